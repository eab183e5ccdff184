// Update step of the HSMA (Sec. II.C) on one GPU: sources -> right-hand side
// at the monitoring points -> least-squares coefficients -> surface images ->
// near-field and surface sums at the particles -> energy and forces.
#include <cmath>

#include "hsma_internal.h"
#include "solve.h"
#include "stages.h"

namespace hsma {

constexpr int WG = 256;

// ---------------------------------------------------------------- layout
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    if (v == nullptr || *v == 0) return dflt;
    return atoi(v);
}

Layout make_layout(const hsma_plan_s* pl, int64_t N, bool grad, int tpl_near_override,
                   int precision_override) {
    Layout ly;
    ly.N = (int)N;
    ly.ns = (pl->bc == HSMA_BC_SLAB_METALLIC_Z) ? 2 * (int)N : (int)N;
    const int prec = precision_override >= 0 ? precision_override : pl->precision;
    const bool f32 = prec == HSMA_FP32_COMP;
    const int tpl_near = tpl_near_override > 0 ? tpl_near_override : env_int("HSMA_TPL_NEAR", 2);
    const int tpl_rhs = env_int("HSMA_TPL_RHS", 1);
    ly.g_rhs = pair_geometry(pl->nchk, ly.ns, tpl_rhs, pl->ncu);
    ly.g_near = pair_geometry(ly.N, ly.ns, tpl_near, pl->ncu);
    ly.g_surf = pair_geometry(ly.N, pl->M, 1, pl->ncu);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    ly.off_src64 = take(sizeof(double4) * (size_t)ly.ns);
    ly.off_src32 = f32 ? take(sizeof(Rec32) * (size_t)ly.ns) : 0;
    ly.off_rhs_part = take(sizeof(double) * (size_t)ly.g_rhs.S * ly.g_rhs.nt_pad);
    ly.off_b = take(sizeof(double) * (size_t)pl->K);
    ly.off_A = take(sizeof(double) * (size_t)pl->nb);
    ly.off_surf = take(sizeof(double) * 8 * (size_t)pl->M);
    ly.off_near_part = take(sizeof(double) * 4 * (size_t)ly.g_near.S * ly.g_near.nt_pad);
    ly.off_surf_part = take(sizeof(double) * 4 * (size_t)ly.g_surf.S * ly.g_surf.nt_pad);
    ly.n_eblk = (ly.N + WG - 1) / WG;
    if (ly.n_eblk < 1) ly.n_eblk = 1;
    ly.off_eblk = take(sizeof(double) * 3 * (size_t)ly.n_eblk);
    ly.off_result = take(sizeof(Result));
    if (grad) {
        ly.g_u = pair_geometry(pl->M, ly.N, 1, pl->ncu);
        ly.g_G = pair_geometry(ly.ns, pl->nchk, tpl_near, pl->ncu);
        ly.off_u_part = take(sizeof(double) * 4 * (size_t)ly.g_u.S * ly.g_u.nt_pad);
        ly.off_tw = take(sizeof(double) * (size_t)pl->nb);
        ly.off_ud = take(sizeof(double) * 2 * (size_t)pl->M);
        ly.off_lam64 = take(sizeof(double4) * (size_t)pl->nchk);
        ly.off_lam32 = f32 ? take(sizeof(Rec32) * (size_t)pl->nchk) : 0;
        ly.off_G_part = take(sizeof(double) * 4 * (size_t)ly.g_G.S * ly.g_G.nt_pad);
    }
    ly.total = o;
    return ly;
}

// ---------------------------------------------------------------- kernels
__global__ void k_prep(const double* __restrict__ x, const double* __restrict__ q, int N, int bc,
                       double L, double4* __restrict__ src, int* __restrict__ status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) prep_body(i, x, q, N, bc, L, src, status);
}

__global__ void k_zero_result(Result* r) {
    if (threadIdx.x == 0) {
        r->energy = 0.0;
        r->qsum = 0.0;
        r->qabs = 0.0;
        r->status = 0;
    }
}

__global__ void k_rhs_finalize(const double* __restrict__ part, int S, int nt_pad, int K,
                               int twins, double* __restrict__ b) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) rhs_body(k, part, S, nt_pad, K, twins, b);
}

__global__ void __launch_bounds__(WG) k_lsq(const double* __restrict__ P, int nu, int K,
                                           const double* __restrict__ b, int k0,
                                           double* __restrict__ A) {
    const int r = blockIdx.x * (WG / 64) + threadIdx.x / 64;
    if (r < nu) lsq_body(r, threadIdx.x & 63, P, K, b, k0, A);
}

__global__ void __launch_bounds__(WG) k_map(const double* __restrict__ Wq,
                                           const double* __restrict__ Wp, int M, int nb,
                                           const double* __restrict__ A,
                                           const double* __restrict__ spos, double Rs,
                                           double* __restrict__ surf) {
    const int j = blockIdx.x * (WG / 64) + threadIdx.x / 64;
    if (j < M) map_body(j, threadIdx.x & 63, Wq, Wp, nb, A, spos, Rs, surf);
}

__global__ void __launch_bounds__(WG)
k_finalize(const double* __restrict__ near, int Sn, int npad, const double* __restrict__ surfp,
           int Ss, int spad, const double4* __restrict__ src, int N, double* __restrict__ phi,
           double* __restrict__ forces, double* __restrict__ dbg_pn, double* __restrict__ dbg_fn,
           double* __restrict__ dbg_po, double* __restrict__ dbg_fo, double* __restrict__ eblk) {
    finalize_body(blockIdx.x, near, Sn, npad, surfp, Ss, spad, src, N, phi, forces, dbg_pn, dbg_fn,
                  dbg_po, dbg_fo, eblk);
}

__global__ void __launch_bounds__(WG) k_energy(const double* __restrict__ eblk, int nblk,
                                              int need_neutral, Result* __restrict__ res) {
    energy_body(eblk, nblk, need_neutral, res);
}

// ---------------------------------------------------------------- pipeline
#define CK(call)                                                                             \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(HSMA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

hsma_status forward(const hsma_plan_s* pl, const Layout& ly, const double* x, const double* q,
                    char* ws, hipStream_t s, double* phi, double* forces,
                    const hsma_intermediates* dbg) {
    const int N = ly.N;
    const bool f32 = pl->precision == HSMA_FP32_COMP;
    double4* src64 = (double4*)(ws + ly.off_src64);
    Rec32* src32 = f32 ? (Rec32*)(ws + ly.off_src32) : nullptr;
    double* rhs_part = (double*)(ws + ly.off_rhs_part);
    double* b = (double*)(ws + ly.off_b);
    double* A = (double*)(ws + ly.off_A);
    double* surf = (double*)(ws + ly.off_surf);
    double* near_part = (double*)(ws + ly.off_near_part);
    double* surf_part = (double*)(ws + ly.off_surf_part);
    double* eblk = (double*)(ws + ly.off_eblk);
    Result* res = (Result*)(ws + ly.off_result);

    hipLaunchKernelGGL(k_zero_result, dim3(1), dim3(64), 0, s, res);
    hipLaunchKernelGGL(k_prep, dim3((N + WG - 1) / WG), dim3(WG), 0, s, x, q, N, pl->bc, pl->L,
                       src64, &res->status);
    CK(hipGetLastError());
    if (f32) CK(launch_make_rec32(src64, ly.ns, pl->L, src32, s));
    // right-hand side at the monitoring points (and twins)
    timing_begin(1, s);
    if (f32)
        CK(launch_pair_f32(pl->img, false, false, pl->d_chk32, src32, ly.g_rhs, pl->L,
                           rhs_part, s));
    else
        CK(launch_pair_f64(pl->img, false, false, pl->d_chk64, src64, ly.g_rhs, pl->L, rhs_part, s));
    timing_end(1, s);
    hipLaunchKernelGGL(k_rhs_finalize, dim3((pl->K + WG - 1) / WG), dim3(WG), 0, s, rhs_part,
                       ly.g_rhs.S, ly.g_rhs.nt_pad, pl->K, pl->img == IMG_PERIODIC ? 1 : 0, b);
    hipLaunchKernelGGL(k_lsq, dim3((pl->nu + 3) / 4), dim3(WG), 0, s, pl->d_P, pl->nu, pl->K, b,
                       pl->nb - pl->nu, A);
    hipLaunchKernelGGL(k_map, dim3((pl->M + 3) / 4), dim3(WG), 0, s, pl->d_Wq, pl->d_Wp, pl->M,
                       pl->nb, A, pl->d_spos, pl->Rs, surf);
    CK(hipGetLastError());
    // near field at the particles: the sources and their 27 images, self excluded
    timing_begin(0, s);
    if (f32)
        CK(launch_pair_f32(pl->img, true, true, src32, src32, ly.g_near, pl->L, near_part, s));
    else
        CK(launch_pair_f64(pl->img, true, true, src64, src64, ly.g_near, pl->L, near_part, s));
    timing_end(0, s);
    // surface images at the particles
    timing_begin(2, s);
    CK(launch_surface_f64(src64, surf, ly.g_surf, surf_part, s));
    timing_end(2, s);
    hipLaunchKernelGGL(k_finalize, dim3(ly.n_eblk), dim3(WG), 0, s, near_part, ly.g_near.S,
                       ly.g_near.nt_pad, surf_part, ly.g_surf.S, ly.g_surf.nt_pad, src64, N, phi,
                       forces, dbg ? dbg->phi_near : nullptr, dbg ? dbg->field_near : nullptr,
                       dbg ? dbg->phi_out : nullptr, dbg ? dbg->field_out : nullptr, eblk);
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(WG), 0, s, eblk, ly.n_eblk,
                       pl->bc != HSMA_BC_METALLIC ? 1 : 0, res);
    CK(hipGetLastError());
    if (dbg) {
        if (dbg->b) CK(hipMemcpyAsync(dbg->b, b, sizeof(double) * pl->K, hipMemcpyDeviceToDevice, s));
        if (dbg->A) CK(hipMemcpyAsync(dbg->A, A, sizeof(double) * pl->nb, hipMemcpyDeviceToDevice, s));
        if (dbg->surf)
            CK(hipMemcpyAsync(dbg->surf, surf, sizeof(double) * 8 * pl->M, hipMemcpyDeviceToDevice, s));
    }
    return HSMA_OK;
}

hsma_status read_result(const Layout& ly, char* ws, hipStream_t s, double* energy) {
    Result h;
    CK(hipMemcpyAsync(&h, ws + ly.off_result, sizeof(Result), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (h.status & 1) return fail(HSMA_E_INVALID, "non-finite position or charge");
    if (h.status & 2) return fail(HSMA_E_OUT_OF_BOX, "position on or outside a grounded wall");
    if (h.status & 4) return fail(HSMA_E_NOT_NEUTRAL, "periodic/slab system is not neutral");
    if (energy) *energy = h.energy;
    return HSMA_OK;
}

}  // namespace hsma
