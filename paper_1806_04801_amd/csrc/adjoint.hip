// Adjoint of the HSMA update step: the exact gradient of the computed energy
// with respect to positions and charges.
//
// E = 1/2 sum_{i real} q_i (phi_near_i + phi_out_i).  The near part is a
// symmetric pair sum, so dE_near/dq_i = phi_near_i and dE_near/dr_i =
// -q_i E_near_i.  The far part E_out = 1/2 u^T T A depends on the charges and
// positions also through the least-squares coefficients A = -P b (Sec. II.A):
//   u_j   = sum_i q_i [1/|d|, d/|d|^3] at the surface points (d = r_i - R_j),
//   tw    = T^T u    (T: A -> surface charges and dipoles, Sec. II.B),
//   lam   = P^T tw   (so that E_out = -1/2 lam^T b),
//   G(r)  = sum_k lam_k g_k(r), g_k the contribution of a unit charge at r to b_k,
// giving dE/dq_i = phi_near_i + 1/2 phi_out_i - 1/2 G(r_i) and
// dE/dr_i = -q_i E_near_i - 1/2 q_i E_out_i - 1/2 q_i grad G(r_i).
// G is itself an image pair sum: the potential at r of charges lam_k at the
// monitoring points (and -lam_k at their twins) with the same 27 images.
// Slab: the mirror charge (x, y, -z; -q) moves with its source, so G and
// grad G at the mirror enter through that map.
#include "hsma_internal.h"
#include "solve.h"

namespace hsma {

constexpr int WG = 256;

// Chunk sums of the surface response: ud[j] = (u_pot_j, n_j . u_vec_j) with
// u_vec = -E (the field of the sources at R_j).
__global__ void k_u_reduce(const double* __restrict__ part, int S, int nt_pad, int M,
                           const double* __restrict__ spos, double Rs, double* __restrict__ ud) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    double v[4];
    for (int comp = 0; comp < 4; ++comp) {
        double a = 0.0;
        for (int c = 0; c < S; ++c) a += part[((size_t)c * 4 + comp) * nt_pad + j];
        v[comp] = a;
    }
    const double nx = spos[4 * j] / Rs, ny = spos[4 * j + 1] / Rs, nz = spos[4 * j + 2] / Rs;
    ud[2 * j] = v[0];
    ud[2 * j + 1] = -(nx * v[1] + ny * v[2] + nz * v[3]);
}

// tw_k = sum_j Wq[j][k] u_pot_j + Wp[j][k] (n_j . u_vec_j)   (T^T u)
__global__ void k_tw(const double* __restrict__ Wq, const double* __restrict__ Wp, int M, int nb,
                     const double* __restrict__ ud, double* __restrict__ tw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    double a = 0.0;
    for (int j = 0; j < M; ++j) {
        a = __builtin_fma(Wq[(size_t)j * nb + k], ud[2 * j], a);
        a = __builtin_fma(Wp[(size_t)j * nb + k], ud[2 * j + 1], a);
    }
    tw[k] = a;
}

// lam = P^T tw' (tw' = the fitted coefficients' part); weighted check points
// as sources: lam_i at x_i and, periodic, -lam_i at the twin x~_i.
__global__ void k_lambda(const double* __restrict__ P, int nu, int K, const double* __restrict__ tw,
                         int k0, const double4* __restrict__ chk, int twins,
                         double4* __restrict__ lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    double a = 0.0;
    for (int r = 0; r < nu; ++r) a = __builtin_fma(P[(size_t)r * K + i], tw[k0 + r], a);
    const double4 x = chk[i];
    lam[i] = make_double4(x.x, x.y, x.z, a);
    if (twins) {
        const double4 t = chk[K + i];
        lam[K + i] = make_double4(t.x, t.y, t.z, -a);
    }
}

__device__ __forceinline__ void chunk_sum4(const double* __restrict__ part, int S, int pad, int i,
                                           double (&v)[4]) {
    for (int comp = 0; comp < 4; ++comp) {
        double a = 0.0;
        for (int c = 0; c < S; ++c) a += part[((size_t)c * 4 + comp) * pad + i];
        v[comp] = a;
    }
}

__global__ void k_grad_finalize(const double* __restrict__ near, int Sn, int npad,
                                const double* __restrict__ surfp, int Ss, int spad,
                                const double* __restrict__ Gp, int Sg, int gpad,
                                const double4* __restrict__ src, int N, int slab, NearFix fix,
                                const double* __restrict__ qnet, double* __restrict__ dEdx,
                                double* __restrict__ dEdq) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double vn[4], vo[4], vg[4];
    chunk_sum4(near, Sn, npad, i, vn);
    chunk_sum4(surfp, Ss, spad, i, vo);
    chunk_sum4(Gp, Sg, gpad, i, vg);
    if (slab) {
        double vm[4];
        chunk_sum4(Gp, Sg, gpad, N + i, vm);
        // G(r) - G(M r); grad: grad G(r) - M grad G(M r), M = diag(1, 1, -1)
        vg[0] -= vm[0];
        vg[1] -= vm[1];
        vg[2] -= vm[2];
        vg[3] += vm[3];
    }
    const double q = src[i].w;
    vn[0] += q * fix.own;   // as in the forward finalize stage
    if (fix.qc != 0.0) vn[0] += *qnet * fix.qc;
    dEdq[i] = vn[0] + 0.5 * vo[0] - 0.5 * vg[0];
    // grad G = -E_G
    for (int a = 0; a < 3; ++a)
        dEdx[3 * i + a] = -q * vn[1 + a] - 0.5 * q * vo[1 + a] + 0.5 * q * vg[1 + a];
}

#define CK(call)                                                                             \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(HSMA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

hsma_status backward(const hsma_plan_s* pl, const Layout& ly, char* ws, hipStream_t s,
                     double* dEdx, double* dEdq) {
    const bool f32 = ly.f32;
    const double4* src64 = (const double4*)(ws + ly.off_src64);
    const Rec32* src32 = f32 ? (const Rec32*)(ws + ly.off_src32) : nullptr;
    double* u_part = (double*)(ws + ly.off_u_part);
    double* ud = (double*)(ws + ly.off_ud);
    double* tw = (double*)(ws + ly.off_tw);
    double4* lam64 = (double4*)(ws + ly.off_lam64);
    Rec32* lam32 = f32 ? (Rec32*)(ws + ly.off_lam32) : nullptr;
    double* G_part = (double*)(ws + ly.off_G_part);
    // response of the real charges at the surface points (no images), double precision
    CK(launch_pair_f64(IMG_FREE, true, false, (const double4*)pl->d_spos, src64, ly.g_u, pl->L,
                       u_part, s));
    hipLaunchKernelGGL(k_u_reduce, dim3((pl->M + WG - 1) / WG), dim3(WG), 0, s, u_part, ly.g_u.S,
                       ly.g_u.nt_pad, pl->M, pl->d_spos, pl->Rs, ud);
    hipLaunchKernelGGL(k_tw, dim3((pl->nb + 63) / 64), dim3(64), 0, s, pl->d_Wq, pl->d_Wp, pl->M,
                       pl->nb, ud, tw);
    hipLaunchKernelGGL(k_lambda, dim3((pl->K + WG - 1) / WG), dim3(WG), 0, s, pl->d_P, pl->nu, pl->K,
                       tw, pl->nb - pl->nu, pl->d_chk64, pl->img == IMG_PERIODIC ? 1 : 0, lam64);
    CK(hipGetLastError());
    // G and its field at every source (real and mirror)
    if (f32) {
        CK(launch_make_rec32(lam64, pl->nchk, pl->L, lam32, s));
        CK(launch_pair_f32(pl->img, true, false, src32, lam32, ly.g_G, pl->L, G_part, s));
    } else {
        CK(launch_pair_f64(pl->img, true, false, src64, lam64, ly.g_G, pl->L, G_part, s));
    }
    hipLaunchKernelGGL(k_grad_finalize, dim3((ly.N + WG - 1) / WG), dim3(WG), 0, s,
                       (const double*)(ws + ly.off_near_part), ly.sym ? ly.g_sym.C + ly.g_sym.s : ly.g_near.S,
                       ly.sym ? ly.g_sym.n_pad : ly.g_near.nt_pad,
                       (const double*)(ws + ly.off_surf_part), ly.g_surf.S, ly.g_surf.nt_pad,
                       G_part, ly.g_G.S, ly.g_G.nt_pad, src64, ly.N,
                       pl->bc == HSMA_BC_SLAB_METALLIC_Z ? 1 : 0, near_fix(pl, ly),
                       &((const Result*)(ws + ly.off_result))->qnet, dEdx, dEdq);
    CK(hipGetLastError());
    return HSMA_OK;
}

}  // namespace hsma
