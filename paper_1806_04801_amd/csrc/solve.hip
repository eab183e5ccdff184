// Update step of the HSMA (Sec. II.C) on one GPU: sources -> right-hand side
// at the monitoring points -> least-squares coefficients -> surface images ->
// near-field and surface sums at the particles -> energy and forces.
#include <cmath>

#include "hsma_internal.h"
#include "solve.h"

namespace hsma {

constexpr int WG = 256;

// ---------------------------------------------------------------- layout
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    if (v == nullptr || *v == 0) return dflt;
    return atoi(v);
}

Layout make_layout(const hsma_plan_s* pl, int64_t N, bool grad) {
    Layout ly;
    ly.N = (int)N;
    ly.ns = (pl->bc == HSMA_BC_SLAB_METALLIC_Z) ? 2 * (int)N : (int)N;
    const bool f32 = pl->precision == HSMA_FP32_COMP;
    const int tpl_near = env_int("HSMA_TPL_NEAR", 2);
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
// Centre (and wrap) the positions, build the source array; grounded slab:
// append the mirror charges -q at z -> -z (mirror reflections plus periodic
// extension turn the slab into a periodic cube of side L).
__global__ void k_prep(const double* __restrict__ x, const double* __restrict__ q, int N, int bc,
                       double L, double4* __restrict__ src, int* __restrict__ status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double c[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    const double qi = q[i];
    int bad = 0;
    if (!isfinite(c[0]) || !isfinite(c[1]) || !isfinite(c[2]) || !isfinite(qi)) bad |= 1;
    const double h = 0.5 * L;
    if (bc == HSMA_BC_PERIODIC) {
        for (int a = 0; a < 3; ++a) {
            double v = c[a] - h;
            v -= L * floor(v / L + 0.5);
            c[a] = v;
        }
    } else if (bc == HSMA_BC_METALLIC) {
        for (int a = 0; a < 3; ++a) {
            c[a] -= h;
            if (!(fabs(c[a]) < h)) bad |= 2;
        }
    } else {
        for (int a = 0; a < 2; ++a) {
            double v = c[a] - h;
            v -= L * floor(v / L + 0.5);
            c[a] = v;
        }
        if (!(c[2] > 0.0 && c[2] < h)) bad |= 2;
    }
    if (bad) atomicOr(status, bad);
    src[i] = make_double4(c[0], c[1], c[2], qi);
    if (bc == HSMA_BC_SLAB_METALLIC_Z) src[N + i] = make_double4(c[0], c[1], -c[2], -qi);
}

__global__ void k_zero_result(Result* r) {
    if (threadIdx.x == 0) {
        r->energy = 0.0;
        r->qsum = 0.0;
        r->qabs = 0.0;
        r->status = 0;
    }
}

// b_k = Phi_in(x_k) (grounded cube) or Phi_in(x_k) - Phi_in(x~_k) (periodic).
__global__ void k_rhs_finalize(const double* __restrict__ part, int S, int nt_pad, int K,
                               int twins, double* __restrict__ b) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double a = 0.0, t = 0.0;
    for (int c = 0; c < S; ++c) a += part[(size_t)c * nt_pad + k];
    if (twins)
        for (int c = 0; c < S; ++c) t += part[(size_t)c * nt_pad + K + k];
    b[k] = a - t;
}

__device__ __forceinline__ double wave_sum(double v) {
    // fixed butterfly order over the 64 lanes
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Least squares (Sec. II.A): A = argmin ||F A + b|| = -R^-1 Q^T b = -P b.
// One wave per coefficient; periodic: A_00 = 0 and the rest follow.
__global__ void __launch_bounds__(WG) k_lsq(const double* __restrict__ P, int nu, int K,
                                           const double* __restrict__ b, int k0,
                                           double* __restrict__ A) {
    const int r = blockIdx.x * (WG / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (r >= nu) return;
    const double* row = P + (size_t)r * K;
    double s = 0.0;
    for (int k = lane; k < K; k += 64) s = __builtin_fma(row[k], b[k], s);
    s = wave_sum(s);
    if (lane == 0) {
        A[k0 + r] = -s;
        if (k0 == 1 && r == 0) A[0] = 0.0;
    }
}

// Harmonic surface mapping (Sec. II.B): surface charge Q_j = Wq_j . A and
// dipole p_j = (Wp_j . A) n_j at the surface points.  One wave per point.
__global__ void __launch_bounds__(WG) k_map(const double* __restrict__ Wq,
                                           const double* __restrict__ Wp, int M, int nb,
                                           const double* __restrict__ A,
                                           const double* __restrict__ spos, double Rs,
                                           double* __restrict__ surf) {
    const int j = blockIdx.x * (WG / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (j >= M) return;
    const double* wq = Wq + (size_t)j * nb;
    const double* wp = Wp + (size_t)j * nb;
    double sq = 0.0, sp = 0.0;
    for (int k = lane; k < nb; k += 64) {
        const double a = A[k];
        sq = __builtin_fma(wq[k], a, sq);
        sp = __builtin_fma(wp[k], a, sp);
    }
    sq = wave_sum(sq);
    sp = wave_sum(sp);
    if (lane == 0) {
        const double X = spos[4 * j], Y = spos[4 * j + 1], Z = spos[4 * j + 2];
        double* o = surf + 8 * (size_t)j;
        o[0] = X; o[1] = Y; o[2] = Z; o[3] = sq;
        o[4] = sp * X / Rs; o[5] = sp * Y / Rs; o[6] = sp * Z / Rs; o[7] = 0.0;
    }
}

// phi = near + surface (chunk sums in fixed order), F = q E, block partial
// sums of q phi, q and |q| for the energy and the neutrality check.
__global__ void __launch_bounds__(WG)
k_finalize(const double* __restrict__ near, int Sn, int npad, const double* __restrict__ surfp,
           int Ss, int spad, const double4* __restrict__ src, int N, double* __restrict__ phi,
           double* __restrict__ forces, double* __restrict__ dbg_pn, double* __restrict__ dbg_fn,
           double* __restrict__ dbg_po, double* __restrict__ dbg_fo, double* __restrict__ eblk) {
    __shared__ double sh[3][WG];
    const int i = blockIdx.x * WG + threadIdx.x;
    double e = 0.0, qs = 0.0, qa = 0.0;
    if (i < N) {
        double vn[4], vo[4];
        for (int comp = 0; comp < 4; ++comp) {
            double a = 0.0, b = 0.0;
            for (int c = 0; c < Sn; ++c) a += near[((size_t)c * 4 + comp) * npad + i];
            for (int c = 0; c < Ss; ++c) b += surfp[((size_t)c * 4 + comp) * spad + i];
            vn[comp] = a;
            vo[comp] = b;
        }
        const double qi = src[i].w;
        const double p = vn[0] + vo[0];
        if (phi) phi[i] = p;
        if (forces) {
            forces[3 * i] = qi * (vn[1] + vo[1]);
            forces[3 * i + 1] = qi * (vn[2] + vo[2]);
            forces[3 * i + 2] = qi * (vn[3] + vo[3]);
        }
        if (dbg_pn) dbg_pn[i] = vn[0];
        if (dbg_po) dbg_po[i] = vo[0];
        if (dbg_fn) { dbg_fn[3 * i] = vn[1]; dbg_fn[3 * i + 1] = vn[2]; dbg_fn[3 * i + 2] = vn[3]; }
        if (dbg_fo) { dbg_fo[3 * i] = vo[1]; dbg_fo[3 * i + 1] = vo[2]; dbg_fo[3 * i + 2] = vo[3]; }
        e = qi * p;
        qs = qi;
        qa = fabs(qi);
    }
    sh[0][threadIdx.x] = e;
    sh[1][threadIdx.x] = qs;
    sh[2][threadIdx.x] = qa;
    __syncthreads();
    for (int w = WG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        eblk[3 * blockIdx.x] = sh[0][0];
        eblk[3 * blockIdx.x + 1] = sh[1][0];
        eblk[3 * blockIdx.x + 2] = sh[2][0];
    }
}

// E = 1/2 sum q phi; neutrality flag for periodic and slab systems.
__global__ void __launch_bounds__(WG) k_energy(const double* __restrict__ eblk, int nblk,
                                              int need_neutral, Result* __restrict__ res) {
    __shared__ double sh[3][WG];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < nblk; k += WG) {
        a += eblk[3 * k];
        b += eblk[3 * k + 1];
        c += eblk[3 * k + 2];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    sh[2][threadIdx.x] = c;
    __syncthreads();
    for (int w = WG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res->energy = 0.5 * sh[0][0];
        res->qsum = sh[1][0];
        res->qabs = sh[2][0];
        if (need_neutral && fabs(sh[1][0]) > 1e-12 * sh[2][0]) res->status |= 4;
    }
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
        CK(launch_pair_f32(pl->img, false, false, pl->d_chk32, src32, ly.g_rhs, (float)pl->L,
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
        CK(launch_pair_f32(pl->img, true, true, src32, src32, ly.g_near, (float)pl->L, near_part, s));
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
