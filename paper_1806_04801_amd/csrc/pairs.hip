// Pair-sum kernels of the HSMA hot path (gfx950, wave64).
//
// One kernel family evaluates, for a set of targets, the Coulomb potential and
// field of a set of sources together with their 27 images in the 3x3x3 block
// of boxes around the central box (the charges inside the auxiliary sphere,
// Sec. II.A; periodic images of Sec. II and the reflected images of Eq. (diel)
// with gamma = -1).  It serves the near-field sum at the particles (Sec. II.C,
// update step), the right-hand side at the monitoring points (Sec. II.A) and
// the two adjoint sums.
//
// Layout of the work: a workgroup of 256 lanes owns 256*T targets (T per
// lane, kept in registers) and one chunk of sources (grid.y).  Sources are
// read at wave-uniform addresses, so they stream through scalar loads into
// SGPRs and feed the vector ALUs directly: no LDS staging and no barriers.
// Images are applied to the per-axis differences: each axis has three
// differences (k = -1, 0, +1) and their squares, so an image costs one add
// for r^2, one rsqrt, and the potential/field updates.  Per-chunk results go to
// a partial buffer that a second kernel sums in a fixed order, so results do
// not depend on scheduling.  In the near sum (SELF) a particle's pairing with
// itself leaves out the central image and, in the periodic block, the images
// of its own charge, whose constant potential the finalize stage adds; in
// single precision the periodic pair potentials are also shifted by a
// constant that the finalize stage restores (images_sum, SHIFT).
#include "hsma_internal.h"
#include "pair_math.h"
#include "stages.h"

namespace hsma {

constexpr int WG = 256;

// One tile: target block tb (256*T targets) against source chunk c.
template <int IMG, bool FIELD, bool SELF, int T>
__device__ __forceinline__ void tile_pair_f64(int tb, int c, const double4* __restrict__ tgt, int nt,
                                              const double4* __restrict__ src, int ns, int chunk,
                                              double L, double* __restrict__ out, int nt_pad,
                                              double gamma = 0.0) {
    const int j0 = c * chunk;
    const int j1 = min(j0 + chunk, ns);
    double tx[T], ty[T], tz[T], ap[T], ax[T], ay[T], az[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        const double4 r = tgt[min(t, nt - 1)];
        tx[u] = r.x; ty[u] = r.y; tz[u] = r.z;
        ap[u] = ax[u] = ay[u] = az[u] = 0.0;
    }
    for (int j = j0; j < j1; ++j) {
        const double4 s = src[j];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            double dx[3], dy[3], dz[3];
            diffs_f64<IMG>(tx[u], s.x, L, dx);
            diffs_f64<IMG>(ty[u], s.y, L, dy);
            diffs_f64<IMG>(tz[u], s.z, L, dz);
            double pot, fx, fy, fz;
            images_sum<double, IMG, FIELD, SELF, false, SELF && IMG == IMG_PERIODIC>(
                dx, dy, dz, pot, fx, fy, fz, nullptr, gamma);
            ap[u] = __builtin_fma(s.w, pot, ap[u]);
            if (FIELD) {
                ax[u] = __builtin_fma(s.w, fx, ax[u]);
                ay[u] = __builtin_fma(s.w, fy, ay[u]);
                az[u] = __builtin_fma(s.w, fz, az[u]);
            }
        }
    }
    constexpr int ncomp = FIELD ? 4 : 1;
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        double* o = out + (size_t)c * ncomp * nt_pad + t;
        o[0] = ap[u];
        if (FIELD) {
            o[(size_t)nt_pad] = ax[u];
            o[(size_t)2 * nt_pad] = ay[u];
            o[(size_t)3 * nt_pad] = az[u];
        }
    }
}

template <int IMG, bool FIELD, bool SELF, int T>
__global__ void __launch_bounds__(WG)
k_pair_f64(const double4* __restrict__ tgt, int nt, const double4* __restrict__ src, int ns,
           int chunk, double L, double* __restrict__ out, int nt_pad, double gamma) {
    tile_pair_f64<IMG, FIELD, SELF, T>(blockIdx.x, blockIdx.y, tgt, nt, src, ns, chunk, L, out, nt_pad,
                                       gamma);
}

// ---------------------------------------------------------------- far images (dielectric box)
// The far part of the dielectric image series at the monitoring points: per
// lane one point; per source of the chunk every image I_k(r) = (-1)^k o r + kL
// with 2 <= max_a |k_a| <= S and weight gamma^|k|, in the order k_x, k_y, k_z
// (the inner block, |k_a| <= 1 on every axis, is skipped).  The powers
// gamma^m, m = 0..S, sit in LDS (every lane reads the same entry); the
// weight of an (x, y) line is hoisted out of the z loop.  The negated sum goes
// to the chunk's partial (the right-hand side is -Phi_far).
constexpr int MAX_FAR_SHELLS = 400;

__global__ void __launch_bounds__(WG)
k_far_shells_f64(const double4* __restrict__ tgt, int nt, const double4* __restrict__ src, int ns,
                 int chunk, double L, double gamma, int S, double* __restrict__ out, int nt_pad) {
    __shared__ double pw[MAX_FAR_SHELLS + 1];
    if (threadIdx.x == 0) {
        double w = 1.0;
        for (int m = 0; m <= S; ++m) {
            pw[m] = w;
            w *= gamma;
        }
    }
    __syncthreads();
    const int t = blockIdx.x * WG + threadIdx.x;
    const double4 p = tgt[min(t, nt - 1)];
    const int j0 = blockIdx.y * chunk;
    const int j1 = min(j0 + chunk, ns);
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double4 r = src[j];
        double sx = 0.0;
        for (int kx = -S; kx <= S; ++kx) {
            const int ax = kx < 0 ? -kx : kx;
            const double dx = p.x - (((kx & 1) ? -r.x : r.x) + kx * L);
            double sy = 0.0;
            for (int ky = -S; ky <= S; ++ky) {
                const int ay = ky < 0 ? -ky : ky;
                const double dy = p.y - (((ky & 1) ? -r.y : r.y) + ky * L);
                const double dxy = __builtin_fma(dy, dy, dx * dx);
                const bool inner = ax <= 1 && ay <= 1;
                double sz = 0.0;
                for (int kz = -S; kz <= S; ++kz) {
                    const int az = kz < 0 ? -kz : kz;
                    if (inner && az <= 1) continue;
                    const double dz = p.z - (((kz & 1) ? -r.z : r.z) + kz * L);
                    sz = __builtin_fma(pw[az], rsqrt_f64(__builtin_fma(dz, dz, dxy)), sz);
                }
                sy = __builtin_fma(pw[ay], sz, sy);
            }
            sx = __builtin_fma(pw[ax], sy, sx);
        }
        acc = __builtin_fma(r.w, sx, acc);
    }
    if (t < nt) out[(size_t)blockIdx.y * nt_pad + t] = -acc;
}

hipError_t launch_far_shells(const double4* tgt, const double4* src, const PairGeom& g, double L,
                             double gamma, int S, double* out, hipStream_t s) {
    if (g.nt <= 0 || g.ns <= 0 || g.tpl != 1) return g.nt <= 0 ? hipSuccess : hipErrorInvalidValue;
    if (S < 1 || S > MAX_FAR_SHELLS) return hipErrorInvalidValue;   // S = 1: no far images, zeros
    hipLaunchKernelGGL(k_far_shells_f64, dim3(g.ntb, g.S), dim3(WG), 0, s, tgt, g.nt, src, g.ns,
                       g.chunk, L, gamma, S, out, g.nt_pad);
    return hipGetLastError();
}

// ---------------------------------------------------------------- single precision
// One tile in single precision.  Each lane sums the (plain float)
// contributions of up to 8 sources into partials and folds them into (hi, lo)
// accumulators with one two-sum per component.  Outputs are scaled back to
// physical units.
template <int IMG, bool FIELD, bool SELF, int T>
__device__ __forceinline__ void tile_pair_f32(int tb, int c, const Rec32* __restrict__ tgt, int nt,
                                              const Rec32* __restrict__ src, int ns, int chunk,
                                              double* __restrict__ out, int nt_pad, double invL) {
    constexpr int G = 8;
    const int j0 = c * chunk;
    const int j1 = min(j0 + chunk, ns);
    Pt32 tp[T];
    float ph[T], pl[T], xh[T], xl[T], yh[T], yl[T], zh[T], zl[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        tp[u] = load_pt32(tgt[min(t, nt - 1)]);
        ph[u] = pl[u] = xh[u] = xl[u] = yh[u] = yl[u] = zh[u] = zl[u] = 0.0f;
    }
    for (int g0 = j0; g0 < j1; g0 += G) {
        const int g1 = min(g0 + G, j1);
        float sp[T], sx[T], sy[T], sz[T];
#pragma unroll
        for (int u = 0; u < T; ++u) sp[u] = sx[u] = sy[u] = sz[u] = 0.0f;
#pragma unroll 2
        for (int j = g0; j < g1; ++j) {
            const Rec32 r0 = src[j];
            const Pt32 s0 = load_pt32(r0);
            const float q0 = r0.v[0].w;
#pragma unroll
            for (int u = 0; u < T; ++u) {
                float dx[3], dy[3], dz[3];
                float p0, fx0, fy0, fz0;
                diffs_f32<IMG>(tp[u], s0, 0, dx);
                diffs_f32<IMG>(tp[u], s0, 1, dy);
                diffs_f32<IMG>(tp[u], s0, 2, dz);
                images_sum<float, IMG, FIELD, SELF, false, SELF, SELF>(dx, dy, dz, p0, fx0, fy0, fz0);
                sp[u] = __builtin_fmaf(q0, p0, sp[u]);
                if (FIELD) {
                    sx[u] = __builtin_fmaf(q0, fx0, sx[u]);
                    sy[u] = __builtin_fmaf(q0, fy0, sy[u]);
                    sz[u] = __builtin_fmaf(q0, fz0, sz[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < T; ++u) {
            two_sum_acc(ph[u], pl[u], sp[u]);
            if (FIELD) {
                two_sum_acc(xh[u], xl[u], sx[u]);
                two_sum_acc(yh[u], yl[u], sy[u]);
                two_sum_acc(zh[u], zl[u], sz[u]);
            }
        }
    }
    constexpr int ncomp = FIELD ? 4 : 1;
    const double invL2 = invL * invL;
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        double* o = out + (size_t)c * ncomp * nt_pad + t;
        o[0] = ((double)ph[u] + (double)pl[u]) * invL;
        if (FIELD) {
            o[(size_t)nt_pad] = ((double)xh[u] + (double)xl[u]) * invL2;
            o[(size_t)2 * nt_pad] = ((double)yh[u] + (double)yl[u]) * invL2;
            o[(size_t)3 * nt_pad] = ((double)zh[u] + (double)zl[u]) * invL2;
        }
    }
}

template <int IMG, bool FIELD, bool SELF, int T>
__global__ void __launch_bounds__(WG)
k_pair_f32(const Rec32* __restrict__ tgt, int nt, const Rec32* __restrict__ src, int ns,
           int chunk, double* __restrict__ out, int nt_pad, double invL) {
    tile_pair_f32<IMG, FIELD, SELF, T>(blockIdx.x, blockIdx.y, tgt, nt, src, ns, chunk, out, nt_pad,
                                       invL);
}

// ---------------------------------------------------------------- explicit charges
// Tiles over an explicit list of point charges (the paper's near set "every
// image inside the auxiliary sphere", generated per source): one pair per
// (target, charge).  SELF: a charge at exactly the target's position (its own
// unshifted copy) is skipped.  The single-precision version sums 8 charges in
// plain float per lane before each two-sum fold.
template <bool FIELD, bool SELF, int T>
__device__ __forceinline__ void tile_free_f64(int tb, int c, const double4* __restrict__ tgt, int nt,
                                              const double4* __restrict__ src, int ns, int chunk,
                                              double* __restrict__ out, int nt_pad) {
    const int j0 = c * chunk;
    const int j1 = min(j0 + chunk, ns);
    double tx[T], ty[T], tz[T], ap[T], ax[T], ay[T], az[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        const double4 r = tgt[min(t, nt - 1)];
        tx[u] = r.x; ty[u] = r.y; tz[u] = r.z;
        ap[u] = ax[u] = ay[u] = az[u] = 0.0;
    }
    auto pair = [&](int j) {
        const double4 s = src[j];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double dx = tx[u] - s.x, dy = ty[u] - s.y, dz = tz[u] - s.z;
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
            double y = rsqrt_f64(r2);
            if (SELF) y = (r2 > 0.0) ? y : 0.0;
            const double qy = s.w * y;
            ap[u] += qy;
            if (FIELD) {
                const double w = qy * (y * y);
                ax[u] = __builtin_fma(w, dx, ax[u]);
                ay[u] = __builtin_fma(w, dy, ay[u]);
                az[u] = __builtin_fma(w, dz, az[u]);
            }
        }
    };
    // groups of four charges are unrolled so that their scalar loads issue together
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) pair(j + k);
    }
    for (; j < j1; ++j) pair(j);
    constexpr int ncomp = FIELD ? 4 : 1;
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        double* o = out + (size_t)c * ncomp * nt_pad + t;
        o[0] = ap[u];
        if (FIELD) {
            o[(size_t)nt_pad] = ax[u];
            o[(size_t)2 * nt_pad] = ay[u];
            o[(size_t)3 * nt_pad] = az[u];
        }
    }
}

template <bool FIELD, bool SELF, int T>
__device__ __forceinline__ void tile_free_f32(int tb, int c, const Rec32* __restrict__ tgt, int nt,
                                              const Rec32* __restrict__ src, int ns, int chunk,
                                              double* __restrict__ out, int nt_pad, double invL) {
    constexpr int G = 8;
    const int j0 = c * chunk;
    const int j1 = min(j0 + chunk, ns);
    float th[T][3], tl[T][3];
    float ph[T], pl[T], xh[T], xl[T], yh[T], yl[T], zh[T], zl[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        const Pt32 p = load_pt32(tgt[min(t, nt - 1)]);
        for (int a = 0; a < 3; ++a) { th[u][a] = p.h0[a]; tl[u][a] = p.l[a]; }
        ph[u] = pl[u] = xh[u] = xl[u] = yh[u] = yl[u] = zh[u] = zl[u] = 0.0f;
    }
    for (int g0 = j0; g0 < j1; g0 += G) {
        const int g1 = min(g0 + G, j1);
        float sp[T], sx[T], sy[T], sz[T];
#pragma unroll
        for (int u = 0; u < T; ++u) sp[u] = sx[u] = sy[u] = sz[u] = 0.0f;
        auto pair = [&](int j) {
            const Pt32 s = load_pt32(src[j]);
            const float q = src[j].v[0].w;
#pragma unroll
            for (int u = 0; u < T; ++u) {
                const float dx = (th[u][0] - s.h0[0]) + (tl[u][0] - s.l[0]);
                const float dy = (th[u][1] - s.h0[1]) + (tl[u][1] - s.l[1]);
                const float dz = (th[u][2] - s.h0[2]) + (tl[u][2] - s.l[2]);
                const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                float y = __builtin_amdgcn_rsqf(r2);
                if (SELF) y = (r2 > 0.0f) ? y : 0.0f;
                const float qy = q * y;
                sp[u] += qy;
                if (FIELD) {
                    const float w = qy * (y * y);
                    sx[u] = __builtin_fmaf(w, dx, sx[u]);
                    sy[u] = __builtin_fmaf(w, dy, sy[u]);
                    sz[u] = __builtin_fmaf(w, dz, sz[u]);
                }
            }
        };
        // a full group is unrolled so that its scalar loads issue together
        if (g1 - g0 == G) {
#pragma unroll
            for (int k = 0; k < G; ++k) pair(g0 + k);
        } else {
            for (int j = g0; j < g1; ++j) pair(j);
        }
#pragma unroll
        for (int u = 0; u < T; ++u) {
            two_sum_acc(ph[u], pl[u], sp[u]);
            if (FIELD) {
                two_sum_acc(xh[u], xl[u], sx[u]);
                two_sum_acc(yh[u], yl[u], sy[u]);
                two_sum_acc(zh[u], zl[u], sz[u]);
            }
        }
    }
    constexpr int ncomp = FIELD ? 4 : 1;
    const double invL2 = invL * invL;
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        double* o = out + (size_t)c * ncomp * nt_pad + t;
        o[0] = ((double)ph[u] + (double)pl[u]) * invL;
        if (FIELD) {
            o[(size_t)nt_pad] = ((double)xh[u] + (double)xl[u]) * invL2;
            o[(size_t)2 * nt_pad] = ((double)yh[u] + (double)yl[u]) * invL2;
            o[(size_t)3 * nt_pad] = ((double)zh[u] + (double)zl[u]) * invL2;
        }
    }
}

template <bool FIELD, bool SELF, int T>
__global__ void __launch_bounds__(WG)
k_free_f64(const double4* __restrict__ tgt, int nt, const double4* __restrict__ src, int ns,
           int chunk, double* __restrict__ out, int nt_pad) {
    tile_free_f64<FIELD, SELF, T>(blockIdx.x, blockIdx.y, tgt, nt, src, ns, chunk, out, nt_pad);
}

template <bool FIELD, bool SELF, int T>
__global__ void __launch_bounds__(WG)
k_free_f32(const Rec32* __restrict__ tgt, int nt, const Rec32* __restrict__ src, int ns,
           int chunk, double* __restrict__ out, int nt_pad, double invL) {
    tile_free_f32<FIELD, SELF, T>(blockIdx.x, blockIdx.y, tgt, nt, src, ns, chunk, out, nt_pad, invL);
}

template <bool FIELD, bool SELF>
static hipError_t free_launch(bool f32, const void* tgt, const void* src, const PairGeom& g,
                              double L, double* out, hipStream_t s) {
    dim3 grid(g.ntb, g.S);
    if (f32) {
        if (g.tpl == 2)
            hipLaunchKernelGGL((k_free_f32<FIELD, SELF, 2>), grid, dim3(WG), 0, s, (const Rec32*)tgt,
                               g.nt, (const Rec32*)src, g.ns, g.chunk, out, g.nt_pad, 1.0 / L);
        else
            hipLaunchKernelGGL((k_free_f32<FIELD, SELF, 1>), grid, dim3(WG), 0, s, (const Rec32*)tgt,
                               g.nt, (const Rec32*)src, g.ns, g.chunk, out, g.nt_pad, 1.0 / L);
    } else {
        if (g.tpl == 2)
            hipLaunchKernelGGL((k_free_f64<FIELD, SELF, 2>), grid, dim3(WG), 0, s, (const double4*)tgt,
                               g.nt, (const double4*)src, g.ns, g.chunk, out, g.nt_pad);
        else
            hipLaunchKernelGGL((k_free_f64<FIELD, SELF, 1>), grid, dim3(WG), 0, s, (const double4*)tgt,
                               g.nt, (const double4*)src, g.ns, g.chunk, out, g.nt_pad);
    }
    return hipGetLastError();
}

hipError_t launch_explicit(bool f32, bool field, bool self, const void* tgt, const void* src,
                           const PairGeom& g, double L, double* out, hipStream_t s) {
    if (g.nt <= 0) return hipSuccess;
    if (g.tpl != 1 && g.tpl != 2) return hipErrorInvalidValue;
    if (field) return self ? free_launch<true, true>(f32, tgt, src, g, L, out, s)
                           : free_launch<true, false>(f32, tgt, src, g, L, out, s);
    if (self) return hipErrorInvalidValue;
    return free_launch<false, false>(f32, tgt, src, g, L, out, s);
}

// ---------------------------------------------------------------- surface images
// Potential and field at targets of M surface points carrying a charge Q_j and
// a point dipole p_j (Sec. II.B; the dipole is the exact limit of the central
// difference of Eq. (cd)):
//   phi = sum Q/|d| + p.d/|d|^3,  E = sum d (Q/|d|^3 + 3 p.d/|d|^5) - p/|d|^3.
template <int T>
__device__ __forceinline__ void tile_surface_f64(int tb, int c, const double4* __restrict__ tgt,
                                                 int nt, const double* __restrict__ surf, int ns,
                                                 int chunk, double* __restrict__ out, int nt_pad) {
    const int j0 = c * chunk;
    const int j1 = min(j0 + chunk, ns);
    double tx[T], ty[T], tz[T], ap[T], ax[T], ay[T], az[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        const double4 r = tgt[min(t, nt - 1)];
        tx[u] = r.x; ty[u] = r.y; tz[u] = r.z;
        ap[u] = ax[u] = ay[u] = az[u] = 0.0;
    }
    for (int j = j0; j < j1; ++j) {
        const double* s = surf + 8 * (size_t)j;
        const double X = s[0], Y = s[1], Z = s[2], Q = s[3], px = s[4], py = s[5], pz = s[6];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double dx = tx[u] - X, dy = ty[u] - Y, dz = tz[u] - Z;
            const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
            const double y = rsqrt_f64(r2);
            const double y2 = y * y;
            const double y3 = y2 * y;
            const double pd = __builtin_fma(px, dx, __builtin_fma(py, dy, pz * dz));
            ap[u] += __builtin_fma(Q, y, pd * y3);
            const double g = y3 * __builtin_fma(3.0 * pd, y2, Q);
            ax[u] += __builtin_fma(g, dx, -px * y3);
            ay[u] += __builtin_fma(g, dy, -py * y3);
            az[u] += __builtin_fma(g, dz, -pz * y3);
        }
    }
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int t = (tb * T + u) * WG + threadIdx.x;
        double* o = out + (size_t)c * 4 * nt_pad + t;
        o[0] = ap[u];
        o[(size_t)nt_pad] = ax[u];
        o[(size_t)2 * nt_pad] = ay[u];
        o[(size_t)3 * nt_pad] = az[u];
    }
}

template <int T>
__global__ void __launch_bounds__(WG)
k_surface_f64(const double4* __restrict__ tgt, int nt, const double* __restrict__ surf, int ns,
              int chunk, double* __restrict__ out, int nt_pad) {
    tile_surface_f64<T>(blockIdx.x, blockIdx.y, tgt, nt, surf, ns, chunk, out, nt_pad);
}

// ---------------------------------------------------------------- helpers
__global__ void k_chunk_reduce(const double* __restrict__ out, int S, int nt, int nt_pad, int ncomp,
                               double* __restrict__ res, int ld) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nt * ncomp) return;
    const int comp = idx / nt, t = idx - comp * nt;
    double acc = 0.0;
    for (int c = 0; c < S; ++c) acc += out[((size_t)c * ncomp + comp) * nt_pad + t];
    res[(size_t)comp * ld + t] = acc;
}

__global__ void k_make_rec32(const double4* __restrict__ p, int n, double L, Rec32* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rec32_body(i, p, L, out);
}

// ---------------------------------------------------------------- grouped tiles
// One launch over the tiles of many requests (continuous batching), all of one
// kind and image mode, so that every launch compiles to the registers of its
// own tile function.  Work-group g finds its group by a binary search over the
// groups' first-tile indices (wave-uniform, so it runs on scalar loads), then
// runs the same tile function as the single-request kernels with one target
// per lane.  The operand pointers come from the descriptors in memory and are
// marked as global memory, so that the wave-uniform source reads compile to
// scalar loads as in the single-request kernels.
template <bool F32, int KIND, int IMG>
__global__ void __launch_bounds__(WG) k_group_tiles(const TileGroup* __restrict__ groups,
                                                   int ngroups) {
    const int g = blockIdx.x;
    int lo = 0, hi = ngroups - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (groups[mid].first <= g) lo = mid;
        else hi = mid - 1;
    }
    const TileGroup* it = groups + lo;
    const int i = g - it->first;
    const int ntb = it->ntb;
    const int c = i / ntb;
    const int tb = i - c * ntb;
    const int nt = it->nt, ns = it->ns, chunk = it->chunk, nt_pad = it->nt_pad;
    double* out = global_ptr(it->out);
    if (KIND == TILE_SURFACE) {
        tile_surface_f64<1>(tb, c, global_ptr((const double4*)it->tgt), nt,
                            global_ptr((const double*)it->src), ns, chunk, out, nt_pad);
    } else if (F32) {
        constexpr bool NEAR = KIND == TILE_NEAR;
        tile_pair_f32<IMG, NEAR, NEAR, 1>(tb, c, global_ptr((const Rec32*)it->tgt), nt,
                                          global_ptr((const Rec32*)it->src), ns, chunk, out, nt_pad,
                                          1.0 / it->L);
    } else {
        constexpr bool NEAR = KIND == TILE_NEAR;
        tile_pair_f64<IMG, NEAR, NEAR, 1>(tb, c, global_ptr((const double4*)it->tgt), nt,
                                          global_ptr((const double4*)it->src), ns, chunk, it->L, out,
                                          nt_pad);
    }
}

template <bool F32>
static void group_tiles(int kind, int img, const TileGroup* groups, int ngroups, int ntiles,
                        hipStream_t s) {
    const dim3 grid(ntiles), blk(WG);
    if (kind == TILE_SURFACE)
        hipLaunchKernelGGL((k_group_tiles<false, TILE_SURFACE, IMG_FREE>), grid, blk, 0, s, groups, ngroups);
    else if (kind == TILE_NEAR && img == IMG_PERIODIC)
        hipLaunchKernelGGL((k_group_tiles<F32, TILE_NEAR, IMG_PERIODIC>), grid, blk, 0, s, groups, ngroups);
    else if (kind == TILE_NEAR)
        hipLaunchKernelGGL((k_group_tiles<F32, TILE_NEAR, IMG_METALLIC>), grid, blk, 0, s, groups, ngroups);
    else if (img == IMG_PERIODIC)
        hipLaunchKernelGGL((k_group_tiles<F32, TILE_RHS, IMG_PERIODIC>), grid, blk, 0, s, groups, ngroups);
    else
        hipLaunchKernelGGL((k_group_tiles<F32, TILE_RHS, IMG_METALLIC>), grid, blk, 0, s, groups, ngroups);
}

hipError_t launch_group_tiles(bool f32, int kind, int img, const TileGroup* groups, int ngroups,
                              int ntiles, hipStream_t s) {
    if (ntiles <= 0 || ngroups <= 0) return hipSuccess;
    if (kind != TILE_SURFACE && img != IMG_PERIODIC && img != IMG_METALLIC) return hipErrorInvalidValue;
    if (f32) group_tiles<true>(kind, img, groups, ngroups, ntiles, s);
    else group_tiles<false>(kind, img, groups, ngroups, ntiles, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launch
PairGeom pair_geometry(int nt, int ns, int tpl, int ncu, int min_chunk) {
    PairGeom g;
    g.nt = nt;
    g.ns = ns;
    g.tpl = tpl;
    g.ntb = (nt + WG * tpl - 1) / (WG * tpl);
    g.nt_pad = g.ntb * WG * tpl;
    if (ns <= 0 || nt <= 0) {
        g.S = 1;
        g.chunk = 0;
        return g;
    }
    // aim at about 20 resident waves per CU times 4 rounds, chunks of at least
    // min_chunk sources (64 for the block images)
    const long want_wg = 20L * ncu;
    long S = (want_wg + g.ntb - 1) / g.ntb;
    const long mc = min_chunk > 0 ? min_chunk : 1;
    long maxS = (ns + mc - 1) / mc;
    if (S > maxS) S = maxS;
    if (S < 1) S = 1;
    g.chunk = (int)((ns + S - 1) / S);
    g.S = (ns + g.chunk - 1) / g.chunk;
    return g;
}

template <int IMG, bool FIELD, bool SELF>
static hipError_t pair64(const double4* tgt, const double4* src, const PairGeom& g, double L,
                         double* out, hipStream_t s, double gamma = 0.0) {
    dim3 grid(g.ntb, g.S);
    if (g.tpl == 2)
        hipLaunchKernelGGL((k_pair_f64<IMG, FIELD, SELF, 2>), grid, dim3(WG), 0, s, tgt, g.nt, src,
                           g.ns, g.chunk, L, out, g.nt_pad, gamma);
    else
        hipLaunchKernelGGL((k_pair_f64<IMG, FIELD, SELF, 1>), grid, dim3(WG), 0, s, tgt, g.nt, src,
                           g.ns, g.chunk, L, out, g.nt_pad, gamma);
    return hipGetLastError();
}

template <int IMG, bool FIELD, bool SELF>
static hipError_t pair32(const Rec32* tgt, const Rec32* src, const PairGeom& g, double* out,
                         double invL, hipStream_t s) {
    dim3 grid(g.ntb, g.S);
    if (g.tpl == 2)
        hipLaunchKernelGGL((k_pair_f32<IMG, FIELD, SELF, 2>), grid, dim3(WG), 0, s, tgt, g.nt, src,
                           g.ns, g.chunk, out, g.nt_pad, invL);
    else
        hipLaunchKernelGGL((k_pair_f32<IMG, FIELD, SELF, 1>), grid, dim3(WG), 0, s, tgt, g.nt, src,
                           g.ns, g.chunk, out, g.nt_pad, invL);
    return hipGetLastError();
}

hipError_t launch_pair_f64(int img, bool field, bool self, const double4* tgt, const double4* src,
                           const PairGeom& g, double L, double* out, hipStream_t s, double gamma) {
    if (g.nt <= 0) return hipSuccess;
    if (img == IMG_DIELECTRIC && field && self)
        return pair64<IMG_DIELECTRIC, true, true>(tgt, src, g, L, out, s, gamma);
    if (g.tpl != 1 && g.tpl != 2) return hipErrorInvalidValue;
    if (img == IMG_PERIODIC) {
        if (field) return self ? pair64<IMG_PERIODIC, true, true>(tgt, src, g, L, out, s)
                               : pair64<IMG_PERIODIC, true, false>(tgt, src, g, L, out, s);
        return pair64<IMG_PERIODIC, false, false>(tgt, src, g, L, out, s);
    }
    if (img == IMG_METALLIC) {
        if (field) return self ? pair64<IMG_METALLIC, true, true>(tgt, src, g, L, out, s)
                               : pair64<IMG_METALLIC, true, false>(tgt, src, g, L, out, s);
        return pair64<IMG_METALLIC, false, false>(tgt, src, g, L, out, s);
    }
    if (img == IMG_FREE && field && !self) return pair64<IMG_FREE, true, false>(tgt, src, g, L, out, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pair_f32(int img, bool field, bool self, const Rec32* tgt, const Rec32* src,
                           const PairGeom& g, double L, double* out, hipStream_t s) {
    if (g.nt <= 0) return hipSuccess;
    if (g.tpl != 1 && g.tpl != 2) return hipErrorInvalidValue;
    const double iL = 1.0 / L;
    if (img == IMG_PERIODIC) {
        if (field) return self ? pair32<IMG_PERIODIC, true, true>(tgt, src, g, out, iL, s)
                               : pair32<IMG_PERIODIC, true, false>(tgt, src, g, out, iL, s);
        return pair32<IMG_PERIODIC, false, false>(tgt, src, g, out, iL, s);
    }
    if (img == IMG_METALLIC) {
        if (field) return self ? pair32<IMG_METALLIC, true, true>(tgt, src, g, out, iL, s)
                               : pair32<IMG_METALLIC, true, false>(tgt, src, g, out, iL, s);
        return pair32<IMG_METALLIC, false, false>(tgt, src, g, out, iL, s);
    }
    if (img == IMG_FREE && field && !self) return pair32<IMG_FREE, true, false>(tgt, src, g, out, iL, s);
    return hipErrorInvalidValue;
}

hipError_t launch_surface_f64(const double4* tgt, const double* surf, const PairGeom& g,
                              double* out, hipStream_t s) {
    if (g.nt <= 0) return hipSuccess;
    dim3 grid(g.ntb, g.S);
    if (g.tpl == 2)
        hipLaunchKernelGGL((k_surface_f64<2>), grid, dim3(WG), 0, s, tgt, g.nt, surf, g.ns, g.chunk,
                           out, g.nt_pad);
    else if (g.tpl == 1)
        hipLaunchKernelGGL((k_surface_f64<1>), grid, dim3(WG), 0, s, tgt, g.nt, surf, g.ns, g.chunk,
                           out, g.nt_pad);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_chunk_reduce(const double* out, const PairGeom& g, int ncomp, double* res, int ld,
                               hipStream_t s) {
    const int n = g.nt * ncomp;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_reduce, dim3((n + 255) / 256), dim3(256), 0, s, out, g.S, g.nt,
                       g.nt_pad, ncomp, res, ld);
    return hipGetLastError();
}

hipError_t launch_make_rec32(const double4* p, int n, double L, Rec32* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_rec32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, L, out);
    return hipGetLastError();
}

}  // namespace hsma
