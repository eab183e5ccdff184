// Near-field sum at the particles with every unordered pair of particles
// evaluated once (Sec. II.C, the near part of the update step; 3x3x3 image
// block of the periodic box or of the grounded box, Eq. (diel) with
// gamma = -1).
//
// The near sum over the image block is symmetric in the two particles of a
// pair: the distance from i to image k of j equals the distance from j to
// image k' of i, where k' = -k on periodic axes and k' = k on reflected axes,
// and the image signs agree.  So one pass over the pair gives both
// directions: the potential term is the same, the field at j is the field at i
// with the sign pattern of images_sum<..., REV>.
//
// Work layout.  Particles are cut into nb blocks of B = 64 * T * s.  The
// block pairs (I, J), I < J, are scheduled as a round-robin tournament: in
// each round every block takes part in exactly one pair, so no two
// work-groups of a round touch the same particle's accumulators and the
// rounds accumulate in place, in a fixed order, without atomics.  A pair is
// split into s row slices and C column parts; work-group (pair, slice,
// part) is one wave that keeps 64 * T rows of block I in registers (T per
// lane) and reads its part of the B columns of block J at wave-uniform
// addresses (scalar loads).  Forward terms (at the rows) accumulate per lane
// as in the plain tile kernel and go to part c's copy of the row
// accumulators; reverse terms (at the columns) are reduced over the wave's
// rows with a 64-lane reduce-scatter and go to slice sigma's copy of the
// column accumulators.  The diagonal pairs (I, I) run first, forward only,
// with the self term of the central image left out; they also initialise
// every accumulator of their rows.
//
// Accumulators: acc[c] = forward from column part c (c < C), acc[C + sigma] =
// reverse from row slice sigma, each 4 components x n_pad doubles (potential,
// field x, y, z), physical units.  The finalize stage sums the C + s copies in
// that order.
#include "hsma_internal.h"
#include "pair_math.h"

namespace hsma {

constexpr int SW = 64;   // one wave per work-group

__device__ __forceinline__ bool parity(int x) { return __builtin_popcount(x) & 1; }

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float lane_f(float x, int src_lane) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(x)));
}

// One halving step of the reduce-scatter: lane l and its partner l ^ m hold
// the same N pairs (v[k], v[k + N]); the lane with f set keeps the upper
// halves, the other the lower ones, and each adds the partner's copy.
template <int N, int CTRL>
__device__ __forceinline__ void rs_step(float (&v)[16], bool f) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float lo = v[k], hi = v[k + N];
        const float keep = f ? hi : lo;
        const float send = f ? lo : hi;
        v[k] = keep + dpp_f<CTRL>(send);
    }
}

// Sum of 16 values over the 64 lanes of the wave.  The row-local partners are
// lane ^ 1, ^ 2 (quad permutations), ^ 7 (half-row mirror) and ^ 15 (row
// mirror); the lane bits that pick the kept half are parities of lane & 5,
// lane & 6, lane & 12 and lane & 8, which form the dual basis of those four
// masks, so partners always hold the same subset.  After the four steps each
// lane of a row holds one distinct value, summed over its row; two exchanges
// across rows (lane ^ 16, lane ^ 32) finish the sum.  Lane l then holds value
// rs_owner(l), and lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same one.
__device__ __forceinline__ int rs_owner(int lane) {
    return parity(lane & 5) * 8 + parity(lane & 6) * 4 + parity(lane & 12) * 2 + ((lane >> 3) & 1);
}

__device__ __forceinline__ float reduce_scatter16(float (&v)[16], int lane) {
    rs_step<8, 0xB1>(v, parity(lane & 5));     // quad_perm [1,0,3,2]
    rs_step<4, 0x4E>(v, parity(lane & 6));     // quad_perm [2,3,0,1]
    rs_step<2, 0x141>(v, parity(lane & 12));   // row_half_mirror
    rs_step<1, 0x140>(v, (lane >> 3) & 1);     // row_mirror
    float e = v[0];
    e += lane_f(e, lane ^ 16);
    e += lane_f(e, lane ^ 32);
    return e;
}

template <int IMG, int T, bool DIAG>
__global__ void __launch_bounds__(SW)
k_sym_f32(const Rec32* __restrict__ pts, SymGeom g, int round, double invL, double* __restrict__ acc) {
    const int lane = threadIdx.x;
    // consecutive work items (the slices of one pair read the same columns)
    // go to the same XCD: the hardware deals work-groups round-robin over 8
    const int per_xcd = gridDim.x >> 3;
    const int id = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const int per_pair = g.s * g.C;
    int I, J, pr;
    if (DIAG) {
        if (id >= g.nb * per_pair) return;
        I = J = pr = id / per_pair;
    } else {
        if (id >= (g.P >> 1) * per_pair) return;
        pr = id / per_pair;
        const int m = g.P - 1;
        if (pr == 0) {
            I = m;
            J = round;
        } else {
            I = (round + pr) % m;
            J = (round - pr + m) % m;
        }
        if (I >= g.nb || J >= g.nb) return;   // the bye of an odd block count
    }
    const int rem = id - pr * per_pair;
    const int sig = rem / g.C;
    const int part = rem - sig * g.C;
    const size_t cs = (size_t)4 * g.n_pad;
    double* __restrict__ fwd = acc + (size_t)part * cs;
    double* __restrict__ rev = acc + (size_t)(g.C + sig) * cs;
    const double invL2 = invL * invL;

    // rows: 64 * T particles of block I; lanes past the end carry no charge
    // and sit far outside every image of the box
    const int r0 = I * g.B + sig * SW * T;
    Pt32 tp[T];
    float qi[T];
    float ph[T], pl[T], xh[T], xl[T], yh[T], yl[T], zh[T], zl[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int i = r0 + u * SW + lane;
        const Rec32 rec = pts[min(i, g.n - 1)];
        tp[u] = load_pt32(rec);
        qi[u] = rec.v[0].w;
        if (i >= g.n) {
            qi[u] = 0.0f;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                tp[u].h0[a] = tp[u].hp[a] = tp[u].hm[a] = 1000.0f;
                tp[u].l[a] = 0.0f;
            }
        }
        ph[u] = pl[u] = xh[u] = xl[u] = yh[u] = yl[u] = zh[u] = zl[u] = 0.0f;
    }

    const int c0 = min(J * g.B + (int)((long)part * g.B / g.C), g.n);
    const int c1 = min(J * g.B + (int)((long)(part + 1) * g.B / g.C), g.n);
    const int kown = rs_owner(lane);
    const int kcol = kown >> 2, kcomp = kown & 3;
    const double oscale = kcomp == 0 ? invL : invL2;
    for (int g0 = c0; g0 < c1; g0 += 8) {
        float sp[T], sx[T], sy[T], sz[T];
#pragma unroll
        for (int u = 0; u < T; ++u) sp[u] = sx[u] = sy[u] = sz[u] = 0.0f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int jb = g0 + 4 * h;
            const int nh = min(4, c1 - jb);
            if (nh <= 0) break;
            double old = 0.0;
            double* dst = nullptr;
            if (!DIAG && lane < 16 && kcol < nh) {
                dst = rev + (size_t)kcomp * g.n_pad + jb + kcol;
                old = *dst;
            }
            float rv[16];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float rp = 0.0f, rx = 0.0f, ry = 0.0f, rz = 0.0f;
                if (q < nh) {
                    const Rec32 rec = pts[jb + q];
                    const Pt32 sj = load_pt32(rec);
                    const float qj = rec.v[0].w;
#pragma unroll
                    for (int u = 0; u < T; ++u) {
                        float dx[3], dy[3], dz[3];
                        diffs_f32<IMG>(tp[u], sj, 0, dx);
                        diffs_f32<IMG>(tp[u], sj, 1, dy);
                        diffs_f32<IMG>(tp[u], sj, 2, dz);
                        float p0, fx0, fy0, fz0, rf[3];
                        images_sum<float, IMG, true, true, !DIAG>(dx, dy, dz, p0, fx0, fy0, fz0, rf);
                        sp[u] = __builtin_fmaf(qj, p0, sp[u]);
                        sx[u] = __builtin_fmaf(qj, fx0, sx[u]);
                        sy[u] = __builtin_fmaf(qj, fy0, sy[u]);
                        sz[u] = __builtin_fmaf(qj, fz0, sz[u]);
                        if (!DIAG) {
                            rp = __builtin_fmaf(qi[u], p0, rp);
                            rx = __builtin_fmaf(qi[u], rf[0], rx);
                            ry = __builtin_fmaf(qi[u], rf[1], ry);
                            rz = __builtin_fmaf(qi[u], rf[2], rz);
                        }
                    }
                }
                rv[4 * q + 0] = rp;
                rv[4 * q + 1] = rx;
                rv[4 * q + 2] = ry;
                rv[4 * q + 3] = rz;
            }
            if (!DIAG) {
                const float e = reduce_scatter16(rv, lane);
                if (dst != nullptr) *dst = old + (double)e * oscale;
            }
        }
#pragma unroll
        for (int u = 0; u < T; ++u) {
            two_sum_acc(ph[u], pl[u], sp[u]);
            two_sum_acc(xh[u], xl[u], sx[u]);
            two_sum_acc(yh[u], yl[u], sy[u]);
            two_sum_acc(zh[u], zl[u], sz[u]);
        }
    }

#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int i = r0 + u * SW + lane;
        if (i >= g.n) continue;
        const double v[4] = {((double)ph[u] + (double)pl[u]) * invL,
                             ((double)xh[u] + (double)xl[u]) * invL2,
                             ((double)yh[u] + (double)yl[u]) * invL2,
                             ((double)zh[u] + (double)zl[u]) * invL2};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double* f = fwd + (size_t)c * g.n_pad + i;
            *f = DIAG ? v[c] : *f + v[c];
        }
        if (DIAG && part == 0) {
            for (int t = 0; t < g.s; ++t) {
                double* r = acc + (size_t)(g.C + t) * cs + i;
#pragma unroll
                for (int c = 0; c < 4; ++c) r[(size_t)c * g.n_pad] = 0.0;
            }
        }
    }
}

// Resident one-wave work-groups per CU for the kernel of T rows per lane.
static int sym_waves_per_cu(int T) {
    int nblk = 0;
    hipError_t e = T == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &nblk, (const void*)k_sym_f32<IMG_PERIODIC, 2, false>, SW, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                &nblk, (const void*)k_sym_f32<IMG_PERIODIC, 1, false>, SW, 0);
    return (e == hipSuccess && nblk > 0) ? nblk : 8;
}

SymGeom sym_geometry(int n, int T, int ncu) {
    SymGeom g;
    g.n = n;
    g.T = T;
    // about 128 rounds (blocks of n / 128), at most 64 row slices
    const long rows = (long)SW * T;
    long s = (n + rows * 128 - 1) / (rows * 128);
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    // keep the accumulators (C + s copies of 32 bytes per particle) under 8 GB
    while (s > 1 && (s + 1) * 32.0 * (double)n > 8e9) --s;
    g.s = (int)s;
    g.B = (int)(rows * s);
    g.nb = (n + g.B - 1) / g.B;
    g.P = g.nb + (g.nb & 1);
    g.n_pad = g.nb * g.B;
    // column parts: as many as keep one round within the resident waves,
    // at least 64 columns each
    const long cap = (long)sym_waves_per_cu(T) * ncu;
    const long w1 = (long)(g.P / 2) * g.s;
    long C = cap / (w1 > 0 ? w1 : 1);
    const long cmax = g.B / 64;
    if (C > cmax) C = cmax;
    if (C < 1) C = 1;
    g.C = (int)C;
    return g;
}

template <int IMG, int T>
static hipError_t sym32(const Rec32* pts, const SymGeom& g, double invL, double* acc, hipStream_t s) {
    auto grid8 = [](long w) { return (unsigned)((w + 7) / 8 * 8); };
    hipLaunchKernelGGL((k_sym_f32<IMG, T, true>), dim3(grid8((long)g.nb * g.s * g.C)), dim3(SW), 0,
                       s, pts, g, -1, invL, acc);
    const unsigned grid = grid8((long)(g.P / 2) * g.s * g.C);
    for (int r = 0; r < g.P - 1; ++r)
        hipLaunchKernelGGL((k_sym_f32<IMG, T, false>), dim3(grid), dim3(SW), 0, s, pts, g, r, invL,
                           acc);
    return hipGetLastError();
}

hipError_t launch_sym_f32(int img, const Rec32* pts, const SymGeom& g, double L, double* acc,
                          hipStream_t s) {
    if (g.n <= 0 || g.nb <= 0) return hipErrorInvalidValue;
    const double invL = 1.0 / L;
    if (img == IMG_PERIODIC)
        return g.T == 2 ? sym32<IMG_PERIODIC, 2>(pts, g, invL, acc, s)
                        : sym32<IMG_PERIODIC, 1>(pts, g, invL, acc, s);
    if (img == IMG_METALLIC)
        return g.T == 2 ? sym32<IMG_METALLIC, 2>(pts, g, invL, acc, s)
                        : sym32<IMG_METALLIC, 1>(pts, g, invL, acc, s);
    return hipErrorInvalidValue;
}

}  // namespace hsma
