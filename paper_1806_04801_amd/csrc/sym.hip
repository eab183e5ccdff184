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
// For the slab (mirror-doubled periodic cube) the rows and columns are the
// real charges and each pair carries two image blocks: the periodic block of
// the charge and that of its mirror (x, y, -z) with the opposite charge.  The
// mirror block is symmetric too, with x and y periodic and z reflected, so
// its reverse field keeps the sign of the z component.
//
// Work layout.  Particles are cut into nb blocks of B = 64 * T * s.  The
// block pairs (I, J), I != J, are scheduled as a round-robin tournament: in
// each round every block takes part in exactly one pair, so no two
// work-groups of a round touch the same particle's accumulators and the
// rounds accumulate in place, in a fixed order, without atomics.  A pair is
// split into s row slices and C column parts; work-group (pair, slice,
// part) is one wave that keeps 64 * T rows of block I in registers (T per
// lane) and reads its part of the B columns of block J at wave-uniform
// addresses (vector loads: every lane fetches the same record, one cache line
// per load, no LDS staging).  Forward terms (at the rows) accumulate per lane
// as in the plain tile kernel and go to part c's copy of the row
// accumulators; reverse terms (at the columns) are summed over the wave's
// rows by a transpose through LDS and go to slice sigma's copy of the column
// accumulators.  The diagonal pairs (I, I) run first, forward only,
// with a particle's pairing with itself reduced to the images of its
// reflections (none in the periodic block, whose own images the finalize
// stage adds exactly); they also initialise every accumulator of their rows.
//
// Accumulators: acc[c] = forward from column part c (c < C), acc[C + sigma] =
// reverse from row slice sigma, each 4 components x n_pad doubles (potential,
// field x, y, z), physical units.  The finalize stage sums the C + s copies in
// that order.
//
// Two precisions: k_sym_f32 on Rec32 records (hi/lo coordinates in units of
// L) with 8-column plain partials folded by two-sum, k_sym_f64 on centred
// double4 records with plain FMA accumulation.
#include <algorithm>
#include <cstdlib>

#include "hsma_internal.h"
#include "pair_math.h"

namespace hsma {

constexpr int SW = 64;   // one wave per work-group

template <int CTRL>
__device__ __forceinline__ float dpp_t(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_t(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Orders the LDS accesses before and after it within the wave.  The
// work-group is one wave and a wave's LDS operations complete in issue order,
// so no hardware wait is needed: a wavefront-scope fence keeps the compiler
// from moving memory operations across.
__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Reverse-term table of one wave in LDS: NV rows (values) of 64 entries
// (lanes), each row padded by 16 bytes.
template <typename R, int NV>
struct RevTable {
    static constexpr int G = SW / NV;                         // lanes per value: 8 or 4
    static constexpr int STRIDE = SW + 16 / (int)sizeof(R);   // row stride in elements
    static constexpr int SIZE = NV * STRIDE;
};

// Sum of NV (8 or 16) values over the 64 lanes of the wave, as a transpose
// through LDS: lane l stores its values in column l of the table; then lane
// l adds the NV consecutive entries [NV (l % G), NV (l % G) + NV) of row
// v = l / G (G = 64 / NV lanes per value), and the G lanes of a value finish
// with DPP exchanges (lane ^ 1, ^ 2 and, for G = 8, the half-row mirror, which
// pairs the two quads).  Every lane of group v returns the total of value v.
// The LDS accesses take no vector-ALU issue slots: per value the ALU work is
// NV - 1 adds plus the exchanges.  Fixed order, so the result is
// deterministic.
template <typename R, int NV>
__device__ __forceinline__ R reduce_lds(const R (&v)[NV], int lane, R* __restrict__ tab) {
    using TT = RevTable<R, NV>;
    static_assert(NV == 8 || NV == 16, "8 or 16 values");
#pragma unroll
    for (int k = 0; k < NV; ++k) tab[k * TT::STRIDE + lane] = v[k];
    wave_order();   // the stores before the loads of other lanes
    const R* row = tab + (lane / TT::G) * TT::STRIDE + (lane % TT::G) * NV;
    R e = row[0];
#pragma unroll
    for (int i = 1; i < NV; ++i) e += row[i];
    wave_order();   // the next call's stores after these loads
    e += dpp_t<0xB1>(e);                     // quad_perm [1,0,3,2]: lane ^ 1
    e += dpp_t<0x4E>(e);                     // quad_perm [2,3,0,1]: lane ^ 2
    if (TT::G == 8) e += dpp_t<0x141>(e);    // row_half_mirror: the other quad
    return e;
}

// The work item of this work-group: row block I, column block J, row slice
// and column part.  Consecutive items (the slices and parts of one block
// pair, which read the same columns) go to the same XCD: the hardware deals
// work-groups round-robin over the 8 XCDs.
struct SymItem {
    int I, J, sig, part;
    bool ok;
};

// Work-group index in XCD order: the launch's grid is a multiple of 8 and
// consecutive indices land on one XCD.
__device__ __forceinline__ int xcd_order_id() {
    const int per_xcd = gridDim.x >> 3;
    return (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
}

template <bool DIAG>
__device__ __forceinline__ SymItem sym_item_of(const SymGeom& g, int round, int id) {
    SymItem it;
    const int per_pair = g.s * g.C;
    int pr;
    it.ok = false;
    if (DIAG) {
        if (id >= g.nb * per_pair) return it;
        it.I = it.J = pr = id / per_pair;
    } else {
        if (id >= (g.P >> 1) * per_pair) return it;
        pr = id / per_pair;
        const int m = g.P - 1;
        if (pr == 0) {
            it.I = m;
            it.J = round;
        } else {
            it.I = (round + pr) % m;
            it.J = (round - pr + m) % m;
        }
        if (it.I >= g.nb || it.J >= g.nb) return it;   // the bye of an odd block count
    }
    const int rem = id - pr * per_pair;
    it.sig = rem / g.C;
    it.part = rem - it.sig * g.C;
    it.ok = true;
    return it;
}

template <bool DIAG>
__device__ __forceinline__ SymItem sym_item(const SymGeom& g, int round) {
    return sym_item_of<DIAG>(g, round, xcd_order_id());
}

// Near terms of one pair per unit charges: potential p, field f at the row,
// and (REV) field rf at the column produced by the row.  OWN (diagonal
// blocks, the only ones where a particle meets itself): a zero central
// distance is skipped and the periodic images of a particle's own charge are
// left to the caller (images_sum).  In single precision both image blocks of the slab are
// shifted by the same constant (images_sum, SHIFT), which cancels in their
// difference.
template <int IMG, bool REV, bool OWN>
__device__ __forceinline__ void pair_terms(const Pt32& t, const Pt32& s, float& p, float (&f)[3],
                                           float (&rf)[3]) {
    constexpr int BI = IMG == IMG_SLAB ? IMG_PERIODIC : IMG;
    float dx[3], dy[3], dz[3];
    diffs_f32<BI>(t, s, 0, dx);
    diffs_f32<BI>(t, s, 1, dy);
    diffs_f32<BI>(t, s, 2, dz);
    images_sum<float, BI, true, OWN, REV, OWN, true>(dx, dy, dz, p, f[0], f[1], f[2], rf);
    if (IMG == IMG_SLAB) {
        // mirror block: z differences t + s - kL (k = -1, 0, +1), charge -1
        const float sl = t.l[2] + s.l[2];
        const float mz[3] = {(t.hm[2] + s.hm[2]) + sl, (t.h0[2] + s.h0[2]) + sl,
                             (t.hp[2] + s.hp[2]) + sl};
        float pm, gx, gy, gz;
        images_sum<float, IMG_PERIODIC, true, false, false, false, true>(dx, dy, mz, pm, gx, gy, gz);
        p -= pm;
        f[0] -= gx;
        f[1] -= gy;
        f[2] -= gz;
        if (REV) {
            rf[0] += gx;
            rf[1] += gy;
            rf[2] -= gz;
        }
    }
}

template <int IMG, bool REV, bool OWN>
__device__ __forceinline__ void pair_terms(const double4& t, const double4& s, double L, double& p,
                                           double (&f)[3], double (&rf)[3]) {
    constexpr int BI = IMG == IMG_SLAB ? IMG_PERIODIC : IMG;
    double dx[3], dy[3], dz[3];
    diffs_f64<BI>(t.x, s.x, L, dx);
    diffs_f64<BI>(t.y, s.y, L, dy);
    diffs_f64<BI>(t.z, s.z, L, dz);
    images_sum<double, BI, true, OWN, REV, OWN>(dx, dy, dz, p, f[0], f[1], f[2], rf);
    if (IMG == IMG_SLAB) {
        const double sm = t.z + s.z;
        const double mz[3] = {sm + L, sm, sm - L};
        double pm, gx, gy, gz;
        images_sum<double, IMG_PERIODIC, true, false>(dx, dy, mz, pm, gx, gy, gz);
        p -= pm;
        f[0] -= gx;
        f[1] -= gy;
        f[2] -= gz;
        if (REV) {
            rf[0] += gx;
            rf[1] += gy;
            rf[2] -= gz;
        }
    }
}

// The grounded-cube and slab kernels with one row per lane are held to 7
// resident waves per SIMD (72 VGPRs instead of 95, with a small spill that is
// reloaded about once per 550 instructions): 1-2.5 % faster by measurement.
// The periodic kernel runs best at its own 76 VGPRs and 6 waves.
template <int IMG, int T, bool DIAG, int QC>
__device__ __forceinline__ void sym_f32_body(const Rec32* __restrict__ pts, const SymGeom& g,
                                             const SymItem& it, double invL,
                                             double* __restrict__ acc, float* __restrict__ tab) {
    constexpr int NV = 4 * QC;   // reverse values per lane and group
    const int lane = threadIdx.x;
    const int I = it.I, J = it.J, sig = it.sig, part = it.part;
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
    // Columns are read with vector loads (every lane the same record, one
    // cache line per load): the index carries a zero that the compiler cannot
    // prove uniform, since scalar loads into SGPRs measured 8.6 % slower here
    // (they share the wait counter of the LDS reduction).
    int vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    // reverse values: lane l owns value l / G of each group when l % G == 0
    constexpr int G = RevTable<float, NV>::G;
    const bool owner = lane % G == 0;
    const int kown = lane / G;
    const int kcol = kown >> 2, kcomp = kown & 3;
    const double oscale = kcomp == 0 ? invL : invL2;
    for (int g0 = c0; g0 < c1; g0 += 8) {
        float sp[T], sx[T], sy[T], sz[T];
#pragma unroll
        for (int u = 0; u < T; ++u) sp[u] = sx[u] = sy[u] = sz[u] = 0.0f;
#pragma unroll
        for (int h = 0; h < 8 / QC; ++h) {
            const int jb = g0 + QC * h;
            const int nh = min(QC, c1 - jb);
            if (nh <= 0) break;
            double old = 0.0;
            double* dst = nullptr;
            if (!DIAG && owner && kcol < nh) {
                dst = rev + (size_t)kcomp * g.n_pad + jb + kcol;
                old = *dst;
            }
            float rv[NV];
#pragma unroll
            for (int q = 0; q < QC; ++q) {
                float rp = 0.0f, rx = 0.0f, ry = 0.0f, rz = 0.0f;
                if (q < nh) {
                    const Rec32 rec = pts[jb + q + vzero];
                    const Pt32 sj = load_pt32(rec);
                    const float qj = rec.v[0].w;
#pragma unroll
                    for (int u = 0; u < T; ++u) {
                        float p0, f0[3], rf[3];
                        pair_terms<IMG, !DIAG, DIAG>(tp[u], sj, p0, f0, rf);
                        sp[u] = __builtin_fmaf(qj, p0, sp[u]);
                        sx[u] = __builtin_fmaf(qj, f0[0], sx[u]);
                        sy[u] = __builtin_fmaf(qj, f0[1], sy[u]);
                        sz[u] = __builtin_fmaf(qj, f0[2], sz[u]);
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
                const float e = reduce_lds(rv, lane, tab);
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

template <int IMG, int T, bool DIAG, int QC>
__global__ void __launch_bounds__(SW, (IMG != IMG_PERIODIC && T == 1) ? 7 : 1)
k_sym_f32(const Rec32* __restrict__ pts, SymGeom g, int round, double invL, double* __restrict__ acc) {
    __shared__ float tab[RevTable<float, 4 * QC>::SIZE];
    const SymItem it = sym_item<DIAG>(g, round);
    if (!it.ok) return;
    sym_f32_body<IMG, T, DIAG, QC>(pts, g, it, invL, acc, tab);
}

// Double precision: one row per lane, positions in physical units (centred
// double4 x, y, z, q), plain FMA accumulation as in the double tile kernel;
// reverse terms are reduced in double.
template <int IMG, bool DIAG, int QC>
__device__ __forceinline__ void sym_f64_body(const double4* __restrict__ pts, const SymGeom& g,
                                             const SymItem& it, double L,
                                             double* __restrict__ acc, double* __restrict__ tab) {
    constexpr int NV = 4 * QC;   // reverse values per lane and group
    const int lane = threadIdx.x;
    const size_t cs = (size_t)4 * g.n_pad;
    double* __restrict__ fwd = acc + (size_t)it.part * cs;
    double* __restrict__ rev = acc + (size_t)(g.C + it.sig) * cs;

    // the row; a lane past the end carries no charge and sits far outside
    // every image of the box
    const int i = it.I * g.B + it.sig * SW + lane;
    double4 t = pts[min(i, g.n - 1)];
    double qi = t.w;
    if (i >= g.n) {
        qi = 0.0;
        t.x = t.y = t.z = 1000.0 * L;
    }
    double ap = 0.0, ax = 0.0, ay = 0.0, az = 0.0;

    const int c0 = min(it.J * g.B + (int)((long)it.part * g.B / g.C), g.n);
    const int c1 = min(it.J * g.B + (int)((long)(it.part + 1) * g.B / g.C), g.n);
    constexpr int G = RevTable<double, NV>::G;
    const bool owner = lane % G == 0;
    const int kown = lane / G;
    const int kcol = kown >> 2, kcomp = kown & 3;
    for (int jb = c0; jb < c1; jb += QC) {
        const int nh = min(QC, c1 - jb);
        double old = 0.0;
        double* dst = nullptr;
        if (!DIAG && owner && kcol < nh) {
            dst = rev + (size_t)kcomp * g.n_pad + jb + kcol;
            old = *dst;
        }
        double rv[NV];
#pragma unroll
        for (int q = 0; q < QC; ++q) {
            double rp = 0.0, rx = 0.0, ry = 0.0, rz = 0.0;
            if (q < nh) {
                const double4 sj = pts[jb + q];
                double p0, f0[3], rf[3];
                pair_terms<IMG, !DIAG, DIAG>(t, sj, L, p0, f0, rf);
                ap = __builtin_fma(sj.w, p0, ap);
                ax = __builtin_fma(sj.w, f0[0], ax);
                ay = __builtin_fma(sj.w, f0[1], ay);
                az = __builtin_fma(sj.w, f0[2], az);
                if (!DIAG) {
                    rp = qi * p0;
                    rx = qi * rf[0];
                    ry = qi * rf[1];
                    rz = qi * rf[2];
                }
            }
            rv[4 * q + 0] = rp;
            rv[4 * q + 1] = rx;
            rv[4 * q + 2] = ry;
            rv[4 * q + 3] = rz;
        }
        if (!DIAG) {
            const double e = reduce_lds(rv, lane, tab);
            if (dst != nullptr) *dst = old + e;
        }
    }

    if (i < g.n) {
        const double v[4] = {ap, ax, ay, az};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double* f = fwd + (size_t)c * g.n_pad + i;
            *f = DIAG ? v[c] : *f + v[c];
        }
        if (DIAG && it.part == 0) {
            for (int r = 0; r < g.s; ++r) {
                double* z = acc + (size_t)(g.C + r) * cs + i;
#pragma unroll
                for (int c = 0; c < 4; ++c) z[(size_t)c * g.n_pad] = 0.0;
            }
        }
    }
}

template <int IMG, bool DIAG, int QC>
__global__ void __launch_bounds__(SW)
k_sym_f64(const double4* __restrict__ pts, SymGeom g, int round, double L, double* __restrict__ acc) {
    __shared__ double tab[RevTable<double, 4 * QC>::SIZE];
    const SymItem it = sym_item<DIAG>(g, round);
    if (!it.ok) return;
    sym_f64_body<IMG, DIAG, QC>(pts, g, it, L, acc, tab);
}

// Resident one-wave work-groups per CU of the round kernel of an image kind
// (T = 0: double precision).
// Columns per reverse group (LDS reduction of 4 x QC values): 2 in single
// precision (fewer registers, more resident waves), 4 in double (measured);
// HSMA_SYM_Q = 2 or 4 overrides.
static int sym_q(bool f64) {
    const char* v = getenv("HSMA_SYM_Q");
    if (v != nullptr && (atoi(v) == 2 || atoi(v) == 4)) return atoi(v);
    return f64 ? 4 : 2;
}

template <int IMG, int QC>
static const void* sym_round_kernel_q(int T) {
    return T == 0   ? (const void*)k_sym_f64<IMG, false, QC>
           : T == 2 ? (const void*)k_sym_f32<IMG, 2, false, QC>
                    : (const void*)k_sym_f32<IMG, 1, false, QC>;
}

template <int IMG>
static const void* sym_round_kernel(int T) {
    return sym_q(T == 0) == 2 ? sym_round_kernel_q<IMG, 2>(T) : sym_round_kernel_q<IMG, 4>(T);
}

static int sym_waves_per_cu(int T, int img) {
    int nblk = 0;
    const void* k = img == IMG_SLAB       ? sym_round_kernel<IMG_SLAB>(T)
                    : img == IMG_METALLIC ? sym_round_kernel<IMG_METALLIC>(T)
                                          : sym_round_kernel<IMG_PERIODIC>(T);
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, k, SW, 0);
    return (e == hipSuccess && nblk > 0) ? nblk : 8;
}

// Target number of rounds: n / 1024 within [2, 128] (measured best from 3e3
// to 1.3e5 particles in both precisions, with up to 64 column parts: fewer,
// larger rounds while a round cannot fill the GPU anyway, and fewer
// launches); HSMA_SYM_ROUNDS overrides.
static long sym_rounds(int n) {
    const char* v = getenv("HSMA_SYM_ROUNDS");
    const long r = v != nullptr ? atol(v) : 0;
    if (r >= 2) return r;
    return std::min(128L, std::max(2L, (long)n / 1024));
}

// Geometry for T rows per lane; *fill is the fraction of resident-wave slots
// that a round's waves occupy over its batches.
static SymGeom sym_geometry_t(int n, int T, bool f64, int img, int ncu, double* fill) {
    SymGeom g;
    g.n = n;
    g.T = T;
    // about R rounds (blocks of n / R), at most 64 row slices
    const long rows = (long)SW * T;
    const long R = sym_rounds(n);
    long s = (n + rows * R - 1) / (rows * R);
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    // keep the accumulators (C + s copies of 32 bytes per particle) under 8 GB
    while (s > 1 && (s + 17) * 32.0 * (double)n > 8e9) --s;
    // an odd block count leaves one block idle in every round (a bye), which
    // costs 1 / nb of each round: larger blocks make the count even
    auto blocks = [&](long sl) { return (n + rows * sl - 1) / (rows * sl); };
    long s2 = s;
    while (blocks(s2) > 1 && (blocks(s2) & 1) && s2 < 64 && (s2 + 18) * 32.0 * (double)n <= 8e9) ++s2;
    if (blocks(s2) == 1 || !(blocks(s2) & 1)) s = s2;
    g.s = (int)s;
    g.B = (int)(rows * s);
    g.nb = (n + g.B - 1) / g.B;
    g.P = g.nb + (g.nb & 1);
    g.n_pad = g.nb * g.B;
    // Column parts: a round's waves all take equally long, so they run in
    // batches of `cap` resident waves and the last batch may be part empty.
    // Pick the part count (at most 64, at least 16 columns per part) whose
    // waves fill their batches best; a larger count wins only by more than 2 %.
    // Small rounds (N up to ~3e4) need many narrow parts to fill the GPU.
    const long cap = (long)sym_waves_per_cu(f64 ? 0 : T, img) * ncu;
    const long w1 = (long)(g.P / 2) * g.s;
    long cmax = g.B / 16;
    if (cmax < 1) cmax = 1;
    if (cmax > 64) cmax = 64;
    long best = 1;
    double best_fill = 0.0;
    for (long C = 1; C <= cmax; ++C) {
        const long w = w1 * C;
        const long batches = (w + cap - 1) / cap;
        const double f = (double)w / (double)(batches * cap);
        if (f > best_fill + 0.02) {
            best_fill = f;
            best = C;
        }
    }
    g.C = (int)best;
    *fill = best_fill;
    return g;
}

SymGeom sym_geometry(int n, int T, bool f64, int img, int ncu) {
    double f1 = 0.0, f2 = 0.0;
    if (f64) return sym_geometry_t(n, 1, true, img, ncu, &f1);
    if (T == 1 || T == 2) return sym_geometry_t(n, T, false, img, ncu, &f1);
    // T = 0: one row per lane (more resident waves) unless two fill the slots
    // better
    const SymGeom g1 = sym_geometry_t(n, 1, false, img, ncu, &f1);
    const SymGeom g2 = sym_geometry_t(n, 2, false, img, ncu, &f2);
    return f2 > f1 + 0.02 ? g2 : g1;
}

template <int IMG, int T, int QC>
static hipError_t sym32(const Rec32* pts, const SymGeom& g, double invL, double* acc, hipStream_t s) {
    auto grid8 = [](long w) { return (unsigned)((w + 7) / 8 * 8); };
    hipLaunchKernelGGL((k_sym_f32<IMG, T, true, QC>), dim3(grid8((long)g.nb * g.s * g.C)), dim3(SW),
                       0, s, pts, g, -1, invL, acc);
    const unsigned grid = grid8((long)(g.P / 2) * g.s * g.C);
    for (int r = 0; r < g.P - 1; ++r)
        hipLaunchKernelGGL((k_sym_f32<IMG, T, false, QC>), dim3(grid), dim3(SW), 0, s, pts, g, r,
                           invL, acc);
    return hipGetLastError();
}

template <int IMG>
static hipError_t sym32_t(const Rec32* pts, const SymGeom& g, double invL, double* acc,
                          hipStream_t s) {
    if (sym_q(false) == 2)
        return g.T == 2 ? sym32<IMG, 2, 2>(pts, g, invL, acc, s) : sym32<IMG, 1, 2>(pts, g, invL, acc, s);
    return g.T == 2 ? sym32<IMG, 2, 4>(pts, g, invL, acc, s) : sym32<IMG, 1, 4>(pts, g, invL, acc, s);
}

hipError_t launch_sym_f32(int img, const Rec32* pts, const SymGeom& g, double L, double* acc,
                          hipStream_t s) {
    if (g.n <= 0 || g.nb <= 0) return hipErrorInvalidValue;
    const double invL = 1.0 / L;
    if (img == IMG_PERIODIC) return sym32_t<IMG_PERIODIC>(pts, g, invL, acc, s);
    if (img == IMG_METALLIC) return sym32_t<IMG_METALLIC>(pts, g, invL, acc, s);
    if (img == IMG_SLAB) return sym32_t<IMG_SLAB>(pts, g, invL, acc, s);
    return hipErrorInvalidValue;
}

template <int IMG, int QC>
static hipError_t sym64(const double4* pts, const SymGeom& g, double L, double* acc, hipStream_t s) {
    auto grid8 = [](long w) { return (unsigned)((w + 7) / 8 * 8); };
    hipLaunchKernelGGL((k_sym_f64<IMG, true, QC>), dim3(grid8((long)g.nb * g.s * g.C)), dim3(SW), 0,
                       s, pts, g, -1, L, acc);
    const unsigned grid = grid8((long)(g.P / 2) * g.s * g.C);
    for (int r = 0; r < g.P - 1; ++r)
        hipLaunchKernelGGL((k_sym_f64<IMG, false, QC>), dim3(grid), dim3(SW), 0, s, pts, g, r, L, acc);
    return hipGetLastError();
}

template <int IMG>
static hipError_t sym64_t(const double4* pts, const SymGeom& g, double L, double* acc, hipStream_t s) {
    return sym_q(true) == 2 ? sym64<IMG, 2>(pts, g, L, acc, s) : sym64<IMG, 4>(pts, g, L, acc, s);
}

hipError_t launch_sym_f64(int img, const double4* pts, const SymGeom& g, double L, double* acc,
                          hipStream_t s) {
    if (g.n <= 0 || g.nb <= 0 || g.T != 1) return hipErrorInvalidValue;
    if (img == IMG_PERIODIC) return sym64_t<IMG_PERIODIC>(pts, g, L, acc, s);
    if (img == IMG_METALLIC) return sym64_t<IMG_METALLIC>(pts, g, L, acc, s);
    if (img == IMG_SLAB) return sym64_t<IMG_SLAB>(pts, g, L, acc, s);
    return hipErrorInvalidValue;
}

}  // namespace hsma
