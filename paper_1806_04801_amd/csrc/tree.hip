// Near-field sum over the 3x3x3 image block by the fast multipole method (the
// O(N) acceleration of the near sum that Sec. II.C and Table I leave to the
// FMM): the same quantity as the direct near kernels, phi_i and E_i from
// every image of every source in the block except the bare self term, to a
// tolerance set by the expansion order.
//
// Sources are the explicit images (27 per source: periodic r + kL, grounded
// (-1)^k o r + kL with charge (-1)^|k| q; the slab's doubled cube like the
// periodic one).  They lie in the cube [-3L/2, 3L/2)^3, which is cut into the
// 27 boxes of the block and each box into a uniform octree: level l has
// 2^l cells per box side (cell side L / 2^l), 3 * 2^l over the cube.  Images
// are sorted by leaf cell (box index, then the Morton code of the cell in its
// box), so that every cell at every level is a contiguous range.
//
// Expansions about cell centres in complex solid harmonics,
//   R_n^m(r) = r^n P_n^m(cos t) e^{i m phi} / (n + m)!,
//   I_n^m(r) = (n - m)! P_n^m(cos t) e^{i m phi} / r^{n + 1}       (m >= 0),
// with 1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x) for |y| < |x| (negative m
// by complex conjugation), built by their Cartesian recurrences:
//   R_m^m = (x + iy) / (2m) R_{m-1}^{m-1},
//   (n^2 - m^2) R_n^m = (2n - 1) z R_{n-1}^m - r^2 R_{n-2}^m,
//   I_m^m = (2m - 1) (x + iy) / r^2 I_{m-1}^{m-1},
//   r^2 I_n^m = (2n - 1) z I_{n-1}^m - ((n - 1)^2 - m^2) I_{n-2}^m.
// In the signed convention X~_n^m = X_n^m for m >= 0 and (-1)^m X_n^m for
// m < 0 the translation theorems are plain convolutions:
//   R~_n^m(a + b) = sum_{j,k} R~_j^k(a) R~_{n-j}^{m-k}(b),
//   I~_n^m(D + d) = sum_{j,k} (-1)^{j+k} R~_j^k(d) I~_{n+j}^{m-k}(D)  (|d| < |D|),
// the second from the Taylor series of a harmonic function with
// d/dz I~_n^m = -I~_{n+1}^m, (d/dx + i d/dy) I~_n^m = -I~_{n+1}^{m+1} and
// (d/dx - i d/dy) I~_n^m = I~_{n+1}^{m-1}.
// Upward pass: leaf multipoles M_n^m = sum_j q_j conj(R_n^m(y_j - c)), coarser
// ones by translation to the parent centre.  Downward pass, for the cells of
// the central box only (they hold the targets): local expansions from the
// multipoles of the interaction list (children of the parent's neighbours that
// are not the cell's own neighbours, up to 189 per level) plus the parent's
// local expansion shifted to the cell.  Targets evaluate their leaf cell's
// local expansion and the sources of the 27 neighbouring leaf cells directly.
// Every sum runs in a fixed order: results are bitwise reproducible.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "hsma_internal.h"
#include "pair_math.h"
#include "tree.h"

namespace hsma {

constexpr int TWG = 64;   // one wave per work-group

__host__ __device__ __forceinline__ int tri(int n, int m) { return n * (n + 1) / 2 + m; }

struct MomPtrs {
    const double2* lev[TREE_MAX_LEVEL + 1];   // multipoles of each level 0..L
};

// Interleaved bits of (ix, iy, iz), 3 x 7 bits.
__device__ __forceinline__ uint32_t morton3(uint32_t ix, uint32_t iy, uint32_t iz) {
    uint32_t k = 0;
#pragma unroll
    for (int b = 0; b < 7; ++b)
        k |= (((ix >> b) & 1u) << (3 * b + 2)) | (((iy >> b) & 1u) << (3 * b + 1)) | (((iz >> b) & 1u) << (3 * b));
    return k;
}

// Leaf-cell key of a point of the image cube at leaf level L.
__device__ __forceinline__ uint32_t leaf_key(double x, double y, double z, double L, int lev) {
    const int G = 3 << lev;
    const double inv_h = (double)(1 << lev) / L;
    int g[3];
    const double v[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int t = (int)floor((v[a] + 1.5 * L) * inv_h);
        g[a] = t < 0 ? 0 : (t >= G ? G - 1 : t);
    }
    const uint32_t box = (uint32_t)((g[0] >> lev) * 9 + (g[1] >> lev) * 3 + (g[2] >> lev));
    const uint32_t mask = (1u << lev) - 1u;
    return (box << (3 * lev)) | morton3((uint32_t)g[0] & mask, (uint32_t)g[1] & mask, (uint32_t)g[2] & mask);
}

// Key of the cell at global grid coordinates (gx, gy, gz) of level l.
__host__ __device__ __forceinline__ uint32_t cell_key(int gx, int gy, int gz, int l) {
    const uint32_t box = (uint32_t)((gx >> l) * 9 + (gy >> l) * 3 + (gz >> l));
    const uint32_t mask = (1u << l) - 1u;
    uint32_t ix = (uint32_t)gx & mask, iy = (uint32_t)gy & mask, iz = (uint32_t)gz & mask, k = 0;
    for (int b = 0; b < 7; ++b)
        k |= (((ix >> b) & 1u) << (3 * b + 2)) | (((iy >> b) & 1u) << (3 * b + 1)) | (((iz >> b) & 1u) << (3 * b));
    return (box << (3 * l)) | k;
}

// ---------------------------------------------------------------- images
// Image k (index kk = (kx+1)*9 + (ky+1)*3 + (kz+1)) of source j goes to slot
// kk * ns + j, with its leaf key; owner[slot] = j for the central image
// (kk = 13) and -1 otherwise (the bare self term is the central image of the
// target itself).
__global__ void k_tree_images(const double4* __restrict__ src, int ns, int img, double gamma, double L,
                              int lev, double4* __restrict__ out, uint32_t* __restrict__ keys,
                              int* __restrict__ vals) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int kk = blockIdx.y;
    if (j >= ns) return;
    const int kx = kk / 9 - 1, ky = (kk / 3) % 3 - 1, kz = kk % 3 - 1;
    const double4 r = src[j];
    double px = r.x, py = r.y, pz = r.z, q = r.w;
    if (img == IMG_METALLIC || img == IMG_DIELECTRIC) {
        // reflections; each weighs -1 (grounded) or gamma (dielectric, Eq. (diel))
        const double w = img == IMG_METALLIC ? -1.0 : gamma;
        if (kx) { px = -px; q *= w; }
        if (ky) { py = -py; q *= w; }
        if (kz) { pz = -pz; q *= w; }
    }
    px += kx * L;
    py += ky * L;
    pz += kz * L;
    const size_t slot = (size_t)kk * ns + j;
    out[slot] = make_double4(px, py, pz, q);
    keys[slot] = leaf_key(px, py, pz, L, lev);
    vals[slot] = (int)slot;
}

// Sorted images and their owners (the target index of a central image).
__global__ void k_tree_gather(const double4* __restrict__ img, const int* __restrict__ order,
                              int64_t n, int ns, double4* __restrict__ sorted, int* __restrict__ owner) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = order[i];
    sorted[i] = img[s];
    owner[i] = (s / ns == 13) ? s % ns : -1;
}

// offs[c] = the first sorted position whose key is >= c, c = 0..ncell (the
// sorted keys do not decrease): leaf cell c holds positions [offs[c], offs[c+1]).
__global__ void k_tree_offsets(const uint32_t* __restrict__ keys, int64_t n, int64_t ncell,
                               int* __restrict__ offs) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncell) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)keys[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    offs[c] = (int)lo;
}

// ---------------------------------------------------------------- leaf moments
// For few leaf cells: one wave per leaf cell, a lane per image (the cell's
// images in turns of 64): for each column m in turn every lane accumulates q
// conj(R_n^m) of its images, n = m..p, then the lanes' sums are combined by a
// fixed butterfly. The loops over n are unrolled to the largest order (guards
// uniform), so the accumulators stay in registers; the recurrence's
// reciprocals depend on (n, m) only.  The lanes read consecutive images, and a
// cell's images are re-read from cache for every m.
__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(64)
k_tree_p2m_wave(const double4* __restrict__ srt, const int* __restrict__ offs, int lev, int p, double L,
                double2* __restrict__ mom) {
    const int64_t cell = blockIdx.x;
    const int lane = threadIdx.x;
    const int b = offs[cell], e = offs[cell + 1];
    double2* out = mom + (size_t)cell * tri(p + 1, 0);
    if (b == e) {
        for (int idx = lane; idx < tri(p + 1, 0); idx += 64) out[idx] = make_double2(0.0, 0.0);
        return;
    }
    // cell centre from its key: box index and Morton code within the box
    const uint32_t key = (uint32_t)cell;
    const uint32_t box = key >> (3 * lev), mc = key & ((1u << (3 * lev)) - 1u);
    uint32_t ix = 0, iy = 0, iz = 0;
    for (int bb = 0; bb < lev; ++bb) {
        ix |= ((mc >> (3 * bb + 2)) & 1u) << bb;
        iy |= ((mc >> (3 * bb + 1)) & 1u) << bb;
        iz |= ((mc >> (3 * bb)) & 1u) << bb;
    }
    const double h = L / (double)(1 << lev);
    const double cx = -1.5 * L + ((double)((box / 9) * (1u << lev) + ix) + 0.5) * h;
    const double cy = -1.5 * L + ((double)(((box / 3) % 3) * (1u << lev) + iy) + 0.5) * h;
    const double cz = -1.5 * L + ((double)((box % 3) * (1u << lev) + iz) + 0.5) * h;
    constexpr int P = TREE_MAX_ORDER;
    for (int m = 0; m <= p; ++m) {
        double ar[P + 1], ai[P + 1], rinv[P + 1];
#pragma unroll
        for (int n = 0; n <= P; ++n) {
            ar[n] = ai[n] = 0.0;
            rinv[n] = (n > m) ? 1.0 / ((double)(n + m) * (double)(n - m)) : 0.0;
        }
        for (int s = b + lane; s < e; s += 64) {
            const double4 y = srt[s];
            const double x = y.x - cx, yy = y.y - cy, z = y.z - cz;
            const double r2 = x * x + yy * yy + z * z;
            // R_m^m = (x + iy)^m / (2^m m!)
            double dr = 1.0, di = 0.0;
#pragma unroll
            for (int k = 1; k <= P; ++k) {
                if (k <= m) {
                    const double c = 0.5 / (double)k;
                    const double nr = (dr * x - di * yy) * c;
                    const double ni = (dr * yy + di * x) * c;
                    dr = nr;
                    di = ni;
                }
            }
            double pr = 0.0, pi = 0.0, cr = dr, ci = di;   // R_{n-2}, R_{n-1}
#pragma unroll
            for (int n = 0; n <= P; ++n) {
                if (n < m || n > p) continue;
                if (n > m) {
                    const double nr = ((2 * n - 1) * z * cr - r2 * pr) * rinv[n];
                    const double ni = ((2 * n - 1) * z * ci - r2 * pi) * rinv[n];
                    pr = cr; pi = ci; cr = nr; ci = ni;
                }
                // M += q conj(R)
                ar[n] = __builtin_fma(y.w, cr, ar[n]);
                ai[n] = __builtin_fma(-y.w, ci, ai[n]);
            }
        }
#pragma unroll
        for (int n = 0; n <= P; ++n) {
            if (n < m || n > p) continue;
            const double vr = wave_sum64(ar[n]);
            const double vi = wave_sum64(ai[n]);
            if (lane == 0) out[tri(n, m)] = make_double2(vr, vi);
        }
    }
}

// For many leaf cells: thread (cell, m), m uniform over the wave: column m of
// the moments of leaf cell `cell`, summed over its sources in sorted order.
// The loops over n are unrolled to the largest order (guards n <= p are
// uniform), so the accumulators stay in registers; the recurrence's
// reciprocals depend on (n, m) only and are formed once per thread.  Work-
// groups go round the XCDs in turn; the p + 1 columns of a block of 64 cells
// are consecutive on one XCD, so that they read the cells' sources through
// one L2.
template <int P>   // largest order the registers hold (p <= P)
__global__ void __launch_bounds__(64)
k_tree_p2m_cols(const double4* __restrict__ srt, const int* __restrict__ offs, int lev, int ncell, int p,
                double L, double2* __restrict__ mom) {
    const int r = blockIdx.x >> 3;
    const int m = r % (p + 1);
    const int64_t cell = ((int64_t)(r / (p + 1)) * 8 + (blockIdx.x & 7)) * 64 + threadIdx.x;
    if (cell >= ncell || m > p) return;
    const int b = offs[cell], e = offs[cell + 1];
    double2* out = mom + (size_t)cell * tri(p + 1, 0);
    const int pm = p - m;   // orders n = m + i, i = 0..pm
    double ar[P + 1], ai[P + 1], rinv[P + 1];
    double dscale = 1.0;   // 1 / (2^m m!)
    for (int k = 1; k <= m; ++k) dscale *= 0.5 / (double)k;
#pragma unroll
    for (int i = 0; i <= P; ++i) {
        ar[i] = ai[i] = 0.0;
        rinv[i] = i > 0 ? 1.0 / ((double)(2 * m + i) * (double)i) : 0.0;   // 1 / ((n + m)(n - m))
    }
    if (b < e) {
        // cell centre from its key: box index and Morton code within the box
        const uint32_t key = (uint32_t)cell;
        const uint32_t box = key >> (3 * lev), mc = key & ((1u << (3 * lev)) - 1u);
        uint32_t ix = 0, iy = 0, iz = 0;
        for (int bb = 0; bb < lev; ++bb) {
            ix |= ((mc >> (3 * bb + 2)) & 1u) << bb;
            iy |= ((mc >> (3 * bb + 1)) & 1u) << bb;
            iz |= ((mc >> (3 * bb)) & 1u) << bb;
        }
        const double h = L / (double)(1 << lev);
        const double cx = -1.5 * L + ((double)((box / 9) * (1u << lev) + ix) + 0.5) * h;
        const double cy = -1.5 * L + ((double)(((box / 3) % 3) * (1u << lev) + iy) + 0.5) * h;
        const double cz = -1.5 * L + ((double)((box % 3) * (1u << lev) + iz) + 0.5) * h;
        // two sources a step (their recurrences interleave; each sum still
        // takes them in order), the next two read one step ahead
        double4 na = srt[b], nb = srt[min(b + 1, e - 1)];
        int s = b;
        for (; s + 1 < e; s += 2) {
            const double4 ya = na, yb = nb;
            na = srt[min(s + 2, e - 1)];
            nb = srt[min(s + 3, e - 1)];
            const double xa = ya.x - cx, ja = ya.y - cy, za = ya.z - cz;
            const double xb = yb.x - cx, jb = yb.y - cy, zb = yb.z - cz;
            const double r2a = xa * xa + ja * ja + za * za, r2b = xb * xb + jb * jb + zb * zb;
            // R_m^m = (x + iy)^m / (2^m m!)
            double wra = 1.0, wia = 0.0, wrb = 1.0, wib = 0.0;
            for (int k = 0; k < m; ++k) {
                const double nra = __builtin_fma(wra, xa, -wia * ja);
                const double nrb = __builtin_fma(wrb, xb, -wib * jb);
                wia = __builtin_fma(wra, ja, wia * xa);
                wib = __builtin_fma(wrb, jb, wib * xb);
                wra = nra;
                wrb = nrb;
            }
            double pra = 0.0, pia = 0.0, cra = wra * dscale, cia = wia * dscale;
            double prb = 0.0, pib = 0.0, crb = wrb * dscale, cib = wib * dscale;
            double zza = (double)(2 * m - 1) * za, zzb = (double)(2 * m - 1) * zb;
            const double z2a = 2.0 * za, z2b = 2.0 * zb;
#pragma unroll
            for (int i = 0; i <= P; ++i) {
                if (i > pm) continue;
                if (i > 0) {
                    zza += z2a;
                    zzb += z2b;
                    const double nra = __builtin_fma(zza, cra, -r2a * pra) * rinv[i];
                    const double nia = __builtin_fma(zza, cia, -r2a * pia) * rinv[i];
                    const double nrb = __builtin_fma(zzb, crb, -r2b * prb) * rinv[i];
                    const double nib = __builtin_fma(zzb, cib, -r2b * pib) * rinv[i];
                    pra = cra; pia = cia; cra = nra; cia = nia;
                    prb = crb; pib = cib; crb = nrb; cib = nib;
                }
                // M += q conj(R), source a then b
                ar[i] = __builtin_fma(yb.w, crb, __builtin_fma(ya.w, cra, ar[i]));
                ai[i] = __builtin_fma(-yb.w, cib, __builtin_fma(-ya.w, cia, ai[i]));
            }
        }
        if (s < e) {   // the last source of an odd count (na holds it)
            const double4 y = na;
            const double x = y.x - cx, yy = y.y - cy, z = y.z - cz;
            const double r2 = x * x + yy * yy + z * z;
            double wr = 1.0, wi = 0.0;
            for (int k = 0; k < m; ++k) {
                const double nr = __builtin_fma(wr, x, -wi * yy);
                wi = __builtin_fma(wr, yy, wi * x);
                wr = nr;
            }
            double pr = 0.0, pi = 0.0, cr = wr * dscale, ci = wi * dscale;   // R_{n-2}, R_{n-1}
            double zz = (double)(2 * m - 1) * z;   // (2n - 1) z, raised by 2z per order
            const double z2 = 2.0 * z;
#pragma unroll
            for (int i = 0; i <= P; ++i) {
                if (i > pm) continue;
                if (i > 0) {
                    zz += z2;
                    const double nr = __builtin_fma(zz, cr, -r2 * pr) * rinv[i];
                    const double ni = __builtin_fma(zz, ci, -r2 * pi) * rinv[i];
                    pr = cr; pi = ci; cr = nr; ci = ni;
                }
                ar[i] = __builtin_fma(y.w, cr, ar[i]);
                ai[i] = __builtin_fma(-y.w, ci, ai[i]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i <= P; ++i)
        if (i <= pm) out[tri(m + i, m)] = make_double2(ar[i], ai[i]);
}

// ---------------------------------------------------------------- translation
// For few parents: a work-group per parent cell of level l and per moment
// M_n^m (m >= 0) of the parent M2M_Q threads, each translating two of its 8
// children at level l + 1 (children with no source skipped), whose moments
// are staged in LDS in the full signed layout; the M2M_Q parts are added in
// order.  tab holds conj(R~_j^k(d_o)) of the 8 child offsets d_o (per axis
// +-1/4 of the parent's side, octant o = Morton digit) for the unit side,
// 8 x (p+1)^2 entries (index j*j + j + k), scaled here by side^j.
constexpr int M2M_Q = 4;
__global__ void __launch_bounds__(1024)
k_tree_m2m_group(const double2* __restrict__ child, const int* __restrict__ offs, int l, int L, int p,
                 double side, const double2* __restrict__ tab, double2* __restrict__ parent) {
    extern __shared__ double2 Ct[];   // 8 (p+1)^2; afterwards the M2M_Q x nc parts
    __shared__ int full[8];
    const int nc = tri(p + 1, 0);
    const int nf = (p + 1) * (p + 1);
    const int ncp = (nc + 63) / 64 * 64;   // threads per child pair
    const int64_t cell = blockIdx.x;
    const int t = threadIdx.x, nt = blockDim.x;
    const int shift = 3 * (L - l - 1);
    if (t < 8) {
        const int64_t c = cell * 8 + t;
        full[t] = offs[(c + 1) << shift] != offs[c << shift];
    }
    for (int idx = t; idx < 8 * nf; idx += nt) {
        const int o = idx / nf, r = idx - o * nf;
        int n = 0;
        while ((n + 1) * (n + 1) <= r) ++n;
        const int m = r - n * n - n;
        double2 v = child[(size_t)(cell * 8 + o) * nc + tri(n, m < 0 ? -m : m)];
        if (m < 0) {
            v.y = -v.y;
            if ((-m) & 1) { v.x = -v.x; v.y = -v.y; }
        }
        Ct[idx] = v;
    }
    __syncthreads();
    const int q = t / ncp, ti = t - q * ncp;
    double sr = 0.0, si = 0.0;
    if (ti < nc) {
        int n = 0;
        while (tri(n + 1, 0) <= ti) ++n;
        const int m = ti - tri(n, 0);
        for (int o = 2 * q; o < 2 * q + 2; ++o) {
            if (!full[o]) continue;
            const double2* M = Ct + (size_t)o * nf;
            const double2* T = tab + (size_t)o * nf;
            double sj = 1.0;
            for (int j = 0; j <= n; ++j) {
                const int nn = n - j;
                for (int k = -j; k <= j; ++k) {
                    const int mm = m - k;
                    if (mm > nn || -mm > nn) continue;
                    const double2 a = T[j * j + j + k];
                    const double2 bb = M[nn * nn + nn + mm];
                    const double ar = a.x * sj, ai = a.y * sj;
                    sr += ar * bb.x - ai * bb.y;
                    si += ar * bb.y + ai * bb.x;
                }
                sj *= side;
            }
        }
    }
    __syncthreads();   // the children's moments are read: their LDS takes the parts
    double2* partq = Ct;
    if (ti < nc) partq[q * nc + ti] = make_double2(sr, si);
    __syncthreads();
    if (q == 0 && ti < nc) {
        double2 v = partq[ti];
        for (int qq = 1; qq < M2M_Q; ++qq) {
            v.x += partq[qq * nc + ti].x;
            v.y += partq[qq * nc + ti].y;
        }
        parent[(size_t)cell * nc + ti] = v;
    }
}

// For many parents: thread (parent cell, n, m >= 0) of level l: the moment
// M_n^m of the parent from its 8 children at level l + 1 (children with no
// source skipped). tab holds conj(R~_j^k(d_o)) of the 8 child offsets d_o (per
// axis +-1/4 of the parent's side, octant o = Morton digit) for the unit side,
// 8 x (p+1)^2 entries (index j*j + j + k), scaled here by side^j.
__global__ void k_tree_m2m_coef(const double2* __restrict__ child, const int* __restrict__ offs, int l,
                                int L, int ncell, int p, double side, const double2* __restrict__ tab,
                                double2* __restrict__ parent) {
    const int nt = tri(p + 1, 0);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cell = t / nt;
    const int idx = (int)(t % nt);
    if (cell >= ncell) return;
    int n = 0;
    while (tri(n + 1, 0) <= idx) ++n;
    const int m = idx - tri(n, 0);
    double sr = 0.0, si = 0.0;
    const int shift = 3 * (L - l - 1);
    for (int o = 0; o < 8; ++o) {
        const int64_t c = cell * 8 + o;
        // the child's leaf range is empty: its moments are zero
        if (offs[(c + 1) << shift] == offs[c << shift]) continue;
        const double2* M = child + (size_t)c * nt;
        const double2* T = tab + (size_t)o * (p + 1) * (p + 1);
        double sj = 1.0;
        for (int j = 0; j <= n; ++j) {
            // the k with |m - k| <= n - j only
            const int nn = n - j;
            const int k0 = max(-j, m - nn), k1 = min(j, m + nn);
            double er = 0.0, ei = 0.0;
            for (int k = k0; k <= k1; ++k) {
                const int mm = m - k;
                const double2 a = T[j * j + j + k];
                // M~_nn^mm: stored for mm >= 0; (-1)^mm conj(M_nn^-mm) below
                const double2 v = M[tri(nn, mm < 0 ? -mm : mm)];
                const double sx = (mm < 0 && (mm & 1)) ? -1.0 : 1.0;
                const double bx = sx * v.x, by = (mm < 0 ? -sx : sx) * v.y;
                er += a.x * bx - a.y * by;
                ei += a.x * by + a.y * bx;
            }
            sr += sj * er;
            si += sj * ei;
            sj *= side;
        }
    }
    parent[(size_t)cell * nt + idx] = make_double2(sr, si);
}

// ---------------------------------------------------------------- downward pass
// Irregular harmonics I~_n^m(D) at the integer offsets D in [-3, 3]^3 (unit
// cell side; offset index (Dx+3)*49 + (Dy+3)*7 + (Dz+3)), orders n <= p2,
// full layout n*n + n + m for m in [-n, n] with I~_n^-m = (-1)^m conj(I_n^m).
// Offsets of neighbouring cells (|D_a| <= 1) are never used and left unset.
__global__ void k_fmm_itab(int p2, double2* __restrict__ tab) {
    // a thread per (offset, column m): I_m^m by the diagonal recurrence, then
    // up the column in n
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int o = id / (p2 + 1), m = id - o * (p2 + 1);
    if (o >= 343) return;
    const int dx = o / 49 - 3, dy = (o / 7) % 7 - 3, dz = o % 7 - 3;
    if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) return;
    const double x = dx, y = dy, z = dz;
    const double r2 = x * x + y * y + z * z, ir2 = 1.0 / r2;
    double2* T = tab + (size_t)o * (p2 + 1) * (p2 + 1);
    double dr = 1.0 / sqrt(r2), di = 0.0;   // I_0^0, then I_k^k up to k = m
    for (int k = 1; k <= m; ++k) {
        const double f = (2 * k - 1) * ir2;
        const double nr = f * (x * dr - y * di);
        const double ni = f * (x * di + y * dr);
        dr = nr;
        di = ni;
    }
    double pr = 0.0, pi = 0.0, cr = dr, ci = di;
    for (int n = m; n <= p2; ++n) {
        if (n > m) {
            const double c2 = (double)((n - 1) * (n - 1) - m * m);
            const double nr = ((2 * n - 1) * z * cr - c2 * pr) * ir2;
            const double ni = ((2 * n - 1) * z * ci - c2 * pi) * ir2;
            pr = cr; pi = ci; cr = nr; ci = ni;
        }
        T[n * n + n + m] = make_double2(cr, ci);
        if (m > 0) {
            const double sg = (m & 1) ? -1.0 : 1.0;
            T[n * n + n - m] = make_double2(sg * cr, -sg * ci);
        }
    }
}

constexpr int FWG = 256;   // threads of a downward-pass work-group (>= outputs (p+1)(p+2)/2)
static_assert(FWG >= 216, "the M2L checks its 216 candidates a thread each");
constexpr int NF = (TREE_MAX_ORDER + 1) * (TREE_MAX_ORDER + 1);
constexpr int NI = (2 * TREE_MAX_ORDER + 1) * (2 * TREE_MAX_ORDER + 1);

// Target cell of the central box at level l from its Morton index.
__device__ __forceinline__ void central_cell(int cid, int l, int& tx, int& ty, int& tz) {
    uint32_t ix = 0, iy = 0, iz = 0;
    for (int b = 0; b < l; ++b) {
        ix |= ((cid >> (3 * b + 2)) & 1u) << b;
        iy |= ((cid >> (3 * b + 1)) & 1u) << b;
        iz |= ((cid >> (3 * b)) & 1u) << b;
    }
    const int side = 1 << l;
    tx = side + (int)ix;
    ty = side + (int)iy;
    tz = side + (int)iz;
}

// Output (j, k) of thread t of a downward-pass work-group (t = tri(j, k)).
__device__ __forceinline__ void coef_of(int t, int& j, int& k) {
    j = 0;
    while (tri(j + 1, 0) <= t) ++j;
    k = t - tri(j, 0);
}

// Full signed table X~_n^m, m in [-n, n] (index n*n + n + m), of expansion
// coefficients stored for m >= 0 (row-packed by tri), times scale^n.
__device__ __forceinline__ void stage_signed(const double2* __restrict__ X, int p, const double* sc,
                                             double2* __restrict__ dst) {
    for (int idx = threadIdx.x; idx < (p + 1) * (p + 1); idx += FWG) {
        int n = 0;
        while ((n + 1) * (n + 1) <= idx) ++n;
        const int m = idx - n * n - n;
        double2 v = X[tri(n, m < 0 ? -m : m)];
        if (m < 0) {
            v.y = -v.y;
            if ((-m) & 1) { v.x = -v.x; v.y = -v.y; }
        }
        const double f = sc ? sc[n] : 1.0;
        dst[idx] = make_double2(v.x * f, v.y * f);
    }
}

// M2L of the cells of the central box at level l: work-group (cell, g), one
// thread per coefficient L_j^k (k >= 0), takes the entries g, g + G, g + 2G,
// ... of the cell's interaction list (children of the parent's neighbours
// that are not neighbours of the cell, non-empty, in a fixed order), D =
// c_T - c_S:
//   part_g L_j^k = (-1)^{j+k} sum_S sum_{n <= p, m} M~_n^m(S) I~_{n+j}^{m-k}(D).
// The source moments (scaled by h^-n) and the irregular harmonics of the
// offset (unit side; the remaining h^-(j+1) is applied at the end) are staged
// in LDS per source cell; the LDS is sized by the order (dynamic), so that
// low orders keep more work-groups resident to hide the staging.
__global__ void __launch_bounds__(FWG)
k_fmm_m2l(const double2* __restrict__ mom, const int* __restrict__ offs, int l, int L, int p,
          double Lbox, const double2* __restrict__ itab, int G, double2* __restrict__ part) {
    extern __shared__ double2 lds[];
    double2* Mt = lds;                              // (p+1)^2
    double2* It = lds + (p + 1) * (p + 1);          // (2p+1)^2
    double* hpow = (double*)(It + (2 * p + 1) * (2 * p + 1));
    const int t = threadIdx.x;
    const int nc = tri(p + 1, 0);
    const int p2 = 2 * p;
    const int ni = (p2 + 1) * (p2 + 1);
    const bool out = t < nc;
    int j = 0, k = 0;
    if (out) coef_of(t, j, k);
    const int cid = blockIdx.x, g = blockIdx.y;
    int tx, ty, tz;
    central_cell(cid, l, tx, ty, tz);
    const double h = Lbox / (double)(1 << l);
    if (t <= p) {
        double v = 1.0;
        for (int n = 0; n < t; ++n) v /= h;
        hpow[t] = v;   // h^-t
    }
    const int GG = 3 << l;
    const int shift = 3 * (L - l);
    const int px = tx >> 1, py = ty >> 1, pz = tz >> 1;
    // the 216 candidates (children of the parent's neighbours) checked at once,
    // a thread each: inside the cube, not a neighbour of the cell, not empty
    __shared__ unsigned char cand_ok[216];
    if (t < 216) {
        const int cx = 2 * px - 2 + t / 36, cy = 2 * py - 2 + (t / 6) % 6, cz = 2 * pz - 2 + t % 6;
        bool ok = cx >= 0 && cx < GG && cy >= 0 && cy < GG && cz >= 0 && cz < GG &&
                  !(abs(cx - tx) <= 1 && abs(cy - ty) <= 1 && abs(cz - tz) <= 1);
        if (ok) {
            const uint32_t ck = cell_key(cx, cy, cz, l);
            ok = offs[(size_t)(ck + 1) << shift] != offs[(size_t)ck << shift];
        }
        cand_ok[t] = ok ? 1 : 0;
    }
    __syncthreads();
    double br = 0.0, bi = 0.0;
    int item = 0;
    for (int cx = 2 * px - 2; cx <= 2 * px + 3; ++cx) {
        for (int cy = 2 * py - 2; cy <= 2 * py + 3; ++cy) {
            for (int cz = 2 * pz - 2; cz <= 2 * pz + 3; ++cz) {
                if (!cand_ok[(cx - 2 * px + 2) * 36 + (cy - 2 * py + 2) * 6 + (cz - 2 * pz + 2)]) continue;
                const uint32_t ck = cell_key(cx, cy, cz, l);
                if ((item++) % G != g) continue;
                stage_signed(mom + (size_t)ck * nc, p, hpow, Mt);
                const int o = (tx - cx + 3) * 49 + (ty - cy + 3) * 7 + (tz - cz + 3);
                const double2* I = itab + (size_t)o * ni;
                for (int idx = t; idx < ni; idx += FWG) It[idx] = I[idx];
                __syncthreads();
                if (out) {
                    for (int n = 0; n <= p; ++n) {
                        const int nn = n + j;
                        const double2* Irow = It + nn * nn + nn - k;
                        const double2* Mrow = Mt + n * n + n;
                        for (int m = -n; m <= n; ++m) {
                            const double2 a = Mrow[m];
                            const double2 c = Irow[m];
                            br += a.x * c.x - a.y * c.y;
                            bi += a.x * c.y + a.y * c.x;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    if (out) {
        double f = ((j + k) & 1) ? -1.0 : 1.0;
        f *= hpow[j] / h;   // h^-(j+1)
        part[((size_t)g * gridDim.x + cid) * nc + t] = make_double2(f * br, f * bi);
    }
}

// M2L of the finer levels, blocked over target cells.  Work-group (tile, g)
// takes M2L_NT cells of the central box that sit at the same corner of their
// parents, so that they share one list of interaction offsets D = c_T - c_S
// (per axis D in [b - 3, b + 2] for the cell's corner bit b, minus the 27
// neighbours: 189 offsets), and the offsets g, g + G, ... of that list; each
// of its waves takes M2L_C of the cells.  Per offset the work-group stages
// I~(D) h^-N in LDS (orders N <= 2p, zero up to 2p + R), and each lane of a
// wave accumulates R consecutive orders j of one k for the wave's cells:
//   part_g L_j^k = (-1)^{j+k} h^-1 sum_D sum_{n <= p, m} M~_n^m(T - D) (I~_{n+j}^{m-k}(D) h^-(n+j)),
// the same sum as (-1)^{j+k} h^-(j+1) sum (M~_n^m h^-n) I~_{n+j}^{m-k}(D) with
// the cell side's powers moved into the table.  The source moments are the
// same for every lane of a wave, so they are read through the scalar cache
// from the multipole array itself (an empty cell's moments are zero); only
// the I~ values come from LDS, R of them sliding by one order along n.  The
// loop over m is outermost.  For m < 0 the source term is s conj(M_n^|m|),
// s = (-1)^m; with y = (s Re I~, -s Im I~) the real part of I~ s conj(M) is
// that of y M and the imaginary part minus it, so the imaginary sums run
// negated through the columns m < 0 and one loop body serves every column.
constexpr int M2L_NT = 16;                  // target cells per work-group
constexpr int M2L_C = 4;                    // target cells per wave
constexpr int M2L_WAVES = M2L_NT / M2L_C;

// Orders j per lane: 3 while the (k, j0) groups fit one wave, else 5.
__host__ __device__ constexpr int m2l_rows(int p) { return p <= 17 ? 3 : 5; }
__host__ __device__ constexpr int m2l_groups(int p, int R) {
    int ng = 0;
    for (int k = 0; k <= p; ++k) ng += (p - k + R) / R;
    return ng;
}
static_assert(m2l_groups(17, 3) <= 64 && m2l_groups(TREE_MAX_ORDER, 5) <= 64, "a (k, j0) group per lane");

template <int R>
__device__ __forceinline__ void m2l_column(const double2* __restrict__ It, const double2* const (&ms)[M2L_C],
                                           int p, int m, int k, int j0, double (&ar)[R][M2L_C],
                                           double (&ai)[R][M2L_C]) {
    const int am = m < 0 ? -m : m;
    const int mu = m - k;
    const double sr = (m < 0 && (am & 1)) ? -1.0 : 1.0;
    const double si = m < 0 ? -sr : sr;
    double xr[R], xi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int N = am + j0 + r;
        const double2 v = It[N * N + N + mu];
        xr[r] = sr * v.x;
        xi[r] = si * v.y;
    }
#pragma unroll 4
    for (int n = am; n <= p; ++n) {
        const int cb = tri(n, am);
        double br[M2L_C], bi[M2L_C];
#pragma unroll
        for (int c = 0; c < M2L_C; ++c) {
            const double2 v = ms[c][cb];
            br[c] = v.x;
            bi[c] = v.y;
        }
        const int N = n + j0 + R;   // the next order's top value (padded table)
        const double2 top = It[N * N + N + mu];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int c = 0; c < M2L_C; ++c) {
                ar[r][c] = __builtin_fma(xr[r], br[c], __builtin_fma(-xi[r], bi[c], ar[r][c]));
                ai[r][c] = __builtin_fma(xi[r], br[c], __builtin_fma(xr[r], bi[c], ai[r][c]));
            }
#pragma unroll
        for (int r = 0; r + 1 < R; ++r) {
            xr[r] = xr[r + 1];
            xi[r] = xi[r + 1];
        }
        xr[R - 1] = sr * top.x;
        xi[R - 1] = si * top.y;
    }
}

template <int R>
__global__ void __launch_bounds__(64 * M2L_WAVES)
k_fmm_m2l_tile(const double2* __restrict__ mom, int l, int p, double Lbox, const double2* __restrict__ itab,
               int G, double2* __restrict__ part) {
    extern __shared__ double2 It[];   // (2p + R + 1)^2
    __shared__ int dlist[189];
    __shared__ double hpow[2 * TREE_MAX_ORDER + 6];
    const int nc = tri(p + 1, 0);
    const int ni = (2 * p + 1) * (2 * p + 1);
    const int nip = (2 * p + R + 1) * (2 * p + R + 1);
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int cls = blockIdx.x & 7, tile = blockIdx.x >> 3, g = blockIdx.y;
    const double h = Lbox / (double)(1 << l);
    const int bx = (cls >> 2) & 1, by = (cls >> 1) & 1, bz = cls & 1;
    if (t == 0) {
        int c = 0;
        for (int dx = bx - 3; dx <= bx + 2; ++dx)
            for (int dy = by - 3; dy <= by + 2; ++dy)
                for (int dz = bz - 3; dz <= bz + 2; ++dz) {
                    if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) continue;
                    dlist[c++] = (dx + 3) * 49 + (dy + 3) * 7 + (dz + 3);
                }
    }
    for (int N = t; N <= 2 * p + R; N += blockDim.x) {
        double v = 1.0;
        for (int i = 0; i < N; ++i) v /= h;
        hpow[N] = v;   // h^-N
    }
    // the wave's cells
    int tc[M2L_C][3];
#pragma unroll
    for (int c = 0; c < M2L_C; ++c)
        central_cell((tile * M2L_NT + wave * M2L_C + c) * 8 + cls, l, tc[c][0], tc[c][1], tc[c][2]);
    // this lane's (k, j0) group
    int k = 0, j0 = 0;
    bool act = false;
    {
        int c = 0;
        for (int kk = 0; kk <= p && !act; ++kk)
            for (int jj = kk; jj <= p; jj += R, ++c)
                if (c == lane) { k = kk; j0 = jj; act = true; break; }
    }
    double ar[R][M2L_C], ai[R][M2L_C];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < M2L_C; ++c) ar[r][c] = ai[r][c] = 0.0;
    for (int it = g; it < 189; it += G) {
        __syncthreads();   // the tables above, or the previous offset's reads, are done
        const int o = dlist[it];
        const int dx = o / 49 - 3, dy = (o / 7) % 7 - 3, dz = o % 7 - 3;
        const double2* I = itab + (size_t)o * ni;
        for (int idx = t; idx < nip; idx += blockDim.x) {
            int N = 0;
            while ((N + 1) * (N + 1) <= idx) ++N;
            double2 v = make_double2(0.0, 0.0);
            if (N <= 2 * p) {
                v = I[idx];
                v.x *= hpow[N];
                v.y *= hpow[N];
            }
            It[idx] = v;
        }
        __syncthreads();
        const double2* ms[M2L_C];
#pragma unroll
        for (int c = 0; c < M2L_C; ++c)
            ms[c] = mom + (size_t)cell_key(tc[c][0] - dx, tc[c][1] - dy, tc[c][2] - dz, l) * nc;
        if (act) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int c = 0; c < M2L_C; ++c) ai[r][c] = -ai[r][c];
            for (int m = -p; m <= p; ++m) {
                if (m == 0) {
#pragma unroll
                    for (int r = 0; r < R; ++r)
#pragma unroll
                        for (int c = 0; c < M2L_C; ++c) ai[r][c] = -ai[r][c];
                }
                m2l_column<R>(It, ms, p, m, k, j0, ar, ai);
            }
        }
    }
    if (act) {
        const int ncell = 1 << (3 * l);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = j0 + r;
            if (j > p) continue;
            const double f = (((j + k) & 1) ? -1.0 : 1.0) / h;
#pragma unroll
            for (int c = 0; c < M2L_C; ++c) {
                const int cid = (tile * M2L_NT + wave * M2L_C + c) * 8 + cls;
                part[((size_t)g * ncell + cid) * nc + tri(j, k)] = make_double2(f * ar[r][c], f * ai[r][c]);
            }
        }
    }
}

// Local expansions of the cells of the central box at level l: the G M2L
// parts in order, plus (l >= 2) the parent's expansion shifted to the cell,
//   L~_j^k += sum_{n >= j, m} L~_n^m(P) R~_{n-j}^{m-k}(c_T - c_P),
// with R~ from the child-offset table (conj(R~) at unit parent side).
__global__ void __launch_bounds__(FWG)
k_fmm_l2l(const double2* __restrict__ part, int G, int l, int p, double Lbox,
          const double2* __restrict__ m2m_tab, const double2* __restrict__ parent_loc,
          double2* __restrict__ loc) {
    __shared__ double2 Lt[NF];
    const int t = threadIdx.x;
    const int nc = tri(p + 1, 0);
    const int nf = (p + 1) * (p + 1);
    const bool out = t < nc;
    int j = 0, k = 0;
    if (out) coef_of(t, j, k);
    const int cid = blockIdx.x;
    double ar = 0.0, ai = 0.0;
    if (out)
        for (int g = 0; g < G; ++g) {
            const double2 v = part[((size_t)g * gridDim.x + cid) * nc + t];
            ar += v.x;
            ai += v.y;
        }
    if (l >= 2) {
        stage_signed(parent_loc + (size_t)(cid >> 3) * nc, p, nullptr, Lt);
        __syncthreads();
        if (out) {
            const double2* T = m2m_tab + (size_t)(cid & 7) * nf;
            const double sp = 2.0 * Lbox / (double)(1 << l);   // parent side
            double sd = 1.0;                                    // sp^(n - j)
            double cr = 0.0, ci = 0.0;
            for (int n = j; n <= p; ++n) {
                const int d = n - j;
                double er = 0.0, ei = 0.0;
                for (int m = -n; m <= n; ++m) {
                    const int mu = m - k;
                    if (mu < -d || mu > d) continue;
                    const double2 a = Lt[n * n + n + m];
                    const double2 r = T[d * d + d + mu];   // conj(R~)
                    er += a.x * r.x + a.y * r.y;
                    ei += a.y * r.x - a.x * r.y;
                }
                cr += sd * er;
                ci += sd * ei;
                sd *= sp;
            }
            ar += cr;
            ai += ci;
        }
    }
    if (out) loc[(size_t)cid * nc + t] = make_double2(ar, ai);
}

// ---------------------------------------------------------------- evaluation
// Work-group (leaf cell of the central box, chunk g of Gs), a lane per target
// (central images of real particles; its waves take the passes of 64 targets
// in turn, reading the same sources together): chunk 0 evaluates the cell's local
// expansion at the target,
//   phi = sum L_n^m R_n^m(d),  E_z = -sum L_n^m R_{n-1}^m(d),
//   E_x + i E_y = sum_{m >= 0} L_n^m R_{n-1}^{m+1}(d) - sum_{m >= 1} conj(L_n^m R_{n-1}^{m-1}(d))
// (d = target - cell centre; d/dz R_n^m = R_{n-1}^m, (d/dx + i d/dy) R_n^m =
// -R_{n-1}^{m+1}), and every chunk sums the sources of the neighbouring leaf
// cells g, g + Gs, ... of the 27 directly.  out[(g * 4 + comp) * npad + i],
// comp 0 = phi, 1..3 = E, for target i.
constexpr int EWG = 256;   // evaluation work-group: a wave per pass of 64 targets
__global__ void __launch_bounds__(EWG)
k_tree_eval(const double4* __restrict__ srt, const int* __restrict__ owner,
            const int* __restrict__ offs, const double2* __restrict__ loc, int L, int p, double Lbox,
            int nt, double* __restrict__ out, int npad) {
    const int g = blockIdx.y, Gs = gridDim.y;
    out += (size_t)g * 4 * npad;
    const int lane = threadIdx.x & 63;
    const int side = 1 << L;
    const int cid = blockIdx.x;   // Morton index within the central box
    uint32_t ix = 0, iy = 0, iz = 0;
    for (int b = 0; b < L; ++b) {
        ix |= ((cid >> (3 * b + 2)) & 1u) << b;
        iy |= ((cid >> (3 * b + 1)) & 1u) << b;
        iz |= ((cid >> (3 * b)) & 1u) << b;
    }
    const int gx = side + (int)ix, gy = side + (int)iy, gz = side + (int)iz;
    const uint32_t key = cell_key(gx, gy, gz, L);
    const int b0 = offs[key], b1 = offs[key + 1];
    const double h = Lbox / (double)side;
    const double ccx = -1.5 * Lbox + (gx + 0.5) * h;
    const double ccy = -1.5 * Lbox + (gy + 0.5) * h;
    const double ccz = -1.5 * Lbox + (gz + 0.5) * h;
    const double2* LL = loc + (size_t)cid * tri(p + 1, 0);
    // the waves take the target passes in turn; they read the same sources
    const int w0 = 64 * __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int base = b0 + w0; base < b1; base += EWG) {
        const int s = base + lane;
        const bool act = s < b1;
        const int me = act ? owner[s] : -1;
        const bool tgt = act && me >= 0 && me < nt;
        const double4 t = srt[act ? s : b0];
        double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        if (g == 0) {
            // columns m of R_n^m(d), n = m..p, each combined with the
            // coefficients of rows n and n + 1
            const double x = t.x - ccx, y = t.y - ccy, z = t.z - ccz;
            const double r2 = x * x + y * y + z * z;
            double dr = 1.0, di = 0.0;   // R_m^m
            for (int m = 0; m <= p; ++m) {
                if (m > 0) {
                    const double nr = (dr * x - di * y) / (2.0 * m);
                    const double ni = (dr * y + di * x) / (2.0 * m);
                    dr = nr;
                    di = ni;
                }
                const double wm = m == 0 ? 1.0 : 2.0;
                double pr = 0.0, pi = 0.0, cr = dr, ci = di;
                for (int n = m; n <= p; ++n) {
                    if (n > m) {
                        const double inv = 1.0 / ((double)(n + m) * (double)(n - m));
                        const double nr = ((2 * n - 1) * z * cr - r2 * pr) * inv;
                        const double ni = ((2 * n - 1) * z * ci - r2 * pi) * inv;
                        pr = cr; pi = ci; cr = nr; ci = ni;
                    }
                    const double2 a = LL[tri(n, m)];
                    phi += wm * (a.x * cr - a.y * ci);
                    if (n + 1 <= p) {
                        const double2 b = LL[tri(n + 1, m)];       // E_z: L_{n+1}^m R_n^m
                        ez -= wm * (b.x * cr - b.y * ci);
                        const double2 c = LL[tri(n + 1, m + 1)];   // -conj(L_{n+1}^{m+1} R_n^m)
                        ex -= c.x * cr - c.y * ci;
                        ey += c.x * ci + c.y * cr;
                        if (m >= 1) {                              // L_{n+1}^{m-1} R_n^m
                            const double2 e = LL[tri(n + 1, m - 1)];
                            ex += e.x * cr - e.y * ci;
                            ey += e.x * ci + e.y * cr;
                        }
                    }
                }
            }
        }
        // neighbouring leaf cells of this chunk, directly
        const int G = 3 << L;
        int item = 0;
        for (int cx = gx - 1; cx <= gx + 1; ++cx) {
            for (int cy = gy - 1; cy <= gy + 1; ++cy) {
                for (int cz = gz - 1; cz <= gz + 1; ++cz) {
                    if ((item++) % Gs != g) continue;
                    if (cx < 0 || cx >= G || cy < 0 || cy >= G || cz < 0 || cz >= G) continue;
                    const uint32_t ck = cell_key(cx, cy, cz, L);
                    const int e0 = offs[ck], e1 = offs[ck + 1];
                    auto term = [&](const double4& r) {
                        const double dx = t.x - r.x, dy = t.y - r.y, dz = t.z - r.z;
                        const double d2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
                        const double y = rsqrt_f64(d2);
                        const double qy = r.w * y;
                        phi += qy;
                        const double w = qy * y * y;
                        ex = __builtin_fma(w, dx, ex);
                        ey = __builtin_fma(w, dy, ey);
                        ez = __builtin_fma(w, dz, ez);
                    };
                    if (cx == gx && cy == gy && cz == gz) {
                        // the target's own cell: skip the bare self term
                        for (int j = e0; j < e1; ++j)
                            if (j != s) term(srt[j]);
                    } else {
                        // four sources a step, summed in order
                        int j = e0;
                        for (; j + 3 < e1; j += 4) {
                            const double4 r0 = srt[j], r1 = srt[j + 1], r2 = srt[j + 2], r3 = srt[j + 3];
                            term(r0);
                            term(r1);
                            term(r2);
                            term(r3);
                        }
                        for (; j < e1; ++j) term(srt[j]);
                    }
                }
            }
        }
        if (tgt) {
            out[me] = phi;
            out[(size_t)npad + me] = ex;
            out[(size_t)2 * npad + me] = ey;
            out[(size_t)3 * npad + me] = ez;
        }
    }
}

// ---------------------------------------------------------------- points
// Potential at a point displaced (x, y, z) from a cell centre, from the
// cell's multipoles (m >= 0, row-packed): phi = sum_{n,m} M_n^m I_n^m.
__device__ double m2p_phi(const double2* __restrict__ M, int p, double x, double y, double z) {
    const double r2 = x * x + y * y + z * z;
    const double ir2 = 1.0 / r2;
    double dr = 1.0 / sqrt(r2), di = 0.0;   // I_m^m
    double phi = 0.0;
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const double f = (2 * m - 1) * ir2;
            const double nr = f * (x * dr - y * di);
            const double ni = f * (x * di + y * dr);
            dr = nr;
            di = ni;
        }
        const double wm = m == 0 ? 1.0 : 2.0;
        double pr = 0.0, pi = 0.0, cr = dr, ci = di;
        double acc = 0.0;
        for (int n = m; n <= p; ++n) {
            if (n > m) {
                const double c2 = (double)((n - 1) * (n - 1) - m * m);
                const double nr = ((2 * n - 1) * z * cr - c2 * pr) * ir2;
                const double ni = ((2 * n - 1) * z * ci - c2 * pi) * ir2;
                pr = cr; pi = ci; cr = nr; ci = ni;
            }
            const double2 a = M[tri(n, m)];
            acc += a.x * cr - a.y * ci;
        }
        phi += wm * acc;
    }
    return phi;
}

constexpr int PT_MAX_ITEMS = 27 + 189 * TREE_MAX_LEVEL;   // far cells of one point, all levels

// A work-group of four waves per point (monitoring points and twins, centred
// coordinates):
// the potential of every image in the 3x3x3 block, from the multipoles of
// the point's far cells at every level and the images of its 27 neighbouring
// leaf cells directly.  Far cells: at level 0 the boxes not adjacent to the
// point's box (a point outside the central box has such boxes), at level
// l >= 1 the children of the neighbours of the point's level-(l - 1) cell
// that are not neighbours of its level-l cell.  The far cells are listed in
// LDS first and then shared out over the work-group's lanes, like the
// neighbours' images; the lane sums are combined by a fixed butterfly in each
// wave and the waves' sums in order.
constexpr int PT_WG = 256;   // a work-group (four waves) per point
__global__ void __launch_bounds__(PT_WG)
k_tree_points(const double4* __restrict__ pts, const int* __restrict__ order, int npts, int share,
              const double4* __restrict__ srt, const int* __restrict__ offs, MomPtrs moms, int L, int p,
              double Lbox, double* __restrict__ out) {
    __shared__ int item_key[PT_MAX_ITEMS];
    __shared__ char item_lev[PT_MAX_ITEMS];
    const int lane = threadIdx.x;   // thread of the work-group (PT_WG)
    // work-groups go round the XCDs in turn: XCD x takes the points x * share
    // .. (x + 1) * share - 1 of the given order, whose far cells overlap in
    // its L2
    const int pos = (blockIdx.x & 7) * share + (blockIdx.x >> 3);
    if (pos >= npts) return;   // the whole work-group, before any barrier
    const int pi = order[pos];
    const double4 P = pts[pi];
    const int GL = 3 << L;
    const double hL = Lbox / (double)(1 << L);
    int g[3];
    const double v[3] = {P.x, P.y, P.z};
    for (int a = 0; a < 3; ++a) {
        const int c = (int)floor((v[a] + 1.5 * Lbox) / hL);
        g[a] = c < 0 ? 0 : (c >= GL ? GL - 1 : c);
    }
    // the candidates of every level checked at once, the lanes sharing them
    // (inside the cube, not adjacent, not empty), then listed in order (every
    // lane walks the flags and writes its share of the list)
    __shared__ unsigned char okf[27 + 216 * TREE_MAX_LEVEL];
    const int bx = g[0] >> L, by = g[1] >> L, bz = g[2] >> L;
    for (int c = lane; c < 27; c += PT_WG) {
        const int cx = c / 9, cy = (c / 3) % 3, cz = c % 3;
        bool ok = !(abs(cx - bx) <= 1 && abs(cy - by) <= 1 && abs(cz - bz) <= 1);
        if (ok) ok = offs[(size_t)(c + 1) << (3 * L)] != offs[(size_t)c << (3 * L)];
        okf[c] = ok ? 1 : 0;
    }
    for (int l = 1; l <= L; ++l) {
        const int G = 3 << l;
        const int shift = 3 * (L - l);
        const int tx = g[0] >> (L - l), ty = g[1] >> (L - l), tz = g[2] >> (L - l);
        const int px = tx >> 1, py = ty >> 1, pz = tz >> 1;
        for (int c = lane; c < 216; c += PT_WG) {
            const int cx = 2 * px - 2 + c / 36, cy = 2 * py - 2 + (c / 6) % 6, cz = 2 * pz - 2 + c % 6;
            bool ok = cx >= 0 && cx < G && cy >= 0 && cy < G && cz >= 0 && cz < G &&
                      !(abs(cx - tx) <= 1 && abs(cy - ty) <= 1 && abs(cz - tz) <= 1);
            if (ok) {
                const uint32_t ck = cell_key(cx, cy, cz, l);
                ok = offs[(size_t)(ck + 1) << shift] != offs[(size_t)ck << shift];
            }
            okf[27 + 216 * (l - 1) + c] = ok ? 1 : 0;
        }
    }
    __syncthreads();
    int nitem = 0;
    for (int c = 0; c < 27; ++c)
        if (okf[c]) {
            if (nitem % PT_WG == lane) { item_key[nitem] = c; item_lev[nitem] = 0; }
            ++nitem;
        }
    for (int l = 1; l <= L; ++l) {
        const int tx = g[0] >> (L - l), ty = g[1] >> (L - l), tz = g[2] >> (L - l);
        const int px = tx >> 1, py = ty >> 1, pz = tz >> 1;
        for (int c = 0; c < 216; ++c)
            if (okf[27 + 216 * (l - 1) + c]) {
                if (nitem % PT_WG == lane) {
                    item_key[nitem] = (int)cell_key(2 * px - 2 + c / 36, 2 * py - 2 + (c / 6) % 6,
                                                    2 * pz - 2 + c % 6, l);
                    item_lev[nitem] = (char)l;
                }
                ++nitem;
            }
    }
    __syncthreads();
    const int nc = tri(p + 1, 0);
    double acc = 0.0;
    for (int i = lane; i < nitem; i += PT_WG) {
        const int l = item_lev[i];
        const uint32_t ck = (uint32_t)item_key[i];
        // centre of cell ck of level l
        const uint32_t box = ck >> (3 * l), mc = ck & ((1u << (3 * l)) - 1u);
        uint32_t ix = 0, iy = 0, iz = 0;
        for (int bb = 0; bb < l; ++bb) {
            ix |= ((mc >> (3 * bb + 2)) & 1u) << bb;
            iy |= ((mc >> (3 * bb + 1)) & 1u) << bb;
            iz |= ((mc >> (3 * bb)) & 1u) << bb;
        }
        const double h = Lbox / (double)(1 << l);
        const double cx = -1.5 * Lbox + ((double)((box / 9) * (1u << l) + ix) + 0.5) * h;
        const double cy = -1.5 * Lbox + ((double)(((box / 3) % 3) * (1u << l) + iy) + 0.5) * h;
        const double cz = -1.5 * Lbox + ((double)((box % 3) * (1u << l) + iz) + 0.5) * h;
        acc += m2p_phi(moms.lev[l] + (size_t)ck * nc, p, P.x - cx, P.y - cy, P.z - cz);
    }
    // neighbouring leaf cells, directly
    for (int cx = g[0] - 1; cx <= g[0] + 1; ++cx) {
        if (cx < 0 || cx >= GL) continue;
        for (int cy = g[1] - 1; cy <= g[1] + 1; ++cy) {
            if (cy < 0 || cy >= GL) continue;
            for (int cz = g[2] - 1; cz <= g[2] + 1; ++cz) {
                if (cz < 0 || cz >= GL) continue;
                const uint32_t ck = cell_key(cx, cy, cz, L);
                const int e1 = offs[ck + 1];
                for (int j = offs[ck] + lane; j < e1; j += PT_WG) {
                    const double4 r = srt[j];
                    const double dx = P.x - r.x, dy = P.y - r.y, dz = P.z - r.z;
                    acc += r.w / sqrt(dx * dx + dy * dy + dz * dz);
                }
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    // the waves' sums, added in order
    __shared__ double wsum[PT_WG / 64];
    if ((lane & 63) == 0) wsum[lane >> 6] = acc;
    __syncthreads();
    if (lane == 0) {
        double v = wsum[0];
        for (int w = 1; w < PT_WG / 64; ++w) v += wsum[w];
        out[pi] = v;
    }
}

// ---------------------------------------------------------------- host
// Dynamic LDS of the blocked M2L: I~ up to order 2p + R (34 KB at order 20).
static size_t m2l_tile_lds(int p) {
    const size_t nip = (size_t)(2 * p + m2l_rows(p) + 1) * (2 * p + m2l_rows(p) + 1);
    return sizeof(double2) * nip;
}

// The blocked M2L serves the levels with at least M2L_NT cells per parent
// corner.
static bool m2l_tiled(int l) { return l >= 3; }

// Work-groups per cell (direct M2L) or per tile of M2L_NT cells (blocked
// M2L) at level l: enough that a level of few cells still spreads over the
// GPU.
static int split_cell(int l) { return std::max(1, std::min(16, 2048 / (1 << (3 * l)))); }
// The blocked M2L keeps 5 work-groups per compute unit resident at 3 orders
// per lane (4 at 5): the split fills the 256 compute units for whole rounds.
static int split_tile(int l, int p) {
    const int round = 256 * (m2l_rows(p) == 3 ? 5 : 4);
    return std::max(1, std::min(48, round / ((1 << (3 * l)) / M2L_NT)));
}

int tree_leaf_level(int64_t ns) {
    // at most tree_leaf_images() images per leaf cell (ns / 8^L: the 27 ns
    // images fill the 27 boxes alike)
    const double cap = tree_leaf_images();
    int L = 1;
    while (L < TREE_MAX_LEVEL && (double)ns / (double)(1LL << (3 * L)) > cap) ++L;
    return L;
}

double tree_leaf_images() {
    static const double v = [] {
        const char* e = getenv("HSMA_TREE_LEAF");
        const double d = e ? atof(e) : 0.0;
        return d >= 1.0 ? d : 1000.0;
    }();
    return v;
}

TreeLayout tree_layout(int64_t ns, int p) {
    TreeLayout t;
    t.L = tree_leaf_level(ns);
    t.p = p;
    t.ns = ns;
    t.nimg = 27 * ns;
    t.ncell_leaf = (int64_t)27 << (3 * t.L);
    // enough evaluation work-groups to spread few leaf cells over the GPU
    t.eval_split = std::max(1, std::min(27, 16384 >> (3 * t.L)));
    const int nc = tri(p + 1, 0);
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = (o + b + 255) & ~(size_t)255; return r; };
    t.off_img = take(sizeof(double4) * (size_t)t.nimg);
    t.off_srt = take(sizeof(double4) * (size_t)t.nimg);
    t.off_keys = take(sizeof(uint32_t) * (size_t)t.nimg);
    t.off_keys2 = take(sizeof(uint32_t) * (size_t)t.nimg);
    t.off_vals = take(sizeof(int) * (size_t)t.nimg);
    t.off_vals2 = take(sizeof(int) * (size_t)t.nimg);
    t.off_owner = take(sizeof(int) * (size_t)t.nimg);
    t.off_offs = take(sizeof(int) * (size_t)(t.ncell_leaf + 1));
    for (int l = 0; l <= t.L; ++l) t.off_mom[l] = take(sizeof(double2) * (size_t)nc * ((size_t)27 << (3 * l)));
    for (int l = 1; l <= t.L; ++l) t.off_loc[l] = take(sizeof(double2) * (size_t)nc * ((size_t)1 << (3 * l)));
    t.off_tab = take(sizeof(double2) * 8 * (size_t)(p + 1) * (p + 1));
    t.off_itab = take(sizeof(double2) * 343 * (size_t)(2 * p + 1) * (2 * p + 1));
    size_t part_cells = 0;
    for (int l = 1; l <= t.L; ++l)   // room for either M2L's parts
        part_cells = std::max(part_cells, (size_t)std::max(split_cell(l), m2l_tiled(l) ? split_tile(l, p) : 0)
                                              << (3 * l));
    t.off_part = take(sizeof(double2) * (size_t)nc * part_cells);
    // hipCUB temporary storage of the sort
    size_t sort_bytes = 0;
    if (t.nimg <= (int64_t)INT32_MAX)   // larger trees are refused before any launch
        hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (int*)nullptr, (int*)nullptr, (int)t.nimg, 0, 32);
    t.cub_bytes = sort_bytes;
    t.off_cub = take(t.cub_bytes);
    t.total = o;
    return t;
}

// conj(R~_j^k(d)) for the 8 child offsets d of a unit-side parent (per axis
// -1/4 or +1/4, octant o = Morton digit), (p+1)^2 entries per octant (index
// j*j + j + k), by the recurrences of the leaf moments.  One thread per octant.
__global__ void k_tree_m2m_table(int p, double2* __restrict__ tab) {
    // a thread per (octant, column m): R_m^m by the diagonal recurrence, then
    // up the column in n
    const int id = threadIdx.x;
    const int o = id / (p + 1), m = id - o * (p + 1);
    if (o >= 8) return;
    const double x = ((o >> 2) & 1) ? 0.25 : -0.25;
    const double y = ((o >> 1) & 1) ? 0.25 : -0.25;
    const double z = (o & 1) ? 0.25 : -0.25;
    const double r2 = x * x + y * y + z * z;
    double2* T = tab + (size_t)o * (p + 1) * (p + 1);
    double dr = 1.0, di = 0.0;   // R_0^0, then R_k^k up to k = m
    for (int k = 1; k <= m; ++k) {
        const double nr = (dr * x - di * y) / (2.0 * k);
        const double ni = (dr * y + di * x) / (2.0 * k);
        dr = nr;
        di = ni;
    }
    double pr = 0.0, pi = 0.0, cr = dr, ci = di;
    for (int n = m; n <= p; ++n) {
        if (n > m) {
            const double inv = 1.0 / ((double)(n + m) * (double)(n - m));
            const double nr = ((2 * n - 1) * z * cr - r2 * pr) * inv;
            const double ni = ((2 * n - 1) * z * ci - r2 * pi) * inv;
            pr = cr; pi = ci; cr = nr; ci = ni;
        }
        // conj(R~_n^m) = conj(R_n^m); conj(R~_n^-m) = (-1)^m R_n^m
        T[n * n + n + m] = make_double2(cr, -ci);
        if (m > 0) {
            const double sg = (m & 1) ? -1.0 : 1.0;
            T[n * n + n - m] = make_double2(sg * cr, sg * ci);
        }
    }
}

hipError_t launch_tree_build(int img, double gamma, const double4* src, int ns, double L, const TreeLayout& t,
                             char* ws, hipStream_t s) {
    if (ns <= 0) return hipSuccess;
    if (t.p < 1 || t.p > TREE_MAX_ORDER || t.L < 1 || t.L > TREE_MAX_LEVEL) return hipErrorInvalidValue;
    double4* img4 = (double4*)(ws + t.off_img);
    double4* srt = (double4*)(ws + t.off_srt);
    uint32_t* keys = (uint32_t*)(ws + t.off_keys);
    uint32_t* keys2 = (uint32_t*)(ws + t.off_keys2);
    int* vals = (int*)(ws + t.off_vals);
    int* vals2 = (int*)(ws + t.off_vals2);
    int* owner = (int*)(ws + t.off_owner);
    int* offs = (int*)(ws + t.off_offs);
    const int64_t n = t.nimg;
    hipLaunchKernelGGL(k_tree_images, dim3((ns + 255) / 256, 27), dim3(256), 0, s, src, ns, img, gamma, L,
                       t.L, img4, keys, vals);
    size_t cub = t.cub_bytes;
    const int end_bit = 3 * t.L + 5;   // box index < 27 < 2^5
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(ws + t.off_cub, cub, keys, keys2, vals, vals2,
                                                      (int)n, 0, end_bit, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tree_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, img4, vals2,
                       n, ns, srt, owner);
    hipLaunchKernelGGL(k_tree_offsets, dim3((unsigned)((t.ncell_leaf + 1 + 255) / 256)), dim3(256), 0, s, keys2,
                       n, t.ncell_leaf, offs);
    // multipoles: leaf level directly, coarser levels (down to the 27 boxes
    // of level 0) by translation
    // leaf multipoles: a wave per cell for leaf levels 1-2 (equal to the
    // columns at level 2), a thread per (cell, m) from level 3 on (1.9 against
    // 1.2 ms at 3e5 particles)
    if (t.ncell_leaf <= 2048)
        hipLaunchKernelGGL(k_tree_p2m_wave, dim3((unsigned)t.ncell_leaf), dim3(64), 0, s, srt, offs, t.L, t.p,
                           L, (double2*)(ws + t.off_mom[t.L]));
    else {
        const dim3 grid((unsigned)((t.ncell_leaf + 511) / 512 * 8 * (t.p + 1)));
        if (t.p <= 16)
            hipLaunchKernelGGL(k_tree_p2m_cols<16>, grid, dim3(64), 0, s, srt, offs, t.L, (int)t.ncell_leaf, t.p,
                               L, (double2*)(ws + t.off_mom[t.L]));
        else
            hipLaunchKernelGGL(k_tree_p2m_cols<TREE_MAX_ORDER>, grid, dim3(64), 0, s, srt, offs, t.L,
                               (int)t.ncell_leaf, t.p, L, (double2*)(ws + t.off_mom[t.L]));
    }
    double2* dtab = (double2*)(ws + t.off_tab);
    hipLaunchKernelGGL(k_tree_m2m_table, dim3(1), dim3(8 * (TREE_MAX_ORDER + 1)), 0, s, t.p, dtab);
    const size_t lds_m2m = sizeof(double2) * 8 * (size_t)(t.p + 1) * (t.p + 1);   // >= M2M_Q nc parts
    const int nc = tri(t.p + 1, 0);
    for (int l = t.L - 1; l >= 0; --l) {
        // a work-group per parent while the parents are few, a thread per
        // coefficient for many (measured faster at each end)
        const int64_t ncell = (int64_t)27 << (3 * l);
        const double side = L / (double)(1 << l);
        if (ncell <= 512)
            hipLaunchKernelGGL(k_tree_m2m_group, dim3((unsigned)ncell), dim3(M2M_Q * ((nc + 63) / 64 * 64)),
                               lds_m2m, s,
                               (const double2*)(ws + t.off_mom[l + 1]), offs, l, t.L, t.p, side, dtab,
                               (double2*)(ws + t.off_mom[l]));
        else
            hipLaunchKernelGGL(k_tree_m2m_coef, dim3((unsigned)((ncell * nc + 255) / 256)), dim3(256), 0, s,
                               (const double2*)(ws + t.off_mom[l + 1]), offs, l, t.L, (int)ncell, t.p, side, dtab,
                               (double2*)(ws + t.off_mom[l]));
    }
    return hipGetLastError();
}

hipError_t launch_tree_points(const double4* pts, const int* order, int npts, double L, const TreeLayout& t,
                              char* ws, double* out, hipStream_t s) {
    if (npts <= 0) return hipSuccess;
    MomPtrs mp;
    for (int l = 0; l <= TREE_MAX_LEVEL; ++l)
        mp.lev[l] = l <= t.L ? (const double2*)(ws + t.off_mom[l]) : nullptr;
    const int share = (npts + 7) / 8;
    hipLaunchKernelGGL(k_tree_points, dim3(8 * share), dim3(PT_WG), 0, s, pts, order, npts, share,
                       (const double4*)(ws + t.off_srt), (const int*)(ws + t.off_offs), mp, t.L, t.p, L, out);
    return hipGetLastError();
}

hipError_t launch_tree_near(int nt, double L, const TreeLayout& t, char* ws, double* out, int npad,
                            hipStream_t s) {
    if (nt <= 0) return hipSuccess;
    const int* offs = (const int*)(ws + t.off_offs);
    const double2* dtab = (const double2*)(ws + t.off_tab);
    // local expansions of the central box, level by level
    double2* itab = (double2*)(ws + t.off_itab);
    hipLaunchKernelGGL(k_fmm_itab, dim3((343 * (2 * t.p + 1) + 255) / 256), dim3(256), 0, s, 2 * t.p, itab);
    double2* part = (double2*)(ws + t.off_part);
    for (int l = 1; l <= t.L; ++l) {
        double2* loc = (double2*)(ws + t.off_loc[l]);
        const double2* ploc = l >= 2 ? (const double2*)(ws + t.off_loc[l - 1]) : nullptr;
        const bool tiled = m2l_tiled(l);
        const int G = tiled ? split_tile(l, t.p) : split_cell(l);
        if (tiled) {
            const dim3 grid((1u << (3 * l)) / M2L_NT, G);
            if (m2l_rows(t.p) == 3)
                hipLaunchKernelGGL(k_fmm_m2l_tile<3>, grid, dim3(64 * M2L_WAVES), m2l_tile_lds(t.p), s,
                                   (const double2*)(ws + t.off_mom[l]), l, t.p, L, itab, G, part);
            else
                hipLaunchKernelGGL(k_fmm_m2l_tile<5>, grid, dim3(64 * M2L_WAVES), m2l_tile_lds(t.p), s,
                                   (const double2*)(ws + t.off_mom[l]), l, t.p, L, itab, G, part);
        } else {
            const size_t lds = sizeof(double2) * ((size_t)(t.p + 1) * (t.p + 1) +
                                                  (size_t)(2 * t.p + 1) * (2 * t.p + 1)) +
                               sizeof(double) * (t.p + 1);
            hipLaunchKernelGGL(k_fmm_m2l, dim3(1u << (3 * l), G), dim3(FWG), lds, s,
                               (const double2*)(ws + t.off_mom[l]), offs, l, t.L, t.p, L, itab, G, part);
        }
        hipLaunchKernelGGL(k_fmm_l2l, dim3(1u << (3 * l)), dim3(FWG), 0, s, part, G, l, t.p, L, dtab, ploc,
                           loc);
    }
    hipLaunchKernelGGL(k_tree_eval, dim3(1u << (3 * t.L), t.eval_split), dim3(EWG), 0, s,
                       (const double4*)(ws + t.off_srt), (const int*)(ws + t.off_owner), offs,
                       (const double2*)(ws + t.off_loc[t.L]), t.L, t.p, L, nt, out, npad);
    return hipGetLastError();
}

}  // namespace hsma
