// Near-field sum over the 3x3x3 image block by a tree code (the O(N log N)
// acceleration of the near sum that Sec. II.C and Table I leave to the FMM):
// the same quantity as the direct near kernels, phi_i and E_i from every
// image of every source in the block except the bare self term, to a
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
// Multipoles about cell centres in complex solid harmonics,
//   R_n^m(r) = r^n P_n^m(cos t) e^{i m phi} / (n + m)!,
//   I_n^m(r) = (n - m)! P_n^m(cos t) e^{i m phi} / r^{n + 1}       (m >= 0),
// with 1/|x - y| = sum_{n,m} conj(R_n^m(y)) I_n^m(x) for |y| < |x| (negative m
// by complex conjugation), built by their Cartesian recurrences:
//   R_m^m = (x + iy) / (2m) R_{m-1}^{m-1},
//   (n^2 - m^2) R_n^m = (2n - 1) z R_{n-1}^m - r^2 R_{n-2}^m,
//   I_m^m = (2m - 1) (x + iy) / r^2 I_{m-1}^{m-1},
//   r^2 I_n^m = (2n - 1) z I_{n-1}^m - ((n - 1)^2 - m^2) I_{n-2}^m.
// Leaf moments M_n^m = sum_j q_j conj(R_n^m(y_j - c)) are summed per cell;
// coarser ones by translation to the parent centre,
//   M~_n^m(P) = sum_{j,k} conj(R~_j^k(c_C - c_P)) M~_{n-j}^{m-k}(C),
// with R~_n^m = R_n^m for m >= 0 and (-1)^m R_n^m for m < 0 (the convention
// in which the addition theorem of the regular harmonics is a plain
// convolution).  A target evaluates, at every level, the cells that are
// children of its parent cell's neighbours but not its own cell's neighbours
// (up to 189 per level), from their moments:
//   phi = sum M_n^m I_n^m,   E_z = sum M_n^m I_{n+1}^m,
//   E_x + i E_y = sum_{m >= 0} M_n^m I_{n+1}^{m+1} - sum_{m >= 1} conj(M_n^m I_{n+1}^{m-1})
// (d/dz I_n^m = -I_{n+1}^m and (d/dx + i d/dy) I_n^m = -I_{n+1}^{m+1} for
// m >= 0), and the sources of the 27 neighbouring leaf cells directly.  Every
// sum runs in a fixed order: results are bitwise reproducible.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "hsma_internal.h"
#include "pair_math.h"
#include "tree.h"

namespace hsma {

constexpr int TWG = 64;   // one wave per work-group

__host__ __device__ __forceinline__ int tri(int n, int m) { return n * (n + 1) / 2 + m; }

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
__global__ void k_tree_images(const double4* __restrict__ src, int ns, int img, double L, int lev,
                              double4* __restrict__ out, uint32_t* __restrict__ keys,
                              int* __restrict__ vals) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int kk = blockIdx.y;
    if (j >= ns) return;
    const int kx = kk / 9 - 1, ky = (kk / 3) % 3 - 1, kz = kk % 3 - 1;
    const double4 r = src[j];
    double px = r.x, py = r.y, pz = r.z, q = r.w;
    if (img == IMG_METALLIC) {
        if (kx) { px = -px; q = -q; }
        if (ky) { py = -py; q = -q; }
        if (kz) { pz = -pz; q = -q; }
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

__global__ void k_tree_count(const uint32_t* __restrict__ keys, int64_t n, int* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&cnt[keys[i]], 1);
}

__global__ void k_tree_zero_int(int* __restrict__ a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

// ---------------------------------------------------------------- leaf moments
// Thread (cell, m): column m of the moments of leaf cell `cell`, summed over
// its sources in sorted order.
__global__ void k_tree_p2m(const double4* __restrict__ srt, const int* __restrict__ offs, int lev,
                           int ncell, int p, double L, double2* __restrict__ mom) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int m = (int)(t % (p + 1));
    const int64_t cell = t / (p + 1);
    if (cell >= ncell) return;
    const int b = offs[cell], e = offs[cell + 1];
    double2* out = mom + (size_t)cell * tri(p + 1, 0);
    double ar[TREE_MAX_ORDER + 1], ai[TREE_MAX_ORDER + 1];
    for (int n = 0; n <= p; ++n) ar[n] = ai[n] = 0.0;
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
        for (int s = b; s < e; ++s) {
            const double4 y = srt[s];
            const double x = y.x - cx, yy = y.y - cy, z = y.z - cz;
            const double r2 = x * x + yy * yy + z * z;
            // R_m^m = (x + iy)^m / (2^m m!)
            double dr = 1.0, di = 0.0;
            for (int k = 1; k <= m; ++k) {
                const double nr = (dr * x - di * yy) / (2.0 * k);
                const double ni = (dr * yy + di * x) / (2.0 * k);
                dr = nr;
                di = ni;
            }
            double pr = 0.0, pi = 0.0, cr = dr, ci = di;   // R_{n-2}, R_{n-1}
            for (int n = m; n <= p; ++n) {
                if (n > m) {
                    const double inv = 1.0 / ((double)(n + m) * (double)(n - m));
                    const double nr = ((2 * n - 1) * z * cr - r2 * pr) * inv;
                    const double ni = ((2 * n - 1) * z * ci - r2 * pi) * inv;
                    pr = cr; pi = ci; cr = nr; ci = ni;
                }
                // M += q conj(R)
                ar[n] = __builtin_fma(y.w, cr, ar[n]);
                ai[n] = __builtin_fma(-y.w, ci, ai[n]);
            }
        }
    }
    for (int n = m; n <= p; ++n) out[tri(n, m)] = make_double2(ar[n], ai[n]);
}

// ---------------------------------------------------------------- translation
// Thread (parent cell, n, m >= 0) of level l: the moment M_n^m of the parent
// from its 8 children at level l + 1 (children with no source skipped).
// tab holds conj(R~_j^k(d_o)) of the 8 child offsets d_o (per axis +-1/4 of
// the parent's side, octant o = Morton digit) for the unit side, 8 x (p+1)^2
// entries (index j*j + j + k), scaled here by side^j.
__global__ void k_tree_m2m(const double2* __restrict__ child, const int* __restrict__ offs, int l,
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
            for (int k = -j; k <= j; ++k) {
                const int mm = m - k, nn = n - j;
                if (mm > nn || -mm > nn) continue;
                const double2 a = T[j * j + j + k];
                // M~_nn^mm: stored for mm >= 0; (-1)^mm conj(M_nn^-mm) below
                double2 b = M[tri(nn, mm < 0 ? -mm : mm)];
                if (mm < 0) {
                    b.y = -b.y;
                    if ((-mm) & 1) { b.x = -b.x; b.y = -b.y; }
                }
                const double ar = a.x * sj, ai = a.y * sj;
                sr += ar * b.x - ai * b.y;
                si += ar * b.y + ai * b.x;
            }
            sj *= side;
        }
    }
    parent[(size_t)cell * nt + idx] = make_double2(sr, si);
}

// ---------------------------------------------------------------- evaluation
// phi and E at a target displaced d from a cell centre, from the cell's
// moments M (m >= 0, row-packed by tri): columns m of I_n^m, n = m..p+1, in
// turn, each combined with the moments of rows n and n - 1.
__device__ __forceinline__ void m2p(const double2* __restrict__ M, int p, double x, double y,
                                    double z, double& phi, double& ez, double& wr, double& wi) {
    const double r2 = x * x + y * y + z * z;
    const double ir2 = 1.0 / r2;
    double dr = rsqrt_f64(r2), di = 0.0;   // I_m^m
    for (int m = 0; m <= p + 1; ++m) {
        if (m > 0) {
            const double f = (2 * m - 1) * ir2;
            const double nr = f * (x * dr - y * di);
            const double ni = f * (x * di + y * dr);
            dr = nr;
            di = ni;
        }
        const double wm = m == 0 ? 1.0 : 2.0;
        double pr = 0.0, pi = 0.0, cr = dr, ci = di;
        for (int n = m; n <= p + 1; ++n) {
            if (n > m) {
                const double c2 = (double)((n - 1) * (n - 1) - m * m);
                const double nr = ((2 * n - 1) * z * cr - c2 * pr) * ir2;
                const double ni = ((2 * n - 1) * z * ci - c2 * pi) * ir2;
                pr = cr; pi = ci; cr = nr; ci = ni;
            }
            if (n <= p) {   // phi: M_n^m I_n^m
                const double2 a = M[tri(n, m)];
                phi += wm * (a.x * cr - a.y * ci);
            }
            if (n >= 1 && m <= n - 1 && n - 1 <= p) {   // E_z: M_{n-1}^m I_n^m
                const double2 a = M[tri(n - 1, m)];
                ez += wm * (a.x * cr - a.y * ci);
            }
            if (m >= 1 && n - 1 <= p) {   // M_{n-1}^{m-1} I_n^m
                const double2 a = M[tri(n - 1, m - 1)];
                wr += a.x * cr - a.y * ci;
                wi += a.x * ci + a.y * cr;
            }
            if (m + 1 <= n - 1 && n - 1 <= p) {   // -conj(M_{n-1}^{m+1} I_n^m)
                const double2 a = M[tri(n - 1, m + 1)];
                wr -= a.x * cr - a.y * ci;
                wi += a.x * ci + a.y * cr;
            }
        }
    }
}

// One wave per leaf cell of the central box: its targets (central images of
// real particles) get the far cells of every level and the direct sum over
// the 27 neighbouring leaf cells.  out[(comp) * npad + i], comp 0 = phi,
// 1..3 = E, for target i.
struct MomPtrs {
    const double2* lev[TREE_MAX_LEVEL + 1];   // moments of each level (index 1..L)
};

__global__ void __launch_bounds__(TWG)
k_tree_eval(const double4* __restrict__ srt, const int* __restrict__ owner,
            const int* __restrict__ offs, MomPtrs moms, int L, int p, double Lbox, int nt,
            double* __restrict__ out, int npad) {
    const int lane = threadIdx.x;
    const int side = 1 << L;
    const int cid = blockIdx.x;   // Morton index within the central box
    // leaf coordinates of the cell (central box: global offset side)
    uint32_t ix = 0, iy = 0, iz = 0;
    for (int b = 0; b < L; ++b) {
        ix |= ((cid >> (3 * b + 2)) & 1u) << b;
        iy |= ((cid >> (3 * b + 1)) & 1u) << b;
        iz |= ((cid >> (3 * b)) & 1u) << b;
    }
    const int gx = side + (int)ix, gy = side + (int)iy, gz = side + (int)iz;
    const uint32_t key = cell_key(gx, gy, gz, L);
    const int b0 = offs[key], b1 = offs[key + 1];
    for (int base = b0; base < b1; base += TWG) {
        const int s = base + lane;
        const bool act = s < b1;
        const int me = act ? owner[s] : -1;
        const bool tgt = act && me >= 0 && me < nt;
        double4 t = srt[act ? s : b0];
        double phi = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        // far cells, level by level
        for (int l = 1; l <= L; ++l) {
            const int G = 3 << l;
            const double h = Lbox / (double)(1 << l);
            const int tx = gx >> (L - l), ty = gy >> (L - l), tz = gz >> (L - l);
            const int px = tx >> 1, py = ty >> 1, pz = tz >> 1;
            const double2* M = moms.lev[l];
            const int nc = tri(p + 1, 0);
            const int shift = 3 * (L - l);
            for (int cx = 2 * px - 2; cx <= 2 * px + 3; ++cx) {
                if (cx < 0 || cx >= G) continue;
                for (int cy = 2 * py - 2; cy <= 2 * py + 3; ++cy) {
                    if (cy < 0 || cy >= G) continue;
                    for (int cz = 2 * pz - 2; cz <= 2 * pz + 3; ++cz) {
                        if (cz < 0 || cz >= G) continue;
                        if (abs(cx - tx) <= 1 && abs(cy - ty) <= 1 && abs(cz - tz) <= 1) continue;
                        const uint32_t ck = cell_key(cx, cy, cz, l);
                        if (offs[(size_t)(ck + 1) << shift] == offs[(size_t)ck << shift]) continue;
                        const double ccx = -1.5 * Lbox + (cx + 0.5) * h;
                        const double ccy = -1.5 * Lbox + (cy + 0.5) * h;
                        const double ccz = -1.5 * Lbox + (cz + 0.5) * h;
                        double f = 0.0, fz = 0.0, wr = 0.0, wi = 0.0;
                        m2p(M + (size_t)ck * nc, p, t.x - ccx, t.y - ccy, t.z - ccz, f, fz, wr, wi);
                        phi += f;
                        ex += wr;
                        ey += wi;
                        ez += fz;
                    }
                }
            }
        }
        // neighbouring leaf cells, directly
        const int G = 3 << L;
        for (int cx = gx - 1; cx <= gx + 1; ++cx) {
            if (cx < 0 || cx >= G) continue;
            for (int cy = gy - 1; cy <= gy + 1; ++cy) {
                if (cy < 0 || cy >= G) continue;
                for (int cz = gz - 1; cz <= gz + 1; ++cz) {
                    if (cz < 0 || cz >= G) continue;
                    const uint32_t ck = cell_key(cx, cy, cz, L);
                    const int e0 = offs[ck], e1 = offs[ck + 1];
                    for (int j = e0; j < e1; ++j) {
                        if (j == s) continue;   // the bare self term
                        const double4 r = srt[j];
                        const double dx = t.x - r.x, dy = t.y - r.y, dz = t.z - r.z;
                        const double d2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz));
                        const double y = rsqrt_f64(d2);
                        const double qy = r.w * y;
                        phi += qy;
                        const double w = qy * y * y;
                        ex = __builtin_fma(w, dx, ex);
                        ey = __builtin_fma(w, dy, ey);
                        ez = __builtin_fma(w, dz, ez);
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

// ---------------------------------------------------------------- host
int tree_leaf_level(int64_t ns) {
    // about 32 sources per leaf cell of the central box
    int L = 1;
    while (L < TREE_MAX_LEVEL && (double)ns / (double)(1LL << (3 * L)) > 45.0) ++L;
    return L;
}

TreeLayout tree_layout(int64_t ns, int p) {
    TreeLayout t;
    t.L = tree_leaf_level(ns);
    t.p = p;
    t.ns = ns;
    t.nimg = 27 * ns;
    t.ncell_leaf = (int64_t)27 << (3 * t.L);
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
    t.off_cnt = take(sizeof(int) * (size_t)(t.ncell_leaf + 1));
    t.off_offs = take(sizeof(int) * (size_t)(t.ncell_leaf + 1));
    for (int l = 1; l <= t.L; ++l) t.off_mom[l] = take(sizeof(double2) * (size_t)nc * ((size_t)27 << (3 * l)));
    t.off_tab = take(sizeof(double2) * 8 * (size_t)(p + 1) * (p + 1));
    // hipCUB temporary storage of the sort and the scan
    size_t sort_bytes = 0, scan_bytes = 0;
    hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                       (int*)nullptr, (int*)nullptr, (int)t.nimg, 0, 32);
    hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int*)nullptr, (int*)nullptr,
                                     (int)(t.ncell_leaf + 1));
    t.cub_bytes = std::max(sort_bytes, scan_bytes);
    t.off_cub = take(t.cub_bytes);
    t.total = o;
    return t;
}

// conj(R~_j^k(d)) for the 8 child offsets d of a unit-side parent (per axis
// -1/4 or +1/4, octant o = Morton digit), (p+1)^2 entries per octant (index
// j*j + j + k), by the recurrences of the leaf moments.  One thread per octant.
__global__ void k_tree_m2m_table(int p, double2* __restrict__ tab) {
    const int o = threadIdx.x;
    if (o >= 8) return;
    const double x = ((o >> 2) & 1) ? 0.25 : -0.25;
    const double y = ((o >> 1) & 1) ? 0.25 : -0.25;
    const double z = (o & 1) ? 0.25 : -0.25;
    const double r2 = x * x + y * y + z * z;
    double2* T = tab + (size_t)o * (p + 1) * (p + 1);
    double dr = 1.0, di = 0.0;   // R_m^m
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            const double nr = (dr * x - di * y) / (2.0 * m);
            const double ni = (dr * y + di * x) / (2.0 * m);
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
}

hipError_t launch_tree_near(int img, const double4* src, int ns, int nt, double L, const TreeLayout& t,
                            char* ws, double* out, int npad, hipStream_t s) {
    if (ns <= 0 || nt <= 0) return hipSuccess;
    if (t.p < 1 || t.p > TREE_MAX_ORDER || t.L < 1 || t.L > TREE_MAX_LEVEL) return hipErrorInvalidValue;
    double4* img4 = (double4*)(ws + t.off_img);
    double4* srt = (double4*)(ws + t.off_srt);
    uint32_t* keys = (uint32_t*)(ws + t.off_keys);
    uint32_t* keys2 = (uint32_t*)(ws + t.off_keys2);
    int* vals = (int*)(ws + t.off_vals);
    int* vals2 = (int*)(ws + t.off_vals2);
    int* owner = (int*)(ws + t.off_owner);
    int* cnt = (int*)(ws + t.off_cnt);
    int* offs = (int*)(ws + t.off_offs);
    const int64_t n = t.nimg;
    hipLaunchKernelGGL(k_tree_images, dim3((ns + 255) / 256, 27), dim3(256), 0, s, src, ns, img, L, t.L,
                       img4, keys, vals);
    size_t cub = t.cub_bytes;
    const int end_bit = 3 * t.L + 5;   // box index < 27 < 2^5
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(ws + t.off_cub, cub, keys, keys2, vals, vals2,
                                                      (int)n, 0, end_bit, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tree_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, img4, vals2,
                       n, ns, srt, owner);
    hipLaunchKernelGGL(k_tree_zero_int, dim3(1024), dim3(256), 0, s, cnt, t.ncell_leaf + 1);
    hipLaunchKernelGGL(k_tree_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, keys2, n, cnt);
    cub = t.cub_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(ws + t.off_cub, cub, cnt, offs, (int)(t.ncell_leaf + 1), s);
    if (e != hipSuccess) return e;
    // moments: leaf level directly, coarser levels by translation
    const int nc = tri(t.p + 1, 0);
    double2* mom[TREE_MAX_LEVEL + 1] = {};
    for (int l = 1; l <= t.L; ++l) mom[l] = (double2*)(ws + t.off_mom[l]);
    {
        const int64_t threads = t.ncell_leaf * (t.p + 1);
        hipLaunchKernelGGL(k_tree_p2m, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, srt, offs,
                           t.L, (int)t.ncell_leaf, t.p, L, mom[t.L]);
    }
    double2* dtab = (double2*)(ws + t.off_tab);
    hipLaunchKernelGGL(k_tree_m2m_table, dim3(1), dim3(64), 0, s, t.p, dtab);
    for (int l = t.L - 1; l >= 1; --l) {
        const int64_t ncell = (int64_t)27 << (3 * l);
        const int64_t threads = ncell * nc;
        hipLaunchKernelGGL(k_tree_m2m, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, mom[l + 1],
                           offs, l, t.L, (int)ncell, t.p, L / (double)(1 << l), dtab, mom[l]);
    }
    MomPtrs mp;
    for (int l = 0; l <= TREE_MAX_LEVEL; ++l) mp.lev[l] = mom[l];
    hipLaunchKernelGGL(k_tree_eval, dim3(1u << (3 * t.L)), dim3(TWG), 0, s, srt, owner, offs, mp, t.L,
                       t.p, L, nt, out, npad);
    return hipGetLastError();
}

}  // namespace hsma
