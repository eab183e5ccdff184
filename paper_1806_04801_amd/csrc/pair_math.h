// Device arithmetic shared by the pair-sum kernels: reciprocal square root in
// double, per-axis image differences in both precisions, the sum over the
// 3x3x3 image block of one source, and the two-sum accumulator.
#pragma once

#include "hsma_internal.h"

namespace hsma {

// 1/sqrt(x) in double: the single-precision hardware estimate of x rounded to
// float (about 2^-23 relative; valid for the distances here, far inside the
// float range) refined by one third-order Newton step,
// y <- y + y e (1/2 + 3/8 e), e = 1 - x y^2, which leaves an error of order
// e^3 below double rounding.
__device__ __forceinline__ double rsqrt_f64(double x) {
    double y = (double)__builtin_amdgcn_rsqf((float)x);
    double t = x * y;
    double e = __builtin_fma(-t, y, 1.0);
    double c = __builtin_fma(e, 0.375, 0.5);
    return __builtin_fma(y * e, c, y);
}

// Per-axis target-minus-image differences for k = -1, 0, +1 (index k + 1).
template <int IMG>
__device__ __forceinline__ void diffs_f64(double t, double s, double L, double (&d)[3]) {
    double d0 = t - s;
    d[1] = d0;
    if (IMG == IMG_PERIODIC) {          // image s + kL
        d[0] = d0 + L;
        d[2] = d0 - L;
    } else if (IMG == IMG_METALLIC || IMG == IMG_DIELECTRIC) {   // image -s + kL
        double sm = t + s;
        d[0] = sm + L;
        d[2] = sm - L;
    } else {
        d[0] = d[2] = 0.0;
    }
}

__device__ __forceinline__ float rsq_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_t(double x) { return rsqrt_f64(x); }

// rsqrt_f64 of x[lo..hi-1] (same operations, same results), the chains
// advancing side by side, a step each in turn, so that no step waits on the
// one before it in the same chain.
template <int lo, int hi>
__device__ __forceinline__ void rsq_col(const double (&x)[3], double (&y)[3]) {
    double y0[3], e[3], c3[3], ye[3];
#pragma unroll
    for (int c = lo; c < hi; ++c) y0[c] = (double)__builtin_amdgcn_rsqf((float)x[c]);
#pragma unroll
    for (int c = lo; c < hi; ++c) e[c] = __builtin_fma(-(x[c] * y0[c]), y0[c], 1.0);
#pragma unroll
    for (int c = lo; c < hi; ++c) c3[c] = __builtin_fma(e[c], 0.375, 0.5);
#pragma unroll
    for (int c = lo; c < hi; ++c) ye[c] = y0[c] * e[c];
#pragma unroll
    for (int c = lo; c < hi; ++c) y[c] = __builtin_fma(ye[c], c3[c], y0[c]);
}
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Sum over the images of one source: pot = sum s_k / |d|, f = sum s_k d / |d|^3,
// s_k the image sign (-1 for the odd reflections of the grounded box).  The
// field goes through the marginals of w = s/|d|^3 over the image cube:
// f_x = sum_a dx_a X_a with X_a = sum_bc w_abc, f_y likewise with
// Y_b = sum_ac w_abc, and f_z with Z_c = sum_ab w_abc.  Per image this costs
// one fused add for r^2, one reciprocal square root, one add for the
// potential, and one product plus two fused adds for w into S_ab = sum_c w
// (from which X and Y follow) and into Z_c.
//
// REV also returns the field that the target, as a unit charge, produces at
// the source through the same images: the potential is symmetric, and each
// field component changes sign on the unreflected image (difference t - s)
// and keeps it on the reflected ones (difference t + s - kL), so
// rf_x = sum_a sigma_a dx_a X_a with sigma = -1 for k = 0 of a grounded axis
// and sigma = -1 for every k of a periodic axis.
//
// OWN (periodic block only): a zero central distance marks the source as the
// target itself.  Its 26 images then lie at the lattice vectors k != 0, a
// potential of OWN_IMAGES_PERIODIC / L per unit charge that the caller adds
// exactly in double, so the pair's potential sum is returned as zero (its
// field is zero by symmetry).  In single precision this keeps the rounding of
// a sum of ~19 / L, the same for every particle and so not cancelling in the
// energy of a neutral system, out of the result.  Distinct particles at the
// same position are invalid input.
//
// SHIFT (single precision, periodic block): as each column (a, b) of the
// image cube starts, the column's value for a unit charge at the target
// itself (OWN_COL_*) is subtracted from that column's first term, off the
// running sum, so the running potential stays of order 1 / L instead of
// growing to ~19 / L.  Its rounding dominates the single-precision error of a
// neutral system's energy, which the shift cuts several-fold (tenfold for a
// periodic cube of 1e6 charges).  The pair's
// potential comes back lowered by OWN_COLS_F32 / L per unit charge, which the
// finalize stage restores exactly.
//
// IMG_DIELECTRIC weighs the images of the grounded-cube positions by
// gamma^|k| (Eq. (diel)), the number of reflections |k| = 0..3.
template <typename R, int IMG, bool FIELD, bool SELF, bool REV = false, bool OWN = false,
          bool SHIFT = false>
__device__ __forceinline__ void images_sum(const R (&dx)[3], const R (&dy)[3], const R (&dz)[3],
                                           R& pot, R& fx, R& fy, R& fz, R* rf = nullptr,
                                           R gamma = R(0)) {
    constexpr int lo = (IMG == IMG_FREE) ? 1 : 0;
    constexpr int hi = (IMG == IMG_FREE) ? 2 : 3;
    R sx[3];
#pragma unroll
    for (int a = lo; a < hi; ++a) sx[a] = dx[a] * dx[a];
    R S[3][3], Z[3];
    R r2c = R(1);
    constexpr bool SH = SHIFT && sizeof(R) == sizeof(float) && IMG == IMG_PERIODIC;
    R wgt[4] = {R(1), gamma, R(0), R(0)};   // gamma^(reflections), dielectric only
    if (IMG == IMG_DIELECTRIC) {
        wgt[2] = gamma * gamma;
        wgt[3] = wgt[2] * gamma;
    }
    pot = R(0);
#pragma unroll
    for (int a = lo; a < hi; ++a) {
#pragma unroll
        for (int b = lo; b < hi; ++b) {
            const R sxy = fma_t(dy[b], dy[b], sx[a]);
            // double: the column's reciprocal square roots first, side by
            // side; single precision: one image at a time (one instruction)
            constexpr bool COL = sizeof(R) == sizeof(double);
            R r2v[3], yv[3];
            if constexpr (COL) {
#pragma unroll
                for (int c = lo; c < hi; ++c) r2v[c] = fma_t(dz[c], dz[c], sxy);
                rsq_col<lo, hi>(r2v, yv);
            }
#pragma unroll
            for (int c = lo; c < hi; ++c) {
                const R r2 = COL ? r2v[c] : fma_t(dz[c], dz[c], sxy);
                if (a == 1 && b == 1 && c == 1) r2c = r2;
                R y = COL ? yv[c] : rsq_t(r2);
                if (SELF && a == 1 && b == 1 && c == 1) y = (r2 > R(0)) ? y : R(0);
                const bool neg = (IMG == IMG_METALLIC) && (((a != 1) + (b != 1) + (c != 1)) & 1);
                const int nref = (a != 1) + (b != 1) + (c != 1);
                const R ys = IMG == IMG_DIELECTRIC ? (nref == 0 ? y : y * wgt[nref]) : neg ? -y : y;
                if (SH && c == lo) {
                    const R cab = (a == 1 && b == 1) ? R(OWN_COL_CENTRE)
                                  : (a == 1 || b == 1) ? R(OWN_COL_EDGE) : R(OWN_COL_CORNER);
                    pot = (a == lo && b == lo) ? ys - cab : pot + (ys - cab);
                } else {
                    pot = (a == lo && b == lo && c == lo) ? ys : pot + ys;
                }
                if (FIELD) {
                    const R y2 = y * y;
                    S[a][b] = (c == lo) ? y2 * ys : fma_t(y2, ys, S[a][b]);
                    Z[c] = (a == lo && b == lo) ? y2 * ys : fma_t(y2, ys, Z[c]);
                }
            }
        }
    }
    if (OWN && IMG == IMG_PERIODIC) pot = (r2c > R(0)) ? pot : R(0);
    if (FIELD) {
        R X[3], Y[3];
#pragma unroll
        for (int a = lo; a < hi; ++a) {
            R x = S[a][lo], yv = S[lo][a];
#pragma unroll
            for (int b = lo + 1; b < hi; ++b) {
                x += S[a][b];
                yv += S[b][a];
            }
            X[a] = x;
            Y[a] = yv;
        }
        if (REV && (IMG == IMG_METALLIC || IMG == IMG_DIELECTRIC)) {
            // reflected images first, then the central one with both signs
            const R ox = fma_t(dx[0], X[0], dx[2] * X[2]);
            const R oy = fma_t(dy[0], Y[0], dy[2] * Y[2]);
            const R oz = fma_t(dz[0], Z[0], dz[2] * Z[2]);
            fx = fma_t(dx[1], X[1], ox);
            fy = fma_t(dy[1], Y[1], oy);
            fz = fma_t(dz[1], Z[1], oz);
            rf[0] = fma_t(-dx[1], X[1], ox);
            rf[1] = fma_t(-dy[1], Y[1], oy);
            rf[2] = fma_t(-dz[1], Z[1], oz);
        } else {
            fx = dx[lo] * X[lo];
            fy = dy[lo] * Y[lo];
            fz = dz[lo] * Z[lo];
#pragma unroll
            for (int a = lo + 1; a < hi; ++a) {
                fx = fma_t(dx[a], X[a], fx);
                fy = fma_t(dy[a], Y[a], fy);
                fz = fma_t(dz[a], Z[a], fz);
            }
            if (REV) {
                rf[0] = -fx;
                rf[1] = -fy;
                rf[2] = -fz;
            }
        }
    } else {
        fx = fy = fz = R(0);
        if (REV) rf[0] = rf[1] = rf[2] = R(0);
    }
}


// Error-free sum (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum_acc(float& hi, float& lo, float b) {
    const float s = hi + b;
    const float bb = s - hi;
    const float e = (hi - (s - bb)) + (b - bb);
    hi = s;
    lo += e;
}

struct Pt32 {
    float h0[3], hp[3], hm[3], l[3];
};

__device__ __forceinline__ Pt32 load_pt32(const Rec32& r) {
    Pt32 p;
    p.h0[0] = r.v[0].x; p.h0[1] = r.v[0].y; p.h0[2] = r.v[0].z;
    p.hp[0] = r.v[1].x; p.hp[1] = r.v[1].y; p.hp[2] = r.v[1].z;
    p.hm[0] = r.v[2].x; p.hm[1] = r.v[2].y; p.hm[2] = r.v[2].z;
    p.l[0] = r.v[1].w; p.l[1] = r.v[2].w; p.l[2] = r.v[3].x;
    return p;
}

// Differences along axis a for k = -1, 0, +1 (box side 1), leading parts exact
// for small results:
//   periodic c_t - c_s - k:  k=+1: (hp_t - hm_s) + (l_t - l_s),  k=-1: (hm_t - hp_s) + (l_t - l_s)
//   metallic c_t + c_s - k:  k=+1: (hp_t + hp_s) + (l_t + l_s),  k=-1: (hm_t + hm_s) + (l_t + l_s)
template <int IMG>
__device__ __forceinline__ void diffs_f32(const Pt32& t, const Pt32& s, int a, float (&d)[3]) {
    const float dl = t.l[a] - s.l[a];
    d[1] = (t.h0[a] - s.h0[a]) + dl;
    if (IMG == IMG_PERIODIC) {
        d[2] = (t.hp[a] - s.hm[a]) + dl;
        d[0] = (t.hm[a] - s.hp[a]) + dl;
    } else if (IMG == IMG_METALLIC) {
        const float sl = t.l[a] + s.l[a];
        d[2] = (t.hp[a] + s.hp[a]) + sl;
        d[0] = (t.hm[a] + s.hm[a]) + sl;
    } else {
        d[0] = d[2] = 0.0f;
    }
}


}  // namespace hsma
