// Device bodies of the per-request stages of the update step, shared by the
// single-request pipeline (solve.hip) and the grouped serving launches
// (serve.hip), so a request computes the same arithmetic in both.
#pragma once

#include "hsma_internal.h"
#include "result_status.h"
#include "solve.h"

namespace hsma {

constexpr int SWG = 256;

// Centre (and wrap) particle i; grounded slab: also write its mirror charge
// -q at z -> -z (mirror reflections plus periodic extension turn the slab into
// a periodic cube of side L).
// Inputs in double or single precision (TI), widened to double here.
template <typename TI = double>
__device__ __forceinline__ void prep_body(int i, const TI* __restrict__ x,
                                          const TI* __restrict__ q, int N, int bc, double L,
                                          double4* __restrict__ src, int* __restrict__ status) {
    double c[3] = {(double)x[3 * i], (double)x[3 * i + 1], (double)x[3 * i + 2]};
    const double qi = (double)q[i];
    int bad = 0;
    if (!isfinite(c[0]) || !isfinite(c[1]) || !isfinite(c[2]) || !isfinite(qi)) bad |= 1;
    const double h = 0.5 * L;
    if (bc == HSMA_BC_PERIODIC) {
        for (int a = 0; a < 3; ++a) {
            double v = c[a] - h;
            v -= L * floor(v / L + 0.5);
            c[a] = v;
        }
    } else if (bc == HSMA_BC_METALLIC || bc == HSMA_BC_DIELECTRIC) {
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
    if (bad) atomicOr(status, bad);   // RS_BAD_INPUT, RS_OUT_OF_BOX
    src[i] = make_double4(c[0], c[1], c[2], qi);
    if (bc == HSMA_BC_SLAB_METALLIC_Z) src[N + i] = make_double4(c[0], c[1], -c[2], -qi);
}

// Exact coincidence of two charges, the one configuration whose Coulomb
// energy is infinite.  Particle i is
// entered, by its centred and wrapped position (the one the pair kernels
// use), into an open-addressing table of mask + 1 slots (a power of two at
// least twice the particle count, all -1 beforehand) with linear probing; a
// slot already holding a particle at the same position sets RS_COINCIDENT.
// Every insertion ends within mask + 1 probes, since the table is never full.
__device__ __forceinline__ uint32_t point_slot(const double4& p, uint32_t mask) {
    // + 0.0 turns -0.0 into +0.0, so that equal positions hash alike; the
    // multipliers and the final mix are those of SplitMix64 (Steele et al. 2014)
    uint64_t h = (uint64_t)__double_as_longlong(p.x + 0.0) * 0x9E3779B97F4A7C15ull;
    h = (h ^ (uint64_t)__double_as_longlong(p.y + 0.0)) * 0xBF58476D1CE4E5B9ull;
    h = (h ^ (uint64_t)__double_as_longlong(p.z + 0.0)) * 0x94D049BB133111EBull;
    h ^= h >> 31;
    return (uint32_t)h & mask;
}

__device__ __forceinline__ void dup_insert_body(int i, const double4* __restrict__ src,
                                                int* __restrict__ tab, uint32_t mask,
                                                int* __restrict__ status) {
    const double4 p = src[i];
    uint32_t slot = point_slot(p, mask);
    for (uint64_t probe = 0; probe <= (uint64_t)mask; ++probe) {
        const int j = atomicCAS(&tab[slot], -1, i);
        if (j < 0) return;
        const double4 o = src[j];
        if (o.x == p.x && o.y == p.y && o.z == p.z) {
            atomicOr(status, RS_COINCIDENT);
            return;
        }
        slot = (slot + 1) & mask;
    }
}

// Single-precision record (see Rec32) of point i: coordinates in units of L,
// hi part rounded to a multiple of 2^-24, lo part the float remainder.
__device__ __forceinline__ void rec32_body(int i, const double4* __restrict__ p, double L,
                                           Rec32* __restrict__ out) {
    const double4 r = p[i];
    const double inv = 1.0 / L;
    const double c[3] = {r.x * inv, r.y * inv, r.z * inv};
    float h[3], l[3];
    for (int a = 0; a < 3; ++a) {
        // inside the box |c| <= 1/2 the 2^-24 grid value is exact in float;
        // outside (check points, images) the float may round it, so the lo
        // part is taken against the stored hi part
        const double hq = rint(c[a] * 16777216.0) * (1.0 / 16777216.0);
        h[a] = (float)hq;
        l[a] = (float)(c[a] - (double)h[a]);
    }
    Rec32 o;
    o.v[0] = make_float4(h[0], h[1], h[2], (float)r.w);
    o.v[1] = make_float4(h[0] - 0.5f, h[1] - 0.5f, h[2] - 0.5f, l[0]);
    o.v[2] = make_float4(h[0] + 0.5f, h[1] + 0.5f, h[2] + 0.5f, l[1]);
    o.v[3] = make_float4(l[2], 0.0f, 0.0f, 0.0f);
    out[i] = o;
}

// b_k = Phi_in(x_k) (grounded cube) or Phi_in(x_k) - Phi_in(x~_k) (periodic).
__device__ __forceinline__ void rhs_body(int k, const double* __restrict__ part, int S, int nt_pad,
                                         int K, int twins, double* __restrict__ b) {
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

// Least squares (Sec. II.A): A = argmin ||F A + b|| = -R^-1 Q^T b = -P b;
// row r of P by one wave; periodic: A_00 = 0.
__device__ __forceinline__ void lsq_body(int r, int lane, const double* __restrict__ P, int K,
                                         const double* __restrict__ b, int k0,
                                         double* __restrict__ A) {
    const double* row = P + (size_t)r * K;
    double s = 0.0;
    for (int k = lane; k < K; k += 64) s = __builtin_fma(row[k], b[k], s);
    s = wave_sum(s);
    if (lane == 0) {
        A[k0 + r] = -s;
        if (k0 == 1 && r == 0) A[0] = 0.0;
    }
}

// Harmonic surface mapping (Sec. II.B) for surface point j by one wave:
// charge Q_j = Wq_j . A and dipole p_j = (Wp_j . A) n_j.
__device__ __forceinline__ void map_body(int j, int lane, const double* __restrict__ Wq,
                                         const double* __restrict__ Wp, int nb,
                                         const double* __restrict__ A,
                                         const double* __restrict__ spos, double Rs,
                                         double* __restrict__ surf) {
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

// The paper's form of the mapping (Eq. (cd), Eq. (integrals)) for surface
// point j: the charge Q_j at R_j and, for the dipole layer, the charges
// +w_j Phi_out(R_j)/(4 pi dr) at (R_s - dr/2) n_j and -w_j Phi_out(R_j)/(4 pi dr)
// at (R_s + dr/2) n_j.  Wp_j . A = -w_j Phi_out(R_j)/(4 pi).  One wave.
__device__ __forceinline__ void map_layers_body(int j, int lane, int M, const double* __restrict__ Wq,
                                                const double* __restrict__ Wp, int nb,
                                                const double* __restrict__ A,
                                                const double* __restrict__ spos, double Rs, double dr,
                                                double4* __restrict__ chg) {
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
        const double nx = spos[4 * j] / Rs, ny = spos[4 * j + 1] / Rs, nz = spos[4 * j + 2] / Rs;
        const double ql = -sp / dr;                 // w_j Phi_out(R_j) / (4 pi dr)
        const double ri = Rs - 0.5 * dr, ro = Rs + 0.5 * dr;
        chg[j] = make_double4(spos[4 * j], spos[4 * j + 1], spos[4 * j + 2], sq);
        chg[M + j] = make_double4(ri * nx, ri * ny, ri * nz, ql);
        chg[2 * M + j] = make_double4(ro * nx, ro * ny, ro * nz, -ql);
    }
}

// Block-wide sums of three values in a fixed tree order.
__device__ __forceinline__ void block_sum3(double (&sh)[3][SWG], double& a, double& b, double& c) {
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    sh[2][threadIdx.x] = c;
    __syncthreads();
    for (int w = SWG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
            sh[2][threadIdx.x] += sh[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    a = sh[0][0];
    b = sh[1][0];
    c = sh[2][0];
}

// Net charge sum_i q_i of src[0 .. N) in a fixed order (one block of SWG
// threads; the result is written by thread 0).
__device__ __forceinline__ void net_charge_body(const double4* __restrict__ src, int N,
                                                double* __restrict__ out) {
    __shared__ double sh[3][SWG];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < N; i += SWG) a += src[i].w;
    block_sum3(sh, a, b, c);
    if (threadIdx.x == 0) *out = a;
}

// phi = near + surface (chunk sums in fixed order) + q * fix.own + Q * fix.qc
// (NearFix; Q = *qnet, read only when fix.qc != 0), F = q E, block partial
// sums of q phi, q and |q| (block blk, all SWG threads participate).  phi and
// F are stored in TO (double, or rounded to single precision); the energy
// sums use the double values.
template <typename TO = double>
__device__ __forceinline__ void finalize_body(int blk, const double* __restrict__ near, int Sn,
                                              int npad, const double* __restrict__ surfp, int Ss,
                                              int spad, const double4* __restrict__ src, int N,
                                              NearFix fix, const double* __restrict__ qnet,
                                              TO* __restrict__ phi,
                                              TO* __restrict__ forces,
                                              double* __restrict__ dbg_pn, double* __restrict__ dbg_fn,
                                              double* __restrict__ dbg_po, double* __restrict__ dbg_fo,
                                              double* __restrict__ eblk) {
    __shared__ double sh[3][SWG];
    const int i = blk * SWG + threadIdx.x;
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
        vn[0] += qi * fix.own;
        if (fix.qc != 0.0) vn[0] += *qnet * fix.qc;
        const double p = vn[0] + vo[0];
        if (phi) phi[i] = (TO)p;
        if (forces) {
            forces[3 * i] = (TO)(qi * (vn[1] + vo[1]));
            forces[3 * i + 1] = (TO)(qi * (vn[2] + vo[2]));
            forces[3 * i + 2] = (TO)(qi * (vn[3] + vo[3]));
        }
        if (dbg_pn) dbg_pn[i] = vn[0];
        if (dbg_po) dbg_po[i] = vo[0];
        if (dbg_fn) { dbg_fn[3 * i] = vn[1]; dbg_fn[3 * i + 1] = vn[2]; dbg_fn[3 * i + 2] = vn[3]; }
        if (dbg_fo) { dbg_fo[3 * i] = vo[1]; dbg_fo[3 * i + 1] = vo[2]; dbg_fo[3 * i + 2] = vo[3]; }
        // a non-finite output (e.g. two distinct charges closer than the
        // single-precision records resolve) makes the energy NaN, which the
        // energy stage reports as RS_NONFINITE
        const bool finite = isfinite(p) && isfinite(vn[1] + vo[1]) && isfinite(vn[2] + vo[2]) &&
                            isfinite(vn[3] + vo[3]);
        e = finite ? qi * p : __builtin_nan("");
        qs = qi;
        qa = fabs(qi);
    }
    block_sum3(sh, e, qs, qa);
    if (threadIdx.x == 0) {
        eblk[3 * blk] = e;
        eblk[3 * blk + 1] = qs;
        eblk[3 * blk + 2] = qa;
    }
}

// E = 1/2 sum q phi; neutrality flag for periodic and slab systems (one block).
__device__ __forceinline__ void energy_body(const double* __restrict__ eblk, int nblk,
                                            int need_neutral, Result* __restrict__ res) {
    __shared__ double sh[3][SWG];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < nblk; k += SWG) {
        a += eblk[3 * k];
        b += eblk[3 * k + 1];
        c += eblk[3 * k + 2];
    }
    block_sum3(sh, a, b, c);
    if (threadIdx.x == 0) {
        res->energy = 0.5 * a;
        res->qsum = b;
        res->qabs = c;
        if (need_neutral && fabs(b) > 1e-12 * c) res->status |= RS_NOT_NEUTRAL;
        if (!isfinite(a)) res->status |= RS_NONFINITE;
    }
}

}  // namespace hsma
