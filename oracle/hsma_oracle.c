/*
 * HSMA oracle: plain double-precision pair sums (test infrastructure only).
 *
 * This file is part of the slow, obviously-correct CPU oracle used to check
 * the GPU library.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may call it.  It shares no code with the GPU library.
 *
 * Notation follows Zhao, Liang & Xu, "Harmonic surface mapping algorithm for
 * fast electrostatic sums" (arXiv:1806.04801):
 *   - Coulomb potential in Gaussian units, Phi(r) = sum_j q_j / |r_j - r|
 *     (Sec. II, Eq. (sum)).
 *   - Images of a source r_j in the 3x3x3 block of boxes around the central
 *     box, k in {-1,0,1}^3:
 *       periodic  : r_j + kL, charge q_j                       (Sec. II, periodic sum)
 *       metallic  : (-1)^k o r_j + kL, charge (-1)^{|k|} q_j   (Eq. (diel), gamma = -1)
 *       dielectric: (-1)^k o r_j + kL, charge gamma^{|k|} q_j   (Eq. (diel), |gamma| < 1)
 *     These are the charges "inside the auxiliary sphere" (Sec. II.A).
 *   - Dielectric boxes also need the images beyond the block, shells
 *     2 <= max|k_a| <= S of the same series (the far part of Eq. (diel)).
 * Coordinates are centred: the central box is [-L/2, L/2]^3.
 * Every loop is a plain double loop in the order of the definition; OpenMP
 * only splits the outer loop over evaluation points.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>

#define BC_PERIODIC 0
#define BC_METALLIC 1
#define BC_DIELECTRIC 3

/* Image k of the source at r for any integer k; returns its weight s_k:
 *   periodic  : r + kL, weight 1
 *   metallic  : (-1)^{k_a} r_a + k_a L per axis, weight (-1)^{|k|}
 *   dielectric: the same positions, weight gamma^{|k|}
 * (|k| = |k_x| + |k_y| + |k_z|, one factor per reflection). */
static double image_of(int bc, double L, double gamma, const int k[3], const double r[3],
                       double out[3])
{
    double w = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (bc == BC_PERIODIC) {
            out[a] = r[a] + k[a] * L;
        } else {
            double refl = (k[a] % 2 == 0) ? r[a] : -r[a];
            out[a] = refl + k[a] * L;
            int n = k[a] < 0 ? -k[a] : k[a];
            for (int t = 0; t < n; ++t) w *= (bc == BC_METALLIC) ? -1.0 : gamma;
        }
    }
    return w;
}

/*
 * Potential of all 27 images of all sources at arbitrary points:
 *   phi[i] = sum_j sum_k s_k q_j / |p_i - I_k(r_j)|
 * src: ns x 4 (x, y, z, q) centred; pts: np x 3.
 * This is Phi_in at the monitoring points (Sec. II.A, the right-hand side of
 * the least-squares system).
 */
void orc_potential_at(int bc, double L, double gamma, const double *src, long ns,
                      const double *pts, long np, double *phi)
{
    #pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < np; ++i) {
        const double *p = pts + 3 * i;
        double acc = 0.0;
        for (long j = 0; j < ns; ++j) {
            const double *r = src + 4 * j;
            for (int kx = -1; kx <= 1; ++kx)
            for (int ky = -1; ky <= 1; ++ky)
            for (int kz = -1; kz <= 1; ++kz) {
                int k[3] = {kx, ky, kz};
                double im[3];
                double s = image_of(bc, L, gamma, k, r, im);
                double dx = p[0] - im[0], dy = p[1] - im[1], dz = p[2] - im[2];
                acc += s * r[3] / sqrt(dx * dx + dy * dy + dz * dz);
            }
        }
        phi[i] = acc;
    }
}

/*
 * Near-field potential and field at source targets (Sec. II.C, update step:
 * contribution of the N_s charges inside the sphere):
 *   phi_i = sum_{(j,k) != (i,0)} s_k q_j / |r_i - I_k(r_j)|
 *   E_i   = -grad phi_i = sum_{(j,k) != (i,0)} s_k q_j (r_i - I_k(r_j)) / |.|^3
 * Only the bare self term (j = i, k = 0) is left out; self-images count.
 * tidx: nt indices of the targets among the sources.
 */
void orc_near(int bc, double L, double gamma, const double *src, long ns,
              const long *tidx, long nt, double *phi, double *field)
{
    #pragma omp parallel for schedule(dynamic, 4)
    for (long t = 0; t < nt; ++t) {
        long i = tidx[t];
        const double *ri = src + 4 * i;
        double ap = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (long j = 0; j < ns; ++j) {
            const double *r = src + 4 * j;
            for (int kx = -1; kx <= 1; ++kx)
            for (int ky = -1; ky <= 1; ++ky)
            for (int kz = -1; kz <= 1; ++kz) {
                if (j == i && kx == 0 && ky == 0 && kz == 0) continue;
                int k[3] = {kx, ky, kz};
                double im[3];
                double s = image_of(bc, L, gamma, k, r, im);
                double dx = ri[0] - im[0], dy = ri[1] - im[1], dz = ri[2] - im[2];
                double d = sqrt(dx * dx + dy * dy + dz * dz);
                double qs = s * r[3];
                ap += qs / d;
                double c = qs / (d * d * d);
                ex += c * dx; ey += c * dy; ez += c * dz;
            }
        }
        phi[t] = ap;
        field[3 * t + 0] = ex; field[3 * t + 1] = ey; field[3 * t + 2] = ez;
    }
}

/*
 * Potential and field of the surface images at arbitrary points (Sec. II.B):
 * a point charge Q_j and a point dipole p_j at R_j (the dipole is the exact
 * limit of the central difference of Eq. (cd)).
 *   phi(r) = sum_j Q_j/|d| + p_j.d/|d|^3,            d = r - R_j
 *   E(r)   = sum_j Q_j d/|d|^3 + 3 (p_j.d) d/|d|^5 - p_j/|d|^3
 * surf: m x 7 (X, Y, Z, Q, px, py, pz); pts: np x 3.
 */
void orc_surface(const double *pts, long np, const double *surf, long m,
                 double *phi, double *field)
{
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < np; ++i) {
        const double *p = pts + 3 * i;
        double ap = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (long j = 0; j < m; ++j) {
            const double *s = surf + 7 * j;
            double dx = p[0] - s[0], dy = p[1] - s[1], dz = p[2] - s[2];
            double d2 = dx * dx + dy * dy + dz * dz;
            double d = sqrt(d2);
            double d3 = d2 * d, d5 = d3 * d2;
            double pd = s[4] * dx + s[5] * dy + s[6] * dz;
            ap += s[3] / d + pd / d3;
            ex += s[3] * dx / d3 + 3.0 * pd * dx / d5 - s[4] / d3;
            ey += s[3] * dy / d3 + 3.0 * pd * dy / d5 - s[5] / d3;
            ez += s[3] * dz / d3 + 3.0 * pd * dz / d5 - s[6] / d3;
        }
        phi[i] = ap;
        field[3 * i + 0] = ex; field[3 * i + 1] = ey; field[3 * i + 2] = ez;
    }
}

/*
 * Potential and field of plain point charges (no images) at points:
 *   phi(r) = sum_j Q_j / |r - R_j|,  E(r) = sum_j Q_j (r - R_j)/|r - R_j|^3
 * chg: m x 4 (X, Y, Z, Q).  Used for the paper-literal surface images
 * (charge layers on the spheres R_s and R_s +- dr/2, Eq. (integrals)) and for
 * the source response at the surface points needed by the adjoint.
 */
void orc_charges(const double *pts, long np, const double *chg, long m,
                 double *phi, double *field)
{
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < np; ++i) {
        const double *p = pts + 3 * i;
        double ap = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (long j = 0; j < m; ++j) {
            const double *s = chg + 4 * j;
            double dx = p[0] - s[0], dy = p[1] - s[1], dz = p[2] - s[2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            ap += s[3] / d;
            double c = s[3] / (d * d * d);
            ex += c * dx; ey += c * dy; ez += c * dz;
        }
        phi[i] = ap;
        field[3 * i + 0] = ex; field[3 * i + 1] = ey; field[3 * i + 2] = ez;
    }
}

/*
 * Adjoint of the right-hand side.  With weights lam_i at points p_i, for each
 * source position r_j (unit charge):
 *   g_j  = sum_i lam_i sum_k s_k / |p_i - I_k(r_j)|
 *   dg_j = d g_j / d r_j = sum_i lam_i sum_k s_k S_k (p_i - I_k(r_j)) / |.|^3
 * where I_k(r) = S_k r + kL (S_k = identity for periodic, the reflection
 * diag((-1)^{k_a}) for metallic).
 * pos: ns x 3 centred; pts: np x 3.
 */
void orc_check_adjoint(int bc, double L, double gamma, const double *pos, long ns,
                       const double *pts, const double *lam, long np,
                       double *g, double *dg)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (long j = 0; j < ns; ++j) {
        const double *r = pos + 3 * j;
        double ag = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        for (long i = 0; i < np; ++i) {
            const double *p = pts + 3 * i;
            for (int kx = -1; kx <= 1; ++kx)
            for (int ky = -1; ky <= 1; ++ky)
            for (int kz = -1; kz <= 1; ++kz) {
                int k[3] = {kx, ky, kz};
                double im[3];
                double s = image_of(bc, L, gamma, k, r, im);
                double dx = p[0] - im[0], dy = p[1] - im[1], dz = p[2] - im[2];
                double d = sqrt(dx * dx + dy * dy + dz * dz);
                ag += lam[i] * s / d;
                double c = lam[i] * s / (d * d * d);
                /* S_k applied to d: reflected axes flip sign (metallic only) */
                double sx = (bc != BC_PERIODIC && kx != 0) ? -1.0 : 1.0;
                double sy = (bc != BC_PERIODIC && ky != 0) ? -1.0 : 1.0;
                double sz = (bc != BC_PERIODIC && kz != 0) ? -1.0 : 1.0;
                gx += c * sx * dx; gy += c * sy * dy; gz += c * sz * dz;
            }
        }
        g[j] = ag;
        dg[3 * j + 0] = gx; dg[3 * j + 1] = gy; dg[3 * j + 2] = gz;
    }
}

/*
 * Near-field potential and field at source targets from an explicit list of
 * charges (image positions and charges, img: m x 4), where entry j belongs to
 * source owner[j] and center[j] != 0 marks the unshifted copy of that source.
 * Only the bare self term (owner == target, center) is left out.  Used for the
 * paper-literal near set "all charges within the auxiliary sphere"
 * (Sec. II.A).
 */
void orc_near_explicit(const double *src, const long *tidx, long nt, const double *img,
                       const long *owner, const int *center, long m, double *phi, double *field)
{
    #pragma omp parallel for schedule(dynamic, 4)
    for (long t = 0; t < nt; ++t) {
        long i = tidx[t];
        const double *ri = src + 4 * i;
        double ap = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (long j = 0; j < m; ++j) {
            if (owner[j] == i && center[j]) continue;
            const double *s = img + 4 * j;
            double dx = ri[0] - s[0], dy = ri[1] - s[1], dz = ri[2] - s[2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            ap += s[3] / d;
            double c = s[3] / (d * d * d);
            ex += c * dx; ey += c * dy; ez += c * dz;
        }
        phi[t] = ap;
        field[3 * t + 0] = ex; field[3 * t + 1] = ey; field[3 * t + 2] = ez;
    }
}

/*
 * The far part of the dielectric image series (Eq. (diel)) at points: every
 * image of every source in the shells 2 <= max_a |k_a| <= S,
 *   phi[i] = sum_j sum_k gamma^{|k|} q_j / |p_i - I_k(r_j)|.
 * These images lie outside the 3x3x3 block, at least 1.5 L from the centre,
 * so the sum is harmonic in the ball of radius 1.5 L (the far field that the
 * least squares fits for a dielectric box).
 */
void orc_far_shells(double L, double gamma, const double *src, long ns,
                    const double *pts, long np, int S, double *phi)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < np; ++i) {
        const double *p = pts + 3 * i;
        double acc = 0.0;
        for (long j = 0; j < ns; ++j) {
            const double *r = src + 4 * j;
            for (int kx = -S; kx <= S; ++kx)
            for (int ky = -S; ky <= S; ++ky)
            for (int kz = -S; kz <= S; ++kz) {
                int m = abs(kx) > abs(ky) ? abs(kx) : abs(ky);
                m = m > abs(kz) ? m : abs(kz);
                if (m < 2) continue;
                int k[3] = {kx, ky, kz};
                double im[3];
                double w = image_of(BC_DIELECTRIC, L, gamma, k, r, im);
                double dx = p[0] - im[0], dy = p[1] - im[1], dz = p[2] - im[2];
                acc += w * r[3] / sqrt(dx * dx + dy * dy + dz * dz);
            }
        }
        phi[i] = acc;
    }
}

/*
 * The image series truncated at shells max_a |k_a| <= S, evaluated at source
 * targets without any splitting (a reference for the whole method):
 *   phi_t = sum_{(j,k) != (i,0)} s_k q_j / |r_i - I_k(r_j)|,  i = tidx[t]
 *   E_t   = sum_{(j,k) != (i,0)} s_k q_j (r_i - I_k(r_j)) / |.|^3
 * (weights and positions of image_of; images held fixed for the field).
 */
void orc_image_series(int bc, double L, double gamma, const double *src, long ns,
                      const long *tidx, long nt, int S, double *phi, double *field)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < nt; ++t) {
        long i = tidx[t];
        const double *ri = src + 4 * i;
        double acc = 0.0, ex = 0.0, ey = 0.0, ez = 0.0;
        for (long j = 0; j < ns; ++j) {
            const double *r = src + 4 * j;
            for (int kx = -S; kx <= S; ++kx)
            for (int ky = -S; ky <= S; ++ky)
            for (int kz = -S; kz <= S; ++kz) {
                if (j == i && kx == 0 && ky == 0 && kz == 0) continue;
                int k[3] = {kx, ky, kz};
                double im[3];
                double w = image_of(bc, L, gamma, k, r, im);
                double dx = ri[0] - im[0], dy = ri[1] - im[1], dz = ri[2] - im[2];
                double d = sqrt(dx * dx + dy * dy + dz * dz);
                acc += w * r[3] / d;
                double c = w * r[3] / (d * d * d);
                ex += c * dx; ey += c * dy; ez += c * dz;
            }
        }
        phi[t] = acc;
        field[3 * t + 0] = ex; field[3 * t + 1] = ey; field[3 * t + 2] = ez;
    }
}
