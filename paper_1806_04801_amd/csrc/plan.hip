// Preparation step of the HSMA (Sec. II.C, Table I) on the GPU: monitoring
// points, fitting matrix of real solid harmonics, Householder QR, the
// pseudo-inverse R^-1 Q^T, Hannay-Nye surface points and the mapping matrices.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>

#include "hsma_internal.h"

namespace hsma {

// ---------------------------------------------------------------- basis
// Real solid harmonics B_k(r) = (|r|/R0)^n Y_nm, k = n^2 + n + m, with Y the
// orthonormal real spherical harmonics without the Condon-Shortley phase
// (Eq. (harmonic); real form as in Sec. II.C).  Evaluated from Cartesian
// coordinates without trigonometry: with u = r/R0,
//   B_{n,0} = Pi_n^0,  B_{n,m} = sqrt2 Pi_n^m Re (u_x + i u_y)^m,
//   B_{n,-m} = sqrt2 Pi_n^m Im (u_x + i u_y)^m,
// where Pi_n^m(u_z, |u|^2) are the normalized homogeneous Legendre
// polynomials: Pi_0^0 = 1/sqrt(4 pi), Pi_m^m = sqrt((2m+1)/(2m)) Pi_{m-1}^{m-1},
// Pi_{m+1}^m = sqrt(2m+3) u_z Pi_m^m and
// Pi_n^m = a (u_z Pi_{n-1}^m - b |u|^2 Pi_{n-2}^m),
// a = sqrt((4n^2-1)/(n^2-m^2)), b = sqrt(((n-1)^2-m^2)/(4(n-1)^2-1)).
// out[i*ld_pt + (k-k0)*ld_k] = (acc ? out : 0) + sign * B_k for k >= k0.
__global__ void k_basis(const double* __restrict__ pts, int npts, int P, double invR0,
                        double* __restrict__ out, int ld_pt, int ld_k, int k0, double sign,
                        int acc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const double x = pts[3 * i] * invR0, y = pts[3 * i + 1] * invR0, z = pts[3 * i + 2] * invR0;
    const double r2 = x * x + y * y + z * z;
    double* o = out + (size_t)i * ld_pt;
    auto put = [&](int k, double v) {
        if (k < k0) return;
        double* d = o + (size_t)(k - k0) * ld_k;
        *d = acc ? *d + sign * v : sign * v;
    };
    const double sq2 = 1.4142135623730951;
    double pmm = 0.28209479177387814;  // 1/sqrt(4 pi)
    double cm = 1.0, sm = 0.0;         // (x + iy)^m
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            pmm *= sqrt((2.0 * m + 1.0) / (2.0 * m));
            const double cn = cm * x - sm * y;
            sm = cm * y + sm * x;
            cm = cn;
        }
        const double fc = (m == 0) ? 1.0 : sq2 * cm;
        const double fs = sq2 * sm;
        double p2 = pmm;  // n = m
        put(m * m + m + m, p2 * fc);
        if (m > 0) put(m * m + m - m, p2 * fs);
        if (m == P) break;
        double p1 = sqrt(2.0 * m + 3.0) * z * pmm;  // n = m + 1
        {
            const int n = m + 1;
            put(n * n + n + m, p1 * fc);
            if (m > 0) put(n * n + n - m, p1 * fs);
        }
        for (int n = m + 2; n <= P; ++n) {
            const double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
            const double b = sqrt((((double)n - 1.0) * (n - 1.0) - (double)m * m) /
                                  (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
            const double p0 = a * (z * p1 - b * r2 * p2);
            put(n * n + n + m, p0 * fc);
            if (m > 0) put(n * n + n - m, p0 * fs);
            p2 = p1;
            p1 = p0;
        }
    }
}

// Far field evaluated from the fitted series (Eq. (harmonic)) at targets:
// phi = sum_k A_k B_k(r), E = -sum_k A_k grad B_k(r).  The recurrence of
// k_basis is carried with its derivatives: Pi_n^m depends on (u_z, |u|^2), so
// grad Pi = (2 u_x Pr, 2 u_y Pr, Pz + 2 u_z Pr) with Pz = dPi/du_z and
// Pr = dPi/d|u|^2 from the differentiated three-term recurrence, and
// d/du_x (u_x + i u_y)^m = m (u_x + i u_y)^(m-1), d/du_y = i m (u_x + i u_y)^(m-1).
__global__ void __launch_bounds__(256) k_far_direct(const double4* __restrict__ tgt, int nt,
                                                   int nt_pad, int P, double invR0,
                                                   const double* __restrict__ A,
                                                   double* __restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt_pad) return;
    const double4 r = tgt[min(t, nt - 1)];
    const double x = r.x * invR0, y = r.y * invR0, z = r.z * invR0;
    const double rho = x * x + y * y + z * z;
    const double sq2 = 1.4142135623730951;
    double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    double pmm = 0.28209479177387814;
    double cm = 1.0, sm = 0.0, cm1 = 0.0, sm1 = 0.0;  // (x+iy)^m and (x+iy)^(m-1)
    for (int m = 0; m <= P; ++m) {
        if (m > 0) {
            pmm *= sqrt((2.0 * m + 1.0) / (2.0 * m));
            cm1 = cm;
            sm1 = sm;
            const double cn = cm * x - sm * y;
            sm = cm * y + sm * x;
            cm = cn;
        }
        // T = C_m (k = n^2+n+m) and S_m (k = n^2+n-m) with their gradients
        const double fc = (m == 0) ? 1.0 : sq2;
        const double dCx = m * cm1, dCy = -m * sm1, dSx = m * sm1, dSy = m * cm1;
        auto acc = [&](int n, double Pi, double Pz, double Pr) {
            const double dPx = 2.0 * x * Pr, dPy = 2.0 * y * Pr, dPz = Pz + 2.0 * z * Pr;
            const int kc = n * n + n + m;
            const double ac = fc * A[kc];
            phi += ac * Pi * cm;
            gx += ac * (dPx * cm + Pi * dCx);
            gy += ac * (dPy * cm + Pi * dCy);
            gz += ac * (dPz * cm);
            if (m > 0) {
                const double as = sq2 * A[n * n + n - m];
                phi += as * Pi * sm;
                gx += as * (dPx * sm + Pi * dSx);
                gy += as * (dPy * sm + Pi * dSy);
                gz += as * (dPz * sm);
            }
        };
        double p2 = pmm, z2 = 0.0, r2 = 0.0;          // n = m
        acc(m, p2, z2, r2);
        if (m == P) break;
        const double c1 = sqrt(2.0 * m + 3.0);
        double p1 = c1 * z * pmm, z1 = c1 * pmm, r1 = 0.0;  // n = m + 1
        acc(m + 1, p1, z1, r1);
        for (int n = m + 2; n <= P; ++n) {
            const double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
            const double b = sqrt((((double)n - 1.0) * (n - 1.0) - (double)m * m) /
                                  (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
            const double p0 = a * (z * p1 - b * rho * p2);
            const double z0 = a * (p1 + z * z1 - b * rho * z2);
            const double r0 = a * (z * r1 - b * p2 - b * rho * r2);
            acc(n, p0, z0, r0);
            p2 = p1; z2 = z1; r2 = r1;
            p1 = p0; z1 = z0; r1 = r0;
        }
    }
    out[t] = phi;
    out[(size_t)nt_pad + t] = -gx * invR0;
    out[(size_t)2 * nt_pad + t] = -gy * invR0;
    out[(size_t)3 * nt_pad + t] = -gz * invR0;
}

hipError_t launch_far_direct(const double4* tgt, int nt, int nt_pad, int P, double invR0,
                             const double* A, double* out, hipStream_t s) {
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_far_direct, dim3((nt_pad + 255) / 256), dim3(256), 0, s, tgt, nt, nt_pad, P,
                       invR0, A, out);
    return hipGetLastError();
}

hipError_t launch_basis(const double* pts, int npts, int P, double invR0, double* out, int ld_pt,
                        int ld_k, int k0, hipStream_t s) {
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_basis, dim3((npts + 127) / 128), dim3(128), 0, s, pts, npts, P, invR0, out,
                       ld_pt, ld_k, k0, 1.0, 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Householder QR
// Fixed-order block sum (deterministic).
template <int NT>
__device__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Reflector of column j of A (column-major, ld = m): v = x - alpha e_1,
// alpha = -sign(x_0) |x|, stored normalized in V[:, j]; R[j][j] = alpha.
__global__ void __launch_bounds__(1024) k_hh_make(double* __restrict__ A, int m, int n, int j,
                                                 double* __restrict__ V, double* __restrict__ R) {
    __shared__ double sh[1024];
    const double* x = A + (size_t)j * m;
    double s = 0.0;
    for (int i = j + threadIdx.x; i < m; i += 1024) s += x[i] * x[i];
    const double nrm2 = block_sum<1024>(s, sh);
    const double x0 = x[j];
    const double nrm = sqrt(nrm2);
    const double alpha = (x0 >= 0.0) ? -nrm : nrm;
    const double v0 = x0 - alpha;
    const double vn2 = nrm2 - x0 * x0 + v0 * v0;
    const double inv = (vn2 > 0.0) ? 1.0 / sqrt(vn2) : 0.0;
    double* v = V + (size_t)j * m;
    for (int i = threadIdx.x; i < m; i += 1024) {
        double val = 0.0;
        if (i == j) val = v0 * inv;
        else if (i > j) val = x[i] * inv;
        v[i] = val;
    }
    if (threadIdx.x == 0) R[(size_t)j * n + j] = alpha;
}

// Apply I - 2 v v^T (v = V[:, j], rows >= j) to columns c0 + blockIdx.x of B
// (column-major, ld = m).  If R is given, record row j of the result in R.
__global__ void __launch_bounds__(256) k_hh_apply(const double* __restrict__ V, int m, int j,
                                                 double* __restrict__ B, int c0, double* R, int n) {
    __shared__ double sh[256];
    const int c = c0 + blockIdx.x;
    const double* v = V + (size_t)j * m;
    double* b = B + (size_t)c * m;
    double s = 0.0;
    for (int i = j + threadIdx.x; i < m; i += 256) s += v[i] * b[i];
    const double dot = 2.0 * block_sum<256>(s, sh);
    for (int i = j + threadIdx.x; i < m; i += 256) b[i] -= dot * v[i];
    if (R != nullptr && threadIdx.x == 0) {
        __threadfence_block();
        R[(size_t)j * n + c] = b[j];
    }
}

// P = R^-1 Q^T: column i of P solves R p = (row i of Q), by back substitution.
// Q column-major (ld = m), R row-major n x n, P row-major n x m.
__global__ void k_pinv(const double* __restrict__ Q, int m, int n, const double* __restrict__ R,
                       double* __restrict__ P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int r = n - 1; r >= 0; --r) {
        double acc = Q[(size_t)r * m + i];
        for (int c = r + 1; c < n; ++c) acc -= R[(size_t)r * n + c] * P[(size_t)c * m + i];
        P[(size_t)r * m + i] = acc / R[(size_t)r * n + r];
    }
}

__global__ void k_eye(double* Q, int m, int n) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)m * n) return;
    const int c = (int)(idx / m), r = (int)(idx % m);
    Q[idx] = (r == c) ? 1.0 : 0.0;
}

// Mapping rows (Sec. II.B): with B_jk = B_k(R_j) in Wp on entry,
//   Wq[j][k] = (w_j / (4 pi Rs)) n_k B_jk   (surface charge sigma = dPhi_out/dn)
//   Wp[j][k] = -(w_j / (4 pi)) B_jk         (surface dipole strength, along n_j)
__global__ void k_map_rows(double* __restrict__ Wq, double* __restrict__ Wp,
                           const double* __restrict__ w, int M, int nb, double Rs) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)M * nb) return;
    const int j = (int)(idx / nb), k = (int)(idx % nb);
    int n = 0;
    while ((n + 1) * (n + 1) <= k) ++n;
    const double B = Wp[idx];
    const double c = w[j] / (4.0 * M_PI);
    Wq[idx] = c * n * B / Rs;
    Wp[idx] = -c * B;
}

// ---------------------------------------------------------------- host geometry
static uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double unit_double(uint64_t z) { return (double)(z >> 11) * (1.0 / 9007199254740992.0); }

// Monitoring points: Fibonacci spiral on the circumsphere (latitude
// asin((2i-1)/K - 1), azimuth 2 pi i w, w the golden ratio conjugate) with
// twins x - L floor(x/L + 1/2) (Sec. II.A, periodic) or without (dielectric
// box: the far images themselves are fitted there); or points on the cube
// faces, point i on face i mod 6, tangential coordinates from SplitMix64.
static void monitoring(hsma_plan_s* pl) {
    const int K = pl->K;
    const double L = pl->L;
    if (pl->img == IMG_PERIODIC || pl->img == IMG_DIELECTRIC) {
        const bool twins = pl->img == IMG_PERIODIC;
        pl->chk.assign((size_t)(twins ? 6 : 3) * K, 0.0);
        const double w = (std::sqrt(5.0) - 1.0) / 2.0;
        for (int i = 1; i <= K; ++i) {
            const double s = (2.0 * i - 1.0) / K - 1.0;
            const double lat = std::asin(s);
            const double az = 2.0 * M_PI * i * w;
            double* x = &pl->chk[(size_t)3 * (i - 1)];
            x[0] = pl->R0 * std::cos(lat) * std::cos(az);
            x[1] = pl->R0 * std::cos(lat) * std::sin(az);
            x[2] = pl->R0 * std::sin(lat);
            if (!twins) continue;
            double* t = &pl->chk[(size_t)3 * (K + i - 1)];
            for (int a = 0; a < 3; ++a) t[a] = x[a] - L * std::floor(x[a] / L + 0.5);
        }
    } else {
        pl->chk.assign((size_t)3 * K, 0.0);
        for (int i = 0; i < K; ++i) {
            const double u = unit_double(splitmix64(pl->desc.seed, 2ull * i));
            const double v = unit_double(splitmix64(pl->desc.seed, 2ull * i + 1));
            const int f = i % 6, axis = f / 2;
            const double side = (f % 2 == 0) ? -1.0 : 1.0;
            const int t0 = (axis == 0) ? 1 : 0, t1 = (axis == 2) ? 1 : 2;
            double* x = &pl->chk[(size_t)3 * i];
            x[axis] = side * 0.5 * L;
            x[t0] = L * (u - 0.5);
            x[t1] = L * (v - 0.5);
        }
    }
}

// Hannay-Nye Fibonacci quadrature on the sphere R_s (Sec. II.B): F1 < F2
// successive Fibonacci numbers with 2(F2+1) nearest to M; for j = 0..F2,
// z_j = -1 + 2j/F2, cos(theta_j) = z_j + sin(pi z_j)/pi, phi_j = pi j F1/F2,
// points at phi_j and phi_j + pi with weight (2 pi Rs^2/F2)(1 + cos(pi z_j)).
static void surface_points(hsma_plan_s* pl) {
    const int M = pl->desc.M;
    long a = 1, b = 2, bf1 = 1, bf2 = 2;
    long best = -1;
    for (;;) {
        const long cnt = 2 * (b + 1);
        const long d = std::labs(cnt - M);
        if (best < 0 || d <= best) { best = d; bf1 = a; bf2 = b; }
        if (cnt > M && d > best) break;
        const long nb = a + b;
        a = b;
        b = nb;
        if (b > 10000000) break;
    }
    pl->F1 = (int)bf1;
    pl->F2 = (int)bf2;
    pl->M = 2 * (pl->F2 + 1);
    pl->spts.assign((size_t)3 * pl->M, 0.0);
    pl->swts.assign(pl->M, 0.0);
    const double Rs = pl->Rs;
    for (int j = 0; j <= pl->F2; ++j) {
        const double z = -1.0 + 2.0 * j / pl->F2;
        double ct = z + std::sin(M_PI * z) / M_PI;
        ct = std::fmax(-1.0, std::fmin(1.0, ct));
        const double st = std::sqrt(std::fmax(0.0, 1.0 - ct * ct));
        const double ph = M_PI * j * pl->F1 / pl->F2;
        const double wt = 2.0 * M_PI * Rs * Rs / pl->F2 * (1.0 + std::cos(M_PI * z));
        for (int e = 0; e < 2; ++e) {
            const double p = ph + e * M_PI;
            double* s = &pl->spts[(size_t)3 * (2 * j + e)];
            s[0] = Rs * st * std::cos(p);
            s[1] = Rs * st * std::sin(p);
            s[2] = Rs * ct;
            pl->swts[2 * j + e] = wt;
        }
    }
}

int far_shell_count(double gamma, double tol) {
    const double g = std::fabs(gamma);
    if (g == 0.0) return 1;
    const double c = 1.0 + 2.0 * g / (1.0 - g);
    int S = 2;
    while (S < 400 && 6.0 * c * c * std::pow(g, S + 1) / ((1.0 - g) * (S + 0.5 - std::sqrt(3.0) / 2.0)) > tol)
        ++S;
    return S;
}

// ---------------------------------------------------------------- plan build
template <typename Tp>
static hsma_status dmalloc(Tp** p, size_t n, size_t* total) {
    if (hipMalloc((void**)p, n * sizeof(Tp)) != hipSuccess) {
        *p = nullptr;
        return fail(HSMA_E_NOMEM, "hipMalloc failed for plan storage");
    }
    *total += n * sizeof(Tp);
    return HSMA_OK;
}

hsma_status build_plan(hsma_plan_s* pl) {
    HSMA_HIP(hipGetDevice(&pl->device));
    hipDeviceProp_t prop;
    HSMA_HIP(hipGetDeviceProperties(&prop, pl->device));
    pl->ncu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    monitoring(pl);
    surface_points(pl);
    const int K = pl->K, nb = pl->nb, nu = pl->nu, M = pl->M;
    pl->nchk = (pl->img == IMG_PERIODIC) ? 2 * K : K;
    hipStream_t s = nullptr;
    size_t tot = 0;
    hsma_status st;
    // temporaries
    double *d_pts = nullptr, *d_F = nullptr, *d_V = nullptr, *d_R = nullptr, *d_Q = nullptr,
           *d_w = nullptr;
    auto cleanup = [&]() {
        hipFree(d_pts); hipFree(d_F); hipFree(d_V); hipFree(d_R); hipFree(d_Q); hipFree(d_w);
    };
    size_t tmp = 0;
    if ((st = dmalloc(&d_pts, (size_t)3 * std::max(pl->nchk, M), &tmp)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&d_F, (size_t)K * nu, &tmp)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&d_V, (size_t)K * nu, &tmp)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&d_R, (size_t)nu * nu, &tmp)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&d_Q, (size_t)K * nu, &tmp)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&d_w, (size_t)M, &tmp)) != HSMA_OK) { cleanup(); return st; }
    // resident
    if ((st = dmalloc(&pl->d_P, (size_t)nu * K, &tot)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&pl->d_Wq, (size_t)M * nb, &tot)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&pl->d_Wp, (size_t)M * nb, &tot)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&pl->d_spos, (size_t)M * 4, &tot)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&pl->d_chk64, (size_t)pl->nchk, &tot)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&pl->d_chk32, (size_t)pl->nchk, &tot)) != HSMA_OK) { cleanup(); return st; }
    if ((st = dmalloc(&pl->d_chk_order, (size_t)pl->nchk, &tot)) != HSMA_OK) { cleanup(); return st; }
    pl->bytes = tot;

#define PLAN_HIP(call)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            cleanup();                                                                      \
            return fail(HSMA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
        }                                                                                   \
    } while (0)

    const double invR0 = 1.0 / pl->R0;
    const int k0 = nb - nu;  // 1 for periodic (A_00 dropped), 0 otherwise
    // fitting matrix F (column-major K x nu): B(x) or B(x) - B(x~)
    PLAN_HIP(hipMemcpy(d_pts, pl->chk.data(), sizeof(double) * 3 * pl->nchk, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_basis, dim3((K + 127) / 128), dim3(128), 0, s, d_pts, K, pl->p, invR0, d_F,
                       1, K, k0, 1.0, 0);
    PLAN_HIP(hipGetLastError());
    if (pl->img == IMG_PERIODIC) {
        hipLaunchKernelGGL(k_basis, dim3((K + 127) / 128), dim3(128), 0, s, d_pts + 3 * (size_t)K,
                           K, pl->p, invR0, d_F, 1, K, k0, -1.0, 1);
        PLAN_HIP(hipGetLastError());
    }
    // check-point records (targets of the right-hand-side kernel)
    {
        std::vector<double> c4((size_t)4 * pl->nchk);
        for (int i = 0; i < pl->nchk; ++i) {
            c4[4 * i] = pl->chk[3 * i];
            c4[4 * i + 1] = pl->chk[3 * i + 1];
            c4[4 * i + 2] = pl->chk[3 * i + 2];
            c4[4 * i + 3] = 0.0;
        }
        PLAN_HIP(hipMemcpy(pl->d_chk64, c4.data(), sizeof(double) * 4 * pl->nchk, hipMemcpyHostToDevice));
        PLAN_HIP(launch_make_rec32(pl->d_chk64, pl->nchk, pl->L, pl->d_chk32, s));
        // the points in Morton order of position over their bounding box, so
        // that the tree right-hand side visits neighbouring points together
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = 0; i < pl->nchk; ++i)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], pl->chk[3 * i + a]);
                hi[a] = std::max(hi[a], pl->chk[3 * i + a]);
            }
        std::vector<std::pair<uint64_t, int>> key((size_t)pl->nchk);
        for (int i = 0; i < pl->nchk; ++i) {
            uint64_t k = 0;
            for (int a = 0; a < 3; ++a) {
                const double w = hi[a] > lo[a] ? (pl->chk[3 * i + a] - lo[a]) / (hi[a] - lo[a]) : 0.0;
                const uint64_t q = (uint64_t)std::min(1048575.0, std::max(0.0, w * 1048576.0));
                for (int b = 0; b < 20; ++b) k |= ((q >> b) & 1u) << (3 * b + 2 - a);
            }
            key[i] = {k, i};
        }
        std::sort(key.begin(), key.end());
        std::vector<int> ord((size_t)pl->nchk);
        for (int i = 0; i < pl->nchk; ++i) ord[i] = key[i].second;
        PLAN_HIP(hipMemcpy(pl->d_chk_order, ord.data(), sizeof(int) * pl->nchk, hipMemcpyHostToDevice));
    }
    // Householder QR of F
    PLAN_HIP(hipMemset(d_R, 0, sizeof(double) * nu * nu));
    for (int j = 0; j < nu; ++j) {
        hipLaunchKernelGGL(k_hh_make, dim3(1), dim3(1024), 0, s, d_F, K, nu, j, d_V, d_R);
        if (j + 1 < nu)
            hipLaunchKernelGGL(k_hh_apply, dim3(nu - j - 1), dim3(256), 0, s, d_V, K, j, d_F, j + 1,
                               d_R, nu);
    }
    PLAN_HIP(hipGetLastError());
    // thin Q = H_0 ... H_{nu-1} [I; 0]
    hipLaunchKernelGGL(k_eye, dim3((unsigned)(((size_t)K * nu + 255) / 256)), dim3(256), 0, s, d_Q, K, nu);
    for (int j = nu - 1; j >= 0; --j)
        hipLaunchKernelGGL(k_hh_apply, dim3(nu - j), dim3(256), 0, s, d_V, K, j, d_Q, j,
                           (double*)nullptr, nu);
    PLAN_HIP(hipGetLastError());
    // rank check on diag(R)
    {
        std::vector<double> Rh((size_t)nu * nu);
        PLAN_HIP(hipMemcpy(Rh.data(), d_R, sizeof(double) * nu * nu, hipMemcpyDeviceToHost));
        double mx = 0.0, mn = INFINITY;
        for (int j = 0; j < nu; ++j) {
            const double d = std::fabs(Rh[(size_t)j * nu + j]);
            mx = std::fmax(mx, d);
            mn = std::fmin(mn, d);
        }
        if (!(mn > 1e-13 * mx)) {
            cleanup();
            return fail(HSMA_E_ILLCOND, "fitting matrix is numerically rank deficient");
        }
    }
    hipLaunchKernelGGL(k_pinv, dim3((K + 63) / 64), dim3(64), 0, s, d_Q, K, nu, d_R, pl->d_P);
    PLAN_HIP(hipGetLastError());
    // surface points and mapping rows (row-major M x nb)
    PLAN_HIP(hipMemcpy(d_pts, pl->spts.data(), sizeof(double) * 3 * M, hipMemcpyHostToDevice));
    PLAN_HIP(hipMemcpy(d_w, pl->swts.data(), sizeof(double) * M, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_basis, dim3((M + 127) / 128), dim3(128), 0, s, d_pts, M, pl->p, invR0,
                       pl->d_Wp, nb, 1, 0, 1.0, 0);
    hipLaunchKernelGGL(k_map_rows, dim3((unsigned)(((size_t)M * nb + 255) / 256)), dim3(256), 0, s,
                       pl->d_Wq, pl->d_Wp, d_w, M, nb, pl->Rs);
    PLAN_HIP(hipGetLastError());
    {
        std::vector<double> s4((size_t)4 * M);
        for (int j = 0; j < M; ++j) {
            s4[4 * j] = pl->spts[3 * j];
            s4[4 * j + 1] = pl->spts[3 * j + 1];
            s4[4 * j + 2] = pl->spts[3 * j + 2];
            s4[4 * j + 3] = 0.0;
        }
        PLAN_HIP(hipMemcpy(pl->d_spos, s4.data(), sizeof(double) * 4 * M, hipMemcpyHostToDevice));
    }
    PLAN_HIP(hipDeviceSynchronize());
#undef PLAN_HIP
    cleanup();
    return HSMA_OK;
}

void free_plan(hsma_plan_s* pl) {
    hipFree(pl->d_P);
    hipFree(pl->d_Wq);
    hipFree(pl->d_Wp);
    hipFree(pl->d_spos);
    hipFree(pl->d_chk64);
    hipFree(pl->d_chk32);
    hipFree(pl->d_chk_order);
    hipFree(pl->host_buf);
}

}  // namespace hsma
