// C ABI of the HSMA library: argument checks, plans, host and device entry
// points, kernel timing.
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hsma_internal.h"
#include "solve.h"

namespace hsma {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

hsma_status fail(hsma_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

// ---------------------------------------------------------------- timing
struct TimingRec {
    int cls;
    hipEvent_t a, b;
};
static std::mutex g_tmu;
static bool g_timing = false;
static std::vector<TimingRec> g_trecs;
static std::vector<hipEvent_t> g_tpool;
static thread_local hipEvent_t g_pending[3] = {nullptr, nullptr, nullptr};

static hipEvent_t take_event() {
    if (!g_tpool.empty()) {
        hipEvent_t e = g_tpool.back();
        g_tpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void timing_begin(int cls, hipStream_t s) {
    if (!g_timing) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) == hipSuccess) g_pending[cls] = e;
}

void timing_end(int cls, hipStream_t s) {
    if (!g_timing || g_pending[cls] == nullptr) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) == hipSuccess) g_trecs.push_back({cls, g_pending[cls], e});
    g_pending[cls] = nullptr;
}

}  // namespace hsma

using namespace hsma;

extern "C" {

const char* hsma_status_string(int st) {
    switch (st) {
        case HSMA_OK: return "ok";
        case HSMA_E_INVALID: return "invalid argument";
        case HSMA_E_NOT_NEUTRAL: return "system not neutral";
        case HSMA_E_OUT_OF_BOX: return "position outside the box";
        case HSMA_E_COINCIDENT: return "two charges at the same position";
        case HSMA_E_NOMEM: return "out of device memory or workspace too small";
        case HSMA_E_DEVICE: return "HIP runtime error";
        case HSMA_E_ILLCOND: return "fitting matrix rank deficient";
        case HSMA_E_NONFINITE: return "non-finite result";
        default: return "unknown status";
    }
}

const char* hsma_last_error(void) { return g_last_error.c_str(); }

int hsma_version(void) { return 6; }

hsma_status hsma_plan_create_ex(const hsma_plan_desc* d, hsma_plan* out) {
    if (d == nullptr || out == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    *out = nullptr;
    if (!(d->L > 0.0) || !std::isfinite(d->L)) return fail(HSMA_E_INVALID, "L must be > 0");
    if (d->bc < 0 || d->bc > 3) return fail(HSMA_E_INVALID, "unknown boundary condition");
    const bool diel = d->bc == HSMA_BC_DIELECTRIC;
    if (diel) {
        if (!(std::fabs(d->gamma) < 1.0)) return fail(HSMA_E_INVALID, "dielectric box needs |gamma| < 1");
        if (d->precision != HSMA_FP64)
            return fail(HSMA_E_INVALID, "the dielectric box runs in double precision only");
        if (d->near_mode != HSMA_NEAR_BLOCK && d->near_mode != HSMA_NEAR_TREE)
            return fail(HSMA_E_INVALID, "the dielectric box uses the block near set (direct or tree)");
        if (d->far_shells < 0 || d->far_shells > 400)
            return fail(HSMA_E_INVALID, "far_shells must be in [0, 400]");
    }
    if (d->p < 1 || d->p > 40) return fail(HSMA_E_INVALID, "p must be in [1, 40]");
    if (d->precision != HSMA_FP64 && d->precision != HSMA_FP32_COMP)
        return fail(HSMA_E_INVALID, "unknown precision");
    const double R0 = std::sqrt(3.0) * d->L / 2.0;
    if (!(d->R > R0) || !std::isfinite(d->R))
        return fail(HSMA_E_INVALID, "R must exceed the circumsphere radius sqrt(3) L / 2");
    const int nb = (d->p + 1) * (d->p + 1);
    const int nu = (d->bc == HSMA_BC_METALLIC || diel) ? nb : nb - 1;
    if (d->K < nu || d->K > (1 << 24)) return fail(HSMA_E_INVALID, "K must be >= number of unknowns");
    if (d->M < 4 || d->M > (1 << 22)) return fail(HSMA_E_INVALID, "M out of range");
    if (d->near_mode != HSMA_NEAR_BLOCK && d->near_mode != HSMA_NEAR_SPHERE &&
        d->near_mode != HSMA_NEAR_TREE)
        return fail(HSMA_E_INVALID, "unknown near mode");
    if (d->near_mode == HSMA_NEAR_TREE) {
        if (d->tree_min_n < 0) return fail(HSMA_E_INVALID, "tree_min_n must be >= 0");
        if (d->tree_order < 0 || d->tree_order > 20)
            return fail(HSMA_E_INVALID, "tree_order must be in [0, 20]");
    }
    if (d->far_mode != HSMA_FAR_SURFACE && d->far_mode != HSMA_FAR_DIRECT)
        return fail(HSMA_E_INVALID, "unknown far-field mode");
    if (d->dipole_mode != HSMA_DIPOLE_EXACT && d->dipole_mode != HSMA_DIPOLE_LAYERS)
        return fail(HSMA_E_INVALID, "unknown dipole mode");
    if (d->dipole_mode == HSMA_DIPOLE_LAYERS && !(d->dr < 0.5 * (d->R - std::sqrt(3.0) * d->L / 2.0)))
        return fail(HSMA_E_INVALID, "layer spacing dr too large for R");
    if (d->near_mode == HSMA_NEAR_SPHERE && d->R > 12.0 * d->L)
        return fail(HSMA_E_INVALID, "sphere near set limited to R <= 12 L");
    hsma_plan_s* pl = new (std::nothrow) hsma_plan_s();
    if (pl == nullptr) return fail(HSMA_E_NOMEM, "host allocation failed");
    pl->desc = *d;
    pl->bc = d->bc;
    pl->img = (d->bc == HSMA_BC_METALLIC) ? IMG_METALLIC : diel ? IMG_DIELECTRIC : IMG_PERIODIC;
    if (diel) {
        pl->gamma = d->gamma;
        pl->far_shells = d->far_shells > 0 ? d->far_shells : far_shell_count(d->gamma, 1e-13);
    }
    pl->p = d->p;
    pl->nb = nb;
    pl->nu = nu;
    pl->K = d->K;
    pl->L = d->L;
    pl->R0 = R0;
    pl->Rs = d->R;
    pl->precision = d->precision;
    pl->near_mode = d->near_mode;
    pl->dipole_mode = d->dipole_mode;
    pl->far_mode = d->far_mode;
    pl->dr = d->dr > 0.0 ? d->dr : 1e-5 * d->R;
    pl->tree_order = d->near_mode == HSMA_NEAR_TREE ? (d->tree_order > 0 ? d->tree_order : 16) : 0;
    pl->tree_min_n = d->near_mode != HSMA_NEAR_TREE ? 0
                     : d->tree_min_n > 0                ? d->tree_min_n
                     : d->precision == HSMA_FP64         ? 16384
                                                         : 24576;
    if (pl->near_mode == HSMA_NEAR_SPHERE) {
        // candidates |k_a| <= kr; a source has at most as many images inside the
        // sphere as there are shifted boxes that reach it
        pl->kr = (int)std::ceil(d->R / d->L + 0.5);
        int cnt = 0;
        for (int a = -pl->kr; a <= pl->kr; ++a)
            for (int b = -pl->kr; b <= pl->kr; ++b)
                for (int c = -pl->kr; c <= pl->kr; ++c) {
                    auto gap = [&](int k) { double g = std::fabs((double)k) - 0.5; return g > 0 ? g * d->L : 0.0; };
                    const double d2 = gap(a) * gap(a) + gap(b) * gap(b) + gap(c) * gap(c);
                    if (d2 < d->R * d->R) ++cnt;
                }
        pl->maxper = cnt;
    }
    hsma_status st = build_plan(pl);
    if (st != HSMA_OK) {
        free_plan(pl);
        delete pl;
        return st;
    }
    if (pl->M < 2 * nb) {
        free_plan(pl);
        delete pl;
        return fail(HSMA_E_INVALID, "too few surface points for the degree (M_eff < 2 N_b)");
    }
    *out = pl;
    return HSMA_OK;
}

hsma_status hsma_plan_create(double L, int bc, int p, int M, int K, double R, hsma_plan* out) {
    hsma_plan_desc d;
    std::memset(&d, 0, sizeof(d));
    d.L = L;
    d.bc = bc;
    d.p = p;
    d.M = M;
    d.K = K;
    d.R = R;
    d.precision = HSMA_FP64;
    d.seed = 12345;
    d.near_mode = HSMA_NEAR_BLOCK;
    d.dipole_mode = HSMA_DIPOLE_EXACT;
    d.dr = 0.0;
    d.far_mode = HSMA_FAR_SURFACE;
    return hsma_plan_create_ex(&d, out);
}

void hsma_plan_destroy(hsma_plan pl) {
    if (pl == nullptr) return;
    free_plan(pl);
    delete pl;
}

hsma_status hsma_plan_info(hsma_plan pl, hsma_plan_info_t* info) {
    if (pl == nullptr || info == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    info->n_basis = pl->nb;
    info->n_unknowns = pl->nu;
    info->K = pl->K;
    info->n_check = pl->nchk;
    info->M_eff = pl->M;
    info->F1 = pl->F1;
    info->F2 = pl->F2;
    info->R0 = pl->R0;
    info->Rs = pl->Rs;
    info->precision = pl->precision;
    info->bc = pl->bc;
    info->bytes_resident = pl->bytes;
    info->near_mode = pl->near_mode;
    info->max_images_per_source = pl->maxper;
    info->dipole_mode = pl->dipole_mode;
    info->dr = pl->dr;
    info->far_mode = pl->far_mode;
    info->gamma = pl->gamma;
    info->far_shells = pl->far_shells;
    info->tree_order = pl->tree_order;
    info->tree_min_n = pl->tree_min_n;
    return HSMA_OK;
}

hsma_status hsma_plan_points(hsma_plan pl, int which, double* xyz, double* w) {
    if (pl == nullptr || xyz == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    if (which == 0) {
        std::memcpy(xyz, pl->chk.data(), sizeof(double) * 3 * pl->K);
    } else if (which == 1) {
        if (pl->img != IMG_PERIODIC) return fail(HSMA_E_INVALID, "no twin points for this plan");
        std::memcpy(xyz, pl->chk.data() + 3 * (size_t)pl->K, sizeof(double) * 3 * pl->K);
    } else if (which == 2) {
        std::memcpy(xyz, pl->spts.data(), sizeof(double) * 3 * pl->M);
        if (w) std::memcpy(w, pl->swts.data(), sizeof(double) * pl->M);
    } else {
        return fail(HSMA_E_INVALID, "which must be 0, 1 or 2");
    }
    return HSMA_OK;
}

size_t hsma_workspace_bytes(hsma_plan pl, int64_t N) {
    if (pl == nullptr || N < 0) return 0;
    return make_layout(pl, N, true).total;
}

hsma_status hsma_near_schedule(hsma_plan pl, int64_t N, hsma_near_schedule_t* out) {
    if (pl == nullptr || out == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    if (N < 1 || N > (int64_t)1 << 28) return fail(HSMA_E_INVALID, "N out of range");
    const Layout ly = make_layout(pl, N, false);
    *out = hsma_near_schedule_t{};
    if (ly.tree) {
        out->kind = 2;
    } else if (ly.sym) {
        out->kind = 1;
        out->rows_per_lane = ly.g_sym.T;
        out->block = ly.g_sym.B;
        out->slices = ly.g_sym.s;
        out->parts = ly.g_sym.C;
        out->blocks = ly.g_sym.nb;
        out->launches = ly.g_sym.P;   // the diagonal launch and P - 1 rounds
    }
    return HSMA_OK;
}

}  // extern "C"

hsma_status hsma::check_sizes(const hsma_plan_s* pl, int64_t N) {
    if (pl == nullptr) return fail(HSMA_E_INVALID, "NULL plan");
    if (N < 1 || N > (int64_t)1 << 28) return fail(HSMA_E_INVALID, "N out of range");
    if (pl->bc == HSMA_BC_SLAB_METALLIC_Z && N > (int64_t)1 << 27)
        return fail(HSMA_E_INVALID, "N out of range for the slab");
    const int64_t ns = (pl->bc == HSMA_BC_SLAB_METALLIC_Z) ? 2 * N : N;
    if (pl->near_mode == HSMA_NEAR_SPHERE && ns * pl->maxper > (int64_t)INT32_MAX)
        return fail(HSMA_E_INVALID, "too many sphere images for N");
    // the tree sorts and indexes its 27 images per source with 32-bit integers
    if (pl->near_mode == HSMA_NEAR_TREE && N >= pl->tree_min_n && 27 * ns > (int64_t)INT32_MAX)
        return fail(HSMA_E_INVALID, "too many images for the tree (27 N_s must stay below 2^31)");
    return HSMA_OK;
}

extern "C" {

hsma_status hsma_energy_forces_device(hsma_plan pl, const double* x, const double* q, int64_t N,
                                      void* stream, void* workspace, size_t workspace_bytes,
                                      double* energy, double* phi, double* forces,
                                      const hsma_intermediates* dbg) {
    hsma_status st = check_sizes(pl, N);
    if (st != HSMA_OK) return st;
    if (x == nullptr || q == nullptr || workspace == nullptr || energy == nullptr)
        return fail(HSMA_E_INVALID, "NULL argument");
    const Layout ly = make_layout(pl, N, false);
    if (workspace_bytes < ly.total) return fail(HSMA_E_NOMEM, "workspace too small");
    HSMA_HIP(hipSetDevice(pl->device));
    hipStream_t s = (hipStream_t)stream;
    st = forward(pl, ly, x, q, HSMA_DTYPE_F64, (char*)workspace, s, phi, forces, dbg);
    if (st != HSMA_OK) return st;
    return read_result(ly, (char*)workspace, s, energy);
}

hsma_status hsma_energy_forces_device_typed(hsma_plan pl, const void* x, const void* q, int64_t N,
                                            int dtype, void* stream, void* workspace,
                                            size_t workspace_bytes, double* energy, void* phi,
                                            void* forces) {
    hsma_status st = check_sizes(pl, N);
    if (st != HSMA_OK) return st;
    if (x == nullptr || q == nullptr || workspace == nullptr || energy == nullptr)
        return fail(HSMA_E_INVALID, "NULL argument");
    if (dtype != HSMA_DTYPE_F64 && dtype != HSMA_DTYPE_F32)
        return fail(HSMA_E_INVALID, "dtype must be HSMA_DTYPE_F64 or HSMA_DTYPE_F32");
    const Layout ly = make_layout(pl, N, false);
    if (workspace_bytes < ly.total) return fail(HSMA_E_NOMEM, "workspace too small");
    HSMA_HIP(hipSetDevice(pl->device));
    hipStream_t s = (hipStream_t)stream;
    st = forward(pl, ly, x, q, dtype, (char*)workspace, s, phi, forces, nullptr);
    if (st != HSMA_OK) return st;
    return read_result(ly, (char*)workspace, s, energy);
}

hsma_status hsma_energy_grad_device(hsma_plan pl, const double* x, const double* q, int64_t N,
                                    void* stream, void* workspace, size_t workspace_bytes,
                                    double* energy, double* dEdx, double* dEdq) {
    hsma_status st = check_sizes(pl, N);
    if (st != HSMA_OK) return st;
    if (x == nullptr || q == nullptr || workspace == nullptr || energy == nullptr ||
        dEdx == nullptr || dEdq == nullptr)
        return fail(HSMA_E_INVALID, "NULL argument");
    if (pl->near_mode != HSMA_NEAR_BLOCK)
        return fail(HSMA_E_INVALID, "the adjoint needs the block near set (the sphere set moves "
                                    "images in and out as charges move)");
    if (pl->bc == HSMA_BC_DIELECTRIC) return fail(HSMA_E_INVALID, "no adjoint for the dielectric box");
    if (pl->near_mode == HSMA_NEAR_TREE)
        return fail(HSMA_E_INVALID, "no adjoint for the tree near sum (an approximation whose "
                                    "gradient is not that of the computed energy)");
    if (pl->dipole_mode != HSMA_DIPOLE_EXACT || pl->far_mode != HSMA_FAR_SURFACE)
        return fail(HSMA_E_INVALID, "the adjoint needs the surface mapping with exact dipoles");
    const Layout ly = make_layout(pl, N, true);
    if (workspace_bytes < ly.total) return fail(HSMA_E_NOMEM, "workspace too small");
    HSMA_HIP(hipSetDevice(pl->device));
    hipStream_t s = (hipStream_t)stream;
    st = forward(pl, ly, x, q, HSMA_DTYPE_F64, (char*)workspace, s, nullptr, nullptr, nullptr);
    if (st != HSMA_OK) return st;
    st = backward(pl, ly, (char*)workspace, s, dEdx, dEdq);
    if (st != HSMA_OK) return st;
    return read_result(ly, (char*)workspace, s, energy);
}

hsma_status hsma_energy_forces(hsma_plan pl, const double* x, const double* q, int64_t N,
                               double* energy, double* phi, double* forces) {
    hsma_status st = check_sizes(pl, N);
    if (st != HSMA_OK) return st;
    if (x == nullptr || q == nullptr || energy == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    // host-side validation before any device work
    double qs = 0.0, qa = 0.0;
    const double h = 0.5 * pl->L;
    for (int64_t i = 0; i < N; ++i) {
        for (int a = 0; a < 3; ++a) {
            const double v = x[3 * i + a];
            if (!std::isfinite(v)) return fail(HSMA_E_INVALID, "non-finite position");
            if ((pl->bc == HSMA_BC_METALLIC || pl->bc == HSMA_BC_DIELECTRIC) && !(std::fabs(v - h) < h))
                return fail(HSMA_E_OUT_OF_BOX, "position on or outside a grounded wall");
            if (pl->bc == HSMA_BC_SLAB_METALLIC_Z && a == 2 && !(v > 0.0 && v < h))
                return fail(HSMA_E_OUT_OF_BOX, "position on or outside a slab wall");
        }
        if (!std::isfinite(q[i])) return fail(HSMA_E_INVALID, "non-finite charge");
        qs += q[i];
        qa += std::fabs(q[i]);
    }
    if (needs_neutral(pl->bc) && std::fabs(qs) > 1e-12 * qa)
        return fail(HSMA_E_NOT_NEUTRAL, "periodic/slab system is not neutral");
    HSMA_HIP(hipSetDevice(pl->device));
    const Layout ly = make_layout(pl, N, false);
    const size_t nx = sizeof(double) * 3 * (size_t)N, nq = sizeof(double) * (size_t)N;
    const size_t off_x = 0, off_q = (nx + 255) & ~(size_t)255,
                 off_phi = off_q + ((nq + 255) & ~(size_t)255),
                 off_f = off_phi + ((nq + 255) & ~(size_t)255),
                 off_ws = off_f + ((nx + 255) & ~(size_t)255);
    // the plan's buffer, grown to this call's need (no allocation once it fits)
    std::lock_guard<std::mutex> lk(pl->host_mu);
    if (pl->host_cap < off_ws + ly.total) {
        hipFree(pl->host_buf);
        pl->host_buf = nullptr;
        pl->host_cap = 0;
        if (hipMalloc((void**)&pl->host_buf, off_ws + ly.total) != hipSuccess) {
            pl->host_buf = nullptr;
            return fail(HSMA_E_NOMEM, "device allocation failed");
        }
        pl->host_cap = off_ws + ly.total;
    }
    char* base = pl->host_buf;
    hipStream_t s = nullptr;
    auto done = [&](hsma_status r) { return r; };
    if (hipMemcpy(base + off_x, x, nx, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + off_q, q, nq, hipMemcpyHostToDevice) != hipSuccess)
        return done(fail(HSMA_E_DEVICE, "host to device copy failed"));
    st = forward(pl, ly, base + off_x, base + off_q, HSMA_DTYPE_F64, base + off_ws, s,
                 (double*)(base + off_phi), (double*)(base + off_f), nullptr);
    if (st != HSMA_OK) return done(st);
    st = read_result(ly, base + off_ws, s, energy);
    if (st != HSMA_OK) return done(st);
    if (phi && hipMemcpy(phi, base + off_phi, nq, hipMemcpyDeviceToHost) != hipSuccess)
        return done(fail(HSMA_E_DEVICE, "device to host copy failed"));
    if (forces && hipMemcpy(forces, base + off_f, nx, hipMemcpyDeviceToHost) != hipSuccess)
        return done(fail(HSMA_E_DEVICE, "device to host copy failed"));
    return done(HSMA_OK);
}

hsma_status hsma_timing_enable(int enable) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = enable != 0;
    return HSMA_OK;
}

hsma_status hsma_timing_read(double* ms, int64_t* launches) {
    if (ms == nullptr || launches == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tmu);
    for (int c = 0; c < 3; ++c) { ms[c] = 0.0; launches[c] = 0; }
    for (auto& r : g_trecs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(HSMA_E_DEVICE, "event wait failed");
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            ms[r.cls] += t;
            launches[r.cls] += 1;
        }
        g_tpool.push_back(r.a);
        g_tpool.push_back(r.b);
    }
    g_trecs.clear();
    return HSMA_OK;
}

}  // extern "C"
