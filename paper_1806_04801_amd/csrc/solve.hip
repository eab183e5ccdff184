// Update step of the HSMA (Sec. II.C) on one GPU: sources -> right-hand side
// at the monitoring points -> least-squares coefficients -> surface images ->
// near-field and surface sums at the particles -> energy and forces.
#include <dlfcn.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "hsma_internal.h"
#include "solve.h"
#include "stages.h"

namespace hsma {

constexpr int WG = 256;

// ---------------------------------------------------------------- layout
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    if (v == nullptr || *v == 0) return dflt;
    return atoi(v);
}

NearFix near_fix(const hsma_plan_s* pl, const Layout& ly) {
    NearFix f;
    if (pl->near_mode == HSMA_NEAR_SPHERE || ly.tree || pl->img != IMG_PERIODIC) return f;
    const double shift = ly.f32 ? OWN_COLS_F32 : 0.0;
    f.own = (OWN_IMAGES_PERIODIC - shift) / pl->L;
    if (pl->bc == HSMA_BC_PERIODIC) f.qc = shift / pl->L;
    return f;
}

Layout make_layout(const hsma_plan_s* pl, int64_t N, bool grad, int tpl_near_override,
                   int precision_override, bool no_tree) {
    Layout ly;
    ly.N = (int)N;
    ly.ns = (pl->bc == HSMA_BC_SLAB_METALLIC_Z) ? 2 * (int)N : (int)N;
    const int prec = precision_override >= 0 ? precision_override : pl->precision;
    const bool f32 = prec == HSMA_FP32_COMP;
    ly.f32 = f32;
    const bool sphere = pl->near_mode == HSMA_NEAR_SPHERE;
    const bool tree = pl->near_mode == HSMA_NEAR_TREE && N >= pl->tree_min_n && !no_tree;
    // targets per lane of the near tiles: the image-block kernels run best
    // with one, the explicit-image tiles with two (measured); an override other
    // than 1 or 2 is ignored
    auto tpl_env = [](const char* name, int dflt) {
        const int v = env_int(name, dflt);
        return (v == 1 || v == 2) ? v : dflt;
    };
    const int tpl_near = tpl_near_override > 0 ? tpl_near_override
                                               : tpl_env("HSMA_TPL_NEAR", sphere ? 2 : 1);
    const int tpl_rhs = tpl_env("HSMA_TPL_RHS", 1);
    // sphere mode: sources are the explicit images (at most maxper per source);
    // partial buffers are sized for that bound
    ly.img_max = sphere ? (int64_t)ly.ns * pl->maxper : 0;
    const int ns_pairs = sphere ? (int)std::min<int64_t>(ly.img_max, INT32_MAX) : ly.ns;
    const bool diel = pl->img == IMG_DIELECTRIC;
    // the far images of a dielectric box: many images per source, so chunks
    // of any size (the block images take at least 64 sources per chunk)
    ly.g_rhs = diel ? pair_geometry(pl->nchk, ns_pairs, 1, pl->ncu, 1)
                    : pair_geometry(pl->nchk, ns_pairs, tpl_rhs, pl->ncu);
    ly.g_near = pair_geometry(ly.N, ns_pairs, tpl_near, pl->ncu);
    // Pair-once near sum: faster than the tiles from 1024 particles in either
    // precision (measured; in the batched server too, where a request's rounds
    // run between the tick's grouped launches).
    // HSMA_SYM=0 turns it off, HSMA_SYM=1 forces it (any N); HSMA_SYM_MIN
    // overrides the threshold.
    {
        const int mode = env_int("HSMA_SYM", -1);
        const int nmin = env_int("HSMA_SYM_MIN", 1024);
        const bool eligible = !sphere && !diel && !tree && ly.N > 0;
        ly.sym = eligible && (mode == 1 || (mode < 0 && ly.N >= nmin));
        ly.sym_img = pl->bc == HSMA_BC_SLAB_METALLIC_Z ? IMG_SLAB : pl->img;
        if (ly.sym) ly.g_sym = sym_geometry(ly.N, env_int("HSMA_SYM_T", 1), !f32, ly.sym_img, pl->ncu);
    }
    const int nsurf = pl->dipole_mode == HSMA_DIPOLE_LAYERS ? 3 * pl->M : pl->M;
    ly.g_surf = pair_geometry(ly.N, nsurf, 1, pl->ncu);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    ly.off_src64 = take(sizeof(double4) * (size_t)ly.ns);
    ly.off_src32 = f32 ? take(sizeof(Rec32) * (size_t)ly.ns) : 0;
    ly.off_rhs_part = take(sizeof(double) * (size_t)ly.g_rhs.S * ly.g_rhs.nt_pad);
    ly.off_b = take(sizeof(double) * (size_t)pl->K);
    ly.off_A = take(sizeof(double) * (size_t)pl->nb);
    ly.off_surf = take(sizeof(double) * 12 * (size_t)pl->M);   // 8 per point, or 3 charges
    if (tree) {
        // the tree writes eval_split copies of phi and E: chunks of the tile
        // layout; the right-hand side comes from the same tree (one chunk),
        // on the caller's stream after the tree is built, except for the
        // dielectric box, whose right-hand side is the far shells'
        ly.tree = true;
        ly.tl = tree_layout(ly.ns, pl->tree_order);
        ly.g_near.S = ly.tl.eval_split;
        if (pl->img != IMG_DIELECTRIC) ly.g_rhs.S = 1;
        ly.single_stream = true;
    }
    {
        size_t near_doubles = 4 * (size_t)ly.g_near.S * ly.g_near.nt_pad;
        if (ly.sym)
            near_doubles = std::max(near_doubles, (size_t)(ly.g_sym.C + ly.g_sym.s) * 4 * ly.g_sym.n_pad);
        ly.off_near_part = take(sizeof(double) * near_doubles);
    }
    ly.off_surf_part = take(sizeof(double) * 4 * (size_t)ly.g_surf.S * ly.g_surf.nt_pad);
    ly.n_eblk = (ly.N + WG - 1) / WG;
    if (ly.n_eblk < 1) ly.n_eblk = 1;
    ly.off_eblk = take(sizeof(double) * 3 * (size_t)ly.n_eblk);
    ly.off_result = take(sizeof(Result));
    ly.dup_T = 64;
    while (ly.dup_T < 2 * (int64_t)ly.N) ly.dup_T *= 2;
    ly.off_dup = take(sizeof(int) * (size_t)ly.dup_T);
    if (sphere) {
        ly.off_cnt = take(sizeof(int) * (size_t)ly.ns);
        ly.off_imgoff = take(sizeof(int) * ((size_t)ly.ns + 1));
        ly.off_img64 = take(sizeof(double4) * (size_t)ly.img_max);
        ly.off_img32 = f32 ? take(sizeof(Rec32) * (size_t)ly.img_max) : 0;
    }
    if (tree) ly.off_tree = take(ly.tl.total);
    if (grad) {
        ly.g_u = pair_geometry(pl->M, ly.N, 1, pl->ncu);
        ly.g_G = pair_geometry(ly.ns, pl->nchk, tpl_near, pl->ncu);
        ly.off_u_part = take(sizeof(double) * 4 * (size_t)ly.g_u.S * ly.g_u.nt_pad);
        ly.off_tw = take(sizeof(double) * (size_t)pl->nb);
        ly.off_ud = take(sizeof(double) * 2 * (size_t)pl->M);
        ly.off_lam64 = take(sizeof(double4) * (size_t)pl->nchk);
        ly.off_lam32 = f32 ? take(sizeof(Rec32) * (size_t)pl->nchk) : 0;
        ly.off_G_part = take(sizeof(double) * 4 * (size_t)ly.g_G.S * ly.g_G.nt_pad);
    }
    ly.total = o;
    return ly;
}

// ---------------------------------------------------------------- kernels
template <typename TI>
__global__ void k_prep(const TI* __restrict__ x, const TI* __restrict__ q, int N, int bc,
                       double L, double4* __restrict__ src, int* __restrict__ status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) prep_body(i, x, q, N, bc, L, src, status);
}

__global__ void k_dup_clear(int* __restrict__ tab, int64_t T) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < T;
         t += (int64_t)gridDim.x * blockDim.x)
        tab[t] = -1;
}

__global__ void k_dup_insert(const double4* __restrict__ src, int N, int* __restrict__ tab,
                             uint32_t mask, int* __restrict__ status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) dup_insert_body(i, src, tab, mask, status);
}

__global__ void k_zero_result(Result* r) {
    if (threadIdx.x == 0) {
        r->energy = 0.0;
        r->qsum = 0.0;
        r->qabs = 0.0;
        r->qnet = 0.0;
        r->status = 0;
    }
}

__global__ void k_rhs_finalize(const double* __restrict__ part, int S, int nt_pad, int K,
                               int twins, double* __restrict__ b) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) rhs_body(k, part, S, nt_pad, K, twins, b);
}

__global__ void __launch_bounds__(WG) k_lsq(const double* __restrict__ P, int nu, int K,
                                           const double* __restrict__ b, int k0,
                                           double* __restrict__ A) {
    const int r = blockIdx.x * (WG / 64) + threadIdx.x / 64;
    if (r < nu) lsq_body(r, threadIdx.x & 63, P, K, b, k0, A);
}

__global__ void __launch_bounds__(WG) k_map(const double* __restrict__ Wq,
                                           const double* __restrict__ Wp, int M, int nb,
                                           const double* __restrict__ A,
                                           const double* __restrict__ spos, double Rs,
                                           double* __restrict__ surf) {
    const int j = blockIdx.x * (WG / 64) + threadIdx.x / 64;
    if (j < M) map_body(j, threadIdx.x & 63, Wq, Wp, nb, A, spos, Rs, surf);
}

__global__ void __launch_bounds__(WG) k_map_layers(const double* __restrict__ Wq,
                                                  const double* __restrict__ Wp, int M, int nb,
                                                  const double* __restrict__ A,
                                                  const double* __restrict__ spos, double Rs,
                                                  double dr, double4* __restrict__ chg) {
    const int j = blockIdx.x * (WG / 64) + threadIdx.x / 64;
    if (j < M) map_layers_body(j, threadIdx.x & 63, M, Wq, Wp, nb, A, spos, Rs, dr, chg);
}

template <typename TO>
__global__ void __launch_bounds__(WG)
k_finalize(const double* __restrict__ near, int Sn, int npad, const double* __restrict__ surfp,
           int Ss, int spad, const double4* __restrict__ src, int N, NearFix fix,
           const double* __restrict__ qnet, TO* __restrict__ phi, TO* __restrict__ forces,
           double* __restrict__ dbg_pn, double* __restrict__ dbg_fn, double* __restrict__ dbg_po,
           double* __restrict__ dbg_fo, double* __restrict__ eblk) {
    finalize_body(blockIdx.x, near, Sn, npad, surfp, Ss, spad, src, N, fix, qnet, phi, forces,
                  dbg_pn, dbg_fn, dbg_po, dbg_fo, eblk);
}

__global__ void __launch_bounds__(SWG) k_net_charge(const double4* __restrict__ src, int N,
                                                    double* __restrict__ out) {
    net_charge_body(src, N, out);
}

__global__ void __launch_bounds__(WG) k_energy(const double* __restrict__ eblk, int nblk,
                                              int need_neutral, Result* __restrict__ res) {
    energy_body(eblk, nblk, need_neutral, res);
}

// The paper's near set: every image of source i with |image| < Rs, for
// |k_a| <= kr (periodic r + kL; grounded (-1)^k o r + kL, charge (-1)^|k| q),
// in lexicographic k order.  count: number of images per source; write: the
// images at the source's offset.
template <bool WRITE>
__global__ void k_sphere_images(const double4* __restrict__ src, int ns, int metallic, double L,
                                double Rs, int kr, int* __restrict__ cnt,
                                const int* __restrict__ off, double4* __restrict__ img) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const double4 c = src[i];
    const double R2 = Rs * Rs;
    int n = 0;
    int o = WRITE ? off[i] : 0;
    for (int a = -kr; a <= kr; ++a)
        for (int b = -kr; b <= kr; ++b)
            for (int k = -kr; k <= kr; ++k) {
                double px = c.x, py = c.y, pz = c.z, sg = 1.0;
                if (metallic) {
                    if (a & 1) { px = -px; sg = -sg; }
                    if (b & 1) { py = -py; sg = -sg; }
                    if (k & 1) { pz = -pz; sg = -sg; }
                }
                px += a * L;
                py += b * L;
                pz += k * L;
                if (px * px + py * py + pz * pz < R2) {
                    if (WRITE) img[o + n] = make_double4(px, py, pz, sg * c.w);
                    ++n;
                }
            }
    if (!WRITE) cnt[i] = n;
}

// Exclusive prefix sum of cnt[0..n) into off[0..n], off[n] = total (one block).
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ cnt, int n,
                                              int* __restrict__ off) {
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int seg = (n + 1023) / 1024;
    const int b = t * seg, e = min(b + seg, n);
    long long s = 0;
    for (int i = b; i < e; ++i) s += cnt[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        long long acc = 0;
        for (int k = 0; k < 1024; ++k) {
            const long long v = part[k];
            part[k] = acc;
            acc += v;
        }
        off[n] = (int)acc;
    }
    __syncthreads();
    long long acc = part[t];
    for (int i = b; i < e; ++i) {
        off[i] = (int)acc;
        acc += cnt[i];
    }
}

// ---------------------------------------------------------------- pipeline
// Auxiliary stream and events of the calling host thread on a device: the
// right-hand-side chain (pairs, reduction, least squares, mapping) runs on it
// while the near-field kernel runs on the caller's stream.  Default priority,
// created once per thread and device.
struct AuxStream {
    int device = -1;
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

static hipError_t aux_stream(int device, AuxStream** out) {
    static thread_local AuxStream aux[16];
    if (device < 0 || device >= 16) return hipErrorInvalidDevice;
    AuxStream& a = aux[device];
    if (a.s == nullptr) {
        hipError_t e = hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&a.join, hipEventDisableTiming)) != hipSuccess) return e;
        a.device = device;
    }
    *out = &a;
    return hipSuccess;
}

static bool overlap_enabled() {
    static const int v = env_int("HSMA_OVERLAP", 1);
    return v != 0;
}

#define CK(call)                                                                             \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(HSMA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

// ---------------------------------------------------------------- profiler ranges
namespace {
struct RoctxApi {
    int (*push)(const char*) = nullptr;
    int (*pop)() = nullptr;
};
const RoctxApi& roctx_api() {
    static const RoctxApi api = [] {
        RoctxApi a;
        const char* e = getenv("HSMA_ROCTX");
        if (e == nullptr || atoi(e) != 1) return a;
        for (const char* lib : {"librocprofiler-sdk-roctx.so.1", "libroctx64.so.4"}) {
            void* h = dlopen(lib, RTLD_NOW | RTLD_LOCAL);
            if (h == nullptr) continue;
            a.push = (int (*)(const char*))dlsym(h, "roctxRangePushA");
            a.pop = (int (*)())dlsym(h, "roctxRangePop");
            if (a.push != nullptr && a.pop != nullptr) break;
            a.push = nullptr;
            a.pop = nullptr;
        }
        return a;
    }();
    return api;
}
}  // namespace

Range::Range(const char* name) {
    const RoctxApi& a = roctx_api();
    if (a.push != nullptr) {
        a.push(name);
        on_ = true;
    }
}

Range::~Range() {
    if (on_) roctx_api().pop();
}

hsma_status forward(const hsma_plan_s* pl, const Layout& ly, const void* x, const void* q,
                    int dtype, char* ws, hipStream_t s, void* phi, void* forces,
                    const hsma_intermediates* dbg) {
    const Range range(ly.tree ? "hsma: update step (fast multipole)" : "hsma: update step");
    if (dtype != HSMA_DTYPE_F64 && dtype != HSMA_DTYPE_F32)
        return fail(HSMA_E_INVALID, "dtype must be HSMA_DTYPE_F64 or HSMA_DTYPE_F32");
    const bool in32 = dtype == HSMA_DTYPE_F32;
    const int N = ly.N;
    const bool f32 = ly.f32;
    double4* src64 = (double4*)(ws + ly.off_src64);
    Rec32* src32 = f32 ? (Rec32*)(ws + ly.off_src32) : nullptr;
    double* rhs_part = (double*)(ws + ly.off_rhs_part);
    double* b = (double*)(ws + ly.off_b);
    double* A = (double*)(ws + ly.off_A);
    double* surf = (double*)(ws + ly.off_surf);
    double* near_part = (double*)(ws + ly.off_near_part);
    double* surf_part = (double*)(ws + ly.off_surf_part);
    double* eblk = (double*)(ws + ly.off_eblk);
    Result* res = (Result*)(ws + ly.off_result);

    hipLaunchKernelGGL(k_zero_result, dim3(1), dim3(64), 0, s, res);
    if (in32)
        hipLaunchKernelGGL(k_prep<float>, dim3((N + WG - 1) / WG), dim3(WG), 0, s, (const float*)x,
                           (const float*)q, N, pl->bc, pl->L, src64, &res->status);
    else
        hipLaunchKernelGGL(k_prep<double>, dim3((N + WG - 1) / WG), dim3(WG), 0, s, (const double*)x,
                           (const double*)q, N, pl->bc, pl->L, src64, &res->status);
    {
        // two charges at the same position (their interaction is infinite)
        int* dup = (int*)(ws + ly.off_dup);
        const int64_t nblk = std::min<int64_t>((ly.dup_T + WG - 1) / WG, 65536);
        hipLaunchKernelGGL(k_dup_clear, dim3((unsigned)nblk), dim3(WG), 0, s, dup, ly.dup_T);
        hipLaunchKernelGGL(k_dup_insert, dim3((N + WG - 1) / WG), dim3(WG), 0, s, src64, N, dup,
                           (uint32_t)(ly.dup_T - 1), &res->status);
    }
    const NearFix fix = near_fix(pl, ly);
    if (fix.qc != 0.0)
        hipLaunchKernelGGL(k_net_charge, dim3(1), dim3(SWG), 0, s, src64, N, &res->qnet);
    CK(hipGetLastError());
    if (f32) CK(launch_make_rec32(src64, ly.ns, pl->L, src32, s));
    PairGeom g_rhs = ly.g_rhs, g_near = ly.g_near;
    const bool sphere = pl->near_mode == HSMA_NEAR_SPHERE;
    double4* img64 = nullptr;
    Rec32* img32 = nullptr;
    if (sphere) {
        // explicit near images; their number sets the launch geometry
        int* cnt = (int*)(ws + ly.off_cnt);
        int* off = (int*)(ws + ly.off_imgoff);
        img64 = (double4*)(ws + ly.off_img64);
        const int metallic = pl->img == IMG_METALLIC ? 1 : 0;
        hipLaunchKernelGGL(k_sphere_images<false>, dim3((ly.ns + WG - 1) / WG), dim3(WG), 0, s,
                           src64, ly.ns, metallic, pl->L, pl->Rs, pl->kr, cnt, (const int*)nullptr,
                           (double4*)nullptr);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, cnt, ly.ns, off);
        hipLaunchKernelGGL(k_sphere_images<true>, dim3((ly.ns + WG - 1) / WG), dim3(WG), 0, s,
                           src64, ly.ns, metallic, pl->L, pl->Rs, pl->kr, (int*)nullptr,
                           (const int*)off, img64);
        CK(hipGetLastError());
        int n_img = 0;
        CK(hipMemcpyAsync(&n_img, off + ly.ns, sizeof(int), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        if (n_img < 0 || (int64_t)n_img > ly.img_max)
            return fail(HSMA_E_DEVICE, "image count out of range");
        g_rhs = pair_geometry(pl->nchk, n_img, ly.g_rhs.tpl, pl->ncu);
        g_near = pair_geometry(ly.N, n_img, ly.g_near.tpl, pl->ncu);
        if (f32) {
            img32 = (Rec32*)(ws + ly.off_img32);
            CK(launch_make_rec32(img64, n_img, pl->L, img32, s));
        }
    }
    if (ly.tree) {
        // the tree (images, sort, multipoles) serves the near sum here and the
        // right-hand side below; the near sum's timing covers the build
        timing_begin(0, s);
        CK(launch_tree_build(pl->img, pl->gamma, src64, ly.ns, pl->L, ly.tl, ws + ly.off_tree, s));
        CK(launch_tree_near(N, pl->L, ly.tl, ws + ly.off_tree, near_part, g_near.nt_pad, s));
        timing_end(0, s);
    }
    // fork: the right-hand-side chain goes to the auxiliary stream; the
    // caller's stream waits for it again before the surface stage, and on
    // every early return (a failed launch), so that no work of this call on
    // the auxiliary stream can outlive the call's use of the workspace
    hipStream_t s1 = s;
    AuxStream* aux = nullptr;
    struct Join {
        AuxStream* a = nullptr;
        hipStream_t s = nullptr;
        ~Join() {
            if (a != nullptr && hipEventRecord(a->join, a->s) == hipSuccess)
                (void)hipStreamWaitEvent(s, a->join, 0);
        }
    } join_on_exit;
    if (overlap_enabled() && !ly.single_stream) {
        CK(aux_stream(pl->device, &aux));
        CK(hipEventRecord(aux->fork, s));
        CK(hipStreamWaitEvent(aux->s, aux->fork, 0));
        s1 = aux->s;
        join_on_exit.a = aux;
        join_on_exit.s = s;
    }
    // right-hand side at the monitoring points (and twins)
    timing_begin(1, s1);
    if (pl->img == IMG_DIELECTRIC)   // the far shells (direct or tree near sum alike)
        CK(launch_far_shells(pl->d_chk64, src64, g_rhs, pl->L, pl->gamma, pl->far_shells, rhs_part, s1));
    else if (ly.tree)
        CK(launch_tree_points(pl->d_chk64, pl->d_chk_order, pl->nchk, pl->L, ly.tl, ws + ly.off_tree, rhs_part, s1));
    else if (sphere)
        CK(launch_explicit(f32, false, false, f32 ? (const void*)pl->d_chk32 : (const void*)pl->d_chk64,
                           f32 ? (const void*)img32 : (const void*)img64, g_rhs, pl->L, rhs_part, s1));
    else if (f32)
        CK(launch_pair_f32(pl->img, false, false, pl->d_chk32, src32, g_rhs, pl->L, rhs_part, s1));
    else
        CK(launch_pair_f64(pl->img, false, false, pl->d_chk64, src64, g_rhs, pl->L, rhs_part, s1));
    timing_end(1, s1);
    hipLaunchKernelGGL(k_rhs_finalize, dim3((pl->K + WG - 1) / WG), dim3(WG), 0, s1, rhs_part,
                       g_rhs.S, g_rhs.nt_pad, pl->K, pl->img == IMG_PERIODIC ? 1 : 0, b);
    hipLaunchKernelGGL(k_lsq, dim3((pl->nu + 3) / 4), dim3(WG), 0, s1, pl->d_P, pl->nu, pl->K, b,
                       pl->nb - pl->nu, A);
    const bool layers = pl->dipole_mode == HSMA_DIPOLE_LAYERS;
    const bool direct = pl->far_mode == HSMA_FAR_DIRECT;
    if (direct) {
        // no mapping: the series is evaluated at the particles below
    } else if (layers)
        hipLaunchKernelGGL(k_map_layers, dim3((pl->M + 3) / 4), dim3(WG), 0, s1, pl->d_Wq, pl->d_Wp,
                           pl->M, pl->nb, A, pl->d_spos, pl->Rs, pl->dr, (double4*)surf);
    else
        hipLaunchKernelGGL(k_map, dim3((pl->M + 3) / 4), dim3(WG), 0, s1, pl->d_Wq, pl->d_Wp, pl->M,
                           pl->nb, A, pl->d_spos, pl->Rs, surf);
    CK(hipGetLastError());
    if (aux != nullptr) CK(hipEventRecord(aux->join, s1));
    // near field at the particles: the sources and their 27 images, self excluded
    if (!ly.tree) timing_begin(0, s);
    if (ly.tree) {
        // computed above
    } else if (sphere)
        CK(launch_explicit(f32, true, true, f32 ? (const void*)src32 : (const void*)src64,
                           f32 ? (const void*)img32 : (const void*)img64, g_near, pl->L, near_part, s));
    else if (ly.sym && f32)
        CK(launch_sym_f32(ly.sym_img, src32, ly.g_sym, pl->L, near_part, s));
    else if (ly.sym)
        CK(launch_sym_f64(ly.sym_img, src64, ly.g_sym, pl->L, near_part, s));
    else if (f32)
        CK(launch_pair_f32(pl->img, true, true, src32, src32, g_near, pl->L, near_part, s));
    else
        CK(launch_pair_f64(pl->img, true, true, src64, src64, g_near, pl->L, near_part, s, pl->gamma));
    if (!ly.tree) timing_end(0, s);
    // join, then the surface images at the particles
    if (aux != nullptr) {
        CK(hipStreamWaitEvent(s, aux->join, 0));
        join_on_exit.a = nullptr;   // joined
    }
    PairGeom g_surf = ly.g_surf;
    timing_begin(2, s);
    if (direct) {
        g_surf.S = 1;
        CK(launch_far_direct(src64, N, g_surf.nt_pad, pl->p, 1.0 / pl->R0, A, surf_part, s));
    } else if (layers) {
        CK(launch_explicit(false, true, false, src64, surf, g_surf, pl->L, surf_part, s));
    } else {
        CK(launch_surface_f64(src64, surf, g_surf, surf_part, s));
    }
    timing_end(2, s);
    const int near_S = ly.sym ? ly.g_sym.C + ly.g_sym.s : g_near.S;
    const int near_pad = ly.sym ? ly.g_sym.n_pad : g_near.nt_pad;
    if (in32)
        hipLaunchKernelGGL(k_finalize<float>, dim3(ly.n_eblk), dim3(WG), 0, s, near_part, near_S,
                           near_pad, surf_part, g_surf.S, g_surf.nt_pad, src64, N, fix, &res->qnet,
                           (float*)phi, (float*)forces, dbg ? dbg->phi_near : nullptr,
                           dbg ? dbg->field_near : nullptr, dbg ? dbg->phi_out : nullptr,
                           dbg ? dbg->field_out : nullptr, eblk);
    else
        hipLaunchKernelGGL(k_finalize<double>, dim3(ly.n_eblk), dim3(WG), 0, s, near_part, near_S,
                           near_pad, surf_part, g_surf.S, g_surf.nt_pad, src64, N, fix, &res->qnet,
                           (double*)phi, (double*)forces, dbg ? dbg->phi_near : nullptr,
                           dbg ? dbg->field_near : nullptr, dbg ? dbg->phi_out : nullptr,
                           dbg ? dbg->field_out : nullptr, eblk);
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(WG), 0, s, eblk, ly.n_eblk,
                       needs_neutral(pl->bc) ? 1 : 0, res);
    CK(hipGetLastError());
    if (dbg) {
        if (dbg->b) CK(hipMemcpyAsync(dbg->b, b, sizeof(double) * pl->K, hipMemcpyDeviceToDevice, s));
        if (dbg->A) CK(hipMemcpyAsync(dbg->A, A, sizeof(double) * pl->nb, hipMemcpyDeviceToDevice, s));
        if (dbg->surf && !layers && !direct)
            CK(hipMemcpyAsync(dbg->surf, surf, sizeof(double) * 8 * pl->M, hipMemcpyDeviceToDevice, s));
    }
    return HSMA_OK;
}

hsma_status read_result(const Layout& ly, char* ws, hipStream_t s, double* energy) {
    Result h;
    CK(hipMemcpyAsync(&h, ws + ly.off_result, sizeof(Result), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    const char* msg = nullptr;
    const hsma_status st = status_of_bits(h.status, &msg);
    if (st != HSMA_OK) return fail(st, msg);
    if (energy) *energy = h.energy;
    return HSMA_OK;
}

}  // namespace hsma
