// Serving runtime: continuous batching of HSMA energy/force requests.
//
// Requests of any N and boundary condition are queued by hsma_server_submit.
// Every tick the server
//   1. retires requests whose results have reached host memory,
//   2. admits queued requests (FIFO) while a request slot is free and the
//      device arena has room for its inputs, outputs and workspace,
//   3. enqueues, on its stream, one set of grouped launches in which every
//      active request advances one stage:
//        stage A (newly admitted): centring, single-precision records, and
//          the right-hand-side and near-field tiles, or for requests of 1024
//          particles and more the pair-once near sum, and for requests on the
//          fast multipole method (tree plans above their threshold) the tree,
//          its near sum and its right-hand side, each on one of a few side
//          streams, so that the near sums of several requests and the
//          grouped tiles run at the same time;
//        stage B (admitted one tick earlier): right-hand-side reduction, least
//          squares, surface mapping, surface tiles, finalization, energy,
//          and the copy of the results to pinned host memory.
//      The pair tiles of all requests (right-hand side and near field of the
//      stage-A requests, surface sums of the stage-B requests) go into a
//      single launch, so the work of requests that arrive while others are
//      running overlaps on the device.
// A request's tiles and reductions depend only on its own N and plan, never on
// the other requests in the mix, so its results are bitwise the same alone
// and in a batch.  At most two ticks are in flight (host flow control).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "hsma_internal.h"
#include "solve.h"
#include "stages.h"

namespace hsma {

// Device descriptor of one request (grouped small kernels read an array).
struct ReqDesc {
    int N, ns, bc, img, K, nchk, nu, nb, M, k0, twins, need_neutral;
    double L, Rs;
    const double* P;
    const double* Wq;
    const double* Wp;
    const double* spos;
    const double* x;
    const double* q;
    double4* src64;
    Rec32* src32;
    double* rhs_part;
    int rhs_S, rhs_pad;
    double* b;
    double* A;
    double* surf;
    double* near_part;
    int near_S, near_pad;
    NearFix fix;   // own-image and shift terms of the near potential
    double* surf_part;
    int surf_S, surf_pad;
    double* eblk;
    int n_eblk, pad0;
    Result* res;
    double* phi;
    double* forces;
    int* dup;            // exact-coincidence table, dup_mask + 1 slots
    uint32_t dup_mask;
};

// ---------------------------------------------------------------- grouped kernels
__global__ void k_g_zero(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.x];
    if (threadIdx.x == 0) {
        d.res->energy = 0.0;
        d.res->qsum = 0.0;
        d.res->qabs = 0.0;
        d.res->qnet = 0.0;
        d.res->status = 0;
    }
}

__global__ void __launch_bounds__(SWG) k_g_net(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    if (d.fix.qc != 0.0) net_charge_body(d.src64, d.N, &d.res->qnet);   // uniform over the block
}

__global__ void __launch_bounds__(SWG) k_g_prep(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    const int i = blockIdx.x * SWG + threadIdx.x;
    if (i < d.N) prep_body(i, d.x, d.q, d.N, d.bc, d.L, d.src64, &d.res->status);
}

// The table of each request is cleared with a grid-stride loop (it holds up
// to 4N slots, the grid covers N), then every real charge enters it.
__global__ void __launch_bounds__(SWG) k_g_dup_clear(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    for (uint64_t t = (uint64_t)blockIdx.x * SWG + threadIdx.x; t <= (uint64_t)d.dup_mask;
         t += (uint64_t)gridDim.x * SWG)
        d.dup[t] = -1;
}

__global__ void __launch_bounds__(SWG) k_g_dup(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    const int i = blockIdx.x * SWG + threadIdx.x;
    if (i < d.N) dup_insert_body(i, d.src64, d.dup, d.dup_mask, &d.res->status);
}

__global__ void __launch_bounds__(SWG) k_g_rec32(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    const int i = blockIdx.x * SWG + threadIdx.x;
    if (d.src32 != nullptr && i < d.ns) rec32_body(i, d.src64, d.L, d.src32);
}

__global__ void __launch_bounds__(SWG) k_g_rhs(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    const int k = blockIdx.x * SWG + threadIdx.x;
    if (k < d.K) rhs_body(k, d.rhs_part, d.rhs_S, d.rhs_pad, d.K, d.twins, d.b);
}

__global__ void __launch_bounds__(SWG) k_g_lsq(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    const int r = blockIdx.x * (SWG / 64) + threadIdx.x / 64;
    if (r < d.nu) lsq_body(r, threadIdx.x & 63, d.P, d.K, d.b, d.k0, d.A);
}

__global__ void __launch_bounds__(SWG) k_g_map(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    const int j = blockIdx.x * (SWG / 64) + threadIdx.x / 64;
    if (j < d.M) map_body(j, threadIdx.x & 63, d.Wq, d.Wp, d.nb, d.A, d.spos, d.Rs, d.surf);
}

__global__ void __launch_bounds__(SWG) k_g_finalize(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    if ((int)blockIdx.x >= d.n_eblk) return;   // uniform over the block
    finalize_body(blockIdx.x, d.near_part, d.near_S, d.near_pad, d.surf_part, d.surf_S, d.surf_pad,
                  d.src64, d.N, d.fix, &d.res->qnet, d.phi, d.forces, nullptr, nullptr, nullptr,
                  nullptr, d.eblk);
}

__global__ void __launch_bounds__(SWG) k_g_energy(const ReqDesc* __restrict__ D) {
    const ReqDesc& d = D[blockIdx.y];
    energy_body(d.eblk, d.n_eblk, d.need_neutral, d.res);
}

// ---------------------------------------------------------------- server
enum { ST_PENDING = 0, ST_STAGE_A = 1, ST_STAGE_B = 2, ST_COPYING = 3, ST_DONE = 4,
       ST_REFINE = 5,         // waiting for arena memory for its double-precision solve
       ST_REFINE_COPY = 6 };  // double-precision solve and result copies enqueued

struct SrvReq {
    int64_t id = 0;
    hsma_plan plan = nullptr;
    int N = 0;
    std::vector<double> hx, hq;
    const double* ext_x = nullptr;   // caller-owned host inputs (trace replay)
    const double* ext_q = nullptr;
    double t_submit = 0.0, t_done = 0.0;
    int state = ST_PENDING;
    size_t off = 0, host_off = 0;
    Layout ly;
    ReqDesc d{};
    double* h_out = nullptr;         // pinned: Result (RES_D doubles), phi, forces
    hipEvent_t ev = nullptr;
    hsma_status status = HSMA_OK;
    double energy = 0.0;
};

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace hsma

struct hsma_server_s {
    hsma_server_desc desc{};
    int device = 0;
    hipStream_t stream = nullptr;
    char* arena_base = nullptr;
    std::unique_ptr<hsma::Arena> arena;
    char* host_base = nullptr;       // pinned result staging
    std::unique_ptr<hsma::Arena> host_arena;
    int64_t next_id = 1;
    std::deque<hsma::SrvReq*> pending;
    std::vector<hsma::SrvReq*> active;
    std::deque<hsma::SrvReq*> refine;   // active requests waiting in ST_REFINE
    std::unordered_map<int64_t, hsma::SrvReq*> all;
    // per-tick tables: ring of device buffers with their events
    static constexpr int RING = 3;
    char* dtab[RING] = {nullptr, nullptr, nullptr};
    char* htab[RING] = {nullptr, nullptr, nullptr};
    size_t tabcap[RING] = {0, 0, 0};
    hipEvent_t tabev[RING] = {nullptr, nullptr, nullptr};
    bool tabused[RING] = {false, false, false};
    int ring = 0;
    std::deque<hipEvent_t> inflight;
    std::vector<hipEvent_t> evpool;
    // side streams of the pair-once near sums (default priority), with the
    // fork event on the server stream and one join event each
    static constexpr int NSIDE = 8;
    int nside = 3;
    double tick_work = 1.5e11;   // pair-image budget of the requests a tick admits
    hipStream_t side[NSIDE] = {};
    hipEvent_t side_ev[NSIDE] = {};
    hipEvent_t fork_ev = nullptr;
    // double-precision refinements run on a stream of their own, beside the ticks
    hipStream_t rstream = nullptr;
    hsma_server_stats_t stats{};
};

namespace hsma {

static hipEvent_t srv_event(hsma_server_s* sv) {
    if (!sv->evpool.empty()) {
        hipEvent_t e = sv->evpool.back();
        sv->evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

static size_t req_device_bytes(const hsma_plan_s* pl, int N, int precision, Layout* ly,
                               bool no_tree = false) {
    *ly = make_layout(pl, N, false, 1, precision, no_tree);
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) & ~(a - 1); };
    return up(sizeof(double) * 3 * N) * 2 + up(sizeof(double) * N) * 2 + ly->total;
}

// Host output of a request: the Result (padded to whole doubles), phi, forces.
constexpr size_t RES_D = (sizeof(Result) + sizeof(double) - 1) / sizeof(double);
static size_t req_host_bytes(int N) { return sizeof(double) * (RES_D + 4 * (size_t)N); }

// A request's arena block: x (N x 3), q, phi, F (N x 3), then the workspace.
struct ReqBlock {
    double *x, *q, *phi, *F;
    char* ws;
};

static ReqBlock carve(char* base, int N) {
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) & ~(a - 1); };
    ReqBlock b;
    b.x = (double*)base;
    b.q = (double*)(base + up(sizeof(double) * 3 * N));
    b.phi = (double*)((char*)b.q + up(sizeof(double) * N));
    b.F = (double*)((char*)b.phi + up(sizeof(double) * N));
    b.ws = (char*)b.F + up(sizeof(double) * 3 * N);
    return b;
}

// Try to admit one request: arena space for x, q, phi, F and workspace.
static bool admit(hsma_server_s* sv, SrvReq* r) {
    Layout ly;
    const size_t bytes = req_device_bytes(r->plan, r->N, sv->desc.precision, &ly);
    size_t off = 0, hoff = 0;
    if (!sv->arena->alloc(bytes, &off)) return false;
    if (!sv->host_arena->alloc(req_host_bytes(r->N), &hoff)) {
        sv->arena->release(off);
        return false;
    }
    r->off = off;
    r->host_off = hoff;
    r->ly = ly;
    r->h_out = (double*)(sv->host_base + hoff);
    const int N = r->N;
    const ReqBlock blk = carve(sv->arena_base + off, N);
    double* dx = blk.x;
    double* dq = blk.q;
    double* dphi = blk.phi;
    double* dF = blk.F;
    char* ws = blk.ws;
    const hsma_plan_s* pl = r->plan;
    ReqDesc& d = r->d;
    d.N = N;
    d.ns = ly.ns;
    d.bc = pl->bc;
    d.img = pl->img;
    d.K = pl->K;
    d.nchk = pl->nchk;
    d.nu = pl->nu;
    d.nb = pl->nb;
    d.M = pl->M;
    d.k0 = pl->nb - pl->nu;
    d.twins = pl->img == IMG_PERIODIC ? 1 : 0;
    d.need_neutral = needs_neutral(pl->bc) ? 1 : 0;
    d.L = pl->L;
    d.Rs = pl->Rs;
    d.P = pl->d_P;
    d.Wq = pl->d_Wq;
    d.Wp = pl->d_Wp;
    d.spos = pl->d_spos;
    d.x = dx;
    d.q = dq;
    d.src64 = (double4*)(ws + ly.off_src64);
    d.src32 = sv->desc.precision == HSMA_FP32_COMP ? (Rec32*)(ws + ly.off_src32) : nullptr;
    d.rhs_part = (double*)(ws + ly.off_rhs_part);
    d.rhs_S = ly.g_rhs.S;
    d.rhs_pad = ly.g_rhs.nt_pad;
    d.b = (double*)(ws + ly.off_b);
    d.A = (double*)(ws + ly.off_A);
    d.surf = (double*)(ws + ly.off_surf);
    d.near_part = (double*)(ws + ly.off_near_part);
    d.near_S = ly.sym ? ly.g_sym.C + ly.g_sym.s : ly.g_near.S;
    d.near_pad = ly.sym ? ly.g_sym.n_pad : ly.g_near.nt_pad;
    d.fix = near_fix(pl, ly);
    d.surf_part = (double*)(ws + ly.off_surf_part);
    d.surf_S = ly.g_surf.S;
    d.surf_pad = ly.g_surf.nt_pad;
    d.eblk = (double*)(ws + ly.off_eblk);
    d.n_eblk = ly.n_eblk;
    d.res = (Result*)(ws + ly.off_result);
    d.phi = dphi;
    d.forces = dF;
    d.dup = (int*)(ws + ly.off_dup);
    d.dup_mask = (uint32_t)(ly.dup_T - 1);
    const double* hx = r->ext_x ? r->ext_x : r->hx.data();
    const double* hq = r->ext_q ? r->ext_q : r->hq.data();
    hipMemcpyAsync(dx, hx, sizeof(double) * 3 * N, hipMemcpyHostToDevice, sv->stream);
    hipMemcpyAsync(dq, hq, sizeof(double) * N, hipMemcpyHostToDevice, sv->stream);
    return true;
}

// The tiles of one pair stage of one request, as one group of the launch.
static void add_group(std::vector<TileGroup>& v, int* ntiles, int kind, int img, const PairGeom& g,
                      const void* tgt, const void* src, double* out, double L) {
    if (g.nt <= 0 || g.ntb <= 0 || g.S <= 0) return;
    TileGroup it;
    it.kind = kind;
    it.img = img;
    it.first = *ntiles;
    it.ntb = g.ntb;
    it.S = g.S;
    it.nt = g.nt;
    it.ns = g.ns;
    it.chunk = g.chunk;
    it.nt_pad = g.nt_pad;
    it.pad = 0;
    it.tgt = tgt;
    it.src = src;
    it.out = out;
    it.L = L;
    v.push_back(it);
    *ntiles += g.ntb * g.S;
}

// Copy the tick's tables to the device through a pinned ring slot.
static hsma_status upload(hsma_server_s* sv, const std::vector<ReqDesc>& da,
                          const std::vector<ReqDesc>& db, const std::vector<TileGroup>& tiles,
                          ReqDesc** dA, ReqDesc** dB, TileGroup** dT) {
    const int slot = sv->ring;
    sv->ring = (sv->ring + 1) % hsma_server_s::RING;
    if (sv->tabused[slot]) HSMA_HIP(hipEventSynchronize(sv->tabev[slot]));
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) & ~(a - 1); };
    const size_t na = up(sizeof(ReqDesc) * da.size()), nb = up(sizeof(ReqDesc) * db.size()),
                 nt = up(sizeof(TileGroup) * tiles.size());
    const size_t need = na + nb + nt + 256;
    if (need > sv->tabcap[slot]) {
        HSMA_HIP(hipStreamSynchronize(sv->stream));
        hipFree(sv->dtab[slot]);
        hipHostFree(sv->htab[slot]);
        sv->dtab[slot] = nullptr;
        sv->htab[slot] = nullptr;
        size_t cap = std::max(need * 2, (size_t)1 << 20);
        if (hipMalloc((void**)&sv->dtab[slot], cap) != hipSuccess ||
            hipHostMalloc((void**)&sv->htab[slot], cap, hipHostMallocDefault) != hipSuccess) {
            sv->tabcap[slot] = 0;
            return fail(HSMA_E_NOMEM, "server table allocation failed");
        }
        sv->tabcap[slot] = cap;
    }
    char* h = sv->htab[slot];
    if (!da.empty()) std::memcpy(h, da.data(), sizeof(ReqDesc) * da.size());
    if (!db.empty()) std::memcpy(h + na, db.data(), sizeof(ReqDesc) * db.size());
    if (!tiles.empty()) std::memcpy(h + na + nb, tiles.data(), sizeof(TileGroup) * tiles.size());
    HSMA_HIP(hipMemcpyAsync(sv->dtab[slot], h, na + nb + nt, hipMemcpyHostToDevice, sv->stream));
    HSMA_HIP(hipEventRecord(sv->tabev[slot], sv->stream));
    sv->tabused[slot] = true;
    *dA = (ReqDesc*)sv->dtab[slot];
    *dB = (ReqDesc*)(sv->dtab[slot] + na);
    *dT = (TileGroup*)(sv->dtab[slot] + na + nb);
    return HSMA_OK;
}

// Whether a finished single-precision or fast-multipole result is recomputed
// with the direct double-precision sums: its energy is below refine_below *
// 1/2 sum |q_i phi_i|, and the double-precision block fits the arena.
static bool wants_refine(const hsma_server_s* sv, const SrvReq* r) {
    if ((sv->desc.precision != HSMA_FP32_COMP && !r->ly.tree) || !(sv->desc.refine_below > 0.0) ||
        r->status != HSMA_OK)
        return false;
    Layout ly64;
    if (req_device_bytes(r->plan, r->N, HSMA_FP64, &ly64, true) > sv->arena->cap()) return false;
    const double* q = r->ext_q ? r->ext_q : r->hq.data();
    const double* phi = r->h_out + RES_D;
    double scale = 0.0;
    for (int i = 0; i < r->N; ++i) scale += std::fabs(q[i] * phi[i]);
    return std::fabs(r->energy) < sv->desc.refine_below * 0.5 * scale;
}

static void retire(hsma_server_s* sv) {
    std::vector<SrvReq*> keep;
    for (SrvReq* r : sv->active) {
        const bool copied = (r->state == ST_COPYING || r->state == ST_REFINE_COPY) &&
                            hipEventQuery(r->ev) == hipSuccess;
        if (!copied) {
            keep.push_back(r);
            continue;
        }
        const Result* res = (const Result*)r->h_out;
        r->energy = res->energy;
        {
            const char* msg = nullptr;
            const hsma_status st = status_of_bits(res->status, &msg);
            if (st != HSMA_OK) r->status = st;
        }
        sv->evpool.push_back(r->ev);
        r->ev = nullptr;
        sv->arena->release(r->off);
        if (r->state == ST_COPYING && wants_refine(sv, r)) {
            // the block is free again: the double-precision solve takes a new
            // one (inputs copied from the host again), so a request waiting
            // for memory holds none
            r->state = ST_REFINE;
            sv->refine.push_back(r);
            keep.push_back(r);
            continue;
        }
        if (r->state == ST_REFINE_COPY) sv->stats.refined += 1;
        r->t_done = now_s();
        r->state = ST_DONE;
        sv->stats.completed += 1;
        // host staging stays until the caller reads the result
    }
    sv->active.swap(keep);
}

// Enqueue the double-precision solves of queued refinements that fit the
// arena, in queue order; false when the head must wait for memory.
static hsma_status start_refinements(hsma_server_s* sv, bool* blocked) {
    *blocked = false;
    hipStream_t s = sv->rstream;
    while (!sv->refine.empty()) {
        SrvReq* r = sv->refine.front();
        // the direct double-precision sums (not the tree's approximation)
        Layout ly64;
        const size_t bytes = req_device_bytes(r->plan, r->N, HSMA_FP64, &ly64, true);
        size_t off = 0;
        if (!sv->arena->alloc(bytes, &off)) {
            *blocked = true;
            return HSMA_OK;
        }
        sv->refine.pop_front();
        r->off = off;
        const int N = r->N;
        const ReqBlock blk = carve(sv->arena_base + off, N);
        const double* hx = r->ext_x ? r->ext_x : r->hx.data();
        const double* hq = r->ext_q ? r->ext_q : r->hq.data();
        HSMA_HIP(hipMemcpyAsync(blk.x, hx, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
        HSMA_HIP(hipMemcpyAsync(blk.q, hq, sizeof(double) * N, hipMemcpyHostToDevice, s));
        hsma_status st = forward(r->plan, ly64, blk.x, blk.q, HSMA_DTYPE_F64, blk.ws, s, blk.phi, blk.F,
                                 nullptr);
        if (st != HSMA_OK) return st;
        HSMA_HIP(hipMemcpyAsync(r->h_out, blk.ws + ly64.off_result, sizeof(Result),
                                hipMemcpyDeviceToHost, s));
        HSMA_HIP(hipMemcpyAsync(r->h_out + RES_D, blk.phi, sizeof(double) * N, hipMemcpyDeviceToHost, s));
        HSMA_HIP(hipMemcpyAsync(r->h_out + RES_D + N, blk.F, sizeof(double) * 3 * N,
                                hipMemcpyDeviceToHost, s));
        r->ev = srv_event(sv);
        if (r->ev == nullptr) return fail(HSMA_E_DEVICE, "event creation failed");
        HSMA_HIP(hipEventRecord(r->ev, s));
        r->state = ST_REFINE_COPY;
    }
    return HSMA_OK;
}

// Pair-image evaluations of a request: the near block (27 N_s per particle)
// and the right-hand side (27 N_s per check point).
static double request_work(const hsma_plan_s* pl, int N) {
    const double ns = pl->bc == HSMA_BC_SLAB_METALLIC_Z ? 2.0 * N : (double)N;
    if (pl->near_mode == HSMA_NEAR_TREE && N >= pl->tree_min_n)
        return 5e5 * ns;   // the tree's near sum and right-hand side, in the same unit (measured)
    return 27.0 * ns * ((double)N + (double)pl->nchk);
}

static hsma_status tick(hsma_server_s* sv) {
    const Range range("hsma: server tick");
    HSMA_HIP(hipSetDevice(sv->device));
    retire(sv);
    // flow control: at most two ticks in flight
    while (sv->inflight.size() >= 2) {
        HSMA_HIP(hipEventSynchronize(sv->inflight.front()));
        sv->evpool.push_back(sv->inflight.front());
        sv->inflight.pop_front();
        retire(sv);
    }
    // double-precision refinements first; while one waits for memory no new
    // request is admitted, so the memory that finishing requests free goes to it
    bool refine_blocked = false;
    const size_t refine_queued = sv->refine.size();
    {
        hsma_status st = start_refinements(sv, &refine_blocked);
        if (st != HSMA_OK) return st;
    }
    const bool refine_started = sv->refine.size() < refine_queued;
    // admission: FIFO while a slot and arena memory are free and the tick's
    // pair work stays within its budget (a request larger than the budget
    // comes alone), so that ticks stay short, two of them keep the GPU busy
    // and a finishing request frees its slot for the queue within a few ticks
    std::vector<SrvReq*> newA;
    double tick_work = 0.0;
    while (!refine_blocked && !sv->pending.empty() &&
           (int)sv->active.size() < sv->desc.max_active) {
        SrvReq* r = sv->pending.front();
        const double w = request_work(r->plan, r->N);
        if (!newA.empty() && tick_work + w > sv->tick_work) break;
        if (!admit(sv, r)) break;
        sv->pending.pop_front();
        r->state = ST_STAGE_A;
        sv->active.push_back(r);
        newA.push_back(r);
        tick_work += w;
    }
    std::vector<SrvReq*> stB;
    for (SrvReq* r : sv->active)
        if (r->state == ST_STAGE_B) stB.push_back(r);
    if (newA.empty() && stB.empty()) {
        if (refine_started) {
            // the refinements are this tick's work: track them like a tick
            hipEvent_t te = srv_event(sv);
            if (te == nullptr) return fail(HSMA_E_DEVICE, "event creation failed");
            HSMA_HIP(hipEventRecord(te, sv->rstream));
            sv->inflight.push_back(te);
            sv->stats.ticks += 1;
        }
        return HSMA_OK;
    }
    const bool f32 = sv->desc.precision == HSMA_FP32_COMP;
    std::vector<ReqDesc> da, db;
    // tile groups in five lists, one launch each: near (periodic, grounded),
    // right-hand side (periodic, grounded), surface
    constexpr int NLIST = 5;
    std::vector<TileGroup> lists[NLIST];
    int nlist_tiles[NLIST] = {0, 0, 0, 0, 0};
    auto list_of = [](int kind, int img) {
        return kind == TILE_SURFACE ? 4 : 2 * (kind == TILE_RHS ? 1 : 0) + (img == IMG_PERIODIC ? 0 : 1);
    };
    int maxA_blk = 1, maxA_ns = 1, maxB_K = 1, maxB_nu = 1, maxB_M = 1, maxB_e = 1;
    for (SrvReq* r : newA) {
        da.push_back(r->d);
        maxA_blk = std::max(maxA_blk, (r->N + SWG - 1) / SWG);
        maxA_ns = std::max(maxA_ns, (r->d.ns + SWG - 1) / SWG);
    }
    for (SrvReq* r : stB) {
        db.push_back(r->d);
        maxB_K = std::max(maxB_K, (r->d.K + SWG - 1) / SWG);
        maxB_nu = std::max(maxB_nu, (r->d.nu + 3) / 4);
        maxB_M = std::max(maxB_M, (r->d.M + 3) / 4);
        maxB_e = std::max(maxB_e, r->d.n_eblk);
    }
    // tile groups: near first (the longest), then right-hand side, then surface;
    // requests large enough for the pair-once near sum run it in rounds of
    // their own instead, and requests on the tree take their near sum and
    // right-hand side from it (see below)
    for (SrvReq* r : newA) {
        const ReqDesc& d = r->d;
        if (r->ly.sym || r->ly.tree) continue;
        const int l = list_of(TILE_NEAR, d.img);
        if (f32) add_group(lists[l], &nlist_tiles[l], TILE_NEAR, d.img, r->ly.g_near, d.src32, d.src32, d.near_part, d.L);
        else add_group(lists[l], &nlist_tiles[l], TILE_NEAR, d.img, r->ly.g_near, d.src64, d.src64, d.near_part, d.L);
    }
    for (SrvReq* r : newA) {
        const hsma_plan_s* pl = r->plan;
        const ReqDesc& d = r->d;
        if (r->ly.tree) continue;
        const int l = list_of(TILE_RHS, d.img);
        if (f32) add_group(lists[l], &nlist_tiles[l], TILE_RHS, d.img, r->ly.g_rhs, pl->d_chk32, d.src32, d.rhs_part, d.L);
        else add_group(lists[l], &nlist_tiles[l], TILE_RHS, d.img, r->ly.g_rhs, pl->d_chk64, d.src64, d.rhs_part, d.L);
    }
    for (SrvReq* r : stB)
        add_group(lists[4], &nlist_tiles[4], TILE_SURFACE, 0, r->ly.g_surf, r->d.src64, r->d.surf, r->d.surf_part, r->d.L);
    std::vector<TileGroup> tiles;
    int list_at[NLIST];
    int ntiles = 0;
    for (int l = 0; l < NLIST; ++l) {
        list_at[l] = (int)tiles.size();
        tiles.insert(tiles.end(), lists[l].begin(), lists[l].end());
        ntiles += nlist_tiles[l];
    }
    ReqDesc *dA = nullptr, *dB = nullptr;
    TileGroup* dT = nullptr;
    hsma_status st = upload(sv, da, db, tiles, &dA, &dB, &dT);
    if (st != HSMA_OK) return st;
    hipStream_t s = sv->stream;
    const unsigned nA = (unsigned)da.size(), nB = (unsigned)db.size();
    // stage B, part 1: right-hand side, least squares, mapping
    if (nB) {
        hipLaunchKernelGGL(k_g_rhs, dim3(maxB_K, nB), dim3(SWG), 0, s, dB);
        hipLaunchKernelGGL(k_g_lsq, dim3(maxB_nu, nB), dim3(SWG), 0, s, dB);
        hipLaunchKernelGGL(k_g_map, dim3(maxB_M, nB), dim3(SWG), 0, s, dB);
    }
    // stage A: centring and records
    if (nA) {
        hipLaunchKernelGGL(k_g_zero, dim3(nA), dim3(64), 0, s, dA);
        hipLaunchKernelGGL(k_g_prep, dim3(maxA_blk, nA), dim3(SWG), 0, s, dA);
        hipLaunchKernelGGL(k_g_dup_clear, dim3(maxA_blk, nA), dim3(SWG), 0, s, dA);
        hipLaunchKernelGGL(k_g_dup, dim3(maxA_blk, nA), dim3(SWG), 0, s, dA);
        hipLaunchKernelGGL(k_g_net, dim3(1, nA), dim3(SWG), 0, s, dA);
        if (f32) hipLaunchKernelGGL(k_g_rec32, dim3(maxA_ns, nA), dim3(SWG), 0, s, dA);
    }
    HSMA_HIP(hipGetLastError());
    // Pair-once near sums of the new requests at or above the threshold, and
    // the tree (build, near sum, right-hand side) of requests on the fast
    // multipole method: each request's launches go to one of the side streams
    // (the one with the least work so far, largest requests first), forked
    // from the server stream after the records above, so that the near sums
    // of several requests and the grouped tiles below run at the same time;
    // the side streams join back at the end of the tick.
    std::vector<SrvReq*> symr;
    for (SrvReq* r : newA)
        if (r->ly.sym || r->ly.tree) symr.push_back(r);
    std::stable_sort(symr.begin(), symr.end(), [](const SrvReq* a, const SrvReq* b) { return a->N > b->N; });
    bool side_used[hsma_server_s::NSIDE] = {};
    if (!symr.empty()) {
        HSMA_HIP(hipEventRecord(sv->fork_ev, s));
        double load[hsma_server_s::NSIDE] = {};
        for (SrvReq* r : symr) {
            int w = 0;
            for (int k = 1; k < sv->nside; ++k)
                if (load[k] < load[w]) w = k;
            // rough cost in one unit: pair-once ~ N^2, the tree ~ 2e4 N (measured)
            load[w] += r->ly.tree ? 2e4 * r->N : (double)r->N * r->N;
            hipStream_t ss = sv->side[w];
            if (!side_used[w]) {
                HSMA_HIP(hipStreamWaitEvent(ss, sv->fork_ev, 0));
                side_used[w] = true;
            }
            if (r->ly.tree) {
                const hsma_plan_s* pl = r->plan;
                char* tws = carve(sv->arena_base + r->off, r->N).ws + r->ly.off_tree;
                HSMA_HIP(launch_tree_build(pl->img, pl->gamma, r->d.src64, r->ly.ns, pl->L, r->ly.tl, tws, ss));
                HSMA_HIP(launch_tree_points(pl->d_chk64, pl->d_chk_order, pl->nchk, pl->L, r->ly.tl, tws, r->d.rhs_part, ss));
                HSMA_HIP(launch_tree_near(r->N, pl->L, r->ly.tl, tws, r->d.near_part, r->ly.g_near.nt_pad, ss));
            } else if (f32)
                HSMA_HIP(launch_sym_f32(r->ly.sym_img, r->d.src32, r->ly.g_sym, r->d.L, r->d.near_part, ss));
            else
                HSMA_HIP(launch_sym_f64(r->ly.sym_img, r->d.src64, r->ly.g_sym, r->d.L, r->d.near_part, ss));
        }
    }
    // the pair tiles of the tick, one launch per kind
    timing_begin(0, s);
    for (int l = 0; l < NLIST; ++l) {
        if (lists[l].empty()) continue;
        const TileGroup& g0 = lists[l].front();
        HSMA_HIP(launch_group_tiles(f32, g0.kind, g0.img, dT + list_at[l], (int)lists[l].size(),
                                    nlist_tiles[l], s));
    }
    timing_end(0, s);
    // stage B, part 2: finalize, energy, results to host
    if (nB) {
        hipLaunchKernelGGL(k_g_finalize, dim3(maxB_e, nB), dim3(SWG), 0, s, dB);
        hipLaunchKernelGGL(k_g_energy, dim3(1, nB), dim3(SWG), 0, s, dB);
        HSMA_HIP(hipGetLastError());
        for (SrvReq* r : stB) {
            HSMA_HIP(hipMemcpyAsync(r->h_out, r->d.res, sizeof(Result), hipMemcpyDeviceToHost, s));
            HSMA_HIP(hipMemcpyAsync(r->h_out + RES_D, r->d.phi, sizeof(double) * r->N,
                                    hipMemcpyDeviceToHost, s));
            HSMA_HIP(hipMemcpyAsync(r->h_out + RES_D + r->N, r->d.forces, sizeof(double) * 3 * r->N,
                                    hipMemcpyDeviceToHost, s));
            r->ev = srv_event(sv);
            HSMA_HIP(hipEventRecord(r->ev, s));
            r->state = ST_COPYING;
        }
    }
    // join the side streams: the next tick's stage B of these requests reads
    // their near sums
    for (int w = 0; w < sv->nside; ++w)
        if (side_used[w]) {
            HSMA_HIP(hipEventRecord(sv->side_ev[w], sv->side[w]));
            HSMA_HIP(hipStreamWaitEvent(s, sv->side_ev[w], 0));
        }
    for (SrvReq* r : newA) r->state = ST_STAGE_B;
    hipEvent_t te = srv_event(sv);
    HSMA_HIP(hipEventRecord(te, s));
    sv->inflight.push_back(te);
    sv->stats.ticks += 1;
    sv->stats.tiles += (int64_t)ntiles;
    return HSMA_OK;
}

static bool busy(const hsma_server_s* sv) { return !sv->pending.empty() || !sv->active.empty(); }

}  // namespace hsma

using namespace hsma;

extern "C" {

hsma_status hsma_server_create(const hsma_server_desc* desc, hsma_server* out) {
    if (desc == nullptr || out == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    *out = nullptr;
    if (desc->memory_bytes < ((size_t)1 << 20) || desc->max_active < 1)
        return fail(HSMA_E_INVALID, "server needs >= 1 MiB of memory and >= 1 slot");
    if (desc->precision != HSMA_FP64 && desc->precision != HSMA_FP32_COMP)
        return fail(HSMA_E_INVALID, "unknown precision");
    if (!(desc->refine_below >= 0.0) || !std::isfinite(desc->refine_below))
        return fail(HSMA_E_INVALID, "refine_below must be finite and >= 0");
    hsma_server_s* sv = new (std::nothrow) hsma_server_s();
    if (sv == nullptr) return fail(HSMA_E_NOMEM, "host allocation failed");
    sv->desc = *desc;
    auto bail = [&](hsma_status st, const char* m) {
        hipFree(sv->arena_base);
        hipHostFree(sv->host_base);
        if (sv->stream) hipStreamDestroy(sv->stream);
        for (int i = 0; i < hsma_server_s::RING; ++i)
            if (sv->tabev[i]) hipEventDestroy(sv->tabev[i]);
        for (int w = 0; w < hsma_server_s::NSIDE; ++w) {
            if (sv->side[w]) hipStreamDestroy(sv->side[w]);
            if (sv->side_ev[w]) hipEventDestroy(sv->side_ev[w]);
        }
        if (sv->fork_ev) hipEventDestroy(sv->fork_ev);
        if (sv->rstream) hipStreamDestroy(sv->rstream);
        delete sv;
        return fail(st, m);
    };
    if (hipGetDevice(&sv->device) != hipSuccess) return bail(HSMA_E_DEVICE, "no HIP device");
    if (hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(HSMA_E_DEVICE, "stream creation failed");
    if (hipMalloc((void**)&sv->arena_base, desc->memory_bytes) != hipSuccess)
        return bail(HSMA_E_NOMEM, "device arena allocation failed");
    // pinned staging for results: sized for the arena's worth of particles
    const size_t host_cap = std::min(desc->memory_bytes / 4, (size_t)1 << 30) + ((size_t)1 << 20);
    if (hipHostMalloc((void**)&sv->host_base, host_cap, hipHostMallocDefault) != hipSuccess)
        return bail(HSMA_E_NOMEM, "pinned host allocation failed");
    sv->arena.reset(new Arena(desc->memory_bytes));
    sv->host_arena.reset(new Arena(host_cap));
    for (int i = 0; i < hsma_server_s::RING; ++i)
        if (hipEventCreateWithFlags(&sv->tabev[i], hipEventDisableTiming) != hipSuccess)
            return bail(HSMA_E_DEVICE, "event creation failed");
    // side streams of the pair-once near sums: HSMA_SRV_STREAMS (1 to 8,
    // default 3) in the environment
    {
        const char* v = getenv("HSMA_SRV_STREAMS");
        const int n = v != nullptr && *v ? atoi(v) : 3;
        sv->nside = std::min(std::max(n, 1), hsma_server_s::NSIDE);
    }
    // pair-image budget of a tick's admissions: HSMA_SRV_TICK_WORK (default
    // 1.5e11, about 17 ms of single-precision near sums)
    {
        const char* v = getenv("HSMA_SRV_TICK_WORK");
        const double w = v != nullptr && *v ? atof(v) : 0.0;
        if (w > 0.0) sv->tick_work = w;
    }
    if (hipEventCreateWithFlags(&sv->fork_ev, hipEventDisableTiming) != hipSuccess)
        return bail(HSMA_E_DEVICE, "event creation failed");
    for (int w = 0; w < sv->nside; ++w)
        if (hipStreamCreateWithFlags(&sv->side[w], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sv->side_ev[w], hipEventDisableTiming) != hipSuccess)
            return bail(HSMA_E_DEVICE, "side stream creation failed");
    if (hipStreamCreateWithFlags(&sv->rstream, hipStreamNonBlocking) != hipSuccess)
        return bail(HSMA_E_DEVICE, "refinement stream creation failed");
    *out = sv;
    return HSMA_OK;
}

void hsma_server_destroy(hsma_server sv) {
    if (sv == nullptr) return;
    hipSetDevice(sv->device);
    hipStreamSynchronize(sv->stream);
    hipStreamSynchronize(sv->rstream);
    for (auto& kv : sv->all) {
        if (kv.second->ev) hipEventDestroy(kv.second->ev);
        delete kv.second;
    }
    for (hipEvent_t e : sv->inflight) hipEventDestroy(e);
    for (hipEvent_t e : sv->evpool) hipEventDestroy(e);
    for (int i = 0; i < hsma_server_s::RING; ++i) {
        hipFree(sv->dtab[i]);
        hipHostFree(sv->htab[i]);
        hipEventDestroy(sv->tabev[i]);
    }
    for (int w = 0; w < sv->nside; ++w) {
        hipStreamSynchronize(sv->side[w]);
        hipStreamDestroy(sv->side[w]);
        hipEventDestroy(sv->side_ev[w]);
    }
    hipEventDestroy(sv->fork_ev);
    hipStreamDestroy(sv->rstream);
    hipFree(sv->arena_base);
    hipHostFree(sv->host_base);
    hipStreamDestroy(sv->stream);
    delete sv;
}

static hsma_status submit_impl(hsma_server sv, hsma_plan plan, const double* x, const double* q,
                               int64_t N, bool copy, int64_t* id) {
    if (sv == nullptr || plan == nullptr || x == nullptr || q == nullptr || id == nullptr)
        return fail(HSMA_E_INVALID, "NULL argument");
    if (N < 1 || N > ((int64_t)1 << 26)) return fail(HSMA_E_INVALID, "N out of range");
    if ((plan->near_mode != HSMA_NEAR_BLOCK && plan->near_mode != HSMA_NEAR_TREE) ||
        plan->dipole_mode != HSMA_DIPOLE_EXACT || plan->far_mode != HSMA_FAR_SURFACE ||
        plan->bc == HSMA_BC_DIELECTRIC)
        return fail(HSMA_E_INVALID, "the server runs block near-set (direct or tree), exact-dipole "
                                    "plans of the periodic, grounded-cube and slab boxes only");
    Layout ly;
    if (req_device_bytes(plan, (int)N, sv->desc.precision, &ly) > sv->arena->cap() ||
        req_host_bytes((int)N) > sv->host_arena->cap()) {
        sv->stats.rejected += 1;
        return fail(HSMA_E_NOMEM, "request can never fit the server's memory");
    }
    SrvReq* r = new (std::nothrow) SrvReq();
    if (r == nullptr) return fail(HSMA_E_NOMEM, "host allocation failed");
    r->id = sv->next_id++;
    r->plan = plan;
    r->N = (int)N;
    if (copy) {
        r->hx.assign(x, x + 3 * N);
        r->hq.assign(q, q + N);
    } else {
        r->ext_x = x;
        r->ext_q = q;
    }
    r->t_submit = now_s();
    sv->pending.push_back(r);
    sv->all[r->id] = r;
    sv->stats.submitted += 1;
    *id = r->id;
    return HSMA_OK;
}

hsma_status hsma_server_submit(hsma_server sv, hsma_plan plan, const double* x, const double* q,
                               int64_t N, int64_t* id) {
    return submit_impl(sv, plan, x, q, N, true, id);
}

hsma_status hsma_server_tick(hsma_server sv) {
    if (sv == nullptr) return fail(HSMA_E_INVALID, "NULL server");
    return tick(sv);
}

hsma_status hsma_server_wait(hsma_server sv, int64_t id) {
    if (sv == nullptr) return fail(HSMA_E_INVALID, "NULL server");
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return fail(HSMA_E_INVALID, "unknown request id");
    while (it->second->state != ST_DONE) {
        if (it->second->state == ST_PENDING && sv->active.empty() && sv->inflight.empty() &&
            sv->pending.front() == it->second) {
            // nothing runs and the head of the queue does not fit: results that
            // were never read hold the pinned staging memory
            Layout ly;
            size_t off = 0;
            (void)ly;
            if (!sv->host_arena->alloc(req_host_bytes(it->second->N), &off))
                return fail(HSMA_E_NOMEM, "result staging full: read finished results first");
            sv->host_arena->release(off);
        }
        hsma_status st = tick(sv);
        if (st != HSMA_OK) return st;
        if (it->second->state == ST_COPYING || it->second->state == ST_REFINE_COPY) {
            HSMA_HIP(hipEventSynchronize(it->second->ev));
            retire(sv);
        }
    }
    return HSMA_OK;
}

hsma_status hsma_server_result(hsma_server sv, int64_t id, int* done, double* energy, double* phi,
                               double* forces, double* latency_s) {
    if (sv == nullptr || done == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return fail(HSMA_E_INVALID, "unknown request id");
    SrvReq* r = it->second;
    if (r->state != ST_DONE) {
        retire(sv);
        if (r->state != ST_DONE) {
            *done = 0;
            return HSMA_OK;
        }
    }
    *done = 1;
    if (energy) *energy = r->energy;
    if (phi) std::memcpy(phi, r->h_out + RES_D, sizeof(double) * r->N);
    if (forces) std::memcpy(forces, r->h_out + RES_D + r->N, sizeof(double) * 3 * r->N);
    if (latency_s) *latency_s = r->t_done - r->t_submit;
    const hsma_status st = r->status;
    sv->host_arena->release(r->host_off);
    sv->all.erase(it);
    delete r;
    if (st != HSMA_OK) return fail(st, "request failed its input checks");
    return HSMA_OK;
}

hsma_status hsma_server_stats(hsma_server sv, hsma_server_stats_t* out) {
    if (sv == nullptr || out == nullptr) return fail(HSMA_E_INVALID, "NULL argument");
    *out = sv->stats;
    out->active = (int)sv->active.size();
    out->pending = (int)sv->pending.size();
    out->arena_bytes = sv->arena->cap();
    out->arena_used = sv->arena->used();
    out->arena_peak = sv->arena->peak();
    return HSMA_OK;
}

// Open-loop replay: request i is submitted when the wall clock passes
// arrival_s[i] (seconds after the call starts); the server ticks until every
// request is done.  energies[i] and latencies_s[i] (completion minus arrival).
hsma_status hsma_server_run_trace(hsma_server sv, int64_t n, const double* arrival_s,
                                  const hsma_plan* plans, const double* const* xs,
                                  const double* const* qs, const int64_t* Ns, double* energies,
                                  double* latencies_s, double* wall_s) {
    if (sv == nullptr || n < 0 || arrival_s == nullptr || plans == nullptr || xs == nullptr ||
        qs == nullptr || Ns == nullptr || energies == nullptr || latencies_s == nullptr)
        return fail(HSMA_E_INVALID, "NULL argument");
    const double t0 = now_s();
    std::vector<int64_t> ids(n, 0);
    std::vector<double> tarr(n, 0.0);
    int64_t next = 0, done = 0;
    while (done < n) {
        const double t = now_s() - t0;
        while (next < n && arrival_s[next] <= t) {
            hsma_status st = submit_impl(sv, plans[next], xs[next], qs[next], Ns[next], false, &ids[next]);
            if (st != HSMA_OK) return st;
            SrvReq* r = sv->all[ids[next]];
            r->t_submit = t0 + arrival_s[next];
            tarr[next] = arrival_s[next];
            ++next;
        }
        if (busy(sv)) {
            hsma_status st = tick(sv);
            if (st != HSMA_OK) return st;
        }
        for (int64_t i = 0; i < next; ++i) {
            if (ids[i] == 0) continue;
            int dn = 0;
            double e = 0.0, lat = 0.0;
            hsma_status st = hsma_server_result(sv, ids[i], &dn, &e, nullptr, nullptr, &lat);
            if (st != HSMA_OK) return st;
            if (dn) {
                energies[i] = e;
                latencies_s[i] = lat;
                ids[i] = 0;
                ++done;
            }
        }
        if (!busy(sv) && next < n) {
            const double wait = arrival_s[next] - (now_s() - t0);
            if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 1e-3)));
        } else if (busy(sv) && sv->pending.empty()) {
            // everything admitted is on the device: wait for the oldest tick
            if (!sv->inflight.empty() && (next >= n || arrival_s[next] > now_s() - t0)) {
                HSMA_HIP(hipEventSynchronize(sv->inflight.front()));
                sv->evpool.push_back(sv->inflight.front());
                sv->inflight.pop_front();
            }
        }
    }
    if (wall_s) *wall_s = now_s() - t0;
    return HSMA_OK;
}

// The same replay with one plain double-precision solve per request, in
// arrival order (hsma_energy_forces_device on the caller's stream), for
// comparison with the batched server.
hsma_status hsma_run_trace_sequential(int64_t n, const double* arrival_s, const hsma_plan* plans,
                                      const double* const* xs, const double* const* qs,
                                      const int64_t* Ns, double* energies, double* latencies_s,
                                      double* wall_s) {
    if (n < 0 || arrival_s == nullptr || plans == nullptr || xs == nullptr || qs == nullptr ||
        Ns == nullptr || energies == nullptr || latencies_s == nullptr)
        return fail(HSMA_E_INVALID, "NULL argument");
    int64_t nmax = 1;
    size_t wsmax = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (plans[i] == nullptr) return fail(HSMA_E_INVALID, "NULL plan");
        nmax = std::max(nmax, Ns[i]);
        wsmax = std::max(wsmax, make_layout(plans[i], Ns[i], false).total);
    }
    char* buf = nullptr;
    const size_t nx = sizeof(double) * 3 * nmax, nq = sizeof(double) * nmax;
    if (hipMalloc((void**)&buf, 2 * nx + 2 * nq + wsmax + 1024) != hipSuccess)
        return fail(HSMA_E_NOMEM, "device allocation failed");
    double* dx = (double*)buf;
    double* dq = (double*)(buf + nx);
    double* dphi = (double*)(buf + nx + nq);
    double* dF = (double*)(buf + nx + 2 * nq);
    char* ws = buf + 2 * nx + 2 * nq;
    hipStream_t s = nullptr;
    const double t0 = now_s();
    for (int64_t i = 0; i < n; ++i) {
        double t = now_s() - t0;
        if (arrival_s[i] > t)
            std::this_thread::sleep_for(std::chrono::duration<double>(arrival_s[i] - t));
        if (hipMemcpyAsync(dx, xs[i], sizeof(double) * 3 * Ns[i], hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(dq, qs[i], sizeof(double) * Ns[i], hipMemcpyHostToDevice, s) != hipSuccess) {
            hipFree(buf);
            return fail(HSMA_E_DEVICE, "copy failed");
        }
        double e = 0.0;
        hsma_status st = hsma_energy_forces_device(plans[i], dx, dq, Ns[i], s, ws, wsmax, &e, dphi,
                                                   dF, nullptr);
        if (st != HSMA_OK) {
            hipFree(buf);
            return st;
        }
        energies[i] = e;
        latencies_s[i] = (now_s() - t0) - arrival_s[i];
    }
    if (wall_s) *wall_s = now_s() - t0;
    hipFree(buf);
    return HSMA_OK;
}

}  // extern "C"
