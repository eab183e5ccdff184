/*
 * hsma.h -- C ABI of the MI355X (gfx950) hot path of the harmonic surface
 * mapping algorithm (HSMA) of Zhao, Liang & Xu, "Harmonic surface mapping
 * algorithm for fast electrostatic sums", arXiv:1806.04801.
 *
 * Problem (paper Sec. II, Eq. (sum)): N point charges q_j at r_j in a cube of
 * side L with a boundary condition represented by image charges; in Gaussian
 * units the potential is Phi(r) = sum q / |r - r'| over sources and images.
 * The library returns the energy E = 1/2 sum_i q_i phi_i, the per-particle
 * potential phi_i (bare self term left out, self-images included) and the
 * forces F_i = q_i E(r_i) = -q_i grad phi(r_i) with the harmonic coefficients
 * held fixed (paper Sec. III, forces as gradients of the potential).
 *
 * Conventions shared by every entry point:
 *   - Coordinates are API coordinates: [0, L)^3 for periodic and grounded
 *     cube, [0, L) x [0, L) x [0, L/2] for the grounded slab.  Arrays of
 *     positions and forces are N x 3 row-major doubles; charges N doubles.
 *   - Periodic positions are wrapped into the box; grounded-cube and slab
 *     positions must lie strictly inside (HSMA_E_OUT_OF_BOX otherwise).
 *   - Periodic and slab systems must be neutral: |sum q| <= 1e-12 sum |q|
 *     (HSMA_E_NOT_NEUTRAL).
 *   - Two charges at exactly the same position (compared after periodic
 *     wrapping) have an infinite interaction: HSMA_E_COINCIDENT.  Close but
 *     distinct positions are accepted.
 *   - The periodic potential is defined up to a constant; the library fixes
 *     it by A_00 = 0 (the constant harmonic carries no information in the
 *     periodic residual of Sec. II.A).
 *   - No exception crosses the ABI.  Every function returns a status; the
 *     text of the last error of the calling thread is in hsma_last_error().
 *     After an error the contents of output arrays are unspecified.
 *   - The caller owns every array it passes.  A plan owns its device-resident
 *     matrices and is immutable after creation: it may be used from several
 *     host threads on distinct streams, each with its own workspace.
 */
#ifndef HSMA_H
#define HSMA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HSMA_BC_PERIODIC = 0,        /* periodic in x, y, z (Sec. II, periodic image sum) */
    HSMA_BC_METALLIC = 1,        /* grounded cube: Eq. (diel) in the conducting limit gamma = -1 */
    HSMA_BC_SLAB_METALLIC_Z = 2, /* periodic in x, y, grounded walls at z = 0 and z = L/2 (mirror
                                    reflections plus periodic extension, Sec. I) */
    HSMA_BC_DIELECTRIC = 3       /* dielectric box: the image series of Eq. (diel) with weight
                                    gamma^|k|, |gamma| < 1 (hsma_plan_desc.gamma); the far images
                                    (shells 2..far_shells of the image lattice) are summed at the
                                    monitoring points and fitted; double precision, block near
                                    set (direct, or the fast multipole method of HSMA_NEAR_TREE),
                                    no adjoint and no serving */
} hsma_bc;

typedef enum {
    HSMA_FP64 = 0,        /* every sum in double precision */
    HSMA_FP32_COMP = 1    /* near and right-hand-side pair sums in single precision with
                             two-sum compensated accumulation; basis, least squares, mapping,
                             surface sum and final reductions in double precision */
} hsma_precision;

typedef enum {
    HSMA_NEAR_BLOCK = 0,   /* near set: the 27 images of every source in the 3x3x3 block of boxes */
    HSMA_NEAR_SPHERE = 1,  /* near set: every image inside the auxiliary sphere |r| < R_s (the
                              paper's literal near set, Sec. II.A); images generated per call;
                              no adjoint and no serving in this mode */
    HSMA_NEAR_TREE = 2     /* near set of HSMA_NEAR_BLOCK; from hsma_plan_desc.tree_min_n
                              particles on, the near sum and the right-hand side are summed by
                              the fast multipole method instead of directly (the O(N)
                              acceleration of Sec. II.C, Table I): multipole and local
                              expansions of order hsma_plan_desc.tree_order about the cells of a
                              uniform octree over the 27 boxes (at most HSMA_TREE_LEAF images
                              per leaf cell, 1000 by default), direct sums between neighbouring
                              leaf cells, in double precision whatever the plan's precision;
                              below tree_min_n the direct kernels of HSMA_NEAR_BLOCK in the
                              plan's precision; at most (2^31 - 1) / 27 sources on the tree
                              (HSMA_E_INVALID above); every box; no adjoint */
} hsma_near_mode;

typedef enum {
    HSMA_DIPOLE_EXACT = 0,  /* surface dipole as exact point dipoles (limit of Eq. (cd)) */
    HSMA_DIPOLE_LAYERS = 1  /* the paper's form: the dipole layer replaced by two charge layers
                               on the spheres R_s -+ dr/2 (Eq. (cd), Eq. (integrals)), i.e. three
                               point charges per surface point; double precision; no adjoint and
                               no serving in this mode */
} hsma_dipole_mode;

typedef enum {
    HSMA_FAR_SURFACE = 0,  /* far field through the harmonic surface mapping (Sec. II.B) */
    HSMA_FAR_DIRECT = 1    /* far field as the fitted series sum_k A_k B_k(r) and its gradient,
                              evaluated at the particles (double precision); no adjoint and no
                              serving in this mode */
} hsma_far_mode;

typedef enum {
    HSMA_OK = 0,
    HSMA_E_INVALID = -1,      /* bad argument (sizes, NULL, non-finite input, K < unknowns, R <= R0) */
    HSMA_E_NOT_NEUTRAL = -2,  /* periodic or slab system with non-zero total charge */
    HSMA_E_OUT_OF_BOX = -3,   /* grounded-cube or slab position on or outside a wall */
    HSMA_E_COINCIDENT = -4,   /* two charges at exactly the same position (after periodic wrapping) */
    HSMA_E_NOMEM = -5,        /* device allocation failed or workspace too small */
    HSMA_E_DEVICE = -6,       /* HIP runtime error */
    HSMA_E_ILLCOND = -7,      /* least-squares matrix numerically rank deficient */
    HSMA_E_NONFINITE = -8     /* the energy, a potential or a force came out non-finite although
                                 the input passed every check (e.g. two distinct charges closer
                                 than single precision resolves); outputs are not usable */
} hsma_status;

typedef struct hsma_plan_s* hsma_plan;

/* Full plan description; hsma_plan_create fills the defaults. */
typedef struct {
    double L;          /* box side (> 0) */
    int bc;            /* hsma_bc */
    int p;             /* harmonic truncation degree P >= 1 (Eq. (harmonic)); N_b = (P+1)^2 */
    int M;             /* requested Fibonacci surface points; the plan uses the Hannay-Nye count
                          2(F2+1) nearest to M (Sec. II.B), reported as M_eff */
    int K;             /* monitoring points N_m (Sec. II.A); K >= unknowns */
    double R;          /* auxiliary sphere radius R_s > sqrt(3) L / 2 (alpha > 1, Sec. III) */
    int precision;     /* hsma_precision */
    uint64_t seed;     /* SplitMix64 seed of the grounded-cube face monitoring points */
    int near_mode;     /* hsma_near_mode (hsma_plan_create: HSMA_NEAR_BLOCK) */
    int dipole_mode;   /* hsma_dipole_mode (hsma_plan_create: HSMA_DIPOLE_EXACT) */
    double dr;         /* layer spacing for HSMA_DIPOLE_LAYERS; <= 0 selects 1e-5 R_s */
    int far_mode;      /* hsma_far_mode (hsma_plan_create: HSMA_FAR_SURFACE) */
    double gamma;      /* HSMA_BC_DIELECTRIC: image weight (1 - eps)/(1 + eps), |gamma| < 1
                          (Eq. (diel)); ignored otherwise */
    int far_shells;    /* HSMA_BC_DIELECTRIC: far image shells S, images with
                          2 <= max_a |k_a| <= S; 0 picks the smallest S whose omitted tail is
                          below 1e-13 sum|q|/L at the monitoring points */
    int tree_order;    /* HSMA_NEAR_TREE: expansion order, 1..20 (0 selects 16) */
    int tree_min_n;    /* HSMA_NEAR_TREE: the fast multipole method from this many particles
                          on, >= 1 (0 selects 16384 for HSMA_FP64 plans and 24576 for
                          HSMA_FP32_COMP plans, near the measured crossovers with the direct
                          double- and single-precision near sums) */
} hsma_plan_desc;

typedef struct {
    int n_basis;       /* N_b = (P+1)^2 */
    int n_unknowns;    /* fitted coefficients: N_b (grounded cube) or N_b - 1 (periodic, slab) */
    int K;             /* monitoring points */
    int n_check;       /* evaluation points of the right-hand side: K, or 2K with the twins */
    int M_eff;         /* surface points 2(F2+1) */
    int F1, F2;        /* Fibonacci pair of the surface quadrature */
    double R0;         /* circumsphere radius sqrt(3) L / 2 */
    double Rs;         /* auxiliary sphere radius */
    int precision;
    int bc;
    size_t bytes_resident;  /* device bytes held by the plan */
    int near_mode;
    int max_images_per_source;  /* near images per source: 27, or the sphere-mode bound */
    int dipole_mode;
    double dr;
    int far_mode;
    double gamma;      /* dielectric box: image weight */
    int far_shells;    /* dielectric box: far image shells in use */
    int tree_order;    /* tree near sum: multipole order in use */
    int tree_min_n;    /* tree near sum: used from this many particles on */
} hsma_plan_info_t;

/* Optional device outputs of the intermediate stages (any pointer may be NULL). */
typedef struct {
    double* b;           /* K values of the least-squares right-hand side */
    double* A;           /* N_b coefficients A_nm, index n^2 + n + m */
    double* surf;        /* M_eff x 8: X, Y, Z, Q, p_x, p_y, p_z, 0 of the surface images
                            (exact-dipole plans; not written with charge layers) */
    double* phi_near;    /* N near-field potentials */
    double* field_near;  /* N x 3 near fields */
    double* phi_out;     /* N far-field potentials (surface images) */
    double* field_out;   /* N x 3 far fields */
} hsma_intermediates;

/* Profiler ranges: with HSMA_ROCTX=1 in the environment (read once per
   process) the library loads the roctx library (rocprofiler-sdk or roctx64)
   and marks every update step ("hsma: update step", "hsma: update step (fast
   multipole)") and every server tick ("hsma: server tick") as a range over
   the host code that enqueues it, for rocprofv3 --marker-trace. */

/* Status text and the calling thread's last error message.  hsma_version()
   is the version of this interface; it changes whenever a declaration or a
   struct layout in this header changes (2: the near-schedule query and the
   server's double-precision refinement; 3: HSMA_E_COINCIDENT; 4:
   HSMA_E_NONFINITE; 5: the dielectric box; 6: the tree-code near sum and
   hsma_energy_forces_device_typed). */
const char* hsma_status_string(int status);
const char* hsma_last_error(void);
int hsma_version(void);

/*
 * Preparation step (Sec. II.C, Table I): monitoring points (Fibonacci grid on
 * the circumsphere with twins for periodic systems, seeded points on the faces
 * of the grounded cube), the fitting matrix of real solid harmonics r^n Y_nm,
 * its Householder QR, the pseudo-inverse R^-1 Q^T, the Hannay-Nye points and
 * weights on the sphere R_s and the mapping matrix.  Runs on the current HIP
 * device and keeps every matrix resident there.  *out receives the plan.
 * Errors: HSMA_E_INVALID, HSMA_E_NOMEM, HSMA_E_DEVICE, HSMA_E_ILLCOND.
 */
hsma_status hsma_plan_create(double L, int bc, int p, int M, int K, double R, hsma_plan* out);
hsma_status hsma_plan_create_ex(const hsma_plan_desc* desc, hsma_plan* out);
void        hsma_plan_destroy(hsma_plan plan);
hsma_status hsma_plan_info(hsma_plan plan, hsma_plan_info_t* info);

/*
 * Host copies of plan geometry, in centred coordinates (box centred at 0):
 *   which = 0: monitoring points (K x 3)      w unused
 *   which = 1: twin points (K x 3, periodic)  w unused
 *   which = 2: surface points (M_eff x 3)     w = quadrature weights (M_eff)
 * xyz and w are host arrays of the stated sizes (w may be NULL).
 */
hsma_status hsma_plan_points(hsma_plan plan, int which, double* xyz, double* w);

/* Device bytes of workspace needed by the device entry points for N particles. */
size_t hsma_workspace_bytes(hsma_plan plan, int64_t N);
/* For tuning, HSMA_TPL_NEAR and HSMA_TPL_RHS in the environment set the
 * targets per lane (1 or 2; other values are ignored) of the per-target near
 * tiles and of the right-hand-side tiles; defaults 1, and 2 for the near tiles
 * of the sphere near set.  These and the HSMA_SYM variables of
 * hsma_near_schedule change the workspace size, so they must not change
 * between this query and the calls that use the workspace. */

/*
 * The near-field kernel that an update step with N particles runs, and its
 * schedule (the near sum of Sec. II.C over the 3x3x3 image block).
 *   kind 0: per-target tiles; each lane sums every source image for its own
 *           targets, so each ordered (target, image) pair is evaluated once.
 *   kind 1: each unordered particle pair is evaluated once and both of its
 *           directions are accumulated (the image-block sum is symmetric in
 *           the two particles; for the slab, the real charges with the
 *           periodic blocks of each charge and of its mirror).  Either
 *           precision, every boundary condition, block near set, N at or
 *           above a threshold (1024 in either precision,
 *           the same for requests of the batched server; the environment
 *           variable HSMA_SYM_MIN overrides it);
 *           HSMA_SYM=0 in the environment turns it off and HSMA_SYM=1 forces
 *           it; for tuning, HSMA_SYM_T (rows per lane: 1, the default, or 2;
 *           0 picks by occupancy), HSMA_SYM_Q (2
 *           or 4 columns per reverse group) and HSMA_SYM_ROUNDS (target round
 *           count) override the choices the library makes.  The particles are cut
 *           into `blocks` blocks of `block`; block pairs run in blocks - 1
 *           (+1 if odd) round-robin rounds after one diagonal launch; a block
 *           pair is split into `slices` row slices of 64 * rows_per_lane rows
 *           and `parts` column parts, one wave each; `launches` counts every
 *           kernel launch of the sum.
 *   kind 2: the fast multipole method (HSMA_NEAR_TREE plans from tree_min_n
 *           particles on).
 * Fields other than kind are 0 for kinds 0 and 2.  Returns HSMA_E_INVALID for a NULL
 * plan or output, or N < 1.
 */
typedef struct {
    int kind;
    int rows_per_lane;
    int block;
    int slices;
    int parts;
    int blocks;
    int launches;
} hsma_near_schedule_t;

hsma_status hsma_near_schedule(hsma_plan plan, int64_t N, hsma_near_schedule_t* out);

/*
 * Update step (Sec. II.C) on host arrays: x (N x 3), q (N); outputs energy
 * (one double), phi (N or NULL) and forces (N x 3 or NULL).  The device
 * buffers live in the plan: the first call, and a call with a larger N than
 * any before, allocate; later calls reuse them.  Calls on one plan run one at
 * a time (a lock of the plan); the call synchronizes before returning.
 */
hsma_status hsma_energy_forces(hsma_plan plan, const double* x, const double* q, int64_t N,
                               double* energy, double* phi, double* forces);

/*
 * Update step on device arrays (all pointers device memory of the plan's
 * device): x (N x 3), q (N), phi (N or NULL), forces (N x 3 or NULL),
 * workspace of hsma_workspace_bytes(plan, N) bytes, all work enqueued on
 * `stream` (a hipStream_t; NULL = default stream).  energy is a host double
 * written after the stream has drained (the call waits for it).  dbg (may be
 * NULL) requests copies of the intermediate stages.  The right-hand-side
 * chain runs on an auxiliary non-blocking stream of the calling host thread
 * (created on its first call on a device), forked from `stream` and joined
 * back into it with events, so that all of a call's work stays ordered on
 * `stream`; HSMA_OVERLAP=0 in the environment (read once per process) keeps
 * it on `stream` itself.
 */
hsma_status hsma_energy_forces_device(hsma_plan plan, const double* x, const double* q, int64_t N,
                                      void* stream, void* workspace, size_t workspace_bytes,
                                      double* energy, double* phi, double* forces,
                                      const hsma_intermediates* dbg);

/*
 * The update step of hsma_energy_forces_device on device arrays of either
 * precision (the interface's dtype argument): dtype HSMA_DTYPE_F64 (double)
 * or HSMA_DTYPE_F32 (float) is the element type of x (N x 3 row-major), q
 * (N), phi (N or NULL) and forces (N x 3 or NULL).  Single-precision inputs
 * are widened to double on the device before anything else (the arithmetic
 * is then the plan's, Sec. II.C); phi and forces are rounded to single
 * precision on output, the energy is a host double.  Workspace, stream,
 * ownership and errors as in hsma_energy_forces_device (HSMA_E_INVALID for
 * any other dtype).
 */
#define HSMA_DTYPE_F64 0
#define HSMA_DTYPE_F32 1
hsma_status hsma_energy_forces_device_typed(hsma_plan plan, const void* x, const void* q, int64_t N,
                                            int dtype, void* stream, void* workspace,
                                            size_t workspace_bytes, double* energy, void* phi,
                                            void* forces);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the update
 * step of hsma_energy_forces_device, with the same kernels and results, run
 * in a static device scratch array of HSMA_NOALLOC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends, instead
 * of a caller workspace.  Every stage runs on `stream` (no auxiliary stream
 * or event is created).  x, q, phi, forces: device arrays as in
 * hsma_energy_forces_device; energy: host double, written after the stream
 * has drained.  The call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).  HSMA_E_NOMEM when the step for N particles
 * needs more scratch than the array holds (hsma_workspace_bytes(plan, N) is
 * an upper bound of the need; about 3e4 particles fit at p = 20).  All calls
 * on one device share its array and it keeps the last call's contents: calls
 * that overlap on one device (other host threads, other streams) race and
 * must be serialized by the caller.
 */
#define HSMA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
hsma_status hsma_energy_forces_noalloc(hsma_plan plan, const double* x, const double* q, int64_t N,
                                       void* stream, double* energy, double* phi, double* forces);

/*
 * Exact gradient of the computed energy (adjoint of the update step):
 * dEdx (N x 3) and dEdq (N) on the device, energy on the host.  Unlike the
 * forces above, -dEdx also differentiates the least-squares coefficients with
 * respect to the positions.  Same conventions as hsma_energy_forces_device.
 */
hsma_status hsma_energy_grad_device(hsma_plan plan, const double* x, const double* q, int64_t N,
                                    void* stream, void* workspace, size_t workspace_bytes,
                                    double* energy, double* dEdx, double* dEdq);

/*
 * Kernel timing for measurement: when enabled, the library records HIP events
 * around every launch of the near-field pair kernel (kernel class 0), the
 * right-hand-side pair kernel (1) and the surface kernel (2) on the stream it
 * launches them on.  hsma_timing_read waits for the recorded events, returns
 * the summed milliseconds and launch counts per class (arrays of 3) and
 * clears the record.
 */
hsma_status hsma_timing_enable(int enable);
hsma_status hsma_timing_read(double* ms, int64_t* launches);

/*
 * Serving: continuous batching of energy/force requests (update steps of
 * possibly different N, boundary condition and plan) on one GPU.
 *
 * A server owns a device arena of memory_bytes for the inputs, outputs and
 * workspace of admitted requests, a pinned host staging area for their
 * results, max_active request slots and a stream.  Requests wait in a FIFO
 * queue until a slot is free and the arena has room (admission by memory).
 * Each hsma_server_tick admits what fits and enqueues one round of grouped
 * launches in which every active request advances one stage; the pair tiles of
 * all requests in the round share one launch per kind (near, right-hand
 * side, surface).  The pair-once near sums of requests at or above the
 * threshold of hsma_near_schedule run on a few side streams of the server
 * (HSMA_SRV_STREAMS in the environment, 1 to 8, default 3, read at server
 * creation), forked from the server stream and joined back within the round,
 * so that the near sums of several requests and the grouped launches of the
 * others run on the GPU at the same time.  A round admits requests while
 * their pair work (27 N_s (N + check points) pair-images each) stays within a
 * budget (HSMA_SRV_TICK_WORK in the environment, default 1.5e11, read at
 * server creation; a larger request is admitted alone), so that rounds stay
 * short and a finished request's slot goes to the queue within a few rounds.  A request's arithmetic depends
 * only on its own inputs and plan, so its result is bitwise the same alone and
 * in any mix.  precision selects the pair sums of every request
 * (HSMA_FP32_COMP: single precision with two-sum accumulation; HSMA_FP64);
 * plans only contribute their geometry and matrices.  A server is used from
 * one host thread; plans must outlive the requests that use them.
 */
typedef struct hsma_server_s* hsma_server;

typedef struct {
    size_t memory_bytes;   /* device arena for admitted requests (>= 1 MiB) */
    int max_active;        /* request slots (>= 1) */
    int precision;         /* hsma_precision of the pair sums */
    double refine_below;   /* 0 = off; applies to the requests of an
                              HSMA_FP32_COMP server and to the requests on the
                              fast multipole method of either: a request whose
                              energy E comes out with |E| below refine_below
                              times 1/2 sum |q_i phi_i| is recomputed with the
                              direct double-precision sums before it completes.  The single-
                              precision error is a small fraction (~4e-9) of
                              that sum, so it is a large relative error only
                              when E is a small difference of large terms;
                              3e-3 kept every energy of a 4096-request
                              synthetic serving mix within 1e-5 of the double-
                              precision one (2 % of the requests refined). */
} hsma_server_desc;

typedef struct {
    int64_t submitted, completed, rejected;
    int active, pending;
    int64_t ticks, tiles;
    size_t arena_bytes, arena_used, arena_peak;
    int64_t refined;       /* requests recomputed in double precision */
} hsma_server_stats_t;

hsma_status hsma_server_create(const hsma_server_desc* desc, hsma_server* out);
void        hsma_server_destroy(hsma_server server);

/* Queue a request; x (N x 3) and q (N) are host arrays, copied.  *id receives
   its handle.  HSMA_E_NOMEM if it could never fit the arena.  The plan must use
   the block near set (HSMA_NEAR_BLOCK, or HSMA_NEAR_TREE: the fast multipole
   method from its tree_min_n on, in double precision whatever the server's
   precision), exact dipoles and the surface mapping, and a periodic, grounded
   cube or slab box (else HSMA_E_INVALID).  The double-precision refinement of
   refine_below recomputes with the direct sums. */
hsma_status hsma_server_submit(hsma_server server, hsma_plan plan, const double* x,
                               const double* q, int64_t N, int64_t* id);

/* One scheduling round (admission, grouped launches, retirement). */
hsma_status hsma_server_tick(hsma_server server);

/* Tick until request id has finished. */
hsma_status hsma_server_wait(hsma_server server, int64_t id);

/* Non-blocking result read: *done = 0 while running; when done, copies the
   energy, phi (N, or NULL) and forces (N x 3, or NULL) to host arrays, the
   latency from submission to completion, and releases the request. */
hsma_status hsma_server_result(hsma_server server, int64_t id, int* done, double* energy,
                               double* phi, double* forces, double* latency_s);

hsma_status hsma_server_stats(hsma_server server, hsma_server_stats_t* stats);

/* Open-loop replay of a request trace through the server: request i (plan
   plans[i], host arrays xs[i], qs[i] of Ns[i] particles, which must stay valid)
   arrives arrival_s[i] seconds after the call starts (non-decreasing).  Fills
   energies[i], latencies_s[i] (completion minus arrival) and the wall time. */
hsma_status hsma_server_run_trace(hsma_server server, int64_t n, const double* arrival_s,
                                  const hsma_plan* plans, const double* const* xs,
                                  const double* const* qs, const int64_t* Ns, double* energies,
                                  double* latencies_s, double* wall_s);

/* The same replay with one hsma_energy_forces_device call per request in
   arrival order (each plan's own precision), for comparison. */
hsma_status hsma_run_trace_sequential(int64_t n, const double* arrival_s, const hsma_plan* plans,
                                      const double* const* xs, const double* const* qs,
                                      const int64_t* Ns, double* energies, double* latencies_s,
                                      double* wall_s);

#ifdef __cplusplus
}
#endif

#endif /* HSMA_H */
