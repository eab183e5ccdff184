// Workspace layout and pipeline entry points of the update step.
#pragma once

#include "hsma_internal.h"
#include "tree.h"

namespace hsma {

struct Result {
    double energy;
    double qsum;
    double qabs;
    double qnet;  // net charge, summed before the finalize stage when NearFix::qc != 0
    int status;   // RS_* bits (result_status.h)
    int pad;
};

struct Layout {
    bool f32 = false;   // single-precision pair sums (records and partials sized for them)
    int N = 0;     // real particles
    int ns = 0;    // sources (2N for the slab: real + mirror)
    PairGeom g_rhs, g_near, g_surf, g_u, g_G;
    size_t off_src64 = 0, off_src32 = 0, off_rhs_part = 0, off_b = 0, off_A = 0, off_surf = 0;
    size_t off_near_part = 0, off_surf_part = 0, off_eblk = 0, off_result = 0;
    size_t off_u_part = 0, off_tw = 0, off_lam64 = 0, off_lam32 = 0, off_G_part = 0,
           off_real32 = 0, off_ud = 0;
    size_t off_cnt = 0, off_imgoff = 0, off_img64 = 0, off_img32 = 0;   // sphere near set
    // exact-coincidence check: open-addressing table of dup_T int slots (a
    // power of two >= 2N), each -1 or the index of a particle
    size_t off_dup = 0;
    int64_t dup_T = 0;
    int64_t img_max = 0;
    // near sum with each unordered pair once (block near set, any boundary
    // condition and precision); its accumulators replace the chunk partials
    bool sym = false;
    int sym_img = 0;   // IMG_* of the pair-once kernel (IMG_SLAB for the slab)
    SymGeom g_sym;
    int n_eblk = 1;
    size_t total = 0;
    // every stage on the caller's stream (no auxiliary stream or events are
    // created): the allocation-free entry point
    bool single_stream = false;
    // tree-code near sum (HSMA_NEAR_TREE): its own workspace at off_tree
    bool tree = false;
    TreeLayout tl;
    size_t off_tree = 0;
};

// What the finalize stages add to the near potential of particle i:
// q_i * own + Q * qc, Q the net charge (Result::qnet).  With the block near
// set of the periodic cube and of the slab (its doubled cube), own restores
// the particle's own periodic images, which the near-sum kernels leave out,
// less the per-pair shift of the single-precision kernels (OWN_COLS_F32 / L,
// images_sum SHIFT); qc restores that shift for the other charges (periodic
// cube; in the slab the mirror charges cancel it).  Both are 0 otherwise.
struct NearFix {
    double own = 0.0, qc = 0.0;
};
// A named range for profilers (rocprofv3 --marker-trace) over a scope of host
// code (the enqueueing of a stage): with HSMA_ROCTX=1 in the environment (read
// once per process) the roctx library is loaded at first use; otherwise, or
// if it cannot be loaded, a no-op.  name must outlive the range.
class Range {
  public:
    explicit Range(const char* name);
    ~Range();
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;

  private:
    bool on_ = false;
};

// The fixed near-potential terms for plan pl under layout ly.
NearFix near_fix(const hsma_plan_s* pl, const Layout& ly);

// no_tree: the direct near kernels even where the plan would use the tree.
Layout make_layout(const hsma_plan_s* pl, int64_t N, bool grad, int tpl_near_override = 0,
                   int precision_override = -1, bool no_tree = false);
// dtype (HSMA_DTYPE_F64 or HSMA_DTYPE_F32) is the type of x, q, phi and forces.
hsma_status forward(const hsma_plan_s* pl, const Layout& ly, const void* x, const void* q,
                    int dtype, char* ws, hipStream_t s, void* phi, void* forces,
                    const hsma_intermediates* dbg);
hsma_status backward(const hsma_plan_s* pl, const Layout& ly, char* ws, hipStream_t s,
                     double* dEdx, double* dEdq);
hsma_status read_result(const Layout& ly, char* ws, hipStream_t s, double* energy);
// Argument checks of the update-step entry points (plan, N).
hsma_status check_sizes(const hsma_plan_s* pl, int64_t N);
hsma_status build_plan(hsma_plan_s* pl);
void free_plan(hsma_plan_s* pl);

}  // namespace hsma
