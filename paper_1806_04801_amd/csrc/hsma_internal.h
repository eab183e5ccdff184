// Internal declarations of the HSMA library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hsma.h"

namespace hsma {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
hsma_status fail(hsma_status st, const std::string& msg);
#define HSMA_HIP(call)                                                               \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::hsma::fail(HSMA_E_DEVICE, std::string(#call) + ": " +          \
                                               hipGetErrorString(e_));               \
    } while (0)

// ---------------------------------------------------------------- geometry modes
// Image maps of the 3x3x3 near block (k in {-1,0,1}^3), applied to a source r:
//   IMG_PERIODIC: r + kL,                  charge q           (periodic sum)
//   IMG_METALLIC: (-1)^k o r + kL,         charge (-1)^|k| q  (Eq. (diel), gamma = -1)
//   IMG_FREE    : r only (no images)
//   IMG_SLAB    : the mirror-doubled periodic cube of the slab, taken over
//                 the real charges only: r + kL with charge q and
//                 (x, y, -z) + kL with charge -q (pair-once kernel only)
//   IMG_DIELECTRIC: the positions of IMG_METALLIC with weight gamma^|k| q
//                 (Eq. (diel), |gamma| < 1; per-target tiles in double)
enum { IMG_PERIODIC = 0, IMG_METALLIC = 1, IMG_FREE = 2, IMG_SLAB = 3, IMG_DIELECTRIC = 4 };

// Potential of the 26 images k != 0 of a unit charge at the origin in the
// periodic 3x3x3 block of unit boxes: 6 + 12 / sqrt(2) + 8 / sqrt(3).  The
// block near-sum kernels leave a particle's own periodic images out and the
// finalize stages add q_i * OWN_IMAGES_PERIODIC / L in double.
constexpr double OWN_IMAGES_PERIODIC = 19.1040835277555764088833;

// The same potential split over the nine columns (k_x, k_y) of the block
// (k_z = -1, 0, 1), rounded to float: the central column (k_x = k_y = 0) 2,
// the four edge columns 1 + sqrt(2), the four corner columns
// 1 / sqrt(2) + 2 / sqrt(3).  The single-precision near sum subtracts them
// per column (images_sum, SHIFT); OWN_COLS_F32 is their sum, exact in double.
constexpr float OWN_COL_CENTRE = 2.0f;
constexpr float OWN_COL_EDGE = 2.41421356237309504880f;
constexpr float OWN_COL_CORNER = 1.86180731956579905342f;
constexpr double OWN_COLS_F32 =
    (double)OWN_COL_CENTRE + 4.0 * (double)OWN_COL_EDGE + 4.0 * (double)OWN_COL_CORNER;

// Single-precision record of a point (target or source), in units of the box
// side L (so the box is [-1/2, 1/2]^3): the centred coordinate c = h0 + l with
// h0 a multiple of 2^-24 and |l| <= 2^-25, so that h0 - 1/2 and h0 + 1/2 are
// exact in float and every image difference keeps its leading part exact
// for close pairs and near walls (Sterbenz); plus the charge.
//   v[0] = (h0x, h0y, h0z, q)
//   v[1] = (hpx, hpy, hpz, lx)      hp = h0 - 1/2
//   v[2] = (hmx, hmy, hmz, ly)      hm = h0 + 1/2
//   v[3] = (lz, 0, 0, 0)
struct Rec32 {
    float4 v[4];
};

// Workspace / launch geometry of a pair-kernel launch.
struct PairGeom {
    int nt = 0;       // targets
    int ns = 0;       // sources
    int tpl = 1;      // targets per lane
    int ntb = 0;      // target blocks (grid.x)
    int nt_pad = 0;   // ntb * 256 * tpl
    int S = 1;        // source chunks (grid.y)
    int chunk = 0;    // sources per chunk
};
PairGeom pair_geometry(int nt, int ns, int tpl, int ncu, int min_chunk = 64);

// Geometry of the near sum that visits every unordered particle pair once:
// blocks of B = 64 * T * s particles, nb blocks (P = nb rounded up to even),
// each block pair split into s row slices and C column parts (one wave each),
// accumulators padded to n_pad = nb * B per component.
struct SymGeom {
    int n = 0;       // particles
    int T = 1;       // rows per lane
    int s = 1;       // row slices per block
    int C = 1;       // column parts per block (one wave per slice and part)
    int B = 64;      // block size
    int nb = 0;      // blocks
    int P = 0;       // nb rounded up to even: P - 1 rounds
    int n_pad = 0;   // nb * B
};
// Single precision: T = 1 or 2 rows per lane, or 0 to choose the one whose
// rounds fill the GPU better (resident waves from the occupancy of each kernel
// variant); the library uses 1, which measured at least as fast everywhere.
// Double precision (f64): one row per lane.
SymGeom sym_geometry(int n, int T, bool f64, int img, int ncu);

// One group of tiles of a grouped pair launch: all tiles of one pair stage of
// one request.  Tile i of the group (0 <= i < ntb * S) is target block
// i % ntb against source chunk i / ntb; work-group g of the launch runs tile
// g - first of the group whose range [first, first + ntb * S) holds g.
enum { TILE_NEAR = 0, TILE_RHS = 1, TILE_SURFACE = 2 };
struct TileGroup {
    int kind, img;        // TILE_*, IMG_* (near and right-hand side)
    int first;            // index of the group's first tile in the launch
    int ntb, S;           // target blocks, source chunks
    int nt, ns, chunk, nt_pad;
    int pad;
    const void* tgt;      // Rec32 / double4 targets
    const void* src;      // Rec32 / double4 sources, or surface records (8 doubles)
    double* out;          // partial buffer of the request's stage
    double L;             // box side (physical units)
};

// A device pointer read from a descriptor in memory, marked as global memory
// (an integer converted to a global pointer), so that accesses through it
// compile to global or scalar loads instead of flat ones.
template <typename P>
__device__ __forceinline__ P* global_ptr(P* p) {
    return (P*)(__attribute__((address_space(1))) P*)(uintptr_t)p;
}

// Periodic and slab systems must be neutral (their energy diverges
// otherwise); grounded and dielectric boxes need not be.
inline bool needs_neutral(int bc) { return bc == HSMA_BC_PERIODIC || bc == HSMA_BC_SLAB_METALLIC_Z; }

// Far image shells S of a dielectric box (image weight gamma) whose omitted
// tail is below tol * sum|q| / L on the circumsphere: shell s >= 2 holds
// images with |k| >= s at distance >= (s - 1/2 - sqrt(3)/2) L from the
// circumsphere's points, and its weights sum to at most 6 |gamma|^s c^2,
// c = 1 + 2|gamma|/(1 - |gamma|).
int far_shell_count(double gamma, double tol);

// ---------------------------------------------------------------- plan
struct hsma_plan_impl;
}  // namespace hsma

struct hsma_plan_s {
    hsma_plan_desc desc{};
    int device = 0;
    int ncu = 256;
    int bc = 0;
    int img = 0;          // image mode of the near block (periodic also for slab)
    int p = 0, nb = 0, nu = 0, K = 0, nchk = 0, M = 0, F1 = 0, F2 = 0;
    double L = 1.0, R0 = 0.0, Rs = 0.0;
    int precision = 0;
    int near_mode = 0;
    int kr = 1;           // sphere mode: images with |k_a| <= kr are candidates
    int maxper = 27;      // near images per source (upper bound in sphere mode)
    int dipole_mode = 0;  // HSMA_DIPOLE_EXACT or HSMA_DIPOLE_LAYERS
    double dr = 0.0;      // layer spacing (charge-layer dipoles)
    int far_mode = 0;     // HSMA_FAR_SURFACE or HSMA_FAR_DIRECT
    double gamma = 0.0;   // dielectric box: image weight
    int far_shells = 0;   // dielectric box: far image shells
    int tree_order = 0;   // tree near sum: multipole order
    int tree_min_n = 0;   // tree near sum: used from this many particles on
    // host geometry (centred)
    std::vector<double> chk;    // nchk x 3: monitoring points then twins
    std::vector<double> spts;   // M x 3
    std::vector<double> swts;   // M
    // device-resident matrices (row-major)
    double* d_P = nullptr;      // nu x K   pseudo-inverse R^-1 Q^T
    double* d_Wq = nullptr;     // M x nb   charge rows  (w_j / (4 pi Rs)) n B_k(R_j)
    double* d_Wp = nullptr;     // M x nb   dipole rows  -(w_j / (4 pi)) B_k(R_j)
    double* d_spos = nullptr;   // M x 4    surface points (X, Y, Z, 0)
    double4* d_chk64 = nullptr; // nchk     check points (x, y, z, 0)
    hsma::Rec32* d_chk32 = nullptr;  // nchk single-precision records
    int* d_chk_order = nullptr;      // nchk check points in Morton order of position (tree right-hand side)
    size_t bytes = 0;
    // device buffer of the host-array entry point (inputs, outputs and
    // workspace), kept between calls and grown when a call needs more; calls
    // of that entry point on one plan take the mutex in turn
    std::mutex host_mu;
    char* host_buf = nullptr;
    size_t host_cap = 0;
};

namespace hsma {

// ---------------------------------------------------------------- kernels
// Pair sums (pairs.hip).  out layout: out[(c * ncomp + comp) * nt_pad + t],
// comp 0 = potential, 1..3 = field E = -grad phi; c = source chunk.
hipError_t launch_pair_f64(int img, bool field, bool self, const double4* tgt, const double4* src,
                           const PairGeom& g, double L, double* out, hipStream_t s,
                           double gamma = 0.0);
// Far images of a dielectric box at points (right-hand side): out[c * nt_pad + t]
// = -sum over the sources of chunk c and the images in shells 2..S of
// gamma^|k| q / |tgt_t - I_k(r)|.
hipError_t launch_far_shells(const double4* tgt, const double4* src, const PairGeom& g, double L,
                             double gamma, int S, double* out, hipStream_t s);
// Single precision: records in units of L; outputs scaled back to physical
// units (potential / L, field / L^2).
hipError_t launch_pair_f32(int img, bool field, bool self, const Rec32* tgt, const Rec32* src,
                           const PairGeom& g, double L, double* out, hipStream_t s);
// Surface images (X, Y, Z, Q, px, py, pz, 0) at targets (x, y, z, q).
hipError_t launch_surface_f64(const double4* tgt, const double* surf, const PairGeom& g,
                              double* out, hipStream_t s);
// Grouped tiles of one kind (TILE_*) and, for near and right-hand-side
// tiles, one image mode (IMG_PERIODIC or IMG_METALLIC); groups ordered by
// first, ntiles tiles in all.
hipError_t launch_group_tiles(bool f32, int kind, int img, const TileGroup* groups, int ngroups,
                              int ntiles, hipStream_t s);
// Near sum at the particles, each unordered pair once (img: IMG_PERIODIC,
// IMG_METALLIC or IMG_SLAB, the last over the n real charges of the slab),
// single precision on Rec32 records.  acc: (g.C + g.s) copies of 4 x g.n_pad
// doubles (forward copies, then reverse copies), written completely for the
// first g.n entries of each component; the caller sums the copies.
hipError_t launch_sym_f32(int img, const Rec32* pts, const SymGeom& g, double L, double* acc,
                          hipStream_t s);
// The same in double precision on centred double4 (x, y, z, q) records.
hipError_t launch_sym_f64(int img, const double4* pts, const SymGeom& g, double L, double* acc,
                          hipStream_t s);
// Pair sums over an explicit list of charges (double4 or Rec32 records).
hipError_t launch_explicit(bool f32, bool field, bool self, const void* tgt, const void* src,
                           const PairGeom& g, double L, double* out, hipStream_t s);
// Sum the chunks of a pair-kernel output: res[comp * ld + t] = sum_c out[...].
hipError_t launch_chunk_reduce(const double* out, const PairGeom& g, int ncomp, double* res, int ld,
                               hipStream_t s);
// Records from centred double positions.
hipError_t launch_make_rec32(const double4* p, int n, double L, Rec32* out, hipStream_t s);

// Far field straight from the fitted series (plan.hip): out[comp * nt_pad + t],
// comp 0 = sum_k A_k B_k(r_t), 1..3 = -grad.
hipError_t launch_far_direct(const double4* tgt, int nt, int nt_pad, int P, double invR0,
                             const double* A, double* out, hipStream_t s);

// Plan kernels (plan.hip).
hipError_t launch_basis(const double* pts, int npts, int P, double invR0, double* out, int ld_pt,
                        int ld_k, int k0, hipStream_t s);

// Timing hooks (api.hip).
void timing_begin(int cls, hipStream_t s);
void timing_end(int cls, hipStream_t s);

}  // namespace hsma
