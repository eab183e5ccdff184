// Tree-code near sum over the 3x3x3 image block (tree.hip): workspace layout
// and launch.
#pragma once

#include "hsma_internal.h"

namespace hsma {

constexpr int TREE_MAX_ORDER = 20;   // expansion order p
constexpr int TREE_MAX_LEVEL = 6;    // leaf level (2^L cells per box side)

struct TreeLayout {
    int L = 1;           // leaf level
    int p = 16;          // expansion order
    int64_t ns = 0;      // sources (N, or 2N for the slab)
    int64_t nimg = 0;    // 27 ns images
    int64_t ncell_leaf = 0;   // 27 * 8^L leaf cells over the image cube
    int eval_split = 1;  // work-groups per leaf cell of the evaluation (output chunks)
    size_t off_img = 0, off_srt = 0, off_keys = 0, off_keys2 = 0, off_vals = 0, off_vals2 = 0,
           off_owner = 0, off_offs = 0, off_tab = 0, off_itab = 0, off_part = 0, off_cub = 0;
    size_t off_mom[TREE_MAX_LEVEL + 1] = {};   // multipoles, all 27 boxes
    size_t off_loc[TREE_MAX_LEVEL + 1] = {};   // local expansions, central box
    size_t cub_bytes = 0;
    size_t total = 0;    // bytes, relative to the tree's own workspace base
};

// Leaf level for ns sources: the smallest with at most tree_leaf_images()
// images per leaf cell (320, or HSMA_TREE_LEAF in the environment).
int tree_leaf_level(int64_t ns);
double tree_leaf_images();
TreeLayout tree_layout(int64_t ns, int p);

// Images of the ns sources (img: IMG_PERIODIC, also for the slab's doubled
// cube, IMG_METALLIC, or IMG_DIELECTRIC with reflection weight gamma), sorted
// into the octree, and their multipoles at every level (ws: t.total bytes).
// Run before the two calls below.
hipError_t launch_tree_build(int img, double gamma, const double4* src, int ns, double L, const TreeLayout& t,
                             char* ws, hipStream_t s);

// Potential of all images at npts points (centred coordinates, inside the
// image cube): out[i], i < npts.  order: a permutation of 0..npts-1 in which
// the points are visited (neighbouring points together share cached cells).
hipError_t launch_tree_points(const double4* pts, const int* order, int npts, double L, const TreeLayout& t,
                              char* ws, double* out, hipStream_t s);

// phi and E at the first nt sources (the real particles) from all 27 images
// of the ns sources, bare self term left out, in t.eval_split chunks whose sum
// is the result: out[(chunk * 4 + comp) * npad + i], comp 0 = phi, 1..3 = E.
hipError_t launch_tree_near(int nt, double L, const TreeLayout& t, char* ws, double* out, int npad,
                            hipStream_t s);

}  // namespace hsma
