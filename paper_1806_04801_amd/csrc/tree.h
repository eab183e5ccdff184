// Tree-code near sum over the 3x3x3 image block (tree.hip): workspace layout
// and launch.
#pragma once

#include "hsma_internal.h"

namespace hsma {

constexpr int TREE_MAX_ORDER = 20;   // expansion order p
constexpr int TREE_MAX_LEVEL = 6;    // leaf level (2^L cells per box side)

struct TreeLayout {
    int L = 1;           // leaf level
    int p = 14;          // expansion order
    int64_t ns = 0;      // sources (N, or 2N for the slab)
    int64_t nimg = 0;    // 27 ns images
    int64_t ncell_leaf = 0;   // 27 * 8^L leaf cells over the image cube
    size_t off_img = 0, off_srt = 0, off_keys = 0, off_keys2 = 0, off_vals = 0, off_vals2 = 0,
           off_owner = 0, off_cnt = 0, off_offs = 0, off_tab = 0, off_cub = 0;
    size_t off_mom[TREE_MAX_LEVEL + 1] = {};
    size_t cub_bytes = 0;
    size_t total = 0;    // bytes, relative to the tree's own workspace base
};

// Leaf level for ns sources: about 32 to 45 sources per leaf cell.
int tree_leaf_level(int64_t ns);
TreeLayout tree_layout(int64_t ns, int p);

// phi and E at the first nt sources (the real particles) from all 27 images
// of the ns sources (img: IMG_PERIODIC, also for the slab's doubled cube, or
// IMG_METALLIC), bare self term left out: out[comp * npad + i], comp 0 = phi,
// 1..3 = E.  ws: t.total bytes.
hipError_t launch_tree_near(int img, const double4* src, int ns, int nt, double L,
                            const TreeLayout& t, char* ws, double* out, int npad, hipStream_t s);

}  // namespace hsma
