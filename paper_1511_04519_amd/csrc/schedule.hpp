// Sweep schedules of the supernodal factor, built on the host (internal).
//
// The substitution pair of Alg. 1 (w = X1^-1 (X2 v_j), X1 = C + gamma G) runs
// as level-scheduled sweeps over the nested-dissection tree. This header
// holds the plain-C++ part: the record layouts the device kernels read and
// the builders of the subtree schedule (the bottom levels swept one subtree
// per workgroup), so the schedule can also be built and checked without a
// GPU.
#pragma once

#include <cstdint>
#include <vector>

#include "factor.hpp"

namespace matex {

// One task of a level sweep: a block (panels with more than 64 rows) or a
// wavefront (the whole supernode, panels with at most 64 rows).
struct PTask {
    int64_t w;       // panel offset of the supernode
    int64_t aux;     // forward: the supernode's update slots; backward: its off-row list
    int32_t c0, nc, nr;
    int32_t first;   // forward: first panel row of the task; backward: first column
    int32_t pos;     // forward: contributor list index of the supernode's panel position 0
    int32_t pad_;
};

// Subtree sweeps of the bottom levels: one block of TW wavefronts per
// subtree (or per few small subtrees), one wavefront per work item.
constexpr int TW = 8;
constexpr int TREE_MAX_NR = 256;   // largest panel (rows) a subtree item takes

struct TItem {
    int64_t w;        // panel offset of the supernode
    int64_t aux;      // forward: global update slots (used by subtree roots);
                      // backward: offset of the off-row list (trow)
    int32_t c0, nc, nr;
    int32_t first, last;   // forward: panel rows [first, last); backward: columns
    int32_t pos;      // forward: contributor list index of panel position 0
    int32_t lds_u;    // forward: LDS offset of the update slots, -1 for a subtree root
    int32_t lds_x;    // LDS offset of the supernode's x
};
static_assert(sizeof(TItem) == 48, "TItem is copied to LDS as 12 words");

// Two 32-bit values (the device reads them as int2).
struct I2 {
    int32_t x, y;
};

// Forward assembly, pull form: panel position p of supernode s has the
// global index pos_base[s] + p, and the children's update slots adding into
// it are cidx[cptr[pos_base[s] + p] .. cptr[pos_base[s] + p + 1]) in child
// order (the inverse of relidx).
struct Contrib {
    std::vector<int32_t> pos_base, cptr, cidx;
};
Contrib contributions(const Symbolic& s);

// Subtree schedule: block b runs forward steps fblk[b] .. fblk[b + 1] - 1
// (children's levels first) and backward steps bblk[b] .. bblk[b + 1] - 1
// (root first), each step TW items (nr = 0: idle). fdesc, per forward item
// and lane: the LDS slots (offset + 1 in each 16-bit half, 0 none) adding
// into btilde at column `lane` (.x) and into panel row first + lane (.y).
// trow, per off row: >= 0 global x index, < 0: -1 - LDS offset of an
// ancestor's x inside the block; one spare entry keeps clamped reads inside.
// LDS of a block: item_doubles (its items), TW wave scratch regions of ws
// doubles, then the shared region (update slots of non-root supernodes and
// every supernode's x) of at most lds_doubles - item_doubles - TW * ws.
struct TreeHost {
    std::vector<TItem> fitems, bitems;
    std::vector<int32_t> fblk{0}, bblk{0};
    std::vector<I2> fdesc;
    std::vector<int32_t> trow;
    std::vector<int64_t> shared;   // shared-region doubles each block uses
    int32_t n_blocks = 0;
    int32_t n_levels = 0;          // levels covered (0 .. n_levels - 1); 0: no subtree sweeps
    int32_t ws = 0;
    int32_t item_doubles = 0;
    int32_t lds_doubles = 0;
};

// The fewest subtree blocks worth a launch (one per compute unit), the most
// supernodes and shared LDS doubles packed into one block.
constexpr int64_t TREE_MIN_BLOCKS = 256;
constexpr int32_t TREE_MAX_NODES = 4 * TW;
constexpr int64_t TREE_MAX_SHARED = 4096;

// Subtree schedule of the bottom `limit` levels at most (limit < 0: none, 0:
// automatic): the most levels whose supernodes all fit a wavefront item
// (nc <= 64, nr <= TREE_MAX_NR, at most two children's slots adding into a
// panel position) that still leave TREE_MIN_BLOCKS subtrees, or every such
// level on a grid with fewer subtrees than that.
TreeHost build_tree_host(const Symbolic& s, const Contrib& c, int32_t limit);

}  // namespace matex
