// Host-side factorisation of the R-MATEX matrices (internal header).
//
// The method factors its shifted matrix once and then only substitutes
// (Alg. 2: LU_Decompose before the time loop; Alg. 1: one forward/backward
// substitution pair per Krylov vector). For R-MATEX the factored matrix is
// C + gamma G (Sec. 3.3.2), and the F/P terms of Eq. 6 need G. Both are
// symmetric positive definite for an RC grid with supply pads, so each is
// factored as P A P^T = L L^T with one shared nested-dissection ordering and
// one shared supernodal structure.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace matex {

struct Csr {
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
};

// Panel columns are padded to whole 128-byte lines (16 doubles) so every
// column starts on a line and a 16-row read touches exactly one line.
constexpr int32_t PANEL_ALIGN = 16;
inline int32_t panel_ld(int32_t nr) { return (nr + PANEL_ALIGN - 1) / PANEL_ALIGN * PANEL_ALIGN; }

// One supernode = one node of the nested-dissection tree: a separator or a
// leaf domain. Its columns are contiguous in the new ordering.
struct Supernode {
    int32_t c0 = 0;       // first column (new ordering)
    int32_t nc = 0;       // number of columns
    int32_t nr = 0;       // rows of the panel: nc diagonal rows + off-diagonal rows
    int32_t parent = -1;  // ND-tree parent (assembly tree)
    int32_t level = 0;    // height above the leaves (0 = leaf)
    int64_t roff = 0;     // offset of the off-diagonal row list in Symbolic::rows
    int64_t w = 0;        // offset of the panel (leading dimension panel_ld(nr)), 128 B aligned
    int64_t u = 0;        // offset of this supernode's forward update slots
};

struct Symbolic {
    int64_t n = 0;
    std::vector<int32_t> perm;    // new -> old
    std::vector<int32_t> iperm;   // old -> new
    std::vector<Supernode> sn;    // postorder
    std::vector<int32_t> rows;    // concatenated off-diagonal rows (new ordering)
    // Forward-sweep assembly: supernode s owns update slots [u, u + nr - nc)
    // holding its subtree's accumulated contribution to its off-diagonal
    // rows. relidx[u + q] is the position of off-diagonal row q of s among
    // the panel rows of its parent ([parent columns ; parent off rows]).
    std::vector<int32_t> relidx;  // n_upd
    std::vector<int32_t> child_ptr, child_idx;   // children of each supernode
    int64_t n_upd = 0;            // sum of off-diagonal row counts
    int64_t n_w = 0;              // total panel storage (sum panel_ld(nr) * nc)
    int64_t nnz_l = 0;            // entries of L in the stored panels (lower part)
    int64_t nnz_exact = 0;        // structural nonzeros of L in this ordering (diagonal included)
    int32_t n_levels = 0;
    std::vector<std::vector<int32_t>> level_sn;   // supernodes per level
    int32_t max_nr = 0, max_nc = 0;
};

// Assemble G (Eq. 1): branch conductance Laplacian plus pad conductances.
Csr assemble_g(int64_t n, int64_t n_branch, const int32_t* a, const int32_t* b,
               const double* g, int32_t n_pad, const int32_t* pad, const double* pad_g);

// Nested-dissection ordering and supernodal symbolic analysis. coord is
// n x 3 (layer, i, j) or null (then a BFS distance is used as coordinate).
Symbolic analyse(const Csr& g, const int32_t* coord, int32_t leaf_max);

// Numeric factor of (alpha * G + diag(d)) on the symbolic structure. Writes
// the panels W_s = [L11^-1 ; L21 L11^-1] (column-major nr x nc, leading
// dimension panel_ld(nr), padding rows zero) into w.
// Returns 0, or 1 + (new-ordering column) of a non-positive pivot.
int64_t factor_panels(const Symbolic& s, const Csr& g, double alpha, const double* d,
                      std::vector<double>& w, int n_threads);

}  // namespace matex
