// Symbolic analysis of one period block A (all N periods share it) extended
// by the 2*Ns border rows [C_1; C_0] of the MPOPF coupling (Eq. B12N).
//
// The factorisation is multifrontal over the augmented matrix
//     M = [ A  Bh^T ]     Bh = [C_1; C_0]   (2Ns x nA)
//         [ Bh  0   ]
// eliminating only A's pivots: the update matrix left on the border rows is
// -Bh A^-1 Bh^T = S_bar_n of Eq. LocalSchurBs3, i.e. the incomplete
// augmented factorisation of section 4.2 (Eq. augmented) applied to the 2Ns
// distinct right-hand sides of section 4.3. Border rows are never pivots and
// are ordered after every A column.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace kkt {

struct SymbolicInput {
    int64_t nA = 0, n_primal = 0, Ns = 0;
    // primal neighbours a dual waits for before it may be eliminated
    // (capped at its count; see amd_order)
    int dual_wait = 4;
    // duals also need an eliminated primal partner of their own (amd_order)
    bool pair_duals = true;
    const int64_t *colptr = nullptr;
    const int32_t *rowind = nullptr;
    const int64_t *C0p = nullptr, *C1p = nullptr;
    const int32_t *C0i = nullptr, *C1i = nullptr;
};

struct Symbolic {
    int64_t nA = 0, n_primal = 0, Ns = 0, nbord = 0, n = 0;  // n = nA + nbord
    int64_t nnzA = 0, nnzC0 = 0, nnzC1 = 0;
    std::vector<int32_t> perm, iperm;   // A part: perm[new] = old

    // supernodes; the last one is the border node (no pivots) when nbord > 0
    int32_t nsup = 0;
    int32_t border_sn = -1;
    std::vector<int32_t> first, ncol, nrow;     // columns [first, first+ncol)
    std::vector<int64_t> rowptr;                // rows of s: rows[rowptr[s] .. +nrow[s]]
    std::vector<int32_t> rows;                  // new-order indices (border row r -> nA + r)
    std::vector<int32_t> parent;                // -1 for a root
    std::vector<int32_t> child_ptr, child_list; // children, increasing order
    std::vector<int64_t> Loff, Uoff;            // panel (nrow x ncol) / update (u x u) offsets
    int64_t Lsize = 0, Usize = 0;
    std::vector<int64_t> relptr;                // rel[relptr[s] .. + (nrow-ncol)]
    std::vector<int32_t> rel;                   // update rows of s -> local rows of parent
    std::vector<int32_t> level;                 // height above the leaves
    int32_t nlevels = 0;
    std::vector<int32_t> level_ptr, level_list; // supernodes grouped by level

    // scatter maps into the per-period panel storage
    std::vector<int64_t> amap;                  // [nnzA]
    std::vector<int8_t> adiag;                  // [nnzA] 0 off-diag, +1 primal diag, -1 dual diag
    std::vector<int64_t> c0map, c1map;          // [nnzC0], [nnzC1]
    std::vector<int32_t> col2sn;                // [nA] new column -> supernode
    std::vector<int8_t> pivsign;                // [nA] new order: +1 primal, -1 dual

    int64_t nnzL = 0, max_front = 0, max_pivots = 0;
    double flops = 0.0;

    int64_t Usize_vec() const { return (int64_t)rel.size(); }  // sum of update rows
};

// Approximate-minimum-degree order of the symmetric graph (xadj/adj without
// self loops). Returns perm[new] = old. With n_primal >= 0, a variable
// i >= n_primal (a dual) becomes eligible only once min(dual_wait, its number
// of primal neighbours) of its primal neighbours (i' < n_primal) of the
// original graph are eliminated; with pair_duals it must also claim eliminated
// primal neighbours of its own, one per dual (see the definition).
std::vector<int32_t> amd_order(int32_t n, const std::vector<int64_t> &xadj,
                               const std::vector<int32_t> &adj, int64_t n_primal = -1, int dual_wait = 4,
                               bool pair_duals = false);

// Full analysis. Returns an empty string on success, else an error message
// (structural problem in the input).
std::string analyze(const SymbolicInput &in, Symbolic &out);

}  // namespace kkt
