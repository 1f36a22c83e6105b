// Host-side symbolic analysis of H_gamma = tril(H) U diag U tril(J^T J).
//
// Sec. 2 (reuse list): ordering and symbolic factorization are done once per
// pattern; Sec. 5.3: the fill-reducing order is approximate minimum degree.
// Everything here is integer work on the host; the result is uploaded once.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hkkt {

using i64 = int64_t;
using i32 = int32_t;

struct AnalyzeOptions {
    int ordering = 0;   // 0 own AMD, 1 natural, 2 nested dissection
    int relax = 1;      // supernode amalgamation level
    int lds_rows = 64;  // fronts with at most this many rows use the LDS kernel
};

// One "big front" work item list per (level, step) of the blocked front
// factorization, built on the host so that kernels only index tables.
struct Symbolic {
    i64 n = 0, m = 0;
    std::vector<i32> perm, iperm;          // perm[k] = original index of pivot k

    // supernodes, numbered in postorder (children before parents)
    i32 ns = 0;
    std::vector<i32> sn_first;             // [ns+1] first column
    std::vector<i64> sn_rowptr;            // [ns+1] into sn_rows
    std::vector<i32> sn_rows;              // sorted row indices; first w are the columns
    std::vector<i64> sn_lptr;              // [ns+1] L storage offsets (nr*w col-major panel)
    std::vector<i64> sn_cbptr;             // [ns+1] contribution block offsets ((nr-w)^2)
    std::vector<i64> sn_uvptr;             // [ns+1] update-vector offsets (nr-w)
    std::vector<i32> sn_parent;            // -1 for roots
    std::vector<i32> child_ptr, child_list;
    std::vector<i32> relmap;               // at sn_uvptr[s]+k: index of rows_below(s)[k] in rows(parent)
    std::vector<i32> ga_row;               // [2*rows] per row slot of a supernode: (start, count) into ga_idx
    std::vector<i32> ga_idx;               //   of its children's update-vector entries (UV offsets, children in order)
    std::vector<i32> col2sn;

    // levels (leaves = 0)
    std::vector<i32> level_ptr, level_sn;  // supernodes grouped by level
    i32 nlevels = 0;

    // structural statistics
    i64 nnzA = 0, nnzL = 0, Lsize = 0, CBsize = 0, UVsize = 0;
    double flops_proxy = 0;                // sum over columns of c_j^2
    i32 max_w = 0, max_nr = 0;
    i64 etree_height = 0;

    // assembly map over the entries of tril(P H_gamma P^T)
    std::vector<i64> a_dst;                // L storage offset
    std::vector<i32> a_h;                  // index into H_val or -1
    std::vector<i32> a_d;                  // original variable for D_x + delta, or -1
    std::vector<i64> a_pptr;               // [nnzA+1] into a_pa/a_pb
    std::vector<i32> a_pa, a_pb;           // J value index pairs: gamma*J[pa]*J[pb]

    // operators in the permuted order
    std::vector<i64> J_rowptr;             // rows of J unchanged
    std::vector<i32> J_colp;               // iperm[col]
    std::vector<i64> JT_rowptr;            // [n+1] J^T rows = permuted columns
    std::vector<i32> JT_col;               // J row index
    std::vector<i32> JT_src;               // index into J_val
    std::vector<i64> HF_rowptr;            // full symmetric H, permuted rows
    std::vector<i32> HF_col;
    std::vector<i32> HF_src;               // index into H_val
    i64 nnzH = 0, nnzJ = 0;

    // members of an uneven group (block-diagonal super-system); G = 1 for a
    // single pattern. Member k owns variables [x_off[k], x_off[k+1]) and J
    // rows [y_off[k], y_off[k+1]); the elimination order keeps every member's
    // variables in its own contiguous range, so the same ranges hold in the
    // permuted order.
    i32 G = 1;
    std::vector<i64> x_off, y_off;
    std::vector<i32> xp_mem;               // [n] member of permuted variable
    std::vector<i32> y_mem;                // [m] member of J row
    std::vector<i32> a_mem;                // [nnzA] member of assembly entry
    std::vector<i32> sn_mem;               // [ns] member of supernode
    // member-aligned reduction blocks (start, end, member) over the J rows
    // and over the combined [x ; y] index space of the KKT residual
    std::vector<i32> mblk, mblk_off;       // mblk_off[k]: first block of member k
    std::vector<i32> rblk, rblk_off;
};

constexpr int kRedBlock = 256;             // rows per reduction block

// Validates the CSR inputs; returns "" if fine, else a message.
std::string validate_pattern(i64 n, i64 m, const i64* Hp, const i32* Hi, const i64* Jp, const i32* Ji);

// Own approximate minimum degree on the symmetric graph (ptr/adj without
// the diagonal). Returns perm[k] = node eliminated k-th.
std::vector<i32> amd_order(i64 n, const std::vector<i64>& ptr, const std::vector<i32>& adj);
std::vector<i32> nd_order(i64 n, const std::vector<i64>& ptr, const std::vector<i32>& adj, int leaf);

// Full analysis. perm_in may be null. For an uneven group, G > 1 members
// with variable offsets x_off[G+1] and J-row offsets y_off[G+1] (entries of
// H and J must stay inside their member's block). Returns "" or an error.
std::string analyze(Symbolic& S, i64 n, i64 m, const i64* Hp, const i32* Hi, const i64* Jp,
                    const i32* Ji, const i32* perm_in, const AnalyzeOptions& opt, int G = 1,
                    const i64* x_off = nullptr, const i64* y_off = nullptr);

}  // namespace hkkt
