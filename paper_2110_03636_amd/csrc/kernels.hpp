// Device kernels of the hybrid direct-iterative KKT solver (gfx950).
//
// Layout conventions (all batch-major, instance b at b * per-instance size):
//  - L storage: supernode s is a dense column-major panel of nr x w entries
//    (rows = the supernode's sorted row list, first w rows are its columns).
//  - contribution blocks (multifrontal update matrices): (nr-w) x (nr-w)
//    column-major, lower triangle used.
//  - update vectors of the forward solve: (nr-w) entries per supernode.
//  - packed solve copy (supernodes of the wavefront solve classes): the
//    entries strictly below the diagonal, column by column (column j holds
//    rows j+1 .. nr-1 contiguously), after one padding entry.
//  - vectors live in the permuted order of the symbolic analysis.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hkkt {

using i64 = int64_t;
using i32 = int32_t;

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kTri = 64;   // diagonal block size of the work-group triangular solves
constexpr int kChunk = 8;  // panel columns prefetched per step by the wavefront solves
constexpr int kTriClasses = 8;   // size classes of the triangular-solve schedule

// Device view of the symbolic analysis.
struct SymView {
    i64 n, m;
    i32 ns;
    const i32* sn_first;
    const i64* sn_rowptr;
    const i32* sn_rows;
    const i64* sn_lptr;
    const i64* sn_cbptr;
    const i64* sn_uvptr;
    const i32* child_ptr;
    const i32* child_list;
    const i32* relmap;
    const i32* ga_row;   // (start, count) pairs per supernode row slot
    const i32* ga_idx;
    const i32* perm;
    i64 Lsize, CBsize, UVsize;
    i64 LPsize;   // entries per instance of the packed solve copy
    // assembly
    i64 nnzA;
    const i64* a_dst;
    const i32* a_h;
    const i32* a_d;
    const i64* a_pptr;
    const i32* a_pa;
    const i32* a_pb;
    // operators
    i64 nnzH, nnzJ, nnzHF;
    const i64* J_rowptr;
    const i32* J_colp;
    const i64* JT_rowptr;
    const i32* JT_col;
    const i32* JT_src;
    const i64* HF_rowptr;
    const i32* HF_col;
    const i32* HF_src;
    // group members (G = 1 for a single pattern): a "CG instance" is
    // c = b * G + k for batch entry b and member k
    i32 G;
    const i32* xp_mem;     // [n] member of permuted variable
    const i32* a_mem;      // [nnzA]
    const i32* sn_mem;     // [ns]
    i32 nbm;               // member-aligned blocks over the J rows
    const i32* mblk;       // (start, end, member) per block
    const i32* mblk_off;   // [G+1]
    i32 nbr;               // member-aligned blocks over [x ; y]
    const i32* rblk;
    const i32* rblk_off;
};

// Packed per-supernode description used by the wavefront triangular solves
// (one broadcast load instead of a chain of metadata loads).
struct TriDesc {
    i64 lptr;    // panel offset in L storage
    i64 uvptr;   // update-vector offset
    i64 rp;      // first row slot (into sn_rows / ga_row)
    i32 f;       // first column
    i32 w;       // width
    i32 nr;      // rows
    i32 nchild;  // number of children (0: leaf, no gather)
    i32 mem;     // group member
    i32 pq;      // descriptor index of the parent supernode, -1 for a root
    i64 pptr;    // offset in the packed solve copy (wavefront classes), -1 if none
};


// Supernode of the tree-traversal solve with the right-hand side of the
// tree's columns held in LDS: slot = LDS index of the first column, rs =
// offset of its below-diagonal rows' LDS indices in the row-slot table.
struct TreeDesc {
    i64 lptr;    // panel offset in L storage
    i64 toff;    // offset of its row-major copy in the staged solves' layout
    i32 f;       // first column (for the reciprocal diagonal)
    i32 w;       // width
    i32 nr;      // rows
    i32 mem;     // group member
    i32 slot;    // LDS index of column f
    i32 rs;      // row-slot table offset of row w
};

// Per-batch numeric values (device, FP64 copies owned by the library).
struct ValView {
    int nb;
    const double* H;      // [nb][nnzH]
    const double* J;      // [nb][nnzJ]
    const double* JT;     // [nb][nnzJ] values of J^T in JT order
    const double* HF;     // [nb][nnzHF] full symmetric H, permuted
    const double* Dxp;    // [nb][n] D_x permuted
    const double* Dx;     // [nb][n] D_x original order
    const double* delta;  // [nb * G]
    const double* gamma;  // [nb * G]
};

// Per-instance CG scalars.
struct CGState {
    double rho, pq, pp, bnorm, alpha, beta, curv0, d2;
    int it, done, breakdown, pad;
};

// Dataflow triangular solves (k_tri_flow): per (instance, descriptor) words.
struct FlowArgs {
    const i32* seg;   // (offset, count) of the descriptors per (level, class), kTriClasses per level
    int nlevels;
    int ndesc;
    const int* ids;   // instance slots, nids of them (null: slot k = instance k)
    int nids;
    const CGState* st;
    int* fcnt;        // [nb][ndesc] children whose forward task is done; reset by the task itself
    int* fflag;       // [nb][ndesc] = app when a root's forward task is done
    int* bflag;       // [nb][ndesc] = app when the backward task is done
    int* abort;       // set when a wait timed out: every later wait returns at once
    int app;          // token of this application (> 0, increasing per batch)
};

}  // namespace hkkt
