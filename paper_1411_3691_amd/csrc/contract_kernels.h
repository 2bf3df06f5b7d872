// Device-side views of a plan and the launcher of the contraction kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mhc {
namespace kern {

// Work of the multi-row group kernels for one method (update tree or plain
// LU), all device memory.  A unit is a row set (a dominator, or a source
// term for the plain LU) with a range of its groups and children; a tile is
// a range of units and a range of sinks whose S rows one workgroup stages
// in LDS at once.
struct RowsTable {
  int32_t n_tiles, max_rows;      // tiles; most rows any tile stages
  const int4* tiles;              // [n_tiles] (u0, u1, s0, s1)
  const int4* unit;               // [n_units] (row set, g0, g1, counts the row set's own term)
  const int2* unit_c;             // [n_units] child range (update tree)
  const int32_t* unit_row;        // [n_units + 1] a unit's staged rows: rows[unit_row[u] ..]
  const int32_t* rows;            // S row index of every staged row: the row set's
                                  // rows (flavour-major), then its children's new rows
  const int32_t* child_lrow;      // [n_children] a child's new row within its unit
};

// Device tables of a plan (all pointers are device memory).
struct PlanView {
  int32_t n_src, n_snk, n_snk_pad, M, F, sn, n_dom;
  int32_t off[9];                 // flavour offsets into a term's tuple
  // update tree, dominators in greedy order
  const int32_t* dom_term;        // [n_dom] source term of each dominator
  const uint32_t* dom_rowoff;     // [n_dom][sn] byte offset a*M*16 of each row
  const int32_t* dom_grp;         // [n_dom+1] group range of each dominator
  const int32_t* grp_fr;          // [n_groups] (f << 8) | r
  const int32_t* grp_ptr;         // [n_groups+1] child range of each group
  const uint32_t* child_rowoff;   // [n_children] byte offset of the new row
  const int32_t* child_term;      // [n_children] source term of the child
  const double* child_wsgn;       // [n_children] sign of the child's row
                                  // permutation (+1 with positional edges)
  // plain method: every source term is its own row set
  const uint32_t* src_rowoff;     // [n_src][sn]
  // per source term: its dominator's term id (itself for a dominator), the
  // (flavour << 8) | row in which it differs from it, plus 1 << 16 where
  // its row permutation is odd (-1 for a dominator), and the byte offset of
  // its new row; read by the per-pair kernels only
  const int32_t* term_owner;      // [n_src]
  const int32_t* term_fr;         // [n_src]
  const uint32_t* term_crow;      // [n_src]
  // sinks, position-major for coalesced loads; padded sinks repeat sink 0
  const uint32_t* snk_coloff;     // [sn][n_snk_pad] byte offset b*16
  // multi-row group kernels (blocks up to 24); n_tiles 0 where not built
  RowsTable rows_tree, rows_plain;
};

// Sink-side update tree (two-sided contraction).  Sink dominators are
// stored in processing order (sorted so that the lanes of a wave have
// similar numbers of groups and children); lanes past n_sdom are padding
// with no groups.  Groups of a dominator are sorted by (flavour, column).
struct SinkTreeView {
  int n_sdom, n_sdom_pad;
  const int32_t* sdom_term;       // [n_sdom_pad] sink term id
  const uint32_t* sdom_coloff;    // [sn][n_sdom_pad] column byte offsets
  const int32_t* sdom_grp;        // [n_sdom_pad + 1] group range
  const int32_t* sgrp_fc;         // [n_sgroups] (flavour << 8) | column
  const int32_t* sgrp_ptr;        // [n_sgroups + 1] child range
  const uint32_t* schild_coloff;  // [n_schildren] new column byte offset
  const int32_t* schild_term;     // [n_schildren] sink term id
  // The children again, slot-major for one coalesced read per lane: row
  // srec_base[f] + i of [rows][n_sdom_pad] holds child i of flavour f of
  // every sink dominator as (new column offset, offset of the column it
  // replaces, sink term or -1 for padding, 0); srec_cnt[f][sink block] is
  // the most children of flavour f in the block (the rows it reads).
  const int4* srec_static;
  const int32_t* srec_cnt;
  int32_t srec_base[9];
  int32_t n_srec;                 // records (rows x n_sdom_pad)
};

// A sink child as the two-sided kernel reads it in one call: its new
// column, the column it replaces (byte offsets; 0xffffffff for padding)
// and its weight (0 for padding).
struct SinkRec {
  uint32_t col, ccol;
  double w;
};

struct ContractArgs {
  PlanView plan;
  SinkTreeView snk;               // used by the two-sided contraction only
  const double2* S;               // [T][M][M]
  const double* w_src;            // [n_src]
  const double* w_snk;            // [n_snk]
  double* partial;                // [T][n_blk_t][3] workgroup partials
  double2* pair_det;              // [T][n_src][n_snk] or null
  unsigned long long* fallback;   // fallback counter or null
  int T, n_items, n_blk_t, n_sblk;
  int tab_rows;                   // two-sided: rows of each wave's LDS table of
                                  // aggregated child rows (0: none)
  SinkRec* srec;                  // two-sided: the sink children's records of this call
  double2* C;                     // outputs, read by the batch reduction only
  double* A;
};

// A batch of jobs for one persistent kernel: tile i = (job, t, chunk, 0)
// in processing order.
struct BatchArgs {
  const ContractArgs* jobs;
  const int4* tiles;
  int n_tiles;
};

// LDS of a two-sided workgroup with its aggregated-row tables and its
// threads' running sums, at most (two workgroups per compute unit), and
// the bytes of those sums (256 threads x 4 complex numbers).
constexpr size_t kTwoSidedLdsLimit = 80 * 1024;
constexpr size_t kTwoSidedSlotBytes = 256 * 4 * 16;

// Flavour blocks supported by the pair-determinant test hook.
constexpr int kPairFlavors = 4;

// Sampled pair determinants: out[q] = d_ij(t) for (t, i, j) = pairs[q],
// evaluated by the method's own arithmetic (plain: one LU per block; tree:
// the owner dominator's factorisation, the shared solve of the changed row
// and the ratio) with the device routines of the contraction kernels.
// Entries with t, i or j out of range give NaN.
struct PairArgs {
  PlanView plan;
  const double2* S;               // [T][M][M]
  const int32_t* pairs;           // [n_pairs][3]
  double2* out;                   // [n_pairs]
  int T, n_pairs;
};
// n: largest flavour block; narrow: every block of size n <= 8 (one
// matrix per lane), else one group of lanes per matrix; pivot as for
// launch_contract (0 none, 1 partial, 2 threshold; narrow only).
hipError_t launch_pairs(const PairArgs& a, int n, bool narrow, bool tree, int pivot,
                        hipStream_t s);

// Enqueues the contraction of all T slices with one matrix per lane (every
// flavour block of size n <= 8) and the final reduction into C[T] (and A[T]
// if non-null).  diag selects the kernels that also produce A and pair
// determinants.  Work items are (row set, block of 64 sinks).
// pivot: 0 none (ablation), 1 partial pivoting, 2 threshold partial pivoting,
// 3 partial pivoting with weighted-row aggregation of each group's children
// (tree only, neither A nor pair determinants).
hipError_t launch_contract(const ContractArgs& a, int n, bool tree, bool diag, int pivot,
                           double2* C, double* A, hipStream_t s);

// The same with one group of lanes per matrix (one row per lane): blocks of
// any sizes up to nmax <= 24, different per flavour.  Work items are
// (row set, block of wide_sinks_per_wave(nmax) sinks).
hipError_t launch_contract_wide(const ContractArgs& a, int nmax, bool tree, bool diag,
                                double2* C, double* A, hipStream_t s, bool agg = false);
int wide_sinks_per_wave(int nmax);

// Multi-row group kernels (several rows of a matrix per lane, blocks up to
// 24, sizes may differ per flavour): buckets 8, 12, 16, 18 and 24 (0 where
// no bucket holds nmax).  Per workgroup: sinks per wave, waves and the bytes of
// the pivot-row buffers; the rows a tile stages get the rest of the LDS.
struct RowsGeometry {
  int spw, waves;
  size_t buf_bytes;
};
// Children whose (new row, weight) one tile stages in LDS, at most; the
// plan splits tiles and units to keep within it.
constexpr int kRowsChildCap = 256;
// LDS of a workgroup besides the pivot-row buffers and the staged rows:
// each wave's sink column offsets (spw sinks x sn positions) and the
// tile's children table.
__host__ __device__ constexpr size_t rows_meta_bytes(int waves, int spw, int sn) {
  return ((size_t)waves * spw * sn * 4 + 15) / 16 * 16 + (size_t)kRowsChildCap * 16;
}
int rows_bucket(int nmax);
RowsGeometry rows_geometry(int nmax, bool tree);
// Enqueues the contraction by the plan's rows table of the method
// (a.n_blk_t chunks per slice, each walking the tiles chunk, chunk +
// n_blk_t, ...) and the final reduction; lds_rows = rows_meta_bytes plus
// the table's max_rows times the padded row bytes.
hipError_t launch_contract_rows(const ContractArgs& a, int nmax, bool tree, bool with_a,
                                bool agg, size_t lds_rows, double2* C, double* A, hipStream_t s);
hipError_t launch_batch_rows(const BatchArgs& b, int nmax, bool tree, bool with_a, int grid,
                             size_t lds_rows, hipStream_t s);
int batch_rows_resident(int nmax, bool tree, bool with_a, size_t lds_rows);

// Two-sided update trees (one matrix per lane, every block of size n <= 8):
// work items are (source dominator, block of 64 sink dominators).
hipError_t launch_contract_two_sided(const ContractArgs& a, int n, double2* C, hipStream_t s);

// Final fixed-order reduction of the workgroup partials into C (and A).
hipError_t launch_reduce(const ContractArgs& a, double2* C, double* A, hipStream_t s);

// Persistent kernels over a tile table (grid workgroups, lds bytes of
// dynamic LDS = the largest slice of S among the jobs); with_a: the
// partials also carry the scale A.
hipError_t launch_batch_lane(const BatchArgs& b, int n, bool tree, bool with_a, int grid,
                             size_t lds, hipStream_t s);
hipError_t launch_batch_wide(const BatchArgs& b, int nmax, bool tree, bool with_a, int grid,
                             size_t lds, hipStream_t s);
int wide_bucket(int nmax);
// Workgroups of a bucket's persistent batch kernel that stay resident on
// one compute unit together, for the LDS bytes one slice of S takes.
int batch_wide_resident(int nmax, bool tree, bool with_a, size_t lds);
// Threads per workgroup of a group kernel (512 or 1024) for a bucket and
// the LDS bytes one slice of S takes.
int wide_block(int nmax, bool tree, size_t lds);
// C_j[t] for each entry (job, t) of jt (n entries).
hipError_t launch_batch_reduce(const ContractArgs* jobs, const int2* jt, int n, hipStream_t s);

}  // namespace kern
}  // namespace mhc

namespace mhc {
namespace kern {

// A child of the update tree as the adjoint reads it: byte offset of its
// new row in the LDS copy of S_t, its source term and that term's weight.
struct ChildRec {
  uint32_t crow;
  int32_t term;
  double w;
};

struct AdjointArgs {
  PlanView plan;
  const double2* S;               // [T][M][M]
  const double* w_src;            // [n_src]
  const double* w_snk;            // [n_snk]
  const double2* gC;              // [T] incoming gradient
  double2* part_gS;               // [T][n_sblk][M*M] workgroup partials
  double* part_wsrc;              // [T][n_src][n_sblk]
  double* part_wsnk;              // [T][n_snk_pad]
  unsigned long long* singular;   // blocks with an exactly zero pivot (skipped)
  uint8_t* dom_flag;              // [T][n_sblk][n_dom] update tree: dominators whose
                                  // lanes need the pair-by-pair route
  ChildRec* child_rec;            // [n_children + 1] update tree: the children's
                                  // records for this call (one spare, read ahead)
  int T, n_sblk, n_children;
};

// Enqueues the adjoint (pair by pair, or by the source update tree) and the
// fixed-order reductions into gS [T][M][M], g_wsrc [n_src], g_wsnk [n_snk]
// (any output may be null).
hipError_t launch_adjoint(const AdjointArgs& a, int n, bool tree, double2* gS, double* g_wsrc,
                          double* g_wsnk, hipStream_t s);

}  // namespace kern
}  // namespace mhc
