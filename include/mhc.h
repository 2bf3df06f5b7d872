/*
 * mhc.h -- multi-hadron correlator contraction on MI355X (gfx950).
 *
 * C ABI of libmhc.so.  For each time slice t the library evaluates
 *
 *     C(t) = sum_{i in src} sum_{j in snk} w_i w'_j prod_f det G_f^(ij)(t),
 *     G_f^(ij)(t)[m][n] = S_t[a_i^{f,m}][a_j^{f,n}],
 *
 * (Vachaspati & Detmold, "Fast Evaluation of Multi-Hadron Correlation
 * Functions", Sec. 1: the correlator as a weighted double sum of
 * determinants, with G block diagonal over quark flavours), either with one
 * pivoted LU per pair and flavour, or with the update tree of Secs. 2-3: a
 * greedy dominating set of the source terms gets LU factorisations, and
 * every other source term is one rank-1 row update away from its dominator
 * (matrix determinant lemma, one shared solve per changed row).
 *
 * Conventions for every function:
 *  - The return value is an mhc_status: MHC_OK (0) or a negative code.  On
 *    error mhc_last_error() returns a message for the calling thread.  No
 *    C++ exception crosses the ABI.
 *  - Host-detectable errors (NULL arguments, shapes, invalid terms) are
 *    reported before anything is enqueued on a stream.
 *  - *_create functions copy every host input; the caller may free its
 *    arrays afterwards.  Handles belong to the library until *_destroy.
 *    *_destroy(NULL) is a no-op.
 *  - Device buffers are caller-owned, contiguous and on the device that was
 *    current when the plan was created.  complex128 means interleaved
 *    (re, im) doubles, the layout of torch.complex128 and hipDoubleComplex.
 *  - A stream argument is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls that take a stream enqueue work and return without
 *    synchronising.
 *  - A handle must not be used from two threads at once; different handles
 *    are independent.
 */
#ifndef MHC_H
#define MHC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MHC_OK = 0,
  MHC_E_ARG = -1,         /* NULL pointer or out-of-range scalar argument    */
  MHC_E_TERM = -2,        /* invalid wavefunction term (index range/repeat)  */
  MHC_E_SHAPE = -3,       /* inconsistent shapes between handles/arguments   */
  MHC_E_DEVICE = -4,      /* HIP runtime error                               */
  MHC_E_OOM = -5,         /* host or device allocation failed                */
  MHC_E_STATE = -6,       /* handle in the wrong state for this call         */
  MHC_E_UNSUPPORTED = -7  /* valid input outside what the kernels implement  */
} mhc_status;

/* Greedy dominating-set rules (Sec. 3).
 * R2 (default): set-cover greedy on closed neighbourhoods -- every term
 *   stays eligible; each step takes the term whose closed neighbourhood holds
 *   the most still-uncovered terms (lowest index on ties).
 * R1: the literal rule -- take the remaining term of highest degree in the
 *   graph of remaining terms (lowest index on ties), then remove it and its
 *   remaining neighbours. */
enum { MHC_GREEDY_R1 = 1, MHC_GREEDY_R2 = 2 };
/* Flag or-ed into the policy of mhc_tree_build: every child gets its own
 * group, so siblings that change the same row do not share the solve
 * (Sec. 2 "updating" without the "caching" of Fig. 1; an ablation). */
enum { MHC_TREE_NO_SHARING = 0x100 };
/* Flag or-ed into the policy of mhc_tree_build: after the greedy rule, a
 * reverse-delete pass over the dominators (last picked first) drops each one
 * whose closed neighbourhood stays dominated by the others kept (Sec. 3
 * names a better dominating set as the first improvement).  The set stays
 * dominating, becomes irredundant and is never larger than the greedy one;
 * a term whose owner was dropped moves to the kept dominator of its closed
 * neighbourhood that was picked first. */
enum { MHC_TREE_PRUNE = 0x200 };
/* Flag or-ed into the policy of mhc_tree_build: edges between terms whose
 * flavour blocks, taken as sets of indices, differ in exactly one element
 * (Sec. 3 links matrices that differ by a single row without fixing the
 * order of the rows; an ablation).  A child's matrix is then a row
 * permutation of its dominator's with one row replaced: its determinant is
 * the permutation's sign times the updated one.  Positional neighbours are
 * set neighbours with sign +1.  Forward contraction only (one-sided tree and
 * plain methods, mhc_contract and the batch); the adjoint and the two-sided
 * method refuse such trees (MHC_E_UNSUPPORTED). */
enum { MHC_TREE_SET_EDGES = 0x400 };

/* Contraction methods. */
enum {
  MHC_PLAIN_LU = 0,    /* pivoted LU of every pair and flavour block (Sec. 2) */
  MHC_UPDATE_TREE = 1, /* dominator LU + rank-1 updates (Secs. 2-3)          */
  MHC_UPDATE_TREE2 = 2, /* source and sink trees: one LU per (source dominator,
                         * sink dominator), rank-1 row and column updates and
                         * the rank-2 form for pairs changed on both sides;
                         * needs mhc_plan_attach_sink_tree                    */
  /* Ablations (Sec. 4 compares LAPACK's pivoted LU with a custom LU without
   * pivoting): the same two methods with the diagonal as every pivot.  Not
   * backward stable; every block must have one size n <= 8. */
  MHC_PLAIN_LU_UNPIVOTED = 3,
  MHC_UPDATE_TREE_UNPIVOTED = 4,
  /* Variants with threshold partial pivoting: the diagonal entry stays the
   * pivot unless it is below 0.1 times the largest |Re|+|Im| among the
   * candidates (growth per step at most 11), so exchanges are rare.  Every
   * block must have one size n <= 8. */
  MHC_PLAIN_LU_THRESHOLD = 5,
  MHC_UPDATE_TREE_THRESHOLD = 6,
  /* The update tree with weighted-row aggregation (an extension of the
   * sharing of Sec. 2): the determinant is multilinear in row r, so the
   * children of a group, which replace the same row r, contribute
   * det G * ((sum_c w_c s_c) . x_r): one dot per group instead of one per
   * child.  No child's own ratio is formed, so A and the dense pair_det
   * form must be NULL; sampled pairs are evaluated as by the update
   * tree. */
  MHC_UPDATE_TREE_AGG = 7
};

typedef struct mhc_terms mhc_terms;
typedef struct mhc_tree mhc_tree;
typedef struct mhc_plan mhc_plan;

/* Message describing the last failure on this thread ("" if none). */
const char* mhc_last_error(void);

/* ABI version (major * 100 + minor). */
int32_t mhc_version(void);

/* Wavefunction terms (Sec. 1: each term is a product of quark creation
 * operators with a weight; the weight tensor is antisymmetric, so it
 * vanishes when an index repeats).
 *   n_terms      >= 1
 *   n_flavors    in [1, 8]; n_per_flavor[f] in [1, 32]
 *   idx          host int32 [n_terms][sum_f n_per_flavor[f]], flavour-major:
 *                the first n_per_flavor[0] entries of a term are its flavour-0
 *                quark indices, in order, then flavour 1, ...
 *   M            size of the quark index space, in [1, 255]; every index
 *                must lie in [0, M)
 * A term with an index outside [0, M), or with a repeated index within one
 * flavour, is rejected with MHC_E_TERM (its weight would be zero).
 * Weights are not part of the terms: they are passed to each contraction. */
mhc_status mhc_terms_create(int32_t n_terms, int32_t n_flavors,
                            const int32_t* n_per_flavor, const int32_t* idx,
                            int32_t M, mhc_terms** out);
void mhc_terms_destroy(mhc_terms* terms);
/* Shape of a term set (any pointer may be NULL): number of terms, number
 * of flavour blocks and the size M of the quark index space (Sec. 1: a term
 * is one product of quark operators per flavour, indices in [0, M)). */
mhc_status mhc_terms_shape(const mhc_terms* terms, int32_t* n_terms,
                           int32_t* n_flavors, int32_t* M);

/* Update tree over source terms (Sec. 3).  Two terms are neighbours when
 * their index tuples differ in exactly one position; that position is the
 * flavour block f and the row r that changes (Sec. 2: G^(jk) = G^(ik) +
 * e_r v^T).  The greedy rule `policy` (MHC_GREEDY_R1 or R2, optionally
 * | MHC_TREE_NO_SHARING and/or | MHC_TREE_PRUNE) picks dominators; every
 * other term becomes a child of the first dominator whose neighbourhood
 * covered it (with MHC_TREE_SET_EDGES the neighbourhood is taken on sets).
 * Host only; depends on neither S nor the weights, so one tree serves every
 * gauge configuration and time slice. */
mhc_status mhc_tree_build(const mhc_terms* src, int32_t policy,
                          mhc_tree** out);
/* Copy the tree out (Sec. 3: the greedy dominating set and the dominator
 * each other term hangs off; Sec. 2: the row in which it differs).  Host
 * arrays of n_terms int32 each, any may be NULL:
 *   n_dom            number of dominators
 *   dom_order[k]     k-th dominator chosen (k < n_dom), -1 after that
 *   owner[u]         dominator owning term u (owner[d] == d for dominators)
 *   flav[u], pos[u]  flavour block and row in which u differs from its
 *                    owner; -1 for dominators */
mhc_status mhc_tree_export(const mhc_tree* tree, int32_t* n_dom,
                           int32_t* dom_order, int32_t* owner, int32_t* flav,
                           int32_t* pos);
/* Per term (host arrays of n_terms int32 each, either may be NULL): the new
 * index in the row that differs from its dominator (Sec. 2: the row s of
 * the update) and the sign of the row permutation between the child's
 * blocks and the dominator's with that row replaced (1 for positional
 * edges); -1 and 0 for dominators.  Errors: MHC_E_ARG (NULL tree). */
mhc_status mhc_tree_children(const mhc_tree* tree, int32_t* new_index, int32_t* sign);
/* Counts of the tree (any pointer may be NULL): dominators (Sec. 3: the
 * matrices that get a full factorisation), (dominator, flavour, row)
 * groups (Sec. 2: children that change the same row of a dominator share
 * one solve) and children (every other term). */
mhc_status mhc_tree_stats(const mhc_tree* tree, int32_t* n_dom,
                          int32_t* n_groups, int32_t* n_children);
/* Copy out the group tables the kernels read (host arrays, caller-owned,
 * sized by mhc_tree_stats; any pointer may be NULL).  Sec. 2: children of a
 * dominator that change the same row r of flavour block f share the solve
 * x = G_f^-1 e_r; Sec. 3: dominators are processed in the order the greedy
 * rule picked them.
 *   dom_grp    [n_dom + 1]   groups of the k-th dominator (dom_order[k]) are
 *                            dom_grp[k] .. dom_grp[k+1]-1
 *   grp_f      [n_groups]    flavour block of each group
 *   grp_r      [n_groups]    changed row of each group
 *   grp_ptr    [n_groups+1]  children of group g are
 *                            grp_child[grp_ptr[g] .. grp_ptr[g+1]-1]
 *   grp_child  [n_children]  term indices
 * Within a dominator groups are sorted by (f, r) ascending; within a group
 * children are in ascending term order.  With MHC_TREE_NO_SHARING every
 * child is a group of its own (same order).
 * Errors: MHC_E_ARG (NULL tree). */
mhc_status mhc_tree_groups(const mhc_tree* tree, int32_t* dom_grp, int32_t* grp_f,
                           int32_t* grp_r, int32_t* grp_ptr, int32_t* grp_child);
void mhc_tree_destroy(mhc_tree* tree);

/* Device plan: the source tree and the sink terms uploaded once to the
 * current HIP device (Sec. 3: built once and reused across configurations).
 * Both term sets must have the same flavour structure and M.  Flavour blocks
 * may differ in size; the largest must be <= 24, and one slice of S as the
 * kernels keep it in LDS (rows padded to M + 1 entries, M * (M + 1) * 16
 * bytes) must fit in 150 KiB (M <= 97); otherwise MHC_E_UNSUPPORTED.
 * Enqueues the uploads on `stream` and waits for them. */
mhc_status mhc_plan_create(const mhc_tree* src_tree, const mhc_terms* snk,
                           void* stream, mhc_plan** out);
void mhc_plan_destroy(mhc_plan* plan);

/* Forward contraction (Sec. 1: C(t) as the weighted double sum of pair
 * determinants; Secs. 2-3: the update tree).  Device pointers,
 * caller-owned:
 *   S         complex128 [T][M][M], row = source quark index, column = sink
 *             quark index (Sec. 1)
 *   w_src     double [n_src];  w_snk  double [n_snk]
 *   C         complex128 [T] (output)
 *   A         double [T] or NULL: A(t) = sum_ij |w_i w'_j d_ij(t)| (output;
 *             the scale the result's accuracy is judged against)
 *   pair_det  NULL, or a test hook (at most 4 flavour blocks) in one of two
 *             forms:
 *             - pairs == NULL: complex128 [T][n_src][n_snk], every
 *               d_ij(t) = prod_f det G_f^(ij)(t), written by the
 *               contraction kernels themselves;
 *             - pairs != NULL: complex128 [n_pairs], d_ij(t) for each
 *               sampled (t, i, j) = pairs[q][0..2] (device int32
 *               [n_pairs][3]), evaluated by the method's arithmetic (plain:
 *               one LU per block; tree: the owner dominator's factorisation,
 *               the solve of the changed row and the ratio) with the device
 *               routines of the contraction kernels, after them on the same
 *               stream; an entry with t, i or j out of range gives NaN.
 *   n_pairs   0 when pairs is NULL, else in [0, 2^31).
 * T in [1, 65535].  Every method returns the same quantities within
 * floating-point rounding: MHC_PLAIN_LU, MHC_UPDATE_TREE (the paper's
 * method), MHC_UPDATE_TREE2 (needs an attached sink tree, computes neither
 * A nor pair_det: both must be NULL), the unpivoted ablations and the
 * threshold-pivoting variants (blocks of one size n <= 8) and
 * MHC_UPDATE_TREE_AGG (no A, no dense pair_det).  Every pointer
 * must stay valid until the stream has run the work.  The plan holds the
 * workgroup partial sums: two contractions on one plan that overlap in
 * time (on different streams) race; a call that needs a larger partial
 * buffer than any before waits for the device, then grows it.
 * Errors: MHC_E_ARG (NULL plan or buffer, T or n_pairs out of range, pairs
 * without pair_det), MHC_E_STATE (MHC_UPDATE_TREE2 without a sink tree),
 * MHC_E_UNSUPPORTED (method not available for these blocks or trees,
 * pair_det with more than 4 blocks, A or dense pair_det with
 * MHC_UPDATE_TREE_AGG), MHC_E_DEVICE, MHC_E_OOM. */
mhc_status mhc_contract(mhc_plan* plan, int32_t method, int32_t T,
                        const void* S, const double* w_src,
                        const double* w_snk, void* C, double* A,
                        void* pair_det, const int32_t* pairs, int64_t n_pairs,
                        void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward contraction of mhc_contract without the pair-determinant hook,
 * with the workgroup partial sums in a static device array of the library
 * (2 MiB per device, held until the process ends) instead of a buffer
 * grown on the plan.  It calls no hipMalloc or hipFree; its first call on a
 * device only looks up that array's address there.  Every valid T fits (the
 * partials take at most 3 * (4096 + T) doubles, 3.5 * (4096 + T) with
 * MHC_UPDATE_TREE2, whose workgroups also leave a flag each); a call that
 * would need more returns MHC_E_UNSUPPORTED.  All calls on one device share the array
 * and its contents: calls that overlap in time on one device (different
 * streams, threads or plans) race.  Arguments, methods and errors as for
 * mhc_contract. */
mhc_status mhc_contract_noalloc(mhc_plan* plan, int32_t method, int32_t T,
                                const void* S, const double* w_src,
                                const double* w_snk, void* C, double* A,
                                void* stream);

/* Adjoint of mhc_contract (every method computes the same C).  For an
 * incoming gradient gC of a real loss (PyTorch's convention for complex
 * tensors):
 *   gS[t][p][q] = gC[t] * conj(dC(t)/dS_t[p][q])      complex128 [T][M][M]
 *   g_wsrc[i]   = Re(sum_t gC[t] * conj(dC(t)/dw_i))   double [n_src]
 *   g_wsnk[j]   = Re(sum_t gC[t] * conj(dC(t)/dw'_j))  double [n_snk]
 * dC/dS follows from Jacobi's formula (d det G / dG[m][n] = det(G)
 * (G^-1)[n][m]) applied to every flavour block of every pair (Sec. 1
 * definitions); dC/dw from bilinearity.  method MHC_PLAIN_LU recomputes
 * every pair's LU and inverse; MHC_UPDATE_TREE factorises dominators only:
 * a child's cofactor matrix is the dominator's updated by Sherman-Morrison
 * (rank 1, Sec. 2), so the weighted sum over a dominator and its children
 * is one scaled inverse plus one rank-1 term per group of siblings.
 * Inputs as for mhc_contract; gC is complex128 [T].  Any output pointer may
 * be NULL (not written).  At most 4 flavour blocks of one size n <= 8; S_t
 * and its gradient must fit in LDS together (2 * M * (M + 1) * 16 bytes).
 * A pair's flavour block with an exactly zero pivot (for MHC_UPDATE_TREE:
 * every pair of a dominator whose block has one) is taken pair by pair; a
 * block that stays singular has no inverse, and its cofactors come from its
 * minors (the definition of the adjugate, by direct LU of each minor); such
 * blocks are counted (mhc_plan_status).  Device scratch is allocated on the plan at the first
 * call (and grown when T grows). */
mhc_status mhc_contract_backward(mhc_plan* plan, int32_t method, int32_t T, const void* S,
                                 const double* w_src, const double* w_snk,
                                 const void* gC, void* gS, double* g_wsrc,
                                 double* g_wsnk, void* stream);

/* Counters summed over all completed calls on this plan (either pointer may
 * be NULL); synchronises the device first.  They count the work the update
 * route of Sec. 2 cannot take (the matrix determinant lemma needs the
 * dominator's inverse), which goes by direct LU instead.
 *   n_fallback       work the update paths took by direct LU because a
 *                    dominator block had an exactly zero pivot (no
 *                    inverse): children (MHC_UPDATE_TREE), or (source
 *                    dominator, sink dominator) pairs (MHC_UPDATE_TREE2);
 *   n_singular_grad  (pair, flavour) blocks with an exactly zero pivot whose
 *                    cofactors the adjoint took from their minors. */
mhc_status mhc_plan_status(mhc_plan* plan, int64_t* n_fallback,
                           int64_t* n_singular_grad);

/* Attaches an update tree over the plan's sink terms (built by
 * mhc_tree_build on sink terms equal to the ones the plan was created with)
 * for method MHC_UPDATE_TREE2.  Sec. 3 links terms that differ in one row
 * or one column but uses rows only; the sink tree adds the columns.  The
 * tree's tables are copied to the device (synchronously on `stream`); a
 * tree attached before is replaced (after waiting for the device).  With
 * MHC_UPDATE_TREE2, mhc_contract needs A == NULL and pair_det == NULL.
 * Errors: MHC_E_ARG (NULL handle), MHC_E_SHAPE (other sink terms),
 * MHC_E_UNSUPPORTED (blocks not all of one size n <= 8), MHC_E_DEVICE,
 * MHC_E_OOM. */
mhc_status mhc_plan_attach_sink_tree(mhc_plan* plan, const mhc_tree* snk_tree, void* stream);

/* Batched jobs.  Many independent contractions (each a plan, its number of
 * slices and its own buffers) run as one captured graph: one persistent
 * kernel per kernel variant walks a table of (job, slice, chunk) tiles,
 * largest predicted cost first, then one kernel writes every job's C (and
 * A).  The paper notes that partitions of the work can be evaluated
 * independently (Sec. 5); here independent jobs share one launch.
 *
 * Schedule (every field 0 = chosen by the library):
 *   kernel          MHC_SCHED_AUTO: one matrix per lane where every flavour
 *                   block of a job has the same size n <= 8, else a group of
 *                   lanes per matrix (several rows per lane);
 *                   MHC_SCHED_LANE forces one matrix per lane (refused for
 *                   other jobs), MHC_SCHED_GROUP one row per lane of a group;
 *   blocks_per_cu   persistent workgroups per compute unit, in [0, 8];
 *   items_per_tile  work items per tile, >= 0 (one row per lane only; the
 *                   several-rows kernels take the plan's tiles).
 * The graph is captured at the first mhc_batch_run and replayed after that
 * (captured again, after waiting for the device, when a run asks for A and
 * the previous did not, or the reverse); the method, the slices per job and
 * the schedule are fixed at creation.
 * Buffers per job j (device, caller-owned): S[j] complex128 [T[j]][M][M],
 * w_src[j], w_snk[j], C[j] complex128 [T[j]], A[j] double [T[j]] (A may be
 * NULL, or any A[j]).  When the buffer pointers differ from the previous
 * run, mhc_batch_run first waits for the device, then updates the job
 * table.  Plans must outlive the batch.  Two runs of one batch that
 * overlap in time (on different streams) share its partial sums and race.
 * Errors: MHC_E_ARG (NULL handle or buffer, bad schedule, T outside
 * [1, 65535]), MHC_E_DEVICE (plan or current device differ),
 * MHC_E_UNSUPPORTED (LANE forced on a job it cannot run), MHC_E_OOM. */
enum { MHC_SCHED_AUTO = 0, MHC_SCHED_LANE = 1, MHC_SCHED_GROUP = 2 };
typedef struct {
  int32_t kernel;
  int32_t blocks_per_cu;
  int32_t items_per_tile;
} mhc_schedule;
typedef struct mhc_batch mhc_batch;

mhc_status mhc_batch_create(mhc_plan* const* plans, const int32_t* T, int32_t n_jobs,
                            int32_t method, const mhc_schedule* sched, mhc_batch** out);
mhc_status mhc_batch_run(mhc_batch* batch, const void* const* S,
                         const double* const* w_src, const double* const* w_snk,
                         void* const* C, double* const* A, void* stream);
/* Tiles, kernels in the graph (persistent kernels + 1), and det-pairs per
 * run (sum over jobs of T * n_src * n_snk); tiles and kernels are 0 before
 * the first run. */
mhc_status mhc_batch_info(const mhc_batch* batch, int32_t* n_tiles, int32_t* n_kernels,
                          int64_t* n_pairs);
void mhc_batch_destroy(mhc_batch* batch);

/* Device probe (not an operation of the paper): the FP64 vector FMA rate
 * that the roofline of the contraction kernels is set against, measured on
 * the current device.  Launches n_blocks workgroups of 256 threads on
 * `stream`; every thread runs `iters` rounds of 16 independent fused
 * multiply-adds a <- a * b + c (32 flop per round) in registers and writes
 * the sum of its 16 values to out[thread].  The caller times the launch:
 * flop per launch = n_blocks * 256 * iters * 32.
 *   out   device, double [n_blocks * 256], caller-owned;
 *   chain values: a_0 = 1 + i / 1024 (i = 0..15), b = 1 - 2^-20,
 *   c = 2^-30 * (1 + (threadIdx & 7)), so out[thread] equals
 *   sum_i (b^iters a_0 + c (1 - b^iters) / (1 - b)) up to rounding.
 * Errors: MHC_E_ARG (NULL out, n_blocks outside [1, 2^20], iters outside
 * [1, 2^24]), MHC_E_DEVICE (launch failure). */
mhc_status mhc_probe_fma64(double* out, int32_t n_blocks, int32_t iters, void* stream);

/* Device probe (not an operation of the paper): the FP64 matrix-core rate,
 * to compare with mhc_probe_fma64.  Every thread runs `iters` rounds of 4
 * independent v_mfma_f64_16x16x4_f64 accumulations (per wave and round
 * 4 x 2048 flop); with_valu != 0 adds the 16 vector FMA chains of
 * mhc_probe_fma64 to every round (32 flop per thread), to measure whether
 * matrix and vector FP64 work add up.  out[thread] receives the sum of the
 * thread's accumulator entries and chain values.  Launch, arguments and
 * errors as for mhc_probe_fma64; flop per launch = n_blocks * 4 waves *
 * iters * 8192 (+ n_blocks * 256 * iters * 32 with with_valu). */
mhc_status mhc_probe_mfma64(double* out, int32_t n_blocks, int32_t iters, int32_t with_valu,
                            void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MHC_H */
