// HIP kernels for gfx950: gather + pivoted complex LU + update tree +
// weighted reduction of the multi-hadron correlator.
//
// Work decomposition.  A work item is (time slice t, source row-set d, sink
// block of 64).  One wavefront takes one item: lane l handles sink
// k = 64*block + l, and every lane of the wave shares the same source row
// set, so the tree structure (groups, children) is wave-uniform and the
// only per-lane data are the sink's column indices.  A workgroup stages the
// slice's propagator S_t into LDS once and its four waves then walk a
// strided subset of that slice's items; every determinant gathers its
// entries from LDS.
//
//  * plain method (Sec. 2, LU route): the row set is one source term;
//    per flavour block: LU with partial pivoting, gathering G_f from LDS as
//    the factorisation proceeds (Crout order, column exchanges), det;
//    d = prod_f det_f.
//  * update tree (Secs. 2-3): the row set is a dominator.  Per flavour
//    block: the same LU keeping L, U and the column order; for every
//    group (f, r) of the dominator one solve x = G_f^-1 e_r (forward and
//    back substitution; with column pivoting e_r is not permuted, so the
//    forward part starts at row r); every child of the group then costs
//    one dot product: det(G with row r := s) = det(G) * (s . x) (matrix
//    determinant lemma, Sec. 2; s . x equals 1 + v^T G^-1 e_r with
//    v = s - old row).  Children with the same (f, r) share x (the
//    "caching" of Sec. 2).
//
// The weighted sum over one item folds the flavours incrementally: with
// P = prod of the dets seen so far and Q = sum over seen flavours f of
// acc_f * prod_{f' != f, seen} det_f',  where acc_f = sum_{children c
// changing flavour f} w_c det(child's block f), the item contributes
// w_k * (w_i * P + Q).  A dominator block with an exactly zero pivot has no
// inverse; its children's blocks are then taken by direct LU (counted in the
// plan's fallback counter).
//
// Reductions are deterministic: per-lane sums, a fixed-order wave and
// workgroup reduction, one partial per workgroup, then a fixed-order final
// kernel.  There are no floating-point atomics.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contract_kernels.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

// Determinant of flavour block f of the pair (row set, sink) with row r
// replaced by the source row `newrow` (byte offset), by direct LU.
template <int N>
__device__ __forceinline__ void child_det_direct(const char* lds,
                                                 const uint32_t* rowoff_dom,
                                                 int r, uint32_t newrow,
                                                 const uint32_t (&coloff)[N],
                                                 double& dre, double& dim) {
  uint32_t ro[N];
#pragma unroll
  for (int m = 0; m < N; ++m) ro[m] = (m == r) ? newrow : rowoff_dom[m];
  double gr[N][N], gi[N][N];
  int perm[N];
  bool z;
  gather<N>(lds, ro, coloff, gr, gi);
  lu<N, false>(gr, gi, dre, dim, perm, z);
}

// MODE bit 0: accumulate A(t) = sum |w w d|; bit 1: write every pair det;
// bit 2: no pivoting (ablation); bit 3: threshold partial pivoting; bit 4:
// weighted-row aggregation (the children of a group enter through one dot
// product of their weighted rows, so no child's own ratio is formed).
// One tile: slice t, the chunk-th strided share of the slice's work items.
// The workgroup stages S_t in LDS (smem), walks its items and writes one
// partial (re, im, A) for (t, chunk).
template <int N, bool TREE, int MODE>
__device__ __forceinline__ void lane_tile(const ContractArgs& a, int t, int chunk,
                                          double2* smem) {
  constexpr bool WITH_A = (MODE & 1) != 0;
  constexpr int PIV = (MODE & 4) ? kNoPivot : (MODE & 8) ? kThresholdPivot : kPartialPivot;
  constexpr bool WITH_PAIRS = (MODE & 2) != 0;
  constexpr bool AGG = (MODE & 16) != 0;
  static_assert(!AGG || (MODE & 3) == 0, "aggregation forms no per-pair values");
  const PlanView& p = a.plan;
  __syncthreads();  // the previous tile of this workgroup is done with LDS
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  const int MM = p.M * p.M;

  // Stage S_t into LDS (16 B per lane per step, coalesced).
  const double2* St = a.S + (size_t)t * MM;
  stage_slice(St, smem, p.M, kBlock);
  __syncthreads();
  const char* lds = reinterpret_cast<const char*>(smem);

  double acc_re = 0.0, acc_im = 0.0, acc_a = 0.0;
  uint32_t n_fallback = 0;
  const int F = p.F;
  const int sn = p.sn;

  for (int item = chunk + a.n_blk_t * wave; item < a.n_items;
       item += a.n_blk_t * kWavesPerBlock) {
    const int d = uniform(item / a.n_sblk);
    const int sb = uniform(item - d * a.n_sblk);
    const int k = sb * kWave + lane;
    const bool valid = k < p.n_snk;
    const int term = TREE ? uniform(p.dom_term[d]) : d;
    const uint32_t* rowoff_d = (TREE ? p.dom_rowoff : p.src_rowoff) + (size_t)d * sn;
    const double wi = a.w_src[term];
    const double wk = valid ? a.w_snk[k] : 0.0;
    const int g_begin = TREE ? uniform(p.dom_grp[d]) : 0;
    const int g_end = TREE ? uniform(p.dom_grp[d + 1]) : 0;

    double Pre = 1.0, Pim = 0.0, Qre = 0.0, Qim = 0.0;
    // Diagnostics: sum over children of |w_c * ratio_c| (A) and the
    // product of the dets of blocks without a zero pivot.
    double sabs_reg = 0.0, sabs_fb = 0.0;
    double Xre = 1.0, Xim = 0.0;
    int nbad = 0, fbad = -1;

    // Test hook: a child's det is ratio * det_f * prod_{g != f} det_g.  The
    // other blocks' dets come from a first pass with the same factorisation
    // routine; the child's own block uses the factorisation its ratio was
    // solved with (for a numerically singular dominator block the two
    // products ratio and det_f are only consistent within one
    // factorisation).  The dominator's own det is written after the main
    // loop.
    double Dpre_re[kPairFlavors], Dpre_im[kPairFlavors];
    if (WITH_PAIRS) {
#pragma unroll
      for (int f = 0; f < kPairFlavors; ++f) {
        Dpre_re[f] = 1.0;
        Dpre_im[f] = 0.0;
        if (f < F) {
          const int o = p.off[f];
          uint32_t ro[N], co[N];
#pragma unroll
          for (int n = 0; n < N; ++n) {
            ro[n] = rowoff_d[o + n];
            co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
          }
          double gr[N][N], gi[N][N];
          bool z;
          lu_crout<N, TREE, PIV>(lds, ro, co, gr, gi, Dpre_re[f], Dpre_im[f], z);
        }
      }
    }

    int g = g_begin;
    for (int f = 0; f < F; ++f) {
      const int o = p.off[f];
      uint32_t ro[N], co[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        ro[n] = rowoff_d[o + n];
        co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
      }
      double gr[N][N], gi[N][N];
      double dre, dim;
      bool zero;
      // groups of this flavour form a contiguous run [g, g_f_end)
      int g_f_end = g;
      if (TREE) {
        while (g_f_end < g_end && uniform(p.grp_fr[g_f_end] >> 8) == f) ++g_f_end;
      }
      double accre = 0.0, accim = 0.0;
      // The tree keeps the multipliers for every dominator block: nearly
      // every dominator has groups in every flavour, and a single
      // factorisation path keeps the register allocation within budget.
      // The factorisation leaves co in its column order, which is the
      // order of the solved vectors x below.
      lu_crout<N, TREE, PIV>(lds, ro, co, gr, gi, dre, dim, zero);
      if (TREE) {
        double sre = 0.0, sim = 0.0;
        for (int gg = g; gg < g_f_end; ++gg) {
          const int r = uniform(p.grp_fr[gg] & 0xff);
          const int c_begin = uniform(p.grp_ptr[gg]);
          const int c_end = uniform(p.grp_ptr[gg + 1]);
          solve_unit_col<N>(gr, gi, r, gg, [&](const double (&xr)[N], const double (&xi)[N]) {
            if constexpr (AGG) {
              // multilinearity in row r: sum_c w_c det(G, row r := s_c) =
              // det(G, row r := sum_c w_c s_c), so the weighted rows are
              // summed first and dotted with x once
              double hr[N], hi[N];
#pragma unroll
              for (int n = 0; n < N; ++n) {
                hr[n] = 0.0;
                hi[n] = 0.0;
              }
              for (int c = c_begin; c < c_end; ++c) {
                const uint32_t crow = uniform(p.child_rowoff[c]);
                const double wc = a.w_src[uniform(p.child_term[c])] * p.child_wsgn[c];
                double2 sv[N];
#pragma unroll
                for (int n = 0; n < N; ++n)
                  sv[n] = *reinterpret_cast<const double2*>(lds + crow + co[n]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int n = 0; n < N; ++n) {
                  hr[n] = hr[n] + wc * sv[n].x;
                  hi[n] = hi[n] + wc * sv[n].y;
                }
              }
#pragma unroll
              for (int n = 0; n < N; ++n) {
                sre = sre + hr[n] * xr[n] - hi[n] * xi[n];
                sim = sim + hr[n] * xi[n] + hi[n] * xr[n];
              }
              return;
            }
            for (int c = c_begin; c < c_end; ++c) {
              const uint32_t crow = uniform(p.child_rowoff[c]);
              const int cterm = uniform(p.child_term[c]);
              // The child's N entries are read before any is used: without
              // the scheduling barrier the compiler, short of registers,
              // waits for each read before issuing the next.
              double2 sv[N];
#pragma unroll
              for (int n = 0; n < N; ++n)
                sv[n] = *reinterpret_cast<const double2*>(lds + crow + co[n]);
              __builtin_amdgcn_sched_barrier(0);
              double rr = 0.0, ri = 0.0;
#pragma unroll
              for (int n = 0; n < N; ++n) {
                rr = rr + sv[n].x * xr[n] - sv[n].y * xi[n];
                ri = ri + sv[n].x * xi[n] + sv[n].y * xr[n];
              }
              // the child's weight carries the sign of its row permutation
              const double sg = p.child_wsgn[c];
              const double wc = a.w_src[cterm] * sg;
              sre += wc * rr;
              sim += wc * ri;
              if (WITH_A && !zero) sabs_reg += fabs(wc) * cabs_scaled(rr, ri);
              if (WITH_PAIRS && valid && a.pair_det && !zero) {
                double cr = sg * (rr * dre - ri * dim), ci = sg * (rr * dim + ri * dre);
#pragma unroll
                for (int q = 0; q < kPairFlavors; ++q) {
                  if (q == f || q >= F) continue;
                  const double tr = cr * Dpre_re[q] - ci * Dpre_im[q];
                  ci = cr * Dpre_im[q] + ci * Dpre_re[q];
                  cr = tr;
                }
                a.pair_det[((size_t)t * p.n_src + cterm) * p.n_snk + k] = make_double2(cr, ci);
              }
            }
          });
        }
        // acc_f = det_f * sum_c w_c ratio_c  (0 for a zero-pivot block)
        accre = zero ? 0.0 : dre * sre - dim * sim;
        accim = zero ? 0.0 : dre * sim + dim * sre;
        if (zero) {
          ++nbad;
          fbad = g_f_end > g ? f : -2;   // -2: singular, but nothing to redo
        }
      } else if (zero) {
        ++nbad;
        fbad = -2;
      }
      g = g_f_end;
      // Q <- Q * D + acc * P ;  P <- P * D
      const double qr = Qre * dre - Qim * dim + accre * Pre - accim * Pim;
      const double qi = Qre * dim + Qim * dre + accre * Pim + accim * Pre;
      Qre = qr;
      Qim = qi;
      const double pr2 = Pre * dre - Pim * dim;
      Pim = Pre * dim + Pim * dre;
      Pre = pr2;
      if (!zero) {
        const double xr2 = Xre * dre - Xim * dim;
        Xim = Xre * dim + Xim * dre;
        Xre = xr2;
      }
    }

    if (WITH_PAIRS && valid && a.pair_det)
      a.pair_det[((size_t)t * p.n_src + term) * p.n_snk + k] = make_double2(Pre, Pim);

    // Fallback: a block with an exactly zero pivot.  If it is the only
    // singular block of the pair and it has children, their blocks are
    // factorised directly; every other block keeps the dominator's det
    // (the product X of the non-singular blocks).
    if (TREE) {
      const bool need = valid && nbad == 1 && fbad >= 0;
      if (__builtin_amdgcn_ballot_w64(need) != 0) {
        for (int f = 0; f < F; ++f) {
          if (__builtin_amdgcn_ballot_w64(need && fbad == f) == 0) continue;
          const int o = p.off[f];
          uint32_t co[N];
#pragma unroll
          for (int n = 0; n < N; ++n) co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
          double fre = 0.0, fim = 0.0;
          for (int gg = g_begin; gg < g_end; ++gg) {
            if (uniform(p.grp_fr[gg] >> 8) != f) continue;
            const int r = uniform(p.grp_fr[gg] & 0xff);
            for (int c = uniform(p.grp_ptr[gg]); c < uniform(p.grp_ptr[gg + 1]); ++c) {
              if (need && fbad == f) {
                double cre, cim;
                child_det_direct<N>(lds, rowoff_d + o, r, p.child_rowoff[c], co, cre, cim);
                cre *= p.child_wsgn[c];
                cim *= p.child_wsgn[c];
                const double wc = a.w_src[p.child_term[c]];
                fre += wc * cre;
                fim += wc * cim;
                const double dr = cre * Xre - cim * Xim, di = cre * Xim + cim * Xre;
                if (WITH_A) sabs_fb += fabs(wc) * cabs_scaled(dr, di);
                if (WITH_PAIRS && a.pair_det)
                  a.pair_det[((size_t)t * p.n_src + p.child_term[c]) * p.n_snk + k] =
                      make_double2(dr, di);
                ++n_fallback;
              }
            }
          }
          if (need && fbad == f) {
            Qre += fre * Xre - fim * Xim;
            Qim += fre * Xim + fim * Xre;
          }
        }
      }
      // Pairs whose blocks are singular in two flavours, or whose singular
      // block has no children, have determinant 0: write zeros for them.
      if (WITH_PAIRS && a.pair_det && valid && nbad > 0) {
        for (int gg = g_begin; gg < g_end; ++gg) {
          const int f = uniform(p.grp_fr[gg] >> 8);
          if (nbad == 1 && fbad == f) continue;   // written above
          for (int c = uniform(p.grp_ptr[gg]); c < uniform(p.grp_ptr[gg + 1]); ++c) {
            // a child of a non-singular flavour still sees the singular
            // block of the other flavour: det 0
            a.pair_det[((size_t)t * p.n_src + p.child_term[c]) * p.n_snk + k] =
                make_double2(0.0, 0.0);
          }
        }
      }
    }

    if (valid) {
      acc_re += wk * (wi * Pre + Qre);
      acc_im += wk * (wi * Pim + Qim);
      if (WITH_A) {
        // |d_child| = |ratio| |P| for children taken by the update; the
        // fallback children carry their own |det| in sabs_fb.
        const double pabs = cabs_scaled(Pre, Pim);
        acc_a += fabs(wk) * ((fabs(wi) + sabs_reg) * pabs + sabs_fb);
      }
    }
  }

  // Workgroup reduction (fixed order) -> one partial per workgroup.
  __shared__ double red[kWavesPerBlock][3];
  const double s0 = wave_sum(acc_re), s1 = wave_sum(acc_im);
  const double s2 = WITH_A ? wave_sum(acc_a) : 0.0;
  if (lane == 0) {
    red[wave][0] = s0;
    red[wave][1] = s1;
    red[wave][2] = s2;
  }
  if (TREE && a.fallback) {
    uint32_t nf = n_fallback;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) nf += __shfl_xor(nf, o, kWave);
    if (lane == 0 && nf) atomicAdd(a.fallback, (unsigned long long)nf);
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) v += red[w][threadIdx.x];
    a.partial[((size_t)t * a.n_blk_t + chunk) * 3 + threadIdx.x] = v;
  }
}

template <int N, bool TREE, int MODE>
__global__ __launch_bounds__(kBlock, 2) void contract_kernel(ContractArgs a) {
  extern __shared__ double2 smem[];
  lane_tile<N, TREE, MODE>(a, blockIdx.y, blockIdx.x, smem);
}

// Persistent form: workgroup w takes tiles w, w + gridDim.x, ... of a tile
// table spanning many jobs.
template <int N, bool TREE, int MODE>
__global__ __launch_bounds__(kBlock, 2) void batch_lane_kernel(BatchArgs b) {
  extern __shared__ double2 smem[];
  for (int i = blockIdx.x; i < b.n_tiles; i += gridDim.x) {
    const int4 tl = b.tiles[i];
    lane_tile<N, TREE, MODE>(b.jobs[tl.x], tl.y, tl.z, smem);
  }
}

// C[t] = sum over workgroups of the partials, in a fixed order.
__global__ __launch_bounds__(kBlock) void reduce_partials(const double* partial, int n_blk_t,
                                                          double2* C, double* A) {
  const int t = blockIdx.x;
  __shared__ double red[3][kBlock];
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < n_blk_t; b += kBlock)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] += partial[((size_t)t * n_blk_t + b) * 3 + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    C[t] = make_double2(red[0][0], red[1][0]);
    if (A) A[t] = red[2][0];
  }
}

template <int N, bool TREE, int MODE>
static hipError_t launch_one(const ContractArgs& a, hipStream_t s) {
  dim3 grid(a.n_blk_t, a.T);
  size_t lds = lds_slice_bytes(a.plan.M);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&contract_kernel<N, TREE, MODE>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((contract_kernel<N, TREE, MODE>), grid, dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_n(const ContractArgs& a, bool tree, bool diag, int pivot,
                           hipStream_t s) {
  if (pivot == 3) return launch_one<N, true, 16>(a, s);   // weighted-row aggregation
  if (pivot == 2) {
    if (tree) return diag ? launch_one<N, true, 11>(a, s) : launch_one<N, true, 8>(a, s);
    return diag ? launch_one<N, false, 11>(a, s) : launch_one<N, false, 8>(a, s);
  }
  if (!pivot) {
    if (tree) return diag ? launch_one<N, true, 7>(a, s) : launch_one<N, true, 4>(a, s);
    return diag ? launch_one<N, false, 7>(a, s) : launch_one<N, false, 4>(a, s);
  }
  if (tree) return diag ? launch_one<N, true, 3>(a, s) : launch_one<N, true, 0>(a, s);
  return diag ? launch_one<N, false, 3>(a, s) : launch_one<N, false, 0>(a, s);
}

hipError_t launch_contract(const ContractArgs& a, int n, bool tree, bool diag, int pivot,
                           double2* C, double* A, hipStream_t s) {
  hipError_t e;
  switch (n) {
    case 1: e = launch_n<1>(a, tree, diag, pivot, s); break;
    case 2: e = launch_n<2>(a, tree, diag, pivot, s); break;
    case 3: e = launch_n<3>(a, tree, diag, pivot, s); break;
    case 4: e = launch_n<4>(a, tree, diag, pivot, s); break;
    case 5: e = launch_n<5>(a, tree, diag, pivot, s); break;
    case 6: e = launch_n<6>(a, tree, diag, pivot, s); break;
    case 7: e = launch_n<7>(a, tree, diag, pivot, s); break;
    case 8: e = launch_n<8>(a, tree, diag, pivot, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return launch_reduce(a, C, A, s);
}

template <int N, bool TREE, int MODE>
static hipError_t launch_batch_lane_m(const BatchArgs& b, int grid, size_t lds, hipStream_t s) {
  hipError_t e =
      hipFuncSetAttribute(reinterpret_cast<const void*>(&batch_lane_kernel<N, TREE, MODE>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_lane_kernel<N, TREE, MODE>), dim3(grid), dim3(kBlock), lds, s, b);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_batch_lane_n(const BatchArgs& b, bool tree, bool with_a, int grid,
                                      size_t lds, hipStream_t s) {
  if (tree)
    return with_a ? launch_batch_lane_m<N, true, 1>(b, grid, lds, s)
                  : launch_batch_lane_m<N, true, 0>(b, grid, lds, s);
  return with_a ? launch_batch_lane_m<N, false, 1>(b, grid, lds, s)
                : launch_batch_lane_m<N, false, 0>(b, grid, lds, s);
}

hipError_t launch_batch_lane(const BatchArgs& b, int n, bool tree, bool with_a, int grid,
                             size_t lds, hipStream_t s) {
  switch (n) {
#define MHC_CASE(NN)                                                             \
  case NN:                                                                       \
    return launch_batch_lane_n<NN>(b, tree, with_a, grid, lds, s);
    MHC_CASE(1) MHC_CASE(2) MHC_CASE(3) MHC_CASE(4) MHC_CASE(5) MHC_CASE(6) MHC_CASE(7)
    MHC_CASE(8)
#undef MHC_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// C_j[t] for every (job, slice) of a batch: one workgroup per entry of pairs
// (job, t), summing that job's partials in a fixed order.
__global__ __launch_bounds__(kBlock) void batch_reduce(const ContractArgs* jobs, const int2* jt) {
  const int2 e = jt[blockIdx.x];
  const ContractArgs& a = jobs[e.x];
  const int t = e.y;
  __shared__ double red[3][kBlock];
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < a.n_blk_t; b += kBlock)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] += a.partial[((size_t)t * a.n_blk_t + b) * 3 + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.C[t] = make_double2(red[0][0], red[1][0]);
    if (a.A) a.A[t] = red[2][0];
  }
}

hipError_t launch_batch_reduce(const ContractArgs* jobs, const int2* jt, int n, hipStream_t s) {
  hipLaunchKernelGGL(batch_reduce, dim3(n), dim3(kBlock), 0, s, jobs, jt);
  return hipGetLastError();
}

hipError_t launch_reduce(const ContractArgs& a, double2* C, double* A, hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials, dim3(a.T), dim3(kBlock), 0, s, a.partial, a.n_blk_t, C, A);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace mhc
