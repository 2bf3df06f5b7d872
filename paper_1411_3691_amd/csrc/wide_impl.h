// Contraction kernels for flavour blocks of any size up to NMAX (gfx950):
// the templates, instantiated per block-size bucket by wide_b*.hip.
//
// One group of GROUP lanes (8, 16 or 32) holds one matrix, one row per
// lane, so a row exchange is a relabelling: no data moves.  Every block of
// every flavour may have its own size n <= NMAX (lanes m >= n hold no row).
//
// Per flavour block of a (row set, sink) pair the group runs Gauss-Jordan
// elimination with partial pivoting (gauss_jordan_rhs: pivot = largest
// |Re| + |Im| among the rows not yet used, lowest row on ties), the pivots
// of GEPP.  For the update tree the elimination carries, as right-hand
// sides, the unit columns e_r of the block's groups (Sec. 2: the children
// that replace row r share x = G^-1 e_r): at the end lane m holds
// x_r[col_m] for every group at once, with no second pass over the row
// operations.  A child whose row r is replaced by s has det = det G *
// (s . x_r) (matrix determinant lemma, Sec. 2): lane m multiplies s[col_m]
// by x_r[col_m].  The products of one dot are summed over the group's lanes
// where a per-pair value is needed (the scale A and the pair-determinant
// hook); otherwise each lane keeps its share of every dot, weighted, in its
// own running sum, and the group's lanes meet only in the final reduction
// of the tile (the weighted sum over children is linear in each dot).
// More groups than RMAX in one block are taken in further eliminations.
//
// Work decomposition: a wave holds 64 / GROUP sinks of one row set (the
// tree structure stays wave-uniform); a workgroup stages S_t in LDS and its
// waves walk a strided share of the slice's items, as in the one-lane-per-
// matrix kernels.  Reductions are fixed-order.
//
// Broadcasts within a group go through a per-group LDS row buffer (the
// pivot lane writes its row, every lane reads it back with one ds_read_b128
// per complex entry) when the workgroup size chooses it and the buffers fit
// beside the copy of S_t; otherwise through ds_bpermute shuffles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "contract_kernels.h"
#include "group_device.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

// Workgroup sizes: 512 threads (two waves per SIMD, up to 256 VGPRs per
// lane), 768 (three, 168) or 1024 (four, 128).
constexpr int kWideBlock = 512;
constexpr int kWideBlockMid = 768;
constexpr int kWideBlockBig = 1024;

// The update tree's unit columns: replayed after the elimination in one
// batched pass (true), or carried through it as right-hand sides (false).
constexpr bool kWideReplay = false;

// Right-hand sides carried per elimination by the update tree (groups of
// one flavour block beyond this take another elimination); the plain LU
// carries none.
template <int NMAX, bool TREE>
constexpr int wide_rmax() {
  return !TREE ? 0 : NMAX < 8 ? NMAX : 8;
}

// Threads per workgroup of a bucket's kernel, from the registers each
// needs: the diagnostic modes (A, pair determinants) and the tree's blocks
// above 12 keep 512; the fast tree up to 12 runs 768 (measured faster than
// 1024 and 512 on the large workload and the batch); the plain LU up to 12
// and 18 fits 1024, the plain LU of 16 and 24 fits 768.
template <int NMAX, bool TREE, int MODE>
constexpr int wide_wb() {
  if ((MODE & 3) != 0) return kWideBlock;
  if (!TREE) return (NMAX == 16 || NMAX == 24) ? kWideBlockMid : kWideBlockBig;
  return NMAX <= 12 ? kWideBlockMid : kWideBlock;
}

// The LDS a workgroup can have: 160 KiB, less 1 KiB for the static arrays
// of the kernels.
constexpr size_t kWideLdsLimit = 159 * 1024;

// Bytes of the groups' row buffers of one workgroup (LDS broadcasts).
template <int GROUP, int NMAX, bool TREE>
constexpr size_t wide_rows_bytes(int wb) {
  // a replay reuses the row buffer (nr <= RMAX <= NMAX entries)
  return (size_t)(wb / GROUP) *
         prow_entries<NMAX, kWideReplay ? 0 : wide_rmax<NMAX, TREE>()>() * 16;
}

// One tile (slice t, chunk) of a job, as lane_tile for one matrix per lane.
// MODE bit 0: accumulate A(t); bit 1: write every pair det.  BCAST: pivot
// rows through the LDS row buffers.
template <int GROUP, int NMAX, bool TREE, int MODE, int WB, bool BCAST>
__device__ __forceinline__ void wide_tile(const ContractArgs& a, int t, int chunk,
                                          double2* smem) {
  constexpr bool WITH_A = (MODE & 1) != 0;
  constexpr bool WITH_PAIRS = (MODE & 2) != 0;
  constexpr bool DIAG = (MODE & 3) != 0;   // per-child ratios summed over the group
  constexpr bool AGG = (MODE & 16) != 0;   // weighted-row aggregation per group
  static_assert(!(AGG && DIAG), "aggregation forms no per-pair values");
  constexpr int SPW = kWave / GROUP;   // sinks per wave
  constexpr int RMAX = wide_rmax<NMAX, TREE>() > 0 ? wide_rmax<NMAX, TREE>() : 1;
  const PlanView& p = a.plan;
  __syncthreads();  // the previous tile of this workgroup is done with LDS
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  const int m = lane % GROUP;          // row of the matrix held by this lane
  const int gsel = lane / GROUP;       // which sink of the wave
  const int MM = p.M * p.M;
  const double2* St = a.S + (size_t)t * MM;
  constexpr int kWaves = WB / kWave;
  // this group's row buffer (LDS broadcasts only), then the copy of S_t
  double2* prow = smem + (threadIdx.x / GROUP) *
                           prow_entries<NMAX, kWideReplay ? 0 : wide_rmax<NMAX, TREE>()>();
  double2* slice = smem + (BCAST ? wide_rows_bytes<GROUP, NMAX, TREE>(WB) / 16 : 0);
  stage_slice(St, slice, p.M, WB);
  __syncthreads();
  const char* lds = reinterpret_cast<const char*>(slice);

  double acc_re = 0.0, acc_im = 0.0, acc_a = 0.0;
  uint32_t n_fallback = 0;
  const int F = p.F;
  const int sn = p.sn;

  for (int item = chunk + a.n_blk_t * wave; item < a.n_items;
       item += a.n_blk_t * kWaves) {
    const int d = uniform(item / a.n_sblk);
    const int sb = uniform(item - d * a.n_sblk);
    const int k = sb * SPW + gsel;
    const bool valid = k < p.n_snk;
    const int term = TREE ? uniform(p.dom_term[d]) : d;
    const uint32_t* rowoff_d = (TREE ? p.dom_rowoff : p.src_rowoff) + (size_t)d * sn;
    const double wi = a.w_src[term];
    const double wk = valid ? a.w_snk[k] : 0.0;
    const int g_begin = TREE ? uniform(p.dom_grp[d]) : 0;
    const int g_end = TREE ? uniform(p.dom_grp[d + 1]) : 0;
    const bool writer = valid && m == 0;

    // P: product of the blocks' dets (the same in every lane of the group);
    // Q: the children's weighted dets folded over the flavours -- the
    // group's value in every lane (DIAG) or this lane's share of it.
    double Pre = 1.0, Pim = 0.0, Qre = 0.0, Qim = 0.0;
    double Xre = 1.0, Xim = 0.0;     // product of the non-singular blocks
    double sabs_reg = 0.0, sabs_fb = 0.0;
    int nbad = 0, fbad = -1;

    // Test hook: a child's det is ratio * det_f * prod_{g != f} det_g; the
    // other blocks' dets come from a first pass (the child's own block uses
    // the elimination its ratio came from).
    double Dpre_re[kPairFlavors], Dpre_im[kPairFlavors];
    if (WITH_PAIRS) {
#pragma unroll
      for (int f = 0; f < kPairFlavors; ++f) {
        Dpre_re[f] = 1.0;
        Dpre_im[f] = 0.0;
        if (f < F) {
          const int o = p.off[f];
          const int n = p.off[f + 1] - o;
          uint32_t co[NMAX];
#pragma unroll
          for (int c = 0; c < NMAX; ++c)
            co[c] = c < n ? p.snk_coloff[(size_t)(o + c) * p.n_snk_pad + k] : 0u;
          const uint32_t myrow = m < n ? rowoff_d[o + m] : 0u;
          block_det_direct<GROUP, NMAX>(lds, myrow, -1, 0u, co, n, m, Dpre_re[f], Dpre_im[f]);
        }
      }
    }

    int g = g_begin;
    double Bre = 0.0, Bim = 0.0;     // direct route: sum of w_c det(child block)
    double babs = 0.0;               // and of |w_c det(child block)|
    for (int f = 0; f < F; ++f) {
      const int o = p.off[f];
      const int n = p.off[f + 1] - o;
      uint32_t co[NMAX];
#pragma unroll
      for (int c = 0; c < NMAX; ++c)
        co[c] = c < n ? p.snk_coloff[(size_t)(o + c) * p.n_snk_pad + k] : 0u;
      const uint32_t myrow = m < n ? rowoff_d[o + m] : 0u;
      int g_f_end = g;
      if (TREE) {
        while (g_f_end < g_end && uniform(p.grp_fr[g_f_end] >> 8) == f) ++g_f_end;
      }
      const int R = g_f_end - g;
      const int npass = R > RMAX ? (R + RMAX - 1) / RMAX : 1;
      const int c_first = TREE && R > 0 ? uniform(p.grp_ptr[g]) : 0;
      const int n_child = TREE && R > 0 ? uniform(p.grp_ptr[g_f_end]) - c_first : 0;
      double dre = 1.0, dim = 0.0;
      bool zero = false;
      double sre = 0.0, sim = 0.0;   // sum over children of w_c * ratio_c (or this lane's share)
      double bre = 0.0, bim = 0.0, bab = 0.0;
      // Eliminations of this block: npass over the dominator's block, each
      // carrying up to RMAX groups' unit columns; then, in a group whose
      // dominator block has an exactly zero pivot (no inverse), one direct
      // elimination per child of the block with the child's row in place.
      // One elimination routine serves all of them.
      int gq = g;                      // group of the next direct child
      for (int pass = 0; pass < npass + (zero ? n_child : 0); ++pass) {
        const bool direct = pass >= npass;
        const int g0 = direct ? 0 : pass * RMAX;
        const int nr = direct ? 0 : (R - g0 < RMAX ? R - g0 : RMAX);
        uint32_t row = myrow;
        int cterm = 0;
        if (direct) {
          // child c_first + (pass - npass): its group and new row
          const int c = c_first + pass - npass;
          while (uniform(p.grp_ptr[gq + 1]) <= c) ++gq;
          const int r = uniform(p.grp_fr[gq] & 0xff);
          cterm = uniform(p.child_term[c]);
          if (m == r) row = uniform(p.child_rowoff[c]);
        } else if (zero) {
          continue;                    // no inverse: no solves to carry
        }
        double ar[NMAX], ai[NMAX];
        load_row<NMAX>(lds, row, co, n, m, ar, ai);
        double brr[RMAX], bri[RMAX];
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
          const int r = q < nr ? uniform(p.grp_fr[g + g0 + q] & 0xff) : -1;
          brr[q] = (m == r) ? 1.0 : 0.0;
          bri[q] = 0.0;
        }
        double ur, ui;
        int col;
        constexpr bool REPLAY = kWideReplay && TREE;
        PivotLanes<NMAX> piv;
        const GJResult res = gauss_jordan_rhs<GROUP, NMAX, RMAX, BCAST, REPLAY>(
            ar, ai, brr, bri, REPLAY ? 0 : nr, n, m, ur, ui, col, prow, &piv);
        if (REPLAY && !direct && !res.zero && nr > 0)
          replay_units<GROUP, NMAX, RMAX, BCAST>(ar, ai, piv, n, m, brr, bri, nr, prow);
        if (direct) {
          // the child's block determinant (its other blocks are the
          // dominator's; the product is formed after the flavour loop),
          // signed by its row permutation
          const double sg = p.child_wsgn[c_first + pass - npass];
          const double wc = a.w_src[cterm] * sg;
          bre += wc * res.dre;
          bim += wc * res.dim;
          if (WITH_A) bab += fabs(wc) * cabs_scaled(res.dre, res.dim);
          if (WITH_PAIRS && writer && a.pair_det) {
            double cr = sg * res.dre, ci = sg * res.dim;
#pragma unroll
            for (int h = 0; h < kPairFlavors; ++h) {
              if (h == f || h >= F) continue;
              const double tr = cr * Dpre_re[h] - ci * Dpre_im[h];
              ci = cr * Dpre_im[h] + ci * Dpre_re[h];
              cr = tr;
            }
            a.pair_det[((size_t)t * p.n_src + cterm) * p.n_snk + k] = make_double2(cr, ci);
          }
          if (m == 0) ++n_fallback;
          continue;
        }
        if (pass == 0) {
          dre = res.dre;
          dim = res.dim;
          zero = res.zero;
        }
        if (!TREE || zero) continue;
        // this lane's pivot column: its sink column offset
        uint32_t mycol = 0;
#pragma unroll
        for (int c = 0; c < NMAX; ++c)
          if (c == col) mycol = co[c];
        static_for<0, RMAX>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          if (q >= nr) return;
          // x_r[col_m] = b'_q[m] / u_m
          const double x_r = brr[q] * ur - bri[q] * ui;
          const double x_i = brr[q] * ui + bri[q] * ur;
          const int gg = g + g0 + q;
          const int c_begin = uniform(p.grp_ptr[gg]);
          const int c_end = uniform(p.grp_ptr[gg + 1]);
          if constexpr (AGG) {
            // multilinearity in row r: the children's weighted rows are
            // summed first (this lane's column), then dotted with x once
            double hr = 0.0, hi = 0.0;
            for (int c = c_begin; c < c_end; ++c) {
              const uint32_t crow = uniform(p.child_rowoff[c]);
              const double wc = a.w_src[uniform(p.child_term[c])] * p.child_wsgn[c];
              if (m < n) {
                const double2 sv = *reinterpret_cast<const double2*>(lds + crow + mycol);
                hr += wc * sv.x;
                hi += wc * sv.y;
              }
            }
            sre += hr * x_r - hi * x_i;
            sim += hr * x_i + hi * x_r;
            return;
          }
          for (int c = c_begin; c < c_end; ++c) {
            const uint32_t crow = uniform(p.child_rowoff[c]);
            const int ct = uniform(p.child_term[c]);
            // the child's weight carries the sign of its row permutation
            const double sg = p.child_wsgn[c];
            const double wc = a.w_src[ct] * sg;
            double pr_ = 0.0, pi_ = 0.0;
            if (m < n) {
              const double2 s = *reinterpret_cast<const double2*>(lds + crow + mycol);
              pr_ = s.x * x_r - s.y * x_i;
              pi_ = s.x * x_i + s.y * x_r;
            }
            if constexpr (DIAG) {
              const double rr = group_sum<GROUP>(pr_);
              const double ri = group_sum<GROUP>(pi_);
              sre += wc * rr;
              sim += wc * ri;
              if (WITH_A) sabs_reg += fabs(wc) * cabs_scaled(rr, ri);
              if (WITH_PAIRS && writer && a.pair_det) {
                double cr = sg * (rr * dre - ri * dim), ci = sg * (rr * dim + ri * dre);
#pragma unroll
                for (int h = 0; h < kPairFlavors; ++h) {
                  if (h == f || h >= F) continue;
                  const double tr = cr * Dpre_re[h] - ci * Dpre_im[h];
                  ci = cr * Dpre_im[h] + ci * Dpre_re[h];
                  cr = tr;
                }
                a.pair_det[((size_t)t * p.n_src + ct) * p.n_snk + k] = make_double2(cr, ci);
              }
            } else {
              sre += wc * pr_;
              sim += wc * pi_;
            }
          }
        });
      }
      // acc_f = det_f * sum_c w_c ratio_c  (0 for a zero-pivot block)
      const double accre = zero ? 0.0 : dre * sre - dim * sim;
      const double accim = zero ? 0.0 : dre * sim + dim * sre;
      if (zero) {
        ++nbad;
        fbad = (TREE && R > 0) ? f : -2;
        Bre = bre;
        Bim = bim;
        babs = bab;
      }
      g = g_f_end;
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

    // The group's values that every lane holds alike enter through lane 0
    // only; in the fast mode Q is already this lane's share.  Children of a
    // singular block (the only singular one) came from the direct route:
    // their determinants are det(child block) times the other blocks' (X).
    double Ure = 0.0, Uim = 0.0;
    if (TREE && nbad == 1 && fbad >= 0) {
      Ure = Bre * Xre - Bim * Xim;
      Uim = Bre * Xim + Bim * Xre;
      if (WITH_A) sabs_fb = babs * cabs_scaled(Xre, Xim);
    }

    if (WITH_PAIRS && a.pair_det && writer) {
      a.pair_det[((size_t)t * p.n_src + term) * p.n_snk + k] = make_double2(Pre, Pim);
    }
    if (valid) {
      const double ure = wi * Pre + Ure + (DIAG ? Qre : 0.0);
      const double uim = wi * Pim + Uim + (DIAG ? Qim : 0.0);
      if (m == 0) {
        acc_re += wk * ure;
        acc_im += wk * uim;
      }
      if (!DIAG) {
        acc_re += wk * Qre;
        acc_im += wk * Qim;
      }
      if (WITH_A && m == 0) {
        const double pabs = cabs_scaled(Pre, Pim);
        acc_a += fabs(wk) * ((fabs(wi) + sabs_reg) * pabs + sabs_fb);
      }
    }
  }

  __shared__ double red[kWaves][3];
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
    for (int w = 0; w < kWaves; ++w) v += red[w][threadIdx.x];
    a.partial[((size_t)t * a.n_blk_t + chunk) * 3 + threadIdx.x] = v;
  }
}

template <int GROUP, int NMAX, bool TREE, int MODE, int WB, bool BCAST>
__global__ __launch_bounds__(WB) void contract_wide_kernel(ContractArgs a) {
  extern __shared__ double2 smem[];
  wide_tile<GROUP, NMAX, TREE, MODE, WB, BCAST>(a, blockIdx.y, blockIdx.x, smem);
}

template <int GROUP, int NMAX, bool TREE, int MODE, int WB, bool BCAST>
__global__ __launch_bounds__(WB) void batch_wide_kernel(BatchArgs b) {
  extern __shared__ double2 smem[];
  for (int i = blockIdx.x; i < b.n_tiles; i += gridDim.x) {
    const int4 tl = b.tiles[i];
    wide_tile<GROUP, NMAX, TREE, MODE, WB, BCAST>(b.jobs[tl.x], tl.y, tl.z, smem);
  }
}

// Pivot rows through LDS where the groups' row buffers fit beside the
// slice of S, else through shuffles.
template <int GROUP, int NMAX, bool TREE, int MODE>
bool wide_bcast(size_t slice) {
  return slice + wide_rows_bytes<GROUP, NMAX, TREE>(wide_wb<NMAX, TREE, MODE>()) <=
         kWideLdsLimit;
}

template <int GROUP, int NMAX, bool TREE, int MODE, bool BCAST>
hipError_t launch_wide_cfg(const ContractArgs& a, size_t slice, hipStream_t s) {
  constexpr int WB = wide_wb<NMAX, TREE, MODE>();
  dim3 grid(a.n_blk_t, a.T);
  const size_t lds = slice + (BCAST ? wide_rows_bytes<GROUP, NMAX, TREE>(WB) : 0);
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&contract_wide_kernel<GROUP, NMAX, TREE, MODE, WB, BCAST>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((contract_wide_kernel<GROUP, NMAX, TREE, MODE, WB, BCAST>), grid, dim3(WB),
                     lds, s, a);
  return hipGetLastError();
}

template <int GROUP, int NMAX, bool TREE, int MODE>
hipError_t launch_wide_one(const ContractArgs& a, hipStream_t s) {
  const size_t slice = lds_slice_bytes(a.plan.M);
  if (wide_bcast<GROUP, NMAX, TREE, MODE>(slice))
    return launch_wide_cfg<GROUP, NMAX, TREE, MODE, true>(a, slice, s);
  return launch_wide_cfg<GROUP, NMAX, TREE, MODE, false>(a, slice, s);
}

// diag: the scale A and/or the dense pair table; the pair table (MODE 3)
// needs a first pass over the blocks, A alone (MODE 1) does not.
template <int GROUP, int NMAX>
hipError_t launch_wide_n(const ContractArgs& a, bool tree, bool diag, bool agg, hipStream_t s) {
  const bool pairs = a.pair_det != nullptr;
  if (tree) {
    if (agg) return launch_wide_one<GROUP, NMAX, true, 16>(a, s);
    if (!diag) return launch_wide_one<GROUP, NMAX, true, 0>(a, s);
    return pairs ? launch_wide_one<GROUP, NMAX, true, 3>(a, s)
                 : launch_wide_one<GROUP, NMAX, true, 1>(a, s);
  }
  if (!diag) return launch_wide_one<GROUP, NMAX, false, 0>(a, s);
  return pairs ? launch_wide_one<GROUP, NMAX, false, 3>(a, s)
               : launch_wide_one<GROUP, NMAX, false, 1>(a, s);
}

template <int GROUP, int NMAX, bool TREE, int MODE, bool BCAST>
hipError_t launch_batch_wide_cfg(const BatchArgs& b, int grid, size_t slice, hipStream_t s) {
  constexpr int WB = wide_wb<NMAX, TREE, MODE>();
  const size_t lds = slice + (BCAST ? wide_rows_bytes<GROUP, NMAX, TREE>(WB) : 0);
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&batch_wide_kernel<GROUP, NMAX, TREE, MODE, WB, BCAST>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_wide_kernel<GROUP, NMAX, TREE, MODE, WB, BCAST>), dim3(grid),
                     dim3(WB), lds, s, b);
  return hipGetLastError();
}

template <int GROUP, int NMAX, bool TREE, int MODE>
hipError_t launch_batch_wide_m(const BatchArgs& b, int grid, size_t slice, hipStream_t s) {
  if (wide_bcast<GROUP, NMAX, TREE, MODE>(slice))
    return launch_batch_wide_cfg<GROUP, NMAX, TREE, MODE, true>(b, grid, slice, s);
  return launch_batch_wide_cfg<GROUP, NMAX, TREE, MODE, false>(b, grid, slice, s);
}

// Workgroups of the batch kernel chosen for this slice size that stay
// resident on one compute unit together (registers and LDS).
template <int GROUP, int NMAX, bool TREE, int MODE>
int batch_wide_resident(size_t slice) {
  constexpr int WB = wide_wb<NMAX, TREE, MODE>();
  const bool bc = wide_bcast<GROUP, NMAX, TREE, MODE>(slice);
  const size_t lds = slice + (bc ? wide_rows_bytes<GROUP, NMAX, TREE>(WB) : 0);
  const void* fn = bc ? reinterpret_cast<const void*>(
                            &batch_wide_kernel<GROUP, NMAX, TREE, MODE, WB, true>)
                      : reinterpret_cast<const void*>(
                            &batch_wide_kernel<GROUP, NMAX, TREE, MODE, WB, false>);
  int n = 0;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, WB, lds) != hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <int GROUP, int NMAX>
int batch_wide_resident_n(bool tree, bool with_a, size_t slice) {
  if (tree)
    return with_a ? batch_wide_resident<GROUP, NMAX, true, 1>(slice)
                  : batch_wide_resident<GROUP, NMAX, true, 0>(slice);
  return with_a ? batch_wide_resident<GROUP, NMAX, false, 1>(slice)
                : batch_wide_resident<GROUP, NMAX, false, 0>(slice);
}

template <int GROUP, int NMAX>
hipError_t launch_batch_wide_n(const BatchArgs& b, bool tree, bool with_a, int grid,
                               size_t slice, hipStream_t s) {
  if (tree)
    return with_a ? launch_batch_wide_m<GROUP, NMAX, true, 1>(b, grid, slice, s)
                  : launch_batch_wide_m<GROUP, NMAX, true, 0>(b, grid, slice, s);
  return with_a ? launch_batch_wide_m<GROUP, NMAX, false, 1>(b, grid, slice, s)
                : launch_batch_wide_m<GROUP, NMAX, false, 0>(b, grid, slice, s);
}

// Per-bucket entry points (one translation unit each, wide_b<NMAX>.hip).
#define MHC_WIDE_BUCKET(GROUP, NMAX)                                                        \
  hipError_t launch_contract_wide_b##NMAX(const ContractArgs& a, bool tree, bool diag,      \
                                          bool agg, hipStream_t s) {                        \
    return launch_wide_n<GROUP, NMAX>(a, tree, diag, agg, s);                               \
  }                                                                                         \
  hipError_t launch_batch_wide_b##NMAX(const BatchArgs& b, bool tree, bool with_a, int grid, \
                                       size_t slice, hipStream_t s) {                       \
    return launch_batch_wide_n<GROUP, NMAX>(b, tree, with_a, grid, slice, s);               \
  }                                                                                         \
  int wide_block_b##NMAX(bool tree, size_t) {                                               \
    return tree ? wide_wb<NMAX, true, 0>() : wide_wb<NMAX, false, 0>();                      \
  }                                                                                         \
  int batch_wide_resident_b##NMAX(bool tree, bool with_a, size_t slice) {                   \
    return batch_wide_resident_n<GROUP, NMAX>(tree, with_a, slice);                          \
  }

}  // namespace kern
}  // namespace mhc
