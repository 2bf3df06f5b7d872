// Contraction kernels for flavour blocks up to 24 with several rows of a
// matrix per lane (gfx950): the templates, instantiated per block-size
// bucket by rows_b*.hip.
//
// A group of GROUP lanes holds one (row set, sink) block, ROWS rows per
// lane (rows_device.h).  Per flavour block the group runs Gauss-Jordan
// elimination with partial pivoting; for the update tree it carries, as
// right-hand sides, the unit columns e_r of the block's groups (Sec. 2:
// the children that replace row r share x = G^-1 e_r).  A child whose row r
// is replaced by s has det = det G * (s . x_r) (matrix determinant lemma,
// Sec. 2): each lane multiplies s at its rows' pivot columns by its
// entries of x_r.  In the fast mode each lane keeps its share of every dot,
// weighted, in its running sum (the weighted sum over children is linear in
// each dot); the scale A needs each child's |ratio| and sums the dot over
// the group first.  More groups than RMAX in one block are taken in further
// eliminations; a dominator block with an exactly zero pivot has no inverse,
// and its children are then eliminated directly with their own row in
// place.
//
// LDS holds, per workgroup, the pivot-row buffers of its groups and the
// rows of S_t its current tile needs: the rows of each unit's row set (a
// dominator, or a source term for the plain LU) and the new rows of the
// unit's children, gathered by the plan (compact staging; a full slice of
// M = 96 would leave no room for the buffers).  A tile is (range of units,
// range of sinks); the waves of the workgroup walk its (unit, block of
// 64 / GROUP sinks) items.  A dominator whose rows do not fit one tile is
// split into units by ranges of its children (only the first unit counts
// the dominator's own term).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contract_kernels.h"
#include "group_device.h"
#include "lu_device.h"
#include "rows_device.h"

namespace mhc {
namespace kern {

// Lanes per matrix, rows per lane, right-hand sides per elimination and
// threads per workgroup of each bucket (largest block NMAX).
template <int NMAX>
struct RowsCfg;
template <>
struct RowsCfg<8> {
  static constexpr int GROUP = 4, ROWS = 2, RMAX = 4, WB = 768;
};
template <>
struct RowsCfg<12> {
  static constexpr int GROUP = 4, ROWS = 3, RMAX = 2, WB = 512;
};
template <>
struct RowsCfg<16> {
  static constexpr int GROUP = 8, ROWS = 2, RMAX = 2, WB = 512;
};
template <>
struct RowsCfg<18> {
  static constexpr int GROUP = 16, ROWS = 2, RMAX = 2, WB = 512;
};
template <>
struct RowsCfg<24> {
  static constexpr int GROUP = 16, ROWS = 2, RMAX = 1, WB = 512;
};

template <int NMAX, bool TREE>
constexpr int rows_rmax() {
  return TREE ? RowsCfg<NMAX>::RMAX : 0;
}

// Bytes of the pivot-row buffers of one workgroup.
template <int NMAX, bool TREE>
constexpr size_t rows_buf_bytes() {
  using C = RowsCfg<NMAX>;
  return (size_t)(C::WB / C::GROUP) * rows_buf_entries<NMAX, rows_rmax<NMAX, TREE>()>() * 16;
}

// A child of the current tile as staged in LDS.
struct ChildInfo {
  uint32_t crow;   // byte offset of its new row among the staged rows
  uint32_t pad;
  double wc;       // its weight times the sign of its row permutation
};

// One chunk of slice t: tiles chunk, chunk + n_blk_t, ... of the method's
// table.  MODE bit 0: accumulate A(t); bit 4: weighted-row aggregation of
// each group's children (one dot per group, no per-child value).
// ARGS: the job's ContractArgs, a kernel argument or an entry of the
// batch's job table read through the constant address space (its fields
// then come by scalar loads where they are used).
template <int NMAX, bool TREE, int MODE, class ARGS>
__device__ __forceinline__ void rows_chunk(ARGS& a, int t, int chunk, double2* smem) {
  using Cfg = RowsCfg<NMAX>;
  constexpr int GROUP = Cfg::GROUP, ROWS = Cfg::ROWS, WB = Cfg::WB;
  constexpr int RMAX = rows_rmax<NMAX, TREE>();
  constexpr int RB = RMAX > 0 ? RMAX : 1;
  constexpr int SPW = kWave / GROUP;   // sinks per wave
  constexpr int kWaves = WB / kWave;
  constexpr int E = rows_buf_entries<NMAX, RMAX>();
  constexpr bool WITH_A = (MODE & 1) != 0;
  constexpr bool AGG = (MODE & 16) != 0;
  static_assert(!(AGG && WITH_A), "aggregation forms no per-child values");
  const auto& p = a.plan;
  const auto& rt = TREE ? p.rows_tree : p.rows_plain;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  const int m = lane % GROUP;      // the group's lane holding rows m, m + GROUP, ...
  const int gsel = lane / GROUP;   // which sink of the wave's block
  // LDS: pivot-row buffers | each wave's sink column offsets | the tile's
  // children (new row, weight) | the staged rows of S_t
  const int sn = p.sn;
  double2* buf = smem + (threadIdx.x / GROUP) * E;
  char* meta = reinterpret_cast<char*>(smem) + (size_t)(WB / GROUP) * E * 16;
  uint32_t* wco = reinterpret_cast<uint32_t*>(meta) + wave * SPW * sn;
  ChildInfo* chi = reinterpret_cast<ChildInfo*>(
      meta + ((size_t)kWaves * SPW * sn * 4 + 15) / 16 * 16);
  double2* rows = reinterpret_cast<double2*>(meta + rows_meta_bytes(kWaves, SPW, sn));
  const char* lds = reinterpret_cast<const char*>(rows);
  const int M = p.M;
  const uint32_t stride = (uint32_t)lds_row(M) * 16u;
  const double2* St = a.S + (size_t)t * M * M;
  const int F = p.F;
  const int n_tiles = rt.n_tiles;

  double acc_re = 0.0, acc_im = 0.0, acc_a = 0.0;
  uint32_t n_fallback = 0;

  for (int ti = chunk; ti < n_tiles; ti += a.n_blk_t) {
    const int4 tl = cload(rt.tiles, ti);
    const int u0 = tl.x, u1 = tl.y, s0 = tl.z, s1 = tl.w;
    const int r0 = cload(rt.unit_row, u0);
    const int nrows = cload(rt.unit_row, u1) - r0;
    __syncthreads();   // the previous tile is done with the rows
    {
      // four entries in flight per thread
      constexpr int U = 4;
      const int total = nrows * M;
      for (int e0 = threadIdx.x; e0 < total; e0 += U * WB) {
        double2 v[U];
        int dst[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int e = e0 + q * WB;
          v[q] = make_double2(0.0, 0.0);
          dst[q] = -1;
          if (e < total) {
            const int r = e / M, c = e - r * M;
            v[q] = St[(size_t)rt.rows[r0 + r] * M + c];
            dst[q] = r * lds_row(M) + c;
          }
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
          if (dst[q] >= 0) rows[dst[q]] = v[q];
      }
    }
    // the tile's children: byte offset of the new row in LDS and weight
    // times the sign of the row permutation
    int tc0 = 0;
    if (TREE) {
      tc0 = cload(rt.unit_c, u0).x;
      for (int u = u0 + wave; u < u1; u += kWaves) {
        const int2 uc = cload(rt.unit_c, u);
        const uint32_t ub = (uint32_t)(cload(rt.unit_row, u) - r0);
        for (int c = uc.x + lane; c < uc.y; c += kWave) {
          ChildInfo ci;
          ci.crow = (ub + (uint32_t)rt.child_lrow[c]) * stride;
          ci.pad = 0u;
          ci.wc = a.w_src[p.child_term[c]] * p.child_wsgn[c];
          chi[c - tc0] = ci;
        }
      }
    }
    __syncthreads();
    const int n_sb = (s1 - s0 + SPW - 1) / SPW;
    const int n_items = (u1 - u0) * n_sb;

    for (int item = wave; item < n_items; item += kWaves) {
      const int uu = uniform(item / n_sb);
      const int u = u0 + uu;
      const int sb = item - uu * n_sb;
      const int k = s0 + sb * SPW + gsel;
      const bool valid = k < s1;
      const int kk = valid ? k : s0;   // lanes past the range compute sink s0, masked
      const int4 ui = cload(rt.unit, u);
      const int rs = ui.x;
      const bool primary = ui.w != 0;
      const int term = TREE ? cload(p.dom_term, rs) : rs;
      const uint32_t ubase = (uint32_t)(cload(rt.unit_row, u) - r0) * stride;
      const int g_begin = TREE ? ui.y : 0;
      const int g_end = TREE ? ui.z : 0;
      int c_lo = 0, c_hi = 0;
      if (TREE) {
        const int2 uc = cload(rt.unit_c, u);
        c_lo = uc.x;
        c_hi = uc.y;
      }
      // this wave's sink column offsets: wco[q * SPW + g] for position q
      // of sink s0 + sb * SPW + g (padded sinks repeat sink s0)
      for (int e = lane; e < SPW * sn; e += kWave) {
        const int q = e / SPW, gl = e - q * SPW;
        const int k2 = s0 + sb * SPW + gl;
        wco[e] = p.snk_coloff[(size_t)q * p.n_snk_pad + (k2 < s1 ? k2 : s0)];
      }
      wave_lds_sync();

      // The group's block of flavour f: the row set's rows, row rrep
      // replaced by the LDS row at crow (a child's), columns of sink kk.
      // Rows past n read the set's first row (never pivots, multiplier 0);
      // columns past n are zero and never read.
      auto load_block = [&](int f, int rrep, uint32_t crow, RowsBlock<ROWS, NMAX, RB>& blk)
                            __attribute__((always_inline)) {
        const int o = p.off[f];
        const int n = p.off[f + 1] - o;
        const uint32_t* cof = wco + (size_t)o * SPW + gsel;
        uint32_t ra[ROWS];
#pragma unroll
        for (int s = 0; s < ROWS; ++s) {
          const int i = m + GROUP * s;
          ra[s] = (i == rrep) ? crow : ubase + (uint32_t)(o + (i < n ? i : 0)) * stride;
        }
        static_for<0, NMAX>([&](auto cc) __attribute__((always_inline)) {
          constexpr int c = decltype(cc)::value;
          if (c < n) {
            const uint32_t co = cof[c * SPW];
#pragma unroll
            for (int s = 0; s < ROWS; ++s) {
              const double2 v = *reinterpret_cast<const double2*>(lds + ra[s] + co);
              blk.ar[s][c] = v.x;
              blk.ai[s][c] = v.y;
            }
          } else {
#pragma unroll
            for (int s = 0; s < ROWS; ++s) {
              blk.ar[s][c] = 0.0;
              blk.ai[s][c] = 0.0;
            }
          }
        });
      };

      // P: product of the blocks' dets (the same in every lane of the
      // group); Q: the children's weighted dets folded over the flavours --
      // the group's value in every lane (with A) or this lane's share.
      double Pre = 1.0, Pim = 0.0, Qre = 0.0, Qim = 0.0;
      double sabs_reg = 0.0;
      bool bad = false;   // some dominator block had an exactly zero pivot

      int g = g_begin;
      for (int f = 0; f < F; ++f) {
        const int o = p.off[f];
        const int n = p.off[f + 1] - o;
        int g_f_end = g;
        if (TREE) {
          while (g_f_end < g_end && (cload(p.grp_fr, g_f_end) >> 8) == f) ++g_f_end;
        }
        const int R = g_f_end - g;
        const int npass = (TREE && R > RB) ? (R + RB - 1) / RB : 1;
        // npass eliminations of the dominator's block, each carrying up to
        // RMAX groups' unit columns.  With D = det of this block the fold
        // over flavours is Q <- D Q + (D P) sum_c w_c ratio_c, P <- D P: the
        // first elimination applies D at once, so that only P and Q stay
        // live across the eliminations.
        RowsBlock<ROWS, NMAX, RB> blk;
        load_block(f, -1, 0u, blk);
        auto set_units = [&](int g0) __attribute__((always_inline)) {
          const int nr = min(R - g0, RB);
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            const int r = q < nr ? (cload(p.grp_fr, g + g0 + q) & 0xff) : -1;
#pragma unroll
            for (int s = 0; s < ROWS; ++s) {
              blk.br[s][q] = (m + GROUP * s == r) ? 1.0 : 0.0;
              blk.bi[s][q] = 0.0;
            }
          }
        };
        if (TREE) set_units(0);
        int col[ROWS];
        PivotRows<NMAX> pivots;
        const RowsResult res =
            rows_gauss_jordan<GROUP, ROWS, NMAX, RMAX, RB, TREE>(blk, n, m, col, buf, pivots);
        {
          const double qr = Qre * res.dre - Qim * res.dim;
          Qim = Qre * res.dim + Qim * res.dre;
          Qre = qr;
          const double pr = Pre * res.dre - Pim * res.dim;
          Pim = Pre * res.dim + Pim * res.dre;
          Pre = pr;
        }
        // no inverse: the item goes the direct route below (a plain LU
        // needs none, its det is 0)
        if (res.zero) bad = true;
        if (TREE && !bad) {
          // x_q[col_i] = b'_q[i] / u_i for this lane's rows (0 for rows
          // past n); the children's rows are read at those columns
          const uint32_t* cof = wco + (size_t)o * SPW + gsel;
          double vr[ROWS], vi[ROWS];
          uint32_t mycol[ROWS];
#pragma unroll
          for (int s = 0; s < ROWS; ++s) {
            rows_pivot_inverse(buf, col[s], vr[s], vi[s]);
            mycol[s] = cof[(col[s] >= 0 ? col[s] : 0) * SPW];
          }
          // groups of this block RB at a time: the first RB rode through
          // the elimination, the others replay its row operations
          for (int pass = 0; pass < npass; ++pass) {
            const int g0 = pass * RB;
            const int nr = min(R - g0, RB);
            if (pass > 0) {
              set_units(g0);
              rows_replay<GROUP, ROWS, NMAX, RB>(blk, n, m, pivots, buf);
            }
            double sre = 0.0, sim = 0.0;   // sum_c w_c ratio_c (or this lane's share)
            static_for<0, RB>([&](auto qc) __attribute__((always_inline)) {
              constexpr int q = decltype(qc)::value;
              if (q >= nr) return;
              double xr[ROWS], xi[ROWS];
  #pragma unroll
              for (int s = 0; s < ROWS; ++s) {
                xr[s] = blk.br[s][q] * vr[s] - blk.bi[s][q] * vi[s];
                xi[s] = blk.br[s][q] * vi[s] + blk.bi[s][q] * vr[s];
              }
              const int gg = g + g0 + q;
              const int cb = max(cload(p.grp_ptr, gg), c_lo);
              const int ce = min(cload(p.grp_ptr, gg + 1), c_hi);
              if constexpr (AGG) {
                // multilinearity in row r: the children's weighted rows are
                // summed first (at this lane's columns), then dotted once
                double hr[ROWS], hi[ROWS];
  #pragma unroll
                for (int s = 0; s < ROWS; ++s) {
                  hr[s] = 0.0;
                  hi[s] = 0.0;
                }
                for (int c = cb; c < ce; ++c) {
                  const ChildInfo ci = chi[c - tc0];
                  const uint32_t cr = ci.crow;
                  const double wc = ci.wc;
                  double2 sv[ROWS];
  #pragma unroll
                  for (int s = 0; s < ROWS; ++s)
                    sv[s] = *reinterpret_cast<const double2*>(lds + cr + mycol[s]);
  #pragma unroll
                  for (int s = 0; s < ROWS; ++s) {
                    hr[s] += wc * sv[s].x;
                    hi[s] += wc * sv[s].y;
                  }
                }
  #pragma unroll
                for (int s = 0; s < ROWS; ++s) {
                  sre += hr[s] * xr[s] - hi[s] * xi[s];
                  sim += hr[s] * xi[s] + hi[s] * xr[s];
                }
                return;
              }
              for (int c = cb; c < ce; ++c) {
                const ChildInfo ci = chi[c - tc0];
                const uint32_t cr = ci.crow;
                const double wc = ci.wc;
                double2 sv[ROWS];
  #pragma unroll
                for (int s = 0; s < ROWS; ++s)
                  sv[s] = *reinterpret_cast<const double2*>(lds + cr + mycol[s]);
                double pr_ = 0.0, pi_ = 0.0;
  #pragma unroll
                for (int s = 0; s < ROWS; ++s) {
                  pr_ += sv[s].x * xr[s] - sv[s].y * xi[s];
                  pi_ += sv[s].x * xi[s] + sv[s].y * xr[s];
                }
                if constexpr (WITH_A) {
                  const double rr = group_sum<GROUP>(pr_);
                  const double ri = group_sum<GROUP>(pi_);
                  sre += wc * rr;
                  sim += wc * ri;
                  sabs_reg += fabs(wc) * cabs_scaled(rr, ri);
                } else {
                  sre += wc * pr_;
                  sim += wc * pi_;
                }
              }
            });
            Qre += Pre * sre - Pim * sim;
            Qim += Pre * sim + Pim * sre;
          }
        }
        g = g_f_end;
      }

      const double wi = cload(a.w_src, term);
      const double wd = primary ? wi : 0.0;
      const double wk = valid ? a.w_snk[kk] : 0.0;
      if (TREE) bad = bad && (g_end > g_begin);   // no children: nothing to redo
      if (!bad) {
        if (valid) {
          if (m == 0) {
            acc_re += wk * (wd * Pre + (WITH_A ? Qre : 0.0));
            acc_im += wk * (wd * Pim + (WITH_A ? Qim : 0.0));
          }
          if (!WITH_A) {
            acc_re += wk * Qre;
            acc_im += wk * Qim;
          }
          if (WITH_A && m == 0)
            acc_a += fabs(wk) * (fabs(wd) + sabs_reg) * cabs_scaled(Pre, Pim);
        }
      } else if (TREE) {
        // Direct route (a dominator block without an inverse; rare): every
        // child's determinant is the product of its own blocks, its changed
        // block eliminated with its row in place, signed by its row
        // permutation.
        double Ure = wd * Pre, Uim = wd * Pim;
        double uab = fabs(wd) * cabs_scaled(Pre, Pim);
        int gq = g_begin;
        const int cb = max(cload(p.grp_ptr, g_begin), c_lo);
        const int ce = min(cload(p.grp_ptr, g_end), c_hi);
        for (int c = cb; c < ce; ++c) {
          while (cload(p.grp_ptr, gq + 1) <= c) ++gq;
          const int fc = cload(p.grp_fr, gq) >> 8;
          const int rc = cload(p.grp_fr, gq) & 0xff;
          const uint32_t crow = ubase + (uint32_t)cload(rt.child_lrow, c) * stride;
          double dr = cload(p.child_wsgn, c), di = 0.0;
          for (int f = 0; f < F; ++f) {
            RowsBlock<ROWS, NMAX, RB> blk;
            load_block(f, f == fc ? rc : -1, crow, blk);
            int col[ROWS];
            PivotRows<NMAX> pivots;
            const RowsResult res = rows_gauss_jordan<GROUP, ROWS, NMAX, 0, RB>(
                blk, p.off[f + 1] - p.off[f], m, col, buf, pivots);
            const double tr = dr * res.dre - di * res.dim;
            di = dr * res.dim + di * res.dre;
            dr = tr;
          }
          const double wc = cload(a.w_src, cload(p.child_term, c));
          Ure += wc * dr;
          Uim += wc * di;
          if (WITH_A) uab += fabs(wc) * cabs_scaled(dr, di);
          if (m == 0 && valid) ++n_fallback;
        }
        if (valid && m == 0) {
          acc_re += wk * Ure;
          acc_im += wk * Uim;
          if (WITH_A) acc_a += fabs(wk) * uab;
        }
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

template <int NMAX, bool TREE, int MODE>
__global__ __launch_bounds__(RowsCfg<NMAX>::WB) void contract_rows_kernel(ContractArgs a) {
  extern __shared__ double2 smem[];
  rows_chunk<NMAX, TREE, MODE>(a, blockIdx.y, blockIdx.x, smem);
}

template <int NMAX, bool TREE, int MODE>
__global__ __launch_bounds__(RowsCfg<NMAX>::WB) void batch_rows_kernel(BatchArgs b) {
  extern __shared__ double2 smem[];
  for (int i = blockIdx.x; i < b.n_tiles; i += gridDim.x) {
    const int4 tl = cload(b.tiles, i);
    const __attribute__((address_space(4))) ContractArgs& a =
        ((const __attribute__((address_space(4))) ContractArgs*)b.jobs)[tl.x];
    rows_chunk<NMAX, TREE, MODE>(a, tl.y, tl.z, smem);
  }
}

template <int NMAX, bool TREE, int MODE>
hipError_t rows_launch_one(const ContractArgs& a, size_t lds_rows, hipStream_t s) {
  constexpr int WB = RowsCfg<NMAX>::WB;
  const size_t lds = rows_buf_bytes<NMAX, TREE>() + lds_rows;
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&contract_rows_kernel<NMAX, TREE, MODE>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((contract_rows_kernel<NMAX, TREE, MODE>), dim3(a.n_blk_t, a.T), dim3(WB),
                     lds, s, a);
  return hipGetLastError();
}

template <int NMAX>
hipError_t rows_launch_n(const ContractArgs& a, bool tree, bool with_a, bool agg, size_t lds_rows,
                         hipStream_t s) {
  if (!tree) return with_a ? rows_launch_one<NMAX, false, 1>(a, lds_rows, s)
                           : rows_launch_one<NMAX, false, 0>(a, lds_rows, s);
  if (agg) return rows_launch_one<NMAX, true, 16>(a, lds_rows, s);
  return with_a ? rows_launch_one<NMAX, true, 1>(a, lds_rows, s)
                : rows_launch_one<NMAX, true, 0>(a, lds_rows, s);
}

template <int NMAX, bool TREE, int MODE>
hipError_t rows_batch_one(const BatchArgs& b, int grid, size_t lds_rows, hipStream_t s) {
  constexpr int WB = RowsCfg<NMAX>::WB;
  const size_t lds = rows_buf_bytes<NMAX, TREE>() + lds_rows;
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&batch_rows_kernel<NMAX, TREE, MODE>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_rows_kernel<NMAX, TREE, MODE>), dim3(grid), dim3(WB), lds, s, b);
  return hipGetLastError();
}

template <int NMAX>
hipError_t rows_batch_n(const BatchArgs& b, bool tree, bool with_a, int grid, size_t lds_rows,
                        hipStream_t s) {
  if (tree) return with_a ? rows_batch_one<NMAX, true, 1>(b, grid, lds_rows, s)
                          : rows_batch_one<NMAX, true, 0>(b, grid, lds_rows, s);
  return with_a ? rows_batch_one<NMAX, false, 1>(b, grid, lds_rows, s)
                : rows_batch_one<NMAX, false, 0>(b, grid, lds_rows, s);
}

template <int NMAX, bool TREE, int MODE>
int rows_resident_one(size_t lds_rows) {
  int nb = 0;
  const size_t lds = rows_buf_bytes<NMAX, TREE>() + lds_rows;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, reinterpret_cast<const void*>(&batch_rows_kernel<NMAX, TREE, MODE>),
          RowsCfg<NMAX>::WB, lds) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

// Entry points of one bucket, defined in its own translation unit.
#define MHC_ROWS_BUCKET(NMAX)                                                                  \
  hipError_t launch_contract_rows_b##NMAX(const ContractArgs& a, bool tree, bool with_a,      \
                                          bool agg, size_t lds_rows, hipStream_t s) {         \
    return rows_launch_n<NMAX>(a, tree, with_a, agg, lds_rows, s);                            \
  }                                                                                           \
  hipError_t launch_batch_rows_b##NMAX(const BatchArgs& b, bool tree, bool with_a, int grid,  \
                                       size_t lds_rows, hipStream_t s) {                      \
    return rows_batch_n<NMAX>(b, tree, with_a, grid, lds_rows, s);                            \
  }                                                                                           \
  int batch_rows_resident_b##NMAX(bool tree, bool with_a, size_t lds_rows) {                  \
    if (tree) return with_a ? rows_resident_one<NMAX, true, 1>(lds_rows)                      \
                            : rows_resident_one<NMAX, true, 0>(lds_rows);                     \
    return with_a ? rows_resident_one<NMAX, false, 1>(lds_rows)                               \
                  : rows_resident_one<NMAX, false, 0>(lds_rows);                              \
  }                                                                                           \
  RowsGeometry rows_geometry_b##NMAX(bool tree) {                                             \
    using C = RowsCfg<NMAX>;                                                                  \
    return RowsGeometry{kWave / C::GROUP, C::WB / kWave,                                      \
                        tree ? rows_buf_bytes<NMAX, true>() : rows_buf_bytes<NMAX, false>()}; \
  }

}  // namespace kern
}  // namespace mhc
