// Contraction kernels for flavour blocks up to 16 with several rows of a
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
  static constexpr int GROUP = 4, ROWS = 2, RMAX = 6, WB = 768;
};
template <>
struct RowsCfg<12> {
  static constexpr int GROUP = 4, ROWS = 3, RMAX = 4, WB = 512;
};
template <>
struct RowsCfg<16> {
  static constexpr int GROUP = 8, ROWS = 2, RMAX = 4, WB = 512;
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

// One chunk of slice t: tiles chunk, chunk + n_blk_t, ... of the method's
// table.  MODE bit 0: accumulate A(t); bit 4: weighted-row aggregation of
// each group's children (one dot per group, no per-child value).
template <int NMAX, bool TREE, int MODE>
__device__ __forceinline__ void rows_chunk(const ContractArgs& a, int t, int chunk,
                                           double2* smem) {
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
  const PlanView& p = a.plan;
  const RowsTable& rt = TREE ? p.rows_tree : p.rows_plain;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  const int m = lane % GROUP;      // the group's lane holding rows m, m + GROUP, ...
  const int gsel = lane / GROUP;   // which sink of the wave's block
  double2* buf = smem + (threadIdx.x / GROUP) * E;
  double2* rows = smem + (WB / GROUP) * E;
  const char* lds = reinterpret_cast<const char*>(rows);
  const int M = p.M;
  const uint32_t stride = (uint32_t)lds_row(M) * 16u;
  const double2* St = a.S + (size_t)t * M * M;
  const int F = p.F;

  double acc_re = 0.0, acc_im = 0.0, acc_a = 0.0;
  uint32_t n_fallback = 0;

  for (int ti = chunk; ti < rt.n_tiles; ti += a.n_blk_t) {
    const int u0 = uniform(rt.tiles[ti].x), u1 = uniform(rt.tiles[ti].y);
    const int s0 = uniform(rt.tiles[ti].z), s1 = uniform(rt.tiles[ti].w);
    const int r0 = uniform(rt.unit_row[u0]);
    const int nrows = uniform(rt.unit_row[u1]) - r0;
    __syncthreads();   // the previous tile is done with the rows
    for (int e = threadIdx.x; e < nrows * M; e += WB) {
      const int r = e / M, c = e - r * M;
      rows[r * lds_row(M) + c] = St[(size_t)rt.rows[r0 + r] * M + c];
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
      const int4 ui = rt.unit[u];
      const int rs = uniform(ui.x);
      const bool primary = uniform(ui.w) != 0;
      const int term = TREE ? uniform(p.dom_term[rs]) : rs;
      const uint32_t ubase = (uint32_t)(uniform(rt.unit_row[u]) - r0) * stride;
      const int g_begin = TREE ? uniform(ui.y) : 0;
      const int g_end = TREE ? uniform(ui.z) : 0;
      const int c_lo = TREE ? uniform(rt.unit_c[u].x) : 0;
      const int c_hi = TREE ? uniform(rt.unit_c[u].y) : 0;

      // The group's block of flavour f: the row set's rows, row rrep
      // replaced by the LDS row at crow (a child's), columns of sink kk.
      auto load_block = [&](int f, int rrep, uint32_t crow, RowsBlock<ROWS, NMAX, RB>& blk) {
        const int o = p.off[f];
        const int n = p.off[f + 1] - o;
        const uint32_t* cof = p.snk_coloff + (size_t)o * p.n_snk_pad + kk;
        uint32_t co[NMAX];
#pragma unroll
        for (int c = 0; c < NMAX; ++c) co[c] = c < n ? cof[(size_t)c * p.n_snk_pad] : 0u;
#pragma unroll
        for (int s = 0; s < ROWS; ++s) {
          const int i = m + GROUP * s;
          const uint32_t ra = (i == rrep) ? crow : ubase + (uint32_t)(o + i) * stride;
#pragma unroll
          for (int c = 0; c < NMAX; ++c) {
            blk.ar[s][c] = 0.0;
            blk.ai[s][c] = 0.0;
            if (c < n && i < n) {
              const double2 v = *reinterpret_cast<const double2*>(lds + ra + co[c]);
              blk.ar[s][c] = v.x;
              blk.ai[s][c] = v.y;
            }
          }
        }
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
          while (g_f_end < g_end && uniform(p.grp_fr[g_f_end] >> 8) == f) ++g_f_end;
        }
        const int R = g_f_end - g;
        const int npass = (TREE && R > RB) ? (R + RB - 1) / RB : 1;
        // npass eliminations of the dominator's block, each carrying up to
        // RMAX groups' unit columns.  With D = det of this block the fold
        // over flavours is Q <- D Q + (D P) sum_c w_c ratio_c, P <- D P: the
        // first elimination applies D at once, so that only P and Q stay
        // live across the eliminations.
        for (int pass = 0; pass < npass; ++pass) {
          const int g0 = pass * RB;
          const int nr = TREE ? min(R - g0, RB) : 0;
          RowsBlock<ROWS, NMAX, RB> blk;
          load_block(f, -1, 0u, blk);
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            const int r = q < nr ? uniform(p.grp_fr[g + g0 + q] & 0xff) : -1;
#pragma unroll
            for (int s = 0; s < ROWS; ++s) {
              blk.br[s][q] = (m + GROUP * s == r) ? 1.0 : 0.0;
              blk.bi[s][q] = 0.0;
            }
          }
          int col[ROWS];
          const RowsResult res =
              rows_gauss_jordan<GROUP, ROWS, NMAX, RMAX, RB>(blk, nr, n, m, col, buf);
          if (pass == 0) {
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
          if (!TREE || bad) continue;
          // x_q[col_i] = b'_q[i] / u_i for this lane's rows; the children's
          // rows are read at those columns
          const uint32_t* cof = p.snk_coloff + (size_t)o * p.n_snk_pad + kk;
          double vr[ROWS], vi[ROWS];
          uint32_t mycol[ROWS];
#pragma unroll
          for (int s = 0; s < ROWS; ++s) {
            rows_pivot_inverse(buf, col[s], vr[s], vi[s]);
            mycol[s] = col[s] >= 0 ? cof[(size_t)col[s] * p.n_snk_pad] : 0u;
          }
          double sre = 0.0, sim = 0.0;   // sum_c w_c ratio_c (or this lane's share)
          static_for<0, RB>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            if (q >= nr) return;
            double xr[ROWS], xi[ROWS];
#pragma unroll
            for (int s = 0; s < ROWS; ++s) {
              xr[s] = blk.br[s][q] * vr[s] - blk.bi[s][q] * vi[s];
              xi[s] = blk.br[s][q] * vi[s] + blk.bi[s][q] * vr[s];
            }
            const int gg = g + g0 + q;
            const int cb = max(uniform(p.grp_ptr[gg]), c_lo);
            const int ce = min(uniform(p.grp_ptr[gg + 1]), c_hi);
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
                const uint32_t cr = ubase + (uint32_t)uniform(rt.child_lrow[c]) * stride;
                const double wc = a.w_src[uniform(p.child_term[c])] * p.child_wsgn[c];
#pragma unroll
                for (int s = 0; s < ROWS; ++s) {
                  if (col[s] >= 0) {
                    const double2 sv = *reinterpret_cast<const double2*>(lds + cr + mycol[s]);
                    hr[s] += wc * sv.x;
                    hi[s] += wc * sv.y;
                  }
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
              const uint32_t cr = ubase + (uint32_t)uniform(rt.child_lrow[c]) * stride;
              const double wc = a.w_src[uniform(p.child_term[c])] * p.child_wsgn[c];
              double pr_ = 0.0, pi_ = 0.0;
#pragma unroll
              for (int s = 0; s < ROWS; ++s) {
                if (col[s] >= 0) {
                  const double2 sv = *reinterpret_cast<const double2*>(lds + cr + mycol[s]);
                  pr_ += sv.x * xr[s] - sv.y * xi[s];
                  pi_ += sv.x * xi[s] + sv.y * xr[s];
                }
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
        g = g_f_end;
      }

      const double wi = a.w_src[term];
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
        const int cb = max(uniform(p.grp_ptr[g_begin]), c_lo);
        const int ce = min(uniform(p.grp_ptr[g_end]), c_hi);
        for (int c = cb; c < ce; ++c) {
          while (uniform(p.grp_ptr[gq + 1]) <= c) ++gq;
          const int fc = uniform(p.grp_fr[gq] >> 8);
          const int rc = uniform(p.grp_fr[gq] & 0xff);
          const uint32_t crow = ubase + (uint32_t)uniform(rt.child_lrow[c]) * stride;
          double dr = p.child_wsgn[c], di = 0.0;
          for (int f = 0; f < F; ++f) {
            RowsBlock<ROWS, NMAX, RB> blk;
            load_block(f, f == fc ? rc : -1, crow, blk);
            int col[ROWS];
            const RowsResult res = rows_gauss_jordan<GROUP, ROWS, NMAX, 0, RB>(
                blk, 0, p.off[f + 1] - p.off[f], m, col, buf);
            const double tr = dr * res.dre - di * res.dim;
            di = dr * res.dim + di * res.dre;
            dr = tr;
          }
          const double wc = a.w_src[uniform(p.child_term[c])];
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
    const int4 tl = b.tiles[i];
    rows_chunk<NMAX, TREE, MODE>(b.jobs[tl.x], tl.y, tl.z, smem);
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
