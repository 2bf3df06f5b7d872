// Two-sided update trees (gfx950): source and sink terms both in dominating
// sets, one pivoted LU per (source dominator, sink dominator, flavour).
//
// The paper's graph links matrices that differ in a single row or column
// (Sec. 3) but builds it over source terms only; here the sink terms get
// their own tree as well.  With G the dominators' block, x_r = G^-1 e_r and
// y_c = e_c^T G^-1, the pairs of one (source partition, sink partition)
// have the determinant ratios (matrix determinant lemma, Sec. 2)
//   source child (row r -> new row s):      rho   = s . x_r
//   sink child (column c -> new column v):  sigma = y_c . v
//   both, in different flavour blocks:      rho * sigma
//   both, in the same block:                tau = rho * sigma - kappa (beta - alpha)
// where kappa = (G^-1)[c][r], beta = s^T G^-1 v and alpha = S[new row][new
// column]; tau is the rank-2 form of the lemma (det(I + V^T G^-1 U) for the
// two changes).  The weighted sum of every pair of the two partitions is
//   prod_f det G_f * ((w_a + sum_c w_c rho_c) (w_b + sum_d w_d sigma_d)
//                     - sum over same-block (c, d) of w_c w_d kappa (beta - alpha)).
//
// Work decomposition: a wave holds one source dominator (wave-uniform
// source tree, as in the one-sided kernel) and 64 sink dominators, one per
// lane, each with its own sink groups and children (per-lane loops; the
// sink dominators are sorted so that neighbouring lanes have similar
// counts).  Per flavour: the source groups and children first (x_r, rho_c);
// then each lane walks its sink groups (y_c) and children (sigma_d) once,
// and where the source dominator has children in the block, solves
// q_d = G^-1 v_d and runs the wave-uniform source loops for the pair terms
// beta - alpha = s_c . q_d - alpha.
//
// A lane whose dominator block has an exactly zero pivot evaluates every
// pair of its two partitions by direct LU instead (counted in the plan's
// fallback counter).

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contract_kernels.h"
#include "group_device.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

// x' = U^-1 L^-1 v in place from the factors of lu_crout<N, true> (G Q =
// L U, diagonal holding 1/U_mm): G^-1 v = Q x', so entry m of x' belongs
// to the factors' column position m.
template <int N>
__device__ __forceinline__ void solve_col(const double (&gr)[N][N], const double (&gi)[N][N],
                                          double (&vr)[N], double (&vi)[N]) {
#pragma unroll
  for (int m = 1; m < N; ++m) {
#pragma unroll
    for (int j = 0; j < m; ++j) {
      vr[m] = vr[m] - gr[m][j] * vr[j] + gi[m][j] * vi[j];
      vi[m] = vi[m] - gr[m][j] * vi[j] - gi[m][j] * vr[j];
    }
  }
#pragma unroll
  for (int m = N - 1; m >= 0; --m) {
    double tr = vr[m], ti = vi[m];
#pragma unroll
    for (int j = m + 1; j < N; ++j) {
      tr = tr - gr[m][j] * vr[j] + gi[m][j] * vi[j];
      ti = ti - gr[m][j] * vi[j] - gi[m][j] * vr[j];
    }
    vr[m] = tr * gr[m][m] - ti * gi[m][m];
    vi[m] = tr * gi[m][m] + ti * gr[m][m];
  }
}

// det of one flavour block with source row r replaced by `newrow` (r < 0:
// none) and sink column c replaced by `newcol` (c < 0: none), by direct LU.
template <int N>
__device__ __forceinline__ void block_det2(const char* lds, const uint32_t* rowoff, int r,
                                           uint32_t newrow, const uint32_t (&co)[N], int c,
                                           uint32_t newcol, double& dre, double& dim) {
  uint32_t ro[N], cl[N];
#pragma unroll
  for (int m = 0; m < N; ++m) ro[m] = (m == r) ? newrow : rowoff[m];
#pragma unroll
  for (int m = 0; m < N; ++m) cl[m] = (m == c) ? newcol : co[m];
  double gr[N][N], gi[N][N];
  int perm[N];
  bool z;
  gather<N>(lds, ro, cl, gr, gi);
  lu<N, false>(gr, gi, dre, dim, perm, z);
}

static_assert(kTwoSidedSlotBytes == (size_t)kBlock * 4 * 16, "one slot per thread");

// A thread's running sums (four complex numbers): in its LDS slot (PARK),
// or in registers where the LDS has no room for the slots.
template <bool PARK>
struct RunningSums {
  double2* slot;
  __device__ double2 get(int i) const { return slot[i]; }
  __device__ void set(int i, double2 v) { slot[i] = v; }
};
template <>
struct RunningSums<false> {
  double2 r[4];
  __device__ double2 get(int i) const { return r[i]; }
  __device__ void set(int i, double2 v) { r[i] = v; }
};

// A wave-uniform double moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double x) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                          __builtin_amdgcn_readfirstlane(__double2loint(x)));
}

// Per (slice, chunk): whether a lane of the chunk met a block with an
// exactly zero pivot; ints after the workgroup partials.
__device__ __forceinline__ int* two_sided_flags(const ContractArgs& a) {
  return reinterpret_cast<int*>(a.partial + (size_t)a.T * a.n_blk_t * 3);
}

template <int N, bool TAB, bool PARK>
__device__ __forceinline__ void two_sided_tile(const ContractArgs& a, int t, int chunk,
                                               double2* smem) {
  const PlanView& p = a.plan;
  const SinkTreeView& q = a.snk;
  __syncthreads();  // the previous tile of this workgroup is done with LDS
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  const int MM = p.M * p.M;
  const double2* St = a.S + (size_t)t * MM;
  stage_slice(St, smem, p.M, kBlock);
  __syncthreads();
  const char* lds = reinterpret_cast<const char*>(smem);

  // Each lane's running sums over the blocks of an item live in LDS between
  // the blocks (PARK: a slot of four complex numbers per thread, after the
  // slice and the tables), so that no register holds them through a
  // factorisation: 0 the product of the block dets, 1 sum_c w_c rho_c,
  // 2 sum_d w_d sigma_d, 3 the same-block pair sum.
  RunningSums<PARK> sums;
  if constexpr (PARK)
    sums.slot = reinterpret_cast<double2*>(reinterpret_cast<char*>(smem) + lds_slice_bytes(p.M) +
                                           (size_t)kWavesPerBlock * a.tab_rows * p.M * 16) +
                (size_t)threadIdx.x * 4;
  double acc_re = 0.0, acc_im = 0.0;  // the wave's total over its items
  bool any_bad = false;  // wave-uniform
  const int F = p.F;
  const int sn = p.sn;
  const int pad = q.n_sdom_pad;

  for (int item = chunk + a.n_blk_t * wave; item < a.n_items;
       item += a.n_blk_t * kWavesPerBlock) {
    const int d = uniform(item / a.n_sblk);
    const int sb = uniform(item - d * a.n_sblk);
    const int k = sb * kWave + lane;
    const bool valid = k < q.n_sdom;
    const int term_a = cload(p.dom_term, d);
    const double wa = cload(a.w_src, term_a);
    const uint32_t* rowoff_d = p.dom_rowoff + (size_t)d * sn;
    const int g_begin = cload(p.dom_grp, d);
    const int g_end = cload(p.dom_grp, d + 1);

    // TAB: row l of this wave's table holds A_g = sum_c w_c S[new row of
    // c][:] for group g = g_begin + l (the source dominator's groups); the
    // previous item's rows were read by this wave only, in program order
    char* tab = reinterpret_cast<char*>(smem) + lds_slice_bytes(p.M) +
                (size_t)wave * a.tab_rows * p.M * 16;
    if (TAB) {
      for (int gg = g_begin; gg < g_end; ++gg) {
        const int c0 = cload(p.grp_ptr, gg), c1 = cload(p.grp_ptr, gg + 1);
        for (int col = lane; col < p.M; col += kWave) {
          double xr = 0.0, xi = 0.0;
          for (int c = c0; c < c1; ++c) {
            const uint32_t crow = cload(p.child_rowoff, c);
            const double wc = cload(a.w_src, cload(p.child_term, c));
            const double2 v = *reinterpret_cast<const double2*>(lds + crow + col * 16);
            xr += wc * v.x;
            xi += wc * v.y;
          }
          *reinterpret_cast<double2*>(tab + ((size_t)(gg - g_begin) * p.M + col) * 16) =
              make_double2(xr, xi);
        }
      }
      wave_lds_sync();
    }

    bool bad = false;
    int g = g_begin;
    for (int f = 0; f < F; ++f) {
      const int o = p.off[f];
      uint32_t co[N], ro[N];
#pragma unroll
      for (int c = 0; c < N; ++c) co[c] = q.sdom_coloff[(size_t)(o + c) * pad + k];
#pragma unroll
      for (int m = 0; m < N; ++m) ro[m] = cload(rowoff_d, o + m);
      // the block transposed (A = G^T, rows = the sink dominator's columns),
      // P A = L U, then V = U^-1 L^-1 in place: G^-1[perm[j]][i] = V[i][j],
      // so x_r = G^-1 e_r is row r of V with entry j at column pcol[j]
      double vr[N][N], vi[N][N];
      // the column offsets ride along with the rows of A: pcol[j] is the
      // offset of column perm[j]
      int pcol[N];
      {
        double dre, dim;
        bool zero;
        gather<N>(lds, co, ro, vr, vi);  // offsets add: vr[j][i] = G[i][j]
#pragma unroll
        for (int j = 0; j < N; ++j) pcol[j] = (int)co[j];
        lu<N, true, true, false, true>(vr, vi, dre, dim, pcol, zero);
        lu_inverse_v<N>(vr, vi);
        bad = bad || zero;
        // the first block sets the sums, the others add to them
        const double2 P = f == 0 ? make_double2(1.0, 0.0) : sums.get(0);
        sums.set(0, make_double2(P.x * dre - P.y * dim, P.x * dim + P.y * dre));
      }
      // the source groups of flavour f (wave-uniform): sum_c w_c rho_c =
      // sigma . x_r with sigma = sum_c w_c s_c, s_c the child's new row
      int g_f_end = g;
      while (g_f_end < g_end && (cload(p.grp_fr, g_f_end) >> 8) == f) ++g_f_end;
      double Rre = 0.0, Rim = 0.0;     // this block's sum_c w_c rho_c
      for (int gg = g; gg < g_f_end; ++gg) {
        const int r = cload(p.grp_fr, gg) & 0xff;
        double sr[N], si[N];
        if (TAB) {
          const char* arow = tab + (size_t)(gg - g_begin) * p.M * 16;
#pragma unroll
          for (int j = 0; j < N; ++j) {
            const double2 sv = *reinterpret_cast<const double2*>(arow + pcol[j]);
            sr[j] = sv.x;
            si[j] = sv.y;
          }
        } else {
#pragma unroll
          for (int j = 0; j < N; ++j) {
            sr[j] = 0.0;
            si[j] = 0.0;
          }
          for (int c = cload(p.grp_ptr, gg); c < cload(p.grp_ptr, gg + 1); ++c) {
            const uint32_t crow = cload(p.child_rowoff, c);
            const double wc = cload(a.w_src, cload(p.child_term, c));
#pragma unroll
            for (int j = 0; j < N; ++j) {
              const double2 sv = *reinterpret_cast<const double2*>(lds + crow + pcol[j]);
              sr[j] += wc * sv.x;
              si[j] += wc * sv.y;
            }
          }
        }
#pragma unroll
        for (int rr = 0; rr < N; ++rr)
          if (rr == r) {
#pragma unroll
            for (int j = 0; j < N; ++j) {
              Rre = Rre + sr[j] * vr[rr][j] - si[j] * vi[rr][j];
              Rim = Rim + sr[j] * vi[rr][j] + si[j] * vr[rr][j];
            }
          }
      }
      // this lane's sink groups in flavour f (column cc -> new column v_d):
      // with p = G^-1 v_d (p[j] its entry perm[j]), sigma_d = y_cc . v_d =
      // p at perm[j] == cc, the position whose column offset pcol[j] is
      // cc's; where the source dominator has children in
      // this block, the same-block pairs take kappa = G^-1[cc][r] and
      // beta - alpha = s_c . p - S[new row][new column]
      {
        const double2 R = f == 0 ? make_double2(0.0, 0.0) : sums.get(1);
        sums.set(1, make_double2(R.x + Rre, R.y + Rim));
      }
      const bool src_kids = g_f_end > g;
      double Sre = 0.0, Sim = 0.0;     // this block's sum_d w_d sigma_d
      double Kre = 0.0, Kim = 0.0;     // and same-block pair sum
      // the sink children of flavour f, one record per step for every lane
      // (coalesced; padding records weigh 0 and match no column): pcol[j]
      // == ccol marks the position of the column the child replaces
      const int nrec = cload(q.srec_cnt, f * a.n_sblk + sb);
      const SinkRec* rec = a.srec + (size_t)q.srec_base[f] * pad + k;
      for (int i_rec = 0; i_rec < nrec; ++i_rec) {
        {
          const SinkRec rc = rec[(size_t)i_rec * pad];
          const uint32_t col = rc.col, ccol = rc.ccol;
          const double wd = rc.w;
          double tr[N], ti[N];
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const double2 v = *reinterpret_cast<const double2*>(lds + ro[i] + col);
            tr[i] = v.x;
            ti[i] = v.y;
          }
          double pr[N], pi[N];
#pragma unroll
          for (int j = 0; j < N; ++j) {
            double xr = 0.0, xi = 0.0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
              xr = xr + vr[i][j] * tr[i] - vi[i][j] * ti[i];
              xi = xi + vr[i][j] * ti[i] + vi[i][j] * tr[i];
            }
            pr[j] = xr;
            pi[j] = xi;
          }
          double sr = 0.0, si = 0.0;
#pragma unroll
          for (int j = 0; j < N; ++j)
            if ((uint32_t)pcol[j] == ccol) {
              sr = pr[j];
              si = pi[j];
            }
          Sre += wd * sr;
          Sim += wd * si;
          if (!src_kids) continue;
          double tre = 0.0, tim = 0.0;
          for (int gg = g; gg < g_f_end; ++gg) {
            const int r = cload(p.grp_fr, gg) & 0xff;
            double kr = 0.0, ki = 0.0;
#pragma unroll
            for (int rr = 0; rr < N; ++rr)
              if (rr == r) {
#pragma unroll
                for (int j = 0; j < N; ++j)
                  if ((uint32_t)pcol[j] == ccol) {
                    kr = vr[rr][j];
                    ki = vi[rr][j];
                  }
              }
            double ure = 0.0, uim = 0.0;
            if (TAB) {
              // sum_c w_c (s_c . p - S[new row][new column]) = A_g . p - A_g[col]
              const char* arow = tab + (size_t)(gg - g_begin) * p.M * 16;
              const double2 al = *reinterpret_cast<const double2*>(arow + col);
              ure = -al.x;
              uim = -al.y;
#pragma unroll
              for (int j = 0; j < N; ++j) {
                const double2 sv = *reinterpret_cast<const double2*>(arow + pcol[j]);
                ure = ure + sv.x * pr[j] - sv.y * pi[j];
                uim = uim + sv.x * pi[j] + sv.y * pr[j];
              }
            } else {
              for (int c = cload(p.grp_ptr, gg); c < cload(p.grp_ptr, gg + 1); ++c) {
                const uint32_t crow = cload(p.child_rowoff, c);
                const double wc = cload(a.w_src, cload(p.child_term, c));
                const double2 al = *reinterpret_cast<const double2*>(lds + crow + col);
                double bre = -al.x, bim = -al.y;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                  const double2 sv = *reinterpret_cast<const double2*>(lds + crow + pcol[j]);
                  bre = bre + sv.x * pr[j] - sv.y * pi[j];
                  bim = bim + sv.x * pi[j] + sv.y * pr[j];
                }
                ure += wc * bre;
                uim += wc * bim;
              }
            }
            tre = tre + kr * ure - ki * uim;
            tim = tim + kr * uim + ki * ure;
          }
          Kre += wd * tre;
          Kim += wd * tim;
        }
      }
      {
        const double2 S2 = f == 0 ? make_double2(0.0, 0.0) : sums.get(2);
        const double2 K2 = f == 0 ? make_double2(0.0, 0.0) : sums.get(3);
        sums.set(2, make_double2(S2.x + Sre, S2.y + Sim));
        sums.set(3, make_double2(K2.x + Kre, K2.y + Kim));
      }
      g = g_f_end;
    }

    // the sink dominator's weight, read here so that it is not held
    // through the blocks
    int kk = k;
    asm volatile("" : "+v"(kk));
    const double wb = valid ? a.w_snk[q.sdom_term[kk]] : 0.0;
    {
      const double2 P = sums.get(0), R = sums.get(1), S2 = sums.get(2), K2 = sums.get(3);
      const double ar_ = wa + R.x, ai_ = R.y;
      const double br_ = wb + S2.x, bi_ = S2.y;
      const double mr = ar_ * br_ - ai_ * bi_ - K2.x;
      const double mi = ar_ * bi_ + ai_ * br_ - K2.y;
      // a lane whose dominators have a block with an exactly zero pivot
      // adds nothing here: two_sided_pairs_tile takes its pairs
      const bool use = valid && !bad;
      const double vre = use ? P.x * mr - P.y * mi : 0.0;
      const double vim = use ? P.x * mi + P.y * mr : 0.0;
      // the wave's item total, accumulated in scalar registers
      acc_re = uniform_f64(acc_re + uniform_f64(wave_sum(vre)));
      acc_im = uniform_f64(acc_im + uniform_f64(wave_sum(vim)));
    }
    any_bad = any_bad || __builtin_amdgcn_ballot_w64(valid && bad) != 0;
  }

  __shared__ double red[kWavesPerBlock][2];
  __shared__ int bad_w[kWavesPerBlock];
  if (lane == 0) {
    red[wave][0] = acc_re;
    red[wave][1] = acc_im;
    bad_w[wave] = any_bad ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double v = 0.0;
    if (threadIdx.x < 2) {
#pragma unroll
      for (int w = 0; w < kWavesPerBlock; ++w) v += red[w][threadIdx.x];
    }
    a.partial[((size_t)t * a.n_blk_t + chunk) * 3 + threadIdx.x] = v;
  }
  if (threadIdx.x == 0) {
    int any = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) any |= bad_w[w];
    two_sided_flags(a)[(size_t)t * a.n_blk_t + chunk] = any;
  }
}

// The lanes of two_sided_tile whose (source dominator, sink dominator)
// blocks include one with an exactly zero pivot (no inverse, so no update
// formula): the same chunk of items, for the workgroups that flagged one;
// each lane refactorises its blocks as two_sided_tile did (same code, same
// operands, so the same lanes find the zero pivot) and evaluates every pair
// of the two partitions by direct LU, counted in the plan's fallback
// counter.  The sums are added to that workgroup's partials.
template <int N>
__device__ __forceinline__ void two_sided_pairs_tile(const ContractArgs& a, int t, int chunk,
                                                     double2* smem) {
  const PlanView& p = a.plan;
  const SinkTreeView& q = a.snk;
  if (two_sided_flags(a)[(size_t)t * a.n_blk_t + chunk] == 0) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  stage_slice(a.S + (size_t)t * p.M * p.M, smem, p.M, kBlock);
  __syncthreads();
  const char* lds = reinterpret_cast<const char*>(smem);
  double acc_re = 0.0, acc_im = 0.0;
  uint32_t n_fallback = 0;
  const int F = p.F;
  const int pad = q.n_sdom_pad;
  for (int item = chunk + a.n_blk_t * wave; item < a.n_items;
       item += a.n_blk_t * kWavesPerBlock) {
    const int d = uniform(item / a.n_sblk);
    const int sb = uniform(item - d * a.n_sblk);
    const int k = sb * kWave + lane;
    const bool valid = k < q.n_sdom;
    const uint32_t* rowoff_d = p.dom_rowoff + (size_t)d * p.sn;
    bool bad = false;
    for (int f = 0; f < F; ++f) {
      const int o = p.off[f];
      uint32_t co[N], ro[N];
#pragma unroll
      for (int c = 0; c < N; ++c) co[c] = q.sdom_coloff[(size_t)(o + c) * pad + k];
#pragma unroll
      for (int m = 0; m < N; ++m) ro[m] = cload(rowoff_d, o + m);
      double vr[N][N], vi[N][N];
      int pcol[N];
      double dre, dim;
      bool zero;
      gather<N>(lds, co, ro, vr, vi);
#pragma unroll
      for (int j = 0; j < N; ++j) pcol[j] = (int)co[j];
      lu<N, true, true, false, true>(vr, vi, dre, dim, pcol, zero);
      bad = bad || zero;
    }
    const bool need = valid && bad;
    if (__builtin_amdgcn_ballot_w64(need) == 0) continue;
    const int g_begin = cload(p.dom_grp, d);
    const int g_end = cload(p.dom_grp, d + 1);
    const int sg_begin = q.sdom_grp[k];
    const int sg_end = q.sdom_grp[k + 1];
    const double wa = cload(a.w_src, cload(p.dom_term, d));
    const double wb = valid ? a.w_snk[q.sdom_term[k]] : 0.0;
    double fre = 0.0, fim = 0.0;
    // source members: the dominator (ci = cs_begin - 1), then its children
    const int cs_begin = cload(p.grp_ptr, g_begin);
    const int cs_end = cload(p.grp_ptr, g_end);
    int gsrc = g_begin;
    for (int ci = cs_begin - 1; ci < cs_end; ++ci) {
      int fs = -1, rs = -1;
      uint32_t srow = 0u;
      double wi = wa;
      if (ci >= cs_begin) {
        while (cload(p.grp_ptr, gsrc + 1) <= ci) ++gsrc;
        fs = cload(p.grp_fr, gsrc) >> 8;
        rs = cload(p.grp_fr, gsrc) & 0xff;
        srow = cload(p.child_rowoff, ci);
        wi = cload(a.w_src, cload(p.child_term, ci));
      }
      // sink members: the dominator, then the children of its groups
      const int cd_begin = q.sgrp_ptr[sg_begin];
      const int cd_end = q.sgrp_ptr[sg_end];
      int gsnk = sg_begin;
      for (int cj = cd_begin - 1; cj < cd_end; ++cj) {
        int fk = -1, ck = -1;
        uint32_t scol = 0u;
        double wj = wb;
        if (cj >= cd_begin) {
          while (q.sgrp_ptr[gsnk + 1] <= cj) ++gsnk;
          fk = q.sgrp_fc[gsnk] >> 8;
          ck = q.sgrp_fc[gsnk] & 0xff;
          scol = q.schild_coloff[cj];
          wj = a.w_snk[q.schild_term[cj]];
        }
        double Dre = 1.0, Dim = 0.0;
        for (int f = 0; f < F; ++f) {
          const int o = p.off[f];
          uint32_t co[N];
#pragma unroll
          for (int c = 0; c < N; ++c) co[c] = q.sdom_coloff[(size_t)(o + c) * pad + k];
          double dre, dim;
          block_det2<N>(lds, rowoff_d + o, f == fs ? rs : -1, srow, co, f == fk ? ck : -1, scol,
                        dre, dim);
          const double tr = Dre * dre - Dim * dim;
          Dim = Dre * dim + Dim * dre;
          Dre = tr;
        }
        if (need) {
          fre += wi * wj * Dre;
          fim += wi * wj * Dim;
        }
      }
    }
    if (need) {
      acc_re += fre;
      acc_im += fim;
      ++n_fallback;
    }
  }
  __shared__ double red[kWavesPerBlock][2];
  const double s0 = wave_sum(acc_re), s1 = wave_sum(acc_im);
  if (lane == 0) {
    red[wave][0] = s0;
    red[wave][1] = s1;
  }
  if (a.fallback) {
    uint32_t nf = n_fallback;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) nf += __shfl_xor(nf, o, kWave);
    if (lane == 0 && nf) atomicAdd(a.fallback, (unsigned long long)nf);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) v += red[w][threadIdx.x];
    a.partial[((size_t)t * a.n_blk_t + chunk) * 3 + threadIdx.x] += v;
  }
}

template <int N>
__global__ __launch_bounds__(kBlock, 2) void contract_two_sided_pairs_kernel(ContractArgs a) {
  extern __shared__ double2 smem[];
  two_sided_pairs_tile<N>(a, blockIdx.y, blockIdx.x, smem);
}

// The sink children's records of one call: the static ones with the
// weight of their term (0 for padding).
__global__ __launch_bounds__(kBlock) void sink_records(const int4* st, const double* w_snk, int n,
                                                       SinkRec* out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const int4 r = st[e];
  SinkRec o;
  o.col = (uint32_t)r.x;
  o.ccol = (uint32_t)r.y;
  o.w = r.z >= 0 ? w_snk[r.z] : 0.0;
  out[e] = o;
}

template <int N, bool TAB, bool PARK>
__global__ __launch_bounds__(kBlock, 2) void contract_two_sided_kernel(ContractArgs a) {
  extern __shared__ double2 smem[];
  two_sided_tile<N, TAB, PARK>(a, blockIdx.y, blockIdx.x, smem);
}

template <int N>
static hipError_t launch_two_sided_n(const ContractArgs& a, hipStream_t s) {
  dim3 grid(a.n_blk_t, a.T);
  // the tables (tab_rows > 0) are sized by the caller to fit beside the
  // slice and the slots within kTwoSidedLdsLimit; without them, the slots
  // where they fit
  const bool tab = a.tab_rows > 0;
  const size_t base = lds_slice_bytes(a.plan.M) +
                      (tab ? (size_t)kWavesPerBlock * a.tab_rows * a.plan.M * 16 : 0);
  const bool park = tab || base + kTwoSidedSlotBytes <= kTwoSidedLdsLimit;
  const size_t lds = base + (park ? kTwoSidedSlotBytes : 0);
  const void* fn = tab    ? reinterpret_cast<const void*>(&contract_two_sided_kernel<N, true, true>)
                   : park ? reinterpret_cast<const void*>(&contract_two_sided_kernel<N, false, true>)
                          : reinterpret_cast<const void*>(&contract_two_sided_kernel<N, false, false>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (tab)
    hipLaunchKernelGGL((contract_two_sided_kernel<N, true, true>), grid, dim3(kBlock), lds, s, a);
  else if (park)
    hipLaunchKernelGGL((contract_two_sided_kernel<N, false, true>), grid, dim3(kBlock), lds, s, a);
  else
    hipLaunchKernelGGL((contract_two_sided_kernel<N, false, false>), grid, dim3(kBlock), lds, s,
                       a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds2 = lds_slice_bytes(a.plan.M);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&contract_two_sided_pairs_kernel<N>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((contract_two_sided_pairs_kernel<N>), grid, dim3(kBlock), lds2, s, a);
  return hipGetLastError();
}

hipError_t launch_contract_two_sided(const ContractArgs& a, int n, double2* C, hipStream_t s) {
  hipError_t e;
  if (a.snk.n_srec > 0) {
    hipLaunchKernelGGL(sink_records, dim3((a.snk.n_srec + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       a.snk.srec_static, a.w_snk, a.snk.n_srec, a.srec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  switch (n) {
#define MHC_CASE(NN)                     \
  case NN:                               \
    e = launch_two_sided_n<NN>(a, s);    \
    break;
    MHC_CASE(1) MHC_CASE(2) MHC_CASE(3) MHC_CASE(4) MHC_CASE(5) MHC_CASE(6) MHC_CASE(7)
    MHC_CASE(8)
#undef MHC_CASE
    default:
      return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return launch_reduce(a, C, nullptr, s);
}

}  // namespace kern
}  // namespace mhc
