// Contraction kernels for flavour blocks of any size up to NMAX (gfx950).
//
// One group of GROUP lanes (16 or 32) holds one matrix, one row per lane, so
// a row exchange is a relabelling: no data moves.  Every block of every
// flavour may have its own size n <= NMAX (lanes m >= n hold no row).
//
// Per flavour block of a (row set, sink) pair the group runs Gauss-Jordan
// elimination with partial pivoting (pivot = largest |Re| + |Im| among the
// rows not yet used, lowest row on ties).  Eliminating every other row at
// every step (not only the rows below) costs nothing extra here -- a lane
// whose row is done would idle otherwise -- and leaves each row m with one
// non-zero, its pivot u_m in column c_m.  det G = sign(pivot order) *
// prod_k u_k, the same pivots as GEPP.  Each row keeps its multipliers in
// the columns the elimination zeroed; replaying those row operations on a
// unit column e_r gives E', and x = G^-1 e_r has x[c_m] = E'_m / u_m: no
// triangular solve is needed, and no appended columns are carried through
// the elimination.  A child whose row r is replaced by s has det = det G *
// (s . x) (matrix determinant lemma, Sec. 2): each lane multiplies s[c_m]
// by x[c_m] and the group sums.
//
// Work decomposition: a wave holds 64 / GROUP sinks of one row set (the
// tree structure stays wave-uniform); a workgroup stages S_t in LDS and its
// waves walk a strided share of the slice's items, as in the one-lane-per-
// matrix kernels.  Reductions are fixed-order.
//
// Broadcasts within a group: in the 1024-thread workgroups (four waves
// per SIMD, where the LDS pipe bounds the elimination) they go through
// LDS: the pivot lane writes its row to the group's row buffer and every
// lane of the group reads it back (one ds_read_b128 per complex entry, all
// lanes of a group on one address).  On gfx950 that moves about 270 B per
// clock and compute unit against about 40 for ds_bpermute_b32, which needs
// four instructions per complex entry.  The row buffers sit at the start
// of the dynamic LDS, the copy of S_t after them.  In the 512-thread
// workgroups (two waves per SIMD, where the latency of each elimination
// step bounds it) the shuffles stay: the write-then-read of the buffer
// lengthens that chain (measured 17 % slower there, 3-11 % faster in the
// 1024-thread kernels).

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "contract_kernels.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

// Workgroup sizes: 512 threads, or 1024 where one slice of S fills most of
// the LDS (one workgroup per CU) and the kernel fits in 128 VGPRs, so that
// four waves per SIMD hide the broadcast latencies of the elimination.
constexpr int kWideBlock = 512;
constexpr int kWideBlockBig = 1024;
// 768 threads: three waves per SIMD for the kernels that need 129..168
// VGPRs (two waves per SIMD at 512 threads).
constexpr int kWideBlockMid = 768;

// Broadcast through LDS row buffers (true) or shuffles, per workgroup size.
constexpr bool wide_lds_bcast(int wb) { return wb == kWideBlockBig; }

// Bytes of the groups' row buffers of one workgroup: NMAX complex entries
// per group, where the broadcast goes through LDS.
constexpr size_t wide_rows_bytes(int group, int nmax, int wb) {
  return wide_lds_bcast(wb) ? (size_t)(wb / group) * nmax * 16 : 0;
}

// A double moved across lanes by a DPP row rotation (within each row of 16
// lanes): lane i receives lane (i + R) mod 16 of its row.
template <int R>
__device__ __forceinline__ double row_ror(double v) {
  constexpr int ctrl = 0x120 + R;   // DPP row_ror:R
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum / max over the GROUP lanes of a group: rotations by 8, 4, 2, 1 within
// each row of 16 (every lane forms the same pairs, so all lanes get the
// same bits), then one exchange between the two rows of a 32-lane group.
template <int GROUP>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(GROUP == 16 || GROUP == 32, "groups are one or two DPP rows");
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  if (GROUP == 32) v += __shfl_xor(v, 16, 32);
  return v;
}

template <int GROUP>
__device__ __forceinline__ double group_max(double v) {
  static_assert(GROUP == 16 || GROUP == 32, "groups are one or two DPP rows");
  v = fmax(v, row_ror<8>(v));
  v = fmax(v, row_ror<4>(v));
  v = fmax(v, row_ror<2>(v));
  v = fmax(v, row_ror<1>(v));
  if (GROUP == 32) v = fmax(v, __shfl_xor(v, 16, 32));
  return v;
}

// The lanes of a group exchange values through LDS with plain stores and
// loads.  Between a lane's store and another lane's load (and between a
// load and the next store to the same place) the compiler must not move
// either: a wavefront-scope release/acquire fence around a wave barrier
// forbids that.  LDS executes one wave's instructions in order, so it
// costs nothing at run time.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// fn(integral_constant<int, i>) for i = B .. E-1: the loop is unrolled in
// the source, so every array index below is a constant expression and the
// per-lane rows stay in registers at any NMAX.
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    static_for<B + 1, E>(fn);
  }
}

// Result of eliminating one flavour block.
struct GJResult {
  double dre, dim;   // det G (same value in every lane of the group)
  bool zero;         // some pivot was exactly zero
};

// Pivot lanes of the elimination steps, 5 bits each.
template <int NMAX>
struct PivotLanes {
  uint32_t w[(NMAX + 5) / 6];
  __device__ __forceinline__ int get(int k) const { return (w[k / 6] >> (5 * (k % 6))) & 31; }
};

// Gauss-Jordan on the group's matrix.  (ar, ai)[c]: this lane's row
// (columns c < n).  Step k eliminates column k from every row but the
// pivot row; a row's multiplier l_{m,k} is kept in its column k (which
// the elimination has just zeroed), so the row operations can be replayed
// on any right-hand side afterwards (replay_unit).  On return, lane m < n
// holds the reciprocal of its pivot in (ur, ui) and the column it pivoted
// in (col); piv holds the pivot lane of every step.
// LDS_BCAST: the pivot row goes through the group's LDS row buffer (the
// factorisations of the main path); otherwise through ds_bpermute shuffles
// (the direct factorisations of the zero-pivot route, where the LDS form,
// inlined into the children loop, made the compiler keep far more
// registers live).
template <int GROUP, int NMAX, bool LDS_BCAST>
__device__ __forceinline__ GJResult gauss_jordan(double (&ar)[NMAX], double (&ai)[NMAX], int n,
                                                 int m, double& ur, double& ui, int& col,
                                                 PivotLanes<NMAX>& piv, double2* prow) {
  static_assert(GROUP <= 32, "lane rank is packed into 5 bits");
  GJResult res{1.0, 0.0, false};
  bool done = m >= n;
  bool neg = false;
  const int gbase = (__lane_id() / GROUP) * GROUP;
  ur = 0.0;
  ui = 0.0;
  col = -1;
  static_for<0, (NMAX + 5) / 6>([&](auto ic) { piv.w[decltype(ic)::value] = 0u; });
  static_for<0, NMAX>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if (k >= n) return;
    // pivot: largest |Re|+|Im| of column k among rows not used yet
    const double mag = fabs(ar[k]) + fabs(ai[k]);
    const uint32_t lo = (__double2loint(mag) & ~31u) | (uint32_t)(31 - m);
    double key = done ? -1.0 : __hiloint2double(__double2hiint(mag), (int)lo);
    key = group_max<GROUP>(key);
    // (some row of the group is always unused at step k < n, so the max
    // carries a rank 0 <= p < GROUP; the mask only keeps the lane in range)
    const int p = (31 - (int)(__double2loint(key) & 31u)) & (GROUP - 1);
    piv.w[k / 6] |= (uint32_t)p << (5 * (k % 6));
    // sign: rows below p that are still unused each contribute one
    // transposition to the pivot permutation
    const uint64_t open = __builtin_amdgcn_ballot_w64(!done);
    const uint32_t below = (uint32_t)((open >> gbase) & ((1ull << p) - 1ull));
    neg = neg != ((__builtin_popcount(below) & 1) != 0);
    // pivot row, broadcast to the group
    const bool me = (m == p);
    const int src = gbase + p;
    double pr, pi;
    if constexpr (LDS_BCAST) {
      if (me) {
        static_for<k, NMAX>([&](auto cc) {
          constexpr int c = decltype(cc)::value;
          if (c < n) prow[c] = make_double2(ar[c], ai[c]);
        });
      }
      wave_lds_sync();
      const double2 pv = prow[k];
      pr = pv.x;
      pi = pv.y;
    } else {
      pr = __shfl(ar[k], src, 64);
      pi = __shfl(ai[k], src, 64);
    }
    const double pmag = fabs(pr) + fabs(pi);
    res.zero = res.zero || (pmag == 0.0);
    const double t = res.dre * pr - res.dim * pi;
    res.dim = res.dre * pi + res.dim * pr;
    res.dre = t;
    double vr, vi;
    cinv(pr, pi, pmag, vr, vi);
    if (me) {
      ur = vr;
      ui = vi;
      col = k;
      done = true;
    }
    // multiplier of this row (0 for the pivot row and empty lanes)
    double lr = ar[k] * vr - ai[k] * vi;
    double li = ar[k] * vi + ai[k] * vr;
    if (me || m >= n) {
      lr = 0.0;
      li = 0.0;
    }
    static_for<k + 1, NMAX>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if (c >= n) return;
      double br, bi;
      if constexpr (LDS_BCAST) {
        const double2 b = prow[c];
        br = b.x;
        bi = b.y;
      } else {
        br = __shfl(ar[c], src, 64);
        bi = __shfl(ai[c], src, 64);
      }
      ar[c] = ar[c] - lr * br + li * bi;
      ai[c] = ai[c] - lr * bi - li * br;
    });
    if constexpr (LDS_BCAST) wave_lds_sync();   // the row is read before the next step writes
    if (!me) {
      ar[k] = lr;
      ai[k] = li;
    }
  });
  if (neg) {
    res.dre = -res.dre;
    res.dim = -res.dim;
  }
  return res;
}

// x = G^-1 e_r from an elimination: replays its row operations on the unit
// column e_r (lane m holds entry m); then x[col_m] = E'_m / u_m, returned
// in (xr, xi) by lane m.  The pivot lane of a step keeps its own column k
// entry (its pivot), which the step does not use.
template <int GROUP, int NMAX, bool LDS_BCAST>
__device__ __forceinline__ void replay_unit(const double (&ar)[NMAX], const double (&ai)[NMAX],
                                            const PivotLanes<NMAX>& piv, int r, int n, int m,
                                            double ur, double ui, double& xr, double& xi,
                                            double2* prow) {
  const int gbase = (__lane_id() / GROUP) * GROUP;
  double er = (m == r) ? 1.0 : 0.0, ei = 0.0;
  static_for<0, NMAX>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if (k >= n) return;
    const int p = piv.get(k);
    // the pivot lane's entry, broadcast to the group
    double br, bi;
    if constexpr (LDS_BCAST) {
      if (m == p) prow[0] = make_double2(er, ei);
      wave_lds_sync();
      const double2 b = prow[0];
      wave_lds_sync();
      br = b.x;
      bi = b.y;
    } else {
      br = __shfl(er, gbase + p, 64);
      bi = __shfl(ei, gbase + p, 64);
    }
    if (m != p && m < n) {
      er = er - ar[k] * br + ai[k] * bi;
      ei = ei - ar[k] * bi - ai[k] * br;
    }
  });
  xr = er * ur - ei * ui;
  xi = er * ui + ei * ur;
}

// det of the block whose row `rrep` is replaced by the LDS row `newrow`
// (direct elimination; used when the dominator block had a zero pivot).
template <int GROUP, int NMAX>
__device__ __forceinline__ void block_det_direct(const char* lds, uint32_t myrow, int rrep,
                                                 uint32_t newrow, const uint32_t (&co)[NMAX],
                                                 int n, int m, double& dre, double& dim,
                                                 double2* prow) {
  const uint32_t row = (m == rrep) ? newrow : myrow;
  double ar[NMAX], ai[NMAX];
#pragma unroll
  for (int c = 0; c < NMAX; ++c) {
    ar[c] = 0.0;
    ai[c] = 0.0;
    if (c < n && m < n) {
      const double2 v = *reinterpret_cast<const double2*>(lds + row + co[c]);
      ar[c] = v.x;
      ai[c] = v.y;
    }
  }
  double ur, ui;
  int col;
  PivotLanes<NMAX> piv;
  const GJResult g = gauss_jordan<GROUP, NMAX, false>(ar, ai, n, m, ur, ui, col, piv, prow);
  dre = g.dre;
  dim = g.dim;
}

// One tile (slice t, chunk) of a job, as lane_tile for one matrix per lane.
template <int GROUP, int NMAX, bool TREE, int MODE, int WB>
__device__ __forceinline__ void wide_tile(const ContractArgs& a, int t, int chunk,
                                          double2* smem) {
  constexpr bool WITH_A = (MODE & 1) != 0;
  constexpr bool WITH_PAIRS = (MODE & 2) != 0;
  constexpr int SPW = kWave / GROUP;   // sinks per wave
  const PlanView& p = a.plan;
  __syncthreads();  // the previous tile of this workgroup is done with LDS
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  const int m = lane % GROUP;          // row of the matrix held by this lane
  const int gsel = lane / GROUP;       // which sink of the wave
  const int MM = p.M * p.M;
  const double2* St = a.S + (size_t)t * MM;
  constexpr int kWaves = WB / kWave;
  // this group's row buffer (used with LDS broadcasts only), then the copy
  // of S_t
  double2* prow = smem + (threadIdx.x / GROUP) * NMAX;
  double2* slice = smem + wide_rows_bytes(GROUP, NMAX, WB) / 16;
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
          block_det_direct<GROUP, NMAX>(lds, myrow, -1, 0u, co, n, m, Dpre_re[f], Dpre_im[f],
                                        prow);
        }
      }
    }

    int g = g_begin;
    for (int f = 0; f < F; ++f) {
      const int o = p.off[f];
      const int n = p.off[f + 1] - o;
      uint32_t co[NMAX];
#pragma unroll
      for (int c = 0; c < NMAX; ++c)
        co[c] = c < n ? p.snk_coloff[(size_t)(o + c) * p.n_snk_pad + k] : 0u;
      const uint32_t myrow = m < n ? rowoff_d[o + m] : 0u;
      double ar[NMAX], ai[NMAX];
#pragma unroll
      for (int c = 0; c < NMAX; ++c) {
        ar[c] = 0.0;
        ai[c] = 0.0;
        if (c < n && m < n) {
          const double2 v = *reinterpret_cast<const double2*>(lds + myrow + co[c]);
          ar[c] = v.x;
          ai[c] = v.y;
        }
      }
      int g_f_end = g;
      if (TREE) {
        while (g_f_end < g_end && uniform(p.grp_fr[g_f_end] >> 8) == f) ++g_f_end;
      }
      const int R = g_f_end - g;
      double ur, ui;
      int col;
      PivotLanes<NMAX> piv;
      const GJResult res =
          gauss_jordan<GROUP, NMAX, wide_lds_bcast(WB)>(ar, ai, n, m, ur, ui, col, piv, prow);
      const double dre = res.dre, dim = res.dim;
      const bool zero = res.zero;
      // this lane's pivot column: its sink column offset
      uint32_t mycol = 0;
#pragma unroll
      for (int c = 0; c < NMAX; ++c)
        if (c == col) mycol = co[c];
      double accre = 0.0, accim = 0.0;
      if (TREE && R > 0) {
        double sre = 0.0, sim = 0.0;
        for (int q = 0; q < R; ++q) {
          // x = G^-1 e_r for this group's row r; lane m holds x[col]
          double x_r, x_i;
          replay_unit<GROUP, NMAX, wide_lds_bcast(WB)>(ar, ai, piv,
                                                       uniform(p.grp_fr[g + q] & 0xff), n, m,
                                                       ur, ui, x_r, x_i, prow);
          const int gg = g + q;
          const int c_begin = uniform(p.grp_ptr[gg]);
          const int c_end = uniform(p.grp_ptr[gg + 1]);
          for (int c = c_begin; c < c_end; ++c) {
            const uint32_t crow = uniform(p.child_rowoff[c]);
            const int cterm = uniform(p.child_term[c]);
            double pr_ = 0.0, pi_ = 0.0;
            if (m < n) {
              const double2 s = *reinterpret_cast<const double2*>(lds + crow + mycol);
              pr_ = s.x * x_r - s.y * x_i;
              pi_ = s.x * x_i + s.y * x_r;
            }
            const double rr = group_sum<GROUP>(pr_);
            const double ri = group_sum<GROUP>(pi_);
            const double wc = a.w_src[cterm];
            sre += wc * rr;
            sim += wc * ri;
            if (WITH_A && !zero) sabs_reg += fabs(wc) * sqrt(rr * rr + ri * ri);
            if (WITH_PAIRS && writer && a.pair_det && !zero) {
              double cr = rr * dre - ri * dim, ci = rr * dim + ri * dre;
#pragma unroll
              for (int h = 0; h < kPairFlavors; ++h) {
                if (h == f || h >= F) continue;
                const double tr = cr * Dpre_re[h] - ci * Dpre_im[h];
                ci = cr * Dpre_im[h] + ci * Dpre_re[h];
                cr = tr;
              }
              a.pair_det[((size_t)t * p.n_src + cterm) * p.n_snk + k] = make_double2(cr, ci);
            }
          }
        }
        accre = zero ? 0.0 : dre * sre - dim * sim;
        accim = zero ? 0.0 : dre * sim + dim * sre;
      }
      if (zero) {
        ++nbad;
        fbad = (TREE && R > 0) ? f : -2;
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

    if (TREE) {
      // children of a singular block (the only singular one): direct
      const bool need = valid && nbad == 1 && fbad >= 0;
      if (__builtin_amdgcn_ballot_w64(need) != 0) {
        for (int f = 0; f < F; ++f) {
          if (__builtin_amdgcn_ballot_w64(need && fbad == f) == 0) continue;
          const int o = p.off[f];
          const int n = p.off[f + 1] - o;
          uint32_t co[NMAX];
#pragma unroll
          for (int c = 0; c < NMAX; ++c)
            co[c] = c < n ? p.snk_coloff[(size_t)(o + c) * p.n_snk_pad + k] : 0u;
          const uint32_t myrow = m < n ? rowoff_d[o + m] : 0u;
          double fre = 0.0, fim = 0.0;
          for (int gg = g_begin; gg < g_end; ++gg) {
            if (uniform(p.grp_fr[gg] >> 8) != f) continue;
            const int r = uniform(p.grp_fr[gg] & 0xff);
            for (int c = uniform(p.grp_ptr[gg]); c < uniform(p.grp_ptr[gg + 1]); ++c) {
              const uint32_t crow = uniform(p.child_rowoff[c]);
              const int cterm = uniform(p.child_term[c]);
              double cre, cim;
              block_det_direct<GROUP, NMAX>(lds, myrow, r, crow, co, n, m, cre, cim, prow);
              if (need && fbad == f) {
                const double wc = a.w_src[cterm];
                fre += wc * cre;
                fim += wc * cim;
                const double dr = cre * Xre - cim * Xim, di = cre * Xim + cim * Xre;
                if (WITH_A) sabs_fb += fabs(wc) * sqrt(dr * dr + di * di);
                if (WITH_PAIRS && writer && a.pair_det)
                  a.pair_det[((size_t)t * p.n_src + cterm) * p.n_snk + k] = make_double2(dr, di);
                if (m == 0) ++n_fallback;
              }
            }
          }
          if (need && fbad == f) {
            Qre += fre * Xre - fim * Xim;
            Qim += fre * Xim + fim * Xre;
          }
        }
      }
    }

    if (WITH_PAIRS && a.pair_det && writer) {
      a.pair_det[((size_t)t * p.n_src + term) * p.n_snk + k] = make_double2(Pre, Pim);
    }
    if (writer) {
      acc_re += wk * (wi * Pre + Qre);
      acc_im += wk * (wi * Pim + Qim);
      if (WITH_A) {
        const double pabs = sqrt(Pre * Pre + Pim * Pim);
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

template <int GROUP, int NMAX, bool TREE, int MODE, int WB>
__global__ __launch_bounds__(WB) void contract_wide_kernel(ContractArgs a) {
  extern __shared__ double2 smem[];
  wide_tile<GROUP, NMAX, TREE, MODE, WB>(a, blockIdx.y, blockIdx.x, smem);
}

template <int GROUP, int NMAX, bool TREE, int MODE, int WB>
__global__ __launch_bounds__(WB) void batch_wide_kernel(BatchArgs b) {
  extern __shared__ double2 smem[];
  for (int i = blockIdx.x; i < b.n_tiles; i += gridDim.x) {
    const int4 tl = b.tiles[i];
    wide_tile<GROUP, NMAX, TREE, MODE, WB>(b.jobs[tl.x], tl.y, tl.z, smem);
  }
}

// 1024-thread workgroups where they measured faster on the batched and
// large workloads: every plain bucket, and the tree's (16, 8) and (16, 12)
// (the larger tree buckets spill too much in 128 VGPRs); only when the
// slice needs over 80 KB of LDS, and not for the test-hook modes.
constexpr bool big_block_allowed(int nmax, bool tree, int mode) {
  return (mode & 2) == 0 && (!tree || nmax <= 12);
}

// The buckets that need 129..168 VGPRs: the tree's from 12 up, the plain
// 16 and 24.
constexpr bool mid_block_allowed(int nmax, bool tree, int mode) {
  return (mode & 2) == 0 && (tree ? nmax >= 12 : (nmax == 16 || nmax == 24));
}

// The LDS a workgroup can have: 160 KiB, less 1 KiB for the static
// arrays of the kernels.
constexpr size_t kWideLdsLimit = 159 * 1024;

int wide_block(int nmax, bool tree, size_t lds) {
  const int b = wide_bucket(nmax);
  const int group = b <= 16 ? 16 : 32;
  // one slice fills most of the LDS (one workgroup per compute unit): 1024
  // threads where the kernel fits 128 VGPRs and the row buffers fit
  if (lds > 80 * 1024 && big_block_allowed(b, tree, 0) &&
      lds + wide_rows_bytes(group, b, kWideBlockBig) <= kWideLdsLimit)
    return kWideBlockBig;
  if (mid_block_allowed(b, tree, 0)) return kWideBlockMid;
  return kWideBlock;
}

template <int GROUP, int NMAX, bool TREE, int MODE, int WB>
static hipError_t launch_wide_wb(const ContractArgs& a, size_t slice, hipStream_t s) {
  dim3 grid(a.n_blk_t, a.T);
  const size_t lds = slice + wide_rows_bytes(GROUP, NMAX, WB);
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&contract_wide_kernel<GROUP, NMAX, TREE, MODE, WB>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((contract_wide_kernel<GROUP, NMAX, TREE, MODE, WB>), grid, dim3(WB), lds,
                     s, a);
  return hipGetLastError();
}

template <int GROUP, int NMAX, bool TREE, int MODE>
static hipError_t launch_wide_one(const ContractArgs& a, hipStream_t s) {
  const size_t lds = lds_slice_bytes(a.plan.M);
  if constexpr (big_block_allowed(NMAX, TREE, MODE)) {
    if (wide_block(NMAX, TREE, lds) == kWideBlockBig)
      return launch_wide_wb<GROUP, NMAX, TREE, MODE, kWideBlockBig>(a, lds, s);
  }
  if constexpr (mid_block_allowed(NMAX, TREE, MODE)) {
    if (wide_block(NMAX, TREE, lds) == kWideBlockMid)
      return launch_wide_wb<GROUP, NMAX, TREE, MODE, kWideBlockMid>(a, lds, s);
  }
  return launch_wide_wb<GROUP, NMAX, TREE, MODE, kWideBlock>(a, lds, s);
}

template <int GROUP, int NMAX>
static hipError_t launch_wide_n(const ContractArgs& a, bool tree, bool diag, hipStream_t s) {
  if (tree)
    return diag ? launch_wide_one<GROUP, NMAX, true, 3>(a, s)
                : launch_wide_one<GROUP, NMAX, true, 0>(a, s);
  return diag ? launch_wide_one<GROUP, NMAX, false, 3>(a, s)
              : launch_wide_one<GROUP, NMAX, false, 0>(a, s);
}

int wide_sinks_per_wave(int nmax) { return nmax <= 16 ? kWave / 16 : kWave / 32; }

template <int GROUP, int NMAX, bool TREE, int MODE, int WB>
static hipError_t launch_batch_wide_wb(const BatchArgs& b, int grid, size_t slice,
                                       hipStream_t s) {
  const size_t lds = slice + wide_rows_bytes(GROUP, NMAX, WB);
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&batch_wide_kernel<GROUP, NMAX, TREE, MODE, WB>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((batch_wide_kernel<GROUP, NMAX, TREE, MODE, WB>), dim3(grid), dim3(WB),
                     lds, s, b);
  return hipGetLastError();
}

template <int GROUP, int NMAX, bool TREE, int MODE>
static hipError_t launch_batch_wide_m(const BatchArgs& b, int grid, size_t lds, hipStream_t s) {
  if constexpr (big_block_allowed(NMAX, TREE, MODE)) {
    if (wide_block(NMAX, TREE, lds) == kWideBlockBig)
      return launch_batch_wide_wb<GROUP, NMAX, TREE, MODE, kWideBlockBig>(b, grid, lds, s);
  }
  if constexpr (mid_block_allowed(NMAX, TREE, MODE)) {
    if (wide_block(NMAX, TREE, lds) == kWideBlockMid)
      return launch_batch_wide_wb<GROUP, NMAX, TREE, MODE, kWideBlockMid>(b, grid, lds, s);
  }
  return launch_batch_wide_wb<GROUP, NMAX, TREE, MODE, kWideBlock>(b, grid, lds, s);
}

template <int GROUP, int NMAX>
static hipError_t launch_batch_wide_n(const BatchArgs& b, bool tree, bool with_a, int grid,
                                      size_t lds, hipStream_t s) {
  if (tree)
    return with_a ? launch_batch_wide_m<GROUP, NMAX, true, 1>(b, grid, lds, s)
                  : launch_batch_wide_m<GROUP, NMAX, true, 0>(b, grid, lds, s);
  return with_a ? launch_batch_wide_m<GROUP, NMAX, false, 1>(b, grid, lds, s)
                : launch_batch_wide_m<GROUP, NMAX, false, 0>(b, grid, lds, s);
}

int wide_bucket(int nmax) {
  return nmax <= 8 ? 8 : nmax <= 12 ? 12 : nmax <= 16 ? 16 : nmax <= 18 ? 18 : 24;
}

hipError_t launch_batch_wide(const BatchArgs& b, int nmax, bool tree, bool with_a, int grid,
                             size_t lds, hipStream_t s) {
  switch (wide_bucket(nmax)) {
    case 8:
      return launch_batch_wide_n<16, 8>(b, tree, with_a, grid, lds, s);
    case 12:
      return launch_batch_wide_n<16, 12>(b, tree, with_a, grid, lds, s);
    case 16:
      return launch_batch_wide_n<16, 16>(b, tree, with_a, grid, lds, s);
    case 18:
      return launch_batch_wide_n<32, 18>(b, tree, with_a, grid, lds, s);
    default:
      return launch_batch_wide_n<32, 24>(b, tree, with_a, grid, lds, s);
  }
}

hipError_t launch_contract_wide(const ContractArgs& a, int nmax, bool tree, bool diag,
                                double2* C, double* A, hipStream_t s) {
  hipError_t e;
  if (nmax <= 8)
    e = launch_wide_n<16, 8>(a, tree, diag, s);
  else if (nmax <= 12)
    e = launch_wide_n<16, 12>(a, tree, diag, s);
  else if (nmax <= 16)
    e = launch_wide_n<16, 16>(a, tree, diag, s);
  else if (nmax <= 18)
    e = launch_wide_n<32, 18>(a, tree, diag, s);
  else if (nmax <= 24)
    e = launch_wide_n<32, 24>(a, tree, diag, s);
  else
    return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  return launch_reduce(a, C, A, s);
}

}  // namespace kern
}  // namespace mhc
