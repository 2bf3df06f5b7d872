// Device building blocks of the group kernels (one group of GROUP lanes per
// matrix, one row per lane): DPP group reductions, the LDS handshake
// between the lanes of a wave, Gauss-Jordan elimination with partial
// pivoting by row relabelling, the replay of its row operations on a unit
// column, and the direct determinant of a block with one row replaced.
// Shared by the contraction kernels and the per-pair kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lu_device.h"

namespace mhc {
namespace kern {

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

}  // namespace kern
}  // namespace mhc
