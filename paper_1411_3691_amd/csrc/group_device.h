// Device building blocks of the group kernels (one group of GROUP lanes per
// matrix, one row per lane): DPP group reductions, the LDS handshake
// between the lanes of a wave, Gauss-Jordan elimination with partial
// pivoting by row relabelling that carries right-hand sides, and the direct
// determinant of a block with one row replaced.  Shared by the contraction
// kernels and the per-pair kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lu_device.h"

namespace mhc {
namespace kern {

// A double moved across lanes by one DPP control (row_ror, quad_perm,
// row_half_mirror): lane i receives the lane the control names within its
// row of 16.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// DPP controls: row_ror:R rotates a row of 16 by R; quad_perm [1,0,3,2] and
// [2,3,0,1] swap neighbours and pairs within each quad; row_half_mirror
// reverses each half row of 8, row_mirror each row of 16.
constexpr int kDppRor8 = 0x128, kDppRor4 = 0x124, kDppRor2 = 0x122, kDppRor1 = 0x121;
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppRowMirror = 0x140;

// Sum / max over the GROUP lanes of a group (4: two exchanges within each
// quad; 8: three steps within each half row; 16: rotations by 8, 4, 2, 1
// within each row; 32: one more exchange between the two rows).  Every lane
// combines the same values in the same order up to commutation, so all
// lanes get the same bits.
template <int GROUP>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(GROUP == 4 || GROUP == 8 || GROUP == 16 || GROUP == 32,
                "groups are 4, 8, 16 or 32 lanes");
  if constexpr (GROUP == 4) {
    v += dpp_move<kDppXor1>(v);
    v += dpp_move<kDppXor2>(v);
  } else if constexpr (GROUP == 8) {
    v += dpp_move<kDppXor1>(v);
    v += dpp_move<kDppXor2>(v);
    v += dpp_move<kDppHalfMirror>(v);
  } else {
    v += dpp_move<kDppRor8>(v);
    v += dpp_move<kDppRor4>(v);
    v += dpp_move<kDppRor2>(v);
    v += dpp_move<kDppRor1>(v);
    if (GROUP == 32) v += __shfl_xor(v, 16, 32);
  }
  return v;
}

template <int GROUP>
__device__ __forceinline__ double group_max(double v) {
  static_assert(GROUP == 4 || GROUP == 8 || GROUP == 16 || GROUP == 32,
                "groups are 4, 8, 16 or 32 lanes");
  if constexpr (GROUP == 4) {
    v = fmax(v, dpp_move<kDppXor1>(v));
    v = fmax(v, dpp_move<kDppXor2>(v));
  } else if constexpr (GROUP == 8) {
    v = fmax(v, dpp_move<kDppXor1>(v));
    v = fmax(v, dpp_move<kDppXor2>(v));
    v = fmax(v, dpp_move<kDppHalfMirror>(v));
  } else {
    v = fmax(v, dpp_move<kDppRor8>(v));
    v = fmax(v, dpp_move<kDppRor4>(v));
    v = fmax(v, dpp_move<kDppRor2>(v));
    v = fmax(v, dpp_move<kDppRor1>(v));
    if (GROUP == 32) v = fmax(v, __shfl_xor(v, 16, 32));
  }
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

// Complex entries of one group's pivot-row buffer in LDS: the row and the
// right-hand sides.
template <int NMAX, int RMAX>
constexpr int prow_entries() {
  return NMAX + RMAX;
}

// Gauss-Jordan elimination with partial pivoting on the group's matrix,
// carrying right-hand sides.  Lane m < n holds row m: (ar, ai)[c] for the
// columns c < n, and (br, bi)[q] for the right-hand sides q < nr (nr <=
// RMAX, the same in every lane of the group; a lane's entry of b_q is row m
// of that column).  Step k takes as pivot the row not used yet with the
// largest |Re| + |Im| in column k (lowest row on ties: one DPP max over the
// group, the lane rank packed into the low mantissa bits); every other row
// subtracts l_m = a_mk / u times the pivot row from its columns above k and
// from its right-hand sides.  Rows are relabelled, never moved.  A row that
// was pivot keeps its pivot u_m in its column col_m (later steps only
// subtract from columns above theirs), so at the end the system reads
// u_m x[col_m] = b'_q[m]: lane m returns 1/u_m in (ur, ui) and col_m in col,
// and x = G^-1 b_q has x[col_m] = b'_q[m] / u_m.  det G = sign of the pivot
// order times the product of the pivots, the pivots of GEPP.  Columns <= k
// of a row are not read after step k and are left as they are.
// LDS_BCAST: the pivot row goes to the group's LDS buffer (prow,
// prow_entries complex entries: the row from column k on, then the
// right-hand sides) and every lane reads it back; otherwise every entry
// moves by a ds_bpermute shuffle.
// Pivot lanes of the elimination steps, 5 bits each.
template <int NMAX>
struct PivotLanes {
  uint32_t w[(NMAX + 5) / 6];
  __device__ __forceinline__ int get(int k) const { return (w[k / 6] >> (5 * (k % 6))) & 31; }
};

// KEEP: each row also keeps its multiplier l_m of step k in its column k
// (which the step no longer needs) and piv records the pivot lane of every
// step, so that replay_units can apply the same row operations to unit
// columns afterwards.
template <int GROUP, int NMAX, int RMAX, bool LDS_BCAST, bool KEEP = false>
__device__ __forceinline__ GJResult gauss_jordan_rhs(double (&ar)[NMAX], double (&ai)[NMAX],
                                                     double (&br)[RMAX], double (&bi)[RMAX],
                                                     int nr, int n, int m, double& ur,
                                                     double& ui, int& col, double2* prow,
                                                     PivotLanes<NMAX>* piv = nullptr) {
  static_assert(GROUP <= 32, "lane rank is packed into 5 bits");
  GJResult res{1.0, 0.0, false};
  bool done = m >= n;
  bool neg = false;
  const int gbase = (__lane_id() / GROUP) * GROUP;
  ur = 0.0;
  ui = 0.0;
  col = -1;
  if constexpr (KEEP) static_for<0, (NMAX + 5) / 6>([&](auto ic) { piv->w[decltype(ic)::value] = 0u; });
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
    if constexpr (KEEP) piv->w[k / 6] |= (uint32_t)p << (5 * (k % 6));
    // sign: rows below p that are still unused each contribute one
    // transposition to the pivot permutation
    const uint64_t open = __builtin_amdgcn_ballot_w64(!done);
    const uint32_t below = (uint32_t)((open >> gbase) & ((1ull << p) - 1ull));
    neg = neg != ((__builtin_popcount(below) & 1) != 0);
    const bool me = (m == p);
    const int src = gbase + p;
    double pr, pi;
    if constexpr (LDS_BCAST) {
      if (me) {
        static_for<k, NMAX>([&](auto cc) {
          constexpr int c = decltype(cc)::value;
          if (c < n) prow[c] = make_double2(ar[c], ai[c]);
        });
        static_for<0, RMAX>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          if (q < nr) prow[NMAX + q] = make_double2(br[q], bi[q]);
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
      double sr, si;
      if constexpr (LDS_BCAST) {
        const double2 b = prow[c];
        sr = b.x;
        si = b.y;
      } else {
        sr = __shfl(ar[c], src, 64);
        si = __shfl(ai[c], src, 64);
      }
      ar[c] = ar[c] - lr * sr + li * si;
      ai[c] = ai[c] - lr * si - li * sr;
      // at most four entries of the pivot row in flight: otherwise the
      // compiler reads the whole row (up to NMAX + RMAX entries) ahead
      if constexpr ((c - k) % 4 == 0) __builtin_amdgcn_sched_barrier(0);
    });
    static_for<0, RMAX>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if (q >= nr) return;
      double sr, si;
      if constexpr (LDS_BCAST) {
        const double2 b = prow[NMAX + q];
        sr = b.x;
        si = b.y;
      } else {
        sr = __shfl(br[q], src, 64);
        si = __shfl(bi[q], src, 64);
      }
      br[q] = br[q] - lr * sr + li * si;
      bi[q] = bi[q] - lr * si - li * sr;
      if constexpr (q % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    });
    if constexpr (LDS_BCAST) wave_lds_sync();   // the row is read before the next step writes
    if constexpr (KEEP) {
      if (!me) {
        ar[k] = lr;
        ai[k] = li;
      }
    }
  });
  if (neg) {
    res.dre = -res.dre;
    res.dim = -res.dim;
  }
  return res;
}

// Applies the row operations of gauss_jordan_rhs<..., KEEP> to nr <= RMAX
// columns b_q at once (lane m holds entry m of each; on entry the unit
// columns e_{r_q}): step k subtracts l_m(k) times the pivot lane's entries.
// On return the system reads u_m x[col_m] = b'_q[m], as if the columns had
// been carried through the elimination.  One pass serves every column, so
// the chain of broadcasts is paid once, not once per column.  The pivot
// lane's entries go through the group's LDS buffer (its first nr entries;
// the elimination no longer needs it) or through shuffles.
template <int GROUP, int NMAX, int RMAX, bool LDS_BCAST>
__device__ __forceinline__ void replay_units(const double (&ar)[NMAX], const double (&ai)[NMAX],
                                             const PivotLanes<NMAX>& piv, int n, int m,
                                             double (&br)[RMAX], double (&bi)[RMAX], int nr,
                                             double2* prow) {
  const int gbase = (__lane_id() / GROUP) * GROUP;
  static_for<0, NMAX>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if (k >= n) return;
    const int p = piv.get(k);
    const bool upd = m != p && m < n;
    if constexpr (LDS_BCAST) {
      if (m == p) {
        static_for<0, RMAX>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          if (q < nr) prow[q] = make_double2(br[q], bi[q]);
        });
      }
      wave_lds_sync();
    }
    static_for<0, RMAX>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if (q >= nr) return;
      double sr, si;
      if constexpr (LDS_BCAST) {
        const double2 b = prow[q];
        sr = b.x;
        si = b.y;
      } else {
        sr = __shfl(br[q], gbase + p, 64);
        si = __shfl(bi[q], gbase + p, 64);
      }
      if (upd) {
        br[q] = br[q] - ar[k] * sr + ai[k] * si;
        bi[q] = bi[q] - ar[k] * si - ai[k] * sr;
      }
    });
    if constexpr (LDS_BCAST) wave_lds_sync();
  });
}

// Loads this lane's row of the block G[m][c] = S_t[row m][col c] from the
// LDS copy of S_t (lanes m >= n and columns c >= n get zeros).
template <int NMAX>
__device__ __forceinline__ void load_row(const char* lds, uint32_t myrow,
                                         const uint32_t (&co)[NMAX], int n, int m,
                                         double (&ar)[NMAX], double (&ai)[NMAX]) {
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
}

// det of the block whose row `rrep` is replaced by the LDS row `newrow`
// (direct elimination, shuffle broadcasts; used when the dominator block had
// a zero pivot).
template <int GROUP, int NMAX>
__device__ __forceinline__ void block_det_direct(const char* lds, uint32_t myrow, int rrep,
                                                 uint32_t newrow, const uint32_t (&co)[NMAX],
                                                 int n, int m, double& dre, double& dim) {
  const uint32_t row = (m == rrep) ? newrow : myrow;
  double ar[NMAX], ai[NMAX];
  load_row<NMAX>(lds, row, co, n, m, ar, ai);
  double ur, ui, b0r[1] = {0.0}, b0i[1] = {0.0};
  int col;
  const GJResult g =
      gauss_jordan_rhs<GROUP, NMAX, 1, false>(ar, ai, b0r, b0i, 0, n, m, ur, ui, col, nullptr);
  dre = g.dre;
  dim = g.dim;
}

}  // namespace kern
}  // namespace mhc
