// Gauss-Jordan elimination with partial pivoting on matrices held by a
// group of GROUP lanes with ROWS rows per lane (row i of the matrix lives in
// lane i % GROUP, slot i / GROUP).  Several rows per lane let one broadcast
// of the pivot row serve ROWS row updates and keep four lanes busy on a
// 12 x 12 block instead of twelve of sixteen: per step the lanes issue
// ROWS times more multiply-adds against the same chain of pivot search,
// broadcast and reciprocal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "group_device.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

// Complex entries of one group's pivot-row buffer (the row from column k
// on, then the right-hand sides), rounded up to an odd count so that the
// 16-byte reads of the groups of one wave fall in different LDS banks.
template <int NMAX, int RMAX>
constexpr int rows_buf_entries() {
  return (NMAX + RMAX) | 1;
}

// Per-lane state of one elimination: ROWS rows of the matrix (columns <
// NMAX) and of RB right-hand sides (storage; an elimination carries at most
// its RMAX <= RB).
template <int ROWS, int NMAX, int RMAX>
struct RowsBlock {
  double ar[ROWS][NMAX], ai[ROWS][NMAX];
  double br[ROWS][RMAX], bi[ROWS][RMAX];
};

// Largest of a 32-bit value over the GROUP lanes of a group (4 or 8).
template <int GROUP>
__device__ __forceinline__ uint32_t group_max_u32(uint32_t v) {
  static_assert(GROUP == 4 || GROUP == 8 || GROUP == 16, "groups of 4, 8 or 16 lanes");
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppXor1, 0xf, 0xf, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppXor2, 0xf, 0xf, false));
  if constexpr (GROUP >= 8)
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppHalfMirror, 0xf, 0xf,
                                                       false));
  if constexpr (GROUP >= 16)
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowMirror, 0xf, 0xf,
                                                       false));
  return v;
}

// Pivot rows of the steps of one elimination, 5 bits each.
template <int NMAX>
struct PivotRows {
  uint32_t w[(NMAX + 5) / 6];
  __device__ __forceinline__ int get(int k) const { return (w[k / 6] >> (5 * (k % 6))) & 31; }
};

struct RowsResult {
  double dre, dim;   // det G (the same in every lane of the group)
  bool zero;         // some pivot was exactly zero
};

// Eliminates the group's n x n block (n <= NMAX, the same in every lane of
// the wave; columns n .. NMAX-1 must hold zeros, rows n .. are ignored)
// with RMAX right-hand sides (unused ones may hold anything finite: no
// per-entry guards, so the steps compile without branches).  Step k takes as pivot the
// row not used yet with the largest |Re| + |Im| in column k, lowest row on
// ties (the row index is packed into the low mantissa bits of the key, one
// DPP max over the group); every other row subtracts l_i = a_ik / u times
// the pivot row from its columns above k and from its right-hand sides.
// Rows are relabelled, never moved: the pivot of column k stays in its row,
// and later steps subtract only pivot rows whose column k is already zero,
// so at the end row i reads u_i x[col_i] = b'_q[i].  Every pivot u is the
// row's entry at its own column, and step k writes the pivot row from
// column k on, so after the elimination entry c of the group's buffer holds
// the pivot of step c: rows_pivot_inverse reads it back.
// col[s] is set to the step at which slot s became a pivot row (-1 for
// slots beyond n).  det G = the product of the pivots times the sign of the
// pivot order (the pivots of GEPP).
// KEEP: every row also keeps its multiplier of step k in its column k and
// pivots records the pivot row of every step, so that
// rows_replay can apply the same row operations to more right-hand sides.
template <int GROUP, int ROWS, int NMAX, int RMAX, int RB, bool KEEP = false>
__device__ __forceinline__ RowsResult rows_gauss_jordan(RowsBlock<ROWS, NMAX, RB>& b, int n,
                                                        int m, int (&col)[ROWS],
                                                        double2* buf, PivotRows<NMAX>& pivots) {
  static_assert(GROUP * ROWS >= NMAX, "the group must hold every row");
  static_assert(GROUP * ROWS <= 32 && NMAX <= 24,
                "the row index is packed into 5 bits; open rows < 24 keep keys above 7");
  static_assert(RMAX <= RB, "right-hand sides beyond the block's storage");
  RowsResult res{1.0, 0.0, false};
#pragma unroll
  for (int w = 0; w < (NMAX + 5) / 6; ++w) pivots.w[w] = 0u;
  uint32_t used = 0u;        // bit s: slot s is a pivot row already
  uint32_t parity = 0u;      // this lane's share of the pivot order's inversions
#pragma unroll
  for (int s = 0; s < ROWS; ++s) col[s] = -1;
  static_for<0, NMAX>([&](auto kc) __attribute__((always_inline)) {
    constexpr int k = decltype(kc)::value;
    if (k >= n) return;
    // pivot: largest |Re| + |Im| of column k among the rows not used yet.
    // The key is the magnitude's high word (non-negative doubles order as
    // their bits) with the row in its 5 low bits, so rows within 2^-15 of
    // the largest count as ties, taken lowest row first; closed rows get 0
    // (open rows are < 24, so their keys are >= 8).
    uint32_t key = 0u;
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
      const int i = m + GROUP * s;
      const double mag = fabs(b.ar[s][k]) + fabs(b.ai[s][k]);
      const uint32_t ks = ((uint32_t)__double2hiint(mag) & ~31u) | (uint32_t)(31 - i);
      const bool open = i < n && !((used >> s) & 1u);
      key = max(key, open ? ks : 0u);
    }
    key = group_max_u32<GROUP>(key);
    const int p = 31 - (int)(key & 31u);   // pivot row, < n
    const int lp = p % GROUP, sp = p / GROUP;
    // sign: every row below p that is still open is one transposition of
    // the pivot order
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
      const int i = m + GROUP * s;
      if (i < p && i < n && !((used >> s) & 1u)) parity ^= 1u;
    }
    if (m == lp) {
      static_for<0, ROWS>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        if (s != sp) return;
        // Each value passes an empty statement in its own branch: otherwise
        // the compiler merges the slots' branches into one store of a value
        // read through a computed slot index, which keeps the rows in
        // scratch memory instead of registers.
        static_for<k, NMAX>([&](auto cc) __attribute__((always_inline)) {
          constexpr int c = decltype(cc)::value;
          const double xr = b.ar[s][c], xi = b.ai[s][c];
          asm volatile("" ::"v"(xr), "v"(xi));
          buf[c] = make_double2(xr, xi);
        });
        static_for<0, RMAX>([&](auto qc) __attribute__((always_inline)) {
          constexpr int q = decltype(qc)::value;
          const double xr = b.br[s][q], xi = b.bi[s][q];
          asm volatile("" ::"v"(xr), "v"(xi));
          buf[NMAX + q] = make_double2(xr, xi);
        });
      });
    }
    wave_lds_sync();
    const double2 pv = buf[k];
    const double pmag = fabs(pv.x) + fabs(pv.y);
    res.zero = res.zero || (pmag == 0.0);
    const double t = res.dre * pv.x - res.dim * pv.y;
    res.dim = res.dre * pv.y + res.dim * pv.x;
    res.dre = t;
    double vr, vi;
    cinv(pv.x, pv.y, pmag, vr, vi);   // 0 for a zero pivot
    // multipliers (0 for the pivot row; rows beyond n follow along with
    // finite values and are never read)
    double lr[ROWS], li[ROWS];
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
      const int i = m + GROUP * s;
      const bool piv = i == p;
      const double wr = piv ? 0.0 : vr, wi = piv ? 0.0 : vi;
      lr[s] = b.ar[s][k] * wr - b.ai[s][k] * wi;
      li[s] = b.ar[s][k] * wi + b.ai[s][k] * wr;
      used |= piv ? 1u << s : 0u;
      col[s] = piv ? k : col[s];
      if constexpr (KEEP) {
        // column k is not read again: it keeps the multiplier for replays
        b.ar[s][k] = lr[s];
        b.ai[s][k] = li[s];
      }
    }
    if constexpr (KEEP) pivots.w[k / 6] |= (uint32_t)p << (5 * (k % 6));
    static_for<k + 1, NMAX>([&](auto cc) __attribute__((always_inline)) {
      constexpr int c = decltype(cc)::value;
      const double2 u = buf[c];
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        b.ar[s][c] = b.ar[s][c] - lr[s] * u.x + li[s] * u.y;
        b.ai[s][c] = b.ai[s][c] - lr[s] * u.y - li[s] * u.x;
      }
    });
    static_for<0, RMAX>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      const double2 u = buf[NMAX + q];
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        b.br[s][q] = b.br[s][q] - lr[s] * u.x + li[s] * u.y;
        b.bi[s][q] = b.bi[s][q] - lr[s] * u.y - li[s] * u.x;
      }
    });
    wave_lds_sync();   // the row is read before the next step writes
  });
  // the group's inversions: the sum of the lanes' shares, mod 2
  uint32_t par = parity;
  if constexpr (GROUP >= 2)
    par ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)par, kDppXor1, 0xf, 0xf, false);
  if constexpr (GROUP >= 4)
    par ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)par, kDppXor2, 0xf, 0xf, false);
  if constexpr (GROUP >= 8)
    par ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)par, kDppHalfMirror, 0xf, 0xf, false);
  if constexpr (GROUP >= 16)
    par ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)par, kDppRowMirror, 0xf, 0xf, false);
  static_assert(GROUP <= 16, "parity reduction covers groups of up to 16 lanes");
  if (par & 1u) {
    res.dre = -res.dre;
    res.dim = -res.dim;
  }
  return res;
}

// Applies the row operations of rows_gauss_jordan<..., KEEP> (multipliers
// in the matrix columns, pivot rows in pivots) to RB right-hand sides at
// once: step k subtracts each row's multiplier times the pivot row's
// entries, so that on return the system reads u_i x[col_i] = b'_q[i], as if
// the columns had been carried through the elimination.  One pass serves
// all RB columns: its chain of broadcasts costs a fraction of another
// elimination.  Uses the right-hand-side part of the group's buffer only;
// the pivots in its first entries stay for rows_pivot_inverse.
template <int GROUP, int ROWS, int NMAX, int RB>
__device__ __forceinline__ void rows_replay(RowsBlock<ROWS, NMAX, RB>& b, int n, int m,
                                            const PivotRows<NMAX>& pivots, double2* buf) {
  static_for<0, NMAX>([&](auto kc) __attribute__((always_inline)) {
    constexpr int k = decltype(kc)::value;
    if (k >= n) return;
    const int p = pivots.get(k);
    const int lp = p % GROUP, sp = p / GROUP;
    if (m == lp) {
      static_for<0, ROWS>([&](auto sc) __attribute__((always_inline)) {
        constexpr int s = decltype(sc)::value;
        if (s != sp) return;
        static_for<0, RB>([&](auto qc) __attribute__((always_inline)) {
          constexpr int q = decltype(qc)::value;
          const double xr = b.br[s][q], xi = b.bi[s][q];
          asm volatile("" ::"v"(xr), "v"(xi));
          buf[NMAX + q] = make_double2(xr, xi);
        });
      });
    }
    wave_lds_sync();
    static_for<0, RB>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      const double2 u = buf[NMAX + q];
#pragma unroll
      for (int s = 0; s < ROWS; ++s) {
        b.br[s][q] = b.br[s][q] - b.ar[s][k] * u.x + b.ai[s][k] * u.y;
        b.bi[s][q] = b.bi[s][q] - b.ar[s][k] * u.y - b.ai[s][k] * u.x;
      }
    });
    wave_lds_sync();
  });
}

// 1 / u for slot s's pivot, read back from the group's buffer (entry col of
// the buffer holds the pivot of step col until the next elimination
// writes it).  Slots without a pivot (beyond n) get 0.
__device__ __forceinline__ void rows_pivot_inverse(const double2* buf, int col, double& vr,
                                                   double& vi) {
  vr = 0.0;
  vi = 0.0;
  if (col >= 0) {
    const double2 u = buf[col];
    cinv(u.x, u.y, fabs(u.x) + fabs(u.y), vr, vi);
  }
}

}  // namespace kern
}  // namespace mhc
