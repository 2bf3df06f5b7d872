// Per-pair determinants at sampled (t, i, j): the test hook of mhc_contract
// for shapes where the dense [T][n_src][n_snk] table does not fit.
//
// Each sampled pair is evaluated by the method's own arithmetic with the
// device routines of the contraction kernels, reading G straight from S in
// global memory (the entries are few and scattered over slices, so nothing
// is staged in LDS):
//  * plain (Sec. 2, LU route): d = prod_f det G_f^(ij), one pivoted LU per
//    block;
//  * update tree (Secs. 2-3): the blocks of the owner dominator d with sink
//    j are factorised; for a child i that differs from d in row r of block
//    f, det G_f^(ij) = det G_f^(dj) * (s . x) with x = G_f^(dj)^-1 e_r and
//    s the child's row r (matrix determinant lemma), every other block is
//    the dominator's; a dominator block with an exactly zero pivot has no
//    inverse, and the child's block is then factorised directly, as in the
//    contraction kernels; with set edges the child's blocks are the
//    dominator's (one row replaced) up to a row permutation, whose sign
//    multiplies the result.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "contract_kernels.h"
#include "group_device.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

namespace {

constexpr int kPairBlock = 256;

// Byte offset of row a of S_t in global memory, from the plan's row offset
// a * (M + 1) * 16 into the padded LDS copy.
__device__ __forceinline__ uint32_t global_row(uint32_t lds_off, int M) {
  return lds_off / (uint32_t)(lds_row(M) * 16) * (uint32_t)(M * 16);
}

struct PairIndex {
  int t, i, j;
  bool ok;
};

__device__ __forceinline__ PairIndex read_pair(const PairArgs& a, int q) {
  PairIndex x{0, 0, 0, false};
  if (q < a.n_pairs) {
    x.t = a.pairs[3 * (size_t)q];
    x.i = a.pairs[3 * (size_t)q + 1];
    x.j = a.pairs[3 * (size_t)q + 2];
    x.ok = x.t >= 0 && x.t < a.T && x.i >= 0 && x.i < a.plan.n_src && x.j >= 0 &&
           x.j < a.plan.n_snk;
  }
  if (!x.ok) x.t = x.i = x.j = 0;   // evaluate a valid pair, write NaN
  return x;
}

__device__ __forceinline__ void cmul(double& ar, double& ai, double br, double bi) {
  const double t = ar * br - ai * bi;
  ai = ar * bi + ai * br;
  ar = t;
}

// One matrix per lane (every block of size N <= 8).
template <int N, bool TREE, int PIV>
__global__ __launch_bounds__(kPairBlock) void pair_lane_kernel(PairArgs a) {
  const int q = blockIdx.x * kPairBlock + threadIdx.x;
  const PairIndex x = read_pair(a, q);
  const PlanView& p = a.plan;
  const char* base = reinterpret_cast<const char*>(a.S + (size_t)x.t * p.M * p.M);
  const int d = TREE ? p.term_owner[x.i] : x.i;
  const int fr = TREE ? p.term_fr[x.i] : -1;
  const int fc = fr >= 0 ? (fr >> 8) & 0xff : -1;
  const int rc = fr & 0xff;
  const double sg = (fr >= 0 && (fr >> 16) & 1) ? -1.0 : 1.0;   // odd row permutation
  double Dre = 1.0, Dim = 0.0;
  for (int f = 0; f < p.F; ++f) {
    const int o = p.off[f];
    uint32_t ro[N], co[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      ro[n] = global_row(p.src_rowoff[(size_t)d * p.sn + o + n], p.M);
      co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + x.j];
    }
    double gr[N][N], gi[N][N];
    double dre, dim;
    bool zero;
    lu_crout<N, TREE, PIV>(base, ro, co, gr, gi, dre, dim, zero);
    if (TREE && f == fc) {
      const uint32_t crow = global_row(p.term_crow[x.i], p.M);
      if (zero) {
        // no inverse: the child's block by direct LU
        uint32_t rc2[N], co2[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
          rc2[n] = (n == rc) ? crow : ro[n];
          co2[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + x.j];
        }
        double hr[N][N], hi[N][N];
        bool z2;
        lu_crout<N, false, PIV>(base, rc2, co2, hr, hi, dre, dim, z2);
      } else {
        double rr = 0.0, ri = 0.0;
        solve_unit_col<N>(gr, gi, rc, 0, [&](const double (&xr)[N], const double (&xi)[N]) {
#pragma unroll
          for (int n = 0; n < N; ++n) {
            const double2 s = *reinterpret_cast<const double2*>(base + crow + co[n]);
            rr = rr + s.x * xr[n] - s.y * xi[n];
            ri = ri + s.x * xi[n] + s.y * xr[n];
          }
        });
        const double cr = rr * dre - ri * dim, ci = rr * dim + ri * dre;
        dre = cr;
        dim = ci;
      }
    }
    cmul(Dre, Dim, dre, dim);
  }
  if (q < a.n_pairs)
    a.out[q] = x.ok ? make_double2(sg * Dre, sg * Dim) : make_double2(NAN, NAN);
}

// One group of GROUP lanes per matrix, one row per lane (blocks up to NMAX,
// sizes may differ per flavour), as in the group contraction kernels: the
// elimination carries e_r of the changed row as its right-hand side.
template <int GROUP, int NMAX, bool TREE>
__global__ __launch_bounds__(kPairBlock) void pair_group_kernel(PairArgs a) {
  const int q = (blockIdx.x * kPairBlock + threadIdx.x) / GROUP;
  const int m = threadIdx.x % GROUP;
  const PairIndex x = read_pair(a, q);
  const PlanView& p = a.plan;
  const char* base = reinterpret_cast<const char*>(a.S + (size_t)x.t * p.M * p.M);
  const int d = TREE ? p.term_owner[x.i] : x.i;
  const int fr = TREE ? p.term_fr[x.i] : -1;
  const int fc = fr >= 0 ? (fr >> 8) & 0xff : -1;
  const int rc = fr & 0xff;
  const double sg = (fr >= 0 && (fr >> 16) & 1) ? -1.0 : 1.0;   // odd row permutation
  double Dre = 1.0, Dim = 0.0;
  for (int f = 0; f < p.F; ++f) {
    const int o = p.off[f];
    const int n = p.off[f + 1] - o;
    uint32_t co[NMAX];
#pragma unroll
    for (int c = 0; c < NMAX; ++c)
      co[c] = c < n ? p.snk_coloff[(size_t)(o + c) * p.n_snk_pad + x.j] : 0u;
    const uint32_t myrow = m < n ? global_row(p.src_rowoff[(size_t)d * p.sn + o + m], p.M) : 0u;
    double ar[NMAX], ai[NMAX];
#pragma unroll
    for (int c = 0; c < NMAX; ++c) {
      ar[c] = 0.0;
      ai[c] = 0.0;
      if (c < n && m < n) {
        const double2 v = *reinterpret_cast<const double2*>(base + myrow + co[c]);
        ar[c] = v.x;
        ai[c] = v.y;
      }
    }
    // the changed row's unit column rides along as the one right-hand side
    double ur, ui, b0r[1] = {(TREE && f == fc && m == rc) ? 1.0 : 0.0}, b0i[1] = {0.0};
    int col;
    const GJResult res = gauss_jordan_rhs<GROUP, NMAX, 1, false>(
        ar, ai, b0r, b0i, (TREE && f == fc) ? 1 : 0, n, m, ur, ui, col, nullptr);
    double dre = res.dre, dim = res.dim;
    if (TREE && f == fc) {
      const uint32_t crow = global_row(p.term_crow[x.i], p.M);
      if (res.zero) {
        block_det_direct<GROUP, NMAX>(base, myrow, rc, crow, co, n, m, dre, dim);
      } else {
        // x = G^-1 e_r: x[col_m] = b'[m] / u_m
        const double x_r = b0r[0] * ur - b0i[0] * ui;
        const double x_i = b0r[0] * ui + b0i[0] * ur;
        uint32_t mycol = 0;
#pragma unroll
        for (int c = 0; c < NMAX; ++c)
          if (c == col) mycol = co[c];
        double pr_ = 0.0, pi_ = 0.0;
        if (m < n) {
          const double2 s = *reinterpret_cast<const double2*>(base + crow + mycol);
          pr_ = s.x * x_r - s.y * x_i;
          pi_ = s.x * x_i + s.y * x_r;
        }
        const double rr = group_sum<GROUP>(pr_);
        const double ri = group_sum<GROUP>(pi_);
        const double cr = rr * dre - ri * dim, ci = rr * dim + ri * dre;
        dre = cr;
        dim = ci;
      }
    }
    cmul(Dre, Dim, dre, dim);
  }
  if (q < a.n_pairs && m == 0)
    a.out[q] = x.ok ? make_double2(sg * Dre, sg * Dim) : make_double2(NAN, NAN);
}

template <int N, bool TREE>
hipError_t launch_lane_piv(const PairArgs& a, int pivot, hipStream_t s) {
  const dim3 grid((a.n_pairs + kPairBlock - 1) / kPairBlock);
  if (pivot == 0)
    hipLaunchKernelGGL((pair_lane_kernel<N, TREE, kNoPivot>), grid, dim3(kPairBlock), 0, s, a);
  else if (pivot == 2)
    hipLaunchKernelGGL((pair_lane_kernel<N, TREE, kThresholdPivot>), grid, dim3(kPairBlock), 0,
                       s, a);
  else
    hipLaunchKernelGGL((pair_lane_kernel<N, TREE, kPartialPivot>), grid, dim3(kPairBlock), 0, s,
                       a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_lane_n(const PairArgs& a, bool tree, int pivot, hipStream_t s) {
  return tree ? launch_lane_piv<N, true>(a, pivot, s) : launch_lane_piv<N, false>(a, pivot, s);
}

template <int GROUP, int NMAX>
hipError_t launch_group(const PairArgs& a, bool tree, hipStream_t s) {
  constexpr int per_block = kPairBlock / GROUP;
  const dim3 grid((a.n_pairs + per_block - 1) / per_block);
  if (tree)
    hipLaunchKernelGGL((pair_group_kernel<GROUP, NMAX, true>), grid, dim3(kPairBlock), 0, s, a);
  else
    hipLaunchKernelGGL((pair_group_kernel<GROUP, NMAX, false>), grid, dim3(kPairBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pairs(const PairArgs& a, int n, bool narrow, bool tree, int pivot,
                        hipStream_t s) {
  if (a.n_pairs <= 0) return hipSuccess;
  if (narrow) {
    switch (n) {
      case 1: return launch_lane_n<1>(a, tree, pivot, s);
      case 2: return launch_lane_n<2>(a, tree, pivot, s);
      case 3: return launch_lane_n<3>(a, tree, pivot, s);
      case 4: return launch_lane_n<4>(a, tree, pivot, s);
      case 5: return launch_lane_n<5>(a, tree, pivot, s);
      case 6: return launch_lane_n<6>(a, tree, pivot, s);
      case 7: return launch_lane_n<7>(a, tree, pivot, s);
      case 8: return launch_lane_n<8>(a, tree, pivot, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (n <= 8) return launch_group<8, 8>(a, tree, s);
  if (n <= 12) return launch_group<16, 12>(a, tree, s);
  if (n <= 16) return launch_group<16, 16>(a, tree, s);
  if (n <= 18) return launch_group<32, 18>(a, tree, s);
  if (n <= 24) return launch_group<32, 24>(a, tree, s);
  return hipErrorInvalidValue;
}

}  // namespace kern
}  // namespace mhc
