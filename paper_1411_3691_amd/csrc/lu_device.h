// Device building blocks shared by the forward and adjoint kernels:
// LDS gather of a flavour block, pivoted complex LU in registers (one matrix
// per lane), unit-vector solves, reciprocal, wave reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mhc {
namespace kern {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// 1 / (pr + i pi) with the magnitude mag = |pr| + |pi| known.  Scaled by a
// power of two so that |pr|^2 + |pi|^2 can neither overflow nor underflow
// (it then lies in [1/8, 1)); a zero pivot gives 0 (the clamp of the scaled
// norm keeps 0 * (1/norm) finite).
__device__ __forceinline__ void cinv(double pr, double pi, double mag,
                                     double& vr, double& vi) {
  const int e = __builtin_amdgcn_frexp_exp(mag);
  const double a = __builtin_amdgcn_ldexp(pr, -e);
  const double b = __builtin_amdgcn_ldexp(pi, -e);
  const double d = fmax(a * a + b * b, 0.125);
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  vr = __builtin_amdgcn_ldexp(a * r, -e);
  vi = __builtin_amdgcn_ldexp(-b * r, -e);
}

// |re + i im|, with both parts scaled by a power of two before squaring so
// that neither square overflows nor underflows (determinants of decayed
// propagators reach 1e-260 and below, where re * re is no longer a normal
// double).  frexp_exp(0) is 0, so a zero argument gives 0.
__device__ __forceinline__ double cabs_scaled(double re, double im) {
  const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(re), fabs(im)));
  const double a = __builtin_amdgcn_ldexp(re, -e);
  const double b = __builtin_amdgcn_ldexp(im, -e);
  return __builtin_amdgcn_ldexp(sqrt(a * a + b * b), e);
}

// The LDS copy of S_t keeps rows of M + 1 complex numbers (one unused):
// with a stride of M * 16 bytes (a multiple of 128 for M = 12 k) the lanes
// that read one column of different rows would all hit the same banks.
__host__ __device__ constexpr int lds_row(int M) { return M + 1; }
__host__ __device__ constexpr size_t lds_slice_bytes(int M) {
  return (size_t)M * lds_row(M) * 16;
}

// Copies S_t (M x M, row-major) into the padded LDS layout.
__device__ __forceinline__ void stage_slice(const double2* St, double2* smem, int M, int nthreads) {
  const int ld = lds_row(M);
  const int dr = nthreads / M, dc = nthreads % M;
  for (int r = threadIdx.x / M, c = threadIdx.x % M; r < M;) {
    smem[r * ld + c] = St[r * M + c];
    r += dr;
    c += dc;
    if (c >= M) {
      c -= M;
      ++r;
    }
  }
}

// G[m][n] = S_t[row_m][col_n]: rowoff/coloff are byte offsets into the LDS
// copy of S_t (row * (M + 1) * 16 and col * 16).
template <int N>
__device__ __forceinline__ void gather(const char* lds, const uint32_t (&rowoff)[N],
                                       const uint32_t (&coloff)[N],
                                       double (&gr)[N][N], double (&gi)[N][N]) {
#pragma unroll
  for (int m = 0; m < N; ++m)
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const double2 v = *reinterpret_cast<const double2*>(lds + rowoff[m] + coloff[n]);
      gr[m][n] = v.x;
      gi[m][n] = v.y;
    }
}

// Exchange of two rows (or columns) in the lanes of `mask` only: a <- b,
// b <- t, where t holds a's old value.  The EXEC mask is narrowed and restored inside one
// straight-line asm block, so the compiler sees no branch.  Every operand,
// t included, is a read-write register operand: outputs never share a
// register, so no value the block reads can sit in a register it has
// already written.  The block writes SCC.
__device__ __forceinline__ void masked_exchange1(uint64_t mask, double (&a)[2], double (&b)[2],
                                                 double (&t)[2]) {
  uint64_t sv;
  asm("s_and_saveexec_b64 %[sv], %[mask]\n\t"
      "v_mov_b64 %[a0], %[b0]\n\t"
      "v_mov_b64 %[a1], %[b1]\n\t"
      "v_mov_b64 %[b0], %[t0]\n\t"
      "v_mov_b64 %[b1], %[t1]\n\t"
      "s_mov_b64 exec, %[sv]"
      : [a0] "+v"(a[0]), [a1] "+v"(a[1]), [b0] "+v"(b[0]), [b1] "+v"(b[1]),
        [t0] "+v"(t[0]), [t1] "+v"(t[1]), [sv] "=&s"(sv)
      : [mask] "s"(mask)
      : "scc");
}

// The same for three complex elements (q = 2 * element + re/im).
__device__ __forceinline__ void masked_exchange3(uint64_t mask, double (&a)[6], double (&b)[6],
                                                 double (&t)[6]) {
  uint64_t sv;
  asm("s_and_saveexec_b64 %[sv], %[mask]\n\t"
      "v_mov_b64 %[a0], %[b0]\n\t"
      "v_mov_b64 %[a1], %[b1]\n\t"
      "v_mov_b64 %[a2], %[b2]\n\t"
      "v_mov_b64 %[a3], %[b3]\n\t"
      "v_mov_b64 %[a4], %[b4]\n\t"
      "v_mov_b64 %[a5], %[b5]\n\t"
      "v_mov_b64 %[b0], %[t0]\n\t"
      "v_mov_b64 %[b1], %[t1]\n\t"
      "v_mov_b64 %[b2], %[t2]\n\t"
      "v_mov_b64 %[b3], %[t3]\n\t"
      "v_mov_b64 %[b4], %[t4]\n\t"
      "v_mov_b64 %[b5], %[t5]\n\t"
      "s_mov_b64 exec, %[sv]"
      : [a0] "+v"(a[0]), [a1] "+v"(a[1]), [a2] "+v"(a[2]), [a3] "+v"(a[3]), [a4] "+v"(a[4]),
        [a5] "+v"(a[5]), [b0] "+v"(b[0]), [b1] "+v"(b[1]), [b2] "+v"(b[2]), [b3] "+v"(b[3]),
        [b4] "+v"(b[4]), [b5] "+v"(b[5]), [t0] "+v"(t[0]), [t1] "+v"(t[1]), [t2] "+v"(t[2]),
        [t3] "+v"(t[3]), [t4] "+v"(t[4]), [t5] "+v"(t[5]), [sv] "=&s"(sv)
      : [mask] "s"(mask)
      : "scc");
}

__device__ __forceinline__ void masked_exchange_i32(uint64_t mask, int& a, int& b, int& t) {
  uint64_t sv;
  asm("s_and_saveexec_b64 %[sv], %[mask]\n\t"
      "v_mov_b32 %[a], %[b]\n\t"
      "v_mov_b32 %[b], %[t]\n\t"
      "s_mov_b64 exec, %[sv]"
      : [a] "+v"(a), [b] "+v"(b), [t] "+v"(t), [sv] "=&s"(sv)
      : [mask] "s"(mask)
      : "scc");
}

// |Re| + |Im| with the row's rank packed into the three lowest mantissa
// bits, so that one max over rows yields the pivot magnitude and row, the
// lowest row winning among equal magnitudes (magnitudes that differ only
// in those bits count as equal).
__device__ __forceinline__ double pivot_key(double re, double im, int m) {
  const double mag = fabs(re) + fabs(im);
  const uint32_t lo = (__double2loint(mag) & ~7u) | (uint32_t)(7 - m);
  return __hiloint2double(__double2hiint(mag), (int)lo);
}

// Gaussian elimination with partial pivoting in registers (pivot = largest
// |Re| + |Im| of the remaining column, lowest row on ties).  Each lane holds
// its own matrix and the pivot row differs from lane to lane: row k is
// saved, then for every candidate row m the lanes that chose m move row m
// into row k and the saved row into row m.
// KEEP: store the multipliers (L, unit diagonal), exchange them with their
// rows (so that P G = L U), replace U_kk by 1/U_kk once it has entered the
// determinant, and keep the permutation (perm[m] = original row now in
// position m).  Returns det = sgn(P) prod U_kk and whether some pivot was
// exactly zero.
// PIVOT = false (an ablation of the paper's unpivoted 6x6 LU, Sec. 4):
// the pivot of step k is the diagonal entry, no rows are exchanged.
// THRESH = true (threshold partial pivoting, a variant): the diagonal entry
// stays the pivot unless it is below kThreshold times the column's largest
// |Re|+|Im|; the growth per step is then at most 1 + 1/kThreshold, and rows
// move only where a lane needs it (a step no lane pivots in is skipped).
constexpr double kThreshold = 0.1;

// TAGS (with KEEP): perm holds a caller's tag per row on entry (a row's
// LDS offset, say) and the tags move with their rows, so that perm[m] is
// the tag of the row now in position m.
template <int N, bool KEEP, bool PIVOT = true, bool THRESH = false, bool TAGS = false>
__device__ __forceinline__ void lu(double (&gr)[N][N], double (&gi)[N][N],
                                   double& dre, double& dim, int (&perm)[N],
                                   bool& zero_pivot) {
  static_assert(N <= 8, "row rank is packed into 3 bits");
  double sre = 1.0, sim = 0.0;
  bool neg = false;
  zero_pivot = false;
  if (KEEP && !TAGS) {
#pragma unroll
    for (int m = 0; m < N; ++m) perm[m] = m;
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (PIVOT) {
    double key = pivot_key(gr[k][k], gi[k][k], k);
#pragma unroll
    for (int m = k + 1; m < N; ++m) key = fmax(key, pivot_key(gr[m][k], gi[m][k], m));
    int p = 7 - (int)(__double2loint(key) & 7u);
    if (THRESH) {
      const double dmag = fabs(gr[k][k]) + fabs(gi[k][k]);
      if (dmag >= kThreshold * key) p = k;
    }
    // Row exchange k <-> p: row k's old value is saved, then for each
    // candidate row m the lanes that chose m move row m into row k and the
    // saved row into row m (the L part too when the factors are kept).
    if (k + 1 < N && (!THRESH || __builtin_amdgcn_ballot_w64(p != k) != 0)) {
      const int jb = KEEP ? 0 : k;
      double tr[N], ti[N];
      int tp = 0;
#pragma unroll
      for (int j = jb; j < N; ++j) {
        tr[j] = gr[k][j];
        ti[j] = gi[k][j];
      }
      if (KEEP) tp = perm[k];
#pragma unroll
      for (int m = k + 1; m < N; ++m) {
        const uint64_t mask = __builtin_amdgcn_ballot_w64(p == m);
        if (THRESH && mask == 0) continue;
#pragma unroll
        for (int j = jb; j < N; j += 3) {
          if (j + 2 < N) {
            double a6[6] = {gr[k][j], gi[k][j], gr[k][j + 1], gi[k][j + 1], gr[k][j + 2], gi[k][j + 2]};
            double b6[6] = {gr[m][j], gi[m][j], gr[m][j + 1], gi[m][j + 1], gr[m][j + 2], gi[m][j + 2]};
            double t6[6] = {tr[j], ti[j], tr[j + 1], ti[j + 1], tr[j + 2], ti[j + 2]};
            masked_exchange3(mask, a6, b6, t6);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              gr[k][j + q] = a6[2 * q];
              gi[k][j + q] = a6[2 * q + 1];
              gr[m][j + q] = b6[2 * q];
              gi[m][j + q] = b6[2 * q + 1];
              tr[j + q] = t6[2 * q];
              ti[j + q] = t6[2 * q + 1];
            }
          } else {
#pragma unroll
            for (int jj = j; jj < N; ++jj) {
              double a2[2] = {gr[k][jj], gi[k][jj]};
              double b2[2] = {gr[m][jj], gi[m][jj]};
              double t2[2] = {tr[jj], ti[jj]};
              masked_exchange1(mask, a2, b2, t2);
              gr[k][jj] = a2[0];
              gi[k][jj] = a2[1];
              gr[m][jj] = b2[0];
              gi[m][jj] = b2[1];
              tr[jj] = t2[0];
              ti[jj] = t2[1];
            }
          }
        }
        if (KEEP) masked_exchange_i32(mask, perm[k], perm[m], tp);
      }
    }
    neg = neg != (p != k);
    }
    const double pr = gr[k][k], pi = gi[k][k];
    const double mag = fabs(pr) + fabs(pi);
    zero_pivot = zero_pivot || (mag == 0.0);
    const double t = sre * pr - sim * pi;
    sim = sre * pi + sim * pr;
    sre = t;
    if (KEEP || k + 1 < N) {
      double vr, vi;
      cinv(pr, pi, mag, vr, vi);
      if (KEEP) {
        gr[k][k] = vr;
        gi[k][k] = vi;
      }
#pragma unroll
      for (int m = k + 1; m < N; ++m) {
        const double lr = gr[m][k] * vr - gi[m][k] * vi;
        const double li = gr[m][k] * vi + gi[m][k] * vr;
        if (KEEP) {
          gr[m][k] = lr;
          gi[m][k] = li;
        }
#pragma unroll
        for (int j = k + 1; j < N; ++j) {
          gr[m][j] = gr[m][j] - lr * gr[k][j] + li * gi[k][j];
          gi[m][j] = gi[m][j] - lr * gi[k][j] - li * gr[k][j];
        }
      }
    }
  }
  dre = neg ? -sre : sre;
  dim = neg ? -sim : sim;
}

// x = G^-1 e_r from the factors of lu<N, true>: solve L y = P e_r (P e_r is
// the unit vector at the position q with perm[q] == r), then U x = y (the
// diagonal of the factors holds 1/U_mm).
template <int N>
__device__ __forceinline__ void solve_unit(const double (&gr)[N][N],
                                           const double (&gi)[N][N],
                                           const int (&perm)[N], int r,
                                           double (&xr)[N], double (&xi)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) {
    double br = perm[m] == r ? 1.0 : 0.0, bi = 0.0;
#pragma unroll
    for (int j = 0; j < m; ++j) {
      br = br - gr[m][j] * xr[j] + gi[m][j] * xi[j];
      bi = bi - gr[m][j] * xi[j] - gi[m][j] * xr[j];
    }
    xr[m] = br;
    xi[m] = bi;
  }
#pragma unroll
  for (int m = N - 1; m >= 0; --m) {
    double br = xr[m], bi = xi[m];
#pragma unroll
    for (int j = m + 1; j < N; ++j) {
      br = br - gr[m][j] * xr[j] + gi[m][j] * xi[j];
      bi = bi - gr[m][j] * xi[j] - gi[m][j] * xr[j];
    }
    xr[m] = br * gr[m][m] - bi * gi[m][m];
    xi[m] = br * gi[m][m] + bi * gr[m][m];
  }
}

// b with h^T G^-1 = b^T P (that is (h^T G^-1)[perm[m]] = b[m]) from the
// factors of lu<N, true> (P G = L U, diagonal holding 1/U_mm): a^T U = h^T,
// then b^T L = a^T.  (br, bi) holds h on entry.
template <int N>
__device__ __forceinline__ void solve_row(const double (&gr)[N][N], const double (&gi)[N][N],
                                          double (&br)[N], double (&bi)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double tr = br[j], ti = bi[j];
#pragma unroll
    for (int i = 0; i < j; ++i) {
      tr = tr - br[i] * gr[i][j] + bi[i] * gi[i][j];
      ti = ti - br[i] * gi[i][j] - bi[i] * gr[i][j];
    }
    br[j] = tr * gr[j][j] - ti * gi[j][j];
    bi[j] = tr * gi[j][j] + ti * gr[j][j];
  }
#pragma unroll
  for (int j = N - 2; j >= 0; --j) {
    double tr = br[j], ti = bi[j];
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      tr = tr - br[i] * gr[i][j] + bi[i] * gi[i][j];
      ti = ti - br[i] * gi[i][j] - bi[i] * gr[i][j];
    }
    br[j] = tr;
    bi[j] = ti;
  }
}

// V = U^-1 L^-1 in place from the factors of lu<N, true> (P A = L U, unit L
// below the diagonal, 1/U_mm on it), so that A^-1 = V P, that is
// A^-1[a][perm[q]] = V[a][q].  First U^-1 over the upper triangle, column
// by column (U^-1[i][j] = -(sum_{i<=k<j} U^-1[i][k] U[k][j]) / U_jj, rows
// in increasing order so that U[k][j], k > i, is still unchanged), then
// V L = U^-1 column by column from the right (V[:, j] = U^-1[:, j] -
// sum_{k>j} V[:, k] L[k][j], with L[k][j] saved before column j is
// overwritten).
template <int N>
__device__ __forceinline__ void lu_inverse_v(double (&gr)[N][N], double (&gi)[N][N]) {
#pragma unroll
  for (int j = 1; j < N; ++j)
#pragma unroll
    for (int i = 0; i < j; ++i) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int k = i; k < j; ++k) {
        sr += gr[i][k] * gr[k][j] - gi[i][k] * gi[k][j];
        si += gr[i][k] * gi[k][j] + gi[i][k] * gr[k][j];
      }
      gr[i][j] = -(sr * gr[j][j] - si * gi[j][j]);
      gi[i][j] = -(sr * gi[j][j] + si * gr[j][j]);
    }
#pragma unroll
  for (int j = N - 2; j >= 0; --j) {
    double lr[N], li[N];
#pragma unroll
    for (int k = j + 1; k < N; ++k) {
      lr[k] = gr[k][j];
      li[k] = gi[k][j];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double vr = i <= j ? gr[i][j] : 0.0, vi = i <= j ? gi[i][j] : 0.0;
#pragma unroll
      for (int k = j + 1; k < N; ++k) {
        vr = vr - gr[i][k] * lr[k] + gi[i][k] * li[k];
        vi = vi - gr[i][k] * li[k] - gi[i][k] * lr[k];
      }
      gr[i][j] = vr;
      gi[i][j] = vi;
    }
  }
}

__device__ __forceinline__ void masked_exchange_u32(uint64_t mask, uint32_t& a, uint32_t& b,
                                                   uint32_t& t) {
  uint64_t sv;
  asm("s_and_saveexec_b64 %[sv], %[mask]\n\t"
      "v_mov_b32 %[a], %[b]\n\t"
      "v_mov_b32 %[b], %[t]\n\t"
      "s_mov_b64 exec, %[sv]"
      : [a] "+v"(a), [b] "+v"(b), [t] "+v"(t), [sv] "=&s"(sv)
      : [mask] "s"(mask)
      : "scc");
}

// Pivot rule of lu_crout.
enum PivotRule { kNoPivot = 0, kPartialPivot = 1, kThresholdPivot = 2 };

// LU of the block G[m][n] = S_t[row m][col n] in Crout order with column
// pivoting, gathering G from LDS as the factorisation needs it (rowoff,
// coloff: byte offsets as for gather).  Step k forms row k of U (columns
// k..N-1) from the original row k, read in the current column order, minus
// its products with the finished rows 0..k-1 of U; the pivot is that row's
// largest |Re| + |Im| (lowest column on ties); then column k of L is formed
// from the original column k, read in the new order.  Because the rows
// below k are still in LDS, a column exchange moves only rows 0..k and the
// column offset: k + 1 complex entries instead of the N of a row exchange
// in right-looking elimination, and no permutation vector is kept.
// On return coloff holds the column order of the factors (G Q = L U, Q the
// exchange of the original columns into that order); the strict lower
// triangle holds L (unit diagonal), the upper triangle U, and with KEEP
// the diagonal holds 1/U_mm.  det = sgn(Q) prod U_mm; zero_pivot reports an
// exactly zero pivot (the row it occurs in is then zero from column k on).
// kThresholdPivot keeps the diagonal candidate unless it is below
// kThreshold times the row's largest entry and skips the exchange when no
// lane of the wave needs it.  kNoPivot reads the whole block first and
// eliminates right-looking (no exchanges, so nothing is gained by reading
// late), leaving coloff and the factor layout as above.
template <int N, bool KEEP, int PIV>
__device__ __forceinline__ void lu_crout(const char* lds, const uint32_t (&rowoff)[N],
                                         uint32_t (&coloff)[N], double (&gr)[N][N],
                                         double (&gi)[N][N], double& dre, double& dim,
                                         bool& zero_pivot) {
  static_assert(N <= 8, "column rank is packed into 3 bits");
  if constexpr (PIV == kNoPivot) {
    int perm[N];
    gather<N>(lds, rowoff, coloff, gr, gi);
    lu<N, KEEP, false>(gr, gi, dre, dim, perm, zero_pivot);
    return;
  }
  double sre = 1.0, sim = 0.0;
  bool neg = false;
  zero_pivot = false;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    // Row k of U: u_j = G[k][j] - sum_{i<k} L[k][i] U[i][j], j >= k.
#pragma unroll
    for (int j = k; j < N; ++j) {
      const double2 v = *reinterpret_cast<const double2*>(lds + rowoff[k] + coloff[j]);
      double ur = v.x, ui = v.y;
#pragma unroll
      for (int i = 0; i < k; ++i) {
        ur = ur - gr[k][i] * gr[i][j] + gi[k][i] * gi[i][j];
        ui = ui - gr[k][i] * gi[i][j] - gi[k][i] * gr[i][j];
      }
      gr[k][j] = ur;
      gi[k][j] = ui;
    }
    if (k + 1 < N) {
      double key = pivot_key(gr[k][k], gi[k][k], k);
#pragma unroll
      for (int j = k + 1; j < N; ++j) key = fmax(key, pivot_key(gr[k][j], gi[k][j], j));
      int p = 7 - (int)(__double2loint(key) & 7u);
      if (PIV == kThresholdPivot) {
        const double dmag = fabs(gr[k][k]) + fabs(gi[k][k]);
        if (dmag >= kThreshold * key) p = k;
      }
      // Exchange columns k and p in rows 0..k: column k's entries are
      // saved, then for each candidate m the lanes that chose m move column
      // m into column k and the saved entries into column m.
      if (PIV == kPartialPivot || __builtin_amdgcn_ballot_w64(p != k) != 0) {
        double tr[N], ti[N];
        uint32_t tc = coloff[k];
#pragma unroll
        for (int i = 0; i <= k; ++i) {
          tr[i] = gr[i][k];
          ti[i] = gi[i][k];
        }
#pragma unroll
        for (int m = k + 1; m < N; ++m) {
          const uint64_t mask = __builtin_amdgcn_ballot_w64(p == m);
          if (PIV == kThresholdPivot && mask == 0) continue;
#pragma unroll
          for (int i = 0; i <= k; i += 3) {
            if (i + 2 <= k) {
              double a6[6] = {gr[i][k], gi[i][k], gr[i + 1][k], gi[i + 1][k], gr[i + 2][k], gi[i + 2][k]};
              double b6[6] = {gr[i][m], gi[i][m], gr[i + 1][m], gi[i + 1][m], gr[i + 2][m], gi[i + 2][m]};
              double t6[6] = {tr[i], ti[i], tr[i + 1], ti[i + 1], tr[i + 2], ti[i + 2]};
              masked_exchange3(mask, a6, b6, t6);
#pragma unroll
              for (int q = 0; q < 3; ++q) {
                gr[i + q][k] = a6[2 * q];
                gi[i + q][k] = a6[2 * q + 1];
                gr[i + q][m] = b6[2 * q];
                gi[i + q][m] = b6[2 * q + 1];
                tr[i + q] = t6[2 * q];
                ti[i + q] = t6[2 * q + 1];
              }
            } else {
#pragma unroll
              for (int ii = i; ii <= k; ++ii) {
                double a2[2] = {gr[ii][k], gi[ii][k]};
                double b2[2] = {gr[ii][m], gi[ii][m]};
                double t2[2] = {tr[ii], ti[ii]};
                masked_exchange1(mask, a2, b2, t2);
                gr[ii][k] = a2[0];
                gi[ii][k] = a2[1];
                gr[ii][m] = b2[0];
                gi[ii][m] = b2[1];
                tr[ii] = t2[0];
                ti[ii] = t2[1];
              }
            }
          }
          masked_exchange_u32(mask, coloff[k], coloff[m], tc);
        }
      }
      neg = neg != (p != k);
    }
    const double pr = gr[k][k], pi = gi[k][k];
    const double mag = fabs(pr) + fabs(pi);
    zero_pivot = zero_pivot || (mag == 0.0);
    const double t = sre * pr - sim * pi;
    sim = sre * pi + sim * pr;
    sre = t;
    if (KEEP || k + 1 < N) {
      double vr, vi;
      cinv(pr, pi, mag, vr, vi);
      if (KEEP) {
        gr[k][k] = vr;
        gi[k][k] = vi;
      }
      // Column k of L: l_m = (G[m][k] - sum_{i<k} L[m][i] U[i][k]) / U[k][k].
#pragma unroll
      for (int m = k + 1; m < N; ++m) {
        const double2 v = *reinterpret_cast<const double2*>(lds + rowoff[m] + coloff[k]);
        double ar = v.x, ai = v.y;
#pragma unroll
        for (int i = 0; i < k; ++i) {
          ar = ar - gr[m][i] * gr[i][k] + gi[m][i] * gi[i][k];
          ai = ai - gr[m][i] * gi[i][k] - gi[m][i] * gr[i][k];
        }
        gr[m][k] = ar * vr - ai * vi;
        gi[m][k] = ar * vi + ai * vr;
      }
    }
  }
  dre = neg ? -sre : sre;
  dim = neg ? -sim : sim;
}

// y = G^-1 e_R, in the column order of the factors of lu_crout<N, true>
// (G Q = L U, so G^-1 e_R = Q U^-1 L^-1 e_R: entry m of y belongs to the
// factors' column position m).  L^-1 e_R is zero above row R and 1 at R, so
// the forward part starts there; R is a compile-time row.
// Every entry of y depends on the first value formed (y_{R+1} of the
// forward part, or y_{N-1} when R = N - 1).  That value passes through an
// empty asm statement that also takes `tag`, a wave-uniform value that
// changes from call to call in the caller's loop: the solve of every R is
// loop-invariant for a given factorisation, and without the tie the
// compiler hoists all N of them out of that loop (N solution vectors live
// at once instead of the few solves needed).  The statement is not
// volatile, so it is no memory access and the caller's loads of read-only
// plan data stay scalar loads.
template <int N, int R>
__device__ __forceinline__ void solve_unit_col_r(const double (&gr)[N][N],
                                                 const double (&gi)[N][N], int tag,
                                                 double (&xr)[N], double (&xi)[N]) {
#pragma unroll
  for (int m = R + 1; m < N; ++m) {
    double br = -gr[m][R], bi = -gi[m][R];
#pragma unroll
    for (int j = R + 1; j < m; ++j) {
      br = br - gr[m][j] * xr[j] + gi[m][j] * xi[j];
      bi = bi - gr[m][j] * xi[j] - gi[m][j] * xr[j];
    }
    if (m == R + 1) asm("" : "+v"(br), "+v"(bi) : "s"(tag));
    xr[m] = br;
    xi[m] = bi;
  }
#pragma unroll
  for (int m = N - 1; m >= 0; --m) {
    double br, bi;
    int j0;
    if (m > R) {
      br = xr[m];
      bi = xi[m];
      j0 = m + 1;
    } else if (m == R) {
      br = 1.0;
      bi = 0.0;
      j0 = m + 1;
      if (m == N - 1) asm("" : "+v"(br), "+v"(bi) : "s"(tag));
    } else {
      br = -(gr[m][m + 1] * xr[m + 1] - gi[m][m + 1] * xi[m + 1]);
      bi = -(gr[m][m + 1] * xi[m + 1] + gi[m][m + 1] * xr[m + 1]);
      j0 = m + 2;
    }
#pragma unroll
    for (int j = j0; j < N; ++j) {
      br = br - gr[m][j] * xr[j] + gi[m][j] * xi[j];
      bi = bi - gr[m][j] * xi[j] - gi[m][j] * xr[j];
    }
    xr[m] = br * gr[m][m] - bi * gi[m][m];
    xi[m] = br * gi[m][m] + bi * gr[m][m];
  }
}

// The same for a wave-uniform runtime row r (0 <= r < N), followed by
// use(xr, xi): one branch per row, each with its own structure and its own
// copy of use, so that no solved vector has to be merged across branches.
template <int N, int R = 0, typename Use>
__device__ __forceinline__ void solve_unit_col(const double (&gr)[N][N],
                                               const double (&gi)[N][N], int r, int tag,
                                               Use&& use) {
  if constexpr (R + 1 < N) {
    if (r != R) {
      solve_unit_col<N, R + 1>(gr, gi, r, tag, use);
      return;
    }
  }
  double xr[N], xi[N];
  solve_unit_col_r<N, R>(gr, gi, tag, xr, xi);
  use(xr, xi);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// A read of plan tables at a wave-uniform index through the constant
// address space, so that it becomes a scalar load (the kernels write
// global memory, and through a generic pointer the compiler keeps such
// reads on the vector path, one memory latency per read).
template <class T>
__device__ __forceinline__ T cload(const T* ptr, long i) {
  static_assert(sizeof(T) % 4 == 0, "read by 32-bit words");
  const __attribute__((address_space(4))) uint32_t* q =
      (const __attribute__((address_space(4))) uint32_t*)(ptr + i);
  T v;
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int w = 0; w < (int)(sizeof(T) / 4); ++w) d[w] = q[w];
  return v;
}

__device__ __forceinline__ int uniform(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace kern
}  // namespace mhc
