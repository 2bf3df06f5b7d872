// HIP kernels for gfx950: gather + pivoted complex LU + update tree +
// weighted reduction of the multi-hadron correlator.
//
// Work decomposition.  A work item is (time slice t, source row-set d, sink
// block of 64).  One wavefront takes one item: lane l handles sink
// k = 64*block + l, and every lane of the wave shares the same source row
// set, so the tree structure (groups, children) is wave-uniform and the
// only per-lane data are the sink's column indices.  A workgroup stages the
// slice's propagator S_t into LDS once and its four waves then walk a
// strided subset of that slice's items; every determinant gathers its
// entries from LDS.
//
//  * plain method (Sec. 2, LU route): the row set is one source term;
//    per flavour block: gather G_f, GEPP, det; d = prod_f det_f.
//  * update tree (Secs. 2-3): the row set is a dominator.  Per flavour
//    block: gather, GEPP keeping L, U and the row permutation; for every
//    group (f, r) of the dominator one solve x = G_f^-1 e_r (forward and
//    back substitution); every child of the group then costs one dot
//    product: det(G with row r := s) = det(G) * (s . x) (matrix determinant
//    lemma, Sec. 2; s . x equals 1 + v^T G^-1 e_r with v = s - old row).
//    Children with the same (f, r) share x (the "caching" of Sec. 2).
//
// The weighted sum over one item folds the flavours incrementally: with
// P = prod of the dets seen so far and Q = sum over seen flavours f of
// acc_f * prod_{f' != f, seen} det_f',  where acc_f = sum_{children c
// changing flavour f} w_c det(child's block f), the item contributes
// w_k * (w_i * P + Q).  A dominator block with an exactly zero pivot has no
// inverse; its children's blocks are then taken by direct LU (counted in the
// plan's fallback counter).
//
// Reductions are deterministic: per-lane sums, a fixed-order wave and
// workgroup reduction, one partial per workgroup, then a fixed-order final
// kernel.  There are no floating-point atomics.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contract_kernels.h"

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

// G[m][n] = S_t[row_m][col_n]: rowoff/coloff are byte offsets into the LDS
// copy of S_t (row * M * 16 and col * 16).
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

// Row exchange in the lanes of `mask` only: a <- b, b <- t, where t holds
// a's old value.  The EXEC mask is narrowed and restored inside one
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
template <int N, bool KEEP>
__device__ __forceinline__ void lu(double (&gr)[N][N], double (&gi)[N][N],
                                   double& dre, double& dim, int (&perm)[N],
                                   bool& zero_pivot) {
  static_assert(N <= 8, "row rank is packed into 3 bits");
  double sre = 1.0, sim = 0.0;
  bool neg = false;
  zero_pivot = false;
  if (KEEP) {
#pragma unroll
    for (int m = 0; m < N; ++m) perm[m] = m;
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double key = pivot_key(gr[k][k], gi[k][k], k);
#pragma unroll
    for (int m = k + 1; m < N; ++m) key = fmax(key, pivot_key(gr[m][k], gi[m][k], m));
    const int p = 7 - (int)(__double2loint(key) & 7u);
    // Row exchange k <-> p: row k's old value is saved, then for each
    // candidate row m the lanes that chose m move row m into row k and the
    // saved row into row m (the L part too when the factors are kept).
    if (k + 1 < N) {
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ int uniform(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}

// Determinant of flavour block f of the pair (row set, sink) with row r
// replaced by the source row `newrow` (byte offset), by direct LU.
template <int N>
__device__ __forceinline__ void child_det_direct(const char* lds,
                                                 const uint32_t* rowoff_dom,
                                                 int r, uint32_t newrow,
                                                 const uint32_t (&coloff)[N],
                                                 double& dre, double& dim) {
  uint32_t ro[N];
#pragma unroll
  for (int m = 0; m < N; ++m) ro[m] = (m == r) ? newrow : rowoff_dom[m];
  double gr[N][N], gi[N][N];
  int perm[N];
  bool z;
  gather<N>(lds, ro, coloff, gr, gi);
  lu<N, false>(gr, gi, dre, dim, perm, z);
}

// MODE bit 0: accumulate A(t) = sum |w w d|; bit 1: write every pair det.
template <int N, bool TREE, int MODE>
__global__ __launch_bounds__(kBlock, 2) void contract_kernel(ContractArgs a) {
  constexpr bool WITH_A = (MODE & 1) != 0;
  constexpr bool WITH_PAIRS = (MODE & 2) != 0;
  extern __shared__ double2 smem[];
  const PlanView& p = a.plan;
  const int t = blockIdx.y;
  const int chunk = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  const int MM = p.M * p.M;

  // Stage S_t into LDS (16 B per lane per step, coalesced).
  const double2* St = a.S + (size_t)t * MM;
  for (int e = threadIdx.x; e < MM; e += kBlock) smem[e] = St[e];
  __syncthreads();
  const char* lds = reinterpret_cast<const char*>(smem);

  double acc_re = 0.0, acc_im = 0.0, acc_a = 0.0;
  uint32_t n_fallback = 0;
  const int F = p.F;
  const int sn = p.sn;

  for (int item = chunk + a.n_blk_t * wave; item < a.n_items;
       item += a.n_blk_t * kWavesPerBlock) {
    const int d = uniform(item / a.n_sblk);
    const int sb = uniform(item - d * a.n_sblk);
    const int k = sb * kWave + lane;
    const bool valid = k < p.n_snk;
    const int term = TREE ? uniform(p.dom_term[d]) : d;
    const uint32_t* rowoff_d = (TREE ? p.dom_rowoff : p.src_rowoff) + (size_t)d * sn;
    const double wi = a.w_src[term];
    const double wk = valid ? a.w_snk[k] : 0.0;
    const int g_begin = TREE ? uniform(p.dom_grp[d]) : 0;
    const int g_end = TREE ? uniform(p.dom_grp[d + 1]) : 0;

    double Pre = 1.0, Pim = 0.0, Qre = 0.0, Qim = 0.0;
    // Diagnostics: sum over children of |w_c * ratio_c| (A) and the
    // product of the dets of blocks without a zero pivot.
    double sabs_reg = 0.0, sabs_fb = 0.0;
    double Xre = 1.0, Xim = 0.0;
    int nbad = 0, fbad = -1;

    // Test hook: the product of all block dets is needed before the
    // children's dets can be written, so take it in a first pass.
    double Dall_re = 0.0, Dall_im = 0.0;
    if (WITH_PAIRS) {
      double pr_ = 1.0, pi_ = 0.0;
      for (int f = 0; f < F; ++f) {
        const int o = p.off[f];
        uint32_t ro[N], co[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
          ro[n] = rowoff_d[o + n];
          co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
        }
        double gr[N][N], gi[N][N], dre, dim;
        int perm[N];
        bool z;
        gather<N>(lds, ro, co, gr, gi);
        lu<N, false>(gr, gi, dre, dim, perm, z);
        const double tr = pr_ * dre - pi_ * dim;
        pi_ = pr_ * dim + pi_ * dre;
        pr_ = tr;
      }
      Dall_re = pr_;
      Dall_im = pi_;
      if (valid && a.pair_det) {
        a.pair_det[((size_t)t * p.n_src + term) * p.n_snk + k] = make_double2(pr_, pi_);
      }
    }

    int g = g_begin;
    for (int f = 0; f < F; ++f) {
      const int o = p.off[f];
      uint32_t ro[N], co[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        ro[n] = rowoff_d[o + n];
        co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
      }
      double gr[N][N], gi[N][N];
      int perm[N];
      double dre, dim;
      bool zero;
      // groups of this flavour form a contiguous run [g, g_f_end)
      int g_f_end = g;
      if (TREE) {
        while (g_f_end < g_end && uniform(p.grp_fr[g_f_end] >> 8) == f) ++g_f_end;
      }
      double accre = 0.0, accim = 0.0;
      gather<N>(lds, ro, co, gr, gi);
      // The tree keeps the multipliers for every dominator block: nearly
      // every dominator has groups in every flavour, and a single
      // factorisation path keeps the register allocation within budget.
      lu<N, TREE>(gr, gi, dre, dim, perm, zero);
      if (TREE) {
        double sre = 0.0, sim = 0.0;
        for (int gg = g; gg < g_f_end; ++gg) {
          const int r = uniform(p.grp_fr[gg] & 0xff);
          double xr[N], xi[N];
          solve_unit<N>(gr, gi, perm, r, xr, xi);
          const int c_begin = uniform(p.grp_ptr[gg]);
          const int c_end = uniform(p.grp_ptr[gg + 1]);
          for (int c = c_begin; c < c_end; ++c) {
            const uint32_t crow = uniform(p.child_rowoff[c]);
            const int cterm = uniform(p.child_term[c]);
            double rr = 0.0, ri = 0.0;
#pragma unroll
            for (int n = 0; n < N; ++n) {
              const double2 s = *reinterpret_cast<const double2*>(lds + crow + co[n]);
              rr = rr + s.x * xr[n] - s.y * xi[n];
              ri = ri + s.x * xi[n] + s.y * xr[n];
            }
            const double wc = a.w_src[cterm];
            sre += wc * rr;
            sim += wc * ri;
            if (WITH_A && !zero) sabs_reg += fabs(wc) * sqrt(rr * rr + ri * ri);
            if (WITH_PAIRS && valid && a.pair_det && !zero) {
              a.pair_det[((size_t)t * p.n_src + cterm) * p.n_snk + k] =
                  make_double2(rr * Dall_re - ri * Dall_im, rr * Dall_im + ri * Dall_re);
            }
          }
        }
        // acc_f = det_f * sum_c w_c ratio_c  (0 for a zero-pivot block)
        accre = zero ? 0.0 : dre * sre - dim * sim;
        accim = zero ? 0.0 : dre * sim + dim * sre;
        if (zero) {
          ++nbad;
          fbad = g_f_end > g ? f : -2;   // -2: singular, but nothing to redo
        }
      } else if (zero) {
        ++nbad;
        fbad = -2;
      }
      g = g_f_end;
      // Q <- Q * D + acc * P ;  P <- P * D
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

    // Fallback: a block with an exactly zero pivot.  If it is the only
    // singular block of the pair and it has children, their blocks are
    // factorised directly; every other block keeps the dominator's det
    // (the product X of the non-singular blocks).
    if (TREE) {
      const bool need = valid && nbad == 1 && fbad >= 0;
      if (__builtin_amdgcn_ballot_w64(need) != 0) {
        for (int f = 0; f < F; ++f) {
          if (__builtin_amdgcn_ballot_w64(need && fbad == f) == 0) continue;
          const int o = p.off[f];
          uint32_t co[N];
#pragma unroll
          for (int n = 0; n < N; ++n) co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
          double fre = 0.0, fim = 0.0;
          for (int gg = g_begin; gg < g_end; ++gg) {
            if (uniform(p.grp_fr[gg] >> 8) != f) continue;
            const int r = uniform(p.grp_fr[gg] & 0xff);
            for (int c = uniform(p.grp_ptr[gg]); c < uniform(p.grp_ptr[gg + 1]); ++c) {
              if (need && fbad == f) {
                double cre, cim;
                child_det_direct<N>(lds, rowoff_d + o, r, p.child_rowoff[c], co, cre, cim);
                const double wc = a.w_src[p.child_term[c]];
                fre += wc * cre;
                fim += wc * cim;
                const double dr = cre * Xre - cim * Xim, di = cre * Xim + cim * Xre;
                if (WITH_A) sabs_fb += fabs(wc) * sqrt(dr * dr + di * di);
                if (WITH_PAIRS && a.pair_det)
                  a.pair_det[((size_t)t * p.n_src + p.child_term[c]) * p.n_snk + k] =
                      make_double2(dr, di);
                ++n_fallback;
              }
            }
          }
          if (need && fbad == f) {
            Qre += fre * Xre - fim * Xim;
            Qim += fre * Xim + fim * Xre;
          }
        }
      }
      // Pairs whose blocks are singular in two flavours, or whose singular
      // block has no children, have determinant 0: write zeros for them.
      if (WITH_PAIRS && a.pair_det && valid && nbad > 0) {
        for (int gg = g_begin; gg < g_end; ++gg) {
          const int f = uniform(p.grp_fr[gg] >> 8);
          if (nbad == 1 && fbad == f) continue;   // written above
          for (int c = uniform(p.grp_ptr[gg]); c < uniform(p.grp_ptr[gg + 1]); ++c) {
            // a child of a non-singular flavour still sees the singular
            // block of the other flavour: det 0
            a.pair_det[((size_t)t * p.n_src + p.child_term[c]) * p.n_snk + k] =
                make_double2(0.0, 0.0);
          }
        }
      }
    }

    if (valid) {
      acc_re += wk * (wi * Pre + Qre);
      acc_im += wk * (wi * Pim + Qim);
      if (WITH_A) {
        // |d_child| = |ratio| |P| for children taken by the update; the
        // fallback children carry their own |det| in sabs_fb.
        const double pabs = sqrt(Pre * Pre + Pim * Pim);
        acc_a += fabs(wk) * ((fabs(wi) + sabs_reg) * pabs + sabs_fb);
      }
    }
  }

  // Workgroup reduction (fixed order) -> one partial per workgroup.
  __shared__ double red[kWavesPerBlock][3];
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
    for (int w = 0; w < kWavesPerBlock; ++w) v += red[w][threadIdx.x];
    a.partial[((size_t)t * a.n_blk_t + chunk) * 3 + threadIdx.x] = v;
  }
}

// C[t] = sum over workgroups of the partials, in a fixed order.
__global__ __launch_bounds__(kBlock) void reduce_partials(const double* partial, int n_blk_t,
                                                          double2* C, double* A) {
  const int t = blockIdx.x;
  __shared__ double red[3][kBlock];
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < n_blk_t; b += kBlock)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] += partial[((size_t)t * n_blk_t + b) * 3 + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    C[t] = make_double2(red[0][0], red[1][0]);
    if (A) A[t] = red[2][0];
  }
}

template <int N, bool TREE, int MODE>
static hipError_t launch_one(const ContractArgs& a, hipStream_t s) {
  dim3 grid(a.n_blk_t, a.T);
  size_t lds = (size_t)a.plan.M * a.plan.M * sizeof(double2);
  hipLaunchKernelGGL((contract_kernel<N, TREE, MODE>), grid, dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

template <int N>
static hipError_t launch_n(const ContractArgs& a, bool tree, bool diag, hipStream_t s) {
  if (tree) return diag ? launch_one<N, true, 3>(a, s) : launch_one<N, true, 0>(a, s);
  return diag ? launch_one<N, false, 3>(a, s) : launch_one<N, false, 0>(a, s);
}

hipError_t launch_contract(const ContractArgs& a, int n, bool tree, bool diag,
                           double2* C, double* A, hipStream_t s) {
  hipError_t e;
  switch (n) {
    case 1: e = launch_n<1>(a, tree, diag, s); break;
    case 2: e = launch_n<2>(a, tree, diag, s); break;
    case 3: e = launch_n<3>(a, tree, diag, s); break;
    case 4: e = launch_n<4>(a, tree, diag, s); break;
    case 5: e = launch_n<5>(a, tree, diag, s); break;
    case 6: e = launch_n<6>(a, tree, diag, s); break;
    case 7: e = launch_n<7>(a, tree, diag, s); break;
    case 8: e = launch_n<8>(a, tree, diag, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_partials, dim3(a.T), dim3(kBlock), 0, s, a.partial, a.n_blk_t, C, A);
  return hipGetLastError();
}

}  // namespace kern
}  // namespace mhc
