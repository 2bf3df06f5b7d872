// Adjoint of the correlator contraction (HIP, gfx950).
//
// For an incoming gradient gC[t] (PyTorch's convention for a real loss):
//   grad S_t[p][q] = gC[t] * conj(dC(t)/dS_t[p][q]),
//   grad w_i       = Re(sum_t gC[t] * conj(sum_j w'_j d_ij(t))),
//   grad w'_j      = Re(sum_t gC[t] * conj(sum_i w_i d_ij(t))),
// with d_ij = prod_f det G_f and, by Jacobi's formula,
//   d det(G_f) / d G_f[r][n] = det(G_f) (G_f^-1)[n][r].
// The LU of every block is recomputed here (no factor is stored by the
// forward pass).  Column r of G_f^-1 is one solve x = G_f^-1 e_r; its n
// entries go to the propagator entries S_t[a_i^{f,r}][a_j^{f,n}].
//
// Work decomposition: a workgroup owns (slice t, sink block of 64) and walks
// every source term (wave w takes sources w, w+4, ...); lane l = sink
// block + l * (number of blocks) (adj_sink).  S_t and an accumulator for
// grad S_t live in LDS; the accumulator takes LDS atomic adds (FP64), then
// goes to a per-workgroup partial that fixed-order kernels reduce.  The weight gradients are reduced
// in a fixed order (bitwise repeatable); grad S is repeatable up to the
// order of the LDS atomics within one workgroup.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contract_kernels.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

constexpr int kMaxAdjFlavors = 4;

// The sinks of one wave share most of their columns and, with them, most
// of their pivot order, and LDS atomics of several lanes to one address
// serialise.  After the inversion each lane rotates the columns of V (and
// their addresses) by lane % kAdjSpread positions: the column index is a
// summation label only, but at each step of a row's adds the lanes of a
// wave then target up to kAdjSpread different columns.
constexpr int kAdjSpread = 4;

// V[i][q] <- V[i][(q + rho) % N], pcol[q] <- pcol[(q + rho) % N], rho =
// lane % R, by selects (no register is indexed at run time).
template <int N, int R>
__device__ __forceinline__ void rotate_columns(double (&vr)[N][N], double (&vi)[N][N],
                                               uint32_t (&pcol)[N], int lane) {
  if constexpr (N > 1 && R > 1) {
    const int rho = lane % R;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double tr[N], ti[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        tr[q] = vr[i][q];
        ti[q] = vi[i][q];
      }
#pragma unroll
      for (int q = 0; q < N; ++q) {
        double xr = tr[q], xi = ti[q];
#pragma unroll
        for (int s = 1; s < R; ++s) {
          xr = rho == s ? tr[(q + s) % N] : xr;
          xi = rho == s ? ti[(q + s) % N] : xi;
        }
        vr[i][q] = xr;
        vi[i][q] = xi;
      }
    }
    uint32_t tc[N];
#pragma unroll
    for (int q = 0; q < N; ++q) tc[q] = pcol[q];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      uint32_t c = tc[q];
#pragma unroll
      for (int s = 1; s < R; ++s) c = rho == s ? tc[(q + s) % N] : c;
      pcol[q] = c;
    }
  }
}

// Sink of lane `lane` in sink block sb: the blocks take the sinks with a
// stride of n_sblk, not 64 consecutive sinks.  Neighbouring sinks of a
// tree-ordered list are siblings that share most of their column indices;
// in one wave their cofactors would be added to the same grad S entries,
// and LDS atomic adds to one address from several lanes serialise.
__device__ __forceinline__ int adj_sink(int sb, int lane, int n_sblk) {
  return sb + n_sblk * lane;
}

// The LDS accumulator of grad S_t holds the real parts and the imaginary
// parts in two planes of M x (M + 1) doubles (`plane` bytes apart), entry
// (row, col) at (row * (M + 1) + col) * 8: half the byte offset of the same
// entry in the complex copy of S_t, so the plan's row and column offsets
// serve both.  With 8-byte steps between columns, 64-bit atomics of lanes
// that add to different columns of one row spread over all LDS bank pairs
// (complex entries, 16 bytes apart, would use every other pair).
__host__ __device__ constexpr uint32_t grad_plane_bytes(int M) {
  return (uint32_t)M * lds_row(M) * 8;
}

__device__ __forceinline__ void grad_add(char* glds, uint32_t plane, uint32_t rowoff,
                                         uint32_t coloff, double re, double im) {
  char* e = glds + ((rowoff + coloff) >> 1);
  atomicAdd(reinterpret_cast<double*>(e), re);
  atomicAdd(reinterpret_cast<double*>(e + plane), im);
}

// Block with an exactly zero pivot (no inverse): its cofactors from the
// definition, adj(G)[n][r] = (-1)^(r+n) det(G without row r and column n),
// each minor by a direct LU (Jacobi's formula d det G / d G[r][n] =
// adj(G)[n][r] holds for singular G too).  Scatters b * conj(adj(G)[n][r])
// into grad S at (row r, column n) for the lanes with `valid`; b = coef *
// conj(prod of the other blocks' determinants).  Rare (singular blocks
// only), so the minor loop is not unrolled.
template <int N>
__device__ __noinline__ void scatter_cofactors(const char* lds, char* glds, uint32_t plane,
                                               const uint32_t (&ro)[N], const uint32_t (&co)[N],
                                               double bre, double bim, bool valid) {
  if constexpr (N == 1) {
    if (valid) grad_add(glds, plane, ro[0], co[0], bre, bim);
  } else {
#pragma unroll 1
    for (int r = 0; r < N; ++r) {
#pragma unroll 1
      for (int n = 0; n < N; ++n) {
        uint32_t rm[N - 1], cm[N - 1];
#pragma unroll
        for (int m = 0; m < N - 1; ++m) {
          rm[m] = m < r ? ro[m] : ro[m + 1];
          cm[m] = m < n ? co[m] : co[m + 1];
        }
        double gr[N - 1][N - 1], gi[N - 1][N - 1];
        int perm[N - 1];
        double mr, mi;
        bool z;
        gather<N - 1>(lds, rm, cm, gr, gi);
        lu<N - 1, false>(gr, gi, mr, mi, perm, z);
        if ((r + n) & 1) {
          mr = -mr;
          mi = -mi;
        }
        // grad S[row r][col n] += b * conj(adj[n][r])
        if (valid) grad_add(glds, plane, ro[r], co[n], bre * mr + bim * mi, bim * mr - bre * mi);
      }
    }
  }
}

// One source term against the lane's sink, pair by pair: the term's rows
// are the row set `rowoff` with, in flavour fs, row rs replaced by the row
// at byte offset srow (fs < 0: no replacement).  Pass 1 forms every block's
// determinant; pass 2 refactorises each block, solves its N unit columns and
// scatters coef * conj(X_f det_f) * conj(x_r[n]) into the LDS accumulator
// (coef = gc * w_i * w_k).  Returns the pair determinant.  A block with an
// exactly zero pivot has no inverse: its cofactors come from its minors
// (scatter_cofactors), and it is counted.
template <int N>
__device__ __forceinline__ double2 member_adjoint(const PlanView& p, const char* lds, char* glds,
                                                  const uint32_t* rowoff, int fs, int rs,
                                                  uint32_t srow, int k, bool valid, double2 gc,
                                                  double cw, uint32_t& n_singular) {
  const int F = p.F;
  double dre[kMaxAdjFlavors], dim[kMaxAdjFlavors];
#pragma unroll
  for (int f = 0; f < kMaxAdjFlavors; ++f) {
    dre[f] = 1.0;
    dim[f] = 0.0;
    if (f < F) {
      const int o = p.off[f];
      uint32_t ro[N], co[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        ro[n] = (f == fs && n == rs) ? srow : rowoff[o + n];
        co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
      }
      double gr[N][N], gi[N][N];
      int perm[N];
      bool z;
      gather<N>(lds, ro, co, gr, gi);
      lu<N, false>(gr, gi, dre[f], dim[f], perm, z);
    }
  }
  double d_re = 1.0, d_im = 0.0;
#pragma unroll
  for (int f = 0; f < kMaxAdjFlavors; ++f) {
    const double tr = d_re * dre[f] - d_im * dim[f];
    d_im = d_re * dim[f] + d_im * dre[f];
    d_re = tr;
  }
  const double cre = gc.x * cw, cim = gc.y * cw;
#pragma unroll
  for (int f = 0; f < kMaxAdjFlavors; ++f) {
    if (f >= F) continue;
    // X_f = prod of the other blocks' determinants
    double xre = 1.0, xim = 0.0;
#pragma unroll
    for (int g = 0; g < kMaxAdjFlavors; ++g) {
      if (g == f) continue;
      const double tr = xre * dre[g] - xim * dim[g];
      xim = xre * dim[g] + xim * dre[g];
      xre = tr;
    }
    // b = coef * conj(X_f det_f)
    const double pre = xre * dre[f] - xim * dim[f];
    const double pim = xre * dim[f] + xim * dre[f];
    const double bre = cre * pre + cim * pim;
    const double bim = cim * pre - cre * pim;
    const int o = p.off[f];
    uint32_t ro[N], co[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
      ro[n] = (f == fs && n == rs) ? srow : rowoff[o + n];
      co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
    }
    double gr[N][N], gi[N][N];
    int perm[N];
    double ddr, ddi;
    bool z;
    gather<N>(lds, ro, co, gr, gi);
    lu<N, true>(gr, gi, ddr, ddi, perm, z);
    if (z) {
      // no inverse: the cofactors from the minors, scaled by
      // coef * conj(X_f) (det_f is not a factor of the adjugate)
      if (valid) ++n_singular;
      scatter_cofactors<N>(lds, glds, grad_plane_bytes(p.M), ro, co, cre * xre + cim * xim,
                           cim * xre - cre * xim, valid);
      continue;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      double xr[N], xi[N];
      solve_unit<N>(gr, gi, perm, r, xr, xi);
#pragma unroll
      for (int n = 0; n < N; ++n) {
        // grad S[row r][col n] += b * conj(x[n])
        const double vr = bre * xr[n] + bim * xi[n];
        const double vi = bim * xr[n] - bre * xi[n];
        if (valid) grad_add(glds, grad_plane_bytes(p.M), ro[r], co[n], vr, vi);
      }
    }
  }
  return make_double2(d_re, d_im);
}

// Stages S_t and clears the grad S_t accumulator (both padded rows).
__device__ __forceinline__ void adjoint_stage(const AdjointArgs& a, int t, double2* smem) {
  const PlanView& p = a.plan;
  const int LL = p.M * lds_row(p.M);
  stage_slice(a.S + (size_t)t * p.M * p.M, smem, p.M, kBlock);
  double2* gl = smem + LL;
  for (int e = threadIdx.x; e < LL; e += kBlock) gl[e] = make_double2(0.0, 0.0);
  __syncthreads();
}

// Per-lane sink-weight partials (waves combined in a fixed order), the
// singular-block counter and the workgroup's grad S_t partial.
__device__ __forceinline__ void adjoint_finish(const AdjointArgs& a, int t, int sb, double acc_wk,
                                               uint32_t n_singular, double2* smem) {
  const PlanView& p = a.plan;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  __shared__ double red[kWavesPerBlock][kWave];
  red[wave][lane] = acc_wk;
  if (a.singular) {
    uint32_t ns = n_singular;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) ns += __shfl_xor(ns, o, kWave);
    if (lane == 0 && ns) atomicAdd(a.singular, (unsigned long long)ns);
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) v += red[w][threadIdx.x];
    a.part_wsnk[(size_t)t * p.n_snk_pad + adj_sink(sb, threadIdx.x, a.n_sblk)] = v;
  }
  const int MM = p.M * p.M;
  const double* re = reinterpret_cast<const double*>(smem + p.M * lds_row(p.M));
  const double* im = re + p.M * lds_row(p.M);
  double2* dst = a.part_gS + ((size_t)t * a.n_sblk + sb) * MM;
  for (int e = threadIdx.x; e < MM; e += kBlock) {
    const int q = (e / p.M) * lds_row(p.M) + e % p.M;
    dst[e] = make_double2(re[q], im[q]);
  }
}

// Plain adjoint: every source term, pair by pair.
template <int N>
__global__ __launch_bounds__(kBlock, 2) void adjoint_kernel(AdjointArgs a) {
  extern __shared__ double2 smem[];
  const PlanView& p = a.plan;
  const int t = blockIdx.y;
  const int sb = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  adjoint_stage(a, t, smem);
  const char* lds = reinterpret_cast<const char*>(smem);
  char* glds = reinterpret_cast<char*>(smem + p.M * lds_row(p.M));
  const int k = adj_sink(sb, lane, a.n_sblk);
  const bool valid = k < p.n_snk;
  const double wk = valid ? a.w_snk[k] : 0.0;
  const double2 gc = a.gC[t];
  double acc_wk = 0.0;
  uint32_t n_singular = 0;
  for (int i = wave; i < p.n_src; i += kWavesPerBlock) {
    const double wi = a.w_src[i];
    const double2 d = member_adjoint<N>(p, lds, glds, p.src_rowoff + (size_t)i * p.sn, -1, -1,
                                        0u, k, valid, gc, wi * wk, n_singular);
    // weights: Re(gc * conj(d))
    const double val = valid ? gc.x * d.x + gc.y * d.y : 0.0;
    acc_wk += wi * val;
    const double s_i = wave_sum(wk * val);
    if (lane == 0) a.part_wsrc[((size_t)t * p.n_src + i) * a.n_sblk + sb] = s_i;
  }
  adjoint_finish(a, t, sb, acc_wk, n_singular, smem);
}

// Every member of dominator d against the lane's sink, pair by pair
// (member_adjoint), for the lanes with `need`; weights added to the
// partials of the update-tree kernel.
template <int N>
__device__ __forceinline__ void dominator_pairs(const AdjointArgs& a, const char* lds, char* glds,
                                             int t, int sb, int d, int k, bool need, double2 gc,
                                             double wk, double& acc_wk, uint32_t& n_singular) {
  const PlanView& p = a.plan;
  const int lane = threadIdx.x & (kWave - 1);
  const int term_d = uniform(p.dom_term[d]);
  const uint32_t* rowoff_d = p.dom_rowoff + (size_t)d * p.sn;
  const double wd = a.w_src[term_d];
  double2 dd = member_adjoint<N>(p, lds, glds, rowoff_d, -1, -1, 0u, k, need, gc, wd * wk,
                                 n_singular);
  double val = need ? gc.x * dd.x + gc.y * dd.y : 0.0;
  acc_wk += wd * val;
  double s_i = wave_sum(wk * val);
  if (lane == 0) a.part_wsrc[((size_t)t * p.n_src + term_d) * a.n_sblk + sb] += s_i;
  for (int gg = uniform(p.dom_grp[d]); gg < uniform(p.dom_grp[d + 1]); ++gg) {
    const int fs = uniform(p.grp_fr[gg] >> 8), rs = uniform(p.grp_fr[gg] & 0xff);
    for (int c = uniform(p.grp_ptr[gg]); c < uniform(p.grp_ptr[gg + 1]); ++c) {
      const uint32_t crow = uniform(p.child_rowoff[c]);
      const int cterm = uniform(p.child_term[c]);
      const double wc = a.w_src[cterm];
      dd = member_adjoint<N>(p, lds, glds, rowoff_d, fs, rs, crow, k, need, gc, wc * wk,
                             n_singular);
      val = need ? gc.x * dd.x + gc.y * dd.y : 0.0;
      acc_wk += wc * val;
      s_i = wave_sum(wk * val);
      if (lane == 0) a.part_wsrc[((size_t)t * p.n_src + cterm) * a.n_sblk + sb] += s_i;
    }
  }
}

// Update-tree adjoint: one (dominator, sink) at a time.  With G the
// dominator's block f, x_m = G^-1 e_m, and the child c of flavour f that
// replaces row r by s_c (z_c = s_c^T G^-1, rho_c = z_c[r]), the cofactor
// matrix of the child is rho_c det G G^-T - det G (z_c - e_r) x_r^T
// (Sherman-Morrison); its row r is det G x_r^T and belongs to the new row
// s_c.  Summed over the partition with the weights, block f's derivative
// on the dominator's rows is
//   X_f det G_f (W (G^-1)^T - sum_groups Z_r x_r^T),  W = w_d + sum_c w_c rho_c,
// Z_r = sum_{c in group r} w_c z_c (children of other flavours enter W
// through their own rho_c; the rank-1 terms vanish on row r), and each
// child adds w_c X_f det G_f x_r to its own row.  Pass A factorises the
// blocks and forms W; pass B refactorises each block transposed, inverts
// it in place and adds each entry of the derivative once (rows of T).  A
// lane whose dominator block has an exactly zero pivot takes every member
// pair by pair (dominator_pairs).
template <int N>
__global__ __launch_bounds__(kBlock, 2) void adjoint_tree_kernel(AdjointArgs a) {
  extern __shared__ double2 smem[];
  const PlanView& p = a.plan;
  const int t = blockIdx.y;
  const int sb = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  adjoint_stage(a, t, smem);
  const char* lds = reinterpret_cast<const char*>(smem);
  char* glds = reinterpret_cast<char*>(smem + p.M * lds_row(p.M));
  const uint32_t plane = grad_plane_bytes(p.M);
  const int k = adj_sink(sb, lane, a.n_sblk);
  const bool valid = k < p.n_snk;
  const double wk = valid ? a.w_snk[k] : 0.0;
  const double2 gc = a.gC[t];
  const int F = p.F;
  const int sn = p.sn;
  double acc_wk = 0.0;
  uint32_t n_singular = 0;

  uint8_t* flag = a.dom_flag + ((size_t)t * a.n_sblk + sb) * p.n_dom;
  for (int d = wave; d < p.n_dom; d += kWavesPerBlock) {
    const int term_d = cload(p.dom_term, d);
    const double wd = cload(a.w_src, term_d);
    const uint32_t* rowoff_d = p.dom_rowoff + (size_t)d * sn;
    const int g_begin = cload(p.dom_grp, d);
    const int g_end = cload(p.dom_grp, d + 1);
    // the sink's column offsets are read again for every dominator: an
    // opaque copy of k keeps their addresses from being hoisted out of the
    // loop (F x N addresses live across it would spill)
    int kk = k;
    asm volatile("" : "+v"(kk));

    // pass A: block determinants and W
    double dre[kMaxAdjFlavors], dim[kMaxAdjFlavors];
    double Wre = wd, Wim = 0.0;
    bool bad = false;
    int g = g_begin;
#pragma unroll
    for (int f = 0; f < kMaxAdjFlavors; ++f) {
      dre[f] = 1.0;
      dim[f] = 0.0;
      if (f >= F) continue;
      const int o = p.off[f];
      uint32_t ro[N], co[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        ro[n] = cload(rowoff_d, o + n);
        co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + kk];
      }
      double gr[N][N], gi[N][N];
      int perm[N];
      bool z;
      gather<N>(lds, ro, co, gr, gi);
      lu<N, true>(gr, gi, dre[f], dim[f], perm, z);
      bad = bad || z;
      for (; g < g_end && (cload(p.grp_fr, g) >> 8) == f; ++g) {
        const int r = cload(p.grp_fr, g) & 0xff;
        double xr[N], xi[N];
        solve_unit<N>(gr, gi, perm, r, xr, xi);
        for (int c = cload(p.grp_ptr, g); c < cload(p.grp_ptr, g + 1); ++c) {
          const uint32_t crow = cload(p.child_rowoff, c);
          const double wc = cload(a.w_src, cload(p.child_term, c));
          double rr = 0.0, ri = 0.0;
#pragma unroll
          for (int n = 0; n < N; ++n) {
            const double2 sv = *reinterpret_cast<const double2*>(lds + crow + co[n]);
            rr = rr + sv.x * xr[n] - sv.y * xi[n];
            ri = ri + sv.x * xi[n] + sv.y * xr[n];
          }
          Wre += wc * rr;
          Wim += wc * ri;
        }
      }
    }
    double Dre = 1.0, Dim = 0.0;
#pragma unroll
    for (int f = 0; f < kMaxAdjFlavors; ++f) {
      const double tr = Dre * dre[f] - Dim * dim[f];
      Dim = Dre * dim[f] + Dim * dre[f];
      Dre = tr;
    }
    const bool fast = valid && !bad;
    // weights of the sink (all members) and of the dominator
    if (fast) {
      const double pr = Dre * Wre - Dim * Wim, pi = Dre * Wim + Dim * Wre;
      acc_wk += gc.x * pr + gc.y * pi;
    }
    {
      const double val = fast ? gc.x * Dre + gc.y * Dim : 0.0;
      const double s_d = wave_sum(wk * val);
      if (lane == 0) a.part_wsrc[((size_t)t * p.n_src + term_d) * a.n_sblk + sb] = s_d;
    }

    // pass B, block by block: with x_m = G^-1 e_m, Z_r = the sum over the
    // group of row r of w_c z_c and T[i][n] = W x_i[n] - sum_r Z_r[i] x_r[n],
    // the dominator's row i takes B conj(T[i][n]) at column n, one add per
    // entry; each child adds B conj(w_c x_r[n]) to its own row.  The block
    // is factorised transposed (A = G^T, rows = the sink's columns,
    // P A = L U) and V = U^-1 L^-1 holds x_i in its row i,
    // x_i[perm[q]] = V[i][q], so a row of T needs no solve and no index
    // that differs between lanes except the column addresses.
    // B = gc * w_k * conj(X_f det_f) = gc * w_k * conj(D)
    const double bre = wk * (gc.x * Dre + gc.y * Dim);
    const double bim = wk * (gc.y * Dre - gc.x * Dim);
    g = g_begin;
#pragma unroll
    for (int f = 0; f < kMaxAdjFlavors; ++f) {
      if (f >= F) continue;
      const int o = p.off[f];
      int g_f_end = g;
      while (g_f_end < g_end && (cload(p.grp_fr, g_f_end) >> 8) == f) ++g_f_end;
      uint32_t ro[N], co[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        ro[n] = cload(rowoff_d, o + n);
        co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + kk];
      }
      double vr[N][N], vi[N][N];
      int perm[N];
      {
        double ddr, ddi;
        bool z;
        gather<N>(lds, co, ro, vr, vi);  // offsets add: vr[q][i] = G[i][q]
        lu<N, true>(vr, vi, ddr, ddi, perm, z);
        lu_inverse_v<N>(vr, vi);
      }
      uint32_t pcol[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        uint32_t v = co[0];
#pragma unroll
        for (int j = 1; j < N; ++j)
          if (perm[q] == j) v = co[j];
        pcol[q] = v;
      }
      rotate_columns<N, kAdjSpread>(vr, vi, pcol, lane);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double tr[N], ti[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
          tr[q] = Wre * vr[i][q] - Wim * vi[i][q];
          ti[q] = Wre * vi[i][q] + Wim * vr[i][q];
        }
        for (int gg = g; gg < g_f_end; ++gg) {
          const int r = cload(p.grp_fr, gg) & 0xff;
          double zr = 0.0, zi = 0.0;
          // the children's records, each read one child ahead
          const int c_end = cload(p.grp_ptr, gg + 1);
          int c = cload(p.grp_ptr, gg);
          ChildRec next = cload(a.child_rec, c);
          for (; c < c_end; ++c) {
            const ChildRec cur = next;
            next = cload(a.child_rec, c + 1);
            const uint32_t crow = cur.crow;
            const int cterm = cur.term;
            const double wc = cur.w;
            // z_c[i] = sum_n s_c[n] x_i[n], s_c = the child's new row
            double dr = 0.0, di = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) {
              const double2 sv = *reinterpret_cast<const double2*>(lds + crow + pcol[q]);
              dr = dr + sv.x * vr[i][q] - sv.y * vi[i][q];
              di = di + sv.x * vi[i][q] + sv.y * vr[i][q];
            }
            zr += wc * dr;
            zi += wc * di;
            if (r == i) {
              // rho_c = z_c[r]: the child's source weight, sum over sinks
              // of w_k Re(gc conj(rho_c D)) = Re(rho_c conj(B)), and its
              // own row
              const double s_c = wave_sum(fast ? dr * bre + di * bim : 0.0);
              if (lane == 0) a.part_wsrc[((size_t)t * p.n_src + cterm) * a.n_sblk + sb] = s_c;
#pragma unroll
              for (int q = 0; q < N; ++q)
                if (fast)
                  grad_add(glds, plane, crow, pcol[q], wc * (bre * vr[i][q] + bim * vi[i][q]),
                           wc * (bim * vr[i][q] - bre * vi[i][q]));
            }
          }
          // T[i] -= Z_r[i] x_r
#pragma unroll
          for (int rr = 0; rr < N; ++rr)
            if (rr == r) {
#pragma unroll
              for (int q = 0; q < N; ++q) {
                tr[q] = tr[q] - zr * vr[rr][q] + zi * vi[rr][q];
                ti[q] = ti[q] - zr * vi[rr][q] - zi * vr[rr][q];
              }
            }
        }
#pragma unroll
        for (int q = 0; q < N; ++q)
          if (fast)
            grad_add(glds, plane, ro[i], pcol[q], bre * tr[q] + bim * ti[q],
                     bim * tr[q] - bre * ti[q]);
      }
      g = g_f_end;
    }

    // a lane whose dominator has a block with an exactly zero pivot: its
    // member pairs go pair by pair in adjoint_tree_pairs_kernel
    const bool need = valid && bad;
    if (lane == 0) flag[d] = __builtin_amdgcn_ballot_w64(need) != 0 ? 1 : 0;
  }
  adjoint_finish(a, t, sb, acc_wk, n_singular, smem);
}

// The lanes of adjoint_tree_kernel whose dominator has a block with an
// exactly zero pivot (no inverse, so no update formula): a workgroup per
// (sink block, slice) as there, for the dominators that kernel flagged;
// each lane refactorises the dominator's blocks as pass A did (same code,
// same operands, so the same lanes find the zero pivot) and takes every
// member pair by pair.  The results are added to that kernel's partials.
// A workgroup without flagged dominators returns at once.
template <int N>
__global__ __launch_bounds__(kBlock, 2) void adjoint_tree_pairs_kernel(AdjointArgs a) {
  extern __shared__ double2 smem[];
  const PlanView& p = a.plan;
  const int t = blockIdx.y;
  const int sb = blockIdx.x;
  const uint8_t* flag = a.dom_flag + ((size_t)t * a.n_sblk + sb) * p.n_dom;
  int any = 0;
  for (int d = threadIdx.x; d < p.n_dom; d += kBlock) any |= flag[d];
  if (!__syncthreads_or(any)) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  adjoint_stage(a, t, smem);
  const char* lds = reinterpret_cast<const char*>(smem);
  char* glds = reinterpret_cast<char*>(smem + p.M * lds_row(p.M));
  const int k = adj_sink(sb, lane, a.n_sblk);
  const bool valid = k < p.n_snk;
  const double wk = valid ? a.w_snk[k] : 0.0;
  const double2 gc = a.gC[t];
  double acc_wk = 0.0;
  uint32_t n_singular = 0;
  for (int d = wave; d < p.n_dom; d += kWavesPerBlock) {
    if (!uniform(flag[d])) continue;
    const uint32_t* rowoff_d = p.dom_rowoff + (size_t)d * p.sn;
    bool bad = false;
#pragma unroll
    for (int f = 0; f < kMaxAdjFlavors; ++f) {
      if (f >= p.F) continue;
      const int o = p.off[f];
      uint32_t ro[N], co[N];
#pragma unroll
      for (int n = 0; n < N; ++n) {
        ro[n] = rowoff_d[o + n];
        co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
      }
      double gr[N][N], gi[N][N];
      int perm[N];
      double dr, di;
      bool z;
      gather<N>(lds, ro, co, gr, gi);
      lu<N, true>(gr, gi, dr, di, perm, z);
      bad = bad || z;
    }
    dominator_pairs<N>(a, lds, glds, t, sb, d, k, valid && bad, gc, wk, acc_wk, n_singular);
  }
  // sink weights (waves in a fixed order), singular blocks, grad S_t
  __shared__ double red[kWavesPerBlock][kWave];
  red[wave][lane] = acc_wk;
  if (a.singular) {
    uint32_t ns = n_singular;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) ns += __shfl_xor(ns, o, kWave);
    if (lane == 0 && ns) atomicAdd(a.singular, (unsigned long long)ns);
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) v += red[w][threadIdx.x];
    a.part_wsnk[(size_t)t * p.n_snk_pad + adj_sink(sb, threadIdx.x, a.n_sblk)] += v;
  }
  const int MM = p.M * p.M;
  const double* re = reinterpret_cast<const double*>(smem + p.M * lds_row(p.M));
  const double* im = re + p.M * lds_row(p.M);
  double2* dst = a.part_gS + ((size_t)t * a.n_sblk + sb) * MM;
  for (int e = threadIdx.x; e < MM; e += kBlock) {
    const int q = (e / p.M) * lds_row(p.M) + e % p.M;
    const double2 v = dst[e];
    dst[e] = make_double2(v.x + re[q], v.y + im[q]);
  }
}

// The update tree's child records for one call: new row, term and weight.
__global__ __launch_bounds__(kBlock) void child_records(const uint32_t* rowoff, const int32_t* term,
                                                        const double* w_src, int n_children,
                                                        ChildRec* out) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n_children) return;
  ChildRec r;
  r.crow = rowoff[c];
  r.term = term[c];
  r.w = w_src[r.term];
  out[c] = r;
}

// grad S[t][e] = sum over sink blocks of the partials (fixed order)
__global__ __launch_bounds__(kBlock) void reduce_gS(const double2* part, int n_sblk, int MM,
                                                    int T, double2* gS) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= (size_t)T * MM) return;
  const int t = (int)(e / MM);
  const int q = (int)(e - (size_t)t * MM);
  double re = 0.0, im = 0.0;
  for (int b = 0; b < n_sblk; ++b) {
    const double2 v = part[((size_t)t * n_sblk + b) * MM + q];
    re += v.x;
    im += v.y;
  }
  gS[e] = make_double2(re, im);
}

// grad w_i = sum over slices and sink blocks; grad w'_k = sum over slices
__global__ __launch_bounds__(kBlock) void reduce_w(const double* part_src, const double* part_snk,
                                                   int T, int n_src, int n_sblk, int n_snk,
                                                   int n_snk_pad, double* g_src, double* g_snk) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (g_src && e < n_src) {
    double s = 0.0;
    for (int t = 0; t < T; ++t)
      for (int b = 0; b < n_sblk; ++b) s += part_src[((size_t)t * n_src + e) * n_sblk + b];
    g_src[e] = s;
  }
  if (g_snk && e < n_snk) {
    double s = 0.0;
    for (int t = 0; t < T; ++t) s += part_snk[(size_t)t * n_snk_pad + e];
    g_snk[e] = s;
  }
}

template <int N>
static hipError_t launch_adj_n(const AdjointArgs& a, bool tree, hipStream_t s) {
  dim3 grid(a.n_sblk, a.T);
  size_t lds = 2 * lds_slice_bytes(a.plan.M);
  const void* fn = tree ? reinterpret_cast<const void*>(&adjoint_tree_kernel<N>)
                        : reinterpret_cast<const void*>(&adjoint_kernel<N>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (!tree) {
    hipLaunchKernelGGL(adjoint_kernel<N>, grid, dim3(kBlock), lds, s, a);
    return hipGetLastError();
  }
  if (a.n_children > 0) {
    hipLaunchKernelGGL(child_records, dim3((a.n_children + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       s, a.plan.child_rowoff, a.plan.child_term, a.w_src, a.n_children,
                       a.child_rec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(adjoint_tree_kernel<N>, grid, dim3(kBlock), lds, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&adjoint_tree_pairs_kernel<N>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_tree_pairs_kernel<N>, grid, dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjointArgs& a, int n, bool tree, double2* gS, double* g_wsrc,
                          double* g_wsnk, hipStream_t s) {
  hipError_t e;
  switch (n) {
    case 1: e = launch_adj_n<1>(a, tree, s); break;
    case 2: e = launch_adj_n<2>(a, tree, s); break;
    case 3: e = launch_adj_n<3>(a, tree, s); break;
    case 4: e = launch_adj_n<4>(a, tree, s); break;
    case 5: e = launch_adj_n<5>(a, tree, s); break;
    case 6: e = launch_adj_n<6>(a, tree, s); break;
    case 7: e = launch_adj_n<7>(a, tree, s); break;
    case 8: e = launch_adj_n<8>(a, tree, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const int MM = a.plan.M * a.plan.M;
  if (gS) {
    const size_t total = (size_t)a.T * MM;
    hipLaunchKernelGGL(reduce_gS, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, a.part_gS, a.n_sblk, MM, a.T, gS);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (g_wsrc || g_wsnk) {
    const int n_max = a.plan.n_src > a.plan.n_snk ? a.plan.n_src : a.plan.n_snk;
    hipLaunchKernelGGL(reduce_w, dim3((n_max + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                       a.part_wsrc, a.part_wsnk, a.T, a.plan.n_src, a.n_sblk, a.plan.n_snk,
                       a.plan.n_snk_pad, g_wsrc, g_wsnk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace kern
}  // namespace mhc
