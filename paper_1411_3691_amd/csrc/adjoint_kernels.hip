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
// 64*block + l.  S_t and an accumulator for grad S_t live in LDS; the
// accumulator takes LDS atomic adds (FP64), then goes to a per-workgroup
// partial that fixed-order kernels reduce.  The weight gradients are reduced
// in a fixed order (bitwise repeatable); grad S is repeatable up to the
// order of the LDS atomics within one workgroup.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contract_kernels.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

constexpr int kMaxAdjFlavors = 4;

template <int N>
__global__ __launch_bounds__(kBlock, 2) void adjoint_kernel(AdjointArgs a) {
  extern __shared__ double2 smem[];
  const PlanView& p = a.plan;
  const int t = blockIdx.y;
  const int sb = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = uniform(threadIdx.x / kWave);
  const int MM = p.M * p.M;
  const int LL = p.M * lds_row(p.M);
  double2* Sl = smem;            // S_t (padded rows)
  double2* gl = smem + LL;       // grad S_t accumulator, same layout
  const double2* St = a.S + (size_t)t * MM;
  stage_slice(St, Sl, p.M, kBlock);
  for (int e = threadIdx.x; e < LL; e += kBlock) gl[e] = make_double2(0.0, 0.0);
  __syncthreads();
  const char* lds = reinterpret_cast<const char*>(Sl);
  char* glds = reinterpret_cast<char*>(gl);

  const int k = sb * kWave + lane;
  const bool valid = k < p.n_snk;
  const double wk = valid ? a.w_snk[k] : 0.0;
  const double2 gc = a.gC[t];
  const int F = p.F;
  const int sn = p.sn;
  double acc_wk = 0.0;
  uint32_t n_singular = 0;

  for (int i = wave; i < p.n_src; i += kWavesPerBlock) {
    const uint32_t* rowoff_i = p.src_rowoff + (size_t)i * sn;
    const double wi = a.w_src[i];
    // pass 1: the determinant of every flavour block
    double dre[kMaxAdjFlavors], dim[kMaxAdjFlavors];
    bool zero[kMaxAdjFlavors];
#pragma unroll
    for (int f = 0; f < kMaxAdjFlavors; ++f) {
      dre[f] = 1.0;
      dim[f] = 0.0;
      zero[f] = false;
      if (f < F) {
        const int o = p.off[f];
        uint32_t ro[N], co[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
          ro[n] = rowoff_i[o + n];
          co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
        }
        double gr[N][N], gi[N][N];
        int perm[N];
        gather<N>(lds, ro, co, gr, gi);
        lu<N, true>(gr, gi, dre[f], dim[f], perm, zero[f]);
      }
    }
    double d_re = 1.0, d_im = 0.0;
#pragma unroll
    for (int f = 0; f < kMaxAdjFlavors; ++f) {
      const double tr = d_re * dre[f] - d_im * dim[f];
      d_im = d_re * dim[f] + d_im * dre[f];
      d_re = tr;
    }
    // weights: Re(gc * conj(d))
    const double val = valid ? gc.x * d_re + gc.y * d_im : 0.0;
    acc_wk += wi * val;
    const double s_i = wave_sum(wk * val);
    if (lane == 0) a.part_wsrc[((size_t)t * p.n_src + i) * a.n_sblk + sb] = s_i;

    // pass 2: grad S.  coef = gc * w_i * w_k (0 on padded lanes)
    const double cw = wi * wk;
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
        ro[n] = rowoff_i[o + n];
        co[n] = p.snk_coloff[(size_t)(o + n) * p.n_snk_pad + k];
      }
      double gr[N][N], gi[N][N];
      int perm[N];
      double ddr, ddi;
      bool z;
      gather<N>(lds, ro, co, gr, gi);
      lu<N, true>(gr, gi, ddr, ddi, perm, z);
      if (z) {
        // det_f = 0 exactly: its adjugate is not formed from an inverse;
        // the block's contribution is skipped and counted
        if (valid) ++n_singular;
        continue;
      }
#pragma unroll
      for (int r = 0; r < N; ++r) {
        double xr[N], xi[N];
        solve_unit<N>(gr, gi, perm, r, xr, xi);
#pragma unroll
        for (int n = 0; n < N; ++n) {
          // grad S[a_i^{f,r}][a_k^{f,n}] += b * conj(x[n])
          const double vr = bre * xr[n] + bim * xi[n];
          const double vi = bim * xr[n] - bre * xi[n];
          double* dst = reinterpret_cast<double*>(glds + ro[r] + co[n]);
          if (valid) {
            atomicAdd(dst, vr);
            atomicAdd(dst + 1, vi);
          }
        }
      }
    }
  }

  // per-lane sink-weight partials, waves combined in a fixed order
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
    a.part_wsnk[(size_t)t * p.n_snk_pad + sb * kWave + threadIdx.x] = v;
  }
  double2* dst = a.part_gS + ((size_t)t * a.n_sblk + sb) * MM;
  for (int e = threadIdx.x; e < MM; e += kBlock) dst[e] = gl[(e / p.M) * lds_row(p.M) + e % p.M];
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
static hipError_t launch_adj_n(const AdjointArgs& a, hipStream_t s) {
  dim3 grid(a.n_sblk, a.T);
  size_t lds = 2 * lds_slice_bytes(a.plan.M);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&adjoint_kernel<N>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_kernel<N>, grid, dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjointArgs& a, int n, double2* gS, double* g_wsrc,
                          double* g_wsnk, hipStream_t s) {
  hipError_t e;
  switch (n) {
    case 1: e = launch_adj_n<1>(a, s); break;
    case 2: e = launch_adj_n<2>(a, s); break;
    case 3: e = launch_adj_n<3>(a, s); break;
    case 4: e = launch_adj_n<4>(a, s); break;
    case 5: e = launch_adj_n<5>(a, s); break;
    case 6: e = launch_adj_n<6>(a, s); break;
    case 7: e = launch_adj_n<7>(a, s); break;
    case 8: e = launch_adj_n<8>(a, s); break;
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
