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
#include "group_device.h"
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
            if (WITH_A && !zero) sabs_reg += fabs(wc) * cabs_scaled(rr, ri);
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
                if (WITH_A) sabs_fb += fabs(wc) * cabs_scaled(dr, di);
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
        const double pabs = cabs_scaled(Pre, Pim);
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
