// Device plans and the forward contraction entry point of libmhc.
//
// A plan holds the tables the kernels read, uploaded once: the dominators
// of the source tree with their row offsets, the group table (flavour,
// changed row, child range), the child table (new row, term) and the sink
// column offsets.  The same plan also carries the plain method's table
// (every source term as its own row set), so both methods run on one plan.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "contract_kernels.h"
#include "mhc_internal.h"

using mhc::fail;

struct mhc_plan {
  int device = 0;
  int32_t n_src = 0, n_snk = 0, n_snk_pad = 0, M = 0, F = 0, sn = 0;
  int32_t n = 0;          // largest flavour block
  bool uniform_n = true;  // every flavour block has size n
  int32_t n_dom = 0, n_groups = 0, n_children = 0;
  std::vector<int32_t> off;
  void* dev_tables = nullptr;          // one allocation for every table
  mhc::kern::PlanView view{};
  double* partial = nullptr;           // workgroup partials
  size_t partial_cap = 0;              // in doubles
  unsigned long long* fallback = nullptr;
  unsigned long long* singular = nullptr;
  // adjoint scratch (grown on demand)
  void* adj_scratch = nullptr;
  size_t adj_cap = 0;
};

namespace {

constexpr int kSinkBlock = 64;
constexpr int kTargetBlocks = 2048;

mhc_status hip_fail(hipError_t e, const char* where) {
  return fail(MHC_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Appends a typed array to a byte image, 256-byte aligned; returns its offset.
template <typename T>
size_t append(std::vector<char>& img, const std::vector<T>& v) {
  size_t at = (img.size() + 255) & ~size_t(255);
  img.resize(at + std::max<size_t>(v.size() * sizeof(T), 1));
  if (!v.empty()) std::memcpy(img.data() + at, v.data(), v.size() * sizeof(T));
  return at;
}

}  // namespace

extern "C" {

mhc_status mhc_plan_create(const mhc_tree* tree, const mhc_terms* snk,
                           void* stream, mhc_plan** out) {
  if (!out) return fail(MHC_E_ARG, "mhc_plan_create: out is NULL");
  *out = nullptr;
  if (!tree || !snk) return fail(MHC_E_ARG, "mhc_plan_create: NULL handle");
  const mhc_terms& src = tree->terms;
  if (src.M != snk->M || src.n_flavors != snk->n_flavors || src.nf != snk->nf)
    return fail(MHC_E_SHAPE,
                "mhc_plan_create: source and sink terms differ in M or in "
                "their flavour blocks");
  int nmax = 0;
  bool uniform_n = true;
  for (int f = 0; f < src.n_flavors; ++f) {
    nmax = std::max(nmax, src.nf[f]);
    uniform_n = uniform_n && src.nf[f] == src.nf[0];
  }
  if (nmax > 24)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_plan_create: flavour blocks larger than 24 are not supported");
  if ((size_t)src.M * src.M * 16 > 150 * 1024)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_plan_create: a slice of S (M*M*16 bytes) must fit in 150 KiB of LDS");

  mhc_plan* pl = new (std::nothrow) mhc_plan();
  if (!pl) return fail(MHC_E_OOM, "mhc_plan_create: out of host memory");
  hipError_t e = hipGetDevice(&pl->device);
  if (e != hipSuccess) {
    delete pl;
    return hip_fail(e, "mhc_plan_create/hipGetDevice");
  }
  pl->n_src = src.n_terms;
  pl->n_snk = snk->n_terms;
  pl->n_snk_pad = (snk->n_terms + kSinkBlock - 1) / kSinkBlock * kSinkBlock;
  pl->M = src.M;
  pl->F = src.n_flavors;
  pl->sn = src.sn;
  pl->n = nmax;
  pl->uniform_n = uniform_n;
  pl->off = src.off;
  pl->n_dom = (int32_t)tree->dom_order.size();
  pl->n_groups = (int32_t)tree->grp_f.size();
  pl->n_children = (int32_t)tree->grp_child.size();

  const int sn = src.sn;
  const uint32_t row_bytes = (uint32_t)src.M * 16u;
  std::vector<int32_t> dom_term(tree->dom_order);
  std::vector<uint32_t> dom_rowoff((size_t)pl->n_dom * sn);
  for (int k = 0; k < pl->n_dom; ++k)
    for (int q = 0; q < sn; ++q)
      dom_rowoff[(size_t)k * sn + q] =
          (uint32_t)src.idx[(size_t)tree->dom_order[k] * sn + q] * row_bytes;
  std::vector<int32_t> grp_fr(pl->n_groups);
  for (int g = 0; g < pl->n_groups; ++g)
    grp_fr[g] = (tree->grp_f[g] << 8) | tree->grp_r[g];
  std::vector<uint32_t> child_rowoff(pl->n_children);
  std::vector<int32_t> child_term(tree->grp_child);
  for (int g = 0; g < pl->n_groups; ++g) {
    const int f = tree->grp_f[g], r = tree->grp_r[g];
    for (int c = tree->grp_ptr[g]; c < tree->grp_ptr[g + 1]; ++c) {
      const int u = tree->grp_child[c];
      child_rowoff[c] =
          (uint32_t)src.idx[(size_t)u * sn + src.off[f] + r] * row_bytes;
    }
  }
  std::vector<uint32_t> src_rowoff((size_t)src.n_terms * sn);
  for (size_t q = 0; q < src_rowoff.size(); ++q)
    src_rowoff[q] = (uint32_t)src.idx[q] * row_bytes;
  std::vector<uint32_t> snk_coloff((size_t)sn * pl->n_snk_pad);
  for (int q = 0; q < sn; ++q)
    for (int k = 0; k < pl->n_snk_pad; ++k) {
      const int kk = k < snk->n_terms ? k : 0;
      snk_coloff[(size_t)q * pl->n_snk_pad + k] =
          (uint32_t)snk->idx[(size_t)kk * sn + q] * 16u;
    }

  std::vector<char> img;
  const size_t o_dom_term = append(img, dom_term);
  const size_t o_dom_rowoff = append(img, dom_rowoff);
  const size_t o_dom_grp = append(img, tree->dom_grp);
  const size_t o_grp_fr = append(img, grp_fr);
  const size_t o_grp_ptr = append(img, tree->grp_ptr);
  const size_t o_child_rowoff = append(img, child_rowoff);
  const size_t o_child_term = append(img, child_term);
  const size_t o_src_rowoff = append(img, src_rowoff);
  const size_t o_snk_coloff = append(img, snk_coloff);
  const size_t o_fallback = append(img, std::vector<unsigned long long>(2, 0ull));

  e = hipMalloc(&pl->dev_tables, img.size());
  if (e != hipSuccess) {
    delete pl;
    return fail(MHC_E_OOM, std::string("mhc_plan_create/hipMalloc: ") +
                               hipGetErrorString(e));
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  e = hipMemcpyAsync(pl->dev_tables, img.data(), img.size(),
                     hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    hipFree(pl->dev_tables);
    delete pl;
    return hip_fail(e, "mhc_plan_create/upload");
  }
  char* base = static_cast<char*>(pl->dev_tables);
  mhc::kern::PlanView& v = pl->view;
  v.n_src = pl->n_src;
  v.n_snk = pl->n_snk;
  v.n_snk_pad = pl->n_snk_pad;
  v.M = pl->M;
  v.F = pl->F;
  v.sn = pl->sn;
  v.n_dom = pl->n_dom;
  for (int f = 0; f < 9; ++f) v.off[f] = f <= pl->F ? pl->off[f] : pl->sn;
  v.dom_term = reinterpret_cast<const int32_t*>(base + o_dom_term);
  v.dom_rowoff = reinterpret_cast<const uint32_t*>(base + o_dom_rowoff);
  v.dom_grp = reinterpret_cast<const int32_t*>(base + o_dom_grp);
  v.grp_fr = reinterpret_cast<const int32_t*>(base + o_grp_fr);
  v.grp_ptr = reinterpret_cast<const int32_t*>(base + o_grp_ptr);
  v.child_rowoff = reinterpret_cast<const uint32_t*>(base + o_child_rowoff);
  v.child_term = reinterpret_cast<const int32_t*>(base + o_child_term);
  v.src_rowoff = reinterpret_cast<const uint32_t*>(base + o_src_rowoff);
  v.snk_coloff = reinterpret_cast<const uint32_t*>(base + o_snk_coloff);
  pl->fallback = reinterpret_cast<unsigned long long*>(base + o_fallback);
  pl->singular = pl->fallback + 1;
  *out = pl;
  return MHC_OK;
}

void mhc_plan_destroy(mhc_plan* pl) {
  if (!pl) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(pl->device);
  hipDeviceSynchronize();
  if (pl->partial) hipFree(pl->partial);
  if (pl->adj_scratch) hipFree(pl->adj_scratch);
  if (pl->dev_tables) hipFree(pl->dev_tables);
  hipSetDevice(cur);
  delete pl;
}

mhc_status mhc_contract(mhc_plan* pl, int32_t method, int32_t T, const void* S,
                        const double* w_src, const double* w_snk, void* C,
                        double* A, void* pair_det, void* stream) {
  if (!pl) return fail(MHC_E_ARG, "mhc_contract: NULL plan");
  if (!S || !w_src || !w_snk || !C)
    return fail(MHC_E_ARG, "mhc_contract: NULL buffer");
  if (T < 1) return fail(MHC_E_ARG, "mhc_contract: T < 1");
  if (T > 65535) return fail(MHC_E_ARG, "mhc_contract: T > 65535");
  if (method != MHC_PLAIN_LU && method != MHC_UPDATE_TREE)
    return fail(MHC_E_ARG, "mhc_contract: unknown method");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "mhc_contract/hipGetDevice");
  if (cur != pl->device)
    return fail(MHC_E_DEVICE, "mhc_contract: current device differs from "
                              "the plan's device");
  if (pair_det && pl->F > 4)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract: pair_det output supports at most 4 flavour blocks");
  const bool tree = method == MHC_UPDATE_TREE;
  const bool diag = A != nullptr || pair_det != nullptr;
  // one matrix per lane when every block has the same size n <= 8, else one
  // group of lanes per matrix
  const bool narrow = pl->uniform_n && pl->n <= 8;
  const int sinks_per_item = narrow ? kSinkBlock : mhc::kern::wide_sinks_per_wave(pl->n);
  const int waves_per_block = narrow ? 4 : 8;
  const int rowsets = tree ? pl->n_dom : pl->n_src;
  const int n_sblk = (pl->n_snk + sinks_per_item - 1) / sinks_per_item;
  const long long n_items = (long long)rowsets * n_sblk;
  if (n_items > 0x7fffffffLL)
    return fail(MHC_E_UNSUPPORTED, "mhc_contract: too many work items");
  int n_blk_t = (kTargetBlocks + T - 1) / T;
  n_blk_t = (int)std::min<long long>(n_blk_t, (n_items + waves_per_block - 1) / waves_per_block);
  n_blk_t = std::max(1, n_blk_t);
  const size_t need = (size_t)T * n_blk_t * 3;
  if (need > pl->partial_cap) {
    if (pl->partial) {
      e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
      if (e != hipSuccess) return hip_fail(e, "mhc_contract/sync");
      hipFree(pl->partial);
      pl->partial = nullptr;
      pl->partial_cap = 0;
    }
    e = hipMalloc(&pl->partial, need * sizeof(double));
    if (e != hipSuccess)
      return fail(MHC_E_OOM, std::string("mhc_contract/hipMalloc: ") +
                                 hipGetErrorString(e));
    pl->partial_cap = need;
  }
  mhc::kern::ContractArgs a{};
  a.plan = pl->view;
  a.S = static_cast<const double2*>(S);
  a.w_src = w_src;
  a.w_snk = w_snk;
  a.partial = pl->partial;
  a.pair_det = static_cast<double2*>(pair_det);
  a.fallback = pl->fallback;
  a.T = T;
  a.n_items = (int)n_items;
  a.n_blk_t = n_blk_t;
  a.n_sblk = n_sblk;
  if (narrow)
    e = mhc::kern::launch_contract(a, pl->n, tree, diag, static_cast<double2*>(C), A,
                                   reinterpret_cast<hipStream_t>(stream));
  else
    e = mhc::kern::launch_contract_wide(a, pl->n, tree, diag, static_cast<double2*>(C), A,
                                        reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mhc_contract/launch");
  return MHC_OK;
}

mhc_status mhc_contract_backward(mhc_plan* pl, int32_t T, const void* S,
                                 const double* w_src, const double* w_snk,
                                 const void* gC, void* gS, double* g_wsrc,
                                 double* g_wsnk, void* stream) {
  if (!pl) return fail(MHC_E_ARG, "mhc_contract_backward: NULL plan");
  if (!S || !w_src || !w_snk || !gC)
    return fail(MHC_E_ARG, "mhc_contract_backward: NULL input buffer");
  if (T < 1 || T > 65535)
    return fail(MHC_E_ARG, "mhc_contract_backward: T outside [1, 65535]");
  if (pl->F > 4)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract_backward: more than 4 flavour blocks");
  if (!pl->uniform_n || pl->n > 8)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract_backward: flavour blocks must share one size n <= 8");
  if ((size_t)2 * pl->M * pl->M * 16 > 160 * 1024 - 4096)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract_backward: S_t and its gradient must fit in LDS");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "mhc_contract_backward/hipGetDevice");
  if (cur != pl->device)
    return fail(MHC_E_DEVICE, "mhc_contract_backward: current device differs "
                              "from the plan's device");
  const int n_sblk = pl->n_snk_pad / kSinkBlock;
  const size_t MM = (size_t)pl->M * pl->M;
  const size_t b_gS = (size_t)T * n_sblk * MM * 16;
  const size_t b_src = ((size_t)T * pl->n_src * n_sblk * 8 + 255) & ~size_t(255);
  const size_t b_snk = (size_t)T * pl->n_snk_pad * 8;
  const size_t need = b_gS + b_src + b_snk;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (need > pl->adj_cap) {
    if (pl->adj_scratch) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_fail(e, "mhc_contract_backward/sync");
      hipFree(pl->adj_scratch);
      pl->adj_scratch = nullptr;
      pl->adj_cap = 0;
    }
    e = hipMalloc(&pl->adj_scratch, need);
    if (e != hipSuccess)
      return fail(MHC_E_OOM, std::string("mhc_contract_backward/hipMalloc: ") +
                                 hipGetErrorString(e));
    pl->adj_cap = need;
  }
  char* base = static_cast<char*>(pl->adj_scratch);
  mhc::kern::AdjointArgs a{};
  a.plan = pl->view;
  a.S = static_cast<const double2*>(S);
  a.w_src = w_src;
  a.w_snk = w_snk;
  a.gC = static_cast<const double2*>(gC);
  a.part_gS = reinterpret_cast<double2*>(base);
  a.part_wsrc = reinterpret_cast<double*>(base + b_gS);
  a.part_wsnk = reinterpret_cast<double*>(base + b_gS + b_src);
  a.singular = pl->singular;
  a.T = T;
  a.n_sblk = n_sblk;
  e = mhc::kern::launch_adjoint(a, pl->n, static_cast<double2*>(gS), g_wsrc, g_wsnk, s);
  if (e != hipSuccess) return hip_fail(e, "mhc_contract_backward/launch");
  return MHC_OK;
}

mhc_status mhc_plan_status(mhc_plan* pl, int64_t* n_fallback,
                           int64_t* n_singular_grad) {
  if (!pl) return fail(MHC_E_ARG, "mhc_plan_status: NULL plan");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "mhc_plan_status/sync");
  unsigned long long v[2] = {0, 0};
  e = hipMemcpy(v, pl->fallback, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "mhc_plan_status/copy");
  if (n_fallback) *n_fallback = (int64_t)v[0];
  if (n_singular_grad) *n_singular_grad = (int64_t)v[1];
  return MHC_OK;
}

}  // extern "C"
