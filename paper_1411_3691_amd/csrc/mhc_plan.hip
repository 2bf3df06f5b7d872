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
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "contract_kernels.h"
#include "lu_device.h"
#include "mhc_internal.h"

using mhc::fail;

struct mhc_plan {
  int device = 0;
  int32_t n_src = 0, n_snk = 0, n_snk_pad = 0, M = 0, F = 0, sn = 0;
  int32_t n = 0;          // largest flavour block
  bool uniform_n = true;  // every flavour block has size n
  int32_t n_dom = 0, n_groups = 0, n_children = 0;
  int32_t max_dom_groups = 0;          // most groups of one dominator
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
  // sink terms (host copy) and the attached sink tree, if any
  std::vector<int32_t> snk_idx;
  void* dev_tree2 = nullptr;
  mhc::kern::SinkTreeView view_snk{};
  mhc::kern::SinkRec* srec_call = nullptr;  // in dev_tree2: the per-call sink records
  int32_t n_sdom = 0, n_sgroups = 0, n_schildren = 0;
  bool set_edges = false;              // the source tree has set edges
  bool rows_built[2] = {false, false}; // multi-row tables: update tree, plain
  std::vector<int4> rows_tiles[2];     // their tiles (host copy, for the batch's costs)
};

// Workgroup partial sums of mhc_contract_noalloc: a file-scope device array
// (each GPU the library runs on holds its own copy until the process ends),
// so that entry point never allocates.  2 MiB covers every valid T: a call
// needs T * ceil(4096 / T) * 3 <= 3 * (4096 + 65534) doubles.
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 18;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {

constexpr int kSinkBlock = 64;
// Workgroups per single-job launch (over all slices): 4096 measured equal
// or faster than 1024, 2048 and 8192 for every lane-kernel method on the
// mid workload (the plain LU 5 % faster than with 2048).
constexpr int kTargetBlocks = 4096;
// The LDS of one workgroup of the multi-row group kernels: 160 KiB less
// 1 KiB for their static arrays.
constexpr size_t kRowsLdsLimit = 159 * 1024;

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

// Device address of `scratch` on each device, taken once per device (with
// that device current) by hipGetSymbolAddress: in host code the array's
// name is only a host-side stand-in.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};

mhc_status noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(MHC_E_DEVICE, "mhc_contract_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "mhc_contract_noalloc/hipGetSymbolAddress");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MHC_OK;
}

// Units and tiles of the multi-row group kernels for one method (host
// copy).  Tree: one unit per dominator, its rows (flavour-major) then the
// distinct new rows of its children; a dominator whose rows exceed cap is
// split by ranges of its children, each unit staging the dominator's rows
// again (only the first counts the dominator's own term).  Plain: one unit
// per source term.  Tiles take consecutive units while their rows fit cap
// and their (unit, sink block) items stay within target; a unit with more
// items than target is cut into tiles by ranges of sinks.
struct RowsHost {
  std::vector<int4> tiles, unit;
  std::vector<int2> unit_c;
  std::vector<int32_t> unit_row, rows, child_lrow;
  int max_rows = 0;
};

bool build_rows(const mhc_terms& src, const mhc_tree* tree, int n_snk, int spw, int waves,
                int cap, RowsHost& h) {
  const int sn = src.sn;
  if (cap < sn + 1 || spw < 1) return false;
  h = RowsHost{};
  h.unit_row.push_back(0);
  auto add_unit = [&](int rs, int g0, int g1, bool primary, int c0, int c1,
                      const std::vector<int32_t>& r) {
    h.unit.push_back(make_int4(rs, g0, g1, primary ? 1 : 0));
    h.unit_c.push_back(make_int2(c0, c1));
    h.rows.insert(h.rows.end(), r.begin(), r.end());
    h.unit_row.push_back((int32_t)h.rows.size());
  };
  if (!tree) {
    for (int i = 0; i < src.n_terms; ++i) {
      std::vector<int32_t> r(src.idx.begin() + (size_t)i * sn,
                             src.idx.begin() + (size_t)(i + 1) * sn);
      add_unit(i, 0, 0, true, 0, 0, r);
    }
  } else {
    h.child_lrow.assign(tree->grp_child.size(), 0);
    const int n_dom = (int)tree->dom_order.size();
    for (int k = 0; k < n_dom; ++k) {
      const int d = tree->dom_order[k];
      const int gb = tree->dom_grp[k], ge = tree->dom_grp[k + 1];
      const int cb = tree->grp_ptr[gb], ce = tree->grp_ptr[ge];
      std::vector<int32_t> base(src.idx.begin() + (size_t)d * sn,
                                src.idx.begin() + (size_t)(d + 1) * sn);
      std::vector<int32_t> r = base;
      int c0 = cb;
      bool primary = true;
      auto close = [&](int c1) {
        // the groups whose children overlap [c0, c1)
        int g0 = gb, g1 = gb;
        if (c1 > c0) {
          while (tree->grp_ptr[g0 + 1] <= c0) ++g0;
          g1 = g0;
          while (g1 < ge && tree->grp_ptr[g1] < c1) ++g1;
        }
        add_unit(k, g0, g1, primary, c0, c1, r);
      };
      for (int c = cb; c < ce; ++c) {
        if (c - c0 >= mhc::kern::kRowsChildCap) {
          close(c);
          primary = false;
          c0 = c;
          r = base;
        }
        const int32_t row = tree->cnew[tree->grp_child[c]];
        int at = -1;
        for (size_t q = 0; q < r.size(); ++q)
          if (r[q] == row) {
            at = (int)q;
            break;
          }
        if (at < 0) {
          if ((int)r.size() + 1 > cap) {
            close(c);
            primary = false;
            c0 = c;
            r = base;
          }
          at = (int)r.size();
          r.push_back(row);
        }
        h.child_lrow[c] = at;
      }
      close(ce);
    }
  }
  // tiles
  const int n_units = (int)h.unit.size();
  const int n_sb = (n_snk + spw - 1) / spw;
  const int target = std::max(waves * 32, 1);
  int u = 0;
  while (u < n_units) {
    const int ur = h.unit_row[u + 1] - h.unit_row[u];
    if (n_sb >= target || u + 1 == n_units) {
      // this unit alone, cut by ranges of sinks
      const int n_split = std::max(1, (n_sb + target - 1) / target);
      const int per = (n_sb + n_split - 1) / n_split * spw;
      for (int s0 = 0; s0 < n_snk; s0 += per)
        h.tiles.push_back(make_int4(u, u + 1, s0, std::min(n_snk, s0 + per)));
      h.max_rows = std::max(h.max_rows, ur);
      ++u;
      continue;
    }
    int u1 = u, rows = 0, items = 0, kids = 0;
    while (u1 < n_units) {
      const int r1 = h.unit_row[u1 + 1] - h.unit_row[u1];
      const int k1 = h.unit_c[u1].y - h.unit_c[u1].x;
      if (u1 > u && (rows + r1 > cap || items + n_sb > target ||
                     kids + k1 > mhc::kern::kRowsChildCap))
        break;
      rows += r1;
      items += n_sb;
      kids += k1;
      ++u1;
    }
    h.tiles.push_back(make_int4(u, u1, 0, n_snk));
    h.max_rows = std::max(h.max_rows, rows);
    u = u1;
  }
  if (n_snk == 0) h.tiles.clear();
  return true;
}

// LDS of a multi-row launch beyond the pivot-row buffers: the wave and
// tile tables and the most rows any tile of the method's table stages.
size_t rows_lds_bytes(const mhc_plan* pl, bool tree) {
  const mhc::kern::RowsGeometry geo = mhc::kern::rows_geometry(pl->n, tree);
  const mhc::kern::RowsTable& rt = tree ? pl->view.rows_tree : pl->view.rows_plain;
  return mhc::kern::rows_meta_bytes(geo.waves, geo.spw, pl->sn) +
         (size_t)rt.max_rows * mhc::kern::lds_row(pl->M) * 16;
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
  if (mhc::kern::lds_slice_bytes(src.M) > 150 * 1024)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_plan_create: a slice of S (M*(M+1)*16 bytes in LDS) must fit in "
                "150 KiB");

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
  for (int k = 0; k < pl->n_dom; ++k)
    pl->max_dom_groups = std::max(pl->max_dom_groups, tree->dom_grp[k + 1] - tree->dom_grp[k]);
  pl->snk_idx = snk->idx;
  pl->set_edges = tree->set_edges;

  const int sn = src.sn;
  const uint32_t row_bytes = (uint32_t)mhc::kern::lds_row(src.M) * 16u;  // LDS row stride
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
  std::vector<double> child_wsgn(pl->n_children);
  for (int c = 0; c < pl->n_children; ++c) {
    const int u = tree->grp_child[c];
    child_rowoff[c] = (uint32_t)tree->cnew[u] * row_bytes;
    child_wsgn[c] = tree->sign[u] < 0 ? -1.0 : 1.0;
  }
  std::vector<int32_t> term_owner(tree->owner), term_fr(src.n_terms, -1);
  std::vector<uint32_t> term_crow(src.n_terms, 0u);
  for (int u = 0; u < src.n_terms; ++u)
    if (tree->owner[u] != u) {
      term_fr[u] = (tree->flav[u] << 8) | tree->pos[u] | (tree->sign[u] < 0 ? 1 << 16 : 0);
      term_crow[u] = (uint32_t)tree->cnew[u] * row_bytes;
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

  // multi-row group kernels: the tables of both methods for the plan's
  // bucket (none where the rows of one unit cannot fit the LDS)
  RowsHost rows_h[2];
  bool rows_ok[2] = {false, false};
  if (mhc::kern::rows_bucket(nmax) > 0) {
    for (int q = 0; q < 2; ++q) {
      const mhc::kern::RowsGeometry geo = mhc::kern::rows_geometry(nmax, q == 0);
      const size_t fixed = geo.buf_bytes + mhc::kern::rows_meta_bytes(geo.waves, geo.spw, sn);
      const size_t avail = fixed < kRowsLdsLimit ? kRowsLdsLimit - fixed : 0;
      const int cap = (int)(avail / row_bytes);
      rows_ok[q] = build_rows(src, q == 0 ? tree : nullptr, snk->n_terms, geo.spw, geo.waves,
                              cap, rows_h[q]);
    }
  }

  std::vector<char> img;
  size_t o_rows[2][7] = {};
  for (int q = 0; q < 2; ++q) {
    if (!rows_ok[q]) continue;
    o_rows[q][0] = append(img, rows_h[q].tiles);
    o_rows[q][1] = append(img, rows_h[q].unit);
    o_rows[q][2] = append(img, rows_h[q].unit_c);
    o_rows[q][3] = append(img, rows_h[q].unit_row);
    o_rows[q][4] = append(img, rows_h[q].rows);
    o_rows[q][5] = append(img, rows_h[q].child_lrow);
  }
  const size_t o_dom_term = append(img, dom_term);
  const size_t o_dom_rowoff = append(img, dom_rowoff);
  const size_t o_dom_grp = append(img, tree->dom_grp);
  const size_t o_grp_fr = append(img, grp_fr);
  const size_t o_grp_ptr = append(img, tree->grp_ptr);
  const size_t o_child_rowoff = append(img, child_rowoff);
  const size_t o_child_term = append(img, child_term);
  const size_t o_child_wsgn = append(img, child_wsgn);
  const size_t o_src_rowoff = append(img, src_rowoff);
  const size_t o_snk_coloff = append(img, snk_coloff);
  const size_t o_term_owner = append(img, term_owner);
  const size_t o_term_fr = append(img, term_fr);
  const size_t o_term_crow = append(img, term_crow);
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
  v.child_wsgn = reinterpret_cast<const double*>(base + o_child_wsgn);
  v.src_rowoff = reinterpret_cast<const uint32_t*>(base + o_src_rowoff);
  v.snk_coloff = reinterpret_cast<const uint32_t*>(base + o_snk_coloff);
  v.term_owner = reinterpret_cast<const int32_t*>(base + o_term_owner);
  v.term_fr = reinterpret_cast<const int32_t*>(base + o_term_fr);
  v.term_crow = reinterpret_cast<const uint32_t*>(base + o_term_crow);
  for (int q = 0; q < 2; ++q) {
    mhc::kern::RowsTable& rt = q == 0 ? v.rows_tree : v.rows_plain;
    rt = mhc::kern::RowsTable{};
    if (!rows_ok[q]) continue;
    rt.n_tiles = (int32_t)rows_h[q].tiles.size();
    rt.max_rows = rows_h[q].max_rows;
    rt.tiles = reinterpret_cast<const int4*>(base + o_rows[q][0]);
    rt.unit = reinterpret_cast<const int4*>(base + o_rows[q][1]);
    rt.unit_c = reinterpret_cast<const int2*>(base + o_rows[q][2]);
    rt.unit_row = reinterpret_cast<const int32_t*>(base + o_rows[q][3]);
    rt.rows = reinterpret_cast<const int32_t*>(base + o_rows[q][4]);
    rt.child_lrow = reinterpret_cast<const int32_t*>(base + o_rows[q][5]);
  }
  pl->rows_built[0] = rows_ok[0];
  pl->rows_built[1] = rows_ok[1];
  pl->rows_tiles[0] = std::move(rows_h[0].tiles);
  pl->rows_tiles[1] = std::move(rows_h[1].tiles);
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
  if (pl->dev_tree2) hipFree(pl->dev_tree2);
  if (pl->dev_tables) hipFree(pl->dev_tables);
  hipSetDevice(cur);
  delete pl;
}

mhc_status mhc_plan_attach_sink_tree(mhc_plan* pl, const mhc_tree* st, void* stream) {
  if (!pl || !st) return fail(MHC_E_ARG, "mhc_plan_attach_sink_tree: NULL handle");
  const mhc_terms& t = st->terms;
  if (t.n_terms != pl->n_snk || t.sn != pl->sn || t.M != pl->M || t.off != pl->off ||
      t.idx != pl->snk_idx)
    return fail(MHC_E_SHAPE,
                "mhc_plan_attach_sink_tree: the tree is not built on the plan's sink terms");
  if (!pl->uniform_n || pl->n > 8)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_plan_attach_sink_tree: two-sided trees need every flavour block of "
                "size n <= 8");
  if (st->set_edges)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_plan_attach_sink_tree: two-sided trees need positional edges");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "mhc_plan_attach_sink_tree/hipGetDevice");
  if (cur != pl->device)
    return fail(MHC_E_DEVICE, "mhc_plan_attach_sink_tree: current device differs from "
                              "the plan's device");
  const int nd = (int)st->dom_order.size();
  // processing order: most children first, then most groups, then tree order
  std::vector<int32_t> order(nd);
  for (int k = 0; k < nd; ++k) order[k] = k;
  auto n_children = [&](int k) {
    return st->grp_ptr[st->dom_grp[k + 1]] - st->grp_ptr[st->dom_grp[k]];
  };
  auto n_groups = [&](int k) { return st->dom_grp[k + 1] - st->dom_grp[k]; };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (n_children(x) != n_children(y)) return n_children(x) > n_children(y);
    return n_groups(x) > n_groups(y);
  });
  const int pad = (nd + kSinkBlock - 1) / kSinkBlock * kSinkBlock;
  const int sn = pl->sn;
  std::vector<int32_t> sdom_term(pad), sdom_grp(pad + 1), sgrp_fc, sgrp_ptr(1, 0), schild_term;
  std::vector<uint32_t> sdom_coloff((size_t)sn * pad), schild_coloff;
  for (int k = 0; k < pad; ++k) {
    const int kk = k < nd ? order[k] : order[0];
    const int term = st->dom_order[kk];
    sdom_term[k] = term;
    for (int q = 0; q < sn; ++q)
      sdom_coloff[(size_t)q * pad + k] = (uint32_t)t.idx[(size_t)term * sn + q] * 16u;
    sdom_grp[k] = (int32_t)sgrp_fc.size();
    if (k >= nd) continue;
    for (int g = st->dom_grp[kk]; g < st->dom_grp[kk + 1]; ++g) {
      const int f = st->grp_f[g], c = st->grp_r[g];
      sgrp_fc.push_back((f << 8) | c);
      for (int ci = st->grp_ptr[g]; ci < st->grp_ptr[g + 1]; ++ci) {
        const int u = st->grp_child[ci];
        schild_term.push_back(u);
        schild_coloff.push_back((uint32_t)t.idx[(size_t)u * sn + t.off[f] + c] * 16u);
      }
      sgrp_ptr.push_back((int32_t)schild_term.size());
    }
  }
  sdom_grp[pad] = (int32_t)sgrp_fc.size();
  // slot-major child records per flavour (processing order of the sink
  // dominators), padded with records that match no column
  const int F = pl->F;
  const int n_sb = pad / kSinkBlock;
  std::vector<int32_t> cnt((size_t)F * pad, 0), srec_cnt((size_t)F * n_sb, 0), rbase(9, 0);
  for (int k = 0; k < nd; ++k)
    for (int g = st->dom_grp[order[k]]; g < st->dom_grp[order[k] + 1]; ++g)
      cnt[(size_t)st->grp_f[g] * pad + k] += st->grp_ptr[g + 1] - st->grp_ptr[g];
  int rows = 0;
  for (int f = 0; f < F; ++f) {
    rbase[f] = rows;
    int mf = 0;
    for (int b = 0; b < n_sb; ++b) {
      int m = 0;
      for (int k = b * kSinkBlock; k < (b + 1) * kSinkBlock; ++k)
        m = std::max(m, cnt[(size_t)f * pad + k]);
      srec_cnt[(size_t)f * n_sb + b] = m;
      mf = std::max(mf, m);
    }
    rows += mf;
  }
  std::vector<int4> srec((size_t)rows * pad, make_int4(0, (int)0xffffffffu, -1, 0));
  {
    std::vector<int32_t> fill((size_t)F * pad, 0);
    for (int k = 0; k < nd; ++k) {
      const int kk = order[k];
      const int dterm = st->dom_order[kk];
      for (int g = st->dom_grp[kk]; g < st->dom_grp[kk + 1]; ++g) {
        const int f = st->grp_f[g], c = st->grp_r[g];
        const uint32_t ccol = (uint32_t)t.idx[(size_t)dterm * sn + t.off[f] + c] * 16u;
        for (int ci = st->grp_ptr[g]; ci < st->grp_ptr[g + 1]; ++ci) {
          const int u = st->grp_child[ci];
          const int i = fill[(size_t)f * pad + k]++;
          srec[(size_t)(rbase[f] + i) * pad + k] =
              make_int4((int)((uint32_t)t.idx[(size_t)u * sn + t.off[f] + c] * 16u), (int)ccol, u, 0);
        }
      }
    }
  }
  std::vector<char> img;
  const size_t o_term = append(img, sdom_term);
  const size_t o_coloff = append(img, sdom_coloff);
  const size_t o_grp = append(img, sdom_grp);
  const size_t o_fc = append(img, sgrp_fc);
  const size_t o_ptr = append(img, sgrp_ptr);
  const size_t o_ccol = append(img, schild_coloff);
  const size_t o_cterm = append(img, schild_term);
  const size_t o_srec = append(img, srec);
  const size_t o_scnt = append(img, srec_cnt);
  // then room for the per-call records (SinkRec, 16 bytes each)
  const size_t o_call = (img.size() + 255) & ~size_t(255);
  const size_t dev_bytes = o_call + srec.size() * sizeof(mhc::kern::SinkRec);
  void* dev = nullptr;
  e = hipMalloc(&dev, dev_bytes);
  if (e != hipSuccess) return fail(MHC_E_OOM, "mhc_plan_attach_sink_tree: device tables");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  e = hipMemcpyAsync(dev, img.data(), img.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    hipFree(dev);
    return hip_fail(e, "mhc_plan_attach_sink_tree/upload");
  }
  if (pl->dev_tree2) {
    // a previous sink tree may still be read by queued work
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      hipFree(dev);
      return hip_fail(e, "mhc_plan_attach_sink_tree/sync");
    }
    hipFree(pl->dev_tree2);
  }
  pl->dev_tree2 = dev;
  char* base = static_cast<char*>(dev);
  mhc::kern::SinkTreeView& v = pl->view_snk;
  v.n_sdom = nd;
  v.n_sdom_pad = pad;
  v.sdom_term = reinterpret_cast<const int32_t*>(base + o_term);
  v.sdom_coloff = reinterpret_cast<const uint32_t*>(base + o_coloff);
  v.sdom_grp = reinterpret_cast<const int32_t*>(base + o_grp);
  v.sgrp_fc = reinterpret_cast<const int32_t*>(base + o_fc);
  v.sgrp_ptr = reinterpret_cast<const int32_t*>(base + o_ptr);
  v.schild_coloff = reinterpret_cast<const uint32_t*>(base + o_ccol);
  v.schild_term = reinterpret_cast<const int32_t*>(base + o_cterm);
  v.srec_static = reinterpret_cast<const int4*>(base + o_srec);
  v.srec_cnt = reinterpret_cast<const int32_t*>(base + o_scnt);
  for (int f = 0; f < 9; ++f) v.srec_base[f] = rbase[f];
  v.n_srec = (int32_t)srec.size();
  pl->srec_call = reinterpret_cast<mhc::kern::SinkRec*>(base + o_call);
  pl->n_sdom = nd;
  pl->n_sgroups = (int32_t)sgrp_fc.size();
  pl->n_schildren = (int32_t)schild_term.size();
  return MHC_OK;
}

// The forward contraction behind mhc_contract and mhc_contract_noalloc:
// `fixed` (capacity fixed_cap doubles) replaces the plan's growing partial
// buffer when not NULL.
static mhc_status contract_impl(mhc_plan* pl, int32_t method, int32_t T, const void* S,
                                const double* w_src, const double* w_snk, void* C,
                                double* A, void* pair_det, const int32_t* pairs,
                                int64_t n_pairs, void* stream, double* fixed,
                                size_t fixed_cap) {
  if (!pl) return fail(MHC_E_ARG, "mhc_contract: NULL plan");
  if (!S || !w_src || !w_snk || !C)
    return fail(MHC_E_ARG, "mhc_contract: NULL buffer");
  if (T < 1) return fail(MHC_E_ARG, "mhc_contract: T < 1");
  if (T > 65535) return fail(MHC_E_ARG, "mhc_contract: T > 65535");
  if (method < MHC_PLAIN_LU || method > MHC_UPDATE_TREE_AGG)
    return fail(MHC_E_ARG, "mhc_contract: unknown method");
  const bool agg = method == MHC_UPDATE_TREE_AGG;
  if (agg && (A || (pair_det && !pairs)))
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract: the weighted-row aggregation forms no per-pair values (A and "
                "the dense pair_det must be NULL; sampled pairs are evaluated by the tree)");
  const int pivot = (method == MHC_PLAIN_LU_UNPIVOTED || method == MHC_UPDATE_TREE_UNPIVOTED) ? 0
                    : (method == MHC_PLAIN_LU_THRESHOLD || method == MHC_UPDATE_TREE_THRESHOLD)
                        ? 2
                        : 1;
  if (pivot != 1 && !(pl->uniform_n && pl->n <= 8))
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract: the unpivoted and threshold-pivoting methods need every flavour "
                "block of size n <= 8");
  if (method == MHC_UPDATE_TREE2) {
    if (pl->set_edges)
      return fail(MHC_E_UNSUPPORTED,
                  "mhc_contract: the two-sided method needs positional edges (the source "
                  "tree was built with MHC_TREE_SET_EDGES)");
    if (!pl->dev_tree2)
      return fail(MHC_E_STATE, "mhc_contract: no sink tree attached to the plan");
    if (A || pair_det)
      return fail(MHC_E_UNSUPPORTED,
                  "mhc_contract: the two-sided method computes neither A nor pair dets");
  }
  if (pairs) {
    if (!pair_det) return fail(MHC_E_ARG, "mhc_contract: pairs given without pair_det");
    if (n_pairs < 0 || n_pairs > 0x7fffffffLL)
      return fail(MHC_E_ARG, "mhc_contract: n_pairs outside [0, 2^31)");
  } else if (n_pairs != 0) {
    return fail(MHC_E_ARG, "mhc_contract: n_pairs without pairs");
  }
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "mhc_contract/hipGetDevice");
  if (cur != pl->device)
    return fail(MHC_E_DEVICE, "mhc_contract: current device differs from "
                              "the plan's device");
  if (pair_det && pl->F > 4)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract: pair_det output supports at most 4 flavour blocks");
  const bool two = method == MHC_UPDATE_TREE2;
  const bool tree = method == MHC_UPDATE_TREE || method == MHC_UPDATE_TREE_UNPIVOTED ||
                    method == MHC_UPDATE_TREE_THRESHOLD || agg;
  // the dense pair table comes from the contraction kernels themselves; a
  // sampled list from the per-pair kernels after them
  void* dense_pairs = pairs ? nullptr : pair_det;
  const bool diag = A != nullptr || dense_pairs != nullptr;
  // one matrix per lane when every block has the same size n <= 8, else one
  // group of lanes per matrix
  const bool narrow = pl->uniform_n && pl->n <= 8;
  // several rows of a matrix per lane (blocks up to 16), from the plan's
  // tiles; the per-pair table and the other pivoting rules keep the
  // one-row-per-lane kernels
  const mhc::kern::RowsTable& rtab = tree ? pl->view.rows_tree : pl->view.rows_plain;
  const bool rows = !narrow && !two && !dense_pairs && pivot == 1 &&
                    pl->rows_built[tree ? 0 : 1] && rtab.n_tiles > 0;
  const int sinks_per_item = narrow ? kSinkBlock : mhc::kern::wide_sinks_per_wave(pl->n);
  const int waves_per_block = narrow ? 4 : 8;
  const int rowsets = (tree || two) ? pl->n_dom : pl->n_src;
  const int n_sblk = two ? pl->view_snk.n_sdom_pad / kSinkBlock
                         : (pl->n_snk + sinks_per_item - 1) / sinks_per_item;
  const long long n_items = (long long)rowsets * n_sblk;
  if (n_items > 0x7fffffffLL)
    return fail(MHC_E_UNSUPPORTED, "mhc_contract: too many work items");
  int n_blk_t = (kTargetBlocks + T - 1) / T;
  if (rows)
    n_blk_t = std::min(n_blk_t, rtab.n_tiles);
  else
    n_blk_t = (int)std::min<long long>(n_blk_t,
                                       (n_items + waves_per_block - 1) / waves_per_block);
  n_blk_t = std::max(1, n_blk_t);
  // two-sided: a flag per workgroup after the partials (ints, two per double)
  const size_t need = (size_t)T * n_blk_t * 3 + (two ? ((size_t)T * n_blk_t + 1) / 2 : 0);
  if (fixed) {
    if (need > fixed_cap)
      return fail(MHC_E_UNSUPPORTED,
                  "mhc_contract_noalloc: the partial sums need " + std::to_string(need) +
                      " doubles, more than the " + std::to_string(fixed_cap) +
                      " of the static scratch");
  } else if (need > pl->partial_cap) {
    if (pl->partial) {
      // earlier calls may still read the old buffer, on any stream
      e = hipDeviceSynchronize();
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
  a.partial = fixed ? fixed : pl->partial;
  a.pair_det = static_cast<double2*>(dense_pairs);
  a.fallback = pl->fallback;
  a.T = T;
  a.n_items = (int)n_items;
  a.n_blk_t = n_blk_t;
  a.n_sblk = n_sblk;
  a.snk = pl->view_snk;
  a.srec = pl->srec_call;
  if (two) {
    // per wave, the source dominator's aggregated child rows (one row of M
    // entries per group) beside the slice, where the LDS holds them
    const size_t tab = (size_t)mhc::kern::kWavesPerBlock * pl->max_dom_groups * pl->M * 16;
    a.tab_rows = mhc::kern::lds_slice_bytes(pl->M) + tab + mhc::kern::kTwoSidedSlotBytes <=
                         mhc::kern::kTwoSidedLdsLimit
                     ? pl->max_dom_groups
                     : 0;
  }
  if (two)
    e = mhc::kern::launch_contract_two_sided(a, pl->n, static_cast<double2*>(C),
                                             reinterpret_cast<hipStream_t>(stream));
  else if (rows)
    e = mhc::kern::launch_contract_rows(
        a, pl->n, tree, A != nullptr, agg,
        rows_lds_bytes(pl, tree), static_cast<double2*>(C), A,
        reinterpret_cast<hipStream_t>(stream));
  else if (narrow)
    e = mhc::kern::launch_contract(a, pl->n, tree, diag, agg ? 3 : pivot,
                                   static_cast<double2*>(C), A,
                                   reinterpret_cast<hipStream_t>(stream));
  else
    e = mhc::kern::launch_contract_wide(a, pl->n, tree, diag, static_cast<double2*>(C), A,
                                        reinterpret_cast<hipStream_t>(stream), agg);
  if (e != hipSuccess) return hip_fail(e, "mhc_contract/launch");
  if (pairs && n_pairs > 0) {
    mhc::kern::PairArgs pa{};
    pa.plan = pl->view;
    pa.S = static_cast<const double2*>(S);
    pa.pairs = pairs;
    pa.out = static_cast<double2*>(pair_det);
    pa.T = T;
    pa.n_pairs = (int)n_pairs;
    e = mhc::kern::launch_pairs(pa, pl->n, narrow, tree, pivot,
                                reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mhc_contract/pairs");
  }
  return MHC_OK;
}

mhc_status mhc_contract(mhc_plan* pl, int32_t method, int32_t T, const void* S,
                        const double* w_src, const double* w_snk, void* C,
                        double* A, void* pair_det, const int32_t* pairs, int64_t n_pairs,
                        void* stream) {
  return contract_impl(pl, method, T, S, w_src, w_snk, C, A, pair_det, pairs, n_pairs, stream,
                       nullptr, 0);
}

mhc_status mhc_contract_noalloc(mhc_plan* pl, int32_t method, int32_t T, const void* S,
                                const double* w_src, const double* w_snk, void* C, double* A,
                                void* stream) {
  if (!pl) return fail(MHC_E_ARG, "mhc_contract_noalloc: NULL plan");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "mhc_contract_noalloc/hipGetDevice");
  if (cur != pl->device)
    return fail(MHC_E_DEVICE, "mhc_contract_noalloc: current device differs from the plan's "
                              "device");
  double* ptr = nullptr;
  const mhc_status st = noalloc_scratch(cur, &ptr);
  if (st != MHC_OK) return st;
  return contract_impl(pl, method, T, S, w_src, w_snk, C, A, nullptr, nullptr, 0, stream, ptr,
                       kNoAllocScratchDoubles);
}

mhc_status mhc_contract_backward(mhc_plan* pl, int32_t method, int32_t T, const void* S,
                                 const double* w_src, const double* w_snk,
                                 const void* gC, void* gS, double* g_wsrc,
                                 double* g_wsnk, void* stream) {
  if (!pl) return fail(MHC_E_ARG, "mhc_contract_backward: NULL plan");
  if (!S || !w_src || !w_snk || !gC)
    return fail(MHC_E_ARG, "mhc_contract_backward: NULL input buffer");
  if (T < 1 || T > 65535)
    return fail(MHC_E_ARG, "mhc_contract_backward: T outside [1, 65535]");
  if (method != MHC_PLAIN_LU && method != MHC_UPDATE_TREE)
    return fail(MHC_E_ARG, "mhc_contract_backward: method must be MHC_PLAIN_LU or MHC_UPDATE_TREE");
  if (method == MHC_UPDATE_TREE && pl->set_edges)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract_backward: the tree adjoint needs positional edges (the source "
                "tree was built with MHC_TREE_SET_EDGES)");
  if (pl->F > 4)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract_backward: more than 4 flavour blocks");
  if (!pl->uniform_n || pl->n > 8)
    return fail(MHC_E_UNSUPPORTED,
                "mhc_contract_backward: flavour blocks must share one size n <= 8");
  if (2 * mhc::kern::lds_slice_bytes(pl->M) > 160 * 1024 - 4096)
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
  const size_t b_snk = ((size_t)T * pl->n_snk_pad * 8 + 255) & ~size_t(255);
  const bool tree_m = method == MHC_UPDATE_TREE;
  const size_t b_flag = tree_m ? ((size_t)T * n_sblk * pl->n_dom + 255) & ~size_t(255) : 0;
  const size_t b_crec = tree_m ? ((size_t)pl->n_children + 1) * sizeof(mhc::kern::ChildRec) : 0;
  const size_t need = b_gS + b_src + b_snk + b_flag + b_crec;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (need > pl->adj_cap) {
    if (pl->adj_scratch) {
      // earlier calls may still use the old scratch, on any stream
      e = hipDeviceSynchronize();
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
  a.dom_flag = tree_m ? reinterpret_cast<uint8_t*>(base + b_gS + b_src + b_snk) : nullptr;
  a.child_rec = tree_m ? reinterpret_cast<mhc::kern::ChildRec*>(base + b_gS + b_src + b_snk +
                                                                b_flag)
                       : nullptr;
  a.n_children = tree_m ? pl->n_children : 0;
  a.singular = pl->singular;
  a.T = T;
  a.n_sblk = n_sblk;
  e = mhc::kern::launch_adjoint(a, pl->n, method == MHC_UPDATE_TREE, static_cast<double2*>(gS),
                                g_wsrc, g_wsnk, s);
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

// ---------------------------------------------------------------- batches
//
// Many independent jobs (plan, slices, method) run as one graph: one
// persistent kernel per kernel variant walks a tile table (job, slice,
// chunk) sorted by predicted cost (largest first, dealt round-robin to the
// workgroups), then one kernel reduces every job's partials.  The graph is
// captured at the first run and replayed afterwards.

struct mhc_batch {
  int device = 0;
  int32_t method = MHC_UPDATE_TREE;
  mhc_schedule sched{};
  std::vector<mhc_plan*> plans;
  std::vector<int32_t> T;
  bool built = false;
  bool with_a = false;               // the captured kernels carry A
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  mhc::kern::ContractArgs* jobs_host = nullptr;  // pinned
  void* dev = nullptr;                           // jobs, tiles, (job, t), partials
  mhc::kern::ContractArgs* jobs_dev = nullptr;
  int n_tiles = 0, n_kernels = 0, n_jt = 0;
  int64_t n_pairs = 0;
  std::vector<const void*> last_ptrs;
};

namespace {

// Kernel families of a batch: one matrix per lane, one row per lane of a
// group, several rows per lane of a group.
enum BatchKind { kLane = 0, kWide = 1, kRows = 2 };

struct Bucket {
  int kind;
  int n;          // block size (lane kernels) or bucket bound (groups of lanes)
  size_t lds;     // slice of S (lane, wide) or most rows any tile stages (rows)
  std::vector<int4> tiles;
  std::vector<double> cost;
};

void batch_release(mhc_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->cap) hipStreamDestroy(b->cap);
  if (b->dev) hipFree(b->dev);
  if (b->jobs_host) hipHostFree(b->jobs_host);
  b->exec = nullptr;
  b->graph = nullptr;
  b->cap = nullptr;
  b->dev = nullptr;
  b->jobs_host = nullptr;
  b->built = false;
}

bool use_lane_kernel(const mhc_plan* pl, int32_t kernel) {
  if (kernel == MHC_SCHED_LANE) return true;
  if (kernel == MHC_SCHED_GROUP) return false;
  return pl->uniform_n && pl->n <= 8;
}

mhc_status batch_build(mhc_batch* b) {
  const int nj = (int)b->plans.size();
  int n_cu = 0;
  hipError_t e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/attribute");
  const bool tree = b->method == MHC_UPDATE_TREE;
  std::vector<mhc::kern::ContractArgs> jobs(nj);
  std::vector<size_t> part_off(nj);
  size_t part_total = 0;
  std::vector<Bucket> buckets;
  std::vector<int2> jt;
  b->n_pairs = 0;
  for (int j = 0; j < nj; ++j) {
    mhc_plan* pl = b->plans[j];
    const bool narrow = use_lane_kernel(pl, b->sched.kernel);
    const int q = tree ? 0 : 1;
    const bool rows = !narrow && b->sched.kernel != MHC_SCHED_GROUP && pl->rows_built[q] &&
                      !pl->rows_tiles[q].empty();
    if (rows) {
      // multi-row group kernels: one chunk per tile of the plan's table
      const mhc::kern::RowsTable& rt = tree ? pl->view.rows_tree : pl->view.rows_plain;
      const mhc::kern::RowsGeometry geo = mhc::kern::rows_geometry(pl->n, tree);
      mhc::kern::ContractArgs& a = jobs[j];
      a = mhc::kern::ContractArgs{};
      a.plan = pl->view;
      a.fallback = pl->fallback;
      a.T = b->T[j];
      a.n_blk_t = rt.n_tiles;
      part_off[j] = part_total;
      part_total += (size_t)a.T * rt.n_tiles * 3;
      b->n_pairs += (int64_t)a.T * pl->n_src * pl->n_snk;
      // predicted cost of one (unit, sink block) item: the eliminations,
      // the solves, the dots
      double item = 0.0;
      for (int f = 0; f < pl->F; ++f) {
        const double nf = pl->off[f + 1] - pl->off[f];
        item += nf * nf * nf;
      }
      if (tree && pl->n_dom > 0)
        item += (double)pl->n_groups / pl->n_dom * pl->n * pl->n +
                (double)pl->n_children / pl->n_dom * pl->n;
      item *= geo.spw;
      const int key_n = mhc::kern::rows_bucket(pl->n);
      Bucket* bk = nullptr;
      for (auto& x : buckets)
        if (x.kind == kRows && x.n == key_n) bk = &x;
      if (!bk) {
        buckets.push_back(Bucket{kRows, key_n, 0, {}, {}});
        bk = &buckets.back();
      }
      bk->lds = std::max(bk->lds, rows_lds_bytes(pl, tree));
      for (int t = 0; t < a.T; ++t) {
        jt.push_back(make_int2(j, t));
        for (int c = 0; c < rt.n_tiles; ++c) {
          const int4 tl = pl->rows_tiles[q][c];
          const double its = (double)(tl.y - tl.x) * ((tl.w - tl.z + geo.spw - 1) / geo.spw);
          bk->tiles.push_back(make_int4(j, t, c, 0));
          bk->cost.push_back(item * its);
        }
      }
      continue;
    }
    const int spi = narrow ? kSinkBlock : mhc::kern::wide_sinks_per_wave(pl->n);
    const int rowsets = tree ? pl->n_dom : pl->n_src;
    const int n_sblk = (pl->n_snk + spi - 1) / spi;
    const long long n_items = (long long)rowsets * n_sblk;
    if (n_items > 0x7fffffffLL) return fail(MHC_E_UNSUPPORTED, "mhc_batch_run: job too large");
    const int ipt = b->sched.items_per_tile > 0 ? b->sched.items_per_tile : (narrow ? 64 : 32);
    const int n_blk_t = (int)std::max<long long>(1, (n_items + ipt - 1) / ipt);
    mhc::kern::ContractArgs& a = jobs[j];
    a = mhc::kern::ContractArgs{};
    a.plan = pl->view;
    a.fallback = pl->fallback;
    a.T = b->T[j];
    a.n_items = (int)n_items;
    a.n_blk_t = n_blk_t;
    a.n_sblk = n_sblk;
    part_off[j] = part_total;
    part_total += (size_t)a.T * n_blk_t * 3;
    b->n_pairs += (int64_t)a.T * pl->n_src * pl->n_snk;
    // predicted cost of one item: the eliminations, the solves, the dots
    double item = 0.0;
    for (int f = 0; f < pl->F; ++f) {
      const double nf = pl->off[f + 1] - pl->off[f];
      item += nf * nf * nf;
    }
    if (tree && pl->n_dom > 0)
      item += (double)pl->n_groups / pl->n_dom * pl->n * pl->n +
              (double)pl->n_children / pl->n_dom * pl->n;
    item *= spi;
    const int key_n = narrow ? pl->n : mhc::kern::wide_bucket(pl->n);
    const int kind = narrow ? kLane : kWide;
    Bucket* bk = nullptr;
    for (auto& x : buckets)
      if (x.kind == kind && x.n == key_n) bk = &x;
    if (!bk) {
      buckets.push_back(Bucket{kind, key_n, 0, {}, {}});
      bk = &buckets.back();
    }
    bk->lds = std::max(bk->lds, mhc::kern::lds_slice_bytes(pl->M));
    for (int t = 0; t < a.T; ++t) {
      jt.push_back(make_int2(j, t));
      for (int c = 0; c < n_blk_t; ++c) {
        const long long its = (n_items - c + n_blk_t - 1) / n_blk_t;  // items of chunk c
        bk->tiles.push_back(make_int4(j, t, c, 0));
        bk->cost.push_back(item * (double)its);
      }
    }
  }
  // largest tiles first within each persistent kernel
  std::vector<int4> tiles;
  std::vector<std::pair<size_t, size_t>> ranges;
  for (auto& bk : buckets) {
    std::vector<size_t> order(bk.tiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return bk.cost[x] > bk.cost[y]; });
    ranges.push_back({tiles.size(), order.size()});
    for (size_t i : order) tiles.push_back(bk.tiles[i]);
  }
  // device image: jobs | tiles | (job, t) | partials
  const size_t o_jobs = 0;
  const size_t o_tiles = (o_jobs + nj * sizeof(mhc::kern::ContractArgs) + 255) & ~size_t(255);
  const size_t o_jt = (o_tiles + tiles.size() * sizeof(int4) + 255) & ~size_t(255);
  const size_t o_part = (o_jt + jt.size() * sizeof(int2) + 255) & ~size_t(255);
  const size_t bytes = o_part + part_total * sizeof(double);
  e = hipMalloc(&b->dev, bytes);
  if (e != hipSuccess) return fail(MHC_E_OOM, "mhc_batch_run: device scratch");
  e = hipHostMalloc(reinterpret_cast<void**>(&b->jobs_host), nj * sizeof(mhc::kern::ContractArgs),
                    hipHostMallocDefault);
  if (e != hipSuccess) return fail(MHC_E_OOM, "mhc_batch_run: pinned job table");
  char* base = static_cast<char*>(b->dev);
  b->jobs_dev = reinterpret_cast<mhc::kern::ContractArgs*>(base + o_jobs);
  int4* tiles_dev = reinterpret_cast<int4*>(base + o_tiles);
  int2* jt_dev = reinterpret_cast<int2*>(base + o_jt);
  double* part_dev = reinterpret_cast<double*>(base + o_part);
  for (int j = 0; j < nj; ++j) {
    jobs[j].partial = part_dev + part_off[j];
    b->jobs_host[j] = jobs[j];
  }
  e = hipMemcpy(tiles_dev, tiles.data(), tiles.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(jt_dev, jt.data(), jt.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/upload");
  // capture the persistent kernels and the reduction
  e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/stream");
  e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/capture");
  hipError_t le = hipSuccess;
  for (size_t i = 0; i < buckets.size() && le == hipSuccess; ++i) {
    const Bucket& bk = buckets[i];
    mhc::kern::BatchArgs ba{b->jobs_dev, tiles_dev + ranges[i].first, (int)ranges[i].second};
    int per_cu = b->sched.blocks_per_cu;
    if (per_cu <= 0) {
      // as many workgroups per compute unit as stay resident together (the
      // group kernels' registers and LDS decide; the lane kernels take two
      // where two copies of the slice fit in LDS)
      per_cu = bk.kind == kLane ? (bk.lds > 72 * 1024 ? 1 : 2)
               : bk.kind == kWide
                   ? std::min(8, mhc::kern::batch_wide_resident(bk.n, tree, b->with_a, bk.lds))
                   : std::min(8, mhc::kern::batch_rows_resident(bk.n, tree, b->with_a, bk.lds));
    }
    const int grid = std::max(1, std::min((int)ranges[i].second, n_cu * per_cu));
    le = bk.kind == kLane
             ? mhc::kern::launch_batch_lane(ba, bk.n, tree, b->with_a, grid, bk.lds, b->cap)
         : bk.kind == kWide
             ? mhc::kern::launch_batch_wide(ba, bk.n, tree, b->with_a, grid, bk.lds, b->cap)
             : mhc::kern::launch_batch_rows(ba, bk.n, tree, b->with_a, grid, bk.lds, b->cap);
  }
  if (le == hipSuccess) le = mhc::kern::launch_batch_reduce(b->jobs_dev, jt_dev, (int)jt.size(), b->cap);
  e = hipStreamEndCapture(b->cap, &b->graph);
  if (le != hipSuccess) return hip_fail(le, "mhc_batch_run/launch");
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/capture end");
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/instantiate");
  b->n_tiles = (int)tiles.size();
  b->n_kernels = (int)buckets.size() + 1;
  b->n_jt = (int)jt.size();
  b->last_ptrs.clear();
  b->built = true;
  return MHC_OK;
}

}  // namespace

extern "C" {

mhc_status mhc_batch_create(mhc_plan* const* plans, const int32_t* T, int32_t n_jobs,
                            int32_t method, const mhc_schedule* sched, mhc_batch** out) {
  if (!out) return fail(MHC_E_ARG, "mhc_batch_create: out is NULL");
  *out = nullptr;
  if (!plans || !T || n_jobs < 1) return fail(MHC_E_ARG, "mhc_batch_create: no jobs");
  if (method != MHC_PLAIN_LU && method != MHC_UPDATE_TREE)
    return fail(MHC_E_ARG, "mhc_batch_create: unknown method");
  mhc_schedule sc{};
  if (sched) sc = *sched;
  if (sc.kernel < MHC_SCHED_AUTO || sc.kernel > MHC_SCHED_GROUP || sc.blocks_per_cu < 0 ||
      sc.blocks_per_cu > 8 || sc.items_per_tile < 0)
    return fail(MHC_E_ARG, "mhc_batch_create: invalid schedule");
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_create/hipGetDevice");
  for (int j = 0; j < n_jobs; ++j) {
    if (!plans[j]) return fail(MHC_E_ARG, "mhc_batch_create: NULL plan");
    if (plans[j]->device != cur)
      return fail(MHC_E_DEVICE, "mhc_batch_create: a plan lives on another device");
    if (T[j] < 1 || T[j] > 65535) return fail(MHC_E_ARG, "mhc_batch_create: T outside [1, 65535]");
    if (sc.kernel == MHC_SCHED_LANE && !(plans[j]->uniform_n && plans[j]->n <= 8))
      return fail(MHC_E_UNSUPPORTED,
                  "mhc_batch_create: the one-matrix-per-lane schedule needs every flavour "
                  "block of size n <= 8");
  }
  mhc_batch* b = new (std::nothrow) mhc_batch();
  if (!b) return fail(MHC_E_OOM, "mhc_batch_create: out of host memory");
  b->device = cur;
  b->method = method;
  b->sched = sc;
  b->plans.assign(plans, plans + n_jobs);
  b->T.assign(T, T + n_jobs);
  *out = b;
  return MHC_OK;
}

mhc_status mhc_batch_run(mhc_batch* b, const void* const* S, const double* const* w_src,
                         const double* const* w_snk, void* const* C, double* const* A,
                         void* stream) {
  if (!b) return fail(MHC_E_ARG, "mhc_batch_run: NULL batch");
  if (!S || !w_src || !w_snk || !C) return fail(MHC_E_ARG, "mhc_batch_run: NULL pointer array");
  const int nj = (int)b->plans.size();
  for (int j = 0; j < nj; ++j)
    if (!S[j] || !w_src[j] || !w_snk[j] || !C[j])
      return fail(MHC_E_ARG, "mhc_batch_run: NULL buffer for job " + std::to_string(j));
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/hipGetDevice");
  if (cur != b->device) return fail(MHC_E_DEVICE, "mhc_batch_run: wrong current device");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool with_a = A != nullptr;
  if (b->built && b->with_a != with_a) {
    // the other kernel variants are needed: capture again
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/sync");
    batch_release(b);
  }
  if (!b->built) {
    b->with_a = with_a;
    mhc_status st = batch_build(b);
    if (st != MHC_OK) {
      batch_release(b);
      return st;
    }
  }
  std::vector<const void*> ptrs;
  ptrs.reserve(5 * nj);
  for (int j = 0; j < nj; ++j) {
    ptrs.push_back(S[j]);
    ptrs.push_back(w_src[j]);
    ptrs.push_back(w_snk[j]);
    ptrs.push_back(C[j]);
    ptrs.push_back(A ? A[j] : nullptr);
  }
  if (ptrs != b->last_ptrs) {
    // the job table is read by the graph: let earlier runs finish first,
    // whichever stream they were launched on
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/sync");
    for (int j = 0; j < nj; ++j) {
      b->jobs_host[j].S = static_cast<const double2*>(S[j]);
      b->jobs_host[j].w_src = w_src[j];
      b->jobs_host[j].w_snk = w_snk[j];
      b->jobs_host[j].C = static_cast<double2*>(C[j]);
      b->jobs_host[j].A = A ? A[j] : nullptr;
    }
    e = hipMemcpy(b->jobs_dev, b->jobs_host, nj * sizeof(mhc::kern::ContractArgs),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/job table");
    b->last_ptrs = ptrs;
  }
  e = hipGraphLaunch(b->exec, s);
  if (e != hipSuccess) return hip_fail(e, "mhc_batch_run/graph launch");
  return MHC_OK;
}

mhc_status mhc_batch_info(const mhc_batch* b, int32_t* n_tiles, int32_t* n_kernels,
                          int64_t* n_pairs) {
  if (!b) return fail(MHC_E_ARG, "mhc_batch_info: NULL batch");
  if (n_tiles) *n_tiles = b->n_tiles;
  if (n_kernels) *n_kernels = b->n_kernels;
  if (n_pairs) {
    int64_t np = 0;
    for (size_t j = 0; j < b->plans.size(); ++j)
      np += (int64_t)b->T[j] * b->plans[j]->n_src * b->plans[j]->n_snk;
    *n_pairs = np;
  }
  return MHC_OK;
}

void mhc_batch_destroy(mhc_batch* b) {
  if (!b) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(b->device);
  hipDeviceSynchronize();
  batch_release(b);
  hipSetDevice(cur);
  delete b;
}

}  // extern "C"
