// Host side of libmhc: error reporting, wavefunction terms and the update
// tree (source-term graph + greedy dominating set + group tables).
//
// Integer work only; nothing here touches the GPU, so these entry points
// work on machines without one.

#include <algorithm>
#include <cstring>
#include <new>
#include <queue>
#include <string>
#include <utility>
#include <vector>

#include "mhc_internal.h"

namespace mhc {

static thread_local std::string g_last_error;

mhc_status fail(mhc_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// ------------------------------------------------------------------ graph
//
// Sec. 3: vertices are source terms, with an edge where two terms differ in
// a single position (one row of one flavour block of G, Sec. 2).  Terms at
// distance exactly 1 agree everywhere except at one position p, so they
// share the key "tuple with position p masked".  For every p the terms are
// sorted by that key; inside a run of equal keys every two terms with
// different values at p are neighbours (equal values would make the terms
// identical: distance 0, no edge).  Each edge is found once, at its
// differing position.
void hamming1_graph(const mhc_terms& t, std::vector<int64_t>& ptr,
                    std::vector<int32_t>& nbr) {
  const int n = t.n_terms, sn = t.sn;
  const int32_t* I = t.idx.data();
  std::vector<std::vector<int32_t>> adj(n);
  std::vector<int32_t> order(n);
  for (int p = 0; p < sn; ++p) {
    for (int u = 0; u < n; ++u) order[u] = u;
    auto less = [&](int32_t a, int32_t b) {
      const int32_t* x = I + (int64_t)a * sn;
      const int32_t* y = I + (int64_t)b * sn;
      for (int q = 0; q < sn; ++q) {
        if (q == p) continue;
        if (x[q] != y[q]) return x[q] < y[q];
      }
      return a < b;
    };
    std::sort(order.begin(), order.end(), less);
    auto same_key = [&](int32_t a, int32_t b) {
      const int32_t* x = I + (int64_t)a * sn;
      const int32_t* y = I + (int64_t)b * sn;
      for (int q = 0; q < sn; ++q)
        if (q != p && x[q] != y[q]) return false;
      return true;
    };
    for (int lo = 0; lo < n;) {
      int hi = lo + 1;
      while (hi < n && same_key(order[lo], order[hi])) ++hi;
      for (int a = lo; a < hi; ++a)
        for (int b = a + 1; b < hi; ++b) {
          int32_t u = order[a], v = order[b];
          if (I[(int64_t)u * sn + p] != I[(int64_t)v * sn + p]) {
            adj[u].push_back(v);
            adj[v].push_back(u);
          }
        }
      lo = hi;
    }
  }
  ptr.assign(n + 1, 0);
  for (int u = 0; u < n; ++u) {
    std::sort(adj[u].begin(), adj[u].end());
    ptr[u + 1] = ptr[u] + (int64_t)adj[u].size();
  }
  nbr.resize(ptr[n]);
  for (int u = 0; u < n; ++u)
    std::copy(adj[u].begin(), adj[u].end(), nbr.begin() + ptr[u]);
}

// Set edges (an ablation of the edge rule): two terms are neighbours when
// their flavour blocks, as sets of indices, differ in exactly one element of
// one block.  With every block sorted, such terms share the key "block f
// without one of its elements, every other block whole" for exactly one
// choice of removed element on each side, and the removed elements differ
// (equal ones would make the sets equal: distance 0, no edge).  For every
// block f all n_f keys of every term are sorted together; inside a run of
// equal keys, entries of two terms with different removed elements are
// neighbours.  Each edge is found once.
void set1_graph(const mhc_terms& t, std::vector<int64_t>& ptr, std::vector<int32_t>& nbr) {
  const int n = t.n_terms, sn = t.sn, F = t.n_flavors;
  std::vector<int32_t> canon(t.idx);
  for (int u = 0; u < n; ++u)
    for (int f = 0; f < F; ++f)
      std::sort(canon.begin() + (int64_t)u * sn + t.off[f],
                canon.begin() + (int64_t)u * sn + t.off[f + 1]);
  const int32_t* C = canon.data();
  std::vector<std::vector<int32_t>> adj(n);
  for (int f = 0; f < F; ++f) {
    const int nf = t.nf[f];
    // entry = (term, position e of the removed element within block f)
    std::vector<std::pair<int32_t, int32_t>> ent;
    ent.reserve((size_t)n * nf);
    for (int u = 0; u < n; ++u)
      for (int e = 0; e < nf; ++e) ent.emplace_back(u, e);
    // key of an entry: the sorted tuple with block f's e-th element skipped
    auto key_at = [&](const std::pair<int32_t, int32_t>& x, int q) {
      // q-th entry of the key (sn - 1 entries)
      const int skip = t.off[f] + x.second;
      return C[(int64_t)x.first * sn + (q < skip ? q : q + 1)];
    };
    auto less = [&](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
      for (int q = 0; q < sn - 1; ++q) {
        const int32_t x = key_at(a, q), y = key_at(b, q);
        if (x != y) return x < y;
      }
      return a < b;
    };
    std::sort(ent.begin(), ent.end(), less);
    auto same = [&](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
      for (int q = 0; q < sn - 1; ++q)
        if (key_at(a, q) != key_at(b, q)) return false;
      return true;
    };
    const size_t m = ent.size();
    for (size_t lo = 0; lo < m;) {
      size_t hi = lo + 1;
      while (hi < m && same(ent[lo], ent[hi])) ++hi;
      for (size_t a = lo; a < hi; ++a)
        for (size_t b = a + 1; b < hi; ++b) {
          const int32_t u = ent[a].first, v = ent[b].first;
          const int32_t xu = C[(int64_t)u * sn + t.off[f] + ent[a].second];
          const int32_t xv = C[(int64_t)v * sn + t.off[f] + ent[b].second];
          if (u != v && xu != xv) {
            adj[u].push_back(v);
            adj[v].push_back(u);
          }
        }
      lo = hi;
    }
  }
  ptr.assign(n + 1, 0);
  for (int u = 0; u < n; ++u) {
    std::sort(adj[u].begin(), adj[u].end());
    ptr[u + 1] = ptr[u] + (int64_t)adj[u].size();
  }
  nbr.resize(ptr[n]);
  for (int u = 0; u < n; ++u)
    std::copy(adj[u].begin(), adj[u].end(), nbr.begin() + ptr[u]);
}

// Sign of the permutation p with dst[m] = src[p(m)] (distinct values), by
// counting inversions.
static int permutation_sign(const int32_t* src, const int32_t* dst, int k) {
  int inv = 0;
  int pos[kMaxPerFlavor];
  for (int m = 0; m < k; ++m) {
    pos[m] = 0;
    for (int j = 0; j < k; ++j)
      if (src[j] == dst[m]) pos[m] = j;
  }
  for (int x = 0; x < k; ++x)
    for (int y = x + 1; y < k; ++y)
      if (pos[x] > pos[y]) ++inv;
  return (inv & 1) ? -1 : 1;
}

}  // namespace mhc

using mhc::fail;

extern "C" {

const char* mhc_last_error(void) { return mhc::g_last_error.c_str(); }

int32_t mhc_version(void) { return 203; }

mhc_status mhc_terms_create(int32_t n_terms, int32_t n_flavors,
                            const int32_t* n_per_flavor, const int32_t* idx,
                            int32_t M, mhc_terms** out) {
  if (!out) return fail(MHC_E_ARG, "mhc_terms_create: out is NULL");
  *out = nullptr;
  if (!n_per_flavor || !idx)
    return fail(MHC_E_ARG, "mhc_terms_create: NULL array");
  if (n_terms < 1) return fail(MHC_E_ARG, "mhc_terms_create: n_terms < 1");
  if (n_flavors < 1 || n_flavors > mhc::kMaxFlavors)
    return fail(MHC_E_ARG, "mhc_terms_create: n_flavors outside [1, 8]");
  if (M < 1 || M > mhc::kMaxM)
    return fail(MHC_E_ARG, "mhc_terms_create: M outside [1, 255]");
  mhc_terms* t = new (std::nothrow) mhc_terms();
  if (!t) return fail(MHC_E_OOM, "mhc_terms_create: out of host memory");
  t->n_terms = n_terms;
  t->n_flavors = n_flavors;
  t->M = M;
  t->off.push_back(0);
  for (int f = 0; f < n_flavors; ++f) {
    int32_t n = n_per_flavor[f];
    if (n < 1 || n > mhc::kMaxPerFlavor || n > M) {
      delete t;
      return fail(MHC_E_ARG,
                  "mhc_terms_create: n_per_flavor[" + std::to_string(f) +
                      "] outside [1, min(32, M)]");
    }
    t->nf.push_back(n);
    t->off.push_back(t->off.back() + n);
  }
  t->sn = t->off.back();
  const int64_t total = (int64_t)n_terms * t->sn;
  try {
    t->idx.assign(idx, idx + total);
  } catch (...) {
    delete t;
    return fail(MHC_E_OOM, "mhc_terms_create: out of host memory");
  }
  for (int64_t i = 0; i < n_terms; ++i) {
    const int32_t* term = t->idx.data() + i * t->sn;
    for (int f = 0; f < n_flavors; ++f) {
      for (int a = t->off[f]; a < t->off[f + 1]; ++a) {
        if (term[a] < 0 || term[a] >= M) {
          delete t;
          return fail(MHC_E_TERM, "mhc_terms_create: term " +
                                      std::to_string(i) +
                                      " has an index outside [0, M)");
        }
        for (int b = t->off[f]; b < a; ++b)
          if (term[a] == term[b]) {
            delete t;
            return fail(MHC_E_TERM,
                        "mhc_terms_create: term " + std::to_string(i) +
                            " repeats index " + std::to_string(term[a]) +
                            " within flavour " + std::to_string(f));
          }
      }
    }
  }
  *out = t;
  return MHC_OK;
}

void mhc_terms_destroy(mhc_terms* terms) { delete terms; }

mhc_status mhc_terms_shape(const mhc_terms* t, int32_t* n_terms,
                           int32_t* n_flavors, int32_t* M) {
  if (!t) return fail(MHC_E_ARG, "mhc_terms_shape: NULL handle");
  if (n_terms) *n_terms = t->n_terms;
  if (n_flavors) *n_flavors = t->n_flavors;
  if (M) *M = t->M;
  return MHC_OK;
}

// Greedy R2: set-cover greedy over closed neighbourhoods.  gain[v] = number
// of still-uncovered terms in N[v]; gains only decrease, so a lazy max-heap
// ordered by (gain desc, index asc) yields, at every step, exactly the
// lowest-index term of maximal current gain: an entry popped with a stale
// gain is pushed back with its current gain.
static void greedy_r2(const std::vector<int64_t>& ptr,
                      const std::vector<int32_t>& nbr, int n,
                      std::vector<int32_t>& dom, std::vector<int32_t>& owner) {
  std::vector<int32_t> gain(n);
  std::vector<char> covered(n, 0);
  using E = std::pair<int32_t, int32_t>;  // (gain, -index)
  std::priority_queue<E> heap;
  for (int v = 0; v < n; ++v) {
    gain[v] = 1 + (int32_t)(ptr[v + 1] - ptr[v]);
    heap.push(E(gain[v], -v));
  }
  int n_cov = 0;
  auto cover = [&](int u, int by) {
    covered[u] = 1;
    owner[u] = by;
    ++n_cov;
    --gain[u];
    for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) --gain[nbr[e]];
  };
  while (n_cov < n) {
    E top = heap.top();
    heap.pop();
    int v = -top.second;
    if (top.first != gain[v]) {
      if (gain[v] > 0) heap.push(E(gain[v], -v));
      continue;
    }
    dom.push_back(v);
    if (!covered[v]) cover(v, v);
    for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e)
      if (!covered[nbr[e]]) cover(nbr[e], v);
    owner[v] = v;
  }
}

// Greedy R1: the literal rule on the graph of remaining terms.  deg[v] =
// number of remaining neighbours of v; same lazy heap, entries of removed
// terms are dropped when popped.
static void greedy_r1(const std::vector<int64_t>& ptr,
                      const std::vector<int32_t>& nbr, int n,
                      std::vector<int32_t>& dom, std::vector<int32_t>& owner) {
  std::vector<int32_t> deg(n);
  std::vector<char> removed(n, 0);
  using E = std::pair<int32_t, int32_t>;
  std::priority_queue<E> heap;
  for (int v = 0; v < n; ++v) {
    deg[v] = (int32_t)(ptr[v + 1] - ptr[v]);
    heap.push(E(deg[v], -v));
  }
  auto remove = [&](int u, int by) {
    removed[u] = 1;
    owner[u] = by;
    for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) --deg[nbr[e]];
  };
  while (!heap.empty()) {
    E top = heap.top();
    heap.pop();
    int v = -top.second;
    if (removed[v]) continue;
    if (top.first != deg[v]) {
      heap.push(E(deg[v], -v));
      continue;
    }
    dom.push_back(v);
    remove(v, v);
    for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e)
      if (!removed[nbr[e]]) remove(nbr[e], v);
  }
}

// Reverse delete over a dominating set: dominators are visited last picked
// first, and one is dropped when every term of its closed neighbourhood is
// dominated by at least one other kept dominator (cnt >= 2 counts itself).
// Terms whose owner was dropped move to the kept dominator of their closed
// neighbourhood with the lowest pick rank.
static void prune_dominators(const std::vector<int64_t>& ptr,
                             const std::vector<int32_t>& nbr, int n,
                             std::vector<int32_t>& dom,
                             std::vector<int32_t>& owner) {
  std::vector<int32_t> cnt(n, 0);
  for (int32_t v : dom) {
    ++cnt[v];
    for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) ++cnt[nbr[e]];
  }
  std::vector<char> kept(n, 0);
  for (int32_t v : dom) kept[v] = 1;
  for (auto it = dom.rbegin(); it != dom.rend(); ++it) {
    const int v = *it;
    bool redundant = cnt[v] >= 2;
    for (int64_t e = ptr[v]; redundant && e < ptr[v + 1]; ++e)
      redundant = cnt[nbr[e]] >= 2;
    if (!redundant) continue;
    kept[v] = 0;
    --cnt[v];
    for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) --cnt[nbr[e]];
  }
  std::vector<int32_t> order;
  std::vector<int32_t> rank(n, -1);
  for (int32_t v : dom)
    if (kept[v]) {
      rank[v] = (int32_t)order.size();
      order.push_back(v);
    }
  for (int u = 0; u < n; ++u) {
    if (kept[owner[u]]) continue;
    int best = kept[u] ? u : -1;
    for (int64_t e = ptr[u]; e < ptr[u + 1]; ++e) {
      const int v = nbr[e];
      if (kept[v] && (best < 0 || rank[v] < rank[best])) best = v;
    }
    owner[u] = best;
  }
  dom.swap(order);
}

mhc_status mhc_tree_build(const mhc_terms* src, int32_t policy,
                          mhc_tree** out) {
  if (!out) return fail(MHC_E_ARG, "mhc_tree_build: out is NULL");
  *out = nullptr;
  if (!src) return fail(MHC_E_ARG, "mhc_tree_build: NULL terms");
  const bool share = (policy & MHC_TREE_NO_SHARING) == 0;
  const bool prune = (policy & MHC_TREE_PRUNE) != 0;
  const bool set_edges = (policy & MHC_TREE_SET_EDGES) != 0;
  policy &= ~(MHC_TREE_NO_SHARING | MHC_TREE_PRUNE | MHC_TREE_SET_EDGES);
  if (policy != MHC_GREEDY_R1 && policy != MHC_GREEDY_R2)
    return fail(MHC_E_ARG, "mhc_tree_build: policy must be R1 or R2");
  mhc_tree* tr = new (std::nothrow) mhc_tree();
  if (!tr) return fail(MHC_E_OOM, "mhc_tree_build: out of host memory");
  try {
    tr->terms = *src;
    tr->policy = policy;
    tr->set_edges = set_edges;
    const int n = src->n_terms, sn = src->sn;
    std::vector<int64_t> ptr;
    std::vector<int32_t> nbr;
    if (set_edges)
      mhc::set1_graph(*src, ptr, nbr);
    else
      mhc::hamming1_graph(*src, ptr, nbr);
    tr->owner.assign(n, -1);
    if (policy == MHC_GREEDY_R2)
      greedy_r2(ptr, nbr, n, tr->dom_order, tr->owner);
    else
      greedy_r1(ptr, nbr, n, tr->dom_order, tr->owner);
    if (prune) prune_dominators(ptr, nbr, n, tr->dom_order, tr->owner);
    // Flavour and row of each child's single difference with its owner.
    tr->flav.assign(n, -1);
    tr->pos.assign(n, -1);
    const int32_t* I = src->idx.data();
    std::vector<int32_t> flav_of(sn), row_of(sn);
    for (int f = 0; f < src->n_flavors; ++f)
      for (int a = src->off[f]; a < src->off[f + 1]; ++a) {
        flav_of[a] = f;
        row_of[a] = a - src->off[f];
      }
    tr->cnew.assign(n, -1);
    tr->sign.assign(n, 0);
    for (int u = 0; u < n; ++u) {
      int d = tr->owner[u];
      if (d == u) continue;
      const int32_t* tu = I + (int64_t)u * sn;
      const int32_t* td = I + (int64_t)d * sn;
      if (!set_edges) {
        int p = -1;
        for (int q = 0; q < sn; ++q)
          if (tu[q] != td[q]) p = q;
        tr->flav[u] = flav_of[p];
        tr->pos[u] = row_of[p];
        tr->cnew[u] = tu[p];
        tr->sign[u] = 1;
        continue;
      }
      // the block whose set differs: the dominator's element missing from
      // the child gives the row r, the child's element missing from the
      // dominator the new index; b = the dominator with that row replaced,
      // and every block of the child holds b's indices in some order
      int32_t b[mhc::kMaxFlavors * mhc::kMaxPerFlavor];
      std::copy(td, td + sn, b);
      for (int f = 0; f < src->n_flavors; ++f) {
        const int o = src->off[f], k = src->nf[f];
        for (int a = 0; a < k; ++a) {
          if (std::find(tu + o, tu + o + k, td[o + a]) != tu + o + k) continue;
          tr->flav[u] = f;
          tr->pos[u] = a;
          for (int c = 0; c < k; ++c)
            if (std::find(td + o, td + o + k, tu[o + c]) == td + o + k) tr->cnew[u] = tu[o + c];
          b[o + a] = tr->cnew[u];
        }
      }
      int sg = 1;
      for (int f = 0; f < src->n_flavors; ++f)
        sg *= mhc::permutation_sign(b + src->off[f], tu + src->off[f], src->nf[f]);
      tr->sign[u] = sg;
    }
    // Group CSR.  Children are visited in ascending term order, then
    // grouped per dominator by (f, r) with a stable sort.
    const int n_dom = (int)tr->dom_order.size();
    std::vector<int32_t> rank(n, -1);
    for (int k = 0; k < n_dom; ++k) rank[tr->dom_order[k]] = k;
    std::vector<int32_t> cnt(n_dom + 1, 0);
    for (int u = 0; u < n; ++u)
      if (tr->owner[u] != u) ++cnt[rank[tr->owner[u]] + 1];
    for (int k = 0; k < n_dom; ++k) cnt[k + 1] += cnt[k];
    std::vector<int32_t> kids(cnt[n_dom]);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int u = 0; u < n; ++u)
      if (tr->owner[u] != u) kids[fill[rank[tr->owner[u]]]++] = u;
    tr->dom_grp.push_back(0);
    tr->grp_ptr.push_back(0);
    for (int k = 0; k < n_dom; ++k) {
      auto b = kids.begin() + cnt[k], e = kids.begin() + cnt[k + 1];
      std::stable_sort(b, e, [&](int32_t x, int32_t y) {
        if (tr->flav[x] != tr->flav[y]) return tr->flav[x] < tr->flav[y];
        return tr->pos[x] < tr->pos[y];
      });
      for (auto it = b; it != e;) {
        auto jt = it + 1;
        while (share && jt != e && tr->flav[*jt] == tr->flav[*it] &&
               tr->pos[*jt] == tr->pos[*it])
          ++jt;
        tr->grp_f.push_back(tr->flav[*it]);
        tr->grp_r.push_back(tr->pos[*it]);
        tr->grp_child.insert(tr->grp_child.end(), it, jt);
        tr->grp_ptr.push_back((int32_t)tr->grp_child.size());
        it = jt;
      }
      tr->dom_grp.push_back((int32_t)tr->grp_f.size());
    }
  } catch (const std::bad_alloc&) {
    delete tr;
    return fail(MHC_E_OOM, "mhc_tree_build: out of host memory");
  }
  *out = tr;
  return MHC_OK;
}

mhc_status mhc_tree_export(const mhc_tree* tr, int32_t* n_dom,
                           int32_t* dom_order, int32_t* owner, int32_t* flav,
                           int32_t* pos) {
  if (!tr) return fail(MHC_E_ARG, "mhc_tree_export: NULL tree");
  const int n = tr->terms.n_terms;
  if (n_dom) *n_dom = (int32_t)tr->dom_order.size();
  if (dom_order) {
    for (int k = 0; k < n; ++k)
      dom_order[k] = k < (int)tr->dom_order.size() ? tr->dom_order[k] : -1;
  }
  if (owner) std::memcpy(owner, tr->owner.data(), n * sizeof(int32_t));
  if (flav) std::memcpy(flav, tr->flav.data(), n * sizeof(int32_t));
  if (pos) std::memcpy(pos, tr->pos.data(), n * sizeof(int32_t));
  return MHC_OK;
}

mhc_status mhc_tree_groups(const mhc_tree* tr, int32_t* dom_grp, int32_t* grp_f,
                           int32_t* grp_r, int32_t* grp_ptr, int32_t* grp_child) {
  if (!tr) return fail(MHC_E_ARG, "mhc_tree_groups: NULL tree");
  auto put = [](int32_t* dst, const std::vector<int32_t>& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int32_t));
  };
  put(dom_grp, tr->dom_grp);
  put(grp_f, tr->grp_f);
  put(grp_r, tr->grp_r);
  put(grp_ptr, tr->grp_ptr);
  put(grp_child, tr->grp_child);
  return MHC_OK;
}

mhc_status mhc_tree_children(const mhc_tree* tr, int32_t* new_index, int32_t* sign) {
  if (!tr) return fail(MHC_E_ARG, "mhc_tree_children: NULL tree");
  const int n = tr->terms.n_terms;
  if (new_index) std::memcpy(new_index, tr->cnew.data(), n * sizeof(int32_t));
  if (sign) std::memcpy(sign, tr->sign.data(), n * sizeof(int32_t));
  return MHC_OK;
}

mhc_status mhc_tree_stats(const mhc_tree* tr, int32_t* n_dom,
                          int32_t* n_groups, int32_t* n_children) {
  if (!tr) return fail(MHC_E_ARG, "mhc_tree_stats: NULL tree");
  if (n_dom) *n_dom = (int32_t)tr->dom_order.size();
  if (n_groups) *n_groups = (int32_t)tr->grp_f.size();
  if (n_children) *n_children = (int32_t)tr->grp_child.size();
  return MHC_OK;
}

void mhc_tree_destroy(mhc_tree* tree) { delete tree; }

}  // extern "C"
