// Internal declarations shared by the host planner, the plan/launch code and
// the kernels of libmhc.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mhc.h"

namespace mhc {

constexpr int kMaxFlavors = 8;
constexpr int kMaxPerFlavor = 32;
constexpr int kMaxM = 255;

// Sets the thread-local error message and returns `code`.
mhc_status fail(mhc_status code, const std::string& msg);

}  // namespace mhc

struct mhc_terms {
  int32_t n_terms = 0;
  int32_t n_flavors = 0;
  int32_t M = 0;
  int32_t sn = 0;                    // sum of n_per_flavor
  std::vector<int32_t> nf;           // [n_flavors]
  std::vector<int32_t> off;          // [n_flavors + 1] flavour offsets
  std::vector<int32_t> idx;          // [n_terms][sn]
};

struct mhc_tree {
  mhc_terms terms;                   // private copy of the source terms
  int32_t policy = MHC_GREEDY_R2;
  std::vector<int32_t> dom_order;    // [n_dom]
  std::vector<int32_t> owner;        // [n]
  std::vector<int32_t> flav;         // [n]
  std::vector<int32_t> pos;          // [n]
  bool set_edges = false;            // MHC_TREE_SET_EDGES
  // per child: the new index of its changed row and the sign of the row
  // permutation that brings its blocks into the dominator's order (always
  // 1 with positional edges); -1 and 0 for dominators
  std::vector<int32_t> cnew;         // [n]
  std::vector<int32_t> sign;         // [n]
  // Group CSR, in dom_order: dominator k owns groups
  // [dom_grp[k], dom_grp[k+1]); group g has flavour grp_f[g], row grp_r[g]
  // and children grp_child[grp_ptr[g] .. grp_ptr[g+1]) (term indices,
  // ascending).  Groups of a dominator are sorted by (f, r).
  std::vector<int32_t> dom_grp;
  std::vector<int32_t> grp_f, grp_r, grp_ptr;
  std::vector<int32_t> grp_child;
};

namespace mhc {
// Builds the neighbour lists (CSR, ascending) of the positional
// Hamming-distance-1 graph.
void hamming1_graph(const mhc_terms& t, std::vector<int64_t>& ptr,
                    std::vector<int32_t>& nbr);
// The same for set edges (blocks that differ as sets in one element).
void set1_graph(const mhc_terms& t, std::vector<int64_t>& ptr, std::vector<int32_t>& nbr);
}  // namespace mhc
