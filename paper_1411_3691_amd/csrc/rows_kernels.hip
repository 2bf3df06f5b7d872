// Dispatch of the multi-row group kernels (rows_impl.h, instantiated per
// block-size bucket in rows_b<NMAX>.hip).

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contract_kernels.h"

namespace mhc {
namespace kern {

#define MHC_ROWS_DECL(NMAX)                                                                    \
  hipError_t launch_contract_rows_b##NMAX(const ContractArgs& a, bool tree, bool with_a,      \
                                          bool agg, size_t lds_rows, hipStream_t s);          \
  hipError_t launch_batch_rows_b##NMAX(const BatchArgs& b, bool tree, bool with_a, int grid,  \
                                       size_t lds_rows, hipStream_t s);                       \
  int batch_rows_resident_b##NMAX(bool tree, bool with_a, size_t lds_rows);                   \
  RowsGeometry rows_geometry_b##NMAX(bool tree);
MHC_ROWS_DECL(8)
MHC_ROWS_DECL(12)
MHC_ROWS_DECL(16)
MHC_ROWS_DECL(18)
MHC_ROWS_DECL(24)

int rows_bucket(int nmax) {
  return nmax <= 8 ? 8 : nmax <= 12 ? 12 : nmax <= 16 ? 16 : nmax <= 18 ? 18 : nmax <= 24 ? 24 : 0;
}

RowsGeometry rows_geometry(int nmax, bool tree) {
  switch (rows_bucket(nmax)) {
    case 8: return rows_geometry_b8(tree);
    case 12: return rows_geometry_b12(tree);
    case 16: return rows_geometry_b16(tree);
    case 18: return rows_geometry_b18(tree);
    case 24: return rows_geometry_b24(tree);
    default: return RowsGeometry{0, 0, 0};
  }
}

hipError_t launch_contract_rows(const ContractArgs& a, int nmax, bool tree, bool with_a,
                                bool agg, size_t lds_rows, double2* C, double* A, hipStream_t s) {
  hipError_t e;
  switch (rows_bucket(nmax)) {
    case 8: e = launch_contract_rows_b8(a, tree, with_a, agg, lds_rows, s); break;
    case 12: e = launch_contract_rows_b12(a, tree, with_a, agg, lds_rows, s); break;
    case 16: e = launch_contract_rows_b16(a, tree, with_a, agg, lds_rows, s); break;
    case 18: e = launch_contract_rows_b18(a, tree, with_a, agg, lds_rows, s); break;
    case 24: e = launch_contract_rows_b24(a, tree, with_a, agg, lds_rows, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return launch_reduce(a, C, A, s);
}

hipError_t launch_batch_rows(const BatchArgs& b, int nmax, bool tree, bool with_a, int grid,
                             size_t lds_rows, hipStream_t s) {
  switch (rows_bucket(nmax)) {
    case 8: return launch_batch_rows_b8(b, tree, with_a, grid, lds_rows, s);
    case 12: return launch_batch_rows_b12(b, tree, with_a, grid, lds_rows, s);
    case 16: return launch_batch_rows_b16(b, tree, with_a, grid, lds_rows, s);
    case 18: return launch_batch_rows_b18(b, tree, with_a, grid, lds_rows, s);
    case 24: return launch_batch_rows_b24(b, tree, with_a, grid, lds_rows, s);
    default: return hipErrorInvalidValue;
  }
}

int batch_rows_resident(int nmax, bool tree, bool with_a, size_t lds_rows) {
  switch (rows_bucket(nmax)) {
    case 8: return batch_rows_resident_b8(tree, with_a, lds_rows);
    case 12: return batch_rows_resident_b12(tree, with_a, lds_rows);
    case 16: return batch_rows_resident_b16(tree, with_a, lds_rows);
    case 18: return batch_rows_resident_b18(tree, with_a, lds_rows);
    case 24: return batch_rows_resident_b24(tree, with_a, lds_rows);
    default: return 1;
  }
}

}  // namespace kern
}  // namespace mhc
