// Dispatch of the group kernels (one group of lanes per matrix, blocks of
// any size up to 24, sizes may differ per flavour) to their block-size
// buckets.  The kernels themselves are in wide_impl.h, instantiated once
// per bucket in wide_b<NMAX>.hip.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contract_kernels.h"
#include "lu_device.h"

namespace mhc {
namespace kern {

hipError_t launch_contract_wide_b8(const ContractArgs& a, bool tree, bool diag, bool agg,
                                   hipStream_t s);
hipError_t launch_contract_wide_b12(const ContractArgs& a, bool tree, bool diag, bool agg,
                                   hipStream_t s);
hipError_t launch_contract_wide_b16(const ContractArgs& a, bool tree, bool diag, bool agg,
                                   hipStream_t s);
hipError_t launch_contract_wide_b18(const ContractArgs& a, bool tree, bool diag, bool agg,
                                   hipStream_t s);
hipError_t launch_contract_wide_b24(const ContractArgs& a, bool tree, bool diag, bool agg,
                                   hipStream_t s);
hipError_t launch_batch_wide_b8(const BatchArgs& b, bool tree, bool with_a, int grid,
                                size_t slice, hipStream_t s);
hipError_t launch_batch_wide_b12(const BatchArgs& b, bool tree, bool with_a, int grid,
                                 size_t slice, hipStream_t s);
hipError_t launch_batch_wide_b16(const BatchArgs& b, bool tree, bool with_a, int grid,
                                 size_t slice, hipStream_t s);
hipError_t launch_batch_wide_b18(const BatchArgs& b, bool tree, bool with_a, int grid,
                                 size_t slice, hipStream_t s);
hipError_t launch_batch_wide_b24(const BatchArgs& b, bool tree, bool with_a, int grid,
                                 size_t slice, hipStream_t s);
int wide_block_b8(bool tree, size_t slice);
int wide_block_b12(bool tree, size_t slice);
int wide_block_b16(bool tree, size_t slice);
int wide_block_b18(bool tree, size_t slice);
int wide_block_b24(bool tree, size_t slice);

int batch_wide_resident_b8(bool tree, bool with_a, size_t slice);
int batch_wide_resident_b12(bool tree, bool with_a, size_t slice);
int batch_wide_resident_b16(bool tree, bool with_a, size_t slice);
int batch_wide_resident_b18(bool tree, bool with_a, size_t slice);
int batch_wide_resident_b24(bool tree, bool with_a, size_t slice);

int wide_bucket(int nmax) {
  return nmax <= 8 ? 8 : nmax <= 12 ? 12 : nmax <= 16 ? 16 : nmax <= 18 ? 18 : 24;
}

// Groups of 8 lanes for blocks up to 8, 16 up to 16, 32 above.
int wide_sinks_per_wave(int nmax) {
  return nmax <= 8 ? kWave / 8 : nmax <= 16 ? kWave / 16 : kWave / 32;
}

int wide_block(int nmax, bool tree, size_t lds) {
  switch (wide_bucket(nmax)) {
    case 8: return wide_block_b8(tree, lds);
    case 12: return wide_block_b12(tree, lds);
    case 16: return wide_block_b16(tree, lds);
    case 18: return wide_block_b18(tree, lds);
    default: return wide_block_b24(tree, lds);
  }
}

int batch_wide_resident(int nmax, bool tree, bool with_a, size_t lds) {
  switch (wide_bucket(nmax)) {
    case 8: return batch_wide_resident_b8(tree, with_a, lds);
    case 12: return batch_wide_resident_b12(tree, with_a, lds);
    case 16: return batch_wide_resident_b16(tree, with_a, lds);
    case 18: return batch_wide_resident_b18(tree, with_a, lds);
    default: return batch_wide_resident_b24(tree, with_a, lds);
  }
}

hipError_t launch_batch_wide(const BatchArgs& b, int nmax, bool tree, bool with_a, int grid,
                             size_t lds, hipStream_t s) {
  switch (wide_bucket(nmax)) {
    case 8: return launch_batch_wide_b8(b, tree, with_a, grid, lds, s);
    case 12: return launch_batch_wide_b12(b, tree, with_a, grid, lds, s);
    case 16: return launch_batch_wide_b16(b, tree, with_a, grid, lds, s);
    case 18: return launch_batch_wide_b18(b, tree, with_a, grid, lds, s);
    default: return launch_batch_wide_b24(b, tree, with_a, grid, lds, s);
  }
}

hipError_t launch_contract_wide(const ContractArgs& a, int nmax, bool tree, bool diag,
                                double2* C, double* A, hipStream_t s, bool agg) {
  if (nmax > 24) return hipErrorInvalidValue;
  hipError_t e;
  switch (wide_bucket(nmax)) {
    case 8: e = launch_contract_wide_b8(a, tree, diag, agg, s); break;
    case 12: e = launch_contract_wide_b12(a, tree, diag, agg, s); break;
    case 16: e = launch_contract_wide_b16(a, tree, diag, agg, s); break;
    case 18: e = launch_contract_wide_b18(a, tree, diag, agg, s); break;
    default: e = launch_contract_wide_b24(a, tree, diag, agg, s); break;
  }
  if (e != hipSuccess) return e;
  return launch_reduce(a, C, A, s);
}

}  // namespace kern
}  // namespace mhc
