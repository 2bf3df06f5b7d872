// Multi-row group kernels for flavour blocks up to 24: one translation unit
// per bucket so the buckets compile in parallel.
#include "rows_impl.h"

namespace mhc {
namespace kern {

MHC_ROWS_BUCKET(24)

}  // namespace kern
}  // namespace mhc
