// Group kernels for flavour blocks up to 24 (groups of 32 lanes): one
// translation unit per bucket so the buckets compile in parallel.
#include "wide_impl.h"

namespace mhc {
namespace kern {

MHC_WIDE_BUCKET(32, 24)

}  // namespace kern
}  // namespace mhc
