// Group kernels for flavour blocks up to 16 (groups of 16 lanes): one
// translation unit per bucket so the buckets compile in parallel.
#include "wide_impl.h"

namespace mhc {
namespace kern {

MHC_WIDE_BUCKET(16, 16)

}  // namespace kern
}  // namespace mhc
