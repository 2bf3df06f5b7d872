// Group kernels for flavour blocks up to 8 (groups of 8 lanes): one
// translation unit per bucket so the buckets compile in parallel.
#include "wide_impl.h"

namespace mhc {
namespace kern {

MHC_WIDE_BUCKET(8, 8)

}  // namespace kern
}  // namespace mhc
