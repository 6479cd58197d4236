// Instantiations of the matching kernels (one group per translation unit,
// so the groups compile in parallel).
#include "glop_kernels_impl.hpp"

namespace glop {
namespace detail {

GLOP_DEFINE_VARIANT(1, 0, 1, 0, 8)
GLOP_DEFINE_VARIANT(1, 1, 1, 0, 8)
GLOP_DEFINE_VARIANT(1, 1, 1, 1, 8)

}  // namespace detail
}  // namespace glop
