// Instantiations of the matching kernels (one group per translation unit,
// so the groups compile in parallel).
#include "glop_kernels_impl.hpp"

namespace glop {
namespace detail {

GLOP_DEFINE_VARIANT(4, 1, 1, 0, 16)
GLOP_DEFINE_VARIANT(4, 1, 1, 1, 16)

}  // namespace detail
}  // namespace glop
