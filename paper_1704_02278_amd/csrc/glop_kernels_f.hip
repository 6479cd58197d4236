// Kernel variants with 4 KiB tiles (4 rounds, 64 bytes per lane per tile) for
// the two default filters: stride 4 with two hash bits, stride 1 blocked.
#include "glop_kernels_impl.hpp"

namespace glop {
namespace detail {

GLOP_DEFINE_VARIANT(4, 1, 2, 1, 4)
GLOP_DEFINE_VARIANT(1, 1, 3, 1, 4)

}  // namespace detail
}  // namespace glop
