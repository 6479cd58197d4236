// Kernel variants: blocked two-bit filter (probe_bits 3), both strides, and the paired
// 16-bit-block filter (probe_bits 4, stride 1, 4-byte q-grams); 8 KiB tiles.
#include "glop_kernels_impl.hpp"

namespace glop {
namespace detail {
GLOP_DEFINE_VARIANT(1, 1, 4, 1, 8)
GLOP_DEFINE_VARIANT(1, 1, 3, 0, 8)
GLOP_DEFINE_VARIANT(1, 1, 3, 1, 8)
GLOP_DEFINE_VARIANT(4, 1, 3, 0, 8)
GLOP_DEFINE_VARIANT(4, 1, 3, 1, 8)
}  // namespace detail
}  // namespace glop
