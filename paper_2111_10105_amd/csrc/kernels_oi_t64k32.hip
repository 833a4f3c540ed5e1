// Orthogonal-iteration kernels (k_oi, k_oi_batch) for windows of at most 64
// frames and k up to 32: one of the four (T, k) classes, each built as a unit
// of its own so that the classes compile in parallel.
#include "oi_device.h"

namespace dmc {
template void launch_oi_t<64, 32>(hipStream_t, const OiArgs&);
template void launch_oi_batch_t<64, 32>(hipStream_t, int, const OiArgs*, const int4*, int);
}  // namespace dmc
