// The cooperative kernels of the batched build for 16-bit pixels (one per
// metric), in a translation unit of their own.
#include "ih_batch_dev.h"

namespace ih {
coop_fn pick_coop_u16(int metric) { return pick_coop_t<uint16_t>(metric); }
}  // namespace ih
