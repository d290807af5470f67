// Evaluation, latency-mode and ratio kernels of BF16 tables.
#include "eval_device.hpp"

namespace bspl {
BSPL_DEFINE_KERNEL_TABLE(BF16)
}  // namespace bspl
