// Evaluation, latency-mode and ratio kernels of F32 tables.
#include "eval_device.hpp"

namespace bspl {
BSPL_DEFINE_KERNEL_TABLE(F32)
}  // namespace bspl
