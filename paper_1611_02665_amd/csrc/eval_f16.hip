// Evaluation, latency-mode and ratio kernels of F16 tables.
#include "eval_device.hpp"

namespace bspl {
BSPL_DEFINE_KERNEL_TABLE(F16)
}  // namespace bspl
