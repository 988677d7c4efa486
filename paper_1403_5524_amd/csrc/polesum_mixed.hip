// Mixed-precision pole sum (placeholder until the FP32/BF16 kernels land).
#include "rm_internal.h"

namespace rmx {

hipError_t launch_polesum_mixed(const Sym &, int, double, const double *,
                                int64_t, double *, int64_t, int,
                                hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace rmx
