// Fast-path step kernels (filled in below as they are written).
#include "internal.h"

namespace maclab {

bool fast_step_supported(const Layout&, const StepParams&) { return false; }

hipError_t launch_step_fast(const Layout&, const void*, void*, const StepParams&, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace maclab
