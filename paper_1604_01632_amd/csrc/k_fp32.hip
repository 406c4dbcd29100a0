// Kernels of the FP32 form.
#include "instantiate.hpp"

namespace fslbm {
Launchers launchers_fp32() { return make_launchers<P32>(); }
}  // namespace fslbm
