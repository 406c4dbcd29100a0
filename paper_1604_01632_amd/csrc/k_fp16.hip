// Kernels of the FP16 form.
#include "instantiate.hpp"

namespace fslbm {
Launchers launchers_fp16() { return make_launchers<P16>(); }
}  // namespace fslbm
