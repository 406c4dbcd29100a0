// Kernels of the FP64 form.
#include "instantiate.hpp"

namespace fslbm {
Launchers launchers_fp64() { return make_launchers<P64>(); }
}  // namespace fslbm
