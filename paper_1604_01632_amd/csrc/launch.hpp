// Launch configuration and the per-precision launcher table.
#pragma once
#include "device.hpp"

namespace fslbm {

struct LaunchCfg {
  int bx;         // threads per block of the bulk kernel (x extent)
  int list_grid;  // blocks of the interface-list kernels
  int small_grid; // blocks of the conversion-list kernels
  int cell_grid;  // blocks of the cell-strided (labelling, init) kernels
  int with_mass; // accumulate the total mass in the stream-collide kernels
};

// Phases of one step, in order; the host may record events between them.
enum Phase { PH_IFACE = 0, PH_BULK, PH_CONVERT, PH_EXCESS, PH_GATHER, PH_LABEL, PH_BUBBLES, PH_COUNT };

struct Launchers {
  void (*phase)(int ph, const Dev &d, const LaunchCfg &c, hipStream_t s);
  void (*init_feq)(const Dev &d, const LaunchCfg &c, const double *rho, const double *u,
                   hipStream_t s);
  void (*init_f)(const Dev &d, const LaunchCfg &c, const double *src, int a, hipStream_t s);
  void (*exportq)(const Dev &d, const LaunchCfg &c, double *out, int what, hipStream_t s);
  int store_bytes;  // bytes per stored PDF value
  int real_bytes;   // bytes per field value (phi, mass, ...)
};

Launchers launchers_fp64();
Launchers launchers_fp32();
Launchers launchers_fp16();

}  // namespace fslbm
