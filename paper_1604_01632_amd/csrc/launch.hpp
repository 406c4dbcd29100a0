// Launch configuration and the per-precision launcher table.
#pragma once
#include "device.hpp"

namespace fslbm {

// Grid classes of the step kernels: how many blocks a domain gets.
enum GridClass {
  G_BULK = 0,  // stream-collide: one chunk of cells per block
  G_LIST,      // interface-list kernels
  G_SMALL,     // conversion-list kernels
  G_TILE,      // interface-list rebuild: one tile of LTILE cells per block
  G_ONE,       // single-block kernels (one per domain)
  G_CELL,      // labelling kernels
  G_EXCOUNT,   // excess mass (G_SMALL blocks) beside the tile counts (G_TILE)
  G_SCANCELL,  // the tile-count scan (one block) beside the labelling init (G_CELL)
  G_TILECELL,  // the list fill (G_TILE) beside the labelling unions (G_CELL)
  G_LISTCELL,  // the gather pass (G_LIST) beside the roots pass (G_CELL)
  G_ONEVOL,    // the assign pass (one block) beside the bubble volumes (one
               // lane per slot and sub-slot)
  G_COUNT
};

struct LaunchCfg {
  int blocks[G_COUNT];
  int bulk_threads;  // threads per stream-collide block (128 or 256)
  int with_mass;     // accumulate the total mass in the stream-collide kernels
};

// Many domains in one launch per kernel: the Dev of every domain (for the
// parity of the step) and, per grid class, the first block of every domain
// (nd + 1 entries; the last is the total).  All pointers are device memory.
struct BatchCfg {
  const Dev *devs;
  int nd;
  const int *off[G_COUNT];
  int total[G_COUNT];
  int bulk_threads;
  int with_mass;
};

// Phases of one step, in order; the host may record events between them.
enum Phase { PH_IFACE = 0, PH_BULK, PH_CONVERT, PH_EXCESS, PH_GATHER, PH_LABEL, PH_BUBBLES, PH_COUNT };

struct Launchers {
  void (*phase)(int ph, const Dev &d, const LaunchCfg &c, hipStream_t s);
  void (*batch_phase)(int ph, const BatchCfg &b, hipStream_t s);
  // stream-collide alone without the mass accumulator (autotuning: it only
  // writes the new lattice and flags, which the next step rewrites)
  void (*batch_bulk_probe)(const BatchCfg &b, hipStream_t s);
  // the geometry kernel alone over the interface lists (autotuning of the
  // list-kernel grid: it only writes per-slot values the next step rewrites)
  void (*batch_list_probe)(const BatchCfg &b, hipStream_t s);
  void (*init_feq)(const Dev &d, const LaunchCfg &c, const double *rho, const double *u,
                   hipStream_t s);
  void (*init_f)(const Dev &d, const LaunchCfg &c, const double *src, int a, hipStream_t s);
  void (*exportq)(const Dev &d, const LaunchCfg &c, double *out, int what, hipStream_t s);
  // invariant checks of the state (the Dev of the next step)
  void (*watchdog)(const Dev &d, const LaunchCfg &c, hipStream_t s);
  int store_bytes;  // bytes per stored PDF value
  int real_bytes;   // bytes per field value (phi, mass, ...)
};

Launchers launchers_fp64();
Launchers launchers_fp32();
Launchers launchers_fp16();

}  // namespace fslbm
