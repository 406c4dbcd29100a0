// Device-side data layout shared by the host API and the kernels of the
// MI355X FSLBM library.  Nothing here is visible across the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exactsum.hpp"

namespace fslbm {

constexpr int Q = 19;

// Cell type in the low three bits of the flag byte (values of the C ABI).
constexpr uint8_t T_GAS = 0, T_IFACE = 1, T_LIQ = 2, T_WALL = 3, T_INLET = 4;
constexpr uint8_t TYPE_MASK = 0x07;
// Static bits, fixed at creation: the cell has a wall / an inlet cell among
// its 18 neighbours.
constexpr uint8_t NEAR_WALL = 0x08;
constexpr uint8_t NEAR_INLET = 0x10;
constexpr uint8_t STATIC_BITS = NEAR_WALL | NEAR_INLET;
// Conversion candidates written by the interface kernel for its new state:
// fill level above 1 + eps (and no inlet neighbour), below -eps.
constexpr uint8_t CAND_F = 0x20;
constexpr uint8_t CAND_E = 0x40;
// Set on interface cells of t+1 that receive excess mass from a converted
// neighbour.
constexpr uint8_t GATHER = 0x80;

// Accumulator replication: atomics of one logical sum are spread over SUB
// slots (picked by block index) to avoid serialising on one address; the
// slots are integers, so the final sum is independent of order.
constexpr int SUB = 16;
// Blocks of `threads` lanes for the per-bubble volume reduction: one lane
// per bubble slot and sub-slot, at most 1024 blocks (grid-stride beyond).
__host__ __device__ constexpr int volume_blocks(int max_bubbles, int threads) {
  const long long n = ((long long)max_bubbles * SUB + threads - 1) / threads;
  return (int)(n < 1024 ? n : 1024);
}
// Blocks of the labelling kernels: one per 4096 cells, at most 1024 (they
// walk the labelled set with grid strides).
__host__ __device__ constexpr int cell_blocks(long long n_cells) {
  const long long b = (n_cells + 4095) / 4096;
  return (int)(b < 1 ? 1 : (b < 1024 ? b : 1024));
}
constexpr int SUB_MASS = 256;

// Fixed-point scale of the two-word integer accumulator of the total mass
// diagnostic (value * 2^FX_VOL rounded to an int64, split into a high and a
// low word); |term| < 2^13.
constexpr int FX_VOL = 50;
constexpr int FX_SPLIT = 25;

// Per-bubble accumulator of the interface cells' gas volumes 1 - phi and
// their count.  A term computed in double from phi in (-1, 3) is an integer
// multiple of 2^-53 below 2 in magnitude (1 - phi lies in [1, 2) for
// phi <= 0 and in (0.5, 1] for 0 < phi < 0.5, where the spacing is 2^-52 or
// 2^-53; for 0.5 <= phi < 3 the difference is exact, a multiple of the
// spacing of phi), so q = (1 - phi) 2^53 is an integer with |q| < 2^54.  It
// is added as three chunks of 18 bits (q = c0 + c1 2^18 + c2 2^36, c2
// signed), whose sums over a wave fit in 32 bits.  Any other term goes into
// the exact-sum words.  Layout: VA_EX exact-sum words, VA_FIX chunk sums,
// the count.
constexpr int VA_EX = 0;
constexpr int VA_FIX = EX_WORDS;
constexpr int VA_FIXN = 3;
constexpr int VA_FIX_BITS = 18;
constexpr int VA_FIX_SCALE = 53;
constexpr int VA_CNT = EX_WORDS + VA_FIXN;
constexpr int VACC = EX_WORDS + VA_FIXN + 1;
// Per-new-component accumulators of a labelling event: exact-sum words of
// the volume and of V*, then ncells, ngas, niface, inlet cells, cells of
// atmosphere bubbles.
constexpr int NACC = 2 * EX_WORDS + 5;

// Bubble flag bits (as in the C ABI).
constexpr int BUBBLE_INLET = 1;
constexpr int BUBBLE_ATMOSPHERE = 2;

struct Scalars {
  long long step;
  long long n_iface;     // interface cells at the end of the last step
  long long n_topology;  // steps in which a labelling run created bubbles
  long long n_label_runs;  // steps with a labelling run
  double bucket;         // orphan excess mass after the last step's phase D
  double share;          // bucket / n_iface, added to every interface cell next step
  double total_mass;
  int next_id;
  int n_live;
  int label_run;         // labelling this step: 1 marked bubbles, 2 all
  int err;               // ERR_* bits
  int nnew;              // new components of the current labelling run
  int nfree;
  int n_il_src;          // interface cells of time t (list length)
  int n_il_dst;          // interface cells of t+1 appended so far
  int n_cand;            // conversion candidates of the current step
  int n_new;             // new interface cells of the current step
  int n_lab;             // cells in the labelled set (listed in clist)
  int n_roots;           // components of the labelled set (roots listed in nlist)
  int if_prev;           // the interface rows of the previous step are valid
  int pad_;
  double mass_ref;       // total mass at creation (watchdog drift reference)
};
constexpr int ERR_CAPACITY = 1;
constexpr int ERR_NONFINITE = 2;
constexpr int ERR_RANGE = 4;
constexpr int ERR_LAYER = 8;    // a liquid cell next to a gas or inlet cell
constexpr int ERR_ORPHAN = 16;  // a gas-region cell without a live bubble
constexpr int ERR_DRIFT = 32;   // total mass drifted beyond the watchdog bound
constexpr int ERR_ILIST = 64;   // more interface cells than the list capacity

// Everything a kernel needs, passed by value.  src/dst refer to time t and
// t+1 of the current step.
struct Dev {
  int nx, ny, nz;
  int per[3];
  int has_walls;
  int max_bubbles;
  int force_topology;
  int freeze;     // no conversions (cell types stay fixed)
  int split_trigger;  // 0 exact 3x3x3 test, 1 anti-parallel normals
  int icap;           // capacity of the interface list and its per-slot arrays
  double trigger_cos;
  double wall_cot;   // cot of the static contact angle (0: mirror at walls)
  int collision;
  double drift_tol;  // watchdog: relative total-mass drift bound (<= 0: off)
  long long N;
  double omega_p, omega_m;
  double sigma, p0, eps, inject;
  double g[3];
  // fields
  void *f_src, *f_dst;
  uint8_t *flag_src, *flag_dst;
  void *phi_src, *phi_dst;
  void *mass, *rhoI, *excess;
  int32_t *bslot;
  int32_t *lab, *aux0, *aux2;
  // bubble table, indexed by slot
  int32_t *b_id, *b_flags, *b_live;
  double *b_vstar, *b_vol, *b_p;
  long long *b_ngas, *b_niface;
  int32_t *b_rmin, *b_rmax, *b_kept;
  int32_t *b_affect;            // marked by the topology trigger this step
  unsigned long long *b_vacc;   // [B][SUB][VACC]
  unsigned long long *c_acc;    // [B][SUB][NACC] per new component (zero between runs)
  int32_t *newroots;            // [B]
  int32_t *newslot;             // [B]
  // cell lists: interface cells of t and t+1, conversion candidates, new
  // interface cells; claim bits of the new-cell list (one byte per cell)
  int32_t *ilist_src, *ilist_dst, *clist, *nlist;
  unsigned *mark;
  // per interface-list slot: gas density (FP64) or its deviation from 1,
  // the bit mask of directions to reconstruct, and the unit normal (split
  // trigger by normals only)
  void *gasv;
  uint32_t *nmask;
  float *nrm;  // [3][icap] by slot of the list of t
  // per tile of the ordered interface-list build: counts and offsets
  int32_t *tilecount, *tileoff;
  // outputs of the interface kernel by list slot (post-collision values,
  // new flag byte), merged into the lattice by the liquid-cell kernel, and
  // the list slot of every interface cell of time t.  Rows and slots are
  // kept for two steps (by step parity): the interface kernel reads the
  // rows of the previous step for the cells that were interface cells then
  void *f_if;
  const void *f_if_prev;
  uint8_t *nflag;
  int32_t *islot;
  int32_t *islot_alt;  // slots of the list of t-1, until k_list_fill writes those of t+1
  // scalars and global accumulators
  Scalars *sc;
  unsigned long long *mass_acc;   // [SUB_MASS][2]
  unsigned long long *bucket_acc; // [SUB][EX_WORDS]
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void fx_split(double v, int scale, long long &hi, long long &lo) {
  long long q = __double2ll_rn(ldexp(v, scale));
  hi = q >> FX_SPLIT;
  lo = q - (hi << FX_SPLIT);
}

__host__ __device__ inline double fx_value(long long hi, long long lo, int scale) {
  return ldexp((double)hi, FX_SPLIT - scale) + ldexp((double)lo, -scale);
}

__device__ __forceinline__ long long wave_sum(long long v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ int wave_sum32(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Block-level combining of keyed sums: a small LDS table with one entry per
// key the block has seen (claimed by compare-and-swap).  Waves add their
// per-key sums into it, and the block adds every entry to global memory
// once (key_sums_flush), so that blocks, not waves, contend for the global
// words.  Keys beyond the table's KB entries go to global memory at once.
// The sums are integers: the result does not depend on the order.
template <int NV, int KB>
struct KeySums {
  int key[KB];
  unsigned long long acc[KB][NV];
};

// Every thread of the block must call it (it synchronises the block).
template <int NV, int KB>
__device__ __forceinline__ void key_sums_init(KeySums<NV, KB> &t) {
  for (int e = threadIdx.x; e < KB; e += blockDim.x) {
    t.key[e] = -1;
#pragma unroll
    for (int k = 0; k < NV; ++k) t.acc[e][k] = 0;
  }
  __syncthreads();
}

// Adds the NV values of every active lane (key >= 0), summed per distinct
// key over the wave (in 64 or, for T = int, 32 bits: the caller bounds the
// sums), into the block's table; the words of a key outside the table go to
// base[(key * stride + sub) * row + off + k] at once.  Every lane of the
// wave must call it.
template <int NV, int KB, class T>
__device__ __forceinline__ void wave_add_by_key_lds(int key, const T *v, KeySums<NV, KB> &t,
                                                    unsigned long long *base, int stride,
                                                    int sub, int row, int off) {
  bool active = key >= 0;
  unsigned long long m = __ballot(active);
  const int lane = __lane_id();
  while (m) {
    int leader = __ffsll((long long)m) - 1;
    int lkey = __shfl(key, leader, 64);
    bool mine = active && key == lkey;
    long long s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      if constexpr (sizeof(T) == 4) s[k] = wave_sum32(mine ? v[k] : 0);
      else s[k] = wave_sum(mine ? (long long)v[k] : 0ll);
    }
    if (lane == leader) {
      int e = 0;
      for (; e < KB; ++e) {
        const int prev = atomicCAS(&t.key[e], -1, lkey);
        if (prev == -1 || prev == lkey) break;
      }
      if (e < KB) {
#pragma unroll
        for (int k = 0; k < NV; ++k) atomicAdd(&t.acc[e][k], (unsigned long long)s[k]);
      } else {
#pragma unroll
        for (int k = 0; k < NV; ++k)
          atomicAdd(&base[((long long)lkey * stride + sub) * row + off + k],
                    (unsigned long long)s[k]);
      }
    }
    unsigned long long mm = __ballot(mine);
    if (mine) active = false;
    m &= ~mm;
  }
}

// Adds the table to base[(key * stride + sub) * row + off + k].  Every
// thread of the block must call it, after its last wave_add_by_key_lds.
template <int NV, int KB>
__device__ __forceinline__ void key_sums_flush(KeySums<NV, KB> &t, unsigned long long *base,
                                               int stride, int sub, int row, int off) {
  __syncthreads();
  for (int q = threadIdx.x; q < KB * NV; q += blockDim.x) {
    const int e = q / NV, k = q % NV;
    const int key = t.key[e];
    const unsigned long long x = t.acc[e][k];
    if (key >= 0 && x != 0)
      atomicAdd(&base[((long long)key * stride + sub) * row + off + k], x);
  }
}

}  // namespace fslbm
