// Kernel launch sequence of one step for one precision, for one domain or
// for a batch of domains.  Included by one translation unit per precision.
#pragma once
#include <type_traits>

#include "kernels.hpp"
#include "launch.hpp"

namespace fslbm {

// One kernel K of grid class G: for one domain or for the whole batch.
template <class K>
static inline void one(const Dev &d, const LaunchCfg &c, int g, hipStream_t s) {
  if (c.blocks[g] > 0) k_one<K><<<c.blocks[g], K::THREADS, 0, s>>>(d);
}
template <class K>
static inline void many(const BatchCfg &b, int g, hipStream_t s) {
  if (b.total[g] > 0) k_many<K><<<b.total[g], K::THREADS, 0, s>>>(b.devs, b.off[g], b.nd);
}

// The kernels of each phase, in order, with their grid classes.  L is a
// launcher object with `template <class K> void operator()(int g)`.
template <class P, class L>
static void phase_kernels(int ph, bool with_mass, int bulk_threads, L &&launch) {
  switch (ph) {
    case PH_IFACE:
      launch.template go<K_geom<P>>(G_LIST);
      // one domain appends its candidates per block, a batch per wave (a
      // domain of a batch has a short list, and the block-wide append's
      // barriers slow the batched kernel by 7 %)
      if constexpr (std::remove_reference_t<L>::kBatch) {
        if (with_mass) launch.template go<K_iface<P, true, false>>(G_LIST);
        else launch.template go<K_iface<P, false, false>>(G_LIST);
      } else {
        if (with_mass) launch.template go<K_iface<P, true, true>>(G_LIST);
        else launch.template go<K_iface<P, false, true>>(G_LIST);
      }
      break;
    case PH_BULK:
      if (bulk_threads == 128) {
        if (with_mass) launch.template go<K_bulk<P, true, 128>>(G_BULK);
        else launch.template go<K_bulk<P, false, 128>>(G_BULK);
      } else {
        if (with_mass) launch.template go<K_bulk<P, true, 256>>(G_BULK);
        else launch.template go<K_bulk<P, false, 256>>(G_BULK);
      }
      break;
    case PH_CONVERT:
      launch.template go<K_conv_types<P>>(G_SMALL);
      launch.template go<K_conv_init<P>>(G_SMALL);
      break;
    case PH_EXCESS:
      if constexpr (std::remove_reference_t<L>::kBatch) {
        // many domains: the tile counts in a launch of their own (the
        // excess pass's registers would hold the tens of thousands of
        // count blocks of a batch to two waves per SIMD)
        launch.template go<K_excess<P>>(G_SMALL);
        launch.template go<K_list_count>(G_TILE);
      } else {
        launch.template go<K_excess_count<P>>(G_EXCOUNT);
      }
      break;
    case PH_GATHER:
      launch.template go<K_scan_label_init>(G_SCANCELL);
      launch.template go<K_fill_label_union>(G_TILECELL);
      launch.template go<K_gather_label_roots<P>>(G_LISTCELL);
      break;
    case PH_LABEL:
      launch.template go<K_assign_volumes>(G_ONEVOL);
      launch.template go<K_label_accumulate<P>>(G_CELL);
      break;
    case PH_BUBBLES:
      launch.template go<K_bubbles>(G_ONE);
      break;
    default:
      break;
  }
}

struct OneLauncher {
  static constexpr bool kBatch = false;
  const Dev &d;
  const LaunchCfg &c;
  hipStream_t s;
  template <class K>
  void go(int g) {
    one<K>(d, c, g, s);
  }
};

struct ManyLauncher {
  static constexpr bool kBatch = true;
  const BatchCfg &b;
  hipStream_t s;
  template <class K>
  void go(int g) {
    many<K>(b, g, s);
  }
};

template <class P>
static void phase_impl(int ph, const Dev &d, const LaunchCfg &c, hipStream_t s) {
  phase_kernels<P>(ph, c.with_mass != 0, c.bulk_threads, OneLauncher{d, c, s});
}

template <class P>
static void batch_phase_impl(int ph, const BatchCfg &b, hipStream_t s) {
  phase_kernels<P>(ph, b.with_mass != 0, b.bulk_threads, ManyLauncher{b, s});
}

template <class P>
static void batch_bulk_probe_impl(const BatchCfg &b, hipStream_t s) {
  if (b.bulk_threads == 128) many<K_bulk<P, false, 128>>(b, G_BULK, s);
  else many<K_bulk<P, false, 256>>(b, G_BULK, s);
}

template <class P>
static void batch_list_probe_impl(const BatchCfg &b, hipStream_t s) {
  many<K_geom<P>>(b, G_LIST, s);
}

template <class P>
static void init_feq_impl(const Dev &d, const LaunchCfg &c, const double *rho, const double *u,
                          hipStream_t s) {
  k_init_feq<P><<<c.blocks[G_CELL], 256, 0, s>>>(d, rho, u);
}

template <class P>
static void init_f_impl(const Dev &d, const LaunchCfg &c, const double *src, int a,
                        hipStream_t s) {
  k_init_f<P><<<c.blocks[G_CELL], 256, 0, s>>>(d, src, a);
}

template <class P>
static void export_impl(const Dev &d, const LaunchCfg &c, double *out, int what, hipStream_t s) {
  k_export<P><<<c.blocks[G_CELL], 256, 0, s>>>(d, out, what);
}

template <class P>
static void watchdog_impl(const Dev &d, const LaunchCfg &c, hipStream_t s) {
  k_one<K_watchdog<P>><<<c.blocks[G_CELL], K_watchdog<P>::THREADS, 0, s>>>(d);
}

template <class P>
static Launchers make_launchers() {
  Launchers L;
  L.phase = phase_impl<P>;
  L.batch_phase = batch_phase_impl<P>;
  L.batch_bulk_probe = batch_bulk_probe_impl<P>;
  L.batch_list_probe = batch_list_probe_impl<P>;
  L.init_feq = init_feq_impl<P>;
  L.init_f = init_f_impl<P>;
  L.exportq = export_impl<P>;
  L.watchdog = watchdog_impl<P>;
  L.store_bytes = (int)sizeof(typename P::S);
  L.real_bytes = (int)sizeof(typename P::R);
  return L;
}

}  // namespace fslbm
