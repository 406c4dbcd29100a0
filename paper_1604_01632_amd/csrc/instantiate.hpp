// Kernel launch sequence of one step for one precision.  Included by one
// translation unit per precision.
#pragma once
#include "kernels.hpp"
#include "launch.hpp"

namespace fslbm {

template <class P>
static void phase_impl(int ph, const Dev &d, const LaunchCfg &c, hipStream_t s) {
  switch (ph) {
    case PH_BULK: {
      const int gx = (d.nx + c.bx - 1) / c.bx;
      const unsigned nb = (unsigned)gx * (unsigned)d.ny * (unsigned)d.nz;
      if (c.with_mass) k_bulk<P, true><<<nb, c.bx, 0, s>>>(d, gx);
      else k_bulk<P, false><<<nb, c.bx, 0, s>>>(d, gx);
      break;
    }
    case PH_IFACE:
      k_geom<P><<<c.list_grid, 256, 0, s>>>(d);
      if (c.with_mass) k_iface<P, true><<<c.list_grid, 256, 0, s>>>(d);
      else k_iface<P, false><<<c.list_grid, 256, 0, s>>>(d);
      break;
    case PH_CONVERT:
      k_conv_types<P><<<c.small_grid, 256, 0, s>>>(d);
      k_conv_init<P><<<c.small_grid, 256, 0, s>>>(d);
      break;
    case PH_EXCESS:
      k_excess<P><<<c.small_grid, 256, 0, s>>>(d);
      break;
    case PH_GATHER: {
      k_gather<P><<<c.list_grid, 256, 0, s>>>(d);
      const int ntiles = (int)((d.N + LTILE - 1) / LTILE);
      k_list_count<<<ntiles, 256, 0, s>>>(d);
      k_list_scan<<<1, 1024, 0, s>>>(d, ntiles);
      k_list_fill<<<ntiles, 256, 0, s>>>(d);
      k_volumes<P><<<1, 1024, 0, s>>>(d);
      break;
    }
    case PH_LABEL:
      k_label_init<<<c.cell_grid, 256, 0, s>>>(d);
      k_label_union<<<c.cell_grid, 256, 0, s>>>(d);
      k_label_roots<<<c.cell_grid, 256, 0, s>>>(d);
      k_label_decide<<<c.cell_grid, 256, 0, s>>>(d);
      k_label_assign<<<1, 1024, 0, s>>>(d);
      k_label_accumulate<P><<<c.cell_grid, 256, 0, s>>>(d);
      k_label_finish<<<1, 1024, 0, s>>>(d);
      k_label_rewrite<<<c.cell_grid, 256, 0, s>>>(d);
      break;
    case PH_BUBBLES:
      k_bubbles<<<1, 1024, 0, s>>>(d);
      break;
    default:
      break;
  }
}

template <class P>
static void init_feq_impl(const Dev &d, const LaunchCfg &c, const double *rho, const double *u,
                          hipStream_t s) {
  k_init_feq<P><<<c.cell_grid, 256, 0, s>>>(d, rho, u);
}

template <class P>
static void init_f_impl(const Dev &d, const LaunchCfg &c, const double *src, int a,
                        hipStream_t s) {
  k_init_f<P><<<c.cell_grid, 256, 0, s>>>(d, src, a);
}

template <class P>
static void export_impl(const Dev &d, const LaunchCfg &c, double *out, int what, hipStream_t s) {
  k_export<P><<<c.cell_grid, 256, 0, s>>>(d, out, what);
}

template <class P>
static Launchers make_launchers() {
  Launchers L;
  L.phase = phase_impl<P>;
  L.init_feq = init_feq_impl<P>;
  L.init_f = init_f_impl<P>;
  L.exportq = export_impl<P>;
  L.store_bytes = (int)sizeof(typename P::S);
  L.real_bytes = (int)sizeof(typename P::R);
  return L;
}

}  // namespace fslbm
