// HIP kernels of one free-surface lattice Boltzmann step with the enhanced
// bubble model (arXiv:1604.01632), templated on the storage precision.
//
// Step pipeline (one HIP stream, no host synchronisation):
//   k_bulk       liquid cells: pull streaming with half-way bounce-back and
//                collision (Sec. 2.1)
//   k_iface      interface cells: Youngs normal and height-function
//                curvature, gas pressure p_V + 2 sigma kappa (Sec. 2.2),
//                reconstruction of gas-side PDFs, mass exchange, collision,
//                fill level, conversion candidates
//   k_convert    new cell types (closed interface layer) and initial values
//                of new interface cells
//   k_excess     excess mass of converted cells, bucket, topology trigger
//   k_gather     interface cells pull excess mass; fill levels; per-bubble
//                volume sums (Sec. 2.3)
//   k_volumes    per-bubble volumes, bucket share, total mass
//   k_label_*    union-find labelling of the gas region and the merge /
//                split rules (Sec. 2.3.1, 2.3.2) - every kernel returns at
//                once unless the trigger fired
//   k_bubbles    injection and ideal-gas pressure (Sec. 2.2)
#pragma once
#include <float.h>
#include <limits.h>

#include "device.hpp"

namespace fslbm {
// Kernels are local to each precision's translation unit.
namespace {

// D3Q19 in the order of the C ABI.
static constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
__host__ __device__ constexpr double wgt(int a) {
  return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Decisions between quantities that are equal in exact arithmetic (axes of
// a symmetric interface, directions tangent to it) use a relative tie band
// so that they do not depend on round-off.
constexpr double TIE_REL = 1e-10;

// ------------------------------------------------------------ precisions

// FP64: PDFs f stored and computed in double, in the operation order of
// the reference definition.  FP32 / FP16DEV: the deviations h = f - w_a
// from the lattice weights are stored (float / half) and all arithmetic is
// done on them in float, so that the weights (which do not sum to one in
// float) never enter a rounded sum and mass is not biased.
struct P64 {
  using S = double;
  using R = double;
  static constexpr bool EXACT = true;
};
struct P32 {
  using S = float;
  using R = float;
  static constexpr bool EXACT = false;
};
struct P16 {
  using S = _Float16;  // round to nearest even on store
  using R = float;
  static constexpr bool EXACT = false;
};

// Stored value of direction a at cell i: f (FP64) or h = f - w (others).
template <class P>
__device__ __forceinline__ typename P::R ld(const void *f, int a, long long N, long long i) {
  return (typename P::R)((const typename P::S *)f)[a * N + i];
}

template <class P>
__device__ __forceinline__ void st(void *f, int a, long long N, long long i, typename P::R v) {
  ((typename P::S *)f)[a * N + i] = (typename P::S)v;
}

// ------------------------------------------------------------- geometry

__device__ __forceinline__ int wrap_axis(int c, int n, int per) {
  if (!per) return c;
  c %= n;
  return c < 0 ? c + n : c;
}

__device__ __forceinline__ long long cidx(const Dev &d, int x, int y, int z) {
  return (long long)x + (long long)d.nx * ((long long)y + (long long)d.ny * z);
}

// Neighbour of an interior cell (fluid and gas cells are interior on
// non-periodic axes, whose face layers are walls or inlets).
__device__ __forceinline__ long long nbr(const Dev &d, int x, int y, int z, int dx, int dy,
                                         int dz) {
  return cidx(d, wrap_axis(x + dx, d.nx, d.per[0]), wrap_axis(y + dy, d.ny, d.per[1]),
              wrap_axis(z + dz, d.nz, d.per[2]));
}

// Neighbour of any cell, -1 outside the box on a non-periodic axis.
__device__ __forceinline__ long long nbr_checked(const Dev &d, int x, int y, int z, int dx,
                                                 int dy, int dz) {
  int xx = wrap_axis(x + dx, d.nx, d.per[0]);
  int yy = wrap_axis(y + dy, d.ny, d.per[1]);
  int zz = wrap_axis(z + dz, d.nz, d.per[2]);
  if (xx < 0 || xx >= d.nx || yy < 0 || yy >= d.ny || zz < 0 || zz >= d.nz) return -1;
  return cidx(d, xx, yy, zz);
}

__device__ __forceinline__ bool in_gas_region(uint8_t t) {
  return t == T_GAS || t == T_IFACE || t == T_INLET;
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ long long ll(unsigned long long v) { return (long long)v; }

// Per-thread two-word fixed-point accumulator.
struct Fx {
  long long hi = 0, lo = 0;
  __device__ void add(double v, int scale) {
    long long h, l;
    fx_split(v, scale, h, l);
    hi += h;
    lo += l;
  }
};

// Block-wide sum of a per-thread Fx into acc[slot][2].
__device__ __forceinline__ void block_fx_add(Fx v, unsigned long long *acc, int slot) {
  __shared__ long long sh[2][16];
  long long h = wave_sum(v.hi), l = wave_sum(v.lo);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nw = (blockDim.x + 63) / 64;
  if (lane == 0) {
    sh[0][w] = h;
    sh[1][w] = l;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long H = 0, L = 0;
    for (int k = 0; k < nw; ++k) {
      H += sh[0][k];
      L += sh[1][k];
    }
    if (H != 0) atomicAdd(&acc[2 * slot], (unsigned long long)H);
    if (L != 0) atomicAdd(&acc[2 * slot + 1], (unsigned long long)L);
  }
}

__device__ __forceinline__ void block_count_add(long long c, unsigned long long *acc, int slot) {
  __shared__ long long shc[16];
  long long s = wave_sum(c);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nw = (blockDim.x + 63) / 64;
  if (lane == 0) shc[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int k = 0; k < nw; ++k) t += shc[k];
    if (t != 0) atomicAdd(&acc[slot], (unsigned long long)t);
  }
}

// Block-wide sum of per-thread exact-sum words into acc[slot][EX_WORDS].
__device__ __forceinline__ void block_ex_add(const ExTerm &v, unsigned long long *acc, int slot) {
  __shared__ long long shx[EX_WORDS][16];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int nw = (blockDim.x + 63) / 64;
#pragma unroll
  for (int c = 0; c < EX_WORDS; ++c) {
    const long long s = wave_sum(v.w[c]);
    if (lane == 0) shx[c][w] = s;
  }
  __syncthreads();
  if (threadIdx.x < EX_WORDS) {
    long long t = 0;
    for (int k = 0; k < nw; ++k) t += shx[threadIdx.x][k];
    if (t != 0) atomicAdd(&acc[slot * EX_WORDS + threadIdx.x], (unsigned long long)t);
  }
}

__device__ __forceinline__ void ex_accumulate(ExTerm &acc, double v) {
  const ExTerm t = ex_split(v);
#pragma unroll
  for (int c = 0; c < EX_WORDS; ++c) acc.w[c] += t.w[c];
}

// ------------------------------------------------------------ equilibrium

// Second-order equilibrium, written in the reference operation order
// (divisions by cs^2) for the FP64 form.
__device__ __forceinline__ void feq_exact(double rho, const double *u, double *out) {
  const double cs2 = 1.0 / 3.0;
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const double cu = CX[a] * u[0] + CY[a] * u[1] + CZ[a] * u[2];
    out[a] = rho * wgt(a) *
             (1.0 + cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

// Equilibrium in the stored representation: f_eq (FP64) or
// f_eq - w = w [drho + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)] with
// drho = rho - 1 (deviation forms).
template <class P>
__device__ __forceinline__ void eqv(typename P::R rho, typename P::R drho,
                                    const typename P::R *u, typename P::R *out) {
  using R = typename P::R;
  if constexpr (P::EXACT) {
    (void)drho;
    feq_exact(rho, u, out);
  } else {
    const R uu15 = (R)1.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const R cu = (R)CX[a] * u[0] + (R)CY[a] * u[1] + (R)CZ[a] * u[2];
      out[a] = (R)wgt(a) * (drho + rho * ((R)3 * cu + (R)4.5 * cu * cu - uu15));
    }
  }
}

// Density, its deviation from 1 and the collision velocity u = sum c f /
// rho - g/2 recovered from stored post-collision values.
template <class P>
__device__ __forceinline__ void recover(const Dev &d, const typename P::R *v, typename P::R &rho,
                                        typename P::R &drho, typename P::R *u) {
  using R = typename P::R;
  R s = (R)0, j[3] = {(R)0, (R)0, (R)0};
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    s += v[a];
    j[0] += CX[a] * v[a];
    j[1] += CY[a] * v[a];
    j[2] += CZ[a] * v[a];
  }
  if constexpr (P::EXACT) {
    rho = s;
    drho = s - (R)1;
  } else {
    drho = s;
    rho = (R)1 + s;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = j[k] / rho - (R)0.5 * (R)d.g[k];
}

// ------------------------------------------------------------- collision

// BGK (omega_m == omega_p) or TRT collision with a Guo body force, in
// place: f holds the streamed PDFs on entry and the post-collision PDFs on
// exit; rho and u are the collision density and velocity
// u = (sum c f + rho g / 2) / rho.
template <class P>
__device__ __forceinline__ void collide(const Dev &d, typename P::R *f, typename P::R &rho_o,
                                        typename P::R *u_o) {
  using R = typename P::R;
  if constexpr (P::EXACT) {
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      rho += f[a];
      jx += CX[a] * f[a];
      jy += CY[a] * f[a];
      jz += CZ[a] * f[a];
    }
    double u[3];
    u[0] = (jx + 0.5 * rho * d.g[0]) / rho;
    u[1] = (jy + 0.5 * rho * d.g[1]) / rho;
    u[2] = (jz + 0.5 * rho * d.g[2]) / rho;
    double fe[Q];
    feq_exact(rho, u, fe);
    const double wp = d.omega_p, wm = d.omega_m;
    const double Fx = rho * d.g[0], Fy = rho * d.g[1], Fz = rho * d.g[2];
    const double uF = u[0] * Fx + u[1] * Fy + u[2] * Fz;
    double out[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int b = opp(a);
      const double cu = CX[a] * u[0] + CY[a] * u[1] + CZ[a] * u[2];
      const double cF = CX[a] * Fx + CY[a] * Fy + CZ[a] * Fz;
      const double s_even = wgt(a) * (-3.0 * uF + 9.0 * cu * cF);
      const double s_odd = wgt(a) * (3.0 * cF);
      const double f_even = 0.5 * (f[a] + f[b]), f_odd = 0.5 * (f[a] - f[b]);
      const double e_even = 0.5 * (fe[a] + fe[b]), e_odd = 0.5 * (fe[a] - fe[b]);
      out[a] = f[a] - wp * (f_even - e_even) - wm * (f_odd - e_odd) +
               (1.0 - 0.5 * wp) * s_even + (1.0 - 0.5 * wm) * s_odd;
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) f[a] = out[a];
    rho_o = rho;
    u_o[0] = u[0];
    u_o[1] = u[1];
    u_o[2] = u[2];
  } else {
    // deviation form: f holds h = f - w
    R dr = (R)0;
#pragma unroll
    for (int a = 0; a < Q; ++a) dr += f[a];
    const R jx = (f[1] - f[2]) + (f[7] - f[8]) + (f[9] - f[10]) + (f[11] - f[12]) + (f[13] - f[14]);
    const R jy = (f[3] - f[4]) + (f[7] - f[8]) - (f[9] - f[10]) + (f[15] - f[16]) + (f[17] - f[18]);
    const R jz = (f[5] - f[6]) + (f[11] - f[12]) - (f[13] - f[14]) + (f[15] - f[16]) - (f[17] - f[18]);
    const R rho = (R)1 + dr;
    const R gx = (R)d.g[0], gy = (R)d.g[1], gz = (R)d.g[2];
    const R inv = (R)1 / rho;
    const R ux = jx * inv + (R)0.5 * gx, uy = jy * inv + (R)0.5 * gy, uz = jz * inv + (R)0.5 * gz;
    const R wp = (R)d.omega_p, wm = (R)d.omega_m;
    const R kp = (R)1 - (R)0.5 * wp, km = (R)1 - (R)0.5 * wm;
    const R uu15 = (R)1.5 * (ux * ux + uy * uy + uz * uz);
    const R ug3 = (R)3 * (ux * gx + uy * gy + uz * gz);
    {
      const R w0 = (R)wgt(0);
      const R eq0 = w0 * (dr - rho * uu15);
      f[0] = f[0] - wp * (f[0] - eq0) - kp * w0 * rho * ug3;
    }
#pragma unroll
    for (int a = 1; a < Q; a += 2) {
      const int b = a + 1;
      const R w = (R)wgt(a);
      const R wr = w * rho;
      const R cu = (R)CX[a] * ux + (R)CY[a] * uy + (R)CZ[a] * uz;
      const R cg = (R)CX[a] * gx + (R)CY[a] * gy + (R)CZ[a] * gz;
      const R eq_even = w * (dr + rho * ((R)4.5 * cu * cu - uu15));
      const R eq_odd = wr * (R)3 * cu;
      const R s_even = wr * ((R)9 * cu * cg - ug3);
      const R s_odd = wr * (R)3 * cg;
      const R fe = (R)0.5 * (f[a] + f[b]), fo = (R)0.5 * (f[a] - f[b]);
      const R de = -wp * (fe - eq_even) + kp * s_even;
      const R dodd = -wm * (fo - eq_odd) + km * s_odd;
      f[a] = f[a] + de + dodd;
      f[b] = f[b] + de - dodd;
    }
    rho_o = rho;
    u_o[0] = ux;
    u_o[1] = uy;
    u_o[2] = uz;
  }
}

// -------------------------------------------------- interface geometry

// Fill level seen by the geometry at integer position (x,y,z): periodic
// axes wrap; samples on wall cells or outside the box take the value of
// their mirror image across the wall plane (half-way between the wall layer
// and the first fluid layer).
template <class R>
__device__ __forceinline__ R phi_sample(const Dev &d, const R *phi, int x, int y, int z) {
  int c[3] = {x, y, z};
  const int n[3] = {d.nx, d.ny, d.nz};
#pragma unroll
  for (int k = 0; k < 3; ++k) c[k] = wrap_axis(c[k], n[k], d.per[k]);
  if (!d.has_walls) return phi[cidx(d, c[0], c[1], c[2])];
  bool inside = true;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (c[k] < 0 || c[k] >= n[k]) inside = false;
  if (inside) {
    const long long i = cidx(d, c[0], c[1], c[2]);
    if ((d.flag_src[i] & TYPE_MASK) != T_WALL) return phi[i];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d.per[k]) continue;
    if (c[k] <= 0) c[k] = 1 - c[k];
    else if (c[k] >= n[k] - 1) c[k] = 2 * n[k] - 3 - c[k];
  }
  return phi[cidx(d, c[0], c[1], c[2])];
}

// Parker-Youngs gradient of the fill level, weights 4/2/1 for face / edge /
// corner offsets; points from gas into liquid.
template <class R>
__device__ __forceinline__ void youngs_normal(const Dev &d, const R *phi, int x, int y, int z,
                                              R *n) {
  n[0] = n[1] = n[2] = (R)0;
#pragma unroll
  for (int p = -1; p <= 1; ++p)
#pragma unroll
    for (int q = -1; q <= 1; ++q) {
      const R w = (R)((p == 0 ? 2 : 1) * (q == 0 ? 2 : 1));
      n[0] += w * (phi_sample(d, phi, x + 1, y + p, z + q) - phi_sample(d, phi, x - 1, y + p, z + q));
      n[1] += w * (phi_sample(d, phi, x + p, y + 1, z + q) - phi_sample(d, phi, x + p, y - 1, z + q));
      n[2] += w * (phi_sample(d, phi, x + p, y + q, z + 1) - phi_sample(d, phi, x + p, y + q, z - 1));
    }
}

// Height-function curvature from 7-cell columns along axis dd over a 3x3
// footprint; kappa > 0 where the liquid is convex.
template <class R>
__device__ __noinline__ R height_curvature_axis(const Dev &d, const R *phi, int x, int y, int z,
                                                int dd) {
  const int e1 = (dd == 0) ? 1 : 0;
  const int e2 = (dd == 2) ? 1 : 2;
  R H[3][3];
#pragma unroll
  for (int a = -1; a <= 1; ++a)
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
      R s = (R)0;
#pragma unroll
      for (int k = -3; k <= 3; ++k) {
        int c[3] = {x, y, z};
        c[e1] += a;
        c[e2] += b;
        c[dd] += k;
        s += phi_sample(d, phi, c[0], c[1], c[2]);
      }
      H[a + 1][b + 1] = s;
    }
  const R Ha = (R)0.5 * (H[2][1] - H[0][1]);
  const R Hb = (R)0.5 * (H[1][2] - H[1][0]);
  const R Haa = H[2][1] - (R)2 * H[1][1] + H[0][1];
  const R Hbb = H[1][2] - (R)2 * H[1][1] + H[1][0];
  const R Hab = (R)0.25 * (H[2][2] - H[2][0] - H[0][2] + H[0][0]);
  const R num = Haa * ((R)1 + Hb * Hb) + Hbb * ((R)1 + Ha * Ha) - (R)2 * Ha * Hb * Hab;
  const R qq = (R)1 + Ha * Ha + Hb * Hb;
  const R den = qq * sqrt(qq);
  return (R)-0.5 * num / den;
}

// Mean curvature: height function along the dominant normal axis; axes
// within the tie band of the largest |n_i| are averaged (order x, y, z).
template <class R>
__device__ __forceinline__ R curvature(const Dev &d, const R *phi, int x, int y, int z,
                                       const R *n) {
  const R an[3] = {fabs(n[0]), fabs(n[1]), fabs(n[2])};
  R m = an[0];
  if (an[1] > m) m = an[1];
  if (an[2] > m) m = an[2];
  if (m == (R)0) return (R)0;
  const R thr = m - (R)TIE_REL * m;
  R sum = (R)0;
  int cnt = 0;
  for (int dd = 0; dd < 3; ++dd)
    if (an[dd] >= thr) {
      sum += height_curvature_axis(d, phi, x, y, z, dd);
      ++cnt;
    }
  return sum / (R)cnt;
}

// ---------------------------------------------------------------- k_bulk

// Liquid cells: pull streaming (half-way bounce-back from walls) and
// collision.  Also copies the flag of gas / wall / inlet cells to the new
// flag field; interface cells are left to k_iface.
template <class P, bool WITH_MASS>
__global__ void __launch_bounds__(256) k_bulk(Dev d) {
  using R = typename P::R;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  Fx mass;
  if (x < d.nx) {
    const long long i = cidx(d, x, y, z);
    const uint8_t fl = d.flag_src[i];
    const uint8_t t = fl & TYPE_MASK;
    if (t == T_LIQ) {
      const int xs[3] = {wrap_axis(x - 1, d.nx, d.per[0]), x, wrap_axis(x + 1, d.nx, d.per[0])};
      const int ys[3] = {wrap_axis(y - 1, d.ny, d.per[1]), y, wrap_axis(y + 1, d.ny, d.per[1])};
      const int zs[3] = {wrap_axis(z - 1, d.nz, d.per[2]), z, wrap_axis(z + 1, d.nz, d.per[2])};
      R f[Q];
      if (!(fl & NEAR_WALL)) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const long long s = cidx(d, xs[1 - CX[a]], ys[1 - CY[a]], zs[1 - CZ[a]]);
          f[a] = ld<P>(d.f_src, a, d.N, s);
        }
      } else {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const long long s = cidx(d, xs[1 - CX[a]], ys[1 - CY[a]], zs[1 - CZ[a]]);
          const uint8_t ts = d.flag_src[s] & TYPE_MASK;
          f[a] = (ts == T_WALL) ? ld<P>(d.f_src, opp(a), d.N, i) : ld<P>(d.f_src, a, d.N, s);
        }
      }
      R rho, u[3];
      collide<P>(d, f, rho, u);
#pragma unroll
      for (int a = 0; a < Q; ++a) st<P>(d.f_dst, a, d.N, i, f[a]);
      if (WITH_MASS) mass.add((double)rho, FX_VOL);
      d.flag_dst[i] = fl & (STATIC_BITS | TYPE_MASK);
    } else if (t != T_IFACE) {
      d.flag_dst[i] = fl & (STATIC_BITS | TYPE_MASK);
    }
  }
  if (WITH_MASS)
    block_fx_add(mass, d.mass_acc, (blockIdx.y + blockIdx.z * gridDim.y) % SUB_MASS);
}

// --------------------------------------------------------------- k_iface

template <class P>
__device__ __forceinline__ double iface_cell(const Dev &d, int x, int y, int z, long long i,
                                             uint8_t fl) {
  using R = typename P::R;
  const R *phi = (const R *)d.phi_src;
  const long long N = d.N;
  R fs[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) fs[a] = ld<P>(d.f_src, a, N, i);

  // interface geometry and gas-side equilibrium
  R n[3];
  youngs_normal(d, phi, x, y, z, n);
  const R kappa = curvature(d, phi, x, y, z, n);
  const int slot = d.bslot[i];
  R rho_gas, drho_gas;
  if constexpr (P::EXACT) {
    const R p_gas = (R)d.b_p[slot] + (R)2.0 * (R)d.sigma * kappa;
    rho_gas = (R)3.0 * p_gas;
    drho_gas = rho_gas - (R)1;
  } else {
    // p = rho cs^2: rho_gas - 1 = (3 p_V - 1) + 6 sigma kappa
    drho_gas = (R)(3.0 * d.b_p[slot] - 1.0) + (R)6 * (R)d.sigma * kappa;
    rho_gas = (R)1 + drho_gas;
  }
  R feq_gas[Q];
  {
    R r, dr, ub[3];
    recover<P>(d, fs, r, dr, ub);
    eqv<P>(rho_gas, drho_gas, ub, feq_gas);
  }
  const R nn = fabs(n[0]) + fabs(n[1]) + fabs(n[2]);

  // pull streaming with bounce-back and reconstruction; keep the raw
  // streamed values for the mass exchange
  R fin[Q], raw[Q];
  uint8_t tsrc[Q];
  fin[0] = fs[0];
  raw[0] = fs[0];
  tsrc[0] = T_IFACE;
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const int b = opp(a);
    const long long s = nbr(d, x, y, z, -CX[a], -CY[a], -CZ[a]);
    const uint8_t ts = d.flag_src[s] & TYPE_MASK;
    tsrc[a] = ts;
    const R recon = feq_gas[a] + feq_gas[b] - fs[b];
    raw[a] = (R)0;
    if (ts == T_WALL) {
      fin[a] = fs[b];
    } else if (ts == T_GAS || ts == T_INLET) {
      fin[a] = recon;
    } else {
      raw[a] = ld<P>(d.f_src, a, N, s);
      fin[a] = raw[a];
      const R cn = CX[a] * n[0] + CY[a] * n[1] + CZ[a] * n[2];
      if (cn > (R)TIE_REL * nn) fin[a] = recon;
    }
  }

  // mass exchange with the neighbour y = x + c_a, whose outgoing value
  // towards x is the raw streamed value of direction opp(a)
  R dm = (R)0;
  const R phi_x = phi[i];
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const int b = opp(a);
    const uint8_t ty = tsrc[b];
    const R diff = (ty == T_LIQ || ty == T_IFACE) ? raw[b] - fs[a] : (R)0;
    if (ty == T_LIQ) {
      dm += diff;
    } else if (ty == T_IFACE) {
      const long long yidx = nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
      dm += (R)0.5 * (phi_x + phi[yidx]) * diff;
    }
  }
  const R m_new = ((R *)d.mass)[i] + dm + (R)d.sc->share;

  R rho, u[3];
  collide<P>(d, fin, rho, u);
#pragma unroll
  for (int a = 0; a < Q; ++a) st<P>(d.f_dst, a, N, i, fin[a]);
  const R phi_new = m_new / rho;
  ((R *)d.mass)[i] = m_new;
  ((R *)d.rhoI)[i] = rho;
  ((R *)d.phi_dst)[i] = phi_new;
  uint8_t nf = fl & (STATIC_BITS | TYPE_MASK);
  if (phi_new > (R)1 + (R)d.eps && !(fl & NEAR_INLET)) nf |= CAND_F;
  if (phi_new < -(R)d.eps) nf |= CAND_E;
  d.flag_dst[i] = nf;
  return (double)m_new;
}

template <class P, bool WITH_MASS>
__global__ void __launch_bounds__(256) k_iface(Dev d) {
  Fx mass;
  const int rows = d.ny * d.nz;
  for (int row = blockIdx.x; row < rows; row += gridDim.x) {
    const int y = row % d.ny, z = row / d.ny;
    for (int x = threadIdx.x; x < d.nx; x += blockDim.x) {
      const long long i = cidx(d, x, y, z);
      const uint8_t fl = d.flag_src[i];
      if ((fl & TYPE_MASK) == T_IFACE) {
        const double m = iface_cell<P>(d, x, y, z, i, fl);
        if (WITH_MASS) mass.add(m, FX_VOL);
      }
    }
  }
  if (WITH_MASS) block_fx_add(mass, d.mass_acc, blockIdx.x % SUB_MASS);
}

// ------------------------------------------------------------- k_convert

// New cell types (phase-synchronous; every rule reads the candidate bits
// and the types of time t):
//   filled interface -> liquid; emptied interface (no filled neighbour)
//   -> gas; gas next to a filled cell -> interface; liquid next to an
//   emptied cell -> interface.
// New interface cells from gas get f = f_eq(mean rho, mean u) of their
// neighbours that were interface or liquid at t, and m = 0; those from
// liquid get m = rho and the smallest bubble ID of their emptied
// neighbours.
template <class P>
__global__ void __launch_bounds__(256) k_convert(Dev d) {
  using R = typename P::R;
  const int rows = d.ny * d.nz;
  for (int row = blockIdx.x; row < rows; row += gridDim.x) {
    const int y = row % d.ny, z = row / d.ny;
    for (int x = threadIdx.x; x < d.nx; x += blockDim.x) {
      const long long i = cidx(d, x, y, z);
      const uint8_t t = d.flag_src[i] & TYPE_MASK;
      if (t == T_WALL || t == T_INLET) continue;
      const uint8_t fd = d.flag_dst[i];
      uint8_t tn = t;
      if (t == T_IFACE) {
        if (fd & CAND_F) {
          tn = T_LIQ;
        } else if (fd & CAND_E) {
          bool nf = false;
#pragma unroll
          for (int a = 1; a < Q; ++a)
            if (d.flag_dst[nbr(d, x, y, z, CX[a], CY[a], CZ[a])] & CAND_F) nf = true;
          if (!nf) tn = T_GAS;
        }
      } else if (t == T_GAS) {
        bool nf = false;
#pragma unroll
        for (int a = 1; a < Q; ++a)
          if (d.flag_dst[nbr(d, x, y, z, CX[a], CY[a], CZ[a])] & CAND_F) nf = true;
        if (nf) {
          tn = T_IFACE;
          // mean density and velocity of the neighbours that were fluid at t,
          // recovered from their post-collision values
          R rs = (R)0, us[3] = {(R)0, (R)0, (R)0};
          int cnt = 0;
          for (int a = 1; a < Q; ++a) {
            const long long j = nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
            const uint8_t tj = d.flag_src[j] & TYPE_MASK;
            if (!(tj == T_IFACE || tj == T_LIQ)) continue;
            R v[Q];
#pragma unroll
            for (int c = 0; c < Q; ++c) v[c] = ld<P>(d.f_dst, c, d.N, j);
            R r, dr, uj[3];
            recover<P>(d, v, r, dr, uj);
            rs += P::EXACT ? r : dr;
#pragma unroll
            for (int k = 0; k < 3; ++k) us[k] += uj[k];
            ++cnt;
          }
          const R mean = rs / (R)cnt;
          const R rb = P::EXACT ? mean : (R)1 + mean;
          const R ub[3] = {us[0] / (R)cnt, us[1] / (R)cnt, us[2] / (R)cnt};
          R fe[Q];
          eqv<P>(rb, P::EXACT ? rb - (R)1 : mean, ub, fe);
#pragma unroll
          for (int c = 0; c < Q; ++c) st<P>(d.f_dst, c, d.N, i, fe[c]);
          ((R *)d.rhoI)[i] = rb;
          ((R *)d.mass)[i] = (R)0;
          atomicAdd((unsigned long long *)&d.b_ngas[d.bslot[i]], (unsigned long long)-1ll);
        }
      } else if (t == T_LIQ) {
        int best_slot = -1, best_id = INT_MAX;
        for (int a = 1; a < Q; ++a) {
          const long long j = nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
          if (!(d.flag_dst[j] & CAND_E)) continue;
          // j is emptied unless one of its neighbours is filled
          const int jx = (int)(j % d.nx), jy = (int)((j / d.nx) % d.ny),
                    jz = (int)(j / ((long long)d.nx * d.ny));
          bool nf = false;
          for (int b = 1; b < Q; ++b)
            if (d.flag_dst[nbr(d, jx, jy, jz, CX[b], CY[b], CZ[b])] & CAND_F) nf = true;
          if (nf) continue;
          const int s = d.bslot[j];
          const int id = d.b_id[s];
          if (id < best_id) {
            best_id = id;
            best_slot = s;
          }
        }
        if (best_slot >= 0) {
          tn = T_IFACE;
          R v[Q];
#pragma unroll
          for (int c = 0; c < Q; ++c) v[c] = ld<P>(d.f_dst, c, d.N, i);
          R r, dr, uu[3];
          recover<P>(d, v, r, dr, uu);
          ((R *)d.mass)[i] = r;
          ((R *)d.rhoI)[i] = r;
          d.bslot[i] = best_slot;
        }
      }
      if (tn != t) d.flag_dst[i] = (uint8_t)((fd & ~TYPE_MASK) | tn);
    }
  }
}

// -------------------------------------------------------------- k_excess

// 3x3x3 block positions p = (dx+1) + 3 (dy+1) + 9 (dz+1); N18 offsets are
// those with 1 <= |dx|+|dy|+|dz| <= 2.
__device__ __forceinline__ int blk_pos(int dx, int dy, int dz) {
  return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}
__device__ __forceinline__ uint32_t adj_mask(int p) {
  // block positions adjacent (18-neighbourhood) to position p
  const int px = p % 3 - 1, py = (p / 3) % 3 - 1, pz = p / 9 - 1;
  uint32_t m = 0;
  for (int q = 0; q < 27; ++q) {
    const int dx = q % 3 - 1 - px, dy = (q / 3) % 3 - 1 - py, dz = q / 9 - 1 - pz;
    const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy, az = dz < 0 ? -dz : dz;
    const int l1 = ax + ay + az;
    if (ax <= 1 && ay <= 1 && az <= 1 && l1 >= 1 && l1 <= 2) m |= 1u << q;
  }
  return m;
}

// Removing the filled cell x from the gas region cannot disconnect it if
// (a) x's gas-region neighbours (new state) are connected inside x's 3x3x3
// block, and (b) every filled neighbour y of x shares a gas-region
// neighbour with x.  Returns true when a relabelling is needed.
__device__ bool split_possible(const Dev &d, int x, int y, int z) {
  uint32_t setm = 0, filled = 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const long long j = nbr(d, x, y, z, dx, dy, dz);
        const uint8_t tn = d.flag_dst[j] & TYPE_MASK;
        const int p = blk_pos(dx, dy, dz);
        if (in_gas_region(tn)) setm |= 1u << p;
        const int l1 = (dx != 0) + (dy != 0) + (dz != 0);
        if (l1 <= 2 && (d.flag_src[j] & TYPE_MASK) == T_IFACE && tn == T_LIQ) filled |= 1u << p;
      }
  const uint32_t n18 = adj_mask(13);
  const uint32_t targets = setm & n18;
  if (!targets) return true;
  uint32_t reach = targets & (~targets + 1u);
  for (;;) {
    uint32_t grow = reach;
    for (int p = 0; p < 27; ++p)
      if (reach & (1u << p)) grow |= adj_mask(p) & setm;
    if (grow == reach) break;
    reach = grow;
  }
  if (targets & ~reach) return true;
  for (int p = 0; p < 27; ++p)
    if (filled & (1u << p))
      if (!(setm & n18 & adj_mask(p))) return true;
  return false;
}

template <class P>
__global__ void __launch_bounds__(256) k_excess(Dev d) {
  using R = typename P::R;
  ExTerm orphan;
#pragma unroll
  for (int c = 0; c < EX_WORDS; ++c) orphan.w[c] = 0;
  bool trig = false;
  const int rows = d.ny * d.nz;
  for (int row = blockIdx.x; row < rows; row += gridDim.x) {
    const int y = row % d.ny, z = row / d.ny;
    for (int x = threadIdx.x; x < d.nx; x += blockDim.x) {
      const long long i = cidx(d, x, y, z);
      const uint8_t t = d.flag_src[i] & TYPE_MASK;
      const uint8_t tn = d.flag_dst[i] & TYPE_MASK;
      if (t == tn) continue;
      if (t == T_IFACE && (tn == T_LIQ || tn == T_GAS)) {
        const bool filled = tn == T_LIQ;
        R *mass = (R *)d.mass;
        const R e = filled ? mass[i] - ((R *)d.rhoI)[i] : mass[i];
        int nI = 0;
#pragma unroll
        for (int a = 1; a < Q; ++a)
          if ((d.flag_dst[nbr(d, x, y, z, CX[a], CY[a], CZ[a])] & TYPE_MASK) == T_IFACE) ++nI;
        if (nI > 0) {
          ((R *)d.excess)[i] = e / (R)nI;
        } else {
          ((R *)d.excess)[i] = (R)0;
          ex_accumulate(orphan, (double)e);
        }
        if (filled) {
          mass[i] = ((R *)d.rhoI)[i];
          ((R *)d.phi_src)[i] = (R)1;
          ((R *)d.phi_dst)[i] = (R)1;
          if (split_possible(d, x, y, z)) trig = true;
          d.bslot[i] = -1;
        } else {
          mass[i] = (R)0;
          ((R *)d.phi_src)[i] = (R)0;
          ((R *)d.phi_dst)[i] = (R)0;
          atomicAdd((unsigned long long *)&d.b_ngas[d.bslot[i]], 1ull);
        }
      } else if (t == T_LIQ && tn == T_IFACE) {
        // a new gas-region cell: a merge if its gas-region neighbours carry
        // another bubble
        const int s = d.bslot[i];
        for (int a = 1; a < Q; ++a) {
          const long long j = nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
          if (in_gas_region(d.flag_dst[j] & TYPE_MASK) && d.bslot[j] != s) trig = true;
        }
      }
    }
  }
  if (trig) d.sc->label_run = 1;
  block_ex_add(orphan, d.bucket_acc, blockIdx.x % SUB);
}

// -------------------------------------------------------------- k_gather

// Final interface cells pull the excess of converted neighbours (in
// direction order), recompute phi = m / rho and add 1 - phi to their
// bubble's volume.
template <class P>
__global__ void __launch_bounds__(256) k_gather(Dev d) {
  using R = typename P::R;
  long long count = 0;
  const int sub = blockIdx.x % SUB;
  const int rows = d.ny * d.nz;
  for (int row = blockIdx.x; row < rows; row += gridDim.x) {
    const int y = row % d.ny, z = row / d.ny;
    for (int x0 = 0; x0 < d.nx; x0 += blockDim.x) {
      const int x = x0 + threadIdx.x;
      int key = -1;
      long long v[VACC] = {0, 0, 0, 0, 0, 1};
      if (x < d.nx) {
        const long long i = cidx(d, x, y, z);
        if ((d.flag_dst[i] & TYPE_MASK) == T_IFACE) {
          R add = (R)0;
          bool touched = false;
#pragma unroll
          for (int a = 1; a < Q; ++a) {
            const long long j = nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
            const uint8_t t0 = d.flag_src[j] & TYPE_MASK;
            const uint8_t t1 = d.flag_dst[j] & TYPE_MASK;
            if (t0 == T_IFACE && (t1 == T_LIQ || t1 == T_GAS)) {
              add += ((const R *)d.excess)[j];
              touched = true;
            }
          }
          R m = ((R *)d.mass)[i];
          if (touched) {
            m += add;
            ((R *)d.mass)[i] = m;
          }
          const R ph = m / ((const R *)d.rhoI)[i];
          ((R *)d.phi_dst)[i] = ph;
          key = d.bslot[i];
          const ExTerm t = ex_split(1.0 - (double)ph);
#pragma unroll
          for (int c = 0; c < EX_WORDS; ++c) v[c] = t.w[c];
          ++count;
        }
      }
      wave_add_by_key<VACC>(key, v, d.b_vacc, SUB, sub);
    }
  }
  block_count_add(count, d.niface_acc, sub);
}

// ------------------------------------------------------------- k_volumes

// Per-bubble volume V = (gas + inlet cells) + sum over interface cells of
// (1 - phi), exactly rounded; orphan bucket; total mass.
template <class P>
__global__ void __launch_bounds__(1024) k_volumes(Dev d) {
  for (int s = threadIdx.x; s < d.max_bubbles; s += blockDim.x) {
    unsigned long long *acc = d.b_vacc + (long long)s * SUB * VACC;
    long long w[EX_WORDS] = {0, 0, 0, 0, 0};
    long long cnt = 0;
    for (int k = 0; k < SUB; ++k) {
      for (int c = 0; c < EX_WORDS; ++c) {
        w[c] += ll(acc[VACC * k + c]);
        acc[VACC * k + c] = 0;
      }
      cnt += ll(acc[VACC * k + EX_WORDS]);
      acc[VACC * k + EX_WORDS] = 0;
    }
    if (d.b_live[s]) {
      const ExTerm g = ex_split((double)d.b_ngas[s]);
      for (int c = 0; c < EX_WORDS; ++c) w[c] += g.w[c];
      d.b_vol[s] = ex_value(w);
      d.b_niface[s] = cnt;
    }
  }
  if (threadIdx.x == 0) {
    Scalars *sc = d.sc;
    long long nI = 0;
    for (int k = 0; k < SUB; ++k) {
      nI += ll(d.niface_acc[k]);
      d.niface_acc[k] = 0;
    }
    // the bucket of the last step was spread over this step's interface
    // cells unless there were none
    const double carry = sc->n_iface > 0 ? 0.0 : sc->bucket;
    long long bw[EX_WORDS] = {0, 0, 0, 0, 0};
    const ExTerm ct = ex_split(carry);
    for (int c = 0; c < EX_WORDS; ++c) bw[c] = ct.w[c];
    for (int k = 0; k < SUB; ++k)
      for (int c = 0; c < EX_WORDS; ++c) {
        bw[c] += ll(d.bucket_acc[EX_WORDS * k + c]);
        d.bucket_acc[EX_WORDS * k + c] = 0;
      }
    const double bucket = ex_value(bw);
    long long mh = 0, ml = 0;
    for (int k = 0; k < SUB_MASS; ++k) {
      mh += ll(d.mass_acc[2 * k]);
      ml += ll(d.mass_acc[2 * k + 1]);
      d.mass_acc[2 * k] = d.mass_acc[2 * k + 1] = 0;
    }
    sc->total_mass = fx_value(mh, ml, FX_VOL) + carry;
    sc->bucket = bucket;
    sc->n_iface = nI;
    sc->share = nI > 0 ? bucket / (double)nI : 0.0;
    if (d.force_topology) sc->label_run = 1;
  }
}

// ---------------------------------------------------------- labelling

// Union-find over the gas region (gas, interface, inlet cells of the new
// state) with 18-neighbour adjacency; every root is the smallest index of
// its component.  Roots only ever point to smaller indices, so every find
// terminates.
__device__ __forceinline__ int lab_load(const int32_t *lab, long long i) {
  return __hip_atomic_load(&lab[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int32_t *lab, int i) {
  int p = lab_load(lab, i);
  while (p != i) {
    i = p;
    p = lab_load(lab, i);
  }
  return i;
}

__device__ __forceinline__ void uf_union(int32_t *lab, int a, int b) {
  for (;;) {
    a = uf_find(lab, a);
    b = uf_find(lab, b);
    if (a == b) return;
    if (a < b) {
      const int old = atomicMin(&lab[b], a);
      if (old == b) return;
      b = old;
    } else {
      const int old = atomicMin(&lab[a], b);
      if (old == a) return;
      a = old;
    }
  }
}

#define FSLBM_GRID_STRIDE(i) \
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < d.N; \
       i += (long long)gridDim.x * blockDim.x)

__device__ __forceinline__ void coords(const Dev &d, long long i, int &x, int &y, int &z) {
  x = (int)(i % d.nx);
  y = (int)((i / d.nx) % d.ny);
  z = (int)(i / ((long long)d.nx * d.ny));
}

__global__ void __launch_bounds__(256) k_label_init(Dev d) {
  if (!d.sc->label_run) return;
  FSLBM_GRID_STRIDE(i) {
    d.lab[i] = in_gas_region(d.flag_dst[i] & TYPE_MASK) ? (int)i : -1;
    d.aux0[i] = INT_MAX;
    d.aux1[i] = -1;
    d.aux2[i] = 0;
  }
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long long t = t0; t < d.max_bubbles; t += (long long)gridDim.x * blockDim.x) {
    d.b_rmin[t] = INT_MAX;
    d.b_rmax[t] = -1;
    d.b_kept[t] = 0;
    for (int k = 0; k < NACC; ++k) d.c_acc[t * NACC + k] = 0;
  }
  if (t0 == 0) d.sc->nnew = 0;
}

__global__ void __launch_bounds__(256) k_label_union(Dev d) {
  if (!d.sc->label_run) return;
  FSLBM_GRID_STRIDE(i) {
    if (d.lab[i] < 0) continue;
    int x, y, z;
    coords(d, i, x, y, z);
    // one direction of every opposite pair covers every edge once
    for (int a = 1; a < Q; a += 2) {
      const long long j = nbr_checked(d, x, y, z, CX[a], CY[a], CZ[a]);
      if (j < 0) continue;
      if (in_gas_region(d.flag_dst[j] & TYPE_MASK)) uf_union(d.lab, (int)i, (int)j);
    }
  }
}

__global__ void __launch_bounds__(256) k_label_roots(Dev d) {
  if (!d.sc->label_run) return;
  FSLBM_GRID_STRIDE(i) {
    if (d.lab[i] < 0) continue;
    const int r = uf_find(d.lab, (int)i);
    d.lab[i] = r;
    const int s = d.bslot[i];
    atomicMin(&d.aux0[r], s);
    atomicMax(&d.aux1[r], s);
    atomicMin(&d.b_rmin[s], r);
    atomicMax(&d.b_rmax[s], r);
    if ((d.flag_dst[i] & TYPE_MASK) == T_INLET) atomicOr(&d.aux2[r], 1);
  }
}

// A component keeps its bubble if it holds exactly one bubble and that
// bubble lies in no other component; every other component is new.
__global__ void __launch_bounds__(256) k_label_decide(Dev d) {
  if (!d.sc->label_run) return;
  FSLBM_GRID_STRIDE(i) {
    if (d.lab[i] != (int)i) continue;
    const int s = d.aux0[i];
    const bool single = d.aux0[i] == d.aux1[i] && d.b_rmin[s] == (int)i && d.b_rmax[s] == (int)i;
    if (single) {
      d.b_kept[s] = 1;
    } else {
      const int k = atomicAdd(&d.sc->nnew, 1);
      if (k < d.max_bubbles) d.newroots[k] = (int)i;
      atomicOr(&d.aux2[i], 2);
    }
  }
}

// Single block: order the new components by their smallest cell index,
// give each the next fresh ID and a free slot, and fix the V* ratio of
// every old bubble.
__global__ void __launch_bounds__(1024) k_label_assign(Dev d) {
  if (!d.sc->label_run) return;
  Scalars *sc = d.sc;
  const int B = d.max_bubbles;
  const int nnew = sc->nnew;
  if (nnew > B) {
    if (threadIdx.x == 0) sc->err |= ERR_CAPACITY;
    return;
  }
  // rank sort of the new roots (distinct values) into newslot as scratch
  for (int k = threadIdx.x; k < nnew; k += blockDim.x) {
    const int r = d.newroots[k];
    int rank = 0;
    for (int j = 0; j < nnew; ++j) rank += d.newroots[j] < r;
    d.newslot[rank] = r;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nnew; k += blockDim.x) d.newroots[k] = d.newslot[k];
  __syncthreads();
  for (int k = threadIdx.x; k < nnew; k += blockDim.x) d.aux0[d.newroots[k]] = k;
  // V* per unit gas volume of every old bubble (per cell if V <= 0)
  for (int s = threadIdx.x; s < B; s += blockDim.x) {
    if (!d.b_live[s]) continue;
    const double v = d.b_vol[s];
    const long long nc = d.b_ngas[s] + d.b_niface[s];
    d.b_ratio[s] = v > 0.0 ? d.b_vstar[s] / v : -(d.b_vstar[s] / (double)(nc > 0 ? nc : 1));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int k = 0;
    for (int s = 0; s < B && k < nnew; ++s) {
      const bool stays = d.b_live[s] && d.b_kept[s];
      if (!stays) d.newslot[k++] = s;
    }
    if (k < nnew) sc->err |= ERR_CAPACITY;
    sc->nfree = k;
  }
}

// Per new component: gas volume V_K = sum (1 - phi) (gas and inlet cells
// count 1), V*_K = sum over its cells of (V*_b / V_b) times the cell's gas
// volume (= sum_b V*_b V(b in K) / V_b), cell counts and the inlet flag.
template <class P>
__global__ void __launch_bounds__(256) k_label_accumulate(Dev d) {
  using R = typename P::R;
  const Scalars *sc = d.sc;
  if (!sc->label_run || sc->nnew > d.max_bubbles || sc->nfree < sc->nnew) return;
  for (long long base = (long long)blockIdx.x * blockDim.x; base < d.N;
       base += (long long)gridDim.x * blockDim.x) {
    const long long i = base + threadIdx.x;
    int key = -1;
    long long v[NACC];
#pragma unroll
    for (int c = 0; c < NACC; ++c) v[c] = 0;
    if (i < d.N && d.lab[i] >= 0) {
      const int r = d.lab[i];
      if (d.aux2[r] & 2) {
        key = d.aux0[r];
        const uint8_t t = d.flag_dst[i] & TYPE_MASK;
        const double w = t == T_IFACE ? 1.0 - (double)((const R *)d.phi_dst)[i] : 1.0;
        const double ratio = d.b_ratio[d.bslot[i]];
        const double ws = ratio >= 0.0 ? ratio * w : -ratio;
        const ExTerm tw = ex_split(w), ts = ex_split(ws);
#pragma unroll
        for (int c = 0; c < EX_WORDS; ++c) {
          v[c] = tw.w[c];
          v[EX_WORDS + c] = ts.w[c];
        }
        v[2 * EX_WORDS] = 1;
        v[2 * EX_WORDS + 1] = (t == T_GAS || t == T_INLET) ? 1 : 0;
        v[2 * EX_WORDS + 2] = t == T_IFACE ? 1 : 0;
        v[2 * EX_WORDS + 3] = t == T_INLET ? 1 : 0;
      }
    }
    wave_add_by_key<NACC>(key, v, d.c_acc, 1, 0);
  }
}

// Single block: install the new bubbles, free the slots of replaced ones.
__global__ void __launch_bounds__(1024) k_label_finish(Dev d) {
  Scalars *sc = d.sc;
  if (!sc->label_run || sc->nnew > d.max_bubbles || sc->nfree < sc->nnew) return;
  const int nnew = sc->nnew;
  const int B = d.max_bubbles;
  for (int s = threadIdx.x; s < B; s += blockDim.x)
    if (d.b_live[s] && !d.b_kept[s]) d.b_live[s] = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < nnew; k += blockDim.x) {
    const unsigned long long *a = d.c_acc + (long long)k * NACC;
    const int s = d.newslot[k];
    d.b_id[s] = sc->next_id + k;
    long long wv[EX_WORDS], ws[EX_WORDS];
    for (int c = 0; c < EX_WORDS; ++c) {
      wv[c] = ll(a[c]);
      ws[c] = ll(a[EX_WORDS + c]);
    }
    d.b_flags[s] = ll(a[2 * EX_WORDS + 3]) > 0 ? 1 : 0;
    d.b_vol[s] = ex_value(wv);
    d.b_vstar[s] = ex_value(ws);
    d.b_ngas[s] = ll(a[2 * EX_WORDS + 1]);
    d.b_niface[s] = ll(a[2 * EX_WORDS + 2]);
    d.b_live[s] = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sc->next_id += nnew;
    if (nnew > 0) sc->n_topology += 1;
  }
}

__global__ void __launch_bounds__(256) k_label_rewrite(Dev d) {
  const Scalars *sc = d.sc;
  if (!sc->label_run || sc->nnew > d.max_bubbles || sc->nfree < sc->nnew) return;
  FSLBM_GRID_STRIDE(i) {
    const int r = d.lab[i];
    if (r >= 0 && (d.aux2[r] & 2)) d.bslot[i] = d.newslot[d.aux0[r]];
  }
}

// ------------------------------------------------------------- k_bubbles

// Single block: gas injection into inlet bubbles and the ideal-gas
// pressure p = p0 V* / max(V, 1e-2); closes the step.
__global__ void __launch_bounds__(1024) k_bubbles(Dev d) {
  __shared__ int live;
  if (threadIdx.x == 0) live = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < d.max_bubbles; s += blockDim.x) {
    if (!d.b_live[s]) continue;
    if (d.b_flags[s] & 1) d.b_vstar[s] += d.inject;
    const double v = d.b_vol[s] > 1e-2 ? d.b_vol[s] : 1e-2;
    d.b_p[s] = d.p0 * d.b_vstar[s] / v;
    atomicAdd(&live, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Scalars *sc = d.sc;
    sc->n_live = live;
    sc->label_run = 0;
    sc->step += 1;
    if (!isfinite(sc->total_mass)) sc->err |= ERR_NONFINITE;
  }
}

// ------------------------------------------------------- create / export

// Stored PDFs of f = f_eq(rho, u) on interface and liquid cells from FP64
// staging arrays rho[N], u[3N] (computed in double); the weights elsewhere.
template <class P>
__global__ void __launch_bounds__(256) k_init_feq(Dev d, const double *rho, const double *u) {
  using R = typename P::R;
  FSLBM_GRID_STRIDE(i) {
    const uint8_t t = d.flag_src[i] & TYPE_MASK;
    double fe[Q];
    if (t == T_IFACE || t == T_LIQ) {
      const double uu[3] = {u[i], u[d.N + i], u[2 * d.N + i]};
      feq_exact(rho[i], uu, fe);
    } else {
      for (int a = 0; a < Q; ++a) fe[a] = wgt(a);
    }
    for (int a = 0; a < Q; ++a) st<P>(d.f_src, a, d.N, i, (R)(P::EXACT ? fe[a] : fe[a] - wgt(a)));
  }
}

// One direction a of f from an FP64 staging array.
template <class P>
__global__ void __launch_bounds__(256) k_init_f(Dev d, const double *src, int a) {
  using R = typename P::R;
  FSLBM_GRID_STRIDE(i) st<P>(d.f_src, a, d.N, i, (R)(P::EXACT ? src[i] : src[i] - wgt(a)));
}

// Export one quantity as FP64: what = 0 phi, 1 mass (rho on liquid cells),
// 2 rho, 3..5 u, 6 + a f_a.
template <class P>
__global__ void __launch_bounds__(256) k_export(Dev d, double *out, int what) {
  using R = typename P::R;
  FSLBM_GRID_STRIDE(i) {
    const uint8_t t = d.flag_src[i] & TYPE_MASK;
    const bool fluid = t == T_IFACE || t == T_LIQ;
    double v = 0.0;
    if (what == 0) {
      v = (double)((const R *)d.phi_src)[i];
    } else if (what >= 6) {
      const double s = (double)ld<P>(d.f_src, what - 6, d.N, i);
      v = fluid ? (P::EXACT ? s : wgt(what - 6) + s) : 0.0;
    } else if (fluid) {
      if constexpr (P::EXACT) {
        R vv[Q];
        for (int a = 0; a < Q; ++a) vv[a] = ld<P>(d.f_src, a, d.N, i);
        R r, dr, uu[3];
        recover<P>(d, vv, r, dr, uu);
        if (what == 1) v = t == T_IFACE ? (double)((const R *)d.mass)[i] : (double)r;
        else if (what == 2) v = (double)r;
        else v = (double)uu[what - 3];
      } else {
        double s = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < Q; ++a) {
          const double h = (double)ld<P>(d.f_src, a, d.N, i);
          s += h;
          j[0] += CX[a] * h;
          j[1] += CY[a] * h;
          j[2] += CZ[a] * h;
        }
        const double r = 1.0 + s;
        if (what == 1) v = t == T_IFACE ? (double)((const R *)d.mass)[i] : r;
        else if (what == 2) v = r;
        else v = j[what - 3] / r - 0.5 * d.g[what - 3];
      }
    }
    out[i] = v;
  }
}

}  // namespace
}  // namespace fslbm
