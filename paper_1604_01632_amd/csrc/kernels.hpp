// HIP kernels of one free-surface lattice Boltzmann step with the enhanced
// bubble model (arXiv:1604.01632), templated on the storage precision.
//
// Step pipeline (one HIP stream, no host synchronisation):
//   k_bulk        liquid cells (dense grid): pull streaming with half-way
//                 bounce-back and collision (Sec. 2.1)
//   k_iface       interface cells (list): Youngs normal and height-function
//                 curvature, gas pressure p_V + 2 sigma kappa (Sec. 2.2),
//                 reconstruction of gas-side PDFs, mass exchange, collision,
//                 fill level; conversion candidates appended to a list
//   k_conv_types  new cell types (closed interface layer); new interface
//                 cells appended to a list (each once)
//   k_conv_init   initial values of the new interface cells
//   k_excess      excess mass of converted cells, bucket, topology trigger
//                 (in one launch with the tile counts of the next
//                 interface list)
//   k_list_*      next interface list in cell order: count, scan (in one
//                 launch with the labelled set of k_label_init), fill (in
//                 one launch with the unions of k_label_union)
//   k_gather      interface cells of t+1 pull excess mass; fill levels;
//                 per-bubble volume sums (Sec. 2.3) (in one launch with the
//                 roots of k_label_roots)
//   k_label_*     per-bubble volumes, bucket share and total mass (in one
//                 launch with k_label_assign, every step); union-find labelling
//                 of the gas region and the merge / split rules
//                 (Sec. 2.3.1, 2.3.2) - the labelling returns at once
//                 unless the trigger fired
//   k_bubbles     new bubbles of a labelling run, injection and ideal-gas
//                 pressure (Sec. 2.2); the list counters of the next step
#pragma once
#include <float.h>
#include <limits.h>

#include "device.hpp"

namespace fslbm {
// Kernels are local to each precision's translation unit.
namespace {

// Block of a kernel as seen by one domain: its index among the domain's
// blocks and their number.
struct Blk {
  int id, n;
};

// Chunk of a list walked by n blocks of `threads` lanes.  The dispatcher
// sends block b to XCD b mod 8; the first n chunks are permuted so that the
// blocks of one XCD take consecutive chunks, and neighbouring interface
// cells (whose stencils share cache lines) meet in that XCD's L2.  Chunks
// beyond the first n (lists longer than the grid) keep the identity order.
__device__ __forceinline__ int xcd_chunk(int c, int m) {
  if (c >= m) return c;
  const int q = m >> 3, r = m & 7, x = c & 7;
  return x * q + (x < r ? x : r) + (c >> 3);
}

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
// Random 32 bits for a (cell, salt) pair: lowbias32 finaliser
// (xorshift-multiply, C. Wellons) of the cell mixed with the salt.
__device__ __forceinline__ uint32_t store_key(long long i, uint32_t salt) {
  uint32_t x = (uint32_t)i ^ (salt * 0x9E3779B9u);
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// x rounded to one of its two neighbouring half values, away from zero
// with probability (|x| - lo) / (hi - lo): unbiased in expectation.  With s
// the half spacing at |x| (2^(e-10) for exponent e, at least 2^-24), the
// result is floor(|x| / s + u) s for u uniform in [0, 1): the scalings are
// exact powers of two and the result is a half value, so the conversion is
// exact.
__device__ __forceinline__ _Float16 half_stochastic(float x, uint32_t r) {
  const uint32_t ab = __float_as_uint(x) & 0x7fffffffu;
  int e = (int)(ab >> 23) - 127;
  e = e < -14 ? -14 : e;
  const float s = __uint_as_float((uint32_t)(e - 10 + 127) << 23);
  const float inv = __uint_as_float((uint32_t)(10 - e + 127) << 23);
  const float u = (float)(r >> 8) * 0x1p-24f;
  const float y = floorf(__uint_as_float(ab) * inv + u) * s;
  return (_Float16)copysignf(y, x);
}

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
  using S = _Float16;  // see to_store
  using R = float;
  static constexpr bool EXACT = false;
};

// The stored values of one cell's new populations.  FP64 and FP32 store
// them as computed.  FP16 rounds the moving populations to nearest and
// gives their rounding residues (exact in float) to the rest population,
// which is rounded stochastically (key: random bits of the cell and step).
// Rounding every deviation to nearest would add the same error to every
// cell of a near-uniform region, step after step, and drift the mass; this
// way a stored cell keeps its deviation sum up to one unbiased rounding.
template <class P>
__device__ __forceinline__ void to_store(const typename P::R (&f)[Q], typename P::S (&out)[Q],
                                         uint32_t key) {
  using S = typename P::S;
  if constexpr (sizeof(S) == 2) {
    float res = 0.0f;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      out[a] = (S)f[a];
      res += f[a] - (float)out[a];
    }
    out[0] = half_stochastic(f[0] + res, key);
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) out[a] = (S)f[a];
  }
}

// Stored value of direction a at cell i: f (FP64) or h = f - w (others).
template <class P>
__device__ __forceinline__ typename P::R ld(const void *f, int a, long long N, long long i) {
  return (typename P::R)((const typename P::S *)f)[a * N + i];
}

// A stored value (exact conversion, or the value of to_store).
template <class P>
__device__ __forceinline__ void st(void *f, int a, long long N, long long i, typename P::S v) {
  ((typename P::S *)f)[a * N + i] = v;
}

// Post-collision populations of the interface cells, by list slot: the Q
// stored values of slot k are contiguous (padded to a multiple of 16
// bytes), so a cell costs one or two cache lines wherever its slot lies,
// and moves with 16-byte accesses.
template <class P>
struct IfRow {
  static constexpr int BYTES = (Q * (int)sizeof(typename P::S) + 15) / 16 * 16;
  static constexpr int WORDS = BYTES / 16;
  static constexpr int SLOTS = BYTES / (int)sizeof(typename P::S);
};

template <class P>
__device__ __forceinline__ void if_load(const void *base, long long k, typename P::R (&f)[Q]) {
  using S = typename P::S;
  uint4 w[IfRow<P>::WORDS];
  const uint4 *p = (const uint4 *)((const char *)base + k * IfRow<P>::BYTES);
#pragma unroll
  for (int q = 0; q < IfRow<P>::WORDS; ++q) w[q] = p[q];
  S v[IfRow<P>::SLOTS];
  __builtin_memcpy(v, w, sizeof w);
#pragma unroll
  for (int a = 0; a < Q; ++a) f[a] = (typename P::R)v[a];
}

template <class P>
__device__ __forceinline__ void if_store(void *base, long long k, const typename P::S (&f)[Q]) {
  using S = typename P::S;
  S v[IfRow<P>::SLOTS];
#pragma unroll
  for (int a = 0; a < IfRow<P>::SLOTS; ++a) v[a] = a < Q ? f[a] : (S)0;
  uint4 w[IfRow<P>::WORDS];
  __builtin_memcpy(w, v, sizeof w);
  uint4 *p = (uint4 *)((char *)base + k * IfRow<P>::BYTES);
#pragma unroll
  for (int q = 0; q < IfRow<P>::WORDS; ++q) p[q] = w[q];
}

// Streaming store of a stored value (non-temporal; half values by their
// 16-bit pattern).
template <class P>
__device__ __forceinline__ void st_stream(void *f, int a, long long N, long long i,
                                          typename P::S sv) {
  using S = typename P::S;
  S *p = (S *)f + a * N + i;
  if constexpr (sizeof(S) == 2) {
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, sv), (unsigned short *)p);
  } else {
    __builtin_nontemporal_store(sv, p);
  }
}

// Streaming load of a stored value (non-temporal: the old lattice is read
// once per step).
template <class P>
__device__ __forceinline__ typename P::R ld_stream(const void *f, int a, long long N, long long i) {
  using S = typename P::S;
  const S *p = (const S *)f + a * N + i;
  if constexpr (sizeof(S) == 2) {
    return (typename P::R)__builtin_bit_cast(S, __builtin_nontemporal_load((const unsigned short *)p));
  } else {
    return (typename P::R)__builtin_nontemporal_load(p);
  }
}

// ------------------------------------------------------------- geometry

// Periodic wrap by adding or subtracting the extent (no integer division;
// offsets are at most a few cells).
__device__ __forceinline__ int wrap_axis(int c, int n, int per) {
  if (!per) return c;
  while (c < 0) c += n;
  while (c >= n) c -= n;
  return c;
}

// Periodic wrap of a coordinate at most one cell outside [0, n).
__device__ __forceinline__ int wrap1(int c, int n, int per) {
  if (!per) return c;
  return c < 0 ? c + n : (c >= n ? c - n : c);
}

// Linear index; the number of cells is below 2^31 (checked at creation).
__device__ __forceinline__ long long cidx(const Dev &d, int x, int y, int z) {
  return (long long)(x + d.nx * (y + d.ny * z));
}

// Neighbour of an interior cell (fluid and gas cells are interior on
// non-periodic axes, whose face layers are walls or inlets).
__device__ __forceinline__ long long nbr(const Dev &d, int x, int y, int z, int dx, int dy,
                                         int dz) {
  return cidx(d, wrap1(x + dx, d.nx, d.per[0]), wrap1(y + dy, d.ny, d.per[1]),
              wrap1(z + dz, d.nz, d.per[2]));
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

__device__ __forceinline__ void coords(const Dev &d, long long i, int &x, int &y, int &z) {
  const unsigned u = (unsigned)i, nx = (unsigned)d.nx, ny = (unsigned)d.ny;
  const unsigned r = u / nx;
  x = (int)(u - r * nx);
  z = (int)(r / ny);
  y = (int)(r - (unsigned)z * ny);
}

// Wrapped coordinates of the 27 cells around (x, y, z) (interior cells).
struct Nb3 {
  int xs[3], ys[3], zs[3];
  __device__ __forceinline__ Nb3(const Dev &d, int x, int y, int z) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xs[k] = wrap1(x + k - 1, d.nx, d.per[0]);
      ys[k] = wrap1(y + k - 1, d.ny, d.per[1]);
      zs[k] = wrap1(z + k - 1, d.nz, d.per[2]);
    }
  }
  __device__ __forceinline__ long long at(const Dev &d, int dx, int dy, int dz) const {
    return (long long)(xs[dx + 1] + d.nx * (ys[dy + 1] + d.ny * zs[dz + 1]));
  }
};

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
    R sum = (R)0;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const R cu = (R)CX[a] * u[0] + (R)CY[a] * u[1] + (R)CZ[a] * u[2];
      out[a] = (R)wgt(a) * (drho + rho * ((R)3 * cu + (R)4.5 * cu * cu - uu15));
      sum += out[a];
    }
    out[0] = drho - sum;  // the deviations sum to rho - 1 (see collide)
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
    // The rest population takes what the moving ones leave of the
    // equilibrium (sum = rho - 1) and of the force term (sum = 0): the float
    // weights do not sum to one, and that bias times rho - 1 (of one sign
    // in a pressurised liquid) would otherwise drift the mass every step.
    R sum_eq = (R)0, sum_s = (R)0;
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
      sum_eq += eq_even;
      sum_s += s_even;
    }
    {
      const R eq0 = dr - (R)2 * sum_eq;
      const R s0 = (R)-2 * sum_s;
      f[0] = f[0] - wp * (f[0] - eq0) + kp * s0;
    }
    rho_o = rho;
    u_o[0] = ux;
    u_o[1] = uy;
    u_o[2] = uz;
  }
}

// -------------------------------------------------- interface geometry

// Parker-Youngs gradient of the fill level (weights 4/2/1 for face / edge /
// corner offsets, pointing from gas into liquid) and the height-function
// curvature are computed by k_geom from the cell's 3x3x3 neighbourhood.

// Fill-level samples at offsets -3..3 per axis from a cell: plain
// coordinates (wrapped on periodic axes) and their mirror images across the
// wall planes on non-periodic axes; a sample on a wall cell or outside the
// box takes the mirrored cell (the rule of phi_sample).
template <class R>
struct PhiWin {
  int xp[7], yp[7], zp[7], xm[7], ym[7], zm[7];
  // bit k: offset k - 3 lies on a face layer of a non-periodic axis or
  // beyond it (interior samples can never be wall cells: walls form the
  // face layers only)
  uint32_t xf = 0, yf = 0, zf = 0;
  __device__ __forceinline__ PhiWin(const Dev &d, int x, int y, int z) {
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      xp[k] = wrap_axis(x + k - 3, d.nx, d.per[0]);
      yp[k] = wrap_axis(y + k - 3, d.ny, d.per[1]);
      zp[k] = wrap_axis(z + k - 3, d.nz, d.per[2]);
      xm[k] = mirror(xp[k], d.nx, d.per[0]);
      ym[k] = mirror(yp[k], d.ny, d.per[1]);
      zm[k] = mirror(zp[k], d.nz, d.per[2]);
      xf |= (uint32_t)(!d.per[0] && (xp[k] <= 0 || xp[k] >= d.nx - 1)) << k;
      yf |= (uint32_t)(!d.per[1] && (yp[k] <= 0 || yp[k] >= d.ny - 1)) << k;
      zf |= (uint32_t)(!d.per[2] && (zp[k] <= 0 || zp[k] >= d.nz - 1)) << k;
    }
  }
  __device__ __forceinline__ static int mirror(int c, int n, int per) {
    if (per) return c;
    if (c <= 0) return 1 - c;
    if (c >= n - 1) return 2 * n - 3 - c;
    return c;
  }
  __device__ __forceinline__ R get(const Dev &d, const R *phi, int ox, int oy, int oz) const {
    const int cx = xp[ox + 3], cy = yp[oy + 3], cz = zp[oz + 3];
    if (!d.has_walls) return phi[cx + d.nx * (cy + d.ny * cz)];
    // an interior sample is an ordinary cell: no flag to look at
    if (!(((xf >> (ox + 3)) | (yf >> (oy + 3)) | (zf >> (oz + 3))) & 1u))
      return phi[cx + d.nx * (cy + d.ny * cz)];
    if (cx >= 0 && cx < d.nx && cy >= 0 && cy < d.ny && cz >= 0 && cz < d.nz) {
      const int i = cx + d.nx * (cy + d.ny * cz);
      if ((d.flag_src[i] & TYPE_MASK) != T_WALL) return phi[i];
    }
    return phi[xm[ox + 3] + d.nx * (ym[oy + 3] + d.ny * zm[oz + 3])];
  }
};

// Height-function curvature along axis DD with the 3x3x3 neighbourhood of
// the cell already in registers (B[dz][dy][dx]); same sums, same order.
template <int DD, class R>
__device__ __forceinline__ R height_curvature_cached(const Dev &d, const R *phi,
                                                     const PhiWin<R> &W, const R (&B)[3][3][3],
                                                     int x, bool rows) {
  R H[3][3];
#pragma unroll
  for (int a = -1; a <= 1; ++a)
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
      // along x with plain rows: x-3, x-2 and x+2, x+3 from two loads
      R ext[4];
      if constexpr (DD == 0 && sizeof(R) == 4) {
        if (rows) {
          const R *rp = phi + (long long)d.nx * (W.yp[a + 3] + (long long)d.ny * W.zp[b + 3]) + x;
          float4 lo;
          float2 hi;
          __builtin_memcpy(&lo, rp - 3, 16);
          __builtin_memcpy(&hi, rp + 2, 8);
          ext[0] = lo.x;
          ext[1] = lo.y;
          ext[2] = hi.x;
          ext[3] = hi.y;
        }
      }
      R s = (R)0;
#pragma unroll
      for (int k = -3; k <= 3; ++k) {
        const int ox = DD == 0 ? k : a;
        const int oy = DD == 0 ? a : (DD == 1 ? k : b);
        const int oz = DD == 2 ? k : b;
        R v;
        if (k >= -1 && k <= 1) v = B[oz + 1][oy + 1][ox + 1];
        else if (DD == 0 && sizeof(R) == 4 && rows) v = ext[k < 0 ? k + 3 : k];
        else v = W.get(d, phi, ox, oy, oz);
        s += v;
      }
      // wetting: a column whose footprint lies in a wall takes the
      // mirrored column's liquid height plus cot(theta) per wall axis
      // crossed (the liquid height of a column parallel to the wall grows
      // by cot(theta) per cell towards a wall met at the static contact
      // angle theta, measured in the liquid)
      if (d.wall_cot != 0.0) {
        const uint32_t f1 = DD == 0 ? W.yf : W.xf;
        const uint32_t f2 = DD == 2 ? W.yf : W.zf;
        const int m = (int)((f1 >> (a + 3)) & 1u) + (int)((f2 >> (b + 3)) & 1u);
        if (m) {
          const int ox = DD == 0 ? 0 : a;
          const int oy = DD == 0 ? a : (DD == 1 ? 0 : b);
          const int oz = DD == 2 ? 0 : b;
          const int cx = W.xp[ox + 3], cy = W.yp[oy + 3], cz = W.zp[oz + 3];
          const bool in = cx >= 0 && cx < d.nx && cy >= 0 && cy < d.ny && cz >= 0 && cz < d.nz;
          if (!in || (d.flag_src[cx + d.nx * (cy + d.ny * cz)] & TYPE_MASK) == T_WALL)
            s += (R)m * (R)d.wall_cot;
        }
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

// Interface geometry of the listed interface cells: Youngs normal and
// height-function curvature from the fill levels of time t, gas density
// from p_V + 2 sigma kappa (Sec. 2.2) and the directions to reconstruct
// (moving from the gas side into the liquid beyond the tie band).  Results
// are stored by list position.
template <class P>
struct K_geom {
  static constexpr int THREADS = 256;
  static constexpr int MIN_WAVES = P::EXACT ? 1 : 4;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  using R = typename P::R;
  const R *phi = (const R *)d.phi_src;
  const int n = d.sc->n_il_src;
  const int nch = (n + THREADS - 1) / THREADS, m = nch < bk.n ? nch : bk.n;
  for (int c = bk.id; c < nch; c += bk.n) {
    const int k = xcd_chunk(c, m) * THREADS + (int)threadIdx.x;
    if (k >= n) continue;
    const long long i = d.ilist_src[k];
    // the bubble pressure in the same rounds as the fill levels
    const int slot = d.bslot[i];
    const double bp = d.b_p[slot];
    int x, y, z;
    coords(d, i, x, y, z);
    const PhiWin<R> W(d, x, y, z);
    R B[3][3][3];
    // plain rows of 4-byte levels: each x-row of the block is one 16-byte
    // load where every sample of those rows is an ordinary cell - x-3..x+3
    // without a periodic wrap, and off the wall layers (walls only form the
    // faces of non-periodic axes) for x-3..x+3 and the rows y-1..y+1,
    // z-1..z+1
    const bool xin = d.per[0] ? (x >= 3 && x + 3 < d.nx) : (x >= 4 && x + 4 < d.nx);
    const bool yin = d.per[1] || (y >= 2 && y + 2 < d.ny);
    const bool zin = d.per[2] || (z >= 2 && z + 2 < d.nz);
    const bool rows = sizeof(R) == 4 && xin && yin && zin;
    if (rows) {
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
          const R *rp = phi + (long long)d.nx * (W.yp[dy + 3] + (long long)d.ny * W.zp[dz + 3]) + x;
          float4 v;
          __builtin_memcpy(&v, rp - 1, 16);
          B[dz + 1][dy + 1][0] = v.x;
          B[dz + 1][dy + 1][1] = v.y;
          B[dz + 1][dy + 1][2] = v.z;
        }
    } else {
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
          for (int dx = -1; dx <= 1; ++dx) B[dz + 1][dy + 1][dx + 1] = W.get(d, phi, dx, dy, dz);
    }
    R nv[3] = {(R)0, (R)0, (R)0};
#pragma unroll
    for (int p = -1; p <= 1; ++p)
#pragma unroll
      for (int q = -1; q <= 1; ++q) {
        const R w = (R)((p == 0 ? 2 : 1) * (q == 0 ? 2 : 1));
        nv[0] += w * (B[q + 1][p + 1][2] - B[q + 1][p + 1][0]);
        nv[1] += w * (B[q + 1][2][p + 1] - B[q + 1][0][p + 1]);
        nv[2] += w * (B[2][q + 1][p + 1] - B[0][q + 1][p + 1]);
      }
    // curvature: dominant axis, ties averaged in the order x, y, z
    const R an[3] = {fabs(nv[0]), fabs(nv[1]), fabs(nv[2])};
    R m = an[0];
    if (an[1] > m) m = an[1];
    if (an[2] > m) m = an[2];
    R kappa = (R)0;
    if (m != (R)0) {
      const R thr = m - (R)TIE_REL * m;
      R sum = (R)0;
      int cnt = 0;
      if (an[0] >= thr) {
        sum += height_curvature_cached<0>(d, phi, W, B, x, rows);
        ++cnt;
      }
      if (an[1] >= thr) {
        sum += height_curvature_cached<1>(d, phi, W, B, x, rows);
        ++cnt;
      }
      if (an[2] >= thr) {
        sum += height_curvature_cached<2>(d, phi, W, B, x, rows);
        ++cnt;
      }
      kappa = sum / (R)cnt;
    }
    R g;
    if constexpr (P::EXACT) {
      const R p_gas = (R)bp + (R)2.0 * (R)d.sigma * kappa;
      g = (R)3.0 * p_gas;  // rho_gas, p = rho cs^2
    } else {
      g = (R)(3.0 * bp - 1.0) + (R)6 * (R)d.sigma * kappa;  // rho_gas - 1
    }
    const R nn = an[0] + an[1] + an[2];
    uint32_t mask = 0;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      const R cn = CX[a] * nv[0] + CY[a] * nv[1] + CZ[a] * nv[2];
      if (cn > (R)TIE_REL * nn) mask |= 1u << a;
    }
    ((R *)d.gasv)[k] = g;
    d.nmask[k] = mask;
    if (d.split_trigger == 1) {
      // unit normal for the split trigger by anti-parallel normals
      const float len = (float)sqrt((double)(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]));
      const float inv = len > 0.0f ? 1.0f / len : 0.0f;
      const long long C = d.icap;
      d.nrm[k] = (float)nv[0] * inv;
      d.nrm[C + k] = (float)nv[1] * inv;
      d.nrm[2 * C + k] = (float)nv[2] * inv;
    }
  }
}
};

// Sum of the gas-side equilibria of direction a and its opposite, in the
// stored representation: f_eq,a + f_eq,abar (FP64, each term in the
// reference operation order) or (f_eq,a - w_a) + (f_eq,abar - w_abar).
template <class P>
__device__ __forceinline__ typename P::R gas_pair(typename P::R rho, typename P::R drho,
                                                  const typename P::R *u, int a) {
  using R = typename P::R;
  if constexpr (P::EXACT) {
    const double cs2 = 1.0 / 3.0;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const int b = opp(a);
    const double cua = CX[a] * u[0] + CY[a] * u[1] + CZ[a] * u[2];
    const double cub = CX[b] * u[0] + CY[b] * u[1] + CZ[b] * u[2];
    const double fa = rho * wgt(a) * (1.0 + cua / cs2 + (cua * cua) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    const double fb = rho * wgt(b) * (1.0 + cub / cs2 + (cub * cub) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    return fa + fb;
  } else {
    const R cu = (R)CX[a] * u[0] + (R)CY[a] * u[1] + (R)CZ[a] * u[2];
    const R uu15 = (R)1.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    return (R)2 * (R)wgt(a) * (drho + rho * ((R)4.5 * cu * cu - uu15));
  }
}

// Candidate bits of a cell's flag byte after the interface kernel: filled
// (becomes liquid) and capped (next to an inlet, over-full: stays interface
// and passes its mass above m = rho on).
__device__ __forceinline__ bool cand_filled(uint8_t f) { return (f & CAND_F) && !(f & NEAR_INLET); }
__device__ __forceinline__ bool cand_capped(uint8_t f) { return (f & CAND_F) && (f & NEAR_INLET); }


// A cell is claimed once per step: one byte of the mark field per cell,
// its low bit set by the first caller.
__device__ __forceinline__ unsigned claim_bit(long long j) { return 1u << (8 * (unsigned)(j & 3)); }

// Sets the claim bit of cell j and returns its word as it was before: the
// claim is won when claim_bit(j) was clear in it.
__device__ __forceinline__ unsigned claim_cell(const Dev &d, long long j) {
  return atomicOr(&d.mark[j >> 2], claim_bit(j));
}

__device__ __forceinline__ void release_cell(const Dev &d, long long j) {
  atomicAnd(&d.mark[j >> 2], ~claim_bit(j));
}

// ---------------------------------------------------------------- k_bulk

// Every cell of a row: liquid cells pull (half-way bounce-back from walls)
// and collide; interface cells take the post-collision values and flag
// that k_iface left at their list slot; gas, wall and inlet cells store
// zeros (their PDFs are undefined).  Every row of the new lattice and flag
// field is thus written whole, in one coalesced pass.
// Stream-collide blocks take consecutive chunks of blockDim.x cells in
// hardware block order.  The dispatcher deals consecutive blocks to the 8
// XCDs round-robin, so all XCDs work on the same few planes at a time and
// share the neighbour planes through the Infinity Cache; on the 256^3 thread
// workload this order measured 480 us per launch against 488 us for
// y-tiled per-XCD ranges and 510 us for contiguous per-XCD ranges.

template <class P, bool WITH_MASS, int TB>
struct K_bulk {
  static constexpr int THREADS = TB;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  using R = typename P::R;
  const int nx = d.nx, ny = d.ny;
  // coordinates: the wave's first cell in scalar arithmetic, then each lane
  // steps over the row (and plane) ends it crosses
  const int lane = (int)threadIdx.x & 63;
  const int w0 = __builtin_amdgcn_readfirstlane(bk.id * (int)blockDim.x +
                                                ((int)threadIdx.x - lane));
  const int r0 = w0 / nx;
  int x = w0 - r0 * nx + lane, y = r0 % ny, z = r0 / ny;
  while (x >= nx) {
    x -= nx;
    if (++y == ny) {
      y = 0;
      ++z;
    }
  }
  Fx mass;
  bool bad = false;  // a non-finite density
  const bool in = (long long)w0 + lane < d.N;
  const long long i = in ? (long long)w0 + lane : 0;
  const uint8_t fl = in ? d.flag_src[i] : (uint8_t)T_GAS;
  const uint8_t t = fl & TYPE_MASK;
  // a wave with no liquid or interface cell leaves its rows untouched
  const bool fluid_wave = __ballot(in && (t == T_LIQ || t == T_IFACE)) != 0ull;
  if (in && fluid_wave) {
    R f[Q];
    uint8_t nfl = fl & (STATIC_BITS | TYPE_MASK);
    if (t == T_LIQ) {
      // source x - c_a of direction a: a fixed offset from i, corrected by
      // the extent where a periodic axis wraps (only on the box faces; on
      // other axes fluid cells never touch the faces)
      const int nxy = nx * ny, NN = (int)d.N;
      const int sxm = (d.per[0] && x == 0) ? nx : 0, sxp = (d.per[0] && x == nx - 1) ? -nx : 0;
      const int sym = (d.per[1] && y == 0) ? nxy : 0, syp = (d.per[1] && y == ny - 1) ? -nxy : 0;
      const int szm = (d.per[2] && z == 0) ? NN : 0, szp = (d.per[2] && z == d.nz - 1) ? -NN : 0;
      auto src = [&](int a) -> long long {
        int v = (int)i - (CX[a] + nx * (CY[a] + ny * CZ[a]));
        v += CX[a] == 1 ? sxm : (CX[a] == -1 ? sxp : 0);
        v += CY[a] == 1 ? sym : (CY[a] == -1 ? syp : 0);
        v += CZ[a] == 1 ? szm : (CZ[a] == -1 ? szp : 0);
        return v;
      };
      // every pulled value is read once in the step: streaming loads keep
      // the old lattice out of the caches as well
      if (!(fl & NEAR_WALL)) {
#pragma unroll
        for (int a = 0; a < Q; ++a) f[a] = ld_stream<P>(d.f_src, a, d.N, src(a));
      } else {
        uint8_t ts[Q];
        R own[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const long long s = src(a);
          ts[a] = d.flag_src[s] & TYPE_MASK;
          f[a] = ld_stream<P>(d.f_src, a, d.N, s);
          own[a] = ld<P>(d.f_src, a, d.N, i);
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) f[a] = (ts[a] == T_WALL) ? own[opp(a)] : f[a];
      }
      R rho, u[3];
      collide<P>(d, f, rho, u);
      if (WITH_MASS) mass.add((double)rho, FX_VOL);
      bad = !isfinite(rho);
    } else if (t == T_IFACE) {
      const int k = d.islot[i];
      if_load<P>(d.f_if, k, f);
      nfl = d.nflag[k];
    } else {
#pragma unroll
      for (int a = 0; a < Q; ++a) f[a] = (R)0;
    }
    // stored values: the collided populations of a liquid cell through
    // to_store, exact copies (interface rows, zeros) otherwise
    typename P::S sv[Q];
    if (t == T_LIQ) {
      to_store<P>(f, sv, store_key(i, (uint32_t)d.sc->step));
    } else {
#pragma unroll
      for (int a = 0; a < Q; ++a) sv[a] = (typename P::S)f[a];
    }
    // the new lattice is written once and read only in the next step:
    // non-temporal stores keep it from evicting the interface data that the
    // following kernels read from the caches
#pragma unroll
    for (int a = 0; a < Q; ++a) st_stream<P>(d.f_dst, a, d.N, i, sv[a]);
    d.flag_dst[i] = nfl;
  } else if (in) {
    d.flag_dst[i] = fl & (STATIC_BITS | TYPE_MASK);
  }
  if (__ballot(bad) && lane == __ffsll((long long)__ballot(bad)) - 1)
    atomicOr(&d.sc->err, ERR_NONFINITE);
  if (WITH_MASS) block_fx_add(mass, d.mass_acc, (int)(bk.id % SUB_MASS));
}
};

// --------------------------------------------------------------- k_iface

// One interface cell: geometry, gas-side equilibrium, pull streaming with
// bounce-back and reconstruction, mass exchange (summed in the order of the
// neighbour directions), collision, new fill level and conversion
// candidates.  Returns the new mass.
template <class P>
__device__ __forceinline__ double iface_cell(const Dev &d, int x, int y, int z, long long i,
                                             int k, uint8_t fl, uint8_t &nf_out) {
  using R = typename P::R;
  const R *phi = (const R *)d.phi_src;
  const long long N = d.N;
  const R g = ((const R *)d.gasv)[k];
  const uint32_t mask = d.nmask[k];
  const R rho_gas = P::EXACT ? g : (R)1 + g;
  const R drho_gas = P::EXACT ? g - (R)1 : g;

  // the cell's own post-collision values: from its row of the previous
  // step if it was an interface cell then (the lattice holds a copy of
  // that row: one or two cache lines instead of one per direction), else
  // from the lattice.  The destination flags still hold the types of t-1.
  R fs[Q];
  if (d.sc->if_prev && (d.flag_dst[i] & TYPE_MASK) == T_IFACE) {
    if_load<P>(d.f_if_prev, d.islot_alt[i], fs);
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) fs[a] = ld<P>(d.f_src, a, N, i);
  }
  R ub[3];
  {
    R r, dr;
    recover<P>(d, fs, r, dr, ub);
  }

  // al: direction towards the neighbour y = x + c_al, which is the source of
  // the pulled direction a = opp(al)
  const Nb3 nb(d, x, y, z);
  R fin[Q];
  fin[0] = fs[0];
  R dm = (R)0;
  bool has_gas = false, has_liq = false;
  const R phi_x = phi[i];
  // the neighbour types first; then, in three groups of six, only the
  // values a neighbour contributes are fetched (streamed value of liquid
  // and interface neighbours, fill level of interface neighbours; gas,
  // inlet and wall neighbours contribute reconstructed or bounced values)
  // and the rules are applied with selects; the mass exchange is summed in
  // direction order
  uint8_t tn[Q];
#pragma unroll
  for (int al = 1; al < Q; ++al) tn[al] = d.flag_src[nb.at(d, CX[al], CY[al], CZ[al])] & TYPE_MASK;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    R raw[6], phn[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int al = 1 + 6 * g + k;
      const uint8_t t = tn[al];
      raw[k] = (R)0;
      phn[k] = (R)0;
      if (t == T_LIQ || t == T_IFACE) {
        const long long s = nb.at(d, CX[al], CY[al], CZ[al]);
        raw[k] = ld<P>(d.f_src, opp(al), N, s);
        if (t == T_IFACE) phn[k] = phi[s];
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int al = 1 + 6 * g + k;
      const int a = opp(al);
      const R recon = gas_pair<P>(rho_gas, drho_gas, ub, a) - fs[al];
      const uint8_t t = tn[al];
      const bool gas_src = t == T_GAS || t == T_INLET;
      const bool fluid_src = t == T_LIQ || t == T_IFACE;
      has_gas = has_gas || gas_src;
      has_liq = has_liq || t == T_LIQ;
      R v = ((mask >> a) & 1u) ? recon : raw[k];
      v = gas_src ? recon : v;
      v = (t == T_WALL) ? fs[al] : v;
      fin[a] = v;
      // mass exchange: liquid 1, interface mean fill level, others 0
      // (adding 0 * diff leaves the sum unchanged)
      const R diff = fluid_src ? raw[k] - fs[al] : (R)0;
      const R w = (t == T_IFACE) ? (R)0.5 * (phi_x + phn[k]) : (R)0;
      dm += (t == T_LIQ) ? diff : w * diff;
    }
  }
  const R m_new = ((R *)d.mass)[i] + dm + (R)d.sc->share;

  R rho, u[3];
  collide<P>(d, fin, rho, u);
  {
    typename P::S sv[Q];
    to_store<P>(fin, sv, store_key(i, (uint32_t)d.sc->step));
    if_store<P>(d.f_if, k, sv);
  }
  const R phi_new = m_new / rho;
  ((R *)d.mass)[i] = m_new;
  ((R *)d.rhoI)[i] = rho;
  ((R *)d.phi_dst)[i] = phi_new;
  // conversion candidates: fill level beyond the thresholds, or the cell
  // no longer separates liquid from gas (no gas / inlet neighbour: filled;
  // no liquid neighbour: emptied).  A cell next to an inlet is never
  // filled: there CAND_F means capped (above 1 + eps, it passes the mass
  // above m = rho on as excess and stays interface)
  uint8_t nf = fl & (STATIC_BITS | TYPE_MASK);
  if (!d.freeze) {
    if (phi_new > (R)1 + (R)d.eps || (!has_gas && !(fl & NEAR_INLET))) nf |= CAND_F;
    if (phi_new < -(R)d.eps || !has_liq) nf |= CAND_E;
  }
  if (!isfinite(m_new) || !isfinite(rho)) atomicOr(&d.sc->err, ERR_NONFINITE);
  d.nflag[k] = nf;
  nf_out = nf;
  return (double)m_new;
}

// Appends the lanes with pred set to a list; returns each such lane's slot,
// -1 for the others.  Every lane of the wave must call it.
__device__ __forceinline__ int wave_append(bool pred, int *counter) {
  const unsigned long long m = __ballot(pred);
  if (!m) return -1;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
  base = __shfl(base, leader, 64);
  return pred ? base + (int)__popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// The same with one atomic for the whole block: the appends of all waves
// serialise on the one counter, which costs more than the block's barriers
// once thousands of waves append to it.  Every thread of the block must
// call it.
__device__ __forceinline__ int block_append(bool pred, int *counter) {
  __shared__ int bw[16];
  __shared__ int bbase;
  const unsigned long long m = __ballot(pred);
  const int lane = __lane_id(), w = (int)threadIdx.x >> 6, nw = ((int)blockDim.x + 63) >> 6;
  if (lane == 0) bw[w] = (int)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < nw; ++k) t += bw[k];
    bbase = t ? atomicAdd(counter, t) : 0;
  }
  __syncthreads();
  int pos = bbase + (int)__popcll(m & ((1ull << lane) - 1ull));
  for (int k = 0; k < w; ++k) pos += bw[k];
  __syncthreads();  // bw and bbase are taken by the next call
  return pred ? pos : -1;
}

// Interface cells of time t (list), one per thread; conversion candidates
// are appended to the candidate list, with one atomic per block
// (BLOCK_APPEND) or per wave.  The list of a step is about one round of
// resident waves, so the FP32/FP16 kernels are held to three waves per SIMD
// (the FP64 one would spill).
template <class P, bool WITH_MASS, bool BLOCK_APPEND>
struct K_iface {
  static constexpr int THREADS = 256;
  static constexpr int MIN_WAVES = P::EXACT ? 1 : 3;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  Fx mass;
  const int n = d.sc->n_il_src;
  const int nch = (n + THREADS - 1) / THREADS, m = nch < bk.n ? nch : bk.n;
  for (int c = bk.id; c < nch; c += bk.n) {
    const int k = xcd_chunk(c, m) * THREADS + (int)threadIdx.x;
    bool cand = false;
    long long i = 0;
    if (k < n) {
      i = d.ilist_src[k];
      int x, y, z;
      coords(d, i, x, y, z);
      uint8_t nf;
      const double m = iface_cell<P>(d, x, y, z, i, k, d.flag_src[i], nf);
      if (WITH_MASS) mass.add(m, FX_VOL);
      cand = (nf & (CAND_F | CAND_E)) != 0;
    }
    // at most one entry per cell and step (the counter is reset at the
    // end of the step); the bound only guards the list
    const int pos = BLOCK_APPEND ? block_append(cand, &d.sc->n_cand)
                                 : wave_append(cand, &d.sc->n_cand);
    if (cand) {
      if (pos < (int)d.N) d.clist[pos] = (int)i;
      else atomicOr(&d.sc->err, ERR_RANGE);
    }
  }
  if (WITH_MASS) block_fx_add(mass, d.mass_acc, bk.id % SUB_MASS);
}
};

// ------------------------------------------------------------- conversions

// Candidates: filled cells -> liquid; emptied cells without a filled
// neighbour -> gas.  Gas neighbours of filled cells and liquid neighbours
// of emptied cells become interface (each listed once).  Every rule reads
// the candidate bits and the types of time t (phase-synchronous).
template <class P>
struct K_conv_types {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  const int n = d.sc->n_cand;
  for (int base = bk.id * blockDim.x; base < n; base += bk.n * blockDim.x) {
    const int k = base + threadIdx.x;
    bool F = false, E = false;
    int x = 0, y = 0, z = 0;
    // the cell's flag and both flags of its neighbours in one batch.  A
    // neighbour's candidate bits do not change here; the flag of t+1 of a
    // gas or liquid neighbour changes only by the same "becomes interface"
    // write from every candidate next to it, so the value read here serves
    // that write.
    uint8_t fdn[Q], fsn[Q];
    if (k < n) {
      const long long i = d.clist[k];
      coords(d, i, x, y, z);
      const uint8_t fd = d.flag_dst[i];
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const long long j = nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
        fdn[a] = d.flag_dst[j];
        fsn[a] = d.flag_src[j];
      }
      if (cand_filled(fd)) {
        F = true;
      } else if (fd & CAND_E) {
        E = true;
#pragma unroll
        for (int a = 1; a < Q; ++a)
          if (cand_filled(fdn[a])) E = false;
      }
      if (F) d.flag_dst[i] = (uint8_t)((fd & ~TYPE_MASK) | T_LIQ);
      if (E) d.flag_dst[i] = (uint8_t)((fd & ~TYPE_MASK) | T_GAS);
    }
    // neighbours that become interface cells: all claims are issued
    // together, then the claimed cells are appended with one atomic per
    // wave
    uint32_t won = 0;
    if (F || E) {
      // every claim in flight before any answer is looked at
      uint32_t want = 0;
      unsigned got[Q];
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const uint8_t tj = fsn[a] & TYPE_MASK;
        got[a] = 0;
        if ((F && tj == T_GAS) || (E && tj == T_LIQ)) {
          const long long j = nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
          d.flag_dst[j] = (uint8_t)((fdn[a] & ~TYPE_MASK) | T_IFACE);
          got[a] = claim_cell(d, j);
          want |= 1u << a;
        }
      }
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const long long j = nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
        if (((want >> a) & 1u) && !(got[a] & claim_bit(j))) won |= 1u << a;
      }
    }
    const int cnt = __popc(won);
    const int lane = (int)threadIdx.x & 63;
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    const int tot = __shfl(incl, 63, 64);
    int wbase = 0;
    if (lane == 0 && tot) wbase = atomicAdd(&d.sc->n_new, tot);
    int pos = __shfl(wbase, 0, 64) + incl - cnt;
#pragma unroll
    for (int a = 1; a < Q; ++a)
      if ((won >> a) & 1u) d.nlist[pos++] = (int)nbr(d, x, y, z, CX[a], CY[a], CZ[a]);
  }
}
};

// New interface cells.  From gas: f = f_eq(mean rho, mean u) of the
// neighbours that were interface or liquid at t (recovered from their
// post-collision values), m = 0, ID kept.  From liquid: m = rho of its own
// post-collision values, the smallest bubble ID of its emptied neighbours.
// D3Q19 velocities for runtime direction indices (one direction per lane).
__constant__ int8_t C19[3][Q] = {
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1}};

// Three new cells per wave, 18 lanes per cell (lanes 54..63 idle): lane q
// of a cell's group looks at its neighbour in direction q + 1 (loads and
// moments in parallel); the group's first lane then adds the 18
// contributions in direction order, so sums keep the order of their
// definition.
template <class P>
struct K_conv_init {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  using R = typename P::R;
  const int n = d.sc->n_new;
  const int lane = (int)threadIdx.x & 63;
  const int g = lane / 18, q = lane % 18, a = q + 1;
  const int wave = (bk.id * (int)blockDim.x + (int)threadIdx.x) >> 6;
  const int nwaves = (bk.n * (int)blockDim.x) >> 6;
  for (int base = 3 * wave; base < n; base += 3 * nwaves) {
    const int k = base + g;
    const bool act = g < 3 && k < n;
    long long i = 0;
    uint8_t t = T_LIQ;
    int x = 0, y = 0, z = 0;
    R cr = (R)0, cu[3] = {(R)0, (R)0, (R)0};
    int valid = 0, eid = INT_MAX, eslot = -1;
    if (act) {
      i = d.nlist[k];
      t = d.flag_src[i] & TYPE_MASK;
      coords(d, i, x, y, z);
      const long long j = nbr(d, x, y, z, C19[0][a], C19[1][a], C19[2][a]);
      const uint8_t tj = d.flag_src[j] & TYPE_MASK;
      if (t == T_GAS) {
        if (tj == T_IFACE || tj == T_LIQ) {
          R v[Q];
#pragma unroll
          for (int c = 0; c < Q; ++c) v[c] = ld<P>(d.f_dst, c, d.N, j);
          R r, dr;
          recover<P>(d, v, r, dr, cu);
          cr = P::EXACT ? r : dr;
          valid = 1;
        }
      } else if (tj == T_IFACE && (d.flag_dst[j] & TYPE_MASK) == T_GAS) {
        eslot = d.bslot[j];
        eid = d.b_id[eslot];
      }
    }
    // ordered sums (all lanes take part in the shuffles)
    R rs = (R)0, us[3] = {(R)0, (R)0, (R)0};
    int cnt = 0, best_id = INT_MAX, best_slot = -1;
    const int g0 = (g < 3 ? g : 2) * 18;
    for (int qq = 0; qq < 18; ++qq) {
      const int src = g0 + qq;
      const R vr = __shfl(cr, src, 64);
      const R v0 = __shfl(cu[0], src, 64), v1 = __shfl(cu[1], src, 64), v2 = __shfl(cu[2], src, 64);
      const int vv = __shfl(valid, src, 64);
      const int ve = __shfl(eid, src, 64), vs = __shfl(eslot, src, 64);
      if (vv) {
        rs += vr;
        us[0] += v0;
        us[1] += v1;
        us[2] += v2;
        ++cnt;
      }
      if (ve < best_id) {
        best_id = ve;
        best_slot = vs;
      }
    }
    if (act && q == 0) {
      if (t == T_GAS) {
        const R mean = rs / (R)cnt;
        const R rb = P::EXACT ? mean : (R)1 + mean;
        const R ubar[3] = {us[0] / (R)cnt, us[1] / (R)cnt, us[2] / (R)cnt};
        R fe[Q];
        eqv<P>(rb, P::EXACT ? rb - (R)1 : mean, ubar, fe);
        {
          typename P::S sv[Q];
          to_store<P>(fe, sv, store_key(i, (uint32_t)d.sc->step));
#pragma unroll
          for (int c = 0; c < Q; ++c) st<P>(d.f_dst, c, d.N, i, sv[c]);
        }
        ((R *)d.rhoI)[i] = rb;
        ((R *)d.mass)[i] = (R)0;
        atomicAdd((unsigned long long *)&d.b_ngas[d.bslot[i]], (unsigned long long)-1ll);
      } else {
        R v[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) v[c] = ld<P>(d.f_dst, c, d.N, i);
        R r, dr, uu[3];
        recover<P>(d, v, r, dr, uu);
        ((R *)d.mass)[i] = r;
        ((R *)d.rhoI)[i] = r;
        d.bslot[i] = best_slot;
      }
      release_cell(d, i);
    }
  }
}
};

// -------------------------------------------------------------- k_excess

// 3x3x3 block positions p = (dx+1) + 3 (dy+1) + 9 (dz+1); N18 offsets are
// those with 1 <= |dx|+|dy|+|dz| <= 2.
__device__ __forceinline__ int blk_pos(int dx, int dy, int dz) {
  return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}
// Block positions adjacent (18-neighbourhood) to each position p.
__constant__ uint32_t ADJ27[27] = {
    0x000161au, 0x0002e3du, 0x0004c32u, 0x000b2d3u, 0x00175efu, 0x0026996u, 0x0019098u,
    0x003a178u, 0x00340b0u, 0x02c340bu, 0x05c7a17u, 0x0986426u, 0x165a659u, 0x2ebdebau,
    0x4d32d34u, 0x32130c8u, 0x742f1d0u, 0x68161a0u, 0x0681600u, 0x0f42e00u, 0x0c84c00u,
    0x34cb200u, 0x7bd7400u, 0x65a6800u, 0x2619000u, 0x5e3a000u, 0x2c34000u};
__device__ __forceinline__ uint32_t adj_mask(int p) { return ADJ27[p]; }

// Removing the filled cell x from the gas region cannot disconnect it if
// (a) x's gas-region neighbours (new state) are connected inside x's 3x3x3
// block, and (b) every filled neighbour y of x shares a gas-region
// neighbour with x.  Returns true when a relabelling is needed.
// n1, n0: the flags of t+1 and t over the block (index blk_pos).
__device__ __forceinline__ bool split_possible(const uint8_t (&n1)[27], const uint8_t (&n0)[27]) {
  uint32_t setm = 0, filled = 0;
#pragma unroll
  for (int p = 0; p < 27; ++p) {
    if (p == 13) continue;
    const uint8_t tn = n1[p] & TYPE_MASK;
    if (in_gas_region(tn)) setm |= 1u << p;
    const int dx = p % 3 - 1, dy = (p / 3) % 3 - 1, dz = p / 9 - 1;
    const int l1 = (dx != 0) + (dy != 0) + (dz != 0);
    if (l1 <= 2 && (n0[p] & TYPE_MASK) == T_IFACE && tn == T_LIQ) filled |= 1u << p;
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

// The split test of the paper (Sec. 2.3.2): among the 18 neighbours of the
// cell that turned liquid, two interface cells of its bubble (interface at
// t and at t + 1, so that they have a normal of this step) whose unit
// normals point in opposite directions, n1.n2 < trigger_cos.
__device__ __forceinline__ bool antiparallel_normals(const Dev &d, int x, int y, int z, int slot,
                                                     const uint8_t (&n1)[27],
                                                     const uint8_t (&n0)[27]) {
  float nx[18], ny[18], nz[18];
  int cnt = 0;
  const long long C = d.icap;
#pragma unroll
  for (int p = 0; p < 27; ++p) {
    const int dx = p % 3 - 1, dy = (p / 3) % 3 - 1, dz = p / 9 - 1;
    const int l1 = (dx != 0) + (dy != 0) + (dz != 0);
    if (l1 == 0 || l1 == 3) continue;
    if ((n1[p] & TYPE_MASK) != T_IFACE || (n0[p] & TYPE_MASK) != T_IFACE) continue;
    const long long j = nbr(d, x, y, z, dx, dy, dz);
    if (d.bslot[j] != slot) continue;
    const int k = d.islot[j];
    nx[cnt] = d.nrm[k];
    ny[cnt] = d.nrm[C + k];
    nz[cnt] = d.nrm[2 * C + k];
    ++cnt;
  }
  const float c = (float)d.trigger_cos;
  for (int a = 0; a < cnt; ++a)
    for (int b = a + 1; b < cnt; ++b)
      if (nx[a] * nx[b] + ny[a] * ny[b] + nz[a] * nz[b] < c) return true;
  return false;
}

template <class P>
struct K_excess {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  using R = typename P::R;
  ExTerm orphan;
#pragma unroll
  for (int c = 0; c < EX_WORDS; ++c) orphan.w[c] = 0;
  bool trig = false;
  const int nc = d.sc->n_cand, nn = d.sc->n_new;
  for (int k = bk.id * blockDim.x + threadIdx.x; k < nc + nn; k += bk.n * blockDim.x) {
    const long long i = k < nc ? d.clist[k] : d.nlist[k - nc];
    int x, y, z;
    coords(d, i, x, y, z);
    // the cell's own values and its neighbours' flags of t+1 in one batch
    // (every rule below uses them; only the gather tags change in this
    // kernel, so a flag read here stays valid for the type tests)
    const uint8_t t = d.flag_src[i] & TYPE_MASK;
    const uint8_t fdi = d.flag_dst[i];
    const uint8_t tn = fdi & TYPE_MASK;
    const int slot = d.bslot[i];
    R *mass = (R *)d.mass;
    const R m_i = mass[i], rho_i = ((const R *)d.rhoI)[i];
    // the flags of t+1 and t over the 3x3x3 block (the split test needs
    // the corners too), also in that batch
    uint8_t n1[27], n0[27];
#pragma unroll
    for (int p = 0; p < 27; ++p) {
      if (p == 13) {
        n1[p] = n0[p] = 0;
        continue;
      }
      const long long j = nbr(d, x, y, z, p % 3 - 1, (p / 3) % 3 - 1, p / 9 - 1);
      n1[p] = d.flag_dst[j];
      n0[p] = d.flag_src[j];
    }
    uint8_t fn[Q];
#pragma unroll
    for (int a = 1; a < Q; ++a) fn[a] = n1[blk_pos(CX[a], CY[a], CZ[a])];
    const bool capped = t == T_IFACE && tn == T_IFACE && cand_capped(fdi);
    if (t == T_IFACE && (tn == T_LIQ || tn == T_GAS || capped)) {
      const bool filled = tn == T_LIQ;
      const R e = (filled || capped) ? m_i - rho_i : m_i;
      // receivers: the interface neighbours of t + 1 that are not capped
      int nI = 0;
#pragma unroll
      for (int a = 1; a < Q; ++a)
        if ((fn[a] & TYPE_MASK) == T_IFACE && !cand_capped(fn[a])) ++nI;
      if (nI > 0) {
        ((R *)d.excess)[i] = e / (R)nI;
        // tag the receivers
#pragma unroll
        for (int a = 1; a < Q; ++a) {
          if ((fn[a] & TYPE_MASK) == T_IFACE && !cand_capped(fn[a]) && !(fn[a] & GATHER))
            d.flag_dst[nbr(d, x, y, z, CX[a], CY[a], CZ[a])] = (uint8_t)(fn[a] | GATHER);
        }
      } else {
        ((R *)d.excess)[i] = (R)0;
        ex_accumulate(orphan, (double)e);
      }
      if (capped) {
        // stays an interface cell with m = rho (its fill level 1 plus what
        // it gathers from converted neighbours)
        mass[i] = rho_i;
        ((R *)d.phi_dst)[i] = (R)1;
      } else if (filled) {
        mass[i] = rho_i;
        ((R *)d.phi_src)[i] = (R)1;
        ((R *)d.phi_dst)[i] = (R)1;
        if (d.split_trigger == 1 ? antiparallel_normals(d, x, y, z, slot, n1, n0)
                                 : split_possible(n1, n0)) {
          trig = true;
          atomicOr(&d.b_affect[slot], 1);
        }
        d.bslot[i] = -1;
      } else {
        mass[i] = (R)0;
        ((R *)d.phi_src)[i] = (R)0;
        ((R *)d.phi_dst)[i] = (R)0;
        atomicAdd((unsigned long long *)&d.b_ngas[slot], 1ull);
      }
    } else if (t == T_LIQ && tn == T_IFACE) {
      // a new gas-region cell: a merge if its gas-region neighbours carry
      // another bubble (their slots read all at once first)
      const int s = slot;
      int sn[Q];
#pragma unroll
      for (int a = 1; a < Q; ++a)
        sn[a] = in_gas_region(fn[a] & TYPE_MASK) ? d.bslot[nbr(d, x, y, z, CX[a], CY[a], CZ[a])]
                                                  : s;
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        if (sn[a] != s) {
          trig = true;
          atomicOr(&d.b_affect[s], 1);
          atomicOr(&d.b_affect[sn[a]], 1);
        }
      }
    }
  }
  if (trig) atomicMax(&d.sc->label_run, 1);
  // a forced topology pass labels the whole gas region every step
  if (d.force_topology && bk.id == 0 && threadIdx.x == 0) atomicMax(&d.sc->label_run, 2);
  block_ex_add(orphan, d.bucket_acc, bk.id % SUB);
}
};

// -------------------------------------------------------------- k_gather

// Over the interface list of t+1 (in cell order): cells that received
// excess (tagged by k_excess) and new interface cells pull the excess of
// converted neighbours (in direction order) and recompute phi = m / rho;
// every cell adds 1 - phi to its bubble's volume (Sec. 2.3).
template <class P>
struct K_gather {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  using R = typename P::R;
  __shared__ KeySums<VA_FIXN + 1, 16> vol;
  key_sums_init(vol);
  const int sub = bk.id % SUB;
  const int n = d.sc->n_il_dst;  // interface list of t+1, rebuilt before this kernel
  const int nch = (n + THREADS - 1) / THREADS, m = nch < bk.n ? nch : bk.n;
  for (int c = bk.id; c < nch; c += bk.n) {
    const int k = xcd_chunk(c, m) * THREADS + (int)threadIdx.x;
    int key = -1;
    int v[VA_FIXN + 1] = {0, 0, 0, 1};  // chunks of (1 - phi) 2^53, count
    if (k < n) {
      const long long i = d.ilist_dst[k];
      // what every listed cell needs, in one batch with its flags
      const uint8_t fd = d.flag_dst[i];
      const uint8_t fsrc = d.flag_src[i];
      const int slot = d.bslot[i];
      R ph = ((const R *)d.phi_dst)[i];
      if ((fd & GATHER) || (fsrc & TYPE_MASK) != T_IFACE) {
        // a receiver of excess or a new interface cell
        R add = (R)0;
        bool touched = false;
        if (fd & GATHER) {
          int x, y, z;
          coords(d, i, x, y, z);
          const Nb3 nb(d, x, y, z);
          bool conv[Q];
          R ex[Q];
#pragma unroll
          for (int a = 1; a < Q; ++a) {
            const long long j = nb.at(d, CX[a], CY[a], CZ[a]);
            const uint8_t t0 = d.flag_src[j] & TYPE_MASK;
            const uint8_t f1 = d.flag_dst[j];
            const uint8_t t1 = f1 & TYPE_MASK;
            conv[a] = t0 == T_IFACE && (t1 == T_LIQ || t1 == T_GAS ||
                                        (t1 == T_IFACE && cand_capped(f1)));
            ex[a] = ((const R *)d.excess)[j];
          }
#pragma unroll
          for (int a = 1; a < Q; ++a) {
            add += conv[a] ? ex[a] : (R)0;
            touched = touched || conv[a];
          }
        }
        R m = ((R *)d.mass)[i];
        if (touched) {
          m += add;
          ((R *)d.mass)[i] = m;
        }
        ph = m / ((const R *)d.rhoI)[i];
        ((R *)d.phi_dst)[i] = ph;
      }
      // (an untouched interface cell keeps phi = m / rho as written by
      // k_iface)
      key = slot;
      const double gv = 1.0 - (double)ph;
      if (fabs(gv) < 2.0) {
        // an integer below 2^54 in magnitude, taken exactly
        const long long q = (long long)(gv * 0x1p53);
        const long long lo = (1ll << VA_FIX_BITS) - 1;
        v[0] = (int)(q & lo);
        v[1] = (int)((q >> VA_FIX_BITS) & lo);
        v[2] = (int)(q >> (2 * VA_FIX_BITS));
      } else {
        // outside the chunk range (a saved state may hold any fill
        // level): straight into the exact-sum words
        const ExTerm t = ex_split(gv);
        unsigned long long *w = d.b_vacc + ((long long)slot * SUB + sub) * VACC + VA_EX;
        for (int c = 0; c < EX_WORDS; ++c)
          if (t.w[c]) atomicAdd(&w[c], (unsigned long long)t.w[c]);
      }
    }
    wave_add_by_key_lds(key, v, vol, d.b_vacc, SUB, sub, VACC, VA_FIX);
  }
  key_sums_flush(vol, d.b_vacc, SUB, sub, VACC, VA_FIX);
}
};

// ------------------------------------------------------ interface list

// The interface cells of t+1 in increasing cell order (stream compaction
// over tiles of LTILE cells: count, scan, fill), so that the list kernels
// of the next step see spatially coherent cells in every wave.
constexpr int LTILE = 4096;

// Each thread of a tile block reads 16 consecutive flag bytes with one
// 16-byte load (tiles are 16-byte aligned; the ragged end of the box is
// read byte by byte).
__device__ __forceinline__ uint32_t iface_bits16(const Dev &d, long long i0) {
  uint32_t bits = 0;
  if (i0 + 16 <= d.N) {
    const uint4 v = *(const uint4 *)(d.flag_dst + i0);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        bits |= (uint32_t)((((w[q] >> (8 * b)) & TYPE_MASK) == T_IFACE) ? 1u : 0u) << (4 * q + b);
  } else {
    for (int b = 0; b < 16; ++b)
      if (i0 + b < d.N && (d.flag_dst[i0 + b] & TYPE_MASK) == T_IFACE) bits |= 1u << b;
  }
  return bits;
}

struct K_list_count {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  __shared__ int part[4];
  const long long i0 = (long long)bk.id * LTILE + 16 * (long long)threadIdx.x;
  int c = i0 < d.N ? __popc(iface_bits16(d, i0)) : 0;
  c = (int)wave_sum((long long)c);
  if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = c;
  __syncthreads();
  if (threadIdx.x == 0) d.tilecount[bk.id] = part[0] + part[1] + part[2] + part[3];
}
};

// The excess-mass pass and the tile counts of the interface list of t+1 in
// one launch: the first blocks take the excess pass, one block per tile
// follows.  The types of t+1 are final once the conversions are applied,
// and the excess pass only adds the receiver bit to flags, so the counts
// may run beside it.
template <class P>
struct K_excess_count {
  static constexpr int THREADS = 256;
  static_assert(K_excess<P>::THREADS == THREADS && K_list_count::THREADS == THREADS,
                "one block size for both parts");
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  const int ntiles = (int)((d.N + LTILE - 1) / LTILE);
  const int nex = bk.n - ntiles;
  if (bk.id < nex) K_excess<P>::run(d, Blk{bk.id, nex});
  else K_list_count::run(d, Blk{bk.id - nex, ntiles});
}
};

// Single block: exclusive scan of the tile counts.
struct K_list_scan {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  __shared__ int wtot[THREADS / 64];
  const int ntiles = (int)((d.N + LTILE - 1) / LTILE);
  const int per = (ntiles + THREADS - 1) / THREADS;
  const int lo = (int)threadIdx.x * per;
  int t = 0;
  for (int k = lo; k < lo + per && k < ntiles; ++k) t += d.tilecount[k];
  // inclusive scan of the per-thread totals: in the wave by shuffles, then
  // over the wave totals
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  int incl = t;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  int run = incl - t, total = 0;
  for (int k = 0; k < THREADS / 64; ++k) {
    if (k < w) run += wtot[k];
    total += wtot[k];
  }
  for (int k = lo; k < lo + per && k < ntiles; ++k) {
    const int c = d.tilecount[k];
    d.tileoff[k] = run;
    run += c;
  }
  if (threadIdx.x == 0) {
    // beyond the capacity the list is cut (an error the host reports)
    if (total > d.icap) atomicOr(&d.sc->err, ERR_ILIST);
    d.sc->n_il_dst = total < d.icap ? total : d.icap;
  }
}
};

struct K_list_fill {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  __shared__ int wsum[4];
  const int tile_base = d.tileoff[bk.id];  // in the same round as the flags
  const long long i0 = (long long)bk.id * LTILE + 16 * (long long)threadIdx.x;
  const uint32_t bits = i0 < d.N ? iface_bits16(d, i0) : 0u;
  const int c = __popc(bits);
  // exclusive prefix of the per-thread counts over the block, in thread
  // (= cell) order
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int before = 0;
  for (int k = 0; k < w; ++k) before += wsum[k];
  int pos = tile_base + before + incl - c;
  for (int b = 0; b < 16; ++b) {
    if ((bits >> b) & 1u) {
      const long long i = i0 + b;
      if (pos < d.icap) {
        d.ilist_dst[pos] = (int)i;
        d.islot_alt[i] = pos;  // the slots of the next step
      }
      ++pos;
    }
  }
}
};

// ------------------------------------------------------- bubble volumes

// Per-bubble volume V = (gas + inlet cells) + sum over interface cells of
// (1 - phi), exactly rounded (SUB lanes per bubble slot over the whole
// grid); orphan bucket and total mass (block 0).  Runs after the gather
// pass, in the blocks after the assign pass's, every step.
__device__ __forceinline__ void bubble_volumes(const Dev &d, Blk bk) {
  __shared__ long long red[4][2];
  // one lane per (slot, sub-slot): the SUB lanes of a slot are
  // consecutive lanes of one wave (SUB divides 64, blocks are whole
  // waves), load and clear their words at once and sum them with shuffles
  static_assert(64 % SUB == 0, "the sub-slots of a slot share a wave");
  const long long nq = (long long)d.max_bubbles * SUB;
  for (long long q0 = (long long)bk.id * blockDim.x; q0 < nq;
       q0 += (long long)bk.n * blockDim.x) {  // uniform per block
    const long long q = q0 + threadIdx.x;
    const long long s = q / SUB;
    const bool live = q < nq && d.b_live[s];
    if (!__ballot(live)) continue;  // no live slot in this wave (uniform per wave)
    long long w[VACC];
#pragma unroll
    for (int c = 0; c < VACC; ++c) w[c] = 0;
    if (live) {
      unsigned long long *acc = d.b_vacc + q * VACC;  // slot s, sub-slot q % SUB
#pragma unroll
      for (int c = 0; c < VACC; ++c) w[c] = ll(acc[c]);
#pragma unroll
      for (int c = 0; c < VACC; ++c) acc[c] = 0;
    }
#pragma unroll
    for (int m = SUB / 2; m >= 1; m >>= 1)
#pragma unroll
      for (int c = 0; c < VACC; ++c) w[c] += __shfl_xor(w[c], m, 64);
    if (live && q % SUB == 0) {
      long long e[EX_WORDS];
#pragma unroll
      for (int c = 0; c < EX_WORDS; ++c) e[c] = w[VA_EX + c];
      // the chunk sums (below 2^42 in magnitude: exact doubles) and the
      // gas cells join the exact sum
#pragma unroll
      for (int c = 0; c < VA_FIXN; ++c) {
        const ExTerm t = ex_split(ldexp((double)w[VA_FIX + c], VA_FIX_BITS * c - VA_FIX_SCALE));
#pragma unroll
        for (int k = 0; k < EX_WORDS; ++k) e[k] += t.w[k];
      }
      const ExTerm g = ex_split((double)d.b_ngas[s]);
#pragma unroll
      for (int c = 0; c < EX_WORDS; ++c) e[c] += g.w[c];
      d.b_vol[s] = ex_value(e);
      d.b_niface[s] = w[VA_CNT];
    }
  }
  if (bk.id != 0) return;  // uniform per block
  // total mass diagnostic: block reduction of the replicated slots
  long long mh = 0, ml = 0;
  for (int k = threadIdx.x; k < SUB_MASS; k += blockDim.x) {
    mh += ll(d.mass_acc[2 * k]);
    ml += ll(d.mass_acc[2 * k + 1]);
    d.mass_acc[2 * k] = d.mass_acc[2 * k + 1] = 0;
  }
  mh = wave_sum(mh);
  ml = wave_sum(ml);
  if (threadIdx.x % 64 == 0) {
    red[threadIdx.x / 64][0] = mh;
    red[threadIdx.x / 64][1] = ml;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Scalars *sc = d.sc;
    long long MH = 0, ML = 0;
    for (int k = 0; k < (int)(blockDim.x + 63) / 64; ++k) {
      MH += red[k][0];
      ML += red[k][1];
    }
    const long long nI = sc->n_il_dst;
    // the bucket of the last step was spread over this step's interface
    // cells unless there were none
    const double carry = sc->n_iface > 0 ? 0.0 : sc->bucket;
    long long bw[EX_WORDS];
    const ExTerm ct = ex_split(carry);
#pragma unroll
    for (int c = 0; c < EX_WORDS; ++c) bw[c] = ct.w[c];
    for (int k = 0; k < SUB; ++k)
#pragma unroll
      for (int c = 0; c < EX_WORDS; ++c) {
        bw[c] += ll(d.bucket_acc[EX_WORDS * k + c]);
        d.bucket_acc[EX_WORDS * k + c] = 0;
      }
    const double bucket = ex_value(bw);
    sc->total_mass = fx_value(MH, ML, FX_VOL) + carry;
    sc->bucket = bucket;
    sc->n_iface = nI;
    sc->share = nI > 0 ? bucket / (double)nI : 0.0;
  }
}

// ---------------------------------------------------------- labelling

// Union-find over the gas region (gas, interface, inlet cells of the new
// state) with 18-neighbour adjacency; every root is the smallest index of
// its component.  Labels only ever decrease and always point to a cell of
// the same component, so every find terminates.
//
// Only the bubbles marked by the topology trigger take part (all bubbles
// on the first step and when labelling is forced): a bubble the trigger did
// not mark has lost no cell and touched no other bubble, so it is still one
// component holding no other bubble and keeps its ID.
// Label reads may see an older value through the caches: an older label
// is still an ancestor (labels only move up their tree and are always
// smaller than the cell), so every walk ends at a cell of the same tree,
// and the linking atomics below act on the current value and retry.  Reads
// with workgroup scope stay in the caches instead of going to memory.
__device__ __forceinline__ int lab_load(const int32_t *lab, long long i) {
  return __hip_atomic_load(&lab[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Find with path halving: every visited cell is re-pointed to its
// grandparent (an ancestor, so the tree stays valid under concurrent
// linking), which keeps the trees shallow.  The re-pointing is a plain
// store: only cells that are no longer roots are re-pointed, and linking
// only writes roots, so a store can at worst put back a less compressed
// ancestor written by another walk; either is valid.  (An atomicMin here
// cost 6 us per labelling run of the 256^3 rupture.)
__device__ __forceinline__ int uf_find(int32_t *lab, int i) {
  int p = lab_load(lab, i);
  while (p != i) {
    const int gp = lab_load(lab, p);
    if (gp == p) return p;
    __hip_atomic_store(&lab[i], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    i = gp;
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
  for (long long i = (long long)bk.id * blockDim.x + threadIdx.x; i < d.N; \
       i += (long long)bk.n * blockDim.x)

// The cells of the labelled set, listed by k_label_init in the candidate
// list (free once the conversions of the step are done); one cell per
// thread in the later passes, whatever the shape of the gas region.
#define FSLBM_LABEL_SET(i) \
  for (int k_ = bk.id * blockDim.x + threadIdx.x, n_ = d.sc->n_lab; k_ < n_; \
       k_ += bk.n * blockDim.x) \
    if (const long long i = d.clist[k_]; true)

// aux2 flags of a root: 1 holds an inlet cell, 2 new component, 4 holds
// cells of more than one bubble.
//
// Labelled set, tile by tile (LTILE consecutive cells, 16 per thread): the
// cells of the set are labelled with the first cell of their x-run inside
// the wave's cells, and listed in cell order.  A block takes a contiguous
// range of tiles and appends the set cells of GROUP tiles at a time with one
// atomic: the appends of all blocks serialise on the one counter.  Cells
// outside the set hold -1 (filled at creation, restored by
// k_label_accumulate).
struct K_label_init {
  static constexpr int THREADS = 256;
  static constexpr int GROUP = 4;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  __shared__ int wsum[GROUP][THREADS / 64];
  __shared__ int base_sh;
  __shared__ int loc[LTILE];
  // per tile of a group: each thread's set cells, and how many set cells
  // the lanes before it in its wave hold (own entries only: no barrier)
  __shared__ uint32_t gbits[GROUP][THREADS];
  __shared__ int gpre[GROUP][THREADS];
  const int run = d.sc->label_run;
  if (!run) return;
  const bool all = run >= 2;
  const int ntiles = (int)((d.N + LTILE - 1) / LTILE);
  const int per = (ntiles + bk.n - 1) / bk.n;
  const int tb = bk.id * per < ntiles ? bk.id * per : ntiles;
  const int te = tb + per < ntiles ? tb + per : ntiles;
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int lb = 16 * (int)threadIdx.x;  // local index of the thread's first cell
  for (int gt = tb; gt < te; gt += GROUP) {  // uniform per block
#pragma unroll 1
  for (int u = 0; u < GROUP; ++u) {
    const int tile = gt + u;
    gbits[u][threadIdx.x] = 0u;
    gpre[u][threadIdx.x] = 0;
    if (tile >= te) {
      if (lane == 63) wsum[u][w] = 0;
      continue;
    }
    const long long t0 = (long long)tile * LTILE;
    const long long i0 = t0 + lb;
    uint32_t bits = 0;
    if (i0 < d.N) {
      uint8_t tt[16];
      if (i0 + 16 <= d.N) {
        const uint4 v = *(const uint4 *)(d.flag_dst + i0);
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 16; ++q) tt[q] = (uint8_t)((wd[q / 4] >> (8 * (q % 4))) & TYPE_MASK);
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q)
          tt[q] = i0 + q < d.N ? (uint8_t)(d.flag_dst[i0 + q] & TYPE_MASK) : (uint8_t)T_WALL;
      }
      uint32_t gas = 0;
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (in_gas_region(tt[q])) gas |= 1u << q;
      if (all || !gas) {
        bits = gas;
      } else if (i0 + 16 <= d.N) {
        // the 16 slots with four 16-byte loads (i0 is a multiple of 16)
        int sl[16];
        __builtin_memcpy(sl, d.bslot + i0, 64);
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (((gas >> q) & 1u) && d.b_affect[sl[q]]) bits |= 1u << q;
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (((gas >> q) & 1u) && d.b_affect[d.bslot[i0 + q]]) bits |= 1u << q;
      }
    }
    // the whole tile outside the set: nothing to do
    if (!__syncthreads_or(bits != 0u)) {
      if (lane == 63) wsum[u][w] = 0;
      continue;
    }
    // initial local labels: the first cell of the cell's x-run inside the
    // wave's 1024 cells, so that every row segment starts as a star (depth
    // one).  A run starts at a set cell that is the wave's first, at x = 0,
    // or after a cell outside the set; the run that enters a thread's cells
    // from the left started at the last start of the lanes before it (a
    // max-scan over the wave).  A run cut at a wave boundary (only where
    // the row length does not divide 1024) is joined by the union pass
    // through its +x edge.
    {
      uint32_t pb = __shfl_up(bits, 1, 64);
      if (lane == 0) pb = 0u;
      const bool left = lane > 0 && ((pb >> 15) & 1u);  // the cell before is set
      const int x0 = (int)(i0 % d.nx);
      int last = -1;
      {
        int x = x0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const bool prev = q > 0 ? ((bits >> (q - 1)) & 1u) != 0u : left;
          if (((bits >> q) & 1u) && (x == 0 || !prev)) last = lb + q;
          if (++x == d.nx) x = 0;
        }
      }
      int incl = last;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off && v > incl) incl = v;
      }
      int carry = __shfl_up(incl, 1, 64);
      if (lane == 0) carry = -1;
      int start = (left && x0 != 0) ? carry : -1;
      int x = x0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (x == 0) start = -1;
        if ((bits >> q) & 1u) {
          if (start < 0) start = lb + q;
          loc[lb + q] = start;
        } else {
          loc[lb + q] = -1;
          start = -1;
        }
        if (++x == d.nx) x = 0;
      }
    }
    __syncthreads();
    // publish the labels of the set cells (lane-consecutive cells)
    for (int r = 0; r < LTILE / THREADS; ++r) {
      const int c = (int)threadIdx.x + THREADS * r;
      const long long i = t0 + c;
      if (i >= d.N) break;
      const int p = loc[c];
      if (p < 0) continue;
      d.lab[i] = (int)(t0 + p);
      d.aux2[i] = 0;
    }
    // the set cells of the lanes before this one in the wave
    const int c = __popc(bits);
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[u][w] = incl;
    gbits[u][threadIdx.x] = bits;
    gpre[u][threadIdx.x] = incl - c;
  }
  // list the set cells of the group: one atomic, cell order
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int u = 0; u < GROUP; ++u)
      for (int k = 0; k < THREADS / 64; ++k) tot += wsum[u][k];
    base_sh = tot ? atomicAdd(&d.sc->n_lab, tot) : 0;
  }
  __syncthreads();
  int pos0 = base_sh;
#pragma unroll 1
  for (int u = 0; u < GROUP; ++u) {
    int pos = pos0 + gpre[u][threadIdx.x];
    for (int k = 0; k < THREADS / 64; ++k) {
      if (k < w) pos += wsum[u][k];
      pos0 += wsum[u][k];
    }
    const uint32_t bits = gbits[u][threadIdx.x];
    const long long i0 = (long long)(gt + u) * LTILE + lb;
    for (int q = 0; q < 16; ++q)
      if ((bits >> q) & 1u) d.clist[pos++] = (int)(i0 + q);
  }
  __syncthreads();  // wsum and base_sh are taken by the next group
  }
  const long long g0 = (long long)bk.id * blockDim.x + threadIdx.x;
  for (long long t = g0; t < d.max_bubbles; t += (long long)bk.n * blockDim.x) {
    d.b_rmin[t] = INT_MAX;
    d.b_rmax[t] = -1;
    // bubbles outside the labelled set keep their entry
    d.b_kept[t] = (!all && d.b_live[t] && !d.b_affect[t]) ? 1 : 0;
  }
  if (g0 == 0) d.sc->nnew = 0;
}
};

// The scan of the interface list's tile counts (block 0) and the labelled
// set (the other blocks) in one launch: the set needs only the types and
// slots of t+1 and the trigger's marks, all final once the excess pass is
// done, and neither part reads what the other writes.
struct K_scan_label_init {
  static constexpr int THREADS = 256;
  static_assert(K_list_scan::THREADS == THREADS && K_label_init::THREADS == THREADS,
                "one block size for both parts");
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  if (bk.id == 0) K_list_scan::run(d, Blk{0, 1});
  else K_label_init::run(d, Blk{bk.id - 1, bk.n - 1});
}
};

// Every edge of the set (one direction of every opposite pair).
// Consecutive set cells usually share their label (one x-run) and so do
// their neighbours in a direction: a lane whose (label, neighbour label)
// pair equals its left neighbour's skips the union, which the left lane
// performs (labels only ever move to ancestors, so equal labels, read at
// any time, mean one tree).
struct K_label_union {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  if (!d.sc->label_run) return;
  const int n = d.sc->n_lab;
  const int lane = (int)threadIdx.x & 63;
  for (int base = bk.id * (int)blockDim.x; base < n; base += bk.n * (int)blockDim.x) {
    const int k = base + (int)threadIdx.x;
    const bool ok = k < n;
    const long long i = ok ? d.clist[k] : 0;
    int x = 0, y = 0, z = 0;
    if (ok) coords(d, i, x, y, z);
    const int li = ok ? d.lab[i] : -1;
    // the neighbours' labels first, all at once (a label read before
    // other unions still lies in its cell's tree: labels only decrease
    // towards the roots)
    int ln[Q / 2];
#pragma unroll
    for (int q = 0; q < Q / 2; ++q) {
      const int a = 2 * q + 1;
      const long long j = ok ? nbr_checked(d, x, y, z, CX[a], CY[a], CZ[a]) : -1;
      ln[q] = j >= 0 ? d.lab[j] : -1;
    }
    // a diagonal edge is implied when one of the two cells beside it (one
    // unit step along either of its axes) is in the set: the two unit
    // edges through that cell are united by their own cells (unit edges
    // are never skipped).  Directions 1, 3, 5 are +x, +y, +z; 7 +x+y,
    // 9 +x-y, 11 +x+z, 13 +x-z, 15 +y+z, 17 +y-z; of the cells beside a
    // diagonal, the +x, +y, +z ones are those read above.
    static_assert(CX[1] == 1 && CY[3] == 1 && CZ[5] == 1 && CX[7] == 1 && CY[7] == 1 &&
                      CX[9] == 1 && CY[9] == -1 && CX[11] == 1 && CZ[11] == 1 && CX[13] == 1 &&
                      CZ[13] == -1 && CY[15] == 1 && CZ[15] == 1 && CY[17] == 1 && CZ[17] == -1,
                  "direction order of the diagonal rule");
    {
      const bool sx = ln[0] >= 0, sy = ln[1] >= 0, sz = ln[2] >= 0;
      if (sx || sy) ln[3] = -1;
      if (sx) ln[4] = -1;
      if (sx || sz) ln[5] = -1;
      if (sx) ln[6] = -1;
      if (sy || sz) ln[7] = -1;
      if (sy) ln[8] = -1;
    }
#pragma unroll
    for (int q = 0; q < Q / 2; ++q) {
      const int lj = ln[q];
      const int pli = __shfl_up(li, 1, 64), plj = __shfl_up(lj, 1, 64);
      const bool dup = lane > 0 && pli == li && plj == lj;
      // outside the set, one tree already, or left to the left lane
      if (lj < 0 || lj == li || dup) continue;
      uf_union(d.lab, li, lj);
    }
  }
}
};

// The fill of the interface list of t+1 (one block per tile) and the
// unions of the labelled set (the blocks after them) in one launch: the
// unions read and write only the labels, which neither the fill nor the
// gather pass after it touch, and the fill reads only the types of t+1
// and the scanned tile offsets.
struct K_fill_label_union {
  static constexpr int THREADS = 256;
  static_assert(K_list_fill::THREADS == THREADS && K_label_union::THREADS == THREADS,
                "one block size for both parts");
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  const int ntiles = (int)((d.N + LTILE - 1) / LTILE);
  if (bk.id < ntiles) K_list_fill::run(d, Blk{bk.id, ntiles});
  else K_label_union::run(d, Blk{bk.id - ntiles, bk.n - ntiles});
}
};

// Final roots (the trees no longer change: plain loads).  Every root
// registers itself with its bubble; an edge between cells of two bubbles
// marks the component as mixed and registers it with both bubbles, so that
// every bubble knows the smallest and largest root of the components that
// hold its cells.
struct K_label_roots {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  if (!d.sc->label_run) return;
  FSLBM_LABEL_SET(i) {
    // the cell's own values and its neighbours' slots are read while the
    // root is found (set membership and slots do not change in this pass)
    const int s = d.bslot[i];
    const bool inlet = (d.flag_dst[i] & TYPE_MASK) == T_INLET;
    int x, y, z;
    coords(d, i, x, y, z);
    int sn[Q / 2];
#pragma unroll
    for (int q = 0; q < Q / 2; ++q) {
      const int a = 2 * q + 1;
      const long long j = nbr_checked(d, x, y, z, CX[a], CY[a], CZ[a]);
      sn[q] = (j < 0 || d.lab[j] < 0) ? -1 : d.bslot[j];
    }
    int r = (int)i, p = d.lab[i];
    while (p != r) {
      r = p;
      p = d.lab[r];
    }
    d.lab[i] = r;
    if (r == (int)i) {
      atomicMin(&d.b_rmin[s], r);
      atomicMax(&d.b_rmax[s], r);
      // the roots are listed (the new-cell list is free during labelling)
      const int q = atomicAdd(&d.sc->n_roots, 1);
      if (q < (int)d.N) d.nlist[q] = r;
    }
    if (inlet) atomicOr(&d.aux2[r], 1);
#pragma unroll
    for (int q = 0; q < Q / 2; ++q) {
      const int sj = sn[q];
      if (sj < 0 || sj == s) continue;
      atomicOr(&d.aux2[r], 4);
      atomicMin(&d.b_rmin[s], r);
      atomicMax(&d.b_rmax[s], r);
      atomicMin(&d.b_rmin[sj], r);
      atomicMax(&d.b_rmax[sj], r);
    }
  }
}
};

// Single block: decide, per listed root, whether its component keeps its
// bubble; order the new components by their smallest cell index, give each
// the next fresh ID and a free slot, and fix the V* ratio of every old
// bubble.
struct K_label_assign {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  if (!d.sc->label_run) return;
  Scalars *sc = d.sc;
  const int B = d.max_bubbles;
  __shared__ int s_nnew;
  if (threadIdx.x == 0) s_nnew = 0;
  __syncthreads();
  // over the listed roots: a component keeps its bubble if it holds
  // exactly one bubble and that bubble lies in no other component; every
  // other component is new
  const int nr = sc->n_roots;
  for (int k = threadIdx.x; k < nr; k += blockDim.x) {
    const int r = d.nlist[k];
    const int s = d.bslot[r];
    const bool single = !(d.aux2[r] & 4) && d.b_rmin[s] == r && d.b_rmax[s] == r;
    if (single) {
      d.b_kept[s] = 1;
    } else {
      const int q = atomicAdd(&s_nnew, 1);
      if (q < B) d.newroots[q] = r;
      atomicOr(&d.aux2[r], 2);
    }
  }
  __syncthreads();
  const int nnew = s_nnew;
  if (threadIdx.x == 0) sc->nnew = nnew;
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
  __syncthreads();
  // the first nnew free slots in increasing order: a block-wide prefix
  // count of the free slots, chunk by chunk
  __shared__ int wfree[THREADS / 64];
  __shared__ int s_base;
  if (threadIdx.x == 0) s_base = 0;
  __syncthreads();
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  for (int s0 = 0; s0 < B; s0 += THREADS) {
    const int s = s0 + (int)threadIdx.x;
    const bool freed = s < B && !(d.b_live[s] && d.b_kept[s]);
    const unsigned long long m = __ballot(freed);
    if (lane == 0) wfree[w] = __popcll(m);
    __syncthreads();
    int before = s_base;
    for (int k = 0; k < w; ++k) before += wfree[k];
    const int pos = before + (int)__popcll(m & ((1ull << lane) - 1ull));
    if (freed && pos < nnew) d.newslot[pos] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int k = 0; k < THREADS / 64; ++k) t += wfree[k];
      s_base += t;
    }
    __syncthreads();
    if (s_base >= nnew) break;  // uniform: read by every thread after the barrier
  }
  if (threadIdx.x == 0) {
    const int k = s_base < nnew ? s_base : nnew;
    if (k < nnew) sc->err |= ERR_CAPACITY;
    sc->nfree = k;
  }
}
};

// The gather pass (its G_LIST blocks) and the roots pass (the blocks after
// them) in one launch: the roots pass reads the labels, slots and types of
// t+1, which the gather pass does not write, and writes only labels, root
// ranges and the root list, which the gather pass does not read.
template <class P>
struct K_gather_label_roots {
  static constexpr int THREADS = 256;
  static_assert(K_gather<P>::THREADS == THREADS && K_label_roots::THREADS == THREADS,
                "one block size for both parts");
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  const int nc = cell_blocks(d.N), ng = bk.n - nc;
  if (bk.id < ng) K_gather<P>::run(d, Blk{bk.id, ng});
  else K_label_roots::run(d, Blk{bk.id - ng, nc});
}
};

// The assign pass (block 0) and the per-bubble volume reduction (the blocks
// after it: one lane per bubble slot and sub-slot) in one launch: the
// volumes need the gather pass, and the accumulate pass after both reads
// them; the assign pass reads none of what the reduction writes.
struct K_assign_volumes {
  static constexpr int THREADS = 256;
  static_assert(K_label_assign::THREADS == THREADS, "one block size for both parts");
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  if (bk.id == 0) K_label_assign::run(d, Blk{0, 1});
  else bubble_volumes(d, Blk{bk.id - 1, bk.n - 1});
}
};

// Per new component: gas volume V_K = sum (1 - phi) (gas and inlet cells
// count 1), V*_K = sum over its cells of (V*_b / V_b) times the cell's gas
// volume (= sum_b V*_b V(b in K) / V_b), cell counts and the inlet flag.
// Each cell of a new component then moves to the component's slot, and
// every cell of the set gets its label -1 back (every cell holds its root
// since k_label_roots), so that the next labelling finds the cells outside
// its set without writing the whole field.
template <class P>
struct K_label_accumulate {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  using R = typename P::R;
  const Scalars *sc = d.sc;
  if (!sc->label_run) return;
  __shared__ KeySums<NACC, 16> comp;
  key_sums_init(comp);
  const bool ok = sc->nnew <= d.max_bubbles && sc->nfree >= sc->nnew;
  const int n = sc->n_lab;
  for (int base = bk.id * blockDim.x; base < n; base += bk.n * blockDim.x) {
    const int k = base + threadIdx.x;
    int key = -1;
    long long v[NACC];
#pragma unroll
    for (int c = 0; c < NACC; ++c) v[c] = 0;
    if (k < n) {
      const long long i = d.clist[k];
      // every value the cell may need, in two rounds (a set cell has a
      // root and a slot)
      const int r = d.lab[i];
      const uint8_t t = d.flag_dst[i] & TYPE_MASK;
      const R ph = ((const R *)d.phi_dst)[i];
      const int sl = d.bslot[i];
      const int a2 = d.aux2[r], a0 = d.aux0[r];
      const double bv = d.b_vol[sl], bvs = d.b_vstar[sl];
      const long long nc = d.b_ngas[sl] + d.b_niface[sl];
      const int bfl = d.b_flags[sl];
      if (ok && (a2 & 2)) {
        key = a0;
        const double w = t == T_IFACE ? 1.0 - (double)ph : 1.0;
        // V* per unit gas volume of the old bubble (per cell if V <= 0)
        const double ratio = bv > 0.0 ? bvs / bv : -(bvs / (double)(nc > 0 ? nc : 1));
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
        v[2 * EX_WORDS + 4] = (bfl & BUBBLE_ATMOSPHERE) ? 1 : 0;
        d.bslot[i] = d.newslot[key];
      }
      d.lab[i] = -1;
    }
    wave_add_by_key_lds(key, v, comp, d.c_acc, SUB, bk.id % SUB, NACC, 0);
  }
  key_sums_flush(comp, d.c_acc, SUB, bk.id % SUB, NACC, 0);
}
};

// ------------------------------------------------------------- k_bubbles

// One new component k of a labelling run, with its summed accumulator
// words a[NACC], into its slot.
__device__ __forceinline__ void install_one(const Dev &d, int k, const unsigned long long *a) {
  const int s = d.newslot[k];
  d.b_id[s] = d.sc->next_id + k;
  long long wv[EX_WORDS], ws[EX_WORDS];
  for (int c = 0; c < EX_WORDS; ++c) {
    wv[c] = ll(a[c]);
    ws[c] = ll(a[EX_WORDS + c]);
  }
  d.b_flags[s] = (ll(a[2 * EX_WORDS + 3]) > 0 ? BUBBLE_INLET : 0) |
                 (ll(a[2 * EX_WORDS + 4]) > 0 ? BUBBLE_ATMOSPHERE : 0);
  d.b_vol[s] = ex_value(wv);
  d.b_vstar[s] = ex_value(ws);
  d.b_ngas[s] = ll(a[2 * EX_WORDS + 1]);
  d.b_niface[s] = ll(a[2 * EX_WORDS + 2]);
  d.b_live[s] = 1;
}

// After a labelling run (one block): free the slots of replaced bubbles
// and install the new components (summing and clearing their partial
// sums).  Every thread of the block must call it.
__device__ __forceinline__ void install_new_bubbles(const Dev &d) {
  Scalars *sc = d.sc;
  const int nnew = sc->nnew;
  const int B = d.max_bubbles;
  for (int s = threadIdx.x; s < B; s += blockDim.x)
    if (d.b_live[s] && !d.b_kept[s]) d.b_live[s] = 0;
  __syncthreads();
  // the SUB partial sums of every word of every new component, one thread
  // per (component, word), through shared memory (a component at a time per
  // thread would walk its SUB * NACC words in series)
  __shared__ unsigned long long comp_sum[64][NACC];
  for (int k0 = 0; k0 < nnew; k0 += 64) {
    const int kn = nnew - k0 < 64 ? nnew - k0 : 64;
    for (int t = threadIdx.x; t < kn * NACC; t += blockDim.x) {
      const int k = k0 + t / NACC, c = t % NACC;
      unsigned long long *p = d.c_acc + (long long)k * SUB * NACC + c;
      unsigned long long v[SUB];
#pragma unroll
      for (int u = 0; u < SUB; ++u) v[u] = p[u * NACC];
      unsigned long long acc = 0;
#pragma unroll
      for (int u = 0; u < SUB; ++u) {
        acc += v[u];
        p[u * NACC] = 0;
      }
      comp_sum[t / NACC][c] = acc;
    }
    __syncthreads();
    for (int kk = threadIdx.x; kk < kn; kk += blockDim.x) install_one(d, k0 + kk, comp_sum[kk]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sc->next_id += nnew;
    if (nnew > 0) sc->n_topology += 1;
  }
}

// Single block: the new bubbles of a labelling run (unless the table
// overflowed, which the labelling flagged), gas injection into inlet
// bubbles and the ideal-gas pressure p = p0 V* / max(V, 1e-2); closes the
// step.
struct K_bubbles {
  static constexpr int THREADS = 1024;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  __shared__ int live;
  const Scalars *sc0 = d.sc;
  // the same values for every thread of the block
  if (sc0->label_run && sc0->nnew <= d.max_bubbles && sc0->nfree >= sc0->nnew)
    install_new_bubbles(d);
  if (threadIdx.x == 0) live = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < d.max_bubbles; s += blockDim.x) {
    d.b_affect[s] = 0;
    if (!d.b_live[s]) continue;
    const int fl = d.b_flags[s];
    if (fl & BUBBLE_INLET) d.b_vstar[s] += d.inject;
    const double v = d.b_vol[s] > 1e-2 ? d.b_vol[s] : 1e-2;
    // an atmosphere (open top) stays at the reference pressure
    d.b_p[s] = (fl & BUBBLE_ATMOSPHERE) ? d.p0 : d.p0 * d.b_vstar[s] / v;
    atomicAdd(&live, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Scalars *sc = d.sc;
    sc->n_live = live;
    if (sc->label_run) sc->n_label_runs += 1;
    sc->label_run = 0;
    // the lists of the next step
    sc->n_il_src = sc->n_il_dst;
    sc->n_il_dst = 0;
    sc->n_cand = 0;
    sc->n_new = 0;
    sc->n_lab = 0;
    sc->n_roots = 0;
    sc->if_prev = 1;  // the interface rows of this step serve the next one
    sc->step += 1;
    if (!isfinite(sc->total_mass)) sc->err |= ERR_NONFINITE;
  }
}
};

// ------------------------------------------------------------ watchdog

// Invariants of the state after a step (launched with the Dev of the next
// step, so the state is in the source arrays): the interface is a closed
// layer (no liquid cell next to a gas or inlet cell, Sec. 2.2), every cell
// of the gas region belongs to a live bubble, interface masses and fill
// levels are finite; block 0 also checks the drift of the total mass
// against the mass at creation.  Failures set error bits only.
template <class P>
struct K_watchdog {
  static constexpr int THREADS = 256;
  static __device__ __forceinline__ void run(const Dev &d, Blk bk) {
  using R = typename P::R;
  int err = 0;
  FSLBM_GRID_STRIDE(i) {
    const uint8_t t = d.flag_src[i] & TYPE_MASK;
    if (t == T_LIQ) {
      int x, y, z;
      coords(d, i, x, y, z);
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const long long j = nbr_checked(d, x, y, z, CX[a], CY[a], CZ[a]);
        if (j < 0) continue;
        const uint8_t tj = d.flag_src[j] & TYPE_MASK;
        if (tj == T_GAS || tj == T_INLET) err |= ERR_LAYER;
      }
    } else if (in_gas_region(t)) {
      const int s = d.bslot[i];
      if (s < 0 || s >= d.max_bubbles || !d.b_live[s]) err |= ERR_ORPHAN;
    }
  }
  // the interface cells of the next step: finite mass and fill level
  const int n = d.sc->n_il_src;
  for (int k = bk.id * blockDim.x + threadIdx.x; k < n; k += bk.n * blockDim.x) {
    const long long i = d.ilist_src[k];
    const R m = ((const R *)d.mass)[i], ph = ((const R *)d.phi_src)[i];
    if (!isfinite(m) || !isfinite(ph)) err |= ERR_NONFINITE;
  }
  int w = err;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) w |= __shfl_xor(w, m, 64);
  if (w && __lane_id() == 0) atomicOr(&d.sc->err, w);
  if (bk.id == 0 && threadIdx.x == 0 && d.drift_tol > 0.0) {
    const double M = d.sc->total_mass, M0 = d.sc->mass_ref;
    if (!(fabs(M - M0) <= d.drift_tol * fabs(M0))) atomicOr(&d.sc->err, ERR_DRIFT);
  }
}
};

// ------------------------------------------------------------ launchers

// A step kernel K launched for one domain (its Dev by value) or for a
// batch of domains: block b of a batch launch belongs to the domain k with
// off[k] <= b < off[k + 1] (found by bisection; domains without blocks
// are skipped).
// Waves per SIMD a kernel must fit (K::MIN_WAVES where given): bounds the
// registers of a kernel whose grid is about one round of resident waves.
template <class K, class = void>
struct MinWaves {
  static constexpr int value = 1;
};
template <class K>
struct MinWaves<K, decltype((void)K::MIN_WAVES)> {
  static constexpr int value = K::MIN_WAVES;
};

template <class K>
__global__ void __launch_bounds__(K::THREADS, MinWaves<K>::value) k_one(Dev d) {
  K::run(d, Blk{(int)blockIdx.x, (int)gridDim.x});
}

__device__ __forceinline__ int batch_domain(const int *off, int nd, int b) {
  int lo = 0, hi = nd;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <class K>
__global__ void __launch_bounds__(K::THREADS, MinWaves<K>::value) k_many(const Dev *devs, const int *off,
                                                                         int nd) {
  const int b = (int)blockIdx.x;
  const int k = batch_domain(off, nd, b);
  K::run(devs[k], Blk{b - off[k], off[k + 1] - off[k]});
}

// ------------------------------------------------------- create / export

// Stored PDFs of f = f_eq(rho, u) on interface and liquid cells from FP64
// staging arrays rho[N], u[3N] (computed in double); the weights elsewhere.
template <class P>
__global__ void __launch_bounds__(256) k_init_feq(Dev d, const double *rho, const double *u) {
  const Blk bk{(int)blockIdx.x, (int)gridDim.x};
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
    R fr[Q];
    for (int a = 0; a < Q; ++a) fr[a] = (R)(P::EXACT ? fe[a] : fe[a] - wgt(a));
    typename P::S sv[Q];
    to_store<P>(fr, sv, store_key(i, 0xFFFFFFFFu));
    for (int a = 0; a < Q; ++a) st<P>(d.f_src, a, d.N, i, sv[a]);
  }
}

// One direction a of f from an FP64 staging array.
template <class P>
__global__ void __launch_bounds__(256) k_init_f(Dev d, const double *src, int a) {
  const Blk bk{(int)blockIdx.x, (int)gridDim.x};
  using R = typename P::R;
  // (an exact conversion for values exported from the same precision)
  FSLBM_GRID_STRIDE(i)
      st<P>(d.f_src, a, d.N, i, (typename P::S)(R)(P::EXACT ? src[i] : src[i] - wgt(a)));
}

// Export one quantity as FP64: what = 0 phi, 1 mass (rho on liquid cells),
// 2 rho, 3..5 u, 6 + a f_a.
template <class P>
__global__ void __launch_bounds__(256) k_export(Dev d, double *out, int what) {
  const Blk bk{(int)blockIdx.x, (int)gridDim.x};
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
