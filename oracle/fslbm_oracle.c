/*
 * Plain FP64 CPU oracle of the free-surface lattice Boltzmann step with the
 * enhanced bubble model (arXiv:1604.01632).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests, by the smoke check and by the CPU
 * baseline leg of the benchmark.  It shares nothing with the GPU library.
 *
 * One step t -> t+1 runs these phases, each reading only the complete
 * output of the previous one:
 *   A  per interface/liquid cell: normal + curvature -> gas pressure
 *      (Sec. 2.2, gas-pressure and Laplace-pressure equations), pull
 *      streaming with bounce-back at walls, reconstruction of the gas-side
 *      PDFs (Sec. 2.2, reconstruction equation), mass exchange (Sec. 2.2,
 *      mass-exchange equation), BGK collision (Sec. 2.1) with a Guo body
 *      force, new fill level.
 *   B  classify filled / emptied interface cells (Sec. 2.2, "fill level
 *      approaches 1 or 0"; the interface stays a closed layer).
 *   C  new cell types and initial values of new interface cells.
 *   D  excess-mass redistribution to interface neighbours.
 *   E  bubble volumes from gas cells and interface fill levels (Sec. 2.3).
 *   F  connected components of the gas region every step (the flood fill of
 *      Sec. 2.3.2) and the merge (Sec. 2.3.1) / split (Sec. 2.3.2) rules.
 *   G  gas injection and ideal-gas pressure p = p0 V* / V (Sec. 2.2,
 *      ideal-gas equation).
 *   H  diagnostics (total mass).
 * Points where the paper is silent follow the readings listed with the
 * design notes (weights, Guo forcing, reconstruction directions, height-
 * function curvature, thresholds, excess mass, split pressure, IDs).
 */
#include "fslbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* D3Q19 velocities (Sec. 2.1; Qian et al.): rest, 6 faces, 12 edges. */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double weight(int a) {
  if (a == 0) return 1.0 / 3.0;
  if (a <= 6) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

/* Opposite direction: the pairs are (1,2), (3,4), ..., (17,18). */
static int opposite(int a) {
  if (a == 0) return 0;
  return (a % 2 == 1) ? a + 1 : a - 1;
}

/* ------------------------------------------------- exactly rounded sums -- */

/* Sums of per-cell quantities (bubble volumes, gas amounts, the orphan
 * bucket, the total mass) are exactly rounded: the result is the exact sum
 * of the terms rounded once to the nearest double, independent of order.
 * Shewchuk's method (1997): keep non-overlapping partials whose sum is
 * exact, updated with error-free two-sums; at the end add them from the
 * largest down and correct a half-way case so that ties round to even
 * (the correction used by R. Hettinger's msum recipe, which is also the
 * algorithm of Python's math.fsum). */
typedef struct {
  double *p;
  int n, cap;
} xsum;

static void xsum_add(xsum *a, double x) {
  int k = 0;
  for (int j = 0; j < a->n; ++j) {
    double y = a->p[j];
    if (fabs(x) < fabs(y)) {
      double t = x;
      x = y;
      y = t;
    }
    double hi = x + y;
    double lo = y - (hi - x);
    if (lo != 0.0) a->p[k++] = lo;
    x = hi;
  }
  if (k == a->cap) {
    a->cap = a->cap ? 2 * a->cap : 8;
    a->p = realloc(a->p, sizeof(double) * a->cap);
  }
  a->p[k++] = x;
  a->n = k;
}

static double xsum_value(const xsum *a) {
  int n = a->n;
  if (n == 0) return 0.0;
  double hi = a->p[--n], lo = 0.0;
  while (n > 0) {
    double x = hi, y = a->p[--n];
    hi = x + y;
    lo = y - (hi - x);
    if (lo != 0.0) break;
  }
  /* the partials left below lo push a half-way result up or down */
  if (n > 0 && ((lo < 0.0 && a->p[n - 1] < 0.0) || (lo > 0.0 && a->p[n - 1] > 0.0))) {
    double y = lo * 2.0;
    double x = hi + y;
    if (y == x - hi) hi = x;
  }
  return hi;
}

static void xsum_free(xsum *a) {
  free(a->p);
  a->p = NULL;
  a->n = a->cap = 0;
}

double orc_fsum(const double *v, int64_t n) {
  xsum a = {0};
  for (int64_t k = 0; k < n; ++k) xsum_add(&a, v[k]);
  double r = xsum_value(&a);
  xsum_free(&a);
  return r;
}

struct part {
  int32_t bubble; /* index into the old bubble table */
  xsum vol;       /* gas volume of the bubble's cells in the component */
  int64_t ncell;
};

struct orc {
  orc_params P;
  int64_t N;
  /* state at time t */
  uint8_t *type;
  double *f;   /* post-collision PDFs [19][N], meaningful on I and L cells */
  double *m;   /* mass: I cells m, L cells rho */
  double *phi; /* fill level: G/IN 0, L 1, I m/rho */
  int32_t *id; /* bubble ID on G, I, IN cells, -1 elsewhere */
  double *rho; /* density of the last collision */
  double *u;   /* velocity of the last collision, [3][N] */
  /* bubbles */
  int32_t nb, cap;
  int32_t *b_id, *b_flags;
  double *b_vstar, *b_vol, *b_p;
  int64_t *b_ncell;
  int32_t next_id;
  double bucket;
  int64_t n_iface; /* number of interface cells at time t */
  int64_t step;
  double mass;
  int64_t n_topology;
  char err[256];
  /* phase outputs (time t+1) */
  uint8_t *type2;
  double *f2, *m2, *phi2, *rho2, *u2, *excess;
  int32_t *id2;
  uint8_t *filled, *emptied0, *emptied, *capped;
  int32_t *label;
};

static int g_threads = 1;
void orc_set_threads(int32_t n) { g_threads = n < 1 ? 1 : n; }
int32_t orc_threads(void) { return g_threads; }

/* ------------------------------------------------------------ geometry -- */

static int64_t cell_index(const orc *o, int x, int y, int z) {
  return (int64_t)x + (int64_t)o->P.nx * ((int64_t)y + (int64_t)o->P.ny * z);
}

static void cell_coords(const orc *o, int64_t i, int *x, int *y, int *z) {
  *x = (int)(i % o->P.nx);
  *y = (int)((i / o->P.nx) % o->P.ny);
  *z = (int)(i / ((int64_t)o->P.nx * o->P.ny));
}

static int wrap(int c, int n, int periodic) {
  if (!periodic) return c;
  c %= n;
  return c < 0 ? c + n : c;
}

/* Neighbour of i at offset (dx,dy,dz) with periodic wrap; -1 outside the
 * box on a non-periodic axis. */
static int64_t neighbour(const orc *o, int64_t i, int dx, int dy, int dz) {
  int x, y, z;
  cell_coords(o, i, &x, &y, &z);
  x = wrap(x + dx, o->P.nx, o->P.periodic[0]);
  y = wrap(y + dy, o->P.ny, o->P.periodic[1]);
  z = wrap(z + dz, o->P.nz, o->P.periodic[2]);
  if (x < 0 || x >= o->P.nx || y < 0 || y >= o->P.ny || z < 0 || z >= o->P.nz) return -1;
  return cell_index(o, x, y, z);
}

static int in_gas_region(uint8_t t) { return t == ORC_G || t == ORC_I || t == ORC_IN; }

/* ---------------------------------------------------------- equilibrium -- */

/* Second-order equilibrium of Sec. 2.1 with cs^2 = 1/3. */
void orc_feq(double rho, const double *u, double *out) {
  const double cs2 = 1.0 / 3.0;
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int a = 0; a < Q; ++a) {
    double cu = CX[a] * u[0] + CY[a] * u[1] + CZ[a] * u[2];
    out[a] = rho * weight(a) * (1.0 + cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

void orc_lattice(int32_t *c, double *w, int32_t *opp) {
  for (int a = 0; a < Q; ++a) {
    c[3 * a] = CX[a];
    c[3 * a + 1] = CY[a];
    c[3 * a + 2] = CZ[a];
    w[a] = weight(a);
    opp[a] = opposite(a);
  }
}

/* Collision of Sec. 2.1: f~ = f - omega (f - f_eq(rho, u)) with moments
 * rho = sum f, rho u = sum c f.  The body force (only g is given, Sec. 3.2)
 * enters by the Guo scheme: u = (sum c f + rho g / 2) / rho and the source
 * (1 - omega/2) w [3 (c - u) + 9 (c.u) c] . rho g.  TRT splits the
 * relaxation into even and odd parts with omega- from the magic parameter. */
void orc_collide(const orc_params *p, const double *fin, double *fout, double *rho_out,
                 double *u_out) {
  double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int a = 0; a < Q; ++a) {
    rho += fin[a];
    jx += CX[a] * fin[a];
    jy += CY[a] * fin[a];
    jz += CZ[a] * fin[a];
  }
  double u[3];
  u[0] = (jx + 0.5 * rho * p->g[0]) / rho;
  u[1] = (jy + 0.5 * rho * p->g[1]) / rho;
  u[2] = (jz + 0.5 * rho * p->g[2]) / rho;
  double feq[Q];
  orc_feq(rho, u, feq);
  double wp = 1.0 / p->tau;
  double wm = wp;
  if (p->collision == 1) wm = 1.0 / (0.5 + p->trt_lambda / (1.0 / wp - 0.5));
  double Fx = rho * p->g[0], Fy = rho * p->g[1], Fz = rho * p->g[2];
  double uF = u[0] * Fx + u[1] * Fy + u[2] * Fz;
  for (int a = 0; a < Q; ++a) {
    int b = opposite(a);
    double cu = CX[a] * u[0] + CY[a] * u[1] + CZ[a] * u[2];
    double cF = CX[a] * Fx + CY[a] * Fy + CZ[a] * Fz;
    double s_even = weight(a) * (-3.0 * uF + 9.0 * cu * cF);
    double s_odd = weight(a) * (3.0 * cF);
    double f_even = 0.5 * (fin[a] + fin[b]), f_odd = 0.5 * (fin[a] - fin[b]);
    double e_even = 0.5 * (feq[a] + feq[b]), e_odd = 0.5 * (feq[a] - feq[b]);
    fout[a] = fin[a] - wp * (f_even - e_even) - wm * (f_odd - e_odd) +
              (1.0 - 0.5 * wp) * s_even + (1.0 - 0.5 * wm) * s_odd;
  }
  *rho_out = rho;
  u_out[0] = u[0];
  u_out[1] = u[1];
  u_out[2] = u[2];
}

/* Velocity at the free boundary (Sec. 2.2: the gas-side equilibrium uses
 * the current velocity at the boundary): the cell's own last collision
 * velocity, recovered from its post-collision PDFs f*.  Under the Guo
 * scheme the collision adds rho g to the momentum, sum c f* = rho u +
 * rho g / 2 with u the collision velocity, so u = sum c f* / rho - g / 2. */
void orc_boundary_velocity(const orc_params *p, const double *fs, double *ub) {
  double r = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < Q; ++a) {
    r += fs[a];
    j[0] += CX[a] * fs[a];
    j[1] += CY[a] * fs[a];
    j[2] += CZ[a] * fs[a];
  }
  for (int k = 0; k < 3; ++k) ub[k] = j[k] / r - 0.5 * p->g[k];
}

/* ------------------------------------------------- normals and curvature -- */

/* Fill level seen by the interface geometry at integer position (x,y,z):
 * periodic axes wrap; a sample on a wall cell or outside the box takes the
 * fill level of its mirror image across the wall plane (wall planes lie
 * half-way between the wall layer and the first fluid layer). */
static double phi_sample(const orc *o, const double *phi, const uint8_t *type, int x, int y,
                         int z) {
  int n[3] = {o->P.nx, o->P.ny, o->P.nz};
  int c[3] = {x, y, z};
  for (int k = 0; k < 3; ++k) c[k] = wrap(c[k], n[k], o->P.periodic[k]);
  int inside = 1;
  for (int k = 0; k < 3; ++k)
    if (c[k] < 0 || c[k] >= n[k]) inside = 0;
  if (inside && type[cell_index(o, c[0], c[1], c[2])] != ORC_W)
    return phi[cell_index(o, c[0], c[1], c[2])];
  for (int k = 0; k < 3; ++k) {
    if (o->P.periodic[k]) continue;
    if (c[k] <= 0) c[k] = 1 - c[k];
    else if (c[k] >= n[k] - 1) c[k] = 2 * n[k] - 3 - c[k];
  }
  return phi[cell_index(o, c[0], c[1], c[2])];
}

/* Interface normal by the Parker-Youngs gradient (Sec. 2.2 cites Parker &
 * Youngs): central differences of the fill level weighted 4/2/1 for face,
 * edge and corner offsets.  Points from gas into liquid. */
static void youngs_normal(const orc *o, const double *phi, const uint8_t *type, int x, int y,
                          int z, double *n) {
  static const double aw[3] = {1.0, 2.0, 1.0};
  n[0] = n[1] = n[2] = 0.0;
  for (int p = -1; p <= 1; ++p)
    for (int q = -1; q <= 1; ++q) {
      double w = aw[p + 1] * aw[q + 1];
      n[0] += w * (phi_sample(o, phi, type, x + 1, y + p, z + q) -
                   phi_sample(o, phi, type, x - 1, y + p, z + q));
      n[1] += w * (phi_sample(o, phi, type, x + p, y + 1, z + q) -
                   phi_sample(o, phi, type, x + p, y - 1, z + q));
      n[2] += w * (phi_sample(o, phi, type, x + p, y + q, z + 1) -
                   phi_sample(o, phi, type, x + p, y + q, z - 1));
    }
}

/* Relative width of a tie: decisions between quantities that are equal
 * in exact arithmetic (axes of a symmetric interface, directions tangent to
 * it) must not depend on round-off. */
#define TIE_REL 1e-10

/* cot of the static contact angle: 0 for the neutral angle (90 degrees,
 * also selected by 0) so that the wall rule is then exactly the mirror. */
static double wall_cot(const orc_params *p) {
  double t = p->contact_angle;
  if (t == 0.0 || t == 90.0) return 0.0;
  double r = t * (3.14159265358979323846 / 180.0);
  return cos(r) / sin(r);
}

/* Number of footprint axes (e1, e2) along which the column through
 * footprint cell c (its own position along d) lies in a wall: the cell is a
 * wall (or outside the box) and the coordinate is on a face layer of a
 * non-periodic axis. */
static int ghost_axes(const orc *o, const uint8_t *type, const int *c, int e1, int e2) {
  int n[3] = {o->P.nx, o->P.ny, o->P.nz};
  int w[3];
  int inside = 1;
  for (int k = 0; k < 3; ++k) {
    w[k] = wrap(c[k], n[k], o->P.periodic[k]);
    if (w[k] < 0 || w[k] >= n[k]) inside = 0;
  }
  if (inside && type[cell_index(o, w[0], w[1], w[2])] != ORC_W) return 0;
  int m = 0;
  if (!o->P.periodic[e1] && (w[e1] <= 0 || w[e1] >= n[e1] - 1)) ++m;
  if (!o->P.periodic[e2] && (w[e2] <= 0 || w[e2] >= n[e2] - 1)) ++m;
  return m;
}

/* Height-function curvature using columns along axis d: columns of 7 fill
 * levels over the 3x3 footprint in the plane of the other two axes give
 * liquid heights H(a,b); kappa follows from their first and second central
 * differences.  kappa > 0 where the liquid is convex (a droplet), < 0 for a
 * bubble; the formula holds for liquid on either side since H counts
 * liquid.
 * Wetting (Sec. 3.2; the paper's model is in a reference that is not
 * available): a column whose footprint lies in a wall is a ghost column.
 * Where the interface meets the wall at the static angle theta (measured in
 * the liquid), the liquid height of a column parallel to the wall grows by
 * cot(theta) per cell towards the wall, whichever side the liquid is on, so
 * the ghost column takes the mirrored column's height plus cot(theta) per
 * wall axis crossed (ghost heights from the contact angle, as in height-
 * function contact-angle methods for VOF).  theta = 90 degrees leaves the
 * mirror. */
static double height_curvature_axis(const orc *o, const double *phi, const uint8_t *type, int x,
                                    int y, int z, int d) {
  int e1 = (d == 0) ? 1 : 0;
  int e2 = (d == 2) ? 1 : 2;
  const double cot = wall_cot(&o->P);
  double H[3][3];
  for (int a = -1; a <= 1; ++a)
    for (int b = -1; b <= 1; ++b) {
      double s = 0.0;
      for (int k = -3; k <= 3; ++k) {
        int c[3] = {x, y, z};
        c[e1] += a;
        c[e2] += b;
        c[d] += k;
        s += phi_sample(o, phi, type, c[0], c[1], c[2]);
      }
      if (cot != 0.0) {
        int c[3] = {x, y, z};
        c[e1] += a;
        c[e2] += b;
        const int m = ghost_axes(o, type, c, e1, e2);
        if (m) s += m * cot;
      }
      H[a + 1][b + 1] = s;
    }
  double Ha = 0.5 * (H[2][1] - H[0][1]);
  double Hb = 0.5 * (H[1][2] - H[1][0]);
  double Haa = H[2][1] - 2.0 * H[1][1] + H[0][1];
  double Hbb = H[1][2] - 2.0 * H[1][1] + H[1][0];
  double Hab = 0.25 * (H[2][2] - H[2][0] - H[0][2] + H[0][0]);
  double num = Haa * (1.0 + Hb * Hb) + Hbb * (1.0 + Ha * Ha) - 2.0 * Ha * Hb * Hab;
  double q = 1.0 + Ha * Ha + Hb * Hb;
  double den = q * sqrt(q);
  return -0.5 * num / den;
}

/* Mean curvature kappa of the interface through cell (x,y,z) (Sec. 2.2,
 * Laplace pressure 2 sigma kappa).  The paper's triangulation is described
 * only in a reference that is not available; this is the height-function
 * estimate along the dominant axis of the normal.  Axes whose |n_i| lies
 * within a relative TIE_REL of the largest one are tied, and kappa is the
 * mean of their estimates (in the order x, y, z). */
static double height_curvature(const orc *o, const double *phi, const uint8_t *type, int x,
                               int y, int z, const double *n) {
  double an[3] = {fabs(n[0]), fabs(n[1]), fabs(n[2])};
  double m = an[0];
  if (an[1] > m) m = an[1];
  if (an[2] > m) m = an[2];
  if (m == 0.0) return 0.0;
  double thr = m - TIE_REL * m;
  double sum = 0.0;
  int cnt = 0;
  for (int d = 0; d < 3; ++d)
    if (an[d] >= thr) {
      sum += height_curvature_axis(o, phi, type, x, y, z, d);
      ++cnt;
    }
  return sum / cnt;
}

void orc_geometry(const orc *o, double *kappa, double *normal) {
  for (int64_t i = 0; i < o->N; ++i) {
    double n[3] = {0.0, 0.0, 0.0}, k = 0.0;
    if (o->type[i] == ORC_I) {
      int x, y, z;
      cell_coords(o, i, &x, &y, &z);
      youngs_normal(o, o->phi, o->type, x, y, z, n);
      k = height_curvature(o, o->phi, o->type, x, y, z, n);
    }
    if (kappa) kappa[i] = k;
    if (normal) {
      normal[i] = n[0];
      normal[o->N + i] = n[1];
      normal[2 * o->N + i] = n[2];
    }
  }
}

/* ------------------------------------------------------------- bubbles -- */

static int32_t bubble_index(const orc *o, int32_t id) {
  for (int32_t k = 0; k < o->nb; ++k)
    if (o->b_id[k] == id) return k;
  return -1;
}

static void bubbles_reserve(orc *o, int32_t n) {
  if (n <= o->cap) return;
  int32_t c = o->cap ? o->cap : 8;
  while (c < n) c *= 2;
  o->b_id = realloc(o->b_id, sizeof(int32_t) * c);
  o->b_flags = realloc(o->b_flags, sizeof(int32_t) * c);
  o->b_vstar = realloc(o->b_vstar, sizeof(double) * c);
  o->b_vol = realloc(o->b_vol, sizeof(double) * c);
  o->b_p = realloc(o->b_p, sizeof(double) * c);
  o->b_ncell = realloc(o->b_ncell, sizeof(int64_t) * c);
  o->cap = c;
}

/* Bubble volume (Sec. 2.3): gas cells count fully, interface cells by their
 * empty fraction 1 - phi (the accumulation rule of Sec. 2.3.2). */
static double cell_gas_volume(uint8_t t, double phi) {
  if (t == ORC_G || t == ORC_IN) return 1.0;
  if (t == ORC_I) return 1.0 - phi;
  return 0.0;
}

/* Ideal-gas pressure (Sec. 2.2): p = V* / V p0; the volume is floored at
 * 1e-2 for vanishing bubbles.  An atmosphere bubble stays at p0. */
static double bubble_pressure(double p0, int32_t flags, double vstar, double vol) {
  if (flags & ORC_BUBBLE_ATMOSPHERE) return p0;
  double v = vol > 1e-2 ? vol : 1e-2;
  return p0 * vstar / v;
}

/* ----------------------------------------------------------- labelling -- */

/* Connected components by breadth-first flood fill (Sec. 2.3.2), visiting
 * seeds in increasing index so that each label is its component's smallest
 * index. */
void orc_label(int32_t nx, int32_t ny, int32_t nz, const int32_t *periodic,
               const uint8_t *inset, int32_t *label) {
  int64_t N = (int64_t)nx * ny * nz;
  int64_t *queue = malloc(sizeof(int64_t) * (N > 0 ? N : 1));
  for (int64_t i = 0; i < N; ++i) label[i] = -1;
  for (int64_t s = 0; s < N; ++s) {
    if (!inset[s] || label[s] >= 0) continue;
    int64_t head = 0, tail = 0;
    queue[tail++] = s;
    label[s] = (int32_t)s;
    while (head < tail) {
      int64_t c = queue[head++];
      int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
      for (int a = 1; a < Q; ++a) {
        int xx = wrap(x + CX[a], nx, periodic[0]);
        int yy = wrap(y + CY[a], ny, periodic[1]);
        int zz = wrap(z + CZ[a], nz, periodic[2]);
        if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) continue;
        int64_t j = (int64_t)xx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * zz);
        if (inset[j] && label[j] < 0) {
          label[j] = (int32_t)s;
          queue[tail++] = j;
        }
      }
    }
  }
  free(queue);
}

/* -------------------------------------------------------------- create -- */

static void set_err(char *err, int32_t len, const char *msg) {
  if (err && len > 0) snprintf(err, (size_t)len, "%s", msg);
}

static void compute_mass(orc *o) {
  xsum M = {0};
  for (int64_t i = 0; i < o->N; ++i)
    if (o->type[i] == ORC_L || o->type[i] == ORC_I) xsum_add(&M, o->m[i]);
  xsum_add(&M, o->bucket);
  o->mass = xsum_value(&M);
  xsum_free(&M);
}

orc *orc_create(const orc_params *p, const uint8_t *type, const double *phi, const double *rho,
                const double *u, const int32_t *id, const int32_t *b_id, const int32_t *b_flags,
                const double *b_vstar, const double *b_pinit, int32_t nb, const double *f_init,
                const double *mass_init, int64_t step0, int32_t next_id0, double bucket0,
                char *err, int32_t errlen) {
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0 || p->tau <= 0.5) {
    set_err(err, errlen, "bad sizes or tau");
    return NULL;
  }
  orc *o = calloc(1, sizeof(orc));
  o->P = *p;
  int64_t N = (int64_t)p->nx * p->ny * p->nz;
  o->N = N;
  o->type = malloc(N);
  o->type2 = malloc(N);
  o->filled = malloc(N);
  o->emptied0 = malloc(N);
  o->emptied = malloc(N);
  o->capped = malloc(N);
  o->f = malloc(sizeof(double) * Q * N);
  o->f2 = malloc(sizeof(double) * Q * N);
  o->m = malloc(sizeof(double) * N);
  o->m2 = malloc(sizeof(double) * N);
  o->phi = malloc(sizeof(double) * N);
  o->phi2 = malloc(sizeof(double) * N);
  o->rho = malloc(sizeof(double) * N);
  o->rho2 = malloc(sizeof(double) * N);
  o->u = malloc(sizeof(double) * 3 * N);
  o->u2 = malloc(sizeof(double) * 3 * N);
  o->excess = malloc(sizeof(double) * N);
  o->id = malloc(sizeof(int32_t) * N);
  o->id2 = malloc(sizeof(int32_t) * N);
  o->label = malloc(sizeof(int32_t) * N);
  char msg[200];
  int n[3] = {p->nx, p->ny, p->nz};
  for (int64_t i = 0; i < N; ++i) {
    int c[3];
    cell_coords(o, i, &c[0], &c[1], &c[2]);
    uint8_t t = type[i];
    if (t > ORC_IN) {
      snprintf(msg, sizeof msg, "cell %lld: bad type %d", (long long)i, t);
      goto fail;
    }
    int face = 0;
    for (int k = 0; k < 3; ++k)
      if (!p->periodic[k] && (c[k] == 0 || c[k] == n[k] - 1)) face = 1;
    if (face && t != ORC_W && t != ORC_IN) {
      snprintf(msg, sizeof msg, "cell %lld: non-periodic face layer must be wall or inlet",
               (long long)i);
      goto fail;
    }
    if (!face && t == ORC_W) {
      snprintf(msg, sizeof msg, "cell %lld: walls only on non-periodic face layers", (long long)i);
      goto fail;
    }
    o->type[i] = t;
    if (t == ORC_I && !isfinite(phi[i])) {
      snprintf(msg, sizeof msg, "cell %lld: interface fill level not finite", (long long)i);
      goto fail;
    }
    if ((t == ORC_I || t == ORC_L) && !(rho[i] > 0.0)) {
      snprintf(msg, sizeof msg, "cell %lld: density must be positive", (long long)i);
      goto fail;
    }
    o->phi[i] = (t == ORC_I) ? phi[i] : (t == ORC_L ? 1.0 : 0.0);
    o->rho[i] = (t == ORC_I || t == ORC_L) ? rho[i] : 0.0;
    for (int k = 0; k < 3; ++k) o->u[k * N + i] = (t == ORC_I || t == ORC_L) ? u[k * N + i] : 0.0;
    o->id[i] = in_gas_region(t) ? id[i] : -1;
  }
  /* closed interface layer and consistent IDs */
  for (int64_t i = 0; i < N; ++i) {
    for (int a = 1; a < Q; ++a) {
      int64_t j = neighbour(o, i, CX[a], CY[a], CZ[a]);
      if (j < 0) continue;
      if (o->type[i] == ORC_L && (o->type[j] == ORC_G || o->type[j] == ORC_IN)) {
        snprintf(msg, sizeof msg, "cell %lld: liquid next to gas", (long long)i);
        goto fail;
      }
      if (in_gas_region(o->type[i]) && in_gas_region(o->type[j]) && o->id[i] != o->id[j]) {
        snprintf(msg, sizeof msg, "cells %lld/%lld: touching gas cells with different IDs",
                 (long long)i, (long long)j);
        goto fail;
      }
    }
  }
  /* bubble table */
  bubbles_reserve(o, nb > 0 ? nb : 1);
  o->nb = nb;
  int32_t maxid = -1;
  for (int32_t k = 0; k < nb; ++k) {
    o->b_id[k] = b_id[k];
    o->b_flags[k] = b_flags[k];
    o->b_vol[k] = 0.0;
    o->b_ncell[k] = 0;
    if (b_id[k] > maxid) maxid = b_id[k];
  }
  xsum *vacc = calloc((size_t)(nb > 0 ? nb : 1), sizeof(xsum));
  for (int64_t i = 0; i < N; ++i) {
    if (!in_gas_region(o->type[i])) continue;
    int32_t k = bubble_index(o, o->id[i]);
    if (k < 0) {
      snprintf(msg, sizeof msg, "cell %lld: bubble ID %d not listed", (long long)i, o->id[i]);
      for (int32_t q = 0; q < nb; ++q) xsum_free(&vacc[q]);
      free(vacc);
      goto fail;
    }
    xsum_add(&vacc[k], cell_gas_volume(o->type[i], o->phi[i]));
    o->b_ncell[k] += 1;
  }
  for (int32_t k = 0; k < nb; ++k) {
    o->b_vol[k] = xsum_value(&vacc[k]);
    xsum_free(&vacc[k]);
  }
  free(vacc);
  for (int32_t k = 0; k < nb; ++k) {
    o->b_vstar[k] = b_vstar[k] > 0.0 ? b_vstar[k] : o->b_vol[k] * b_pinit[k] / p->p0;
    o->b_p[k] = bubble_pressure(p->p0, o->b_flags[k], o->b_vstar[k], o->b_vol[k]);
  }
  o->next_id = next_id0 > maxid ? next_id0 : maxid + 1;
  o->step = step0;
  o->bucket = bucket0;
  /* PDFs and masses */
  o->n_iface = 0;
  for (int64_t i = 0; i < N; ++i) {
    uint8_t t = o->type[i];
    if (t == ORC_I || t == ORC_L) {
      double fe[Q], uu[3] = {o->u[i], o->u[N + i], o->u[2 * N + i]};
      orc_feq(o->rho[i], uu, fe);
      for (int a = 0; a < Q; ++a) o->f[a * N + i] = f_init ? f_init[a * N + i] : fe[a];
    } else {
      for (int a = 0; a < Q; ++a) o->f[a * N + i] = 0.0;
    }
    if (t == ORC_I) {
      /* m = phi rho (Sec. 2.2), or the mass of a saved state */
      o->m[i] = mass_init ? mass_init[i] : o->phi[i] * o->rho[i];
      o->n_iface += 1;
    } else if (t == ORC_L) {
      o->m[i] = o->rho[i];
    } else {
      o->m[i] = 0.0;
    }
  }
  compute_mass(o);
  return o;
fail:
  set_err(err, errlen, msg);
  orc_destroy(o);
  return NULL;
}

void orc_destroy(orc *o) {
  if (!o) return;
  void *ptrs[] = {o->type, o->type2, o->filled, o->emptied0, o->emptied, o->capped, o->f, o->f2, o->m,
                  o->m2, o->phi, o->phi2, o->rho, o->rho2, o->u, o->u2, o->excess, o->id,
                  o->id2, o->label, o->b_id, o->b_flags, o->b_vstar, o->b_vol, o->b_p,
                  o->b_ncell};
  for (size_t k = 0; k < sizeof ptrs / sizeof ptrs[0]; ++k) free(ptrs[k]);
  free(o);
}

const char *orc_error(const orc *o) { return o->err; }

/* ------------------------------------------------------------- phase A -- */

/* Stream, reconstruct, exchange mass and collide one interface or liquid
 * cell i, reading only the state at time t. */
static void phase_a_cell(orc *o, int64_t i, double bucket_share) {
  const int64_t N = o->N;
  const uint8_t t = o->type[i];
  double fs[Q]; /* own post-collision values f*(x, t) */
  for (int a = 0; a < Q; ++a) fs[a] = o->f[a * N + i];

  /* Interface geometry and gas-side equilibrium (Sec. 2.2). */
  double n[3] = {0.0, 0.0, 0.0};
  double feq_gas[Q];
  if (t == ORC_I) {
    int x, y, z;
    cell_coords(o, i, &x, &y, &z);
    youngs_normal(o, o->phi, o->type, x, y, z, n);
    double kappa = height_curvature(o, o->phi, o->type, x, y, z, n);
    int32_t b = bubble_index(o, o->id[i]);
    double p_gas = o->b_p[b] + 2.0 * o->P.sigma * kappa; /* p_V + 2 sigma kappa */
    double rho_gas = 3.0 * p_gas;                        /* p = rho cs^2 */
    double ub[3];
    orc_boundary_velocity(&o->P, fs, ub);
    orc_feq(rho_gas, ub, feq_gas);
  }

  /* Pull streaming (Sec. 2.1) with half-way bounce-back at walls and the
   * free-surface reconstruction f_a = f_a^gas + f_abar^gas - f*_abar(x). */
  double fin[Q];
  fin[0] = fs[0];
  for (int a = 1; a < Q; ++a) {
    int b = opposite(a);
    int64_t s = neighbour(o, i, -CX[a], -CY[a], -CZ[a]);
    uint8_t ts = s >= 0 ? o->type[s] : (uint8_t)ORC_W; /* fluid cells are interior */
    double recon = (t == ORC_I) ? feq_gas[a] + feq_gas[b] - fs[b] : 0.0;
    if (ts == ORC_W) {
      fin[a] = fs[b];
    } else if (ts == ORC_G || ts == ORC_IN) {
      fin[a] = recon; /* missing PDF from the gas side */
    } else {
      fin[a] = o->f[a * N + s];
      /* moving from the gas side into the liquid, beyond a tie band
       * around the tangent plane */
      double cn = CX[a] * n[0] + CY[a] * n[1] + CZ[a] * n[2];
      double nn = fabs(n[0]) + fabs(n[1]) + fabs(n[2]);
      if (t == ORC_I && cn > TIE_REL * nn) fin[a] = recon;
    }
  }

  /* Mass exchange of interface cells with their neighbours (Sec. 2.2):
   * liquid neighbours exchange the full PDF difference, interface
   * neighbours weighted by the mean fill level, gas (and wall, inlet)
   * neighbours nothing. */
  double m_new = o->m[i];
  if (t == ORC_I) {
    double dm = 0.0;
    for (int a = 1; a < Q; ++a) {
      int b = opposite(a);
      int64_t y = neighbour(o, i, CX[a], CY[a], CZ[a]);
      uint8_t ty = y >= 0 ? o->type[y] : (uint8_t)ORC_W;
      double diff = (ty == ORC_L || ty == ORC_I) ? o->f[b * N + y] - fs[a] : 0.0;
      if (ty == ORC_L) dm += diff;
      else if (ty == ORC_I) dm += 0.5 * (o->phi[i] + o->phi[y]) * diff;
    }
    m_new = o->m[i] + dm + bucket_share;
  }

  double fout[Q], rho, u[3];
  orc_collide(&o->P, fin, fout, &rho, u);
  for (int a = 0; a < Q; ++a) o->f2[a * N + i] = fout[a];
  o->rho2[i] = rho;
  for (int k = 0; k < 3; ++k) o->u2[k * N + i] = u[k];
  if (t == ORC_I) {
    o->m2[i] = m_new;
    o->phi2[i] = m_new / rho; /* phi = m / rho */
  } else {
    o->m2[i] = rho;
    o->phi2[i] = 1.0;
  }
}

/* -------------------------------------------------------- phases B - D -- */

static int any_neighbour_flag(const orc *o, int64_t i, const uint8_t *flag) {
  for (int a = 1; a < Q; ++a) {
    int64_t j = neighbour(o, i, CX[a], CY[a], CZ[a]);
    if (j >= 0 && flag[j]) return 1;
  }
  return 0;
}

static int any_neighbour_type(const orc *o, int64_t i, uint8_t t) {
  for (int a = 1; a < Q; ++a) {
    int64_t j = neighbour(o, i, CX[a], CY[a], CZ[a]);
    if (j >= 0 && o->type[j] == t) return 1;
  }
  return 0;
}

/* ------------------------------------------------------------- phase F -- */

struct comp {
  int64_t root;
  int32_t *ids; /* distinct old bubbles (table indices) in the component */
  int32_t nids, cap;
  xsum vol, vstar;
  int inlet, atmosphere;
  int64_t ncell;
};

static void comp_note(struct comp *c, int32_t b) {
  for (int32_t k = 0; k < c->nids; ++k)
    if (c->ids[k] == b) return;
  if (c->nids == c->cap) {
    c->cap = c->cap ? 2 * c->cap : 4;
    c->ids = realloc(c->ids, sizeof(int32_t) * c->cap);
  }
  c->ids[c->nids++] = b;
}

/* Merge (Sec. 2.3.1) and split (Sec. 2.3.2) through one canonical rule on
 * the connected components K of the gas region:
 *  - K keeps the ID b if b is the only bubble in K and K the only
 *    component of b;
 *  - otherwise K becomes a new bubble with a fresh ID (in order of K's
 *    smallest cell index) whose volume is the gas volume of its cells and
 *    whose gas amount V* is carried by its cells: each cell of an old bubble
 *    b brings V*_b / V_b times its gas volume (per cell V*_b / n_b if
 *    V_b <= 0), i.e. V*_K = sum_b V*_b V(b in K) / V_b.
 * For a pure merge this gives V* = sum V*_b and V = sum V_b (Sec. 2.3.1);
 * for a pure split every daughter keeps the mother's pressure (Sec. 2.3.2).
 * K owns inlet cells if it holds one, and is an atmosphere if it holds
 * cells of an atmosphere bubble (a bubble that reaches the open top joins
 * it and takes its constant pressure).
 * Returns 1 if a new ID was created. */
static int phase_f(orc *o, const double *old_vol, const int64_t *old_ncell) {
  const int64_t N = o->N;
  uint8_t *inset = o->filled; /* reuse as a scratch mask */
  for (int64_t i = 0; i < N; ++i) inset[i] = (uint8_t)in_gas_region(o->type2[i]);
  orc_label(o->P.nx, o->P.ny, o->P.nz, o->P.periodic, inset, o->label);
  /* components in increasing order of their smallest index */
  int64_t ncomp = 0;
  for (int64_t i = 0; i < N; ++i)
    if (o->label[i] == i) ++ncomp;
  struct comp *comps = calloc((size_t)(ncomp > 0 ? ncomp : 1), sizeof(struct comp));
  int64_t *root_to_comp = malloc(sizeof(int64_t) * (N > 0 ? N : 1));
  int64_t k = 0;
  for (int64_t i = 0; i < N; ++i)
    if (o->label[i] == i) {
      comps[k].root = i;
      root_to_comp[i] = k;
      ++k;
    }
  /* gas amount per unit gas volume of every old bubble */
  double *ratio = calloc((size_t)(o->nb > 0 ? o->nb : 1), sizeof(double));
  for (int32_t b = 0; b < o->nb; ++b)
    ratio[b] = old_vol[b] > 0.0 ? o->b_vstar[b] / old_vol[b] : 0.0;
  for (int64_t i = 0; i < N; ++i) {
    if (!inset[i]) continue;
    struct comp *c = &comps[root_to_comp[o->label[i]]];
    int32_t b = bubble_index(o, o->id2[i]);
    comp_note(c, b);
    double w = cell_gas_volume(o->type2[i], o->phi2[i]);
    xsum_add(&c->vol, w);
    xsum_add(&c->vstar, old_vol[b] > 0.0 ? ratio[b] * w : o->b_vstar[b] / (double)old_ncell[b]);
    c->ncell += 1;
    if (o->type2[i] == ORC_IN) c->inlet = 1;
    if (o->b_flags[b] & ORC_BUBBLE_ATMOSPHERE) c->atmosphere = 1;
  }
  /* number of components each old bubble appears in */
  int32_t *ncomp_of = calloc((size_t)(o->nb > 0 ? o->nb : 1), sizeof(int32_t));
  for (int64_t c = 0; c < ncomp; ++c)
    for (int32_t q = 0; q < comps[c].nids; ++q) ncomp_of[comps[c].ids[q]] += 1;
  /* new table */
  int32_t nb_new = (int32_t)ncomp;
  int32_t *nid = malloc(sizeof(int32_t) * (nb_new > 0 ? nb_new : 1));
  int32_t *nflags = malloc(sizeof(int32_t) * (nb_new > 0 ? nb_new : 1));
  double *nvstar = malloc(sizeof(double) * (nb_new > 0 ? nb_new : 1));
  double *nvol = malloc(sizeof(double) * (nb_new > 0 ? nb_new : 1));
  int64_t *nncell = malloc(sizeof(int64_t) * (nb_new > 0 ? nb_new : 1));
  int created = 0;
  for (int64_t c = 0; c < ncomp; ++c) {
    struct comp *K = &comps[c];
    int keep = (K->nids == 1) && (ncomp_of[K->ids[0]] == 1);
    if (keep) {
      int32_t b = K->ids[0];
      nid[c] = o->b_id[b];
      nvstar[c] = o->b_vstar[b];
      nvol[c] = old_vol[b];
    } else {
      nid[c] = o->next_id++;
      created = 1;
      nvstar[c] = xsum_value(&K->vstar);
      nvol[c] = xsum_value(&K->vol);
    }
    nflags[c] = (K->inlet ? ORC_BUBBLE_INLET : 0) | (K->atmosphere ? ORC_BUBBLE_ATMOSPHERE : 0);
    nncell[c] = K->ncell;
  }
  for (int64_t i = 0; i < N; ++i)
    if (inset[i]) o->id2[i] = nid[root_to_comp[o->label[i]]];
  /* install */
  bubbles_reserve(o, nb_new > 0 ? nb_new : 1);
  o->nb = nb_new;
  for (int32_t c = 0; c < nb_new; ++c) {
    o->b_id[c] = nid[c];
    o->b_flags[c] = nflags[c];
    o->b_vstar[c] = nvstar[c];
    o->b_vol[c] = nvol[c];
    o->b_ncell[c] = nncell[c];
  }
  for (int64_t c = 0; c < ncomp; ++c) {
    free(comps[c].ids);
    xsum_free(&comps[c].vol);
    xsum_free(&comps[c].vstar);
  }
  free(comps);
  free(root_to_comp);
  free(ratio);
  free(ncomp_of);
  free(nid);
  free(nflags);
  free(nvstar);
  free(nvol);
  free(nncell);
  return created;
}

/* Density and velocity of a cell recovered from its post-collision PDFs:
 * rho = sum f*, u = sum c f* / rho - g / 2 (the Guo collision velocity). */
static void recover_moments(const orc *o, const double *f, int64_t j, double *rho, double *u) {
  const int64_t N = o->N;
  double r = 0.0, m[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < Q; ++c) {
    double v = f[c * N + j];
    r += v;
    m[0] += CX[c] * v;
    m[1] += CY[c] * v;
    m[2] += CZ[c] * v;
  }
  *rho = r;
  for (int k = 0; k < 3; ++k) u[k] = m[k] / r - 0.5 * o->P.g[k];
}

/* ---------------------------------------------------------------- step -- */

static int one_step(orc *o) {
  const int64_t N = o->N;
  const double eps = o->P.eps;

  /* Phase A.  The orphan-mass bucket of the previous step is spread evenly
   * over the interface cells of time t. */
  double share = 0.0;
  if (o->n_iface > 0) {
    share = o->bucket / (double)o->n_iface;
    o->bucket = 0.0;
  }
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (int64_t i = 0; i < N; ++i) {
    uint8_t t = o->type[i];
    if (t == ORC_I || t == ORC_L) {
      phase_a_cell(o, i, share);
    } else {
      for (int a = 0; a < Q; ++a) o->f2[a * N + i] = 0.0;
      o->m2[i] = 0.0;
      o->phi2[i] = 0.0;
      o->rho2[i] = 0.0;
      o->u2[i] = o->u2[N + i] = o->u2[2 * N + i] = 0.0;
    }
  }

  /* Phase B: filled interface cells (phi > 1 + eps, never next to an
   * inlet), emptied interface cells (phi < -eps); an emptied cell next to
   * a filled one stays interface so that the layer stays closed.  An
   * interface cell that no longer separates liquid from gas is converted
   * whatever its fill level (the closed-layer rule of Sec. 2.2 read as in
   * the cited FSLBM of Koerner et al.): without a gas or inlet neighbour
   * it is filled, without a liquid neighbour it is emptied; filling wins
   * when both hold.  A cell next to an inlet never fills (the layer around
   * the inlet stays closed); above 1 + eps it is capped instead: it passes
   * the mass above m = rho on as excess (phase D) and stays interface, so
   * that its fill level, the liquid fraction of the cell, stays bounded. */
  for (int64_t i = 0; i < N; ++i) {
    o->filled[i] = 0;
    o->emptied0[i] = 0;
    o->capped[i] = 0;
    if (o->type[i] != ORC_I) continue;
    int near_in = any_neighbour_type(o, i, ORC_IN);
    int no_gas = !near_in && !any_neighbour_type(o, i, ORC_G);
    int no_liq = !any_neighbour_type(o, i, ORC_L);
    o->filled[i] = (uint8_t)(!near_in && (o->phi2[i] > 1.0 + eps || no_gas));
    o->emptied0[i] = (uint8_t)(o->phi2[i] < -eps || no_liq);
    o->capped[i] = (uint8_t)(near_in && o->phi2[i] > 1.0 + eps);
    if (o->P.freeze_conversions) /* fixed geometry */
      o->filled[i] = o->emptied0[i] = o->capped[i] = 0;
  }
  for (int64_t i = 0; i < N; ++i)
    o->emptied[i] = (uint8_t)(o->emptied0[i] && !o->filled[i] &&
                              !any_neighbour_flag(o, i, o->filled));
  for (int64_t i = 0; i < N; ++i)
    if (o->emptied[i]) o->capped[i] = 0;

  /* Phase C: new types.  Filled -> liquid, emptied -> gas, gas next to a
   * filled cell -> interface, liquid next to an emptied cell -> interface. */
  for (int64_t i = 0; i < N; ++i) {
    uint8_t t = o->type[i];
    uint8_t t2 = t;
    if (o->filled[i]) t2 = ORC_L;
    else if (o->emptied[i]) t2 = ORC_G;
    else if (t == ORC_G && any_neighbour_flag(o, i, o->filled)) t2 = ORC_I;
    else if (t == ORC_L && any_neighbour_flag(o, i, o->emptied)) t2 = ORC_I;
    o->type2[i] = t2;
    o->id2[i] = o->id[i];
  }
  for (int64_t i = 0; i < N; ++i) {
    uint8_t t = o->type[i], t2 = o->type2[i];
    if (t == ORC_G && t2 == ORC_I) {
      /* new interface cell from gas: equilibrium at the mean density and
       * velocity (recovered from the post-collision PDFs) of the neighbours
       * that were interface or liquid at t; empty; keeps its bubble ID */
      double rs = 0.0, us[3] = {0.0, 0.0, 0.0};
      int cnt = 0;
      for (int a = 1; a < Q; ++a) {
        int64_t j = neighbour(o, i, CX[a], CY[a], CZ[a]);
        if (j < 0 || !(o->type[j] == ORC_I || o->type[j] == ORC_L)) continue;
        double rj, uj[3];
        recover_moments(o, o->f2, j, &rj, uj);
        rs += rj;
        for (int k = 0; k < 3; ++k) us[k] += uj[k];
        ++cnt;
      }
      double rb = rs / cnt, ub[3] = {us[0] / cnt, us[1] / cnt, us[2] / cnt};
      double fe[Q];
      orc_feq(rb, ub, fe);
      for (int a = 0; a < Q; ++a) o->f2[a * N + i] = fe[a];
      o->rho2[i] = rb;
      for (int k = 0; k < 3; ++k) o->u2[k * N + i] = ub[k];
      o->m2[i] = 0.0;
    } else if (t == ORC_L && t2 == ORC_I) {
      /* new interface cell from liquid: full (m = rho recovered from its
       * post-collision PDFs), ID of the smallest emptied neighbour ID */
      double rr, uu[3];
      recover_moments(o, o->f2, i, &rr, uu);
      o->m2[i] = rr;
      o->rho2[i] = rr;
      int32_t best = -1;
      for (int a = 1; a < Q; ++a) {
        int64_t j = neighbour(o, i, CX[a], CY[a], CZ[a]);
        if (j >= 0 && o->emptied[j] && (best < 0 || o->id[j] < best)) best = o->id[j];
      }
      o->id2[i] = best;
    } else if (t == ORC_I && t2 == ORC_L) {
      o->id2[i] = -1;
    }
  }

  /* Phase D: excess mass.  A filled (or capped) cell keeps m = rho and
   * passes on m - rho; an emptied cell passes on its whole mass.  The
   * excess is split evenly over the neighbours that are interface cells
   * after the conversion and not capped (a capped cell neither receives
   * excess nor keeps it); without such a neighbour it goes to the bucket. */
  xsum bucket = {0};
  xsum_add(&bucket, o->bucket); /* carried if there was no interface cell */
  for (int64_t i = 0; i < N; ++i) {
    o->excess[i] = 0.0;
    if (!(o->filled[i] || o->emptied[i] || o->capped[i])) continue;
    double e;
    if (o->filled[i] || o->capped[i]) {
      e = o->m2[i] - o->rho2[i];
      o->m2[i] = o->rho2[i];
    } else {
      e = o->m2[i];
      o->m2[i] = 0.0;
    }
    int nI = 0;
    for (int a = 1; a < Q; ++a) {
      int64_t j = neighbour(o, i, CX[a], CY[a], CZ[a]);
      if (j >= 0 && o->type2[j] == ORC_I && !o->capped[j]) ++nI;
    }
    if (nI > 0) o->excess[i] = e / nI;
    else xsum_add(&bucket, e);
  }
  o->bucket = xsum_value(&bucket);
  xsum_free(&bucket);
  for (int64_t i = 0; i < N; ++i) {
    uint8_t t2 = o->type2[i];
    if (t2 == ORC_I) {
      double add = 0.0;
      int touched = 0;
      for (int a = 1; a < Q && !o->capped[i]; ++a) {
        int64_t j = neighbour(o, i, CX[a], CY[a], CZ[a]);
        if (j >= 0 && (o->filled[j] || o->emptied[j] || o->capped[j])) {
          add += o->excess[j];
          touched = 1;
        }
      }
      if (touched) o->m2[i] += add;
      o->phi2[i] = o->m2[i] / o->rho2[i];
    } else if (t2 == ORC_L) {
      o->phi2[i] = 1.0;
    } else {
      o->phi2[i] = 0.0;
    }
    if (t2 == ORC_G || t2 == ORC_IN || t2 == ORC_W) o->m2[i] = 0.0;
  }

  /* Phase E: volumes of the old bubbles on the new state. */
  double *old_vol = calloc((size_t)(o->nb > 0 ? o->nb : 1), sizeof(double));
  int64_t *old_ncell = calloc((size_t)(o->nb > 0 ? o->nb : 1), sizeof(int64_t));
  xsum *vacc = calloc((size_t)(o->nb > 0 ? o->nb : 1), sizeof(xsum));
  int bad = 0;
  for (int64_t i = 0; i < N && !bad; ++i) {
    if (!in_gas_region(o->type2[i])) continue;
    int32_t b = bubble_index(o, o->id2[i]);
    if (b < 0) {
      snprintf(o->err, sizeof o->err, "step %lld: cell %lld has no bubble", (long long)o->step,
               (long long)i);
      bad = 1;
      break;
    }
    xsum_add(&vacc[b], cell_gas_volume(o->type2[i], o->phi2[i]));
    old_ncell[b] += 1;
  }
  for (int32_t b = 0; b < o->nb; ++b) {
    old_vol[b] = xsum_value(&vacc[b]);
    xsum_free(&vacc[b]);
  }
  free(vacc);
  if (bad) {
    free(old_vol);
    free(old_ncell);
    return -1;
  }

  /* Phase F: topology every step. */
  if (phase_f(o, old_vol, old_ncell)) o->n_topology += 1;
  free(old_vol);
  free(old_ncell);

  /* Phase G: injection and ideal-gas pressure. */
  for (int32_t b = 0; b < o->nb; ++b) {
    if (o->b_flags[b] & ORC_BUBBLE_INLET) o->b_vstar[b] += o->P.inject_rate;
    o->b_p[b] = bubble_pressure(o->P.p0, o->b_flags[b], o->b_vstar[b], o->b_vol[b]);
  }

  /* commit t+1 */
  uint8_t *tt = o->type; o->type = o->type2; o->type2 = tt;
  double *tf = o->f; o->f = o->f2; o->f2 = tf;
  double *tm = o->m; o->m = o->m2; o->m2 = tm;
  double *tp = o->phi; o->phi = o->phi2; o->phi2 = tp;
  double *tr = o->rho; o->rho = o->rho2; o->rho2 = tr;
  double *tu = o->u; o->u = o->u2; o->u2 = tu;
  int32_t *ti = o->id; o->id = o->id2; o->id2 = ti;
  o->n_iface = 0;
  for (int64_t i = 0; i < N; ++i)
    if (o->type[i] == ORC_I) o->n_iface += 1;
  o->step += 1;

  /* Phase H */
  compute_mass(o);
  return 0;
}

int32_t orc_step(orc *o, int32_t n) {
  for (int32_t s = 0; s < n; ++s)
    if (one_step(o) != 0) return -1;
  return 0;
}

/* ---------------------------------------------------------------- read -- */

void orc_read(const orc *o, uint8_t *type, double *phi, double *mass, double *f, int32_t *id,
              double *rho, double *u) {
  const int64_t N = o->N;
  if (type) memcpy(type, o->type, N);
  if (phi) memcpy(phi, o->phi, sizeof(double) * N);
  if (mass) memcpy(mass, o->m, sizeof(double) * N);
  if (f) memcpy(f, o->f, sizeof(double) * Q * N);
  if (id) memcpy(id, o->id, sizeof(int32_t) * N);
  if (rho) memcpy(rho, o->rho, sizeof(double) * N);
  if (u) memcpy(u, o->u, sizeof(double) * 3 * N);
}

int32_t orc_nbubbles(const orc *o) { return o->nb; }

void orc_bubbles(const orc *o, int32_t *id, int32_t *flags, double *vol, double *vstar,
                 double *p, int64_t *ncells) {
  /* selection order by ID */
  int32_t *ord = malloc(sizeof(int32_t) * (o->nb > 0 ? o->nb : 1));
  for (int32_t k = 0; k < o->nb; ++k) ord[k] = k;
  for (int32_t a = 0; a < o->nb; ++a)
    for (int32_t b = a + 1; b < o->nb; ++b)
      if (o->b_id[ord[b]] < o->b_id[ord[a]]) {
        int32_t t = ord[a];
        ord[a] = ord[b];
        ord[b] = t;
      }
  for (int32_t k = 0; k < o->nb; ++k) {
    int32_t s = ord[k];
    if (id) id[k] = o->b_id[s];
    if (flags) flags[k] = o->b_flags[s];
    if (vol) vol[k] = o->b_vol[s];
    if (vstar) vstar[k] = o->b_vstar[s];
    if (p) p[k] = o->b_p[s];
    if (ncells) ncells[k] = o->b_ncell[s];
  }
  free(ord);
}

void orc_scalars(const orc *o, int64_t *step, int32_t *next_id, double *bucket, double *mass,
                 int64_t *n_topology) {
  if (step) *step = o->step;
  if (next_id) *next_id = o->next_id;
  if (bucket) *bucket = o->bucket;
  if (mass) *mass = o->mass;
  if (n_topology) *n_topology = o->n_topology;
}
