/*
 * Plain FP64 CPU oracle of one free-surface lattice Boltzmann step with the
 * enhanced bubble model (Anderl, Bogner, Rauh, Ruede, Delgado: "Free Surface
 * Lattice Boltzmann with Enhanced Bubble Model", arXiv:1604.01632).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the checker that the GPU library
 * is compared against; it shares no code, header, table or helper with the
 * GPU path, and nothing in the product path may link or call it.
 *
 * Every phase reads only the complete output of the previous phase (phase-
 * synchronous update), so the result does not depend on cell visiting order.
 */
#ifndef FSLBM_ORACLE_H
#define FSLBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_G = 0, ORC_I = 1, ORC_L = 2, ORC_W = 3, ORC_IN = 4 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t periodic[3];
  int32_t collision;   /* 0: BGK (Sec. 2.1), 1: TRT (optional reading) */
  int32_t freeze_conversions; /* 1: no interface cell is filled or emptied */
  double tau;          /* omega = 1 / tau */
  double trt_lambda;   /* TRT magic parameter */
  double sigma;        /* surface tension (Sec. 2.2, Laplace pressure) */
  double g[3];         /* body-force acceleration (Sec. 3.2) */
  double p0;           /* reference pressure rho0 cs^2, rho0 = 1 */
  double eps;          /* conversion threshold margin */
  double inject_rate;  /* V* added per step to inlet-owning bubbles */
  double contact_angle; /* static contact angle at walls in degrees, measured
                           in the liquid (Sec. 3.2); 0 or 90: neutral (mirror) */
} orc_params;

/* Bubble flags: bit 0 the bubble owns inlet cells (gas is injected);
 * bit 1 an "atmosphere" held at the reference pressure p0 whatever its
 * volume (the open top of the pore case, Sec. 3.2). */
#define ORC_BUBBLE_INLET 1
#define ORC_BUBBLE_ATMOSPHERE 2

typedef struct orc orc;

/* Build the oracle state.  Arrays are flat, i = x + nx*(y + ny*z); u is SoA
 * [3][N].  bubbles: b_vstar[k] > 0 is used as the initial volume V*, else
 * V* = V(0) * b_pinit[k] / p0.  f_init may be NULL (then f = f_eq(rho, u)).
 * mass_init may be NULL (then an interface cell starts with m = phi rho,
 * Sec. 2.2); otherwise it gives the interface masses of a saved state, so
 * that a run continues from that state exactly.
 * Returns NULL and writes a message into err on invalid input. */
orc *orc_create(const orc_params *p, const uint8_t *type, const double *phi,
                const double *rho, const double *u, const int32_t *id,
                const int32_t *b_id, const int32_t *b_flags, const double *b_vstar,
                const double *b_pinit, int32_t nb, const double *f_init,
                const double *mass_init, int64_t step0, int32_t next_id0, double bucket0,
                char *err, int32_t errlen);
void orc_destroy(orc *o);
void orc_set_threads(int32_t n);
int32_t orc_threads(void);

/* Advance n steps.  Returns 0, or -1 after an internal inconsistency (the
 * message is in orc_error). */
int32_t orc_step(orc *o, int32_t n);
const char *orc_error(const orc *o);

/* Read the state: any pointer may be NULL.  f is [19][N] post-collision;
 * rho and u are the values of the last collision (inputs before the first
 * step). */
void orc_read(const orc *o, uint8_t *type, double *phi, double *mass, double *f,
              int32_t *id, double *rho, double *u);
int32_t orc_nbubbles(const orc *o);
/* Bubbles sorted by ID. */
void orc_bubbles(const orc *o, int32_t *id, int32_t *flags, double *vol, double *vstar,
                 double *p, int64_t *ncells);
/* step count, next free ID, orphan-mass bucket, total mass (sum over liquid
 * cells of rho plus interface masses plus bucket), number of steps in which
 * some component received a new ID. */
void orc_scalars(const orc *o, int64_t *step, int32_t *next_id, double *bucket,
                 double *mass, int64_t *n_topology);

/* ---- pieces exposed for tests ---- */
void orc_lattice(int32_t *c /*[19][3]*/, double *w /*[19]*/, int32_t *opp /*[19]*/);
void orc_feq(double rho, const double *u, double *out /*19*/);
/* One collision of fin (19 values) with the oracle's parameters; writes the
 * post-collision values and the collision density and velocity. */
void orc_collide(const orc_params *p, const double *fin, double *fout, double *rho, double *u);
/* Velocity of the free boundary used in the gas-side equilibrium of an
 * interface cell, from its post-collision PDFs fs[19]. */
void orc_boundary_velocity(const orc_params *p, const double *fs, double *u /*3*/);
/* Normal (Youngs gradient) and curvature (height function) of every
 * interface cell of the current state; other cells get 0. */
void orc_geometry(const orc *o, double *kappa /*N*/, double *normal /*3N*/);
/* Exactly rounded sum of n doubles (the exact sum rounded once to the
 * nearest double, ties to even), as used for all per-cell sums. */
double orc_fsum(const double *v, int64_t n);
/* Connected components of the cells with inset[i] != 0 under 18-neighbour
 * adjacency; label = smallest linear index of the component, -1 outside. */
void orc_label(int32_t nx, int32_t ny, int32_t nz, const int32_t *periodic,
               const uint8_t *inset, int32_t *label);

#ifdef __cplusplus
}
#endif
#endif
