/*
 * fslbm.h - C ABI of the MI355X free-surface lattice Boltzmann library with
 * the enhanced bubble model of Anderl, Bogner, Rauh, Ruede, Delgado,
 * "Free Surface Lattice Boltzmann with Enhanced Bubble Model"
 * (arXiv:1604.01632).
 *
 * One call of fslbm_step advances one domain by whole time steps:
 *   - D3Q19 stream and BGK (or TRT) collision with a Guo body force
 *     (Sec. 2.1);
 *   - interface mass exchange (Sec. 2.2, mass-exchange equation) and fill
 *     levels phi = m / rho;
 *   - reconstruction of the PDFs missing on the gas side from the gas
 *     pressure p_V + 2 sigma kappa (Sec. 2.2, reconstruction and gas-pressure
 *     equations);
 *   - interface -> liquid / gas conversion keeping a closed interface layer,
 *     with excess-mass redistribution (Sec. 2.2);
 *   - per-bubble volume, ideal-gas pressure p = p0 V* / V (Sec. 2.2,
 *     ideal-gas equation), and bubble merge (Sec. 2.3.1) and split
 *     (Sec. 2.3.2) by connected-component labelling of the gas region, run
 *     only when a conversion can change the topology.
 *
 * Conventions
 *   Cell index i = x + nx * (y + ny * z).  PDFs are SoA: f[a * N + i] with
 *   the D3Q19 order: 0 rest; 1..6 = +x, -x, +y, -y, +z, -z; 7,8 = (1,1,0),
 *   (-1,-1,0); 9,10 = (1,-1,0), (-1,1,0); 11,12 = (1,0,1), (-1,0,-1);
 *   13,14 = (1,0,-1), (-1,0,1); 15,16 = (0,1,1), (0,-1,-1); 17,18 = (0,1,-1),
 *   (0,-1,1).  Velocities are SoA u[c * N + i].
 *   Host arrays on this boundary are always FP64, whatever the internal
 *   precision; the library converts.
 *   Ownership: the caller owns every host array and the device workspace
 *   (one allocation of fslbm_workspace_bytes() bytes, e.g. a torch uint8
 *   tensor).  The library allocates no device memory beyond it and frees
 *   nothing it did not allocate; a handle owns only host metadata and must
 *   not outlive its workspace.
 *   Streams: all device work of a handle is enqueued on the HIP stream given
 *   at creation; fslbm_step returns after enqueueing.  Reads synchronise that
 *   stream.  One handle must not be used from two threads at once; distinct
 *   handles are independent.
 *   Errors: every call returns FSLBM_OK (0) or a negative status;
 *   fslbm_last_error() returns the calling thread's message for the last
 *   failure.  Device-side failures (bubble table full, non-finite values,
 *   a failed watchdog check) are reported by the next synchronising call.
 */
#ifndef FSLBM_H
#define FSLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FSLBM_OK = 0,
  FSLBM_EINVAL = -1,    /* invalid argument or input state */
  FSLBM_ENOMEM = -2,    /* workspace too small */
  FSLBM_EDEVICE = -3,   /* HIP runtime error */
  FSLBM_ENUMERIC = -4,  /* non-finite density, mass or fill level; a broken
                           interface layer or mass drift found by the
                           watchdog; an internal list overflow */
  FSLBM_ECAPACITY = -5  /* bubble table or interface list full */
};

/* Cell types (Sec. 2.2, Fig. 1, plus walls and gas inlets of Sec. 3.2). */
enum { FSLBM_GAS = 0, FSLBM_INTERFACE = 1, FSLBM_LIQUID = 2, FSLBM_WALL = 3, FSLBM_INLET = 4 };

/* Storage precision of PDFs and fields.  FP64: FP64 arithmetic.  FP32 and
 * FP16DEV (PDFs stored as FP16 deviations from the lattice weights):
 * FP32 arithmetic; per-bubble volumes, pressures and the total mass are
 * always accumulated in FP64. */
enum { FSLBM_FP64 = 0, FSLBM_FP32 = 1, FSLBM_FP16DEV = 2 };

/* Collision operator: BGK (Sec. 2.1) or two-relaxation-time. */
enum { FSLBM_BGK = 0, FSLBM_TRT = 1 };

/* Bubble flag bits: INLET the bubble owns inlet cells (gas is injected,
 * Sec. 3.2); ATMOSPHERE the bubble is held at the reference pressure p0
 * whatever its volume (the open top of the pore case, Sec. 3.2).  A
 * component formed by a merge or split owns inlet cells if it holds one,
 * and is an atmosphere if it holds cells of an atmosphere. */
enum { FSLBM_BUBBLE_INLET = 1, FSLBM_BUBBLE_ATMOSPHERE = 2 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t periodic[3];  /* 1: periodic axis; 0: the two face layers must be
                           WALL or INLET cells */
  int32_t precision;    /* FSLBM_FP64 / FSLBM_FP32 / FSLBM_FP16DEV */
  int32_t collision;    /* FSLBM_BGK / FSLBM_TRT */
  double tau;           /* relaxation time, omega = 1 / tau; > 1/2 */
  double trt_lambda;    /* TRT magic parameter (3/16 is typical) */
  double sigma;         /* surface tension (Laplace pressure 2 sigma kappa) */
  double g[3];          /* body-force acceleration */
  double p0;            /* reference pressure rho0 cs^2 = 1/3 */
  double eps_convert;   /* interface -> liquid when phi > 1 + eps,
                           interface -> gas when phi < -eps */
  double inject_rate;   /* V* added per step to each bubble owning INLET cells */
  int32_t max_bubbles;  /* capacity of the device bubble table (>= 1) */
  int32_t force_topology; /* 1: label the gas region every step (testing) */
  int32_t freeze_conversions; /* 1: no interface cell is filled or emptied,
                                 so cell types and bubbles stay fixed
                                 (testing the flow and the interface update
                                 on a fixed geometry) */
  int32_t watchdog_every; /* K > 0: after every K-th step (counted from step
                             0 of the run) a device check runs, and
                             fslbm_step waits for it and returns
                             FSLBM_ENUMERIC if it failed: a liquid cell next
                             to a gas or inlet cell (the interface must stay
                             a closed layer, Sec. 2.2), a gas-region cell
                             without a live bubble, or a relative drift of
                             the total mass beyond watchdog_drift.  0: off */
  double watchdog_drift;  /* relative total-mass drift (against the mass at
                             creation) tolerated by the watchdog; <= 0: not
                             checked */
  int32_t debug_flags;    /* FSLBM_DEBUG_* bits (testing only) */
  int32_t split_trigger;  /* FSLBM_TRIGGER_EXACT (default) or
                             FSLBM_TRIGGER_NORMALS */
  double trigger_cos;     /* FSLBM_TRIGGER_NORMALS: two unit normals are
                             anti-parallel when their dot product is below
                             this value (e.g. -0.5) */
  int32_t iface_capacity; /* interface cells the per-slot arrays of the
                             interface list hold (0: min(N, max(N/6,
                             65536))); more interface cells in a step is
                             FSLBM_ECAPACITY */
  int32_t pad_;
  double contact_angle;   /* static contact angle at walls in degrees,
                             measured in the liquid (Sec. 3.2): a column of
                             the height-function stencil that lies in a wall
                             takes the mirrored column's liquid height plus
                             cot(angle) per wall axis crossed.  0 or 90: the
                             plain mirror (neutral wetting); else 0 < angle <
                             180 */
} fslbm_params;

/* What starts the connected-component labelling of a bubble (Sec. 2.3).
 * Merges are found exactly in both cases: a cell that joins the gas region
 * next to another bubble's cell (Sec. 2.3.1).  Splits (Sec. 2.3.2):
 *   EXACT    a cell that leaves the gas region and whose remaining
 *            gas-region neighbours are not connected inside its 3x3x3
 *            block, or that touches another such cell: never misses a
 *            split (the result equals labelling every step);
 *   NORMALS  the paper's test: a cell that turns liquid and has, among its
 *            18 neighbours, two interface cells of the same bubble whose
 *            normals (fill-level gradients of the step) are anti-parallel,
 *            n1.n2 < trigger_cos |n1| |n2|.  Cheaper in labelling runs, but
 *            a split it does not see stays undetected until it fires. */
enum { FSLBM_TRIGGER_EXACT = 0, FSLBM_TRIGGER_NORMALS = 1 };

/* debug_flags: accept a liquid cell next to a gas or inlet cell at
 * creation (for tests of the watchdog; the step is not defined on such a
 * state, but every kernel still reads and writes only inside the
 * workspace). */
enum { FSLBM_DEBUG_NO_LAYER_CHECK = 1 };

/* Initial bubble: v_star > 0 gives V* directly (restart); otherwise
 * V* = V(0) p_init / p0, with V(0) the volume of the initial state. */
typedef struct {
  int32_t id;
  int32_t flags;
  double v_star;
  double p_init;
} fslbm_bubble_init;

typedef struct {
  int32_t id;
  int32_t flags;     /* FSLBM_BUBBLE_* bits */
  double volume;     /* V: gas cells count 1, interface cells 1 - phi */
  double v_star;     /* V*: gas amount at the reference pressure */
  double pressure;   /* p0 V* / max(V, 1e-2) */
  int64_t n_cells;   /* gas + interface + inlet cells carrying this ID */
} fslbm_bubble;

typedef struct {
  int64_t step;        /* time steps done */
  int32_t next_id;     /* next fresh bubble ID */
  int32_t n_bubbles;   /* live bubbles */
  double bucket;       /* excess mass without an interface neighbour, spread
                          over all interface cells in the next step */
  double total_mass;   /* sum over liquid rho + interface m + bucket, FP64,
                          of the last step */
  int64_t n_topology;  /* steps in which a merge or split created bubbles */
  int64_t n_label_runs; /* steps in which the labelling ran (the trigger
                           fired, or the first step) */
} fslbm_scalars;

/* Exact device workspace size for these parameters (0 on invalid params). */
size_t fslbm_workspace_bytes(const fslbm_params *params);

/* Validate and upload an initial state and create a handle.
 *   cell_type[N] (u8), phi[N] (interface fill levels; ignored elsewhere),
 *   rho[N] and u[3N] (used to build f = f_eq(rho, u) when f_init is NULL),
 *   bubble_id[N] (IDs of GAS / INTERFACE / INLET cells; ignored elsewhere),
 *   bubbles[n_bubbles], f_init[19N] or NULL, mass_init[N] (interface masses
 *   of a checkpoint; NULL: m = phi rho, Sec. 2.2), restore (step, next_id,
 *   bucket of a checkpoint) or NULL.  A checkpoint read with
 *   fslbm_read_fields / fslbm_bubbles and passed back through f_init,
 *   mass_init, restore and v_star continues bit for bit.
 *   device_workspace: device pointer to >= fslbm_workspace_bytes() bytes,
 *   256-byte aligned; stream: hipStream_t (NULL = default stream).
 * EINVAL if: sizes or tau out of range; a type is unknown; a non-periodic
 * face layer holds a cell that is not WALL or INLET, or a WALL cell lies
 * elsewhere; a LIQUID cell touches a GAS or INLET cell (18-neighbourhood);
 * touching gas-region cells carry different IDs; an ID is not listed; an
 * interface fill level is not finite (any finite value is accepted: a
 * checkpoint may hold levels beyond [0, 1] that convert in the next step);
 * rho <= 0 on a fluid cell;
 * more bubbles than max_bubbles.  ENOMEM if the workspace is too small. */
int fslbm_create(const fslbm_params *params, const uint8_t *cell_type, const double *phi,
                 const double *rho, const double *u, const int32_t *bubble_id,
                 const fslbm_bubble_init *bubbles, int32_t n_bubbles, const double *f_init,
                 const double *mass_init, const fslbm_scalars *restore, void *device_workspace,
                 size_t workspace_bytes, void *stream, void **out_handle);

/* Enqueue n_steps >= 0 time steps on the handle's stream.  One step is the
 * update of Sec. 2: stream and collide (Sec. 2.1), the free-surface
 * boundary condition, mass exchange and cell conversion (Sec. 2.2), bubble
 * volumes and pressures (Sec. 2.2, ideal-gas equation) and the merge and
 * split rules (Sec. 2.3.1, 2.3.2).  Returns after enqueueing, except when
 * the watchdog is due (watchdog_every): then it waits for the check and
 * returns FSLBM_ENUMERIC (after the failing step; later steps are not
 * enqueued) if it failed. */
int fslbm_step(void *handle, int32_t n_steps);

/* Synchronise and copy state to the host; any pointer may be NULL.  The
 * state is that of Sec. 2.2: cell types, fill levels phi = m / rho, masses
 * and the PDFs of interface and liquid cells, plus the bubble ID of every
 * gas-region cell (Sec. 2.3).
 * f[19N] is the post-collision PDF set (undefined on GAS / WALL / INLET
 * cells), mass is m on interface cells and rho on liquid cells, rho and u
 * are recovered from f (u = sum c f / rho - g / 2).  Returns the first
 * asynchronous error of past steps (ECAPACITY, ENUMERIC) instead, if any. */
int fslbm_read_fields(void *handle, uint8_t *cell_type, double *phi, double *mass, double *f,
                      int32_t *bubble_id, double *rho, double *u, fslbm_scalars *scalars);

/* Synchronise and copy the live bubbles, sorted by ID, into out[capacity];
 * *n_out receives the number of live bubbles (ECAPACITY if > capacity).
 * A bubble is the data set {ID, V*, V} of Sec. 2.2 and 2.3 with the
 * pressure of the ideal-gas equation (Sec. 2.2), p = p0 V* / max(V, 1e-2). */
int fslbm_bubbles(void *handle, fslbm_bubble *out, int32_t capacity, int32_t *n_out);

/* Synchronise and report device-side failures of past steps. */
int fslbm_sync(void *handle);

/* GPU time per phase of the sampled steps enqueued while timing was
 * enabled, measured with HIP events on the handle's stream (bulk = liquid-cell
 * stream-collide kernel, iface = geometry and interface kernels, convert =
 * new cell types and new interface cells, excess = excess mass, topology
 * trigger and the tile counts of the next interface list, gather = the rest
 * of the list rebuild, the excess gather, and the labelled set, unions and
 * roots of a labelling run (independent work that shares their launches),
 * label = per-bubble volume sums (every step) and the rest of the labelling,
 * bubbles = installing the new bubbles of a labelling run and the pressure
 * update).  The labelling kernels return at once unless a topology change
 * is possible. */
typedef struct {
  double bulk_ms, iface_ms, convert_ms, excess_ms, gather_ms, label_ms, bubbles_ms;
  double step_ms;   /* sum of the above */
  int64_t steps;    /* sampled (timed) steps */
} fslbm_timing;

/* Phases of a step, as bits of the timing mask. */
enum {
  FSLBM_PHASE_IFACE = 1, FSLBM_PHASE_BULK = 2, FSLBM_PHASE_CONVERT = 4, FSLBM_PHASE_EXCESS = 8,
  FSLBM_PHASE_GATHER = 16, FSLBM_PHASE_LABEL = 32, FSLBM_PHASE_BUBBLES = 64, FSLBM_PHASE_ALL = 127
};

/* Event timing of every period-th step enqueued from now on (the first of
 * them included); period 1 times every step, 0 disables timing.  Only the
 * phases in phase_mask (FSLBM_PHASE_* bits; 0 means all) are bracketed by
 * events, the others report 0.  Each event delays the next kernel by a few
 * microseconds, so a period well above 1 and a narrow mask keep the timed
 * stream close to an untimed one.  Waits for the handle's stream and clears
 * the accumulated times.  FSLBM_EINVAL for period < 0. */
int fslbm_set_timing(void *handle, int32_t period, uint32_t phase_mask);

/* Synchronise, report the accumulated times and clear them. */
int fslbm_get_timing(void *handle, fslbm_timing *out);

/* Diagnostics: achievable HBM bandwidth on this device.  Copies `bytes`
 * (a multiple of 16) from src to dst, both device buffers owned by the
 * caller and 16-byte aligned, reps times with a plain streaming copy kernel
 * (16-byte non-temporal loads and stores) on `stream`, and writes to
 * *gbs_out the bytes read plus written per second, averaged over the reps
 * (HIP events).  EINVAL on bad arguments, EDEVICE on HIP errors. */
int fslbm_copy_bandwidth(void *dst, const void *src, size_t bytes, int32_t reps, void *stream,
                         double *gbs_out);

/* Destroy the handle (no device memory is freed: it belongs to the caller). */
int fslbm_destroy(void *handle);

/* Message of the calling thread's last failure ("" if none). */
const char *fslbm_last_error(void);

/* ---------------------------------------------------------------------
 * Batched form: many independent domains (uneven sizes, each created with
 * fslbm_create, all of one precision) advanced together.  Every kernel of
 * a step is launched once for all domains (each block finds its domain
 * from per-kernel block-offset tables), and one whole step of all domains
 * is captured in a HIP graph at creation, so that a batch step is one
 * graph launch.  Each domain computes exactly what fslbm_step computes for
 * it alone (bit for bit).
 *
 * Autotuning at creation, 18 points: the stream-collide block size (128 or
 * 256 threads) and the order of domains in the block map (as given, by
 * decreasing or by increasing size) are chosen by timing the
 * stream-collide kernel of the batch on the live state (a probe without
 * the mass accumulator that only writes buffers the next step rewrites),
 * and the grid density of the interface-list kernels (one block per 1024,
 * 2048 or 4096 cells) by timing the geometry kernel (which only writes
 * per-slot values the next step rewrites).  The choice is appended to the
 * text file tuning_cache_path (may be NULL: tune without caching) under a
 * key made of the precision and the domain extents, and read from it next
 * time.  An empty string "" skips tuning (256 threads, domains as given,
 * 2048 cells per list block), for callers that rebuild batches often.
 * --------------------------------------------------------------------- */

/* Device bytes of the batch tables for n_domains (0 if n_domains < 1). */
size_t fslbm_batch_workspace_bytes(int32_t n_domains);

typedef struct {
  int32_t bulk_threads;  /* chosen stream-collide block size (128 or 256) */
  int32_t order;         /* 0: domains as given, 1: by decreasing size,
                            2: by increasing size */
  int32_t from_cache;    /* 1 if the choice came from the tuning cache */
  int32_t list_cells;    /* cells per block of the interface-list kernels'
                            grids (1024, 2048 or 4096) */
  int64_t cells;         /* cells of all domains */
  float probe_ms[9];     /* stream-collide probes of (256 or 128 threads) x
                            (order 0, 1, 2) in that order, then geometry
                            probes of 1024, 2048 and 4096 cells per block */
  int32_t pad;
} fslbm_batch_info;

/* Build a batch over handles[n] (distinct, same precision).  The device
 * workspace (>= fslbm_batch_workspace_bytes(n), 256-byte aligned) holds
 * the tables and belongs to the caller; it and the handles must outlive the
 * batch.  stream: the caller's hipStream_t (NULL = default); batch steps
 * are ordered after work already queued on it and on the domains' own
 * streams, and before work queued there afterwards.  The batch runs on a
 * stream of its own (default priority).  Stepping a member domain on its
 * own between batch steps is allowed (the batch then rebuilds its tables).
 * EINVAL on NULL or repeated handles or mixed precisions, ENOMEM if the
 * workspace is too small, EDEVICE on HIP failures. */
int fslbm_batch_create(void *const *handles, int32_t n, const char *tuning_cache_path,
                       void *device_workspace, size_t workspace_bytes, void *stream,
                       void **out_batch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * batched form of fslbm_batch_create with its tables in a static device
 * array of the library (4 MiB per GPU, held until the process ends) instead
 * of a caller workspace.  No device memory is allocated and no stream,
 * event or graph is created: every domain must have been created on
 * `stream`, and each batch step is the plain launch of the step kernels on
 * it (no tuning: 256-thread stream-collide blocks, domains as given).  The
 * domains compute bit for bit what they compute alone or in any batch.
 * At most about 3700 domains (EINVAL beyond the array, with the sizes in
 * the message).  All such batches on one GPU share the one array: creating
 * one overwrites the tables of the one before, which must not be stepped
 * again; calls that overlap on one GPU race.  Use fslbm_batch_step and
 * fslbm_batch_destroy on the returned batch. */
int fslbm_batch_create_noalloc(void *const *handles, int32_t n, void *stream, void **out_batch);

/* Enqueue n_steps >= 0 steps of every domain of the batch (n_steps graph
 * launches).  Asynchronous errors of a domain are reported by fslbm_sync,
 * fslbm_read_fields or fslbm_bubbles on its handle. */
int fslbm_batch_step(void *batch, int32_t n_steps);

/* Replace the members of a batch by handles[n] (same precision; n at most
 * the domains its table space holds: the workspace size given at creation,
 * see fslbm_batch_workspace_bytes).  Domains may come and go this way, as
 * in a serving loop, without creating a new batch: the tables are
 * rewritten in place, ordered on the batch's stream after the steps already
 * queued (no wait for them), and from the first reset on the batch's steps
 * are plain kernel launches instead of graph replays (its graphs are
 * dropped; the kernels and results are the same).  A batch of
 * fslbm_batch_create_noalloc keeps its rule: every domain on its stream. */
int fslbm_batch_reset(void *batch, void *const *handles, int32_t n);

/* The autotuning outcome of the batch. */
int fslbm_batch_info_get(void *batch, fslbm_batch_info *out);

/* Wait for the batch's work and release its host resources. */
int fslbm_batch_destroy(void *batch);

#ifdef __cplusplus
}
#endif
#endif
