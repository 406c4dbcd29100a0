// Host implementation of the C ABI declared in include/fslbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fslbm.h"
#include "launch.hpp"

using namespace fslbm;

// The batch tables of fslbm_batch_create_noalloc: a static device array
// (one copy per GPU, kept until the process ends).  In host code `scratch`
// only names the symbol; its device address on the current device comes
// from hipGetSymbolAddress, once per device (scratch_address below), and
// only that address is used (kernel arguments, copies).
static constexpr size_t SCRATCH_BYTES = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(FSLBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

constexpr int HOST_CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int HOST_CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int HOST_CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

bool launchers_for(int precision, Launchers &L) {
  if (precision == FSLBM_FP64) L = launchers_fp64();
  else if (precision == FSLBM_FP32) L = launchers_fp32();
  else if (precision == FSLBM_FP16DEV) L = launchers_fp16();
  else return false;
  return true;
}

// ------------------------------------------------------------- layout

enum Arr {
  A_F0, A_F1, A_FLAG0, A_FLAG1, A_PHI0, A_PHI1, A_MASS, A_RHOI, A_EXCESS, A_BSLOT, A_LAB,
  A_AUX0, A_AUX2, A_BID, A_BFLAGS, A_BLIVE, A_BRMIN, A_BRMAX, A_BKEPT, A_BAFFECT, A_NEWROOTS,
  A_NEWSLOT, A_BVSTAR, A_BVOL, A_BP, A_BNGAS, A_BNIFACE, A_BVACC, A_CACC,
  A_SCALARS, A_MASSACC, A_BUCKETACC, A_ILIST0, A_ILIST1, A_CLIST, A_NLIST, A_MARK, A_GASV, A_NMASK, A_NRM, A_TILECOUNT, A_TILEOFF,
  A_FIF0, A_FIF1, A_NFLAG, A_ISLOT0, A_ISLOT1, A_COUNT
};

struct Layout {
  size_t off[A_COUNT];
  size_t total;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Interface cells the list and its per-slot arrays hold.
long long iface_capacity(const fslbm_params &p) {
  const long long N = (long long)p.nx * p.ny * p.nz;
  if (p.iface_capacity > 0) return std::min<long long>(p.iface_capacity, N);
  return std::min<long long>(N, std::max<long long>(N / 6, 65536));
}

Layout make_layout(const fslbm_params &p, const Launchers &L) {
  const size_t N = (size_t)p.nx * p.ny * p.nz;
  const size_t C = (size_t)iface_capacity(p);
  const size_t B = (size_t)p.max_bubbles;
  size_t sz[A_COUNT];
  sz[A_F0] = sz[A_F1] = (size_t)Q * N * L.store_bytes;
  sz[A_FLAG0] = sz[A_FLAG1] = N;
  sz[A_PHI0] = sz[A_PHI1] = sz[A_MASS] = sz[A_RHOI] = sz[A_EXCESS] = N * L.real_bytes;
  sz[A_BSLOT] = sz[A_LAB] = sz[A_AUX0] = sz[A_AUX2] = N * 4;
  sz[A_BID] = sz[A_BFLAGS] = sz[A_BLIVE] = sz[A_BRMIN] = sz[A_BRMAX] = sz[A_BKEPT] = sz[A_BAFFECT] =
      sz[A_NEWROOTS] = sz[A_NEWSLOT] = B * 4;
  sz[A_BVSTAR] = sz[A_BVOL] = sz[A_BP] = sz[A_BNGAS] = sz[A_BNIFACE] = B * 8;
  sz[A_BVACC] = B * SUB * VACC * 8;
  sz[A_CACC] = B * SUB * NACC * 8;
  sz[A_SCALARS] = sizeof(Scalars);
  sz[A_MASSACC] = SUB_MASS * 2 * 8;
  sz[A_BUCKETACC] = SUB * EX_WORDS * 8;
  sz[A_ILIST0] = sz[A_ILIST1] = C * 4;
  sz[A_CLIST] = sz[A_NLIST] = N * 4;
  sz[A_MARK] = ((N + 3) / 4) * 4;
  sz[A_GASV] = C * L.real_bytes;
  sz[A_NMASK] = C * 4;
  sz[A_NRM] = p.split_trigger == FSLBM_TRIGGER_NORMALS ? 3 * C * 4 : 0;
  sz[A_TILECOUNT] = sz[A_TILEOFF] = ((N + 4095) / 4096) * 4;
  sz[A_FIF0] = sz[A_FIF1] = C * (((size_t)Q * L.store_bytes + 15) / 16 * 16);  // one padded row per slot
  sz[A_NFLAG] = C;
  sz[A_ISLOT0] = sz[A_ISLOT1] = N * 4;
  Layout lay;
  size_t o = 0;
  for (int k = 0; k < A_COUNT; ++k) {
    lay.off[k] = o;
    o = align256(o + sz[k]);
  }
  lay.total = o;
  return lay;
}

const char *check_params(const fslbm_params *p) {
  if (!p) return "params is NULL";
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "sizes must be >= 1";
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int k = 0; k < 3; ++k)
    if (!p->periodic[k] && n[k] < 5) return "a non-periodic axis needs at least 5 cells";
  if ((long long)p->nx * p->ny * p->nz >= (1ll << 31)) return "more than 2^31 - 1 cells";
  if (p->ny > 65535 || p->nz > 65535) return "ny and nz must be <= 65535";
  if (!(p->tau > 0.5)) return "tau must be > 1/2";
  if (p->collision != FSLBM_BGK && p->collision != FSLBM_TRT) return "unknown collision";
  if (p->collision == FSLBM_TRT && !(p->trt_lambda > 0.0)) return "trt_lambda must be > 0";
  if (p->precision < FSLBM_FP64 || p->precision > FSLBM_FP16DEV) return "unknown precision";
  if (p->max_bubbles < 1 || p->max_bubbles > (1 << 20)) return "max_bubbles out of range";
  if (!(p->eps_convert >= 0.0)) return "eps_convert must be >= 0";
  if (!(p->p0 > 0.0)) return "p0 must be > 0";
  if (p->force_topology != 0 && p->force_topology != 1) return "force_topology must be 0 or 1";
  if (p->freeze_conversions != 0 && p->freeze_conversions != 1)
    return "freeze_conversions must be 0 or 1";
  if (p->watchdog_every < 0) return "watchdog_every must be >= 0";
  if (p->debug_flags & ~FSLBM_DEBUG_NO_LAYER_CHECK) return "unknown debug_flags bits";
  if (p->iface_capacity < 0) return "iface_capacity must be >= 0";
  if (p->split_trigger != FSLBM_TRIGGER_EXACT && p->split_trigger != FSLBM_TRIGGER_NORMALS)
    return "unknown split_trigger";
  if (p->split_trigger == FSLBM_TRIGGER_NORMALS && !(p->trigger_cos >= -1.0 && p->trigger_cos <= 1.0))
    return "trigger_cos must lie in [-1, 1]";
  if (!(p->contact_angle >= 0.0 && p->contact_angle < 180.0))
    return "contact_angle must be 0 (neutral) or lie in (0, 180) degrees";
  return nullptr;
}

// cot of the static contact angle; exactly 0 for the neutral angle (90
// degrees, or 0 for unset), so that the wall rule is then the mirror.
double wall_cot(const fslbm_params &p) {
  const double t = p.contact_angle;
  if (t == 0.0 || t == 90.0) return 0.0;
  const double r = t * (3.14159265358979323846 / 180.0);
  return std::cos(r) / std::sin(r);
}

// --------------------------------------------------------------- context

struct Ctx {
  // per-phase event timing (fslbm_set_timing): on every timing_period-th
  // step enqueued since it was set, each phase in timing_mask is bracketed
  // by a pair of events
  int timing_period = 0;
  unsigned timing_mask = 0;
  long long timing_count = 0;
  long long timed_steps = 0;
  std::vector<hipEvent_t> events;  // two per timed phase
  std::vector<int> event_phase;    // the phase of each pair
  size_t used = 0;                 // pairs in use
  long long host_step = 0;         // steps enqueued since step 0 of the run
  fslbm_params P;
  Launchers L;
  LaunchCfg cfg;
  Layout lay;
  Dev dev[2];  // dev[c]: src buffers = c
  int cur = 0;
  long long N = 0;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
};

template <class T>
T *at(char *ws, const Layout &lay, Arr a) {
  return (T *)(ws + lay.off[a]);
}

void build_devs(Ctx &c) {
  const Layout &lay = c.lay;
  char *ws = c.ws;
  Dev d{};
  d.nx = c.P.nx;
  d.ny = c.P.ny;
  d.nz = c.P.nz;
  for (int k = 0; k < 3; ++k) d.per[k] = c.P.periodic[k] ? 1 : 0;
  d.has_walls = !(d.per[0] && d.per[1] && d.per[2]);
  d.max_bubbles = c.P.max_bubbles;
  d.force_topology = c.P.force_topology;
  d.freeze = c.P.freeze_conversions;
  d.split_trigger = c.P.split_trigger;
  d.icap = (int)iface_capacity(c.P);
  d.trigger_cos = c.P.trigger_cos;
  d.wall_cot = wall_cot(c.P);
  d.drift_tol = c.P.watchdog_drift;
  d.collision = c.P.collision;
  d.N = c.N;
  d.omega_p = 1.0 / c.P.tau;
  d.omega_m = d.omega_p;
  if (c.P.collision == FSLBM_TRT) d.omega_m = 1.0 / (0.5 + c.P.trt_lambda / (1.0 / d.omega_p - 0.5));
  d.sigma = c.P.sigma;
  d.p0 = c.P.p0;
  d.eps = c.P.eps_convert;
  d.inject = c.P.inject_rate;
  for (int k = 0; k < 3; ++k) d.g[k] = c.P.g[k];
  d.mass = ws + lay.off[A_MASS];
  d.rhoI = ws + lay.off[A_RHOI];
  d.excess = ws + lay.off[A_EXCESS];
  d.bslot = at<int32_t>(ws, lay, A_BSLOT);
  d.lab = at<int32_t>(ws, lay, A_LAB);
  d.aux0 = at<int32_t>(ws, lay, A_AUX0);
  d.aux2 = at<int32_t>(ws, lay, A_AUX2);
  d.b_id = at<int32_t>(ws, lay, A_BID);
  d.b_flags = at<int32_t>(ws, lay, A_BFLAGS);
  d.b_live = at<int32_t>(ws, lay, A_BLIVE);
  d.b_rmin = at<int32_t>(ws, lay, A_BRMIN);
  d.b_rmax = at<int32_t>(ws, lay, A_BRMAX);
  d.b_kept = at<int32_t>(ws, lay, A_BKEPT);
  d.b_affect = at<int32_t>(ws, lay, A_BAFFECT);
  d.newroots = at<int32_t>(ws, lay, A_NEWROOTS);
  d.newslot = at<int32_t>(ws, lay, A_NEWSLOT);
  d.b_vstar = at<double>(ws, lay, A_BVSTAR);
  d.b_vol = at<double>(ws, lay, A_BVOL);
  d.b_p = at<double>(ws, lay, A_BP);
  d.b_ngas = at<long long>(ws, lay, A_BNGAS);
  d.b_niface = at<long long>(ws, lay, A_BNIFACE);
  d.b_vacc = at<unsigned long long>(ws, lay, A_BVACC);
  d.c_acc = at<unsigned long long>(ws, lay, A_CACC);
  d.sc = at<Scalars>(ws, lay, A_SCALARS);
  d.mass_acc = at<unsigned long long>(ws, lay, A_MASSACC);
  d.bucket_acc = at<unsigned long long>(ws, lay, A_BUCKETACC);
  d.clist = at<int32_t>(ws, lay, A_CLIST);
  d.nlist = at<int32_t>(ws, lay, A_NLIST);
  d.mark = at<unsigned>(ws, lay, A_MARK);
  d.gasv = ws + lay.off[A_GASV];
  d.nmask = at<uint32_t>(ws, lay, A_NMASK);
  d.nrm = at<float>(ws, lay, A_NRM);
  d.tilecount = at<int32_t>(ws, lay, A_TILECOUNT);
  d.tileoff = at<int32_t>(ws, lay, A_TILEOFF);
  d.nflag = at<uint8_t>(ws, lay, A_NFLAG);
  for (int s = 0; s < 2; ++s) {
    Dev e = d;
    e.f_src = ws + lay.off[s == 0 ? A_F0 : A_F1];
    e.f_dst = ws + lay.off[s == 0 ? A_F1 : A_F0];
    e.flag_src = at<uint8_t>(ws, lay, s == 0 ? A_FLAG0 : A_FLAG1);
    e.flag_dst = at<uint8_t>(ws, lay, s == 0 ? A_FLAG1 : A_FLAG0);
    e.phi_src = ws + lay.off[s == 0 ? A_PHI0 : A_PHI1];
    e.phi_dst = ws + lay.off[s == 0 ? A_PHI1 : A_PHI0];
    e.ilist_src = at<int32_t>(ws, lay, s == 0 ? A_ILIST0 : A_ILIST1);
    e.ilist_dst = at<int32_t>(ws, lay, s == 0 ? A_ILIST1 : A_ILIST0);
    e.f_if = ws + lay.off[s == 0 ? A_FIF0 : A_FIF1];
    e.f_if_prev = ws + lay.off[s == 0 ? A_FIF1 : A_FIF0];
    e.islot = at<int32_t>(ws, lay, s == 0 ? A_ISLOT0 : A_ISLOT1);
    e.islot_alt = at<int32_t>(ws, lay, s == 0 ? A_ISLOT1 : A_ISLOT0);
    c.dev[s] = e;
  }
}

LaunchCfg make_cfg(const fslbm_params &p, int bulk_threads = 256, int list_cells = 2048) {
  LaunchCfg cfg;
  const long long N = (long long)p.nx * p.ny * p.nz;
  auto clampb = [&](long long per, long long cap) {
    return (int)std::max<long long>(1, std::min<long long>((N + per - 1) / per, cap));
  };
  cfg.bulk_threads = bulk_threads;
  cfg.blocks[G_BULK] = (int)((N + bulk_threads - 1) / bulk_threads);
  // The list and labelling kernels walk lists a few per cent of the cells
  // long with grid-stride loops: one block per 2048 or 4096 cells is ample,
  // and a block that finds no work still costs its dispatch (a batch of
  // small domains would otherwise launch hundreds of thousands of them).
  // Large boxes reach the caps.
  cfg.blocks[G_LIST] = clampb(list_cells, 2048);
  cfg.blocks[G_SMALL] = clampb(4096, 256);
  cfg.blocks[G_TILE] = (int)((N + 4095) / 4096);
  cfg.blocks[G_ONE] = 1;
  cfg.blocks[G_CELL] = cell_blocks(N);
  cfg.blocks[G_EXCOUNT] = cfg.blocks[G_SMALL] + cfg.blocks[G_TILE];
  cfg.blocks[G_SCANCELL] = 1 + cfg.blocks[G_CELL];
  cfg.blocks[G_TILECELL] = cfg.blocks[G_TILE] + cfg.blocks[G_CELL];
  cfg.blocks[G_LISTCELL] = cfg.blocks[G_LIST] + cfg.blocks[G_CELL];
  // the volume reduction walks the bubble slots with grid strides: a small
  // domain of a batch gets no more blocks for it than for its labelling
  cfg.blocks[G_ONEVOL] = 1 + std::min(volume_blocks(p.max_bubbles, 256), cell_blocks(N));
  cfg.with_mass = 1;
  return cfg;
}

// host-side conversions for uploads
template <class T>
std::vector<char> pack_real(const std::vector<double> &v, int bytes) {
  (void)sizeof(T);
  std::vector<char> out(v.size() * bytes);
  if (bytes == 8) {
    std::memcpy(out.data(), v.data(), v.size() * 8);
  } else {
    float *o = (float *)out.data();
    for (size_t k = 0; k < v.size(); ++k) o[k] = (float)v[k];
  }
  return out;
}

// ------------------------------------------------------------- batches

struct Batch {
  std::vector<Ctx *> dom;       // launch order
  std::vector<int> base_cur;    // parity of every domain when the tables were built
  Launchers L;
  int precision = 0;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;  // own stream: captured and replayed
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  char *ws = nullptr;
  Dev *d_devs[2] = {nullptr, nullptr};
  int *d_off[G_COUNT] = {};
  BatchCfg cfg[2];
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  fslbm_batch_info info{};
  // tables in the library's static scratch array: no own stream, events or
  // graphs; steps are plain launches on the caller's stream
  bool in_scratch = false;
  // steps as plain launches instead of graph replays (after a reset)
  bool direct = false;
  int cap = 0;  // domains the table space holds (fixed table offsets)
  // pinned host staging of the tables, two buffers used in turn, each
  // reusable once the copy out of it (event) has completed
  char *stage[2] = {nullptr, nullptr};
  hipEvent_t stage_ev[2] = {nullptr, nullptr};
  int stage_cur = 0;
};

size_t batch_bytes(int nd) {
  return align256(2 * (size_t)nd * sizeof(Dev)) + G_COUNT * align256((size_t)(nd + 1) * 4);
}

// Domains a table space of `bytes` holds.
int batch_capacity(size_t bytes) {
  int lo = 0, hi = 1 << 24;
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (batch_bytes(mid) <= bytes) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Device tables for the current domain order and parities: the Dev of
// every domain for the next step (relative parity 0) and the one after
// (1), and per grid class the first block of every domain.
// Tables at fixed offsets for the batch's capacity (the kernel arguments
// that point at them stay valid when the members change): the Devs of the
// two parities, then per grid class the block offsets.  Written through the
// pinned staging buffers without waiting for the stream, or, for a batch in
// the scratch array (which allocates nothing, not even pinned host memory),
// from pageable memory with a wait.
int batch_tables(Batch &b, int bulk_threads, int list_cells = 2048) {
  const int nd = (int)b.dom.size();
  const int cap = b.cap > 0 ? b.cap : nd;
  std::vector<Dev> devs(2 * (size_t)nd);
  std::vector<int> off[G_COUNT];
  for (int g = 0; g < G_COUNT; ++g) off[g].assign(nd + 1, 0);
  b.base_cur.resize(nd);
  for (int k = 0; k < nd; ++k) {
    Ctx &c = *b.dom[k];
    b.base_cur[k] = c.cur;
    devs[k] = c.dev[c.cur];
    devs[nd + k] = c.dev[c.cur ^ 1];
    const LaunchCfg lc = make_cfg(c.P, bulk_threads, list_cells);
    for (int g = 0; g < G_COUNT; ++g) off[g][k + 1] = off[g][k] + lc.blocks[g];
  }
  // the image of the table space: [Dev x cap][Dev x cap] then per class
  // (cap + 1) offsets, each part 256-byte aligned
  const size_t dev_part = align256(2 * (size_t)cap * sizeof(Dev));
  const size_t off_part = align256((size_t)(cap + 1) * 4);
  const size_t total = dev_part + G_COUNT * off_part;
  std::vector<char> pageable;
  char *img;
  if (b.stage[0]) {
    const int k = b.stage_cur;
    HIP_TRY(hipEventSynchronize(b.stage_ev[k]));  // its previous copy is done
    img = b.stage[k];
  } else {
    pageable.resize(total);
    img = pageable.data();
  }
  std::memcpy(img, devs.data(), (size_t)nd * sizeof(Dev));
  std::memcpy(img + (size_t)cap * sizeof(Dev), devs.data() + nd, (size_t)nd * sizeof(Dev));
  for (int g = 0; g < G_COUNT; ++g)
    std::memcpy(img + dev_part + g * off_part, off[g].data(), (size_t)(nd + 1) * 4);
  char *p = b.ws;
  b.d_devs[0] = (Dev *)p;
  b.d_devs[1] = (Dev *)p + cap;
  for (int g = 0; g < G_COUNT; ++g) b.d_off[g] = (int *)(p + dev_part + g * off_part);
  HIP_TRY(hipMemcpyAsync(p, img, total, hipMemcpyHostToDevice, b.stream));
  if (b.stage[0]) {
    HIP_TRY(hipEventRecord(b.stage_ev[b.stage_cur], b.stream));
    b.stage_cur ^= 1;
  } else {
    HIP_TRY(hipStreamSynchronize(b.stream));
  }
  for (int r = 0; r < 2; ++r) {
    BatchCfg &bc = b.cfg[r];
    bc.devs = b.d_devs[r];
    bc.nd = nd;
    for (int g = 0; g < G_COUNT; ++g) {
      bc.off[g] = b.d_off[g];
      bc.total[g] = off[g][nd];
    }
    bc.bulk_threads = bulk_threads;
    bc.with_mass = 1;
  }
  return FSLBM_OK;
}

void batch_drop_graphs(Batch &b) {
  for (int r = 0; r < 2; ++r) {
    if (b.exec[r]) hipGraphExecDestroy(b.exec[r]);
    if (b.graph[r]) hipGraphDestroy(b.graph[r]);
    b.exec[r] = nullptr;
    b.graph[r] = nullptr;
  }
}

// One graph per relative parity, each holding one whole step of every
// domain (the kernels only; no memory operations are captured).
int batch_capture(Batch &b) {
  batch_drop_graphs(b);
  for (int r = 0; r < 2; ++r) {
    HIP_TRY(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
    for (int ph = 0; ph < PH_COUNT; ++ph) b.L.batch_phase(ph, b.cfg[r], b.stream);
    HIP_TRY(hipStreamEndCapture(b.stream, &b.graph[r]));
    HIP_TRY(hipGraphInstantiate(&b.exec[r], b.graph[r], nullptr, nullptr, 0));
  }
  return FSLBM_OK;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the scratch array on the current device.
int scratch_address(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(FSLBM_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || ((uintptr_t)ptr & 255)) return fail(FSLBM_EDEVICE, "scratch array not aligned");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FSLBM_OK;
}

// Tuning key: precision and the sequence of domain extents (FNV-1a).
std::string batch_key(const Batch &b) {
  unsigned long long h = 1469598103934665603ull;
  auto mix = [&](long long v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (unsigned long long)((v >> (8 * k)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (Ctx *c : b.dom) {
    mix(c->P.nx);
    mix(c->P.ny);
    mix(c->P.nz);
  }
  char buf[96];
  std::snprintf(buf, sizeof buf, "p%d-n%zu-%016llx", b.precision, b.dom.size(), h);
  return buf;
}

bool batch_cache_lookup(const char *path, const std::string &key, int &threads, int &order,
                        int &list_cells) {
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char k[128];
    int t, o, l;
    if (std::sscanf(line, "%127s %d %d %d", k, &t, &o, &l) != 4) continue;
    if (key == k && (t == 128 || t == 256) && o >= 0 && o <= 2 &&
        (l == 1024 || l == 2048 || l == 4096)) {
      threads = t;
      order = o;
      list_cells = l;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void batch_cache_store(const char *path, const std::string &key, int threads, int order,
                       int list_cells) {
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d\n", key.c_str(), threads, order, list_cells);
  std::fclose(f);
}

// Average duration (ms) of a probe over reps launches: the stream-collide
// kernel (list = false) or the geometry kernel (list = true).
int batch_probe(Batch &b, int reps, float &ms, bool list = false) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto probe = [&]() {
    if (list) b.L.batch_list_probe(b.cfg[0], b.stream);
    else b.L.batch_bulk_probe(b.cfg[0], b.stream);
  };
  for (int w = 0; w < 2; ++w) probe();
  HIP_TRY(hipEventRecord(e0, b.stream));
  for (int r = 0; r < reps; ++r) probe();
  HIP_TRY(hipEventRecord(e1, b.stream));
  HIP_TRY(hipEventSynchronize(e1));
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  ms /= reps;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return FSLBM_OK;
}

void batch_order(Batch &b, const std::vector<Ctx *> &given, int order) {
  b.dom = given;
  if (order == 1)
    std::stable_sort(b.dom.begin(), b.dom.end(), [](const Ctx *x, const Ctx *y) { return x->N > y->N; });
  if (order == 2)
    std::stable_sort(b.dom.begin(), b.dom.end(), [](const Ctx *x, const Ctx *y) { return x->N < y->N; });
}

void batch_free(Batch *b) {
  if (!b) return;
  if (b->in_scratch) {
    // nothing of its own on the device: wait for its work and drop the host part
    hipStreamSynchronize(b->stream);
    delete b;
    return;
  }
  if (b->stream) hipStreamSynchronize(b->stream);
  batch_drop_graphs(*b);
  for (int k = 0; k < 2; ++k) {
    if (b->stage_ev[k]) hipEventDestroy(b->stage_ev[k]);
    if (b->stage[k]) hipHostFree(b->stage[k]);
  }
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
}

int sync_and_check(Ctx &c) {
  HIP_TRY(hipStreamSynchronize(c.stream));
  Scalars sc;
  HIP_TRY(hipMemcpy(&sc, c.dev[0].sc, sizeof sc, hipMemcpyDeviceToHost));
  if (sc.err & ERR_CAPACITY) return fail(FSLBM_ECAPACITY, "bubble table full (max_bubbles)");
  if (sc.err & ERR_NONFINITE)
    return fail(FSLBM_ENUMERIC, "non-finite density, mass or fill level (or total mass)");
  if (sc.err & ERR_RANGE) return fail(FSLBM_ENUMERIC, "conversion candidate list overflow");
  if (sc.err & ERR_ILIST)
    return fail(FSLBM_ECAPACITY, "interface list full: more interface cells than iface_capacity (" +
                                     std::to_string(iface_capacity(c.P)) + ")");
  if (sc.err & ERR_LAYER)
    return fail(FSLBM_ENUMERIC, "watchdog: a liquid cell touches a gas or inlet cell "
                                "(the interface layer is not closed)");
  if (sc.err & ERR_ORPHAN)
    return fail(FSLBM_ENUMERIC, "watchdog: a gas-region cell has no live bubble");
  if (sc.err & ERR_DRIFT) {
    char m[160];
    std::snprintf(m, sizeof m, "watchdog: total mass %.17g drifted from %.17g beyond %g relative",
                  sc.total_mass, sc.mass_ref, c.P.watchdog_drift);
    return fail(FSLBM_ENUMERIC, m);
  }
  return FSLBM_OK;
}

bool watchdog_due(const Ctx &c) {
  return c.P.watchdog_every > 0 && c.host_step % c.P.watchdog_every == 0;
}

// Achievable-bandwidth probe: a plain streaming copy with 16-byte
// non-temporal loads and stores (each byte is read and written once).  It
// gives the bandwidth a kernel that only streams can reach on the device,
// as context for the roofline of the step kernels.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy_stream(const v4u *__restrict__ src,
                                                      v4u *__restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

// ==================================================================== ABI

extern "C" {

const char *fslbm_last_error(void) { return g_err.c_str(); }

size_t fslbm_workspace_bytes(const fslbm_params *params) {
  if (check_params(params)) return 0;
  Launchers L;
  if (!launchers_for(params->precision, L)) return 0;
  return make_layout(*params, L).total;
}

int fslbm_create(const fslbm_params *params, const uint8_t *cell_type, const double *phi,
                 const double *rho, const double *u, const int32_t *bubble_id,
                 const fslbm_bubble_init *bubbles, int32_t n_bubbles, const double *f_init,
                 const double *mass_init, const fslbm_scalars *restore, void *device_workspace,
                 size_t workspace_bytes, void *stream, void **out_handle) {
  if (!out_handle) return fail(FSLBM_EINVAL, "out_handle is NULL");
  *out_handle = nullptr;
  if (const char *m = check_params(params)) return fail(FSLBM_EINVAL, m);
  const fslbm_params &p = *params;
  if (!cell_type || !phi || !rho || !u || !bubble_id || (n_bubbles > 0 && !bubbles))
    return fail(FSLBM_EINVAL, "an input array is NULL");
  if (n_bubbles < 0 || n_bubbles > p.max_bubbles)
    return fail(FSLBM_EINVAL, "n_bubbles out of range (max_bubbles)");
  Launchers L;
  launchers_for(p.precision, L);
  const Layout lay = make_layout(p, L);
  if (!device_workspace) return fail(FSLBM_EINVAL, "device_workspace is NULL");
  if (((uintptr_t)device_workspace) % 256 != 0)
    return fail(FSLBM_EINVAL, "device_workspace must be 256-byte aligned");
  if (workspace_bytes < lay.total)
    return fail(FSLBM_ENOMEM, "workspace too small: need " + std::to_string(lay.total) + " bytes");

  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const long long N = (long long)nx * ny * nz;
  const int n3[3] = {nx, ny, nz};
  auto nb = [&](long long i, int a) -> long long {
    int c[3] = {(int)(i % nx), (int)((i / nx) % ny), (int)(i / ((long long)nx * ny))};
    const int dc[3] = {HOST_CX[a], HOST_CY[a], HOST_CZ[a]};
    for (int k = 0; k < 3; ++k) {
      c[k] += dc[k];
      if (p.periodic[k]) c[k] = (c[k] % n3[k] + n3[k]) % n3[k];
      if (c[k] < 0 || c[k] >= n3[k]) return -1;
    }
    return c[0] + (long long)nx * (c[1] + (long long)ny * c[2]);
  };
  auto gasreg = [](uint8_t t) { return t == T_GAS || t == T_IFACE || t == T_INLET; };

  // ---- validation (same rules as the problem statement: closed interface
  // layer, walls only on non-periodic faces, consistent bubble IDs)
  std::vector<int> slot_of_index(n_bubbles);
  int32_t max_id = -1;
  for (int k = 0; k < n_bubbles; ++k) {
    if (bubbles[k].id < 0) return fail(FSLBM_EINVAL, "bubble IDs must be >= 0");
    for (int j = 0; j < k; ++j)
      if (bubbles[j].id == bubbles[k].id) return fail(FSLBM_EINVAL, "duplicate bubble ID");
    max_id = std::max(max_id, bubbles[k].id);
  }
  auto slot_of_id = [&](int32_t id) -> int {
    for (int k = 0; k < n_bubbles; ++k)
      if (bubbles[k].id == id) return k;
    return -1;
  };
  std::vector<uint8_t> flag(N);
  std::vector<int32_t> bslot(N, -1);
  char msg[256];
  for (long long i = 0; i < N; ++i) {
    const uint8_t t = cell_type[i];
    const int c[3] = {(int)(i % nx), (int)((i / nx) % ny), (int)(i / ((long long)nx * ny))};
    if (t > T_INLET) {
      snprintf(msg, sizeof msg, "cell %lld: unknown type %d", i, t);
      return fail(FSLBM_EINVAL, msg);
    }
    bool face = false;
    for (int k = 0; k < 3; ++k)
      if (!p.periodic[k] && (c[k] == 0 || c[k] == n3[k] - 1)) face = true;
    if (face && t != T_WALL && t != T_INLET) {
      snprintf(msg, sizeof msg, "cell %lld: non-periodic face layer must be wall or inlet", i);
      return fail(FSLBM_EINVAL, msg);
    }
    if (!face && t == T_WALL) {
      snprintf(msg, sizeof msg, "cell %lld: walls only on non-periodic face layers", i);
      return fail(FSLBM_EINVAL, msg);
    }
    if (t == T_IFACE && !std::isfinite(phi[i])) {
      snprintf(msg, sizeof msg, "cell %lld: interface fill level not finite", i);
      return fail(FSLBM_EINVAL, msg);
    }
    if ((t == T_IFACE || t == T_LIQ) && !(rho[i] > 0.0)) {
      snprintf(msg, sizeof msg, "cell %lld: density must be positive", i);
      return fail(FSLBM_EINVAL, msg);
    }
    if (gasreg(t)) {
      const int s = slot_of_id(bubble_id[i]);
      if (s < 0) {
        snprintf(msg, sizeof msg, "cell %lld: bubble ID %d not listed", i, bubble_id[i]);
        return fail(FSLBM_EINVAL, msg);
      }
      bslot[i] = s;
    }
    uint8_t f = t;
    for (int a = 1; a < Q; ++a) {
      const long long j = nb(i, a);
      if (j < 0) continue;
      const uint8_t tj = cell_type[j];
      if (tj == T_WALL) f |= NEAR_WALL;
      if (tj == T_INLET) f |= NEAR_INLET;
      if (t == T_LIQ && (tj == T_GAS || tj == T_INLET) &&
          !(p.debug_flags & FSLBM_DEBUG_NO_LAYER_CHECK)) {
        snprintf(msg, sizeof msg, "cell %lld: liquid next to gas", i);
        return fail(FSLBM_EINVAL, msg);
      }
      if (gasreg(t) && gasreg(tj) && bubble_id[i] != bubble_id[j]) {
        snprintf(msg, sizeof msg, "cells %lld/%lld: touching gas cells with different IDs", i, j);
        return fail(FSLBM_EINVAL, msg);
      }
    }
    flag[i] = f;
  }

  // ---- initial bubble table (volumes summed in cell order)
  const int B = p.max_bubbles;
  std::vector<int32_t> b_id(B, 0), b_flags(B, 0), b_live(B, 0);
  std::vector<double> b_vol(B, 0.0), b_vstar(B, 0.0), b_p(B, 0.0);
  std::vector<long long> b_ngas(B, 0), b_niface(B, 0);
  // exactly rounded volume sums, as in every step
  std::vector<long long> vw((size_t)B * EX_WORDS, 0);
  for (long long i = 0; i < N; ++i) {
    const uint8_t t = cell_type[i];
    if (!gasreg(t)) continue;
    const int s = bslot[i];
    const ExTerm term = ex_split(t == T_IFACE ? 1.0 - phi[i] : 1.0);
    for (int c = 0; c < EX_WORDS; ++c) vw[(size_t)s * EX_WORDS + c] += term.w[c];
    if (t == T_IFACE) b_niface[s] += 1;
    else b_ngas[s] += 1;
  }
  for (int s = 0; s < n_bubbles; ++s) b_vol[s] = ex_value(&vw[(size_t)s * EX_WORDS]);
  for (int k = 0; k < n_bubbles; ++k) {
    b_id[k] = bubbles[k].id;
    b_flags[k] = bubbles[k].flags & (FSLBM_BUBBLE_INLET | FSLBM_BUBBLE_ATMOSPHERE);
    b_live[k] = 1;
    b_vstar[k] = bubbles[k].v_star > 0.0 ? bubbles[k].v_star : b_vol[k] * bubbles[k].p_init / p.p0;
    const double v = b_vol[k] > 1e-2 ? b_vol[k] : 1e-2;
    b_p[k] = (b_flags[k] & FSLBM_BUBBLE_ATMOSPHERE) ? p.p0 : p.p0 * b_vstar[k] / v;
  }

  // ---- fields
  std::vector<double> phi_h(N), mass_h(N), rhoi_h(N, 0.0);
  std::vector<int32_t> ilist, islot(N, 0);
  long long n_iface = 0;
  long long Mw[EX_WORDS] = {0, 0, 0, 0, 0};
  auto madd = [&](double v) {
    const ExTerm t = ex_split(v);
    for (int c = 0; c < EX_WORDS; ++c) Mw[c] += t.w[c];
  };
  for (long long i = 0; i < N; ++i) {
    const uint8_t t = cell_type[i];
    if (t == T_IFACE) {
      phi_h[i] = phi[i];
      mass_h[i] = mass_init ? mass_init[i] : phi[i] * rho[i];
      rhoi_h[i] = rho[i];
      madd(mass_h[i]);
      islot[i] = (int32_t)ilist.size();
      ilist.push_back((int32_t)i);
      ++n_iface;
    } else if (t == T_LIQ) {
      phi_h[i] = 1.0;
      mass_h[i] = rho[i];
      madd(mass_h[i]);
    } else {
      phi_h[i] = 0.0;
      mass_h[i] = 0.0;
    }
  }
  if (n_iface > iface_capacity(p))
    return fail(FSLBM_ECAPACITY, "the initial state has " + std::to_string(n_iface) +
                                     " interface cells, more than iface_capacity (" +
                                     std::to_string(iface_capacity(p)) + ")");

  Ctx *c = new Ctx();
  c->P = p;
  c->L = L;
  c->cfg = make_cfg(p);
  c->lay = lay;
  c->N = N;
  c->stream = (hipStream_t)stream;
  c->ws = (char *)device_workspace;
  build_devs(*c);
  c->cur = 0;
  c->host_step = restore ? restore->step : 0;
  const Dev &d = c->dev[0];
  hipStream_t st = c->stream;
  auto cleanup_fail = [&](int code) {
    delete c;
    return code;
  };
#define UP(dst, src, bytes) \
  do { hipError_t e_ = hipMemcpyAsync((dst), (src), (bytes), hipMemcpyHostToDevice, st); \
       if (e_ != hipSuccess) { fail(FSLBM_EDEVICE, std::string("upload: ") + hipGetErrorString(e_)); \
                               return cleanup_fail(FSLBM_EDEVICE); } } while (0)
  // zero everything first (not captured in any graph)
  {
    hipError_t e = hipMemsetAsync(c->ws, 0, lay.total, st);
    if (e != hipSuccess) {
      fail(FSLBM_EDEVICE, std::string("memset: ") + hipGetErrorString(e));
      return cleanup_fail(FSLBM_EDEVICE);
    }
  }
  {
    // labels: -1 outside the labelled set of a step (see k_label_init)
    hipError_t e = hipMemsetAsync(d.lab, 0xFF, (size_t)N * 4, st);
    if (e != hipSuccess) {
      fail(FSLBM_EDEVICE, std::string("memset: ") + hipGetErrorString(e));
      return cleanup_fail(FSLBM_EDEVICE);
    }
  }
  UP(d.flag_src, flag.data(), N);
  UP(d.flag_dst, flag.data(), N);
  std::vector<char> phi_p = pack_real<double>(phi_h, L.real_bytes);
  std::vector<char> mass_p = pack_real<double>(mass_h, L.real_bytes);
  std::vector<char> rhoi_p = pack_real<double>(rhoi_h, L.real_bytes);
  UP(d.phi_src, phi_p.data(), phi_p.size());
  UP(d.phi_dst, phi_p.data(), phi_p.size());
  UP(d.mass, mass_p.data(), mass_p.size());
  UP(d.rhoI, rhoi_p.data(), rhoi_p.size());
  UP(d.bslot, bslot.data(), N * 4);
  if (!ilist.empty()) UP(d.ilist_src, ilist.data(), ilist.size() * 4);
  UP(d.islot, islot.data(), N * 4);
  UP(d.b_id, b_id.data(), B * 4);
  UP(d.b_flags, b_flags.data(), B * 4);
  UP(d.b_live, b_live.data(), B * 4);
  UP(d.b_vol, b_vol.data(), B * 8);
  UP(d.b_vstar, b_vstar.data(), B * 8);
  UP(d.b_p, b_p.data(), B * 8);
  UP(d.b_ngas, b_ngas.data(), B * 8);
  UP(d.b_niface, b_niface.data(), B * 8);
  Scalars sc{};
  sc.step = restore ? restore->step : 0;
  sc.next_id = std::max(restore ? restore->next_id : 0, max_id + 1);
  sc.bucket = restore ? restore->bucket : 0.0;
  sc.n_iface = n_iface;
  sc.share = n_iface > 0 ? sc.bucket / (double)n_iface : 0.0;
  madd(sc.bucket);
  sc.total_mass = ex_value(Mw);
  sc.mass_ref = sc.total_mass;
  sc.n_live = n_bubbles;
  sc.label_run = 2;  // the first step labels the whole gas region
  sc.n_il_src = (int)n_iface;
  UP(d.sc, &sc, sizeof sc);
  // PDFs, through the destination lattice as FP64 staging
  double *staging = (double *)d.f_dst;
  if (f_init) {
    for (int a = 0; a < Q; ++a) {
      UP(staging, f_init + (size_t)a * N, N * 8);
      c->L.init_f(d, c->cfg, staging, a, st);
    }
  } else {
    UP(staging, rho, N * 8);
    UP(staging + N, u, 3 * N * 8);
    c->L.init_feq(d, c->cfg, staging, staging + N, st);
  }
  {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
      fail(FSLBM_EDEVICE, std::string("create: ") + hipGetErrorString(e));
      return cleanup_fail(FSLBM_EDEVICE);
    }
  }
#undef UP
  *out_handle = c;
  g_err.clear();
  return FSLBM_OK;
}

int fslbm_step(void *handle, int32_t n_steps) {
  if (!handle) return fail(FSLBM_EINVAL, "handle is NULL");
  if (n_steps < 0) return fail(FSLBM_EINVAL, "n_steps < 0");
  Ctx &c = *(Ctx *)handle;
  for (int s = 0; s < n_steps; ++s) {
    const Dev &d = c.dev[c.cur];
    if (c.timing_period > 0 && c.timing_count++ % c.timing_period == 0) {
      for (int ph = 0; ph < PH_COUNT; ++ph) {
        if (!((c.timing_mask >> ph) & 1u)) {
          c.L.phase(ph, d, c.cfg, c.stream);
          continue;
        }
        while (c.events.size() < 2 * (c.used + 1)) {
          hipEvent_t e;
          HIP_TRY(hipEventCreate(&e));
          c.events.push_back(e);
        }
        if (c.event_phase.size() < c.used + 1) c.event_phase.resize(c.used + 1);
        HIP_TRY(hipEventRecord(c.events[2 * c.used], c.stream));
        c.L.phase(ph, d, c.cfg, c.stream);
        HIP_TRY(hipEventRecord(c.events[2 * c.used + 1], c.stream));
        c.event_phase[c.used] = ph;
        c.used += 1;
      }
      c.timed_steps += 1;
    } else {
      for (int ph = 0; ph < PH_COUNT; ++ph) c.L.phase(ph, d, c.cfg, c.stream);
    }
    c.cur ^= 1;
    c.host_step += 1;
    if (watchdog_due(c)) {
      c.L.watchdog(c.dev[c.cur], c.cfg, c.stream);
      HIP_TRY(hipGetLastError());
      const int rc = sync_and_check(c);
      if (rc != FSLBM_OK) return rc;
    }
  }
  HIP_TRY(hipGetLastError());
  return FSLBM_OK;
}

int fslbm_set_timing(void *handle, int32_t period, uint32_t phase_mask) {
  if (!handle) return fail(FSLBM_EINVAL, "handle is NULL");
  if (period < 0) return fail(FSLBM_EINVAL, "timing period < 0");
  if (phase_mask & ~(uint32_t)FSLBM_PHASE_ALL) return fail(FSLBM_EINVAL, "unknown phase bits");
  Ctx &c = *(Ctx *)handle;
  HIP_TRY(hipStreamSynchronize(c.stream));
  c.timing_period = period;
  c.timing_mask = phase_mask ? phase_mask : (uint32_t)FSLBM_PHASE_ALL;
  c.timing_count = 0;
  c.timed_steps = 0;
  c.used = 0;
  return FSLBM_OK;
}

int fslbm_get_timing(void *handle, fslbm_timing *out) {
  if (!handle || !out) return fail(FSLBM_EINVAL, "NULL argument");
  Ctx &c = *(Ctx *)handle;
  HIP_TRY(hipStreamSynchronize(c.stream));
  double ms[PH_COUNT] = {0};
  for (size_t k = 0; k < c.used; ++k) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, c.events[2 * k], c.events[2 * k + 1]));
    ms[c.event_phase[k]] += t;
  }
  out->steps = (int64_t)c.timed_steps;
  out->bulk_ms = ms[PH_BULK];
  out->iface_ms = ms[PH_IFACE];
  out->convert_ms = ms[PH_CONVERT];
  out->excess_ms = ms[PH_EXCESS];
  out->gather_ms = ms[PH_GATHER];
  out->label_ms = ms[PH_LABEL];
  out->bubbles_ms = ms[PH_BUBBLES];
  double tot = 0.0;
  for (int ph = 0; ph < PH_COUNT; ++ph) tot += ms[ph];
  out->step_ms = tot;
  c.used = 0;
  c.timed_steps = 0;
  return FSLBM_OK;
}

int fslbm_sync(void *handle) {
  if (!handle) return fail(FSLBM_EINVAL, "handle is NULL");
  return sync_and_check(*(Ctx *)handle);
}

int fslbm_read_fields(void *handle, uint8_t *cell_type, double *phi, double *mass, double *f,
                      int32_t *bubble_id, double *rho, double *u, fslbm_scalars *scalars) {
  if (!handle) return fail(FSLBM_EINVAL, "handle is NULL");
  Ctx &c = *(Ctx *)handle;
  int rc = sync_and_check(c);
  if (rc != FSLBM_OK) return rc;
  const Dev &d = c.dev[c.cur];
  const long long N = c.N;
  double *staging = (double *)d.f_dst;
  auto fetch = [&](int what, double *out) -> int {
    c.L.exportq(d, c.cfg, staging, what, c.stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, staging, N * 8, hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
    return FSLBM_OK;
  };
  if (cell_type) {
    HIP_TRY(hipMemcpy(cell_type, d.flag_src, N, hipMemcpyDeviceToHost));
    for (long long i = 0; i < N; ++i) cell_type[i] &= TYPE_MASK;
  }
  if (phi && (rc = fetch(0, phi))) return rc;
  if (mass && (rc = fetch(1, mass))) return rc;
  if (rho && (rc = fetch(2, rho))) return rc;
  if (u)
    for (int k = 0; k < 3; ++k)
      if ((rc = fetch(3 + k, u + k * N))) return rc;
  if (f)
    for (int a = 0; a < Q; ++a)
      if ((rc = fetch(6 + a, f + (size_t)a * N))) return rc;
  if (bubble_id) {
    std::vector<int32_t> slot(N), ids(c.P.max_bubbles);
    HIP_TRY(hipMemcpy(slot.data(), d.bslot, N * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ids.data(), d.b_id, c.P.max_bubbles * 4, hipMemcpyDeviceToHost));
    std::vector<uint8_t> t(N);
    HIP_TRY(hipMemcpy(t.data(), d.flag_src, N, hipMemcpyDeviceToHost));
    for (long long i = 0; i < N; ++i) {
      const uint8_t ty = t[i] & TYPE_MASK;
      const bool g = ty == T_GAS || ty == T_IFACE || ty == T_INLET;
      bubble_id[i] = (g && slot[i] >= 0) ? ids[slot[i]] : -1;
    }
  }
  if (scalars) {
    Scalars sc;
    HIP_TRY(hipMemcpy(&sc, d.sc, sizeof sc, hipMemcpyDeviceToHost));
    scalars->step = sc.step;
    scalars->next_id = sc.next_id;
    scalars->n_bubbles = sc.n_live;
    scalars->bucket = sc.bucket;
    scalars->total_mass = sc.total_mass;
    scalars->n_topology = sc.n_topology;
    scalars->n_label_runs = sc.n_label_runs;
  }
  return FSLBM_OK;
}

int fslbm_bubbles(void *handle, fslbm_bubble *out, int32_t capacity, int32_t *n_out) {
  if (!handle) return fail(FSLBM_EINVAL, "handle is NULL");
  Ctx &c = *(Ctx *)handle;
  int rc = sync_and_check(c);
  if (rc != FSLBM_OK) return rc;
  const Dev &d = c.dev[c.cur];
  const int B = c.P.max_bubbles;
  std::vector<int32_t> id(B), fl(B), live(B);
  std::vector<double> vol(B), vs(B), pr(B);
  std::vector<long long> ng(B), ni(B);
  HIP_TRY(hipMemcpy(id.data(), d.b_id, B * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(fl.data(), d.b_flags, B * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(live.data(), d.b_live, B * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(vol.data(), d.b_vol, B * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(vs.data(), d.b_vstar, B * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(pr.data(), d.b_p, B * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ng.data(), d.b_ngas, B * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(ni.data(), d.b_niface, B * 8, hipMemcpyDeviceToHost));
  std::vector<fslbm_bubble> v;
  for (int s = 0; s < B; ++s)
    if (live[s]) v.push_back(fslbm_bubble{id[s], fl[s], vol[s], vs[s], pr[s], ng[s] + ni[s]});
  std::sort(v.begin(), v.end(), [](const fslbm_bubble &a, const fslbm_bubble &b) { return a.id < b.id; });
  if (n_out) *n_out = (int32_t)v.size();
  if ((int32_t)v.size() > capacity) return fail(FSLBM_ECAPACITY, "output capacity too small");
  if (out) std::copy(v.begin(), v.end(), out);
  return FSLBM_OK;
}

int fslbm_copy_bandwidth(void *dst, const void *src, size_t bytes, int32_t reps, void *stream,
                         double *gbs_out) {
  if (!dst || !src || !gbs_out) return fail(FSLBM_EINVAL, "NULL argument");
  if (bytes == 0 || bytes % 16 || reps < 1) return fail(FSLBM_EINVAL, "bytes or reps out of range");
  if (((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
    return fail(FSLBM_EINVAL, "buffers must be 16-byte aligned");
  const long long n = (long long)(bytes / 16);
  // about four vectors per thread over the grid
  const long long want = (n + 4 * 256 - 1) / (4 * 256);
  const int blocks = (int)(want < 1 ? 1 : (want > 65536 ? 65536 : want));
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  // one untimed pass first
  k_copy_stream<<<blocks, 256, 0, st>>>((const v4u *)src, (v4u *)dst, n);
  HIP_TRY(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) k_copy_stream<<<blocks, 256, 0, st>>>((const v4u *)src, (v4u *)dst, n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *gbs_out = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
  return FSLBM_OK;
}

int fslbm_destroy(void *handle) {
  if (!handle) return fail(FSLBM_EINVAL, "handle is NULL");
  Ctx *c = (Ctx *)handle;
  hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->events) hipEventDestroy(e);
  delete c;
  return FSLBM_OK;
}

size_t fslbm_batch_workspace_bytes(int32_t n_domains) {
  if (n_domains < 1) return 0;
  return batch_bytes(n_domains);
}

int fslbm_batch_create(void *const *handles, int32_t n, const char *tuning_cache_path,
                       void *device_workspace, size_t workspace_bytes, void *stream,
                       void **out_batch) {
  if (!out_batch) return fail(FSLBM_EINVAL, "out_batch is NULL");
  *out_batch = nullptr;
  if (!handles || n < 1) return fail(FSLBM_EINVAL, "no handles");
  if (!device_workspace || ((uintptr_t)device_workspace & 255))
    return fail(FSLBM_EINVAL, "device_workspace must be 256-byte aligned");
  if (workspace_bytes < batch_bytes(n)) return fail(FSLBM_ENOMEM, "batch workspace too small");
  std::vector<Ctx *> given(n);
  for (int k = 0; k < n; ++k) {
    if (!handles[k]) return fail(FSLBM_EINVAL, "a handle is NULL");
    given[k] = (Ctx *)handles[k];
    for (int j = 0; j < k; ++j)
      if (given[j] == given[k]) return fail(FSLBM_EINVAL, "a handle is listed twice");
    if (given[k]->P.precision != given[0]->P.precision)
      return fail(FSLBM_EINVAL, "all domains of a batch must have the same precision");
  }
  Batch *b = new Batch();
  b->precision = given[0]->P.precision;
  b->L = given[0]->L;
  b->user_stream = (hipStream_t)stream;
  b->ws = (char *)device_workspace;
  b->cap = batch_capacity(workspace_bytes);
  auto bail = [&](int code) {
    std::string msg = g_err;
    batch_free(b);
    g_err = msg;
    return code;
  };
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
    fail(FSLBM_EDEVICE, "batch: stream or event creation failed");
    return bail(FSLBM_EDEVICE);
  }
  for (int k = 0; k < 2; ++k) {
    if (hipHostMalloc((void **)&b->stage[k], batch_bytes(b->cap), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&b->stage_ev[k], hipEventDisableTiming) != hipSuccess) {
      fail(FSLBM_EDEVICE, "batch: pinned staging or event creation failed");
      return bail(FSLBM_EDEVICE);
    }
    // a recorded event that has completed: the buffer is free
    if (hipEventRecord(b->stage_ev[k], b->stream) != hipSuccess) {
      fail(FSLBM_EDEVICE, "batch: event record failed");
      return bail(FSLBM_EDEVICE);
    }
  }
  // finish whatever the domains' own streams hold (creation uploads)
  for (Ctx *c : given)
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
      fail(FSLBM_EDEVICE, "batch: domain stream sync failed");
      return bail(FSLBM_EDEVICE);
    }
  long long cells = 0;
  for (Ctx *c : given) cells += c->N;
  b->info.cells = cells;
  // autotuning: stream-collide block size and block-to-domain order
  b->dom = given;
  const std::string key = batch_key(*b);
  int threads = 256, order = 0, list_cells = 2048;
  if (tuning_cache_path && !tuning_cache_path[0]) {
    // "": no tuning (callers that rebuild batches often)
  } else if (batch_cache_lookup(tuning_cache_path, key, threads, order, list_cells)) {
    b->info.from_cache = 1;
  } else {
    // the stream-collide grid (block size x domain order), then the list
    // kernels' grid density with the chosen order; the two grids are
    // independent, so 9 probes cover the 18 points
    float best = 1e30f;
    int ci = 0;
    for (int t : {256, 128})
      for (int o : {0, 1, 2}) {
        batch_order(*b, given, o);
        int rc = batch_tables(*b, t);
        float ms = 0.f;
        if (rc == FSLBM_OK) rc = batch_probe(*b, 5, ms);
        if (rc != FSLBM_OK) return bail(rc);
        b->info.probe_ms[ci++] = ms;
        if (ms < best) {
          best = ms;
          threads = t;
          order = o;
        }
      }
    batch_order(*b, given, order);
    best = 1e30f;
    for (int l : {1024, 2048, 4096}) {
      int rc = batch_tables(*b, threads, l);
      float ms = 0.f;
      if (rc == FSLBM_OK) rc = batch_probe(*b, 5, ms, true);
      if (rc != FSLBM_OK) return bail(rc);
      b->info.probe_ms[ci++] = ms;
      if (ms < best) {
        best = ms;
        list_cells = l;
      }
    }
    batch_cache_store(tuning_cache_path, key, threads, order, list_cells);
  }
  b->info.bulk_threads = threads;
  b->info.order = order;
  b->info.list_cells = list_cells;
  batch_order(*b, given, order);
  int rc = batch_tables(*b, threads, list_cells);
  if (rc == FSLBM_OK) rc = batch_capture(*b);
  if (rc == FSLBM_OK && hipStreamSynchronize(b->stream) != hipSuccess) {
    fail(FSLBM_EDEVICE, "batch: table upload failed");
    rc = FSLBM_EDEVICE;
  }
  if (rc != FSLBM_OK) return bail(rc);
  *out_batch = b;
  g_err.clear();
  return FSLBM_OK;
}

int fslbm_batch_create_noalloc(void *const *handles, int32_t n, void *stream, void **out_batch) {
  if (!out_batch) return fail(FSLBM_EINVAL, "out_batch is NULL");
  *out_batch = nullptr;
  if (!handles || n < 1) return fail(FSLBM_EINVAL, "no handles");
  if (batch_bytes(n) > SCRATCH_BYTES)
    return fail(FSLBM_EINVAL, "too many domains for the static batch tables: " + std::to_string(n) +
                                  " domains need " + std::to_string(batch_bytes(n)) +
                                  " bytes, the array holds " + std::to_string(SCRATCH_BYTES));
  std::vector<Ctx *> given(n);
  for (int k = 0; k < n; ++k) {
    if (!handles[k]) return fail(FSLBM_EINVAL, "a handle is NULL");
    given[k] = (Ctx *)handles[k];
    for (int j = 0; j < k; ++j)
      if (given[j] == given[k]) return fail(FSLBM_EINVAL, "a handle is listed twice");
    if (given[k]->P.precision != given[0]->P.precision)
      return fail(FSLBM_EINVAL, "all domains of a batch must have the same precision");
    if (given[k]->stream != (hipStream_t)stream)
      return fail(FSLBM_EINVAL, "every domain must have been created on the batch's stream");
  }
  void *ptr = nullptr;
  if (int rc = scratch_address(&ptr)) return rc;
  Batch *b = new Batch();
  b->in_scratch = true;
  b->precision = given[0]->P.precision;
  b->L = given[0]->L;
  b->user_stream = (hipStream_t)stream;
  b->stream = (hipStream_t)stream;
  b->ws = (char *)ptr;
  b->dom = given;
  long long cells = 0;
  for (Ctx *c : given) cells += c->N;
  b->info.cells = cells;
  b->info.bulk_threads = 256;
  b->info.list_cells = 2048;
  b->cap = batch_capacity(SCRATCH_BYTES);
  int rc = batch_tables(*b, 256);
  if (rc != FSLBM_OK) {
    delete b;
    return rc;
  }
  *out_batch = b;
  g_err.clear();
  return FSLBM_OK;
}

int fslbm_batch_step(void *batch, int32_t n_steps) {
  if (!batch) return fail(FSLBM_EINVAL, "batch is NULL");
  if (n_steps < 0) return fail(FSLBM_EINVAL, "n_steps < 0");
  Batch &b = *(Batch *)batch;
  if (n_steps == 0) return FSLBM_OK;
  // a domain stepped on its own since the tables were built shifts its
  // parity: rebuild the tables and graphs
  const int nd = (int)b.dom.size();
  const int r0 = (b.dom[0]->cur - b.base_cur[0]) & 1;
  bool same = true;
  for (int k = 1; k < nd; ++k) same = same && (((b.dom[k]->cur - b.base_cur[k]) & 1) == r0);
  int r = r0;
  if (!same) {
    int rc = batch_tables(b, b.info.bulk_threads, b.info.list_cells);
    if (rc == FSLBM_OK && !b.in_scratch && !b.direct) rc = batch_capture(b);
    if (rc != FSLBM_OK) return rc;
    r = 0;
  }
  // order after the work already queued on the caller's and the domains'
  // streams, and before whatever they queue next (a batch in the scratch
  // array runs on the one stream of the caller and its domains)
  std::vector<hipStream_t> streams{b.user_stream};
  if (!b.in_scratch) {
    for (Ctx *c : b.dom)
      if (std::find(streams.begin(), streams.end(), c->stream) == streams.end())
        streams.push_back(c->stream);
    for (hipStream_t st : streams) {
      HIP_TRY(hipEventRecord(b.ev_in, st));
      HIP_TRY(hipStreamWaitEvent(b.stream, b.ev_in, 0));
    }
  }
  int rc = FSLBM_OK;
  int done = 0;
  for (int s = 0; s < n_steps && rc == FSLBM_OK; ++s) {
    if (b.in_scratch || b.direct) {
      for (int ph = 0; ph < PH_COUNT; ++ph) b.L.batch_phase(ph, b.cfg[(r + s) & 1], b.stream);
    } else {
      HIP_TRY(hipGraphLaunch(b.exec[(r + s) & 1], b.stream));
    }
    done = s + 1;
    // the watchdog of every member whose check is due after this step
    bool due = false;
    for (Ctx *c : b.dom) {
      c->host_step += 1;
      if (watchdog_due(*c)) {
        c->L.watchdog(c->dev[c->cur ^ (done & 1)], c->cfg, b.stream);
        due = true;
      }
    }
    if (due) {
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipStreamSynchronize(b.stream));
      for (size_t k = 0; k < b.dom.size() && rc == FSLBM_OK; ++k) {
        Ctx &c = *b.dom[k];
        if (!watchdog_due(c)) continue;
        Scalars sc;
        HIP_TRY(hipMemcpy(&sc, c.dev[0].sc, sizeof sc, hipMemcpyDeviceToHost));
        if (sc.err) {
          // the same message as the domain's own calls give
          HIP_TRY(hipStreamSynchronize(c.stream));
          rc = sync_and_check(c);
          if (rc != FSLBM_OK) g_err = "batch member " + std::to_string(k) + ": " + g_err;
        }
      }
    }
  }
  if (!b.in_scratch) {
    HIP_TRY(hipEventRecord(b.ev_out, b.stream));
    for (hipStream_t st : streams) HIP_TRY(hipStreamWaitEvent(st, b.ev_out, 0));
  }
  for (Ctx *c : b.dom) c->cur ^= (done & 1);
  return rc;
}

int fslbm_batch_reset(void *batch, void *const *handles, int32_t n) {
  if (!batch) return fail(FSLBM_EINVAL, "batch is NULL");
  Batch &b = *(Batch *)batch;
  if (!handles || n < 1) return fail(FSLBM_EINVAL, "no handles");
  if (n > b.cap)
    return fail(FSLBM_EINVAL, "batch reset: " + std::to_string(n) + " domains, the table space holds " +
                                  std::to_string(b.cap));
  std::vector<Ctx *> given(n);
  for (int k = 0; k < n; ++k) {
    if (!handles[k]) return fail(FSLBM_EINVAL, "a handle is NULL");
    given[k] = (Ctx *)handles[k];
    for (int j = 0; j < k; ++j)
      if (given[j] == given[k]) return fail(FSLBM_EINVAL, "a handle is listed twice");
    if (given[k]->P.precision != b.precision)
      return fail(FSLBM_EINVAL, "all domains of a batch must have the same precision");
    if (b.in_scratch && given[k]->stream != b.stream)
      return fail(FSLBM_EINVAL, "every domain must have been created on the batch's stream");
  }
  // from now on steps are plain launches: the tables change in place
  batch_drop_graphs(b);
  b.direct = true;
  b.dom = given;
  long long cells = 0;
  for (Ctx *c : given) cells += c->N;
  b.info.cells = cells;
  return batch_tables(b, b.info.bulk_threads, b.info.list_cells);
}

int fslbm_batch_info_get(void *batch, fslbm_batch_info *out) {
  if (!batch || !out) return fail(FSLBM_EINVAL, "NULL argument");
  *out = ((Batch *)batch)->info;
  return FSLBM_OK;
}

int fslbm_batch_destroy(void *batch) {
  if (!batch) return fail(FSLBM_EINVAL, "batch is NULL");
  batch_free((Batch *)batch);
  return FSLBM_OK;
}

}  // extern "C"
