// Host runtime behind the C ABI (include/gpf.h): contexts, plans, bodies,
// batches, and the launch sequence of a solve.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "gpf_internal.h"

namespace gpf {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
gpf_status fail(gpf_status st, const std::string &msg) {
  set_error(msg);
  return st;
}

DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}
gpf_status DevBuf::alloc(size_t nbytes) {
  if (p) {
    if (bytes >= nbytes) return GPF_OK;
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  if (nbytes == 0) nbytes = 256;
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    return fail(GPF_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  bytes = nbytes;
  return GPF_OK;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
static thread_local KernelTimer *g_timer = nullptr;

void timer_install(KernelTimer *t) { g_timer = t; }

// more events for a timer whose pool runs short (host-side creation only)
static bool timer_refill(KernelTimer *t) {
  for (int i = 0; i < 1024; ++i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) break;
    t->pool.push_back(e);
  }
  return t->pool.size() >= 2;
}

void timer_begin(int kind, hipStream_t s) {
  KernelTimer *t = g_timer;
  if (!t || (t->pool.size() < 2 && !timer_refill(t))) return;  // no timer, or out of events
  hipEvent_t a = t->pool.back();
  t->pool.pop_back();
  if (hipEventRecord(a, s) != hipSuccess) {
    t->pool.push_back(a);
    return;
  }
  t->open_a = a;
  t->open_kind = kind;
}

void timer_end(hipStream_t s) {
  KernelTimer *t = g_timer;
  if (!t || !t->open_a) return;
  if (t->pool.empty() && !timer_refill(t)) {
    t->pool.push_back(t->open_a);
    t->open_a = nullptr;
    return;
  }
  hipEvent_t b = t->pool.back();
  t->pool.pop_back();
  (void)hipEventRecord(b, s);
  t->pending.push_back({t->open_a, b, t->open_kind});
  t->open_a = nullptr;
}

KernelTimer::~KernelTimer() {
  for (auto &r : pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

void KernelTimer::reset() {
  for (int k = 0; k < GPF_TK_COUNT; ++k) {
    total_ms[k] = 0.0;
    count[k] = 0;
  }
  for (auto &r : pending) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
  while (pool.size() < 8192) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) break;
    pool.push_back(e);
  }
}

gpf_status KernelTimer::flush() {
  for (auto &r : pending) {
    GPF_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    GPF_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    total_ms[r.kind] += ms;
    count[r.kind] += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  pending.clear();
  return GPF_OK;
}

// ---------------------------------------------------------------------------
// descriptor ring
// ---------------------------------------------------------------------------
DescRing::~DescRing() {
  for (auto e : ev) (void)hipEventDestroy(e);
  if (host) (void)hipHostFree(host);
}

gpf_status DescRing::init(int nslots, size_t bytes_per_slot) {
  slots = nslots;
  slot_bytes = (bytes_per_slot + 255) / 256 * 256;
  GPF_HIP(hipHostMalloc(reinterpret_cast<void **>(&host), slots * slot_bytes, hipHostMallocDefault));
  GPF_TRY(dev.alloc(slots * slot_bytes));
  ev.resize(slots);
  for (auto &e : ev) GPF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  busy.assign(slots, 0);
  pinned.assign(slots, 0);
  return GPF_OK;
}

gpf_status DescRing::push(const void *src, size_t nbytes, hipStream_t s, void **dptr) {
  if (nbytes > slot_bytes) return fail(GPF_E_INVALID, "descriptor block larger than a ring slot");
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  GPF_HIP(hipStreamIsCapturing(s, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  int slot = -1;
  for (int tries = 0; tries < slots; ++tries) {
    const int k = (next + tries) % slots;
    if (!pinned[k]) {
      slot = k;
      break;
    }
  }
  if (slot < 0) return fail(GPF_E_NOMEM, "all descriptor slots are held by captured graphs");
  next = (slot + 1) % slots;
  if (busy[slot] && !capturing) GPF_HIP(hipEventSynchronize(ev[slot]));
  char *h = host + (size_t)slot * slot_bytes;
  char *d = dev.as<char>() + (size_t)slot * slot_bytes;
  std::memcpy(h, src, nbytes);
  if (capturing && defer_captured)
    deferred.emplace_back(slot, nbytes);   // copied once the capture has ended
  else
    GPF_HIP(hipMemcpyAsync(d, h, nbytes, hipMemcpyHostToDevice, s));
  if (capturing) {
    pinned[slot] = 1;  // the graph reads this slot: keep it until the graph is gone
  } else {
    GPF_HIP(hipEventRecord(ev[slot], s));
    busy[slot] = 1;
  }
  *dptr = d;
  return GPF_OK;
}

gpf_status DescRing::flush_deferred() {
  gpf_status st = GPF_OK;
  for (const auto &p : deferred) {
    const hipError_t e = hipMemcpy(dev.as<char>() + (size_t)p.first * slot_bytes,
                                   host + (size_t)p.first * slot_bytes, p.second,
                                   hipMemcpyHostToDevice);
    if (e != hipSuccess && st == GPF_OK) st = fail(GPF_E_DEVICE, "descriptor copy after capture failed");
  }
  deferred.clear();
  return st;
}

namespace {

// cache of host LGF tables and unscaled spectra, keyed by n
struct HostCache {
  std::mutex mu;
  std::map<int, std::shared_ptr<std::vector<double>>> tables;
  std::map<int, std::pair<double, std::shared_ptr<std::vector<double>>>> spectra;
};
HostCache &cache() {
  static HostCache c;
  return c;
}

std::shared_ptr<std::vector<double>> get_table(int n) {
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto it = cache().tables.find(n);
    if (it != cache().tables.end()) return it->second;
  }
  auto t = std::make_shared<std::vector<double>>((size_t)(n + 1) * (n + 1));
  lgf_table_host(n, t->data());
  std::lock_guard<std::mutex> lk(cache().mu);
  cache().tables[n] = t;
  return t;
}

std::pair<double, std::shared_ptr<std::vector<double>>> get_spectrum(int n) {
  {
    std::lock_guard<std::mutex> lk(cache().mu);
    auto it = cache().spectra.find(n);
    if (it != cache().spectra.end()) return it->second;
  }
  auto tab = get_table(n);
  auto sp = std::make_shared<std::vector<double>>((size_t)(n + 1) * (n + 1));
  double c = lgf_spectrum_host(n, tab->data(), sp->data());
  std::lock_guard<std::mutex> lk(cache().mu);
  cache().spectra[n] = {c, sp};
  return {c, sp};
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
bool is_finite(double v) { return std::isfinite(v); }
hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

int xcd_count(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 1;
  std::string arch = prop.gcnArchName;
  if (arch.rfind("gfx942", 0) == 0 || arch.rfind("gfx950", 0) == 0) return 8;
  return 1;
}

template <class T>
gpf_status upload_spectrum(gpf_plan *p, DevBuf &spec, DevBuf &tw) {
  const int n = p->grid.n, N = 2 * n;
  auto sp = get_spectrum(n);
  p->gauge_c = sp.first;
  const double scale = -p->grid.dx * p->grid.dx / (double(N) * double(N));
  std::vector<T> hs((size_t)(n + 1) * (n + 1));
  for (size_t i = 0; i < hs.size(); ++i) hs[i] = (T)((*sp.second)[i] * scale);
  GPF_TRY(spec.alloc(hs.size() * sizeof(T)));
  GPF_HIP(hipMemcpy(spec.p, hs.data(), hs.size() * sizeof(T), hipMemcpyHostToDevice));
  std::vector<T> ht(2 * (size_t)N);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < N; ++k) {
    ht[2 * k] = (T)std::cos(-2.0 * pi * k / N);
    ht[2 * k + 1] = (T)std::sin(-2.0 * pi * k / N);
  }
  GPF_TRY(tw.alloc(ht.size() * sizeof(T)));
  GPF_HIP(hipMemcpy(tw.p, ht.data(), ht.size() * sizeof(T), hipMemcpyHostToDevice));
  return GPF_OK;
}

// Fill device memory and wait for the fill: the memory is then ready for
// work on any stream, including non-blocking ones, which do not order after
// the null stream that hipMemset runs on.  Used where buffers are created or
// grown, never in a launch sequence.
gpf_status fill_now(void *p, int value, size_t bytes) {
  GPF_HIP(hipMemset(p, value, bytes));
  GPF_HIP(hipStreamSynchronize(nullptr));
  return GPF_OK;
}

constexpr int kPlanRingSlots = 64;
constexpr size_t kProblemDescBytes = sizeof(ProbDesc) + 2 * sizeof(ConvDesc);

}  // namespace
}  // namespace gpf

using namespace gpf;

gpf_status gpf_workspace::ensure(int nn, bool need32, bool need64, int nns, int band) {
  const size_t cells = (size_t)nn * nn, half = (size_t)(nn + 1) * nn;
  // source fields start zeroed; the last reader of a source leaves it zero
  auto zeroed = [&](DevBuf &b, size_t bytes) -> gpf_status {
    if (b.bytes >= bytes) return GPF_OK;
    GPF_TRY(b.alloc(bytes));
    GPF_TRY(fill_now(b.p, 0, b.bytes));
    return GPF_OK;
  };
  if (need32) {
    GPF_TRY(zeroed(w32, cells * 4));
    GPF_TRY(x32.alloc(half * 8));
  }
  if (need64) {
    GPF_TRY(zeroed(w64, cells * 8));
    GPF_TRY(x64.alloc(half * 16));
    GPF_TRY(s64.alloc(cells * 8));
  }
  GPF_TRY(zeroed(aux, AUX_BYTES));
  GPF_TRY(part.alloc(sizeof(double) * 5 * (size_t)kPartStride));
  if (band > 0) GPF_TRY(xb.alloc((size_t)(nn + 1) * band * 16));   // complex FP64 at most
  if (nns > 0) {
    const size_t cols = 1 + GPF_MAX_EDGES;
    GPF_TRY(rhs.alloc(cols * nns * sizeof(double)));
    GPF_TRY(y.alloc(cols * nns * sizeof(double)));
    GPF_TRY(fsurf.alloc(nns * sizeof(double)));
    ns = std::max(ns, nns);
  }
  n = std::max(n, nn);
  return GPF_OK;
}

gpf_status gpf_workspace::ensure_vortices(int nvv) {
  if (n > 0) {
    const size_t tiles = (size_t)bin_tiles(n) + 1;
    if (bin_cnt.bytes < tiles * sizeof(int)) {
      GPF_TRY(bin_cnt.alloc(tiles * sizeof(int)));
      GPF_TRY(fill_now(bin_cnt.p, 0, bin_cnt.bytes));  // counts start (and end) at zero
    }
    GPF_TRY(bin_start.alloc(tiles * sizeof(int)));
  }
  if (nvv > nv || !rank.p) {
    const size_t cap = std::max<size_t>(1024, (size_t)nvv);
    GPF_TRY(rank.alloc(cap * sizeof(int)));
    GPF_TRY(sorted.alloc(4 * cap * sizeof(double)));
    nv = (int)cap;
  }
  if (n > 0) {
    GPF_TRY(items.alloc(4 * sizeof(int) * (1 + (size_t)tile_items_max(n, nv))));
    GPF_TRY(halo.alloc(sizeof(double) * kHaloRing * (size_t)std::max(1, bin_tiles(n))));
  }
  GPF_TRY(splits.alloc(4 * sizeof(int) * (1 + (size_t)split_tiles_max(nv))));
  GPF_TRY(splitwin.alloc(sizeof(long long) * kSplitWin * (size_t)std::max(1, split_items_max(nv))));
  return GPF_OK;
}

gpf_batch::~gpf_batch() {
  for (int l = 0; l < kMaxLanes; ++l) {
    if (lane_stream[l]) (void)hipStreamDestroy(lane_stream[l]);
    if (join_ev[l]) (void)hipEventDestroy(join_ev[l]);
  }
  if (fork_ev) (void)hipEventDestroy(fork_ev);
  if (side) (void)hipStreamDestroy(side);
  if (side_fork) (void)hipEventDestroy(side_fork);
  if (side_join) (void)hipEventDestroy(side_join);
  if (side2) (void)hipStreamDestroy(side2);
  if (side2_join) (void)hipEventDestroy(side2_join);
  for (auto *w : ws) delete w;
}

gpf_status gpf_plan::ensure_fp64() {
  if (!spec64.p) GPF_TRY(upload_spectrum<double>(this, spec64, tw64));
  return ws.ensure(grid.n, false, true, 0);
}

// ---------------------------------------------------------------------------
// launch sequence of one group (same n and precision; 1..nb problems)
// ---------------------------------------------------------------------------
namespace gpf {
namespace {

struct GroupCfg {
  int n = 0;
  bool body = false;
  bool fp64_plan = false;  // all fields FP64
  bool conv1_fp64 = false; // FP32 plan with an FP64 first convolution
  bool parts = false;      // a body of several parts (GPF_PARTS)
};

struct ProblemRef {
  gpf_plan *plan;
  const gpf_body *body;
  const gpf_inputs *in;
  const gpf_outputs *out;
  gpf_workspace *ws;
  int znew_from = -1;   // >= 0: the new vortices are vortices znew_from.. of in
  const double *pgw_dev = nullptr;   // GPF_PARTS: per-part Gamma_w on the device
};

GroupCfg config_of(const ProblemRef &r) {
  GroupCfg c;
  c.n = r.plan->grid.n;
  c.body = r.in->mode != GPF_NOBODY;
  c.fp64_plan = r.plan->fp64;
  c.conv1_fp64 = !c.fp64_plan && c.body && r.body->conv1_fp64;
  c.parts = r.in->mode == GPF_PARTS;
  return c;
}

bool same_cfg(const GroupCfg &a, const GroupCfg &b) {
  return a.n == b.n && a.body == b.body && a.fp64_plan == b.fp64_plan &&
         a.conv1_fp64 == b.conv1_fp64 && a.parts == b.parts;
}

// rows of a body's band: the 16-row groups spanning its surface stencils
int body_band(const gpf_body *b) { return (b->row_hi | 15) - (b->row_lo & ~15) + 1; }

// fill the descriptors of one problem
void describe(const ProblemRef &r, const GroupCfg &cfg, ProbDesc &pd, ConvDesc &c1, ConvDesc &c2) {
  const gpf_plan *p = r.plan;
  const gpf_inputs *in = r.in;
  const gpf_outputs *out = r.out;
  gpf_workspace *ws = r.ws;
  const bool w64 = cfg.fp64_plan || cfg.conv1_fp64;
  std::memset(&pd, 0, sizeof(pd));
  std::memset(&c1, 0, sizeof(c1));
  std::memset(&c2, 0, sizeof(c2));
  c1.row_lo = c2.row_lo = 0;
  c1.row_hi = c2.row_hi = p->grid.n - 1;
  c1.fwd_lo = c2.fwd_lo = 0;
  c1.fwd_hi = c2.fwd_hi = p->grid.n - 1;
  c1.keep_lo = c2.keep_lo = 0;   // empty: nothing kept
  c1.keep_end = c2.keep_end = 0;
  pd.n = p->grid.n;
  pd.dx = p->grid.dx;
  pd.x0 = p->grid.x0;
  pd.y0 = p->grid.y0;
  // dense clouds: velocities tile by tile through LDS
  pd.vel_tiles = (long long)in->nv * 4 >= (long long)p->grid.n * p->grid.n ? 1 : 0;
  pd.lgf = p->lgf.as<double>();
  pd.nv = in->nv;
  pd.xv = in->d_xv;
  pd.yv = in->d_yv;
  pd.gv = in->d_gv;
  pd.w = w64 ? ws->w64.p : ws->w32.p;
  pd.w64 = w64 ? 1 : 0;
  pd.aux = ws->aux.as<double>();
  pd.partials = ws->part.as<double>();
  pd.bin_cnt = ws->bin_cnt.as<int>();
  pd.bin_start = ws->bin_start.as<int>();
  pd.items = ws->items.as<int>();
  pd.halo = ws->halo.p;
  pd.splits = ws->splits.as<int>();
  pd.splitwin = ws->splitwin.as<long long>();
  pd.rank = ws->rank.as<int>();
  pd.sorted = ws->sorted.as<double>();
  pd.status = out->d_status;
  pd.psi = out->d_psi;
  pd.u = (out->d_u && out->d_v) ? out->d_u : nullptr;
  pd.v = out->d_v;
  pd.sc_out = out->d_scalars;
  pd.imp_out = out->d_impulse;
  SolveScalars &sv = pd.sv;
  sv.u_inf = in->u_inf;
  sv.v_inf = in->v_inf;
  sv.ub = in->ub;
  sv.vb = in->vb;
  sv.omega = in->omega;
  sv.gamma_b = in->gamma_b;
  sv.gamma_w_in = in->gamma_w;
  sv.mode = in->mode;
  sv.m = (in->mode == GPF_KUTTA_SHED || in->mode == GPF_PARTS) ? in->m : 0;
  sv.znew_from = r.znew_from;
  for (int j = 0; j < sv.m; ++j) {
    sv.xnew[j] = in->h_xnew[j];
    sv.ynew[j] = in->h_ynew[j];
    sv.fmin[j] = in->fmin[j];
    sv.fmax[j] = in->fmax[j];
  }
  const void *spec2 = cfg.fp64_plan ? p->spec64.p : p->spec32.p;
  const void *tw2 = cfg.fp64_plan ? p->tw64.p : p->tw32.p;
  void *x2 = cfg.fp64_plan ? ws->x64.p : ws->x32.p;
  c1.in = pd.w;
  // Every reader of the field in a solve is a convolution's forward row
  // pass (the surface step only adds to it): those passes add R_v's tile
  // halos as they read, and the scatter skips its halo pass
  pd.halo_defer = pd.nv > 0 && halo_tiles(p->grid.n) > 0 ? 1 : 0;
  c1.halo = pd.halo_defer ? pd.halo : nullptr;
  c1.c = p->gauge_c;
  c1.gamma = pd.aux + SC_GAMMA_W;
  // the final convolution adds s_inf when the plan stores the total psi
  const bool total = (p->flags & GPF_PSI_TOTAL) != 0;
  pd.psi_total = total ? 1 : 0;
  auto set_inf = [&](ConvDesc &cd) {
    cd.add_inf = total ? 1 : 0;
    cd.inf_u = in->u_inf;
    cd.inf_v = in->v_inf;
    cd.ox = p->grid.x0;
    cd.oy = p->grid.y0;
    cd.h = p->grid.dx;
  };
  if (!cfg.body) {
    // one convolution
    set_inf(c1);
    c1.X = x2;
    c1.out = out->d_psi;
    c1.spec = spec2;
    c1.tw = tw2;
    c1.zero_in = 1;   // the only reader of the source: leave it zero
    pd.s1 = out->d_psi;
    c2 = c1;
    return;
  }
  const gpf_body *b = r.body;
  for (int e = 0; e < b->nedge; ++e) sv.edges[e] = b->edges[e];
  if (in->mode == GPF_PARTS) {
    // per part: mode, constraint values, motion; new vortices at the edges
    // of the shedding parts (body edge order); each steady-Kutta part's edge
    sv.m = in->m;
    sv.nparts = in->nparts;
    for (int j = 0; j < in->nparts; ++j) {
      const gpf_part &q = in->parts[j];
      sv.pmode[j] = q.mode;
      sv.pgb[j] = q.gamma_b;
      sv.pgw[j] = q.gamma_w;
      sv.pub[j] = q.ub;
      sv.pvb[j] = q.vb;
      sv.pom[j] = q.omega;
      sv.kedge[j] = -1;
    }
    int i = 0;
    for (int e = 0; e < b->nedge; ++e) {
      const int j = b->edge_part[e];
      if (in->parts[j].mode == GPF_KUTTA_SHED) {
        sv.edges[i] = b->edges[e];
        sv.epart[i] = j;
        ++i;
      } else if (in->parts[j].mode == GPF_KUTTA_STEADY && sv.kedge[j] < 0) {
        sv.kedge[j] = b->edges[e];
      }
    }
    pd.part = b->part.as<int>();
    pd.gpart = b->gpart.as<double>();
    pd.zpart = b->zpart.as<double>();
    pd.cpart = b->cpart.as<double>();
    pd.pgw_dev = r.pgw_dev;
  }
  pd.ns = b->ns;
  pd.xs = b->xs.as<double>();
  pd.ys = b->ys.as<double>();
  pd.ds = b->ds.as<double>();
  pd.sinv = b->sinv.as<double>();
  pd.f0 = b->f0.as<double>();
  pd.ghat = b->ghat.as<double>();
  pd.mom_x = b->mom_x;
  pd.mom_y = b->mom_y;
  pd.mom_r2 = b->mom_r2;
  pd.st_i = b->st_i.as<int>();
  pd.st_w = b->st_w.as<double>();
  pd.gamma0 = b->gamma0;
  pd.rhs = ws->rhs.as<double>();
  pd.fs = ws->fsurf.as<double>();
  pd.rs_node = b->rs_node.as<int>();
  pd.rs_off = b->rs_off.as<int>();
  pd.rs_code = b->rs_code.as<int>();
  pd.rs_nodes = b->rs_nodes;
  pd.f_out = out->d_f;
  pd.ft_out = out->d_ftilde;
  pd.nx = b->nx.as<double>();
  pd.ny = b->ny.as<double>();
  // first convolution: only its surface values are used
  c1.X = cfg.conv1_fp64 ? ws->x64.p : x2;
  c1.out = cfg.conv1_fp64 ? ws->s64.p : out->d_psi;
  c1.spec = cfg.conv1_fp64 ? p->spec64.p : spec2;
  c1.tw = cfg.conv1_fp64 ? p->tw64.p : tw2;
  c1.zero_in = 0;
  c1.row_lo = b->row_lo;   // only the surface stencils read this field
  c1.row_hi = b->row_hi;
  {
    const int band = body_band(b);
    if (ws->xb.bytes >= (size_t)(p->grid.n + 1) * band * (w64 ? 16 : 8)) {
      c1.Xb = ws->xb.p;
      c1.band_pitch = band;
    }
  }
  pd.s1 = c1.out;
  // final convolution of all vorticity
  c2.in = pd.w;
  c2.halo = c1.halo;
  c2.X = x2;
  c2.out = out->d_psi;
  c2.spec = spec2;
  c2.tw = tw2;
  c2.gamma = pd.aux + SC_GAMMA_SRC2;
  c2.c = p->gauge_c;
  c2.zero_in = 1;   // the last reader of the source: leave it zero
  set_inf(c2);
  // Between the two convolutions the source changes only where R_s f lands,
  // the rows of the surface stencils (no new vortices in the modes without
  // them).  When both convolutions share the intermediate (the first one's
  // column pass writes only its band rows to X, or none), the second one's
  // forward row pass redoes only the band rows: the others of X still hold
  // the first pass's transforms.  The first pass then clears the rows
  // outside the band, the second the band rows.
  if (c1.X == c2.X && pd.sv.m == 0 && !pd.w_accumulate) {
    const int lo = b->row_lo & ~15, hi = std::min(p->grid.n - 1, b->row_hi | 15);
    c1.zero_in = 1;
    c1.keep_lo = lo;
    c1.keep_end = hi + 1;
    c2.fwd_lo = lo;
    c2.fwd_hi = hi;
  }
}

template <class TW, class T1, class T2>
gpf_status launch_group(const GroupCfg &cfg, int nb, const ProbDesc *pd, const ConvDesc *c1,
                        const ConvDesc *c2, int nv_max, int ns_max, int m_max, bool impulse,
                        int band, int xcds, const ConvSched &sc1, const ConvSched &sc2,
                        bool shared, const double *shared_sinv, int vel_kinds, int fband2,
                        bool halo_pass, int rs_blocks, hipStream_t s) {
  GPF_HIP(launch_scatter_vortices<TW>(pd, nb, cfg.n, nv_max, s, nullptr, halo_pass));
  GPF_HIP((launch_convolve<TW, T1>(cfg.n, c1, nb, xcds, cfg.body ? band : 0, s, sc1)));
  if (cfg.body) {
    GPF_HIP(launch_surface_rhs<T1>(pd, nb, ns_max, m_max, s));
    if (cfg.parts) {
      GPF_HIP(launch_schur_apply_parts<TW>(pd, nb, ns_max, s));
    } else {
      if (shared) GPF_HIP(launch_schur_gemm(pd, nb, ns_max, m_max, shared_sinv, s));
      GPF_HIP(launch_schur_apply<TW>(pd, nb, ns_max, m_max, s));
    }
    timer_begin(GPF_TK_SURFACE, s);
    GPF_HIP(launch_rs_apply(pd, nb, rs_blocks, s));
    timer_end(s);
    GPF_HIP((launch_convolve<TW, T2>(cfg.n, c2, nb, xcds, 0, s, sc2, fband2)));
  }
  GPF_HIP(launch_solve_velocity<T2>(pd, nb, cfg.n, nv_max, s, nullptr, vel_kinds));
  if (impulse) GPF_HIP(launch_impulse(pd, nb, s));
  return GPF_OK;
}

// Run problems that share one configuration as one launch sequence.
gpf_status run_group(const GroupCfg &cfg, const std::vector<ProblemRef> &probs, DescRing &ring,
                     int xcds, hipStream_t s) {
  const int nb = (int)probs.size();
  std::vector<char> blk(nb * kProblemDescBytes);
  ProbDesc *pd = reinterpret_cast<ProbDesc *>(blk.data());
  ConvDesc *c1 = reinterpret_cast<ConvDesc *>(blk.data() + nb * sizeof(ProbDesc));
  ConvDesc *c2 = c1 + nb;
  int nv_max = 0, ns_max = 0, m_max = 0;
  int band = 0;   // rows of the first convolution's last pass (16-row groups)
  bool impulse = false;
  int vel_kinds = 0;   // velocity kernels the group needs: 1 vortex by vortex, 2 tile by tile
  int fband2 = 0;      // source rows the second forward row pass transforms (most of any problem)
  bool halo_pass = false;   // some problem's halos are added by the scatter's halo pass
  int rs_blocks = 0;        // workgroups of the R_s gather per problem (most of any)
  for (int i = 0; i < nb; ++i) {
    describe(probs[i], cfg, pd[i], c1[i], c2[i]);
    if (cfg.body) rs_blocks = std::max(rs_blocks, rs_apply_blocks(pd[i].rs_nodes, pd[i].sv.m));
    halo_pass = halo_pass || (pd[i].nv > 0 && !pd[i].halo_defer);
    fband2 = std::max(fband2, c2[i].fwd_hi - c2[i].fwd_lo + 1);
    if (pd[i].u && pd[i].nv > 0) vel_kinds |= pd[i].vel_tiles ? 2 : 1;
    nv_max = std::max(nv_max, pd[i].nv);
    ns_max = std::max(ns_max, pd[i].ns);
    m_max = std::max(m_max, pd[i].sv.m);
    band = std::max(band, (c1[i].row_hi | 15) - (c1[i].row_lo & ~15) + 1);
    impulse = impulse || pd[i].imp_out != nullptr;
  }
  // problems that share one body (one-part modes): S^-1 is applied to all
  // their right-hand sides as one product on the matrix cores
  bool shared = cfg.body && !cfg.parts && nb >= 2;
  for (int i = 1; i < nb && shared; ++i) shared = probs[i].body == probs[0].body;
  for (int i = 0; i < nb && shared; ++i) shared = probs[i].ws->y.p != nullptr;
  if (shared)
    for (int i = 0; i < nb; ++i) pd[i].y = probs[i].ws->y.as<double>();
  void *dev = nullptr;
  GPF_TRY(ring.push(blk.data(), blk.size(), s, &dev));
  const ProbDesc *dpd = static_cast<const ProbDesc *>(dev);
  const ConvDesc *dc1 =
      reinterpret_cast<const ConvDesc *>(static_cast<char *>(dev) + nb * sizeof(ProbDesc));
  const ConvDesc *dc2 = dc1 + nb;
  gpf_ctx *ctx = probs[0].plan->ctx;
  const bool d1 = cfg.fp64_plan || cfg.conv1_fp64;
  const ConvSched sc1 = ctx->sched_for(cfg.n, d1, nb);
  const ConvSched sc2 = ctx->sched_for(cfg.n, cfg.fp64_plan, nb);
  if (cfg.fp64_plan)
    return launch_group<double, double, double>(cfg, nb, dpd, dc1, dc2, nv_max, ns_max, m_max, impulse,
                                                   band, xcds, sc1, sc2, shared,
                                                   shared ? probs[0].body->sinv.as<double>() : nullptr, vel_kinds, fband2, halo_pass, rs_blocks, s);
  if (cfg.conv1_fp64)
    return launch_group<double, double, float>(cfg, nb, dpd, dc1, dc2, nv_max, ns_max, m_max, impulse,
                                                   band, xcds, sc1, sc2, shared,
                                                   shared ? probs[0].body->sinv.as<double>() : nullptr, vel_kinds, fband2, halo_pass, rs_blocks, s);
  return launch_group<float, float, float>(cfg, nb, dpd, dc1, dc2, nv_max, ns_max, m_max, impulse,
                                                   band, xcds, sc1, sc2, shared,
                                                   shared ? probs[0].body->sinv.as<double>() : nullptr, vel_kinds, fband2, halo_pass, rs_blocks, s);
}

// A batch can run merged when its problems differ only in grid size and in
// the precision of the first convolution: bodies of one part, FP32 fields,
// grids the multi-size transforms cover (n from 64 to 2048).
bool mergeable(const GroupCfg &c) {
  return c.body && !c.parts && !c.fp64_plan && c.n >= 64 && c.n <= 2048;
}

// Bytes of the descriptor block of a merged batch of nb problems: the
// problem and convolution descriptors, the work tables of the multi-size
// passes (three per convolution, two convolutions, two classes), then the
// flat block maps (per class: bin count, tile scatter, halo pass, bin
// place, split tiles, R_s gather; over all problems: two velocity kernels).
size_t merged_block_bytes(int nb) {
  return ((size_t)nb * kProblemDescBytes + 15) / 16 * 16 + 9 * (size_t)nb * sizeof(MultiEntry) +
         8 * (size_t)nb * sizeof(FlatEntry);   // six maps per class, two velocity maps
}

// Every stage of the solve as one launch per precision class over problems
// of all grid sizes (class A: FP32 first convolution, class B: FP64 first
// convolution).  The transforms of FP32 fields are the multi-size passes,
// whose work lists take the largest grids first; FP64 first convolutions
// run per grid size (in order of decreasing n).
// side: the batch, whose side stream and events take class B's first half
// when both classes are present (nullptr: one stream)
gpf_status run_merged(std::vector<ProblemRef> probs, DescRing &ring, int xcds, hipStream_t s,
                      gpf_batch *side) {
  const int nb = (int)probs.size();
  // class A before class B, each by decreasing n (stable: input order kept)
  std::stable_sort(probs.begin(), probs.end(), [](const ProblemRef &a, const ProblemRef &b) {
    const GroupCfg ca = config_of(a), cb = config_of(b);
    if (ca.conv1_fp64 != cb.conv1_fp64) return !ca.conv1_fp64;
    return ca.n > cb.n;
  });
  int na = 0;
  while (na < nb && !config_of(probs[na]).conv1_fp64) ++na;
  const int nbb = nb - na;
  std::vector<char> blk(merged_block_bytes(nb), 0);
  ProbDesc *pd = reinterpret_cast<ProbDesc *>(blk.data());
  ConvDesc *c1 = reinterpret_cast<ConvDesc *>(blk.data() + nb * sizeof(ProbDesc));
  ConvDesc *c2 = c1 + nb;
  const size_t tab_off = ((size_t)nb * kProblemDescBytes + 15) / 16 * 16;
  MultiEntry *tab = reinterpret_cast<MultiEntry *>(blk.data() + tab_off);
  struct ClassInfo {
    int nv_max = 0, ns_max = 0, m_max = 0, n_max = 0;
  } ca, cbi, ca1, ca2;
  // with the side streams, class A runs as two parts on two streams: A1 the
  // problems of its largest grid size, A2 the rest
  int na1 = 0;
  while (na1 < na && config_of(probs[na1]).n == config_of(probs[0]).n) ++na1;
  bool impulse = false;
  for (int i = 0; i < nb; ++i) {
    const GroupCfg cfg = config_of(probs[i]);
    describe(probs[i], cfg, pd[i], c1[i], c2[i]);
    for (ClassInfo *cp : {i < na ? &ca : &cbi, i < na1 ? &ca1 : (i < na ? &ca2 : &cbi)}) {
      ClassInfo &ci = *cp;
      ci.nv_max = std::max(ci.nv_max, pd[i].nv);
      ci.ns_max = std::max(ci.ns_max, pd[i].ns);
      ci.m_max = std::max(ci.m_max, pd[i].sv.m);
      ci.n_max = std::max(ci.n_max, cfg.n);
    }
    impulse = impulse || pd[i].imp_out != nullptr;
  }
  // work tables: pass kind per table (0 rows forward, 1 columns, 2 band rows
  // inverse, 3 all rows inverse) over problems [lo, hi) of `cd`
  int used = 0;
  auto make_table = [&](int kind, const ConvDesc *cd, int lo, int hi, MultiPass *mp) {
    MultiEntry *e = tab + used;
    int first = 0;
    for (int i = lo; i < hi; ++i) {
      const int n = pd[i].n;
      int lg = 0;
      while ((1 << lg) < n) ++lg;
      e[i - lo].first = first;
      e[i - lo].prob = i - lo;
      e[i - lo].logn = lg;
      // band flag: the inverse pass of a first convolution covers its output
      // band; a forward pass covers its source rows fwd_lo .. fwd_hi
      e[i - lo].band = kind == 2 || (kind == 0 && (cd[i].fwd_lo != 0 || cd[i].fwd_hi != n - 1)) ? 1 : 0;
      first += multi_blocks(kind, n, cd[i]);
    }
    mp->nprob = hi - lo;
    mp->total = first;
    // row passes: neighbouring row blocks share cache lines, so each XCD
    // takes a contiguous part of the list; column blocks share nothing
    mp->xcds = kind == 1 ? 1 : std::max(1, xcds);
    mp->e = reinterpret_cast<const MultiEntry *>(tab_off + used * sizeof(MultiEntry));  // offset for now
    used += hi - lo;
  };
  // flat grids of the binning, tile and velocity kernels: problem i of
  // [lo, hi) takes blocks(i) blocks (maps of the binning and tile kernels
  // per class, velocity maps over every problem)
  const size_t flat_off = tab_off + 9 * (size_t)nb * sizeof(MultiEntry);
  FlatEntry *ftab = reinterpret_cast<FlatEntry *>(blk.data() + flat_off);
  int fused = 0;
  auto make_flat = [&](int lo, int hi, auto blocks, FlatMap *fm) {
    FlatEntry *e = ftab + fused;
    int first = 0;
    for (int i = lo; i < hi; ++i) {
      const int k = blocks(i);
      e[i - lo] = FlatEntry{first, i - lo, k, 0};
      first += k;
    }
    fm->nprob = hi - lo;
    fm->total = first;
    fm->e = reinterpret_cast<const FlatEntry *>(flat_off + fused * sizeof(FlatEntry));  // offset for now
    fused += hi - lo;
  };
  auto bin_blocks = [&](int i) { return pd[i].nv > 0 ? bin_count_blocks(pd[i].nv) : 1; };
  auto place_map_blocks = [&](int i) { return place_blocks(pd[i].nv); };
  auto split_tile_blocks = [&](int i) { return pd[i].nv > 0 ? split_blocks(pd[i].nv) : 0; };
  auto rs_blocks = [&](int i) { return rs_apply_blocks(pd[i].rs_nodes, pd[i].sv.m); };
  auto tile_blocks = [&](int i) { return tile_items_max(pd[i].n, pd[i].nv); };
  auto vel_gather = [&](int i) { return pd[i].u && !pd[i].vel_tiles ? (pd[i].nv + 255) / 256 : 0; };
  auto vel_tiles = [&](int i) { return pd[i].u && pd[i].vel_tiles ? tile_blocks(i) : 0; };
  auto halo_blocks = [&](int i) { return pd[i].nv > 0 && !pd[i].halo_defer ? fixup_blocks(pd[i].n) : 0; };
  // per class: bin count, tile scatter, halo pass, bin place (fs*[4] stays
  // empty), split tiles, R_s gather; over all problems: two velocity kernels
  FlatMap fsb[5] = {}, fcomb[2] = {}, frs[2] = {}, fvel[2];
  struct Sub {
    int lo = 0, hi = 0;
    ClassInfo ci;
    FlatMap fs[5] = {}, fcomb = {}, frs = {}, fvel[2] = {};
    MultiPass mp1[3], mp2[3];
    hipStream_t st = nullptr;
  } subs[2];
  const bool split = side != nullptr && na1 > 0 && na1 < na;
  const int nsub = na > 0 ? (split ? 2 : 1) : 0;
  if (split) {
    subs[0].lo = 0, subs[0].hi = na1, subs[0].ci = ca1, subs[0].st = s;
    subs[1].lo = na1, subs[1].hi = na, subs[1].ci = ca2, subs[1].st = side->side2;
  } else {
    subs[0].lo = 0, subs[0].hi = na, subs[0].ci = ca, subs[0].st = s;
  }
  for (int k = 0; k < nsub; ++k) {
    Sub &u = subs[k];
    make_flat(u.lo, u.hi, bin_blocks, &u.fs[0]);
    make_flat(u.lo, u.hi, tile_blocks, &u.fs[1]);
    make_flat(u.lo, u.hi, halo_blocks, &u.fs[2]);
    make_flat(u.lo, u.hi, place_map_blocks, &u.fs[3]);
    make_flat(u.lo, u.hi, split_tile_blocks, &u.fcomb);
    make_flat(u.lo, u.hi, rs_blocks, &u.frs);
  }
  if (nbb > 0) {
    make_flat(na, nb, bin_blocks, &fsb[0]);
    make_flat(na, nb, tile_blocks, &fsb[1]);
    make_flat(na, nb, halo_blocks, &fsb[2]);
    make_flat(na, nb, place_map_blocks, &fsb[3]);
    make_flat(na, nb, split_tile_blocks, &fcomb[1]);
  }
  if (nbb > 0) make_flat(na, nb, rs_blocks, &frs[1]);
  // velocity maps: per part with the side streams, else over every problem
  const bool vsplit = side != nullptr && ((na > 0 && nbb > 0) || split);
  FlatMap fvelb[2] = {};
  if (vsplit) {
    for (int k = 0; k < nsub; ++k) {
      make_flat(subs[k].lo, subs[k].hi, vel_gather, &subs[k].fvel[0]);
      make_flat(subs[k].lo, subs[k].hi, vel_tiles, &subs[k].fvel[1]);
    }
    if (nbb > 0) {
      make_flat(na, nb, vel_gather, &fvelb[0]);
      make_flat(na, nb, vel_tiles, &fvelb[1]);
    }
  } else {
    make_flat(0, nb, vel_gather, &fvel[0]);
    make_flat(0, nb, vel_tiles, &fvel[1]);
  }
  MultiPass mp2b[3];
  for (int k = 0; k < nsub; ++k) {
    Sub &u = subs[k];
    make_table(0, c1, u.lo, u.hi, &u.mp1[0]);
    make_table(1, c1, u.lo, u.hi, &u.mp1[1]);
    make_table(2, c1, u.lo, u.hi, &u.mp1[2]);
    make_table(0, c2, u.lo, u.hi, &u.mp2[0]);
    make_table(1, c2, u.lo, u.hi, &u.mp2[1]);
    make_table(3, c2, u.lo, u.hi, &u.mp2[2]);
  }
  if (nbb > 0) {
    make_table(0, c2, na, nb, &mp2b[0]);
    make_table(1, c2, na, nb, &mp2b[1]);
    make_table(3, c2, na, nb, &mp2b[2]);
  }
  void *dev = nullptr;
  GPF_TRY(ring.push(blk.data(), blk.size(), s, &dev));
  char *base = static_cast<char *>(dev);
  auto fix = [&](MultiPass *mp) {   // table offsets -> device addresses
    for (int k = 0; k < 3; ++k) mp[k].e = reinterpret_cast<const MultiEntry *>(base + (size_t)mp[k].e);
  };
  for (int k = 0; k < nsub; ++k) {
    fix(subs[k].mp1);
    fix(subs[k].mp2);
  }
  if (nbb > 0) fix(mp2b);
  auto fixf = [&](FlatMap *fm, int k) {
    for (int i = 0; i < k; ++i) fm[i].e = reinterpret_cast<const FlatEntry *>(base + (size_t)fm[i].e);
  };
  for (int k = 0; k < nsub; ++k) {
    fixf(subs[k].fs, 4);
    fixf(&subs[k].fcomb, 1);
    fixf(&subs[k].frs, 1);
  }
  if (nbb > 0) {
    fixf(fsb, 4);
    fixf(&fcomb[1], 1);
    fixf(&frs[1], 1);
  }
  if (vsplit) {
    for (int k = 0; k < nsub; ++k) fixf(subs[k].fvel, 2);
    if (nbb > 0) fixf(fvelb, 2);
  } else {
    fixf(fvel, 2);
  }
  const ProbDesc *dpd = reinterpret_cast<const ProbDesc *>(base);
  const ConvDesc *dc1 = reinterpret_cast<const ConvDesc *>(base + nb * sizeof(ProbDesc));
  const ConvDesc *dc2 = dc1 + nb;
  gpf_ctx *ctx = probs[0].plan->ctx;
  // each class up to its velocities: R_v (scatter, split tiles), the first
  // convolution (surface band only), surface right-hand sides, Schur
  // complement and constraints, R_s f, the final convolution.  Class B's
  // kernels are few and small (FP64 transforms of a handful of problems):
  // with both classes present they run on the side stream, issued first,
  // beside class A's.  Class A's two parts run on the caller's stream (A1)
  // and the second side stream (A2), so that one part's latency-bound
  // stages overlap the other's transforms.  With the side streams each part
  // also takes its velocities on its own stream, after its final
  // convolution; the main stream waits for the side streams before the
  // impulses.
  const bool fork = side != nullptr && na > 0 && nbb > 0;
  const hipStream_t sb = fork ? side->side : s;
  auto class_a = [&](Sub &u) -> gpf_status {
    const int lo = u.lo, m = u.hi - u.lo;
    const hipStream_t st = u.st;
    GPF_HIP(launch_scatter_vortices<float>(dpd + lo, m, u.ci.n_max, u.ci.nv_max, st, u.fs));
    timer_begin(GPF_TK_SCATTER, st);
    GPF_HIP(launch_split_combine(dpd + lo, m, 0, st, &u.fcomb));
    timer_end(st);
    GPF_HIP((launch_convolve_multi<float, float>(dc1 + lo, u.mp1, st)));
    GPF_HIP(launch_surface_rhs<float>(dpd + lo, m, u.ci.ns_max, u.ci.m_max, st));
    GPF_HIP(launch_schur_apply<float>(dpd + lo, m, u.ci.ns_max, u.ci.m_max, st));
    timer_begin(GPF_TK_SURFACE, st);
    GPF_HIP(launch_rs_apply(dpd + lo, m, 0, st, &u.frs));
    timer_end(st);
    GPF_HIP((launch_convolve_multi<float, float>(dc2 + lo, u.mp2, st)));
    if (vsplit) GPF_HIP(launch_solve_velocity<float>(dpd + lo, m, u.ci.n_max, u.ci.nv_max, st, u.fvel));
    return GPF_OK;
  };
  auto class_b = [&]() -> gpf_status {
    GPF_HIP(launch_scatter_vortices<double>(dpd + na, nbb, cbi.n_max, cbi.nv_max, sb, fsb));
    timer_begin(GPF_TK_SCATTER, sb);
    GPF_HIP(launch_split_combine(dpd + na, nbb, 0, sb, &fcomb[1]));
    timer_end(sb);
    for (int i = na; i < nb;) {
      int j = i;
      int band = 0;
      while (j < nb && pd[j].n == pd[i].n) {
        band = std::max(band, (c1[j].row_hi | 15) - (c1[j].row_lo & ~15) + 1);
        ++j;
      }
      const ConvSched sc = ctx->sched_for(pd[i].n, true, j - i);
      GPF_HIP((launch_convolve<double, double>(pd[i].n, dc1 + i, j - i, xcds, band, sb, sc)));
      i = j;
    }
    GPF_HIP(launch_surface_rhs<double>(dpd + na, nbb, cbi.ns_max, cbi.m_max, sb));
    GPF_HIP(launch_schur_apply<double>(dpd + na, nbb, cbi.ns_max, cbi.m_max, sb));
    timer_begin(GPF_TK_SURFACE, sb);
    GPF_HIP(launch_rs_apply(dpd + na, nbb, 0, sb, &frs[1]));
    timer_end(sb);
    GPF_HIP((launch_convolve_multi<double, float>(dc2 + na, mp2b, sb)));
    if (vsplit) GPF_HIP(launch_solve_velocity<float>(dpd + na, nbb, cbi.n_max, cbi.nv_max, sb, fvelb));
    return GPF_OK;
  };
  if (fork || split) {
    // after the descriptor copy on s, and after every earlier use of these
    // problems' buffers on s
    GPF_HIP(hipEventRecord(side->side_fork, s));
    if (fork) GPF_HIP(hipStreamWaitEvent(sb, side->side_fork, 0));
    if (split) GPF_HIP(hipStreamWaitEvent(side->side2, side->side_fork, 0));
    if (fork) {
      GPF_TRY(class_b());
      GPF_HIP(hipEventRecord(side->side_join, sb));
    }
    if (split) {
      GPF_TRY(class_a(subs[1]));
      GPF_HIP(hipEventRecord(side->side2_join, side->side2));
    }
    GPF_TRY(class_a(subs[0]));
    if (fork) GPF_HIP(hipStreamWaitEvent(s, side->side_join, 0));
    if (split) GPF_HIP(hipStreamWaitEvent(s, side->side2_join, 0));
  } else {
    for (int k = 0; k < nsub; ++k) GPF_TRY(class_a(subs[k]));
    if (nbb > 0) GPF_TRY(class_b());
  }
  // velocities of every problem (per part above with the side streams),
  // then impulses where asked
  if (!vsplit)
    GPF_HIP(launch_solve_velocity<float>(dpd, nb, std::max(ca.n_max, cbi.n_max),
                                         std::max(ca.nv_max, cbi.nv_max), s, fvel));
  if (impulse) GPF_HIP(launch_impulse(dpd, nb, s));
  return GPF_OK;
}

gpf_status validate(const gpf_plan *plan, const gpf_body *body, const gpf_inputs *in,
                    const gpf_outputs *out) {
  if (!plan || !in || !out) return fail(GPF_E_INVALID, "solve: null argument");
  if (!out->d_psi || !out->d_status) return fail(GPF_E_INVALID, "solve: d_psi and d_status are required");
  if (out->d_impulse && in->mode != GPF_NOBODY && !out->d_f)
    return fail(GPF_E_INVALID, "solve: the impulse with a body needs d_f");
  if (in->nv < 0 || in->nv > kMaxVortices) return fail(GPF_E_UNSUPPORTED, "solve: nv must be in [0, 2^22]");
  if (in->nv > 0 && (!in->d_xv || !in->d_yv || !in->d_gv))
    return fail(GPF_E_INVALID, "solve: null vortex arrays");
  if (!is_finite(in->u_inf) || !is_finite(in->v_inf) || !is_finite(in->ub) || !is_finite(in->vb) ||
      !is_finite(in->omega))
    return fail(GPF_E_INVALID, "solve: non-finite freestream or body motion");
  if (in->mode < GPF_NOBODY || in->mode > GPF_PARTS) return fail(GPF_E_INVALID, "solve: unknown mode");
  if (in->mode != GPF_NOBODY) {
    if (!body) return fail(GPF_E_INVALID, "solve: this mode needs a body");
    if (body->plan != plan) return fail(GPF_E_INVALID, "solve: body belongs to another plan");
  }
  if (in->mode == GPF_CIRCULATION && !is_finite(in->gamma_b))
    return fail(GPF_E_INVALID, "solve: non-finite gamma_b");
  if (in->mode == GPF_KUTTA_STEADY && body->nedge < 1)
    return fail(GPF_E_INVALID, "solve: steady Kutta needs a body with an edge");
  if (in->mode == GPF_KUTTA_SHED) {
    if (in->m < 1 || in->m != body->nedge)
      return fail(GPF_E_INVALID, "solve: shedding needs one new vortex per body edge");
    for (int j = 0; j < in->m; ++j) {
      if (!is_finite(in->h_xnew[j]) || !is_finite(in->h_ynew[j]))
        return fail(GPF_E_INVALID, "solve: non-finite new vortex position");
      // NaN fails the comparison; infinite bounds leave the edge free
      if (!(in->fmin[j] <= in->fmax[j]))
        return fail(GPF_E_INVALID, "solve: edge bounds need fmin <= fmax");
    }
    if (!std::isnan(in->gamma_w) && !is_finite(in->gamma_w))
      return fail(GPF_E_INVALID, "solve: gamma_w must be finite or NaN");
  }
  if (in->mode == GPF_PARTS) {
    if (body->nparts < 2 || in->nparts != body->nparts)
      return fail(GPF_E_INVALID, "solve: GPF_PARTS needs a body split by gpf_body_set_parts, "
                                 "with nparts equal to its part count");
    int nshed = 0;
    for (int j = 0; j < in->nparts; ++j) {
      const gpf_part &q = in->parts[j];
      if (q.mode != GPF_CIRCULATION && q.mode != GPF_KUTTA_STEADY && q.mode != GPF_KUTTA_SHED)
        return fail(GPF_E_INVALID, "solve: a part's mode must be circulation, steady Kutta or shedding");
      if (!is_finite(q.gamma_b) || !is_finite(q.gamma_w) || !is_finite(q.ub) || !is_finite(q.vb) ||
          !is_finite(q.omega))
        return fail(GPF_E_INVALID, "solve: non-finite part value");
      int edges = 0;
      for (int e = 0; e < body->nedge; ++e) edges += body->edge_part[e] == j;
      if (q.mode == GPF_KUTTA_STEADY && edges < 1)
        return fail(GPF_E_INVALID, "solve: a steady-Kutta part needs an edge");
      if (q.mode == GPF_KUTTA_SHED) nshed += edges;
    }
    if (in->m != nshed)
      return fail(GPF_E_INVALID, "solve: m must equal the edge count of the shedding parts");
    for (int i = 0; i < in->m; ++i) {
      if (!is_finite(in->h_xnew[i]) || !is_finite(in->h_ynew[i]))
        return fail(GPF_E_INVALID, "solve: non-finite new vortex position");
      if (!(in->fmin[i] <= in->fmax[i]))
        return fail(GPF_E_INVALID, "solve: edge bounds need fmin <= fmax");
    }
  }
  return GPF_OK;
}

ProbDesc single_problem(const gpf_plan *plan) {
  ProbDesc pd;
  std::memset(&pd, 0, sizeof(pd));
  pd.n = plan->grid.n;
  pd.dx = plan->grid.dx;
  pd.x0 = plan->grid.x0;
  pd.y0 = plan->grid.y0;
  pd.status = plan->status_scratch.as<unsigned>();
  return pd;
}

}  // namespace
}  // namespace gpf

extern "C" {

const char *gpf_last_error(void) { return g_last_error.c_str(); }
const char *gpf_version(void) { return "gpf 0.2 (gfx950)"; }

gpf_status gpf_invert_fp64(gpf_ctx *ctx, int n, const double *d_a, double *d_ainv,
                           void *hip_stream, double *min_pivot_rel) {
  if (!ctx || n < 1 || n > 8192 || !d_a || !d_ainv || d_a == d_ainv)
    return fail(GPF_E_INVALID, "gpf_invert_fp64: bad arguments");
  GPF_HIP(hipSetDevice(ctx->device));
  double mp = 0.0;
  GPF_TRY(invert_fp64(n, const_cast<double *>(d_a), d_ainv, as_stream(hip_stream), &mp));
  if (min_pivot_rel) *min_pivot_rel = mp;
  return GPF_OK;
}

gpf_status gpf_lgf_table(int nmax, double *h_table) {
  if (nmax < 0 || nmax > 8192 || !h_table) return fail(GPF_E_INVALID, "gpf_lgf_table: bad arguments");
  lgf_table_host(nmax, h_table);
  return GPF_OK;
}

gpf_status gpf_ctx_create(int device, gpf_ctx **out) {
  if (!out) return fail(GPF_E_INVALID, "gpf_ctx_create: null out");
  *out = nullptr;
  int count = 0;
  GPF_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(GPF_E_INVALID, "gpf_ctx_create: bad device");
  GPF_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  GPF_HIP(hipGetDeviceProperties(&prop, device));
  // the allocation-free entry point's scratch address on this device
  GPF_TRY(noalloc_init(device));
  auto *c = new gpf_ctx;
  c->device = device;
  c->num_cu = prop.multiProcessorCount;
  c->xcds = xcd_count(device);
  std::snprintf(c->arch, sizeof(c->arch), "%s", prop.gcnArchName);
  for (char *q = c->arch; *q; ++q)   // the target name without its feature suffixes
    if (*q == ':' || *q == ' ') { *q = 0; break; }
  *out = c;
  return GPF_OK;
}

void gpf_ctx_destroy(gpf_ctx *ctx) { delete ctx; }

gpf_status gpf_plan_create(gpf_ctx *ctx, const gpf_grid *grid, unsigned flags, gpf_plan **out) {
  if (!ctx || !grid || !out) return fail(GPF_E_INVALID, "gpf_plan_create: null argument");
  *out = nullptr;
  const int n = grid->n;
  if (!is_pow2(n) || n < 16 || n > 2048)
    return fail(GPF_E_UNSUPPORTED, "gpf_plan_create: n must be a power of two in [16, 2048]");
  if (!(grid->dx > 0.0) || !is_finite(grid->dx) || !is_finite(grid->x0) || !is_finite(grid->y0))
    return fail(GPF_E_INVALID, "gpf_plan_create: dx must be positive and x0, y0 finite");
  if (flags & ~(GPF_FP64 | GPF_CONV1_FP64 | GPF_POLICY_AUTO | GPF_PSI_TOTAL | GPF_PLAN_MULTISTREAM))
    return fail(GPF_E_INVALID, "gpf_plan_create: unknown flag");
  GPF_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<gpf_plan> p(new gpf_plan);
  p->ctx = ctx;
  p->grid = *grid;
  p->flags = flags;
  p->fp64 = (flags & GPF_FP64) != 0;
  auto tab = get_table(n);
  GPF_TRY(p->lgf.alloc(tab->size() * sizeof(double)));
  GPF_HIP(hipMemcpy(p->lgf.p, tab->data(), tab->size() * sizeof(double), hipMemcpyHostToDevice));
  if (p->fp64 || (flags & GPF_CONV1_FP64)) GPF_TRY(p->ensure_fp64());
  if (!p->fp64) {
    GPF_TRY(upload_spectrum<float>(p.get(), p->spec32, p->tw32));
    GPF_TRY(p->ws.ensure(n, true, false, 0));
  }
  GPF_TRY(p->status_scratch.alloc(256));
  GPF_TRY(fill_now(p->status_scratch.p, 0, 256));
  GPF_TRY(p->ring.init(kPlanRingSlots, kProblemDescBytes));
  GPF_HIP(hipDeviceSynchronize());
  *out = p.release();
  return GPF_OK;
}

void gpf_plan_destroy(gpf_plan *plan) { delete plan; }

gpf_status gpf_body_create(gpf_plan *plan, int ns, const double *h_xs, const double *h_ys,
                           const double *h_ds, int nedge, const int *h_edges, gpf_body **out) {
  if (!plan || !h_xs || !h_ys || !h_ds || !out || (nedge > 0 && !h_edges))
    return fail(GPF_E_INVALID, "gpf_body_create: null argument");
  *out = nullptr;
  if (ns < 2 || ns > 8192) return fail(GPF_E_UNSUPPORTED, "gpf_body_create: ns must be in [2, 8192]");
  if (nedge < 0 || nedge > GPF_MAX_EDGES) return fail(GPF_E_INVALID, "gpf_body_create: bad edge count");
  const gpf_grid &g = plan->grid;
  for (int p = 0; p < ns; ++p) {
    if (!is_finite(h_xs[p]) || !is_finite(h_ys[p]) || !(h_ds[p] > 0.0) || !is_finite(h_ds[p]))
      return fail(GPF_E_INVALID, "gpf_body_create: non-finite point or non-positive ds");
    const double xi = (h_xs[p] - g.x0) / g.dx, eta = (h_ys[p] - g.y0) / g.dx;
    if (!(xi >= 1.0 && xi < g.n - 2.0 && eta >= 1.0 && eta < g.n - 2.0))
      return fail(GPF_E_OUT_OF_GRID, "gpf_body_create: surface stencil leaves the grid window");
  }
  for (int e = 0; e < nedge; ++e)
    if (h_edges[e] < 0 || h_edges[e] >= ns) return fail(GPF_E_INVALID, "gpf_body_create: bad edge index");
  GPF_HIP(hipSetDevice(plan->ctx->device));
  std::unique_ptr<gpf_body> b(new gpf_body);
  b->plan = plan;
  b->ns = ns;
  b->nedge = nedge;
  b->row_lo = g.n;
  b->row_hi = -1;
  for (int p = 0; p < ns; ++p) {
    const int j0 = (int)std::floor((h_ys[p] - g.y0) / g.dx) - 1;  // lowest stencil row
    b->row_lo = std::min(b->row_lo, j0);
    b->row_hi = std::max(b->row_hi, j0 + 3);
  }
  for (int e = 0; e < nedge; ++e) b->edges[e] = h_edges[e];
  const size_t vb = ns * sizeof(double);
  GPF_TRY(b->xs.alloc(vb));
  GPF_TRY(b->ys.alloc(vb));
  GPF_TRY(b->ds.alloc(vb));
  GPF_TRY(b->st_i.alloc(2 * ns * sizeof(int)));
  GPF_TRY(b->st_w.alloc(8 * vb));
  GPF_TRY(b->sinv.alloc((size_t)ns * vb));
  GPF_TRY(b->f0.alloc(vb));
  GPF_TRY(b->ghat.alloc(vb));
  GPF_TRY(b->nx.alloc(vb));
  GPF_TRY(b->ny.alloc(vb));
  GPF_TRY(fill_now(b->nx.p, 0, vb));
  GPF_TRY(fill_now(b->ny.p, 0, vb));
  b->hxs.assign(h_xs, h_xs + ns);
  b->hys.assign(h_ys, h_ys + ns);
  b->hds.assign(h_ds, h_ds + ns);
  {
    // no normals yet: zero area, arc-length centroid
    double L = 0.0, sx = 0.0, sy = 0.0;
    for (int p = 0; p < ns; ++p) {
      L += h_ds[p];
      sx += h_ds[p] * h_xs[p];
      sy += h_ds[p] * h_ys[p];
    }
    b->xc = sx / L;
    b->yc = sy / L;
  }
  GPF_TRY(plan->ws.ensure(g.n, !plan->fp64, plan->fp64, ns, body_band(b.get())));
  GPF_HIP(hipMemcpy(b->xs.p, h_xs, vb, hipMemcpyHostToDevice));
  GPF_HIP(hipMemcpy(b->ys.p, h_ys, vb, hipMemcpyHostToDevice));
  GPF_HIP(hipMemcpy(b->ds.p, h_ds, vb, hipMemcpyHostToDevice));
  hipStream_t s = nullptr;
  unsigned *status = plan->status_scratch.as<unsigned>();
  GPF_HIP(launch_surface_stencils(g.n, g.dx, g.x0, g.y0, ns, b->xs.as<double>(), b->ys.as<double>(),
                                  b->st_i.as<int>(), b->st_w.as<double>(), status, s));
  DevBuf S;
  GPF_TRY(S.alloc((size_t)ns * vb));
  GPF_HIP(launch_schur_build(g.n, ns, b->st_i.as<int>(), b->st_w.as<double>(), b->ds.as<double>(),
                             plan->lgf.as<double>(), S.as<double>(), s));
  double min_piv = 0.0;
  GPF_TRY(invert_fp64(ns, S.as<double>(), b->sinv.as<double>(), s, &min_piv));
  if (!(min_piv > 1e-14)) return fail(GPF_E_SINGULAR, "gpf_body_create: Schur complement is singular");
  // f0 = S^-1 1; amplification probe: r = -y_s and the alternating vector
  std::vector<double> X(3 * (size_t)ns);
  double rmax = 0.0;
  for (int p = 0; p < ns; ++p) {
    X[p] = 1.0;
    X[ns + p] = -h_ys[p];
    rmax = std::max(rmax, std::fabs(h_ys[p]));
  }
  if (rmax == 0.0) rmax = 1.0;
  for (int p = 0; p < ns; ++p) X[2 * ns + p] = (p & 1) ? -rmax : rmax;
  DevBuf dX, dY;
  GPF_TRY(dX.alloc(3 * vb));
  GPF_TRY(dY.alloc(3 * vb));
  GPF_HIP(hipMemcpy(dX.p, X.data(), 3 * vb, hipMemcpyHostToDevice));
  GPF_HIP(launch_gemv(ns, 3, b->sinv.as<double>(), dX.as<double>(), dY.as<double>(), s));
  std::vector<double> Y(3 * (size_t)ns);
  GPF_HIP(hipMemcpy(Y.data(), dY.p, 3 * vb, hipMemcpyDeviceToHost));
  unsigned hstatus = 0;
  GPF_HIP(hipMemcpy(&hstatus, status, sizeof(unsigned), hipMemcpyDeviceToHost));
  GPF_TRY(fill_now(status, 0, sizeof(unsigned)));
  if (hstatus & GPF_DEV_OUT_OF_GRID) return fail(GPF_E_OUT_OF_GRID, "gpf_body_create: stencil outside grid");
  {
    // R_s as a gather (Sec. 2.2, eq. basicblock: R_s spreads each point's
    // value over its 4 x 4 stencil): the nodes the stencils reach, each with
    // its (point, a, b) entries in point order, so that a solve adds R_s f
    // node by node in a fixed order
    std::vector<int> sti(2 * (size_t)ns);
    GPF_HIP(hipMemcpy(sti.data(), b->st_i.p, sti.size() * sizeof(int), hipMemcpyDeviceToHost));
    std::vector<std::pair<int, int>> e;
    e.reserve(16 * (size_t)ns);
    for (int p = 0; p < ns; ++p)
      for (int bb = 0; bb < 4; ++bb)
        for (int a = 0; a < 4; ++a)
          e.emplace_back((sti[2 * p + 1] + bb) * g.n + sti[2 * p] + a, 16 * p + 4 * bb + a);
    std::sort(e.begin(), e.end());
    std::vector<int> node, off, code(e.size());
    for (size_t k = 0; k < e.size(); ++k) {
      if (k == 0 || e[k].first != e[k - 1].first) {
        node.push_back(e[k].first);
        off.push_back((int)k);
      }
      code[k] = e[k].second;
    }
    off.push_back((int)e.size());
    b->rs_nodes = (int)node.size();
    GPF_TRY(b->rs_node.alloc(node.size() * sizeof(int)));
    GPF_TRY(b->rs_off.alloc(off.size() * sizeof(int)));
    GPF_TRY(b->rs_code.alloc(code.size() * sizeof(int)));
    GPF_HIP(hipMemcpy(b->rs_node.p, node.data(), node.size() * sizeof(int), hipMemcpyHostToDevice));
    GPF_HIP(hipMemcpy(b->rs_off.p, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
    GPF_HIP(hipMemcpy(b->rs_code.p, code.data(), code.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  double g0 = 0.0, nr = 0.0, nf = 0.0, nrhs = 0.0, npert = 0.0;
  double mx = 0.0, my = 0.0, mr2 = 0.0;
  for (int p = 0; p < ns; ++p) {
    const double fh = h_ds[p] * Y[p];
    g0 += fh;
    mx += fh * h_xs[p];
    my += fh * h_ys[p];
    mr2 += fh * (h_xs[p] * h_xs[p] + h_ys[p] * h_ys[p]);
    nr += Y[ns + p] * Y[ns + p];
    nf += Y[2 * ns + p] * Y[2 * ns + p];
    nrhs += X[ns + p] * X[ns + p];
    npert += X[2 * ns + p] * X[2 * ns + p];
  }
  for (int p = 0; p < ns; ++p)
    if (!(std::fabs(Y[p]) > 0.0) || !is_finite(Y[p]))
      return fail(GPF_E_SINGULAR, "gpf_body_create: f0 has a zero or non-finite entry");
  if (!(std::fabs(g0) > 0.0) || !is_finite(g0)) return fail(GPF_E_SINGULAR, "gpf_body_create: Gamma0 is zero");
  b->gamma0 = g0;
  b->mom_x = mx;
  b->mom_y = my;
  b->mom_r2 = mr2;
  b->amp = (nr > 0.0 && npert > 0.0) ? std::sqrt(nf / nr) / std::sqrt(npert / nrhs) : INFINITY;
  b->conv1_fp64 = !plan->fp64 && ((plan->flags & GPF_CONV1_FP64) ||
                                  ((plan->flags & GPF_POLICY_AUTO) && b->amp > GPF_AMP_THRESHOLD));
  if (b->conv1_fp64) GPF_TRY(plan->ensure_fp64());
  GPF_HIP(hipMemcpy(b->f0.p, Y.data(), vb, hipMemcpyHostToDevice));
  b->hf0.assign(Y.begin(), Y.begin() + ns);
  GPF_HIP(launch_gemv_t(ns, b->sinv.as<double>(), b->ds.as<double>(), b->ghat.as<double>(), s));
  GPF_HIP(hipDeviceSynchronize());
  *out = b.release();
  return GPF_OK;
}

void gpf_body_destroy(gpf_body *body) { delete body; }

gpf_status gpf_body_info(const gpf_body *body, double *gamma0, double *amp, int *conv1_fp64) {
  if (!body) return fail(GPF_E_INVALID, "gpf_body_info: null body");
  if (gamma0) *gamma0 = body->gamma0;
  if (amp) *amp = body->amp;
  if (conv1_fp64) *conv1_fp64 = body->conv1_fp64 ? 1 : 0;
  return GPF_OK;
}

gpf_status gpf_body_f0(const gpf_body *body, double *h_f0) {
  if (!body || !h_f0) return fail(GPF_E_INVALID, "gpf_body_f0: null argument");
  GPF_HIP(hipMemcpy(h_f0, body->f0.p, body->ns * sizeof(double), hipMemcpyDeviceToHost));
  return GPF_OK;
}

namespace {

// Pressure operators of a body with normals (Sec. 2.6.1):
// Q = -(C_s L^-1 C_s^T)^+ C_s L^-1 R_s; for a closed surface the operator's
// uniform direction is removed by bordering it with 1 and dS (dS-weighted
// mean of dphi zero), an open one is inverted as it is.
gpf_status pressure_setup(gpf_body *b) {
  b->has_pressure = false;
  const gpf_plan *pl = b->plan;
  const gpf_grid &g = pl->grid;
  const int ns = b->ns;
  for (int p = 0; p < ns; ++p) {   // face stencils need one more node of margin
    const double xi = (b->hxs[p] - g.x0) / g.dx, eta = (b->hys[p] - g.y0) / g.dx;
    if (!(xi >= 2.0 && xi < g.n - 3.0 && eta >= 2.0 && eta < g.n - 3.0)) return GPF_OK;
  }
  if (ns > 4096) return GPF_OK;
  hipStream_t s = nullptr;
  const size_t vb = ns * sizeof(double);
  GPF_TRY(b->pst.alloc(ns * sizeof(PresStencil)));
  GPF_TRY(b->qpres.alloc((size_t)ns * vb));
  const int nb = b->nparts;
  const int N = b->closed ? ns + nb : ns;
  DevBuf M, K, A, Ainv;
  GPF_TRY(M.alloc((size_t)ns * vb));
  GPF_TRY(K.alloc((size_t)ns * vb));
  GPF_TRY(A.alloc((size_t)N * N * sizeof(double)));
  GPF_TRY(Ainv.alloc((size_t)N * N * sizeof(double)));
  GPF_HIP(launch_pres_stencils(ns, b->xs.as<double>(), b->ys.as<double>(), g.x0, g.y0, g.dx,
                               b->pst.as<PresStencil>(), s));
  GPF_HIP(launch_pres_build(g.n, ns, b->pst.as<PresStencil>(), b->pnx.as<double>(),
                            b->pny.as<double>(), b->st_i.as<int>(), b->st_w.as<double>(),
                            b->ds.as<double>(), g.dx, pl->lgf.as<double>(), M.as<double>(),
                            K.as<double>(), s));
  if (b->closed) {
    // [M 1_j; (dS o 1_j)^T 0], one border per part, assembled on the host
    std::vector<double> hm((size_t)ns * ns), ha((size_t)N * N, 0.0);
    GPF_HIP(hipMemcpy(hm.data(), M.p, (size_t)ns * vb, hipMemcpyDeviceToHost));
    for (int p = 0; p < ns; ++p) {
      const int j = nb > 1 ? b->hpart[p] : 0;
      for (int q = 0; q < ns; ++q) ha[(size_t)p * N + q] = hm[(size_t)p * ns + q];
      ha[(size_t)p * N + ns + j] = 1.0;
      ha[(size_t)(ns + j) * N + p] = b->hds[p];
    }
    GPF_HIP(hipMemcpy(A.p, ha.data(), ha.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    GPF_HIP(hipMemcpy(A.p, M.p, (size_t)ns * vb, hipMemcpyDeviceToDevice));
  }
  double min_piv = 0.0;
  GPF_TRY(invert_fp64(N, A.as<double>(), Ainv.as<double>(), s, &min_piv));
  if (!(min_piv > 1e-14)) return GPF_OK;
  GPF_HIP(launch_pres_q(ns, N, Ainv.as<double>(), K.as<double>(), b->qpres.as<double>(), s));
  GPF_HIP(hipDeviceSynchronize());
  b->has_pressure = true;
  return GPF_OK;
}

}  // namespace

gpf_status gpf_body_set_normals(gpf_body *body, const double *h_nx, const double *h_ny, int closed) {
  if (!body || !h_nx || !h_ny) return fail(GPF_E_INVALID, "gpf_body_set_normals: null argument");
  const int ns = body->ns;
  for (int p = 0; p < ns; ++p)
    if (!is_finite(h_nx[p]) || !is_finite(h_ny[p]))
      return fail(GPF_E_INVALID, "gpf_body_set_normals: non-finite normal");
  GPF_HIP(hipSetDevice(body->plan->ctx->device));
  const size_t vb = ns * sizeof(double);
  GPF_TRY(body->pnx.alloc(vb));
  GPF_TRY(body->pny.alloc(vb));
  GPF_HIP(hipMemcpy(body->pnx.p, h_nx, vb, hipMemcpyHostToDevice));
  GPF_HIP(hipMemcpy(body->pny.p, h_ny, vb, hipMemcpyHostToDevice));
  body->closed = closed != 0;
  body->has_normals = true;
  if (body->closed) {
    // the impulse's motion term, area and centroid (eq. centroid); the area
    // as the mean of its two forms
    GPF_HIP(hipMemcpy(body->nx.p, h_nx, vb, hipMemcpyHostToDevice));
    GPF_HIP(hipMemcpy(body->ny.p, h_ny, vb, hipMemcpyHostToDevice));
    double vx = 0.0, vy = 0.0, cx = 0.0, cy = 0.0;
    for (int p = 0; p < ns; ++p) {
      const double x = body->hxs[p], y = body->hys[p], w = body->hds[p];
      const double r2 = x * x + y * y;
      vx += w * x * h_nx[p];
      vy += w * y * h_ny[p];
      cx += w * r2 * h_nx[p];
      cy += w * r2 * h_ny[p];
    }
    const double V = 0.5 * (vx + vy);
    body->area = V;
    if (V != 0.0) {
      body->xc = cx / (2.0 * V);
      body->yc = cy / (2.0 * V);
    }
  } else {
    // zero thickness: its two faces cancel in the motion term
    GPF_TRY(fill_now(body->nx.p, 0, vb));
    GPF_TRY(fill_now(body->ny.p, 0, vb));
    body->area = 0.0;
    double L = 0.0, sx = 0.0, sy = 0.0;
    for (int p = 0; p < ns; ++p) {
      L += body->hds[p];
      sx += body->hds[p] * body->hxs[p];
      sy += body->hds[p] * body->hys[p];
    }
    body->xc = sx / L;
    body->yc = sy / L;
  }
  return pressure_setup(body);
}

gpf_status gpf_pressure(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in, const void *d_psi,
                        const double *d_f, const double *d_dphi_prev, double dt, double rho,
                        double *d_dphi, double *d_dp, double *d_p, double *d_pside,
                        void *hip_stream) {
  if (!plan || !body || !in || !d_psi || !d_f || !d_dphi || !d_dp || !is_finite(rho) ||
      (d_dphi_prev && !(dt > 0.0 && is_finite(dt))) || (d_pside && !d_p))
    return fail(GPF_E_INVALID, "gpf_pressure: bad arguments");
  if (body->plan != plan) return fail(GPF_E_INVALID, "gpf_pressure: body belongs to another plan");
  if (!body->has_normals) return fail(GPF_E_INVALID, "gpf_pressure: the body has no normals");
  if (!body->has_pressure)
    return fail(GPF_E_UNSUPPORTED, "gpf_pressure: no pressure operators for this body (surface "
                                   "within two nodes of the window edge, ns > 4096, or singular)");
  GPF_HIP(hipSetDevice(plan->ctx->device));
  hipStream_t s = as_stream(hip_stream);
  const gpf_grid &g = plan->grid;
  const int n = g.n, ns = body->ns;
  GPF_TRY(plan->pres_ddt.alloc(ns * sizeof(double)));
  PresDesc D;
  std::memset(&D, 0, sizeof(D));
  D.n = n;
  D.ns = ns;
  D.psi_total = (plan->flags & GPF_PSI_TOTAL) ? 1 : 0;
  D.dx = g.dx;
  D.x0 = g.x0;
  D.y0 = g.y0;
  D.rho = rho;
  D.dt = d_dphi_prev ? dt : 1.0;
  D.u_inf = in->u_inf;
  D.v_inf = in->v_inf;
  D.ub = in->ub;
  D.vb = in->vb;
  D.omega = in->omega;
  D.psi = d_psi;
  D.f = d_f;
  D.Q = body->qpres.as<double>();
  D.dphi_prev = d_dphi_prev;
  D.xs = body->xs.as<double>();
  D.ys = body->ys.as<double>();
  D.ds = body->ds.as<double>();
  D.pnx = body->pnx.as<double>();
  D.pny = body->pny.as<double>();
  D.st = body->pst.as<PresStencil>();
  D.st_i = body->st_i.as<int>();
  D.st_w = body->st_w.as<double>();
  if (in->mode == GPF_PARTS && body->nparts > 1) {
    D.part = body->part.as<int>();
    for (int j = 0; j < in->nparts && j < GPF_MAX_PARTS; ++j) {
      D.pub[j] = in->parts[j].ub;
      D.pvb[j] = in->parts[j].vb;
      D.pom[j] = in->parts[j].omega;
    }
  }
  D.dphi = d_dphi;
  D.dp = d_dp;
  D.ddt = plan->pres_ddt.as<double>();
  if (plan->fp64)
    GPF_HIP(launch_pres_surface_part<double>(D, s));
  else
    GPF_HIP(launch_pres_surface_part<float>(D, s));
  if (!d_p) return GPF_OK;
  // grid pressure: source on the cells, one FP64 convolution, finish
  const size_t fb = (size_t)n * n * sizeof(double);
  GPF_TRY(plan->ensure_fp64());
  GPF_TRY(plan->pres_w.alloc(fb));
  GPF_TRY(plan->pres_fx.alloc(fb));
  GPF_TRY(plan->pres_fy.alloc(fb));
  GPF_TRY(plan->pres_src.alloc(fb));
  GPF_TRY(plan->pres_tmp.alloc(fb));
  GPF_TRY(plan->pres_X.alloc((size_t)(n + 1) * n * 16));
  GPF_HIP(launch_fill(plan->pres_w.p, fb, s));
  GPF_HIP(launch_fill(plan->pres_fx.p, fb, s));
  GPF_HIP(launch_fill(plan->pres_fy.p, fb, s));
  D.wsheet = plan->pres_w.as<double>();
  D.fx = plan->pres_fx.as<double>();
  D.fy = plan->pres_fy.as<double>();
  D.src = plan->pres_src.as<double>();
  D.tmp = plan->pres_tmp.as<double>();
  D.p = d_p;
  D.pside = d_pside;
  if (plan->fp64)
    GPF_HIP(launch_pres_field_part<double>(D, s));
  else
    GPF_HIP(launch_pres_field_part<float>(D, s));
  ConvDesc cd;
  std::memset(&cd, 0, sizeof(cd));
  cd.in = D.src;
  cd.X = plan->pres_X.p;
  cd.out = D.tmp;
  cd.spec = plan->spec64.p;
  cd.tw = plan->tw64.p;
  cd.gamma = nullptr;
  cd.gamma_val = 0.0;   // a divergence: no net source; the pressure's constant is free
  cd.c = plan->gauge_c;
  cd.zero_in = 0;
  cd.row_lo = 0;
  cd.row_hi = n - 1;
  void *dev = nullptr;
  GPF_TRY(plan->ring.push(&cd, sizeof(cd), s, &dev));
  GPF_HIP((launch_convolve<double, double>(n, static_cast<ConvDesc *>(dev), 1, plan->ctx->xcds, 0, s,
                                            plan->ctx->sched_for(n, true, 1))));
  if (plan->fp64)
    GPF_HIP(launch_pres_finish<double>(D, s));
  else
    GPF_HIP(launch_pres_finish<float>(D, s));
  return GPF_OK;
}

gpf_status gpf_body_set_parts(gpf_body *body, int nparts, const int *h_part) {
  if (!body || !h_part) return fail(GPF_E_INVALID, "gpf_body_set_parts: null argument");
  if (nparts < 2 || nparts > GPF_MAX_PARTS)
    return fail(GPF_E_UNSUPPORTED, "gpf_body_set_parts: nparts must be in [2, GPF_MAX_PARTS]");
  const int ns = body->ns;
  std::vector<int> count(nparts, 0);
  for (int p = 0; p < ns; ++p) {
    if (h_part[p] < 0 || h_part[p] >= nparts)
      return fail(GPF_E_INVALID, "gpf_body_set_parts: part index out of range");
    ++count[h_part[p]];
  }
  for (int j = 0; j < nparts; ++j)
    if (count[j] == 0) return fail(GPF_E_INVALID, "gpf_body_set_parts: empty part");
  GPF_HIP(hipSetDevice(body->plan->ctx->device));
  const size_t vb = ns * sizeof(double);
  // indicator columns 1_j and dS o 1_j
  std::vector<double> ind((size_t)nparts * ns, 0.0), wind((size_t)nparts * ns, 0.0);
  for (int p = 0; p < ns; ++p) {
    ind[(size_t)h_part[p] * ns + p] = 1.0;
    wind[(size_t)h_part[p] * ns + p] = body->hds[p];
  }
  DevBuf dInd, dW, part, gpart, zpart, cpart;
  GPF_TRY(dInd.alloc(nparts * vb));
  GPF_TRY(dW.alloc(nparts * vb));
  GPF_TRY(part.alloc(ns * sizeof(int)));
  GPF_TRY(gpart.alloc(nparts * vb));
  GPF_TRY(zpart.alloc(nparts * vb));
  GPF_TRY(cpart.alloc((size_t)nparts * nparts * sizeof(double)));
  hipStream_t s = nullptr;
  GPF_HIP(hipMemcpy(dInd.p, ind.data(), nparts * vb, hipMemcpyHostToDevice));
  GPF_HIP(hipMemcpy(dW.p, wind.data(), nparts * vb, hipMemcpyHostToDevice));
  GPF_HIP(hipMemcpy(part.p, h_part, ns * sizeof(int), hipMemcpyHostToDevice));
  // z_j = S^-1 1_j; g_j = S^-T (dS o 1_j)
  GPF_HIP(launch_gemv(ns, nparts, body->sinv.as<double>(), dInd.as<double>(), zpart.as<double>(), s));
  for (int j = 0; j < nparts; ++j)
    GPF_HIP(launch_gemv_t(ns, body->sinv.as<double>(), dW.as<double>() + (size_t)j * ns,
                          gpart.as<double>() + (size_t)j * ns, s));
  // C_jl = sum over part j of dS z_l (host, FP64)
  std::vector<double> z((size_t)nparts * ns), C((size_t)nparts * nparts, 0.0);
  GPF_HIP(hipMemcpy(z.data(), zpart.p, nparts * vb, hipMemcpyDeviceToHost));
  for (int l = 0; l < nparts; ++l)
    for (int p = 0; p < ns; ++p) C[(size_t)h_part[p] * nparts + l] += body->hds[p] * z[(size_t)l * ns + p];
  GPF_HIP(hipMemcpy(cpart.p, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice));
  GPF_HIP(hipDeviceSynchronize());
  body->nparts = nparts;
  body->hpart.assign(h_part, h_part + ns);
  for (int e = 0; e < body->nedge; ++e) body->edge_part[e] = h_part[body->edges[e]];
  body->part.swap(part);
  body->gpart.swap(gpart);
  body->zpart.swap(zpart);
  body->cpart.swap(cpart);
  if (body->has_normals) return pressure_setup(body);   // one border per part
  return GPF_OK;
}

gpf_status gpf_body_geometry(const gpf_body *body, double *area, double *xc, double *yc) {
  if (!body) return fail(GPF_E_INVALID, "gpf_body_geometry: null body");
  if (area) *area = body->area;
  if (xc) *xc = body->xc;
  if (yc) *yc = body->yc;
  return GPF_OK;
}

gpf_status gpf_body_added_mass(const gpf_body *body, double rho, double *h_m) {
  if (!body || !h_m || !is_finite(rho)) return fail(GPF_E_INVALID, "gpf_body_added_mass: bad arguments");
  const int ns = body->ns;
  GPF_HIP(hipSetDevice(body->plan->ctx->device));
  // surface streamfunctions of the unit motions, circulation removed:
  // P^Gamma s = s - 1 (fhat0 . s)/Gamma0
  std::vector<double> X(3 * (size_t)ns);
  for (int p = 0; p < ns; ++p) {
    const double x = body->hxs[p], y = body->hys[p];
    X[p] = y;
    X[ns + p] = -x;
    X[2 * ns + p] = -0.5 * (x * x + y * y);
  }
  for (int c = 0; c < 3; ++c) {
    double fs = 0.0;
    for (int p = 0; p < ns; ++p) fs += body->hds[p] * body->hf0[p] * X[c * ns + p];
    const double sh = fs / body->gamma0;
    for (int p = 0; p < ns; ++p) X[c * ns + p] -= sh;
  }
  const size_t vb = ns * sizeof(double);
  DevBuf dX, dF, dImp, dDesc;
  GPF_TRY(dX.alloc(3 * vb));
  GPF_TRY(dF.alloc(3 * vb));
  GPF_TRY(dImp.alloc(9 * sizeof(double)));
  GPF_TRY(dDesc.alloc(3 * sizeof(ProbDesc)));
  hipStream_t s = nullptr;
  GPF_HIP(hipMemcpy(dX.p, X.data(), 3 * vb, hipMemcpyHostToDevice));
  GPF_HIP(launch_gemv(ns, 3, body->sinv.as<double>(), dX.as<double>(), dF.as<double>(), s));
  // the impulse of each sheet with its motion (no vortices)
  ProbDesc pd[3];
  const double motion[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};  // ub, vb, omega
  for (int c = 0; c < 3; ++c) {
    std::memset(&pd[c], 0, sizeof(ProbDesc));
    pd[c].ns = ns;
    pd[c].xs = body->xs.as<double>();
    pd[c].ys = body->ys.as<double>();
    pd[c].ds = body->ds.as<double>();
    pd[c].nx = body->nx.as<double>();
    pd[c].ny = body->ny.as<double>();
    pd[c].f_out = dF.as<double>() + (size_t)c * ns;
    pd[c].imp_out = dImp.as<double>() + 3 * c;
    pd[c].sv.mode = GPF_NOBODY;
    pd[c].sv.ub = motion[c][0];
    pd[c].sv.vb = motion[c][1];
    pd[c].sv.omega = motion[c][2];
    pd[c].sv.znew_from = -1;
  }
  GPF_HIP(hipMemcpy(dDesc.p, pd, sizeof(pd), hipMemcpyHostToDevice));
  GPF_HIP(launch_impulse(static_cast<const ProbDesc *>(dDesc.p), 3, s));
  double imp[9];
  GPF_HIP(hipMemcpy(imp, dImp.p, sizeof(imp), hipMemcpyDeviceToHost));
  for (int c = 0; c < 3; ++c) {
    const double px = imp[3 * c], py = imp[3 * c + 1], pi = imp[3 * c + 2];
    h_m[3 * c] = rho * px;
    h_m[3 * c + 1] = rho * py;
    h_m[3 * c + 2] = rho * (pi - (body->xc * py - body->yc * px));
  }
  return GPF_OK;
}

// ---------------------------------------------------------------------------
// building blocks
// ---------------------------------------------------------------------------

gpf_status gpf_regularize_vortices(gpf_plan *plan, int nv, const double *d_xv, const double *d_yv,
                                   const double *d_gv, void *d_w, int accumulate,
                                   unsigned int *d_status, void *hip_stream) {
  if (!plan || !d_w || nv < 0 || (nv > 0 && (!d_xv || !d_yv || !d_gv)))
    return fail(GPF_E_INVALID, "gpf_regularize_vortices: bad arguments");
  if (nv > kMaxVortices) return fail(GPF_E_UNSUPPORTED, "gpf_regularize_vortices: nv above 2^22");
  hipStream_t s = as_stream(hip_stream);
  TimerScope scope(plan->timing ? &plan->timer : nullptr);
  const int n = plan->grid.n;
  GPF_TRY(plan->ws.ensure_vortices(nv));
  if (!accumulate) GPF_HIP(launch_fill(d_w, (size_t)n * n * (plan->fp64 ? 8 : 4), s));
  ProbDesc pd = single_problem(plan);
  pd.nv = nv;
  pd.xv = d_xv;
  pd.yv = d_yv;
  pd.gv = d_gv;
  pd.w = d_w;
  pd.w_accumulate = accumulate ? 1 : 0;
  pd.w64 = plan->fp64 ? 1 : 0;
  pd.aux = plan->ws.aux.as<double>();
  pd.partials = plan->ws.part.as<double>();
  pd.bin_cnt = plan->ws.bin_cnt.as<int>();
  pd.bin_start = plan->ws.bin_start.as<int>();
  pd.items = plan->ws.items.as<int>();
  pd.halo = plan->ws.halo.p;
  pd.splits = plan->ws.splits.as<int>();
  pd.splitwin = plan->ws.splitwin.as<long long>();
  pd.rank = plan->ws.rank.as<int>();
  pd.sorted = plan->ws.sorted.as<double>();
  if (d_status) pd.status = d_status;
  void *dev = nullptr;
  GPF_TRY(plan->ring.push(&pd, sizeof(pd), s, &dev));
  if (plan->fp64)
    GPF_HIP(launch_scatter_vortices<double>(static_cast<ProbDesc *>(dev), 1, n, nv, s));
  else
    GPF_HIP(launch_scatter_vortices<float>(static_cast<ProbDesc *>(dev), 1, n, nv, s));
  return GPF_OK;
}

gpf_status gpf_convolve(gpf_plan *plan, const void *d_w, void *d_s, double gamma_src,
                        void *hip_stream) {
  if (!plan || !d_w || !d_s || !is_finite(gamma_src))
    return fail(GPF_E_INVALID, "gpf_convolve: bad arguments");
  hipStream_t s = as_stream(hip_stream);
  TimerScope scope(plan->timing ? &plan->timer : nullptr);
  ConvDesc cd;
  std::memset(&cd, 0, sizeof(cd));
  cd.in = const_cast<void *>(d_w);
  cd.X = plan->fp64 ? plan->ws.x64.p : plan->ws.x32.p;
  cd.out = d_s;
  cd.spec = plan->fp64 ? plan->spec64.p : plan->spec32.p;
  cd.tw = plan->fp64 ? plan->tw64.p : plan->tw32.p;
  cd.gamma = nullptr;
  cd.gamma_val = gamma_src;
  cd.c = plan->gauge_c;
  cd.zero_in = 0;
  cd.row_lo = 0;
  cd.row_hi = plan->grid.n - 1;
  void *dev = nullptr;
  GPF_TRY(plan->ring.push(&cd, sizeof(cd), s, &dev));
  const int n = plan->grid.n;
  const int x = plan->ctx->xcds;
  const ConvSched sc = plan->ctx->sched_for(n, plan->fp64, 1);
  if (plan->fp64)
    GPF_HIP((launch_convolve<double, double>(n, static_cast<ConvDesc *>(dev), 1, x, 0, s, sc)));
  else
    GPF_HIP((launch_convolve<float, float>(n, static_cast<ConvDesc *>(dev), 1, x, 0, s, sc)));
  return GPF_OK;
}

gpf_status gpf_interpolate_surface(const gpf_body *body, const void *d_s, double *d_r,
                                   void *hip_stream) {
  if (!body || !d_s || !d_r) return fail(GPF_E_INVALID, "gpf_interpolate_surface: bad arguments");
  hipStream_t s = as_stream(hip_stream);
  const gpf_plan *p = body->plan;
  if (p->fp64)
    GPF_HIP(launch_interp_surface<double>(p->grid.n, body->ns, body->st_i.as<int>(),
                                          body->st_w.as<double>(), (const double *)d_s, d_r, s));
  else
    GPF_HIP(launch_interp_surface<float>(p->grid.n, body->ns, body->st_i.as<int>(),
                                         body->st_w.as<double>(), (const float *)d_s, d_r, s));
  return GPF_OK;
}

gpf_status gpf_vortex_velocity(gpf_plan *plan, const void *d_s, int nv, const double *d_xv,
                               const double *d_yv, double u_inf, double v_inf, double *d_u,
                               double *d_v, unsigned int *d_status, void *hip_stream) {
  if (!plan || !d_s || nv < 0 || (nv > 0 && (!d_xv || !d_yv || !d_u || !d_v)) ||
      !is_finite(u_inf) || !is_finite(v_inf))
    return fail(GPF_E_INVALID, "gpf_vortex_velocity: bad arguments");
  if (nv > kMaxVortices) return fail(GPF_E_UNSUPPORTED, "gpf_vortex_velocity: nv above 2^22");
  hipStream_t s = as_stream(hip_stream);
  TimerScope scope(plan->timing ? &plan->timer : nullptr);
  ProbDesc pd = single_problem(plan);
  pd.nv = nv;
  pd.xv = d_xv;
  pd.yv = d_yv;
  pd.psi = d_s;
  pd.u = d_u;
  pd.v = d_v;
  pd.sv.u_inf = u_inf;
  pd.sv.v_inf = v_inf;
  if (d_status) pd.status = d_status;
  void *dev = nullptr;
  GPF_TRY(plan->ring.push(&pd, sizeof(pd), s, &dev));
  if (plan->fp64)
    GPF_HIP(launch_vortex_velocity<double>(static_cast<ProbDesc *>(dev), 1, nv, s));
  else
    GPF_HIP(launch_vortex_velocity<float>(static_cast<ProbDesc *>(dev), 1, nv, s));
  return GPF_OK;
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------

gpf_status gpf_plan::slot_for(hipStream_t s, gpf_stream_slot **out) {
  std::lock_guard<std::mutex> lk(slots_mu);
  for (auto &sl : slots)
    if (sl->stream == s) {
      *out = sl.get();
      return GPF_OK;
    }
  std::unique_ptr<gpf_stream_slot> sl(new gpf_stream_slot);
  sl->stream = s;
  GPF_TRY(sl->ring.init(kPlanRingSlots, kProblemDescBytes));
  *out = sl.get();
  slots.push_back(std::move(sl));
  return GPF_OK;
}

gpf_status gpf_solve(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in,
                     const gpf_outputs *out, void *hip_stream) {
  GPF_TRY(validate(plan, body, in, out));
  hipError_t e = hipSetDevice(plan->ctx->device);
  if (e != hipSuccess) return fail(GPF_E_DEVICE, hipGetErrorString(e));
  hipStream_t s = as_stream(hip_stream);
  gpf_workspace *ws = &plan->ws;
  DescRing *ring = &plan->ring;
  if (plan->flags & GPF_PLAN_MULTISTREAM) {
    gpf_stream_slot *sl = nullptr;
    GPF_TRY(plan->slot_for(s, &sl));
    ws = &sl->ws;
    ring = &sl->ring;
  }
  ProblemRef r{plan, in->mode == GPF_NOBODY ? nullptr : body, in, out, ws};
  const GroupCfg cfg = config_of(r);
  GPF_TRY(ws->ensure(cfg.n, !cfg.fp64_plan, cfg.fp64_plan || cfg.conv1_fp64,
                     r.body ? r.body->ns : 0, r.body ? body_band(r.body) : 0));
  GPF_TRY(ws->ensure_vortices(in->nv));
  TimerScope scope(plan->timing && ws == &plan->ws ? &plan->timer : nullptr);
  std::vector<ProblemRef> one{r};
  return run_group(cfg, one, *ring, plan->ctx->xcds, s);
}

gpf_status gpf_batch_create(gpf_ctx *ctx, int max_problems, gpf_batch **out) {
  if (!ctx || !out || max_problems < 1 || max_problems > 4096)
    return fail(GPF_E_INVALID, "gpf_batch_create: bad arguments");
  *out = nullptr;
  GPF_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<gpf_batch> b(new gpf_batch);
  b->ctx = ctx;
  b->max_problems = max_problems;
  b->ws.resize(max_problems, nullptr);
  for (auto &w : b->ws) w = new gpf_workspace;
  GPF_TRY(b->ring.init(16, merged_block_bytes(max_problems)));
  *out = b.release();
  return GPF_OK;
}

void gpf_batch_destroy(gpf_batch *batch) { delete batch; }

gpf_status gpf_batch_set_lanes(gpf_batch *batch, int lanes) {
  if (!batch || lanes < 1 || lanes > gpf_batch::kMaxLanes)
    return fail(GPF_E_INVALID, "gpf_batch_set_lanes: lanes must be in [1, 4]");
  GPF_HIP(hipSetDevice(batch->ctx->device));
  if (lanes > 1 && !batch->fork_ev)
    GPF_HIP(hipEventCreateWithFlags(&batch->fork_ev, hipEventDisableTiming));
  for (int l = 0; l < lanes && lanes > 1; ++l) {
    if (!batch->lane_stream[l])
      GPF_HIP(hipStreamCreateWithFlags(&batch->lane_stream[l], hipStreamNonBlocking));
    if (!batch->join_ev[l]) GPF_HIP(hipEventCreateWithFlags(&batch->join_ev[l], hipEventDisableTiming));
  }
  batch->lanes = lanes;
  return GPF_OK;
}

int gpf_batch_get_lanes(const gpf_batch *batch) { return batch ? batch->lanes : 0; }

gpf_status gpf_batch_set_merge(gpf_batch *batch, int merge) {
  if (!batch || merge < 0 || merge > 2)
    return fail(GPF_E_INVALID, "gpf_batch_set_merge: null batch or merge not in [0, 2]");
  batch->merge = merge;
  return GPF_OK;
}

gpf_status gpf_solve_batched(gpf_batch *batch, int nprob, gpf_plan *const *plans,
                             const gpf_body *const *bodies, const gpf_inputs *inputs,
                             const gpf_outputs *outputs, void *hip_stream) {
  if (!batch || nprob < 0 || (nprob > 0 && (!plans || !inputs || !outputs)))
    return fail(GPF_E_INVALID, "gpf_solve_batched: bad arguments");
  if (nprob > batch->max_problems)
    return fail(GPF_E_INVALID, "gpf_solve_batched: more problems than the batch holds");
  GPF_HIP(hipSetDevice(batch->ctx->device));
  std::vector<ProblemRef> refs;
  for (int i = 0; i < nprob; ++i) {
    const gpf_body *b = bodies ? bodies[i] : nullptr;
    GPF_TRY(validate(plans[i], b, &inputs[i], &outputs[i]));
    if (plans[i]->ctx->device != batch->ctx->device)
      return fail(GPF_E_INVALID, "gpf_solve_batched: plan on another device");
    for (int k = 0; k < i; ++k)
      if (outputs[k].d_psi == outputs[i].d_psi)
        return fail(GPF_E_INVALID, "gpf_solve_batched: two problems share an output field");
    ProblemRef r{plans[i], inputs[i].mode == GPF_NOBODY ? nullptr : b, &inputs[i], &outputs[i],
                 batch->ws[i]};
    const GroupCfg cfg = config_of(r);
    if (batch->hw_all) {
      batch->hw_n = std::max(batch->hw_n, cfg.n);
      batch->hw_nv = std::max(batch->hw_nv, inputs[i].nv);
      if (r.body) {
        batch->hw_ns = std::max(batch->hw_ns, r.body->ns);
        batch->hw_band = std::max(batch->hw_band, body_band(r.body));
      }
      batch->hw_w32 = batch->hw_w32 || !cfg.fp64_plan;
      batch->hw_w64 = batch->hw_w64 || cfg.fp64_plan || cfg.conv1_fp64;
    } else {
      const bool w64 = cfg.fp64_plan || cfg.conv1_fp64;
      GPF_TRY(r.ws->ensure(cfg.n, !cfg.fp64_plan, w64, r.body ? r.body->ns : 0,
                           r.body ? body_band(r.body) : 0));
      GPF_TRY(r.ws->ensure_vortices(inputs[i].nv));
    }
    refs.push_back(r);
  }
  if (batch->hw_all) {
    for (ProblemRef &r : refs) {
      GPF_TRY(r.ws->ensure(batch->hw_n, batch->hw_w32, batch->hw_w64, batch->hw_ns, batch->hw_band));
      GPF_TRY(r.ws->ensure_vortices(batch->hw_nv));
    }
  }
  if (nprob == 0) return GPF_OK;
  hipStream_t s = as_stream(hip_stream);
  TimerScope scope(plans[0]->timing ? &plans[0]->timer : nullptr);
  const int lanes = std::min(batch->lanes, nprob);
  if (lanes > 1) {
    GPF_HIP(hipEventRecord(batch->fork_ev, s));
    for (int l = 0; l < lanes; ++l) GPF_HIP(hipStreamWaitEvent(batch->lane_stream[l], batch->fork_ev, 0));
  }
  // group by configuration, keeping the first-seen order of the groups
  std::vector<char> done(nprob, 0);
  std::vector<GroupCfg> cfgs;
  std::vector<std::vector<ProblemRef>> groups;
  for (int i = 0; i < nprob; ++i) {
    if (done[i]) continue;
    const GroupCfg cfg = config_of(refs[i]);
    std::vector<ProblemRef> grp;
    for (int k = i; k < nprob; ++k)
      if (!done[k] && same_cfg(cfg, config_of(refs[k]))) {
        grp.push_back(refs[k]);
        done[k] = 1;
      }
    cfgs.push_back(cfg);
    groups.push_back(std::move(grp));
  }
  const int ng = (int)groups.size();
  bool merge = batch->merge && ng >= 2 && nprob <= kMaxMultiProblems;
  for (int g = 0; g < ng && merge; ++g) merge = mergeable(cfgs[g]);
  if (merge) {
    // one launch per stage and precision class over every grid size; the
    // lanes, if any, wait for nothing and join at once
    if (batch->merge == 1 && !batch->side) {
      GPF_HIP(hipStreamCreateWithFlags(&batch->side, hipStreamNonBlocking));
      GPF_HIP(hipEventCreateWithFlags(&batch->side_fork, hipEventDisableTiming));
      GPF_HIP(hipEventCreateWithFlags(&batch->side_join, hipEventDisableTiming));
      GPF_HIP(hipStreamCreateWithFlags(&batch->side2, hipStreamNonBlocking));
      GPF_HIP(hipEventCreateWithFlags(&batch->side2_join, hipEventDisableTiming));
    }
    GPF_TRY(run_merged(refs, batch->ring, batch->ctx->xcds, s, batch->merge == 1 ? batch : nullptr));
  } else if (lanes == 1) {
    for (int g = 0; g < ng; ++g) GPF_TRY(run_group(cfgs[g], groups[g], batch->ring, batch->ctx->xcds, s));
  } else if (ng >= 2) {
    // several groups: whole groups to lanes, the costliest first to the
    // least loaded lane (cost ~ problems x n^2), so that small grids run
    // beside large ones
    std::vector<int> order(ng);
    for (int g = 0; g < ng; ++g) order[g] = g;
    auto cost = [&](int g) { return (double)groups[g].size() * cfgs[g].n * cfgs[g].n; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<double> load(lanes, 0.0);
    for (int g : order) {
      const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[l] += cost(g);
      GPF_TRY(run_group(cfgs[g], groups[g], batch->ring, batch->ctx->xcds, batch->lane_stream[l]));
    }
  } else {
    // one group: its members dealt out over the lanes
    const std::vector<ProblemRef> &grp = groups[0];
    const int per = ((int)grp.size() + lanes - 1) / lanes;
    for (int l = 0; l < lanes; ++l) {
      const int a = l * per, b = std::min((int)grp.size(), a + per);
      if (a >= b) break;
      std::vector<ProblemRef> part(grp.begin() + a, grp.begin() + b);
      GPF_TRY(run_group(cfgs[0], part, batch->ring, batch->ctx->xcds, batch->lane_stream[l]));
    }
  }
  if (lanes > 1) {
    for (int l = 0; l < lanes; ++l) {
      GPF_HIP(hipEventRecord(batch->join_ev[l], batch->lane_stream[l]));
      GPF_HIP(hipStreamWaitEvent(s, batch->join_ev[l], 0));
    }
  }
  return GPF_OK;
}

// ---------------------------------------------------------------------------
// explicit-midpoint time stepping
// ---------------------------------------------------------------------------

gpf_rk2::~gpf_rk2() {
  // the ring slots the graph replays are released once its last replay is done
  if (done) {
    (void)hipEventSynchronize(done);
    (void)hipEventDestroy(done);
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (cap) (void)hipStreamDestroy(cap);
  for (int k : held) plan->ring.unpin(k);
}

namespace gpf {
namespace {

// one step: two solves and two position updates, enqueued on s
gpf_status rk2_enqueue(gpf_rk2 *rk, hipStream_t s) {
  gpf_plan *plan = rk->plan;
  ProblemRef r1{plan, rk->body, &rk->in1, &rk->out1, &rk->ws};
  ProblemRef r2{plan, rk->body, &rk->in2, &rk->out2, &rk->ws};
  const GroupCfg cfg = config_of(r1);
  std::vector<ProblemRef> one{r1};
  GPF_TRY(run_group(cfg, one, plan->ring, plan->ctx->xcds, s));
  GPF_HIP(launch_axpy2(rk->nv, rk->x, rk->y, rk->u1.as<double>(), rk->v1.as<double>(),
                       0.5 * rk->dt, rk->xm.as<double>(), rk->ym.as<double>(), s));
  one[0] = r2;
  GPF_TRY(run_group(cfg, one, plan->ring, plan->ctx->xcds, s));
  GPF_HIP(launch_axpy2(rk->nv, rk->x, rk->y, rk->u2.as<double>(), rk->v2.as<double>(), rk->dt,
                       rk->x, rk->y, s));
  return GPF_OK;
}

}  // namespace
}  // namespace gpf

gpf_status gpf_rk2_create(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in, double *d_x,
                          double *d_y, double dt, int use_graph, gpf_rk2 **out) {
  if (!plan || !in || !out || (in->nv > 0 && (!d_x || !d_y)) || !is_finite(dt))
    return fail(GPF_E_INVALID, "gpf_rk2_create: bad arguments");
  *out = nullptr;
  if (in->mode == GPF_KUTTA_SHED || (in->mode == GPF_PARTS && in->m > 0))
    return fail(GPF_E_UNSUPPORTED, "gpf_rk2_create: the shedding mode needs a vortex release rule");
  GPF_HIP(hipSetDevice(plan->ctx->device));
  std::unique_ptr<gpf_rk2> rk(new gpf_rk2);
  rk->plan = plan;
  rk->body = in->mode == GPF_NOBODY ? nullptr : body;
  rk->x = d_x;
  rk->y = d_y;
  rk->dt = dt;
  rk->nv = in->nv;
  rk->use_graph = use_graph != 0;
  const int n = plan->grid.n;
  const size_t vb = std::max(1, in->nv) * sizeof(double);
  const int ns = rk->body ? rk->body->ns : 1;
  GPF_TRY(rk->xm.alloc(vb));
  GPF_TRY(rk->ym.alloc(vb));
  GPF_TRY(rk->u1.alloc(vb));
  GPF_TRY(rk->v1.alloc(vb));
  GPF_TRY(rk->u2.alloc(vb));
  GPF_TRY(rk->v2.alloc(vb));
  GPF_TRY(rk->psi.alloc((size_t)n * n * (plan->fp64 ? 8 : 4)));
  GPF_TRY(rk->f.alloc(ns * sizeof(double)));
  GPF_TRY(rk->ft.alloc(ns * sizeof(double)));
  GPF_TRY(rk->sc.alloc(SC_COUNT * sizeof(double)));
  GPF_TRY(rk->status.alloc(sizeof(unsigned)));
  GPF_TRY(fill_now(rk->status.p, 0, sizeof(unsigned)));
  rk->in1 = *in;
  rk->in1.d_xv = d_x;
  rk->in1.d_yv = d_y;
  rk->in2 = rk->in1;
  rk->in2.d_xv = rk->xm.as<double>();
  rk->in2.d_yv = rk->ym.as<double>();
  gpf_outputs o{};
  o.d_psi = rk->psi.p;
  o.d_f = rk->body ? rk->f.as<double>() : nullptr;
  o.d_ftilde = rk->body ? rk->ft.as<double>() : nullptr;
  o.d_scalars = rk->sc.as<double>();
  o.d_status = rk->status.as<unsigned>();
  rk->out1 = o;
  rk->out1.d_u = rk->u1.as<double>();
  rk->out1.d_v = rk->v1.as<double>();
  rk->out2 = o;
  rk->out2.d_u = rk->u2.as<double>();
  rk->out2.d_v = rk->v2.as<double>();
  GPF_TRY(validate(plan, rk->body, &rk->in1, &rk->out1));
  {
    // a workspace of its own: a captured step keeps pointing at it, and
    // other calls on the plan may grow (reallocate) the plan's workspace
    ProblemRef r{plan, rk->body, &rk->in1, &rk->out1, &rk->ws};
    const GroupCfg cfg = config_of(r);
    GPF_TRY(rk->ws.ensure(cfg.n, !cfg.fp64_plan, cfg.fp64_plan || cfg.conv1_fp64,
                          rk->body ? rk->body->ns : 0, rk->body ? body_band(rk->body) : 0));
    GPF_TRY(rk->ws.ensure_vortices(in->nv));
  }
  if (rk->use_graph) {
    GPF_HIP(hipStreamCreateWithFlags(&rk->cap, hipStreamNonBlocking));
    GPF_HIP(hipEventCreateWithFlags(&rk->done, hipEventDisableTiming));
    // capture one step; descriptors pushed while capturing stay reserved
    // (rk->held) until the handle is destroyed
    const std::vector<char> pinned_before = plan->ring.pinned;
    GPF_HIP(hipStreamBeginCapture(rk->cap, hipStreamCaptureModeThreadLocal));
    gpf_status st;
    {
      TimerScope none(nullptr);
      plan->ring.defer_captured = true;   // the slots get one copy, below
      st = rk2_enqueue(rk.get(), rk->cap);
      plan->ring.defer_captured = false;
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(rk->cap, &g);
    for (int k = 0; k < plan->ring.slots; ++k)
      if (plan->ring.pinned[k] && !pinned_before[k]) rk->held.push_back(k);
    const gpf_status fst = plan->ring.flush_deferred();
    if (st == GPF_OK) st = fst;
    if (st != GPF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;   // ~gpf_rk2 releases the slots: nothing was replayed
    }
    GPF_HIP(e);
    rk->graph = g;
    GPF_HIP(hipGraphInstantiate(&rk->exec, rk->graph, nullptr, nullptr, 0));
  }
  *out = rk.release();
  return GPF_OK;
}

gpf_status gpf_rk2_run(gpf_rk2 *rk, int nsteps, void *hip_stream) {
  if (!rk || nsteps < 0) return fail(GPF_E_INVALID, "gpf_rk2_run: bad arguments");
  hipStream_t s = as_stream(hip_stream);
  GPF_HIP(hipSetDevice(rk->plan->ctx->device));
  for (int k = 0; k < nsteps; ++k) {
    if (rk->use_graph) {
      GPF_HIP(hipGraphLaunch(rk->exec, s));
    } else {
      TimerScope scope(rk->plan->timing ? &rk->plan->timer : nullptr);
      GPF_TRY(rk2_enqueue(rk, s));
    }
  }
  if (rk->use_graph && nsteps > 0) GPF_HIP(hipEventRecord(rk->done, s));
  return GPF_OK;
}

gpf_status gpf_rk2_fields(const gpf_rk2 *rk, const void **d_psi, const double **d_u,
                          const double **d_v, const double **d_f, const double **d_scalars,
                          unsigned int **d_status) {
  if (!rk) return fail(GPF_E_INVALID, "gpf_rk2_fields: null object");
  if (d_psi) *d_psi = rk->psi.p;
  if (d_u) *d_u = rk->u2.as<double>();
  if (d_v) *d_v = rk->v2.as<double>();
  if (d_f) *d_f = rk->body ? rk->f.as<double>() : nullptr;
  if (d_scalars) *d_scalars = rk->sc.as<double>();
  if (d_status) *d_status = rk->status.as<unsigned>();
  return GPF_OK;
}

void gpf_rk2_destroy(gpf_rk2 *rk) { delete rk; }

// ---------------------------------------------------------------------------
// shedding with forward Euler steps
// ---------------------------------------------------------------------------

namespace gpf {
namespace {

// one step: place the new vortices, solve, store strengths and move
gpf_status shed_enqueue(gpf_shed *sh, const ShedGeom &geom, hipStream_t s) {
  gpf_plan *plan = sh->plan;
  const int nv = sh->nv + sh->m;
  double *x = sh->x, *y = sh->y, *g = sh->g;
  int *last = sh->last.as<int>();
  GPF_HIP(launch_shed_place(geom, sh->nv, last, x, y, g, s));
  sh->in.nv = nv;
  gpf_outputs o = sh->out;   // the impulse, if asked for, goes to this step's row
  if (o.d_impulse) o.d_impulse += 3 * (size_t)sh->steps;
  double *gw = sh->in.mode == GPF_PARTS ? sh->gw.as<double>() : nullptr;
  ProblemRef r{plan, sh->body, &sh->in, &o, &plan->ws, sh->nv, gw};
  const GroupCfg cfg = config_of(r);
  std::vector<ProblemRef> one{r};
  GPF_TRY(run_group(cfg, one, plan->ring, plan->ctx->xcds, s));
  GPF_HIP(launch_shed_advance(geom, nv, sh->out.d_scalars, last, gw, x, y, g, sh->out.d_u,
                              sh->out.d_v, sh->dt, s));
  sh->nv = nv;
  ++sh->steps;
  return GPF_OK;
}

}  // namespace
}  // namespace gpf

gpf_status gpf_shed_create(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in,
                           const gpf_outputs *out, double *d_x, double *d_y, double *d_g,
                           int capacity, double dt, const double *h_first, gpf_shed **psh) {
  if (!plan || !body || !in || !out || !psh || !h_first || !is_finite(dt) || in->nv < 0 ||
      !d_x || !d_y || !d_g)
    return fail(GPF_E_INVALID, "gpf_shed_create: bad arguments");
  *psh = nullptr;
  if (!out->d_u || !out->d_v || !out->d_scalars)
    return fail(GPF_E_INVALID, "gpf_shed_create: d_u, d_v and d_scalars are required");
  const bool parts = in->mode == GPF_PARTS;
  if (in->mode != GPF_KUTTA_SHED && !parts)
    return fail(GPF_E_INVALID, "gpf_shed_create: needs the shedding mode or GPF_PARTS");
  if (in->ub != 0.0 || in->vb != 0.0 || in->omega != 0.0)
    return fail(GPF_E_UNSUPPORTED,
                "gpf_shed_create: the body stays in place; give a translation as the uniform flow");
  // the shedding edges, in body edge order, and the part of each
  int m = 0;
  int edge_idx[GPF_MAX_EDGES], epart[GPF_MAX_EDGES] = {};
  if (parts) {
    if (body->nparts < 2 || in->nparts != body->nparts)
      return fail(GPF_E_INVALID, "gpf_shed_create: GPF_PARTS needs a body split into in->nparts parts");
    for (int j = 0; j < in->nparts; ++j) {
      const gpf_part &q = in->parts[j];
      if (q.ub != 0.0 || q.vb != 0.0 || q.omega != 0.0)
        return fail(GPF_E_UNSUPPORTED, "gpf_shed_create: every part stays in place");
    }
    for (int e = 0; e < body->nedge; ++e) {
      const int j = body->edge_part[e];
      if (j >= 0 && j < in->nparts && in->parts[j].mode == GPF_KUTTA_SHED) {
        edge_idx[m] = body->edges[e];
        epart[m] = j;
        ++m;
      }
    }
  } else {
    m = body->nedge;
    for (int e = 0; e < m; ++e) edge_idx[e] = body->edges[e];
  }
  if (m < 1 || in->m != m)
    return fail(GPF_E_INVALID, "gpf_shed_create: one new vortex per shedding edge");
  if (capacity < in->nv + m) return fail(GPF_E_INVALID, "gpf_shed_create: capacity below nv + m");
  for (int j = 0; j < 2 * m; ++j)
    if (!is_finite(h_first[j])) return fail(GPF_E_INVALID, "gpf_shed_create: non-finite h_first");
  GPF_HIP(hipSetDevice(plan->ctx->device));
  std::unique_ptr<gpf_shed> sh(new gpf_shed);
  sh->plan = plan;
  sh->body = body;
  sh->nv = in->nv;
  sh->capacity = capacity;
  sh->m = m;
  sh->dt = dt;
  for (int j = 0; j < 2 * m; ++j) sh->first[j] = h_first[j];
  for (int j = 0; j < m; ++j) {
    sh->epart[j] = epart[j];
    const size_t k = (size_t)edge_idx[j];
    GPF_HIP(hipMemcpy(&sh->edge_xy[2 * j], body->xs.as<double>() + k, sizeof(double),
                      hipMemcpyDeviceToHost));
    GPF_HIP(hipMemcpy(&sh->edge_xy[2 * j + 1], body->ys.as<double>() + k, sizeof(double),
                      hipMemcpyDeviceToHost));
  }
  GPF_TRY(sh->last.alloc(GPF_MAX_EDGES * sizeof(int)));
  GPF_TRY(fill_now(sh->last.p, 0xff, GPF_MAX_EDGES * sizeof(int)));   // -1: nothing released
  if (parts) {
    double gw0[GPF_MAX_PARTS] = {};
    for (int j = 0; j < in->nparts; ++j) gw0[j] = in->parts[j].gamma_w;
    GPF_TRY(sh->gw.alloc(GPF_MAX_PARTS * sizeof(double)));
    GPF_HIP(hipMemcpy(sh->gw.p, gw0, sizeof(gw0), hipMemcpyHostToDevice));
  }
  sh->x = d_x;
  sh->y = d_y;
  sh->g = d_g;
  sh->in = *in;
  sh->in.d_xv = d_x;
  sh->in.d_yv = d_y;
  sh->in.d_gv = d_g;
  sh->in.nv = in->nv + m;
  sh->in.gamma_w = std::nan("");
  for (int j = 0; j < GPF_MAX_EDGES; ++j) sh->in.h_xnew[j] = sh->in.h_ynew[j] = 0.0;
  sh->out = *out;
  GPF_TRY(validate(plan, body, &sh->in, &sh->out));
  ProblemRef r{plan, body, &sh->in, &sh->out, &plan->ws, in->nv};
  const GroupCfg cfg = config_of(r);
  GPF_TRY(plan->ws.ensure(cfg.n, !cfg.fp64_plan, cfg.fp64_plan || cfg.conv1_fp64, body->ns,
                          body_band(body)));
  GPF_TRY(plan->ws.ensure_vortices(capacity));
  *psh = sh.release();
  return GPF_OK;
}

gpf_status gpf_shed_run(gpf_shed *sh, int nsteps, void *hip_stream) {
  if (!sh || nsteps < 0) return fail(GPF_E_INVALID, "gpf_shed_run: bad arguments");
  if ((long long)sh->nv + (long long)nsteps * sh->m > sh->capacity)
    return fail(GPF_E_INVALID, "gpf_shed_run: the steps would exceed the vortex capacity");
  hipStream_t s = as_stream(hip_stream);
  GPF_HIP(hipSetDevice(sh->plan->ctx->device));
  ShedGeom geom{};
  geom.m = sh->m;
  for (int j = 0; j < sh->m; ++j) {
    geom.ex[j] = sh->edge_xy[2 * j];
    geom.ey[j] = sh->edge_xy[2 * j + 1];
    geom.fx[j] = sh->first[2 * j];
    geom.fy[j] = sh->first[2 * j + 1];
    geom.epart[j] = sh->epart[j];
  }
  TimerScope scope(sh->plan->timing ? &sh->plan->timer : nullptr);
  for (int k = 0; k < nsteps; ++k) GPF_TRY(shed_enqueue(sh, geom, s));
  return GPF_OK;
}

int gpf_shed_count(const gpf_shed *sh) { return sh ? sh->nv : -1; }

void gpf_shed_destroy(gpf_shed *sh) { delete sh; }

gpf_status gpf_timing_enable(gpf_plan *plan, int enable) {
  if (!plan) return fail(GPF_E_INVALID, "gpf_timing_enable: null plan");
  if (enable) plan->timer.reset();
  plan->timing = enable != 0;
  return GPF_OK;
}

gpf_status gpf_timing_read(gpf_plan *plan, int kind, long long *count, double *total_ms) {
  if (!plan || kind < 0 || kind >= GPF_TK_COUNT || !count || !total_ms)
    return fail(GPF_E_INVALID, "gpf_timing_read: bad arguments");
  GPF_TRY(plan->timer.flush());
  *count = plan->timer.count[kind];
  *total_ms = plan->timer.total_ms[kind];
  return GPF_OK;
}

gpf_status gpf_sync(void *hip_stream, unsigned int *d_status) {
  if (!d_status) return fail(GPF_E_INVALID, "gpf_sync: null status");
  hipStream_t s = as_stream(hip_stream);
  unsigned h = 0;
  GPF_HIP(hipMemcpyAsync(&h, d_status, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  GPF_HIP(hipStreamSynchronize(s));
  if (h) {
    unsigned zero = 0;
    GPF_HIP(hipMemcpy(d_status, &zero, sizeof(unsigned), hipMemcpyHostToDevice));
  }
  if (h & GPF_DEV_OUT_OF_GRID) return fail(GPF_E_OUT_OF_GRID, "a stencil left the grid window");
  if (h & GPF_DEV_SINGULAR) return fail(GPF_E_SINGULAR, "singular edge system");
  return GPF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// convolution schedules and the autotuner
// ---------------------------------------------------------------------------

int sched_class(int nb) { return nb <= 1 ? 0 : (nb < 8 ? 1 : (nb < 32 ? 2 : 3)); }

namespace {
long long sched_key(int n, bool fp64, int cls) {
  return ((long long)n << 8) | ((fp64 ? 1 : 0) << 4) | cls;
}
bool sched_valid(const gpf_schedule &s) {
  return s.rows >= 0 && s.rows <= 2 && s.order >= 0 && s.order <= 2 && s.cols >= 0 && s.cols <= 2;
}
}  // namespace

gpf::ConvSched gpf_ctx::sched_for(int n, bool fp64, int nb) {
  std::lock_guard<std::mutex> lk(sched_mu);
  auto it = sched.find(sched_key(n, fp64, sched_class(nb)));
  return it == sched.end() ? gpf::ConvSched{} : it->second;
}

gpf_status gpf_schedule_set(gpf_ctx *ctx, int n, int fp64, int nb, const gpf_schedule *s) {
  if (!ctx || nb < 1) return fail(GPF_E_INVALID, "gpf_schedule_set: bad arguments");
  if (s && !sched_valid(*s)) return fail(GPF_E_INVALID, "gpf_schedule_set: value out of range");
  std::lock_guard<std::mutex> lk(ctx->sched_mu);
  const long long key = sched_key(n, fp64 != 0, sched_class(nb));
  if (s) {
    gpf::ConvSched c;
    c.rows = s->rows;
    c.order = s->order;
    c.cols = s->cols;
    ctx->sched[key] = c;
  } else {
    ctx->sched.erase(key);
  }
  return GPF_OK;
}

gpf_status gpf_schedule_get(gpf_ctx *ctx, int n, int fp64, int nb, gpf_schedule *s) {
  if (!ctx || nb < 1 || !s) return fail(GPF_E_INVALID, "gpf_schedule_get: bad arguments");
  const gpf::ConvSched c = ctx->sched_for(n, fp64 != 0, nb);
  s->rows = c.rows;
  s->order = c.order;
  s->cols = c.cols;
  return GPF_OK;
}

namespace gpf {
namespace {

// the schedules the tuners try: the rules first, then every explicit shape
std::vector<ConvSched> sched_candidates(bool fp64, int n) {
  std::vector<ConvSched> c(1);
  const int ncols = (fp64 && n >= 512) ? 2 : 1;
  for (int r = 1; r <= 2; ++r)
    for (int o = 1; o <= 2; ++o)
      for (int k = 0; k < ncols; ++k) {
        ConvSched x;
        x.rows = r;
        x.order = o;
        x.cols = ncols == 2 ? 1 + k : 0;
        c.push_back(x);
      }
  return c;
}

// a cached result for (arch, n, precision, class), or false
bool tune_cache_read(const char *path, const char *arch, int n, int fp64, int cls, ConvSched *sc,
                     double *us) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char a[64];
    int nn, d, c, r, o, k;
    double t;
    if (std::sscanf(line, "%63s %d %d %d %d %d %d %lf", a, &nn, &d, &c, &r, &o, &k, &t) != 8) continue;
    if (std::strcmp(a, arch) || nn != n || d != fp64 || c != cls) continue;
    gpf_schedule g{r, o, k};
    if (!sched_valid(g)) continue;
    sc->rows = r;
    sc->order = o;
    sc->cols = k;
    *us = t;
    found = true;   // the last matching line wins
  }
  std::fclose(f);
  return found;
}

template <class T>
gpf_status tune_precision(gpf_plan *plan, int nb, ConvSched *best, double *best_us) {
  const int n = plan->grid.n;
  constexpr bool D = std::is_same<T, double>::value;
  const size_t cells = (size_t)n * n, half = (size_t)(n + 1) * n;
  const size_t per = cells * sizeof(T) * 2 + half * 2 * sizeof(T);
  if ((double)per * nb > 16.0 * (1ull << 30)) return fail(GPF_E_NOMEM, "gpf_autotune: more than 16 GiB");
  DevBuf src, X, out, desc;
  GPF_TRY(src.alloc(cells * sizeof(T) * nb));
  GPF_TRY(X.alloc(half * 2 * sizeof(T) * nb));
  GPF_TRY(out.alloc(cells * sizeof(T) * nb));
  GPF_TRY(desc.alloc(sizeof(ConvDesc) * nb));
  GPF_TRY(fill_now(src.p, 0, src.bytes));
  std::vector<ConvDesc> cd(nb);
  for (int i = 0; i < nb; ++i) {
    ConvDesc &c = cd[i];
    std::memset(&c, 0, sizeof(c));
    c.in = src.as<char>() + cells * sizeof(T) * i;
    c.X = X.as<char>() + half * 2 * sizeof(T) * i;
    c.out = out.as<char>() + cells * sizeof(T) * i;
    c.spec = D ? plan->spec64.p : plan->spec32.p;
    c.tw = D ? plan->tw64.p : plan->tw32.p;
    c.c = plan->gauge_c;
    c.row_lo = 0;
    c.row_hi = n - 1;
  }
  GPF_HIP(hipMemcpy(desc.p, cd.data(), sizeof(ConvDesc) * nb, hipMemcpyHostToDevice));
  const ConvDesc *d = desc.as<const ConvDesc>();
  const std::vector<ConvSched> cands = sched_candidates(D, n);
  hipStream_t s = nullptr;
  GPF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  gpf_status st = GPF_OK;
  auto run = [&]() -> gpf_status {
    GPF_HIP(hipEventCreate(&e0));
    GPF_HIP(hipEventCreate(&e1));
    const int xcds = plan->ctx->xcds;
    constexpr int kReps = 10;
    *best_us = 1e30;
    for (const ConvSched &c : cands) {
      for (int w = 0; w < 2; ++w) GPF_HIP((launch_convolve<T, T>(n, d, nb, xcds, 0, s, c)));
      double t_min = 1e30;
      for (int round = 0; round < 2; ++round) {
        GPF_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < kReps; ++k) GPF_HIP((launch_convolve<T, T>(n, d, nb, xcds, 0, s, c)));
        GPF_HIP(hipEventRecord(e1, s));
        GPF_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        GPF_HIP(hipEventElapsedTime(&ms, e0, e1));
        t_min = std::min(t_min, 1e3 * ms / kReps);
      }
      if (t_min < *best_us) {
        *best_us = t_min;
        *best = c;
      }
    }
    return GPF_OK;
  };
  {
    TimerScope none(nullptr);
    st = run();
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipStreamDestroy(s);
  return st;
}

}  // namespace
}  // namespace gpf

gpf_status gpf_autotune(gpf_plan *plan, int fp64, int nb, const char *cache_path,
                        gpf_schedule *chosen, double *us) {
  if (!plan || nb < 1 || nb > 1024) return fail(GPF_E_INVALID, "gpf_autotune: bad arguments");
  GPF_HIP(hipSetDevice(plan->ctx->device));
  gpf_ctx *ctx = plan->ctx;
  const int n = plan->grid.n;
  const int cls = sched_class(nb);
  ConvSched best;
  double t = 0.0;
  if (!(cache_path && tune_cache_read(cache_path, ctx->arch, n, fp64 ? 1 : 0, cls, &best, &t))) {
    if (fp64) {
      if (!plan->spec64.p) GPF_TRY(upload_spectrum<double>(plan, plan->spec64, plan->tw64));
      GPF_TRY(tune_precision<double>(plan, nb, &best, &t));
    } else {
      if (!plan->spec32.p) GPF_TRY(upload_spectrum<float>(plan, plan->spec32, plan->tw32));
      GPF_TRY(tune_precision<float>(plan, nb, &best, &t));
    }
    if (cache_path) {
      FILE *f = std::fopen(cache_path, "a");
      if (!f) return fail(GPF_E_INVALID, "gpf_autotune: cannot append to the cache file");
      std::fprintf(f, "%s %d %d %d %d %d %d %.3f\n", ctx->arch, n, fp64 ? 1 : 0, cls, best.rows,
                   best.order, best.cols, t);
      std::fclose(f);
    }
  }
  gpf_schedule g{best.rows, best.order, best.cols};
  GPF_TRY(gpf_schedule_set(ctx, n, fp64, nb, &g));
  if (chosen) *chosen = g;
  if (us) *us = t;
  return GPF_OK;
}

gpf_status gpf_autotune_batched(gpf_batch *batch, int nprob, gpf_plan *const *plans,
                                const gpf_body *const *bodies, const gpf_inputs *inputs,
                                const gpf_outputs *outputs, void *hip_stream) {
  if (!batch || nprob < 1 || nprob > batch->max_problems || !plans || !inputs || !outputs)
    return fail(GPF_E_INVALID, "gpf_autotune_batched: bad arguments");
  GPF_HIP(hipSetDevice(batch->ctx->device));
  gpf_ctx *ctx = batch->ctx;
  // the groups gpf_solve_batched forms, and the schedule entries they use
  std::vector<GroupCfg> cfgs;
  std::vector<int> counts;
  for (int i = 0; i < nprob; ++i) {
    const gpf_body *b = bodies ? bodies[i] : nullptr;
    GPF_TRY(validate(plans[i], b, &inputs[i], &outputs[i]));
    ProblemRef r{plans[i], inputs[i].mode == GPF_NOBODY ? nullptr : b, &inputs[i], &outputs[i],
                 batch->ws[i]};
    const GroupCfg cfg = config_of(r);
    size_t g = 0;
    while (g < cfgs.size() && !same_cfg(cfgs[g], cfg)) ++g;
    if (g == cfgs.size()) {
      cfgs.push_back(cfg);
      counts.push_back(0);
    }
    ++counts[g];
  }
  hipStream_t s = as_stream(hip_stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GPF_HIP(hipEventCreate(&e0));
  GPF_HIP(hipEventCreate(&e1));
  constexpr int kLaneWarm = 400;
  auto timed = [&](double *us) -> gpf_status {
    GPF_TRY(gpf_solve_batched(batch, nprob, plans, bodies, inputs, outputs, hip_stream));
    constexpr int kReps = 3;
    double best = 1e30;
    for (int round = 0; round < 2; ++round) {
      GPF_HIP(hipEventRecord(e0, s));
      for (int k = 0; k < kReps; ++k)
        GPF_TRY(gpf_solve_batched(batch, nprob, plans, bodies, inputs, outputs, hip_stream));
      GPF_HIP(hipEventRecord(e1, s));
      GPF_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      GPF_HIP(hipEventElapsedTime(&ms, e0, e1));
      best = std::min(best, 1e3 * ms / kReps);
    }
    *us = best;
    return GPF_OK;
  };
  gpf_status st = GPF_OK;
  // the lane count first, with the schedules as they stand
  {
    int best_l = batch->lanes;
    double best_us = 1e30;
    for (int l = 1; l <= gpf_batch::kMaxLanes && st == GPF_OK; ++l) {
      st = gpf_batch_set_lanes(batch, l);
      // several lanes run on streams of their own, whose first few hundred
      // solves of a workload run up to 3x slower (measured on the 512^2
      // plate batch with two lanes: settled after ~250): run them in first
      // (the same workload: a lighter one does not do it)
      for (int k = 0; l > 1 && k < kLaneWarm && st == GPF_OK; ++k)
        st = gpf_solve_batched(batch, nprob, plans, bodies, inputs, outputs, hip_stream);
      double us = 0.0;
      if (st == GPF_OK) st = timed(&us);
      if (st == GPF_OK && us < best_us) {
        best_us = us;
        best_l = l;
      }
    }
    if (st == GPF_OK) st = gpf_batch_set_lanes(batch, best_l);
  }
  const int lanes = std::min(batch->lanes, nprob);
  struct Key {
    int n, nb;
    bool fp64;
  };
  std::vector<Key> keys;
  auto add = [&](int n, bool fp64, int nb) {
    for (const Key &k : keys)
      if (k.n == n && k.fp64 == fp64 && sched_class(k.nb) == sched_class(nb)) return;
    keys.push_back(Key{n, nb, fp64});
  };
  for (size_t g = 0; g < cfgs.size(); ++g) {
    // launch size of the group: whole groups go to lanes when there are
    // several, a single group is dealt out over them
    const int nb = (lanes > 1 && cfgs.size() == 1) ? (counts[g] + lanes - 1) / lanes : counts[g];
    add(cfgs[g].n, cfgs[g].fp64_plan || cfgs[g].conv1_fp64, nb);
    if (cfgs[g].body) add(cfgs[g].n, cfgs[g].fp64_plan, nb);
  }
  for (const Key &k : keys) {
    if (st != GPF_OK) break;
    ConvSched best;
    double best_us = 1e30;
    for (const ConvSched &c : sched_candidates(k.fp64, k.n)) {
      gpf_schedule g{c.rows, c.order, c.cols};
      st = gpf_schedule_set(ctx, k.n, k.fp64, k.nb, &g);
      double us = 0.0;
      if (st == GPF_OK) st = timed(&us);
      if (st != GPF_OK) break;
      if (us < best_us) {
        best_us = us;
        best = c;
      }
    }
    if (st != GPF_OK) break;
    gpf_schedule g{best.rows, best.order, best.cols};
    GPF_TRY(gpf_schedule_set(ctx, k.n, k.fp64, k.nb, &g));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// ---------------------------------------------------------------------------
// Schur complement built column by column through batched convolutions
// ---------------------------------------------------------------------------

namespace gpf {
namespace {

template <class T>
gpf_status schur_by_columns(gpf_body *b, int batch, double *S, hipStream_t s) {
  gpf_plan *pl = b->plan;
  const int n = pl->grid.n, ns = b->ns;
  constexpr bool D = std::is_same<T, double>::value;
  const size_t cells = (size_t)n * n, half = (size_t)(n + 1) * n;
  DevBuf w, X, out, desc;
  GPF_TRY(w.alloc(cells * sizeof(T) * batch));
  GPF_TRY(X.alloc(half * 2 * sizeof(T) * batch));
  GPF_TRY(out.alloc(cells * sizeof(T) * batch));
  GPF_TRY(desc.alloc(sizeof(ConvDesc) * batch));
  GPF_HIP(launch_fill(w.p, w.bytes, s));   // sources start zero; the row pass leaves them zero
  std::vector<ConvDesc> cd(batch);
  const int band = body_band(b);
  for (int q0 = 0; q0 < ns; q0 += batch) {
    const int nb = std::min(batch, ns - q0);
    for (int i = 0; i < nb; ++i) {
      ConvDesc &c = cd[i];
      std::memset(&c, 0, sizeof(c));
      c.in = w.as<char>() + cells * sizeof(T) * i;
      c.X = X.as<char>() + half * 2 * sizeof(T) * i;
      c.out = out.as<char>() + cells * sizeof(T) * i;
      c.spec = D ? pl->spec64.p : pl->spec32.p;
      c.tw = D ? pl->tw64.p : pl->tw32.p;
      c.gamma_val = b->hds[q0 + i];   // circulation of the unit sheet: dS_q
      c.c = pl->gauge_c;
      c.zero_in = 1;
      c.row_lo = b->row_lo;            // only the surface stencils read the result
      c.row_hi = b->row_hi;
    }
    GPF_HIP(hipMemcpyAsync(desc.p, cd.data(), sizeof(ConvDesc) * nb, hipMemcpyHostToDevice, s));
    GPF_HIP(launch_unit_sheets<T>(n, ns, q0, nb, pl->grid.dx, b->st_i.as<int>(),
                                  b->st_w.as<double>(), b->ds.as<double>(), w.as<T>(), cells, s));
    GPF_HIP((launch_convolve<T, T>(n, desc.as<const ConvDesc>(), nb, pl->ctx->xcds, band, s,
                                   pl->ctx->sched_for(n, D, nb))));
    GPF_HIP(launch_interp_columns<T>(n, ns, q0, nb, b->st_i.as<int>(), b->st_w.as<double>(),
                                     out.as<const T>(), cells, S, s));
    GPF_HIP(hipStreamSynchronize(s));   // the descriptors are rewritten for the next batch
  }
  return GPF_OK;
}

}  // namespace
}  // namespace gpf

gpf_status gpf_body_schur_by_convolution(gpf_body *body, int fp64, int batch, double *h_rel_s,
                                         double *h_rel_f, double *h_ms) {
  if (!body || batch < 1 || batch > 1024)
    return fail(GPF_E_INVALID, "gpf_body_schur_by_convolution: bad arguments");
  gpf_plan *pl = body->plan;
  GPF_HIP(hipSetDevice(pl->ctx->device));
  const int n = pl->grid.n, ns = body->ns;
  const size_t T = fp64 ? 8 : 4;
  if ((double)batch * ((double)n * n * 2 * T + (double)(n + 1) * n * 2 * T) > 16.0 * (1ull << 30))
    return fail(GPF_E_NOMEM, "gpf_body_schur_by_convolution: more than 16 GiB");
  if (fp64) {
    if (!pl->spec64.p) GPF_TRY(upload_spectrum<double>(pl, pl->spec64, pl->tw64));
  } else {
    if (!pl->spec32.p) GPF_TRY(upload_spectrum<float>(pl, pl->spec32, pl->tw32));
  }
  hipStream_t s = nullptr;
  const size_t mb = (size_t)ns * ns * sizeof(double);
  DevBuf Sc, Se, Sinv, R, F;
  GPF_TRY(Sc.alloc(mb));
  GPF_TRY(Se.alloc(mb));
  GPF_TRY(Sinv.alloc(mb));
  GPF_TRY(R.alloc(ns * sizeof(double)));
  GPF_TRY(F.alloc(2 * ns * sizeof(double)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  GPF_HIP(hipDeviceSynchronize());
  GPF_HIP(hipEventCreate(&e0));
  GPF_HIP(hipEventCreate(&e1));
  gpf_status st;
  {
    TimerScope none(nullptr);
    GPF_HIP(hipEventRecord(e0, s));
    st = fp64 ? schur_by_columns<double>(body, batch, Sc.as<double>(), s)
              : schur_by_columns<float>(body, batch, Sc.as<double>(), s);
    GPF_HIP(hipEventRecord(e1, s));
  }
  GPF_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  GPF_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  GPF_TRY(st);
  // the exact S, from the LGF table, and the two sheets of a unit uniform flow
  GPF_HIP(launch_schur_build(n, ns, body->st_i.as<int>(), body->st_w.as<double>(),
                             body->ds.as<double>(), pl->lgf.as<double>(), Se.as<double>(), s));
  std::vector<double> hc((size_t)ns * ns), he((size_t)ns * ns);
  GPF_HIP(hipMemcpy(hc.data(), Sc.p, mb, hipMemcpyDeviceToHost));
  GPF_HIP(hipMemcpy(he.data(), Se.p, mb, hipMemcpyDeviceToHost));
  double dn = 0.0, en = 0.0;
  for (size_t k = 0; k < hc.size(); ++k) {
    dn += (hc[k] - he[k]) * (hc[k] - he[k]);
    en += he[k] * he[k];
  }
  double min_piv = 0.0;
  GPF_TRY(invert_fp64(ns, Sc.as<double>(), Sinv.as<double>(), s, &min_piv));
  std::vector<double> r(ns);
  for (int p = 0; p < ns; ++p) r[p] = -body->hys[p];
  GPF_HIP(hipMemcpy(R.p, r.data(), ns * sizeof(double), hipMemcpyHostToDevice));
  GPF_HIP(launch_gemv(ns, 1, Sinv.as<double>(), R.as<double>(), F.as<double>(), s));
  GPF_HIP(launch_gemv(ns, 1, body->sinv.as<double>(), R.as<double>(), F.as<double>() + ns, s));
  std::vector<double> hf(2 * (size_t)ns);
  GPF_HIP(hipMemcpy(hf.data(), F.p, 2 * ns * sizeof(double), hipMemcpyDeviceToHost));
  double df = 0.0, fn = 0.0;
  for (int p = 0; p < ns; ++p) {
    df += (hf[p] - hf[ns + p]) * (hf[p] - hf[ns + p]);
    fn += hf[ns + p] * hf[ns + p];
  }
  if (h_rel_s) *h_rel_s = std::sqrt(dn / en);
  if (h_rel_f) *h_rel_f = min_piv > 1e-14 ? std::sqrt(df / fn) : INFINITY;
  if (h_ms) *h_ms = ms;
  return GPF_OK;
}
