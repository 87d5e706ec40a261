// Host runtime behind the C ABI (include/gpf.h): contexts, plans, bodies and
// the per-solve launch sequence.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>
#include <map>
#include <memory>
#include <mutex>

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

static thread_local KernelTimer *g_timer = nullptr;

void timer_install(KernelTimer *t) { g_timer = t; }

void timer_begin(int kind, hipStream_t s) {
  KernelTimer *t = g_timer;
  if (!t) return;
  if (t->pool.size() < 2) return;  // out of events: stop recording
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

GridGeom geom(const gpf_plan *p) {
  return GridGeom{p->grid.n, p->grid.dx, p->grid.x0, p->grid.y0};
}

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
  gpf_status st;
  if ((st = spec.alloc(hs.size() * sizeof(T))) != GPF_OK) return st;
  GPF_HIP(hipMemcpy(spec.p, hs.data(), hs.size() * sizeof(T), hipMemcpyHostToDevice));
  std::vector<T> ht(2 * (size_t)N);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < N; ++k) {
    ht[2 * k] = (T)std::cos(-2.0 * pi * k / N);
    ht[2 * k + 1] = (T)std::sin(-2.0 * pi * k / N);
  }
  if ((st = tw.alloc(ht.size() * sizeof(T))) != GPF_OK) return st;
  GPF_HIP(hipMemcpy(tw.p, ht.data(), ht.size() * sizeof(T), hipMemcpyHostToDevice));
  return GPF_OK;
}

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace
}  // namespace gpf

using namespace gpf;

gpf_status gpf_plan::ensure_fp64_conv() {
  const int n = grid.n;
  gpf_status st;
  if (!spec64.p && (st = upload_spectrum<double>(this, spec64, tw64)) != GPF_OK) return st;
  if ((st = w64.alloc((size_t)n * n * sizeof(double))) != GPF_OK) return st;
  if ((st = x64.alloc((size_t)(n + 1) * n * 2 * sizeof(double))) != GPF_OK) return st;
  if ((st = s64.alloc((size_t)n * n * sizeof(double))) != GPF_OK) return st;
  return GPF_OK;
}

gpf_status gpf_plan::ensure_schur_ws(int ns) {
  if (ns <= ns_cap) return GPF_OK;
  gpf_status st;
  const size_t cols = 1 + GPF_MAX_EDGES;
  if ((st = rhs.alloc(cols * ns * sizeof(double))) != GPF_OK) return st;
  if ((st = y.alloc(cols * ns * sizeof(double))) != GPF_OK) return st;
  if ((st = fbuf.alloc(ns * sizeof(double))) != GPF_OK) return st;
  if ((st = fwork.alloc(ns * sizeof(double))) != GPF_OK) return st;
  ns_cap = ns;
  return GPF_OK;
}

namespace gpf {
namespace {

template <class TP>
gpf_status solve_impl(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in,
                      const gpf_outputs *out, hipStream_t s, bool conv1_fp64) {
  const GridGeom g = geom(plan);
  const int n = g.n;
  const int x = plan->ctx->xcds;
  unsigned *status = out->d_status;
  double *sc = plan->sc.as<double>();
  unsigned *counter = reinterpret_cast<unsigned *>(plan->sc.as<char>() + SC_COUNTER_OFFSET_BYTES);
  TP *psi = static_cast<TP *>(out->d_psi);
  // the source field of both convolutions: FP64 when the first one runs in FP64
  const bool w_fp64 = conv1_fp64 || std::is_same<TP, double>::value;
  void *w = w_fp64 ? plan->w64.p : plan->w32.p;
  const size_t wbytes = (size_t)n * n * (w_fp64 ? 8 : 4);
  GPF_HIP(launch_fill(w, wbytes, s));
  if (w_fp64)
    GPF_HIP(launch_scatter_vortices<double>(g, in->nv, in->d_xv, in->d_yv, in->d_gv, (double *)w,
                                            plan->part.as<double>(), sc + SC_GAMMA_W, counter,
                                            status, s));
  else
    GPF_HIP(launch_scatter_vortices<float>(g, in->nv, in->d_xv, in->d_yv, in->d_gv, (float *)w,
                                           plan->part.as<double>(), sc + SC_GAMMA_W, counter,
                                           status, s));
  const TP *spec = std::is_same<TP, double>::value ? (const TP *)plan->spec64.p : (const TP *)plan->spec32.p;
  const TP *tw = std::is_same<TP, double>::value ? (const TP *)plan->tw64.p : (const TP *)plan->tw32.p;
  void *xw = std::is_same<TP, double>::value ? plan->x64.p : plan->x32.p;

  if (in->mode == GPF_NOBODY) {
    if (w_fp64 && std::is_same<TP, float>::value)
      GPF_HIP((launch_convolve<double, float>(n, (const double *)w, xw, (float *)psi,
                                              (const float *)spec, (const float *)tw,
                                              plan->gauge_c, sc + SC_GAMMA_W, x, s)));
    else
      GPF_HIP((launch_convolve<TP, TP>(n, (const TP *)w, xw, psi, spec, tw, plan->gauge_c,
                                       sc + SC_GAMMA_W, x, s)));
    if (out->d_u && out->d_v)
      GPF_HIP(launch_vortex_velocity<TP>(g, in->nv, in->d_xv, in->d_yv, psi, in->u_inf,
                                         in->v_inf, out->d_u, out->d_v, status, s));
    if (out->d_scalars) GPF_HIP(launch_copy_doubles(sc, out->d_scalars, SC_COUNT, s));
    return GPF_OK;
  }

  // first convolution: s* (only its surface values are used)
  const int ns = body->ns;
  SolveScalars sv{};
  sv.u_inf = in->u_inf;
  sv.v_inf = in->v_inf;
  sv.ub = in->ub;
  sv.vb = in->vb;
  sv.omega = in->omega;
  sv.gamma_b = in->gamma_b;
  sv.gamma_w_in = in->gamma_w;
  sv.mode = in->mode;
  sv.m = in->mode == GPF_KUTTA_SHED ? in->m : 0;
  for (int e = 0; e < body->nedge; ++e) sv.edges[e] = body->edges[e];
  for (int j = 0; j < sv.m; ++j) {
    sv.xnew[j] = in->h_xnew[j];
    sv.ynew[j] = in->h_ynew[j];
  }
  double *rhs = plan->rhs.as<double>();
  const auto surface_rhs_timed = [&](auto *sfield) -> gpf_status {
    timer_begin(GPF_TK_SURFACE, s);
    GPF_HIP(launch_surface_rhs(g, ns, body->xs.as<double>(), body->ys.as<double>(),
                               body->st_i.as<int>(), body->st_w.as<double>(), sfield,
                               plan->lgf.as<double>(), sv, rhs, status, s));
    return GPF_OK;
  };
  if (conv1_fp64) {
    double *sstar = plan->s64.as<double>();
    GPF_HIP((launch_convolve<double, double>(n, (const double *)w, plan->x64.p, sstar,
                                             plan->spec64.as<double>(), plan->tw64.as<double>(),
                                             plan->gauge_c, sc + SC_GAMMA_W, x, s)));
    gpf_status st = surface_rhs_timed(sstar);
    if (st != GPF_OK) return st;
  } else {
    // s* goes into the caller's psi buffer, overwritten by the final field
    GPF_HIP((launch_convolve<TP, TP>(n, (const TP *)w, xw, psi, spec, tw, plan->gauge_c,
                                     sc + SC_GAMMA_W, x, s)));
    gpf_status st = surface_rhs_timed(psi);
    if (st != GPF_OK) return st;
  }
  GPF_HIP(launch_gemv(ns, 1 + sv.m, body->sinv.as<double>(), rhs, plan->y.as<double>(), s));
  double *ft = out->d_ftilde ? out->d_ftilde : plan->fwork.as<double>();
  GPF_HIP(launch_constraints(ns, plan->y.as<double>(), body->f0.as<double>(), body->ds.as<double>(),
                             body->gamma0, body->xs.as<double>(), body->ys.as<double>(), sv, sc,
                             plan->fbuf.as<double>(), ft, status, s));
  if (w_fp64)
    GPF_HIP(launch_scatter_sheet<double>(g, ns, body->st_i.as<int>(), body->st_w.as<double>(),
                                         body->ds.as<double>(), plan->fbuf.as<double>(), sv, sc,
                                         (double *)w, s));
  else
    GPF_HIP(launch_scatter_sheet<float>(g, ns, body->st_i.as<int>(), body->st_w.as<double>(),
                                        body->ds.as<double>(), plan->fbuf.as<double>(), sv, sc,
                                        (float *)w, s));
  timer_end(s);
  // final convolution of all vorticity
  if (w_fp64 && std::is_same<TP, float>::value)
    GPF_HIP((launch_convolve<double, float>(n, (const double *)w, xw, (float *)psi,
                                            (const float *)spec, (const float *)tw, plan->gauge_c,
                                            sc + SC_GAMMA_SRC2, x, s)));
  else
    GPF_HIP((launch_convolve<TP, TP>(n, (const TP *)w, xw, psi, spec, tw, plan->gauge_c,
                                     sc + SC_GAMMA_SRC2, x, s)));
  if (out->d_u && out->d_v)
    GPF_HIP(launch_vortex_velocity<TP>(g, in->nv, in->d_xv, in->d_yv, psi, in->u_inf, in->v_inf,
                                       out->d_u, out->d_v, status, s));
  if (out->d_f) GPF_HIP(launch_copy_doubles(plan->fbuf.as<double>(), out->d_f, ns, s));
  if (out->d_scalars) GPF_HIP(launch_copy_doubles(sc, out->d_scalars, SC_COUNT, s));
  return GPF_OK;
}

}  // namespace
}  // namespace gpf

extern "C" {

const char *gpf_last_error(void) { return g_last_error.c_str(); }
const char *gpf_version(void) { return "gpf 0.1 (gfx950)"; }

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
  auto *c = new gpf_ctx;
  c->device = device;
  hipDeviceProp_t prop;
  GPF_HIP(hipGetDeviceProperties(&prop, device));
  c->num_cu = prop.multiProcessorCount;
  c->xcds = xcd_count(device);
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
  if (flags & ~(GPF_FP64 | GPF_CONV1_FP64 | GPF_POLICY_AUTO))
    return fail(GPF_E_INVALID, "gpf_plan_create: unknown flag");
  GPF_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<gpf_plan> p(new gpf_plan);
  p->ctx = ctx;
  p->grid = *grid;
  p->flags = flags;
  p->fp64 = (flags & GPF_FP64) != 0;
  gpf_status st;
  auto tab = get_table(n);
  p->host_lgf = *tab;
  if ((st = p->lgf.alloc(tab->size() * sizeof(double))) != GPF_OK) return st;
  GPF_HIP(hipMemcpy(p->lgf.p, tab->data(), tab->size() * sizeof(double), hipMemcpyHostToDevice));
  if (p->fp64) {
    if ((st = p->ensure_fp64_conv()) != GPF_OK) return st;
  } else {
    if ((st = upload_spectrum<float>(p.get(), p->spec32, p->tw32)) != GPF_OK) return st;
    if ((st = p->w32.alloc((size_t)n * n * sizeof(float))) != GPF_OK) return st;
    if ((st = p->x32.alloc((size_t)(n + 1) * n * 2 * sizeof(float))) != GPF_OK) return st;
    if (flags & GPF_CONV1_FP64)
      if ((st = p->ensure_fp64_conv()) != GPF_OK) return st;
  }
  if ((st = p->sc.alloc(512)) != GPF_OK) return st;
  GPF_HIP(hipMemset(p->sc.p, 0, 512));
  if ((st = p->part.alloc(sizeof(double) * (size_t)scatter_vortex_blocks(1 << 22))) != GPF_OK)
    return st;
  if ((st = p->status_scratch.alloc(256)) != GPF_OK) return st;
  GPF_HIP(hipMemset(p->status_scratch.p, 0, 256));
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
  for (int e = 0; e < nedge; ++e) b->edges[e] = h_edges[e];
  b->hx.assign(h_xs, h_xs + ns);
  b->hy.assign(h_ys, h_ys + ns);
  b->hds.assign(h_ds, h_ds + ns);
  gpf_status st;
  const size_t vb = ns * sizeof(double);
  if ((st = b->xs.alloc(vb)) || (st = b->ys.alloc(vb)) || (st = b->ds.alloc(vb)) ||
      (st = b->st_i.alloc(2 * ns * sizeof(int))) || (st = b->st_w.alloc(8 * vb)) ||
      (st = b->sinv.alloc((size_t)ns * vb)) || (st = b->f0.alloc(vb)) || (st = b->fhat0.alloc(vb)))
    return st;
  if ((st = plan->ensure_schur_ws(ns)) != GPF_OK) return st;
  GPF_HIP(hipMemcpy(b->xs.p, h_xs, vb, hipMemcpyHostToDevice));
  GPF_HIP(hipMemcpy(b->ys.p, h_ys, vb, hipMemcpyHostToDevice));
  GPF_HIP(hipMemcpy(b->ds.p, h_ds, vb, hipMemcpyHostToDevice));
  hipStream_t s = nullptr;
  unsigned *status = plan->status_scratch.as<unsigned>();
  GPF_HIP(launch_surface_stencils(geom(plan), ns, b->xs.as<double>(), b->ys.as<double>(),
                                  b->st_i.as<int>(), b->st_w.as<double>(), status, s));
  DevBuf S;
  if ((st = S.alloc((size_t)ns * vb)) != GPF_OK) return st;
  GPF_HIP(launch_schur_build(g.n, ns, b->st_i.as<int>(), b->st_w.as<double>(), b->ds.as<double>(),
                             plan->lgf.as<double>(), S.as<double>(), s));
  double min_piv = 0.0;
  if ((st = invert_fp64(ns, S.as<double>(), b->sinv.as<double>(), s, &min_piv)) != GPF_OK) return st;
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
  if ((st = dX.alloc(3 * vb)) || (st = dY.alloc(3 * vb))) return st;
  GPF_HIP(hipMemcpy(dX.p, X.data(), 3 * vb, hipMemcpyHostToDevice));
  GPF_HIP(launch_gemv(ns, 3, b->sinv.as<double>(), dX.as<double>(), dY.as<double>(), s));
  std::vector<double> Y(3 * (size_t)ns);
  GPF_HIP(hipMemcpy(Y.data(), dY.p, 3 * vb, hipMemcpyDeviceToHost));
  unsigned hstatus = 0;
  GPF_HIP(hipMemcpy(&hstatus, status, sizeof(unsigned), hipMemcpyDeviceToHost));
  GPF_HIP(hipMemset(status, 0, sizeof(unsigned)));
  if (hstatus & GPF_DEV_OUT_OF_GRID) return fail(GPF_E_OUT_OF_GRID, "gpf_body_create: stencil outside grid");
  double g0 = 0.0, nr = 0.0, nf = 0.0, nrhs = 0.0, npert = 0.0;
  std::vector<double> fh(ns);
  for (int p = 0; p < ns; ++p) {
    g0 += h_ds[p] * Y[p];
    fh[p] = h_ds[p] * Y[p];
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
  b->amp = (nr > 0.0 && npert > 0.0) ? std::sqrt(nf / nr) / std::sqrt(npert / nrhs) : INFINITY;
  const bool fp32_plan = !plan->fp64;
  b->conv1_fp64 = fp32_plan && ((plan->flags & GPF_CONV1_FP64) ||
                                ((plan->flags & GPF_POLICY_AUTO) && b->amp > GPF_AMP_THRESHOLD));
  if (b->conv1_fp64)
    if ((st = plan->ensure_fp64_conv()) != GPF_OK) return st;
  GPF_HIP(hipMemcpy(b->f0.p, Y.data(), vb, hipMemcpyHostToDevice));
  GPF_HIP(hipMemcpy(b->fhat0.p, fh.data(), vb, hipMemcpyHostToDevice));
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

// ---------------------------------------------------------------------------
// building blocks
// ---------------------------------------------------------------------------

gpf_status gpf_regularize_vortices(gpf_plan *plan, int nv, const double *d_xv, const double *d_yv,
                                   const double *d_gv, void *d_w, int accumulate,
                                   unsigned int *d_status, void *hip_stream) {
  if (!plan || !d_w || nv < 0 || (nv > 0 && (!d_xv || !d_yv || !d_gv)))
    return fail(GPF_E_INVALID, "gpf_regularize_vortices: bad arguments");
  if (nv > (1 << 22)) return fail(GPF_E_UNSUPPORTED, "gpf_regularize_vortices: nv above 2^22");
  hipStream_t s = as_stream(hip_stream);
  const int n = plan->grid.n;
  const size_t bytes = (size_t)n * n * (plan->fp64 ? 8 : 4);
  if (!accumulate) GPF_HIP(launch_fill(d_w, bytes, s));
  unsigned *status = d_status ? d_status : plan->status_scratch.as<unsigned>();
  double *sc = plan->sc.as<double>();
  unsigned *counter = reinterpret_cast<unsigned *>(plan->sc.as<char>() + SC_COUNTER_OFFSET_BYTES);
  if (plan->fp64)
    GPF_HIP(launch_scatter_vortices<double>(geom(plan), nv, d_xv, d_yv, d_gv, (double *)d_w,
                                            plan->part.as<double>(), sc + SC_GAMMA_W, counter,
                                            status, s));
  else
    GPF_HIP(launch_scatter_vortices<float>(geom(plan), nv, d_xv, d_yv, d_gv, (float *)d_w,
                                           plan->part.as<double>(), sc + SC_GAMMA_W, counter,
                                           status, s));
  return GPF_OK;
}

gpf_status gpf_convolve(gpf_plan *plan, const void *d_w, void *d_s, double gamma_src,
                        void *hip_stream) {
  if (!plan || !d_w || !d_s || !is_finite(gamma_src))
    return fail(GPF_E_INVALID, "gpf_convolve: bad arguments");
  hipStream_t s = as_stream(hip_stream);
  TimerScope scope(plan->timing ? &plan->timer : nullptr);
  // the gauge term is read from device memory by the last pass
  double *slot = plan->sc.as<double>() + SC_COUNT;  // scratch slot after the named ones
  GPF_HIP(hipMemcpyAsync(slot, &gamma_src, sizeof(double), hipMemcpyHostToDevice, s));
  const int n = plan->grid.n;
  const int x = plan->ctx->xcds;
  if (plan->fp64)
    GPF_HIP((launch_convolve<double, double>(n, (const double *)d_w, plan->x64.p, (double *)d_s,
                                             plan->spec64.as<double>(), plan->tw64.as<double>(),
                                             plan->gauge_c, slot, x, s)));
  else
    GPF_HIP((launch_convolve<float, float>(n, (const float *)d_w, plan->x32.p, (float *)d_s,
                                           plan->spec32.as<float>(), plan->tw32.as<float>(),
                                           plan->gauge_c, slot, x, s)));
  // the host value must stay alive until the copy has been issued
  GPF_HIP(hipStreamSynchronize(s));
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
  hipStream_t s = as_stream(hip_stream);
  unsigned *status = d_status ? d_status : plan->status_scratch.as<unsigned>();
  if (plan->fp64)
    GPF_HIP(launch_vortex_velocity<double>(geom(plan), nv, d_xv, d_yv, (const double *)d_s, u_inf,
                                           v_inf, d_u, d_v, status, s));
  else
    GPF_HIP(launch_vortex_velocity<float>(geom(plan), nv, d_xv, d_yv, (const float *)d_s, u_inf,
                                          v_inf, d_u, d_v, status, s));
  return GPF_OK;
}

// ---------------------------------------------------------------------------
// full solve
// ---------------------------------------------------------------------------


gpf_status gpf_solve(gpf_plan *plan, const gpf_body *body, const gpf_inputs *in,
                     const gpf_outputs *out, void *hip_stream) {
  if (!plan || !in || !out) return fail(GPF_E_INVALID, "gpf_solve: null argument");
  if (!out->d_psi || !out->d_status) return fail(GPF_E_INVALID, "gpf_solve: d_psi and d_status are required");
  if (in->nv < 0 || in->nv > (1 << 22)) return fail(GPF_E_UNSUPPORTED, "gpf_solve: nv must be in [0, 2^22]");
  if (in->nv > 0 && (!in->d_xv || !in->d_yv || !in->d_gv))
    return fail(GPF_E_INVALID, "gpf_solve: null vortex arrays");
  if (!is_finite(in->u_inf) || !is_finite(in->v_inf) || !is_finite(in->ub) || !is_finite(in->vb) ||
      !is_finite(in->omega))
    return fail(GPF_E_INVALID, "gpf_solve: non-finite freestream or body motion");
  if (in->mode < GPF_NOBODY || in->mode > GPF_KUTTA_SHED)
    return fail(GPF_E_INVALID, "gpf_solve: unknown mode");
  if (in->mode != GPF_NOBODY) {
    if (!body) return fail(GPF_E_INVALID, "gpf_solve: this mode needs a body");
    if (body->plan != plan) return fail(GPF_E_INVALID, "gpf_solve: body belongs to another plan");
  }
  if (in->mode == GPF_CIRCULATION && !is_finite(in->gamma_b))
    return fail(GPF_E_INVALID, "gpf_solve: non-finite gamma_b");
  if (in->mode == GPF_KUTTA_STEADY && body->nedge < 1)
    return fail(GPF_E_INVALID, "gpf_solve: steady Kutta needs a body with an edge");
  if (in->mode == GPF_KUTTA_SHED) {
    if (in->m < 1 || in->m != body->nedge)
      return fail(GPF_E_INVALID, "gpf_solve: shedding needs one new vortex per body edge");
    for (int j = 0; j < in->m; ++j)
      if (!is_finite(in->h_xnew[j]) || !is_finite(in->h_ynew[j]))
        return fail(GPF_E_INVALID, "gpf_solve: non-finite new vortex position");
    if (!std::isnan(in->gamma_w) && !is_finite(in->gamma_w))
      return fail(GPF_E_INVALID, "gpf_solve: gamma_w must be finite or NaN");
  }
  hipError_t e = hipSetDevice(plan->ctx->device);
  if (e != hipSuccess) return fail(GPF_E_DEVICE, hipGetErrorString(e));
  hipStream_t s = as_stream(hip_stream);
  TimerScope scope(plan->timing ? &plan->timer : nullptr);
  const bool conv1_fp64 = body && body->conv1_fp64 && in->mode != GPF_NOBODY;
  if (plan->fp64) return solve_impl<double>(plan, body, in, out, s, false);
  return solve_impl<float>(plan, body, in, out, s, conv1_fp64);
}

gpf_status gpf_timing_enable(gpf_plan *plan, int enable) {
  if (!plan) return fail(GPF_E_INVALID, "gpf_timing_enable: null plan");
  if (enable) plan->timer.reset();
  plan->timing = enable != 0;
  return GPF_OK;
}

gpf_status gpf_timing_read(gpf_plan *plan, int kind, long long *count, double *total_ms) {
  if (!plan || kind < 0 || kind >= GPF_TK_COUNT || !count || !total_ms)
    return fail(GPF_E_INVALID, "gpf_timing_read: bad arguments");
  gpf_status st = plan->timer.flush();
  if (st != GPF_OK) return st;
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
