// Internal declarations of the gpf library (host runtime + HIP kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gpf.h"

namespace gpf {

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
gpf_status fail(gpf_status st, const std::string &msg);

#define GPF_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::gpf::fail(GPF_E_DEVICE, std::string(#call ": ") +             \
                                           hipGetErrorString(e_));           \
  } while (0)

// ---------------------------------------------------------------------------
// host numerics (lgf_host.cpp)
// ---------------------------------------------------------------------------
// G(a, b) for 0 <= a, b <= nmax into table[a*(nmax+1)+b].
void lgf_table_host(int nmax, double *table);
// Real spectrum of the (2n)^2 even extension of the table, minus a constant
// c, restricted to 0 <= k1, k2 <= n: spec[k1*(n+1)+k2] (unscaled).  The
// constant c (mean of G over offsets <= n/2) is returned.
double lgf_spectrum_host(int n, const double *table, double *spec);

// ---------------------------------------------------------------------------
// device objects
// ---------------------------------------------------------------------------
// Per-kernel event timing (opt-in).  Launchers bracket their kernels with
// timer_begin/timer_end; the marks go to the timer installed for the
// current thread by the API entry point (none: no-op).
struct KernelTimer {
  struct Rec {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  hipEvent_t open_a = nullptr;
  int open_kind = -1;
  double total_ms[GPF_TK_COUNT] = {0};
  long long count[GPF_TK_COUNT] = {0};
  ~KernelTimer();
  void reset();
  gpf_status flush();
};
void timer_install(KernelTimer *t);
void timer_begin(int kind, hipStream_t s);
void timer_end(hipStream_t s);
struct TimerScope {
  explicit TimerScope(KernelTimer *t) { timer_install(t); }
  ~TimerScope() { timer_install(nullptr); }
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf();
  gpf_status alloc(size_t nbytes);
  template <class T> T *as() const { return static_cast<T *>(p); }
};

}  // namespace gpf

struct gpf_ctx {
  int device = 0;
  int num_cu = 0;
  int xcds = 8;
};

struct gpf_plan {
  gpf_ctx *ctx = nullptr;
  gpf_grid grid{};
  unsigned flags = 0;
  bool fp64 = false;          // field type double
  double gauge_c = 0.0;       // spectrum shift restored as -c * gamma_src
  // resident constants
  gpf::DevBuf lgf;            // (n+1)^2 double LGF table (Schur build, new vortices)
  gpf::DevBuf spec32, spec64; // (n+1)^2 scaled, centred spectrum
  gpf::DevBuf tw32, tw64;     // 2n twiddles exp(-2 pi i k / 2n)
  // workspaces
  gpf::DevBuf w32, w64;       // n*n source fields
  gpf::DevBuf x32, x64;       // (n+1)*n complex intermediate, k-major
  gpf::DevBuf s64;            // n*n FP64 field (first convolution in FP64)
  gpf::DevBuf sc;             // device scalars (double) and counters
  gpf::DevBuf part;           // block partial sums (double)
  gpf::DevBuf rhs, y;         // ns x (1+m) Schur right-hand sides and results
  gpf::DevBuf fbuf;           // ns sheet strength scratch
  gpf::DevBuf fwork;          // ns ftilde scratch
  gpf::DevBuf status_scratch; // used when building blocks get no status word
  int ns_cap = 0;
  std::vector<double> host_lgf;  // host copy of the table
  gpf::KernelTimer timer;
  bool timing = false;
  gpf_status ensure_fp64_conv();
  gpf_status ensure_schur_ws(int ns);
};

struct gpf_body {
  gpf_plan *plan = nullptr;
  int ns = 0;
  int nedge = 0;
  int edges[GPF_MAX_EDGES] = {0};
  double gamma0 = 0.0;
  double amp = 0.0;
  bool conv1_fp64 = false;
  std::vector<double> hx, hy, hds;
  gpf::DevBuf xs, ys, ds;     // surface geometry (double)
  gpf::DevBuf st_i, st_w;     // stencils: int2 base per point, 8 doubles weights
  gpf::DevBuf sinv;           // ns x ns S^-1, row-major, FP64
  gpf::DevBuf f0, fhat0;      // ns each
};

namespace gpf {

// ---------------------------------------------------------------------------
// kernel launchers (all asynchronous on `stream`)
// ---------------------------------------------------------------------------
struct GridGeom {
  int n;
  double dx, x0, y0;
};

// fields
hipError_t launch_fill(void *p, size_t bytes, hipStream_t s);
template <class T>
hipError_t launch_scatter_vortices(const GridGeom &g, int nv, const double *x,
                                   const double *y, const double *gam, T *w,
                                   double *partials, double *gamma_out,
                                   unsigned *counter, unsigned *status,
                                   hipStream_t s);
int scatter_vortex_blocks(int nv);

// convolution: s = conv(w) - c * (*gamma_src); Tin = type of w, T = compute/out type
template <class Tin, class T>
hipError_t launch_convolve(int n, const Tin *w, void *xwork, T *s, const T *spec,
                           const T *tw, double c, const double *gamma_src,
                           int xcds, hipStream_t st);

// surface stencils and gathers
hipError_t launch_surface_stencils(const GridGeom &g, int ns, const double *xs,
                                   const double *ys, int *st_i, double *st_w,
                                   unsigned *status, hipStream_t s);
template <class T>
hipError_t launch_interp_surface(int n, int ns, const int *st_i,
                                 const double *st_w, const T *field, double *r,
                                 hipStream_t s);

// Schur complement build and inversion (FP64)
hipError_t launch_schur_build(int n, int ns, const int *st_i, const double *st_w,
                              const double *ds, const double *lgf, double *S,
                              hipStream_t s);
gpf_status invert_fp64(int ns, double *A, double *Ainv, hipStream_t s, double *min_pivot_rel);
hipError_t launch_gemv(int ns, int ncol, const double *A, const double *X,
                       double *Y, hipStream_t s);

// per-solve surface right-hand sides: rhs[:,0] = s_b' - E_s s*,
// rhs[:,1+j] = E_s L^-1 d_j (direct LGF sums)
struct SolveScalars {
  double u_inf, v_inf, ub, vb, omega;
  double gamma_b, gamma_w_in;   // gamma_w_in NaN -> use device sum
  int mode, m;
  int edges[GPF_MAX_EDGES];
  double xnew[GPF_MAX_EDGES], ynew[GPF_MAX_EDGES];
};
template <class T>
hipError_t launch_surface_rhs(const GridGeom &g, int ns, const double *xs,
                              const double *ys, const int *st_i,
                              const double *st_w, const T *sstar,
                              const double *lgf, const SolveScalars &sv,
                              double *rhs, unsigned *status, hipStream_t s);
// constraint solve (one workgroup): writes f (ns), ftilde, scalars
hipError_t launch_constraints(int ns, const double *y, const double *f0,
                              const double *ds, double gamma0,
                              const double *xs, const double *ys,
                              const SolveScalars &sv, double *dev_scalars,
                              double *f, double *ftilde, unsigned *status,
                              hipStream_t s);
// w += R_s f + sum_j Gamma_j d_j
template <class T>
hipError_t launch_scatter_sheet(const GridGeom &g, int ns, const int *st_i,
                                const double *st_w, const double *ds,
                                const double *f, const SolveScalars &sv,
                                const double *dev_scalars, T *w, hipStream_t s);
template <class T>
hipError_t launch_vortex_velocity(const GridGeom &g, int nv, const double *x,
                                  const double *y, const T *s, double uinf,
                                  double vinf, double *u, double *v,
                                  unsigned *status, hipStream_t st);
hipError_t launch_copy_doubles(const double *dev_scalars, double *out, int count,
                               hipStream_t s);

// device scalar slots (doubles) inside plan->sc
enum ScalarSlot {
  SC_GAMMA_W = 0,     // circulation of the vortices (sum Gamma_q)
  SC_GAMMA_SRC2 = 1,  // source circulation of the final convolution
  SC_S0 = 2,
  SC_GAMMA_B = 3,
  SC_GAMMA_NEW = 4,   // .. 4 + GPF_MAX_EDGES
  SC_COUNT = 4 + GPF_MAX_EDGES,
  SC_COUNTER_OFFSET_BYTES = 256  // unsigned counter lives after the doubles
};

}  // namespace gpf
