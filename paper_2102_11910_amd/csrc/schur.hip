// Schur complement of the immersed-surface saddle system and the constraint
// solves (Sec. 2.2-2.4, appendix A), all in FP64.
//
// * S = -E_s L^-1 R_s (Sec. 2.2.2) built exactly from the LGF table:
//     S_pq = -dS_q sum_{a in st(p)} sum_{b in st(q)} e_pa e_qb G(a - b)
//   (dx^2 of L^-1 cancels dx^-2 of R_s).  S is indefinite, so it is
//   inverted by Gauss-Jordan elimination with partial pivoting.
// * Per solve, with y0 = S^-1 (s_b' - E_s s*) and y_j = S^-1 E_s L^-1 d_j:
//   prescribed circulation (eq. circsystem, circs0):
//       s0 = (<1, y0> - Gamma_b)/Gamma0, f = y0 - s0 f0
//   steady Kutta at edge k (eq. kuttasystem, intermedsoln, s0):
//       f~* = y0/f0 - c1 (c1 = fhat0.s_b'/Gamma0 from P^Gamma, using S^-1 1 = f0),
//       s0 = f~*_k, f~ = f~* - s0
//   Kutta at m edges with new vortices (eq. kuttasystem2/3, twovortex):
//       sum_j (1 + fhat0.P_{k_i} f~_j) Gamma_j = -(Gamma_w + fhat0.P_{k_i} f~*),
//       x = f~* + sum Gamma_j f~_j, s0 = mean_i x_{k_i}, f~ = x - s0
#include "gpf_internal.h"

namespace gpf {
namespace {

__device__ __forceinline__ double m4p(double r) {
  r = fabs(r);
  if (r <= 1.0) return 1.0 - 2.5 * r * r + 1.5 * r * r * r;
  if (r <= 2.0) return 0.5 * (2.0 - r) * (2.0 - r) * (1.0 - r);
  return 0.0;
}

// S[p][q], one thread per entry
__global__ __launch_bounds__(256) void k_schur_build(int n, int ns, const int *__restrict__ st_i,
                                                     const double *__restrict__ st_w,
                                                     const double *__restrict__ ds,
                                                     const double *__restrict__ lgf,
                                                     double *__restrict__ S) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (q >= ns) return;
  const int w = n + 1;
  const int ip = st_i[2 * p], jp = st_i[2 * p + 1];
  const int iq = st_i[2 * q], jq = st_i[2 * q + 1];
  double acc = 0.0;
  for (int b = 0; b < 4; ++b) {
    for (int d = 0; d < 4; ++d) {
      const int dj = abs(jp + b - jq - d);
      const double wyy = st_w[8 * p + 4 + b] * st_w[8 * q + 4 + d];
      double racc = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int di = abs(ip + a - iq - c);
          racc += st_w[8 * p + a] * st_w[8 * q + c] * lgf[(size_t)di * w + dj];
        }
      }
      acc += wyy * racc;
    }
  }
  S[(size_t)p * ns + q] = -ds[q] * acc;
}

// Gauss-Jordan step k on the augmented matrix M = [A | B] (ns x 2ns):
// pivot search, row swap, pivot-row scaling, and column capture.
__global__ __launch_bounds__(256) void k_gj_pivot(int ns, int k, double *__restrict__ M,
                                                  double *__restrict__ col,
                                                  double *__restrict__ piv_log) {
  __shared__ double best[256];
  __shared__ int bidx[256];
  const int tid = threadIdx.x, ld = 2 * ns;
  double bv = -1.0;
  int bi = k;
  for (int i = k + tid; i < ns; i += 256) {
    const double a = fabs(M[(size_t)i * ld + k]);
    if (a > bv) { bv = a; bi = i; }
  }
  best[tid] = bv;
  bidx[tid] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      if (best[tid + s] > best[tid] || (best[tid + s] == best[tid] && bidx[tid + s] < bidx[tid])) {
        best[tid] = best[tid + s];
        bidx[tid] = bidx[tid + s];
      }
    }
    __syncthreads();
  }
  const int pr = bidx[0];
  if (pr != k) {
    for (int j = tid; j < ld; j += 256) {
      const double t = M[(size_t)k * ld + j];
      M[(size_t)k * ld + j] = M[(size_t)pr * ld + j];
      M[(size_t)pr * ld + j] = t;
    }
  }
  __syncthreads();
  const double pv = M[(size_t)k * ld + k];
  if (tid == 0) piv_log[k] = pv;
  const double inv = pv != 0.0 ? 1.0 / pv : 0.0;
  __syncthreads();
  for (int j = tid; j < ld; j += 256) M[(size_t)k * ld + j] *= inv;
  for (int i = tid; i < ns; i += 256) col[i] = (i == k) ? 0.0 : M[(size_t)i * ld + k];
}

__global__ __launch_bounds__(256) void k_gj_eliminate(int ns, int k, double *__restrict__ M,
                                                      const double *__restrict__ col) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  const int ld = 2 * ns;
  if (j >= ld || i == k) return;
  const double c = col[i];
  if (c != 0.0) M[(size_t)i * ld + j] -= c * M[(size_t)k * ld + j];
}

__global__ void k_gj_init(int ns, const double *__restrict__ A, double *__restrict__ M) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  const int ld = 2 * ns;
  if (j >= ld) return;
  M[(size_t)i * ld + j] = j < ns ? A[(size_t)i * ns + j] : (j - ns == i ? 1.0 : 0.0);
}

__global__ void k_gj_extract(int ns, const double *__restrict__ M, double *__restrict__ Ainv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= ns) return;
  Ainv[(size_t)i * ns + j] = M[(size_t)i * 2 * ns + ns + j];
}

// Y[:, c] = A X[:, c] for c < ncol; X, Y column-major (ns x ncol); one wave per row
__global__ __launch_bounds__(256) void k_gemv(int ns, int ncol, const double *__restrict__ A,
                                              const double *__restrict__ X,
                                              double *__restrict__ Y) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= ns) return;
  double acc[1 + GPF_MAX_EDGES];
#pragma unroll
  for (int c = 0; c < 1 + GPF_MAX_EDGES; ++c) acc[c] = 0.0;
  const double *a = A + (size_t)row * ns;
  for (int q = lane; q < ns; q += 64) {
    const double aq = a[q];
#pragma unroll
    for (int c = 0; c < 1 + GPF_MAX_EDGES; ++c)
      if (c < ncol) acc[c] += aq * X[(size_t)c * ns + q];
  }
#pragma unroll
  for (int c = 0; c < 1 + GPF_MAX_EDGES; ++c) {
    if (c < ncol) {
      double v = acc[c];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) Y[(size_t)c * ns + row] = v;
    }
  }
}

// rhs[:,0] = s_b' - E_s s*;  rhs[:,1+j] = (E_s L^-1 d_j) by direct LGF sums.
// Blocks [0, nbe) give one thread per surface point for the first column;
// the remaining blocks give 16 lanes per (point, new vortex) pair, one lane
// per node of the surface stencil, each summing the 16 nodes of the vortex
// stencil.
constexpr int kRB = 256;

template <class T>
__global__ __launch_bounds__(kRB) void k_surface_rhs(const ProbDesc *__restrict__ d, int nbe) {
  const ProbDesc &P = d[blockIdx.y];
  const int ns = P.ns, n = P.n;
  const SolveScalars &sv = P.sv;
  if ((int)blockIdx.x < nbe) {
    const int p = blockIdx.x * kRB + threadIdx.x;
    if (p >= ns) return;
    const int i0 = P.st_i[2 * p], j0 = P.st_i[2 * p + 1];
    const double *ew = P.st_w + 8 * p;
    const T *s1 = static_cast<const T *>(P.s1);
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double r = 0.0;
#pragma unroll
      for (int a = 0; a < 4; ++a) r += ew[a] * (double)s1[(size_t)(j0 + b) * n + i0 + a];
      acc += ew[4 + b] * r;
    }
    const double x = P.xs[p], y = P.ys[p];
    const double sb = (sv.ub - sv.u_inf) * y - (sv.vb - sv.v_inf) * x -
                      0.5 * sv.omega * (x * x + y * y);
    P.rhs[p] = sb - acc;
    return;
  }
  if (sv.mode != GPF_KUTTA_SHED) return;
  const int m = sv.m;
  const int pj = ((int)blockIdx.x - nbe) * (kRB / 16) + (int)threadIdx.x / 16;
  const int lane = threadIdx.x & 15;
  const bool active = pj < ns * m;
  double val = 0.0;
  int p = 0, j = 0;
  if (active) {
    p = pj % ns;
    j = pj / ns;
    const double xi = (sv.xnew[j] - P.x0) / P.dx, eta = (sv.ynew[j] - P.y0) / P.dx;
    if (xi >= 2.0 && xi < n - 3.0 && eta >= 2.0 && eta < n - 3.0) {
      const int vi = (int)floor(xi) - 1, vj = (int)floor(eta) - 1;
      const double fx = xi - floor(xi), fy = eta - floor(eta);
      const int a = lane & 3, b = lane >> 2;
      const int ia = P.st_i[2 * p] + a, jb = P.st_i[2 * p + 1] + b;
      const int w = n + 1;
      double r = 0.0;
#pragma unroll
      for (int dd = 0; dd < 4; ++dd) {
        const int dj = abs(jb - vj - dd);
        double rr = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) rr += m4p(fx + 1.0 - c) * P.lgf[(size_t)abs(ia - vi - c) * w + dj];
        r += m4p(fy + 1.0 - dd) * rr;
      }
      val = P.st_w[8 * p + a] * P.st_w[8 * p + 4 + b] * r;
    } else if (lane == 0 && p == 0) {
      atomicOr(P.status, GPF_DEV_OUT_OF_GRID);
    }
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) val += __shfl_xor(val, off);
  if (active && lane == 0) P.rhs[(size_t)(1 + j) * ns + p] = val;
}

constexpr int kCB = 256;

// sum over the workgroup (kCB = 4 waves): wave shuffles, then the four
// wave totals through LDS; every thread gets the result
__device__ double block_sum(double v, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int wave = threadIdx.x >> 6;
  __syncthreads();  // red[] may still be read by the previous call
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Constraint solve of one problem by one workgroup: reads Y = S^-1 rhs,
// writes f, f~ and the scalar slots.
struct ConstraintScratch {
  double red[kCB];
  double gam[GPF_MAX_EDGES];
  double dj[GPF_MAX_EDGES];
  double A[GPF_MAX_EDGES][GPF_MAX_EDGES + 1];
  double s0;
};

__device__ void constraints_block(const ProbDesc &P, const double *__restrict__ Y,
                                  const double *__restrict__ f0, const double *__restrict__ ds,
                                  ConstraintScratch &cs) {
  double *red = cs.red;
  double *gam = cs.gam;
  double *dj = cs.dj;
  const int tid = threadIdx.x;
  const int ns = P.ns;
  const SolveScalars &sv = P.sv;
  double *__restrict__ f = P.f;
  double *__restrict__ ft = P.ft;
  double *sc = P.aux;
  const double gamma0 = P.gamma0;
  const double gamma_w_dev = sc[SC_GAMMA_W];
  const int m = sv.mode == GPF_KUTTA_SHED ? sv.m : 0;

  if (sv.mode == GPF_CIRCULATION) {
    double part = 0.0;
    for (int p = tid; p < ns; p += kCB) part += ds[p] * Y[p];
    const double circ = block_sum(part, red);
    const double s0 = (circ - sv.gamma_b) / gamma0;
    double pb = 0.0;
    for (int p = tid; p < ns; p += kCB) {
      const double fp = Y[p] - s0 * f0[p];
      f[p] = fp;
      ft[p] = fp / f0[p];
      pb += ds[p] * fp;
    }
    const double gb = block_sum(pb, red);
    if (tid == 0) {
      sc[SC_S0] = s0;
      sc[SC_GAMMA_B] = gb;
      sc[SC_GAMMA_SRC2] = gamma_w_dev + gb;
    }
    return;
  }

  // Kutta modes: c1 = fhat0 . s_b' / Gamma0 (circulation removal of the rhs)
  double part = 0.0;
  for (int p = tid; p < ns; p += kCB) {
    const double x = P.xs[p], y = P.ys[p];
    const double sb = (sv.ub - sv.u_inf) * y - (sv.vb - sv.v_inf) * x -
                      0.5 * sv.omega * (x * x + y * y);
    part += ds[p] * f0[p] * sb;
  }
  const double c1 = block_sum(part, red) / gamma0;
  // ft <- f~* = y0/f0 - c1
  for (int p = tid; p < ns; p += kCB) ft[p] = Y[p] / f0[p] - c1;
  __syncthreads();

  if (sv.mode == GPF_KUTTA_STEADY) {
    const double s0 = ft[sv.edges[0]];
    __syncthreads();  // every thread has read f~*_k before any thread shifts it
    double pb = 0.0;
    for (int p = tid; p < ns; p += kCB) {
      const double t = ft[p] - s0;
      ft[p] = t;
      const double fp = f0[p] * t;
      f[p] = fp;
      pb += ds[p] * fp;
    }
    const double gb = block_sum(pb, red);
    if (tid == 0) {
      sc[SC_S0] = s0;
      sc[SC_GAMMA_B] = gb;
      sc[SC_GAMMA_SRC2] = gamma_w_dev + gb;
    }
    return;
  }

  // shedding at m edges
  const double gamma_w = isnan(sv.gamma_w_in) ? gamma_w_dev : sv.gamma_w_in;
  double dstar = 0.0;
  for (int p = tid; p < ns; p += kCB) dstar += ds[p] * f0[p] * ft[p];
  dstar = block_sum(dstar, red);
  for (int j = 0; j < m; ++j) {
    double pj = 0.0;
    for (int p = tid; p < ns; p += kCB) pj += ds[p] * Y[(size_t)(1 + j) * ns + p];
    const double v = block_sum(pj, red);   // fhat0 . f~_j = sum dS f0 (y_j / f0)
    if (tid == 0) dj[j] = v;
  }
  if (tid == 0) {
    auto &A = cs.A;
    for (int i = 0; i < m; ++i) {
      const int k = sv.edges[i];
      for (int j = 0; j < m; ++j)
        A[i][j] = 1.0 + dj[j] - gamma0 * Y[(size_t)(1 + j) * ns + k] / f0[k];
      A[i][m] = -(gamma_w + dstar - gamma0 * ft[k]);
    }
    bool singular = false;
    double amax = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) amax = fmax(amax, fabs(A[i][j]));
    for (int c = 0; c < m; ++c) {
      int pr = c;
      for (int i = c + 1; i < m; ++i)
        if (fabs(A[i][c]) > fabs(A[pr][c])) pr = i;
      if (!(fabs(A[pr][c]) > 1e-13 * amax)) { singular = true; break; }
      if (pr != c)
        for (int j = 0; j <= m; ++j) { double t = A[c][j]; A[c][j] = A[pr][j]; A[pr][j] = t; }
      for (int i = 0; i < m; ++i) {
        if (i == c) continue;
        const double fct = A[i][c] / A[c][c];
        for (int j = c; j <= m; ++j) A[i][j] -= fct * A[c][j];
      }
    }
    for (int j = 0; j < m; ++j) gam[j] = singular ? 0.0 : A[j][m] / A[j][j];
    if (singular) atomicOr(P.status, GPF_DEV_SINGULAR);
    // s0 = mean over edges of x_k, x = f~* + sum_j Gamma_j f~_j
    double s0 = 0.0;
    for (int i = 0; i < m; ++i) {
      const int k = sv.edges[i];
      double xk = ft[k];
      for (int j = 0; j < m; ++j) xk += gam[j] * Y[(size_t)(1 + j) * ns + k] / f0[k];
      s0 += xk;
    }
    cs.s0 = s0 / m;
  }
  __syncthreads();
  const double s0 = cs.s0;
  double pb = 0.0;
  for (int p = tid; p < ns; p += kCB) {
    double x = ft[p];
    for (int j = 0; j < m; ++j) x += gam[j] * Y[(size_t)(1 + j) * ns + p] / f0[p];
    const double t = x - s0;
    ft[p] = t;
    const double fp = f0[p] * t;
    f[p] = fp;
    pb += ds[p] * fp;
  }
  const double gb = block_sum(pb, red);
  if (tid == 0) {
    double gsum = 0.0;
    for (int j = 0; j < m; ++j) {
      sc[SC_GAMMA_NEW + j] = gam[j];
      gsum += gam[j];
    }
    sc[SC_S0] = s0;
    sc[SC_GAMMA_B] = gb;
    sc[SC_GAMMA_SRC2] = gamma_w_dev + gb + gsum;
  }
}

__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

// Y = S^-1 [rhs columns] (one wave per row); the last workgroup of each
// problem then solves the constraints, scatters R_s f and the new vortices
// into the source field and copies the outputs.
constexpr int kStageDoubles = 3072;

template <class T>
__global__ __launch_bounds__(kCB) void k_schur_apply(const ProbDesc *__restrict__ d) {
  __shared__ double stage[kStageDoubles];
  __shared__ ConstraintScratch cs;
  __shared__ bool last;
  double *gam = cs.gam;
  const ProbDesc &P = d[blockIdx.y];
  const int ns = P.ns;
  const int ncol = 1 + (P.sv.mode == GPF_KUTTA_SHED ? P.sv.m : 0);
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row < ns) {
    double acc[1 + GPF_MAX_EDGES];
#pragma unroll
    for (int c = 0; c < 1 + GPF_MAX_EDGES; ++c) acc[c] = 0.0;
    const double *a = P.sinv + (size_t)row * ns;
    for (int q = lane; q < ns; q += 64) {
      const double aq = a[q];
#pragma unroll
      for (int c = 0; c < 1 + GPF_MAX_EDGES; ++c)
        if (c < ncol) acc[c] += aq * P.rhs[(size_t)c * ns + q];
    }
#pragma unroll
    for (int c = 0; c < 1 + GPF_MAX_EDGES; ++c) {
      if (c < ncol) {
        double v = acc[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) P.y[(size_t)c * ns + row] = v;
      }
    }
  }
  __syncthreads();
  unsigned *counter = aux_counter(P.aux, 1);
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned done = atomicAdd(counter, 1u);
    last = (done == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  // the constraint phases read Y, f0 and dS several times: stage them in
  // LDS once when they fit (Y was just written by other workgroups)
  const double *Y = P.y, *f0 = P.f0, *ds = P.ds;
  if ((size_t)ns * (ncol + 2) <= kStageDoubles) {
    double *Ys = stage, *f0s = stage + (size_t)ncol * ns, *dss = f0s + ns;
    for (int k = threadIdx.x; k < ncol * ns; k += kCB) Ys[k] = P.y[k];
    for (int k = threadIdx.x; k < ns; k += kCB) {
      f0s[k] = P.f0[k];
      dss[k] = P.ds[k];
    }
    __syncthreads();
    Y = Ys;
    f0 = f0s;
    ds = dss;
  }
  constraints_block(P, Y, f0, ds, cs);
  __syncthreads();
  // R_s f and the new vortices into the source field
  T *w = static_cast<T *>(P.w);
  const int n = P.n;
  const double inv = 1.0 / (P.dx * P.dx);
  for (int p = threadIdx.x; p < ns; p += kCB) {
    const int i0 = P.st_i[2 * p], j0 = P.st_i[2 * p + 1];
    const double amp = P.ds[p] * P.f[p] * inv;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double ab = amp * P.st_w[8 * p + 4 + b];
      T *r = w + (size_t)(j0 + b) * n + i0;
#pragma unroll
      for (int a = 0; a < 4; ++a) atomic_add(r + a, (T)(ab * P.st_w[8 * p + a]));
    }
  }
  if (P.sv.mode == GPF_KUTTA_SHED && (int)threadIdx.x < P.sv.m) {
    const int j = threadIdx.x;
    const double xi = (P.sv.xnew[j] - P.x0) / P.dx, eta = (P.sv.ynew[j] - P.y0) / P.dx;
    if (xi >= 2.0 && xi < n - 3.0 && eta >= 2.0 && eta < n - 3.0) {
      const int i0 = (int)floor(xi) - 1, j0 = (int)floor(eta) - 1;
      const double fx = xi - floor(xi), fy = eta - floor(eta);
      const double amp = gam[j] * inv;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double ab = amp * m4p(fy + 1.0 - b);
        T *r = w + (size_t)(j0 + b) * n + i0;
#pragma unroll
        for (int a = 0; a < 4; ++a) atomic_add(r + a, (T)(ab * m4p(fx + 1.0 - a)));
      }
    }
  }
  // outputs
  for (int p = threadIdx.x; p < ns; p += kCB) {
    if (P.f_out) P.f_out[p] = P.f[p];
    if (P.ft_out) P.ft_out[p] = P.ft[p];
  }
  __syncthreads();
  if (P.sc_out && (int)threadIdx.x < SC_COUNT) P.sc_out[threadIdx.x] = P.aux[threadIdx.x];
  if (threadIdx.x == 0) atomicExch(counter, 0u);
}

}  // namespace

hipError_t launch_schur_build(int n, int ns, const int *st_i, const double *st_w,
                              const double *ds, const double *lgf, double *S, hipStream_t s) {
  hipLaunchKernelGGL(k_schur_build, dim3((ns + 255) / 256, ns), dim3(256), 0, s, n, ns, st_i, st_w,
                     ds, lgf, S);
  return hipGetLastError();
}

gpf_status invert_fp64(int ns, double *A, double *Ainv, hipStream_t s, double *min_pivot_rel) {
  DevBuf M, col, piv;
  gpf_status st;
  if ((st = M.alloc((size_t)ns * 2 * ns * sizeof(double))) != GPF_OK) return st;
  if ((st = col.alloc((size_t)ns * sizeof(double))) != GPF_OK) return st;
  if ((st = piv.alloc((size_t)ns * sizeof(double))) != GPF_OK) return st;
  const dim3 g2((2 * ns + 255) / 256, ns);
  hipLaunchKernelGGL(k_gj_init, g2, dim3(256), 0, s, ns, A, M.as<double>());
  for (int k = 0; k < ns; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, ns, k, M.as<double>(),
                       col.as<double>(), piv.as<double>());
    hipLaunchKernelGGL(k_gj_eliminate, g2, dim3(256), 0, s, ns, k, M.as<double>(),
                       col.as<double>());
  }
  const dim3 g1((ns + 255) / 256, ns);
  hipLaunchKernelGGL(k_gj_extract, g1, dim3(256), 0, s, ns, M.as<double>(), Ainv);
  GPF_HIP(hipGetLastError());
  std::vector<double> hp(ns), ha((size_t)ns * ns);
  GPF_HIP(hipMemcpyAsync(hp.data(), piv.p, ns * sizeof(double), hipMemcpyDeviceToHost, s));
  GPF_HIP(hipMemcpyAsync(ha.data(), A, (size_t)ns * ns * sizeof(double), hipMemcpyDeviceToHost, s));
  GPF_HIP(hipStreamSynchronize(s));
  double amax = 0.0, pmin = 1e300;
  for (double v : ha) amax = std::max(amax, std::fabs(v));
  for (double v : hp) pmin = std::min(pmin, std::fabs(v));
  *min_pivot_rel = amax > 0.0 ? pmin / amax : 0.0;
  return GPF_OK;
}

hipError_t launch_gemv(int ns, int ncol, const double *A, const double *X, double *Y,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_gemv, dim3((ns + 3) / 4), dim3(256), 0, s, ns, ncol, A, X, Y);
  return hipGetLastError();
}

template <class T>
hipError_t launch_surface_rhs(const ProbDesc *d, int nb, int ns_max, int m_max, hipStream_t s) {
  const int nbe = (ns_max + kRB - 1) / kRB;
  const int nbl = (ns_max * m_max + kRB / 16 - 1) / (kRB / 16);
  timer_begin(GPF_TK_SURFACE, s);
  hipLaunchKernelGGL((k_surface_rhs<T>), dim3(nbe + nbl, nb), dim3(kRB), 0, s, d, nbe);
  return hipGetLastError();
}
template hipError_t launch_surface_rhs<float>(const ProbDesc *, int, int, int, hipStream_t);
template hipError_t launch_surface_rhs<double>(const ProbDesc *, int, int, int, hipStream_t);

template <class T>
hipError_t launch_schur_apply(const ProbDesc *d, int nb, int ns_max, hipStream_t s) {
  hipLaunchKernelGGL((k_schur_apply<T>), dim3((ns_max + 3) / 4, nb), dim3(kCB), 0, s, d);
  timer_end(s);
  return hipGetLastError();
}
template hipError_t launch_schur_apply<float>(const ProbDesc *, int, int, hipStream_t);
template hipError_t launch_schur_apply<double>(const ProbDesc *, int, int, hipStream_t);

}  // namespace gpf
