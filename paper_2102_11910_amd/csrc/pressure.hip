// Pressure (Sec. 2.6.1): the potential jump dphi across the surface, the
// surface Bernoulli equation (eq. surfbernoulli) for the pressure jump, and
// the grid pressure on the cell centres (eq. pgrid).
//
// Staggered layout: psi and vorticity on the nodes (x_i, y_j); u on the
// x-faces (x_i, y_j + dx/2), v on the y-faces (x_i + dx/2, y_j), from the
// curl u = (psi[j+1][i] - psi[j][i])/dx, v = -(psi[j][i+1] - psi[j][i])/dx;
// pressure on the cell centres (x_i + dx/2, y_j + dx/2).  Face data reach
// the surface through the smoothed three-point function (E_f) and back
// through its transpose (R_f = dx^-2 E_f^T diag(dS)).
#include <cmath>

#include "gpf_internal.h"
#include "weights.h"

namespace gpf {
namespace {

// three-point weights of one point on the u-lattice and on the v-lattice
__device__ void face_weights(double x, double y, double x0, double y0, double dx, PresStencil &st) {
  const double xi = (x - x0) / dx, eta = (y - y0) / dx;
  const double eu = eta - 0.5, xv = xi - 0.5;
  st.iu = (int)floor(xi) - 1;
  st.ju = (int)floor(eu) - 1;
  st.iv = (int)floor(xv) - 1;
  st.jv = (int)floor(eta) - 1;
  for (int a = 0; a < 4; ++a) {
    st.wxu[a] = yang3(xi - (st.iu + a));
    st.wyu[a] = yang3(eu - (st.ju + a));
    st.wxv[a] = yang3(xv - (st.iv + a));
    st.wyv[a] = yang3(eta - (st.jv + a));
  }
}

__global__ void k_pres_stencils(int ns, const double *__restrict__ xs, const double *__restrict__ ys,
                                double x0, double y0, double dx, PresStencil *st) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  PresStencil s;
  face_weights(xs[p], ys[p], x0, y0, dx, s);
  st[p] = s;
}

// Node weights of the surface curl C_s psi = n . E_f curl psi as two
// separable stencils: U (4 x 5 nodes from (iu, ju)), V (5 x 4 from (iv, jv)).
//   U: nx/dx wxu[a] (wyu[b-1] - wyu[b]),  V: ny/dx (wxv[a] - wxv[a-1]) wyv[b]
__device__ __forceinline__ double dlo(const double *w, int k) {   // w[k-1] - w[k], w outside 0..3 = 0
  return (k >= 1 ? w[k - 1] : 0.0) - (k <= 3 ? w[k] : 0.0);
}

// sum over the 20 x 20 (or 20 x 16) node pairs of two separable stencils of
// G(|di|, |dj|), G the lattice Green's function table ((n+1)^2)
__device__ double pair_sum(const double *lgf, int w, int ia, int ja, const double *xa, int nxa,
                           const double *ya, int nya, int ib, int jb, const double *xb, int nxb,
                           const double *yb, int nyb) {
  double acc = 0.0;
  for (int b = 0; b < nya; ++b) {
    for (int d = 0; d < nyb; ++d) {
      const int dj = abs(ja + b - jb - d);
      double racc = 0.0;
      for (int a = 0; a < nxa; ++a)
        for (int c = 0; c < nxb; ++c) racc += xa[a] * xb[c] * lgf[(size_t)abs(ia + a - ib - c) * w + dj];
      acc += ya[b] * yb[d] * racc;
    }
  }
  return acc;
}

struct CsSep {   // the two separable stencils of C_s at one point
  int iu, ju, iv, jv;
  double ux[4], uy[5], vx[5], vy[4];
};

__device__ void cs_sep(const PresStencil &s, double nx, double ny, double dx, CsSep &c) {
  c.iu = s.iu;
  c.ju = s.ju;
  c.iv = s.iv;
  c.jv = s.jv;
  for (int a = 0; a < 4; ++a) c.ux[a] = nx / dx * s.wxu[a];
  for (int b = 0; b < 5; ++b) c.uy[b] = dlo(s.wyu, b);
  for (int a = 0; a < 5; ++a) c.vx[a] = -ny / dx * dlo(s.wxv, a);
  for (int b = 0; b < 4; ++b) c.vy[b] = s.wyv[b];
}

// M[p][q] = dS_q sum C_s(p) C_s(q) G,  K[p][q] = dS_q sum C_s(p) E_s(q) G
// (M = C_s L^-1 C_s^T, K = C_s L^-1 R_s; L^-1 = dx^2 G and the dx^2 of R
// cancel).  One thread per (p, q); M row-major, K column-major.
__global__ __launch_bounds__(256) void k_pres_build(int n, int ns, const PresStencil *__restrict__ st,
                                                    const double *__restrict__ pnx,
                                                    const double *__restrict__ pny,
                                                    const int *__restrict__ st_i,
                                                    const double *__restrict__ st_w,
                                                    const double *__restrict__ ds, double dx,
                                                    const double *__restrict__ lgf, double *M,
                                                    double *K) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (q >= ns) return;
  const int w = n + 1;
  CsSep cp, cq;
  cs_sep(st[p], pnx[p], pny[p], dx, cp);
  cs_sep(st[q], pnx[q], pny[q], dx, cq);
  double m = 0.0;
  m += pair_sum(lgf, w, cp.iu, cp.ju, cp.ux, 4, cp.uy, 5, cq.iu, cq.ju, cq.ux, 4, cq.uy, 5);
  m += pair_sum(lgf, w, cp.iu, cp.ju, cp.ux, 4, cp.uy, 5, cq.iv, cq.jv, cq.vx, 5, cq.vy, 4);
  m += pair_sum(lgf, w, cp.iv, cp.jv, cp.vx, 5, cp.vy, 4, cq.iu, cq.ju, cq.ux, 4, cq.uy, 5);
  m += pair_sum(lgf, w, cp.iv, cp.jv, cp.vx, 5, cp.vy, 4, cq.iv, cq.jv, cq.vx, 5, cq.vy, 4);
  const double *ex = st_w + 8 * q;
  double k = 0.0;
  k += pair_sum(lgf, w, cp.iu, cp.ju, cp.ux, 4, cp.uy, 5, st_i[2 * q], st_i[2 * q + 1], ex, 4, ex + 4, 4);
  k += pair_sum(lgf, w, cp.iv, cp.jv, cp.vx, 5, cp.vy, 4, st_i[2 * q], st_i[2 * q + 1], ex, 4, ex + 4, 4);
  M[(size_t)p * ns + q] = ds[q] * m;
  K[(size_t)q * ns + p] = ds[q] * k;
}

template <class T>
__device__ __forceinline__ double face_u(const T *psi, int n, int i, int j, double dx) {
  return ((double)psi[(size_t)(j + 1) * n + i] - (double)psi[(size_t)j * n + i]) / dx;
}
template <class T>
__device__ __forceinline__ double face_v(const T *psi, int n, int i, int j, double dx) {
  return -((double)psi[(size_t)j * n + i + 1] - (double)psi[(size_t)j * n + i]) / dx;
}

// surface velocity of point p (rigid motion of the body, or of its part)
__device__ __forceinline__ void surf_velocity(const PresDesc &D, int p, double x, double y,
                                              double &vx, double &vy) {
  double ub = D.ub, vb = D.vb, om = D.omega;
  if (D.part) {
    const int j = D.part[p];
    ub = D.pub[j];
    vb = D.pvb[j];
    om = D.pom[j];
  }
  vx = ub - om * y;
  vy = vb + om * x;
}

// One thread per surface point: dphi = Q f (Q column-major, so the threads
// of a wave read consecutive entries), d(dphi)/dt, E_f v and the pressure
// jump of the surface Bernoulli equation.
template <class T>
__global__ __launch_bounds__(256) void k_pres_surface(PresDesc D) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= D.ns) return;
  double acc = 0.0;
  for (int q = 0; q < D.ns; ++q) acc += D.Q[(size_t)q * D.ns + p] * D.f[q];
  const double dphi = acc;
  const double ddt = D.dphi_prev ? (dphi - D.dphi_prev[p]) / D.dt : 0.0;
  const PresStencil s = D.st[p];
  const T *psi = static_cast<const T *>(D.psi);
  const int n = D.n;
  double eu = 0.0, ev = 0.0;
  for (int b = 0; b < 4; ++b)
    for (int a = 0; a < 4; ++a) {
      eu += s.wxu[a] * s.wyu[b] * face_u(psi, n, s.iu + a, s.ju + b, D.dx);
      ev += s.wxv[a] * s.wyv[b] * face_v(psi, n, s.iv + a, s.jv + b, D.dx);
    }
  if (!D.psi_total) {
    eu += D.u_inf;
    ev += D.v_inf;
  }
  const double x = D.xs[p], y = D.ys[p];
  double vsx, vsy;
  surf_velocity(D, p, x, y, vsx, vsy);
  const double f = D.f[p], nx = D.pnx[p], ny = D.pny[p];
  // gamma x n = f (-n_y, n_x)
  const double dp = -D.rho * ((eu - vsx) * (-f * ny) + (ev - vsy) * (f * nx)) - D.rho * ddt;
  D.dphi[p] = dphi;
  D.dp[p] = dp;
  D.ddt[p] = ddt;
}

// R_s f onto the nodes and R_f (n d(dphi)/dt - v_s x gamma) onto the faces
// (16 lanes per point, one per stencil node; FP64 atomics)
__global__ __launch_bounds__(256) void k_pres_scatter(PresDesc D) {
  const int p = blockIdx.x * 16 + (threadIdx.x >> 4), k = threadIdx.x & 15;
  if (p >= D.ns) return;
  const int n = D.n;
  const int a = k & 3, b = k >> 2;
  const double inv = D.ds[p] / (D.dx * D.dx);
  const double f = D.f[p];
  // sheet onto the nodes (same stencil as the solve's R_s)
  const int i0 = D.st_i[2 * p], j0 = D.st_i[2 * p + 1];
  atomicAdd(D.wsheet + (size_t)(j0 + b) * n + i0 + a,
            inv * f * D.st_w[8 * p + a] * D.st_w[8 * p + 4 + b]);
  // surface force terms onto the faces
  const PresStencil s = D.st[p];
  double vsx, vsy;
  surf_velocity(D, p, D.xs[p], D.ys[p], vsx, vsy);
  const double ddt = D.ddt[p];
  const double qx = D.pnx[p] * ddt - vsy * f;   // v_s x gamma = (v_sy f, -v_sx f)
  const double qy = D.pny[p] * ddt + vsx * f;
  atomicAdd(D.fx + (size_t)(s.ju + b) * n + s.iu + a, inv * qx * s.wxu[a] * s.wyu[b]);
  atomicAdd(D.fy + (size_t)(s.jv + b) * n + s.iv + a, inv * qy * s.wxv[a] * s.wyv[b]);
}

// node vorticity of the fluid: -(Delta_h psi)/dx^2 minus the sheet's part
template <class T>
__device__ __forceinline__ double fluid_vorticity(const T *psi, const double *wsheet, int n, int i, int j,
                                                  double dx) {
  if (i < 1 || j < 1 || i > n - 2 || j > n - 2) return 0.0;
  const size_t c = (size_t)j * n + i;
  const double lap = (double)psi[c + 1] + (double)psi[c - 1] + (double)psi[c + n] + (double)psi[c - n] -
                     4.0 * (double)psi[c];
  return -lap / (dx * dx) - wsheet[c];
}

// Lamb vector w x v on the x-face (x_i, y_j+1/2): -w v, w from its two
// nodes, v from its four y-faces
template <class T>
__device__ double lamb_x(const T *psi, const double *wsheet, int n, int i, int j, double dx, double vinf) {
  if (i < 1 || i > n - 2 || j < 0 || j > n - 2) return 0.0;
  const double wv = 0.5 * (fluid_vorticity(psi, wsheet, n, i, j, dx) +
                           fluid_vorticity(psi, wsheet, n, i, j + 1, dx));
  const double vb = 0.25 * (face_v(psi, n, i - 1, j, dx) + face_v(psi, n, i, j, dx) +
                            face_v(psi, n, i - 1, j + 1, dx) + face_v(psi, n, i, j + 1, dx)) + vinf;
  return -wv * vb;
}

// on the y-face (x_i+1/2, y_j): +w u
template <class T>
__device__ double lamb_y(const T *psi, const double *wsheet, int n, int i, int j, double dx, double uinf) {
  if (j < 1 || j > n - 2 || i < 0 || i > n - 2) return 0.0;
  const double wv = 0.5 * (fluid_vorticity(psi, wsheet, n, i, j, dx) +
                           fluid_vorticity(psi, wsheet, n, i + 1, j, dx));
  const double ub = 0.25 * (face_u(psi, n, i, j - 1, dx) + face_u(psi, n, i, j, dx) +
                            face_u(psi, n, i + 1, j - 1, dx) + face_u(psi, n, i + 1, j, dx)) + uinf;
  return wv * ub;
}

// source of the cell pressure Poisson equation: D (w x v + R_f terms) on the
// (n-1)^2 cells, stored n x n with a zero last row and column
template <class T>
__global__ __launch_bounds__(256) void k_pres_source(PresDesc D) {
  const int n = D.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  const size_t c = (size_t)j * n + i;
  if (i > n - 2 || j > n - 2) {
    D.src[c] = 0.0;
    return;
  }
  const T *psi = static_cast<const T *>(D.psi);
  const double dx = D.dx;
  const double uinf = D.psi_total ? 0.0 : D.u_inf, vinf = D.psi_total ? 0.0 : D.v_inf;
  const double fx1 = lamb_x(psi, D.wsheet, n, i + 1, j, dx, vinf) + D.fx[c + 1];
  const double fx0 = lamb_x(psi, D.wsheet, n, i, j, dx, vinf) + D.fx[c];
  const double fy1 = lamb_y(psi, D.wsheet, n, i, j + 1, dx, uinf) + D.fy[c + n];
  const double fy0 = lamb_y(psi, D.wsheet, n, i, j, dx, uinf) + D.fy[c];
  D.src[c] = (fx1 - fx0) / dx + (fy1 - fy0) / dx;
}

// p = -rho |v|^2 / 2 + rho (-L^-1 src) (the convolution gives -L^-1 src up to
// a uniform value); zero outside the (n-1)^2 cells
template <class T>
__global__ __launch_bounds__(256) void k_pres_finish(PresDesc D) {
  const int n = D.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= n) return;
  const size_t c = (size_t)j * n + i;
  if (i > n - 2 || j > n - 2) {
    D.p[c] = 0.0;
    return;
  }
  const T *psi = static_cast<const T *>(D.psi);
  const double uinf = D.psi_total ? 0.0 : D.u_inf, vinf = D.psi_total ? 0.0 : D.v_inf;
  const double uc = 0.5 * (face_u(psi, n, i, j, D.dx) + face_u(psi, n, i + 1, j, D.dx)) + uinf;
  const double vc = 0.5 * (face_v(psi, n, i, j, D.dx) + face_v(psi, n, i, j + 1, D.dx)) + vinf;
  D.p[c] = -0.5 * D.rho * (uc * uc + vc * vc) + D.rho * D.tmp[c];
}

// p+- = E_c p +- dp/2 at the surface points (E_c: three-point weights on the
// cell lattice)
__global__ void k_pres_sides(PresDesc D) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= D.ns) return;
  const int n = D.n;
  const double xi = (D.xs[p] - D.x0) / D.dx - 0.5, eta = (D.ys[p] - D.y0) / D.dx - 0.5;
  const int i0 = (int)floor(xi) - 1, j0 = (int)floor(eta) - 1;
  double acc = 0.0;
  for (int b = 0; b < 4; ++b) {
    const double wy = yang3(eta - (j0 + b));
    for (int a = 0; a < 4; ++a) acc += yang3(xi - (i0 + a)) * wy * D.p[(size_t)(j0 + b) * n + i0 + a];
  }
  D.pside[p] = acc + 0.5 * D.dp[p];
  D.pside[D.ns + p] = acc - 0.5 * D.dp[p];
}

// Q = -A K over the first ns rows and columns of A (leading dimension lda):
// Q[c][p] column-major, one thread per (p, c)
__global__ __launch_bounds__(256) void k_pres_q(int ns, int lda, const double *__restrict__ A,
                                                const double *__restrict__ K, double *Q) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
  if (p >= ns) return;
  const double *a = A + (size_t)p * lda;
  const double *k = K + (size_t)c * ns;
  double acc = 0.0;
  for (int q = 0; q < ns; ++q) acc += a[q] * k[q];
  Q[(size_t)c * ns + p] = -acc;
}

}  // namespace

hipError_t launch_pres_q(int ns, int lda, const double *A, const double *K, double *Q, hipStream_t s) {
  hipLaunchKernelGGL(k_pres_q, dim3((ns + 255) / 256, ns), dim3(256), 0, s, ns, lda, A, K, Q);
  return hipGetLastError();
}

hipError_t launch_pres_stencils(int ns, const double *xs, const double *ys, double x0, double y0,
                                double dx, PresStencil *st, hipStream_t s) {
  hipLaunchKernelGGL(k_pres_stencils, dim3((ns + 127) / 128), dim3(128), 0, s, ns, xs, ys, x0, y0, dx, st);
  return hipGetLastError();
}

hipError_t launch_pres_build(int n, int ns, const PresStencil *st, const double *pnx, const double *pny,
                             const int *st_i, const double *st_w, const double *ds, double dx,
                             const double *lgf, double *M, double *K, hipStream_t s) {
  hipLaunchKernelGGL(k_pres_build, dim3((ns + 255) / 256, ns), dim3(256), 0, s, n, ns, st, pnx, pny,
                     st_i, st_w, ds, dx, lgf, M, K);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pres_surface_part(const PresDesc &D, hipStream_t s) {
  hipLaunchKernelGGL((k_pres_surface<T>), dim3((D.ns + 255) / 256), dim3(256), 0, s, D);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pres_field_part(const PresDesc &D, hipStream_t s) {
  hipLaunchKernelGGL(k_pres_scatter, dim3((D.ns + 15) / 16), dim3(256), 0, s, D);
  hipLaunchKernelGGL((k_pres_source<T>), dim3((D.n + 255) / 256, D.n), dim3(256), 0, s, D);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pres_finish(const PresDesc &D, hipStream_t s) {
  hipLaunchKernelGGL((k_pres_finish<T>), dim3((D.n + 255) / 256, D.n), dim3(256), 0, s, D);
  if (D.pside) hipLaunchKernelGGL(k_pres_sides, dim3((D.ns + 127) / 128), dim3(128), 0, s, D);
  return hipGetLastError();
}

template hipError_t launch_pres_surface_part<float>(const PresDesc &, hipStream_t);
template hipError_t launch_pres_surface_part<double>(const PresDesc &, hipStream_t);
template hipError_t launch_pres_field_part<float>(const PresDesc &, hipStream_t);
template hipError_t launch_pres_field_part<double>(const PresDesc &, hipStream_t);
template hipError_t launch_pres_finish<float>(const PresDesc &, hipStream_t);
template hipError_t launch_pres_finish<double>(const PresDesc &, hipStream_t);

}  // namespace gpf
