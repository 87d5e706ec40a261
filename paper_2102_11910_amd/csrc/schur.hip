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
#include "weights.h"

namespace gpf {
namespace {


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

// y = A^T x, one thread per column of A (row-major, ns x ns)
__global__ __launch_bounds__(256) void k_gemv_t(int ns, const double *__restrict__ A,
                                                const double *__restrict__ x,
                                                double *__restrict__ y) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ns) return;
  double acc = 0.0;
  for (int p = 0; p < ns; ++p) acc += x[p] * A[(size_t)p * ns + q];
  y[q] = acc;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Impulse about the origin (eqs. linimpxd, linimpyd, angimpd), one
// workgroup per problem that asks for it.  The node inner products of the
// regularized vortices equal the point sums (the M4' weights reproduce x, y
// and x^2 + y^2), so the fluid part comes from the moments that binning
// already summed per workgroup; new vortices add their strengths at their
// positions; the body adds dS (f + n_x v_y - n_y v_x), with the surface
// velocity relative to the fluid at infinity.
__global__ __launch_bounds__(256) void k_impulse(const ProbDesc *__restrict__ d) {
  const ProbDesc &P = d[blockIdx.y];
  if (!P.imp_out) return;
  __shared__ double red[3][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const SolveScalars &sv = P.sv;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;   // sums of (y, x, x^2 + y^2) times strength
  const int nvb = P.nv > 0 ? bin_count_blocks(P.nv) : 0;   // workgroups of the binning count
  for (int b = tid; b < nvb; b += 256) {
    a0 += P.partials[2 * (size_t)kPartStride + b];
    a1 += P.partials[1 * (size_t)kPartStride + b];
    a2 += P.partials[3 * (size_t)kPartStride + b];
  }
  if (tid < sv.m) {
    const double g = P.aux[SC_GAMMA_NEW + tid];
    const double x = sv.znew_from >= 0 ? P.xv[sv.znew_from + tid] : sv.xnew[tid];
    const double y = sv.znew_from >= 0 ? P.yv[sv.znew_from + tid] : sv.ynew[tid];
    a0 += g * y;
    a1 += g * x;
    a2 += g * (x * x + y * y);
  }
  if (P.ns > 0 && P.f_out) {
    for (int p = tid; p < P.ns; p += 256) {
      const double x = P.xs[p], y = P.ys[p];
      const int j = P.part ? P.part[p] : 0;
      const double ub = P.part ? sv.pub[j] : sv.ub, vb = P.part ? sv.pvb[j] : sv.vb;
      const double om = P.part ? sv.pom[j] : sv.omega;
      const double vx = ub - sv.u_inf - om * y, vy = vb - sv.v_inf + om * x;
      const double q = P.ds[p] * (P.f_out[p] + P.nx[p] * vy - P.ny[p] * vx);
      a0 += y * q;
      a1 += x * q;
      a2 += (x * x + y * y) * q;
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  if (lane == 0) {
    red[0][wave] = a0;
    red[1][wave] = a1;
    red[2][wave] = a2;
  }
  __syncthreads();
  if (tid == 0) {
    const double s0 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double s1 = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const double s2 = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    P.imp_out[0] = s0;
    P.imp_out[1] = -s1;
    P.imp_out[2] = -0.5 * s2;
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
    double ub = sv.ub, vb = sv.vb, om = sv.omega;
    if (P.part) {   // several parts: the motion of this point's part
      const int j = P.part[p];
      ub = sv.pub[j];
      vb = sv.pvb[j];
      om = sv.pom[j];
    }
    const double sb = (ub - sv.u_inf) * y - (vb - sv.v_inf) * x - 0.5 * om * (x * x + y * y);
    P.rhs[p] = sb - acc;
    return;
  }
  if (sv.m <= 0) return;
  const int m = sv.m;
  const int pj = ((int)blockIdx.x - nbe) * (kRB / 16) + (int)threadIdx.x / 16;
  const int lane = threadIdx.x & 15;
  const bool active = pj < ns * m;
  double val = 0.0;
  int p = 0, j = 0;
  if (active) {
    p = pj % ns;
    j = pj / ns;
    const double zx = sv.znew_from >= 0 ? P.xv[sv.znew_from + j] : sv.xnew[j];
    const double zy = sv.znew_from >= 0 ? P.yv[sv.znew_from + j] : sv.ynew[j];
    const double xi = (zx - P.x0) / P.dx, eta = (zy - P.y0) / P.dx;
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



// Surface solve of one batch in one launch.  Every scalar the constraint
// modes need is a dot product with the rhs columns: the circulations
// sum_p dS_p y_c[p] = ghat . rhs_c (ghat = S^-T dS, a body constant) and the
// values y_c[k] at the edge points (rows k of S^-1).  Each workgroup forms
// them itself, solves the small constraint system, then finishes its own
// rows of f and f~: outputs and R_s f into the source field.  Workgroup 0
// writes the scalars and adds the new vortices.  No workgroup waits for
// another.
constexpr int kCB = 256;                       // 4 waves
constexpr int kRowsPerWave = 4;
constexpr int kCRows = 4 * kRowsPerWave;       // surface rows per workgroup
constexpr int kMaxCol = 1 + GPF_MAX_EDGES;
constexpr int kRStage = 6144;                  // rhs doubles staged in LDS

constexpr int kPre = 4;   // slices of 64 of each S^-1 row a wave loads up front

// MC: columns of the rhs a launch can have (1 + the largest m).  RPW: rows
// of S^-1 per wave (4 rows per workgroup and wave count); launches with few
// workgroups take one row per wave, so that more workgroups share the rows.
template <class T, int MC, int RPW>
__global__ __launch_bounds__(kCB) void k_schur_apply(const ProbDesc *__restrict__ d) {
  constexpr int CR = 4 * RPW;      // surface rows per workgroup
  constexpr int PRE = 16 / RPW;    // slices of 64 of each row a wave loads up front
  __shared__ double rs[kRStage];
  __shared__ double red[4][MC];                  // per-wave parts of ghat . rhs_c
  __shared__ double ye[GPF_MAX_EDGES][MC];       // y_c / f0 at the edge points
  __shared__ double yr[CR][MC];              // y_c at this workgroup's rows
  __shared__ double scal[3 + GPF_MAX_EDGES];     // c1, s0, Gamma_b, Gamma_j
  __shared__ double circ[MC];                    // ghat . rhs_c
  __shared__ double A[GPF_MAX_EDGES][GPF_MAX_EDGES + 1];
  __shared__ double gsrc2;                       // circulation of the final source
  __shared__ int singular_flag;
  const ProbDesc &P = d[blockIdx.y];
  const int ns = P.ns;
  const int row0 = blockIdx.x * CR;
  if (row0 >= ns) return;
  const SolveScalars &sv = P.sv;
  const int mode = sv.mode;
  const int m = mode == GPF_KUTTA_SHED ? sv.m : 0;
  const int ncol = 1 + m;
  const int ne = mode == GPF_KUTTA_SHED ? m : (mode == GPF_KUTTA_STEADY ? 1 : 0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  const double gw_dev = P.aux[SC_GAMMA_W];
  // the finishing step's load (this thread's row) does not depend on the
  // solve: issued first
  const int lr = tid >> 4, node = tid & 15;
  const int pf = min(row0 + min(lr, CR - 1), ns - 1);
  const double f0p = P.f0[pf];
  size_t coff[MC];   // column offsets, clamped to the last column
#pragma unroll
  for (int c = 0; c < MC; ++c) coff[c] = (size_t)min(c, ncol - 1) * ns;
  if (P.y) {
    // y_c = S^-1 r_c was formed for the whole launch: ghat . r_c = dS . y_c,
    // and the edge rows and this workgroup's rows are read from y
    const double *Y = P.y;
    double acc[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[c] = 0.0;
    for (int q = tid; q < ns; q += kCB) {
      const double w = P.ds[q];
#pragma unroll
      for (int c = 0; c < MC; ++c) acc[c] += w * Y[coff[c] + q];
    }
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      if (c < ncol) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) red[wave][c] = v;
      }
    }
    if (tid < ne * MC) {
      const int e = tid / MC, c = tid - e * MC;
      const int kp = sv.edges[e];
      if (c < ncol) ye[e][c] = Y[(size_t)c * ns + kp] / P.f0[kp];
    }
    if (tid < CR * MC) {
      const int rr = tid / MC, c = tid - rr * MC;
      if (c < ncol && row0 + rr < ns) yr[rr][c] = Y[(size_t)c * ns + row0 + rr];
    }
  } else {
  // Loads below are unconditional, with indices clamped into range, so
  // that each wave keeps many of them in flight; sums of clamped terms
  // are discarded.  The first slices of this wave's rows of S^-1 and of
  // ghat do not depend on the rhs: they are issued before it is staged.
  const int r0 = row0 + wave * RPW;
  const int nr = min(RPW, ns - r0);
  const double *arow[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) arow[r] = P.sinv + (size_t)min(r0 + r, ns - 1) * ns;
  double apre[PRE][RPW];
#pragma unroll
  for (int i = 0; i < PRE; ++i)
#pragma unroll
    for (int r = 0; r < RPW; ++r) apre[i][r] = arow[r][min(lane + 64 * i, ns - 1)];
  const double gpre = P.ghat[min(tid, ns - 1)];
  const double *R = P.rhs;
  if (ncol * ns <= kRStage) {
#pragma unroll 4
    for (int k = tid; k < ncol * ns; k += kCB) rs[k] = P.rhs[k];
    __syncthreads();
    R = rs;
  }
  // ghat . rhs_c, all columns in one sweep
  {
    double acc[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[c] = tid < ns ? gpre * R[coff[c] + min(tid, ns - 1)] : 0.0;
#pragma unroll 2
    for (int q = tid + kCB; q < ns; q += kCB) {
      const double g = P.ghat[q];
#pragma unroll
      for (int c = 0; c < MC; ++c) acc[c] += g * R[coff[c] + q];
    }
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      if (c < ncol) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) red[wave][c] = v;
      }
    }
  }
  // rows of S^-1 at the edge points, one wave each
  for (int e = wave; e < ne; e += 4) {
    const int k = sv.edges[e];
    const double inv_f0 = 1.0 / P.f0[k];
    const double *a = P.sinv + (size_t)k * ns;
    double acc[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[c] = 0.0;
#pragma unroll 4
    for (int q = lane; q < ns; q += 64) {
      const double aq = a[q];
#pragma unroll
      for (int c = 0; c < MC; ++c) acc[c] += aq * R[coff[c] + q];
    }
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      if (c < ncol) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) ye[e][c] = v * inv_f0;
      }
    }
  }
  // this workgroup's rows: RPW per wave, interleaved over q
  {
    double acc[RPW][MC];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
      for (int c = 0; c < MC; ++c) acc[r][c] = 0.0;
    if (nr > 0) {
#pragma unroll
      for (int i = 0; i < PRE; ++i) {
        const int q = lane + 64 * i;
        if (q < ns) {
          double rq[MC];
#pragma unroll
          for (int c = 0; c < MC; ++c) rq[c] = R[coff[c] + q];
#pragma unroll
          for (int r = 0; r < RPW; ++r)
#pragma unroll
            for (int c = 0; c < MC; ++c) acc[r][c] += apre[i][r] * rq[c];
        }
      }
#pragma unroll 2
      for (int q = lane + 64 * PRE; q < ns; q += 64) {
        double aq[RPW], rq[MC];
#pragma unroll
        for (int r = 0; r < RPW; ++r) aq[r] = arow[r][q];
#pragma unroll
        for (int c = 0; c < MC; ++c) rq[c] = R[coff[c] + q];
#pragma unroll
        for (int r = 0; r < RPW; ++r)
#pragma unroll
          for (int c = 0; c < MC; ++c) acc[r][c] += aq[r] * rq[c];
      }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      if (r < nr) {
#pragma unroll
        for (int c = 0; c < MC; ++c) {
          if (c < ncol) {
            const double v = wave_sum(acc[r][c]);
            if (lane == 0) yr[wave * RPW + r][c] = v;
          }
        }
      }
    }
  }
  }
  __syncthreads();

  // constraint scalars (one thread; every workgroup gets the same values)
  if (tid == 0) {
    for (int c = 0; c < ncol; ++c) circ[c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    const double g0 = P.gamma0;
    double c1 = 0.0, s0 = 0.0, gb = 0.0, gsum = 0.0;
    singular_flag = 0;
    double *gam = scal + 3;
    for (int j = 0; j < GPF_MAX_EDGES; ++j) gam[j] = 0.0;
    if (mode == GPF_CIRCULATION) {
      s0 = (circ[0] - sv.gamma_b) / g0;
      gb = circ[0] - s0 * g0;
    } else {
      // c1 = fhat0 . s_b' / Gamma0 through the body moments of fhat0
      c1 = ((sv.ub - sv.u_inf) * P.mom_y - (sv.vb - sv.v_inf) * P.mom_x -
            0.5 * sv.omega * P.mom_r2) / g0;
      if (mode == GPF_KUTTA_STEADY) {
        s0 = ye[0][0] - c1;
        gb = circ[0] - (c1 + s0) * g0;
      } else {
        const double gamma_w = isnan(sv.gamma_w_in) ? gw_dev : sv.gamma_w_in;
        const double dstar = circ[0] - c1 * g0;   // fhat0 . f~*
        // Generalized edge conditions (Sec. 2.5): edge i takes part when the
        // intermediate sheet lies outside [fmin_i, fmax_i] at k_i, with the
        // violated bound as its target; the others shed nothing.  Kutta is
        // fmin = fmax = 0.  The sheet tested is the one the body carries if
        // nothing is shed, f~* - s0 with Kelvin's s0 = (fhat0 . f~* +
        // Gamma_w)/Gamma0: independent of the Green's function gauge, and
        // the shed strength vanishes as it reaches a bound.
        const double s0_keep = (dstar + gamma_w) / g0;
        int act[GPF_MAX_EDGES];
        double tgt[GPF_MAX_EDGES];
        int na = 0;
        for (int i = 0; i < m; ++i) {
          const double fs = ye[i][0] - c1 - s0_keep;
          if (fs < sv.fmin[i]) { act[na] = i; tgt[na++] = sv.fmin[i]; }
          else if (fs > sv.fmax[i]) { act[na] = i; tgt[na++] = sv.fmax[i]; }
        }
        // rows of eq. twovortex-gen over the active edges:
        // sum_j (1 + fhat0 . P_k f~_j) Gamma_j = -(Gamma_w + fhat0 . P_k f~* + Gamma0 t)
        double amax = 0.0;
        for (int r = 0; r < na; ++r) {
          const int i = act[r];
          for (int c = 0; c < na; ++c) {
            const int j = act[c];
            A[r][c] = 1.0 + circ[1 + j] - g0 * ye[i][1 + j];
            amax = fmax(amax, fabs(A[r][c]));
          }
          A[r][na] = -(gamma_w + dstar - g0 * (ye[i][0] - c1) + g0 * tgt[r]);
        }
        bool singular = false;
        for (int c = 0; c < na; ++c) {
          int pr = c;
          for (int i = c + 1; i < na; ++i)
            if (fabs(A[i][c]) > fabs(A[pr][c])) pr = i;
          if (!(fabs(A[pr][c]) > 1e-13 * amax)) { singular = true; break; }
          if (pr != c)
            for (int j = 0; j <= na; ++j) { const double t = A[c][j]; A[c][j] = A[pr][j]; A[pr][j] = t; }
          for (int i = 0; i < na; ++i) {
            if (i == c) continue;
            const double fct = A[i][c] / A[c][c];
            for (int j = c; j <= na; ++j) A[i][j] -= fct * A[c][j];
          }
        }
        for (int r = 0; r < na; ++r) gam[act[r]] = singular ? 0.0 : A[r][na] / A[r][r];
        singular_flag = singular ? 1 : 0;
        if (na > 0) {
          // s0: mean over the active edges of x_k - t, x = f~* + sum_j Gamma_j f~_j
          for (int r = 0; r < na; ++r) {
            const int i = act[r];
            double xk = ye[i][0] - c1;
            for (int j = 0; j < m; ++j) xk += gam[j] * ye[i][1 + j];
            s0 += xk - tgt[r];
          }
          s0 /= na;
        } else {
          s0 = s0_keep;   // nothing shed: Kelvin's theorem alone fixes s0
        }
        double gj = 0.0;
        for (int j = 0; j < m; ++j) {
          gj += gam[j] * circ[1 + j];
          gsum += gam[j];
        }
        gb = dstar + gj - s0 * g0;
      }
    }
    scal[0] = c1;
    scal[1] = s0;
    scal[2] = gb;
    gsrc2 = gw_dev + gb + gsum;
  }
  __syncthreads();

  // f, f~ of the rows (R_s f and the new vortices go to the field in
  // k_rs_apply, node by node)
  const double c1 = scal[0], s0 = scal[1];
  {
    const int p = row0 + lr;
    if (lr < CR && p < ns && node == 0) {
      double ft, f;
      if (mode == GPF_CIRCULATION) {
        f = yr[lr][0] - s0 * f0p;
        ft = f / f0p;
      } else {
        double x = yr[lr][0] / f0p - c1;
        for (int j = 0; j < m; ++j) x += scal[3 + j] * yr[lr][1 + j] / f0p;
        ft = x - s0;
        f = f0p * ft;
      }
      P.fs[p] = f;
      if (P.f_out) P.f_out[p] = f;
      if (P.ft_out) P.ft_out[p] = ft;
    }
  }
  // workgroup 0 writes the scalars last, so that no barrier waits on them
  if (blockIdx.x == 0 && tid == 0) {
    const double s0 = scal[1], gb = scal[2];
    P.aux[SC_GAMMA_SRC2] = gsrc2;
    P.aux[SC_S0] = s0;
    P.aux[SC_GAMMA_B] = gb;
    for (int j = 0; j < GPF_MAX_EDGES; ++j) P.aux[SC_GAMMA_NEW + j] = scal[3 + j];
    if (P.sc_out) {
      P.sc_out[SC_GAMMA_W] = gw_dev;
      P.sc_out[SC_GAMMA_SRC2] = gsrc2;
      P.sc_out[SC_S0] = s0;
      P.sc_out[SC_GAMMA_B] = gb;
      for (int j = 0; j < GPF_MAX_EDGES; ++j) P.sc_out[SC_GAMMA_NEW + j] = scal[3 + j];
    }
    if (singular_flag) atomicOr(P.status, GPF_DEV_SINGULAR);
  }
}

// y = S^-1 rhs for problems that share one body: the right-hand-side
// columns of all problems side by side (problem b's column c at b * ncol + c)
// times S^-1, a dense FP64 product on the matrix cores.  One workgroup of
// four wavefronts per 16 x 16 tile of y; wavefront w takes the quarter w of
// the k range, 16 steps of v_mfma_f64_16x16x4f64 at a time with all their
// operands loaded first (lane l holds A[l % 16][k + l / 16] and
// B[k + l / 16][l % 16]; output item r of lane l is row 4 r + l / 16,
// column l % 16 of the tile), and the four partial tiles are summed in LDS.
typedef double double4v __attribute__((ext_vector_type(4)));
constexpr int kGemmSteps = 16;
__global__ __launch_bounds__(256) void k_schur_gemm(const ProbDesc *__restrict__ d, int nb,
                                                    int ncol, int ns,
                                                    const double *__restrict__ A) {
  __shared__ double part[3][64][4];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int i0 = blockIdx.x * 16;
  const int g = blockIdx.y * 16 + li;   // column of the launch
  const int b = min(g / ncol, nb - 1), c = g - (g / ncol) * ncol;
  // this lane's problem: its column count and buffers, loaded together
  const ProbDesc &P = d[b];
  const int mode = P.sv.mode, mm = P.sv.m;
  const double *Rb = P.rhs + (size_t)c * ns;
  double *Yb = P.y + (size_t)c * ns;
  const bool colok = g / ncol < nb && c <= (mode == GPF_KUTTA_SHED ? mm : 0);
  const double *Ar = A + (size_t)min(i0 + li, ns - 1) * ns;
  const int kq = (((ns + 3) / 4 + 3) / 4) * 4;   // this wavefront's k range, a multiple of 4
  const int kbeg = wave * kq, kend = min(ns, kbeg + kq);
  double4v acc = {0.0, 0.0, 0.0, 0.0};
  for (int kc = kbeg; kc < kend; kc += 4 * kGemmSteps) {
    double av[kGemmSteps], bv[kGemmSteps];
#pragma unroll
    for (int t = 0; t < kGemmSteps; ++t) {
      const int k = kc + 4 * t + lk;
      const bool in = k < kend;
      av[t] = in ? Ar[k] : 0.0;
      bv[t] = (colok && in) ? Rb[k] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kGemmSteps; ++t)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], acc, 0, 0, 0);
  }
  if (wave > 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wave - 1][l][r] = acc[r];
  }
  __syncthreads();
  if (wave == 0 && colok) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = i0 + 4 * r + lk;
      const double v = acc[r] + part[0][l][r] + part[1][l][r] + part[2][l][r];
      if (row < ns) Yb[row] = v;
    }
  }
}

// Surface solve for a body of several parts (Sec. 2.7, eq. kuttasystem4).
// Part j has its own uniform value s0_j, so
//     f = y_0 + sum_i Gamma_i y_i - sum_j s0_j z_j,
// y_c = S^-1 r_c (rhs columns), z_j = S^-1 1_j (per body).  The rows, one per
// part and one per new vortex, need the part circulations of each column
// (gpart_j . r_c), the columns at the edge points (rows of S^-1) and the
// body constants C_jl (circulation of z_l over part j) and z_l at the edges.
// Every workgroup forms and solves the (nparts + m) system itself (a second
// time when edge bounds make some edges shed), then finishes its rows as in
// k_schur_apply.
constexpr int kMaxUnk = GPF_MAX_PARTS + GPF_MAX_EDGES;
constexpr int kMaxERows = GPF_MAX_EDGES + GPF_MAX_PARTS;

// Gauss-Jordan with partial pivoting on A (n x n, augmented); false when a
// pivot is below 1e-13 of the largest entry
__device__ bool solve_small(double (*A)[kMaxUnk + 1], int n, double *x) {
  double amax = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) amax = fmax(amax, fabs(A[i][j]));
  for (int c = 0; c < n; ++c) {
    int pr = c;
    for (int i = c + 1; i < n; ++i)
      if (fabs(A[i][c]) > fabs(A[pr][c])) pr = i;
    if (!(fabs(A[pr][c]) > 1e-13 * amax)) return false;
    if (pr != c)
      for (int j = 0; j <= n; ++j) {
        const double t = A[c][j];
        A[c][j] = A[pr][j];
        A[pr][j] = t;
      }
    for (int i = 0; i < n; ++i) {
      if (i == c) continue;
      const double fct = A[i][c] / A[c][c];
      for (int j = c; j <= n; ++j) A[i][j] -= fct * A[c][j];
    }
  }
  for (int i = 0; i < n; ++i) x[i] = A[i][n] / A[i][i];
  return true;
}

template <class T>
__global__ __launch_bounds__(kCB) void k_schur_apply_parts(const ProbDesc *__restrict__ d) {
  __shared__ double rs[kRStage];
  __shared__ double red[4][GPF_MAX_PARTS][kMaxCol];
  __shared__ double circ[GPF_MAX_PARTS][kMaxCol];   // gpart_j . r_c
  __shared__ double ye[kMaxERows][kMaxCol];         // (S^-1 r_c) at the edge rows
  __shared__ double yr[kCRows][kMaxCol];            // (S^-1 r_c) at this workgroup's rows
  __shared__ double A[kMaxUnk][kMaxUnk + 1];
  __shared__ double sol[kMaxUnk];                   // s0_1.., Gamma_1..
  __shared__ double zed[GPF_MAX_PARTS][kMaxERows];  // z_l at the edge rows
  __shared__ double cjl[GPF_MAX_PARTS * GPF_MAX_PARTS];
  __shared__ double f0e[kMaxERows];
  const ProbDesc &P = d[blockIdx.y];
  const int ns = P.ns;
  const int row0 = blockIdx.x * kCRows;
  if (row0 >= ns) return;
  const SolveScalars &sv = P.sv;
  const int np = sv.nparts, m = sv.m, ncol = 1 + m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // edge rows: the m new-vortex edges, then each steady-Kutta part's edge
  __shared__ int erow_k[kMaxERows];
  int ne = m;
  for (int j = 0; j < np; ++j) ne += sv.pmode[j] == GPF_KUTTA_STEADY;
  if (tid == 0) {
    int e = 0;
    for (int i = 0; i < m; ++i) erow_k[e++] = sv.edges[i];
    for (int j = 0; j < np; ++j)
      if (sv.pmode[j] == GPF_KUTTA_STEADY) erow_k[e++] = sv.kedge[j];
  }
  __syncthreads();
  // the body constants the constraint rows read, staged in parallel
  for (int t = tid; t < np * ne; t += kCB) {
    const int l = t / ne, e = t % ne;
    zed[l][e] = P.zpart[(size_t)l * ns + erow_k[e]];
  }
  for (int t = tid; t < np * np; t += kCB) cjl[t] = P.cpart[t];
  for (int e = tid; e < ne; e += kCB) f0e[e] = P.f0[erow_k[e]];

  const double gw_dev = P.aux[SC_GAMMA_W];
  const double *R = P.rhs;
  if (ncol * ns <= kRStage) {
#pragma unroll 4
    for (int k = tid; k < ncol * ns; k += kCB) rs[k] = P.rhs[k];
    __syncthreads();
    R = rs;
  }
  size_t coff[kMaxCol];
#pragma unroll
  for (int c = 0; c < kMaxCol; ++c) coff[c] = (size_t)min(c, ncol - 1) * ns;
  // part circulations of every column, one sweep per part
  for (int j = 0; j < np; ++j) {
    const double *g = P.gpart + (size_t)j * ns;
    double acc[kMaxCol];
#pragma unroll
    for (int c = 0; c < kMaxCol; ++c) acc[c] = 0.0;
#pragma unroll 2
    for (int q = tid; q < ns; q += kCB) {
      const double gq = g[q];
#pragma unroll
      for (int c = 0; c < kMaxCol; ++c) acc[c] += gq * R[coff[c] + q];
    }
#pragma unroll
    for (int c = 0; c < kMaxCol; ++c) {
      if (c < ncol) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) red[wave][j][c] = v;
      }
    }
  }
  // the columns at the edge rows, one wave each
  for (int e = wave; e < ne; e += 4) {
    const double *a = P.sinv + (size_t)erow_k[e] * ns;
    double acc[kMaxCol];
#pragma unroll
    for (int c = 0; c < kMaxCol; ++c) acc[c] = 0.0;
#pragma unroll 4
    for (int q = lane; q < ns; q += 64) {
      const double aq = a[q];
#pragma unroll
      for (int c = 0; c < kMaxCol; ++c) acc[c] += aq * R[coff[c] + q];
    }
#pragma unroll
    for (int c = 0; c < kMaxCol; ++c) {
      if (c < ncol) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) ye[e][c] = v;
      }
    }
  }
  // this workgroup's rows
  {
    const int r0 = row0 + wave * kRowsPerWave;
    const int nr = min(kRowsPerWave, ns - r0);
    double acc[kRowsPerWave][kMaxCol];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
      for (int c = 0; c < kMaxCol; ++c) acc[r][c] = 0.0;
    if (nr > 0) {
      const double *arow[kRowsPerWave];
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r) arow[r] = P.sinv + (size_t)min(r0 + r, ns - 1) * ns;
#pragma unroll 2
      for (int q = lane; q < ns; q += 64) {
        double aq[kRowsPerWave], rq[kMaxCol];
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) aq[r] = arow[r][q];
#pragma unroll
        for (int c = 0; c < kMaxCol; ++c) rq[c] = R[coff[c] + q];
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r)
#pragma unroll
          for (int c = 0; c < kMaxCol; ++c) acc[r][c] += aq[r] * rq[c];
      }
    }
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      if (r < nr) {
#pragma unroll
        for (int c = 0; c < kMaxCol; ++c) {
          if (c < ncol) {
            const double v = wave_sum(acc[r][c]);
            if (lane == 0) yr[wave * kRowsPerWave + r][c] = v;
          }
        }
      }
    }
  }
  __syncthreads();

  if (tid == 0) {
    for (int j = 0; j < np; ++j)
      for (int c = 0; c < ncol; ++c)
        circ[j][c] = red[0][j][c] + red[1][j][c] + red[2][j][c] + red[3][j][c];
    const int N = np + m;
    const double *C = cjl;
    bool active[GPF_MAX_EDGES];
    double tgt[GPF_MAX_EDGES];
    for (int i = 0; i < m; ++i) {
      active[i] = false;
      tgt[i] = 0.0;
    }
    bool ok = true;
    for (int pass = 0; pass < 2; ++pass) {
      // one row per part
      int kr = m;   // next steady-Kutta edge row
      for (int j = 0; j < np; ++j) {
        const int mode = sv.pmode[j];
        if (mode == GPF_KUTTA_STEADY) {
          const int e = kr++;
          for (int l = 0; l < np; ++l) A[j][l] = -zed[l][e];
          for (int i = 0; i < m; ++i) A[j][np + i] = ye[e][1 + i];
          A[j][N] = -ye[e][0];
        } else {
          for (int l = 0; l < np; ++l) A[j][l] = -C[j * np + l];
          for (int i = 0; i < m; ++i)
            A[j][np + i] = circ[j][1 + i] + ((mode == GPF_KUTTA_SHED && sv.epart[i] == j) ? 1.0 : 0.0);
          const double gw = P.pgw_dev ? P.pgw_dev[j] : sv.pgw[j];
          A[j][N] = (mode == GPF_CIRCULATION ? sv.pgb[j] : -gw) - circ[j][0];
        }
      }
      // one row per new vortex: held at its target, or shedding nothing
      for (int i = 0; i < m; ++i) {
        const int r = np + i;
        for (int c = 0; c <= N; ++c) A[r][c] = 0.0;
        if (active[i]) {
          for (int l = 0; l < np; ++l) A[r][l] = -zed[l][i];
          for (int i2 = 0; i2 < m; ++i2) A[r][np + i2] = ye[i][1 + i2];
          A[r][N] = f0e[i] * tgt[i] - ye[i][0];
        } else {
          A[r][np + i] = 1.0;
        }
      }
      ok = solve_small(A, N, sol);
      if (!ok || pass == 1) break;
      // which edges shed: the sheet with nothing shed against the bounds
      bool any = false;
      for (int i = 0; i < m; ++i) {
        double fk = ye[i][0];
        for (int l = 0; l < np; ++l) fk -= sol[l] * zed[l][i];
        const double ft = fk / f0e[i];
        if (ft < sv.fmin[i]) { active[i] = true; tgt[i] = sv.fmin[i]; any = true; }
        else if (ft > sv.fmax[i]) { active[i] = true; tgt[i] = sv.fmax[i]; any = true; }
      }
      if (!any) break;
    }
    if (!ok) {
      for (int c = 0; c < N; ++c) sol[c] = 0.0;
      if (blockIdx.x == 0) atomicOr(P.status, GPF_DEV_SINGULAR);
    }
    if (blockIdx.x == 0) {
      double gsum = 0.0, gb_tot = 0.0;
      for (int i = 0; i < m; ++i) gsum += sol[np + i];
      for (int j = 0; j < np; ++j) {
        double gb = circ[j][0];
        for (int i = 0; i < m; ++i) gb += sol[np + i] * circ[j][1 + i];
        for (int l = 0; l < np; ++l) gb -= sol[l] * C[j * np + l];
        gb_tot += gb;
        P.aux[SC_PART_S0 + j] = sol[j];
        P.aux[SC_PART_GB + j] = gb;
        if (P.sc_out) {
          P.sc_out[SC_PART_S0 + j] = sol[j];
          P.sc_out[SC_PART_GB + j] = gb;
        }
      }
      P.aux[SC_GAMMA_SRC2] = gw_dev + gb_tot + gsum;
      P.aux[SC_S0] = sol[0];
      P.aux[SC_GAMMA_B] = gb_tot;
      for (int i = 0; i < GPF_MAX_EDGES; ++i) P.aux[SC_GAMMA_NEW + i] = i < m ? sol[np + i] : 0.0;
      if (P.sc_out) {
        P.sc_out[SC_GAMMA_W] = gw_dev;
        P.sc_out[SC_GAMMA_SRC2] = gw_dev + gb_tot + gsum;
        P.sc_out[SC_S0] = sol[0];
        P.sc_out[SC_GAMMA_B] = gb_tot;
        for (int i = 0; i < GPF_MAX_EDGES; ++i) P.sc_out[SC_GAMMA_NEW + i] = i < m ? sol[np + i] : 0.0;
      }
    }
  }
  __syncthreads();

  // f, f~ of the rows (R_s f and the new vortices go to the field in
  // k_rs_apply, node by node)
  {
    const int lr = tid >> 4, node = tid & 15;
    const int p = row0 + lr;
    if (p < ns && node == 0) {
      double f = yr[lr][0];
      for (int i = 0; i < m; ++i) f += sol[np + i] * yr[lr][1 + i];
      for (int l = 0; l < np; ++l) f -= sol[l] * P.zpart[(size_t)l * ns + p];
      P.fs[p] = f;
      if (P.f_out) P.f_out[p] = f;
      if (P.ft_out) P.ft_out[p] = f / P.f0[p];
    }
  }
}

// R_s f and the new vortices' stencils added to the source field (Sec. 2.2,
// eq. basicblock; new vortices Sec. 2.4.2), node by node: one thread per
// node the surface stencils reach sums its entries in point order, then the
// new vortices reaching the node in their order, and adds the sum once; the
// last workgroup of a problem that adds new vortices takes their nodes
// outside that list (the first of equal candidates).  No two threads write
// one node, so the field is the same bits on every run.
// new vortex j's base node (i0, j0) and fractions; false outside the window
__device__ __forceinline__ bool new_vortex_cell(const ProbDesc &P, int j, int *i0, int *j0, double *fx,
                                                double *fy) {
  const SolveScalars &sv = P.sv;
  const int n = P.n;
  const double zx = sv.znew_from >= 0 ? P.xv[sv.znew_from + j] : sv.xnew[j];
  const double zy = sv.znew_from >= 0 ? P.yv[sv.znew_from + j] : sv.ynew[j];
  const double xi = (zx - P.x0) / P.dx, eta = (zy - P.y0) / P.dx;
  if (!(xi >= 2.0 && xi < n - 3.0 && eta >= 2.0 && eta < n - 3.0)) return false;
  *i0 = (int)floor(xi) - 1;
  *j0 = (int)floor(eta) - 1;
  *fx = xi - floor(xi);
  *fy = eta - floor(eta);
  return true;
}

// sum over new vortices 0 .. m-1 whose stencils reach node (ix, iy) of
// Gamma_j times the stencil weight there
__device__ __forceinline__ double new_vortex_weights(const ProbDesc &P, int m, int ix, int iy) {
  double v = 0.0;
  for (int j = 0; j < m; ++j) {
    int i0, j0;
    double fx, fy;
    if (!new_vortex_cell(P, j, &i0, &j0, &fx, &fy)) continue;
    const int a = ix - i0, b = iy - j0;
    if (a < 0 || a > 3 || b < 0 || b > 3) continue;
    v += P.aux[SC_GAMMA_NEW + j] * m4p(fy + 1.0 - b) * m4p(fx + 1.0 - a);
  }
  return v;
}

template <class T>
__device__ __forceinline__ void rs_apply_body(const ProbDesc &P, const FlatBlock &fb) {
  const int K = P.rs_nodes, n = P.n, m = P.sv.m;
  const int kb = (K + 255) / 256;
  T *w = static_cast<T *>(P.w);
  const double inv_dx2 = 1.0 / (P.dx * P.dx);
  if (fb.blk < kb) {
    const int k = fb.blk * 256 + threadIdx.x;
    if (k >= K) return;
    const int node = P.rs_node[k], e1 = P.rs_off[k + 1];
    double v = 0.0;
    for (int e = P.rs_off[k]; e < e1; ++e) {
      const int c = P.rs_code[e], p = c >> 4, b = (c >> 2) & 3, a = c & 3;
      v += P.ds[p] * P.fs[p] * inv_dx2 * P.st_w[8 * p + a] * P.st_w[8 * p + 4 + b];
    }
    if (m > 0) v += new_vortex_weights(P, m, node % n, node / n) * inv_dx2;
    w[node] = (T)((double)w[node] + v);
  } else if (fb.blk == kb && m > 0) {
    // candidates: node (a, b) of new vortex j, thread 16 j + 4 b + a
    const int t = threadIdx.x, j = t >> 4, a = t & 3, b = (t >> 2) & 3;
    if (j >= m) return;
    int i0, j0;
    double fx, fy;
    if (!new_vortex_cell(P, j, &i0, &j0, &fx, &fy)) return;
    const int ix = i0 + a, iy = j0 + b, node = iy * n + ix;
    // a node on the list is its thread's; one an earlier new vortex
    // reaches is that vortex's candidate
    int lo = 0, hi = K;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (P.rs_node[mid] < node) lo = mid + 1; else hi = mid;
    }
    if (lo < K && P.rs_node[lo] == node) return;
    for (int jj = 0; jj < j; ++jj) {
      int ki, kj;
      double gx, gy;
      if (new_vortex_cell(P, jj, &ki, &kj, &gx, &gy) && ix - ki >= 0 && ix - ki <= 3 && iy - kj >= 0 &&
          iy - kj <= 3)
        return;
    }
    w[node] = (T)((double)w[node] + new_vortex_weights(P, m, ix, iy) * inv_dx2);
  }
}

__global__ __launch_bounds__(256) void k_rs_apply(const ProbDesc *__restrict__ d, FlatMap fm) {
  FlatBlock fb;
  if (!flat_block(fm, &fb)) return;
  const ProbDesc &P = d[fb.prob];
  if (P.w64)
    rs_apply_body<double>(P, fb);
  else
    rs_apply_body<float>(P, fb);
}


// ---------------------------------------------------------------------------
// Blocked in-place Gauss-Jordan inverse with partial pivoting (the FP64
// inverse of the Schur complement S, Sec. 2.2.2 and App. A), by panels of
// kGjPanel columns K, out of place between two buffers (cur -> next):
//  1. k_bgj_panel: one workgroup holds the n x |K| panel in registers and
//     runs the column steps of K on it (pivot row = largest |entry| among
//     the rows not yet pivotal, row exchange, in-place sweep), so that the
//     panel's pivot rows hold A_KK^-1 and its other rows -A_IK A_KK^-1 (in
//     the exchanged row order).  It records the pivots and the source row of
//     every row after the exchanges.
//  2. k_bgj_update: the other columns J, on FP64 matrix cores:
//     next[K, J] = A_KK^-1 A_KJ,  next[I, J] = A_IJ - A_IK A_KK^-1 A_KJ,
//     i.e. next[i, J] = (i in K ? 0 : cur[src(i), J]) + panel[i, :] cur[src(K), J].
// After the last panel the exchanges are undone on the columns (k_bgj_order,
// k_bgj_gather).
// ---------------------------------------------------------------------------
constexpr int kGjPanel = 16;
constexpr int kGjThreads = 512;
constexpr int kGjMaxN = 4 * kGjThreads;   // rows a panel workgroup holds (4 per thread)

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int R>
__global__ __launch_bounds__(kGjThreads) void k_bgj_panel(int n, int k0, const double *__restrict__ cur,
                                                         double *__restrict__ next, int *__restrict__ src,
                                                         int *__restrict__ piv, double *__restrict__ pval) {
  constexpr int NW = kGjThreads / 64;
  __shared__ double red_v[NW];
  __shared__ int red_i[NW];
  __shared__ double prow_s[kGjPanel], swap_s[kGjPanel];
  __shared__ int pr_s[kGjPanel], pos_s[2 * kGjPanel], from_s[2 * kGjPanel];
  const int w = min(kGjPanel, n - k0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double v[R][kGjPanel];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + r * kGjThreads;
#pragma unroll
    for (int c = 0; c < kGjPanel; ++c) v[r][c] = (i < n && c < w) ? cur[(size_t)i * n + k0 + c] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < kGjPanel; ++c) {
    if (c >= w) continue;
    const int k = k0 + c;
    // pivot: largest |entry| of column k among rows >= k, lowest row on
    // ties; row k itself when no entry compares (all NaN), so the pivot
    // row is always in [k, n)
    double bv = -1.0;
    int bi = k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + r * kGjThreads;
      const double a = fabs(v[r][c]);
      if (i >= k && i < n && a > bv) {
        bv = a;
        bi = i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[wave] = bv;
      red_i[wave] = bi;
    }
    __syncthreads();
    double pbest = red_v[0];
    int pr = red_i[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) {
      const double ov = red_v[q];
      const int oi = red_i[q];
      if (ov > pbest || (ov == pbest && oi < pr)) {
        pbest = ov;
        pr = oi;
      }
    }
    if (tid == 0) pr_s[c] = pr;
    // the pivot row to LDS; row k to LDS when it moves to row pr
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + r * kGjThreads;
      if (i == pr) {
#pragma unroll
        for (int cc = 0; cc < kGjPanel; ++cc) prow_s[cc] = v[r][cc];
      }
      if (i == k && pr != k) {
#pragma unroll
        for (int cc = 0; cc < kGjPanel; ++cc) swap_s[cc] = v[r][cc];
      }
    }
    __syncthreads();
    double prow[kGjPanel];
#pragma unroll
    for (int cc = 0; cc < kGjPanel; ++cc) prow[cc] = prow_s[cc];
    const double p = prow[c];
    if (tid == 0) {
      piv[k] = pr;
      pval[k] = p;
    }
    const double ip = p != 0.0 ? 1.0 / p : 0.0;
#pragma unroll
    for (int cc = 0; cc < kGjPanel; ++cc) prow[cc] = cc == c ? ip : prow[cc] * ip;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + r * kGjThreads;
      if (i == pr && pr != k) {
#pragma unroll
        for (int cc = 0; cc < kGjPanel; ++cc) v[r][cc] = swap_s[cc];
      }
      if (i == k) {
#pragma unroll
        for (int cc = 0; cc < kGjPanel; ++cc) v[r][cc] = prow[cc];
      } else {
        const double m = v[r][c];
#pragma unroll
        for (int cc = 0; cc < kGjPanel; ++cc) v[r][cc] = cc == c ? -m * ip : v[r][cc] - m * prow[cc];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = tid + r * kGjThreads;
    if (i < n) {
#pragma unroll
      for (int c = 0; c < kGjPanel; ++c)
        if (c < w) next[(size_t)i * n + k0 + c] = v[r][c];
      src[i] = i;
    }
  }
  __syncthreads();   // the identity map is in place before the moved rows overwrite it
  if (tid == 0) {
    // rows the exchanges moved: replay them on the (at most 2w) rows involved
    int m = 0;
    for (int c = 0; c < w; ++c) {
      const int a = k0 + c, b = pr_s[c];
      int ia = -1, ib = -1;
      for (int q = 0; q < m; ++q) {
        if (pos_s[q] == a) ia = q;
        if (pos_s[q] == b) ib = q;
      }
      if (ia < 0) {
        pos_s[m] = a;
        from_s[m] = a;
        ia = m++;
      }
      if (ib < 0) {
        pos_s[m] = b;
        from_s[m] = b;
        ib = m++;
      }
      const int t = from_s[ia];
      from_s[ia] = from_s[ib];
      from_s[ib] = t;
    }
    for (int q = 0; q < m; ++q) src[pos_s[q]] = from_s[q];
  }
}

// next[i, j] for j outside the panel: 64 x 64 tiles, one 16-row band per
// wave, 16 x 16 x 4 FP64 MFMA (lane l holds A[l % 16][l / 16], B[l / 16][l % 16]
// and, in accumulator register e = 0..3, D[4 e + l / 16][l % 16])
__global__ __launch_bounds__(256) void k_bgj_update(int n, int k0, const double *__restrict__ cur,
                                                    double *__restrict__ next, const int *__restrict__ src) {
  const int w = min(kGjPanel, n - k0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * 64 + wave * 16, col0 = blockIdx.x * 64;
  const int lr = lane & 15, lk = lane >> 4;
  // A operand: panel rows of this band (already in the exchanged order)
  double a[kGjPanel / 4];
#pragma unroll
  for (int kk = 0; kk < kGjPanel / 4; ++kk) {
    const int c = 4 * kk + lk, i = row0 + lr;
    a[kk] = (c < w && i < n) ? next[(size_t)i * n + k0 + c] : 0.0;
  }
  // B operand rows: cur at the source rows of the panel rows
  int srck[kGjPanel / 4];
#pragma unroll
  for (int kk = 0; kk < kGjPanel / 4; ++kk) {
    const int c = 4 * kk + lk;
    srck[kk] = c < w ? src[k0 + c] : 0;
  }
  f64x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = col0 + 16 * t + lr;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = row0 + 4 * e + lk;
      acc[t][e] = (i < n && j < n && (i < k0 || i >= k0 + w)) ? cur[(size_t)src[i] * n + j] : 0.0;
    }
  }
#pragma unroll
  for (int kk = 0; kk < kGjPanel / 4; ++kk) {
    const int c = 4 * kk + lk;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = col0 + 16 * t + lr;
      const double b = (c < w && j < n) ? cur[(size_t)srck[kk] * n + j] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = col0 + 16 * t + lr;
    if (j >= n || (j >= k0 && j < k0 + w)) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = row0 + 4 * e + lk;
      if (i < n) next[(size_t)i * n + j] = acc[t][e];
    }
  }
}

// column order of the inverse: the row exchanges replayed, in reverse, on
// an index array (one workgroup; the array in LDS)
__global__ __launch_bounds__(256) void k_bgj_order(int n, const int *__restrict__ piv, int *__restrict__ idx) {
  __shared__ int ix[kGjMaxN];
  for (int j = threadIdx.x; j < n; j += 256) ix[j] = j;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = n - 1; k >= 0; --k) {
      const int r = piv[k];
      const int t = ix[k];
      ix[k] = ix[r];
      ix[r] = t;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += 256) idx[j] = ix[j];
}

__global__ void k_bgj_gather(int n, const double *__restrict__ M, const int *__restrict__ idx,
                             double *__restrict__ Ainv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  Ainv[(size_t)i * n + j] = M[(size_t)i * n + idx[j]];
}
}  // namespace

hipError_t launch_schur_build(int n, int ns, const int *st_i, const double *st_w,
                              const double *ds, const double *lgf, double *S, hipStream_t s) {
  hipLaunchKernelGGL(k_schur_build, dim3((ns + 255) / 256, ns), dim3(256), 0, s, n, ns, st_i, st_w,
                     ds, lgf, S);
  return hipGetLastError();
}

static gpf_status invert_blocked(int n, const double *A, double *Ainv, hipStream_t s, DevBuf &pval) {
  DevBuf W0, W1, src, piv, idx;
  gpf_status st;
  const size_t mb = (size_t)n * n * sizeof(double);
  if ((st = W0.alloc(mb)) != GPF_OK) return st;
  if ((st = W1.alloc(mb)) != GPF_OK) return st;
  if ((st = src.alloc((size_t)n * sizeof(int))) != GPF_OK) return st;
  if ((st = piv.alloc((size_t)n * sizeof(int))) != GPF_OK) return st;
  if ((st = idx.alloc((size_t)n * sizeof(int))) != GPF_OK) return st;
  if ((st = pval.alloc((size_t)n * sizeof(double))) != GPF_OK) return st;
  const int R = (n + kGjThreads - 1) / kGjThreads;
  const dim3 gu((n + 63) / 64, (n + 63) / 64);
  const double *cur = A;
  double *next = W0.as<double>();
  for (int k0 = 0; k0 < n; k0 += kGjPanel) {
    if (R <= 1)
      hipLaunchKernelGGL(k_bgj_panel<1>, dim3(1), dim3(kGjThreads), 0, s, n, k0, cur, next, src.as<int>(),
                         piv.as<int>(), pval.as<double>());
    else if (R == 2)
      hipLaunchKernelGGL(k_bgj_panel<2>, dim3(1), dim3(kGjThreads), 0, s, n, k0, cur, next, src.as<int>(),
                         piv.as<int>(), pval.as<double>());
    else
      hipLaunchKernelGGL(k_bgj_panel<4>, dim3(1), dim3(kGjThreads), 0, s, n, k0, cur, next, src.as<int>(),
                         piv.as<int>(), pval.as<double>());
    hipLaunchKernelGGL(k_bgj_update, gu, dim3(256), 0, s, n, k0, cur, next, src.as<int>());
    cur = next;
    next = next == W0.as<double>() ? W1.as<double>() : W0.as<double>();
  }
  hipLaunchKernelGGL(k_bgj_order, dim3(1), dim3(256), 0, s, n, piv.as<int>(), idx.as<int>());
  hipLaunchKernelGGL(k_bgj_gather, dim3((n + 255) / 256, n), dim3(256), 0, s, n, cur, idx.as<int>(), Ainv);
  GPF_HIP(hipGetLastError());
  GPF_HIP(hipStreamSynchronize(s));   // the work buffers are freed on return
  return GPF_OK;
}

gpf_status invert_fp64(int ns, double *A, double *Ainv, hipStream_t s, double *min_pivot_rel) {
  if (ns <= kGjMaxN) {
    DevBuf pval;
    GPF_TRY(invert_blocked(ns, A, Ainv, s, pval));
    std::vector<double> hp(ns), ha((size_t)ns * ns);
    GPF_HIP(hipMemcpyAsync(hp.data(), pval.p, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    GPF_HIP(hipMemcpyAsync(ha.data(), A, (size_t)ns * ns * sizeof(double), hipMemcpyDeviceToHost, s));
    GPF_HIP(hipStreamSynchronize(s));
    double amax = 0.0, pmin = 1e300;
    for (double v : ha) amax = std::max(amax, std::fabs(v));
    for (double v : hp) pmin = std::min(pmin, std::fabs(v));
    *min_pivot_rel = amax > 0.0 ? pmin / amax : 0.0;
    return GPF_OK;
  }
  // larger systems: Gauss-Jordan on [A | I], two launches per column
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

hipError_t launch_impulse(const ProbDesc *d, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_impulse, dim3(1, nb), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_gemv_t(int ns, const double *A, const double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv_t, dim3((ns + 255) / 256), dim3(256), 0, s, ns, A, x, y);
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

hipError_t launch_schur_gemm(const ProbDesc *d, int nb, int ns, int m_max, const double *sinv,
                             hipStream_t s) {
  const int cols = nb * (1 + m_max);
  hipLaunchKernelGGL(k_schur_gemm, dim3((ns + 15) / 16, (cols + 15) / 16), dim3(256), 0, s, d, nb,
                     1 + m_max, ns, sinv);
  return hipGetLastError();
}

template <class T>
hipError_t launch_schur_apply(const ProbDesc *d, int nb, int ns_max, int m_max, hipStream_t s) {
  // one row per wave unless that makes more than 2048 workgroups
  const int narrow = (ns_max + 3) / 4;
  if ((long)narrow * nb <= 2048) {
    const dim3 grid(narrow, nb);
    if (m_max <= 2)
      hipLaunchKernelGGL((k_schur_apply<T, 3, 1>), grid, dim3(kCB), 0, s, d);
    else
      hipLaunchKernelGGL((k_schur_apply<T, kMaxCol, 1>), grid, dim3(kCB), 0, s, d);
  } else {
    const dim3 grid((ns_max + 15) / 16, nb);
    if (m_max <= 2)
      hipLaunchKernelGGL((k_schur_apply<T, 3, 4>), grid, dim3(kCB), 0, s, d);
    else
      hipLaunchKernelGGL((k_schur_apply<T, kMaxCol, 4>), grid, dim3(kCB), 0, s, d);
  }
  timer_end(s);
  return hipGetLastError();
}
template hipError_t launch_schur_apply<float>(const ProbDesc *, int, int, int, hipStream_t);
template hipError_t launch_schur_apply<double>(const ProbDesc *, int, int, int, hipStream_t);

template <class T>
hipError_t launch_schur_apply_parts(const ProbDesc *d, int nb, int ns_max, hipStream_t s) {
  hipLaunchKernelGGL((k_schur_apply_parts<T>), dim3((ns_max + kCRows - 1) / kCRows, nb), dim3(kCB),
                     0, s, d);
  timer_end(s);
  return hipGetLastError();
}
template hipError_t launch_schur_apply_parts<float>(const ProbDesc *, int, int, hipStream_t);
template hipError_t launch_schur_apply_parts<double>(const ProbDesc *, int, int, hipStream_t);

hipError_t launch_rs_apply(const ProbDesc *d, int nb, int blocks, hipStream_t s, const FlatMap *fm) {
  if (fm ? fm->total <= 0 : blocks <= 0) return hipSuccess;
  const dim3 grid = fm ? dim3(fm->total) : dim3(blocks, nb);
  hipLaunchKernelGGL(k_rs_apply, grid, dim3(256), 0, s, d, fm ? *fm : FlatMap{nullptr, 0, 0});
  return hipGetLastError();
}

}  // namespace gpf
