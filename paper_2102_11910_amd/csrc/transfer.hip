// Regularization and interpolation between Lagrangian points and grid nodes.
//
// * R_v (Sec. 2.1, eq. vortexregularization): w += Gamma_q / dx^2 times the
//   tensor product of M4' weights on the 4 x 4 nodes around the vortex.
// * E_v (Sec. 2.1): the same weights applied to node velocities, which are
//   centred differences of s (face velocities of the discrete curl averaged
//   to nodes).
// * R_s, E_s (Sec. 2.2.1): smoothed 3-point kernel; R_s = dx^-2 E_s^T diag(dS).
//
// Cell indices and fractions are computed in FP64 from FP64 positions, then
// the weights are rounded to the field type.  Stencils that would leave the
// window are skipped and reported in the device status word.
#include <algorithm>

#include "gpf_internal.h"
#include "weights.h"

namespace gpf {
namespace {



// base node (lowest stencil index) and fraction; true if [lo, hi) holds xi
__device__ __forceinline__ bool cell(double p, double o, double dx, int lo, int hi,
                                     int *base, double *frac) {
  const double xi = (p - o) / dx;
  if (!(xi >= (double)lo && xi < (double)hi)) return false;  // also rejects NaN
  const double fl = floor(xi);
  *base = (int)fl - 1;
  *frac = xi - fl;
  return true;
}


constexpr int kScatterBlock = 256;
static_assert(kPartStride * kScatterBlock == kMaxVortices, "one partial per bin_count workgroup");

__global__ void k_fill(unsigned *p, size_t words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------------------
// R_v by tiles of ts x ts cells.  The vortices are counted and sorted by the
// tile of their cell floor(xi); a vortex's 4 x 4 stencil (nodes floor(xi)-1
// .. floor(xi)+2) then reaches only its own tile and the eight around it.
// A workgroup takes one item of a work list (a tile, or up to kTileChunk
// records of a dense tile), sums its stencils in an LDS window around the
// tile in 64-bit fixed point with a per-problem power-of-two scale (no sum
// can overflow, and the window's sums do not depend on the order of the
// additions), and stores the tile's own nodes into the field and the
// others into the tile's halo slot; the windows of a dense tile's items
// are summed by a second kernel.
// ---------------------------------------------------------------------------
__host__ __device__ inline int tile_cells(int n) { return n <= 32 ? n : 32; }
constexpr int kMaxTiles = 4096;
constexpr int kMaxTileCells = 32;

// log2 of a power of two
__device__ __forceinline__ int ilog2(int x) { return 31 - __clz(x); }
// grid sizes are powers of two, so are ts and n / ts: shifts, not divisions
__device__ __forceinline__ int vortex_tile(int i0, int j0, int ts, int tps) {
  const int sh = ilog2(ts);
  return ((j0 + 1) >> sh) * tps + ((i0 + 1) >> sh);
}

// 1. count vortices per tile.  A workgroup histograms its 256 PER vortices
//    in LDS, then adds each non-empty bin to the global count once; a
//    vortex's rank in its tile = the workgroup's offset for the tile + its
//    rank within the workgroup.  Each workgroup also stores its partial
//    circulation, the moments of the circulation and the partial sum of
//    |Gamma|, summed per thread in vortex order, then across the workgroup
//    in a fixed order.
template <int PER>
__device__ __forceinline__ void bin_count_body(const ProbDesc &P, int blk, int *hist,
                                               double (*red)[kScatterBlock / 64]) {
  const int n = P.n, ts = tile_cells(n), tps = n / ts, ntiles = tps * tps;
  for (int t = threadIdx.x; t < ntiles; t += kScatterBlock) hist[t] = 0;
  // every load first; a thread past the last vortex reads the last one again
  // and counts nothing
  const int base = blk * kScatterBlock * PER + threadIdx.x;
  double xs[PER], ys[PER], gs[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int q = min(base + k * kScatterBlock, P.nv - 1);
    xs[k] = P.xv[q];
    ys[k] = P.yv[q];
    gs[k] = P.gv[q];
  }
  __syncthreads();
  int tile[PER], lrank[PER];
  double mom[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    tile[k] = -1;
    lrank[k] = 0;
    if (base + k * kScatterBlock >= P.nv) continue;
    int i0, j0;
    double fx, fy;
    if (cell(xs[k], P.x0, P.dx, 2, n - 3, &i0, &fx) && cell(ys[k], P.y0, P.dx, 2, n - 3, &j0, &fy)) {
      // circulation and its first and second moments (the impulse of the
      // vortices: the M4' weights reproduce x, y and x^2 + y^2 exactly), and
      // sum |Gamma| for the fixed-point scale
      const double g = gs[k], x = xs[k], y = ys[k];
      mom[0] += g;
      mom[1] += g * x;
      mom[2] += g * y;
      mom[3] += g * (x * x + y * y);
      mom[4] += fabs(g);
      tile[k] = vortex_tile(i0, j0, ts, tps);
      lrank[k] = atomicAdd(hist + tile[k], 1);
    } else {
      atomicOr(P.status, GPF_DEV_OUT_OF_GRID);
    }
  }
  __syncthreads();
  {
    // the atomics of one thread are independent: issue them all before
    // using the results
    constexpr int kPer = kMaxTiles / kScatterBlock;
    int ret[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int t = threadIdx.x + k * kScatterBlock;
      const int c = t < ntiles ? hist[t] : 0;
      ret[k] = c ? atomicAdd(P.bin_cnt + t, c) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int t = threadIdx.x + k * kScatterBlock;
      if (t < ntiles) hist[t] = ret[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int q = base + k * kScatterBlock;
    if (q < P.nv) P.rank[q] = tile[k] >= 0 ? hist[tile[k]] + lrank[k] : -1;
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mom[c] += __shfl_xor(mom[c], off);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < 5; ++c) red[c][threadIdx.x >> 6] = mom[c];
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double s = 0.0;
    for (int w = 0; w < kScatterBlock / 64; ++w) s += red[threadIdx.x][w];
    P.partials[(size_t)threadIdx.x * kPartStride + blk] = s;
  }
}

__global__ __launch_bounds__(kScatterBlock) void k_bin_count(const ProbDesc *__restrict__ d, FlatMap fm) {
  __shared__ int hist[kMaxTiles];
  __shared__ double red[5][kScatterBlock / 64];
  FlatBlock fb;
  if (!flat_block(fm, &fb)) return;
  const ProbDesc &P = d[fb.prob];
  // workgroups past this problem's vortices (a 2-D grid covers the largest
  // problem of the launch) have nothing to do
  if (P.nv <= 0 || fb.blk >= bin_count_blocks(P.nv)) return;
  switch (bin_per_thread(P.nv)) {
    case 1: bin_count_body<1>(P, fb.blk, hist, red); break;
    case 2: bin_count_body<2>(P, fb.blk, hist, red); break;
    case 4: bin_count_body<4>(P, fb.blk, hist, red); break;
    default: bin_count_body<8>(P, fb.blk, hist, red); break;
  }
}

// 2. tile starts, work list, scalars and the records, in one kernel: every
//    workgroup of a problem scans the tile counts (at most kMaxTiles) in
//    LDS for the starts its vortices need; workgroup 0 also writes the
//    starts, the work list of the tile kernels, the circulation and sum
//    |Gamma| (partials summed in a fixed order, so every solve gives the
//    same bits) and the fixed-point scale.  Each vortex goes to slot
//    start + rank of the tile-sorted list as (xi, eta, Gamma / dx^2, q):
//    32 bytes, the vortex's own index last (the tile velocity kernel writes
//    its result there).  A vortex outside the window (already reported)
//    gets no record and NaN velocities.
constexpr int kPlacePer = 4;                               // vortices per thread
constexpr int kPlaceBlock = kPlacePer * kScatterBlock;     // vortices per workgroup
__global__ __launch_bounds__(kScatterBlock) void k_bin_place(const ProbDesc *__restrict__ d, FlatMap fm) {
  __shared__ int start_s[kMaxTiles];
  __shared__ int wsum[kScatterBlock / 64], wsum2[kScatterBlock / 64];
  __shared__ double gsum[2][kScatterBlock / 64];
  FlatBlock fb;
  if (!flat_block(fm, &fb)) return;
  const ProbDesc &P = d[fb.prob];
  const bool lead = fb.blk == 0;
  if (!lead && fb.blk * kPlaceBlock >= P.nv) return;   // no vortex of its own to place
  const int n = P.n, ts = tile_cells(n), tps = n / ts, ntiles = tps * tps;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int kPer = kMaxTiles / kScatterBlock;
  const int per = (ntiles + kScatterBlock - 1) / kScatterBlock;
  const int lo = tid * per;
  int cnts[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) cnts[k] = (k < per && lo + k < ntiles) ? P.bin_cnt[lo + k] : 0;
  int run = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) run += cnts[k];
  int incl = run;   // inclusive scan of the run totals: waves, then across waves
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wsum[wave] = incl;
  // circulation and sum |Gamma| over the bin_count partials, strided per
  // thread, then waves, in a fixed order
  double g = 0.0, ga = 0.0;
  const int nvb = lead && P.nv > 0 ? bin_count_blocks(P.nv) : 0;   // workgroups of bin_count
  for (int b = tid; b < nvb; b += kScatterBlock) {
    g += P.partials[b];
    ga += P.partials[4 * (size_t)kPartStride + b];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    g += __shfl_xor(g, off);
    ga += __shfl_xor(ga, off);
  }
  if (lane == 0) {
    gsum[0][wave] = g;
    gsum[1][wave] = ga;
  }
  __syncthreads();
  int pos = incl - run, total = 0;
#pragma unroll
  for (int w = 0; w < kScatterBlock / 64; ++w) {
    if (w < wave) pos += wsum[w];
    total += wsum[w];
  }
  const int pos0 = pos;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (k < per && lo + k < ntiles) {
      start_s[lo + k] = pos;
      if (lead) P.bin_start[lo + k] = pos;
      pos += cnts[k];
    }
  }
  if (lead) {
    // work list of the tile kernels, in tile order: a tile of c records
    // gives ceil(c / kTileChunk) items of consecutive records, an empty tile
    // one empty item (which clears the tile's halo slot).  A tile of
    // several items goes on the split list with the first of its items'
    // window slots.
    auto parts_of = [&](int k) {
      return k < per && lo + k < ntiles ? max(1, (cnts[k] + kTileChunk - 1) / kTileChunk) : 0;
    };
    // items; split tiles (low 16 bits) and their items (high bits): both
    // below 2^15 (tiles + nv / kTileChunk, split_items_max)
    int ni = 0, sp = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int q = parts_of(k);
      ni += q;
      if (q > 1) sp += 1 + (q << 16);
    }
    int a = ni, b = sp;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int va = __shfl_up(a, off), vb = __shfl_up(b, off);
      if (lane >= off) {
        a += va;
        b += vb;
      }
    }
    __syncthreads();   // wsum is reused
    if (lane == 63) {
      wsum[wave] = a;
      wsum2[wave] = b;
    }
    __syncthreads();
    int at = a - ni, sat = b - sp, tot_items = 0, tot_sp = 0;
#pragma unroll
    for (int w = 0; w < kScatterBlock / 64; ++w) {
      if (w < wave) {
        at += wsum[w];
        sat += wsum2[w];
      }
      tot_items += wsum[w];
      tot_sp += wsum2[w];
    }
    int stile = sat & 0xffff, slot = sat >> 16;
    int r = pos0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int parts = parts_of(k), c = cnts[k];
      // last field: 0 the tile's only item, else 1 + the item's window slot
      for (int j = 0; j < parts; ++j) {
        const int4 it = make_int4(lo + k, r + j * kTileChunk, min(r + c, r + (j + 1) * kTileChunk),
                                  parts > 1 ? 1 + slot + j : 0);
        *reinterpret_cast<int4 *>(P.items + 4 * (1 + at++)) = it;
      }
      if (parts > 1) {
        *reinterpret_cast<int4 *>(P.splits + 4 * (1 + stile++)) = make_int4(lo + k, slot, parts, 0);
        slot += parts;
      }
      r += c;
    }
    if (tid == 0) {
      *reinterpret_cast<int4 *>(P.splits) = make_int4(tot_sp & 0xffff, 0, 0, 0);
      *reinterpret_cast<int4 *>(P.items) = make_int4(tot_items, 0, 0, 0);
      P.bin_start[ntiles] = total;
      double gw = 0.0, gabs = 0.0;
      for (int w = 0; w < kScatterBlock / 64; ++w) {
        gw += gsum[0][w];
        gabs += gsum[1][w];
      }
      P.aux[SC_GAMMA_W] = gw;
      if (P.sc_out) P.sc_out[SC_GAMMA_W] = gw;
      // no node sum exceeds sum |Gamma| / dx^2 (each 1-D weight is at most 1
      // in magnitude); the sums are scaled to below 2^B (FixedPoint<T>)
      const double smax = gabs / (P.dx * P.dx);
      int e = 0;
      if (smax > 0.0) {
        frexp(smax, &e);   // smax < 2^e
      }
      P.aux[SC_RV_SCALE] = (double)e;   // sum |Gamma| / dx^2 < 2^e
    }
  }
  __syncthreads();   // start_s is complete
  // kPlacePer vortices per thread, all loads issued first
  const int *__restrict__ rank = P.rank;
  const double *__restrict__ xv = P.xv;
  const double *__restrict__ yv = P.yv;
  const double *__restrict__ gv = P.gv;
  double *__restrict__ sorted = P.sorted;
  const double inv_dx2 = 1.0 / (P.dx * P.dx);
  for (int q0 = fb.blk * kPlaceBlock + tid; q0 < P.nv; q0 += fb.nblk * kPlaceBlock) {
    int rk[kPlacePer];
    double x[kPlacePer], y[kPlacePer], gq[kPlacePer];
#pragma unroll
    for (int u = 0; u < kPlacePer; ++u) {
      const int q = min(q0 + u * kScatterBlock, P.nv - 1);
      rk[u] = rank[q];
      x[u] = xv[q];
      y[u] = yv[q];
      gq[u] = gv[q];
    }
#pragma unroll
    for (int u = 0; u < kPlacePer; ++u) {
      const int q = q0 + u * kScatterBlock;
      if (q >= P.nv) break;
      if (rk[u] < 0) {
        if (P.u) {
          P.u[q] = NAN;
          P.v[q] = NAN;
        }
        continue;
      }
      const double xi = (x[u] - P.x0) / P.dx, eta = (y[u] - P.y0) / P.dx;
      const int t = vortex_tile((int)floor(xi) - 1, (int)floor(eta) - 1, ts, tps);
      double4 o;
      o.x = xi;
      o.y = eta;
      o.z = gq[u] * inv_dx2;
      o.w = (double)q;
      *reinterpret_cast<double4 *>(sorted + 4 * (size_t)(start_s[t] + rk[u])) = o;
    }
  }
}

// 3. one workgroup per item of the work list (a tile, or a part of a dense
//    tile's records): the item's vortices add their 4 x 4 stencils to an
//    LDS window of (ts+3)^2 nodes (nodes X0-1 .. X0+ts+1) in 64-bit fixed
//    point, so the window's sums do not depend on the order of the
//    additions.  The tile's own ts^2 nodes (window-local 1 .. ts) are then
//    stored into the field (zero, or the values to add to); the other
//    6 ts + 9 window nodes belong to neighbouring tiles and are stored in
//    the tile's halo slot, which the convolutions (or step 4) add to their
//    owners.  A dense tile's workgroup takes its records kTileChunk at a
//    time into the same window: no global atomic, and the field is the same
//    bits on every run.  The tile's count is cleared for the next solve.
// 4. one workgroup per tile whose neighbours' windows can reach it: each of
//    its 6 ts - 9 border nodes (local 0, 1 or ts-1 on an axis) adds, in a
//    fixed order, the halo values of the non-empty neighbours that reach it.
constexpr int kTileBlock = 128;
static_assert(kTileChunk % kTileBlock == 0, "an item's records are a whole number per thread");

// index in a tile's halo slot of window node (kx, ky), a node outside the
// tile's own 1 .. ts range on some axis: the row ky = 0, the rows ts+1 and
// ts+2, then columns 0, ts+1 and ts+2 of rows 1 .. ts
__device__ __forceinline__ int halo_index(int kx, int ky, int ts) {
  const int bw = ts + 3;
  if (ky == 0) return kx;
  if (ky > ts) return bw + (ky - ts - 1) * bw + kx;
  return 3 * bw + (ky - 1) * 3 + (kx == 0 ? 0 : kx - ts);
}

// Workgroup barrier that orders LDS accesses only: global stores and atomics
// issued before it stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
constexpr int kMaxWin = (kMaxTileCells + 3) * (kMaxTileCells + 3);

// Fixed point of the window sums: terms scaled to below 2^B in magnitude.
// FP32 fields: B = 50, where one add of 1.5 * 2^52 rounds a term to an
// integer in its low mantissa bits (exact below 2^51), a resolution of
// 2^-50 of the largest possible sum, far below the FP32 rounding of the
// field.  FP64 fields: B = 61 and the exact double -> int64 conversion.
template <class T> struct FixedPoint;
template <> struct FixedPoint<float> {
  static constexpr int B = 50;
  static __device__ __forceinline__ long long to_int(double x) {
    const double t = x + 6755399441055744.0;   // 1.5 * 2^52
    return __double_as_longlong(t) - 0x4338000000000000LL;
  }
};
template <> struct FixedPoint<double> {
  static constexpr int B = 61;
  static __device__ __forceinline__ long long to_int(double x) { return __double2ll_rn(x); }
};

// A tile's summed window (fixed point; value_at(u, k) is node k, the u-th
// of this thread): its own nodes go to the field (zero, or the values to
// add to), the others to the tile's halo slot (every entry, zeros included)
constexpr int kWinPer = (kSplitWin + kTileBlock - 1) / kTileBlock;   // nodes per thread
// UNROLLED: the loop over a thread's nodes is unrolled (value_at may then
// index registers by u); otherwise u is 0
template <class T, bool UNROLLED, class F>
__device__ __forceinline__ void store_tile_window(const ProbDesc &P, int t, int ts, int tps, int X0,
                                                  int Y0, double inv, F value_at) {
  const int n = P.n, bw = ts + 3, nwin = bw * bw;
  T *w = static_cast<T *>(P.w);
  T *hal = static_cast<T *>(P.halo) + (size_t)t * kHaloRing;
  auto store = [&](long long v, int k) {
    const int kx = k % bw, ky = k / bw;
    const T val = (T)((double)v * inv);
    if (kx >= 1 && kx <= ts && ky >= 1 && ky <= ts) {
      if (v == 0) return;
      T *node = w + (size_t)(Y0 + ky) * n + X0 + kx;
      *node = P.w_accumulate ? *node + val : val;
    } else {
      hal[halo_index(kx, ky, ts)] = val;
    }
  };
  if constexpr (UNROLLED) {
#pragma unroll
    for (int u = 0; u < kWinPer; ++u) {
      const int k = threadIdx.x + u * kTileBlock;
      if (k < nwin) store(value_at(u, k), k);
    }
  } else {
    for (int k = threadIdx.x; k < nwin; k += kTileBlock) store(value_at(0, k), k);
  }
}

// store_tile_window for 32-cell tiles and a window in LDS: the own nodes by
// rows of 32 (one line of the field each), then the halo ring decoded in
// its own order (window row 0, rows 33 and 34, then columns 0, 33 and 34
// of rows 1 .. 32), without a division by the window width per entry
template <class T>
__device__ __forceinline__ void store_window32(const ProbDesc &P, int t, int X0, int Y0, double inv,
                                               const long long *win) {
  constexpr int bw = 32 + 3;
  const int n = P.n;
  T *w = static_cast<T *>(P.w);
  T *hal = static_cast<T *>(P.halo) + (size_t)t * kHaloRing;
  for (int e = threadIdx.x; e < 32 * 32; e += kTileBlock) {
    const int r = e >> 5, c = e & 31;
    const long long v = win[(r + 1) * bw + c + 1];
    if (v == 0) continue;
    const T val = (T)((double)v * inv);
    T *node = w + (size_t)(Y0 + 1 + r) * n + X0 + 1 + c;
    *node = P.w_accumulate ? *node + val : val;
  }
  for (int h = threadIdx.x; h < kHaloRing; h += kTileBlock) {
    int kx, ky;
    if (h < 3 * bw) {
      const int row = h / bw;   // 0, 1, 2: window rows 0, 33, 34
      ky = row == 0 ? 0 : 32 + row;
      kx = h - row * bw;
    } else {
      const int q = h - 3 * bw, c = q % 3;
      ky = 1 + q / 3;
      kx = c == 0 ? 0 : 32 + c;
    }
    hal[h] = (T)((double)win[ky * bw + kx] * inv);
  }
}

// TS: the tile size when it is known at compile time (32, every grid of
// n >= 32), 0 otherwise: the window loops then divide by constants
template <class T, int TS>
__device__ __forceinline__ void tile_scatter_body(const ProbDesc &P, const FlatBlock &fb,
                                                  long long *win) {
  const int cnt = P.items[0];
  if (fb.blk >= cnt) return;
  const int n = P.n, ts = TS ? TS : tile_cells(n), tps = n / ts, tpsh = ilog2(tps);
  const int tid = threadIdx.x;
  const int bw = ts + 3, nwin = bw * bw;
  const int sexp = FixedPoint<T>::B - (int)P.aux[SC_RV_SCALE];
  const double scale = ldexp(1.0, sexp), inv = ldexp(1.0, -sexp);
  T *halo = static_cast<T *>(P.halo);
  // one item per workgroup when the launch covers the work list (it is
  // sized for the most items a problem can have)
  for (int i = fb.blk; i < cnt; i += fb.nblk) {
    const int4 it = *reinterpret_cast<const int4 *>(P.items + 4 * (1 + i));
    const int t = it.x, b0 = it.y, b1 = it.z;
    if (b0 == b1) {
      // a tile without vortices: its halo slot holds zeros for the readers
      // that add every neighbour's slot (the LDS window is not touched)
      T *hal = halo + (size_t)t * kHaloRing;
      for (int k = tid; k < kHaloRing; k += kTileBlock) hal[k] = (T)0;
      continue;
    }
    const int X0 = (t & (tps - 1)) * ts - 1, Y0 = (t >> tpsh) * ts - 1;   // window origin
    // the item's records (at most kTileChunk), loaded before the window is
    // cleared; clamped duplicates past the end add zero
    constexpr int kPer = kTileChunk / kTileBlock;
    double rec[kPer][3];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int k = b0 + j * kTileBlock + tid;
      const double *r = P.sorted + 4 * (size_t)min(k, b1 - 1);
      rec[j][0] = r[0];
      rec[j][1] = r[1];
      rec[j][2] = k < b1 ? r[2] : 0.0;
    }
    for (int k = tid; k < nwin; k += kTileBlock) win[k] = 0;
    lds_barrier();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      if (b0 + j * kTileBlock + tid >= b1) continue;
      const double xi = rec[j][0], eta = rec[j][1], amp = rec[j][2] * scale;
      const double flx = floor(xi), fly = floor(eta);
      const double fx = xi - flx, fy = eta - fly;
      double wx[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) wx[a] = m4p(fx + 1.0 - a);
      long long *row = win + ((int)fly - 1 - Y0) * bw + ((int)flx - 1 - X0);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double ab = amp * m4p(fy + 1.0 - b);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const long long v = FixedPoint<T>::to_int(ab * wx[a]);
          if (v != 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(row + b * bw + a), (unsigned long long)v);
        }
      }
    }
    lds_barrier();
    if (it.w == 0) {
      if (tid == 0) P.bin_cnt[t] = 0;
      if constexpr (TS == 32)
        store_window32<T>(P, t, X0, Y0, inv, win);
      else
        store_tile_window<T, false>(P, t, ts, tps, X0, Y0, inv, [&](int, int k) { return win[k]; });
    } else {
      // an item of a split tile: its window goes to its own slot, and
      // k_split_combine stores the tile's sum after this launch
      long long *mine = P.splitwin + (size_t)(it.w - 1) * kSplitWin;
      for (int k = tid; k < nwin; k += kTileBlock) mine[k] = win[k];
    }
    if (i + fb.nblk < cnt) lds_barrier();   // the window is cleared for the next item
  }
}

template <class T>
__global__ __launch_bounds__(kTileBlock) void k_tile_scatter(const ProbDesc *__restrict__ d, FlatMap fm) {
  __shared__ long long win[kMaxWin];
  FlatBlock fb;
  if (!flat_block(fm, &fb)) return;
  const ProbDesc &P = d[fb.prob];
  if (tile_cells(P.n) == 32)
    tile_scatter_body<T, 32>(P, fb, win);
  else
    tile_scatter_body<T, 0>(P, fb, win);
}

// 3b. one workgroup per tile of several items (after the tile kernel): the
//     items' windows summed in integers (exact, so neither the order nor
//     the split changes a bit), stored as a lone item's window would be
template <class T>
__device__ __forceinline__ void split_combine_body(const ProbDesc &P, const FlatBlock &fb) {
  const int nsplit = P.splits[0];
  const int n = P.n, ts = tile_cells(n), tps = n / ts;
  const double inv = ldexp(1.0, (int)P.aux[SC_RV_SCALE] - FixedPoint<T>::B);
  for (int e = fb.blk; e < nsplit; e += fb.nblk) {
    const int4 sp = *reinterpret_cast<const int4 *>(P.splits + 4 * (1 + e));
    const int t = sp.x, parts = sp.z;
    const long long *win = P.splitwin + (size_t)sp.y * kSplitWin;
    const int X0 = (t % tps) * ts - 1, Y0 = (t / tps) * ts - 1;
    // each thread's nodes summed part by part: the loads of one part are
    // issued together
    long long acc[kWinPer];
#pragma unroll
    for (int u = 0; u < kWinPer; ++u) acc[u] = 0;
    for (int q = 0; q < parts; ++q) {
      const long long *wq = win + (size_t)q * kSplitWin;
#pragma unroll
      for (int u = 0; u < kWinPer; ++u) {
        const int k = threadIdx.x + u * kTileBlock;
        acc[u] += k < kSplitWin ? wq[k] : 0;
      }
    }
    store_tile_window<T, true>(P, t, ts, tps, X0, Y0, inv, [&](int u, int) { return acc[u]; });
    if (threadIdx.x == 0) P.bin_cnt[t] = 0;
  }
}

__global__ __launch_bounds__(kTileBlock) void k_split_combine(const ProbDesc *__restrict__ d, FlatMap fm) {
  FlatBlock fb;
  if (!flat_block(fm, &fb)) return;
  const ProbDesc &P = d[fb.prob];
  if (P.nv <= 0) return;
  if (P.w64)
    split_combine_body<double>(P, fb);
  else
    split_combine_body<float>(P, fb);
}

// 4.: kFixupTiles tiles per workgroup, a few border nodes per thread; every
// load a node needs (the neighbours' tile counts, their halo entries, the
// node) is issued before any is used, and a neighbour without vortices
// (whose halo slot holds nothing of this solve) is dropped by a select.
constexpr int kFixupBlock = 256;
constexpr int kFixupTiles = 4;
constexpr int kBorderNodes = 6 * 32 - 9;   // of a 32 x 32 tile
constexpr int kFixupPer = (kFixupTiles * kBorderNodes + kFixupBlock - 1) / kFixupBlock;

template <class T>
__global__ __launch_bounds__(kFixupBlock) void k_halo_fixup(const ProbDesc *__restrict__ d, FlatMap fm) {
  FlatBlock fb;
  if (!flat_block(fm, &fb)) return;
  const ProbDesc &P = d[fb.prob];
  const int n = P.n, ts = tile_cells(n), tps = n / ts, ntiles = tps * tps;
  if (tps < 2 || P.nv <= 0 || P.halo_defer) return;
  const T *__restrict__ halo = static_cast<const T *>(P.halo);
  const int *__restrict__ start = P.bin_start;
  T *w = static_cast<T *>(P.w);
  size_t at[kFixupPer];
  T own[kFixupPer], h[kFixupPer][3];
  bool ok[kFixupPer], valid[kFixupPer][3];
#pragma unroll
  for (int u = 0; u < kFixupPer; ++u) {
    const int e = threadIdx.x + u * kFixupBlock;
    const int t = fb.blk * kFixupTiles + e / kBorderNodes, i = e % kBorderNodes;
    ok[u] = e < kFixupTiles * kBorderNodes && t < ntiles;
    // border node i of tile t: rows 0, 1 and ts-1, then columns 0, 1 and
    // ts-1 of rows 2 .. ts-2
    int lx, ly;
    if (i < 3 * ts) {
      const int r = i / ts;
      ly = r < 2 ? r : ts - 1;
      lx = i % ts;
    } else {
      const int j = i - 3 * ts, c = j % 3;
      ly = 2 + j / 3;
      lx = c < 2 ? c : ts - 1;
    }
    const int tc = ok[u] ? t : 0;
    const int tx = tc % tps, ty = tc / tps;
    const int x = tx * ts + lx, y = ty * ts + ly;
    at[u] = (size_t)y * n + x;
    own[u] = ok[u] ? w[at[u]] : (T)0;
    // the (up to three) neighbours whose windows reach the node: the
    // left/lower ones reach local 0 and 1, the right/upper ones local ts-1
    const int sx = lx <= 1 ? -1 : (lx == ts - 1 ? 1 : 0);
    const int sy = ly <= 1 ? -1 : (ly == ts - 1 ? 1 : 0);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int dx = q == 1 ? 0 : sx, dy = q == 0 ? 0 : sy;   // (sx,0), (0,sy), (sx,sy)
      const int nx = tx + dx, ny = ty + dy;
      valid[u][q] = ok[u] && (dx != 0 || dy != 0) && !(q == 2 && (dx == 0 || dy == 0)) &&
                    nx >= 0 && nx < tps && ny >= 0 && ny < tps;
      const int nt = valid[u][q] ? ny * tps + nx : 0;
      const int kx = x - (nx * ts - 1), ky = y - (ny * ts - 1);
      h[u][q] = valid[u][q] ? halo[(size_t)nt * kHaloRing + halo_index(kx, ky, ts)] : (T)0;
      // a neighbour without vortices wrote no halo: its count decides
      valid[u][q] = valid[u][q] && start[nt + 1] != start[nt];
    }
  }
#pragma unroll
  for (int u = 0; u < kFixupPer; ++u) {
    if (!(valid[u][0] || valid[u][1] || valid[u][2])) continue;
    T add = (T)0;
#pragma unroll
    for (int q = 0; q < 3; ++q) add += valid[u][q] ? h[u][q] : (T)0;
    w[at[u]] = own[u] + add;
  }
}

__global__ void k_surface_stencils(int n, double dx, double x0, double y0, int ns,
                                   const double *__restrict__ xs, const double *__restrict__ ys,
                                   int *__restrict__ st_i, double *__restrict__ st_w,
                                   unsigned *__restrict__ status) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  int i0, j0;
  double fx, fy;
  const bool okx = cell(xs[p], x0, dx, 1, n - 2, &i0, &fx);
  const bool oky = cell(ys[p], y0, dx, 1, n - 2, &j0, &fy);
  if (!(okx && oky)) {
    atomicOr(status, GPF_DEV_OUT_OF_GRID);
    i0 = j0 = 1;
    fx = fy = 0.0;
  }
  st_i[2 * p] = i0;
  st_i[2 * p + 1] = j0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    st_w[8 * p + a] = yang3(fx + 1.0 - a);
    st_w[8 * p + 4 + a] = yang3(fy + 1.0 - a);
  }
}

template <class T>
__global__ void k_interp_surface(int n, int ns, const int *__restrict__ st_i,
                                 const double *__restrict__ st_w, const T *__restrict__ f,
                                 double *__restrict__ r) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const int i0 = st_i[2 * p], j0 = st_i[2 * p + 1];
  double acc = 0.0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double rowacc = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
      rowacc += st_w[8 * p + a] * (double)f[(size_t)(j0 + b) * n + i0 + a];
    acc += st_w[8 * p + 4 + b] * rowacc;
  }
  r[p] = acc;
}

// Unit sheets for a column-by-column Schur build: field b of the batch gets
// R_s e_q, q = q0 + b, i.e. dS_q / dx^2 times the 4 x 4 stencil weights of
// surface point q (distinct nodes: plain stores into a zeroed field).
template <class T>
__global__ void k_unit_sheets(int n, int ns, int q0, double inv_dx2, const int *__restrict__ st_i,
                              const double *__restrict__ st_w, const double *__restrict__ ds,
                              T *w, size_t stride) {
  const int q = q0 + blockIdx.x;
  if (q >= ns || threadIdx.x >= 16) return;
  const int a = threadIdx.x & 3, b = threadIdx.x >> 2;
  const int i0 = st_i[2 * q], j0 = st_i[2 * q + 1];
  w[stride * blockIdx.x + (size_t)(j0 + b) * n + i0 + a] =
      (T)(ds[q] * inv_dx2 * st_w[8 * q + a] * st_w[8 * q + 4 + b]);
}

// E_s of field b of the batch at every surface point, into column q0 + b of
// the row-major ns x ns matrix S
template <class T>
__global__ void k_interp_columns(int n, int ns, int q0, const int *__restrict__ st_i,
                                 const double *__restrict__ st_w, const T *__restrict__ f,
                                 size_t stride, double *__restrict__ S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = q0 + blockIdx.y;
  if (p >= ns || q >= ns) return;
  const T *fb = f + stride * blockIdx.y;
  const int i0 = st_i[2 * p], j0 = st_i[2 * p + 1];
  double acc = 0.0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double rowacc = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
      rowacc += st_w[8 * p + a] * (double)fb[(size_t)(j0 + b) * n + i0 + a];
    acc += st_w[8 * p + 4 + b] * rowacc;
  }
  S[(size_t)p * ns + q] = acc;
}

// Velocity at a vortex (E_v of the node velocities, Sec. 2.1): the centred
// differences u = (s[j+1] - s[j-1]) / 2dx, v = -(s[i+1] - s[i-1]) / 2dx at
// the 4 x 4 stencil nodes, interpolated with M4' weights.  s points at node
// (i0 - 1, j0 - 1) of a field of row pitch `pitch`: rows j0-1 .. j0+4 and
// columns i0-1 .. i0+4 are read.
template <class T>
__device__ __forceinline__ void stencil_velocity(const T *s, int pitch, double fx, double fy,
                                                 double h, double *u, double *v) {
  double wx[4], wy[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    wx[a] = m4p(fx + 1.0 - a);
    wy[a] = m4p(fy + 1.0 - a);
  }
  double uacc = 0.0, vacc = 0.0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double ur = 0.0, vr = 0.0;
    const T *rm = s + (size_t)b * pitch;   // row j0+b-1
    const T *rc = rm + pitch;              // row j0+b
    const T *rp = rc + pitch;              // row j0+b+1
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ur += wx[a] * ((double)rp[a + 1] - (double)rm[a + 1]);
      vr += wx[a] * ((double)rc[a + 2] - (double)rc[a]);
    }
    uacc += wy[b] * ur;
    vacc += wy[b] * vr;
  }
  *u = uacc * h;
  *v = -vacc * h;
}

// Velocities of the binned vortices tile by tile, for dense clouds (at
// least one vortex per four nodes; the vortex-by-vortex kernel's 36
// scattered loads per vortex then cost more than loading the field once):
// a workgroup takes one item of the work list, loads the window of s its
// tile's vortices read (nodes X0-2 .. X0+ts+3 on each axis: the 4 x 4
// stencil of a vortex in the tile, plus the one-node halo of the centred
// differences) into LDS with row-wise coalesced loads, then every vortex of
// the item forms its velocity from LDS and writes it at its own index.
constexpr int kVelWin = kMaxTileCells + 6;

template <class T, int TS>
__device__ __forceinline__ void tile_velocity_body(const ProbDesc &P, const FlatBlock &fb, T *win) {
  const int cnt = P.items[0];
  if (fb.blk >= cnt) return;
  const int n = P.n, ts = TS ? TS : tile_cells(n), tps = n / ts, tpsh = ilog2(tps);
  const int tid = threadIdx.x;
  const int bw = ts + 6, nwin = bw * bw;
  const T *s = static_cast<const T *>(P.psi);
  const double h = 0.5 / P.dx;
  const double ui = P.psi_total ? 0.0 : P.sv.u_inf, vi = P.psi_total ? 0.0 : P.sv.v_inf;
  constexpr int kPer = kTileChunk / kTileBlock;
  for (int i = fb.blk; i < cnt; i += fb.nblk) {
    const int4 it = *reinterpret_cast<const int4 *>(P.items + 4 * (1 + i));
    const int t = it.x, b0 = it.y, b1 = it.z;
    if (b0 == b1) continue;   // an empty tile's item
    const int X0 = (t & (tps - 1)) * ts - 2, Y0 = (t >> tpsh) * ts - 2;   // window origin
    double4 rec[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j)
      rec[j] = *reinterpret_cast<const double4 *>(P.sorted + 4 * (size_t)min(b0 + j * kTileBlock + tid, b1 - 1));
    for (int k = tid; k < nwin; k += kTileBlock) {
      const int gx = X0 + k % bw, gy = Y0 + k / bw;
      win[k] = (gx >= 0 && gx < n && gy >= 0 && gy < n) ? s[(size_t)gy * n + gx] : (T)0;
    }
    lds_barrier();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      if (b0 + j * kTileBlock + tid >= b1) continue;
      const double flx = floor(rec[j].x), fly = floor(rec[j].y);
      // rows j0-1 .. j0+4, columns i0-1 .. i0+4 of s, i0 = floor(xi) - 1
      double u, v;
      stencil_velocity(win + ((int)fly - 2 - Y0) * bw + ((int)flx - 2 - X0), bw, rec[j].x - flx,
                       rec[j].y - fly, h, &u, &v);
      const int q = (int)rec[j].w;
      P.u[q] = u + ui;
      P.v[q] = v + vi;
    }
    if (i + fb.nblk < cnt) lds_barrier();   // the window is reloaded for the next item
  }
}

template <class T>
__global__ __launch_bounds__(kTileBlock) void k_tile_velocity(const ProbDesc *__restrict__ d, FlatMap fm) {
  __shared__ T win[kVelWin * kVelWin];
  FlatBlock fb;
  if (!flat_block(fm, &fb)) return;
  const ProbDesc &P = d[fb.prob];
  if (P.u == nullptr || !P.vel_tiles) return;
  if (tile_cells(P.n) == 32)
    tile_velocity_body<T, 32>(P, fb, win);
  else
    tile_velocity_body<T, 0>(P, fb, win);
}

// Velocities vortex by vortex, reading s from global memory.  After R_v of
// the same solve (from_records) the threads take the tile-sorted records, so
// neighbouring threads read neighbouring rows of s; the records hold only
// vortices inside the window (the others got NaN velocities when sorted).
// Otherwise they take the vortices in input order and check the window.
template <class T>
__global__ __launch_bounds__(256) void k_vortex_velocity(const ProbDesc *__restrict__ d, FlatMap fm,
                                                         int from_records) {
  FlatBlock fb;
  if (!flat_block(fm, &fb)) return;
  const ProbDesc &P = d[fb.prob];
  if (P.u == nullptr || P.vel_tiles) return;
  const int n = P.n;
  const int k = fb.blk * blockDim.x + threadIdx.x;
  int i0, j0, q;
  double fx, fy;
  if (from_records) {
    const int ts = tile_cells(n), tps = n / ts;
    if (k >= P.bin_start[tps * tps]) return;
    const double4 rec = *reinterpret_cast<const double4 *>(P.sorted + 4 * (size_t)k);
    const double flx = floor(rec.x), fly = floor(rec.y);
    i0 = (int)flx - 1;
    j0 = (int)fly - 1;
    fx = rec.x - flx;
    fy = rec.y - fly;
    q = (int)rec.w;
  } else {
    q = k;
    if (q >= P.nv) return;
    if (!(cell(P.xv[q], P.x0, P.dx, 2, n - 3, &i0, &fx) &&
          cell(P.yv[q], P.y0, P.dx, 2, n - 3, &j0, &fy))) {
      atomicOr(P.status, GPF_DEV_OUT_OF_GRID);
      P.u[q] = NAN;
      P.v[q] = NAN;
      return;
    }
  }
  double u, v;
  stencil_velocity(static_cast<const T *>(P.psi) + (size_t)(j0 - 1) * n + (i0 - 1), n, fx, fy,
                   0.5 / P.dx, &u, &v);
  const double ui = P.psi_total ? 0.0 : P.sv.u_inf, vi = P.psi_total ? 0.0 : P.sv.v_inf;
  P.u[q] = u + ui;
  P.v[q] = v + vi;
}

__global__ void k_axpy2(int nv, const double *__restrict__ x, const double *__restrict__ y,
                        const double *__restrict__ u, const double *__restrict__ v, double a,
                        double *xo, double *yo) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nv) return;
  xo[q] = x[q] + a * u[q];
  yo[q] = y[q] + a * v[q];
}

// Shedding step, before the solve: new vortex j goes one third of the way
// from edge point e_j to the last vortex that edge released (Sec. 2.4.2),
// or to e_j + first_j before the first release; appended with strength 0.
__global__ void k_shed_place(ShedGeom sg, int nv, const int *__restrict__ last, double *x,
                             double *y, double *g) {
  const int j = threadIdx.x;
  if (j >= sg.m) return;
  const int l = last[j];
  double zx, zy;
  if (l >= 0) {
    zx = sg.ex[j] + (x[l] - sg.ex[j]) / 3.0;
    zy = sg.ey[j] + (y[l] - sg.ey[j]) / 3.0;
  } else {
    zx = sg.ex[j] + sg.fx[j];
    zy = sg.ey[j] + sg.fy[j];
  }
  x[nv + j] = zx;
  y[nv + j] = zy;
  g[nv + j] = 0.0;
}

// Shedding step, after the solve: the new vortices (the last m of nv) take
// their strengths from the scalar block; an edge that shed a nonzero
// strength records its new vortex as its last release; with several parts
// each part's released circulation grows by its edges' strengths (one lane,
// in edge order); every vortex moves by forward Euler.
__global__ void k_shed_advance(ShedGeom sg, int nv, const double *__restrict__ sc, int *last,
                               double *gw, double *x, double *y, double *g,
                               const double *__restrict__ u, const double *__restrict__ v,
                               double dt) {
  const int m = sg.m;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) {
    const double gj = sc[SC_GAMMA_NEW + q];
    g[nv - m + q] = gj;
    if (gj != 0.0) last[q] = nv - m + q;
  }
  if (gw && q == 0) {
    for (int j = 0; j < m; ++j) gw[sg.epart[j]] += sc[SC_GAMMA_NEW + j];
  }
  if (q < nv) {
    x[q] += dt * u[q];
    y[q] += dt * v[q];
  }
}

}  // namespace

hipError_t launch_shed_place(const ShedGeom &sg, int nv, const int *last, double *x, double *y,
                             double *g, hipStream_t s) {
  hipLaunchKernelGGL(k_shed_place, dim3(1), dim3(64), 0, s, sg, nv, last, x, y, g);
  return hipGetLastError();
}

hipError_t launch_shed_advance(const ShedGeom &sg, int nv, const double *sc, int *last, double *gw,
                               double *x, double *y, double *g, const double *u, const double *v,
                               double dt, hipStream_t s) {
  hipLaunchKernelGGL(k_shed_advance, dim3((nv + 255) / 256), dim3(256), 0, s, sg, nv, sc, last, gw,
                     x, y, g, u, v, dt);
  return hipGetLastError();
}

hipError_t launch_axpy2(int nv, const double *x, const double *y, const double *u,
                        const double *v, double a, double *xo, double *yo, hipStream_t s) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy2, dim3((nv + 255) / 256), dim3(256), 0, s, nv, x, y, u, v, a, xo, yo);
  return hipGetLastError();
}

int scatter_blocks(int nv_max) { return nv_max > 0 ? (nv_max + kScatterBlock - 1) / kScatterBlock : 1; }

int place_blocks(int nv) { return nv > 0 ? (nv + kPlaceBlock - 1) / kPlaceBlock : 1; }

hipError_t launch_fill(void *p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  int blocks = (int)std::min<size_t>((words + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, static_cast<unsigned *>(p), words);
  return hipGetLastError();
}

int bin_tiles(int n) {
  const int ts = tile_cells(n);
  return (n / ts) * (n / ts);
}

int halo_tiles(int n) { return bin_tiles(n) > 1 ? bin_tiles(n) : 0; }

int fixup_blocks(int n) { return (halo_tiles(n) + kFixupTiles - 1) / kFixupTiles; }

// items of a problem: one per tile plus one per further kTileChunk records
// of a tile (sum over tiles of floor((c - 1) / kTileChunk) <= nv / kTileChunk)
int tile_items_max(int n, int nv) { return nv > 0 ? bin_tiles(n) + nv / kTileChunk : 0; }

int split_blocks(int nv) { return std::min(64, split_tiles_max(nv)); }

// grid of a launch: the flat map's blocks, or nb problems of `per` blocks
static dim3 grid_of(const FlatMap *fm, int per, int nb) {
  return fm ? dim3(std::max(1, fm->total)) : dim3(std::max(1, per), nb);
}

template <class T>
hipError_t launch_scatter_vortices(const ProbDesc *d, int nb, int n, int nv_max, hipStream_t s,
                                   const FlatMap *fm, bool halo_pass) {
  timer_begin(GPF_TK_SCATTER, s);
  const FlatMap none{nullptr, 0, 0};
  const FlatMap mb = fm ? fm[0] : none, mt = fm ? fm[1] : none, mh = fm ? fm[2] : none;
  const FlatMap mp = fm ? fm[3] : none;
  // the count's workgroups take up to 2048 vortices (bin_per_thread); the
  // place kernel one per thread
  const int cb = nv_max > 0 ? bin_count_blocks(nv_max) : 1, vb = place_blocks(nv_max);
  hipLaunchKernelGGL(k_bin_count, grid_of(fm ? &mb : nullptr, cb, nb), dim3(kScatterBlock), 0, s, d, mb);
  hipLaunchKernelGGL(k_bin_place, grid_of(fm ? &mp : nullptr, vb, nb), dim3(kScatterBlock), 0, s, d, mp);
  // one workgroup per item of the work list, then one per tile for the halos
  hipLaunchKernelGGL((k_tile_scatter<T>), grid_of(fm ? &mt : nullptr, tile_items_max(n, nv_max), nb),
                     dim3(kTileBlock), 0, s, d, mt);
  // tiles of several items: their windows summed after the tile kernel
  if (fm ? fm[4].total > 0 : split_blocks(nv_max) > 0) {
    const hipError_t e = launch_split_combine(d, nb, split_blocks(nv_max), s, fm ? &fm[4] : nullptr);
    if (e != hipSuccess) return e;
  }
  if (fm ? mh.total > 0 : (halo_pass && nv_max > 0 && halo_tiles(n) > 0))
    hipLaunchKernelGGL((k_halo_fixup<T>), grid_of(fm ? &mh : nullptr, fixup_blocks(n), nb), dim3(kFixupBlock),
                       0, s, d, mh);
  timer_end(s);
  return hipGetLastError();
}
template hipError_t launch_scatter_vortices<float>(const ProbDesc *, int, int, int, hipStream_t,
                                                   const FlatMap *, bool);
template hipError_t launch_scatter_vortices<double>(const ProbDesc *, int, int, int, hipStream_t,
                                                    const FlatMap *, bool);

hipError_t launch_split_combine(const ProbDesc *d, int nb, int blocks, hipStream_t s, const FlatMap *fm) {
  if (fm ? fm->total <= 0 : blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split_combine, grid_of(fm, blocks, nb), dim3(kTileBlock), 0, s, d,
                     fm ? *fm : FlatMap{nullptr, 0, 0});
  return hipGetLastError();
}

hipError_t launch_surface_stencils(int n, double dx, double x0, double y0, int ns,
                                   const double *xs, const double *ys, int *st_i, double *st_w,
                                   unsigned *status, hipStream_t s) {
  hipLaunchKernelGGL(k_surface_stencils, dim3((ns + 127) / 128), dim3(128), 0, s, n, dx, x0, y0,
                     ns, xs, ys, st_i, st_w, status);
  return hipGetLastError();
}

template <class T>
hipError_t launch_interp_surface(int n, int ns, const int *st_i, const double *st_w,
                                 const T *field, double *r, hipStream_t s) {
  hipLaunchKernelGGL((k_interp_surface<T>), dim3((ns + 127) / 128), dim3(128), 0, s, n, ns,
                     st_i, st_w, field, r);
  return hipGetLastError();
}
template hipError_t launch_interp_surface<float>(int, int, const int *, const double *,
                                                 const float *, double *, hipStream_t);
template hipError_t launch_interp_surface<double>(int, int, const int *, const double *,
                                                  const double *, double *, hipStream_t);

template <class T>
hipError_t launch_unit_sheets(int n, int ns, int q0, int nb, double dx, const int *st_i,
                              const double *st_w, const double *ds, T *w, size_t stride,
                              hipStream_t s) {
  hipLaunchKernelGGL((k_unit_sheets<T>), dim3(nb), dim3(64), 0, s, n, ns, q0, 1.0 / (dx * dx), st_i,
                     st_w, ds, w, stride);
  return hipGetLastError();
}
template hipError_t launch_unit_sheets<float>(int, int, int, int, double, const int *,
                                              const double *, const double *, float *, size_t,
                                              hipStream_t);
template hipError_t launch_unit_sheets<double>(int, int, int, int, double, const int *,
                                               const double *, const double *, double *, size_t,
                                               hipStream_t);

template <class T>
hipError_t launch_interp_columns(int n, int ns, int q0, int nb, const int *st_i,
                                 const double *st_w, const T *f, size_t stride, double *S,
                                 hipStream_t s) {
  hipLaunchKernelGGL((k_interp_columns<T>), dim3((ns + 127) / 128, nb), dim3(128), 0, s, n, ns, q0,
                     st_i, st_w, f, stride, S);
  return hipGetLastError();
}
template hipError_t launch_interp_columns<float>(int, int, int, int, const int *, const double *,
                                                 const float *, size_t, double *, hipStream_t);
template hipError_t launch_interp_columns<double>(int, int, int, int, const int *, const double *,
                                                  const double *, size_t, double *, hipStream_t);

template <class T>
hipError_t launch_solve_velocity(const ProbDesc *d, int nb, int n, int nv_max, hipStream_t s,
                                 const FlatMap *fm, int kinds) {
  if (nv_max <= 0) return hipSuccess;
  timer_begin(GPF_TK_VELOCITY, s);
  const FlatMap none{nullptr, 0, 0};
  const FlatMap mg = fm ? fm[0] : none, mt = fm ? fm[1] : none;
  if (fm ? mg.total > 0 : (kinds & 1) != 0)
    hipLaunchKernelGGL((k_vortex_velocity<T>), grid_of(fm ? &mg : nullptr, (nv_max + 255) / 256, nb),
                       dim3(256), 0, s, d, mg, 1);
  if (fm ? mt.total > 0 : (kinds & 2) != 0)
    hipLaunchKernelGGL((k_tile_velocity<T>), grid_of(fm ? &mt : nullptr, tile_items_max(n, nv_max), nb),
                       dim3(kTileBlock), 0, s, d, mt);
  timer_end(s);
  return hipGetLastError();
}
template hipError_t launch_solve_velocity<float>(const ProbDesc *, int, int, int, hipStream_t,
                                                 const FlatMap *, int);
template hipError_t launch_solve_velocity<double>(const ProbDesc *, int, int, int, hipStream_t,
                                                  const FlatMap *, int);

template <class T>
hipError_t launch_vortex_velocity(const ProbDesc *d, int nb, int nv_max, hipStream_t s) {
  if (nv_max <= 0) return hipSuccess;
  timer_begin(GPF_TK_VELOCITY, s);
  hipLaunchKernelGGL((k_vortex_velocity<T>), dim3((nv_max + 255) / 256, nb), dim3(256), 0, s, d,
                     FlatMap{nullptr, 0, 0}, 0);
  timer_end(s);
  return hipGetLastError();
}
template hipError_t launch_vortex_velocity<float>(const ProbDesc *, int, int, hipStream_t);
template hipError_t launch_vortex_velocity<double>(const ProbDesc *, int, int, hipStream_t);

}  // namespace gpf
