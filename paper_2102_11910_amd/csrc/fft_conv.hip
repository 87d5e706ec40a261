// Zero-padded lattice-Green's-function convolution s = -L^-1 w on gfx950.
//
// The particular solution of the unbounded discrete Poisson problem
// (Sec. 2.1, eq. poisson) is s = -dx^2 (G * w) over the infinite lattice.
// For w supported on the n x n window this equals the circular convolution
// of the zero-padded (2n)^2 source with the even kernel
// K(i,j) = G(min(i,2n-i), min(j,2n-j)), whose 2-D DFT is real.
//
// Three passes, N = 2n:
//   1. rows:    two real rows packed as one complex sequence, length-N FFT
//               (upper half of the input is zero), unpacked into the two
//               half spectra and stored k-major: X[k1][j], k1 in [0, n].
//   2. columns: per k1, length-N FFT of X[k1][0..n) (upper half zero),
//               times the real spectrum, inverse FFT, first n outputs kept.
//   3. rows:    two half spectra packed as one Hermitian-pair sequence,
//               inverse FFT, first n outputs of each row kept, minus the
//               exact gauge term c * gamma_src.
// The spectrum already holds -dx^2/N^2 and the gauge shift by c.
//
// FFT core: a group of N/16 lanes owns one sequence in LDS; every stage is a
// Stockham radix-R step (R = 16 except a last 2/4/8 step), each lane doing
// 16/R butterflies with its values in registers.  LDS rows are padded by one
// element every 16 to spread the strided stores over the banks.
#include <algorithm>
#include <type_traits>

#include "gpf_internal.h"

namespace gpf {
namespace {

template <class T> struct CT;
template <> struct CT<float> { using V = float2; using V2 = float4; };
template <> struct CT<double> { using V = double2; using V2 = double4; };

template <class V> __device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// a * b + c, rounded once
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <class V> __device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <class V> __device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }

// cos / sin of 2 pi k / 16, k = 0..7
__device__ constexpr double kC16[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                       0.38268343236508977173, 0.0, -0.38268343236508977173,
                                       -0.70710678118654752440, -0.92387953251128675613};
__device__ constexpr double kS16[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                                       0.92387953251128675613, 1.0, 0.92387953251128675613,
                                       0.70710678118654752440, 0.38268343236508977173};

template <int R> __host__ __device__ constexpr int bitrev(int x) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}

// In-register R-point DFT (natural order in and out), radix-2 DIT network.
// INV selects the e^{+i} kernel (unnormalized).
template <int R, bool INV, class V>
__device__ __forceinline__ void dft_reg(V *v) {
  using S = decltype(v[0].x);
  V t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[bitrev<R>(i)] = v[i];
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) {
        const int idx = k * (16 / len);
        V b = t[i + k + len / 2];
        if (idx == 4) {  // multiply by -i (forward) or +i (inverse)
          V r;
          if (INV) { r.x = -b.y; r.y = b.x; } else { r.x = b.y; r.y = -b.x; }
          b = r;
        } else if (idx != 0) {
          // a +- b w with w = (c, s) in the fused multiply-add form of
          // Linzer and Feig: b w = m (b.x - t b.y, b.y + t b.x) with m = c,
          // t = s / c where |c| >= |s|, else m = s, t = c / s and
          // b w = m (t b.x - b.y, t b.y + b.x); |t| <= 1 either way.  Six
          // FMAs per butterfly instead of a complex product and four adds.
          const double cw = kC16[idx], sw = INV ? kS16[idx] : -kS16[idx];
          const V a = t[i + k];
          S bx, by, m;
          if (__builtin_fabs(cw) >= __builtin_fabs(sw)) {
            const S tn = (S)(sw / cw);
            m = (S)cw;
            bx = fmad(-tn, b.y, b.x);
            by = fmad(tn, b.x, b.y);
          } else {
            const S tn = (S)(cw / sw);
            m = (S)sw;
            bx = fmad(tn, b.x, -b.y);
            by = fmad(tn, b.y, b.x);
          }
          t[i + k].x = fmad(m, bx, a.x);
          t[i + k].y = fmad(m, by, a.y);
          t[i + k + len / 2].x = fmad(-m, bx, a.x);
          t[i + k + len / 2].y = fmad(-m, by, a.y);
          continue;
        }
        V a = t[i + k];
        t[i + k] = cadd(a, b);
        t[i + k + len / 2] = csub(a, b);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = t[i];
}

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

constexpr int kE = 16;  // values per lane

template <int N> struct Plan {
  static constexpr int TPS = N / kE;          // lanes per sequence
  static constexpr int SEQ = N <= 256 ? 8 : (N == 512 ? 4 : (N <= 2048 ? 2 : 1));
  static constexpr int WGT = TPS * SEQ;        // threads per workgroup
  static constexpr int LDS_SEQ = N + N / 16;   // padded elements per sequence
};

// Row passes: a workgroup holds 2 SEQ rows, so each k-major row of the
// intermediate is touched in runs of 2 SEQ elements; the wide SEQ gives
// 128-byte runs within about 72 KB of LDS (two workgroups per CU).
// The wide shape suits launches with many row blocks (batches); single
// problems and row-pruned passes keep the narrow shape for more workgroups.
// Shapes of a pass: narrow and wide as above; multi = the 256-thread
// workgroup of the launches that cover problems of several grid sizes at once
// (N / 16 lanes per sequence, 4096 / N sequences: the same LDS footprint for
// every N).
constexpr int kNarrow = 0, kWide = 1, kMulti = 2;
constexpr int kMultiThreads = 256;

template <class T, int N, int SH> struct RowPlan {
  static constexpr int TPS = N / kE;
  static constexpr int LDS_SEQ = N + N / 16;
  static constexpr int ELEM = 2 * (int)sizeof(T);
  static constexpr int fit(int s) {
    while (s > 1 && s * LDS_SEQ * ELEM > 72 * 1024) s /= 2;
    return s;
  }
  static constexpr int SEQ = SH == kMulti ? kMultiThreads / TPS
                                          : (SH == kWide ? fit(64 / ELEM) : Plan<N>::SEQ);
  static constexpr int WGT = TPS * SEQ;
  // a workgroup's run of each k-major row fills whole 128-byte lines
  static constexpr bool FULL_LINES = 2 * SEQ * ELEM >= 128;
};

// radix of stage `s` for a length-N transform with 16 values per lane
template <int N> __host__ __device__ constexpr int stage_radix(int s) {
  int rem = N, r = 16;
  for (int i = 0; i <= s; ++i) {
    r = rem >= 16 ? 16 : rem;
    if (i < s) rem /= r;
  }
  return r;
}
template <int N> __host__ __device__ constexpr int num_stages() {
  int rem = N, s = 0;
  while (rem > 1) {
    rem /= (rem >= 16 ? 16 : rem);
    ++s;
  }
  return s;
}
// stride NS of stage s (product of the earlier radices)
template <int N> __host__ __device__ constexpr int stage_ns(int s) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= stage_radix<N>(i);
  return ns;
}
// base twiddles a lane keeps for stages before s (stage 0 needs none): the
// R-1 factors of its first butterfly.  Only a last stage has more than one
// butterfly per lane, and there butterfly b sits at j + b N/16, so its
// factors are the base ones times 16th roots of unity.
template <int N> __host__ __device__ constexpr int tw_before(int s) {
  int c = 0;
  for (int i = 1; i < s; ++i) c += stage_radix<N>(i) - 1;
  return c;
}
template <int N> __host__ __device__ constexpr int tw_regs() {
  return tw_before<N>(num_stages<N>()) > 0 ? tw_before<N>(num_stages<N>()) : 1;
}

// Twiddles in registers for FP32 transforms up to N = 1024, where the
// kernel's occupancy is bounded by LDS anyway.  FP64 transforms (and larger
// ones) read the table instead; FP64 forms the factors of a butterfly as
// powers of its first one (one table load, and the products of at most 15
// factors stay within a few ulps), which keeps its register count, and with
// it the occupancy of the FP64 passes, down.
template <class T, int N> __host__ __device__ constexpr bool tw_in_regs() {
  return N <= 4096 && !std::is_same<T, double>::value;
}

// x_r *= w^r (r = 1..R-1) for w the first twiddle of the butterfly
template <int R, class V>
__device__ __forceinline__ void twiddle_powers(V (&v)[R], V w1) {
  V w = w1;
#pragma unroll
  for (int r = 1; r < R; ++r) {
    v[r] = cmul(v[r], w);
    if (r + 1 < R) w = cmul(w, w1);
  }
}

// Every twiddle factor a lane uses, loaded once at kernel start (the loads
// overlap the data loads instead of waiting behind each stage's barrier);
// inverse transforms use their conjugates.
template <class T, int N, int S>
__device__ __forceinline__ void load_twiddles(typename CT<T>::V (&wr)[tw_regs<N>()],
                                              const typename CT<T>::V *tw, int lane) {
  if constexpr (S < num_stages<N>()) {
    if constexpr (S >= 1) {
      constexpr int R = stage_radix<N>(S), NS = stage_ns<N>(S), OFF = tw_before<N>(S);
      const int j = lane % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) wr[OFF + r - 1] = tw[j * r * (N / (NS * R))];
    }
    load_twiddles<T, N, S + 1>(wr, tw, lane);
  }
}

// w * exp(-+2 pi i k / 16); k is a constant once the callers' loops unroll
template <bool INV, class V> __device__ __forceinline__ V rot16(V w, int k) {
  using S = decltype(w.x);
  k &= 15;
  if (k == 0) return w;
  V c;
  c.x = (S)(k < 8 ? kC16[k] : -kC16[k - 8]);
  const S sn = (S)(k < 8 ? kS16[k] : -kS16[k - 8]);
  c.y = INV ? sn : -sn;
  return cmul(w, c);
}

// Exchange barrier of one sequence.  Where a sequence lies inside one
// wavefront (N / 16 <= 64 lanes) and no other wavefront touches its LDS rows,
// the wavefront orders its own LDS traffic (its LDS instructions execute in
// order), so only the compiler must keep the order: a wavefront-scope fence,
// with no wait for the stores and no workgroup barrier.
template <bool WAVE>
__device__ __forceinline__ void seq_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// One Stockham stage.  Lane `lane` of the group owning a sequence handles
// butterflies bf = lane + b * TPS (b < 16/R), each reading elements
// bf + r * N/R and writing base + r * NS.  With IN_REGS the stage reads its
// 16 values from x[] instead of LDS, where x[k] holds element lane + k * TPS
// (the stage-0 layout, radix 16).  With OUT_REGS the results stay in x[],
// again as x[k] = element lane + k * TPS: in the last stage the butterfly
// b, output r lands at lane + TPS * (b + r * 16/R).
template <class T, int N, int S, bool INV, bool ZERO_UPPER, bool LOWER_OUT, bool IN_REGS,
          bool OUT_REGS, bool WAVE>
__device__ __forceinline__ void fft_stage(typename CT<T>::V (&x)[kE], typename CT<T>::V *lds,
                                          const typename CT<T>::V (&wr)[tw_regs<N>()],
                                          const typename CT<T>::V *tw, int lane) {
  using V = typename CT<T>::V;
  constexpr int TPS = N / kE;
  constexpr int R = stage_radix<N>(S), NS = stage_ns<N>(S);
  constexpr int NB = kE / R;   // butterflies per lane
  static_assert(!IN_REGS || R == kE, "register input needs a radix-16 first stage");
  static_assert(NB == 1 || (S == num_stages<N>() - 1 && NS * R == N),
                "several butterflies per lane only in a last stage");
  V v[NB][R];
  if (IN_REGS) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (ZERO_UPPER && r >= R / 2) {
        v[0][r].x = (T)0;
        v[0][r].y = (T)0;
      } else {
        v[0][r] = x[r];
      }
    }
  } else {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int bf = lane + b * TPS;
      const int pbf = pad(bf);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (ZERO_UPPER && r >= R / 2) {
          v[b][r].x = (T)0;
          v[b][r].y = (T)0;
        } else if constexpr ((N / R) % 16 == 0) {
          v[b][r] = lds[pbf + r * (N / R) + r * (N / R) / 16];
        } else {
          v[b][r] = lds[pad(bf + r * (N / R))];
        }
      }
    }
    seq_sync<WAVE>();
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int bf = lane + b * TPS;
    const int j = bf % NS;
    if (NS > 1) {
      if constexpr (!tw_in_regs<T, N>() && std::is_same<T, double>::value) {
        V w1 = tw[j * (N / (NS * R))];
        if (INV) w1.y = -w1.y;
        twiddle_powers<R>(v[b], w1);
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V w;
          if constexpr (tw_in_regs<T, N>()) {
            w = wr[tw_before<N>(S) + r - 1];
            if (INV) w.y = -w.y;
            if (NB > 1) w = rot16<INV>(w, b * r);   // butterfly b sits at j + b N/16
          } else {
            w = tw[j * r * (N / (NS * R))];
            if (INV) w.y = -w.y;
          }
          v[b][r] = cmul(v[b][r], w);
        }
      }
    }
    dft_reg<R, INV>(v[b]);
    if (OUT_REGS) {
#pragma unroll
      for (int r = 0; r < R; ++r) x[b + r * NB] = v[b][r];
    } else {
      const int base = (bf / NS) * NS * R + j;
      // NS a multiple of 16: constant offsets from pad(base); NS = 1 with a
      // radix-16 step: base = 16 bf, so pad(base + r) = 17 bf + r
      const int pbase = (NS == 1 && R == 16) ? 17 * bf : pad(base);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (LOWER_OUT && r >= R / 2) continue;
        if constexpr (NS % 16 == 0) {
          lds[pbase + r * NS + r * NS / 16] = v[b][r];
        } else if constexpr (NS == 1 && R == 16) {
          lds[pbase + r] = v[b][r];
        } else {
          lds[pad(base + r * NS)] = v[b][r];
        }
      }
    }
  }
  if (!OUT_REGS) seq_sync<WAVE>();
}

template <class T, int N, int S, bool INV, bool ZIN, bool LOUT, bool IN_REGS, bool OUT_REGS,
          bool WAVE>
__device__ __forceinline__ void fft_stages(typename CT<T>::V (&x)[kE], typename CT<T>::V *lds,
                                           const typename CT<T>::V (&wr)[tw_regs<N>()],
                                           const typename CT<T>::V *tw, int lane) {
  constexpr int NST = num_stages<N>();
  if constexpr (S < NST) {
    fft_stage<T, N, S, INV, ZIN && S == 0, LOUT && S == NST - 1, IN_REGS && S == 0,
              OUT_REGS && S == NST - 1, WAVE>(x, lds, wr, tw, lane);
    fft_stages<T, N, S + 1, INV, ZIN, LOUT, IN_REGS, OUT_REGS, WAVE>(x, lds, wr, tw, lane);
  }
}

// Length-N transform of one sequence; all threads of the block must call it
// (it synchronizes the block, or with WAVE only the compiler's order: for
// callers whose sequences each lie inside one wavefront and whose LDS rows
// no other wavefront touches).  IN_REGS / OUT_REGS: input / output in x[]
// (x[k] = element lane + k * N/16), otherwise in natural order in lds.
template <class T, int N, bool INV, bool ZIN, bool LOUT, bool IN_REGS, bool OUT_REGS,
          bool WAVE = false>
__device__ __forceinline__ void fft_seq(typename CT<T>::V (&x)[kE], typename CT<T>::V *lds,
                                        const typename CT<T>::V (&wr)[tw_regs<N>()],
                                        const typename CT<T>::V *tw, int lane) {
  static_assert(!WAVE || N / kE <= 64, "a wavefront-ordered sequence fits one wavefront");
  fft_stages<T, N, 0, INV, ZIN, LOUT, IN_REGS, OUT_REGS, WAVE>(x, lds, wr, tw, lane);
}

// Row-pass block index.  Workgroups are dispatched round-robin over the
// XCDs.  remap <= 1 keeps that order, which spreads every band of rows over
// all XCDs even where some rows are empty or skipped; remap = the XCD count
// puts consecutive logical blocks on one XCD, so that workgroups whose runs
// of each k-major row share cache lines also share an L2.  The launcher
// picks it (see row_remap).
__device__ __forceinline__ int xcd_block(int remap) {
  const int nb = gridDim.x, b = blockIdx.x;
  if (remap <= 1 || nb % remap) return b;
  return (b % remap) * (nb / remap) + b / remap;
}

// ---------------------------------------------------------------------------
// pass 1: rows, real -> half spectrum, stored k-major
// ---------------------------------------------------------------------------
// R_v halos added as the source is read.  The scatter stores each 32 x 32
// cell tile's own nodes into the field and the window nodes its neighbours
// own into the tile's halo slot (a ring of kHaloRing entries: window row 0,
// rows 33 and 34, then columns 0, 33 and 34 of rows 1 .. 32; a tile without
// vortices holds zeros).  A node on a tile's columns 0, 1 (31) takes the
// left (right) neighbour's entry, a node on rows 0, 1 (31) the lower (upper)
// neighbour's, a corner node also the diagonal one's: added in that order to
// source rows ja, ja + 1 (ja even, so both lie in one tile row) at columns
// lane + k TPS.  Each part is one branch whose loads are issued together;
// a neighbour outside the grid is replaced by the own tile (a valid
// address) and its value dropped.
template <class Tin, int N>
__device__ __forceinline__ void add_halos(const Tin *__restrict__ hal, Tin (&ra)[kE / 2],
                                          Tin (&rb)[kE / 2], int ja, int lane) {
  constexpr int n = N / 2;
  if constexpr (n >= 64) {
    constexpr int TPS = N / kE, bw = 32 + 3, tps = n / 32, R = kHaloRing;
    const int ty = ja >> 5, la = ja & 31;
    bool anyc = false;
#pragma unroll
    for (int k = 0; k < kE / 2; ++k) {
      const int lx = (lane + k * TPS) & 31;
      anyc = anyc || lx <= 1 || lx == 31;
    }
    if (anyc) {
      Tin ha[kE / 2], hb[kE / 2];
      bool ok[kE / 2];
#pragma unroll
      for (int k = 0; k < kE / 2; ++k) {
        const int i = lane + k * TPS, tx = i >> 5, lx = i & 31;
        const int hx = lx <= 1 ? tx - 1 : tx + 1;
        ok[k] = (lx <= 1 || lx == 31) && hx >= 0 && hx < tps;
        // window column 33, 34 of the left neighbour, 0 of the right one
        const size_t at = (size_t)(ty * tps + (ok[k] ? hx : tx)) * R + 3 * bw + 3 * la +
                          (lx <= 1 ? lx + 1 : 0);
        ha[k] = hal[at];
        hb[k] = hal[at + 3];
      }
#pragma unroll
      for (int k = 0; k < kE / 2; ++k) {
        ra[k] += ok[k] ? ha[k] : (Tin)0;
        rb[k] += ok[k] ? hb[k] : (Tin)0;
      }
    }
    // rows 0 and 1 of a tile take window rows 33 and 34 of the lower
    // neighbour; row 31 (the second row of the pair at la = 30) window row 0
    // of the upper one.  One row at a time, to keep fewer values live.
    const bool low = la == 0 && ty > 0, up = la == 30 && ty + 1 < tps;
    if (low || up) {
      const int vy = low ? ty - 1 : ty + 1;
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) {
        if (rr == 0 && !low) continue;
        const int off = rr == 0 ? bw : (low ? 2 * bw : 0);
        Tin (&r)[kE / 2] = rr == 0 ? ra : rb;
        Tin v[kE / 2], dg[kE / 2];
        bool okd[kE / 2];
#pragma unroll
        for (int k = 0; k < kE / 2; ++k) {
          const int i = lane + k * TPS, tx = i >> 5, lx = i & 31;
          const int hx = lx <= 1 ? tx - 1 : tx + 1;
          okd[k] = (lx <= 1 || lx == 31) && hx >= 0 && hx < tps;
          v[k] = hal[(size_t)(vy * tps + tx) * R + off + lx + 1];
          dg[k] = hal[(size_t)(vy * tps + (okd[k] ? hx : tx)) * R + off + (lx <= 1 ? lx + 33 : 0)];
        }
#pragma unroll
        for (int k = 0; k < kE / 2; ++k) {
          r[k] += v[k];
          r[k] += okd[k] ? dg[k] : (Tin)0;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// row-pair block `blk` of one problem (rows 2 SEQ blk ..), LDS of SEQ rows
template <class Tin, class T, int N, int SH>
__device__ __forceinline__ void rows_fwd_body(const ConvDesc &C, int blk, int band,
                                              typename CT<T>::V *lds) {
  using V = typename CT<T>::V;
  using P = RowPlan<T, N, SH>;
  constexpr int n = N / 2;
  Tin *__restrict__ w = static_cast<Tin *>(C.in);
  V *__restrict__ X = static_cast<V *>(C.X);
  const V *__restrict__ tw = static_cast<const V *>(C.tw);
  const int tid = threadIdx.x;
  // band: the grid covers source rows fwd_lo .. fwd_hi only (the other rows
  // of X keep an earlier pass's transforms); a workgroup of more than 16
  // rows may reach past fwd_hi and neither transforms nor stores those rows
  const int lo = band ? C.fwd_lo : 0;
  const int hi_row = band ? C.fwd_hi : n - 1;
  const int j0 = lo + blk * 2 * P::SEQ;
  if (j0 > hi_row) return;

  const int q = tid / P::TPS, lane = tid % P::TPS;
  const bool live = j0 + 2 * q <= hi_row;   // this sequence's row pair is transformed
  V x[kE];
  V wr[tw_regs<N>()];
  {
    // elements lane + k * TPS of the packed row pair; k >= 8 is the zero half.
    // A sequence past the range reads the workgroup's first pair (j0 is even
    // and hi_row odd, so j0 + 1 <= hi_row) and drops it by a select: the
    // loads stay unconditional and are issued together.
    const int ja = live ? j0 + 2 * q : j0;
    const size_t row = (size_t)ja * n;
    Tin ra[kE / 2], rb[kE / 2];
#pragma unroll
    for (int k = 0; k < kE / 2; ++k) {
      ra[k] = w[row + lane + k * P::TPS];
      rb[k] = w[row + n + lane + k * P::TPS];
    }
    if (C.halo) add_halos<Tin, N>(static_cast<const Tin *>(C.halo), ra, rb, ja, lane);
#pragma unroll
    for (int k = 0; k < kE / 2; ++k) {
      x[k].x = live ? (T)ra[k] : (T)0;
      x[k].y = live ? (T)rb[k] : (T)0;
    }
  }
  // the first stage needs no twiddles: loaded after the source
  if constexpr (tw_in_regs<T, N>()) load_twiddles<T, N, 0>(wr, tw, lane);
  constexpr int RW = 2 * P::SEQ;
  // rows j0 .. j0 + nr - 1 of the workgroup are covered; nr < RW only where
  // a band ends inside the workgroup, and the guarded loops below run only
  // there
  const int nr = min(RW, hi_row - j0 + 1);
  if (C.zero_in) {
    // the source is cleared after it is read, which needs a barrier; the
    // same barrier tells whether the workgroup's rows hold anything.  Rows
    // that hold nothing (a band away from the vortices and the body)
    // transform to nothing: the workgroup then only stores zeros, and has
    // nothing to clear.  Rows keep_lo .. keep_end-1 stay for a later pass.
    bool nz = false;
#pragma unroll
    for (int k = 0; k < kE / 2; ++k) nz = nz || x[k].x != (T)0 || x[k].y != (T)0;
    if (!__syncthreads_or(nz)) {
      V zero;
      zero.x = (T)0;
      zero.y = (T)0;
      for (int idx = tid; idx < (n + 1) * RW; idx += P::WGT)
        if (idx % RW < nr) X[(size_t)(idx / RW) * n + j0 + idx % RW] = zero;
      return;
    }
    if (nr == RW && (C.keep_end <= j0 || C.keep_lo >= j0 + RW)) {
      for (int idx = tid; idx < RW * n; idx += P::WGT) w[(size_t)j0 * n + idx] = (Tin)0;
    } else {
      for (int idx = tid; idx < RW * n; idx += P::WGT) {
        const int r = j0 + idx / n;
        if (r - j0 < nr && (r < C.keep_lo || r >= C.keep_end)) w[(size_t)j0 * n + idx] = (Tin)0;
      }
    }
  }
  fft_seq<T, N, false, true, false, true, false>(x, lds + q * P::LDS_SEQ, wr, tw, lane);

  // unpack: A = (Z[k] + conj Z[N-k]) / 2, B = (Z[k] - conj Z[N-k]) / (2i)
  auto unpack = [&](int idx) {
    const int k = idx / RW, jj = idx % RW;
    const V *L = lds + (jj >> 1) * P::LDS_SEQ;
    const V zk = L[pad(k)];
    const V zm = L[pad((N - k) & (N - 1))];
    V o;
    if ((jj & 1) == 0) {
      o.x = (T)0.5 * (zk.x + zm.x);
      o.y = (T)0.5 * (zk.y - zm.y);
    } else {
      o.x = (T)0.5 * (zk.y + zm.y);
      o.y = (T)0.5 * (zm.x - zk.x);
    }
    X[(size_t)k * n + j0 + jj] = o;
  };
  if (nr == RW) {
    for (int idx = tid; idx < (n + 1) * RW; idx += P::WGT) unpack(idx);
  } else {
    for (int idx = tid; idx < (n + 1) * RW; idx += P::WGT)
      if (idx % RW < nr) unpack(idx);
  }
}

template <class Tin, class T, int N, bool WIDE>
__global__ __launch_bounds__((RowPlan<T, N, WIDE ? kWide : kNarrow>::WGT)) void k_rows_fwd(
    const ConvDesc *__restrict__ cd, int remap, int band) {
  using P = RowPlan<T, N, WIDE ? kWide : kNarrow>;
  __shared__ typename CT<T>::V lds[P::SEQ * P::LDS_SEQ];
  rows_fwd_body<Tin, T, N, WIDE ? kWide : kNarrow>(cd[blockIdx.y], xcd_block(remap), band, lds);
}

// ---------------------------------------------------------------------------
// pass 2: columns, forward FFT x spectrum x inverse FFT
// ---------------------------------------------------------------------------
// column block `blk` of one problem: columns SEQ blk .. (SEQ sequences)
template <class T, int N, int SEQ>
__device__ __forceinline__ void cols_body(const ConvDesc &C, int blk, typename CT<T>::V *lds) {
  using V = typename CT<T>::V;
  using P = Plan<N>;   // lanes per sequence and padded sequence length
  constexpr int n = N / 2;
  V *__restrict__ X = static_cast<V *>(C.X);
  const T *__restrict__ spec = static_cast<const T *>(C.spec);
  const V *__restrict__ tw = static_cast<const V *>(C.tw);
  const int tid = threadIdx.x;
  const int c0 = blk * SEQ;
  const int q = tid / P::TPS, lane = tid % P::TPS;
  const int k1 = min(c0 + q, n);   // blocks past the last column redo it and store nothing
  V *col = X + (size_t)k1 * n;
  V x[kE];
#pragma unroll
  for (int k = 0; k < kE / 2; ++k) x[k] = col[lane + k * P::TPS];
  // the spectrum row (and, when kept in registers, the twiddles) are loaded
  // up front, beside the column
  T g[kE];
  {
    // element lane + k TPS: below n for k < 8 (8 TPS = n), else mirrored;
    // at k = 8, lane 0 both forms give n
    const T *sp = spec + (size_t)k1 * (n + 1);
#pragma unroll
    for (int k = 0; k < kE; ++k) g[k] = k < kE / 2 ? sp[lane + k * P::TPS] : sp[N - lane - k * P::TPS];
  }
  V wr[tw_regs<N>()];
  if constexpr (tw_in_regs<T, N>()) load_twiddles<T, N, 0>(wr, tw, lane);
  V *L = lds + q * P::LDS_SEQ;
  // each sequence is one wavefront's (or part of one) and so are its LDS rows
  constexpr bool kWave = P::TPS <= 64;
  fft_seq<T, N, false, true, false, true, true, kWave>(x, L, wr, tw, lane);
#pragma unroll
  for (int k = 0; k < kE; ++k) {
    x[k].x *= g[k];
    x[k].y *= g[k];
  }
  fft_seq<T, N, true, false, true, true, true, kWave>(x, L, wr, tw, lane);
  if (c0 + q <= n) {
    // only the rows the last pass reads: all, unless the first convolution
    // feeds the surface stencils alone.  The last pass transforms rows in
    // pairs inside 16-row-aligned workgroups, and an unwritten (stale) partner
    // row would add its rounding noise, so whole 16-row groups are kept.
    const int lo = C.row_lo & ~15, hi = C.row_hi | 15;
    V *dst = C.Xb ? static_cast<V *>(C.Xb) + (size_t)k1 * C.band_pitch - lo : col;
#pragma unroll
    for (int k = 0; k < kE / 2; ++k) {
      const int j = lane + k * P::TPS;
      if (j >= lo && j <= hi) dst[j] = x[k];
    }
  }
}

template <class T, int N>
__global__ __launch_bounds__(Plan<N>::WGT) void k_cols_conv(const ConvDesc *__restrict__ cd) {
  using P = Plan<N>;
  __shared__ typename CT<T>::V lds[P::SEQ * P::LDS_SEQ];
  cols_body<T, N, P::SEQ>(cd[blockIdx.y], blockIdx.x, lds);
}

// FP64 column pass for N >= 1024: one sequence per workgroup (N/16 lanes)
// with the data in registers between stages; each exchange goes through LDS
// one real component at a time, so a sequence needs N + N/16 scalars of LDS
// instead of complex values, and the twiddles are powers of one table value.
// Both cut the footprint that bounds the FP64 pass's occupancy (measured on
// the 512^2 batch: 74 -> 64 us).
// one padding scalar per 16 (8 and 32 per measured slower on the 512^2 batch)
constexpr int kSplitPad = 4;
__device__ __forceinline__ int spad(int i) { return i + (i >> kSplitPad); }

template <class T, int N, int S, bool INV, bool ZIN>
__device__ __forceinline__ void split_stages(typename CT<T>::V (&x)[kE], T *lds,
                                             const typename CT<T>::V *tw, int lane) {
  using V = typename CT<T>::V;
  constexpr int NST = num_stages<N>();
  constexpr int TPS = N / kE;
  constexpr int R = stage_radix<N>(S), NS = stage_ns<N>(S), NB = kE / R;
  // x holds this stage's inputs as v[b][r] = x[b * R + r]
  V v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (ZIN && S == 0 && r >= R / 2) {
        v[b][r].x = (T)0;
        v[b][r].y = (T)0;
      } else {
        v[b][r] = x[b * R + r];
      }
    }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int bf = lane + b * TPS;
    const int j = bf % NS;
    if (NS > 1) {
      V w1 = tw[j * (N / (NS * R))];
      if (INV) w1.y = -w1.y;
      V w = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        v[b][r] = cmul(v[b][r], w);
        if (r + 1 < R) w = cmul(w, w1);
      }
    }
    dft_reg<R, INV>(v[b]);
  }
  if constexpr (S == NST - 1) {
    // last stage: butterfly b, output r is element lane + TPS (b + r NB)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) x[b + r * NB] = v[b][r];
  } else {
    constexpr int R2 = stage_radix<N>(S + 1), NB2 = kE / R2;
    // real parts, then imaginary parts: write this stage's outputs at
    // base + r NS, read the next stage's inputs bf2 + r2 N/R2
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int bf = lane + b * TPS;
        const int j = bf % NS;
        const int base = (bf / NS) * NS * R + j;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[spad(base + r * NS)] = part ? v[b][r].y : v[b][r].x;
      }
      seq_sync<(TPS <= 64)>();   // the workgroup is the sequence
#pragma unroll
      for (int b2 = 0; b2 < NB2; ++b2) {
        const int bf2 = lane + b2 * TPS;
#pragma unroll
        for (int r2 = 0; r2 < R2; ++r2) {
          const T val = lds[spad(bf2 + r2 * (N / R2))];
          if (part)
            x[b2 * R2 + r2].y = val;
          else
            x[b2 * R2 + r2].x = val;
        }
      }
      seq_sync<(TPS <= 64)>();
    }
    split_stages<T, N, S + 1, INV, ZIN>(x, lds, tw, lane);
  }
}

template <class T, int N>
__global__ __launch_bounds__(N / kE) void k_cols_conv_split(const ConvDesc *__restrict__ cd) {
  using V = typename CT<T>::V;
  constexpr int TPS = N / kE;
  constexpr int n = N / 2;
  __shared__ T lds[N + (N >> kSplitPad)];
  const ConvDesc &C = cd[blockIdx.y];
  V *__restrict__ X = static_cast<V *>(C.X);
  const T *__restrict__ spec = static_cast<const T *>(C.spec);
  const V *__restrict__ tw = static_cast<const V *>(C.tw);
  const int lane = threadIdx.x;
  const int k1 = blockIdx.x;
  V *col = X + (size_t)k1 * n;
  V x[kE];
#pragma unroll
  for (int k = 0; k < kE / 2; ++k) x[k] = col[lane + k * TPS];
  split_stages<T, N, 0, false, true>(x, lds, tw, lane);
  {
    const T *sp = spec + (size_t)k1 * (n + 1);
#pragma unroll
    for (int k = 0; k < kE; ++k) {
      const int k2 = lane + k * TPS;
      const T g = sp[k2 <= n ? k2 : N - k2];
      x[k].x *= g;
      x[k].y *= g;
    }
  }
  split_stages<T, N, 0, true, false>(x, lds, tw, lane);
  const int lo = C.row_lo & ~15, hi = C.row_hi | 15;
  V *dst = C.Xb ? static_cast<V *>(C.Xb) + (size_t)k1 * C.band_pitch - lo : col;
#pragma unroll
  for (int k = 0; k < kE / 2; ++k) {
    const int j = lane + k * TPS;
    if (j >= lo && j <= hi) dst[j] = x[k];
  }
}

// ---------------------------------------------------------------------------
// pass 3: rows, two half spectra -> two real rows, gauge epilogue
// ---------------------------------------------------------------------------
// row-pair block `blk` of one problem; band: blocks count from the 16-row
// group of row_lo, and rows past the band's last 16-row group (a workgroup
// of more than 16 rows can reach them) are neither read nor written
template <class T, int N, int SH>
__device__ __forceinline__ void rows_inv_body(const ConvDesc &C, int blk, int band,
                                              typename CT<T>::V *lds) {
  using V = typename CT<T>::V;
  using V2 = typename CT<T>::V2;
  using P = RowPlan<T, N, SH>;
  constexpr int n = N / 2;
  T *__restrict__ s = static_cast<T *>(C.out);
  const V *__restrict__ tw = static_cast<const V *>(C.tw);
  const int tid = threadIdx.x;
  // band: the grid covers the rows from the 16-row group of row_lo on, read
  // from the compact band when the column pass stored one
  const int lo = band ? C.row_lo & ~15 : 0;
  const int hi_row = band ? (C.row_hi | 15) : n - 1;
  const int j0 = lo + blk * 2 * P::SEQ;
  if (j0 + 2 * P::SEQ <= C.row_lo || j0 > C.row_hi) return;  // rows nobody reads
  const bool compact = band && C.Xb;
  const V *__restrict__ X = compact ? static_cast<const V *>(C.Xb) - lo : static_cast<const V *>(C.X);
  const int pitch = compact ? C.band_pitch : n;
  V wr[tw_regs<N>()];
  if constexpr (tw_in_regs<T, N>()) load_twiddles<T, N, 0>(wr, tw, tid % P::TPS);

  // Z[k] = A[k] + i B[k], Z[N-k] = conj(A[k]) + i conj(B[k]); the imaginary
  // parts of A and B at k = 0 and k = n are dropped (real rows).  Every
  // load of a thread is issued before any is unpacked.
  constexpr int ITEMS = (n + 1) * P::SEQ, ITER = (ITEMS + P::WGT - 1) / P::WGT;
  V2 abv[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int idx = min(tid + it * P::WGT, ITEMS - 1);
    if (P::SEQ * 2 > 16 && j0 + 2 * (idx % P::SEQ) > hi_row) {
      abv[it].x = abv[it].y = abv[it].z = abv[it].w = (T)0;   // past the band
    } else {
      abv[it] = *reinterpret_cast<const V2 *>(X + (size_t)(idx / P::SEQ) * pitch + j0 + 2 * (idx % P::SEQ));
    }
  }
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int idx = tid + it * P::WGT;
    if (idx >= ITEMS) break;
    const int k = idx / P::SEQ, q = idx % P::SEQ;
    const V2 ab = abv[it];
    V *L = lds + q * P::LDS_SEQ;
    V z;
    if (k == 0 || k == n) {
      z.x = ab.x;
      z.y = ab.z;
      L[pad(k)] = z;
    } else {
      z.x = ab.x - ab.w;
      z.y = ab.y + ab.z;
      L[pad(k)] = z;
      z.x = ab.x + ab.w;
      z.y = ab.z - ab.y;
      L[pad(N - k)] = z;
    }
  }
  __syncthreads();
  const int q = tid / P::TPS, lane = tid % P::TPS;
  V x[kE];
  fft_seq<T, N, true, false, true, false, true>(x, lds + q * P::LDS_SEQ, wr, tw, lane);
  const T shift = (T)(C.c * (C.gamma ? C.gamma[0] : C.gamma_val));
  const int j = j0 + 2 * q;
  if (P::SEQ * 2 > 16 && j > hi_row) return;   // past the band: nothing to store
  const size_t row = (size_t)j * n;
  if (C.add_inf) {
    // total psi: + U_inf y - V_inf x, added in FP64 before the one rounding
    const double ya = C.inf_u * (C.oy + j * C.h), yb = C.inf_u * (C.oy + (j + 1) * C.h);
    const double sh = C.c * (C.gamma ? C.gamma[0] : C.gamma_val);
#pragma unroll
    for (int k = 0; k < kE / 2; ++k) {
      const int i = lane + k * P::TPS;
      const double xi = C.inf_v * (C.ox + i * C.h);
      s[row + i] = (T)((double)x[k].x - sh + (ya - xi));
      s[row + n + i] = (T)((double)x[k].y - sh + (yb - xi));
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < kE / 2; ++k) {
    s[row + lane + k * P::TPS] = x[k].x - shift;
    s[row + n + lane + k * P::TPS] = x[k].y - shift;
  }
}

template <class T, int N, bool WIDE>
__global__ __launch_bounds__((RowPlan<T, N, WIDE ? kWide : kNarrow>::WGT),
                             (std::is_same<T, float>::value ? 4 : 1)) void k_rows_inv(
    const ConvDesc *__restrict__ cd, int remap, int band) {
  using P = RowPlan<T, N, WIDE ? kWide : kNarrow>;
  __shared__ typename CT<T>::V lds[P::SEQ * P::LDS_SEQ];
  rows_inv_body<T, N, WIDE ? kWide : kNarrow>(cd[blockIdx.y], xcd_block(remap), band, lds);
}

int num_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
  }
  return cus;
}

// XCD order of a row pass (ConvSched::order): 0 plain where a workgroup's
// runs fill whole 128-byte lines, consecutive blocks per XCD otherwise;
// 1 plain; 2 consecutive blocks
template <class T, int N, bool WIDE>
int row_remap(const ConvSched &sc, int xcds) {
  if (sc.order == 1) return 1;
  if (sc.order == 2) return xcds;
  return RowPlan<T, N, WIDE ? kWide : kNarrow>::FULL_LINES ? 1 : xcds;
}

template <class Tin, class T, int N, bool WIDE>
// fband > 0: only that many source rows per problem, from its fwd_lo on
void launch_rows_fwd(const ConvDesc *d, int nb, int xcds, const ConvSched &sc, hipStream_t st,
                     int fband) {
  using RP = RowPlan<T, N, WIDE ? kWide : kNarrow>;
  const int rows = fband > 0 ? std::min(fband, N / 2) : N / 2;
  hipLaunchKernelGGL((k_rows_fwd<Tin, T, N, WIDE>), dim3((rows + 2 * RP::SEQ - 1) / (2 * RP::SEQ), nb),
                     dim3(RP::WGT), 0, st, d, row_remap<T, N, WIDE>(sc, xcds), fband > 0 ? 1 : 0);
}
// band > 0: only that many rows per problem, from its row_lo's 16-row group
template <class T, int N, bool WIDE>
void launch_rows_inv(const ConvDesc *d, int nb, int xcds, int band, const ConvSched &sc,
                     hipStream_t st) {
  using RP = RowPlan<T, N, WIDE ? kWide : kNarrow>;
  const int rows = band > 0 ? std::min(band, N / 2) : N / 2;
  hipLaunchKernelGGL((k_rows_inv<T, N, WIDE>), dim3((rows + 2 * RP::SEQ - 1) / (2 * RP::SEQ), nb),
                     dim3(RP::WGT), 0, st, d, row_remap<T, N, WIDE>(sc, xcds), band > 0 ? 1 : 0);
}

template <class Tin, class T, int N>
hipError_t run_conv(const ConvDesc *d, int nb, int xcds, int band, const ConvSched &sc,
                    hipStream_t st, int fband) {
  const bool pruned = band > 0;
  using P = Plan<N>;
  constexpr int n = N / 2;
  // wide row blocks when they still give two or more workgroups per CU
  // (ConvSched::rows 0), or as the schedule says
  const bool wide = sc.rows == 2 ||
                    (sc.rows == 0 && (n / (2 * RowPlan<T, N, kWide>::SEQ)) * nb >= 2 * num_cus());
  constexpr bool D = std::is_same<T, double>::value;
  timer_begin(D ? GPF_TK_ROWS_FWD64 : GPF_TK_ROWS_FWD, st);
  if (wide)
    launch_rows_fwd<Tin, T, N, true>(d, nb, xcds, sc, st, fband);
  else
    launch_rows_fwd<Tin, T, N, false>(d, nb, xcds, sc, st, fband);
  timer_end(st);
  timer_begin(D ? GPF_TK_COLS64 : GPF_TK_COLS, st);
  // FP64 from N = 1024 on: the split-exchange column pass unless the
  // schedule asks for the complex exchange
  bool split = false;
  if constexpr (D && N >= 1024) split = sc.cols != 1;
  if (split) {
    if constexpr (D && N >= 1024)
      hipLaunchKernelGGL((k_cols_conv_split<T, N>), dim3(n + 1, nb), dim3(N / kE), 0, st, d);
  } else {
    hipLaunchKernelGGL((k_cols_conv<T, N>), dim3((n + 1 + P::SEQ - 1) / P::SEQ, nb), dim3(P::WGT),
                       0, st, d);
  }
  timer_end(st);
  timer_begin(D ? GPF_TK_ROWS_INV64 : GPF_TK_ROWS_INV, st);
  if (wide && !pruned)
    launch_rows_inv<T, N, true>(d, nb, xcds, 0, sc, st);
  else
    launch_rows_inv<T, N, false>(d, nb, xcds, band, sc, st);
  timer_end(st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// passes over problems of several grid sizes in one launch
// ---------------------------------------------------------------------------
// The launch's blocks form one work list: the table orders the problems by
// decreasing grid size and gives each its first block, so the largest
// transforms are dispatched first and the small ones fill in behind them as
// workgroups retire.  (A persistent loop over a work counter was compiled
// too: the loop around the transform bodies raised the register count from
// 113 to 178-214, i.e. from four waves per SIMD to two, so each workgroup
// takes one block.)  Block g belongs to the last entry whose first block is
// <= g: every wave loads the table (up to 256 entries, four per lane), counts
// the entries at or below g by ballots and reads the entry from its lane.
constexpr int kMultiLds = kMultiThreads * 17;   // SEQ (N + N/16) elements for every N

__device__ __forceinline__ bool multi_locate(const MultiPass &mp, int *prob, int *logn, int *band,
                                             int *blk) {
  // workgroups are dealt round-robin to the XCDs; every block of these
  // passes is the same work (4096 transform points), so each XCD takes one
  // contiguous 1/xcds of the list (the grid is padded to a multiple of
  // xcds), and neighbouring row blocks, whose runs share cache lines, share
  // an L2
  const int per = gridDim.x / mp.xcds;
  const int g = (blockIdx.x % mp.xcds) * per + blockIdx.x / mp.xcds;
  if (g >= mp.total) return false;
  const int lane = threadIdx.x & 63;
  int e[4][4];
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k * 64 < mp.nprob) {
      const int i = lane + 64 * k;
      if (i < mp.nprob) {
        const int4 v = *reinterpret_cast<const int4 *>(mp.e + i);
        e[k][0] = v.x; e[k][1] = v.y; e[k][2] = v.z; e[k][3] = v.w;
      } else {
        e[k][0] = 0x7fffffff; e[k][1] = e[k][2] = e[k][3] = 0;
      }
      cnt += __popcll(__ballot(e[k][0] <= g));
    }
  }
  const int idx = __builtin_amdgcn_readfirstlane(cnt - 1);
  const int k = idx >> 6, l = idx & 63;
  int f[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
    f[c] = k == 0 ? e[0][c] : (k == 1 ? e[1][c] : (k == 2 ? e[2][c] : e[3][c]));
  const int first = __builtin_amdgcn_readlane(f[0], l);
  *prob = __builtin_amdgcn_readlane(f[1], l);
  *logn = __builtin_amdgcn_readlane(f[2], l);
  *band = __builtin_amdgcn_readlane(f[3], l);
  *blk = g - first;
  return true;
}

template <class Tin, class T>
__global__ __launch_bounds__(kMultiThreads) void k_rows_fwd_multi(const ConvDesc *__restrict__ cd,
                                                                  MultiPass mp) {
  __shared__ typename CT<T>::V lds[kMultiLds];
  int p, logn, band, blk;
  if (!multi_locate(mp, &p, &logn, &band, &blk)) return;
  const ConvDesc &C = cd[p];
  switch (logn) {
    case 6: rows_fwd_body<Tin, T, 128, kMulti>(C, blk, band, lds); break;
    case 7: rows_fwd_body<Tin, T, 256, kMulti>(C, blk, band, lds); break;
    case 8: rows_fwd_body<Tin, T, 512, kMulti>(C, blk, band, lds); break;
    case 9: rows_fwd_body<Tin, T, 1024, kMulti>(C, blk, band, lds); break;
    case 10: rows_fwd_body<Tin, T, 2048, kMulti>(C, blk, band, lds); break;
    case 11: rows_fwd_body<Tin, T, 4096, kMulti>(C, blk, band, lds); break;
    default: break;
  }
}

template <class T>
__global__ __launch_bounds__(kMultiThreads) void k_cols_multi(const ConvDesc *__restrict__ cd,
                                                              MultiPass mp) {
  __shared__ typename CT<T>::V lds[kMultiLds];
  int p, logn, band, blk;
  if (!multi_locate(mp, &p, &logn, &band, &blk)) return;
  const ConvDesc &C = cd[p];
  switch (logn) {
    case 6: cols_body<T, 128, kMultiThreads / 8>(C, blk, lds); break;
    case 7: cols_body<T, 256, kMultiThreads / 16>(C, blk, lds); break;
    case 8: cols_body<T, 512, kMultiThreads / 32>(C, blk, lds); break;
    case 9: cols_body<T, 1024, kMultiThreads / 64>(C, blk, lds); break;
    case 10: cols_body<T, 2048, kMultiThreads / 128>(C, blk, lds); break;
    case 11: cols_body<T, 4096, kMultiThreads / 256>(C, blk, lds); break;
    default: break;
  }
}

template <class T>
__global__ __launch_bounds__(kMultiThreads) void k_rows_inv_multi(const ConvDesc *__restrict__ cd,
                                                                  MultiPass mp) {
  __shared__ typename CT<T>::V lds[kMultiLds];
  int p, logn, band, blk;
  if (!multi_locate(mp, &p, &logn, &band, &blk)) return;
  const ConvDesc &C = cd[p];
  switch (logn) {
    case 6: rows_inv_body<T, 128, kMulti>(C, blk, band, lds); break;
    case 7: rows_inv_body<T, 256, kMulti>(C, blk, band, lds); break;
    case 8: rows_inv_body<T, 512, kMulti>(C, blk, band, lds); break;
    case 9: rows_inv_body<T, 1024, kMulti>(C, blk, band, lds); break;
    case 10: rows_inv_body<T, 2048, kMulti>(C, blk, band, lds); break;
    case 11: rows_inv_body<T, 4096, kMulti>(C, blk, band, lds); break;
    default: break;
  }
}

}  // namespace

int multi_blocks(int pass, int n, const ConvDesc &c) {
  const int rows = 4096 / n;              // rows per workgroup (two per sequence)
  if (pass == 1) {
    const int seq = 2048 / n;             // columns per workgroup
    return (n + 1 + seq - 1) / seq;
  }
  if (pass == 2) {                        // band of the first convolution
    const int band = (c.row_hi | 15) - (c.row_lo & ~15) + 1;
    return (band + rows - 1) / rows;
  }
  if (pass == 0) return (c.fwd_hi - c.fwd_lo + 1 + rows - 1) / rows;   // source rows transformed
  return n / rows;                        // 3: every row of the inverse
}

template <class Tin, class T>
hipError_t launch_convolve_multi(const ConvDesc *d, const MultiPass *mp, hipStream_t st) {
  static_assert(std::is_same<T, float>::value, "multi-size passes are FP32 transforms");
  auto grid = [](const MultiPass &m) { return dim3((m.total + m.xcds - 1) / m.xcds * m.xcds); };
  timer_begin(GPF_TK_ROWS_FWD, st);
  hipLaunchKernelGGL((k_rows_fwd_multi<Tin, T>), grid(mp[0]), dim3(kMultiThreads), 0, st, d, mp[0]);
  timer_end(st);
  timer_begin(GPF_TK_COLS, st);
  hipLaunchKernelGGL((k_cols_multi<T>), grid(mp[1]), dim3(kMultiThreads), 0, st, d, mp[1]);
  timer_end(st);
  timer_begin(GPF_TK_ROWS_INV, st);
  hipLaunchKernelGGL((k_rows_inv_multi<T>), grid(mp[2]), dim3(kMultiThreads), 0, st, d, mp[2]);
  timer_end(st);
  return hipGetLastError();
}
template hipError_t launch_convolve_multi<float, float>(const ConvDesc *, const MultiPass *, hipStream_t);
template hipError_t launch_convolve_multi<double, float>(const ConvDesc *, const MultiPass *, hipStream_t);

template <class Tin, class T>
hipError_t launch_convolve(int n, const ConvDesc *d, int nb, int xcds, int band, hipStream_t st,
                           const ConvSched &sc, int fband) {
  switch (n) {
    case 16: return run_conv<Tin, T, 32>(d, nb, xcds, band, sc, st, fband);
    case 32: return run_conv<Tin, T, 64>(d, nb, xcds, band, sc, st, fband);
    case 64: return run_conv<Tin, T, 128>(d, nb, xcds, band, sc, st, fband);
    case 128: return run_conv<Tin, T, 256>(d, nb, xcds, band, sc, st, fband);
    case 256: return run_conv<Tin, T, 512>(d, nb, xcds, band, sc, st, fband);
    case 512: return run_conv<Tin, T, 1024>(d, nb, xcds, band, sc, st, fband);
    case 1024: return run_conv<Tin, T, 2048>(d, nb, xcds, band, sc, st, fband);
    case 2048: return run_conv<Tin, T, 4096>(d, nb, xcds, band, sc, st, fband);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_convolve<float, float>(int, const ConvDesc *, int, int, int, hipStream_t,
                                                     const ConvSched &, int);
template hipError_t launch_convolve<double, double>(int, const ConvDesc *, int, int, int, hipStream_t,
                                                     const ConvSched &, int);
template hipError_t launch_convolve<double, float>(int, const ConvDesc *, int, int, int, hipStream_t,
                                                     const ConvSched &, int);

}  // namespace gpf
