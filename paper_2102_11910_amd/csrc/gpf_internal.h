// Internal declarations of the gpf library (host runtime + HIP kernels).
//
// Every solve kernel works on a batch of independent problems: blockIdx.y
// selects a problem, whose pointers and scalars come from a descriptor in
// device memory.  A plain solve is a batch of one.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <map>
#include <mutex>
#include <string>
#include <utility>
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

#define GPF_TRY(call)                \
  do {                               \
    gpf_status s_ = (call);          \
    if (s_ != GPF_OK) return s_;     \
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
// device memory and timing
// ---------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf();
  gpf_status alloc(size_t nbytes);  // keeps the buffer if it is large enough
  template <class T> T *as() const { return static_cast<T *>(p); }
  void swap(DevBuf &o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
  }
};

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

// Ring of descriptor slots: host staging in pinned memory, copied to device
// memory on the caller's stream.  A slot is reused only after the event
// recorded behind its copy has completed; slots taken while the stream is
// being captured into a graph stay reserved until unpin() (called by the
// owner of the graph once no replay can still read them).
struct DescRing {
  int slots = 0;
  size_t slot_bytes = 0;
  char *host = nullptr;
  DevBuf dev;
  std::vector<hipEvent_t> ev;
  std::vector<char> busy, pinned;
  int next = 0;
  // set by the library around a capture of its own: a block pushed while
  // capturing is copied once after the capture (flush_deferred) instead of
  // by a copy node that every replay would repeat
  bool defer_captured = false;
  std::vector<std::pair<int, size_t>> deferred;   // (slot, bytes)
  DescRing() = default;
  DescRing(const DescRing &) = delete;
  DescRing &operator=(const DescRing &) = delete;
  ~DescRing();
  gpf_status init(int nslots, size_t bytes_per_slot);
  gpf_status push(const void *src, size_t bytes, hipStream_t s, void **dptr);
  gpf_status flush_deferred();   // synchronous copies of the deferred blocks
  void unpin(int slot) {
    pinned[slot] = 0;
    busy[slot] = 0;
  }
};

// ---------------------------------------------------------------------------
// descriptors
// ---------------------------------------------------------------------------
// scalar slots (doubles) of a problem's aux block
enum ScalarSlot {
  SC_GAMMA_W = 0,     // circulation of the vortices (sum Gamma_q)
  SC_GAMMA_SRC2 = 1,  // source circulation of the final convolution
  SC_S0 = 2,
  SC_GAMMA_B = 3,
  SC_GAMMA_NEW = 4,   // .. 4 + GPF_MAX_EDGES
  SC_PART_S0 = 4 + GPF_MAX_EDGES,                 // GPF_PARTS: s0_j
  SC_PART_GB = 4 + GPF_MAX_EDGES + GPF_MAX_PARTS, // GPF_PARTS: bound circulation per part
  SC_COUNT = 4 + GPF_MAX_EDGES + 2 * GPF_MAX_PARTS,
  SC_RV_SCALE = 31,   // R_v: power-of-two scale of the fixed-point sums
  AUX_DOUBLES = 32,
  AUX_BYTES = AUX_DOUBLES * 8
};

struct SolveScalars {
  double u_inf, v_inf, ub, vb, omega;
  double gamma_b, gamma_w_in;   // gamma_w_in NaN -> use the device sum
  int mode, m;
  int edges[GPF_MAX_EDGES];
  double xnew[GPF_MAX_EDGES], ynew[GPF_MAX_EDGES];
  double fmin[GPF_MAX_EDGES], fmax[GPF_MAX_EDGES];   // edge bounds on f~
  int znew_from;   // >= 0: new vortex j sits at vortex znew_from + j (device
                   // arrays) instead of (xnew[j], ynew[j])
  // GPF_PARTS: per part its mode, constraint values and motion; the part of
  // each new vortex's edge; the steady-Kutta edge of each part (or -1)
  int nparts;
  int pmode[GPF_MAX_PARTS];
  double pgb[GPF_MAX_PARTS], pgw[GPF_MAX_PARTS];
  double pub[GPF_MAX_PARTS], pvb[GPF_MAX_PARTS], pom[GPF_MAX_PARTS];
  int epart[GPF_MAX_EDGES];
  int kedge[GPF_MAX_PARTS];
};

// Launch schedule of the convolution passes (the same arithmetic in every
// schedule; they differ in how work maps to workgroups and XCDs).
struct ConvSched {
  int rows = 0;    // row passes: 0 wide when it gives two workgroups per CU, 1 narrow, 2 wide
  int order = 0;   // row-pass XCD order: 0 by line fill, 1 dispatch order, 2 blocks per XCD
  int cols = 0;    // FP64 column pass from N = 1024: 0 or 2 split exchange, 1 complex exchange
};

// one convolution of one problem: out = conv(in) - c * gamma[0]
struct ConvDesc {
  void *in;            // n*n source (zeroed after it is read when zero_in)
  void *X;             // (n+1)*n complex intermediate
  void *out;           // n*n result
  const void *spec;    // (n+1)^2 scaled spectrum
  const void *tw;      // 2n twiddles
  const double *gamma; // source circulation (device); null: use gamma_val
  double gamma_val;
  double c;            // gauge shift of the spectrum
  int zero_in;
  int row_lo, row_hi;  // rows of `out` that are needed (inclusive)
  // optional compact band: the column pass stores rows (row_lo & ~15) ..
  // (row_hi | 15) as Xb[k1 * band_pitch + j - (row_lo & ~15)] and the band
  // inverse row pass reads them from there (null: in place in X)
  void *Xb;
  int band_pitch;
  int add_inf;         // add s_inf = inf_u (oy + j h) - inf_v (ox + i h) to the output
  double inf_u, inf_v, ox, oy, h;
  // forward row pass: with its band flag it transforms only source rows
  // fwd_lo .. fwd_hi (fwd_lo a multiple of 16), the other rows of X holding
  // the transforms of an earlier pass over the same source; when it clears
  // the source (zero_in) it leaves rows keep_lo <= j < keep_end for a later
  // pass (a zeroed descriptor keeps nothing)
  int fwd_lo, fwd_hi;
  int keep_lo, keep_end;
  // halo slots of the source's R_v tiles (32 x 32 cells, n / 32 per side,
  // kHaloRing entries each, of the source's type), added to the border
  // nodes of every source row the forward row pass reads; nullptr: none
  const void *halo;
};

struct ProbDesc {
  // grid
  int n;
  double dx, x0, y0;
  const double *lgf;            // (n+1)^2 LGF table
  // vortices
  int nv;
  const double *xv, *yv, *gv;
  // fields
  void *w;                      // source field (zero on entry, or the values R_v adds to)
  int w_accumulate;             // 1: w holds values R_v adds to; 0: w is zero on entry
  int w64;                      // 1: the source field w is FP64, 0: FP32
  int halo_defer;               // 1: the solve's convolutions add the tiles' halos as
                                // they read w (no halo pass); 0: the halo pass adds them
  int vel_tiles;                // 1: velocities tile by tile through LDS (dense clouds)
  const void *s1;               // result of the first convolution
  // per-problem aux: scalars and partial sums
  double *aux;
  double *partials;
  unsigned *status;
  // vortex binning by tiles of cells: counts (zero between solves), tile
  // starts, rank of each vortex in its tile, tile-sorted (xi, eta, Gamma/dx^2)
  int *bin_cnt, *bin_start, *rank;
  void *halo;                   // per tile, the window nodes its neighbours own
                                // (kHaloRing values of the field type)
  int *items;                   // work list of the tile kernels, 4 ints per item:
                                // [0] = {count, 0, 0, 0}, then {tile, first record,
                                // end record, 0 alone or 1 + window slot}
  int *splits;                  // tiles of several items: [0] = {count, 0, 0, 0},
                                // then {tile, first window slot, items, 0}
  long long *splitwin;          // window slots of split tiles' items (kSplitWin each)
  double *sorted;
  // body
  int ns;
  const double *xs, *ys, *ds, *sinv, *f0;
  const double *ghat;           // S^-T dS: circulation of S^-1 r is ghat . r
  const int *st_i;
  const double *st_w;
  double gamma0;
  double mom_x, mom_y, mom_r2;  // sums of fhat0 x, fhat0 y, fhat0 (x^2 + y^2)
  double *rhs;                  // Schur right-hand sides: ns x (1+m)
  double *fs;                   // f per surface point, written by the surface step
  // R_s as a gather: the rs_nodes grid nodes (n j + i, ascending) the surface
  // stencils reach, node k's entries rs_code[rs_off[k] .. rs_off[k+1]) =
  // 16 p + 4 b + a (stencil weight a, b of point p), in point order
  const int *rs_node, *rs_off, *rs_code;
  int rs_nodes;
  double *y;                    // S^-1 rhs, formed for the whole launch (problems sharing
                                // one body), or null: each workgroup forms its rows
  // outputs (nullable)
  const void *psi;              // final field (velocities read it)
  double *u, *v, *f_out, *ft_out, *sc_out;
  double *imp_out;              // impulse (P_x, P_y, Pi_O), or null
  const double *nx, *ny;        // body normals into the fluid (zeros: thin body)
  // GPF_PARTS: part of each point; per part S^-T (dS o 1_j) and S^-1 1_j
  // (ns each, part-major) and the circulations C_jl of S^-1 1_l over part j
  const int *part;
  const double *gpart, *zpart, *cpart;
  const double *pgw_dev;        // GPF_PARTS: per-part released circulation on
                                // the device (replaces sv.pgw), or null
  int psi_total;                // psi holds s + s_inf: velocities add no U_inf
  SolveScalars sv;
};

// ---------------------------------------------------------------------------
// kernel launchers (asynchronous on `s`; `nb` problems, same n)
// ---------------------------------------------------------------------------
int scatter_blocks(int nv_max);
int place_blocks(int nv);   // workgroups of the binning place kernel of one problem
// binning partials per workgroup of vortices, five planes of kPartStride:
// sum Gamma, sum Gamma x, sum Gamma y, sum Gamma (x^2 + y^2), sum |Gamma|
constexpr int kMaxVortices = 1 << 22;
constexpr int kPartStride = kMaxVortices / 256;
// Vortices per thread of the binning count (256 threads per workgroup), a
// power of two from 1 to 8 (16 made the kernel, which holds every case,
// keep 144 VGPRs instead of 81).  A workgroup adds one device atomic per
// non-empty tile to the tile counts, and the atomics on one counter are
// carried out one after another; a thread's vortices, on the other hand,
// are a serial chain of FP64 cell arithmetic and LDS atomics.  About 64
// workgroups per problem measured best (32, 128 and 256, and one vortex
// per thread, were slower on the 64-problem batch and the 1e5-vortex
// single solve).
__host__ __device__ inline int bin_per_thread(int nv) {
  const int want = (nv + 256 * 64 - 1) / (256 * 64);
  int p = 1;
  while (p < want && p < 8) p *= 2;
  return p;
}
// workgroups of the binning count of a problem (one partial each)
__host__ __device__ inline int bin_count_blocks(int nv) {
  const int per = 256 * bin_per_thread(nv);
  return nv > 0 ? (nv + per - 1) / per : 1;
}
int bin_tiles(int n);  // tiles per grid (square tiles of 32 cells, fewer for n < 32)
// A tile of more than kTileChunk vortices is split into items of at most
// kTileChunk records each, and a tile without vortices is one empty item
// (it clears its halo slot); tile_items_max bounds the items of a problem.
// The items of a split tile store their fixed-point windows ((32 + 3)^2
// nodes) in slots of their own, which a second kernel sums; a problem has
// at most split_tiles_max such tiles and split_items_max such items.
constexpr int kTileChunk = 512;
int tile_items_max(int n, int nv);
constexpr int kSplitWin = (32 + 3) * (32 + 3);
inline int split_tiles_max(int nv) { return nv / (kTileChunk + 1); }
inline int split_items_max(int nv) { return nv / kTileChunk + split_tiles_max(nv); }
int split_blocks(int nv);   // workgroups of the split-tile kernel of one problem
// A tile's window (ts + 3)^2 nodes minus its own ts^2: 6 ts + 9 at most.
constexpr int kHaloRing = 6 * 32 + 9;
int halo_tiles(int n);   // tiles that neighbours' windows reach (0 for one tile)
int fixup_blocks(int n); // workgroups of the halo pass of one problem

// Flat grids of merged batches for the kernels that read n, nv and ns from
// their descriptors: entry i gives the first block of problem `prob` in the
// launch and its number of blocks (entries ordered, firsts ascending; a
// problem with no blocks has an entry of nblk 0).  Without a table (e ==
// nullptr) blockIdx.y is the problem and gridDim.x its block count.
struct FlatEntry {
  int first, prob, nblk, pad;
};
struct FlatMap {
  const FlatEntry *e;   // device table of nprob entries (16-byte aligned), or nullptr
  int nprob;
  int total;            // blocks of the launch
};
struct FlatBlock {
  int prob, blk, nblk;
};
// this workgroup's problem and block; false past the last block.  Every wave
// loads the table (up to 256 entries, four per lane) and counts the entries
// at or below its block by ballots.
__device__ __forceinline__ bool flat_block(const FlatMap &fm, FlatBlock *fb) {
  int prob = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  bool ok = true;
  if (fm.e) {
    const int g = blockIdx.x;
    const int lane = threadIdx.x & 63;
    int first = 0, pr = 0, nb = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k * 64 < fm.nprob) {
        const int i = lane + 64 * k;
        int4 v = make_int4(0x7fffffff, 0, 0, 0);
        if (i < fm.nprob) v = *reinterpret_cast<const int4 *>(fm.e + i);
        const int c = __popcll(__ballot(v.x <= g));
        // the entry sits in this quarter when the count ends inside it
        const int idx = __builtin_amdgcn_readfirstlane(cnt + c - 1);
        if (c > 0 && idx >= 64 * k) {
          const int l = idx & 63;
          first = __builtin_amdgcn_readlane(v.x, l);
          pr = __builtin_amdgcn_readlane(v.y, l);
          nb = __builtin_amdgcn_readlane(v.z, l);
        }
        cnt += c;
      }
    }
    prob = pr;
    blk = g - first;
    nblk = nb;
    ok = g < fm.total;
  }
  fb->prob = prob;
  fb->blk = blk;
  fb->nblk = nblk;
  return ok;
}
// R_v: bin and sort the vortices by tile; one workgroup per work item sums
// its vortices' stencils in an LDS window in fixed point, stores the tile's
// own nodes into the source field (zero, or the values to add to) and the
// nodes its neighbours own into the tile's halo slot; then one workgroup per
// tile adds the neighbours' halos to its border nodes in a fixed order, so
// the field is the same bits on every run (split dense tiles use atomics).
// Problems with halo_defer skip that last pass: their convolutions add the
// halos as they read the field.
// fm (merged batches): fm[0] the count's map, fm[1] the tile kernel's,
// fm[2] the halo kernel's, fm[3] the place kernel's (one block per 256
// vortices), fm[4] the split-tile kernel's (total 0: the caller launches it
// with launch_split_combine); nullptr: a 2-D grid of nb problems, with the
// halo pass when `halo_pass` is set
template <class T>
hipError_t launch_scatter_vortices(const ProbDesc *d, int nb, int n, int nv_max, hipStream_t s,
                                   const FlatMap *fm = nullptr, bool halo_pass = true);
// Launches that cover problems of several grid sizes (FP32 transforms, n from
// 64 to 2048): entry i of a pass's table gives the first of its blocks,
// problem `prob` (an index into the launch's ConvDesc array) and log2 n;
// entries are ordered by decreasing n, firsts ascending.  band = 1 in the
// last pass of a first convolution (only the band of surface rows).
constexpr int kMaxMultiProblems = 256;
struct MultiEntry {
  int first, prob, logn, band;
};
struct MultiPass {
  const MultiEntry *e;  // device table of nprob entries (16-byte aligned)
  int nprob;
  int total;            // blocks of the launch
  int xcds;             // XCDs the workgroups are dealt to (>= 1)
};
// blocks of one problem in a multi-size pass (0 rows forward over the
// descriptor's source rows fwd_lo .. fwd_hi, 1 columns, 2 rows inverse over
// the band of the descriptor, 3 rows inverse, all rows)
int multi_blocks(int pass, int n, const ConvDesc &c);
// the three passes of one convolution per problem; mp[0..2] the passes' tables
template <class Tin, class T>
hipError_t launch_convolve_multi(const ConvDesc *d, const MultiPass *mp, hipStream_t s);
// band > 0: the descriptors restrict the output rows, and no problem needs
// more than `band` rows from the 16-row group of its row_lo (narrow inverse
// rows over that band only); 0: every row.  fband > 0: the forward row pass
// transforms only each descriptor's source rows fwd_lo .. fwd_hi, at most
// fband of them (the other rows of X are kept); 0: every row.  sc: launch
// schedule.
template <class Tin, class T>
hipError_t launch_convolve(int n, const ConvDesc *d, int nb, int xcds, int band, hipStream_t s,
                           const ConvSched &sc, int fband = 0);
// the fixed device scratch of gpf_convolve_noalloc: its address on `device`
// (which must be current) is taken once; called when a context is created
gpf_status noalloc_init(int device);
size_t noalloc_scratch_bytes();
template <class T>
hipError_t launch_surface_rhs(const ProbDesc *d, int nb, int ns_max, int m_max, hipStream_t s);
template <class T>
hipError_t launch_schur_apply(const ProbDesc *d, int nb, int ns_max, int m_max, hipStream_t s);
// y = S^-1 rhs for nb problems that share one body (ns points, S^-1 = sinv),
// on the matrix cores; every descriptor's y must be set
hipError_t launch_schur_gemm(const ProbDesc *d, int nb, int ns, int m_max, const double *sinv,
                             hipStream_t s);
// the same for bodies of several parts (mode GPF_PARTS)
template <class T>
hipError_t launch_schur_apply_parts(const ProbDesc *d, int nb, int ns_max, hipStream_t s);
// R_s f and the new vortices' stencils added to the source field after the
// surface step, node by node in a fixed order (FP32 and FP64 fields in one
// launch, by each problem's w64); `blocks` per problem (the most of
// rs_apply_blocks over the launch), or the flat map fm
hipError_t launch_rs_apply(const ProbDesc *d, int nb, int blocks, hipStream_t s,
                           const FlatMap *fm = nullptr);
// the split tiles' windows summed into the field after R_v's tile kernel,
// for FP32 and FP64 fields in one launch; `blocks` per problem
// (split_blocks of the most vortices), or the flat map fm
hipError_t launch_split_combine(const ProbDesc *d, int nb, int blocks, hipStream_t s,
                                const FlatMap *fm = nullptr);
inline int rs_apply_blocks(int rs_nodes, int m) { return (rs_nodes + 255) / 256 + (m > 0 ? 1 : 0); }
template <class T>
hipError_t launch_vortex_velocity(const ProbDesc *d, int nb, int nv_max, hipStream_t s);
// velocities of a solve's vortices from their tile-sorted records (after
// launch_scatter_vortices of the same solve): problems with vel_tiles set
// tile by tile through LDS, the others vortex by vortex in record order; n
// the largest grid of the launch
// fm (merged batches): fm[0] the vortex-by-vortex kernel's map, fm[1] the
// tile kernel's; nullptr: 2-D grids of nb problems, of the kernels `kinds`
// asks for (1 vortex by vortex, 2 tile by tile, 3 both)
template <class T>
hipError_t launch_solve_velocity(const ProbDesc *d, int nb, int n, int nv_max, hipStream_t s,
                                 const FlatMap *fm = nullptr, int kinds = 3);

// xo = x + a u, yo = y + a v (in place allowed)
// pressure (Sec. 2.6.1): three-point weights of a surface point on the
// u-faces (x_i, y_j + dx/2) and the v-faces (x_i + dx/2, y_j)
struct PresStencil {
  int iu, ju, iv, jv;
  double wxu[4], wyu[4], wxv[4], wyv[4];
};
struct PresDesc {
  int n, ns, psi_total;
  double dx, x0, y0, rho, dt, u_inf, v_inf, ub, vb, omega;
  const void *psi;             // final field of the solve (plan field type)
  const double *f, *Q, *dphi_prev;
  const double *xs, *ys, *ds, *pnx, *pny;
  const PresStencil *st;
  const int *st_i;
  const double *st_w;
  const int *part;             // GPF_PARTS: part of each point, else null
  double pub[GPF_MAX_PARTS], pvb[GPF_MAX_PARTS], pom[GPF_MAX_PARTS];
  double *dphi, *dp, *ddt;     // ns each
  double *wsheet, *fx, *fy, *src, *tmp;   // n x n FP64 work fields
  double *p, *pside;           // outputs of the field part (nullable)
};
hipError_t launch_pres_stencils(int ns, const double *xs, const double *ys, double x0, double y0,
                                double dx, PresStencil *st, hipStream_t s);
hipError_t launch_pres_build(int n, int ns, const PresStencil *st, const double *pnx, const double *pny,
                             const int *st_i, const double *st_w, const double *ds, double dx,
                             const double *lgf, double *M, double *K, hipStream_t s);
// Q = -A K (A: leading dimension lda, first ns rows/columns; K, Q column-major)
hipError_t launch_pres_q(int ns, int lda, const double *A, const double *K, double *Q, hipStream_t s);
template <class T>
hipError_t launch_pres_surface_part(const PresDesc &D, hipStream_t s);
template <class T>
hipError_t launch_pres_field_part(const PresDesc &D, hipStream_t s);
template <class T>
hipError_t launch_pres_finish(const PresDesc &D, hipStream_t s);

// shedding steps (nv counts the new vortices; nv >= m >= 1)
struct ShedGeom {
  int m;
  double ex[GPF_MAX_EDGES], ey[GPF_MAX_EDGES];   // edge points
  double fx[GPF_MAX_EDGES], fy[GPF_MAX_EDGES];   // offsets of the first release
  int epart[GPF_MAX_EDGES];                       // GPF_PARTS: part of each edge
};
hipError_t launch_shed_place(const ShedGeom &sg, int nv, const int *last, double *x, double *y,
                             double *g, hipStream_t s);
// gw (nullable): per-part released circulation, to which each new vortex
// adds its strength (part sg.epart[j])
hipError_t launch_shed_advance(const ShedGeom &sg, int nv, const double *sc, int *last, double *gw,
                               double *x, double *y, double *g, const double *u, const double *v,
                               double dt,
                               hipStream_t s);
hipError_t launch_axpy2(int nv, const double *x, const double *y, const double *u,
                        const double *v, double a, double *xo, double *yo, hipStream_t s);

// single-problem helpers used at setup and by the building blocks
hipError_t launch_fill(void *p, size_t bytes, hipStream_t s);   // zero bytes (a multiple of 4)
// Schur build by columns: field b (stride elements apart) gets R_s e_{q0+b};
// column q0 + b of the row-major S gets E_s of field b
template <class T>
hipError_t launch_unit_sheets(int n, int ns, int q0, int nb, double dx, const int *st_i,
                              const double *st_w, const double *ds, T *w, size_t stride,
                              hipStream_t s);
template <class T>
hipError_t launch_interp_columns(int n, int ns, int q0, int nb, const int *st_i,
                                 const double *st_w, const T *f, size_t stride, double *S,
                                 hipStream_t s);
hipError_t launch_surface_stencils(int n, double dx, double x0, double y0, int ns,
                                   const double *xs, const double *ys, int *st_i,
                                   double *st_w, unsigned *status, hipStream_t s);
template <class T>
hipError_t launch_interp_surface(int n, int ns, const int *st_i, const double *st_w,
                                 const T *field, double *r, hipStream_t s);
hipError_t launch_schur_build(int n, int ns, const int *st_i, const double *st_w,
                              const double *ds, const double *lgf, double *S, hipStream_t s);
gpf_status invert_fp64(int ns, double *A, double *Ainv, hipStream_t s, double *min_pivot_rel);
hipError_t launch_gemv(int ns, int ncol, const double *A, const double *X, double *Y,
                       hipStream_t s);
hipError_t launch_gemv_t(int ns, const double *A, const double *x, double *y, hipStream_t s);
// impulse of each problem whose imp_out is set (after the surface solve)
hipError_t launch_impulse(const ProbDesc *d, int nb, hipStream_t s);

}  // namespace gpf

// ---------------------------------------------------------------------------
// handles
// ---------------------------------------------------------------------------
struct gpf_ctx {
  int device = 0;
  int num_cu = 0;
  int xcds = 8;
  char arch[64] = {};
  // convolution schedules by (n, precision, batch-size class); absent
  // entries use the default rules
  std::mutex sched_mu;
  std::map<long long, gpf::ConvSched> sched;
  gpf::ConvSched sched_for(int n, bool fp64, int nb);
};
// batch-size classes of the schedule table: 1, 2-7, 8-31, 32 and more
int sched_class(int nb);

// Workspace of one problem slot: source fields, intermediates, first
// convolution output, aux block and Schur vectors.
struct gpf_workspace {
  int n = 0, ns = 0, nv = 0;
  gpf::DevBuf w32, w64, x32, x64, s64, aux, part, rhs, y, fsurf;
  gpf::DevBuf xb;   // compact band of the first convolution's column pass
  gpf::DevBuf bin_cnt, bin_start, items, rank, sorted, halo, splits, splitwin;
  // band: rows of a body's band (16-row groups), 0 without a body
  gpf_status ensure(int n, bool need32, bool need64, int ns, int band = 0);
  gpf_status ensure_vortices(int nv);
};

// workspace and descriptor ring of one stream (GPF_PLAN_MULTISTREAM)
struct gpf_stream_slot {
  hipStream_t stream = nullptr;
  gpf_workspace ws;
  gpf::DescRing ring;
};

struct gpf_plan {
  gpf_ctx *ctx = nullptr;
  gpf_grid grid{};
  unsigned flags = 0;
  bool fp64 = false;          // field type double
  double gauge_c = 0.0;       // spectrum shift restored as -c * gamma_src
  gpf::DevBuf lgf;            // (n+1)^2 double LGF table
  gpf::DevBuf spec32, spec64; // (n+1)^2 scaled, centred spectrum
  gpf::DevBuf tw32, tw64;     // 2n twiddles exp(-2 pi i k / 2n)
  gpf::DevBuf status_scratch; // status word for building blocks given none
  gpf_workspace ws;           // workspace of plain solves
  gpf::DescRing ring;         // descriptors of plain solves
  gpf::KernelTimer timer;
  bool timing = false;
  std::mutex slots_mu;
  std::vector<std::unique_ptr<gpf_stream_slot>> slots;   // GPF_PLAN_MULTISTREAM
  gpf_status ensure_fp64();
  gpf_status slot_for(hipStream_t s, gpf_stream_slot **out);
  // pressure work fields (n x n FP64: sheet vorticity, face terms, source,
  // convolution result) and the FP64 convolution intermediate; ns scratch
  gpf::DevBuf pres_w, pres_fx, pres_fy, pres_src, pres_tmp, pres_X, pres_ddt;
};

struct gpf_body {
  gpf_plan *plan = nullptr;
  int ns = 0;
  int nedge = 0;
  int edges[GPF_MAX_EDGES] = {0};
  double gamma0 = 0.0;
  double amp = 0.0;
  bool conv1_fp64 = false;
  int row_lo = 0, row_hi = 0; // grid rows read by the surface stencils
  gpf::DevBuf xs, ys, ds;     // surface geometry (double)
  gpf::DevBuf st_i, st_w;     // stencils: base (i0, j0) per point, 8 weights
  gpf::DevBuf rs_node, rs_off, rs_code;   // R_s as a gather (ProbDesc)
  int rs_nodes = 0;
  gpf::DevBuf sinv;           // ns x ns S^-1, row-major, FP64
  gpf::DevBuf f0;             // S^-1 1
  gpf::DevBuf ghat;           // S^-T dS
  gpf::DevBuf nx, ny;         // normals of the impulse's motion term (zeros: thin body)
  bool has_normals = false;
  // pressure: unit normals of the sides (+ side = normal side), the
  // stencils and Q = -(C_s L^-1 C_s^T)^+ C_s L^-1 R_s (column-major)
  bool closed = false, has_pressure = false;
  gpf::DevBuf pnx, pny, pst, qpres;
  double area = 0.0, xc = 0.0, yc = 0.0;   // enclosed area and centroid
  std::vector<double> hxs, hys, hds, hf0;  // host copies of the geometry and f0
  // parts (gpf_body_set_parts); nparts = 1 without
  int nparts = 1;
  std::vector<int> hpart;
  int edge_part[GPF_MAX_EDGES] = {0};
  gpf::DevBuf part, gpart, zpart, cpart;
  double mom_x = 0.0, mom_y = 0.0, mom_r2 = 0.0;  // moments of fhat0 = dS f0
};

struct gpf_batch {
  static constexpr int kMaxLanes = 4;
  gpf_ctx *ctx = nullptr;
  int max_problems = 0;
  std::vector<gpf_workspace *> ws;
  gpf::DescRing ring;
  // lanes > 1: the batch is split over that many internal streams, forked
  // from and joined to the caller's stream with events
  int lanes = 1;
  // batches of several grid sizes run merged (one launch per stage over all
  // sizes): 1 with the side stream below, 2 on the caller's stream alone;
  // 0 runs them group by group
  int merge = 1;
  // with hw_all set (the request server's batches), every workspace of a
  // call is kept at the high-water sizes: the largest grid, vortex count,
  // surface and band the batch has held, and whether FP32 / FP64 fields were
  // needed, which the server raises to its own admission marks before each
  // batch.  A slot grown only to the problem in hand grows again, and
  // hipFree then waits for the whole device, each time a larger problem
  // than it has held lands on it.  Other batches size each slot to its
  // problem (a mix of very different sizes would otherwise multiply the
  // largest problem's footprint by the slot count).
  bool hw_all = false;
  int hw_n = 0, hw_nv = 0, hw_ns = 0, hw_band = 0;
  bool hw_w32 = false, hw_w64 = false;
  hipStream_t lane_stream[kMaxLanes] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kMaxLanes] = {};
  // side stream of merged batches (created at the first merged batch with
  // both precision classes): the class with an FP64 first convolution runs
  // there, velocities included, beside the FP32 class
  hipStream_t side = nullptr;
  hipEvent_t side_fork = nullptr, side_join = nullptr;
  // second side stream: the FP32 class's problems below its largest grid
  // size, beside those of the largest
  hipStream_t side2 = nullptr;
  hipEvent_t side2_join = nullptr;
  ~gpf_batch();
};

struct gpf_shed {
  gpf_plan *plan = nullptr;
  const gpf_body *body = nullptr;
  gpf_inputs in{};
  gpf_outputs out{};
  int nv = 0, capacity = 0, m = 0;
  int steps = 0;   // steps enqueued so far
  double dt = 0.0;
  double first[2 * GPF_MAX_EDGES] = {};     // offsets of each edge's first release
  double edge_xy[2 * GPF_MAX_EDGES] = {};   // edge points
  double *x = nullptr, *y = nullptr, *g = nullptr;   // caller's vortex arrays
  gpf::DevBuf last;   // per edge: index of its last nonzero release, or -1
  // GPF_PARTS: part of each shedding edge, and per part the circulation it
  // has released (device, GPF_MAX_PARTS doubles)
  int epart[GPF_MAX_EDGES] = {};
  gpf::DevBuf gw;
};

struct gpf_rk2 {
  gpf_plan *plan = nullptr;
  const gpf_body *body = nullptr;
  gpf_inputs in1{}, in2{};
  gpf_outputs out1{}, out2{};
  double *x = nullptr, *y = nullptr;
  double dt = 0.0;
  int nv = 0;
  bool use_graph = false;
  gpf::DevBuf xm, ym, u1, v1, u2, v2, psi, f, ft, sc, status;
  gpf_workspace ws;   // private: a captured step refers to its buffers
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> held;          // descriptor-ring slots the captured step replays
  hipEvent_t done = nullptr;      // recorded behind the last replay
  ~gpf_rk2();
};
