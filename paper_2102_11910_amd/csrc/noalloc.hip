// Allocation-free variant of the LGF convolution s = -L^-1 w (Sec. 2.1,
// eq. poisson), for callers that cannot allocate device memory: code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
//
// gpf_convolve keeps its (n+1) x n complex intermediate in the plan's
// workspace and its launch descriptor in the plan's descriptor ring (a
// pinned host buffer copied to the device).  This variant keeps both in one
// file-scope device array instead: the descriptor is written by a one-wave
// kernel that takes it by value, so no host-to-device copy is enqueued and
// nothing is allocated.  The transform kernels are the ones gpf_convolve
// launches.
//
// The array lives on every device the library runs on until the process
// ends.  Its address on a device is taken once (hipGetSymbolAddress, with
// that device current) when a context is created on it; host code uses only
// that address, never the array's name, which is a host-side stand-in.
// Every call on a device shares its array: calls that overlap on one device
// race.  No field of the array needs to start at zero (the row pass writes
// every element of the intermediate that the later passes read).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "gpf_internal.h"

namespace gpf {
namespace {

constexpr size_t kDescBytes = 256;
static_assert(sizeof(ConvDesc) <= kDescBytes, "ConvDesc must fit its scratch slot");
// intermediate of the largest supported grid: FP32 n = 2048 (and FP64 n = 1024)
constexpr size_t kIntermediateBytes = (size_t)2049 * 2048 * 8;
constexpr size_t kScratchBytes = kDescBytes + kIntermediateBytes;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

__global__ void k_put_desc(ConvDesc cd, ConvDesc *dst) {
  // one wave copies the descriptor word by word with vector stores
  const unsigned *src = reinterpret_cast<const unsigned *>(&cd);
  unsigned *d = reinterpret_cast<unsigned *>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(ConvDesc) / 4); i += blockDim.x) d[i] = src[i];
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

gpf_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(GPF_E_UNSUPPORTED, "allocation-free scratch: device index above 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return GPF_OK;
  int cur = -1;
  GPF_HIP(hipGetDevice(&cur));
  if (cur != device) return fail(GPF_E_INVALID, "allocation-free scratch: device not current");
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(GPF_E_DEVICE, "allocation-free scratch: hipGetSymbolAddress failed");
  g_scratch[device] = p;
  return GPF_OK;
}

}  // namespace gpf

using namespace gpf;

extern "C" gpf_status gpf_convolve_noalloc(gpf_plan *plan, const void *d_w, void *d_s,
                                           double gamma_src, void *hip_stream) {
  if (!plan || !d_w || !d_s || !std::isfinite(gamma_src))
    return fail(GPF_E_INVALID, "gpf_convolve_noalloc: bad arguments");
  const int n = plan->grid.n;
  const size_t need = (size_t)(n + 1) * n * 2 * (plan->fp64 ? sizeof(double) : sizeof(float));
  if (need > kIntermediateBytes)
    return fail(GPF_E_UNSUPPORTED,
                "gpf_convolve_noalloc: the intermediate of this grid exceeds the fixed scratch "
                "(FP32 n <= 2048, FP64 n <= 1024)");
  const int dev = plan->ctx->device;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
  }
  if (!base) return fail(GPF_E_INVALID, "gpf_convolve_noalloc: scratch not set up on this device");
  GPF_HIP(hipSetDevice(dev));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  TimerScope none(nullptr);
  ConvDesc cd;
  std::memset(&cd, 0, sizeof(cd));
  cd.in = const_cast<void *>(d_w);
  cd.X = static_cast<char *>(base) + kDescBytes;
  cd.out = d_s;
  cd.spec = plan->fp64 ? plan->spec64.p : plan->spec32.p;
  cd.tw = plan->fp64 ? plan->tw64.p : plan->tw32.p;
  cd.gamma = nullptr;
  cd.gamma_val = gamma_src;
  cd.c = plan->gauge_c;
  cd.zero_in = 0;
  cd.row_lo = 0;
  cd.row_hi = n - 1;
  ConvDesc *dd = static_cast<ConvDesc *>(base);
  hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, cd, dd);
  GPF_HIP(hipGetLastError());
  const ConvSched sc = plan->ctx->sched_for(n, plan->fp64, 1);
  const int x = plan->ctx->xcds;
  if (plan->fp64)
    GPF_HIP((launch_convolve<double, double>(n, dd, 1, x, 0, s, sc)));
  else
    GPF_HIP((launch_convolve<float, float>(n, dd, 1, x, 0, s, sc)));
  return GPF_OK;
}
