// Allocation-free FP64 direct forces (tg_direct_fp64_noalloc): the kernels
// and split of tg_direct_fp64, with no context.  The device memory beyond
// the caller's inputs and outputs (the segment table and the per-block
// compensated partial sums) is one fixed array of the library, `scratch`,
// which every GPU the library runs on holds until the process ends.
//
// Host code never passes the array's name to a kernel: on the host it is a
// stand-in, not a device address.  The address of each GPU's copy comes
// from hipGetSymbolAddress, taken once per device with that device current,
// and only that address reaches the kernels.
#include <atomic>
#include <mutex>

#include "tg_internal.h"

namespace {

constexpr int kMaxSeg = TG_NOALLOC_MAX_SEG;
constexpr size_t kSegBytes = 4096;                        // segment table region
constexpr int64_t kPartDoubles = (int64_t)8 * 131072;     // as a context's partials
constexpr size_t kScratchBytes = kSegBytes + sizeof(double) * (size_t)kPartDoubles;
static_assert(sizeof(int64_t) * 2 * (kMaxSeg + 1) <= kSegBytes, "segment table region");
static_assert(kScratchBytes == TG_NOALLOC_SCRATCH_BYTES, "scratch size stated in tg.h");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
std::atomic<unsigned char *> g_ptr[kMaxDevices];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace tg {
namespace {

// The segment offsets travel by value in the kernel arguments and are
// stored into the scratch table, so the call needs no host-to-device copy.
struct SegArg {
  int64_t v[2 * (kMaxSeg + 1)];
  int32_t n;
};

__global__ __launch_bounds__(64) void k_store_segs(SegArg a, int64_t *__restrict__ dst) {
  for (int t = threadIdx.x; t < a.n; t += blockDim.x) dst[t] = a.v[t];
}

// Device address of the current device's scratch (null on failure, with
// *err set to a static message).
unsigned char *scratch_here(const char **err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    *err = "tg_direct_fp64_noalloc: hipGetDevice failed";
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *err = "tg_direct_fp64_noalloc: device ordinal beyond 63";
    return nullptr;
  }
  unsigned char *p = g_ptr[dev].load(std::memory_order_acquire);
  if (p) return p;
  std::lock_guard<std::mutex> lock(g_mu);
  p = g_ptr[dev].load(std::memory_order_relaxed);
  if (p) return p;
  void *addr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !addr) {
    *err = e != hipSuccess ? hipGetErrorString(e)
                           : "tg_direct_fp64_noalloc: no scratch address";
    return nullptr;
  }
  p = static_cast<unsigned char *>(addr);
  g_ptr[dev].store(p, std::memory_order_release);
  return p;
}

}  // namespace
}  // namespace tg

using namespace tg;

extern "C" tg_status tg_direct_fp64_noalloc(
    const double *spos, const double *sm, const double *seps, int64_t ns,
    const double *tpos, const double *teps, int64_t nt, const int64_t *sseg,
    const int64_t *tseg, int32_t nseg, int32_t self_pairs, int32_t accumulate,
    int32_t softening, double *acc, double *pot, void *stream) {
  if (ns < 0 || nt < 0) return fail_literal(TG_EINVAL, "tg_direct_fp64_noalloc: negative size");
  if (softening != TG_SOFT_PLUMMER && softening != TG_SOFT_SPLINE)
    return fail_literal(TG_EINVAL, "tg_direct_fp64_noalloc: unknown softening");
  if (nseg < 0) return fail_literal(TG_EINVAL, "tg_direct_fp64_noalloc: nseg < 0");
  if (nseg > kMaxSeg)
    return fail_literal(TG_ECAPACITY,
                        "tg_direct_fp64_noalloc: nseg exceeds TG_NOALLOC_MAX_SEG (64)");
  if (nt == 0) return TG_OK;
  if (!tpos || !teps || !acc || (ns > 0 && (!spos || !sm || !seps)))
    return fail_literal(TG_EINVAL, "tg_direct_fp64_noalloc: NULL pointer");
  if (self_pairs && ns != nt)
    return fail_literal(TG_EINVAL, "tg_direct_fp64_noalloc: self_pairs needs ns == nt");
  SegArg a;
  int nseg_eff = nseg;
  if (nseg == 0) {
    a.v[0] = 0; a.v[1] = ns; a.v[2] = 0; a.v[3] = nt;
    nseg_eff = 1;
  } else {
    if (!sseg || !tseg) return fail_literal(TG_EINVAL, "tg_direct_fp64_noalloc: NULL segments");
    for (int s = 0; s <= nseg; ++s) { a.v[s] = sseg[s]; a.v[nseg + 1 + s] = tseg[s]; }
    if (a.v[0] != 0 || a.v[nseg] != ns || a.v[nseg + 1] != 0 || a.v[2 * nseg + 1] != nt)
      return fail_literal(TG_EINVAL, "tg_direct_fp64_noalloc: segment offsets must span 0..n");
    for (int s = 0; s < nseg; ++s)
      if (a.v[s + 1] < a.v[s] || a.v[nseg + 2 + s] < a.v[nseg + 1 + s])
        return fail_literal(TG_EINVAL, "tg_direct_fp64_noalloc: segment offsets not ascending");
  }
  a.n = 2 * (nseg_eff + 1);
  int64_t max_src = 0;
  for (int s = 0; s < nseg_eff; ++s) max_src = std::max(max_src, a.v[s + 1] - a.v[s]);
  const char *err = nullptr;
  unsigned char *base = scratch_here(&err);
  if (!base) return fail_literal(TG_EHIP, err);
  int64_t *dseg = reinterpret_cast<int64_t *>(base);
  double *part = reinterpret_cast<double *>(base + kSegBytes);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_store_segs, dim3(1), dim3(64), 0, st, a, dseg);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    const DirectEnv env{st, softening, part, kPartDoubles};
    e = launch_direct_env(env, dseg, spos, sm, seps, 0.0, tpos, teps, nt, nseg_eff, max_src,
                          self_pairs, accumulate, acc, pot);
  }
  if (e != hipSuccess) return fail_literal(TG_EHIP, hipGetErrorString(e));
  return TG_OK;
}
