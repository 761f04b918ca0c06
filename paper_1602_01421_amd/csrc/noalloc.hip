// fe_gram_noalloc: fe_gram without any allocation, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
//
// fe_gram's row-interval partial sums (the first stage of its two-stage
// reduction) go to a buffer it allocates per call; here they go to a
// file-scope device array instead.  Each GPU holds its own copy of the array
// until the process ends, at an address read once per device with
// hipGetSymbolAddress (the array's name is not a device address in host
// code).  Every call on a GPU shares that GPU's copy: calls that overlap in
// time on one GPU (different streams, or a second host thread) race.  The
// Gram kernels write every partial they later read, so nothing needs clearing
// between calls.
#include <mutex>

#include "fe_internal.h"

namespace fe {
namespace {

constexpr size_t kScratchDoubles = size_t(1) << 20;  // 8 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {nullptr};

// Device address of this GPU's copy of `scratch` (looked up once per device,
// with that device current).
fe_status scratch_ptr(double** out) {
  int dev = 0;
  FE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FE_EUNSUPPORTED, "fe_gram_noalloc: device %d", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FE_EDEVICE, "fe_gram_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return FE_OK;
}

}  // namespace
}  // namespace fe

using namespace fe;

extern "C" fe_status fe_gram_noalloc(const void* V, int32_t nblk, int64_t stride, const void* W,
                                     int64_t n, int32_t b, fe_dtype dt, double alpha, double* C,
                                     void* stream) {
  if (!V || !W || !C) return fail(FE_EINVAL, "fe_gram_noalloc: NULL argument");
  if (n < 1 || b < 1 || b > 64 || nblk < 1)
    return fail(FE_EINVAL, "fe_gram_noalloc: bad sizes n=%lld b=%d nblk=%d", (long long)n, b, nblk);
  if (!dtype_ok(dt)) return fail(FE_EINVAL, "fe_gram_noalloc: bad dtype");
  if (nblk > 1 && stride < n * b) return fail(FE_EINVAL, "fe_gram_noalloc: blk_stride < n*b");
  if ((int64_t)nblk * b > 1024) return fail(FE_EINVAL, "fe_gram_noalloc: k = nblk*b > 1024");
  if ((reinterpret_cast<uintptr_t>(V) | reinterpret_cast<uintptr_t>(W)) % dtype_size(dt))
    return fail(FE_EINVAL, "fe_gram_noalloc: misaligned V or W");
  const size_t need = gram_sets_partials_doubles(n, nblk * b, b);
  if (need > kScratchDoubles)
    return fail(FE_EUNSUPPORTED,
                "fe_gram_noalloc: needs %zu partial doubles, the static scratch holds %zu "
                "(k*b <= 2048 at any n)", need, kScratchDoubles);
  double* part = nullptr;
  FE_TRY(scratch_ptr(&part));
  return gram_launch(V, nblk, stride, W, n, b, dt, alpha, C, part, (hipStream_t)stream);
}
