// The sparse product's memory traffic without its rows, as a measurement of
// the product's ceiling on a given matrix: every stored column index, in
// storage order, fetches its X row in the same VEC-element chunks as the
// product (CPAD lanes per row, consecutive lanes on consecutive nonzeros, the
// index stream read non-temporally), and the sums are only reduced per
// workgroup.  Its time is what the product's gathers alone cost on this
// matrix.  The same kernel over a caller's index stream measures what another
// order of the same gathers would cost.
#include "dev_common.h"
#include "fe_internal.h"

namespace fe {
namespace {

constexpr int kWG = 256;
constexpr int kGatherSets = 16384;

// CLAMP: indices from a caller's stream are clamped to [0, n) (the product's own
// column indices are valid by construction).
template <typename T, int VEC, int CPAD, bool CLAMP>
__global__ __launch_bounds__(kWG) void gather_bound_kernel(const int32_t* __restrict__ col,
                                                           int64_t nnz, const T* __restrict__ X,
                                                           int32_t b, int64_t n,
                                                           double* __restrict__ out) {
  using A = typename Acc<T>::type;
  constexpr int U = 8;
  constexpr int SLOTS = kWG / CPAD;
  const int t = threadIdx.x, slot = t / CPAD, chunk = t % CPAD;
  const int64_t nslots = (int64_t)gridDim.x * SLOTS;
  A acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0;
  if (chunk * VEC < b) {
    const T* Xc = X + chunk * VEC;
    for (int64_t e = (int64_t)blockIdx.x * SLOTS + slot; e < nnz; e += nslots * U) {
      int32_t j[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t q = e + u * nslots;
        j[u] = __builtin_nontemporal_load(col + (q < nnz ? q : nnz - 1));
      }
      A v[U][VEC];
      if constexpr (CLAMP) {
#pragma unroll
        for (int u = 0; u < U; ++u) j[u] = j[u] < 0 ? 0 : ((int64_t)j[u] >= n ? (int32_t)(n - 1) : j[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) load_vec<T, VEC>(Xc + (int64_t)j[u] * b, v[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool ok = e + u * nslots < nnz;
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[c] += ok ? v[u][c] : (A)0;
      }
    }
  }
  __shared__ double red[kWG];
  double sum = 0.0;
#pragma unroll
  for (int v = 0; v < VEC; ++v) sum += (double)acc[v];
  red[t] = sum;
  __syncthreads();
  for (int h = kWG / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) out[blockIdx.x] = red[0];
}

template <typename T>
fe_status gather_bound_t(const int32_t* idx, int64_t count, bool clamp, const void* X, int64_t n,
                         double* out, int32_t b, hipStream_t s) {
  constexpr int maxvec = 16 / sizeof(T);
  int vec = 1;
  const uintptr_t align = reinterpret_cast<uintptr_t>(X);
  while (vec * 2 <= maxvec && b % (vec * 2) == 0 && align % (vec * 2 * sizeof(T)) == 0) vec *= 2;
  int c = b / vec, cpad = 1;
  while (cpad < c) cpad *= 2;
  const T* Xp = static_cast<const T*>(X);
#define FE_GB(V, C)                                                                          \
  if (vec == V && cpad == C) {                                                               \
    if (clamp)                                                                               \
      hipLaunchKernelGGL((gather_bound_kernel<T, V, C, true>), dim3(kGatherSets), dim3(kWG),  \
                         0, s, idx, count, Xp, b, n, out);                                   \
    else                                                                                     \
      hipLaunchKernelGGL((gather_bound_kernel<T, V, C, false>), dim3(kGatherSets), dim3(kWG), \
                         0, s, idx, count, Xp, b, n, out);                                   \
    FE_HIP(hipGetLastError());                                                               \
    return FE_OK;                                                                            \
  }
  FE_GB(1, 1) FE_GB(1, 2) FE_GB(1, 4) FE_GB(1, 8) FE_GB(1, 16) FE_GB(1, 32) FE_GB(1, 64)
  FE_GB(2, 1) FE_GB(2, 2) FE_GB(2, 4) FE_GB(2, 8) FE_GB(2, 16) FE_GB(2, 32)
  if constexpr (maxvec >= 4) { FE_GB(4, 1) FE_GB(4, 2) FE_GB(4, 4) FE_GB(4, 8) FE_GB(4, 16) }
  if constexpr (maxvec >= 8) { FE_GB(8, 1) FE_GB(8, 2) FE_GB(8, 4) FE_GB(8, 8) }
#undef FE_GB
  return fail(FE_EUNSUPPORTED, "gather bound: no kernel for b=%d vec=%d", b, vec);
}

}  // namespace

int32_t gather_bound_sets() { return kGatherSets; }

fe_status gather_rows_launch(const int32_t* idx, int64_t count, bool clamp, const void* X,
                             int64_t n, double* out, int32_t b, fe_dtype dt, hipStream_t s) {
  switch (dt) {  // count == 0: every workgroup writes 0
    case FE_F64: return gather_bound_t<double>(idx, count, clamp, X, n, out, b, s);
    case FE_F32: return gather_bound_t<float>(idx, count, clamp, X, n, out, b, s);
    case FE_BF16: return gather_bound_t<bf16_t>(idx, count, clamp, X, n, out, b, s);
  }
  return fail(FE_EINVAL, "gather bound: bad dtype");
}

fe_status gather_bound_launch(const Csr& A, const void* X, double* out, int32_t b, fe_dtype dt,
                              hipStream_t s) {
  return gather_rows_launch(A.d_col, A.nnz, false, X, A.n, out, b, dt, s);
}

}  // namespace fe
