// Y = A X for a 0/1 pattern CSR matrix (the sparse matrix multiplication
// section of the paper): row i of Y is the sum of the rows of X named by row
// i's column indices.  There is no value array and no multiply.
//
// Scheduling (the paper's answer to power-law degree skew is dynamic
// partitions with work stealing; on the GPU the same skew is absorbed by
// degree binning).  Rows are visited in descending-degree order (either the
// handle's own numbering after degree relabelling, or through an order array)
// and cut into bins; ONE launch covers every bin, the workgroup index picking
// its bin from a small prefix table, heaviest bins first so long workgroups
// start early:
//   split  : degree > 16384 -> chunks of 8192 nonzeros, one workgroup each,
//            writing partial sums; a second small launch adds each row's
//            partials in chunk order, so results are deterministic
//   block  : 2048 < degree <= 16384 -> one 256-lane workgroup per row, LDS
//            reduction across its four wavefronts
//   group  : smaller rows -> groups of E*CPAD lanes per row inside a 64-wide
//            wavefront (E edge slots x CPAD column chunks), E chosen from the
//            degree so each lane gathers one or two X rows; cross-lane
//            butterfly reduction over the slots
//   zero   : empty rows -> store zeros, no index traffic
// Each lane gathers one 16-byte chunk of an X row per nonzero (VEC elements;
// CPAD chunks cover the b columns), so a row of X is read with full-width
// vector loads, the analogue of the paper's fixed-width vectorised row add.
// Column indices and Y are streamed with non-temporal accesses so that they do
// not evict X, which is the only operand with reuse.
#include "dev_common.h"
#include "fe_internal.h"

namespace fe {
namespace {

enum Kind : int32_t { K_ZERO = 0, K_GROUP = 1, K_BLOCK = 2, K_SPLIT = 3, K_WAVE = 4 };
constexpr int kMaxBins = 16;
constexpr int kWG = 256;

struct Bin {
  int32_t kind;
  int32_t E;      // edge slots per row (group kind)
  int64_t pos0;   // first position (in degree order) of the bin
  int64_t nrows;  // rows (or chunks for K_SPLIT)
  int64_t wg0;    // first workgroup of the bin
};

struct Plan {
  const int64_t* row_ptr;
  const int32_t* col;
  const int32_t* order;  // null: position == row
  const SplitChunk* chunks;
  void* partials;
  int32_t b;
  int32_t nbins;
  Bin bins[kMaxBins];
};

// Sum the X rows named by col[e], col[e + SLOTS], ... (< e1) into acc.  Each
// pass issues U index loads and then U gathers per lane before consuming any
// of them, so a whole row's traffic is in flight at once.  Out-of-range slots
// re-read the row's last index (a cache hit) and contribute zero, which keeps
// the loop free of divergent branches.
template <typename T, int VEC, int CPAD, int SLOTS, int U, typename A>
__device__ __forceinline__ void gather_rows(const Plan& P, const T* __restrict__ X, int64_t e,
                                            int64_t e1, int chunk, bool live, A* acc) {
  const int32_t* __restrict__ col = P.col;
  const int64_t b = P.b;
  const T* Xc = X + chunk * VEC;
  if (!live) return;
  for (; e < e1; e += U * SLOTS) {
    int32_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t idx = e + u * SLOTS;
      j[u] = __builtin_nontemporal_load(col + (idx < e1 ? idx : e1 - 1));
    }
    A v[U][VEC];
#pragma unroll
    for (int u = 0; u < U; ++u) load_vec<T, VEC>(Xc + j[u] * b, v[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = e + u * SLOTS < e1;
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[c] += ok ? v[u][c] : (A)0;
    }
  }
}

// Butterfly sum over the E slots of a group (slot stride CPAD lanes).
template <int E, int CPAD, typename A, int VEC>
__device__ __forceinline__ void reduce_slots(A* acc) {
#pragma unroll
  for (int off = E / 2; off >= 1; off >>= 1) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[v] += __shfl_xor(acc[v], off * CPAD, 64);
  }
}

template <typename T, int VEC, int CPAD, int E, int U>
__device__ __forceinline__ void run_group(const Plan& P, const Bin& B, int64_t local, const T* __restrict__ X,
                          T* __restrict__ Y) {
  using A = typename Acc<T>::type;
  constexpr int G = E * CPAD;
  constexpr int RPW = kWG / G;
  const int t = threadIdx.x;
  const int g = t / G, in = t % G, slot = in / CPAD, chunk = in % CPAD;
  const int64_t idx = local * RPW + g;
  if (idx >= B.nrows) return;  // whole group leaves together
  const int64_t pos = B.pos0 + idx;
  const int64_t row = P.order ? (int64_t)P.order[pos] : pos;
  const int64_t e0 = __builtin_nontemporal_load(P.row_ptr + row);
  const int64_t e1 = __builtin_nontemporal_load(P.row_ptr + row + 1);
  const bool live = chunk * VEC < P.b;
  A acc[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0;
  gather_rows<T, VEC, CPAD, E, U>(P, X, e0 + slot, e1, chunk, live, acc);
  reduce_slots<E, CPAD, A, VEC>(acc);
  if (slot == 0 && live) store_vec_nt<T, VEC>(Y + row * P.b + chunk * VEC, acc);
}

// One 256-lane workgroup over the nonzero range [e0, e1); returns the row sum
// in lanes t < CPAD of wave 0 (others hold garbage).
template <typename T, int VEC, int CPAD>
__device__ __forceinline__ void run_wg_range(const Plan& P, const T* __restrict__ X, int64_t e0,
                                             int64_t e1, typename Acc<T>::type* acc) {
  using A = typename Acc<T>::type;
  constexpr int SLOTS = kWG / CPAD;
  __shared__ A red[4][CPAD * VEC];
  const int t = threadIdx.x;
  const int slot = t / CPAD, chunk = t % CPAD;
  const bool live = chunk * VEC < P.b;
#pragma unroll
  for (int v = 0; v < VEC; ++v) acc[v] = 0;
  gather_rows<T, VEC, CPAD, SLOTS, 8>(P, X, e0 + slot, e1, chunk, live, acc);
  reduce_slots<64 / CPAD, CPAD, A, VEC>(acc);
  const int w = t >> 6, l = t & 63;
  if (l < CPAD) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) red[w][l * VEC + v] = acc[v];
  }
  __syncthreads();
  if (t < CPAD) {
#pragma unroll
    for (int v = 0; v < VEC; ++v)
      acc[v] = (red[0][t * VEC + v] + red[1][t * VEC + v]) + (red[2][t * VEC + v] + red[3][t * VEC + v]);
  }
}

template <typename T, int VEC, int CPAD>
__device__ __forceinline__ void run_block(const Plan& P, const Bin& B, int64_t local, const T* __restrict__ X,
                          T* __restrict__ Y) {
  using A = typename Acc<T>::type;
  const int64_t pos = B.pos0 + local;
  const int64_t row = P.order ? (int64_t)P.order[pos] : pos;
  const int64_t e0 = P.row_ptr[row], e1 = P.row_ptr[row + 1];
  A acc[VEC];
  run_wg_range<T, VEC, CPAD>(P, X, e0, e1, acc);
  const int t = threadIdx.x;
  if (t < CPAD && t * VEC < P.b) store_vec_nt<T, VEC>(Y + row * P.b + t * VEC, acc);
}

// A chunk of a hub row: its partial sum goes to the partials buffer; the
// combine kernel adds a row's partials in chunk order after this launch
// (stream order makes them visible without device-scope fences, which write
// back the L2 of every XCD on this part).
template <typename T, int VEC, int CPAD>
__device__ __forceinline__ void run_split(const Plan& P, const Bin& B, int64_t local,
                                          const T* __restrict__ X) {
  using A = typename Acc<T>::type;
  const int64_t ci = B.pos0 + local;
  const SplitChunk c = P.chunks[ci];
  A acc[VEC];
  run_wg_range<T, VEC, CPAD>(P, X, c.e0, c.e1, acc);
  const int t = threadIdx.x;
  A* part = reinterpret_cast<A*>(P.partials);
  if (t < CPAD && t * VEC < P.b) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) part[ci * P.b + t * VEC + v] = acc[v];
  }
}

template <typename T, int VEC, int CPAD>
__device__ __forceinline__ void run_zero(const Plan& P, const Bin& B, int64_t local, T* __restrict__ Y) {
  using A = typename Acc<T>::type;
  A z[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) z[v] = 0;
  const int64_t b = P.b;
  const int64_t nchunk = b / VEC;  // VEC divides b
  const int64_t i = local * kWG + threadIdx.x;  // chunk index inside the bin
  if (P.order == nullptr) {
    if (i < B.nrows * nchunk) store_vec_nt<T, VEC>(Y + B.pos0 * b + i * VEC, z);
  } else {
    if (i < B.nrows * nchunk) {
      const int64_t r = i / nchunk, c = i % nchunk;
      const int64_t row = P.order[B.pos0 + r];
      store_vec_nt<T, VEC>(Y + row * b + c * VEC, z);
    }
  }
}

template <typename T, int VEC, int CPAD>
__global__ __launch_bounds__(kWG) void spmm_kernel(Plan P, const T* __restrict__ X,
                                                   T* __restrict__ Y) {
  const int64_t wg = blockIdx.x;
  int bi = 0;
  while (bi + 1 < P.nbins && wg >= P.bins[bi + 1].wg0) ++bi;
  const Bin B = P.bins[bi];
  const int64_t local = wg - B.wg0;
  switch (B.kind) {
    case K_SPLIT:
      run_split<T, VEC, CPAD>(P, B, local, X);
      break;
    case K_BLOCK:
      run_block<T, VEC, CPAD>(P, B, local, X, Y);
      break;
    case K_ZERO:
      run_zero<T, VEC, CPAD>(P, B, local, Y);
      break;
    case K_WAVE:  // one wavefront (64 / CPAD slots) per row, long rows
      run_group<T, VEC, CPAD, 64 / CPAD, 8>(P, B, local, X, Y);
      break;
    default:  // short rows: E slots, at most two nonzeros per slot
      switch (B.E) {
        case 1: run_group<T, VEC, CPAD, 1, 2>(P, B, local, X, Y); break;
        case 2: if constexpr (2 * CPAD <= 64) run_group<T, VEC, CPAD, 2, 2>(P, B, local, X, Y); break;
        case 4: if constexpr (4 * CPAD <= 64) run_group<T, VEC, CPAD, 4, 2>(P, B, local, X, Y); break;
        case 8: if constexpr (8 * CPAD <= 64) run_group<T, VEC, CPAD, 8, 2>(P, B, local, X, Y); break;
        case 16: if constexpr (16 * CPAD <= 64) run_group<T, VEC, CPAD, 16, 2>(P, B, local, X, Y); break;
        case 32: if constexpr (32 * CPAD <= 64) run_group<T, VEC, CPAD, 32, 2>(P, B, local, X, Y); break;
      }
  }
}

// Y row of hub `pos` = sum of its chunk partials, in chunk order.
template <typename T>
__global__ __launch_bounds__(64) void split_combine_kernel(const SplitChunk* __restrict__ chunks,
                                                           const int64_t* __restrict__ first_chunk,
                                                           const int32_t* __restrict__ order,
                                                           const void* __restrict__ partials,
                                                           int32_t b, T* __restrict__ Y) {
  using A = typename Acc<T>::type;
  const int64_t pos = blockIdx.x;
  const int64_t f = first_chunk[pos];
  const int32_t cnt = chunks[f].count;
  const A* part = reinterpret_cast<const A*>(partials);
  const int64_t row = order ? (int64_t)order[pos] : pos;
  for (int c = threadIdx.x; c < b; c += 64) {
    A s = 0;
    for (int32_t i = 0; i < cnt; ++i) s += part[(f + i) * b + c];
    Y[row * b + c] = to_storage<T, A>(s);
  }
}

int ilog2_floor(int64_t x) {
  int r = -1;
  while (x) {
    x >>= 1;
    ++r;
  }
  return r;
}

// Build the bin table for column-chunk count CPAD.  Positions run over rows
// in descending-degree order; rows_deg_gt gives the bin boundaries.
fe_status make_plan(const Csr& A, int32_t b, int cpad, int vec, Plan* P, int64_t* total_wg) {
  P->row_ptr = A.d_row_ptr;
  P->col = A.d_col;
  P->order = A.d_order;
  P->chunks = A.d_chunks;
  P->partials = A.d_partials;
  P->b = b;
  int nb = 0;
  int64_t wg = 0;
  auto add_n = [&](int32_t kind, int32_t E, int64_t pos0, int64_t nrows, int64_t nwg) {
    if (nrows <= 0 || nb >= kMaxBins) return;
    Bin& B = P->bins[nb++];
    B.kind = kind;
    B.E = E;
    B.pos0 = pos0;
    B.nrows = nrows;
    B.wg0 = wg;
    wg += nwg;
  };
  auto add = [&](int32_t kind, int32_t E, int64_t pos0, int64_t nrows, int64_t per_wg) {
    add_n(kind, E, pos0, nrows, (nrows + per_wg - 1) / per_wg);
  };
  const int ecap = 64 / cpad;
  // split chunks (positions [0, n_split_rows) in degree order)
  add(K_SPLIT, 0, 0, A.n_chunks, 1);
  const int64_t c_split = rows_deg_gt(A, kSplitThreshold);
  const int64_t c_block = rows_deg_gt(A, kBlockThreshold);
  add(K_BLOCK, 0, c_split, c_block - c_split, 1);
  // wave-size groups: ecap < deg <= kBlockThreshold
  const int64_t c_ecap = rows_deg_gt(A, ecap);
  add(K_WAVE, ecap, c_block, c_ecap - c_block, kWG / (ecap * cpad));
  // group bins: deg in (2^(g-1), 2^g] with E = 2^(g-1) < ecap, then deg == 1 with E = 1
  int64_t hi_pos = c_ecap;
  for (int g = ilog2_floor(ecap); g >= 1; --g) {
    const int64_t lo = (int64_t)1 << (g - 1);  // deg > lo
    const int64_t c_lo = rows_deg_gt(A, lo);
    const int E = (int)lo;
    add(K_GROUP, E, hi_pos, c_lo - hi_pos, kWG / (E * cpad));
    hi_pos = c_lo;
  }
  const int64_t c_zero = rows_deg_gt(A, 0);
  add(K_GROUP, 1, hi_pos, c_zero - hi_pos, kWG / cpad);
  // empty rows: one VEC-chunk store per lane
  const int64_t zchunks = (A.n - c_zero) * (b / vec);
  add_n(K_ZERO, 0, c_zero, A.n - c_zero, (zchunks + kWG - 1) / kWG);
  P->nbins = nb;
  *total_wg = wg;
  return FE_OK;
}

template <typename T, int VEC, int CPAD>
fe_status launch_t(const Csr& A, const void* X, void* Y, int32_t b, hipStream_t s) {
  Plan P;
  int64_t wg = 0;
  FE_TRY(make_plan(A, b, CPAD, VEC, &P, &wg));
  if (wg == 0) return FE_OK;
  if (wg > 0x7FFFFFFF) return fail(FE_EUNSUPPORTED, "spmm grid too large");
  hipLaunchKernelGGL((spmm_kernel<T, VEC, CPAD>), dim3((uint32_t)wg), dim3(kWG), 0, s, P,
                     static_cast<const T*>(X), static_cast<T*>(Y));
  FE_HIP(hipGetLastError());
  if (A.n_split_rows > 0) {
    hipLaunchKernelGGL((split_combine_kernel<T>), dim3((uint32_t)A.n_split_rows), dim3(64), 0, s,
                       A.d_chunks, A.d_first_chunk, A.d_order, A.d_partials, b,
                       static_cast<T*>(Y));
    FE_HIP(hipGetLastError());
  }
  return FE_OK;
}

// VEC: largest power of two dividing b with VEC*sizeof(T) <= 16 and the
// pointers aligned to it; CPAD: next power of two >= b / VEC.
template <typename T>
fe_status dispatch(const Csr& A, const void* X, void* Y, int32_t b, hipStream_t s) {
  constexpr int maxvec = 16 / sizeof(T);
  int vec = 1;
  const uintptr_t align = reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y);
  while (vec * 2 <= maxvec && b % (vec * 2) == 0 && align % (vec * 2 * sizeof(T)) == 0) vec *= 2;
  int c = b / vec, cpad = 1;
  while (cpad < c) cpad *= 2;
#define FE_CASE(V, C) \
  if (vec == V && cpad == C) return launch_t<T, V, C>(A, X, Y, b, s);
  FE_CASE(1, 1) FE_CASE(1, 2) FE_CASE(1, 4) FE_CASE(1, 8) FE_CASE(1, 16) FE_CASE(1, 32)
  FE_CASE(1, 64) FE_CASE(2, 1) FE_CASE(2, 2) FE_CASE(2, 4) FE_CASE(2, 8) FE_CASE(2, 16)
  FE_CASE(2, 32)
  if constexpr (maxvec >= 4) {
    FE_CASE(4, 1) FE_CASE(4, 2) FE_CASE(4, 4) FE_CASE(4, 8) FE_CASE(4, 16)
  }
  if constexpr (maxvec >= 8) {
    FE_CASE(8, 1) FE_CASE(8, 2) FE_CASE(8, 4) FE_CASE(8, 8)
  }
#undef FE_CASE
  return fail(FE_EUNSUPPORTED, "spmm: no kernel for b=%d vec=%d", b, vec);
}

}  // namespace

fe_status spmm_launch(const Csr& A, const void* X, void* Y, int32_t b, fe_dtype dt,
                      hipStream_t s) {
  switch (dt) {
    case FE_F64: return dispatch<double>(A, X, Y, b, s);
    case FE_F32: return dispatch<float>(A, X, Y, b, s);
    case FE_BF16: return dispatch<bf16_t>(A, X, Y, b, s);
  }
  return fail(FE_EINVAL, "spmm: bad dtype");
}

}  // namespace fe
