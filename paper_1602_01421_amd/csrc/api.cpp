// C ABI: errors, CSR handles (graph -> pattern CSR on the host, then upload),
// and the validated entry points of the sparse and dense kernels.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "fe_internal.h"

namespace fe {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

fe_status fail(fe_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

void clear_error() { g_err.clear(); }

// ------------------------------------------------------------ host threads
static int host_threads() {
  int t = (int)std::thread::hardware_concurrency();
  if (const char* e = getenv("OMP_NUM_THREADS")) {
    int v = atoi(e);
    if (v > 0) t = std::min(t > 0 ? t : v, v);
  }
  return std::max(1, std::min(t, 64));
}

// f(begin, end) over [0, n) in dynamically claimed chunks
template <class F>
static void parallel_chunks(int64_t n, int64_t chunk, F f) {
  const int T = host_threads();
  if (T == 1 || n <= chunk) {
    f((int64_t)0, n);
    return;
  }
  std::atomic<int64_t> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t)
    th.emplace_back([&] {
      for (;;) {
        int64_t b = next.fetch_add(chunk);
        if (b >= n) break;
        f(b, std::min(n, b + chunk));
      }
    });
  for (auto& x : th) x.join();
}

int64_t rows_deg_gt(const Csr& A, int64_t t) {
  if (t <= 0) return A.cnt_gt[0];
  int e = 0;
  while (((int64_t)1 << e) < t) ++e;
  return A.cnt_gt[std::min(e + 1, 33)];
}

// Rows ordered by descending degree, ties by ascending id (stable counting sort).
static std::vector<int32_t> degree_order(const std::vector<int64_t>& row_ptr, int64_t n,
                                         int64_t max_deg) {
  std::vector<int64_t> start((size_t)max_deg + 2, 0);
  for (int64_t i = 0; i < n; ++i) start[(size_t)(row_ptr[i + 1] - row_ptr[i])]++;
  int64_t acc = 0;
  for (int64_t d = max_deg; d >= 0; --d) {
    int64_t c = start[(size_t)d];
    start[(size_t)d] = acc;
    acc += c;
  }
  std::vector<int32_t> order((size_t)n);
  for (int64_t i = 0; i < n; ++i) order[(size_t)start[(size_t)(row_ptr[i + 1] - row_ptr[i])]++] = (int32_t)i;
  return order;
}

static void free_device(Csr* A) {
  hipFree(A->d_row_ptr);
  hipFree(A->d_col);
  hipFree(A->d_order);
  hipFree(A->d_perm);
  hipFree(A->d_chunks);
  hipFree(A->d_first_chunk);
  hipFree(A->d_partials);
  A->d_row_ptr = nullptr;
  A->d_col = nullptr;
  A->d_order = A->d_perm = nullptr;
  A->d_chunks = nullptr;
  A->d_first_chunk = nullptr;
  A->d_partials = nullptr;
}

template <class T>
static fe_status upload(T** dptr, const T* h, size_t count) {
  if (count == 0) {
    *dptr = nullptr;
    return FE_OK;
  }
  hipError_t e = hipMalloc((void**)dptr, count * sizeof(T));
  if (e != hipSuccess) return fail(FE_ENOMEM, "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
  FE_HIP(hipMemcpy(*dptr, h, count * sizeof(T), hipMemcpyHostToDevice));
  return FE_OK;
}

// Finalise a host CSR (rows strictly sorted): optional degree relabelling,
// degree census, hub chunk table, upload.
fe_status csr_upload(Csr* A, std::vector<int64_t>&& row_ptr, std::vector<int32_t>&& col,
                     bool relabel) {
  const int64_t n = (int64_t)row_ptr.size() - 1;
  int64_t max_deg = 0;
  for (int64_t i = 0; i < n; ++i) max_deg = std::max(max_deg, row_ptr[i + 1] - row_ptr[i]);
  std::vector<int32_t> order = degree_order(row_ptr, n, max_deg);
  if (relabel) {
    std::vector<int32_t> inv((size_t)n);
    for (int64_t i = 0; i < n; ++i) inv[(size_t)order[i]] = (int32_t)i;
    std::vector<int64_t> rp2((size_t)n + 1);
    rp2[0] = 0;
    for (int64_t i = 0; i < n; ++i)
      rp2[i + 1] = rp2[i] + (row_ptr[order[i] + 1] - row_ptr[order[i]]);
    std::vector<int32_t> col2(col.size());
    parallel_chunks(n, 4096, [&](int64_t b, int64_t e) {
      for (int64_t r = b; r < e; ++r) {
        const int64_t o = order[r];
        int32_t* dst = col2.data() + rp2[r];
        const int64_t d = row_ptr[o + 1] - row_ptr[o];
        for (int64_t t = 0; t < d; ++t) dst[t] = inv[(size_t)col[row_ptr[o] + t]];
        std::sort(dst, dst + d);
      }
    });
    row_ptr.swap(rp2);
    col.swap(col2);
    A->perm = order;  // new -> old
    A->relabeled = true;
  } else {
    A->perm.clear();
    A->relabeled = false;
  }
  A->n = n;
  A->nnz = row_ptr[n];
  A->max_deg = max_deg;
  // census: cnt_gt[0] = #deg > 0; cnt_gt[i] = #deg > 2^(i-1)
  for (int i = 0; i < 34; ++i) A->cnt_gt[i] = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t d = row_ptr[i + 1] - row_ptr[i];
    if (d > 0) A->cnt_gt[0]++;
    for (int e = 0; e < 33; ++e) {
      if (d > ((int64_t)1 << e)) A->cnt_gt[e + 1]++;
      else break;
    }
  }
  // hub chunks: positions [0, n_split) in degree order
  const int64_t n_split = rows_deg_gt(*A, kSplitThreshold);
  std::vector<SplitChunk> chunks;
  std::vector<int64_t> first_chunk;
  for (int64_t pos = 0; pos < n_split; ++pos) {
    const int64_t row = relabel ? pos : order[pos];
    const int64_t e0 = row_ptr[row], e1 = row_ptr[row + 1];
    const int32_t cnt = (int32_t)((e1 - e0 + kSplitChunk - 1) / kSplitChunk);
    const int32_t first = (int32_t)chunks.size();
    first_chunk.push_back(first);
    for (int32_t c = 0; c < cnt; ++c) {
      SplitChunk s;
      s.e0 = e0 + c * kSplitChunk;
      s.e1 = std::min(e1, s.e0 + kSplitChunk);
      s.pos = (int32_t)pos;
      s.first = first;
      s.count = cnt;
      s.pad = 0;
      chunks.push_back(s);
    }
  }
  A->n_split_rows = n_split;
  A->n_chunks = (int64_t)chunks.size();
  FE_HIP(hipGetDevice(&A->device));
  fe_status st = FE_OK;
  if ((st = upload(&A->d_row_ptr, row_ptr.data(), row_ptr.size())) != FE_OK) goto err;
  if ((st = upload(&A->d_col, col.data(), col.size())) != FE_OK) goto err;
  if (relabel) {
    if ((st = upload(&A->d_perm, A->perm.data(), A->perm.size())) != FE_OK) goto err;
  } else {
    if ((st = upload(&A->d_order, order.data(), order.size())) != FE_OK) goto err;
  }
  if (A->n_chunks) {
    if ((st = upload(&A->d_chunks, chunks.data(), chunks.size())) != FE_OK) goto err;
    if ((st = upload(&A->d_first_chunk, first_chunk.data(), first_chunk.size())) != FE_OK) goto err;
    if (hipMalloc(&A->d_partials, sizeof(double) * 64 * A->n_chunks) != hipSuccess) {
      st = fail(FE_ENOMEM, "hipMalloc for hub partials failed");
      goto err;
    }
  }
  return FE_OK;
err:
  free_device(A);
  return st;
}

}  // namespace fe

using namespace fe;

extern "C" {

const char* fe_last_error(void) { return g_err.c_str(); }

int32_t fe_version(void) { return 10000 * 0 + 100 * 3 + 0; }

fe_status fe_csr_build(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       uint32_t flags, fe_csr** out) {
  if (!out) return fail(FE_EINVAL, "fe_csr_build: out is NULL");
  if (n <= 0 || n > 0x7FFFFFFFLL) return fail(FE_EINVAL, "fe_csr_build: n=%lld out of range", (long long)n);
  if (m < 0 || (m > 0 && (!src || !dst))) return fail(FE_EINVAL, "fe_csr_build: bad edge list");
  const bool sym = flags & FE_SYMMETRIZE, dedupe = flags & FE_DEDUPE, noself = flags & FE_DROP_SELF;
  // validate ids
  std::atomic<bool> bad(false);
  parallel_chunks(m, 1 << 20, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i)
      if ((uint32_t)src[i] >= (uint64_t)n || (uint32_t)dst[i] >= (uint64_t)n) {
        bad = true;
        return;
      }
  });
  if (bad) return fail(FE_EINVAL, "fe_csr_build: vertex id out of [0, n)");
  try {
    std::vector<uint32_t> cnt((size_t)n, 0);
    parallel_chunks(m, 1 << 20, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e; ++i) {
        const int32_t u = src[i], v = dst[i];
        if (noself && u == v) continue;
        __atomic_fetch_add(&cnt[(size_t)u], 1u, __ATOMIC_RELAXED);
        if (sym) __atomic_fetch_add(&cnt[(size_t)v], 1u, __ATOMIC_RELAXED);
      }
    });
    std::vector<int64_t> off((size_t)n + 1);
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + cnt[(size_t)i];
    std::vector<int32_t> raw((size_t)off[n]);
    {
      std::vector<int64_t> cur(off.begin(), off.end() - 1);
      parallel_chunks(m, 1 << 20, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
          const int32_t u = src[i], v = dst[i];
          if (noself && u == v) continue;
          raw[(size_t)__atomic_fetch_add(&cur[(size_t)u], 1, __ATOMIC_RELAXED)] = v;
          if (sym) raw[(size_t)__atomic_fetch_add(&cur[(size_t)v], 1, __ATOMIC_RELAXED)] = u;
        }
      });
    }
    // sort (and dedupe) each row in place; new degree into cnt
    parallel_chunks(n, 2048, [&](int64_t b, int64_t e) {
      for (int64_t r = b; r < e; ++r) {
        int32_t* s = raw.data() + off[r];
        int32_t* t = raw.data() + off[r + 1];
        std::sort(s, t);
        cnt[(size_t)r] = (uint32_t)((dedupe ? std::unique(s, t) : t) - s);
      }
    });
    std::vector<int64_t> row_ptr((size_t)n + 1);
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[(size_t)i];
    std::vector<int32_t> col((size_t)row_ptr[n]);
    parallel_chunks(n, 4096, [&](int64_t b, int64_t e) {
      for (int64_t r = b; r < e; ++r)
        std::memcpy(col.data() + row_ptr[r], raw.data() + off[r], sizeof(int32_t) * cnt[(size_t)r]);
    });
    std::vector<int32_t>().swap(raw);
    std::vector<uint32_t>().swap(cnt);
    fe_csr* A = new fe_csr();
    fe_status st = csr_upload(A, std::move(row_ptr), std::move(col), flags & FE_RELABEL_BY_DEGREE);
    if (st != FE_OK) {
      delete A;
      return st;
    }
    *out = A;
    return FE_OK;
  } catch (const std::bad_alloc&) {
    return fail(FE_ENOMEM, "fe_csr_build: host allocation failed");
  }
}

fe_status fe_csr_from_csr(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                          uint32_t flags, fe_csr** out) {
  if (!out || !row_ptr) return fail(FE_EINVAL, "fe_csr_from_csr: NULL argument");
  if (n <= 0 || n > 0x7FFFFFFFLL) return fail(FE_EINVAL, "fe_csr_from_csr: n out of range");
  if (row_ptr[0] != 0) return fail(FE_EINVAL, "fe_csr_from_csr: row_ptr[0] != 0");
  for (int64_t i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return fail(FE_EINVAL, "fe_csr_from_csr: row_ptr decreases at %lld", (long long)i);
  if (row_ptr[n] > 0 && !col_idx) return fail(FE_EINVAL, "fe_csr_from_csr: col_idx is NULL");
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      if (col_idx[e] < 0 || col_idx[e] >= n)
        return fail(FE_EINVAL, "fe_csr_from_csr: column out of range in row %lld", (long long)i);
      if (e > row_ptr[i] && col_idx[e] <= col_idx[e - 1])
        return fail(FE_EINVAL, "fe_csr_from_csr: row %lld not strictly increasing", (long long)i);
    }
  try {
    std::vector<int64_t> rp(row_ptr, row_ptr + n + 1);
    std::vector<int32_t> ci(col_idx, col_idx + row_ptr[n]);
    fe_csr* A = new fe_csr();
    fe_status st = csr_upload(A, std::move(rp), std::move(ci), flags & FE_RELABEL_BY_DEGREE);
    if (st != FE_OK) {
      delete A;
      return st;
    }
    *out = A;
    return FE_OK;
  } catch (const std::bad_alloc&) {
    return fail(FE_ENOMEM, "fe_csr_from_csr: host allocation failed");
  }
}

fe_status fe_csr_info(const fe_csr* A, int64_t* n, int64_t* nnz, int64_t* max_deg) {
  if (!A) return fail(FE_EINVAL, "fe_csr_info: NULL handle");
  if (n) *n = A->n;
  if (nnz) *nnz = A->nnz;
  if (max_deg) *max_deg = A->max_deg;
  return FE_OK;
}

fe_status fe_csr_perm(const fe_csr* A, int32_t* perm) {
  if (!A || !perm) return fail(FE_EINVAL, "fe_csr_perm: NULL argument");
  if (A->relabeled)
    std::memcpy(perm, A->perm.data(), sizeof(int32_t) * A->n);
  else
    for (int64_t i = 0; i < A->n; ++i) perm[i] = (int32_t)i;
  return FE_OK;
}

fe_status fe_csr_export(const fe_csr* A, int64_t* row_ptr, int32_t* col_idx) {
  if (!A || !row_ptr || (A->nnz && !col_idx)) return fail(FE_EINVAL, "fe_csr_export: NULL argument");
  FE_HIP(hipMemcpy(row_ptr, A->d_row_ptr, sizeof(int64_t) * (A->n + 1), hipMemcpyDeviceToHost));
  if (A->nnz) FE_HIP(hipMemcpy(col_idx, A->d_col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToHost));
  return FE_OK;
}

void fe_csr_free(fe_csr* A) {
  if (!A) return;
  free_device(A);
  delete A;
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char *pa = (const char*)a, *pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

fe_status fe_spmm(const fe_csr* A, const void* X, void* Y, int32_t b, fe_dtype dt, void* stream) {
  if (!A || !X || !Y) return fail(FE_EINVAL, "fe_spmm: NULL argument");
  if (b < 1 || b > 64) return fail(FE_EINVAL, "fe_spmm: b=%d not in [1, 64]", b);
  if (!dtype_ok(dt)) return fail(FE_EINVAL, "fe_spmm: bad dtype");
  const size_t bytes = (size_t)A->n * b * dtype_size(dt);
  if (overlap(X, bytes, Y, bytes)) return fail(FE_EINVAL, "fe_spmm: X and Y overlap");
  if ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) % dtype_size(dt))
    return fail(FE_EINVAL, "fe_spmm: X/Y not aligned to the element size");
  return spmm_launch(*A, X, Y, b, dt, (hipStream_t)stream);
}

fe_status fe_spmm_gather_bound(const fe_csr* A, const void* X, double* out, int32_t b,
                              fe_dtype dt, void* stream) {
  if (!A || !X || !out) return fail(FE_EINVAL, "fe_spmm_gather_bound: NULL argument");
  if (b < 1 || b > 64) return fail(FE_EINVAL, "fe_spmm_gather_bound: b=%d not in [1, 64]", b);
  if (!dtype_ok(dt)) return fail(FE_EINVAL, "fe_spmm_gather_bound: bad dtype");
  if (reinterpret_cast<uintptr_t>(X) % dtype_size(dt))
    return fail(FE_EINVAL, "fe_spmm_gather_bound: X not aligned to the element size");
  return gather_bound_launch(*A, X, out, b, dt, (hipStream_t)stream);
}

int32_t fe_spmm_gather_bound_sets(void) { return gather_bound_sets(); }

fe_status fe_gather_rows(const int32_t* idx, int64_t count, const void* X, int64_t n, int32_t b,
                         fe_dtype dt, double* out, void* stream) {
  if (!X || !out || (count > 0 && !idx)) return fail(FE_EINVAL, "fe_gather_rows: NULL argument");
  if (count < 0 || n < 1) return fail(FE_EINVAL, "fe_gather_rows: bad sizes");
  if (b < 1 || b > 64) return fail(FE_EINVAL, "fe_gather_rows: b=%d not in [1, 64]", b);
  if (!dtype_ok(dt)) return fail(FE_EINVAL, "fe_gather_rows: bad dtype");
  if (reinterpret_cast<uintptr_t>(X) % dtype_size(dt))
    return fail(FE_EINVAL, "fe_gather_rows: X not aligned to the element size");
  return gather_rows_launch(idx, count, true, X, n, out, b, dt, (hipStream_t)stream);
}

static fe_status check_blocks(const char* fn, const void* V, int32_t nblk, int64_t stride,
                              int64_t n, int32_t b, fe_dtype dt) {
  if (!V) return fail(FE_EINVAL, "%s: V is NULL", fn);
  if (n < 1 || b < 1 || b > 64 || nblk < 1) return fail(FE_EINVAL, "%s: bad sizes n=%lld b=%d nblk=%d", fn, (long long)n, b, nblk);
  if (!dtype_ok(dt)) return fail(FE_EINVAL, "%s: bad dtype", fn);
  if (nblk > 1 && stride < n * b) return fail(FE_EINVAL, "%s: blk_stride < n*b", fn);
  if ((int64_t)nblk * b > 1024) return fail(FE_EINVAL, "%s: k = nblk*b > 1024", fn);
  if (reinterpret_cast<uintptr_t>(V) % dtype_size(dt)) return fail(FE_EINVAL, "%s: misaligned V", fn);
  return FE_OK;
}

fe_status fe_gram(const void* V, int32_t nblk, int64_t stride, const void* W, int64_t n, int32_t b,
                  fe_dtype dt, double alpha, double* C, void* stream) {
  FE_TRY(check_blocks("fe_gram", V, nblk, stride, n, b, dt));
  if (!W || !C) return fail(FE_EINVAL, "fe_gram: NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const size_t np = gram_partials_doubles(n, nblk * b, b);
  double* part = nullptr;
  hipError_t e = hipMallocAsync((void**)&part, np * sizeof(double), s);
  if (e != hipSuccess) return fail(FE_ENOMEM, "fe_gram: hipMallocAsync: %s", hipGetErrorString(e));
  fe_status st = gram_launch(V, nblk, stride, W, n, b, dt, alpha, C, part, s);
  hipError_t e2 = hipFreeAsync(part, s);
  if (st != FE_OK) return st;
  if (e2 != hipSuccess) return fail(FE_EDEVICE, "fe_gram: hipFreeAsync: %s", hipGetErrorString(e2));
  return FE_OK;
}

fe_status fe_block_update(void* W, int64_t n, int32_t b, const void* V, int32_t nblk, int64_t stride,
                          const double* C, double alpha, double beta, fe_dtype dt, void* stream) {
  FE_TRY(check_blocks("fe_block_update", V, nblk, stride, n, b, dt));
  if (!W || !C) return fail(FE_EINVAL, "fe_block_update: NULL argument");
  const size_t es = dtype_size(dt);
  const size_t wbytes = (size_t)n * b * es;
  const size_t vbytes = ((size_t)(nblk - 1) * stride + (size_t)n * b) * es;
  if (overlap(W, wbytes, V, vbytes)) {
    if (!(nblk == 1 && W == V && b <= 16))
      return fail(FE_EINVAL, "fe_block_update: W overlaps V (only W == V with nblk == 1, b <= 16 is allowed)");
  }
  // at b = 8 and 16 the solver's MFMA kernel (V read as min(16, 4 x element
  // size)-byte column groups, C staged in LDS for k <= 256)
  const size_t va = std::min<size_t>(16, 4 * es);
  if ((b == 8 || b == 16) && (int64_t)nblk * b <= 256 && reinterpret_cast<uintptr_t>(V) % va == 0 &&
      ((size_t)stride * es) % va == 0)
    return mult_update_launch(W, n, b, V, nblk, stride, C, alpha, beta, nullptr, dt,
                              (hipStream_t)stream);
  return update_launch(W, n, b, V, nblk, stride, C, alpha, beta, dt, (hipStream_t)stream);
}

fe_status fe_block_update_gram(void* W, int64_t n, int32_t b, const void* V, int32_t nblk,
                               int64_t stride, const double* C, double* Cout, fe_dtype dt,
                               void* stream) {
  FE_TRY(check_blocks("fe_block_update_gram", V, nblk, stride, n, b, dt));
  if (!W || !C || !Cout) return fail(FE_EINVAL, "fe_block_update_gram: NULL argument");
  const bool fused = cgs_mid_supported(b, nblk, dt);
  if (!fused && (!(b == 1 || b == 2 || b == 4 || b == 8 || b == 16) || nblk * b > 64))
    return fail(FE_EUNSUPPORTED,
                "fe_block_update_gram: needs b in {1,2,4,8,16} and k <= 64 (k + b <= 128 at b = 4, 16)");
  const size_t es = dtype_size(dt);
  const size_t vbytes = ((size_t)(nblk - 1) * stride + (size_t)n * b) * es;
  if (overlap(W, (size_t)n * b * es, V, vbytes))
    return fail(FE_EINVAL, "fe_block_update_gram: W overlaps V");
  const size_t va = std::min<size_t>(16, 4 * es);  // the fused kernels' vector loads
  if (fused && (reinterpret_cast<uintptr_t>(W) % va || reinterpret_cast<uintptr_t>(V) % va ||
                ((size_t)stride * es) % va))
    return fail(FE_EINVAL, "fe_block_update_gram: W and the blocks must be %zu-byte aligned", va);
  hipStream_t s = (hipStream_t)stream;
  const size_t np = gram_partials_doubles(n, nblk * b + b, b);
  double* part = nullptr;
  hipError_t e = hipMallocAsync((void**)&part, np * sizeof(double), s);
  if (e != hipSuccess)
    return fail(FE_ENOMEM, "fe_block_update_gram: hipMallocAsync: %s", hipGetErrorString(e));
  fe_status st = fused ? cgs_mid_launch(W, n, b, V, nblk, stride, C, Cout, part, dt, s)
                       : update_gram_launch(W, n, b, V, nblk, stride, C, Cout, part, dt, s);
  hipError_t e2 = hipFreeAsync(part, s);
  if (st != FE_OK) return st;
  if (e2 != hipSuccess)
    return fail(FE_EDEVICE, "fe_block_update_gram: hipFreeAsync: %s", hipGetErrorString(e2));
  return FE_OK;
}

}  // extern "C"
