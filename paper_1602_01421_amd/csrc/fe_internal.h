// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fe.h"

namespace fe {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
fe_status fail(fe_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define FE_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::fe::fail(FE_EDEVICE, "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                          \
  } while (0)

#define FE_TRY(expr)               \
  do {                             \
    fe_status s_ = (expr);         \
    if (s_ != FE_OK) return s_;    \
  } while (0)

inline size_t dtype_size(fe_dtype dt) { return dt == FE_F64 ? 8 : dt == FE_F32 ? 4 : 2; }
inline bool dtype_ok(fe_dtype dt) { return dt == FE_F64 || dt == FE_F32 || dt == FE_BF16; }

// ------------------------------------------------------------- sparse side
// Rows with more nonzeros than kSplitThreshold are cut into chunks of
// kSplitChunk nonzeros, one workgroup each; a second launch adds the chunk
// partials of each row in chunk order (deterministic).
constexpr int64_t kSplitThreshold = 16384;
constexpr int64_t kSplitChunk = 8192;
constexpr int64_t kBlockThreshold = 2048;  // rows above this get a whole workgroup

struct SplitChunk {
  int64_t e0, e1;    // nonzero range of this chunk
  int32_t pos;       // position of the row in degree order
  int32_t first;     // index of the row's first chunk
  int32_t count;     // chunks of this row
  int32_t pad;
};

struct Csr {
  int device = 0;
  int64_t n = 0, nnz = 0, max_deg = 0;
  bool relabeled = false;
  int64_t* d_row_ptr = nullptr;  // n+1
  int32_t* d_col = nullptr;      // nnz
  int32_t* d_order = nullptr;    // rows by descending degree; null when relabeled (identity)
  int32_t* d_perm = nullptr;     // new -> old (relabeled only)
  std::vector<int32_t> perm;     // host copy of d_perm (empty = identity)
  // cnt_gt[i] = number of rows with degree > thr(i), thr(0) = 0, thr(i) = 2^(i-1)
  int64_t cnt_gt[34] = {0};
  // split rows
  int64_t n_split_rows = 0, n_chunks = 0;
  SplitChunk* d_chunks = nullptr;
  int64_t* d_first_chunk = nullptr;  // n_split_rows: index of each hub row's first chunk
  void* d_partials = nullptr;        // n_chunks * 64 doubles
};

// number of rows with degree > t for t = 0 or a power of two
int64_t rows_deg_gt(const Csr& A, int64_t t);

fe_status csr_upload(Csr* A, std::vector<int64_t>&& row_ptr, std::vector<int32_t>&& col,
                     bool relabel);

fe_status spmm_launch(const Csr& A, const void* X, void* Y, int32_t b, fe_dtype dt,
                      hipStream_t s);
// The product's gathers without its rows (a measurement of its memory
// ceiling on this matrix): out gets gather_bound_sets() FP64 workgroup sums.
int32_t gather_bound_sets();
fe_status gather_bound_launch(const Csr& A, const void* X, double* out, int32_t b, fe_dtype dt,
                              hipStream_t s);
// The same gathers over a caller's index stream (clamp: indices clamped to [0, n)).
fe_status gather_rows_launch(const int32_t* idx, int64_t count, bool clamp, const void* X,
                             int64_t n, double* out, int32_t b, fe_dtype dt, hipStream_t s);

// ------------------------------------------------------------- dense side
// partial buffer size (doubles) needed by gram_launch, update_gram_launch and
// cgs_mid_launch for (n, k, b); gram_sets_partials_doubles: gram_launch alone
size_t gram_partials_doubles(int64_t n, int32_t k, int32_t b);
size_t gram_sets_partials_doubles(int64_t n, int32_t k, int32_t b);
fe_status gram_launch(const void* V, int32_t nblk, int64_t blk_stride, const void* W, int64_t n,
                      int32_t b, fe_dtype dt, double alpha, double* C, double* partials,
                      hipStream_t s);
// Block QR factors of one orthogonalisation step on the device (b <= 16):
// first pass from the two Grams C1, C2 ((k+b) x b): rec = C1 + C2 (k x b),
// R1 = chol(W2^T W2), M = R1^-1, flag = 1 on a dependent column; second pass
// from G = W^T W: M = chol(G)^-1, recR = chol(G) R1, flag += 2 on failure.
fe_status chol_first_launch(const double* C1, const double* C2, int32_t k, int32_t b, double eta,
                            double* rec, double* R1, double* M, double* flag, hipStream_t s);
fe_status chol_second_launch(const double* G, int32_t b, const double* R1, double* M,
                             double* recR, double* flag, hipStream_t s);
// Z ((k+b) x b) = [-C2 M; M] (C2: first k rows of the second Gram, M: b x b):
// W <- [V W] Z is the second Gram-Schmidt update followed by W M in one pass.
fe_status cgs_coef_launch(const double* C2, const double* M, int32_t k, int32_t b, double* Z,
                          hipStream_t s);
// W <- W - V C (C: k x b FP64, k = nblk*b <= 64, b in {1,2,4,8,16}) and, in
// the same pass, Cout ((k+b) x b) = [V W']^T W' of the rounded result;
// partials sized by gram_partials_doubles(n, k + b, b).
fe_status update_gram_launch(void* W, int64_t n, int32_t b, const void* V, int32_t nblk,
                             int64_t blk_stride, const double* C, double* Cout, double* partials,
                             fe_dtype dt, hipStream_t s);
// CGS2's middle step in one pass over V, at b = 4, 8 or 16: W <- W - V[:, :b nblk_v] C1,
// then Cout ((b nblk_v + b) x b) = [V W']^T W' with the rounded W' (W its own
// n x b block, not overlapping V).  Up to 128 columns of [V W], fewer at b = 8 in
// FP64 (cgs_mid_supported); partials as for gram_launch.
bool cgs_mid_supported(int32_t b, int32_t nblk_v, fe_dtype dt);
// The last pass of an orthogonalisation step at b = 8 or 16, in place:
// W <- [V W] Z (nblocks = blocks of [V W], W the last, up to 128 columns;
// Z (b nblocks) x b FP64) and G = W^T W (b x b) of the rounded result;
// partials as for gram_launch.
bool cgs_last_supported(int32_t b, int32_t nblocks);
fe_status cgs_last_launch(void* V, int32_t b, int32_t nblocks, int64_t blk_stride, int64_t n,
                          const double* Z, double* G, double* partials, fe_dtype dt,
                          hipStream_t s);
fe_status cgs_mid_launch(void* W, int64_t n, int32_t b, const void* V, int32_t nblk_v,
                         int64_t blk_stride, const double* C1, double* Cout, double* partials,
                         fe_dtype dt, hipStream_t s);
fe_status update_launch(void* W, int64_t n, int32_t b, const void* V, int32_t nblk,
                        int64_t blk_stride, const double* C, double alpha, double beta,
                        fe_dtype dt, hipStream_t s);
// The contractions below (m <= 256 input columns, p <= 128 outputs) keep Y in
// LDS up to 64 outputs and m16 x p16 <= 64 KB; beyond that they need `ypad`,
// a device buffer of rotate_pad_doubles(m, p) doubles (else FE_EUNSUPPORTED).
size_t rotate_pad_doubles(int32_t m, int32_t p);
// V[:, 0:p] <- V[:, 0:m] * Y[:, 0:p] in place (Y: device FP64, m x p row-major)
fe_status rotate_launch(void* V, int64_t n, int32_t b, int32_t nblk_in, int32_t nblk_out,
                        int64_t blk_stride, const double* Y, double* ypad, fe_dtype dt,
                        hipStream_t s);
// W <- beta W + alpha V[:, 0:k] C on the MFMA contraction of the restart
// (C: device FP64, k x b row-major; W (n x b) may be V's own single block).
// Same result as update_launch up to the order of the FP64 sums.
fe_status mult_update_launch(void* W, int64_t n, int32_t b, const void* V, int32_t nblk,
                             int64_t blk_stride, const double* C, double alpha, double beta,
                             double* ypad, fe_dtype dt, hipStream_t s);
// Out (n x c packed, FP64) <- V[:, 0:m] * Y (m x c), V as blocks in dt.
fe_status combine_launch(double* Out, int32_t c, int64_t n, int32_t b, const void* V, int32_t nblk,
                         int64_t blk_stride, const double* Y, double* ypad, fe_dtype dt,
                         hipStream_t s);
// FP64 X, AX (n x c): sums[3i] = x_i.ax_i, sums[3i+1] = x_i.x_i,
// sums[3i+2] = ||ax_i - theta_i x_i||^2
size_t resid_partials_doubles(int64_t n, int32_t c);
fe_status resid_launch(const double* AX, const double* X, int64_t n, int32_t c,
                       const double* theta, double* sums, double* partials, hipStream_t s);
// dst (n x c in dt) <- src (FP64), row r stored at perm[r] when perm is given
fe_status store_rows(void* dst, const double* src, const int32_t* perm, int64_t n, int32_t c,
                     fe_dtype dt, hipStream_t s);
// copy an n x b block (same dtype)
fe_status copy_block(void* dst, const void* src, int64_t n, int32_t b, fe_dtype dt,
                     hipStream_t s);
// dst[new] = src[perm[new]] (gather) or dst[perm[new]] = src[new] (scatter), rows of width c
fe_status permute_rows(void* dst, const void* src, const int32_t* perm, int64_t n, int32_t c,
                       fe_dtype dt, bool scatter, hipStream_t s);
// fill columns with Philox draws: mode 0 = N(0,1) (start block), 1 = uniform [-1,1) refill
// Row r draws with counter row id perm[r] (original vertex id; perm null = identity).
fe_status random_fill(void* W, int64_t n, int32_t b, uint32_t col_mask, int32_t mode,
                      uint64_t seed, uint32_t step, const int32_t* perm, fe_dtype dt,
                      hipStream_t s);

// dst (count elements of ddt) <- src (sdt), rounded to nearest even
fe_status convert_launch(void* dst, fe_dtype ddt, const void* src, fe_dtype sdt, int64_t count,
                         hipStream_t s);

bool sym_eig(int n, double* a, double* w, double* z);

}  // namespace fe

struct fe_csr : fe::Csr {};
