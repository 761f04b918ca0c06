// Block Krylov-Schur driver (host control loop, device subspace).
//
// The paper's eigensolver is Anasazi's block Krylov-Schur, following its
// generic eigen-iteration: (1) update the subspace (sparse product plus
// reorthogonalisation), (2) solve the projected m x m problem, (3) Ritz
// pairs and residuals, (4) convergence test; with the block extension b
// vectors enter per step and the subspace holds m = b * NB vectors.  This is
// Stewart's Krylov-Schur for symmetric A (block thick-restart Lanczos with
// full reorthogonalisation):
//
//   state   A V = V T + Q B,  V n x k orthonormal, Q n x b orthonormal, Q _|_ V
//   expand  V <- [V Q]; W = A Q; C = CGS2(V, W); W = Q' R; T gets C; B = [0 R]
//   check   S = sym(T) = Y diag(theta) Y^T, |theta| descending; rho_i = ||B y_i||
//   restart V[:, :p] <- V Y[:, :p], T <- diag(theta_1..p), B <- B Y[:, :p]
//
// Device memory holds the whole subspace: m/b + 1 packed n x b blocks.  The
// block after the last basis block holds W, which becomes the next Q in
// place, so a Gram product over k/b + 1 blocks returns both V^T W and W^T W.
// Only small FP64 matrices (<= (m+b) x b, m x m) cross to the host.
//
// Readings where the paper is silent: dependence threshold eta (a column is
// dependent when its norm after projection against V and the earlier
// accepted columns is <= eta times its norm before projection; 1e-10 for
// FP64 storage, decided with directly computed norms), and a Cholesky QR
// guard eta_chol = 1e-6 below which the column-wise factors replace Cholesky
// QR twice (see set_eta); dependent columns are refilled with Philox uniform
// [-1, 1) draws orthogonalised against everything accepted; kept Ritz vectors p = m - b*max(1,
// floor((m-nev)/(2b))); convergence rho_i <= tol * max(eps^(2/3), |theta_i|)
// with eps the FP64 unit roundoff (ARPACK's convention).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "fe_internal.h"

namespace fe {
namespace {

using clk = std::chrono::steady_clock;
// Denominator of the convergence test: max(eps^(2/3), |theta|), eps = 2^-52.
static double ritz_scale(double theta) {
  return std::max(std::fabs(theta), std::cbrt(2.220446049250313e-16 * 2.220446049250313e-16));
}

// Ritz vectors kept at a restart: the caller's count, or the default
// m - b max(1, floor((m - nev) / (2 b))) (a reading; m - p stays a multiple of b).
static int restart_size(int m, int b, int nev, int keep) {
  return keep > 0 ? keep : m - b * std::max(1, (m - nev) / (2 * b));
}

static double secs(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

enum ProfCls { P_SPMM = 0, P_GRAM = 1, P_UPDATE = 2, P_OTHER = 3 };

struct Prof {
  bool on = false;
  hipStream_t s = nullptr;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  double t[4] = {0, 0, 0, 0};
  int open_cls = -1;
  hipEvent_t open_a = nullptr;
  // st: the stream the timed work runs on (default: the solve's stream)
  void begin(int cls, hipStream_t st = nullptr) {
    if (!on) return;
    hipEventCreate(&open_a);
    hipEventRecord(open_a, st ? st : s);
    open_cls = cls;
  }
  void end(hipStream_t st = nullptr) {
    if (!on || open_cls < 0) return;
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, st ? st : s);
    recs.push_back({open_cls, open_a, e});
    open_cls = -1;
  }
  void flush() {  // stream must be synchronised
    for (auto& r : recs) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, r.a, r.b);
      t[r.cls] += ms * 1e-3;
      hipEventDestroy(r.a);
      hipEventDestroy(r.b);
    }
    recs.clear();
  }
  ~Prof() { flush(); }
};

// Every device buffer of a solve, in 256-byte units: from hipMalloc (freed
// when the solve returns), or carved in order from a caller's workspace.
static size_t ws_round(size_t bytes) { return (std::max<size_t>(bytes, 256) + 255) / 256 * 256; }

struct DevBuf {
  std::vector<void*> ptrs;
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  int allocs = 0;  // hipMalloc calls made
  ~DevBuf() {
    for (void* p : ptrs) hipFree(p);
  }
  void release(void* p) {
    if (arena) return;
    for (auto& q : ptrs)
      if (q == p) {
        (void)hipFree(q);
        q = nullptr;
      }
  }
  fe_status get(void** p, size_t bytes) {
    const size_t sz = ws_round(bytes);
    if (arena) {
      if (arena_used + sz > arena_bytes)
        return fail(FE_ENOMEM, "fe_krylov_schur: workspace of %zu bytes is too small",
                    arena_bytes);
      *p = arena + arena_used;
      arena_used += sz;
      return FE_OK;
    }
    hipError_t e = hipMalloc(p, sz);
    if (e != hipSuccess)
      return fail(FE_ENOMEM, "fe_krylov_schur: hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    ++allocs;
    ptrs.push_back(*p);
    return FE_OK;
  }
};

// The sum of every DevBuf::get of a solve (the order does not matter to the
// bump allocation): setup(), the mixed start block and switch, the final check.
static size_t ks_workspace_plan(int64_t n, int nev, int b, int m, fe_dtype dt, bool mixed,
                                bool start) {
  const fe_dtype dt0 = mixed ? FE_BF16 : dt;
  const size_t es0 = dtype_size(dt0), esf = dtype_size(dt);
  const size_t nblk = (size_t)(m / b + 1), kmax = (size_t)(m + b), stride = (size_t)n * b;
  const size_t d = sizeof(double);
  size_t t = ws_round(nblk * stride * es0);
  t += ws_round(d * 2 * kmax * b) + ws_round(d * b * b) + ws_round(d * kmax * b) +
       ws_round(d * m * m);
  t += ws_round(d * rotate_pad_doubles(m + b, std::max(m, 64)));
  t += ws_round(d * 64) + ws_round(d * 3 * 64);
  t += ws_round(d * gram_partials_doubles(n, (int32_t)kmax, b));
  t += ws_round(d * resid_partials_doubles(n, 64));
  t += ws_round(d * ((size_t)m * b + (size_t)b * b + 1) * nblk);
  t += ws_round(d * b * b);
  if (mixed && start) t += ws_round(stride * esf);
  if (mixed) t += ws_round(nblk * stride * esf) + ws_round(d * stride);
  t += 2 * ws_round(d * (size_t)n * nev);
  t += ws_round(stride * std::max(es0, esf));  // the restart overlap's spare block
  return t;
}

struct HostBuf {
  std::vector<void*> ptrs;
  ~HostBuf() {
    for (void* p : ptrs) hipHostFree(p);
  }
  fe_status get(double** p, size_t count) {
    hipError_t e = hipHostMalloc((void**)p, std::max<size_t>(count, 32) * sizeof(double));
    if (e != hipSuccess) return fail(FE_ENOMEM, "fe_krylov_schur: hipHostMalloc failed");
    ptrs.push_back(*p);
    return FE_OK;
  }
};

// upper-triangular inverse of the na x na matrix R (row-major, ld = ld)
static void inv_upper(int na, const double* R, int ld, double* Ri, int ldi) {
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < na; ++j) Ri[i * ldi + j] = 0.0;
  for (int j = 0; j < na; ++j) {
    Ri[j * ldi + j] = 1.0 / R[j * ld + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int t = i + 1; t <= j; ++t) s += R[i * ld + t] * Ri[t * ldi + j];
      Ri[i * ldi + j] = -s / R[i * ld + i];
    }
  }
}

class Solver {
 public:
  const Csr& A;
  const Csr* At = nullptr;  // set for the singular value problem: the operator is A^T A
  void* Tb = nullptr;       // n x b block between the two products (A^T A)
  // Restart overlap: the next expansion's first product (from Q, which the
  // rotation neither reads nor writes) runs on a second stream into `spare`
  // while the restart rotation runs on the solve's stream.
  hipStream_t s2 = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  void* spare = nullptr;
  bool pre_product = false;
  double* T64 = nullptr;    // n x nev FP64, the final check's A X (A^T A)
  int nev, b, m;
  double tol, eta, eta_chol;
  fe_ks_opts o;
  hipStream_t s;
  fe_dtype dt, dt_final;
  size_t es;
  bool mixed = false;
  double mixed_switch = 1e-3;
  int switch_restart = -1, spmm_low = 0;
  int64_t n, stride;
  char* V = nullptr;  // m/b + 1 blocks
  double *dC = nullptr, *dM = nullptr, *dZ = nullptr, *dY = nullptr, *dYpad = nullptr, *dTheta = nullptr,
         *dSums = nullptr;
  double *dPart = nullptr, *dPartRes = nullptr;
  double *hC1 = nullptr, *hC2 = nullptr, *hG = nullptr, *hM = nullptr, *hY = nullptr,
         *hSums = nullptr, *hTheta = nullptr;
  // Per-step records of the device-side orthogonalisation (one slot per
  // block): C (k x b, stride m*b), R (b x b), status flag.
  double *dRec = nullptr, *hRec = nullptr, *dR1 = nullptr;
  size_t rec_stride = 0;
  DevBuf dev;
  HostBuf host;
  Prof prof;
  std::vector<double> T, Bk;
  int step = 0, refills = 0, spmm_calls = 0, spmm_cols = 0, gram_calls = 0, update_calls = 0;
  double t_host = 0.0;
  double bytes[4] = {0, 0, 0, 0};  // algorithmic HBM bytes per kernel class
  std::vector<double> worst_hist;

  Solver(const Csr& A_, int nev_, int b_, int m_, double tol_, const fe_ks_opts& o_)
      : A(A_), nev(nev_), b(b_), m(m_), tol(tol_), o(o_) {
    s = (hipStream_t)o.hip_stream;
    dt_final = o.dt;
    mixed = o.mixed != 0 && o.dt != FE_BF16;
    if (o.mixed_switch > 0) mixed_switch = o.mixed_switch;
    dt = mixed ? FE_BF16 : o.dt;
    es = dtype_size(dt);
    n = A.n;
    stride = n * b;
    set_eta();
    prof.on = o.profile != 0;
    prof.s = s;
    if (o.workspace) {
      dev.arena = static_cast<char*>(o.workspace);
      dev.arena_bytes = o.workspace_bytes;
    }
  }
  ~Solver() {
    if (s2) {
      (void)hipStreamSynchronize(s2);  // before the buffers it may still use are freed
      (void)hipStreamDestroy(s2);
    }
    if (ev_a) (void)hipEventDestroy(ev_a);
    if (ev_b) (void)hipEventDestroy(ev_b);
  }

  // eta: refill threshold on the column-wise ratio (reading: 1e-10 for FP64
  // storage, 1e-5 FP32, 3e-2 BF16, near each storage's rounding level);
  // eta_chol: below this ratio Cholesky QR twice is not trusted (its first
  // pass loses orthogonality like u kappa^2), and the device path hands the
  // step to the column-wise path.  The device screen reads the ratio from a
  // Schur complement of the Gram matrix, which resolves it down to about
  // sqrt(u) = 1.5e-8, so eta_chol >= 1e-6.
  void set_eta() {
    eta = o.eta > 0 ? o.eta : (dt == FE_F64 ? 1e-10 : dt == FE_F32 ? 1e-5 : 3e-2);
    eta_chol = std::max(eta, 1e-6);
  }

  void* blk(int j) { return V + (size_t)j * stride * es; }

  // Mixed precision switch.  Widening the BF16 basis in place would keep the
  // Krylov relation A V = V T + Q B only to BF16 accuracy, and thick restarts
  // never purge that error (the implicit residuals keep falling while the
  // explicit ones stay near 2^-8).  Instead the solve restarts explicitly in
  // dt_final from one block that sums the wanted Ritz vectors: column j holds
  // sum_{i = j mod b, i < q} V y_i with q = nev rounded up to a multiple of b,
  // so q/b block steps already span every wanted Ritz direction again.
  fe_status widen_restart(const std::vector<double>& Y) {
    const int nblk = m / b + 1;
    const int q = std::min(m, (nev + b - 1) / b * b);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < b; ++j) {
        double sum = 0.0;
        for (int t = j; t < q; t += b) sum += Y[(size_t)i * m + t];
        hY[(size_t)i * b + j] = sum;
      }
    FE_HIP(hipMemcpyAsync(dY, hY, sizeof(double) * m * b, hipMemcpyHostToDevice, s));
    const size_t es2 = dtype_size(dt_final);
    char* V2 = nullptr;
    double* tmp = nullptr;
    FE_TRY(dev.get((void**)&V2, (size_t)nblk * stride * es2));
    FE_TRY(dev.get((void**)&tmp, (size_t)n * b * sizeof(double)));
    prof.begin(P_OTHER);
    FE_TRY(combine_launch(tmp, b, n, b, V, m / b, stride, dY, dYpad, dt, s));
    FE_TRY(convert_launch(V2, dt_final, tmp, FE_F64, (int64_t)n * b, s));
    prof.end();
    FE_TRY(sync());
    dev.release(tmp);
    dev.release(V);
    V = V2;
    dt = dt_final;
    es = es2;
    set_eta();
    return FE_OK;
  }

  fe_status setup() {
    const int nblk = m / b + 1;
    FE_TRY(dev.get((void**)&V, (size_t)nblk * stride * es));
    const int kmax = m + b;
    FE_TRY(dev.get((void**)&dC, sizeof(double) * 2 * kmax * b));
    FE_TRY(dev.get((void**)&dM, sizeof(double) * b * b));
    FE_TRY(dev.get((void**)&dZ, sizeof(double) * (m + b) * b));
    FE_TRY(dev.get((void**)&dY, sizeof(double) * m * m));
    FE_TRY(dev.get((void**)&dYpad, sizeof(double) * rotate_pad_doubles(m + b, std::max(m, 64))));
    FE_TRY(dev.get((void**)&dTheta, sizeof(double) * 64));
    FE_TRY(dev.get((void**)&dSums, sizeof(double) * 3 * 64));
    FE_TRY(dev.get((void**)&dPart, sizeof(double) * gram_partials_doubles(n, kmax, b)));
    FE_TRY(dev.get((void**)&dPartRes, sizeof(double) * resid_partials_doubles(n, 64)));
    FE_TRY(host.get(&hC1, kmax * b));
    FE_TRY(host.get(&hC2, kmax * b));
    FE_TRY(host.get(&hG, kmax * b));
    FE_TRY(host.get(&hM, b * b));
    FE_TRY(host.get(&hY, m * m));
    FE_TRY(host.get(&hSums, 3 * 64));
    FE_TRY(host.get(&hTheta, 64));
    rec_stride = (size_t)m * b + (size_t)b * b + 1;
    FE_TRY(dev.get((void**)&dRec, sizeof(double) * rec_stride * (m / b + 1)));
    FE_TRY(host.get(&hRec, rec_stride * (m / b + 1)));
    FE_TRY(dev.get((void**)&dR1, sizeof(double) * b * b));
    if (At) FE_TRY(dev.get(&Tb, (size_t)n * b * std::max(es, dtype_size(dt_final))));
    FE_TRY(dev.get(&spare, (size_t)n * b * std::max(es, dtype_size(dt_final))));
    FE_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    FE_HIP(hipEventCreateWithFlags(&ev_a, hipEventDisableTiming));
    FE_HIP(hipEventCreateWithFlags(&ev_b, hipEventDisableTiming));
    T.assign((size_t)m * m, 0.0);
    Bk.assign((size_t)b * m, 0.0);
    return FE_OK;
  }

  fe_status sync() {
    FE_HIP(hipStreamSynchronize(s));
    prof.flush();
    return FE_OK;
  }

  fe_status gram(int nblk, const void* W, double* C) {
    prof.begin(P_GRAM);
    fe_status st = gram_launch(V, nblk, stride, W, n, b, dt, 1.0, C, dPart, s);
    prof.end();
    ++gram_calls;
    bytes[P_GRAM] += (double)n * nblk * b * es;  // W is the last of the nblk blocks
    return st;
  }
  // Wide blocks (b >= 8) go to the MFMA contraction: the one-thread-per-row
  // kernel's 2 k b FP64 FMAs per row make it VALU bound there.
  fe_status update(void* W, const void* Vp, int nblk, const double* C, double alpha, double beta) {
    prof.begin(P_UPDATE);
    fe_status st = b >= 8 ? mult_update_launch(W, n, b, Vp, nblk, stride, C, alpha, beta, dYpad, dt, s)
                          : update_launch(W, n, b, Vp, nblk, stride, C, alpha, beta, dt, s);
    prof.end();
    ++update_calls;
    const bool in_place = (W == Vp);
    bytes[P_UPDATE] += (double)n * b * es * ((in_place ? 0 : nblk) + (beta != 0.0 || in_place) + 1);
    return st;
  }
  fe_status spmm(const void* X, void* Y, int cols) { return spmm_on(X, Y, cols, s); }
  fe_status spmm_on(const void* X, void* Y, int cols, hipStream_t st_) {
    prof.begin(P_SPMM, st_);
    fe_status st = At ? spmm_launch(A, X, Tb, cols, dt, st_) : spmm_launch(A, X, Y, cols, dt, st_);
    if (st == FE_OK && At) st = spmm_launch(*At, Tb, Y, cols, dt, st_);
    prof.end(st_);
    spmm_cols += cols;
    bytes[P_SPMM] += (At ? 2.0 : 1.0) * (4.0 * A.nnz + 8.0 * (n + 1) + 2.0 * n * cols * es);
    return st;
  }
  // hM is pinned host memory reused by the next factor: the copy must have
  // read it before the host writes it again, so the upload waits for it.
  fe_status upload_M() {
    FE_HIP(hipMemcpyAsync(dM, hM, sizeof(double) * b * b, hipMemcpyHostToDevice, s));
    FE_HIP(hipStreamSynchronize(s));
    return FE_OK;
  }
  // W <- W * hM (in place)
  fe_status right_mult(void* W) {
    FE_TRY(upload_M());
    return update(W, W, 1, dM, 1.0, 0.0);
  }
  // G = W^T W of block wb into hG (synchronises)
  fe_status self_gram(int wb) {
    prof.begin(P_GRAM);
    FE_TRY(gram_launch(blk(wb), 1, stride, blk(wb), n, b, dt, 1.0, dC, dPart, s));
    prof.end();
    ++gram_calls;
    bytes[P_GRAM] += (double)n * b * es;
    FE_HIP(hipMemcpyAsync(hG, dC, sizeof(double) * b * b, hipMemcpyDeviceToHost, s));
    return sync();
  }

  // orth_block without host round trips, for the common case: the same
  // kernels, with the rank-revealing Cholesky, the triangular inverses and the
  // second Cholesky QR pass done by small device kernels (bitwise the host's
  // arithmetic).  C, R and a status flag go to the step's record; a nonzero
  // flag (dependent column, failed factorisation) makes the caller redo the
  // step with orth_block, which handles refills.
  fe_status orth_fast(int wb, double* rec) {
    const int nk = wb;
    const int k = nk * b;
    void* W = blk(wb);
    double* dC1 = dC;
    double* dC2 = dC + (size_t)(k + b) * b;
    double* flag = rec + (size_t)m * b + (size_t)b * b;
    FE_TRY(gram(nk + 1, W, dC1));
    if (cgs_mid_supported(b, nk, dt)) {
      // first update and second Gram in one pass over [V W]
      prof.begin(P_GRAM);
      FE_TRY(cgs_mid_launch(W, n, b, V, nk, stride, dC1, dC2, dPart, dt, s));
      prof.end();
      ++gram_calls;
      ++update_calls;
      bytes[P_GRAM] += (double)n * (nk + 2) * b * es;  // [V W] read, W' written
    } else {
      FE_TRY(update(W, V, nk, dC1, -1.0, 1.0));
      FE_TRY(gram(nk + 1, W, dC2));
    }
    FE_TRY(chol_first_launch(dC1, dC2, k, b, eta_chol, rec, dR1, dM, flag, s));
    if (cgs_last_supported(b, nk + 1)) {
      // W <- (W - V C2) R1^-1 as one in-place right-multiplication of [V W]
      // (W is the block after V), with W^T W of the result in the same pass
      FE_TRY(cgs_coef_launch(dC2, dM, k, b, dZ, s));
      prof.begin(P_UPDATE);
      FE_TRY(cgs_last_launch(V, b, nk + 1, stride, n, dZ, dC, dPart, dt, s));
      prof.end();
      ++update_calls;
      ++gram_calls;
      bytes[P_UPDATE] += (double)n * b * es * (nk + 2);  // [V W] read, W written
      FE_TRY(chol_second_launch(dC, b, dR1, dM, rec + (size_t)m * b, flag, s));
      return update(W, W, 1, dM, 1.0, 0.0);
    }
    if (b >= 8) {
      // W <- (W - V C2) R1^-1 as one in-place right-multiplication of [V W]
      // (W is the block after V; each output row is written after its reads)
      FE_TRY(cgs_coef_launch(dC2, dM, k, b, dZ, s));
      FE_TRY(update(W, V, nk + 1, dZ, 1.0, 0.0));
    } else {
      FE_TRY(update(W, V, nk, dC2, -1.0, 1.0));
      FE_TRY(update(W, W, 1, dM, 1.0, 0.0));
    }
    prof.begin(P_GRAM);
    FE_TRY(gram_launch(W, 1, stride, W, n, b, dt, 1.0, dC, dPart, s));
    prof.end();
    ++gram_calls;
    bytes[P_GRAM] += (double)n * b * es;
    FE_TRY(chol_second_launch(dC, b, dR1, dM, rec + (size_t)m * b, flag, s));
    return update(W, W, 1, dM, 1.0, 0.0);
  }

  // T gets C as the new columns k-b..k-1 (and their mirror), Bk the new R.
  void absorb(int k, const double* C, const double* R) {
    auto th = clk::now();
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < b; ++j) {
        T[(size_t)i * m + (k - b + j)] = C[(size_t)i * b + j];
        T[(size_t)(k - b + j) * m + i] = C[(size_t)i * b + j];
      }
    std::fill(Bk.begin(), Bk.end(), 0.0);
    for (int i = 0; i < b; ++i)
      for (int j = 0; j < b; ++j) Bk[(size_t)i * m + (k - b + j)] = R[(size_t)i * b + j];
    t_host += secs(th, clk::now());
  }

  // W <- W * M with M the identity except the entries set by the caller
  // (hM is reset to the identity by reset_M).
  void reset_M() {
    std::fill(hM, hM + b * b, 0.0);
    for (int i = 0; i < b; ++i) hM[i * b + i] = 1.0;
  }

  // Column j of block wb against the accepted (orthonormal) columns `acc`,
  // twice (classical Gram-Schmidt twice); the coefficients are added to
  // R[acc, j].  Returns the norm of the projected column, taken directly
  // from the block's own Gram matrix (no cancellation against earlier norms).
  fe_status project_column(int wb, int j, const std::vector<int>& acc, std::vector<double>& R,
                           double* norm) {
    void* W = blk(wb);
    for (int pass = 0; pass < 2 && !acc.empty(); ++pass) {
      FE_TRY(self_gram(wb));
      reset_M();
      for (int i : acc) {
        const double c = hG[i * b + j];
        hM[i * b + j] = -c;
        R[(size_t)i * b + j] += c;
      }
      FE_TRY(right_mult(W));
    }
    FE_TRY(self_gram(wb));
    *norm = std::sqrt(std::max(0.0, hG[j * b + j]));
    return FE_OK;
  }

  fe_status scale_column(int wb, int j, double f) {
    reset_M();
    hM[j * b + j] = f;
    return right_mult(blk(wb));
  }

  // Cholesky QR twice of block wb in place: R (b x b) with W_in = Q R.
  // Returns false (W untouched) when a factorisation fails.
  fe_status cholqr2(int wb, std::vector<double>& R, bool* ok) {
    std::vector<double> Rt((size_t)b * b, 0.0), Racc((size_t)b * b, 0.0), Ri((size_t)b * b);
    for (int i = 0; i < b; ++i) Racc[i * b + i] = 1.0;
    *ok = false;
    for (int pass = 0; pass < 2; ++pass) {
      FE_TRY(self_gram(wb));
      std::fill(Rt.begin(), Rt.end(), 0.0);
      for (int j = 0; j < b; ++j) {
        double d = hG[j * b + j];
        for (int i = 0; i < j; ++i) d -= Rt[i * b + j] * Rt[i * b + j];
        if (!(d > 0.0)) {
          if (pass == 1) return fail(FE_EBREAKDOWN, "fe_krylov_schur: block QR lost rank (step %d)", step);
          return FE_OK;
        }
        Rt[j * b + j] = std::sqrt(d);
        for (int l = j + 1; l < b; ++l) {
          double g = hG[j * b + l];
          for (int i = 0; i < j; ++i) g -= Rt[i * b + j] * Rt[i * b + l];
          Rt[j * b + l] = g / Rt[j * b + j];
        }
      }
      inv_upper(b, Rt.data(), b, Ri.data(), b);
      std::copy(Ri.begin(), Ri.end(), hM);
      FE_TRY(right_mult(blk(wb)));
      std::vector<double> tmp((size_t)b * b, 0.0);  // Racc <- Rt Racc
      for (int i = 0; i < b; ++i)
        for (int j = 0; j < b; ++j) {
          double sum = 0.0;
          for (int t = 0; t < b; ++t) sum += Rt[i * b + t] * Racc[t * b + j];
          tmp[i * b + j] = sum;
        }
      Racc.swap(tmp);
    }
    R = Racc;
    *ok = true;
    return FE_OK;
  }

  // Orthogonalise W (block wb) against V[:, :k] (blocks 0..k/b-1, k = wb*b) and
  // orthonormalise it.  Out: C (k x b) and R (b x b) with W_in = V C + Q R.
  // The careful path, taken for the start block and for every step the
  // device-side factors flagged: CGS2 against V, then column-wise CGS2 inside
  // the block in column order with each column's norm read directly from the
  // block's Gram matrix, so that the dependence ratio (norm after projection
  // over norm before) is resolved down to the storage's rounding, not to the
  // square root of it as a Schur complement of the Gram matrix would be.
  // Column j is dependent when that ratio is not above eta (or the column is
  // not finite): its row of R is zero and it is refilled with Philox draws
  // orthogonalised against V and every column kept so far.  With no
  // dependent column and every ratio at least eta_chol the block is
  // refactored by Cholesky QR twice (the device path's factorisation);
  // otherwise the column-wise factors stand.
  fe_status orth_block(int wb, std::vector<double>& C, std::vector<double>& R) {
    const int nk = wb;  // basis blocks
    const int k = nk * b;
    void* W = blk(wb);
    double* dC1 = dC;
    double* dC2 = dC + (size_t)(k + b) * b;
    // CGS2 against V: pass 1 gives [V W]^T W (W's own norms in its last rows)
    FE_TRY(gram(nk + 1, W, dC1));
    FE_HIP(hipMemcpyAsync(hC1, dC1, sizeof(double) * (k + b) * b, hipMemcpyDeviceToHost, s));
    if (nk > 0) {
      FE_TRY(update(W, V, nk, dC1, -1.0, 1.0));
      FE_TRY(gram(nk + 1, W, dC2));
      FE_HIP(hipMemcpyAsync(hC2, dC2, sizeof(double) * (k + b) * b, hipMemcpyDeviceToHost, s));
      FE_TRY(update(W, V, nk, dC2, -1.0, 1.0));
    }
    FE_TRY(sync());
    std::vector<double> nb(b);
    for (int j = 0; j < b; ++j) nb[j] = std::sqrt(std::max(0.0, hC1[(size_t)(k + j) * b + j]));
    C.assign((size_t)k * b, 0.0);
    for (int i = 0; i < k * b; ++i) C[i] = hC1[i] + (nk > 0 ? hC2[i] : 0.0);
    if (o.verbose >= 2) {
      int bad1 = 0, bad2 = 0;
      for (int i = 0; i < (k + b) * b; ++i) {
        bad1 += !std::isfinite(hC1[i]);
        if (nk > 0) bad2 += !std::isfinite(hC2[i]);
      }
      fprintf(stderr, "[fe_krylov_schur] careful step %d (block %d): non-finite Gram entries %d / %d;"
              " norms before projection:", step, wb, bad1, bad2);
      for (int j = 0; j < b; ++j) fprintf(stderr, " %.3e", hC1[(size_t)(k + j) * b + j]);
      fprintf(stderr, "\n");
    }
    // A non-finite column (a caller's start block) is dependent outright and
    // is overwritten by its refill draws at once: the right multiplications
    // below combine all columns, and NaN x 0 would spread it.
    uint32_t bad_mask = 0;
    for (int j = 0; j < b; ++j)
      if (!std::isfinite(hC1[(size_t)(k + j) * b + j])) bad_mask |= 1u << j;
    const int32_t* perm = A.relabeled ? A.d_perm : nullptr;
    if (bad_mask)
      FE_TRY(random_fill(W, n, b, bad_mask, 1, o.seed, (uint32_t)step, perm, dt, s));
    // column-wise CGS2 in column order
    R.assign((size_t)b * b, 0.0);
    std::vector<int> acc, dep;
    double min_ratio = 1.0;
    for (int j = 0; j < b; ++j) {
      if (bad_mask & (1u << j)) {
        dep.push_back(j);
        continue;
      }
      double nw = 0.0;
      FE_TRY(project_column(wb, j, acc, R, &nw));
      min_ratio = std::min(min_ratio, nb[j] > 0.0 ? nw / nb[j] : 0.0);
      if (o.verbose >= 2)
        fprintf(stderr, "[fe_krylov_schur]   column %d: norm after %.3e (G_jj %.3e), ratio %.3e -> %s\n",
                j, nw, hG[j * b + j], nb[j] > 0.0 ? nw / nb[j] : 0.0,
                (!(nw > eta * nb[j]) || !(nw > 0.0)) ? "dependent" : "kept");
      if (!(nw > eta * nb[j]) || !(nw > 0.0)) {
        dep.push_back(j);
        continue;
      }
      FE_TRY(scale_column(wb, j, 1.0 / nw));
      R[(size_t)j * b + j] = nw;
      acc.push_back(j);
    }
    if (dep.empty()) {
      if (min_ratio >= eta_chol) {
        // well conditioned: Cholesky QR twice of the projected block, rebuilt
        // as Q R from the column-wise factors
        std::copy(R.begin(), R.end(), hM);
        FE_TRY(right_mult(W));
        std::vector<double> Rq;
        bool ok = false;
        FE_TRY(cholqr2(wb, Rq, &ok));
        if (ok) {
          R = Rq;
        } else {  // back to the column-wise factors: W <- W R^-1
          std::vector<double> Ri((size_t)b * b);
          inv_upper(b, R.data(), b, Ri.data(), b);
          std::copy(Ri.begin(), Ri.end(), hM);
          FE_TRY(right_mult(W));
        }
      }
      return FE_OK;
    }
    // refills, in column order, against V (twice) and the kept columns (twice)
    uint32_t mask = 0;
    for (int j : dep) mask |= 1u << j;
    FE_TRY(random_fill(W, n, b, mask, 1, o.seed, (uint32_t)step, perm, dt, s));
    if (nk > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        FE_TRY(gram(nk + 1, W, dC2));
        FE_TRY(update(W, V, nk, dC2, -1.0, 1.0));
      }
    }
    for (int j : dep) {
      std::vector<double> Rdrop((size_t)b * b, 0.0);  // a refill's coefficients are not kept
      double nw = 0.0;
      FE_TRY(project_column(wb, j, acc, Rdrop, &nw));
      if (o.verbose >= 2)
        fprintf(stderr, "[fe_krylov_schur]   refill %d: norm %.3e (G_jj %.3e)\n", j, nw, hG[j * b + j]);
      if (!(nw > 0.0) || !std::isfinite(nw))
        return fail(FE_EBREAKDOWN, "fe_krylov_schur: refill of column %d is dependent (step %d)", j, step);
      FE_TRY(scale_column(wb, j, 1.0 / nw));
      acc.push_back(j);
    }
    refills += (int)dep.size();
    return FE_OK;
  }

  // The start block (no basis yet).  Its Gram matrix decides first: with every
  // column's ratio (Schur complement of the Gram matrix over its diagonal) at
  // least eta_chol, Cholesky QR twice runs on the device, which is what the
  // careful path settles on for such a block; otherwise (a dependent, nearly
  // dependent or non-finite column) the careful path runs.  For a random or
  // learned block this replaces 16 column-by-column passes over the block by
  // four.
  fe_status orth_start(std::vector<double>& C, std::vector<double>& R) {
    void* W = blk(0);
    double* rec = dRec;  // block 0's record: R at m b, the flag after it
    double* flag = rec + (size_t)m * b + (size_t)b * b;
    double* hflag = hRec + (size_t)m * b + (size_t)b * b;
    FE_TRY(gram(1, W, dC));
    FE_TRY(chol_first_launch(dC, dC, 0, b, eta_chol, rec, dR1, dM, flag, s));
    FE_HIP(hipMemcpyAsync(hflag, flag, sizeof(double), hipMemcpyDeviceToHost, s));
    FE_TRY(sync());
    if (*hflag != 0.0) return orth_block(0, C, R);
    FE_TRY(update(W, W, 1, dM, 1.0, 0.0));
    FE_TRY(gram(1, W, dC));
    FE_TRY(chol_second_launch(dC, b, dR1, dM, rec + (size_t)m * b, flag, s));
    FE_HIP(hipMemcpyAsync(hflag, flag, sizeof(double), hipMemcpyDeviceToHost, s));
    FE_TRY(sync());
    if (*hflag != 0.0) return orth_block(0, C, R);  // W R1^-1 spans the same space
    FE_TRY(update(W, W, 1, dM, 1.0, 0.0));
    C.clear();
    R.assign((size_t)b * b, 0.0);  // the start block's factor is not used
    return FE_OK;
  }

  fe_status run(double* evals, void* evecs, fe_ks_report* rep) {
    auto t0 = clk::now();
    FE_TRY(setup());
    const int max_restarts = o.max_restarts > 0 ? o.max_restarts : 500;
    const int32_t* perm = A.relabeled ? A.d_perm : nullptr;
    // start block into block 0 (internal numbering)
    prof.begin(P_OTHER);
    if (o.start && dt != dt_final) {  // mixed: bring the caller's block to the storage dtype
      void* tmp = nullptr;
      FE_TRY(dev.get(&tmp, (size_t)n * b * dtype_size(dt_final)));
      if (perm)
        FE_TRY(permute_rows(tmp, o.start, perm, n, b, dt_final, false, s));
      else
        FE_TRY(copy_block(tmp, o.start, n, b, dt_final, s));
      FE_TRY(convert_launch(blk(0), dt, tmp, dt_final, n * b, s));
      FE_TRY(sync());
      dev.release(tmp);
    } else if (o.start) {
      if (perm)
        FE_TRY(permute_rows(blk(0), o.start, perm, n, b, dt, false, s));
      else
        FE_TRY(copy_block(blk(0), o.start, n, b, dt, s));
    } else {
      FE_TRY(random_fill(blk(0), n, b, 0xFFFFFFFFu, 0, o.seed, 0, perm, dt, s));
    }
    prof.end();
    std::vector<double> C, R;
    step = 0;
    FE_TRY(orth_start(C, R));
    int k = 0;  // basis columns; Q is block k/b
    int restarts = 0;
    std::vector<double> theta(m), Y((size_t)m * m), rho(m);
    bool converged = false;
    int nconv = 0;
    // Start-block check: the worst wanted estimate at the first Rayleigh-Ritz
    // step is the reference; the caller's block is kept once an estimate falls
    // start_drop-fold below it, and abandoned if none has by restart
    // start_check.
    bool start_watch = o.start != nullptr && o.start_check > 0;
    const double start_drop = o.start_drop > 0 ? o.start_drop : 10.0;
    double start_ref = 0.0;
    int start_fallback = -1;
    struct Pending {
      int wb, step0;
    };
    std::vector<Pending> pend;
    for (;;) {
      // Expansion.  Steps run with device-side factors and are checked when
      // the expansion ends; the first flagged step (and every later one) is
      // discarded and redone from its product on, that step on the host path.
      int force_host = -1;
      for (bool redo = true; redo;) {
        redo = false;
        while (k < m) {
          k += b;
          const int wb = k / b;
          const int step0 = step;
          if (pre_product)  // computed during the restart rotation
            pre_product = false;
          else
            FE_TRY(spmm(blk(wb - 1), blk(wb), b));
          ++spmm_calls;
          if (dt != dt_final) ++spmm_low;
          ++step;
          if (wb == force_host) {
            FE_TRY(orth_block(wb, C, R));
            absorb(k, C.data(), R.data());
          } else {
            FE_TRY(orth_fast(wb, dRec + (size_t)wb * rec_stride));
            pend.push_back({wb, step0});
          }
        }
        if (pend.empty()) break;
        const int w0 = pend.front().wb, w1 = pend.back().wb;
        FE_HIP(hipMemcpyAsync(hRec + (size_t)w0 * rec_stride, dRec + (size_t)w0 * rec_stride,
                              sizeof(double) * rec_stride * (w1 - w0 + 1),
                              hipMemcpyDeviceToHost, s));
        FE_TRY(sync());
        for (size_t i = 0; i < pend.size(); ++i) {
          const Pending& P = pend[i];
          const double* rec = hRec + (size_t)P.wb * rec_stride;
          if (rec[(size_t)m * b + (size_t)b * b] != 0.0) {
            if (o.verbose >= 2)
              fprintf(stderr, "[fe_krylov_schur] step %d flagged (%g): redone on the careful path\n",
                      P.step0 + 1, rec[(size_t)m * b + (size_t)b * b]);
            const int dropped = (int)(pend.size() - i);
            spmm_calls -= dropped;
            spmm_cols -= dropped * b;
            if (dt != dt_final) spmm_low -= dropped;
            k = (P.wb - 1) * b;
            step = P.step0;
            force_host = P.wb;
            redo = true;
            break;
          }
          absorb(P.wb * b, rec, rec + (size_t)m * b);
        }
        pend.clear();
      }
      // Rayleigh-Ritz on the symmetric part of T
      auto th = clk::now();
      std::vector<double> S((size_t)m * m), w(m), Z((size_t)m * m);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) S[(size_t)i * m + j] = 0.5 * (T[(size_t)i * m + j] + T[(size_t)j * m + i]);
      if (!sym_eig(m, S.data(), w.data(), Z.data()))
        return fail(FE_ENOCONV, "fe_krylov_schur: projected eigenproblem did not converge");
      std::vector<int> idx(m);
      for (int i = 0; i < m; ++i) idx[i] = i;
      std::sort(idx.begin(), idx.end(), [&](int a, int c) {
        const double fa = std::fabs(w[a]), fc = std::fabs(w[c]);
        if (fa != fc) return fa > fc;
        if (w[a] != w[c]) return w[a] > w[c];
        return a < c;
      });
      for (int j = 0; j < m; ++j) {
        theta[j] = w[idx[j]];
        for (int i = 0; i < m; ++i) Y[(size_t)i * m + j] = Z[(size_t)i * m + idx[j]];
      }
      nconv = 0;
      for (int j = 0; j < m; ++j) {
        double r2 = 0.0;
        for (int i = 0; i < b; ++i) {
          double sum = 0.0;
          for (int t = 0; t < m; ++t) sum += Bk[(size_t)i * m + t] * Y[(size_t)t * m + j];
          r2 += sum * sum;
        }
        rho[j] = std::sqrt(r2) / ritz_scale(theta[j]);
        if (j < nev && rho[j] <= tol) ++nconv;
      }
      converged = nconv == nev;
      t_host += secs(th, clk::now());
      if (o.verbose) {
        double worst = 0.0;
        for (int j = 0; j < nev; ++j) worst = std::max(worst, rho[j]);
        fprintf(stderr, "[fe_krylov_schur] restart %d spmm %d conv %d/%d max rho %.3e theta0 %.12g\n",
                restarts, spmm_calls, nconv, nev, worst, theta[0]);
      }
      if (converged || restarts >= max_restarts) break;
      if (start_watch) {
        double worst = 0.0;
        for (int j = 0; j < nev; ++j) worst = std::max(worst, rho[j]);
        if (restarts == 0) {
          start_ref = worst;
        } else if (worst * start_drop <= start_ref) {
          start_watch = false;
        } else if (restarts >= o.start_check) {
          // a fresh start from the seed's N(0,1) block; with the step count
          // reset the refill draws are those of a solve without a start block
          start_watch = false;
          start_fallback = restarts;
          prof.begin(P_OTHER);
          FE_TRY(random_fill(blk(0), n, b, 0xFFFFFFFFu, 0, o.seed, 0, perm, dt, s));
          prof.end();
          worst_hist.clear();
          std::fill(T.begin(), T.end(), 0.0);
          std::fill(Bk.begin(), Bk.end(), 0.0);
          step = 0;
          FE_TRY(orth_start(C, R));
          k = 0;
          ++restarts;
          continue;
        }
      }
      if (dt != dt_final) {  // mixed: widen once BF16 stalls or is good enough
        double worst = 0.0;
        for (int j = 0; j < nev; ++j) worst = std::max(worst, rho[j]);
        worst_hist.push_back(worst);
        const size_t h = worst_hist.size();
        // stalled: no 10% gain over the best of the three restarts before
        const bool stalled =
            h >= 4 && worst > 0.9 * std::min({worst_hist[h - 2], worst_hist[h - 3], worst_hist[h - 4]});
        if (worst < mixed_switch || stalled) {
          FE_TRY(widen_restart(Y));
          switch_restart = restarts;
          std::fill(T.begin(), T.end(), 0.0);
          std::fill(Bk.begin(), Bk.end(), 0.0);
          FE_TRY(orth_start(C, R));
          k = 0;
          ++restarts;
          continue;
        }
      }
      // restart
      const int p = restart_size(m, b, nev, o.keep);
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < p; ++j) hY[(size_t)i * p + j] = Y[(size_t)i * m + j];
      FE_HIP(hipMemcpyAsync(dY, hY, sizeof(double) * m * p, hipMemcpyHostToDevice, s));
      // the next expansion's first product A Q (Q = block m/b, which the
      // rotation neither reads nor writes) on the second stream, into the
      // spare block, while the rotation runs here
      FE_HIP(hipEventRecord(ev_a, s));
      FE_HIP(hipStreamWaitEvent(s2, ev_a, 0));
      FE_TRY(spmm_on(blk(m / b), spare, b, s2));
      FE_HIP(hipEventRecord(ev_b, s2));
      prof.begin(P_OTHER);
      FE_TRY(rotate_launch(V, n, b, m / b, p / b, stride, dY, dYpad, dt, s));
      FE_TRY(copy_block(blk(p / b), blk(m / b), n, b, dt, s));
      FE_HIP(hipStreamWaitEvent(s, ev_b, 0));
      FE_TRY(copy_block(blk(p / b + 1), spare, n, b, dt, s));
      prof.end();
      pre_product = true;
      std::vector<double> Bn((size_t)b * m, 0.0);
      for (int i = 0; i < b; ++i)
        for (int j = 0; j < p; ++j) {
          double sum = 0.0;
          for (int t = 0; t < m; ++t) sum += Bk[(size_t)i * m + t] * Y[(size_t)t * m + j];
          Bn[(size_t)i * m + j] = sum;
        }
      Bk.swap(Bn);
      std::fill(T.begin(), T.end(), 0.0);
      for (int j = 0; j < p; ++j) T[(size_t)j * m + j] = theta[j];
      k = p;
      ++restarts;
      FE_TRY(sync());  // hY reused next restart
    }
    // final check in FP64: X = V Y[:, :nev], AX = A X, Rayleigh quotients and
    // explicit residuals (the solver's own check of its answer)
    double *X = nullptr, *AX = nullptr;
    FE_TRY(dev.get((void**)&X, (size_t)n * nev * sizeof(double)));
    FE_TRY(dev.get((void**)&AX, (size_t)n * nev * sizeof(double)));
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < nev; ++j) hY[(size_t)i * nev + j] = Y[(size_t)i * m + j];
    for (int j = 0; j < nev; ++j) hTheta[j] = 0.0;
    FE_HIP(hipMemcpyAsync(dY, hY, sizeof(double) * m * nev, hipMemcpyHostToDevice, s));
    FE_HIP(hipMemcpyAsync(dTheta, hTheta, sizeof(double) * nev, hipMemcpyHostToDevice, s));
    prof.begin(P_OTHER);
    FE_TRY(combine_launch(X, nev, n, b, V, m / b, stride, dY, dYpad, dt, s));
    prof.end();
    prof.begin(P_OTHER);
    if (At) {
      FE_TRY(dev.get((void**)&T64, (size_t)n * nev * sizeof(double)));
      FE_TRY(spmm_launch(A, X, T64, nev, FE_F64, s));
      FE_TRY(spmm_launch(*At, T64, AX, nev, FE_F64, s));
    } else {
      FE_TRY(spmm_launch(A, X, AX, nev, FE_F64, s));
    }
    prof.end();
    spmm_cols += nev;
    prof.begin(P_OTHER);
    FE_TRY(resid_launch(AX, X, n, nev, dTheta, dSums, dPartRes, s));
    prof.end();
    FE_HIP(hipMemcpyAsync(hSums, dSums, sizeof(double) * 3 * nev, hipMemcpyDeviceToHost, s));
    FE_TRY(sync());
    std::vector<double> rq(nev), xx(nev);
    for (int j = 0; j < nev; ++j) {
      xx[j] = hSums[3 * j + 1];
      rq[j] = hSums[3 * j] / xx[j];
      hTheta[j] = rq[j];
    }
    FE_HIP(hipMemcpyAsync(dTheta, hTheta, sizeof(double) * nev, hipMemcpyHostToDevice, s));
    prof.begin(P_OTHER);
    FE_TRY(resid_launch(AX, X, n, nev, dTheta, dSums, dPartRes, s));
    if (evecs) FE_TRY(store_rows(evecs, X, perm, n, nev, dt_final, s));  // caller's dtype
    prof.end();
    FE_HIP(hipMemcpyAsync(hSums, dSums, sizeof(double) * 3 * nev, hipMemcpyDeviceToHost, s));
    FE_TRY(sync());
    for (int j = 0; j < nev; ++j) evals[j] = rq[j];
    if (rep) {
      std::memset(rep, 0, sizeof(*rep));
      rep->restarts = restarts;
      rep->spmm_calls = spmm_calls;
      rep->spmm_cols = spmm_cols;
      rep->converged = nconv;
      rep->refills = refills;
      rep->gram_calls = gram_calls;
      rep->update_calls = update_calls;
      rep->switch_restart = switch_restart;
      rep->spmm_calls_low = spmm_low;
      rep->start_fallback = start_fallback;
      rep->device_allocs = dev.allocs;
      for (int j = 0; j < nev; ++j) {
        rep->rho[j] = rho[j];
        rep->ritz[j] = theta[j];
        rep->resid[j] = std::sqrt(std::max(0.0, hSums[3 * j + 2])) /
                        (ritz_scale(rq[j]) * std::sqrt(xx[j]));
      }
      rep->t_spmm = prof.t[P_SPMM];
      rep->t_gram = prof.t[P_GRAM];
      rep->t_update = prof.t[P_UPDATE];
      rep->t_other_dev = prof.t[P_OTHER];
      rep->bytes_spmm = bytes[P_SPMM];
      rep->bytes_gram = bytes[P_GRAM];
      rep->bytes_update = bytes[P_UPDATE];
      rep->t_host = t_host;
      rep->t_total = secs(t0, clk::now());
    }
    return converged ? FE_OK : fail(FE_ENOCONV, "fe_krylov_schur: %d of %d pairs converged after %d restarts", nconv, nev, restarts);
  }
};

}  // namespace
}  // namespace fe

namespace {
fe_status ks_check(const fe::Csr* A, int32_t nev, int32_t block, int32_t m, double tol,
                   const fe_ks_opts& o) {
  using namespace fe;
  if (!A) return fail(FE_EINVAL, "fe_krylov_schur: NULL argument");
  if (!dtype_ok(o.dt)) return fail(FE_EINVAL, "fe_krylov_schur: bad dtype");
  if (block < 1 || block > 16 || m < 1 || m % block || nev < 1 || nev > m - block || !(tol > 0))
    return fail(FE_EINVAL, "fe_krylov_schur: need 1<=block<=16, m %% block == 0, 1<=nev<=m-block, tol>0");
  if (o.which != 0) return fail(FE_EUNSUPPORTED, "fe_krylov_schur: only largest magnitude");
  if (o.keep && (o.keep < nev || o.keep > m - block || (m - o.keep) % block))
    return fail(FE_EINVAL, "fe_krylov_schur: keep=%d needs nev <= keep <= m - block, (m - keep) %% block == 0",
                o.keep);
  const int p = restart_size(m, block, nev, o.keep);
  if (m > 256 || p > 128 || nev > 64)
    return fail(FE_EUNSUPPORTED, "fe_krylov_schur: m=%d keeps p=%d (limits m<=256, p<=128, nev<=64)", m, p);
  if (block != 1 && block != 2 && block != 4 && block != 8 && block != 16)
    return fail(FE_EUNSUPPORTED, "fe_krylov_schur: block must be 1, 2, 4, 8 or 16");
  if ((int64_t)m + block > A->n) return fail(FE_EINVAL, "fe_krylov_schur: m + block > n");
  if (o.workspace && reinterpret_cast<uintptr_t>(o.workspace) % 256)
    return fail(FE_EINVAL, "fe_krylov_schur: workspace not 256-byte aligned");
  return FE_OK;
}
}  // namespace

extern "C" fe_status fe_svds(const fe_csr* A, const fe_csr* At, int32_t nsv, int32_t block,
                             int32_t m, double tol, const fe_ks_opts* opts, double* svals,
                             void* vecs, fe_ks_report* rep) {
  using namespace fe;
  if (!A || !At || !svals) return fail(FE_EINVAL, "fe_svds: NULL argument");
  if (A->n != At->n || A->nnz != At->nnz)
    return fail(FE_EINVAL, "fe_svds: A (n=%lld, nnz=%lld) and At (n=%lld, nnz=%lld) differ",
                (long long)A->n, (long long)A->nnz, (long long)At->n, (long long)At->nnz);
  if (A->relabeled || At->relabeled)
    return fail(FE_EINVAL, "fe_svds: handles must keep the vertex numbering (no FE_RELABEL_BY_DEGREE)");
  fe_ks_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  if (o.workspace) return fail(FE_EUNSUPPORTED, "fe_svds: no caller workspace");
  FE_TRY(ks_check(A, nsv, block, m, tol, o));
  clear_error();
  std::vector<double> lam((size_t)nsv);
  Solver S(*A, nsv, block, m, tol, o);
  S.At = At;
  const fe_status st = S.run(lam.data(), vecs, rep);
  for (int i = 0; i < nsv; ++i) svals[i] = std::sqrt(std::max(lam[(size_t)i], 0.0));
  return st;
}

extern "C" fe_status fe_ks_workspace_bytes(const fe_csr* A, int32_t nev, int32_t block, int32_t m,
                                           const fe_ks_opts* opts, uint64_t* bytes) {
  using namespace fe;
  if (!bytes) return fail(FE_EINVAL, "fe_ks_workspace_bytes: NULL argument");
  fe_ks_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  o.workspace = nullptr;
  FE_TRY(ks_check(A, nev, block, m, 1.0, o));
  const bool mixed = o.mixed != 0 && o.dt != FE_BF16;
  *bytes = ks_workspace_plan(A->n, nev, block, m, o.dt, mixed, o.start != nullptr);
  return FE_OK;
}

extern "C" fe_status fe_krylov_schur(const fe_csr* A, int32_t nev, int32_t block, int32_t m,
                                     double tol, const fe_ks_opts* opts, double* evals,
                                     void* evecs, fe_ks_report* rep) {
  using namespace fe;
  if (!A || !evals) return fail(FE_EINVAL, "fe_krylov_schur: NULL argument");
  fe_ks_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  FE_TRY(ks_check(A, nev, block, m, tol, o));
  if (o.workspace) {
    const bool mixed = o.mixed != 0 && o.dt != FE_BF16;
    const size_t need = ks_workspace_plan(A->n, nev, block, m, o.dt, mixed, o.start != nullptr);
    if (o.workspace_bytes < need)
      return fail(FE_EINVAL, "fe_krylov_schur: workspace of %llu bytes, needs %zu",
                  (unsigned long long)o.workspace_bytes, need);
  }
  clear_error();
  Solver S(*A, nev, block, m, tol, o);
  return S.run(evals, evecs, rep);
}
