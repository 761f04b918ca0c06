/*
 * fe.h -- C ABI of the MI355X block Krylov-Schur hot path.
 *
 * The operations follow the paper's statement of the problem:
 *   - the generic eigen-iteration of its eigensolver-algorithm subsection
 *     (update the subspace, solve the projected problem, residual of the
 *     Ritz pairs, convergence test) with the block extension: b vectors per
 *     step, so the sparse product is a sparse-matrix x dense-block product;
 *   - the sparse matrix multiplication section (pattern matrix, each nonzero
 *     adds an input row to an output row);
 *   - the table of dense operations the eigensolver requires (MvTransMv and
 *     MvTimesMatAddMv with their alpha/beta scalars) in the vector-subspace
 *     section;
 *   - the two-stage reduction for operations whose output is a small matrix
 *     and the row-interval parallelisation of tall-and-skinny operations
 *     (the subsection on parallelising matrix operations).
 *
 * Conventions
 *   - Every function returns fe_status and never throws across the ABI.  On a
 *     non-OK status, fe_last_error() returns a message for the calling thread.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.
 *   - Dense tall-and-skinny blocks are row-major with leading dimension equal
 *     to their width ("packed"): element (i, c) of an n x b block is at
 *     index i*b + c.  A subspace of k = nblk*b columns is a list of nblk such
 *     blocks, block j starting blk_stride elements after block j-1.
 *   - Storage dtypes: FE_F64, FE_F32, FE_BF16 (raw bfloat16 bits, uint16_t).
 *     Sparse sums accumulate in FP32 (FP64 for FE_F64 storage); Gram and
 *     update arithmetic is FP64; results are rounded to the storage dtype by
 *     round-to-nearest-even.
 *   - Kernels run asynchronously on the HIP stream passed as `hip_stream`
 *     (hipStream_t cast to void*; NULL = the null stream).  Callers own all
 *     buffers they pass; the library owns fe_csr handles.
 *   - Calls on distinct handles/streams may run concurrently.  Calls on one
 *     fe_csr handle share its split-row scratch and must not overlap in time.
 */
#ifndef FE_H
#define FE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FE_OK = 0,
  FE_EINVAL = 1,       /* invalid argument (sizes, null pointers, bad CSR) */
  FE_ENOMEM = 2,       /* host or device allocation failed */
  FE_EDEVICE = 3,      /* a HIP runtime call failed; text in fe_last_error() */
  FE_ENOCONV = 4,      /* solver stopped at max_restarts; outputs hold best estimates */
  FE_EBREAKDOWN = 5,   /* subspace could not be extended (refill failed) */
  FE_EUNSUPPORTED = 6  /* valid request outside the library's limits (sizes, shapes) */
} fe_status;

typedef enum { FE_F64 = 0, FE_F32 = 1, FE_BF16 = 2 } fe_dtype;

/* Flags for fe_csr_build / fe_csr_from_csr. */
#define FE_SYMMETRIZE 0x1u        /* add (v,u) for every (u,v) */
#define FE_DEDUPE 0x2u            /* merge repeated (u,v) */
#define FE_DROP_SELF 0x4u         /* drop (u,u) */
#define FE_RELABEL_BY_DEGREE 0x8u /* renumber vertices by descending degree (ties: lower id first) */
#define FE_GRAPH_DEFAULT (FE_SYMMETRIZE | FE_DEDUPE | FE_DROP_SELF)

/* Opaque device CSR: int64 row_ptr[n+1], int32 col_idx[nnz], no value array
   (the adjacency is a 0/1 pattern), plus the degree-binned row schedule and,
   with FE_RELABEL_BY_DEGREE, the vertex permutation. */
typedef struct fe_csr fe_csr;

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *fe_last_error(void);

/* Library version as 10000*major + 100*minor + patch. */
int32_t fe_version(void);

/*
 * Build the device CSR of a graph from a host edge list (src[e], dst[e]),
 * 0 <= src, dst < n < 2^31.  Flags select symmetrising, deduplication,
 * self-loop removal and degree relabelling; each row's columns come out
 * strictly increasing when FE_DEDUPE is set (non-decreasing otherwise).
 * The edge arrays are read only during the call.  The sparse matrix format
 * section of the paper motivates a compact, pattern-only format.
 * Errors: FE_EINVAL (n <= 0, n_edges < 0, null pointers, ids out of range),
 * FE_ENOMEM, FE_EDEVICE.  *out is set only on FE_OK; free with fe_csr_free.
 */
fe_status fe_csr_build(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst,
                       uint32_t flags, fe_csr **out);

/*
 * Adopt an existing host CSR (row_ptr[n+1] int64, col_idx[row_ptr[n]] int32),
 * validated: row_ptr[0] == 0, non-decreasing, columns in [0, n) and strictly
 * increasing within each row.  Only FE_RELABEL_BY_DEGREE is honoured in flags.
 * Errors: FE_EINVAL on any violation, FE_ENOMEM, FE_EDEVICE.
 */
fe_status fe_csr_from_csr(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                          uint32_t flags, fe_csr **out);

/* Sizes of a handle (any output pointer may be NULL). */
fe_status fe_csr_info(const fe_csr *A, int64_t *n, int64_t *nnz, int64_t *max_deg);

/*
 * Host copy of the vertex order used inside the handle: perm[new] = old.
 * Identity unless built with FE_RELABEL_BY_DEGREE.  fe_spmm works in the
 * handle's (new) numbering: row `new` of X/Y belongs to vertex perm[new].
 */
fe_status fe_csr_perm(const fe_csr *A, int32_t *perm);

/* Host copy of the handle's CSR in its own numbering (row_ptr[n+1], col_idx[nnz]). */
fe_status fe_csr_export(const fe_csr *A, int64_t *row_ptr, int32_t *col_idx);

void fe_csr_free(fe_csr *A);

/*
 * Y = A X  (the sparse matrix multiplication section).  X, Y: device, n x b
 * packed row-major in dtype dt, 1 <= b <= 64, must not overlap.  Row i of Y is
 * the sum of the rows of X indexed by row i's columns (an empty row gives 0).
 * Accumulates in FP32 (FP64 for FE_F64); the result is rounded to dt.
 * Errors: FE_EINVAL (b out of range, null pointers, X/Y overlap), FE_EDEVICE.
 */
fe_status fe_spmm(const fe_csr *A, const void *X, void *Y, int32_t b, fe_dtype dt,
                  void *hip_stream);

/*
 * Measurement aid for fe_spmm's memory ceiling on this matrix: the same
 * gathers without the rows.  Every stored column index, in storage order,
 * fetches its row of X (n x b in dt, as in fe_spmm) in the same vector-wide
 * chunks as fe_spmm; the values are summed per workgroup into out (device,
 * fe_spmm_gather_bound_sets() doubles; their values carry no meaning beyond
 * keeping the loads).  Its duration is what the product's gathers alone take
 * (the product itself also reads row offsets, reduces rows and writes Y).
 * Errors: FE_EINVAL (b out of range, NULL, misaligned X), FE_EDEVICE.
 */
fe_status fe_spmm_gather_bound(const fe_csr *A, const void *X, double *out, int32_t b,
                               fe_dtype dt, void *hip_stream);
int32_t fe_spmm_gather_bound_sets(void);

/*
 * The same gathers over a caller's index stream, to measure what another
 * order of the product's gathers would cost: X row idx[e] (device int32,
 * count entries, clamped to [0, n)) for e = 0 .. count-1 in order, X device
 * n x b in dt; out as for fe_spmm_gather_bound.
 * Errors: FE_EINVAL (NULL, sizes, b out of range, misaligned X), FE_EDEVICE.
 */
fe_status fe_gather_rows(const int32_t *idx, int64_t count, const void *X, int64_t n, int32_t b,
                         fe_dtype dt, double *out, void *hip_stream);

/*
 * C = alpha * V^T W  (MvTransMv).  V: device, nblk >= 1 blocks of n x b, block
 * j at V + j*blk_stride elements (blk_stride >= n*b); W: device n x b.
 * C: device FP64, k x b row-major with k = nblk*b.  Arithmetic FP64; the sum
 * over rows is split into fixed row intervals whose partial k x b matrices
 * are added in a fixed order (the two-stage reduction), so repeated calls
 * are bitwise identical.  W may be one of V's blocks.
 * Allocates a stream-ordered partials buffer (freed stream-ordered).
 * Errors: FE_EINVAL (n < 1, b not in [1,64], nblk < 1, k > 1024, null), FE_EDEVICE.
 */
fe_status fe_gram(const void *V, int32_t nblk, int64_t blk_stride, const void *W, int64_t n,
                  int32_t b, fe_dtype dt, double alpha, double *C, void *hip_stream);

/*
 * fe_gram without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it).  Same arguments, result and errors as fe_gram, and the same
 * kernels, so the result is bitwise fe_gram's.  The row-interval partial
 * sums go to a static device array of 2^20 doubles (8 MiB) that each GPU the
 * library runs on holds until the process ends, instead of a per-call
 * buffer.  The partials take min(512, ceil(n/128)) * k * b doubles, so any n
 * works for k * b <= 2048; larger requests return FE_EUNSUPPORTED before
 * anything is launched.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (other streams, other host threads)
 * race and must be serialised by the caller.
 */
fe_status fe_gram_noalloc(const void *V, int32_t nblk, int64_t blk_stride, const void *W,
                          int64_t n, int32_t b, fe_dtype dt, double alpha, double *C,
                          void *hip_stream);

/*
 * W = beta * W + alpha * V C  (MvTimesMatAddMv).  W: device n x b; V: nblk
 * blocks as in fe_gram; C: device FP64 k x b row-major.  FP64 arithmetic,
 * rounded to dt.  Every output row depends only on the same row of V and W
 * (row-interval parallelism).  W may equal V only when nblk == 1 and b <= 16
 * (in-place right multiplication, W <- beta W + alpha W C); any other overlap
 * is FE_EINVAL.  With beta == 0, W is not read (NaNs in it do not propagate).
 * At b = 8 and 16 with k <= 256 and V and the block stride aligned to
 * min(16, 4 x element size) bytes, the solver's MFMA kernel runs (FP64 MFMA
 * contraction, so the FP64 sums are taken in another order than the
 * one-thread-per-row kernel used otherwise).
 * Errors: FE_EINVAL, FE_EDEVICE.
 */
fe_status fe_block_update(void *W, int64_t n, int32_t b, const void *V, int32_t nblk,
                          int64_t blk_stride, const double *C, double alpha, double beta,
                          fe_dtype dt, void *hip_stream);

/*
 * The middle step of classical Gram-Schmidt twice (the reorthogonalisation
 * of Algorithm 1's step (1)) fused into one pass over V:
 *   W <- W - V C            (C: device FP64 k x b, k = nblk*b; FP64
 *                            arithmetic, rounded to dt)
 *   Cout = [V W]^T W        (device FP64 (k + b) x b row-major, taken from
 *                            the rounded W; rows 0..k-1 are V^T W, the last
 *                            b rows W^T W)
 * Equal to fe_block_update (alpha -1, beta 1) followed by fe_gram over the
 * nblk blocks plus W, up to the order of the FP64 sums.  V and W as in
 * fe_gram; W must not overlap V.  At b = 4, 8 and 16 with k + b <= 128 (at
 * b = 8 in FP64: k <= 96) the solver's register-resident kernels run (W, V
 * and the block stride then aligned to min(16, 4 x element size) bytes);
 * otherwise an LDS-tiled kernel with k <= 64.
 * Errors: FE_EINVAL (sizes, NULL, overlap, alignment), FE_EUNSUPPORTED (b not
 * in {1,2,4,8,16}, or k beyond those limits), FE_ENOMEM, FE_EDEVICE.
 */
fe_status fe_block_update_gram(void *W, int64_t n, int32_t b, const void *V, int32_t nblk,
                               int64_t blk_stride, const double *C, double *Cout, fe_dtype dt,
                               void *hip_stream);

/* Options of fe_krylov_schur.  Zero-initialise, then set what you need. */
typedef struct {
  fe_dtype dt;           /* storage dtype of the subspace (default FE_F64 = 0) */
  int32_t which;         /* 0 = largest magnitude (only mode) */
  int32_t max_restarts;  /* 0 -> 500 */
  uint64_t seed;         /* random start and refill draws */
  const void *start;     /* device n x block start block in dt, original vertex
                            order; NULL = N(0,1) drawn from `seed` */
  void *hip_stream;      /* stream for all work (NULL = null stream) */
  double eta;            /* refill threshold: a new column whose norm after projection
                            (against the basis and the block's earlier kept columns,
                            column by column) is <= eta x its norm before is refilled;
                            0 -> 1e-10 (F64), 1e-5 (F32), 3e-2 (BF16).  Blocks with a
                            column ratio below max(eta, 1e-6) are factored column by
                            column instead of by Cholesky QR twice. */
  int32_t profile;       /* 1 = time each kernel class with HIP events */
  int32_t verbose;       /* 1 = print one line per restart to stderr; 2 = also the
                            block QR's column decisions on its careful path */
  int32_t mixed;         /* 1 = mixed-precision storage: the subspace starts in BF16;
                            once the worst wanted residual estimate drops below
                            mixed_switch, or gains less than 10% on the best of the
                            three restarts before (stall), the solve restarts in dt
                            (FP32 or FP64) from one block that sums the wanted Ritz
                            vectors (column j: those with index = j mod block).
                            The caller's start block, if any, is rounded to BF16. */
  double mixed_switch;   /* 0 -> 1e-3 */
  int32_t start_check;   /* with a caller's start block: 0 = keep it whatever happens;
                            c > 0 = abandon it if the worst wanted residual estimate
                            has not fallen start_drop-fold below its value at the first
                            Rayleigh-Ritz step by the c-th restart.  The solve then
                            starts again from the N(0,1) block of `seed` (the block
                            and refill draws of a solve without a start block) in its
                            current storage; the products spent so far stay counted.
                            Ignored without a start block.  (A fallback rule for
                            learned start blocks; not in the paper.) */
  double start_drop;     /* 0 -> 10 */
  void *workspace;       /* NULL: the solve allocates its device memory (hipMalloc) and
                            frees it before returning.  Otherwise a device buffer of at
                            least fe_ks_workspace_bytes() bytes, 256-byte aligned, owned
                            by the caller and used for every device buffer of the solve
                            (the solve then makes no device allocation; it still uses
                            a few KB of pinned host memory).  Its contents on entry do
                            not matter; on return they are undefined. */
  uint64_t workspace_bytes; /* size of `workspace` */
  int32_t keep;          /* Ritz vectors kept at a restart: 0 -> m - block * max(1,
                            (m - nev) / (2 block)); otherwise nev <= keep <= m - block
                            with m - keep a multiple of block (FE_EINVAL if not) */
} fe_ks_opts;

/* Per-solve report (all times in seconds). */
typedef struct {
  int32_t restarts;        /* restarts performed */
  int32_t spmm_calls;      /* width-`block` products in the iteration */
  int32_t spmm_cols;       /* columns multiplied, including the final check */
  int32_t converged;       /* number of wanted pairs meeting tol at the last check */
  int32_t refills;         /* dependent columns replaced by random vectors */
  int32_t gram_calls, update_calls;
  int32_t switch_restart;  /* restart at which a mixed solve widened its storage, -1 if never */
  int32_t spmm_calls_low;  /* products done while the storage was BF16 (mixed solves) */
  double rho[64];          /* Krylov-Schur residual estimate / max(eps^(2/3),|theta|) per pair */
  double ritz[64];         /* Ritz values of the projected matrix at the last check */
  double resid[64];        /* explicit ||A x - q x|| / (max(eps^(2/3),|q|) ||x||), q the
                              FP64 Rayleigh quotient returned in evals */
  double t_spmm, t_gram, t_update, t_other_dev; /* event-timed kernel time (profile=1);
                              t_spmm covers the width-`block` products only */
  double bytes_spmm, bytes_gram, bytes_update;   /* algorithmic HBM bytes moved by those
                              kernel classes: SpMM 4 nnz + 8 (n+1) + 2 n b s; Gram n k s;
                              update n b s (k/b + 2) (s = element size) */
  double t_host, t_total;  /* host small-matrix work; wall clock of the solve */
  int32_t start_fallback;  /* restart at which the caller's start block was abandoned
                              (opts.start_check), -1 if never */
  int32_t device_allocs;   /* device allocations the solve made (0 with a workspace) */
} fe_ks_report;

/*
 * Block Krylov-Schur for the nev largest-magnitude eigenpairs of the
 * symmetric pattern matrix A (the paper's selected solver, following its
 * generic eigen-iteration with the block extension).  block = b vectors per
 * step, m = subspace size (m % block == 0, 1 <= nev <= m - block, nev <= 64,
 * m <= 256, block in {1,2,4,8,16}, m + block <= n; the restart keeps
 * p = opts->keep or m - block * max(1, (m - nev) / (2 block)) vectors,
 * p <= 128), tol > 0: pair i is converged when its
 * Krylov-Schur residual estimate is <= tol * max(eps^(2/3), |theta_i|), eps
 * the FP64 unit roundoff.
 * Final check (FP64 whatever the storage dtype): the Ritz vectors X = V Y are
 * formed in FP64, multiplied by A in FP64, and each value returned is the
 * Rayleigh quotient x^T A x / x^T x with its explicit residual.  The stop
 * test trusts the Krylov relation, which a basis stored in FP32 or BF16
 * carries only to that storage's unit roundoff u_s, so there the explicit
 * residual may exceed tol |theta_i| by about 2 u_s |lambda_1|.
 * Outputs: evals (host double[nev], pairs ordered by Ritz value |theta|
 * descending, ties to the larger theta); evecs (device n x nev in opts->dt,
 * original vertex order, 2-norm 1 up to storage rounding) or NULL; rep (host)
 * or NULL.
 * Device memory: (m + 2 block) * n elements of dt (mixed: of BF16, then from
 * the switch of dt, with n * block doubles during the switch), 2 * nev * n
 * doubles and small FP64 buffers; allocated for the call and freed before
 * return, or carved from opts->workspace (fe_ks_workspace_bytes gives the
 * size).  The solve also runs work on a second stream of its own (created
 * and destroyed by the call, default priority): at each restart the next
 * expansion's first product overlaps the restart rotation, which touches
 * other blocks.  Synchronises the stream before returning.
 * Errors: FE_EINVAL (also a workspace smaller than fe_ks_workspace_bytes or
 * not 256-byte aligned), FE_ENOMEM, FE_EDEVICE, FE_ENOCONV (max_restarts reached;
 * outputs hold the current estimates), FE_EUNSUPPORTED (sizes beyond the limits).
 */
fe_status fe_krylov_schur(const fe_csr *A, int32_t nev, int32_t block, int32_t m, double tol,
                          const fe_ks_opts *opts, double *evals, void *evecs,
                          fe_ks_report *rep);

/*
 * The nsv largest singular values of a square pattern matrix A that need not
 * be symmetric (a directed graph: the paper's billion-node run is the SVD of
 * its directed page graph), with the same block Krylov-Schur applied to the
 * symmetric positive semidefinite operator A^T A: each step's product is
 * A^T (A X), two sparse products.  A and At are handles of the matrix and of
 * its transpose (fe_csr_build on the same arcs with src and dst swapped,
 * both without FE_SYMMETRIZE and without FE_RELABEL_BY_DEGREE).  Options,
 * shapes, tol (relative to each eigenvalue of A^T A) and the report as in
 * fe_krylov_schur (rep->resid: residuals of A^T A x = lambda x; the width-
 * block products are counted once per A^T A application).
 * Outputs: svals (host double[nsv], descending) = sqrt of the eigenvalues of
 * A^T A; vecs (device n x nsv in opts->dt) the right singular vectors, or
 * NULL; left singular vectors are A v / sigma (fe_spmm with A).
 * Errors: as fe_krylov_schur; FE_EINVAL when A and At differ in size or are
 * relabelled; FE_EUNSUPPORTED with opts->workspace.
 */
fe_status fe_svds(const fe_csr *A, const fe_csr *At, int32_t nsv, int32_t block, int32_t m,
                  double tol, const fe_ks_opts *opts, double *svals, void *vecs,
                  fe_ks_report *rep);

/*
 * Device memory fe_krylov_schur needs for these arguments (the options that
 * matter: dt, mixed, and whether a start block is given), so that a caller
 * can pass it as opts->workspace (e.g. a buffer from its own allocator).
 * Same argument checks as fe_krylov_schur (tol is not checked).
 * Errors: FE_EINVAL, FE_EUNSUPPORTED.
 */
fe_status fe_ks_workspace_bytes(const fe_csr *A, int32_t nev, int32_t block, int32_t m,
                                const fe_ks_opts *opts, uint64_t *bytes);

/* ------------------------------------------------------------------------
 * Learned start block (not in the paper: a learned warm start for the
 * solver).  A three-layer graph network over Ahat = D^-1/2 A D^-1/2:
 *   h0_i = [log(1 + deg_i), z_i (15 values)]
 *   S_l = Ahat H_{l-1};  H_l = relu(S_l W_l + H_{l-1} U_l + b_l)   (hidden 64)
 *   X = H_3 P                                                      (8 columns)
 * Parameters live on the device as FP32 masters (flattened in the order
 * W0 U0 b0 W1 U1 b1 W2 U2 b2 P, matrices row-major, 19,136 floats); the dense
 * transforms run on BF16 (or FP32) MFMA with FP32 accumulation, aggregation on fe_spmm
 * in FP32.  z, V and X are device FP32 blocks in the ORIGINAL vertex order
 * (the library permutes for relabelled handles).  Loss against eigenvectors
 * V (n x 8, orthonormal): L = 1 - ||V^T Q||_F^2 / 8 with Q an orthonormal
 * basis of span(X).
 *
 * Memory: each handle owns a device workspace sized to the largest call it
 * has served (inference: 4 x n x 64 + 9n floats; training keeps every
 * activation), held until fe_gnn_free; a call that needs more than the
 * current workspace takes stream-ordered allocations once and the next call
 * grows the workspace.  Calls on one handle must not overlap (they share the
 * workspace, the gradients and the Adam state).
 * ---------------------------------------------------------------------- */
typedef struct fe_gnn fe_gnn;

/* Number of parameters (19,136). */
int64_t fe_gnn_param_count(void);

/* New network with Glorot-uniform weights drawn from Philox(seed), zero
   biases and a fresh Adam state.  compute = FE_BF16 runs the forward
   transforms on BF16 MFMA (BF16 copies of the FP32 weights, FP32
   accumulation); FE_F32 runs them on FP32 MFMA.  Backward contractions are
   FP32 in both modes.  Errors: FE_EINVAL (NULL, other dtype), FE_ENOMEM. */
fe_status fe_gnn_create(uint64_t seed, fe_dtype compute, fe_gnn **out);
void fe_gnn_free(fe_gnn *g);

/* Host copies of the FP32 parameters in the flattened order.  set also
   clears the stored gradients and the Adam state. */
fe_status fe_gnn_get_params(const fe_gnn *g, float *host);
fe_status fe_gnn_set_params(fe_gnn *g, const float *host);

/* Start block X (device n x block FP32, original vertex order) from the
   network's 8 outputs for graph A with random features z (device n x 15
   FP32): block = 8 returns the outputs; block = 1, 2 or 4 folds them, column
   c summing the outputs j = c (mod block), so the block still carries every
   output direction for a solver that starts from fewer columns.
   Synchronises the stream.  Errors: FE_EINVAL (NULL, block not in
   {1,2,4,8}), FE_ENOMEM, FE_EDEVICE. */
fe_status fe_gnn_forward(fe_gnn *g, const fe_csr *A, const float *z, float *X, int32_t block,
                         void *hip_stream);

/* Forward, loss against V (device n x 8 FP32, orthonormal columns) and
   backward; the gradients are kept in g (and copied to grads_host, 19,136
   floats, when not NULL); *loss receives L.  Synchronises the stream. */
fe_status fe_gnn_backward(fe_gnn *g, const fe_csr *A, const float *z, const float *V,
                          double *loss, float *grads_host, void *hip_stream);

/* One Adam step (Kingma & Ba: beta1 0.9, beta2 0.999, eps 1e-8, bias
   corrected) with the gradients stored by the last fe_gnn_backward.  clip > 0
   first scales the gradients by min(1, clip / ||g||_2), the norm taken over
   all parameters (global-norm clipping); clip == 0 disables it.  Asynchronous
   on the stream.  Errors: FE_EINVAL (NULL, no stored gradients, clip < 0). */
fe_status fe_gnn_adam(fe_gnn *g, double lr, double clip, void *hip_stream);

/*
 * Host utility: eigendecomposition of a small dense symmetric matrix (the
 * projected problem of the eigen-iteration, which the paper solves with
 * LAPACK-class code).  a: host n x n row-major (read only); w: host n
 * eigenvalues, unordered; z: host n x n row-major, column j the unit
 * eigenvector of w[j].  Householder tridiagonalisation + implicit-shift QR.
 * Errors: FE_EINVAL (n < 1, NULL), FE_ENOCONV (QL iteration limit).
 */
fe_status fe_dense_symeig(int32_t n, const double *a, double *w, double *z);

#ifdef __cplusplus
}
#endif
#endif /* FE_H */
