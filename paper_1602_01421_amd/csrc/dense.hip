// Tall-and-skinny subspace kernels (the vector-subspace section's table of
// dense operations and its subsection on parallelising them).
//
//   gram    C = alpha V^T W          (MvTransMv)       -- FP64 MFMA, two stages
//   update  W = beta W + alpha V C   (MvTimesMatAddMv) -- FP64 FMA per row
//   rotate  V[:, :p] = V[:, :m] Y    (restart: Ritz vectors in place)
//   combine Out = V Y                (final Ritz vectors)
//   resid   ||A x_i - theta_i x_i||^2 and ||x_i||^2 per column (MvNorm/MvAddMv/MvScale2 fused)
//   permute, copy, random fill
//
// A subspace of k columns is a list of k/b blocks, each n x b row-major
// (packed); row r of every block is contiguous, so a row interval of all
// blocks is read with coalesced vector loads.  Outputs that are small
// matrices are reduced in two stages: per-workgroup partials over a fixed
// row interval, then a fixed-order sum (deterministic), as the paper
// describes for non-tall-and-skinny outputs.
#include "dev_common.h"
#include "fe_internal.h"

namespace fe {
namespace {

// ----------------------------------------------------------------- Gram
// v_mfma_f64_4x4x4f64 computes four independent 4x4x4 products per
// wavefront.  Operand layout (measured on gfx950): lane = 16*kk + 4*blk + x,
// where kk is the contraction index, blk the block, and x the output row i
// for A or the output column j for B.  The accumulator of lane
// 16*i + 4*blk + j holds D_blk[i][j].
// Mapping: contraction index = one of four consecutive matrix rows; block
// blk = a group of four V columns; the same four W columns feed all blocks.
// One instruction therefore performs 4 rows x 16 V-columns x 4 W-columns.
constexpr int kGramWG = 512;          // 8 wavefronts
constexpr int kGramRowsPerIter = 16;  // rows per wavefront per iteration (4 MFMA steps)
constexpr int kGramPG = 4;            // 16-column V groups per workgroup (64 V columns)
constexpr int kCgsWG = 256;           // cgs_last16_kernel: 4 wavefronts
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T, int NQG>
__global__ __launch_bounds__(kGramWG) void gram_kernel(const T* __restrict__ V, int64_t stride,
                                                       const T* __restrict__ W, int64_t n,
                                                       int32_t b, int32_t k, int64_t rows_per_wg,
                                                       double* __restrict__ partials) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kk = lane >> 4, blk = (lane >> 2) & 3, x = lane & 3;
  const int p_base = blockIdx.y * (16 * kGramPG);
  const int q_base = blockIdx.z * (4 * NQG);
  const int npg = min(kGramPG, (k - p_base + 15) / 16);
  const int nqg = min(NQG, (b - q_base + 3) / 4);
  int64_t aoff[kGramPG];
  bool aval[kGramPG];
#pragma unroll
  for (int pg = 0; pg < kGramPG; ++pg) {
    const int p = p_base + pg * 16 + 4 * blk + x;
    aval[pg] = p < k;
    aoff[pg] = aval[pg] ? (int64_t)(p / b) * stride + (p % b) : 0;
  }
  int boff[NQG];
  bool bval[NQG];
#pragma unroll
  for (int qg = 0; qg < NQG; ++qg) {
    const int q = q_base + qg * 4 + x;
    bval[qg] = q < b;
    boff[qg] = bval[qg] ? q : 0;
  }
  double acc[kGramPG][NQG];
#pragma unroll
  for (int pg = 0; pg < kGramPG; ++pg)
#pragma unroll
    for (int qg = 0; qg < NQG; ++qg) acc[pg][qg] = 0.0;

  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r_end = min(n, r_begin + rows_per_wg);
  for (int64_t r0 = r_begin + wave * kGramRowsPerIter; r0 < r_end;
       r0 += (kGramWG / 64) * kGramRowsPerIter) {
    // Unconditional loads from clamped (always valid) addresses, masked after
    // the fact: a guarded load would serialise on its own wait.
    double a[4][kGramPG], bb[4][NQG];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = r0 + 4 * u + kk;
      const bool rv = row < r_end;
      const int64_t rb = (rv ? row : r_end - 1) * b;
#pragma unroll
      for (int pg = 0; pg < kGramPG; ++pg) {
        const double x = load_f64(V + aoff[pg] + rb);
        a[u][pg] = (rv && aval[pg]) ? x : 0.0;
      }
#pragma unroll
      for (int qg = 0; qg < NQG; ++qg) {
        const double x = load_f64(W + rb + boff[qg]);
        bb[u][qg] = (rv && bval[qg]) ? x : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int pg = 0; pg < kGramPG; ++pg)
        if (pg < npg)
#pragma unroll
          for (int qg = 0; qg < NQG; ++qg)
            if (qg < nqg)
              acc[pg][qg] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u][pg], bb[u][qg], acc[pg][qg],
                                                               0, 0, 0);
  }
  // wavefront partials added in wavefront order (deterministic)
  __shared__ double red[kGramPG][NQG][64];
  for (int w = 0; w < kGramWG / 64; ++w) {
    if (wave == w) {
#pragma unroll
      for (int pg = 0; pg < kGramPG; ++pg)
#pragma unroll
        for (int qg = 0; qg < NQG; ++qg)
          red[pg][qg][lane] = (w == 0 ? 0.0 : red[pg][qg][lane]) + acc[pg][qg];
    }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * k * b;
  for (int idx = threadIdx.x; idx < kGramPG * NQG * 64; idx += kGramWG) {
    const int l = idx & 63, qg = (idx >> 6) % NQG, pg = (idx >> 6) / NQG;
    const int i = l >> 4, bl = (l >> 2) & 3, j = l & 3;
    const int p = p_base + pg * 16 + 4 * bl + i, q = q_base + qg * 4 + j;
    if (p < k && q < b) out[(int64_t)p * b + q] = red[pg][qg][l];
  }
}

// Same contraction for b a multiple of 4, with 16-byte row loads: lane x of
// each quad loads the four consecutive columns of row r0 + 4x + kk that its
// quad needs, and a 4 x 4 transpose across the quad (two DPP quad_perm
// stages, 32-bit lanes) hands every lane the operand the plain kernel would
// have loaded with four separate element loads.  Four times fewer load
// instructions; the texture-address unit was 64% busy with element loads.
template <int CTRL>
__device__ __forceinline__ float quad_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_dpp(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// v[c] of quad lane x becomes v[c] of lane c before the call (4 x 4 transpose):
// stage 1 exchanges, between lanes x and x^2, the components c whose bit 1
// differs from x's; stage 2 does the same for bit 0 between x and x^1.
template <typename A>
__device__ __forceinline__ void quad_transpose(A (&v)[4], int x) {
  {
    const A a0 = quad_dpp<0x4E>(v[0]), a1 = quad_dpp<0x4E>(v[1]);  // quad_perm 2,3,0,1
    const A a2 = quad_dpp<0x4E>(v[2]), a3 = quad_dpp<0x4E>(v[3]);
    const bool hi = x & 2;
    v[0] = hi ? a2 : v[0];
    v[1] = hi ? a3 : v[1];
    v[2] = hi ? v[2] : a0;
    v[3] = hi ? v[3] : a1;
  }
  {
    const A a0 = quad_dpp<0xB1>(v[0]), a1 = quad_dpp<0xB1>(v[1]);  // quad_perm 1,0,3,2
    const A a2 = quad_dpp<0xB1>(v[2]), a3 = quad_dpp<0xB1>(v[3]);
    const bool odd = x & 1;
    v[0] = odd ? a1 : v[0];
    v[1] = odd ? v[1] : a0;
    v[2] = odd ? a3 : v[2];
    v[3] = odd ? v[3] : a2;
  }
}

template <typename T, int NQG, int NPG>
__global__ __launch_bounds__(kGramWG) void gram_wide_kernel(const T* __restrict__ V,
                                                            int64_t stride,
                                                            const T* __restrict__ W, int64_t n,
                                                            int32_t b, int32_t k,
                                                            int64_t rows_per_wg,
                                                            double* __restrict__ partials) {
  using A = typename Acc<T>::type;
  constexpr int VEC = 16 / sizeof(T) < 4 ? 16 / sizeof(T) : 4;  // 4 elements per load group
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kk = lane >> 4, blk = (lane >> 2) & 3, x = lane & 3;
  const int p_base = blockIdx.y * (16 * NPG);
  const int q_base = blockIdx.z * (4 * NQG);
  const int nqg = min(NQG, (b - q_base + 3) / 4);
  // column group of this lane's quad: 4 consecutive columns inside one block;
  // quads past k load the last 4 columns (k - 4.., in this slice, loaded by
  // the quad that owns them: the same cache lines) and discard the values
  int64_t aoff[NPG];
  bool aval[NPG];
#pragma unroll
  for (int pg = 0; pg < NPG; ++pg) {
    const int c0 = p_base + pg * 16 + 4 * blk;
    aval[pg] = c0 < k;
    const int cc = aval[pg] ? c0 : k - 4;
    aoff[pg] = (int64_t)(cc / b) * stride + (cc % b);
  }
  int boff[NQG];
  bool bval[NQG];
#pragma unroll
  for (int qg = 0; qg < NQG; ++qg) {
    const int q0 = q_base + qg * 4;
    bval[qg] = q0 < b;
    boff[qg] = bval[qg] ? q0 : 0;
  }
  double acc[NPG][NQG];
#pragma unroll
  for (int pg = 0; pg < NPG; ++pg)
#pragma unroll
    for (int qg = 0; qg < NQG; ++qg) acc[pg][qg] = 0.0;

  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r_end = min(n, r_begin + rows_per_wg);
  for (int64_t r0 = r_begin + wave * kGramRowsPerIter; r0 < r_end;
       r0 += (kGramWG / 64) * kGramRowsPerIter) {
    const int64_t row = r0 + 4 * x + kk;  // the row this lane loads
    const bool rv = row < r_end;
    const int64_t rb = (rv ? row : r_end - 1) * b;
    double a[4][NPG], bb[4][NQG];
#pragma unroll
    for (int pg = 0; pg < NPG; ++pg) {
      A v[4];
#pragma unroll
      for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(V + aoff[pg] + rb + c, v + c);
      const bool ok = rv && aval[pg];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = ok ? v[c] : (A)0;
      quad_transpose(v, x);  // v[u] = element (row r0 + 4u + kk, column c0 + x)
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u][pg] = (double)v[u];
    }
#pragma unroll
    for (int qg = 0; qg < NQG; ++qg) {
      A v[4];
#pragma unroll
      for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(W + rb + boff[qg] + c, v + c);
      const bool ok = rv && bval[qg];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = ok ? v[c] : (A)0;
      quad_transpose(v, x);
#pragma unroll
      for (int u = 0; u < 4; ++u) bb[u][qg] = (double)v[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int pg = 0; pg < NPG; ++pg)
#pragma unroll
          for (int qg = 0; qg < NQG; ++qg)
            if (qg < nqg)
              acc[pg][qg] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u][pg], bb[u][qg], acc[pg][qg],
                                                               0, 0, 0);
  }
  __shared__ double red[NPG][NQG][64];
  for (int w = 0; w < kGramWG / 64; ++w) {
    if (wave == w) {
#pragma unroll
      for (int pg = 0; pg < NPG; ++pg)
#pragma unroll
        for (int qg = 0; qg < NQG; ++qg)
          red[pg][qg][lane] = (w == 0 ? 0.0 : red[pg][qg][lane]) + acc[pg][qg];
    }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * k * b;
  for (int idx = threadIdx.x; idx < NPG * NQG * 64; idx += kGramWG) {
    const int l = idx & 63, qg = (idx >> 6) % NQG, pg = (idx >> 6) / NQG;
    const int i = l >> 4, bl = (l >> 2) & 3, j = l & 3;
    const int p = p_base + pg * 16 + 4 * bl + i, q = q_base + qg * 4 + j;
    if (p < k && q < b) out[(int64_t)p * b + q] = red[pg][qg][l];
  }
}

// CGS2's middle step at b = 4 in one pass over [V W]: W <- W - V C1 and the
// Gram partials of [V W']^T W' (the layout of gram_wide_kernel<T, 1, NPG>).
// V has kv columns; the lanes whose column group is W's (group kv/4) load
// W's old values.  Each lane forms, in FP64, the dot products of its
// 16 V columns with C1 (staged in LDS, zero past kv); a butterfly over the
// four lanes holding the row's other column groups completes them.  W' is
// rounded to T once: that value is stored (by one lane per row) and is what
// the Gram contracts, both as the last V group and as the W operand.  Rows
// of a wavefront are its own, so reading W before writing it is safe.
template <typename T, int NPG>
__global__ __launch_bounds__(kGramWG) void cgs_mid_kernel(const T* __restrict__ V, int64_t stride,
                                                          T* __restrict__ W, int64_t n, int32_t kv,
                                                          const double* __restrict__ C1,
                                                          int64_t rows_per_wg,
                                                          double* __restrict__ partials) {
  using A = typename Acc<T>::type;
  constexpr int VEC = 16 / sizeof(T) < 4 ? 16 / sizeof(T) : 4;
  constexpr int B = 4;
  const int k = kv + B;
  __shared__ double Cs[16 * NPG * B];  // C1 rows, zero from row kv on
  for (int i = threadIdx.x; i < 16 * NPG * B; i += kGramWG) Cs[i] = (i / B < kv) ? C1[i] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kk = lane >> 4, blk = (lane >> 2) & 3, x = lane & 3;
  int64_t aoff[NPG];
  bool aval[NPG], isw[NPG];
#pragma unroll
  for (int pg = 0; pg < NPG; ++pg) {
    const int c0 = pg * 16 + 4 * blk;
    aval[pg] = c0 < k;
    isw[pg] = c0 == kv;
    aoff[pg] = (aval[pg] && !isw[pg]) ? (int64_t)(c0 / B) * stride + (c0 % B) : 0;
  }
  double acc[NPG];
#pragma unroll
  for (int pg = 0; pg < NPG; ++pg) acc[pg] = 0.0;
  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r_end = min(n, r_begin + rows_per_wg);
  for (int64_t r0 = r_begin + wave * kGramRowsPerIter; r0 < r_end;
       r0 += (kGramWG / 64) * kGramRowsPerIter) {
    asm volatile("" ::: "memory");  // keep the C1 reads inside the loop (no hoisting)
    const int64_t row = r0 + 4 * x + kk;  // the row this lane loads
    const bool rv = row < r_end;
    const int64_t rb = (rv ? row : r_end - 1) * B;
    A v[NPG][4], w[4];
#pragma unroll
    for (int pg = 0; pg < NPG; ++pg) {
      const T* src = isw[pg] ? W + rb : V + aoff[pg] + rb;
#pragma unroll
      for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(src + c, v[pg] + c);
      const bool ok = rv && aval[pg];
#pragma unroll
      for (int c = 0; c < 4; ++c) v[pg][c] = ok ? v[pg][c] : (A)0;
    }
#pragma unroll
    for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(W + rb + c, w + c);
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = rv ? w[c] : (A)0;
    // V C1 over this lane's columns, then over the row's four lanes
    double s[B] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int pg = 0; pg < NPG; ++pg)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int col = pg * 16 + 4 * blk + c;
        const double vv = (col < kv) ? (double)v[pg][c] : 0.0;
        const double* cr = Cs + col * B;
#pragma unroll
        for (int j = 0; j < B; ++j) s[j] = fma(vv, cr[j], s[j]);
      }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      s[j] += __shfl_xor(s[j], 4, 64);
      s[j] += __shfl_xor(s[j], 8, 64);
    }
    double d[B];
    A wr[4];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      d[j] = (double)w[j] - s[j];
      const T t = to_storage<T, double>(d[j]);
      if constexpr (sizeof(T) == 2)
        wr[j] = (A)bf16_to_f32(t);
      else
        wr[j] = (A)t;
      d[j] = (double)wr[j];
    }
    if (blk == 0 && rv) {
#pragma unroll
      for (int c = 0; c < 4; c += VEC) store_vec<T, VEC, double>(W + rb + c, d + c);
    }
    double a[4][NPG], bb[4];
#pragma unroll
    for (int pg = 0; pg < NPG; ++pg) {
#pragma unroll
      for (int c = 0; c < 4; ++c) v[pg][c] = isw[pg] ? wr[c] : v[pg][c];
      quad_transpose(v[pg], x);  // v[u] = element (row r0 + 4u + kk, column c0 + x)
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u][pg] = (double)v[pg][u];
    }
    {
      A t[4] = {wr[0], wr[1], wr[2], wr[3]};
      quad_transpose(t, x);
#pragma unroll
      for (int u = 0; u < 4; ++u) bb[u] = (double)t[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int pg = 0; pg < NPG; ++pg)
        acc[pg] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[u][pg], bb[u], acc[pg], 0, 0, 0);
  }
  __shared__ double red[NPG][64];
  for (int wv = 0; wv < kGramWG / 64; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int pg = 0; pg < NPG; ++pg) red[pg][lane] = (wv == 0 ? 0.0 : red[pg][lane]) + acc[pg];
    }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * k * B;
  for (int idx = threadIdx.x; idx < NPG * 64; idx += kGramWG) {
    const int l = idx & 63, pg = idx >> 6;
    const int i = l >> 4, bl = (l >> 2) & 3, j = l & 3;
    const int p = pg * 16 + 4 * bl + i;
    if (p < k) out[(int64_t)p * B + j] = red[pg][l];
  }
}

// CGS2's middle step at b = 16: W <- W - V C1 (V: kv = 16 G columns) and the
// Gram partials of [V W']^T W', one pass over V from memory.  Per 16-row
// group a wavefront forms V C1 on v_mfma_f64_16x16x4f64 in the restart
// contraction's layout (lane (i, k) holds row i, columns 4k..4k+3 of each
// group; output lane j + 16 (i mod 4), register i / 4 = row 4 reg + k,
// column j), rounds W' once to T, stores it, and passes it through a 2 KB
// LDS tile to the Gram's layout (lane (i, k) of step s = row 4k + s, column
// i), in which the G + 1 tiles of [V W']^T W' accumulate as in gram16_kernel.
// V reaches the Gram layout from the registers the update used: a lane
// permutation (ds_bpermute, no LDS storage) gives lane qx + 4 jq + 16 lk the
// four columns 4 jq..4 jq+3 of row 4 lk + qx, then a quad transpose.  The
// next group's V and W loads are issued before this group's W' and Gram
// work, so one group's memory latency overlaps the previous group's MFMAs.
__device__ __forceinline__ float lane_pull(float v, int src4) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src4, __float_as_int(v)));
}
__device__ __forceinline__ double lane_pull(double v, int src4) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src4, (int)(u & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src4, (int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// B = 16: G basis blocks, one 16-column tile each.  B = 8: kv = 8 nblk_v
// basis columns in G = ceil(nblk_v / 2) tiles (tile g = blocks 2g and
// 2g + 1, the second absent when nblk_v is odd); W's 8 columns fill half of
// each 16 x 16 MFMA tile, the other half is fed zeros.
template <typename T, int G, int B>
__global__ __launch_bounds__(kGramWG) void cgs_mid16_kernel(const T* __restrict__ V,
                                                            int64_t stride, T* __restrict__ W,
                                                            int64_t n, int32_t kv,
                                                            const double* __restrict__ C1,
                                                            int64_t rows_per_wg,
                                                            double* __restrict__ partials) {
  using A = typename Acc<T>::type;
  constexpr int VEC = 16 / sizeof(T) < 4 ? 16 / sizeof(T) : 4;
  static_assert(B == 8 || B == 16, "cgs_mid16: b = 8 or 16");
  if constexpr (B == 16) kv = 16 * G;  // a compile-time constant there
  const int k = kv + B;
  constexpr int64_t kStep = (kGramWG / 64) * kGramRowsPerIter;
  __shared__ double Cs[16 * G * B];      // C1 (kv x B), zero rows up to 16 G
  __shared__ double Wt[kGramWG / 64][256];  // per wavefront: W' rows r0..r0+15
  for (int i = threadIdx.x; i < 16 * G * B; i += kGramWG) Cs[i] = i < kv * B ? C1[i] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int qx = li & 3, jq = li >> 2;
  const int pull = 4 * ((4 * lk + qx) + 16 * jq);  // ds_bpermute byte address of the source lane
  f64x4 acc[G + 1];
#pragma unroll
  for (int t = 0; t <= G; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r_end = min(n, r_begin + rows_per_wg);
  const int64_t last = r_end - 1;
  // one 16-row group's loads: V in the update layout, W in the update's output
  // layout (register reg: row r + 4 reg + lk, column li); rows clamped to the
  // workgroup's last row (in bounds; such lanes are masked where used)
  // this lane's four columns 16 g + 4 lk .. + 3 of tile g: block and offset
  // (columns past kv, B = 8 only, read block 0 and meet zero rows of Cs; their
  // Gram rows are not written)
  auto voff = [&](int g) -> int64_t {
    if constexpr (B == 16) {
      return (int64_t)g * stride + 4 * lk;
    } else {
      const int c = 16 * g + 4 * lk;
      return c < kv ? (int64_t)(2 * g + (lk >> 1)) * stride + 4 * (lk & 1) : 0;
    }
  };
  const int lw = li < B ? li : 0;  // W column of this lane (B = 8: lanes 8..15 idle)
  A v[G][4], w[4];
  auto load_group = [&](int64_t r) {
    const int64_t ra = min(r + li, last);
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(V + voff(g) + ra * B + c, v[g] + c);
#pragma unroll
    for (int reg = 0; reg < 4; ++reg)
      w[reg] = (A)load_f64(W + min(r + 4 * reg + lk, last) * B + lw);
  };
  int64_t r0 = r_begin + wave * kGramRowsPerIter;
  if (r0 < r_end) load_group(r0);
  for (; r0 < r_end; r0 += kStep) {
    asm volatile("" ::: "memory");  // keep the C1 reads inside the loop (no hoisting)
    // V C1 for rows r0..r0+15
    f64x4 u = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int st = 0; st < 4; ++st)
        u = __builtin_amdgcn_mfma_f64_16x16x4f64(
            (double)v[g][st], li < B ? Cs[(16 * g + 4 * lk + st) * B + lw] : 0.0, u, 0, 0, 0);
    // this group's V in the Gram layout (before the quad transpose), and its W
    A vg[G][4], wc[4];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int c = 0; c < 4; ++c) vg[g][c] = lane_pull(v[g][c], pull);
#pragma unroll
    for (int reg = 0; reg < 4; ++reg) wc[reg] = w[reg];
    // the next group's loads (past r_end they re-read the last row and are unused)
    load_group(r0 + kStep);
    // W' = W - V C1 in the output layout: register reg = row r0 + 4 reg + lk, column li
#pragma unroll
    for (int reg = 0; reg < 4; ++reg) {
      const int64_t row = r0 + 4 * reg + lk;
      const bool rv = row < r_end;
      const double d = (double)wc[reg] - u[reg];
      const T t = to_storage<T, double>(d);
      double wr;
      if constexpr (sizeof(T) == 2)
        wr = (double)bf16_to_f32(t);
      else
        wr = (double)t;
      if (rv && li < B) W[row * B + li] = t;
      Wt[wave][(4 * reg + lk) * 16 + li] = (rv && li < B) ? wr : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // [V W']^T W' over the same rows in the Gram layout (lane (i, k) of step s:
    // row 4k + s, column i)
    double bw[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) bw[st] = Wt[wave][(4 * lk + st) * 16 + li];
    const bool gv = r0 + 4 * lk + qx < r_end;  // the row this lane's vg holds
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int c = 0; c < 4; ++c) vg[g][c] = gv ? vg[g][c] : (A)0;
      quad_transpose(vg[g], qx);
#pragma unroll
      for (int st = 0; st < 4; ++st)
        acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)vg[g][st], bw[st], acc[g], 0, 0, 0);
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
      acc[G] = __builtin_amdgcn_mfma_f64_16x16x4f64(bw[st], bw[st], acc[G], 0, 0, 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the tile's reads finish before the next rows' writes
  }
  // wavefront partials added in wavefront order (deterministic)
  __shared__ double red[G + 1][4][64];
  for (int w2 = 0; w2 < kGramWG / 64; ++w2) {
    if (wave == w2) {
#pragma unroll
      for (int t = 0; t <= G; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[t][r][lane] = (w2 == 0 ? 0.0 : red[t][r][lane]) + acc[t][r];
    }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * k * B;
  for (int idx = threadIdx.x; idx < (G + 1) * 4 * 64; idx += kGramWG) {
    const int l = idx & 63, r = (idx >> 6) & 3, t = idx >> 8;
    const int i = 4 * r + (l >> 4), q = l & 15;  // row of the 16 x 16 tile, column
    const int p = t < G ? 16 * t + i : kv + i;    // V rows, then W's
    if (q < B && (t < G ? p < kv : i < B)) out[(int64_t)p * B + q] = red[t][r][l];
  }
}

// C[e] = alpha * sum over partial sets x (fixed order: strided lanes, then group order)
__global__ __launch_bounds__(1024) void reduce_partials(const double* __restrict__ partials,
                                                        int32_t nsets, int32_t len, double alpha,
                                                        double* __restrict__ out) {
  const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + l;
  double s = 0.0;
  if (e < len)
    for (int x = g; x < nsets; x += 16) s += partials[(int64_t)x * len + e];
  __shared__ double red[16][64];
  red[g][l] = s;
  __syncthreads();
  if (g == 0 && e < len) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) t += red[i][l];
    out[e] = alpha * t;
  }
}

// Same contraction for b = 16 on v_mfma_f64_16x16x4f64 (A lane i + 16k,
// B lane j + 16k, D lane j + 16 (i mod 4), register i / 4): the output tile is
// 16 V columns x 16 W columns and the contraction runs over rows, four per
// step.  Lane (i, k) of step s needs column i of row r0 + 4k + s; it is
// loaded as one 16-byte group of four columns per lane (lane x of quad q
// loads columns 4q..4q+3 of row r0 + 4k + x) and a quad transpose hands the
// operands over, four times fewer load instructions than element loads.  (At b = 8 half of each tile would be
// padding; the quad-transpose kernel is faster there.)  NPG 16-column V tiles
// per workgroup slice;
// tiles past k are fed zeros (their MFMAs are not skipped, which keeps every
// accumulator chain unconditional).
template <typename T, int NPG>
__global__ __launch_bounds__(kGramWG) void gram16_kernel(const T* __restrict__ V, int64_t stride,
                                                         const T* __restrict__ W, int64_t n,
                                                         int32_t b, int32_t k,
                                                         int64_t rows_per_wg,
                                                         double* __restrict__ partials) {
  using A = typename Acc<T>::type;
  constexpr int VEC = 16 / sizeof(T) < 4 ? 16 / sizeof(T) : 4;
  constexpr int B = 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int x = li & 3, jq = li >> 2;  // quad lane, quad: columns 4 jq .. 4 jq + 3
  const int p_base = blockIdx.y * (16 * NPG);  // slices of NPG whole 16-column blocks
  int64_t aoff[NPG];
  bool aval[NPG];
#pragma unroll
  for (int pg = 0; pg < NPG; ++pg) {
    const int c0 = p_base + 16 * pg;  // a whole block of 16 columns
    aval[pg] = c0 < k;
    aoff[pg] = aval[pg] ? (int64_t)(c0 / B) * stride + 4 * jq : 0;
  }
  f64x4 acc[NPG];
#pragma unroll
  for (int pg = 0; pg < NPG; ++pg) acc[pg] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r_end = min(n, r_begin + rows_per_wg);
  const int64_t last = r_end - 1;
  constexpr int64_t kStep = (kGramWG / 64) * kGramRowsPerIter;
  // each lane loads 4 consecutive columns of row r0 + 4 lk + x (clamped to the
  // workgroup's last row, masked afterwards); the quad transpose then gives
  // lane (4 jq + x) column 4 jq + x of rows r0 + 4 lk + u, u = 0..3: the MFMA
  // operands of steps u.  The next group's loads are issued before this
  // group's MFMAs.
  A wr[4], vr[NPG][4];
  auto load_group = [&](int64_t r) {
    const int64_t rb = min(r + 4 * lk + x, last) * B;
#pragma unroll
    for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(W + rb + 4 * jq + c, wr + c);
#pragma unroll
    for (int pg = 0; pg < NPG; ++pg)
#pragma unroll
      for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(V + aoff[pg] + rb + c, vr[pg] + c);
  };
  int64_t r0 = r_begin + wave * kGramRowsPerIter;
  if (r0 < r_end) load_group(r0);
  for (; r0 < r_end; r0 += kStep) {
    const bool rv = r0 + 4 * lk + x < r_end;
    A w[4], v[NPG][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) w[c] = rv ? wr[c] : (A)0;
#pragma unroll
    for (int pg = 0; pg < NPG; ++pg)
#pragma unroll
      for (int c = 0; c < 4; ++c) v[pg][c] = (rv && aval[pg]) ? vr[pg][c] : (A)0;
    load_group(r0 + kStep);  // past r_end: re-reads the last row, unused
    quad_transpose(w, x);
    double bw[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) bw[u] = (double)w[u];
#pragma unroll
    for (int pg = 0; pg < NPG; ++pg) quad_transpose(v[pg], x);
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int pg = 0; pg < NPG; ++pg)
        acc[pg] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)v[pg][st], bw[st], acc[pg], 0, 0, 0);
  }
  // wavefront partials added in wavefront order (deterministic)
  __shared__ double red[NPG][4][64];
  for (int w = 0; w < kGramWG / 64; ++w) {
    if (wave == w) {
#pragma unroll
      for (int pg = 0; pg < NPG; ++pg)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[pg][r][lane] = (w == 0 ? 0.0 : red[pg][r][lane]) + acc[pg][r];
    }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * k * b;
  for (int idx = threadIdx.x; idx < NPG * 4 * 64; idx += kGramWG) {
    const int l = idx & 63, r = (idx >> 6) & 3, pg = idx >> 8;
    const int p = p_base + 16 * pg + 4 * r + (l >> 4), q = l & 15;
    if (p < k && q < b) out[(int64_t)p * b + q] = red[pg][r][l];
  }
}

int gram_sets(int64_t n) {
  // ~2 workgroups of 8 wavefronts per CU; never fewer rows than one iteration
  int64_t by_rows = (n + 8 * kGramRowsPerIter - 1) / (8 * kGramRowsPerIter);
  return (int)std::max<int64_t>(1, std::min<int64_t>(512, by_rows));
}

// Row intervals of cgs_last16_kernel: four-wavefront workgroups over twice as
// many intervals as the Gram's (measured a little faster there; the middle
// step, at up to ~180 VGPRs, was slower in this shape and keeps the Gram's).
int cgs_sets(int64_t n) {
  int64_t by_rows = (n + 4 * kGramRowsPerIter - 1) / (4 * kGramRowsPerIter);
  return (int)std::max<int64_t>(1, std::min<int64_t>(1024, by_rows));
}

template <typename T>
fe_status gram_t(const void* V, int32_t nblk, int64_t stride, const void* W, int64_t n, int32_t b,
                 double alpha, double* C, double* partials, hipStream_t s) {
  const int32_t k = nblk * b;
  const int gx = gram_sets(n);
  int64_t rows_per_wg = (n + gx - 1) / gx;
  rows_per_wg = (rows_per_wg + 15) / 16 * 16;
  const int gy = (k + 16 * kGramPG - 1) / (16 * kGramPG);
  const int gz = (b + 15) / 16;
  dim3 grid(gx, gy, gz);
  const T* Vp = static_cast<const T*>(V);
  const T* Wp = static_cast<const T*>(W);
#define FE_GRAM(KERNEL, Q)                                                                    \
  hipLaunchKernelGGL((KERNEL<T, Q>), grid, dim3(kGramWG), 0, s, Vp, stride, Wp, n, b, k,      \
                     rows_per_wg, partials)
#define FE_GRAM2(KERNEL, Q, P)                                                                \
  hipLaunchKernelGGL((KERNEL<T, Q, P>), grid, dim3(kGramWG), 0, s, Vp, stride, Wp, n, b, k,   \
                     rows_per_wg, partials)
  if (b == 16) {  // whole 16 x 16 MFMA tiles; the k / 16 tiles split evenly over the slices
    // up to 8 tiles per slice for 4- and 2-byte storage (one pass over W up to
    // 128 columns), 4 for FP64 (register-bound)
    constexpr int max_pg = sizeof(T) <= 4 ? 8 : kGramPG;
    const int tiles = (k + 15) / 16;
    const int slices = (tiles + max_pg - 1) / max_pg;
    const int npg = (tiles + slices - 1) / slices;
    grid.y = slices;
    if (npg == 1) FE_GRAM(gram16_kernel, 1);
    else if (npg == 2) FE_GRAM(gram16_kernel, 2);
    else if (npg == 3) FE_GRAM(gram16_kernel, 3);
    else if (npg == 4) FE_GRAM(gram16_kernel, 4);
    else if constexpr (max_pg == 8) {
      if (npg == 5) FE_GRAM(gram16_kernel, 5);
      else if (npg == 6) FE_GRAM(gram16_kernel, 6);
      else if (npg == 7) FE_GRAM(gram16_kernel, 7);
      else FE_GRAM(gram16_kernel, 8);
    }
  } else if (b % 4 == 0) {  // 16-byte row loads and quad transposes
    // NPG: 16-column V groups per slice, a template parameter so that no MFMA
    // chain is guarded (groups past k are fed zeros); the groups split evenly
    // over the slices, up to 8 per slice at b = 4 and 8 in 4- and 2-byte
    // storage (one pass over W up to 128 columns: each slice reads W), else 4
    constexpr int max_pg = sizeof(T) <= 4 ? 8 : kGramPG;
    const int groups = (k + 15) / 16;
    const int cap = b <= 8 ? max_pg : kGramPG;
    const int slices = (groups + cap - 1) / cap;
    const int npg = (groups + slices - 1) / slices;
    grid.y = slices;
#define FE_GRAM_W(Q)                                                                          \
  if (npg == 1) FE_GRAM2(gram_wide_kernel, Q, 1);                                             \
  else if (npg == 2) FE_GRAM2(gram_wide_kernel, Q, 2);                                        \
  else if (npg == 3) FE_GRAM2(gram_wide_kernel, Q, 3);                                        \
  else if (npg == 4) FE_GRAM2(gram_wide_kernel, Q, 4);                                        \
  else if constexpr (max_pg == 8 && Q <= 2) {                                                 \
    if (npg == 5) FE_GRAM2(gram_wide_kernel, Q, 5);                                           \
    else if (npg == 6) FE_GRAM2(gram_wide_kernel, Q, 6);                                      \
    else if (npg == 7) FE_GRAM2(gram_wide_kernel, Q, 7);                                      \
    else FE_GRAM2(gram_wide_kernel, Q, 8);                                                    \
  }
    if (b == 4) { FE_GRAM_W(1) }
    else if (b == 8) { FE_GRAM_W(2) }
    else { FE_GRAM_W(4) }  // 16 W columns per z-slice
#undef FE_GRAM_W
  } else if (b <= 4) {
    FE_GRAM(gram_kernel, 1);
  } else if (b <= 8) {
    FE_GRAM(gram_kernel, 2);
  } else {
    FE_GRAM(gram_kernel, 4);
  }
#undef FE_GRAM
#undef FE_GRAM2
  FE_HIP(hipGetLastError());
  const int len = k * b;
  hipLaunchKernelGGL(reduce_partials, dim3((len + 63) / 64), dim3(1024), 0, s, partials, gx, len,
                     alpha, C);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// ---------------------------------------------------------------- update
// One thread per row; C (k x B, pre-scaled by alpha) is staged in LDS and read
// with wavefront-uniform addresses (broadcast).
template <typename T, int B>
__global__ __launch_bounds__(256) void update_kernel(T* W, int64_t n,
                                                     const T* V, int32_t nblk,
                                                     int64_t stride, const double* __restrict__ C,
                                                     double alpha, double beta) {
  extern __shared__ double Cs[];
  const int k = nblk * B;
  for (int i = threadIdx.x; i < k * B; i += blockDim.x) Cs[i] = alpha * C[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  constexpr int VEC = (B * sizeof(T) >= 16) ? 16 / sizeof(T) : B;
  double acc[B];
#pragma unroll
  for (int q = 0; q < B; ++q) acc[q] = 0.0;
  for (int jb = 0; jb < nblk; ++jb) {
    const T* vp = V + jb * stride + r * B;
    double v[B];
#pragma unroll
    for (int c0 = 0; c0 < B; c0 += VEC) {
      double tmp[VEC];
      load_vec<T, VEC>(vp + c0, tmp);
#pragma unroll
      for (int c = 0; c < VEC; ++c) v[c0 + c] = tmp[c];
    }
    const double* cr = Cs + jb * B * B;
#pragma unroll
    for (int c = 0; c < B; ++c)
#pragma unroll
      for (int q = 0; q < B; ++q) acc[q] = fma(v[c], cr[c * B + q], acc[q]);
  }
  T* wp = W + r * B;
  if (beta != 0.0) {
#pragma unroll
    for (int c0 = 0; c0 < B; c0 += VEC) {
      double tmp[VEC];
      load_vec<T, VEC>(wp + c0, tmp);
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[c0 + c] = fma(beta, tmp[c], acc[c0 + c]);
    }
  }
#pragma unroll
  for (int c0 = 0; c0 < B; c0 += VEC) store_vec<T, VEC>(wp + c0, acc + c0);
}

// Any b: one thread per output element.
// In-place right multiplication W <- beta W + alpha W C (nblk == 1, b <= 16)
// at widths without a specialised kernel: one thread per row reads its whole
// row before writing any of it (the per-element kernel below would let one
// wavefront overwrite a row another is still reading).  Same arithmetic and
// order as update_generic.
template <typename T>
__global__ __launch_bounds__(256) void update_inplace_generic(T* W, int64_t n, int32_t b,
                                                              const double* __restrict__ C,
                                                              double alpha, double beta) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = c < b ? load_f64(W + r * b + c) : 0.0;
  double y[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c < b && q < b) acc = fma(x[c], C[c * b + q], acc);
    acc *= alpha;
    if (beta != 0.0) acc = fma(beta, x[q], acc);
    y[q] = acc;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (q < b) W[r * b + q] = to_storage<T, double>(y[q]);
}

template <typename T>
__global__ __launch_bounds__(256) void update_generic(T* __restrict__ W, int64_t n, int32_t b,
                                                      const T* __restrict__ V, int32_t nblk,
                                                      int64_t stride, const double* __restrict__ C,
                                                      double alpha, double beta) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  const int64_t r = e / b;
  const int q = (int)(e % b);
  double acc = 0.0;
  for (int jb = 0; jb < nblk; ++jb)
    for (int c = 0; c < b; ++c)
      acc = fma(load_f64(V + jb * stride + r * b + c), C[(int64_t)(jb * b + c) * b + q], acc);
  acc *= alpha;
  if (beta != 0.0) acc = fma(beta, load_f64(W + e), acc);
  W[e] = to_storage<T, double>(acc);
}

// ------------------------------------------------- fused update + Gram
// The middle of a classical Gram-Schmidt sweep in one pass over V:
//   W' = W - V C          (C: the first k rows of the previous Gram, FP64)
//   partial sums of [V W']^T W'   ((k + B) x B, the Gram kernel's layout)
// W' is rounded to T, written back, and the Gram uses the ROUNDED values, so
// the result equals a separate update followed by a Gram up to the order of
// the sums.  Tiles of kUgRows rows of [V W] are staged in LDS as FP64 (exact
// widening of every storage type); arithmetic is FP64.  Each workgroup walks
// a fixed row range; its four wavefronts take interleaved rows and their
// partials are added in wavefront order (deterministic).
constexpr int kUgRows = 64;
constexpr int kUgWG = 256;

int ug_sets(int64_t n) {  // up to 8 resident workgroups per CU on 256 CUs
  const int64_t by_rows = (n + 4 * kUgRows - 1) / (4 * kUgRows);
  return (int)std::max<int64_t>(1, std::min<int64_t>(2048, by_rows));
}

template <typename T, int B>
__global__ __launch_bounds__(kUgWG) void update_gram_kernel(T* __restrict__ W, int64_t n,
                                                            const T* __restrict__ V, int32_t nblk,
                                                            int64_t stride,
                                                            const double* __restrict__ C,
                                                            int64_t rows_per_wg,
                                                            double* __restrict__ partials) {
  constexpr int VEC = (B * sizeof(T) >= 16) ? 16 / sizeof(T) : B;
  constexpr int NU = (kUgRows * B + kUgWG - 1) / kUgWG;  // update outputs per thread
  constexpr int NW = kUgWG / 64;                          // wavefronts
  extern __shared__ double smem[];
  const int k = nblk * B, kk = k + B, ld = kk | 1;  // odd row stride spreads LDS banks
  double* Cs = smem;              // k x B
  double* X = smem + k * B;       // kUgRows x ld: [V row | W row], FP64 (exact widening)
  double* red = X;                // reused at the end: NW x (kk x B) wave partials
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  for (int i = t; i < k * B; i += kUgWG) Cs[i] = C[i];
  // Gram outputs: lane owns columns p = lane and lane + 64 (kk <= 80) and all
  // B columns q of W'; the wavefronts split each tile's rows (r = wave mod NW)
  double acc[2][B];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int q = 0; q < B; ++q) acc[h][q] = 0.0;
  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r_end = min(n, r_begin + rows_per_wg);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kUgRows) {
    const int nr = (int)min((int64_t)kUgRows, r_end - r0);
    __syncthreads();  // Cs staged; the previous tile fully consumed
    const int per = nr * B / VEC;  // vector chunks per block row-range
    for (int c = t; c < (nblk + 1) * per; c += kUgWG) {
      const int j = c / per, off = (c - j * per) * VEC;
      const T* src = (j < nblk ? V + (int64_t)j * stride : W) + r0 * B + off;
      double v[VEC];
      load_vec<T, VEC>(src, v);
      const int r = off / B, col = j * B + off % B;
#pragma unroll
      for (int e = 0; e < VEC; ++e) X[r * ld + col + e] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      const int e = t + i * kUgWG;
      if (e < nr * B) {
        const int r = e / B, q = e % B;
        const double* xr = X + r * ld;
        // same order as the update kernel (sum of V C first, then W), so W'
        // is bitwise what fe_block_update(alpha -1, beta 1) produces
        double a = 0.0;
        for (int p = 0; p < k; ++p) a = fma(xr[p], -Cs[p * B + q], a);
        a = fma(1.0, xr[k + q], a);
        const T o = to_storage<T, double>(a);
        W[(r0 + r) * B + q] = o;
        X[r * ld + k + q] = load_f64(&o);  // only this thread reads this entry
      }
    }
    __syncthreads();
    for (int r = wave; r < nr; r += NW) {
      const double* xr = X + r * ld;
      double w[B];
#pragma unroll
      for (int q = 0; q < B; ++q) w[q] = xr[k + q];  // same address in every lane
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = lane + 64 * h;
        const double x = xr[p < kk ? p : 0];
#pragma unroll
        for (int q = 0; q < B; ++q) acc[h][q] = fma(x, w[q], acc[h][q]);
      }
    }
  }
  // wavefront partials added in wavefront order (deterministic)
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int p = lane + 64 * h;
    if (p < kk)
#pragma unroll
      for (int q = 0; q < B; ++q) red[(wave * kk + p) * B + q] = acc[h][q];
  }
  __syncthreads();
  double* out = partials + (int64_t)blockIdx.x * kk * B;
  for (int e = t; e < kk * B; e += kUgWG) {
    double sum = red[e];
    for (int w2 = 1; w2 < NW; ++w2) sum += red[w2 * kk * B + e];
    out[e] = sum;
  }
}

template <typename T>
fe_status update_gram_t(void* W, int64_t n, int32_t b, const void* V, int32_t nblk,
                        int64_t stride, const double* C, double* Cout, double* partials,
                        hipStream_t s) {
  const int k = nblk * b, kk = k + b, ld = kk | 1;
  if (k > 64 || nblk < 1)
    return fail(FE_EUNSUPPORTED, "update_gram: %d basis columns (1 block .. 64 columns)", k);
  const int gx = ug_sets(n);
  int64_t rows_per_wg = (n + gx - 1) / gx;
  rows_per_wg = (rows_per_wg + kUgRows - 1) / kUgRows * kUgRows;
  // Cs + the tile; the tile area is reused for the 4 wavefronts' partials
  const size_t lds = sizeof(double) * ((size_t)k * b + std::max<size_t>((size_t)kUgRows * ld,
                                                                         (size_t)4 * kk * b));
  T* Wp = static_cast<T*>(W);
  const T* Vp = static_cast<const T*>(V);
#define FE_UG(BB)                                                                              \
  case BB:                                                                                     \
    hipLaunchKernelGGL((update_gram_kernel<T, BB>), dim3(gx), dim3(kUgWG), lds, s, Wp, n, Vp,   \
                       nblk, stride, C, rows_per_wg, partials);                                \
    break;
  switch (b) {
    FE_UG(1) FE_UG(2) FE_UG(4) FE_UG(8) FE_UG(16)
    default:
      return fail(FE_EUNSUPPORTED, "update_gram: block %d not in {1,2,4,8,16}", b);
  }
#undef FE_UG
  FE_HIP(hipGetLastError());
  const int len = kk * b;
  hipLaunchKernelGGL(reduce_partials, dim3((len + 63) / 64), dim3(1024), 0, s, partials, gx, len,
                     1.0, Cout);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

template <typename T>
fe_status update_t(void* W, int64_t n, int32_t b, const void* V, int32_t nblk, int64_t stride,
                   const double* C, double alpha, double beta, hipStream_t s) {
  T* Wp = static_cast<T*>(W);
  const T* Vp = static_cast<const T*>(V);
  const int64_t g = (n + 255) / 256;
  const size_t lds = (size_t)nblk * b * b * sizeof(double);
  if (g > 0x7FFFFFFF) return fail(FE_EUNSUPPORTED, "update: n too large");
#define FE_UPD(BB)                                                                          \
  case BB:                                                                                  \
    hipLaunchKernelGGL((update_kernel<T, BB>), dim3((uint32_t)g), dim3(256), lds, s, Wp, n, Vp, \
                       nblk, stride, C, alpha, beta);                                      \
    break;
  if (lds <= 64 * 1024 && (b == 1 || b == 2 || b == 4 || b == 8 || b == 16)) {
    switch (b) { FE_UPD(1) FE_UPD(2) FE_UPD(4) FE_UPD(8) FE_UPD(16) }
  } else if (W == V && nblk == 1 && b <= 16) {
    hipLaunchKernelGGL((update_inplace_generic<T>), dim3((uint32_t)g), dim3(256), 0, s, Wp, n, b,
                       C, alpha, beta);
  } else {
    const int64_t ge = (n * b + 255) / 256;
    if (ge > 0x7FFFFFFF) return fail(FE_EUNSUPPORTED, "update: n*b too large");
    hipLaunchKernelGGL((update_generic<T>), dim3((uint32_t)ge), dim3(256), 0, s, Wp, n, b, Vp, nblk,
                       stride, C, alpha, beta);
  }
#undef FE_UPD
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// ------------------------------------------------------- rotate / combine
// Out = beta Out + V (alpha Y) for V (n x m, m/B packed blocks) and Y (m x p,
// FP64): the restart V[:, :p] <- V Y in place, the packed FP64 Ritz vectors,
// and the solver's block updates W <- W - V C at wide blocks.  A dense
// tall-and-skinny contraction, so it runs on v_mfma_f64_16x16x4f64 (lane
// layouts measured on gfx950: A lane i + 16k, B lane j + 16k, D lane
// j + 16 (i mod 4), register i / 4): a wavefront owns 16 rows and stores only
// after its last step, so every input of its rows is read before any output
// of them is written and the in-place forms are safe.  When B is a multiple
// of 4 the columns are taken sixteen at a time: lane (i, k) loads the four
// consecutive columns 4k..4k+3 of its row with one vector load and feeds them
// to four MFMA steps, step s contracting over columns {4k + s} (the B
// operand, alpha Y from LDS padded with zeros to whole 16 x 16 tiles, is
// indexed the same way).  Sixteen wavefronts per workgroup share the LDS copy
// of Y.  FP64 arithmetic for every storage type.
// Up to 64 output columns with m16 x p16 <= 64 KB the scaled, zero-padded Y
// sits in LDS; wider (p up to 128) or taller (m up to 256) products read it
// from a padded copy in device memory (GY), where the sixteen lanes of each
// operand read hit the same cache lines.
constexpr int kRotMax = 128;   // p (or c_out): at most eight 16-column tiles
constexpr int kRotRows = 256;  // largest m
constexpr int kRotLdsMax = 64;  // largest p (or c_out) with Y in LDS
constexpr int kRotWG = 512;

// Ypad (m16 x p16) = alpha Y (m x p), zero beyond m and p.
__global__ void pad_y_kernel(const double* __restrict__ Y, int32_t m, int32_t p, int32_t m16,
                             int32_t p16, double alpha, double* __restrict__ Ypad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m16 * p16) return;
  const int t = i / p16, c = i - t * p16;
  Ypad[i] = (t < m && c < p) ? alpha * Y[t * p + c] : 0.0;
}

template <typename T, typename TO, int B, int NT, bool GY>
__global__ __launch_bounds__(kRotWG) void rotate_kernel(TO* Out, int32_t out_mode,  // may alias V
                                                        int32_t c_out, double beta, int64_t n,
                                                        const T* V, int32_t nblk, int64_t stride,
                                                        const double* __restrict__ Y, double alpha,
                                                        int32_t p, int32_t p16, int32_t m16) {
  extern __shared__ double Ysh[];  // m16 x p16: alpha Y, zero beyond m and p
  const int m = nblk * B;
  const double* Ys;
  if constexpr (GY) {
    Ys = Y;  // already scaled and padded to m16 x p16
  } else {
    for (int i = threadIdx.x; i < m16 * p16; i += blockDim.x) {
      const int t = i / p16, c = i - t * p16;
      Ysh[i] = (t < m && c < p) ? alpha * Y[t * p + c] : 0.0;
    }
    __syncthreads();
    Ys = Ysh;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nwave = blockDim.x >> 6;
  const int64_t ngroups = (n + 15) / 16;
  for (int64_t g = (int64_t)blockIdx.x * nwave + wave; g < ngroups;
       g += (int64_t)gridDim.x * nwave) {
    const int64_t r0 = g * 16;
    const int64_t ra = min(r0 + li, n - 1);  // this lane's A row (clamped; not stored)
    f64x4 acc[NT];  // NT = p16 / 16 output tiles
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    if constexpr (B % 4 == 0) {
      constexpr int VEC = 16 / sizeof(T) < 4 ? 16 / sizeof(T) : 4;
      using A = typename Acc<T>::type;
#pragma unroll 1
      for (int kb = 0; kb < m; kb += 16) {
        const int c0 = kb + 4 * lk;  // m is a multiple of 4: all four columns or none
        const bool ok = c0 < m;
        const int cc = ok ? c0 : 0;
        const T* vp = V + (int64_t)(cc / B) * stride + ra * B + (cc % B);
        A v[4];
#pragma unroll
        for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(vp + c, v + c);
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const double a = ok ? (double)v[st] : 0.0;
          const double* yr = Ys + (c0 + st) * p16 + li;  // c0 + st < m16
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, yr[16 * t], acc[t], 0, 0, 0);
        }
      }
    } else {
#pragma unroll 4
      for (int kb = 0; kb < m; kb += 4) {
        const int col = kb + lk;
        const double a = col < m ? load_f64(V + (int64_t)(col / B) * stride + ra * B + (col % B)) : 0.0;
        const double* yr = Ys + (col < m ? col : 0) * p16 + li;
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, yr[16 * t], acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      {
        const int c = 16 * t + li;
#pragma unroll
        for (int reg = 0; reg < 4; ++reg) {
          const int64_t row = r0 + 4 * reg + lk;
          if (row < n) {
            if (out_mode == 0) {
              if (c < p) Out[(int64_t)(c / B) * stride + row * B + (c % B)] = to_storage<TO, double>(acc[t][reg]);
            } else if (c < c_out) {
              TO* o = Out + row * c_out + c;
              const double x = beta != 0.0 ? fma(beta, load_f64(o), acc[t][reg]) : acc[t][reg];
              *o = to_storage<TO, double>(x);
            }
          }
        }
      }
    }
  }
}

template <typename T, typename TO = T>
fe_status rotate_t(void* Out, int32_t out_mode, int32_t c_out, double beta, int64_t n, int32_t b,
                   const void* V, int32_t nblk, int64_t stride, const double* Y, double alpha,
                   int32_t p, double* ypad, hipStream_t s) {
  const int m = nblk * b;
  const int p16 = (p + 15) / 16 * 16;
  const int m16 = (m + 15) / 16 * 16;
  const size_t lds_need = (size_t)m16 * p16 * sizeof(double);
  if (p > kRotMax || m > kRotRows)
    return fail(FE_EUNSUPPORTED, "rotate: m=%d (max %d), p=%d (max %d)", m, kRotRows, p, kRotMax);
  const bool gy = p16 > kRotLdsMax || lds_need > 64 * 1024;
  if (gy && !ypad)
    return fail(FE_EUNSUPPORTED, "rotate: m=%d, p=%d needs the padded-Y buffer", m, p);
  const size_t lds = gy ? 0 : lds_need;
  const double* Yk = Y;
  double a = alpha;
  if (gy) {
    const int cnt = m16 * p16;
    hipLaunchKernelGGL(pad_y_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, Y, m, p, m16, p16,
                       alpha, ypad);
    FE_HIP(hipGetLastError());
    Yk = ypad;
    a = 1.0;
  }
  const int64_t groups = (n + 15) / 16;
  const int wpg = kRotWG / 64;
  const uint32_t grid = (uint32_t)std::max<int64_t>(1, std::min<int64_t>((groups + wpg - 1) / wpg, 2048));
  TO* O = static_cast<TO*>(Out);
  const T* Vp = static_cast<const T*>(V);
#define FE_ROT(BB, NTT, G)                                                                        \
  if (b == BB && p16 == 16 * NTT && gy == G) {                                                    \
    hipLaunchKernelGGL((rotate_kernel<T, TO, BB, NTT, G>), dim3(grid), dim3(kRotWG), lds, s, O,   \
                       out_mode, c_out, beta, n, Vp, nblk, stride, Yk, a, p, p16, m16);          \
    FE_HIP(hipGetLastError());                                                                    \
    return FE_OK;                                                                                 \
  }
#define FE_ROT_B(BB)                                                                              \
  FE_ROT(BB, 1, false) FE_ROT(BB, 2, false) FE_ROT(BB, 3, false) FE_ROT(BB, 4, false)             \
  FE_ROT(BB, 1, true) FE_ROT(BB, 2, true) FE_ROT(BB, 3, true) FE_ROT(BB, 4, true)                 \
  FE_ROT(BB, 5, true) FE_ROT(BB, 6, true) FE_ROT(BB, 7, true) FE_ROT(BB, 8, true)
  FE_ROT_B(1) FE_ROT_B(2) FE_ROT_B(4) FE_ROT_B(8) FE_ROT_B(16)
#undef FE_ROT_B
#undef FE_ROT
  return fail(FE_EUNSUPPORTED, "rotate: block %d not in {1,2,4,8,16}", b);
}

// -------------------------------------------------------------- residual
// Per workgroup, for each column i < c of the FP64 blocks X and AX (n x c):
// sums of x*ax, x*x and (ax - theta_i x)^2; partials reduced later.
constexpr int kResCols = 64;
__global__ __launch_bounds__(256) void resid_kernel(const double* __restrict__ AX,
                                                    const double* __restrict__ X, int64_t n,
                                                    int32_t c, const double* __restrict__ theta,
                                                    int64_t rows_per_wg,
                                                    double* __restrict__ partials) {
  __shared__ double red[4][3 * kResCols];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(n, r0 + rows_per_wg);
  for (int i0 = 0; i0 < c; i0 += 8) {
    double s0[8], s1[8], s2[8], th[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s0[u] = s1[u] = s2[u] = 0.0;
      th[u] = (i0 + u < c) ? theta[i0 + u] : 0.0;
    }
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = r * c + (i0 + u < c ? i0 + u : c - 1);  // clamped, masked below
        const double xr = X[e], axr = AX[e];
        const double x = (i0 + u < c) ? xr : 0.0, ax = (i0 + u < c) ? axr : 0.0;
        const double d = ax - th[u] * x;
        s0[u] = fma(x, ax, s0[u]);
        s1[u] = fma(x, x, s1[u]);
        s2[u] = fma(d, d, s2[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        s0[u] += __shfl_xor(s0[u], off, 64);
        s1[u] += __shfl_xor(s1[u], off, 64);
        s2[u] += __shfl_xor(s2[u], off, 64);
      }
    if (lane == 0)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < c) {
          red[wave][3 * (i0 + u)] = s0[u];
          red[wave][3 * (i0 + u) + 1] = s1[u];
          red[wave][3 * (i0 + u) + 2] = s2[u];
        }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * c; e += 256)
    partials[(int64_t)blockIdx.x * 3 * c + e] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
}

int resid_sets(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 1023) / 1024));
}

// FP64 rows -> storage dtype, optionally scattered through perm (dst[perm[r]] = src[r])
template <typename T>
__global__ void store_rows_kernel(T* __restrict__ dst, const double* __restrict__ src,
                                  const int32_t* __restrict__ perm, int64_t n, int32_t c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t r = e / c, j = e % c;
  const int64_t o = perm ? (int64_t)perm[r] : r;
  dst[o * c + j] = to_storage<T, double>(src[e]);
}

// ------------------------------------------------------------- permute/rng
template <typename T>
__global__ void permute_kernel(T* __restrict__ dst, const T* __restrict__ src,
                               const int32_t* __restrict__ perm, int64_t n, int32_t c,
                               int32_t scatter) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t r = e / c, j = e % c;
  const int64_t o = perm[r];
  if (scatter)
    dst[o * c + j] = src[e];
  else
    dst[e] = src[o * c + j];
}

template <typename T>
__global__ void random_kernel(T* __restrict__ W, int64_t n, int32_t b, uint32_t mask, int32_t mode,
                              uint32_t k0, uint32_t k1, uint32_t step,
                              const int32_t* __restrict__ perm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * b) return;
  const int64_t r = e / b;
  const int j = (int)(e % b);
  if (!((mask >> j) & 1u)) return;
  const uint64_t i = perm ? (uint64_t)(uint32_t)perm[r] : (uint64_t)r;
  double v;
  if (mode == 1) {  // refill: uniform [-1, 1), exact in FP32
    uint4 w = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), step, 0x52460000u + j),
                            k0, k1);
    v = (double)(w.x >> 8) * (1.0 / 8388608.0) - 1.0;
  } else {  // start block: N(0,1) by Box-Muller
    uint4 w = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), j, 0x53545254u), k0, k1);
    const double u1 = 1.0 - ((double)(w.x >> 5) * 67108864.0 + (double)(w.y >> 6)) *
                                (1.0 / 9007199254740992.0);
    const double u2 = ((double)(w.z >> 5) * 67108864.0 + (double)(w.w >> 6)) *
                      (1.0 / 9007199254740992.0);
    v = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
  W[e] = to_storage<T, double>(v);
}

template <typename S, typename D>
__global__ void convert_kernel(D* __restrict__ dst, const S* __restrict__ src, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = to_storage<D, double>(load_f64(src + e));
}

template <typename S>
fe_status convert_from(void* dst, fe_dtype ddt, const S* src, int64_t count, hipStream_t s) {
  const int64_t g = (count + 255) / 256;
  if (g > 0x7FFFFFFF) return fail(FE_EUNSUPPORTED, "convert: too large");
  switch (ddt) {
    case FE_F64:
      hipLaunchKernelGGL((convert_kernel<S, double>), dim3((uint32_t)g), dim3(256), 0, s,
                         static_cast<double*>(dst), src, count);
      break;
    case FE_F32:
      hipLaunchKernelGGL((convert_kernel<S, float>), dim3((uint32_t)g), dim3(256), 0, s,
                         static_cast<float*>(dst), src, count);
      break;
    case FE_BF16:
      hipLaunchKernelGGL((convert_kernel<S, bf16_t>), dim3((uint32_t)g), dim3(256), 0, s,
                         static_cast<bf16_t*>(dst), src, count);
      break;
  }
  FE_HIP(hipGetLastError());
  return FE_OK;
}

}  // namespace

size_t rotate_pad_doubles(int32_t m, int32_t p) {
  return (size_t)((m + 15) / 16 * 16) * (size_t)((p + 15) / 16 * 16);
}

// ------------------------------------------------------------- launchers
size_t gram_partials_doubles(int64_t n, int32_t k, int32_t b) {
  return (size_t)std::max({gram_sets(n), ug_sets(n), cgs_sets(n)}) * (size_t)k * (size_t)b;
}

size_t gram_sets_partials_doubles(int64_t n, int32_t k, int32_t b) {
  return (size_t)gram_sets(n) * (size_t)k * (size_t)b;
}

fe_status update_gram_launch(void* W, int64_t n, int32_t b, const void* V, int32_t nblk,
                             int64_t stride, const double* C, double* Cout, double* partials,
                             fe_dtype dt, hipStream_t s) {
  switch (dt) {
    case FE_F64: return update_gram_t<double>(W, n, b, V, nblk, stride, C, Cout, partials, s);
    case FE_F32: return update_gram_t<float>(W, n, b, V, nblk, stride, C, Cout, partials, s);
    case FE_BF16: return update_gram_t<bf16_t>(W, n, b, V, nblk, stride, C, Cout, partials, s);
  }
  return fail(FE_EINVAL, "update_gram: bad dtype");
}

fe_status gram_launch(const void* V, int32_t nblk, int64_t stride, const void* W, int64_t n,
                      int32_t b, fe_dtype dt, double alpha, double* C, double* partials,
                      hipStream_t s) {
  switch (dt) {
    case FE_F64: return gram_t<double>(V, nblk, stride, W, n, b, alpha, C, partials, s);
    case FE_F32: return gram_t<float>(V, nblk, stride, W, n, b, alpha, C, partials, s);
    case FE_BF16: return gram_t<bf16_t>(V, nblk, stride, W, n, b, alpha, C, partials, s);
  }
  return fail(FE_EINVAL, "gram: bad dtype");
}

template <typename T>
fe_status cgs_mid16_t(void* W, int64_t n, int32_t b, const void* V, int32_t nblk_v, int64_t stride,
                      const double* C1, double* Cout, double* partials, hipStream_t s) {
  const int32_t kv = nblk_v * b, k = kv + b;
  if (nblk_v < 1 || k > 128 || (b != 8 && b != 16))
    return fail(FE_EUNSUPPORTED, "cgs_mid: %d columns at b = %d", k, b);
  const int tiles = (kv + 15) / 16;
  const int gx = gram_sets(n);
  int64_t rows_per_wg = (n + gx - 1) / gx;
  rows_per_wg = (rows_per_wg + 15) / 16 * 16;
  const T* Vp = static_cast<const T*>(V);
  T* Wp = static_cast<T*>(W);
#define FE_MID16(G, BB)                                                                        \
  case G:                                                                                      \
    hipLaunchKernelGGL((cgs_mid16_kernel<T, G, BB>), dim3(gx), dim3(kGramWG), 0, s, Vp, stride, \
                       Wp, n, kv, C1, rows_per_wg, partials);                                  \
    break;
  if (b == 16) {
    switch (tiles) { FE_MID16(1, 16) FE_MID16(2, 16) FE_MID16(3, 16) FE_MID16(4, 16) FE_MID16(5, 16)
                     FE_MID16(6, 16) FE_MID16(7, 16) }
  } else if constexpr (sizeof(T) <= 4) {
    switch (tiles) { FE_MID16(1, 8) FE_MID16(2, 8) FE_MID16(3, 8) FE_MID16(4, 8) FE_MID16(5, 8)
                     FE_MID16(6, 8) FE_MID16(7, 8) FE_MID16(8, 8) }
  } else {
    if (tiles > 6) return fail(FE_EUNSUPPORTED, "cgs_mid: %d columns at b = 8 in FP64", k);
    switch (tiles) { FE_MID16(1, 8) FE_MID16(2, 8) FE_MID16(3, 8) FE_MID16(4, 8) FE_MID16(5, 8)
                     FE_MID16(6, 8) }
  }
#undef FE_MID16
  FE_HIP(hipGetLastError());
  const int len = k * b;
  hipLaunchKernelGGL(reduce_partials, dim3((len + 63) / 64), dim3(1024), 0, s, partials, gx, len,
                     1.0, Cout);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

template <typename T>
fe_status cgs_mid_t(void* W, int64_t n, const void* V, int32_t nblk_v, int64_t stride,
                    const double* C1, double* Cout, double* partials, hipStream_t s) {
  const int32_t kv = nblk_v * 4, k = kv + 4;
  if (k > 128) return fail(FE_EUNSUPPORTED, "cgs_mid: %d columns (max 128)", k);
  const int gx = gram_sets(n);
  int64_t rows_per_wg = (n + gx - 1) / gx;
  rows_per_wg = (rows_per_wg + 15) / 16 * 16;
  const T* Vp = static_cast<const T*>(V);
  T* Wp = static_cast<T*>(W);
  const int npg = (k + 15) / 16;
#define FE_MID(P)                                                                              \
  hipLaunchKernelGGL((cgs_mid_kernel<T, P>), dim3(gx), dim3(kGramWG), 0, s, Vp, stride, Wp, n, \
                     kv, C1, rows_per_wg, partials)
  switch (npg) {
    case 1: FE_MID(1); break;
    case 2: FE_MID(2); break;
    case 3: FE_MID(3); break;
    case 4: FE_MID(4); break;
    case 5: FE_MID(5); break;
    case 6: FE_MID(6); break;
    case 7: FE_MID(7); break;
    default: FE_MID(8); break;
  }
#undef FE_MID
  FE_HIP(hipGetLastError());
  const int len = k * 4;
  hipLaunchKernelGGL(reduce_partials, dim3((len + 63) / 64), dim3(1024), 0, s, partials, gx, len,
                     1.0, Cout);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// The last pass of an orthogonalisation step at b = 8 or 16, in place:
// W <- [V W] Z (Z: kcols x B, the second Gram-Schmidt update and the first
// Cholesky factor's inverse together) and, from the rounded result, the
// partials of W^T W for the second Cholesky factor.  [V W] has kcols columns
// (W its last block) in NT 16-column tiles: at B = 16 one block per tile, at
// B = 8 tile g holds blocks 2g and 2g + 1 (the second absent when the block
// count is odd: those lanes read block 0 and meet zero rows of Z).  W's B
// columns fill the 16 x 16 MFMA tile's first B columns, the rest are fed
// zeros.  Per 16-row group a wavefront forms the product in the restart
// contraction's layout, stores it, and passes it through a 2 KB LDS tile to
// the Gram layout as cgs_mid16_kernel does.  The next group's loads are
// issued before this group's store and Gram.  Every row of W is read by the
// wavefront that writes it, before it writes it.
template <typename T, int NT, int B>
__global__ __launch_bounds__(kCgsWG) void cgs_last16_kernel(T* V, int64_t stride, int64_t n,
                                                             int32_t kcols,
                                                             const double* __restrict__ Z,
                                                             int64_t rows_per_wg,
                                                             double* __restrict__ partials) {
  using A = typename Acc<T>::type;
  constexpr int VEC = 16 / sizeof(T) < 4 ? 16 / sizeof(T) : 4;
  static_assert(B == 8 || B == 16, "cgs_last16: b = 8 or 16");
  if constexpr (B == 16) kcols = 16 * NT;  // a compile-time constant there
  constexpr int64_t kStep = (kCgsWG / 64) * kGramRowsPerIter;
  __shared__ double Zs[16 * NT * 16];  // Z padded to 16 NT x 16 with zeros
  __shared__ double Wt[kCgsWG / 64][256];
  for (int i = threadIdx.x; i < 16 * NT * 16; i += kCgsWG) {
    const int r = i >> 4, j = i & 15;
    Zs[i] = (r < kcols && j < B) ? Z[r * B + j] : 0.0;
  }
  __syncthreads();
  T* W = V + (int64_t)(kcols / B - 1) * stride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r_end = min(n, r_begin + rows_per_wg);
  const int64_t last = r_end - 1;
  // this lane's four columns 16 g + 4 lk .. + 3 of tile g: block and offset
  auto voff = [&](int g) -> int64_t {
    if constexpr (B == 16) {
      return (int64_t)g * stride + 4 * lk;
    } else {
      const int c = 16 * g + 4 * lk;
      return c < kcols ? (int64_t)(2 * g + (lk >> 1)) * stride + 4 * (lk & 1) : 0;
    }
  };
  A v[NT][4];
  auto load_group = [&](int64_t r) {
    const int64_t ra = min(r + li, last);
#pragma unroll
    for (int g = 0; g < NT; ++g)
#pragma unroll
      for (int c = 0; c < 4; c += VEC) load_vec<T, VEC>(V + voff(g) + ra * B + c, v[g] + c);
  };
  int64_t r0 = r_begin + wave * kGramRowsPerIter;
  if (r0 < r_end) load_group(r0);
  for (; r0 < r_end; r0 += kStep) {
    asm volatile("" ::: "memory");  // keep the Z reads inside the loop (no hoisting)
    f64x4 u = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < NT; ++g)
#pragma unroll
      for (int st = 0; st < 4; ++st)
        u = __builtin_amdgcn_mfma_f64_16x16x4f64((double)v[g][st],
                                                 Zs[(16 * g + 4 * lk + st) * 16 + li], u, 0, 0, 0);
    load_group(r0 + kStep);  // past r_end: re-reads the last row, unused
#pragma unroll
    for (int reg = 0; reg < 4; ++reg) {
      const int64_t row = r0 + 4 * reg + lk;
      const bool rv = row < r_end && li < B;
      const T t = to_storage<T, double>(u[reg]);
      double wr;
      if constexpr (sizeof(T) == 2)
        wr = (double)bf16_to_f32(t);
      else
        wr = (double)t;
      if (rv) W[row * B + li] = t;
      Wt[wave][(4 * reg + lk) * 16 + li] = rv ? wr : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double bw[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) bw[st] = Wt[wave][(4 * lk + st) * 16 + li];
#pragma unroll
    for (int st = 0; st < 4; ++st) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bw[st], bw[st], acc, 0, 0, 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // the tile's reads finish before the next rows' writes
  }
  // wavefront partials added in wavefront order (deterministic)
  __shared__ double red[4][64];
  for (int w2 = 0; w2 < kCgsWG / 64; ++w2) {
    if (wave == w2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) red[r][lane] = (w2 == 0 ? 0.0 : red[r][lane]) + acc[r];
    }
    __syncthreads();
  }
  double* out = partials + (int64_t)blockIdx.x * B * B;
  for (int idx = threadIdx.x; idx < 4 * 64; idx += kCgsWG) {
    const int l = idx & 63, r = idx >> 6;
    const int i = 4 * r + (l >> 4), j = l & 15;
    if (i < B && j < B) out[i * B + j] = red[r][l];
  }
}

template <typename T>
fe_status cgs_last16_t(void* V, int32_t b, int32_t nblocks, int64_t stride, int64_t n,
                       const double* Z, double* G, double* partials, hipStream_t s) {
  const int gx = cgs_sets(n);
  int64_t rows_per_wg = (n + gx - 1) / gx;
  rows_per_wg = (rows_per_wg + 15) / 16 * 16;
  T* Vp = static_cast<T*>(V);
  const int32_t kcols = nblocks * b;
  const int tiles = (kcols + 15) / 16;
#define FE_LAST16(NT, BB)                                                                      \
  case NT:                                                                                     \
    hipLaunchKernelGGL((cgs_last16_kernel<T, NT, BB>), dim3(gx), dim3(kCgsWG), 0, s, Vp, stride, \
                       n, kcols, Z, rows_per_wg, partials);                                    \
    break;
  if (b == 16) {
    switch (tiles) {
      FE_LAST16(2, 16) FE_LAST16(3, 16) FE_LAST16(4, 16) FE_LAST16(5, 16) FE_LAST16(6, 16)
      FE_LAST16(7, 16) FE_LAST16(8, 16)
      default:
        return fail(FE_EUNSUPPORTED, "cgs_last: %d blocks at b = 16", nblocks);
    }
  } else {
    switch (tiles) {
      FE_LAST16(1, 8) FE_LAST16(2, 8) FE_LAST16(3, 8) FE_LAST16(4, 8) FE_LAST16(5, 8)
      FE_LAST16(6, 8) FE_LAST16(7, 8) FE_LAST16(8, 8)
      default:
        return fail(FE_EUNSUPPORTED, "cgs_last: %d blocks at b = 8", nblocks);
    }
  }
#undef FE_LAST16
  FE_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_partials, dim3((b * b + 63) / 64), dim3(1024), 0, s, partials, gx,
                     b * b, 1.0, G);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

bool cgs_last_supported(int32_t b, int32_t nblocks) {
  if (b == 16) return nblocks >= 2 && nblocks <= 8;
  if (b == 8) return nblocks >= 2 && nblocks <= 16;
  return false;
}

fe_status cgs_last_launch(void* V, int32_t b, int32_t nblocks, int64_t stride, int64_t n,
                          const double* Z, double* G, double* partials, fe_dtype dt,
                          hipStream_t s) {
  if (!cgs_last_supported(b, nblocks))
    return fail(FE_EUNSUPPORTED, "cgs_last: b=%d with %d blocks", b, nblocks);
  switch (dt) {
    case FE_F64: return cgs_last16_t<double>(V, b, nblocks, stride, n, Z, G, partials, s);
    case FE_F32: return cgs_last16_t<float>(V, b, nblocks, stride, n, Z, G, partials, s);
    case FE_BF16: return cgs_last16_t<bf16_t>(V, b, nblocks, stride, n, Z, G, partials, s);
  }
  return fail(FE_EINVAL, "cgs_last: bad dtype");
}

bool cgs_mid_supported(int32_t b, int32_t nblk_v, fe_dtype dt) {
  if (b == 4 || b == 16) return nblk_v >= 1 && nblk_v * b + b <= 128;
  // b = 8: up to 15 basis blocks (8 tiles) in 4- and 2-byte storage, 12 (6
  // tiles) in FP64, whose register tiles would spill beyond
  if (b == 8) return nblk_v >= 1 && nblk_v <= (dt == FE_F64 ? 12 : 15);
  return false;
}

fe_status cgs_mid_launch(void* W, int64_t n, int32_t b, const void* V, int32_t nblk_v,
                         int64_t stride, const double* C1, double* Cout, double* partials,
                         fe_dtype dt, hipStream_t s) {
  if (!cgs_mid_supported(b, nblk_v, dt))
    return fail(FE_EUNSUPPORTED, "cgs_mid: b=%d with %d basis blocks", b, nblk_v);
  if (b == 8 || b == 16) {
    switch (dt) {
      case FE_F64: return cgs_mid16_t<double>(W, n, b, V, nblk_v, stride, C1, Cout, partials, s);
      case FE_F32: return cgs_mid16_t<float>(W, n, b, V, nblk_v, stride, C1, Cout, partials, s);
      case FE_BF16: return cgs_mid16_t<bf16_t>(W, n, b, V, nblk_v, stride, C1, Cout, partials, s);
    }
  } else {
    switch (dt) {
      case FE_F64: return cgs_mid_t<double>(W, n, V, nblk_v, stride, C1, Cout, partials, s);
      case FE_F32: return cgs_mid_t<float>(W, n, V, nblk_v, stride, C1, Cout, partials, s);
      case FE_BF16: return cgs_mid_t<bf16_t>(W, n, V, nblk_v, stride, C1, Cout, partials, s);
    }
  }
  return fail(FE_EINVAL, "cgs_mid: bad dtype");
}

fe_status update_launch(void* W, int64_t n, int32_t b, const void* V, int32_t nblk, int64_t stride,
                        const double* C, double alpha, double beta, fe_dtype dt, hipStream_t s) {
  switch (dt) {
    case FE_F64: return update_t<double>(W, n, b, V, nblk, stride, C, alpha, beta, s);
    case FE_F32: return update_t<float>(W, n, b, V, nblk, stride, C, alpha, beta, s);
    case FE_BF16: return update_t<bf16_t>(W, n, b, V, nblk, stride, C, alpha, beta, s);
  }
  return fail(FE_EINVAL, "update: bad dtype");
}

fe_status rotate_launch(void* V, int64_t n, int32_t b, int32_t nblk_in, int32_t nblk_out,
                        int64_t stride, const double* Y, double* ypad, fe_dtype dt, hipStream_t s) {
  const int32_t p = nblk_out * b;
  switch (dt) {
    case FE_F64: return rotate_t<double>(V, 0, 0, 0.0, n, b, V, nblk_in, stride, Y, 1.0, p, ypad, s);
    case FE_F32: return rotate_t<float>(V, 0, 0, 0.0, n, b, V, nblk_in, stride, Y, 1.0, p, ypad, s);
    case FE_BF16: return rotate_t<bf16_t>(V, 0, 0, 0.0, n, b, V, nblk_in, stride, Y, 1.0, p, ypad, s);
  }
  return fail(FE_EINVAL, "rotate: bad dtype");
}

fe_status combine_launch(double* Out, int32_t c, int64_t n, int32_t b, const void* V, int32_t nblk,
                         int64_t stride, const double* Y, double* ypad, fe_dtype dt, hipStream_t s) {
  switch (dt) {
    case FE_F64: return rotate_t<double, double>(Out, 1, c, 0.0, n, b, V, nblk, stride, Y, 1.0, c, ypad, s);
    case FE_F32: return rotate_t<float, double>(Out, 1, c, 0.0, n, b, V, nblk, stride, Y, 1.0, c, ypad, s);
    case FE_BF16: return rotate_t<bf16_t, double>(Out, 1, c, 0.0, n, b, V, nblk, stride, Y, 1.0, c, ypad, s);
  }
  return fail(FE_EINVAL, "combine: bad dtype");
}

fe_status mult_update_launch(void* W, int64_t n, int32_t b, const void* V, int32_t nblk,
                             int64_t stride, const double* C, double alpha, double beta,
                             double* ypad, fe_dtype dt, hipStream_t s) {
  switch (dt) {
    case FE_F64: return rotate_t<double>(W, 1, b, beta, n, b, V, nblk, stride, C, alpha, b, ypad, s);
    case FE_F32: return rotate_t<float>(W, 1, b, beta, n, b, V, nblk, stride, C, alpha, b, ypad, s);
    case FE_BF16: return rotate_t<bf16_t>(W, 1, b, beta, n, b, V, nblk, stride, C, alpha, b, ypad, s);
  }
  return fail(FE_EINVAL, "update: bad dtype");
}

// ------------------------------------------- block QR factors on the device
// The small factorisations of one orthogonalisation step, done on the GPU so
// that the common case (no dependent column) needs no host round trip.  One
// workgroup; the b x b Gram of the step is formed in parallel, then thread 0
// runs exactly the host's serial FP64 recurrences (same operations, same
// order), so the factors are bitwise those of the host path.
constexpr int kCholMaxB = 16;

// Column j of the inverse of the upper-triangular R (nb x nb), the host's
// recurrence; columns are independent, so threads take one each.
__device__ void dev_inv_upper_col(int nb, const double* R, double* Ri, int j) {
  for (int i = j + 1; i < nb; ++i) Ri[i * nb + j] = 0.0;
  Ri[j * nb + j] = 1.0 / R[j * nb + j];
  for (int i = j - 1; i >= 0; --i) {
    double acc = 0.0;
    for (int t = i + 1; t <= j; ++t) acc += R[i * nb + t] * Ri[t * nb + j];
    Ri[i * nb + j] = -acc / R[i * nb + i];
  }
}

// Thread 0 factors G (b x b, LDS) into R (LDS) with the dependence test of the
// first pass (eta > 0, column norms before projection from C1) or plainly
// (eta < 0); returns through *ok.
__device__ void dev_chol(const double* G, double* R, int b, double eta, const double* C1, int k,
                         int* ok) {
  for (int i = 0; i < b * b; ++i) R[i] = 0.0;
  int good = 1;
  for (int j = 0; j < b && good; ++j) {
    double d = G[j * b + j];
    for (int i = 0; i < j; ++i) d -= R[i * b + j] * R[i * b + j];
    double thr = 0.0;
    if (eta > 0.0) thr = eta * sqrt(fmax(0.0, C1[(k + j) * b + j]));
    if (!(d > thr * thr) || !(d > 0.0)) {
      good = 0;
      break;
    }
    const double rjj = sqrt(d);
    R[j * b + j] = rjj;
    for (int l = j + 1; l < b; ++l) {
      double g = G[j * b + l];
      for (int i = 0; i < j; ++i) g -= R[i * b + j] * R[i * b + l];
      R[j * b + l] = g / rjj;
    }
  }
  *ok = good;
}

// First pass.  C1, C2: (k + b) x b Grams of [V W] with W before / after the
// first projection.  Writes C = C1 + C2 (rows < k) to rec, the factor R1 of
// G = W2^T W2 = C2[k:] - C2[:k]^T C2[:k] to R1, M = R1^-1, and *flag = 1 when a
// column is dependent (norm after projection <= eta x norm before).
__global__ __launch_bounds__(256) void chol_first_kernel(const double* __restrict__ C1,
                                                         const double* __restrict__ C2, int k,
                                                         int b, double eta, double* __restrict__ rec,
                                                         double* __restrict__ R1,
                                                         double* __restrict__ M,
                                                         double* __restrict__ flag) {
  __shared__ double G[kCholMaxB * kCholMaxB], R[kCholMaxB * kCholMaxB];
  __shared__ int ok;
  for (int e = threadIdx.x; e < k * b; e += blockDim.x) rec[e] = C1[e] + C2[e];
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    double g = C2[(k + i) * b + j];
    for (int t = 0; t < k; ++t) g -= C2[t * b + i] * C2[t * b + j];
    G[e] = g;
  }
  __syncthreads();
  if (threadIdx.x == 0) dev_chol(G, R, b, eta, C1, k, &ok);
  __syncthreads();
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) R1[e] = R[e];
  if (ok) {
    if ((int)threadIdx.x < b) dev_inv_upper_col(b, R, M, threadIdx.x);
  } else {
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) M[e] = (e / b == e % b) ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) flag[0] = ok ? 0.0 : 1.0;
}

// Second pass (Cholesky QR of the right-multiplied block): G = W^T W (b x b),
// Rp its Cholesky factor, M = Rp^-1, recR = Rp R1; flag += 2 on failure.
__global__ __launch_bounds__(256) void chol_second_kernel(const double* __restrict__ G, int b,
                                                          const double* __restrict__ R1,
                                                          double* __restrict__ M,
                                                          double* __restrict__ recR,
                                                          double* __restrict__ flag) {
  __shared__ double Gs[kCholMaxB * kCholMaxB], Rp[kCholMaxB * kCholMaxB];
  __shared__ int ok;
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) Gs[e] = G[e];
  __syncthreads();
  if (threadIdx.x == 0) dev_chol(Gs, Rp, b, -1.0, nullptr, 0, &ok);
  __syncthreads();
  if (!ok) {
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) M[e] = (e / b == e % b) ? 1.0 : 0.0;
    if (threadIdx.x == 0) flag[0] += 2.0;
    return;
  }
  if ((int)threadIdx.x < b) dev_inv_upper_col(b, Rp, M, threadIdx.x);
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    double acc = 0.0;
    for (int t = 0; t < b; ++t) acc += Rp[i * b + t] * R1[t * b + j];
    recR[e] = acc;
  }
}

fe_status chol_first_launch(const double* C1, const double* C2, int32_t k, int32_t b, double eta,
                            double* rec, double* R1, double* M, double* flag, hipStream_t s) {
  if (b > kCholMaxB) return fail(FE_EUNSUPPORTED, "chol: block %d > %d", b, kCholMaxB);
  hipLaunchKernelGGL(chol_first_kernel, dim3(1), dim3(256), 0, s, C1, C2, k, b, eta, rec, R1, M,
                     flag);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

fe_status chol_second_launch(const double* G, int32_t b, const double* R1, double* M,
                             double* recR, double* flag, hipStream_t s) {
  if (b > kCholMaxB) return fail(FE_EUNSUPPORTED, "chol: block %d > %d", b, kCholMaxB);
  hipLaunchKernelGGL(chol_second_kernel, dim3(1), dim3(256), 0, s, G, b, R1, M, recR, flag);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// Z ((k + b) x b, row-major) = [-C2 M; M]: with it one right-multiplication
// W <- [V W] Z applies the second Gram-Schmidt update (W - V C2) and the
// inverse of the first Cholesky factor (M) together, one pass over [V W]
// instead of an update pass and an in-place pass over W.
__global__ __launch_bounds__(256) void cgs_coef_kernel(const double* __restrict__ C2,
                                                       const double* __restrict__ M, int k, int b,
                                                       double* __restrict__ Z) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < (k + b) * b; e += gridDim.x * blockDim.x) {
    const int i = e / b, j = e % b;
    double z;
    if (i < k) {
      double acc = 0.0;
      for (int l = 0; l < b; ++l) acc = fma(C2[i * b + l], M[l * b + j], acc);
      z = -acc;
    } else {
      z = M[(i - k) * b + j];
    }
    Z[e] = z;
  }
}

fe_status cgs_coef_launch(const double* C2, const double* M, int32_t k, int32_t b, double* Z,
                          hipStream_t s) {
  const int cnt = (k + b) * b;
  hipLaunchKernelGGL(cgs_coef_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, C2, M, k, b, Z);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

size_t resid_partials_doubles(int64_t n, int32_t c) { return (size_t)resid_sets(n) * 3 * c; }

fe_status resid_launch(const double* AX, const double* X, int64_t n, int32_t c,
                       const double* theta, double* sums, double* partials, hipStream_t s) {
  if (c > kResCols) return fail(FE_EUNSUPPORTED, "resid: %d columns (max %d)", c, kResCols);
  const int g = resid_sets(n);
  const int64_t rpw = (n + g - 1) / g;
  hipLaunchKernelGGL(resid_kernel, dim3(g), dim3(256), 0, s, AX, X, n, c, theta, rpw, partials);
  FE_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_partials, dim3((3 * c + 63) / 64), dim3(1024), 0, s, partials, g,
                     3 * c, 1.0, sums);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

fe_status store_rows(void* dst, const double* src, const int32_t* perm, int64_t n, int32_t c,
                     fe_dtype dt, hipStream_t s) {
  const int64_t g = (n * c + 255) / 256;
  if (g > 0x7FFFFFFF) return fail(FE_EUNSUPPORTED, "store_rows: too large");
#define FE_ST(TT)                                                                                 \
  hipLaunchKernelGGL((store_rows_kernel<TT>), dim3((uint32_t)g), dim3(256), 0, s, static_cast<TT*>(dst), \
                     src, perm, n, c);
  switch (dt) {
    case FE_F64: FE_ST(double) break;
    case FE_F32: FE_ST(float) break;
    case FE_BF16: FE_ST(bf16_t) break;
  }
#undef FE_ST
  FE_HIP(hipGetLastError());
  return FE_OK;
}

fe_status copy_block(void* dst, const void* src, int64_t n, int32_t b, fe_dtype dt,
                     hipStream_t s) {
  FE_HIP(hipMemcpyAsync(dst, src, (size_t)n * b * dtype_size(dt), hipMemcpyDeviceToDevice, s));
  return FE_OK;
}

fe_status permute_rows(void* dst, const void* src, const int32_t* perm, int64_t n, int32_t c,
                       fe_dtype dt, bool scatter, hipStream_t s) {
  const int64_t g = (n * c + 255) / 256;
  if (g > 0x7FFFFFFF) return fail(FE_EUNSUPPORTED, "permute: too large");
#define FE_PERM(TT)                                                                              \
  hipLaunchKernelGGL((permute_kernel<TT>), dim3((uint32_t)g), dim3(256), 0, s, static_cast<TT*>(dst), \
                     static_cast<const TT*>(src), perm, n, c, (int32_t)scatter);
  switch (dt) {
    case FE_F64: FE_PERM(double) break;
    case FE_F32: FE_PERM(float) break;
    case FE_BF16: FE_PERM(bf16_t) break;
  }
#undef FE_PERM
  FE_HIP(hipGetLastError());
  return FE_OK;
}

fe_status random_fill(void* W, int64_t n, int32_t b, uint32_t mask, int32_t mode, uint64_t seed,
                      uint32_t step, const int32_t* perm, fe_dtype dt, hipStream_t s) {
  const int64_t g = (n * b + 255) / 256;
  if (g > 0x7FFFFFFF) return fail(FE_EUNSUPPORTED, "random_fill: too large");
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#define FE_RNG(TT)                                                                               \
  hipLaunchKernelGGL((random_kernel<TT>), dim3((uint32_t)g), dim3(256), 0, s, static_cast<TT*>(W), n, \
                     b, mask, mode, k0, k1, step, perm);
  switch (dt) {
    case FE_F64: FE_RNG(double) break;
    case FE_F32: FE_RNG(float) break;
    case FE_BF16: FE_RNG(bf16_t) break;
  }
#undef FE_RNG
  FE_HIP(hipGetLastError());
  return FE_OK;
}

}  // namespace fe

namespace fe {
fe_status convert_launch(void* dst, fe_dtype ddt, const void* src, fe_dtype sdt, int64_t count,
                         hipStream_t s) {
  switch (sdt) {
    case FE_F64: return convert_from(dst, ddt, static_cast<const double*>(src), count, s);
    case FE_F32: return convert_from(dst, ddt, static_cast<const float*>(src), count, s);
    case FE_BF16: return convert_from(dst, ddt, static_cast<const bf16_t*>(src), count, s);
  }
  return fail(FE_EINVAL, "convert: bad dtype");
}
}  // namespace fe
