// Learned start block: a three-layer graph network over Ahat = D^-1/2 A D^-1/2
// (not part of the paper; see fe.h).  Forward, loss gradient, backward and
// Adam run here; aggregation uses the pattern SpMM.  The forward transforms
// run on BF16 MFMA (v_mfma_f32_16x16x32_bf16: BF16 copies of the FP32 master
// weights, FP32 accumulation); the backward contractions (input and weight
// gradients, long sums with cancellation) run on FP32 MFMA.
//
// MFMA 16x16x32 bf16 lane layout (measured on gfx950): A[i][k] is element
// k % 8 of lane i + 16 * (k / 8); B[k][j] is element k % 8 of lane
// j + 16 * (k / 8); D[i][j] is register i % 4 of lane j + 16 * (i / 4).
#include <cmath>
#include <cstring>
#include <vector>

#include "dev_common.h"
#include "fe_internal.h"

namespace fe {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int HID = 64, IN0 = 16, NOUT = 8, NZ = 15, NLAYER = 3;

struct Offsets {
  int W[NLAYER], U[NLAYER], b[NLAYER], P, total;
};
Offsets offsets() {
  Offsets o;
  int at = 0, din = IN0;
  for (int l = 0; l < NLAYER; ++l) {
    o.W[l] = at;
    at += din * HID;
    o.U[l] = at;
    at += din * HID;
    o.b[l] = at;
    at += HID;
    din = HID;
  }
  o.P = at;
  at += HID * NOUT;
  o.total = at;
  return o;
}

__device__ __forceinline__ bf16x8 pack_bf16(const float* x) {
  u16x8 u;
#pragma unroll
  for (int e = 0; e < 8; ++e) u[e] = (uint16_t)f32_to_bf16(x[e]);
  return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ elementwise
__global__ void features_kernel(const int64_t* __restrict__ row_ptr, const float* __restrict__ z,
                                const int32_t* __restrict__ perm, int64_t n,
                                float* __restrict__ H0, float* __restrict__ Hs0,
                                float* __restrict__ dinv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t deg = row_ptr[r + 1] - row_ptr[r];
  const int64_t o = perm ? (int64_t)perm[r] : r;
  const float di = deg > 0 ? (float)(1.0 / sqrt((double)deg)) : 0.0f;
  dinv[r] = di;
  float h = (float)log1p((double)deg);
  H0[r * IN0] = h;
  Hs0[r * IN0] = di * h;
  for (int c = 0; c < NZ; ++c) {
    h = z[o * NZ + c];
    H0[r * IN0 + 1 + c] = h;
    Hs0[r * IN0 + 1 + c] = di * h;
  }
}

// dHprev = dHp + dinv * Q (rows of width d)
__global__ void combine_kernel(float* __restrict__ out, const float* __restrict__ dHp,
                               const float* __restrict__ Q, const float* __restrict__ dinv,
                               int64_t n, int d) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  out[e] = dHp[e] + dinv[e / d] * Q[e];
}

// X = H3 P (row r of the internal order is written to row perm[r] of Xout too)
// X = H3 P (internal order, kept for the backward pass) and/or Xout in the
// original vertex order with wout columns: column c of Xout sums the outputs
// j = c (mod wout) in ascending j (wout = 8: the outputs themselves).
__global__ void out_fwd_kernel(const float* __restrict__ H3, const float* __restrict__ P,
                               int64_t n, float* __restrict__ X, const int32_t* __restrict__ perm,
                               float* __restrict__ Xout, int32_t wout) {
  __shared__ float Ps[HID * NOUT];
  for (int i = threadIdx.x; i < HID * NOUT; i += blockDim.x) Ps[i] = P[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  float acc[NOUT];
#pragma unroll
  for (int j = 0; j < NOUT; ++j) acc[j] = 0.f;
  for (int k = 0; k < HID; ++k) {
    const float h = H3[r * HID + k];
#pragma unroll
    for (int j = 0; j < NOUT; ++j) acc[j] = fmaf(h, Ps[k * NOUT + j], acc[j]);
  }
  const int64_t o = perm ? (int64_t)perm[r] : r;
  if (X) {
#pragma unroll
    for (int j = 0; j < NOUT; ++j) X[r * NOUT + j] = acc[j];
  }
  if (Xout) {
    for (int c = 0; c < wout; ++c) {
      float sum = acc[c];
      for (int j = c + wout; j < NOUT; j += wout) sum += acc[j];
      Xout[o * wout + c] = sum;
    }
  }
}

// dH3 = dX P^T
__global__ void out_bwd_kernel(const float* __restrict__ dX, const float* __restrict__ P,
                               int64_t n, float* __restrict__ dH3) {
  __shared__ float Ps[HID * NOUT];
  for (int i = threadIdx.x; i < HID * NOUT; i += blockDim.x) Ps[i] = P[i];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * HID) return;
  const int64_t r = e / HID;
  const int k = (int)(e % HID);
  float acc = 0.f;
#pragma unroll
  for (int j = 0; j < NOUT; ++j) acc = fmaf(dX[r * NOUT + j], Ps[k * NOUT + j], acc);
  dH3[e] = acc;
}

// ------------------------------------------------------ MFMA row GEMMs
// Forward layer: H = relu([dinv*T, Hprev] [W; U] + b), Hs = dinv * H.
// A workgroup handles 64-row tiles (wavefront w: rows 16w..16w+15) and all 64
// output columns (four 16x16 accumulator tiles); [W; U] is staged in LDS as
// BF16, transposed (output column major) with a padded row stride.
template <int DIN>
__global__ __launch_bounds__(256) void layer_fwd_kernel(const float* __restrict__ T,
                                                        const float* __restrict__ Hp,
                                                        const float* __restrict__ dinv,
                                                        const float* __restrict__ W,
                                                        const float* __restrict__ U,
                                                        const float* __restrict__ bias, int64_t n,
                                                        float* __restrict__ H,
                                                        float* __restrict__ Hs) {
  constexpr int K = 2 * DIN, KS = K + 8;
  __shared__ __align__(16) uint16_t Bs[HID * KS];
  __shared__ float bs[HID];
  for (int e = threadIdx.x; e < K * HID; e += blockDim.x) {
    const int k = e / HID, j = e % HID;  // [W; U][k][j]
    const float w = k < DIN ? W[k * HID + j] : U[(k - DIN) * HID + j];
    Bs[j * KS + k] = (uint16_t)f32_to_bf16(w);
  }
  for (int j = threadIdx.x; j < HID; j += blockDim.x) bs[j] = bias[j];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kg = lane >> 4;
  for (int64_t tile = blockIdx.x; tile * 64 < n; tile += gridDim.x) {
    // At 64 input features the compiler would hoist every LDS weight read out
    // of the row-tile loop (100-174 VGPRs); a compiler barrier keeps them inside.
    if constexpr (DIN > 16) asm volatile("" ::: "memory");
    const int64_t r0 = tile * 64 + wave * 16;
    const int64_t row = r0 + i;
    const int64_t rc = row < n ? row : n - 1;
    const float di = dinv[rc];
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < K / 32; ++ks) {
      const int k0 = ks * 32 + kg * 8;
      float x[8];
      const float* src = k0 < DIN ? T + rc * DIN + k0 : Hp + rc * DIN + (k0 - DIN);
      const float4 p0 = *reinterpret_cast<const float4*>(src);
      const float4 p1 = *reinterpret_cast<const float4*>(src + 4);
      x[0] = p0.x; x[1] = p0.y; x[2] = p0.z; x[3] = p0.w;
      x[4] = p1.x; x[5] = p1.y; x[6] = p1.z; x[7] = p1.w;
      const float sc = (row < n) ? (k0 < DIN ? di : 1.0f) : 0.0f;
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] *= sc;
      const bf16x8 a = pack_bf16(x);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bs + (16 * t + i) * KS + k0);
        acc[t] = mfma_bf16(a, b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = r0 + 4 * kg + r;
        const int col = 16 * t + i;
        if (orow < n) {
          const float h = fmaxf(acc[t][r] + bs[col], 0.0f);
          H[orow * HID + col] = h;
          Hs[orow * HID + col] = dinv[orow] * h;
        }
      }
  }
}

// Forward layer in FP32 (FP32 MFMA 16x16x4), for the FP32 compute mode.  The
// contraction index k = (K / 4) * kk + ks is mapped so that lane (i, kk)
// reads K / 4 contiguous inputs of its row (each range lies in one source).
template <int DIN>
__global__ __launch_bounds__(256) void layer_fwd_f32_kernel(const float* __restrict__ T,
                                                            const float* __restrict__ Hp,
                                                            const float* __restrict__ dinv,
                                                            const float* __restrict__ W,
                                                            const float* __restrict__ U,
                                                            const float* __restrict__ bias,
                                                            int64_t n, float* __restrict__ H,
                                                            float* __restrict__ Hs) {
  constexpr int K = 2 * DIN, KQ = K / 4, KS = K + 1;
  __shared__ float Bs[HID * KS];
  __shared__ float bs[HID];
  for (int e = threadIdx.x; e < K * HID; e += blockDim.x) {
    const int k = e / HID, j = e % HID;
    Bs[j * KS + k] = k < DIN ? W[k * HID + j] : U[(k - DIN) * HID + j];
  }
  for (int j = threadIdx.x; j < HID; j += blockDim.x) bs[j] = bias[j];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kk = lane >> 4;
  const int k0 = KQ * kk;
  for (int64_t tile = blockIdx.x; tile * 64 < n; tile += gridDim.x) {
    // At 64 input features the compiler would hoist every LDS weight read out
    // of the row-tile loop (100-174 VGPRs); a compiler barrier keeps them inside.
    if constexpr (DIN > 16) asm volatile("" ::: "memory");
    const int64_t r0 = tile * 64 + wave * 16;
    const int64_t row = r0 + i;
    const int64_t rc = row < n ? row : n - 1;
    const float sc = (row < n) ? (k0 < DIN ? dinv[rc] : 1.0f) : 0.0f;
    const float* src = k0 < DIN ? T + rc * DIN + k0 : Hp + rc * DIN + (k0 - DIN);
    float x[KQ];
#pragma unroll
    for (int q = 0; q < KQ; q += 4) {
      const float4 p = *reinterpret_cast<const float4*>(src + q);
      x[q] = p.x * sc;
      x[q + 1] = p.y * sc;
      x[q + 2] = p.z * sc;
      x[q + 3] = p.w * sc;
    }
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KQ; ++ks)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ks], Bs[(16 * t + i) * KS + k0 + ks],
                                                      acc[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = r0 + 4 * kk + r;
        const int col = 16 * t + i;
        if (orow < n) {
          const float h = fmaxf(acc[t][r] + bs[col], 0.0f);
          H[orow * HID + col] = h;
          Hs[orow * HID + col] = dinv[orow] * h;
        }
      }
  }
}

// Backward through a layer's inputs: with dZ = dH * (H > 0),
//   G1 = dinv * (dZ W^T)   (the input of the aggregation transpose)
//   dHp = dZ U^T
// on FP32 MFMA (16x16x4).  The contraction index k = 16 * kk + ks of step ks
// is mapped so that lane (i, kk) reads 16 contiguous dZ values of its row;
// B = [W; U] (row j' is an output column here) is staged in LDS as FP32.
template <int DIN>
__global__ __launch_bounds__(256) void layer_bwd_kernel(const float* __restrict__ dH,
                                                        const float* __restrict__ H,
                                                        const float* __restrict__ dinv,
                                                        const float* __restrict__ W,
                                                        const float* __restrict__ U, int64_t n,
                                                        float* __restrict__ G1,
                                                        float* __restrict__ dHp) {
  constexpr int N = 2 * DIN, NT = N / 16, KS = HID + 1;
  __shared__ float Bs[N * KS];
  for (int e = threadIdx.x; e < N * HID; e += blockDim.x) {
    const int jp = e / HID, k = e % HID;
    Bs[jp * KS + k] = jp < DIN ? W[jp * HID + k] : U[(jp - DIN) * HID + k];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kk = lane >> 4;
  for (int64_t tile = blockIdx.x; tile * 64 < n; tile += gridDim.x) {
    // At 64 input features the compiler would hoist every LDS weight read out
    // of the row-tile loop (100-174 VGPRs); a compiler barrier keeps them inside.
    if constexpr (DIN > 16) asm volatile("" ::: "memory");
    const int64_t r0 = tile * 64 + wave * 16;
    const int64_t row = r0 + i;
    const int64_t rc = row < n ? row : n - 1;
    const bool ok = row < n;
    float x[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 g = *reinterpret_cast<const float4*>(dH + rc * HID + 16 * kk + 4 * q);
      const float4 h = *reinterpret_cast<const float4*>(H + rc * HID + 16 * kk + 4 * q);
      x[4 * q + 0] = (ok && h.x > 0.f) ? g.x : 0.f;
      x[4 * q + 1] = (ok && h.y > 0.f) ? g.y : 0.f;
      x[4 * q + 2] = (ok && h.z > 0.f) ? g.z : 0.f;
      x[4 * q + 3] = (ok && h.w > 0.f) ? g.w : 0.f;
    }
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[ks], Bs[(16 * t + i) * KS + 16 * kk + ks],
                                                      acc[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = r0 + 4 * kk + r;
        const int col = 16 * t + i;
        if (orow < n) {
          if (col < DIN)
            G1[orow * DIN + col] = dinv[orow] * acc[t][r];
          else
            dHp[orow * DIN + (col - DIN)] = acc[t][r];
        }
      }
  }
}

// Weight gradients of a layer: C = F^T dZ with F = [dinv*T, Hprev, 1]
// (2*DIN + 1 features; the column of ones yields the bias gradient) and
// dZ = dH * (H > 0), summed over a fixed row interval per workgroup.  This is
// a long sum with cancellation, so it runs on FP32 MFMA
// (v_mfma_f32_16x16x4f32: A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// D[i][j] in register i % 4 of lane j + 16 (i / 4), measured on gfx950).
// Each 32-row step is read with 16-byte loads and staged in LDS transposed
// (feature / column major, odd row stride, so every operand read is a
// conflict-free 4-byte read).  Several workgroups per CU keep loads in
// flight while others compute.
template <int DIN>
__global__ __launch_bounds__(256) void wgrad_kernel(const float* __restrict__ T,
                                                    const float* __restrict__ Hp,
                                                    const float* __restrict__ dinv,
                                                    const float* __restrict__ dH,
                                                    const float* __restrict__ H, int64_t n,
                                                    int64_t rows_per_wg,
                                                    float* __restrict__ partials) {
  constexpr int NF = 2 * DIN + 1, MT = (NF + 15) / 16, NFP = MT * 16;
  constexpr int RS = 32 + 1;
  constexpr int D4 = DIN / 4, H4 = HID / 4;
  __shared__ float Fs[NFP * RS];
  __shared__ float Zs[HID * RS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, kk = lane >> 4;
  constexpr int TPW = (MT * 4 + 3) / 4;  // accumulator tiles per wavefront
  f32x4 acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  // constant feature rows: the ones column and the zero padding (rows past
  // the interval have dZ = 0, so their ones contribute nothing)
  for (int e = threadIdx.x; e < (NFP - 2 * DIN) * 32; e += blockDim.x) {
    const int f = 2 * DIN + e / 32, rr = e % 32;
    Fs[f * RS + rr] = f == 2 * DIN ? 1.0f : 0.0f;
  }
  const int64_t rb = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t re = min(n, rb + rows_per_wg);
  for (int64_t r0 = rb; r0 < re; r0 += 32) {
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * D4; e += blockDim.x) {
      const int rr = e / D4, f4 = e % D4;
      const int64_t row = r0 + rr;
      float4 t = make_float4(0.f, 0.f, 0.f, 0.f), h = t;
      if (row < re) {
        const float dv = dinv[row];
        t = *reinterpret_cast<const float4*>(T + row * DIN + 4 * f4);
        h = *reinterpret_cast<const float4*>(Hp + row * DIN + 4 * f4);
        t.x = dv * t.x;
        t.y = dv * t.y;
        t.z = dv * t.z;
        t.w = dv * t.w;
      }
      float* ft = Fs + (4 * f4) * RS + rr;
      ft[0] = t.x;
      ft[RS] = t.y;
      ft[2 * RS] = t.z;
      ft[3 * RS] = t.w;
      float* fh = Fs + (DIN + 4 * f4) * RS + rr;
      fh[0] = h.x;
      fh[RS] = h.y;
      fh[2 * RS] = h.z;
      fh[3 * RS] = h.w;
    }
    for (int e = threadIdx.x; e < 32 * H4; e += blockDim.x) {
      const int rr = e / H4, c4 = e % H4;
      const int64_t row = r0 + rr;
      float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row < re) {
        const float4 g = *reinterpret_cast<const float4*>(dH + row * HID + 4 * c4);
        const float4 a = *reinterpret_cast<const float4*>(H + row * HID + 4 * c4);
        z.x = a.x > 0.f ? g.x : 0.f;
        z.y = a.y > 0.f ? g.y : 0.f;
        z.z = a.z > 0.f ? g.z : 0.f;
        z.w = a.w > 0.f ? g.w : 0.f;
      }
      float* zz = Zs + (4 * c4) * RS + rr;
      zz[0] = z.x;
      zz[RS] = z.y;
      zz[2 * RS] = z.z;
      zz[3 * RS] = z.w;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int tile = wave * TPW + q;
      if (tile < MT * 4) {
        const int mt = tile / 4, nt = tile % 4;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          const float a = Fs[(16 * mt + i) * RS + 4 * ks + kk];
          const float b = Zs[(16 * nt + i) * RS + 4 * ks + kk];
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
        }
      }
    }
  }
  float* out = partials + (int64_t)blockIdx.x * NF * HID;
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int tile = wave * TPW + q;
    if (tile < MT * 4) {
      const int mt = tile / 4, nt = tile % 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = 16 * mt + 4 * kk + r, c = 16 * nt + i;
        if (f < NF) out[f * HID + c] = acc[q][r];
      }
    }
  }
}

// dP = H3^T dX over a fixed row interval per workgroup.  Lane k owns feature
// k and all NOUT columns; wavefront w takes rows rb + w, rb + w + 4, ... with
// four rows in flight, and the four wavefront sums are added in LDS in a
// fixed order.
__global__ __launch_bounds__(256) void pgrad_kernel(const float* __restrict__ H3,
                                                    const float* __restrict__ dX, int64_t n,
                                                    int64_t rows_per_wg,
                                                    float* __restrict__ partials) {
  static_assert(NOUT == 8, "two float4 per output row");
  __shared__ float red[4][HID * NOUT];
  const int k = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t re = min(n, rb + rows_per_wg);
  float a[NOUT];
#pragma unroll
  for (int j = 0; j < NOUT; ++j) a[j] = 0.f;
  int64_t r = rb + w;
  for (; r + 12 < re; r += 16) {
    float h[4];
    float4 x0[4], x1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t rr = r + 4 * u;
      h[u] = H3[rr * HID + k];
      x0[u] = *reinterpret_cast<const float4*>(dX + rr * NOUT);
      x1[u] = *reinterpret_cast<const float4*>(dX + rr * NOUT + 4);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[0] = fmaf(h[u], x0[u].x, a[0]);
      a[1] = fmaf(h[u], x0[u].y, a[1]);
      a[2] = fmaf(h[u], x0[u].z, a[2]);
      a[3] = fmaf(h[u], x0[u].w, a[3]);
      a[4] = fmaf(h[u], x1[u].x, a[4]);
      a[5] = fmaf(h[u], x1[u].y, a[5]);
      a[6] = fmaf(h[u], x1[u].z, a[6]);
      a[7] = fmaf(h[u], x1[u].w, a[7]);
    }
  }
  for (; r < re; r += 4) {
    const float h = H3[r * HID + k];
#pragma unroll
    for (int j = 0; j < NOUT; ++j) a[j] = fmaf(h, dX[r * NOUT + j], a[j]);
  }
#pragma unroll
  for (int j = 0; j < NOUT; ++j) red[w][k * NOUT + j] = a[j];
  __syncthreads();
  for (int e = threadIdx.x; e < HID * NOUT; e += blockDim.x)
    partials[(int64_t)blockIdx.x * HID * NOUT + e] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
}

// Fixed-order sum of per-workgroup partials in two stages:
// stage[g][e] = sum of partials[x][e] over the sets x of group g (kSetGroup
// consecutive sets), then out[e] = sum over g of stage[g][e], both in FP64.
constexpr int kSetGroup = 32;

__global__ void sum_sets_stage_kernel(const float* __restrict__ partials, int nsets, int len,
                                      double* __restrict__ stage) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const int g = blockIdx.y;
  const int x1 = min(nsets, (g + 1) * kSetGroup);
  double s = 0.0;
  for (int x = g * kSetGroup; x < x1; ++x) s += partials[(int64_t)x * len + e];
  stage[(int64_t)g * len + e] = s;
}

__global__ void sum_stage_kernel(const double* __restrict__ stage, int ngroups, int len,
                                 float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int g = 0; g < ngroups; ++g) s += stage[(int64_t)g * len + e];
  out[e] = (float)s;
}

// scatter a layer's [C rows: W (DIN), U (DIN), b (1)] into the flat gradient
__global__ void place_grads_kernel(const float* __restrict__ C, int din, float* __restrict__ gW,
                                   float* __restrict__ gU, float* __restrict__ gb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (2 * din + 1) * HID) return;
  const int f = e / HID, c = e % HID;
  if (f < din) gW[f * HID + c] = C[e];
  else if (f < 2 * din) gU[(f - din) * HID + c] = C[e];
  else gb[c] = C[e];
}

// scale = min(1, clip / ||g||_2) over all parameters; one workgroup, fixed
// summation order (strided FP64 partial sums, then a tree in LDS).
__global__ __launch_bounds__(1024) void clip_scale_kernel(const float* __restrict__ g, int count,
                                                          float clip, float* __restrict__ scale) {
  __shared__ double red[1024];
  double sum = 0.0;
  for (int e = threadIdx.x; e < count; e += 1024) sum += (double)g[e] * (double)g[e];
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 512; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double norm = sqrt(red[0]);
    scale[0] = norm > clip ? (float)(clip / norm) : 1.0f;
  }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int count, float lr,
                            float c1, float c2, const float* __restrict__ scale) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const float gi = scale ? g[e] * scale[0] : g[e];
  const float mi = 0.9f * m[e] + 0.1f * gi;
  const float vi = 0.999f * v[e] + 0.001f * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// Workgroups (partial-sum sets) of the row reductions: at least 256 rows
// each, at most 1024 sets (four workgroups per CU at the largest sizes).
int wgrad_sets(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256));
}

}  // namespace

// ------------------------------------------------------------------ host
struct Gnn {
  int device = 0;
  bool f32 = false;  // forward transforms on FP32 MFMA instead of BF16
  float* params = nullptr;  // FP32 masters
  float* grads = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* gscale = nullptr;  // gradient clipping factor (device scalar)
  int step = 0;
  bool have_grads = false;
  // Workspace arena: grown (at the start of a call) to the largest total a
  // previous call needed, so steady-state calls allocate nothing.
  char* arena = nullptr;
  size_t arena_cap = 0, arena_need = 0;
};

namespace {

// Workspace of one call: bump allocation from the handle's arena; a request
// that does not fit (first calls, or a larger graph) falls back to a
// stream-ordered allocation and raises the arena's target size, which the
// next call allocates before it starts.
struct Ws {
  hipStream_t s;
  Gnn* g;
  size_t off = 0, need = 0;
  std::vector<void*> ptrs;
  Ws(hipStream_t st, Gnn* gn) : s(st), g(gn) {}
  fe_status grow() {
    if (g->arena_need <= g->arena_cap) return FE_OK;
    if (g->arena) {
      FE_HIP(hipStreamSynchronize(s));
      FE_HIP(hipFree(g->arena));
      g->arena = nullptr;
      g->arena_cap = 0;
    }
    if (hipMalloc((void**)&g->arena, g->arena_need) != hipSuccess) {
      g->arena = nullptr;
      return fail(FE_ENOMEM, "gnn workspace: %zu bytes", g->arena_need);
    }
    g->arena_cap = g->arena_need;
    return FE_OK;
  }
  // Overflow allocations go back to the stream-ordered pool, and the pool is
  // trimmed here: otherwise the pool would hand the memory back to the device
  // at some later synchronisation of the caller's, inside unrelated work.
  ~Ws() {
    for (void* p : ptrs) (void)hipFreeAsync(p, s);
    if (!ptrs.empty()) {
      int dev = 0;
      hipMemPool_t pool = nullptr;
      if (hipStreamSynchronize(s) == hipSuccess && hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess)
        (void)hipMemPoolTrimTo(pool, 0);
    }
    g->arena_need = std::max(g->arena_need, need);
  }
  template <class T>
  fe_status get(T** p, size_t count) {
    const size_t bytes = (std::max<size_t>(count, 64) * sizeof(T) + 255) & ~(size_t)255;
    need += bytes;
    if (off + bytes <= g->arena_cap) {
      *p = reinterpret_cast<T*>(g->arena + off);
      off += bytes;
      return FE_OK;
    }
    hipError_t e = hipMallocAsync((void**)p, bytes, s);
    if (e != hipSuccess) return fail(FE_ENOMEM, "gnn workspace: %s", hipGetErrorString(e));
    ptrs.push_back(*p);
    return FE_OK;
  }
};

inline dim3 grid1(int64_t count, int block = 256) {
  return dim3((uint32_t)((count + block - 1) / block));
}

struct Fwd {
  float *dinv, *H[4], *Hs[4], *T[3], *X, *Xorig;
};

// Forward pass.  With keep, every activation stays for the backward pass;
// without it (inference) four n x 64 buffers are reused across layers: layer l
// reads H[l] and T[l] and writes H[l+1] and Hs[l+1], so H alternates between
// two buffers, while Hs and T each need one (Hs[l] is consumed by the product
// that makes T[l] before layer l writes Hs[l+1]; T[l] is read only by layer l).
fe_status forward(const Gnn& g, const Csr& A, const float* z, Ws& ws, Fwd& f, float* Xorig,
                  bool keep = true, int32_t wout = NOUT) {
  const int64_t n = A.n;
  const Offsets o = offsets();
  hipStream_t s = ws.s;
  const int32_t* perm = A.relabeled ? A.d_perm : nullptr;
  FE_TRY(ws.get(&f.dinv, n));
  if (keep) {
    FE_TRY(ws.get(&f.H[0], n * IN0));
    FE_TRY(ws.get(&f.Hs[0], n * IN0));
    for (int l = 1; l <= NLAYER; ++l) {
      FE_TRY(ws.get(&f.H[l], n * HID));
      FE_TRY(ws.get(&f.Hs[l], n * HID));
    }
    FE_TRY(ws.get(&f.T[0], n * IN0));
    FE_TRY(ws.get(&f.T[1], n * HID));
    FE_TRY(ws.get(&f.T[2], n * HID));
  } else {
    float *ha, *hb, *hs, *t;
    FE_TRY(ws.get(&ha, n * HID));
    FE_TRY(ws.get(&hb, n * HID));
    FE_TRY(ws.get(&hs, n * HID));
    FE_TRY(ws.get(&t, n * HID));
    for (int l = 0; l <= NLAYER; ++l) {
      f.H[l] = (l % 2) ? hb : ha;
      f.Hs[l] = hs;
    }
    for (int l = 0; l < NLAYER; ++l) f.T[l] = t;
  }
  FE_TRY(ws.get(&f.X, n * NOUT));
  hipLaunchKernelGGL(features_kernel, grid1(n), dim3(256), 0, s, A.d_row_ptr, z, perm, n, f.H[0],
                     f.Hs[0], f.dinv);
  FE_HIP(hipGetLastError());
  const uint32_t tiles = (uint32_t)std::min<int64_t>((n + 63) / 64, 2048);
  for (int l = 0; l < NLAYER; ++l) {
    const int din = l == 0 ? IN0 : HID;
    FE_TRY(spmm_launch(A, f.Hs[l], f.T[l], din, FE_F32, s));  // T = A (dinv * H)
#define FE_FWD(KERNEL, D)                                                                  \
  hipLaunchKernelGGL((KERNEL<D>), dim3(tiles), dim3(256), 0, s, f.T[l], f.H[l], f.dinv,     \
                     g.params + o.W[l], g.params + o.U[l], g.params + o.b[l], n, f.H[l + 1], \
                     f.Hs[l + 1]);
    if (l == 0) {
      if (g.f32) FE_FWD(layer_fwd_f32_kernel, IN0) else FE_FWD(layer_fwd_kernel, IN0)
    } else {
      if (g.f32) FE_FWD(layer_fwd_f32_kernel, HID) else FE_FWD(layer_fwd_kernel, HID)
    }
#undef FE_FWD
    FE_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(out_fwd_kernel, grid1(n), dim3(256), 0, s, f.H[NLAYER], g.params + o.P, n,
                     keep ? f.X : nullptr, perm, Xorig, wout);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

}  // namespace
}  // namespace fe

struct fe_gnn : fe::Gnn {};

using namespace fe;

extern "C" {

int64_t fe_gnn_param_count(void) { return offsets().total; }

fe_status fe_gnn_create(uint64_t seed, fe_dtype compute, fe_gnn** out) {
  if (!out) return fail(FE_EINVAL, "fe_gnn_create: out is NULL");
  if (compute != FE_BF16 && compute != FE_F32)
    return fail(FE_EINVAL, "fe_gnn_create: compute must be FE_BF16 or FE_F32");
  const Offsets o = offsets();
  std::vector<float> h((size_t)o.total, 0.0f);
  // Glorot-uniform weights from Philox4x32-10 draws (counter: index, tensor id)
  auto philox = [](uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1) {
    uint32_t c2 = 0x474e4e31u, c3 = 0;
    for (int r = 0; r < 10; ++r) {
      if (r) {
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
      }
      const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
      const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
      const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
      c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    return c0;
  };
  auto fill = [&](int off, int rows, int cols, uint32_t tid) {
    const double lim = std::sqrt(6.0 / (rows + cols));
    for (int e = 0; e < rows * cols; ++e) {
      const uint32_t w = philox((uint32_t)e, tid, (uint32_t)seed, (uint32_t)(seed >> 32));
      h[(size_t)off + e] = (float)((2.0 * (w * (1.0 / 4294967296.0)) - 1.0) * lim);
    }
  };
  int din = IN0;
  for (int l = 0; l < NLAYER; ++l) {
    fill(o.W[l], din, HID, 10 * l + 1);
    fill(o.U[l], din, HID, 10 * l + 2);
    din = HID;
  }
  fill(o.P, HID, NOUT, 99);
  fe_gnn* g = new fe_gnn();
  g->f32 = compute == FE_F32;
  if (hipGetDevice(&g->device) != hipSuccess) {
    delete g;
    return fail(FE_EDEVICE, "fe_gnn_create: no device");
  }
  const size_t bytes = sizeof(float) * o.total;
  if (hipMalloc((void**)&g->params, bytes) != hipSuccess ||
      hipMalloc((void**)&g->grads, bytes) != hipSuccess ||
      hipMalloc((void**)&g->m, bytes) != hipSuccess || hipMalloc((void**)&g->v, bytes) != hipSuccess ||
      hipMalloc((void**)&g->gscale, sizeof(float)) != hipSuccess) {
    fe_gnn_free(g);
    return fail(FE_ENOMEM, "fe_gnn_create: hipMalloc failed");
  }
  if (hipMemcpy(g->params, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(g->grads, 0, bytes) != hipSuccess || hipMemset(g->m, 0, bytes) != hipSuccess ||
      hipMemset(g->v, 0, bytes) != hipSuccess) {
    fe_gnn_free(g);
    return fail(FE_EDEVICE, "fe_gnn_create: upload failed");
  }
  *out = g;
  return FE_OK;
}

void fe_gnn_free(fe_gnn* g) {
  if (!g) return;
  (void)hipFree(g->params);
  (void)hipFree(g->grads);
  (void)hipFree(g->gscale);
  (void)hipFree(g->arena);
  (void)hipFree(g->m);
  (void)hipFree(g->v);
  delete g;
}

fe_status fe_gnn_get_params(const fe_gnn* g, float* host) {
  if (!g || !host) return fail(FE_EINVAL, "fe_gnn_get_params: NULL argument");
  FE_HIP(hipMemcpy(host, g->params, sizeof(float) * offsets().total, hipMemcpyDeviceToHost));
  return FE_OK;
}

fe_status fe_gnn_set_params(fe_gnn* g, const float* host) {
  if (!g || !host) return fail(FE_EINVAL, "fe_gnn_set_params: NULL argument");
  const size_t bytes = sizeof(float) * offsets().total;
  FE_HIP(hipMemcpy(g->params, host, bytes, hipMemcpyHostToDevice));
  FE_HIP(hipMemset(g->grads, 0, bytes));
  FE_HIP(hipMemset(g->m, 0, bytes));
  FE_HIP(hipMemset(g->v, 0, bytes));
  g->step = 0;
  g->have_grads = false;
  return FE_OK;
}

fe_status fe_gnn_forward(fe_gnn* g, const fe_csr* A, const float* z, float* X, int32_t block,
                         void* stream) {
  if (!g || !A || !z || !X) return fail(FE_EINVAL, "fe_gnn_forward: NULL argument");
  if (block != 1 && block != 2 && block != 4 && block != 8)
    return fail(FE_EINVAL, "fe_gnn_forward: block must be 1, 2, 4 or 8");
  hipStream_t s = (hipStream_t)stream;
  {
    Ws ws(s, g);
    FE_TRY(ws.grow());
    Fwd f;
    FE_TRY(forward(*g, *A, z, ws, f, X, false, block));
  }
  FE_HIP(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status fe_gnn_backward(fe_gnn* g, const fe_csr* A, const float* z, const float* V, double* loss,
                          float* grads_host, void* stream) {
  if (!g || !A || !z || !V) return fail(FE_EINVAL, "fe_gnn_backward: NULL argument");
  const int64_t n = A->n;
  if (n < NOUT) return fail(FE_EINVAL, "fe_gnn_backward: n < 8");
  hipStream_t s = (hipStream_t)stream;
  const Offsets o = offsets();
  const int32_t* perm = A->relabeled ? A->d_perm : nullptr;
  {
    Ws ws(s, g);
    FE_TRY(ws.grow());
    Fwd f;
    FE_TRY(forward(*g, *A, z, ws, f, nullptr));
    // targets in the internal order
    float *Vi, *dX;
    FE_TRY(ws.get(&Vi, n * NOUT));
    FE_TRY(ws.get(&dX, n * NOUT));
    if (perm)
      FE_TRY(permute_rows(Vi, V, perm, n, NOUT, FE_F32, false, s));
    else
      FE_HIP(hipMemcpyAsync(Vi, V, sizeof(float) * n * NOUT, hipMemcpyDeviceToDevice, s));
    // M = V^T X, G = X^T X (FP64)
    double *dMG, *part, *dC;
    FE_TRY(ws.get(&dMG, 2 * NOUT * NOUT));
    FE_TRY(ws.get(&part, gram_partials_doubles(n, NOUT, NOUT)));
    FE_TRY(ws.get(&dC, 2 * NOUT * NOUT));
    FE_TRY(gram_launch(Vi, 1, n * NOUT, f.X, n, NOUT, FE_F32, 1.0, dMG, part, s));
    FE_TRY(gram_launch(f.X, 1, n * NOUT, f.X, n, NOUT, FE_F32, 1.0, dMG + NOUT * NOUT, part, s));
    double MG[2 * NOUT * NOUT];
    FE_HIP(hipMemcpyAsync(MG, dMG, sizeof MG, hipMemcpyDeviceToHost, s));
    FE_HIP(hipStreamSynchronize(s));
    // host: Gi = G^-1 (Gauss-Jordan with partial pivoting), loss and dL/dX factors
    const double* M = MG;
    double G[NOUT][2 * NOUT];
    for (int i = 0; i < NOUT; ++i)
      for (int j = 0; j < 2 * NOUT; ++j) G[i][j] = j < NOUT ? MG[NOUT * NOUT + i * NOUT + j] : (j - NOUT == i);
    for (int c = 0; c < NOUT; ++c) {
      int piv = c;
      for (int r = c + 1; r < NOUT; ++r)
        if (std::fabs(G[r][c]) > std::fabs(G[piv][c])) piv = r;
      if (!(std::fabs(G[piv][c]) > 0.0)) return fail(FE_EBREAKDOWN, "fe_gnn_backward: X^T X is singular");
      if (piv != c)
        for (int j = 0; j < 2 * NOUT; ++j) std::swap(G[c][j], G[piv][j]);
      const double d = G[c][c];
      for (int j = 0; j < 2 * NOUT; ++j) G[c][j] /= d;
      for (int r = 0; r < NOUT; ++r)
        if (r != c) {
          const double f0 = G[r][c];
          for (int j = 0; j < 2 * NOUT; ++j) G[r][j] -= f0 * G[c][j];
        }
    }
    double Gi[NOUT][NOUT], MGi[NOUT][NOUT], MtM[NOUT][NOUT], C1[NOUT * NOUT], C2[NOUT * NOUT];
    for (int i = 0; i < NOUT; ++i)
      for (int j = 0; j < NOUT; ++j) Gi[i][j] = G[i][NOUT + j];
    for (int i = 0; i < NOUT; ++i)
      for (int j = 0; j < NOUT; ++j) {
        double a = 0.0, b = 0.0;
        for (int t = 0; t < NOUT; ++t) {
          a += M[i * NOUT + t] * Gi[t][j];
          b += M[t * NOUT + i] * M[t * NOUT + j];
        }
        MGi[i][j] = a;
        MtM[i][j] = b;
      }
    double tr = 0.0;
    for (int i = 0; i < NOUT; ++i)
      for (int t = 0; t < NOUT; ++t) tr += MGi[i][t] * M[i * NOUT + t];
    if (loss) *loss = 1.0 - tr / NOUT;
    const double sc = 2.0 / NOUT;
    for (int i = 0; i < NOUT; ++i)
      for (int j = 0; j < NOUT; ++j) {
        C1[i * NOUT + j] = -sc * MGi[i][j];  // dX = V C1 + X C2
        double a = 0.0;
        for (int t = 0; t < NOUT; ++t)
          for (int u = 0; u < NOUT; ++u) a += Gi[i][t] * MtM[t][u] * Gi[u][j];
        C2[i * NOUT + j] = sc * a;
      }
    double hc[2 * NOUT * NOUT];
    std::memcpy(hc, C1, sizeof C1);
    std::memcpy(hc + NOUT * NOUT, C2, sizeof C2);
    FE_HIP(hipMemcpyAsync(dC, hc, sizeof hc, hipMemcpyHostToDevice, s));
    FE_TRY(update_launch(dX, n, NOUT, Vi, 1, n * NOUT, dC, 1.0, 0.0, FE_F32, s));
    FE_TRY(update_launch(dX, n, NOUT, f.X, 1, n * NOUT, dC + NOUT * NOUT, 1.0, 1.0, FE_F32, s));
    // output layer
    float *dH, *dHn, *G1, *Q, *dHp, *pP, *wpart, *C;
    FE_TRY(ws.get(&dH, n * HID));
    FE_TRY(ws.get(&dHn, n * HID));
    FE_TRY(ws.get(&G1, n * HID));
    FE_TRY(ws.get(&Q, n * HID));
    FE_TRY(ws.get(&dHp, n * HID));
    const int ps = wgrad_sets(n);
    const int64_t prow = (n + ps - 1) / ps;
    const int ngroups = (ps + kSetGroup - 1) / kSetGroup;
    double* stage;
    FE_TRY(ws.get(&stage, (size_t)ngroups * (2 * HID + 1) * HID));
    auto sum_sets = [&](const float* part, int len, float* out) {
      hipLaunchKernelGGL(sum_sets_stage_kernel, dim3((len + 255) / 256, ngroups), dim3(256), 0, s,
                         part, ps, len, stage);
      hipLaunchKernelGGL(sum_stage_kernel, grid1(len), dim3(256), 0, s, stage, ngroups, len, out);
    };
    FE_TRY(ws.get(&pP, (size_t)ps * HID * NOUT));
    hipLaunchKernelGGL(pgrad_kernel, dim3(ps), dim3(256), 0, s, f.H[NLAYER], dX, n, prow, pP);
    sum_sets(pP, HID * NOUT, g->grads + o.P);
    hipLaunchKernelGGL(out_bwd_kernel, grid1(n * HID), dim3(256), 0, s, dX, g->params + o.P, n, dH);
    FE_HIP(hipGetLastError());
    FE_TRY(ws.get(&wpart, (size_t)ps * (2 * HID + 1) * HID));
    FE_TRY(ws.get(&C, (2 * HID + 1) * HID));
    int64_t wrow = (n + ps - 1) / ps;
    wrow = (wrow + 31) / 32 * 32;
    const uint32_t tiles = (uint32_t)std::min<int64_t>((n + 63) / 64, 2048);
    for (int l = NLAYER - 1; l >= 0; --l) {
      const int din = l == 0 ? IN0 : HID;
      const int nf = 2 * din + 1;
      if (l == 0)
        hipLaunchKernelGGL((wgrad_kernel<IN0>), dim3(ps), dim3(256), 0, s, f.T[0], f.H[0], f.dinv,
                           dH, f.H[1], n, wrow, wpart);
      else
        hipLaunchKernelGGL((wgrad_kernel<HID>), dim3(ps), dim3(256), 0, s, f.T[l], f.H[l], f.dinv,
                           dH, f.H[l + 1], n, wrow, wpart);
      sum_sets(wpart, nf * HID, C);
      hipLaunchKernelGGL(place_grads_kernel, grid1(nf * HID), dim3(256), 0, s, C, din,
                         g->grads + o.W[l], g->grads + o.U[l], g->grads + o.b[l]);
      FE_HIP(hipGetLastError());
      if (l == 0) break;
      hipLaunchKernelGGL((layer_bwd_kernel<HID>), dim3(tiles), dim3(256), 0, s, dH, f.H[l + 1],
                         f.dinv, g->params + o.W[l], g->params + o.U[l], n, G1, dHp);
      FE_HIP(hipGetLastError());
      FE_TRY(spmm_launch(*A, G1, Q, HID, FE_F32, s));  // Ahat is symmetric
      hipLaunchKernelGGL(combine_kernel, grid1(n * HID), dim3(256), 0, s, dHn, dHp, Q, f.dinv, n,
                         HID);
      FE_HIP(hipGetLastError());
      std::swap(dH, dHn);
    }
    if (grads_host)
      FE_HIP(hipMemcpyAsync(grads_host, g->grads, sizeof(float) * o.total, hipMemcpyDeviceToHost, s));
  }
  FE_HIP(hipStreamSynchronize(s));
  g->have_grads = true;
  return FE_OK;
}

fe_status fe_gnn_adam(fe_gnn* g, double lr, double clip, void* stream) {
  if (!g) return fail(FE_EINVAL, "fe_gnn_adam: NULL");
  if (!(clip >= 0.0)) return fail(FE_EINVAL, "fe_gnn_adam: clip must be >= 0");
  if (!g->have_grads) return fail(FE_EINVAL, "fe_gnn_adam: no gradients (call fe_gnn_backward)");
  hipStream_t s = (hipStream_t)stream;
  g->step += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, g->step));
  const float c2 = (float)(1.0 - std::pow(0.999, g->step));
  const int count = offsets().total;
  if (clip > 0.0) {
    hipLaunchKernelGGL(clip_scale_kernel, dim3(1), dim3(1024), 0, s, g->grads, count, (float)clip,
                       g->gscale);
    FE_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(adam_kernel, grid1(count), dim3(256), 0, s, g->params, g->grads, g->m, g->v,
                     count, (float)lr, c1, c2, clip > 0.0 ? g->gscale : nullptr);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

}  // extern "C"
