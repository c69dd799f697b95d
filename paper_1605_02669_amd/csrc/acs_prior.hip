// Learned edge prior on gfx950: a 4 -> 64 -> 64 -> 1 MLP (ReLU hidden
// layers) whose sigmoid output scores candidate edges; the scores replace
// eta^beta of the candidates in the transition rule (Eq. 1, Eq. 2 of the
// paper's Sec. 3).  This is an addition of this project, not the paper's.
//
// The matrix products run on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16,
// fp32 accumulation).  Lane layout of that instruction (checked on the GPU):
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + 0..7]
//   B (32 x 16): lane l holds B[8 (l / 16) + 0..7][l % 16]
//   D (16 x 16): lane l holds D[4 (l / 16) + 0..3][l % 16]
// Weights are kept in fp32 (master copy, optimizer state) and rounded to
// bf16 when staged into LDS; activations are rounded to bf16 between layers.
//
// Parameter vector (floats): W1[4][64] | b1[64] | W2[64][64] | b2[64] |
// W3[64] | b3[1] (row-major, x @ W + b).
#include <hip/hip_runtime.h>

#include "acs_internal.hpp"

namespace acs {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int H = 64;
constexpr int OW1 = 0, OB1 = 256, OW2 = 320, OB2 = 4416, OW3 = 4480, OB3 = 4544;

// Weights staged in LDS, transposed so that a B operand is one 16-byte read:
//   w1t[n][k]  (64 x 32, k >= 4 zero)        B[k][n] = W1[k][n]
//   w2t[n][k]  (64 x 64)                      B[k][n] = W2[k][n]
//   w2r[n][k]  (64 x 64) = W2 row-major       B[k][n] = W2[n][k]   (W2^T)
//   w3t[n][k]  (16 x 64, n >= 1 zero)         B[k][n] = W3[k]
struct alignas(16) Stage {
  __bf16 w1t[H * 32];
  __bf16 w2t[H * H];
  __bf16 w2r[H * H];
  __bf16 w3t[16 * H];
  float b1[H], b2[H], w3[H], b3;
};

__device__ __forceinline__ void stage_weights(Stage &S, const float *P) {
  for (int e = threadIdx.x; e < H * 32; e += blockDim.x) {
    const int n = e / 32, k = e % 32;
    S.w1t[e] = (__bf16)(k < 4 ? P[OW1 + k * H + n] : 0.f);
  }
  for (int e = threadIdx.x; e < H * H; e += blockDim.x) {
    const int n = e / H, k = e % H;
    S.w2t[e] = (__bf16)P[OW2 + k * H + n];
    S.w2r[e] = (__bf16)P[OW2 + e];
  }
  for (int e = threadIdx.x; e < 16 * H; e += blockDim.x) {
    const int n = e / H, k = e % H;
    S.w3t[e] = (__bf16)(n == 0 ? P[OW3 + k] : 0.f);
  }
  for (int e = threadIdx.x; e < H; e += blockDim.x) {
    S.b1[e] = P[OB1 + e];
    S.b2[e] = P[OB2 + e];
    S.w3[e] = P[OW3 + e];
  }
  if (threadIdx.x == 0) S.b3 = P[OB3];
  __syncthreads();
}

// The lanes of a wave exchange activations through LDS.  LDS operations of
// one wave complete in issue order; this keeps the compiler from moving LDS
// accesses across the exchange points.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ bf16x8 ld8(const __bf16 *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Forward pass of 16 rows held by one wave.  x: this lane's row features
// (valid in lane group 0).  Writes relu activations (bf16, row-major
// [16][64]) to h1 and h2 and returns the logit of rows 4g + v in z[v] for
// lanes with l % 16 == 0.
__device__ __forceinline__ f32x4 forward16(const Stage &S, float4 x, int lane, __bf16 *h1,
                                           __bf16 *h2) {
  const int g = lane >> 4, c16 = lane & 15;
  bf16x8 a1;
  for (int q = 0; q < 8; ++q) a1[q] = (__bf16)0.f;
  if (g == 0) {
    a1[0] = (__bf16)x.x;
    a1[1] = (__bf16)x.y;
    a1[2] = (__bf16)x.z;
    a1[3] = (__bf16)x.w;
  }
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const f32x4 d = mfma(a1, ld8(S.w1t + (16 * t + c16) * 32 + 8 * g), zero);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      h1[(4 * g + v) * H + 16 * t + c16] = (__bf16)fmaxf(d[v] + S.b1[16 * t + c16], 0.f);
  }
  wave_sync();
  const bf16x8 a2a = ld8(h1 + c16 * H + 8 * g), a2b = ld8(h1 + c16 * H + 32 + 8 * g);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 d = mfma(a2a, ld8(S.w2t + (16 * t + c16) * H + 8 * g), zero);
    d = mfma(a2b, ld8(S.w2t + (16 * t + c16) * H + 32 + 8 * g), d);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      h2[(4 * g + v) * H + 16 * t + c16] = (__bf16)fmaxf(d[v] + S.b2[16 * t + c16], 0.f);
  }
  wave_sync();
  const bf16x8 a3a = ld8(h2 + c16 * H + 8 * g), a3b = ld8(h2 + c16 * H + 32 + 8 * g);
  f32x4 d = mfma(a3a, ld8(S.w3t + c16 * H + 8 * g), zero);
  d = mfma(a3b, ld8(S.w3t + c16 * H + 32 + 8 * g), d);
  for (int v = 0; v < 4; ++v) d[v] += S.b3;
  return d;
}

// Inference with everything in registers.  The products are computed
// transposed, Z^T = W^T H^T, so a layer's output tile (lane l: hidden units
// 16t + 4(l/16) + v of row l % 16) is already the next layer's B operand
// once the K index of that layer is permuted to match: within K block b,
// B-row 8g + q is hidden unit 32b + 4g + q for q < 4 and 32b + 16 + 4g +
// (q - 4) for q >= 4.  The weight tiles (A operands) are built in that
// order once per wave.  The 64 -> 1 layer runs on the vector unit, on the
// bf16-rounded activations, and the four lane groups' partial sums meet by
// lane swaps.  No LDS.
struct RegNet {
  bf16x8 w1[4];     // A of layer 1, tile t: W1^T[16t + l%16][8(l/16) + q] (k < 4)
  bf16x8 w2[4][2];  // A of layer 2, tile t, K block b (permuted K)
  float b1[4][4], b2[4][4], w3[4][4];  // [t][v] at hidden 16t + 4(l/16) + v
  float b3;
};

__device__ __forceinline__ int perm_k(int b, int g, int q) {
  return q < 4 ? 32 * b + 4 * g + q : 32 * b + 16 + 4 * g + (q - 4);
}

__device__ __forceinline__ void load_regnet(RegNet &R, const float *P, int lane) {
  const int g = lane >> 4, c16 = lane & 15;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = 8 * g + q;
      R.w1[t][q] = (__bf16)(k < 4 ? P[OW1 + k * H + 16 * t + c16] : 0.f);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        R.w2[t][b][q] = (__bf16)P[OW2 + perm_k(b, g, q) * H + 16 * t + c16];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int h = 16 * t + 4 * g + v;
      R.b1[t][v] = P[OB1 + h];
      R.b2[t][v] = P[OB2 + h];
      R.w3[t][v] = (float)(__bf16)P[OW3 + h];
    }
  }
  R.b3 = P[OB3];
}

// Logit of row l % 16 of a 16-row tile (every lane of the row's four lane
// groups gets it); x: the row's features.
__device__ __forceinline__ float forward16r(const RegNet &R, float4 x, int lane) {
  const int g = lane >> 4;
  bf16x8 bx;
#pragma unroll
  for (int q = 0; q < 8; ++q) bx[q] = (__bf16)0.f;
  if (g == 0) {
    bx[0] = (__bf16)x.x;
    bx[1] = (__bf16)x.y;
    bx[2] = (__bf16)x.z;
    bx[3] = (__bf16)x.w;
  }
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  bf16x8 h1[2];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const f32x4 d = mfma(R.w1[t], bx, zero);
#pragma unroll
    for (int v = 0; v < 4; ++v) h1[t >> 1][4 * (t & 1) + v] = (__bf16)fmaxf(d[v] + R.b1[t][v], 0.f);
  }
  float part = 0.f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 d = mfma(R.w2[t][0], h1[0], zero);
    d = mfma(R.w2[t][1], h1[1], d);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      part = fmaf((float)(__bf16)fmaxf(d[v] + R.b2[t][v], 0.f), R.w3[t][v], part);
  }
  // sum over the four lane groups: each swap pairs a lane with its partner,
  // and the two results of a swap add up to own + partner
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(part), __float_as_uint(part),
                                                  false, false);
  part = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(part), __float_as_uint(part),
                                                  false, false);
  part = __uint_as_float(b[0]) + __uint_as_float(b[1]);
  return part + R.b3;
}

__device__ __forceinline__ float4 load_x(const float *X, int row, int rows) {
  return row < rows ? *reinterpret_cast<const float4 *>(X + (size_t)row * 4)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Logits of `rows` feature rows: four waves per block share the staged
// weights; each wave takes 16-row tiles with its own activation buffers.
constexpr int kFwdWaves = 4;

__global__ __launch_bounds__(64 * kFwdWaves) void k_prior_forward(const float *P, const float *X,
                                                                  int rows, float *Z) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  RegNet R;
  load_regnet(R, P, lane);
  // two independent 16-row tiles per pass (their matrix and vector work
  // interleave), the next pass's features loaded ahead
  const int stride = gridDim.x * kFwdWaves * 32;
  int r0 = (blockIdx.x * kFwdWaves + wv) * 32;
  float4 xa = load_x(X, r0 + (lane & 15), rows), xb = load_x(X, r0 + 16 + (lane & 15), rows);
  for (; r0 < rows; r0 += stride) {
    const float4 na = load_x(X, r0 + stride + (lane & 15), rows);
    const float4 nb = load_x(X, r0 + stride + 16 + (lane & 15), rows);
    const float za = forward16r(R, xa, lane), zb = forward16r(R, xb, lane);
    const int row = r0 + (lane & 15);
    if (lane < 16 && row < rows) Z[row] = za;
    if (lane < 16 && row + 16 < rows) Z[row + 16] = zb;
    xa = na;
    xb = nb;
  }
}

// Gradient of the mean binary cross-entropy (with logits) over all `rows`
// rows, accumulated into G; loss sum into *L.  kGradWaves waves per block
// share the staged weights; each wave takes 32-row tiles (two 16-row
// forward passes) with its own buffers.  dW2 = H1^T dH2 and dH1 = dH2 W2^T
// run on the matrix cores; the 4-wide first layer, the 64 -> 1 last layer
// and the biases on the vector units.  The waves' partial sums meet in LDS,
// and each block adds its total to G once per parameter.
constexpr int kGradWaves = 3;

struct GradWave {
  __bf16 h1[32 * H];    // row-major activations of the first hidden layer
  __bf16 h2[32 * H];    // second hidden layer, then (in place) dL/dH2
  __bf16 h1t[H * 32];   // H1^T [feature][row]: each feature's four 8-row
  __bf16 dh2t[H * 32];  //   chunks in the order chunk ^ ((feature >> 2) & 3), so
                        //   the transposing stores of 64 features spread over
                        //   more banks while a chunk stays one 16-byte load
  float zs[32], dzs[32], xs[32 * 4];
};

__global__ __launch_bounds__(64 * kGradWaves) void k_prior_grad(const float *P, const float *X,
                                                                const float *Y, int rows,
                                                                float *G, float *L) {
  __shared__ Stage S;
  __shared__ union alignas(16) {
    GradWave w[kGradWaves];
    float red[kPriorParams + 1];  // block totals (the last entry: loss)
  } U;
  stage_weights(S, P);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  GradWave &B = U.w[wv];
  __bf16 *h1 = B.h1, *h2 = B.h2, *dh2 = B.h2, *h1t = B.h1t, *dh2t = B.dh2t;
  float *zs = B.zs, *dzs = B.dzs, *xs = B.xs;
  const float inv_rows = 1.f / (float)rows;
  f32x4 gw2[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) gw2[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  float gw1[4][4] = {};  // [nt][input] partials for feature 16 nt + c16
  float gb1[4] = {};
  float gw3 = 0.f, gb2 = 0.f, gb3 = 0.f, loss = 0.f;  // lane = feature
  const float w3f = (float)S.w3t[lane];  // W3 as the forward pass used it (bf16)

  for (int r0 = (blockIdx.x * kGradWaves + wv) * 32; r0 < rows;
       r0 += gridDim.x * kGradWaves * 32) {
    wave_sync();
    // forward of two 16-row halves; the first layer's inputs are kept as the
    // bf16 values the matrix cores multiplied (for its weight gradient)
    for (int hf = 0; hf < 2; ++hf) {
      const int row = r0 + 16 * hf + c16;
      const float4 x = load_x(X, row, rows);
      if (g == 0) {
        xs[(16 * hf + c16) * 4 + 0] = (float)(__bf16)x.x;
        xs[(16 * hf + c16) * 4 + 1] = (float)(__bf16)x.y;
        xs[(16 * hf + c16) * 4 + 2] = (float)(__bf16)x.z;
        xs[(16 * hf + c16) * 4 + 3] = (float)(__bf16)x.w;
      }
      const f32x4 z = forward16(S, x, lane, h1 + 16 * hf * H, h2 + 16 * hf * H);
      if (c16 == 0)
        for (int v = 0; v < 4; ++v) zs[16 * hf + 4 * g + v] = z[v];
    }
    wave_sync();
    // dz = (sigmoid(z) - y) / rows, loss = softplus(z) - y z (rows past the end: 0)
    if (lane < 32) {
      const int row = r0 + lane;
      float dz = 0.f;
      if (row < rows) {
        const float z = zs[lane], y = Y[row];
        dz = (1.f / (1.f + __expf(-z)) - y) * inv_rows;
        loss += fmaxf(z, 0.f) + log1pf(__expf(-fabsf(z))) - y * z;
      }
      dzs[lane] = dz;
    }
    wave_sync();
    // last layer and dH2 (lane = feature f), dH2 written over H2 in place
    {
      const int f = lane;
      // unrolled by 8 so the rows' LDS loads and stores overlap (1.17 ->
      // 0.73 ms per 4.2 M rows; full unrolling is no faster than none)
#pragma unroll 8
      for (int r = 0; r < 32; ++r) {
        const float hv = (float)h2[r * H + f];
        const float dz = dzs[r];
        gw3 += hv * dz;
        const float dh = hv > 0.f ? dz * w3f : 0.f;
        gb2 += dh;
        dh2[r * H + f] = (__bf16)dh;
        const int rs = r ^ (8 * ((f >> 2) & 3));  // 16-byte chunks swizzled by feature
        dh2t[f * 32 + rs] = (__bf16)dh;
        h1t[f * 32 + rs] = h1[r * H + f];
      }
      if (lane < 32) gb3 += dzs[lane];
    }
    wave_sync();
    // dW2 += H1^T dH2: M = 64 features (4 tiles), N = 64 (4 tiles), K = 32 rows
    for (int mt = 0; mt < 4; ++mt) {
      const int fa = 16 * mt + c16;
      const bf16x8 a = ld8(h1t + fa * 32 + 8 * (g ^ ((fa >> 2) & 3)));
      for (int nt = 0; nt < 4; ++nt)
        gw2[mt][nt] = mfma(a, ld8(dh2t + (16 * nt + c16) * 32 + 8 * (g ^ (((16 * nt + c16) >> 2) & 3))),
                           gw2[mt][nt]);
    }
    // dH1 = dH2 W2^T, masked by H1 > 0: M = 32 rows (2 tiles), N = 64, K = 64
    for (int mh = 0; mh < 2; ++mh) {
      const bf16x8 aa = ld8(dh2 + (16 * mh + c16) * H + 8 * g);
      const bf16x8 ab = ld8(dh2 + (16 * mh + c16) * H + 32 + 8 * g);
      for (int nt = 0; nt < 4; ++nt) {
        const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
        f32x4 d = mfma(aa, ld8(S.w2r + (16 * nt + c16) * H + 8 * g), zero);
        d = mfma(ab, ld8(S.w2r + (16 * nt + c16) * H + 32 + 8 * g), d);
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * mh + 4 * g + v;
          const int f = 16 * nt + c16;
          const float dh1 = (float)h1[r * H + f] > 0.f ? d[v] : 0.f;
          gb1[nt] += dh1;
          for (int c = 0; c < 4; ++c) gw1[nt][c] += xs[r * 4 + c] * dh1;
        }
      }
    }
  }
  // the waves' partial sums meet in LDS (over the now unused wave buffers)
  __syncthreads();
  for (int e = threadIdx.x; e <= kPriorParams; e += blockDim.x) U.red[e] = 0.f;
  __syncthreads();
  for (int mt = 0; mt < 4; ++mt)
    for (int nt = 0; nt < 4; ++nt)
      for (int v = 0; v < 4; ++v)
        atomicAdd(&U.red[OW2 + (16 * mt + 4 * g + v) * H + 16 * nt + c16], gw2[mt][nt][v]);
  for (int nt = 0; nt < 4; ++nt) {
    atomicAdd(&U.red[OB1 + 16 * nt + c16], gb1[nt]);
    for (int c = 0; c < 4; ++c) atomicAdd(&U.red[OW1 + c * H + 16 * nt + c16], gw1[nt][c]);
  }
  atomicAdd(&U.red[OW3 + lane], gw3);
  atomicAdd(&U.red[OB2 + lane], gb2);
  if (lane < 32) {
    atomicAdd(&U.red[OB3], gb3);
    atomicAdd(&U.red[kPriorParams], loss);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kPriorParams; e += blockDim.x) atomicAdd(&G[e], U.red[e]);
  if (threadIdx.x == 0) atomicAdd(L, U.red[kPriorParams]);
}

// Adam (Kingma and Ba, 2015) on the fp32 parameters; clears the gradient.
__global__ __launch_bounds__(256) void k_prior_adam(float *P, float *G, float *M, float *V,
                                                    int t, float lr, float b1, float b2,
                                                    float eps) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kPriorParams) return;
  const float g = G[e];
  const float m = b1 * M[e] + (1.f - b1) * g;
  const float v = b2 * V[e] + (1.f - b2) * g * g;
  M[e] = m;
  V[e] = v;
  const float mh = m / (1.f - powf(b1, (float)t));
  const float vh = v / (1.f - powf(b2, (float)t));
  P[e] -= lr * mh / (sqrtf(vh) + eps);
  G[e] = 0.f;
}

// Features of the first 16 candidates of every city (row i * 16 + r):
// (dx / s_i, dy / s_i, d_ij / s_i, r / 15), s_i = d(i, 16th neighbour).
__device__ __forceinline__ float4 edge_features(const Dev &D, int i, int r) {
  const uint4 rec = D.crec[(size_t)i * D.cl + r];
  const uint32_t s16 = D.crec[(size_t)i * D.cl + 15].y;
  const double s = s16 ? (double)s16 : 1.0;
  const int j = (int)rec.x;
  return make_float4((float)((D.xy[2 * j] - D.xy[2 * i]) / s),
                     (float)((D.xy[2 * j + 1] - D.xy[2 * i + 1]) / s), (float)(rec.y / s),
                     (float)(r / 15.0));
}

__global__ __launch_bounds__(256) void k_prior_features(Dev D, float *X) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D.n * 16) return;
  *reinterpret_cast<float4 *>(X + (size_t)e * 4) = edge_features(D, e / 16, e % 16);
}

// Scores of every candidate edge of the instance straight into the
// eta^beta word of the candidate records: max(sigmoid(z), 1e-6).
__global__ __launch_bounds__(64 * kFwdWaves) void k_prior_apply(Dev D, const float *P) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  RegNet R;
  load_regnet(R, P, lane);
  const int rows = D.n * 16;
  for (int r0 = (blockIdx.x * kFwdWaves + wv) * 16; r0 < rows;
       r0 += gridDim.x * kFwdWaves * 16) {
    const int row = r0 + (lane & 15);
    const float4 x = row < rows ? edge_features(D, row / 16, row % 16)
                                : make_float4(0.f, 0.f, 0.f, 0.f);
    const float z = forward16r(R, x, lane);
    if (lane < 16 && row < rows) {
      const float sc = fmaxf(1.f / (1.f + __expf(-z)), 1e-6f);
      const_cast<uint4 *>(D.crec)[(size_t)(row / 16) * D.cl + row % 16].z = __float_as_uint(sc);
    }
  }
}

}  // namespace

hipError_t launch_prior_forward(const float *P, const float *X, int rows, float *Z,
                                hipStream_t s) {
  const int tiles = (rows + 31) / 32;
  int blocks = (tiles + kFwdWaves - 1) / kFwdWaves;
  blocks = blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024;
  hipLaunchKernelGGL(k_prior_forward, dim3(blocks), dim3(64 * kFwdWaves), 0, s, P, X, rows, Z);
  return hipGetLastError();
}

hipError_t launch_prior_grad(const float *P, const float *X, const float *Y, int rows, float *G,
                             float *L, hipStream_t s) {
  const int tiles = (rows + 31) / 32;
  int blocks = (tiles + kGradWaves - 1) / kGradWaves;
  blocks = blocks < 512 ? (blocks > 0 ? blocks : 1) : 512;
  hipLaunchKernelGGL(k_prior_grad, dim3(blocks), dim3(64 * kGradWaves), 0, s, P, X, Y, rows, G,
                     L);
  return hipGetLastError();
}

hipError_t launch_prior_adam(float *P, float *G, float *M, float *V, int t, float lr, float b1,
                             float b2, float eps, hipStream_t s) {
  hipLaunchKernelGGL(k_prior_adam, dim3((kPriorParams + 255) / 256), dim3(256), 0, s, P, G, M, V,
                     t, lr, b1, b2, eps);
  return hipGetLastError();
}

hipError_t launch_prior_features(const Dev &d, float *X, hipStream_t s) {
  hipLaunchKernelGGL(k_prior_features, dim3((d.n * 16 + 255) / 256), dim3(256), 0, s, d, X);
  return hipGetLastError();
}

hipError_t launch_prior_apply(const Dev &d, const float *P, hipStream_t s) {
  const int tiles = d.n;  // 16 rows per city
  int blocks = (tiles + kFwdWaves - 1) / kFwdWaves;
  blocks = blocks < 1024 ? blocks : 1024;
  hipLaunchKernelGGL(k_prior_apply, dim3(blocks), dim3(64 * kFwdWaves), 0, s, d, P);
  return hipGetLastError();
}

}  // namespace acs
