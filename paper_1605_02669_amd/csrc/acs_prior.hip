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
// bf16 when a wave loads its operand tiles; activations are rounded to bf16
// between layers.
//
// Parameter vector (floats): W1[4][64] | b1[64] | W2[64][64] | b2[64] |
// W3[64] | b3[1] (row-major, x @ W + b).
#include <hip/hip_runtime.h>

#include "acs_internal.hpp"

namespace acs {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2;
// an operand as four dwords: bf16 entries 2p (low half) and 2p + 1 (high
// half) share dword p
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int H = 64;
constexpr int OW1 = 0, OB1 = 256, OW2 = 320, OB2 = 4416, OW3 = 4480, OB3 = 4544;

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, u32x4 b, f32x4 c) {
  return mfma(a, __builtin_bit_cast(bf16x8, b), c);
}
__device__ __forceinline__ f32x4 mfma(u32x4 a, bf16x8 b, f32x4 c) {
  return mfma(__builtin_bit_cast(bf16x8, a), b, c);
}
__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
  return mfma(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c);
}

// the K = 16 product: A lane l holds A[l % 16][4 (l / 16) + 0..3], B lane l
// holds B[4 (l / 16) + 0..3][l % 16], D as above
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short s16x4;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f32x4 mfma16(u32x2 a, u32x2 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a),
                                                   __builtin_bit_cast(s16x4, b), c, 0, 0, 0);
}

// two floats rounded to bf16 (to nearest, ties to even) in one dword, a in
// the low half; and the two halves back as floats
__device__ __forceinline__ unsigned pk2(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
__device__ __forceinline__ float lo_f(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_f(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// max(x, 0) as one integer max on the bits: a float with the sign bit set
// (negative, or -0) is a negative integer and becomes +0
__device__ __forceinline__ float relu(float x) {
  return __int_as_float(max(__float_as_int(x), 0));
}

// Inference with everything in registers.  The products are computed
// transposed, Z^T = W^T H^T, so a layer's output tile (lane l: hidden units
// 16t + 4(l/16) + v of row l % 16) is already the next layer's B operand
// once the K index of that layer is permuted to match: within K block b,
// B-row 8g + q is hidden unit 32b + 4g + q for q < 4 and 32b + 16 + 4g +
// (q - 4) for q >= 4.  The weight tiles (A operands) are built in that
// order once per wave.  The biases start the accumulators.  The 64 -> 1
// layer is one more product whose A operand repeats W3 in all 16 rows, so
// that every lane of a row receives the row's logit.  No LDS.
struct RegNet {
  bf16x8 w1[4];     // A of layer 1, tile t: W1^T[16t + l%16][8(l/16) + q] (k < 4)
  bf16x8 w2[4][2];  // A of layer 2, tile t, K block b (permuted K)
  bf16x8 w3[2];     // A of layer 3, K block b: W3[perm_k(b, l/16, q)] in every row
  f32x4 b1[4], b2[4];  // [t][v] at hidden 16t + 4(l/16) + v
  f32x4 b3;            // b3 in every entry
  __device__ __forceinline__ bf16x8 W1(int t) const { return w1[t]; }
  __device__ __forceinline__ bf16x8 W2(int t, int b) const { return w2[t][b]; }
  __device__ __forceinline__ bf16x8 W3(int b) const { return w3[b]; }
  __device__ __forceinline__ f32x4 B1(int t) const { return b1[t]; }
  __device__ __forceinline__ f32x4 B2(int t) const { return b2[t]; }
  __device__ __forceinline__ f32x4 B3() const { return b3; }
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
    }
  }
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int q = 0; q < 8; ++q) R.w3[b][q] = (__bf16)P[OW3 + perm_k(b, g, q)];
  const float b3 = P[OB3];
  R.b3 = (f32x4){b3, b3, b3, b3};
}

// Logit of row l % 16 of a 16-row tile (every lane of the row's four lane
// groups gets it); x: the row's features.  Also leaves the activations as
// the gradient needs them: h1 and h2 = H1^T and H2^T as B operands (K
// blocks 0 and 1), so entry 4(t & 1) + v of block t >> 1 is hidden unit
// 16t + 4(l/16) + v of the row.
template <class Net>
__device__ __forceinline__ float forward16r(const Net &R, float4 x, int lane, u32x4 h1[2],
                                            u32x4 h2[2]) {
  const int g = lane >> 4;
  const u32x4 bx = g == 0 ? (u32x4){pk2(x.x, x.y), pk2(x.z, x.w), 0u, 0u} : (u32x4){0u, 0u, 0u, 0u};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const f32x4 d = mfma(R.W1(t), bx, R.B1(t));
    h1[t >> 1][2 * (t & 1)] = pk2(relu(d[0]), relu(d[1]));
    h1[t >> 1][2 * (t & 1) + 1] = pk2(relu(d[2]), relu(d[3]));
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 d = mfma(R.W2(t, 0), h1[0], R.B2(t));
    d = mfma(R.W2(t, 1), h1[1], d);
    h2[t >> 1][2 * (t & 1)] = pk2(relu(d[0]), relu(d[1]));
    h2[t >> 1][2 * (t & 1) + 1] = pk2(relu(d[2]), relu(d[3]));
  }
  f32x4 z = mfma(R.W3(0), h2[0], R.B3());
  z = mfma(R.W3(1), h2[1], z);
  return z[0];
}

__device__ __forceinline__ float forward16r(const RegNet &R, float4 x, int lane) {
  u32x4 h1[2], h2[2];
  return forward16r(R, x, lane, h1, h2);
}

__device__ __forceinline__ float4 load_x(const float *X, int row, int rows) {
  return row < rows ? *reinterpret_cast<const float4 *>(X + (size_t)row * 4)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
}

// Logits of `rows` feature rows: each wave builds its weight tiles in
// registers and takes two 16-row tiles per pass.
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
// rows, accumulated into G; loss sum into *L.  Each wave takes 32-row tiles
// (two 16-row halves, one after the other) and keeps activations and
// partial sums in registers:
//   forward   as in inference, the products transposed (rows across lanes);
//   dH2       dz w3 masked by H2 > 0, lane by lane; dW3, db2, db3 as
//             lane-local sums on the vector unit;
//   turn      H1 and dH2 turned around (rows within a lane);
//   dH1       dH2 W2^T on the matrix cores, masked by H1 > 0;
//   dW2       H1^T dH2 on the matrix cores (K = 16, the half's rows);
//   dW1, db1  dH1^T [X 1] on the matrix cores, dH1 carried as a sum of two
//             bf16 values (16 significant bits) against the bf16 inputs.
// A product with a 0/1 selection matrix turns a 16 x 16 block around
// exactly: each sum has one nonzero term, a bf16 value times 1.  Afterwards
// lane l holds rows 4(l/16) + v of one hidden unit, which is the K = 16
// operand layout.  The weight tiles sit in LDS, one 16-byte entry per lane,
// and are read where they are used, so that a wave holds at most 256
// registers and two waves share a SIMD.  The lanes' and waves' partial sums
// meet in LDS at the end, and each block adds its total to G once per
// parameter.
constexpr int kGradWaves = 8;  // two per SIMD: a wave holds 256 registers

// B operand that picks hidden units 16 (2b + odd) + l % 16 out of K block b
// of a transposed tile (the inverse of perm_k).
__device__ __forceinline__ bf16x8 pick_tile(int lane, int odd) {
  const int g = lane >> 4, c16 = lane & 15;
  bf16x8 s;
#pragma unroll
  for (int q = 0; q < 8; ++q)
    s[q] = (__bf16)(g == (c16 >> 2) && q == 4 * odd + (c16 & 3) ? 1.f : 0.f);
  return s;
}

// Every lane's operand tiles in LDS, one 16-byte entry per tile and lane
// (lane l reads entry [tile][l]: no bank conflicts), read where they are
// used instead of held in registers across the loop.
enum : int {
  kTW1 = 0, kTW2 = 4, kTW3 = 12, kTB1 = 14, kTB2 = 18, kTB3 = 22, kTW2b = 23, kTPick = 31,
  kTPickX = 33, kTW3f = 34, kTiles = 38
};

struct LdsNet {
  const u32x4 (*tl)[64];
  int lane;
  __device__ __forceinline__ u32x4 at(int i) const { return tl[i][lane]; }
  __device__ __forceinline__ bf16x8 W1(int t) const {
    return __builtin_bit_cast(bf16x8, at(kTW1 + t));
  }
  __device__ __forceinline__ bf16x8 W2(int t, int b) const {
    return __builtin_bit_cast(bf16x8, at(kTW2 + 2 * t + b));
  }
  __device__ __forceinline__ bf16x8 W3(int b) const {
    return __builtin_bit_cast(bf16x8, at(kTW3 + b));
  }
  __device__ __forceinline__ f32x4 B1(int t) const {
    return __builtin_bit_cast(f32x4, at(kTB1 + t));
  }
  __device__ __forceinline__ f32x4 B2(int t) const {
    return __builtin_bit_cast(f32x4, at(kTB2 + t));
  }
  __device__ __forceinline__ f32x4 B3() const { return __builtin_bit_cast(f32x4, at(kTB3)); }
  __device__ __forceinline__ bf16x8 W2b(int t, int b) const {
    return __builtin_bit_cast(bf16x8, at(kTW2b + 2 * t + b));
  }
  __device__ __forceinline__ bf16x8 Pick(int odd) const {
    return __builtin_bit_cast(bf16x8, at(kTPick + odd));
  }
  __device__ __forceinline__ bf16x8 PickX() const {
    return __builtin_bit_cast(bf16x8, at(kTPickX));
  }
  __device__ __forceinline__ f32x4 W3f(int t) const {
    return __builtin_bit_cast(f32x4, at(kTW3f + t));
  }
};

__global__ __launch_bounds__(64 * kGradWaves) void k_prior_grad(const float *P, const float *X,
                                                                const float *Y, int rows,
                                                                float *G, float *L) {
  __shared__ union alignas(16) {
    u32x4 tl[kTiles][64];         // operand tiles
    float red[kPriorParams + 1];  // block totals (the last entry: loss)
  } U;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  {
    RegNet N;
    load_regnet(N, P, lane);
    // B of dH1 = dH2 W2^T, tile t, K block b: W2[16t + l%16][perm_k(b, g, q)]
    bf16x8 w2b[4][2];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 8; ++q)
          w2b[t][b][q] = (__bf16)P[OW2 + (16 * t + c16) * H + perm_k(b, g, q)];
    f32x4 w3f[4];  // W3 (bf16) at hidden 16t + 4g + v
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) w3f[t][v] = (float)(__bf16)P[OW3 + 16 * t + 4 * g + v];
    bf16x8 pickx;  // B operand that picks input column l % 16 (identity)
#pragma unroll
    for (int q = 0; q < 8; ++q) pickx[q] = (__bf16)(8 * g + q == c16 ? 1.f : 0.f);
    // the waves store the tiles in turn
    auto put = [&](int i, auto v) {
      if (i % kGradWaves == wv) U.tl[i][lane] = __builtin_bit_cast(u32x4, v);
    };
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      put(kTW1 + t, N.w1[t]);
      put(kTW2 + 2 * t, N.w2[t][0]);
      put(kTW2 + 2 * t + 1, N.w2[t][1]);
      put(kTB1 + t, N.b1[t]);
      put(kTB2 + t, N.b2[t]);
      put(kTW2b + 2 * t, w2b[t][0]);
      put(kTW2b + 2 * t + 1, w2b[t][1]);
      put(kTW3f + t, w3f[t]);
    }
    put(kTW3, N.w3[0]);
    put(kTW3 + 1, N.w3[1]);
    put(kTB3, N.b3);
    put(kTPick, pick_tile(lane, 0));
    put(kTPick + 1, pick_tile(lane, 1));
    put(kTPickX, pickx);
  }
  __syncthreads();
  const LdsNet R{U.tl, lane};
  const float inv_rows = 1.f / (float)rows;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 gw2[4][4];  // dW2[16mt + 4g + v][16nt + l%16]
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) gw2[a][b] = zero;
  // [dW1; db1]^T[16mt + 4g + v][c] at lane column c = l%16 (c < 4: input c;
  // c = 4: the bias)
  f32x4 gw1[4] = {zero, zero, zero, zero};
  // lane-local partial sums at hidden 16t + 4g + v over the lane's rows
  float gw3[4][4] = {}, gb2[4][4] = {};
  float gb3 = 0.f, loss = 0.f;  // lanes 0..15 only (one lane per row)

  const int stride = gridDim.x * kGradWaves * 32;
  int r0 = (blockIdx.x * kGradWaves + wv) * 32;
  float4 xn[2];
  float yn[2];
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    const int row = r0 + 16 * hf + c16;
    xn[hf] = load_x(X, row, rows);
    yn[hf] = row < rows ? Y[row] : 0.f;
  }
  for (; r0 < rows; r0 += stride) {
    // the tiles are read from LDS where they are used, every pass (a
    // compiler barrier: not hoisted out of the loop)
    __asm__ volatile("" ::: "memory");
    const float4 x[2] = {xn[0], xn[1]};
    const float y[2] = {yn[0], yn[1]};
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {  // the next tile's rows, loaded ahead
      const int row = r0 + stride + 16 * hf + c16;
      xn[hf] = load_x(X, row, rows);
      yn[hf] = row < rows ? Y[row] : 0.f;
    }
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      u32x4 h1[2], h2[2], dh2[2];
      __builtin_amdgcn_sched_barrier(0);
      const float z = forward16r(R, x[hf], lane, h1, h2);
      __builtin_amdgcn_sched_barrier(0);
      // dz = (sigmoid(z) - y) / rows, loss = softplus(z) - y z (rows past
      // the end: 0); the reciprocal and logarithm of the vector unit (about
      // 1 ulp) are ample for a training signal
      const int row = r0 + 16 * hf + c16;
      float dz = 0.f;
      if (row < rows) {
        const float e = __expf(-fabsf(z));
        const float sg = __builtin_amdgcn_rcpf(1.f + e);  // sigmoid(|z|)
        dz = ((z >= 0.f ? sg : e * sg) - y[hf]) * inv_rows;
        if (g == 0) loss += fmaxf(z, 0.f) + __logf(1.f + e) - y[hf] * z;
      }
      if (g == 0) gb3 += dz;
      // last layer and dH2^T (bf16, in H1^T's operand layout)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const f32x4 w3t = R.W3f(t);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const unsigned w = h2[t >> 1][2 * (t & 1) + p];
          float dh[2];
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            const int v = 2 * p + o;
            const float hv = o ? hi_f(w) : lo_f(w);
            gw3[t][v] = fmaf(hv, dz, gw3[t][v]);
            dh[o] = hv > 0.f ? dz * w3t[v] : 0.f;
            gb2[t][v] += dh[o];
          }
          dh2[t >> 1][2 * (t & 1) + p] = pk2(dh[0], dh[1]);
        }
      }
      // the inputs (bf16, as the first layer multiplied them) and a 1 for
      // the bias, turned around: lane l holds column l%16 of rows 4g + v
      const u32x4 xe = g == 0 ? (u32x4){pk2(x[hf].x, x[hf].y), pk2(x[hf].z, x[hf].w),
                                        pk2(1.f, 0.f), 0u}
                              : (u32x4){0u, 0u, 0u, 0u};
      const f32x4 tx = mfma(xe, R.PickX(), zero);
      const u32x2 bx = {pk2(tx[0], tx[1]), pk2(tx[2], tx[3])};
      // operands over the half's 16 rows: K position 4g + v is row 4g + v
      u32x2 ah1[4], bdh2[4], adh1[4], adh1l[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        // H1 and dH2 turned around: rows 4g + v of hidden unit 16t + l%16
        const bf16x8 pick = R.Pick(t & 1);
        const f32x4 t1 = mfma(h1[t >> 1], pick, zero);
        const f32x4 t2 = mfma(dh2[t >> 1], pick, zero);
        // dH1 at the same positions, masked by H1 > 0, as a bf16 pair
        // hi + lo
        f32x4 d = mfma(dh2[0], R.W2b(t, 0), zero);
        d = mfma(dh2[1], R.W2b(t, 1), d);
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          ah1[t][p] = pk2(t1[2 * p], t1[2 * p + 1]);
          bdh2[t][p] = pk2(t2[2 * p], t2[2 * p + 1]);
          const float d0 = t1[2 * p] > 0.f ? d[2 * p] : 0.f;
          const float d1 = t1[2 * p + 1] > 0.f ? d[2 * p + 1] : 0.f;
          const unsigned hi = pk2(d0, d1);
          adh1[t][p] = hi;
          adh1l[t][p] = pk2(d0 - lo_f(hi), d1 - hi_f(hi));
        }
      }
      // dW2 += H1^T dH2 and [dW1; db1]^T += dH1^T [X 1] over the half
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) gw2[mt][nt] = mfma16(ah1[mt], bdh2[nt], gw2[mt][nt]);
        gw1[mt] = mfma16(adh1[mt], bx, gw1[mt]);
        gw1[mt] = mfma16(adh1l[mt], bx, gw1[mt]);
      }
    }
  }
  __syncthreads();  // every wave is done with the tiles
  for (int e = threadIdx.x; e <= kPriorParams; e += blockDim.x) U.red[e] = 0.f;
  __syncthreads();
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int h = 16 * mt + 4 * g + v;
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        atomicAdd(&U.red[OW2 + h * H + 16 * nt + c16], gw2[mt][nt][v]);
      if (c16 < 4) atomicAdd(&U.red[OW1 + c16 * H + h], gw1[mt][v]);
      if (c16 == 4) atomicAdd(&U.red[OB1 + h], gw1[mt][v]);
      atomicAdd(&U.red[OW3 + h], gw3[mt][v]);
      atomicAdd(&U.red[OB2 + h], gb2[mt][v]);
    }
  if (lane < 16) {
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
  // one block per CU (fewer block totals to add into G)
  int blocks = (tiles + kGradWaves - 1) / kGradWaves;
  blocks = blocks < 256 ? (blocks > 0 ? blocks : 1) : 256;
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
