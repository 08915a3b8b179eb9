// Contact-force surrogate: a 12 -> 128 -> 128 -> 2 tanh MLP on pair
// features, with hand-written forward, backward and Adam kernels for gfx950.
// Products run on the matrix cores (v_mfma_f32_16x16x16_bf16, and for the
// K = 128 layers of inference v_mfma_f32_16x16x32_bf16: BF16 operands, FP32
// accumulation); biases, activations, losses and optimiser state are
// FP32.
//
// Fragment layouts of the 16x16x16 BF16 MFMA (wave64): for A (16 x 16,
// row-major, K contiguous) lane l holds row l % 16, columns 4 (l / 16) .. +3;
// for B given as B^T (16 x 16, K contiguous) lane l holds column l % 16,
// k = 4 (l / 16) .. +3; the 16 x 16 FP32 result gives lane l the column
// l % 16, rows 4 (l / 16) .. +3. Every product below is written as
// C = A B^T with both operands staged row-major with K contiguous.
//
// One workgroup of 4 wavefronts handles 64 rows (pairs), 16 per wavefront.
// The weight gradient of a workgroup is a partial over its 64 rows; partials
// are summed over workgroups in a fixed order by a second kernel, so
// training is deterministic (no float atomics).

#include <hip/hip_runtime.h>

#include "vmas_internal.h"

namespace vmas {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NI = 12, NIP = 16, NH = 128, NO = 2, NOP = 16;
constexpr int ROWS = 64;        // rows per workgroup
constexpr int LDH = NH + 8;     // padded row stride (bf16) of 128-wide operands
constexpr int LDI = NIP + 8;    // padded row stride of 16-wide operands
constexpr int LDR = ROWS + 8;   // padded row stride of transposed (K = rows) operands

// BF16 from FP32, round to nearest even (the hardware conversion).
__device__ __forceinline__ unsigned short to_bf16(float f) {
  return __builtin_bit_cast(unsigned short, (__bf16)f);
}

// tanh x = (e^{2x} - 1) / (e^{2x} + 1) with the hardware exp2 and reciprocal
// (each about 1 ulp): absolute error of a few 1e-7, far below the BF16
// rounding the activations go through; |x| is clamped to 9, where tanh is 1
// in FP32. Inference uses it; training (activations kept for the backward
// pass) uses tanhf, so a training run does not depend on this shortcut.
__device__ __forceinline__ float tanh_fast(float x) {
  const float c = fminf(fmaxf(x, -9.0f), 9.0f);
  const float e = __builtin_amdgcn_exp2f(c * 2.8853900817779268f);  // 2 / ln 2
  return (e - 1.0f) * __builtin_amdgcn_rcpf(e + 1.0f);
}
template <bool TRAIN> __device__ __forceinline__ float act(float x) {
  if constexpr (TRAIN) return tanhf(x);
  else return tanh_fast(x);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// 4 consecutive bf16 of a row-major operand as one MFMA fragment.
// (row * ld + k0 is a multiple of 4 elements: one aligned 8-byte LDS read)
__device__ __forceinline__ s4 frag(const unsigned short* base, int ld, int row, int k0) {
  return *reinterpret_cast<const s4*>(base + row * ld + k0);
}

// acc += A[r0 .. r0+15][0 .. K) * Bt[c0 .. c0+15][0 .. K)^T
__device__ __forceinline__ f4 mma(f4 acc, const unsigned short* A, int lda, int r0,
                                  const unsigned short* Bt, int ldb, int c0, int K, int lane) {
  const int r = lane & 15, kq = (lane >> 4) * 4;
  for (int k = 0; k < K; k += 16) {
    const s4 a = frag(A, lda, r0 + r, k + kq);
    const s4 b = frag(Bt, ldb, c0 + r, k + kq);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

struct MlpArgs {
  const unsigned short* W1;  // [NH][NIP]  bf16, columns >= NI are zero
  const unsigned short* W2;  // [NH][NH]
  const unsigned short* W3;  // [NOP][NH], rows >= NO are zero
  const float* b1;           // [NH]
  const float* b2;           // [NH]
  const float* b3;           // [NO]
};

// Stages the three weight matrices of one network into LDS, 8 BF16 values
// (16 bytes) per load and store; every row length (16, 128) and LDS row
// stride (LDI, LDH) is a multiple of 8 elements, so each access is aligned.
__device__ void stage_weights(const MlpArgs& m, unsigned short* w1, unsigned short* w2,
                              unsigned short* w3) {
  using u4 = uint4;
  const u4* g1 = reinterpret_cast<const u4*>(m.W1);
  const u4* g2 = reinterpret_cast<const u4*>(m.W2);
  const u4* g3 = reinterpret_cast<const u4*>(m.W3);
  for (int i = threadIdx.x; i < NH * NIP / 8; i += blockDim.x) {
    const int row = i / (NIP / 8), col = (i % (NIP / 8)) * 8;
    *reinterpret_cast<u4*>(w1 + row * LDI + col) = g1[i];
  }
#pragma unroll 4
  for (int i = threadIdx.x; i < NH * NH / 8; i += blockDim.x) {
    const int row = i / (NH / 8), col = (i % (NH / 8)) * 8;
    *reinterpret_cast<u4*>(w2 + row * LDH + col) = g2[i];
  }
  for (int i = threadIdx.x; i < NOP * NH / 8; i += blockDim.x) {
    const int row = i / (NH / 8), col = (i % (NH / 8)) * 8;
    *reinterpret_cast<u4*>(w3 + row * LDH + col) = g3[i];
  }
}

// The weights of the inference kernel: W1 as stage_weights stores it; in W2
// and W3 every 32-column block is permuted so that the K values lane group
// g (= lane / 16) supplies to a 16x16x32 product -- columns 4g .. 4g+3 and
// 16+4g .. 16+4g+3 of the block -- are the 8 consecutive columns 8g .. 8g+7
// (one 16-byte LDS read). Each 4-column group moves as a whole (8 bytes).
__device__ __forceinline__ int k32_col(int c) {
  const int r = c & 31;
  return (c & ~31) + 8 * ((r & 15) >> 2) + 4 * (r >> 4) + (r & 3);
}
__device__ void stage_weights_k32(const MlpArgs& m, unsigned short* w1, unsigned short* w2,
                                  unsigned short* w3) {
  using u2 = uint2;
  using u4 = uint4;
  const u4* g1 = reinterpret_cast<const u4*>(m.W1);
  const u4* g2 = reinterpret_cast<const u4*>(m.W2);
  const u4* g3 = reinterpret_cast<const u4*>(m.W3);
  for (int i = threadIdx.x; i < NH * NIP / 8; i += blockDim.x) {
    const int row = i / (NIP / 8), col = (i % (NIP / 8)) * 8;
    *reinterpret_cast<u4*>(w1 + row * LDI + col) = g1[i];
  }
  auto put = [](unsigned short* w, int row, int col, u4 v) {
    *reinterpret_cast<u2*>(w + row * LDH + k32_col(col)) = make_uint2(v.x, v.y);
    *reinterpret_cast<u2*>(w + row * LDH + k32_col(col + 4)) = make_uint2(v.z, v.w);
  };
#pragma unroll 4
  for (int i = threadIdx.x; i < NH * NH / 8; i += blockDim.x)
    put(w2, i / (NH / 8), (i % (NH / 8)) * 8, g2[i]);
  for (int i = threadIdx.x; i < NOP * NH / 8; i += blockDim.x)
    put(w3, i / (NH / 8), (i % (NH / 8)) * 8, g3[i]);
}

typedef __bf16 b8 __attribute__((ext_vector_type(8)));
// 8 consecutive bf16 of a staged (permuted) row as one 16x16x32 fragment
__device__ __forceinline__ b8 frag8(const unsigned short* base, int ld, int row, int k0) {
  return *reinterpret_cast<const b8*>(base + row * ld + k0);
}
// the B fragment of one 32-wide K step from two 16-unit result fragments
__device__ __forceinline__ b8 cat8(s4 lo, s4 hi) {
  return __builtin_bit_cast(b8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

// Forward pass over 64-row tiles. X [n][12] -> Y [n][2]; TRAIN: also the FP32
// activations H1, H2 [n][128] for the backward pass. With n_dev set, the row
// count is min(n, *n_dev), read on the device.
template <bool TRAIN>
__global__ void __launch_bounds__(256) k_mlp_forward(MlpArgs m, const float* __restrict__ X,
                                                     int64_t n, const int32_t* __restrict__ n_dev,
                                                     float* __restrict__ Y,
                                                     float* __restrict__ H1, float* __restrict__ H2) {
  if (n_dev) n = min(n, (int64_t)max(*n_dev, 0));
  const int64_t tiles = (n + ROWS - 1) / ROWS;
  if ((int64_t)blockIdx.x >= tiles) return;  // uniform per workgroup, before any barrier
  __shared__ __attribute__((aligned(16))) unsigned short w1[NH * LDI], w2[NH * LDH], w3[NOP * LDH];
  __shared__ __attribute__((aligned(16))) unsigned short xs[ROWS * LDI], h1s[ROWS * LDH];
  __shared__ float bias[NH + NH + NO];
  stage_weights(m, w1, w2, w3);
  for (int i = threadIdx.x; i < NH; i += blockDim.x) {
    bias[i] = m.b1[i];
    bias[NH + i] = m.b2[i];
  }
  if (threadIdx.x < NO) bias[2 * NH + threadIdx.x] = m.b3[threadIdx.x];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = wv * 16, col = lane & 15, rq = (lane >> 4) * 4;
  // the workgroup walks row tiles; the weights stay staged in LDS
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t row0 = tile * ROWS;
    __syncthreads();  // the previous tile's activations are consumed
    for (int i = threadIdx.x; i < ROWS * NIP; i += blockDim.x) {
      const int r = i / NIP, c = i % NIP;
      const int64_t g = row0 + r;
      xs[r * LDI + c] = to_bf16((c < NI && g < n) ? X[g * NI + c] : 0.0f);
    }
    __syncthreads();
    // layer 1: h1 = tanh(x W1^T + b1)
    for (int j = 0; j < NH / 16; ++j) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = mma(acc, xs, LDI, r0, w1, LDI, j * 16, NIP, lane);
      const int c = j * 16 + col;
      for (int i = 0; i < 4; ++i) {
        const float h = act<TRAIN>(acc[i] + bias[c]);
        const int r = r0 + rq + i;
        h1s[r * LDH + c] = to_bf16(h);
        if (H1 && row0 + r < n) H1[(row0 + r) * NH + c] = h;
      }
    }
    __syncthreads();
    // layer 2: h2 = tanh(h1 W2^T + b2); all 8 column tiles are accumulated in
    // registers first, then h2 overwrites this wavefront's own rows of h1
    // (the wavefront's 16 rows of h1 are read from LDS once, as 8 fragments)
    f4 acc2[NH / 16];
    {
      s4 a[NH / 16];
#pragma unroll
      for (int kk = 0; kk < NH / 16; ++kk) a[kk] = frag(h1s, LDH, r0 + col, kk * 16 + rq);
#pragma unroll
      for (int j = 0; j < NH / 16; ++j) {
        acc2[j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < NH / 16; ++kk)
          acc2[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
              a[kk], frag(w2, LDH, j * 16 + col, kk * 16 + rq), acc2[j], 0, 0, 0);
      }
    }
    for (int j = 0; j < NH / 16; ++j) {
      const int c = j * 16 + col;
      for (int i = 0; i < 4; ++i) {
        const float h = act<TRAIN>(acc2[j][i] + bias[NH + c]);
        const int r = r0 + rq + i;
        h1s[r * LDH + c] = to_bf16(h);
        if (H2 && row0 + r < n) H2[(row0 + r) * NH + c] = h;
      }
    }
    __syncthreads();
    // layer 3: y = h2 W3^T + b3
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mma(acc, h1s, LDH, r0, w3, LDH, 0, NH, lane);
    if (col < NO) {
      for (int i = 0; i < 4; ++i) {
        const int64_t g = row0 + r0 + rq + i;
        if (g < n) Y[g * NO + col] = acc[i] + bias[2 * NH + col];
      }
    }
  }
}

// Inference forward pass with the layers transposed: a wavefront computes
// H1^T = tanh(W1 X^T + b1), H2^T = tanh(W2 H1^T + b2), Y^T = W3 H2^T + b3 for
// 16 rows. The 16 x 16 result of one matrix-core product gives lane l the
// hidden units 4 (l / 16) .. +3 of row l % 16, which is the B fragment
// (k = those hidden units, column = that row) of the next layer's product,
// so activations stay in registers: no LDS round trip and no barrier between
// layers. The weights are staged in LDS once per workgroup.
//
// Layers 2 and 3 (K = 128) run on the 16x16x32 BF16 product of gfx950 (half
// the instructions of 16x16x16 at the same FLOP): lane l supplies 8 values
// of K, and the same 8 positions of K for the A and the B operand. Those 8
// are taken as the hidden units 4 (l / 16) .. +3 of two consecutive 16-unit
// blocks -- the two result fragments the lane already holds -- so the K
// order of a 32-wide step is a permutation of the hidden units, which the
// staging applies to the weight columns (stage_weights_k32).
constexpr int INFER_WAVES = 8;                  // wavefronts per workgroup (one weight copy)
constexpr int INFER_ROWS = 16 * INFER_WAVES;     // rows per workgroup tile
__global__ void __launch_bounds__(64 * INFER_WAVES)
k_mlp_infer(MlpArgs m, const float* __restrict__ X, int64_t n, const int32_t* __restrict__ n_dev,
            const int32_t* __restrict__ out_idx, float* __restrict__ Y) {
  if (n_dev) n = min(n, (int64_t)max(*n_dev, 0));
  const int64_t tiles = (n + INFER_ROWS - 1) / INFER_ROWS;
  if ((int64_t)blockIdx.x >= tiles) return;  // uniform per workgroup, before any barrier
  __shared__ __attribute__((aligned(16))) unsigned short w1[NH * LDI], w2[NH * LDH], w3[NOP * LDH];
  __shared__ __attribute__((aligned(16))) float bias[NH + NH + NOP];
  stage_weights_k32(m, w1, w2, w3);
  for (int i = threadIdx.x; i < NH; i += blockDim.x) {
    bias[i] = m.b1[i];
    bias[NH + i] = m.b2[i];
  }
  if (threadIdx.x < NOP) bias[2 * NH + threadIdx.x] = threadIdx.x < NO ? m.b3[threadIdx.x] : 0.0f;
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, kq = (lane >> 4) * 4;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t row = tile * INFER_ROWS + wv * 16 + col;  // this lane's row (column of the products)
    // B fragment of X^T: features kq .. kq + 3 of the row (zero past 12 and past n)
    s4 bx;
    {
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (row < n && kq < NI) v = *reinterpret_cast<const float4*>(X + row * NI + kq);
      bx = s4{(short)to_bf16(v.x), (short)to_bf16(v.y), (short)to_bf16(v.z), (short)to_bf16(v.w)};
    }
    auto activate = [&](f4 acc, int boff) {
      const float4 b = *reinterpret_cast<const float4*>(bias + boff + kq);
      return s4{(short)to_bf16(tanh_fast(acc[0] + b.x)), (short)to_bf16(tanh_fast(acc[1] + b.y)),
                (short)to_bf16(tanh_fast(acc[2] + b.z)), (short)to_bf16(tanh_fast(acc[3] + b.w))};
    };
    // layer 1: 8 blocks of 16 hidden units
    s4 h1[NH / 16];
#pragma unroll
    for (int t = 0; t < NH / 16; ++t) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(frag(w1, LDI, t * 16 + col, kq), bx, acc, 0, 0, 0);
      h1[t] = activate(acc, t * 16);
    }
    // layer 2: the 8 output blocks advance together (independent
    // accumulators keep the matrix cores busy), 32 input units at a time
    f4 acc2[NH / 16];
#pragma unroll
    for (int u = 0; u < NH / 16; ++u) acc2[u] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < NH / 32; ++t) {
      const b8 bh = cat8(h1[2 * t], h1[2 * t + 1]);
#pragma unroll
      for (int u = 0; u < NH / 16; ++u)
        acc2[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag8(w2, LDH, u * 16 + col, t * 32 + 2 * kq),
                                                          bh, acc2[u], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);  // 8 weight fragments live at a time
    }
    s4 h2[NH / 16];
#pragma unroll
    for (int u = 0; u < NH / 16; ++u) h2[u] = activate(acc2[u], NH + u * 16);
    // layer 3: outputs 0 and 1 land in lanes 0 .. 15, elements 0 and 1
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < NH / 32; ++t)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag8(w3, LDH, col, t * 32 + 2 * kq),
                                                    cat8(h2[2 * t], h2[2 * t + 1]), acc, 0, 0, 0);
    if (kq == 0 && row < n) {
      const int64_t o = out_idx ? (int64_t)out_idx[row] : row;
      Y[o * NO] = acc[0] + bias[2 * NH];
      Y[o * NO + 1] = acc[1] + bias[2 * NH + 1];
    }
  }
}

// Backward pass of 64 rows given dY [n][2] and the forward activations.
// Writes dX [n][12] (optional) and this workgroup's partial gradient of all
// parameters, in the canonical order W1 (128x12), b1, W2 (128x128), b2,
// W3 (2x128), b3, into part[blockIdx.x][NPARAM].
constexpr int NPARAM = NH * NI + NH + NH * NH + NH + NO * NH + NO;

__global__ void __launch_bounds__(256) k_mlp_backward(MlpArgs m, const float* __restrict__ X,
                                                      const float* __restrict__ H1,
                                                      const float* __restrict__ H2,
                                                      const float* __restrict__ dY, int64_t n,
                                                      float* __restrict__ dX,
                                                      float* __restrict__ part) {
  // transposed weights: W3^T [NH][NOP], W2^T [NH][NH], W1^T [NIP][NH]
  __shared__ __attribute__((aligned(16))) unsigned short w3t[NH * LDI], w2t[NH * LDH], w1t[NIP * LDH];
  // per-row operands (row-major, K = features) and their transposes (K = rows)
  __shared__ __attribute__((aligned(16))) unsigned short dys[ROWS * LDI], dz2s[ROWS * LDH], dz1s[ROWS * LDH];
  __shared__ __attribute__((aligned(16))) unsigned short dyT[NOP * LDR], dz2T[NH * LDR], dz1T[NH * LDR];
  __shared__ __attribute__((aligned(16))) unsigned short h1T[NH * LDR], xT[NIP * LDR];
  __shared__ float bsum[4][NH + NH + NOP];
  // 8 consecutive weights of a row per 16-byte load, stored transposed
  auto stage_t = [&](const unsigned short* W, int rows, int cols, unsigned short* dst, int ld) {
    const uint4* g = reinterpret_cast<const uint4*>(W);
    for (int i = threadIdx.x; i < rows * cols / 8; i += blockDim.x) {
      const int o = i / (cols / 8), k0 = (i % (cols / 8)) * 8;
      const uint4 v = g[i];
      const unsigned short* e = reinterpret_cast<const unsigned short*>(&v);
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[(k0 + j) * ld + o] = e[j];
    }
  };
  stage_t(m.W1, NH, NIP, w1t, LDH);
  stage_t(m.W2, NH, NH, w2t, LDH);
  stage_t(m.W3, NOP, NH, w3t, LDI);
  const int64_t row0 = (int64_t)blockIdx.x * ROWS;
  for (int i = threadIdx.x; i < ROWS * NH; i += blockDim.x) {
    const int r = i / NH, c = i % NH;
    const int64_t g = row0 + r;
    h1T[c * LDR + r] = to_bf16(g < n ? H1[g * NH + c] : 0.0f);
  }
  for (int i = threadIdx.x; i < ROWS * NOP; i += blockDim.x) {
    const int r = i / NOP, c = i % NOP;
    const int64_t g = row0 + r;
    const float v = (c < NO && g < n) ? dY[g * NO + c] : 0.0f;
    dys[r * LDI + c] = to_bf16(v);
    dyT[c * LDR + r] = to_bf16(v);
    xT[c * LDR + r] = to_bf16((c < NI && g < n) ? X[g * NI + c] : 0.0f);
  }
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = wv * 16, col = lane & 15, rq = (lane >> 4) * 4;
  float* bs = bsum[wv];
  // dz2 = (dy W3) * (1 - h2^2)
  for (int j = 0; j < NH / 16; ++j) {
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mma(acc, dys, LDI, r0, w3t, LDI, j * 16, NOP, lane);
    const int c = j * 16 + col;
    float cs = 0.0f;
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + rq + i;
      const int64_t g = row0 + r;
      const float h = g < n ? H2[g * NH + c] : 0.0f;
      const float dz = acc[i] * (1.0f - h * h);
      cs += dz;
      const unsigned short b = to_bf16(dz);
      dz2s[r * LDH + c] = b;
      dz2T[c * LDR + r] = b;
    }
    // column sum over the 16 rows of this wavefront (4 lanes share a column)
    cs += __shfl_xor(cs, 16);
    cs += __shfl_xor(cs, 32);
    if (lane < 16) bs[NH + c] = cs;
  }
  __syncthreads();
  // dz1 = (dz2 W2) * (1 - h1^2)
  for (int j = 0; j < NH / 16; ++j) {
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mma(acc, dz2s, LDH, r0, w2t, LDH, j * 16, NH, lane);
    const int c = j * 16 + col;
    float cs = 0.0f;
    for (int i = 0; i < 4; ++i) {
      const int r = r0 + rq + i;
      const int64_t g = row0 + r;
      const float h = g < n ? H1[g * NH + c] : 0.0f;
      const float dz = acc[i] * (1.0f - h * h);
      cs += dz;
      const unsigned short b = to_bf16(dz);
      dz1s[r * LDH + c] = b;
      dz1T[c * LDR + r] = b;
    }
    cs += __shfl_xor(cs, 16);
    cs += __shfl_xor(cs, 32);
    if (lane < 16) bs[c] = cs;
  }
  // db3: column sums of dy
  if (lane < NO) {
    float cs = 0.0f;
    for (int i = 0; i < 16; ++i) {
      const int64_t g = row0 + r0 + i;
      cs += g < n ? dY[g * NO + lane] : 0.0f;
    }
    bs[2 * NH + lane] = cs;
  }
  __syncthreads();
  // dX = dz1 W1 (first 12 columns)
  if (dX) {
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mma(acc, dz1s, LDH, r0, w1t, LDH, 0, NH, lane);
    if (col < NI)
      for (int i = 0; i < 4; ++i) {
        const int64_t g = row0 + r0 + rq + i;
        if (g < n) dX[g * NI + col] = acc[i];
      }
  }
  float* P = part + (size_t)blockIdx.x * NPARAM;
  // dW2 = dz2^T h1 (128 x 128, K = 64 rows): 64 output tiles, 16 per wavefront
  for (int t = wv; t < 64; t += 4) {
    const int ti = t / 8, tj = t % 8;
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mma(acc, dz2T, LDR, ti * 16, h1T, LDR, tj * 16, ROWS, lane);
    for (int i = 0; i < 4; ++i)
      P[NH * NI + NH + (ti * 16 + rq + i) * NH + tj * 16 + col] = acc[i];
  }
  // dW1 = dz1^T x (128 x 12): 8 tiles, 2 per wavefront
  for (int t = wv; t < 8; t += 4) {
    f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = mma(acc, dz1T, LDR, t * 16, xT, LDR, 0, ROWS, lane);
    if (col < NI)
      for (int i = 0; i < 4; ++i) P[(t * 16 + rq + i) * NI + col] = acc[i];
  }
  // dW3 = dy^T h2 (2 x 128, K = 64 rows) on the vector units, one output per
  // thread, BF16-rounded operands as in the matrix-core products
  {
    const int o = threadIdx.x / NH, k = threadIdx.x % NH;
    float acc = 0.0f;
    for (int r = 0; r < ROWS; ++r) {
      const int64_t g = row0 + r;
      if (g < n)
        acc = fmaf(from_bf16(to_bf16(dY[g * NO + o])), from_bf16(to_bf16(H2[g * NH + k])), acc);
    }
    P[NH * NI + NH + NH * NH + NH + o * NH + k] = acc;
  }
  __syncthreads();
  // bias partials: wavefront partial sums added in a fixed order
  for (int c = threadIdx.x; c < NH; c += blockDim.x) {
    P[NH * NI + c] = ((bsum[0][c] + bsum[1][c]) + bsum[2][c]) + bsum[3][c];
    P[NH * NI + NH + NH * NH + c] =
        ((bsum[0][NH + c] + bsum[1][NH + c]) + bsum[2][NH + c]) + bsum[3][NH + c];
  }
  if (threadIdx.x < NO) {
    const int c = threadIdx.x;
    P[NPARAM - NO + c] =
        ((bsum[0][2 * NH + c] + bsum[1][2 * NH + c]) + bsum[2][2 * NH + c]) + bsum[3][2 * NH + c];
  }
}

// grad[p] = sum over workgroups b (in order) of part[b][p].
__global__ void k_reduce_parts(const float* __restrict__ part, int nparts, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float s = 0.0f;
  for (int b = 0; b < nparts; ++b) s += part[(size_t)b * NPARAM + p];
  grad[p] = s;
}

// dY = (Y - target) / n, and the loss sum (Y - target)^2 / (2n) per row.
__global__ void k_mse_grad(const float* __restrict__ Y, const float* __restrict__ tgt, int64_t n,
                           float* __restrict__ dY, float* __restrict__ row_loss) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float inv = 1.0f / (float)n;
  float l = 0.0f;
  for (int c = 0; c < NO; ++c) {
    const float e = Y[i * NO + c] - tgt[i * NO + c];
    dY[i * NO + c] = e * inv;
    l += e * e;
  }
  if (row_loss) row_loss[i] = 0.5f * l * inv;
}

// Adam on the FP32 master parameters; refreshes the BF16 padded copies.
__global__ void k_adam(float* __restrict__ master, float* __restrict__ mom, float* __restrict__ var,
                       const float* __restrict__ grad, float lr, float b1, float b2, float eps,
                       float c1, float c2, unsigned short* __restrict__ W1,
                       unsigned short* __restrict__ W2, unsigned short* __restrict__ W3,
                       float* __restrict__ bias1, float* __restrict__ bias2, float* __restrict__ bias3) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = grad[p];
  const float mm = b1 * mom[p] + (1.0f - b1) * g;
  const float vv = b2 * var[p] + (1.0f - b2) * g * g;
  mom[p] = mm;
  var[p] = vv;
  const float w = master[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  master[p] = w;
  int q = p;
  if (q < NH * NI) {
    W1[(q / NI) * NIP + q % NI] = to_bf16(w);
    return;
  }
  q -= NH * NI;
  if (q < NH) {
    bias1[q] = w;
    return;
  }
  q -= NH;
  if (q < NH * NH) {
    W2[q] = to_bf16(w);
    return;
  }
  q -= NH * NH;
  if (q < NH) {
    bias2[q] = w;
    return;
  }
  q -= NH;
  if (q < NO * NH) {
    W3[q] = to_bf16(w);
    return;
  }
  q -= NO * NH;
  bias3[q] = w;
}

// Copies FP32 master parameters into the kernel layouts (no update).
__global__ void k_unpack(const float* __restrict__ master, unsigned short* __restrict__ W1,
                         unsigned short* __restrict__ W2, unsigned short* __restrict__ W3,
                         float* __restrict__ bias1, float* __restrict__ bias2,
                         float* __restrict__ bias3) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float w = master[p];
  int q = p;
  if (q < NH * NI) { W1[(q / NI) * NIP + q % NI] = to_bf16(w); return; }
  q -= NH * NI;
  if (q < NH) { bias1[q] = w; return; }
  q -= NH;
  if (q < NH * NH) { W2[q] = to_bf16(w); return; }
  q -= NH * NH;
  if (q < NH) { bias2[q] = w; return; }
  q -= NH;
  if (q < NO * NH) { W3[q] = to_bf16(w); return; }
  q -= NO * NH;
  bias3[q] = w;
}

// loss[0] = sum of row losses, one workgroup, fixed order.
__global__ void k_sum(const float* __restrict__ v, int64_t n, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

hipError_t mlp_launch_sum(const float* v, int64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

int mlp_nparam() { return NPARAM; }

hipError_t mlp_launch_forward(const unsigned short* W1, const unsigned short* W2,
                              const unsigned short* W3, const float* b1, const float* b2,
                              const float* b3, const float* X, int64_t n, const int32_t* n_dev,
                              const int32_t* out_idx, float* Y, float* H1, float* H2,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (out_idx && (H1 || H2)) return hipErrorInvalidValue;  // scattered outputs: inference only
  MlpArgs m{W1, W2, W3, b1, b2, b3};
  const int64_t tiles = (n + ROWS - 1) / ROWS;
  const int64_t blocks = tiles < 2048 ? tiles : 2048;  // 8 workgroups per CU walk the tiles
  if (H1 || H2)
    hipLaunchKernelGGL(k_mlp_forward<true>, dim3((unsigned)blocks), dim3(256), 0, s, m, X, n, n_dev,
                       Y, H1, H2);
  else {
    const int64_t itiles = (n + INFER_ROWS - 1) / INFER_ROWS;
    const int64_t iblocks = itiles < 768 ? itiles : 768;  // 3 workgroups per CU walk the tiles
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)iblocks), dim3(64 * INFER_WAVES), 0, s, m, X, n,
                       n_dev, out_idx, Y);
  }
  return hipGetLastError();
}

hipError_t mlp_launch_backward(const unsigned short* W1, const unsigned short* W2,
                               const unsigned short* W3, const float* b1, const float* b2,
                               const float* b3, const float* X, const float* H1, const float* H2,
                               const float* dY, int64_t n, float* dX, float* part, float* grad,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  MlpArgs m{W1, W2, W3, b1, b2, b3};
  const int64_t blocks = (n + ROWS - 1) / ROWS;
  hipLaunchKernelGGL(k_mlp_backward, dim3((unsigned)blocks), dim3(256), 0, s, m, X, H1, H2, dY, n,
                     dX, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !grad) return e;
  hipLaunchKernelGGL(k_reduce_parts, dim3((NPARAM + 255) / 256), dim3(256), 0, s, part,
                     (int)blocks, grad);
  return hipGetLastError();
}

hipError_t mlp_launch_mse(const float* Y, const float* tgt, int64_t n, float* dY, float* row_loss,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mse_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Y, tgt, n, dY,
                     row_loss);
  return hipGetLastError();
}

hipError_t mlp_launch_adam(float* master, float* mom, float* var, const float* grad, float lr,
                           float b1, float b2, float eps, int step, unsigned short* W1,
                           unsigned short* W2, unsigned short* W3, float* bias1, float* bias2,
                           float* bias3, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, master, mom, var, grad,
                     lr, b1, b2, eps, c1, c2, W1, W2, W3, bias1, bias2, bias3);
  return hipGetLastError();
}

hipError_t mlp_launch_unpack(const float* master, unsigned short* W1, unsigned short* W2,
                             unsigned short* W3, float* bias1, float* bias2, float* bias3,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3((NPARAM + 255) / 256), dim3(256), 0, s, master, W1, W2, W3,
                     bias1, bias2, bias3);
  return hipGetLastError();
}

int64_t mlp_parts_for(int64_t n) { return (n + ROWS - 1) / ROWS; }

}  // namespace vmas
