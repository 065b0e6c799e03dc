// Slosh-wrench surrogate: a 128 -> 4 x (256, GELU) -> 3 MLP on gfx950 MFMA.
//
// Every dense product is one kernel, gemm_tn: C[m][n] = sum_k A[m][k] B[n][k]
// with both operands BF16 and contiguous along k, accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16.  Each product of the network is cast in that form
// by choosing what the epilogues store:
//   forward   z_l = a_{l-1} W_l^T + b_l          A = a_{l-1} [B][in],  B = W_l [out][in]
//   dgrad     g_{l-1} = (g_l W_l) * gelu'(z)     A = g_l [B][out],     B = W_l^T [in][out]
//   wgrad     dW_l = g_l^T a_{l-1}                A = g_l^T [out][B],   B = a_{l-1}^T [in][B]
//             (the batch split into up to 16 parts, their results summed in order)
// so the forward epilogue also writes the transposed activation and the
// pre-activation, and the dgrad epilogue writes the gradient both ways.  The
// 3-wide head, the loss, the bias gradients and Adam are small VALU kernels.
// GELU is the tanh form; Adam keeps FP32 master weights and refreshes the
// BF16 copies (row-major and transposed) after every step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>

#include "slosh.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 128, kHid = 256, kOut = 3, kLayers = 5;
constexpr int kDims[kLayers + 1] = {kIn, kHid, kHid, kHid, kHid, kOut};
// packed parameter offsets: W_l then b_l for l = 0..4
constexpr int kOffW[kLayers] = {0, 33024, 98816, 164608, 230400};
constexpr int kOffB[kLayers] = {32768, 98560, 164352, 230144, 231168};
static_assert(kOffB[4] + kOut == MLP_N_PARAMS, "packing");

constexpr float kGeluK = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float kGeluC = 0.044715f;

constexpr float kLog2e = 1.4426950408889634f;

// The logistic function of 2u, 1 / (1 + e^(-2u)), from the hardware base-2
// exponential and reciprocal (about 1 ulp each; e^(-2u) overflowing to +inf
// gives 0, underflowing to 0 gives 1).
__device__ __forceinline__ float sigmoid2(float u) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-2.0f * kLog2e * u));
}

// The tanh form x/2 (1 + tanh(u)), u = sqrt(2/pi)(x + 0.044715 x^3), written
// as x s with s = 1 / (1 + e^(-2u)) (1 + tanh(u) = 2 / (1 + e^(-2u))), and
// -2u log2(e) = x (A + B x^2): branch-free, 5 instructions and the hardware
// exponential and reciprocal.
constexpr float kGeluA = -2.0f * kLog2e * kGeluK;
constexpr float kGeluB = kGeluA * kGeluC;

__device__ __forceinline__ float gelu(float x) {
  const float v = x * fmaf(kGeluB, x * x, kGeluA);
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(v));
}

// Its derivative, s + 2 x s (1 - s) u'(x) (the tanh form's
// (1 + t)/2 + x (1 - t^2) u'/2 with 1 + t = 2 s, 1 - t^2 = 4 s (1 - s)).
__device__ __forceinline__ float gelu_grad(float x) {
  const float x2 = x * x;
  const float sg = sigmoid2(kGeluK * x * fmaf(kGeluC, x2, 1.0f));
  const float du = kGeluK * fmaf(3.0f * kGeluC, x2, 1.0f);
  return sg + 2.0f * x * sg * (1.0f - sg) * du;
}

// ---------------------------------------------------------------------------
// gemm_tn: 256 threads = 4 waves in a 2x2 arrangement, 64x64 output tile, each
// wave 32x32 = 2x2 MFMA tiles of 16x16.  Lane l holds row (l % 16) of A and
// column (l % 16) of B for k in [8 (l / 16), 8 (l / 16) + 8) of each 32-wide
// k step; the result element e of lane l is row 4 (l / 16) + e, column
// l % 16, or, for an epilogue that asks for B as the first MFMA operand
// (kBFirst), row l % 16, column 4 (l / 16) + e.
// Rows m >= M and columns n >= N read zeros and are not stored.  K % 32 == 0.
// A grid with gridDim.z > 1 splits the k range into gridDim.z equal parts
// (K % (32 gridDim.z) == 0); part z covers [z K/Z, (z+1) K/Z) and its
// epilogue sees blockIdx.z (EpiPart stores each part in its own slab).
// ---------------------------------------------------------------------------

struct EpiFwd {            // hidden forward layer
  static constexpr bool kBFirst = true;   // two of its three stores are transposed
  const float* bias;       // [N]
  bf16* act;               // [M][ld_act] row-major, next layer's A
  int ld_act;
  bf16* actT;              // [N][ldT] or null (training)
  float* zT;               // [N][ldT] or null (training)
  int ldT;
  __device__ void operator()(int m, int n, float v) const {
    float z = v + bias[n];
    float a = gelu(z);
    act[(size_t)m * ld_act + n] = (bf16)a;
    if (actT) {
      actT[(size_t)n * ldT + m] = (bf16)a;
      zT[(size_t)n * ldT + m] = z;
    }
  }
};

struct EpiDgrad {          // g_{l-1} = (g_l W_l) * gelu'(z_{l-1})
  static constexpr bool kBFirst = false;
  const float* zT;         // [N][ldT] pre-activation of the layer below
  bf16* g;                 // [M][ld_g] row-major or null
  int ld_g;
  bf16* gT;                // [N][ldT]
  int ldT;
  __device__ void operator()(int m, int n, float v) const {
    float gv = v * gelu_grad(zT[(size_t)n * ldT + m]);
    if (g) g[(size_t)m * ld_g + n] = (bf16)gv;
    gT[(size_t)n * ldT + m] = (bf16)gv;
  }
};

struct EpiPart {           // k-split part z of a weight gradient, into slab z
  static constexpr bool kBFirst = false;
  float* c;
  int ldc;
  size_t slab;
  __device__ void operator()(int m, int n, float v) const { c[blockIdx.z * slab + (size_t)m * ldc + n] = v; }
};

template <class Epi>
__global__ void __launch_bounds__(256) gemm_tn(const bf16* __restrict__ A, int lda,
                                               const bf16* __restrict__ B, int ldb, int M, int N,
                                               int K, Epi epi) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int m0 = blockIdx.y * 64 + wy * 32;
  const int n0 = blockIdx.x * 64 + wx * 32;
  const int li = lane & 15, kq = (lane >> 4) * 8;
  floatx4 acc[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = {};
  const int kz = K / (int)gridDim.z, kb = (int)blockIdx.z * kz;
  for (int k0 = kb; k0 < kb + kz; k0 += 32) {
    bf16x8 a[2], b[2];
    for (int r = 0; r < 2; ++r) {
      int m = m0 + r * 16 + li;
      a[r] = m < M ? *reinterpret_cast<const bf16x8*>(A + (size_t)m * lda + k0 + kq) : zero;
    }
    for (int c = 0; c < 2; ++c) {
      int n = n0 + c * 16 + li;
      b[c] = n < N ? *reinterpret_cast<const bf16x8*>(B + (size_t)n * ldb + k0 + kq) : zero;
    }
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c)
        acc[r][c] = Epi::kBFirst ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[c], a[r], acc[r][c], 0, 0, 0)
                                 : __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[r], b[c], acc[r][c], 0, 0, 0);
  }
  const int q4 = (lane >> 4) * 4;
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c)
      for (int e = 0; e < 4; ++e) {
        // B first: element e of lane l is row 16 r + l % 16, column
        // 16 c + 4 (l / 16) + e (the lanes of a store hold consecutive rows,
        // so transposed stores are contiguous); A first: row 16 r + 4 (l / 16)
        // + e, column 16 c + l % 16 (row-major stores are)
        const int m = m0 + r * 16 + (Epi::kBFirst ? li : q4 + e);
        const int n = n0 + c * 16 + (Epi::kBFirst ? q4 + e : li);
        if (m < M && n < N) epi(m, n, acc[r][c][e]);
      }
}

// Inference: the whole network for a tile of kRows rows in one workgroup.
// Activations stay in LDS (two BF16 buffers, rows padded by 16 bytes); each of
// the 4 waves computes kRows x 64 outputs of a layer as 4 x 4 MFMA tiles with
// the weights read from L2 (accumulators starting from the biases); GELU is
// applied in the epilogue; the 3-wide head is one MFMA tile per 16 rows.
constexpr int kRows = 64;
constexpr int kLdsStride = kHid + 8;

// The products of a layer are taken with the weights as the first MFMA
// operand and the activations as the second, so that acc[r][c] holds, in
// lane l, outputs n0 + 16 c + rq .. + 3 (rq = 4 (l / 16)) of row 16 r +
// l % 16: four consecutive outputs of one row, stored as one 8-byte word.
// The accumulators start from the biases (bias_acc), so a layer's output
// is GELU of the accumulator (tile_out).

// Accumulators of a layer set to this lane's biases: bn[c] holds the biases
// of outputs n0 + 16 c + rq .. + 3, the outputs acc[r][c] holds.
template <int RT>
__device__ __forceinline__ void bias_acc(floatx4 (&acc)[RT][4], const float4 (&bn)[4]) {
  for (int r = 0; r < RT; ++r)
    for (int c = 0; c < 4; ++c) acc[r][c] = floatx4{bn[c].x, bn[c].y, bn[c].z, bn[c].w};
}

// This lane's biases of layer l (the outputs bias_acc gives them to).
__device__ __forceinline__ void load_bias(float4 (&bn)[4], const float* __restrict__ master, int l, int n0, int rq) {
  for (int c = 0; c < 4; ++c) bn[c] = *reinterpret_cast<const float4*>(master + kOffB[l] + n0 + c * 16 + rq);
}

// Weight fragments are requested this many k steps ahead of their use.
constexpr int kAhead = 2;

template <int L>
constexpr int layer_in() { return L == 0 ? kIn : kHid; }

// GELU of one 16 x 16 output tile (row tile r, column tile c) of this wave
// into dst (BF16): the lane's four consecutive outputs of one row as one
// 8-byte word.
__device__ __forceinline__ void tile_out(const floatx4& acc, bf16* dst, int r, int c, int n0, int li, int rq) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  bf16x4 v;
  v[0] = (bf16)gelu(acc[0]);
  v[1] = (bf16)gelu(acc[1]);
  v[2] = (bf16)gelu(acc[2]);
  v[3] = (bf16)gelu(acc[3]);
  *reinterpret_cast<bf16x4*>(&dst[(r * 16 + li) * kLdsStride + n0 + c * 16 + rq]) = v;
}

// The weight fragments of column tiles 2h and 2h + 1 at k step ks.
template <int K>
__device__ __forceinline__ void load_w2(bf16x8 (&b)[2], const bf16* __restrict__ W, int ks, int h, int n0, int li,
                                        int kq) {
  for (int c = 0; c < 2; ++c)
    b[c] = *reinterpret_cast<const bf16x8*>(W + (size_t)(n0 + (2 * h + c) * 16 + li) * K + ks * 32 + kq);
}

// Hidden layer L of a full row tile (kRows rows, RT = 4), in two halves of
// the wave's 64 outputs (column tiles 0-1, then 2-3), with the weight loads
// software-pipelined over the 2 K/32 steps of both halves: pre holds the
// fragments of the first kAhead steps and bn the biases, both requested
// before the previous layer's epilogue; step s requests step s + kAhead.
// The first half's epilogue is interleaved with the second half's products
// (one 16 x 16 tile per step or two), so that the matrix cores and the
// vector unit of a wave work at once; before the second half's epilogue the
// next layer's first steps and biases are requested.
template <int L, int ROWS>
__device__ __forceinline__ void layer_pipe(bf16 (*buf)[ROWS * kLdsStride], const bf16* __restrict__ wb,
                                           const float* __restrict__ master, bf16x8 (&pre)[kAhead][2],
                                           float4 (&bn)[4], int n0, int li, int kq, int rq) {
  constexpr int RT = ROWS / 16, K = layer_in<L>(), KS = K / 32, S = 2 * KS;
  static_assert(KS > kAhead, "the prefetch distance fits the layer");
  const bf16* W = wb + kOffW[L];
  const bf16* src = buf[L & 1];
  bf16* dst = buf[1 - (L & 1)];
  floatx4 acc[RT][4];
  bias_acc<RT>(acc, bn);
  bf16x8 b[S][2];
#pragma unroll
  for (int s = 0; s < kAhead; ++s)
    for (int c = 0; c < 2; ++c) b[s][c] = pre[s][c];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int h = s / KS, ks = s % KS;
    if (s + kAhead < S) load_w2<K>(b[s + kAhead], W, (s + kAhead) % KS, (s + kAhead) / KS, n0, li, kq);
    if (h == 1 && ks == KS - 1 && L < 3) {
      // the next layer's first steps and biases
      constexpr int KN = layer_in<(L < 3 ? L + 1 : L)>();
#pragma unroll
      for (int t = 0; t < kAhead; ++t) load_w2<KN>(pre[t], wb + kOffW[L < 3 ? L + 1 : L], t, 0, n0, li, kq);
      load_bias(bn, master, L < 3 ? L + 1 : L, n0, rq);
    }
    bf16x8 a[RT];
    for (int r = 0; r < RT; ++r)
      a[r] = *reinterpret_cast<const bf16x8*>(&src[(r * 16 + li) * kLdsStride + ks * 32 + kq]);
    for (int r = 0; r < RT; ++r)
      for (int c = 0; c < 2; ++c)
        acc[r][2 * h + c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[s][c], a[r], acc[r][2 * h + c], 0, 0, 0);
    if (h == 1)   // the first half's tiles g (2 RT of them) spread over the KS steps
      for (int g = 0; g < 2 * RT; ++g)
        if (g * KS / (2 * RT) == ks) tile_out(acc[g >> 1][g & 1], dst, g >> 1, g & 1, n0, li, rq);
    __builtin_amdgcn_sched_barrier(0);   // keep each step's requests and epilogue tiles in its own step
  }
  for (int r = 0; r < RT; ++r)
    for (int c = 2; c < 4; ++c) tile_out(acc[r][c], dst, r, c, n0, li, rq);
  __syncthreads();
}

// The network on the ROWS rows (a multiple of 16, at most kRows) staged in
// buf[0] as BF16: the four hidden layers on MFMA (ping-pong between the two
// buffers; each of the 4 waves computes ROWS x 64 outputs of a layer as
// ROWS/16 x 4 MFMA tiles), then the head, whose result for row r and output
// o goes to out(r, o, value) (called by one lane of the row's wave).  w4s
// is the head's weight matrix (3 x 256) staged in LDS by the caller.  All
// 256 threads; ends without a barrier.
template <int ROWS, class Out>
__device__ __forceinline__ void net_rows(bf16 (*buf)[ROWS * kLdsStride], const bf16* __restrict__ wb,
                                         const float* __restrict__ master, const bf16* w4s, Out&& out) {
  static_assert(ROWS % 16 == 0 && ROWS <= kRows, "row tiles of 16");
  constexpr int RT = ROWS / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4;
  const int n0 = wave * 64;
  // the head's biases, fetched now so that their round trip is hidden
  const float hb0 = master[kOffB[4]], hb1 = master[kOffB[4] + 1], hb2 = master[kOffB[4] + 2];
  // the pipelined layers; layer L writes buf[1 - (L & 1)], so the last
  // hidden layer's outputs are in buf[0]
  bf16x8 pre[kAhead][2];
  float4 bn[4];
#pragma unroll
  for (int s = 0; s < kAhead; ++s) load_w2<kIn>(pre[s], wb + kOffW[0], s, 0, n0, li, kq);
  load_bias(bn, master, 0, n0, rq);
  layer_pipe<0, ROWS>(buf, wb, master, pre, bn, n0, li, kq, rq);
  layer_pipe<1, ROWS>(buf, wb, master, pre, bn, n0, li, kq, rq);
  layer_pipe<2, ROWS>(buf, wb, master, pre, bn, n0, li, kq, rq);
  layer_pipe<3, ROWS>(buf, wb, master, pre, bn, n0, li, kq, rq);
  static_assert(((4 - 1) & 1) == 1, "an even number of hidden layers ends in buf[0]");
  constexpr int cur = 0;
  // the head on MFMA: wave w takes row tile w, its 3 outputs padded to a
  // 16-wide tile with zero weights; lane l < 16 ends with outputs 0-2 of
  // row 16 w + l (the accumulator starts from the head's biases)
  static_assert(kOut == 3, "head layout");
  if (wave >= RT) return;
  floatx4 h = rq == 0 ? floatx4{hb0, hb1, hb2, 0.f} : floatx4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero = {};
#pragma unroll
  for (int ks = 0; ks < kHid / 32; ++ks) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(&buf[cur][(wave * 16 + li) * kLdsStride + ks * 32 + kq]);
    const bf16x8 b = li < kOut ? *reinterpret_cast<const bf16x8*>(&w4s[li * kHid + ks * 32 + kq]) : zero;
    h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a, h, 0, 0, 0);
  }
  if (lane < 16) {
    out(wave * 16 + li, 0, h[0]);
    out(wave * 16 + li, 1, h[1]);
    out(wave * 16 + li, 2, h[2]);
  }
}

// The head's weights (3 x 256 BF16, 96 fragments of 8) into LDS; threads
// 0-95.  The caller's barrier publishes them.
__device__ __forceinline__ void stage_head(const bf16* __restrict__ wb, bf16* w4s) {
  if (threadIdx.x < kOut * kHid / 8)
    *reinterpret_cast<bf16x8*>(w4s + 8 * threadIdx.x) =
        *reinterpret_cast<const bf16x8*>(wb + kOffW[4] + 8 * threadIdx.x);
}

__global__ void __launch_bounds__(256) mlp_forward_fused(const float* __restrict__ x, int B,
                                                         const bf16* __restrict__ wb,
                                                         const float* __restrict__ master,
                                                         float* __restrict__ y) {
  __shared__ __align__(16) bf16 buf[2][kRows * kLdsStride];
  __shared__ __align__(16) bf16 w4s[kOut * kHid];
  const int row0 = blockIdx.x * kRows;
  // the tile's inputs, 4 floats per load and all of a thread's loads issued
  // before the first is used (rows past B read as zeros)
  constexpr int kQ = kRows * kIn / 4 / 256;
  const float* xt = x + (size_t)row0 * kIn;
  float4 xv[kQ];
  if (row0 + kRows <= B) {
#pragma unroll
    for (int i = 0; i < kQ; ++i) xv[i] = *reinterpret_cast<const float4*>(xt + 4 * ((int)threadIdx.x + 256 * i));
  } else {
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int e = 4 * ((int)threadIdx.x + 256 * i);
      xv[i] = row0 + e / kIn < B ? *reinterpret_cast<const float4*>(xt + e) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  stage_head(wb, w4s);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int e = 4 * ((int)threadIdx.x + 256 * i), r = e / kIn, k = e - r * kIn;
    bf16* d = &buf[0][r * kLdsStride + k];
    d[0] = (bf16)xv[i].x;
    d[1] = (bf16)xv[i].y;
    d[2] = (bf16)xv[i].z;
    d[3] = (bf16)xv[i].w;
  }
  __syncthreads();
  net_rows<kRows>(buf, wb, master, w4s, [&](int r, int o, float v) {
    const int m = row0 + r;
    if (m < B) y[(size_t)m * kOut + o] = v;
  });
}

// FP32 input [B][128] -> BF16 row-major and (training) transposed copies,
// kCastRows rows a workgroup: the rows read and the row-major copy written
// four values a thread at a time, the transposed copy through LDS, kCastRows
// consecutive values of each of its rows at a time.  (64 rows a workgroup
// left a batch of 4,096 with 64 workgroups, and the training step took 199
// instead of 171 us.)
constexpr int kCastRows = 16;

__global__ void __launch_bounds__(256) mlp_cast_input(const float* __restrict__ x, int B, bf16* __restrict__ xb,
                                                      bf16* __restrict__ xT, int ldT) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  __shared__ bf16 tT[kIn][kCastRows + 2];   // transposed tile (rows padded against bank conflicts)
  const int row0 = blockIdx.x * kCastRows;
  const int nr = B - row0 < kCastRows ? B - row0 : kCastRows;
  for (int i = threadIdx.x; i < kCastRows * kIn / 4; i += 256) {
    const int rr = i / (kIn / 4), k = (i - rr * (kIn / 4)) * 4;
    if (rr >= nr) continue;
    const float4 v = *reinterpret_cast<const float4*>(x + (size_t)(row0 + rr) * kIn + k);
    bf16x4 b;
    b[0] = (bf16)v.x;
    b[1] = (bf16)v.y;
    b[2] = (bf16)v.z;
    b[3] = (bf16)v.w;
    *reinterpret_cast<bf16x4*>(xb + (size_t)(row0 + rr) * kIn + k) = b;
    if (xT) {
      tT[k][rr] = b[0];
      tT[k + 1][rr] = b[1];
      tT[k + 2][rr] = b[2];
      tT[k + 3][rr] = b[3];
    }
  }
  if (!xT) return;
  __syncthreads();
  for (int i = threadIdx.x; i < kIn * kCastRows; i += 256) {
    const int k = i / kCastRows, rr = i - k * kCastRows;
    if (rr < nr) xT[(size_t)k * ldT + row0 + rr] = tT[k][rr];
  }
}

// Head y = a4 W4^T + b4 for kHeadRows rows a workgroup.  Training: loss terms,
// dL/dy, and g4 = (dL/dy W4) * gelu'(z4) written both ways.  The dot
// products take one wavefront per row; g4 is computed with the lanes along
// the rows, so that the feature-major pre-activation and gradient are read
// and written contiguously, and reaches its row-major copy through LDS.
constexpr int kHeadRows = 16;

__global__ void __launch_bounds__(256) mlp_head(const bf16* __restrict__ a4, const bf16* __restrict__ W4,
                                                const float* __restrict__ b4, int B, float* __restrict__ y,
                                                const float* __restrict__ target, float* __restrict__ gy,
                                                float* __restrict__ loss_rows, const float* __restrict__ z4T,
                                                bf16* __restrict__ g4, bf16* __restrict__ g4T, int ldT,
                                                const float* __restrict__ dy_in) {
  __shared__ float gs[kHeadRows][kOut];                      // dL/dy of the workgroup's rows
  __shared__ __align__(16) bf16 tile[kHeadRows][kLdsStride];   // their g4, row-major
  const int row0 = blockIdx.x * kHeadRows, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nr = B - row0 < kHeadRows ? B - row0 : kHeadRows;
  const bool train = target || dy_in;
  // every load of the kernel requested up front: the wave's rows of a4 and
  // this thread's pre-activations of the g4 part (kHeadRows consecutive rows
  // of a feature per kHeadRows threads)
  constexpr int kRowsPerWave = kHeadRows / 4, kZPer = kHeadRows * kHid / 256;
  float av[kRowsPerWave][4];
#pragma unroll
  for (int j = 0; j < kRowsPerWave; ++j) {
    const int rr = wave + 4 * j;
    for (int q = 0; q < 4; ++q) av[j][q] = rr < nr ? (float)a4[(size_t)(row0 + rr) * kHid + lane * 4 + q] : 0.f;
  }
  float zv[kZPer];
#pragma unroll
  for (int j = 0; j < kZPer; ++j) {
    const int i = threadIdx.x + 256 * j, k = i / kHeadRows, rr = i - k * kHeadRows;
    zv[j] = train && rr < nr ? z4T[(size_t)k * ldT + row0 + rr] : 0.f;
  }
#pragma unroll
  for (int j = 0; j < kRowsPerWave; ++j) {
    const int rr = wave + 4 * j;
    if (rr >= nr) break;
    const int row = row0 + rr;
    const float* a = av[j];
    float out[kOut];
    for (int o = 0; o < kOut; ++o) {
      float s = 0.f;
      for (int q = 0; q < 4; ++q) s += a[q] * (float)W4[o * kHid + lane * 4 + q];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      out[o] = s + b4[o];
    }
    if (lane == 0)
      for (int o = 0; o < kOut; ++o) y[(size_t)row * kOut + o] = out[o];
    if (!train) continue;
    float g[kOut], l = 0.f;
    if (dy_in) {
      // back-propagation of a caller's output gradient dL/dy
      for (int o = 0; o < kOut; ++o) g[o] = dy_in[(size_t)row * kOut + o];
    } else {
      float scale = 2.0f / (float(B) * kOut);
      for (int o = 0; o < kOut; ++o) {
        float d = out[o] - target[(size_t)row * kOut + o];
        g[o] = scale * d;
        l += d * d;
      }
    }
    if (lane == 0) {
      if (!dy_in) loss_rows[row] = l;
      for (int o = 0; o < kOut; ++o) {
        gy[(size_t)row * kOut + o] = g[o];
        gs[rr][o] = g[o];
      }
    }
  }
  if (!train) return;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kZPer; ++j) {
    const int i = threadIdx.x + 256 * j, k = i / kHeadRows, rr = i - k * kHeadRows;
    if (rr >= nr) continue;
    float s = 0.f;
    for (int o = 0; o < kOut; ++o) s += gs[rr][o] * (float)W4[o * kHid + k];
    const bf16 v = (bf16)(s * gelu_grad(zv[j]));
    g4T[(size_t)k * ldT + row0 + rr] = v;
    tile[rr][k] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHeadRows * (kHid / 8); i += 256) {
    const int rr = i / (kHid / 8), c = (i - rr * (kHid / 8)) * 8;
    if (rr < nr)
      *reinterpret_cast<bf16x8*>(&g4[(size_t)(row0 + rr) * kHid + c]) = *reinterpret_cast<const bf16x8*>(&tile[rr][c]);
  }
}

// The batch loss, the mean of the per-row squared errors over B rows and
// the 3 outputs: 256 threads striding over the rows, then a tree in LDS.
// All 256 threads of a block.
__device__ void loss_sum(const float* __restrict__ rows, int B, float* __restrict__ out) {
  __shared__ float part[256];
  float s = 0.f;
  for (int b = threadIdx.x; b < B; b += 256) s += rows[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0] / (float(B) * kOut);
}

// The gradient reductions of back-propagation in one launch.  Blocks
// [0, blk0[4]) sum the k-split parts of the hidden layers' weight gradients,
// slab by slab in order (256 elements a block, the layers' blocks back to
// back from blk0[l]); the next 4 kHid blocks each sum one hidden bias
// gradient, db_l[n] = sum_b g_l[b][n]; the last 3 (kHid + 1) blocks one of
// the head's, dW4[o][k] = sum_b gy[b][o] a4[b][k] (k = kHid: db4[o] =
// sum_b gy[b][o]); with rows, one more block the batch loss (loss_sum).
// A sum over the batch: 256 threads striding over it, wavefront sums, then
// the four wavefronts' sums in order.
struct GradReduce {
  float* part[4];          // layer l's parts, slab[l] floats each (written by gemm_tn<EpiPart>)
  int slab[4];
  int blk0[5];
  const bf16* gT[4];       // dL/dz of hidden layer l, feature-major
  int parts;
  const float* gy;         // dL/dy [B][3]
  const bf16* a4T;         // last hidden activations, feature-major
  const float* rows;       // per-row squared errors, or null (no loss)
  float* loss;             // the batch loss (mean squared error), if rows
};

__global__ void __launch_bounds__(256) mlp_grad_reduce(GradReduce a, int ldT, int B, float* __restrict__ grad) {
  const int blk = blockIdx.x;
  if (blk < a.blk0[4]) {   // the same branch for the whole block
    int l = 0;
    while (l < 3 && blk >= a.blk0[l + 1]) ++l;
    const int i = (blk - a.blk0[l]) * 256 + (int)threadIdx.x;
    if (i >= a.slab[l]) return;
    float s = 0.f;
#pragma unroll 4
    for (int z = 0; z < a.parts; ++z) s += a.part[l][(size_t)z * a.slab[l] + i];
    grad[kOffW[l] + i] = s;
    return;
  }
  const int q = blk - a.blk0[4];
  if (q == 4 * kHid + kOut * (kHid + 1)) {   // the loss block (launched only with rows)
    loss_sum(a.rows, B, a.loss);
    return;
  }
  __shared__ float red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float s = 0.f;
  int dst;
  if (q < 4 * kHid) {
    const int l = q / kHid, n = q - l * kHid;
    const bf16* g = a.gT[l] + (size_t)n * ldT;
#pragma unroll 4
    for (int b = threadIdx.x; b < B; b += 256) s += (float)g[b];
    dst = kOffB[l] + n;
  } else {
    const int t = q - 4 * kHid, o = t / (kHid + 1), k = t - o * (kHid + 1);
    if (k < kHid) {
      const bf16* x = a.a4T + (size_t)k * ldT;
#pragma unroll 4
      for (int b = threadIdx.x; b < B; b += 256) s += a.gy[(size_t)b * kOut + o] * (float)x[b];
    } else {
#pragma unroll 4
      for (int b = threadIdx.x; b < B; b += 256) s += a.gy[(size_t)b * kOut + o];
    }
    dst = k < kHid ? kOffW[4] + o * kHid + k : kOffB[4] + o;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) red[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) grad[dst] = (red[0] + red[1]) + (red[2] + red[3]);
}


// Parameter i's BF16 copies from its FP32 value: the row-major copy of all
// parameters and, for W1..W3, the transposed copy.
__device__ __forceinline__ void refresh_one(int i, float w, bf16* __restrict__ wb, bf16* __restrict__ wT) {
  const bf16 v = (bf16)w;
  wb[i] = v;
  for (int l = 1; l <= 3; ++l) {
    const int off = kOffW[l];
    if (i >= off && i < off + kHid * kHid) {
      const int r = (i - off) / kHid, c = (i - off) % kHid;     // W_l[r][c], r = out, c = in
      wT[(size_t)(l - 1) * kHid * kHid + (size_t)c * kHid + r] = v;
    }
  }
}

// Adam with bias correction on the FP32 master weights, then their BF16
// copies (one pass over the parameters).
__global__ void mlp_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                         const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2,
                         bf16* __restrict__ wb, bf16* __restrict__ wT) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_N_PARAMS) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.0f - b1) * gi;
  float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  refresh_one(i, wi, wb, wT);
}

// The BF16 copies of all parameters (after they are set).
__global__ void mlp_refresh(const float* __restrict__ w, bf16* __restrict__ wb, bf16* __restrict__ wT) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_N_PARAMS) return;
  refresh_one(i, w[i], wb, wT);
}

// Surrogate inputs from rollout logs: window w of rollout r holds samples
// t = w .. w + window - 1 of (theta, omega, input torque) and the fill ratio,
// each standardised; its target is the wrench at the window's last sample.
//   x [(r * n_win + w)][t * 4 + c],  y [(r * n_win + w)][3],  n_win = T - window + 1.
// per-rollout constants in the fourth input channel (fill ratio, tank
// descriptors), at most this many
constexpr int kMaxStatic = 8;

struct WinNorm {
  float in_mean[3 + kMaxStatic], in_inv[3 + kMaxStatic], out_mean[3], out_inv[3], out_std[3];
};

__global__ void mlp_windows(const float* __restrict__ feat, const float* __restrict__ stat, int n_static,
                            const float* __restrict__ wrench, int R, int T, int window, WinNorm nm,
                            float* __restrict__ x, float* __restrict__ y) {
  const int n_win = T - window + 1;
  const long long width = (long long)window * 4;
  const long long total = (long long)R * n_win * width;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  long long row = e / width;
  int k = (int)(e - row * width);
  int ti = k >> 2, c = k & 3;
  int r = (int)(row / n_win), w = (int)(row - (long long)r * n_win);
  int t = w + ti;
  // channel 3 of sample ti carries the rollout's constant ti % n_static
  const int q = c < 3 ? c : 3 + ti % n_static;
  float v = c < 3 ? feat[((size_t)r * T + t) * 3 + c] : stat[(size_t)r * n_static + (q - 3)];
  x[e] = (v - nm.in_mean[q]) * nm.in_inv[q];
  if (y && k < 3) {
    float o = wrench[((size_t)r * T + w + window - 1) * 3 + k];
    y[row * 3 + k] = (o - nm.out_mean[k]) * nm.out_inv[k];
  }
}

// Window width of the coupled rollout: the network's 128 inputs are 32
// samples of 4 channels.
constexpr int kWin = kIn / 4;

// Rollouts per workgroup of the coupled rollout: one row tile, so that a few
// hundred rollouts spread over as many CUs (each interval's network work per
// wave is a quarter of a 64-row tile's).
constexpr int kCRows = 16;

// The rigid body of kCRows rollouts per workgroup driven by the network, all
// log intervals in one launch (the rollouts are independent).  Per interval
// k: the window of samples k - 31 .. k, standardised from a ring of the last
// 32 samples in LDS (mlp_windows' layout; an input further than z_max
// standard deviations from the training mean, or not a number, sets
// MLP_FLAG_OUT_OF_RANGE); the network on MFMA; then thread r integrates its
// rollout over the interval's steps with the de-standardised wrench held:
// eq. tankdynamics without an attitude law, first-order symplectic Euler
// (Section 3.4; velocities first, then positions with the new velocities),
// and logs sample k + 1 (state; theta, thetadot, the input torque of the
// sample's step, also into the ring).
// The network on a 16-row tile, out of line: inlined into the coupled
// rollout's time loop, its weight requests made ahead took every register
// and spilled (512 registers a lane and 412 B of scratch); as a call, 134.
__device__ __attribute__((noinline)) void net16(bf16 (*buf)[kCRows * kLdsStride], const bf16* __restrict__ wb,
                                              const float* __restrict__ master, const bf16* w4s, float* hout) {
  net_rows<kCRows>(buf, wb, master, w4s, [&](int r, int o, float v) { hout[r * kOut + o] = v; });
}

__global__ void __launch_bounds__(256) mlp_coupled(const float* __restrict__ stat, int n_static, int R, int T,
                                                   WinNorm nm, float z_max, const double* __restrict__ body,
                                                   const float* __restrict__ u_seq, int n_steps, int stride,
                                                   const bf16* __restrict__ wb, const float* __restrict__ master,
                                                   double* __restrict__ rigid, float* __restrict__ feat,
                                                   float* __restrict__ y_log, float* __restrict__ w_log,
                                                   unsigned* __restrict__ flags) {
  __shared__ __align__(16) bf16 buf[2][kCRows * kLdsStride];
  __shared__ float ring[kCRows][kWin][3];
  __shared__ float hout[kCRows * kOut];
  __shared__ unsigned fl[kCRows];
  __shared__ __align__(16) bf16 w4s[kOut * kHid];
  const int row0 = blockIdx.x * kCRows, t = threadIdx.x;
  stage_head(wb, w4s);
  for (int e = t; e < kCRows * kWin * 3; e += 256) {
    const int r = e / (kWin * 3), q = e - r * (kWin * 3);
    const int m = row0 + r;
    ring[r][q / 3][q % 3] = m < R ? feat[((size_t)m * T + q / 3) * 3 + q % 3] : 0.0f;
  }
  if (t < kCRows) fl[t] = 0u;
  const int mine = row0 + t;
  const bool owner = t < kCRows && mine < R;
  double x0 = 0.0, x1 = 0.0, th = 0.0, v0 = 0.0, v1 = 0.0, om = 0.0, mass = 1.0, inertia = 1.0, dt = 0.0;
  if (owner) {
    const double* st = rigid + 6 * (size_t)mine;
    x0 = st[0];
    x1 = st[1];
    th = st[2];
    v0 = st[3];
    v1 = st[4];
    om = st[5];
    mass = body[3 * (size_t)mine];
    inertia = body[3 * (size_t)mine + 1];
    dt = body[3 * (size_t)mine + 2];
  }
  __syncthreads();
  for (int k = kWin - 1; k < T; ++k) {
    for (int e = t; e < kCRows * kIn; e += 256) {
      const int r = e / kIn, kk = e - r * kIn;
      const int ti = kk >> 2, c = kk & 3;
      const int m = row0 + r;
      const int q = c < 3 ? c : 3 + ti % n_static;
      float z = 0.0f;
      if (m < R) {
        const float v = c < 3 ? ring[r][(k - kWin + 1 + ti) % kWin][c] : stat[(size_t)m * n_static + (q - 3)];
        z = (v - nm.in_mean[q]) * nm.in_inv[q];
        if (!(fabsf(z) <= z_max)) atomicOr(&fl[r], MLP_FLAG_OUT_OF_RANGE);
      }
      buf[0][r * kLdsStride + kk] = (bf16)z;
    }
    __syncthreads();
    net16(buf, wb, master, w4s, hout);
    __syncthreads();
    if (owner) {
      double F[3];
      for (int d = 0; d < 3; ++d) {
        const float f = hout[t * kOut + d] * nm.out_std[d] + nm.out_mean[d];
        F[d] = (double)f;
        w_log[((size_t)mine * T + k) * 3 + d] = f;
      }
      const int n0 = k * stride, n1 = n0 + stride < n_steps ? n0 + stride : n_steps;
      for (int n = n0; n < n1; ++n) {
        const float* u = u_seq + ((size_t)mine * n_steps + n) * 3;
        double sn, cs;
        sincos(th, &sn, &cs);
        const double a0 = (cs * F[0] - sn * F[1] + (double)u[0]) / mass;
        const double a1 = (sn * F[0] + cs * F[1] + (double)u[1]) / mass;
        const double a2 = (F[2] + (double)u[2]) / inertia;
        v0 += dt * a0;
        v1 += dt * a1;
        om += dt * a2;
        x0 += dt * v0;
        x1 += dt * v1;
        th += dt * om;
      }
      if (k + 1 < T) {
        float* y = y_log + ((size_t)mine * T + k + 1) * 6;
        y[0] = (float)x0;
        y[1] = (float)x1;
        y[2] = (float)th;
        y[3] = (float)v0;
        y[4] = (float)v1;
        y[5] = (float)om;
        const float f0 = (float)th, f1 = (float)om;
        const float f2 = u_seq[((size_t)mine * n_steps + (size_t)(k + 1) * stride) * 3 + 2];
        float* f = feat + ((size_t)mine * T + k + 1) * 3;
        f[0] = f0;
        f[1] = f1;
        f[2] = f2;
        float* g = ring[t][(k + 1) % kWin];
        g[0] = f0;
        g[1] = f1;
        g[2] = f2;
      }
    }
    __syncthreads();
  }
  if (owner) {
    double* st = rigid + 6 * (size_t)mine;
    st[0] = x0;
    st[1] = x1;
    st[2] = th;
    st[3] = v0;
    st[4] = v1;
    st[5] = om;
    flags[mine] = fl[t];
  }
}

// The norm vector of mlp_make_windows into kernel form; false if a std is
// not positive.
bool win_norm(const float* norm, int n_static, WinNorm* nm) {
  const int ni = 3 + n_static;   // input channels with a mean and a std: theta, thetadot, torque, constants
  for (int c = 0; c < ni; ++c) {
    if (!(norm[ni + c] > 0.0f)) return false;
    nm->in_mean[c] = norm[c];
    nm->in_inv[c] = 1.0f / norm[ni + c];
  }
  for (int c = 0; c < 3; ++c) {
    if (!(norm[2 * ni + 3 + c] > 0.0f)) return false;
    nm->out_mean[c] = norm[2 * ni + c];
    nm->out_std[c] = norm[2 * ni + 3 + c];
    nm->out_inv[c] = 1.0f / norm[2 * ni + 3 + c];
  }
  return true;
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// The network's input rows are read four floats at a time.
bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

struct MlpLayout {
  size_t master, m, v, grad, wb, wT, xb, xT, act[4], actT[4], zT[4], g[4], gT[4], y, gy, rows,
      loss, part, total;
  int ldT;   // leading dimension of the feature-major (transposed) buffers, a multiple of 32
};

// k-split of the weight gradients: a batch is cut into parts of at least
// 256 rows, at most kMaxParts of them (the 4x4 or 4x2 output tiles of a
// layer alone would occupy a few dozen of the 256 CUs)
constexpr int kMaxParts = 16;

int wgrad_parts(int B) {
  int z = 1;
  while (z < kMaxParts && B % (64 * z) == 0 && B / (2 * z) >= 256) z *= 2;
  return z;
}

MlpLayout mlp_layout(int maxB) {
  MlpLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += al(bytes > 0 ? bytes : 1);
    return at;
  };
  size_t B = (size_t)maxB, P = MLP_N_PARAMS;
  L.ldT = (maxB + 31) & ~31;
  size_t BT = (size_t)L.ldT;
  L.master = take(P * 4);
  L.m = take(P * 4);
  L.v = take(P * 4);
  L.grad = take(P * 4);
  L.wb = take(P * 2);
  L.wT = take((size_t)3 * kHid * kHid * 2);
  L.xb = take(B * kIn * 2);
  L.xT = take(BT * kIn * 2);
  for (int l = 0; l < 4; ++l) {
    L.act[l] = take(B * kHid * 2);
    L.actT[l] = take(BT * kHid * 2);
    L.zT[l] = take(BT * kHid * 4);
    L.g[l] = take(B * kHid * 2);
    L.gT[l] = take(BT * kHid * 2);
  }
  L.y = take(B * kOut * 4);
  L.gy = take(B * kOut * 4);
  L.rows = take(B * 4);
  L.loss = take(4);
  L.part = take((size_t)kMaxParts * kHid * (kIn + 3 * kHid) * 4);   // every hidden layer's parts
  L.total = o;
  return L;
}

thread_local char m_err[256];

int mlp_hip_fail(hipError_t e, const char* what) {
  snprintf(m_err, sizeof m_err, "%s: %s", what, hipGetErrorString(e));
  return SPH_E_HIP;
}

#define MHIP(x)                                        \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return mlp_hip_fail(e_, #x); \
  } while (0)

}  // namespace

struct mlp_handle {
  int maxB;
  hipStream_t stream;
  char* ws;
  MlpLayout L;
  long long t;   // Adam step counter
  template <class T>
  T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
};

namespace {

// Forward through the four hidden layers; training keeps transposes and z.
void forward(mlp_handle* h, const float* x, int B, bool train) {
  const int ldT = h->L.ldT;
  hipLaunchKernelGGL(mlp_cast_input, dim3((B + kCastRows - 1) / kCastRows), dim3(256), 0, h->stream, x, B,
                     h->at<bf16>(h->L.xb), train ? h->at<bf16>(h->L.xT) : nullptr, ldT);
  const bf16* a = h->at<bf16>(h->L.xb);
  int lda = kIn;
  for (int l = 0; l < 4; ++l) {
    EpiFwd e;
    e.bias = h->at<float>(h->L.master) + kOffB[l];
    e.act = h->at<bf16>(h->L.act[l]);
    e.ld_act = kHid;
    e.actT = train ? h->at<bf16>(h->L.actT[l]) : nullptr;
    e.zT = train ? h->at<float>(h->L.zT[l]) : nullptr;
    e.ldT = ldT;
    dim3 grid((kHid + 63) / 64, (B + 63) / 64);
    hipLaunchKernelGGL(gemm_tn<EpiFwd>, grid, dim3(256), 0, h->stream, a, lda,
                       h->at<bf16>(h->L.wb) + kOffW[l], kDims[l], B, kHid, kDims[l], e);
    a = e.act;
    lda = kHid;
  }
}

}  // namespace

extern "C" {

int mlp_workspace_bytes(int32_t max_batch, size_t* bytes) {
  if (max_batch < 1 || max_batch > (1 << 24) || !bytes) return SPH_E_INVAL;
  *bytes = mlp_layout(max_batch).total;
  return SPH_OK;
}

int mlp_init(const float* params_dev, int32_t max_batch, void* ws_dev, size_t ws_bytes, void* stream,
             mlp_handle** out) {
  if (!out || !params_dev || !ws_dev || max_batch < 1 || max_batch > (1 << 24)) return SPH_E_INVAL;
  if (reinterpret_cast<uintptr_t>(ws_dev) & 255) return SPH_E_INVAL;
  MlpLayout L = mlp_layout(max_batch);
  if (ws_bytes < L.total) return SPH_E_CAPACITY;
  mlp_handle* h = new (std::nothrow) mlp_handle();
  if (!h) return SPH_E_INVAL;
  h->maxB = max_batch;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->ws = reinterpret_cast<char*>(ws_dev);
  h->L = L;
  h->t = 0;
  hipError_t e = hipMemsetAsync(h->ws, 0, L.total, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->at<float>(L.master), params_dev, (size_t)MLP_N_PARAMS * 4,
                       hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) {
    delete h;
    return mlp_hip_fail(e, "mlp_init copy");
  }
  hipLaunchKernelGGL(mlp_refresh, dim3((MLP_N_PARAMS + 255) / 256), dim3(256), 0, h->stream,
                     h->at<float>(L.master), h->at<bf16>(L.wb), h->at<bf16>(L.wT));
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return mlp_hip_fail(e, "mlp_init");
  }
  *out = h;
  return SPH_OK;
}

int mlp_destroy(mlp_handle* h) {
  if (!h) return SPH_E_INVAL;
  delete h;
  return SPH_OK;
}

int mlp_forward(mlp_handle* h, const float* x_dev, int32_t batch, float* y_dev) {
  if (!h || !x_dev || !y_dev || batch < 1 || batch > h->maxB || !aligned16(x_dev)) return SPH_E_INVAL;
  hipLaunchKernelGGL(mlp_forward_fused, dim3((batch + kRows - 1) / kRows), dim3(256), 0, h->stream, x_dev,
                     batch, h->at<bf16>(h->L.wb), h->at<float>(h->L.master), y_dev);
  MHIP(hipGetLastError());
  return SPH_OK;
}

}  // extern "C"

namespace {

// Forward with the activations kept, then back-propagation into the
// handle's gradient buffer, from the mean-squared-error gradient against
// target (the batch loss into loss_dev, if given) or from a given dL/dy.
void run_backward(mlp_handle* h, const float* x_dev, const float* target_dev, const float* dy_dev, int B,
                  float* loss_dev = nullptr) {
  const int ldT = h->L.ldT;
  forward(h, x_dev, B, true);
  float* grad = h->at<float>(h->L.grad);
  hipLaunchKernelGGL(mlp_head, dim3((B + kHeadRows - 1) / kHeadRows), dim3(256), 0, h->stream, h->at<bf16>(h->L.act[3]),
                     h->at<bf16>(h->L.wb) + kOffW[4], h->at<float>(h->L.master) + kOffB[4], B,
                     h->at<float>(h->L.y), target_dev, h->at<float>(h->L.gy), h->at<float>(h->L.rows),
                     h->at<float>(h->L.zT[3]), h->at<bf16>(h->L.g[3]), h->at<bf16>(h->L.gT[3]), ldT, dy_dev);
  // hidden layers, top down: g[l] holds dL/dz of hidden layer l (output of
  // W_l); each layer's weight gradient in k-split parts, reduced with the
  // bias gradients in one launch at the end
  const int parts = wgrad_parts(B);
  GradReduce gr;
  gr.parts = parts;
  gr.gy = h->at<float>(h->L.gy);
  gr.a4T = h->at<bf16>(h->L.actT[3]);
  gr.rows = loss_dev ? h->at<float>(h->L.rows) : nullptr;
  gr.loss = loss_dev;
  gr.blk0[0] = 0;
  size_t off = 0;
  for (int l = 0; l < 4; ++l) {
    gr.slab[l] = kHid * kDims[l];
    gr.part[l] = h->at<float>(h->L.part) + off;
    gr.gT[l] = h->at<bf16>(h->L.gT[l]);
    gr.blk0[l + 1] = gr.blk0[l] + (gr.slab[l] + 255) / 256;
    off += (size_t)kMaxParts * gr.slab[l];
  }
  for (int l = 3; l >= 0; --l) {
    const bf16* aT = l > 0 ? h->at<bf16>(h->L.actT[l - 1]) : h->at<bf16>(h->L.xT);
    EpiPart ep{gr.part[l], kDims[l], (size_t)gr.slab[l]};
    dim3 gw((kDims[l] + 63) / 64, (kHid + 63) / 64, parts);
    hipLaunchKernelGGL(gemm_tn<EpiPart>, gw, dim3(256), 0, h->stream, h->at<bf16>(h->L.gT[l]), ldT, aT,
                       ldT, kHid, kDims[l], B, ep);
    if (l > 0) {
      EpiDgrad ed;
      ed.zT = h->at<float>(h->L.zT[l - 1]);
      ed.g = h->at<bf16>(h->L.g[l - 1]);
      ed.ld_g = kHid;
      ed.gT = h->at<bf16>(h->L.gT[l - 1]);
      ed.ldT = ldT;
      dim3 gd((kHid + 63) / 64, (B + 63) / 64);
      hipLaunchKernelGGL(gemm_tn<EpiDgrad>, gd, dim3(256), 0, h->stream, h->at<bf16>(h->L.g[l]), kHid,
                         h->at<bf16>(h->L.wT) + (size_t)(l - 1) * kHid * kHid, kHid, B, kHid, kHid, ed);
    }
  }
  hipLaunchKernelGGL(mlp_grad_reduce, dim3(gr.blk0[4] + 4 * kHid + kOut * (kHid + 1) + (loss_dev ? 1 : 0)), dim3(256),
                     0, h->stream, gr, ldT, B, grad);
}

// Adam with bias correction at step t on the master weights from grad, then
// the BF16 copies refreshed.
void run_adam(mlp_handle* h, const float* grad, float lr, float beta1, float beta2, float eps, long long t) {
  float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
  hipLaunchKernelGGL(mlp_adam, dim3((MLP_N_PARAMS + 255) / 256), dim3(256), 0, h->stream,
                     h->at<float>(h->L.master), h->at<float>(h->L.m), h->at<float>(h->L.v), grad, lr, beta1,
                     beta2, eps, c1, c2, h->at<bf16>(h->L.wb), h->at<bf16>(h->L.wT));
}

bool train_batch_ok(const mlp_handle* h, int batch) {
  return batch >= 32 && batch <= h->maxB && batch % 32 == 0;
}

}  // namespace

extern "C" {

int mlp_train_step(mlp_handle* h, const float* x_dev, const float* target_dev, int32_t batch, float lr,
                   float beta1, float beta2, float eps, float* grad_dev, float* loss_dev) {
  if (!h || !x_dev || !target_dev || !train_batch_ok(h, batch) || !aligned16(x_dev)) return SPH_E_INVAL;
  const int B = batch;
  run_backward(h, x_dev, target_dev, nullptr, B, loss_dev ? loss_dev : h->at<float>(h->L.loss));
  float* grad = h->at<float>(h->L.grad);
  if (grad_dev)
    MHIP(hipMemcpyAsync(grad_dev, grad, (size_t)MLP_N_PARAMS * 4, hipMemcpyDeviceToDevice, h->stream));
  h->t += 1;
  run_adam(h, grad, lr, beta1, beta2, eps, h->t);
  MHIP(hipGetLastError());
  return SPH_OK;
}

int mlp_backward(mlp_handle* h, const float* x_dev, const float* dy_dev, int32_t batch, float* grads_dev) {
  if (!h || !x_dev || !dy_dev || !grads_dev || !train_batch_ok(h, batch) || !aligned16(x_dev)) return SPH_E_INVAL;
  run_backward(h, x_dev, nullptr, dy_dev, batch);
  MHIP(hipMemcpyAsync(grads_dev, h->at<float>(h->L.grad), (size_t)MLP_N_PARAMS * 4, hipMemcpyDeviceToDevice,
                      h->stream));
  MHIP(hipGetLastError());
  return SPH_OK;
}

int mlp_adam_step(mlp_handle* h, const float* grads_dev, float lr, float beta1, float beta2, float eps,
                  int32_t t) {
  if (!h || !grads_dev || t < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return SPH_E_INVAL;
  run_adam(h, grads_dev, lr, beta1, beta2, eps, t);
  h->t = t;
  MHIP(hipGetLastError());
  return SPH_OK;
}

int mlp_make_windows(const float* feat_dev, const float* static_dev, int32_t n_static, const float* wrench_dev,
                     int32_t n_roll, int32_t n_t, int32_t window, const float* norm, float* x_dev, float* y_dev,
                     void* stream) {
  if (!feat_dev || !static_dev || !norm || !x_dev || n_roll < 1 || window < 1 || n_t < window) return SPH_E_INVAL;
  if (n_static < 1 || n_static > kMaxStatic || n_static > window) return SPH_E_INVAL;
  if (y_dev && !wrench_dev) return SPH_E_INVAL;
  WinNorm nm;
  if (!win_norm(norm, n_static, &nm)) return SPH_E_INVAL;
  long long total = (long long)n_roll * (n_t - window + 1) * window * 4;
  long long blocks = (total + 255) / 256;
  if (blocks > 0x7fffffffLL) return SPH_E_INVAL;
  hipLaunchKernelGGL(mlp_windows, dim3((unsigned)blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     feat_dev, static_dev, n_static, wrench_dev, n_roll, n_t, window, nm, x_dev, y_dev);
  MHIP(hipGetLastError());
  return SPH_OK;
}

int mlp_coupled_rollout(mlp_handle* h, int32_t n_roll, int32_t n_steps, int32_t log_stride, int32_t window,
                        const double* body_dev, const float* u_seq_dev, const float* static_dev, int32_t n_static,
                        const float* norm, float z_max, double* rigid_dev, float* feat_dev, float* y_log_dev,
                        float* wrench_log_dev, uint32_t* flags_dev) {
  if (!h || !body_dev || !u_seq_dev || !static_dev || !norm || !rigid_dev || !feat_dev || !y_log_dev ||
      !wrench_log_dev || !flags_dev)
    return SPH_E_INVAL;
  if (window != kWin || n_roll < 1 || n_roll > h->maxB || log_stride < 1 || n_steps < 1) return SPH_E_INVAL;
  if (n_static < 1 || n_static > kMaxStatic || !(z_max > 0.0f)) return SPH_E_INVAL;
  const long long T = ((long long)n_steps + log_stride - 1) / log_stride;
  if (T < window || (long long)n_roll * T * 6 > 0x7fffffffLL || (long long)n_roll * n_steps * 3 > 0x7fffffffLL)
    return SPH_E_INVAL;
  WinNorm nm;
  if (!win_norm(norm, n_static, &nm)) return SPH_E_INVAL;
  hipLaunchKernelGGL(mlp_coupled, dim3((n_roll + kCRows - 1) / kCRows), dim3(256), 0, h->stream, static_dev,
                     n_static, n_roll, (int)T, nm, z_max, body_dev, u_seq_dev, n_steps, log_stride,
                     h->at<bf16>(h->L.wb), h->at<float>(h->L.master), rigid_dev, feat_dev, y_log_dev,
                     wrench_log_dev, flags_dev);
  MHIP(hipGetLastError());
  return SPH_OK;
}

int mlp_get_params(mlp_handle* h, float* params_dev) {
  if (!h || !params_dev) return SPH_E_INVAL;
  MHIP(hipMemcpyAsync(params_dev, h->at<float>(h->L.master), (size_t)MLP_N_PARAMS * 4,
                      hipMemcpyDeviceToDevice, h->stream));
  return SPH_OK;
}

}  // extern "C"
