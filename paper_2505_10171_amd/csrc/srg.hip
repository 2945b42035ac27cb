// srg.hip -- BF16 matrix-core training and inference of the run-outcome
// surrogate (see include/srg.h) for gfx950.
//
// Every layer product is one GEMM kernel: a 64x64 output tile per 256-thread
// workgroup, K in steps of 32 staged through LDS (both operands stored with K
// contiguous, so each lane reads its eight-element fragment with one 16-byte
// LDS load), and each of the four waves accumulating a 32x32 sub-tile with
// four v_mfma_f32_16x16x32_bf16 per K step.  The forward products read a BF16
// copy of each weight matrix kept transposed (N x K), so both operands stage
// with 16-byte copies; the backward products transpose W^T (dX) and X^T (dW)
// while staging.  Epilogues fuse the bias, the ReLU and the ReLU derivative.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <random>
#include <vector>

#include "../../include/lbm.h"
#include "../../include/srg.h"

namespace srg {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NL = 5;                                  // layers
constexpr int KIN[NL] = {32, 256, 256, 256, 256};      // padded fan-in
constexpr int NOUT[NL] = {256, 256, 256, 256, 64};     // padded fan-out
constexpr int KREAL[NL] = {SRG_IN, 256, 256, 256, 256};
constexpr int NREAL[NL] = {256, 256, 256, 256, SRG_OUT};
constexpr int NCLS = 3, NTRAJ = 48;
constexpr int ALIGN = 256;

enum { EPI_RELU_BF16 = 0, EPI_LINEAR_F32 = 1, EPI_DRELU_BF16 = 2, EPI_F32 = 3 };

// C[M x N] = A[M x K] * B[K x N].  TA: A stored as [K x M] (lda = its row
// length); TB: B stored as [N x K].  M, N multiples of 8 (rows/columns outside
// are skipped), K a multiple of 32.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const bf16* __restrict__ A,
                                              int lda, const bf16* __restrict__ B, int ldb,
                                              const float* __restrict__ bias,
                                              const bf16* __restrict__ act, int ldact,
                                              bf16* __restrict__ Cb, float* __restrict__ Cf,
                                              int ldc) {
  constexpr int LD = 40;  // LDS row: 32 K values + 8 padding (80 bytes)
  __shared__ __attribute__((aligned(16))) bf16 As[64 * LD];
  __shared__ __attribute__((aligned(16))) bf16 Bs[64 * LD];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bf16x8 zero8 = {};
  for (int k0 = 0; k0 < K; k0 += 32) {
    __syncthreads();
    // stage A tile (64 rows of M, 32 of K)
    if (!TA) {
      const int r = t >> 2, kc = (t & 3) * 8;
      bf16x8 v = zero8;
      if (m0 + r < M) v = *(const bf16x8*)(A + (long long)(m0 + r) * lda + k0 + kc);
      *(bf16x8*)(As + r * LD + kc) = v;
    } else {
      const int k = t >> 3, mc = (t & 7) * 8;
      bf16x8 v = zero8;
      if (m0 + mc < M) v = *(const bf16x8*)(A + (long long)(k0 + k) * lda + m0 + mc);
#pragma unroll
      for (int j = 0; j < 8; ++j) As[(mc + j) * LD + k] = v[j];
    }
    // stage B tile (64 columns of N, 32 of K), stored column-major in LDS
    if (TB) {
      const int r = t >> 2, kc = (t & 3) * 8;
      bf16x8 v = zero8;
      if (n0 + r < N) v = *(const bf16x8*)(B + (long long)(n0 + r) * ldb + k0 + kc);
      *(bf16x8*)(Bs + r * LD + kc) = v;
    } else {
      const int k = t >> 3, nc = (t & 7) * 8;
      bf16x8 v = zero8;
      if (n0 + nc < N) v = *(const bf16x8*)(B + (long long)(k0 + k) * ldb + n0 + nc);
#pragma unroll
      for (int j = 0; j < 8; ++j) Bs[(nc + j) * LD + k] = v[j];
    }
    __syncthreads();
    // lane l: row (l % 16) of each 16-row block, K elements (l / 16) * 8 .. + 7
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8*)(As + (wm + i * 16 + fr) * LD + fk);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8*)(Bs + (wn + j * 16 + fr) * LD + fk);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  // lane l holds C rows (l / 16) * 4 + r (r = 0..3) of column l % 16 per block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + j * 16 + (lane & 15);
      if (n >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
        if (m >= M) continue;
        const float c = acc[i][j][r];
        const long long o = (long long)m * ldc + n;
        if (EPI == EPI_RELU_BF16) {
          Cb[o] = (bf16)fmaxf(c + bias[n], 0.f);
        } else if (EPI == EPI_LINEAR_F32) {
          Cf[o] = c + bias[n];
        } else if (EPI == EPI_DRELU_BF16) {
          Cb[o] = (bf16)((float)act[(long long)m * ldact + n] > 0.f ? c : 0.f);
        } else {
          Cf[o] = c;
        }
      }
    }
}

// Forward product on larger tiles: C[M x N] = A[M x K] * B^T with A and B both
// K-contiguous (B stored N x K), M and N multiples of 128, K of 32.  A
// workgroup computes a 128x128 tile, each wave a 64x64 sub-tile with
// v_mfma_f32_32x32x16_bf16 (twice the FLOPs per LDS fragment of the 16x16x32
// form); the next K step's tiles are fetched into registers while the current
// one is multiplied.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_big(int M, int N, int K, const bf16* __restrict__ A,
                                                  int lda, const bf16* __restrict__ B, int ldb,
                                                  const float* __restrict__ bias,
                                                  bf16* __restrict__ Cb, float* __restrict__ Cf,
                                                  int ldc) {
  constexpr int LD = 40;
  __shared__ __attribute__((aligned(16))) bf16 As[128 * LD];
  __shared__ __attribute__((aligned(16))) bf16 Bs[128 * LD];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * 128, n0 = blockIdx.x * 128;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  // staging: thread t moves rows r0 and r0 + 64 of both tiles, chunk kc
  const int r0 = t >> 2, kc = (t & 3) * 8;
  const bf16* a0 = A + (long long)(m0 + r0) * lda + kc;
  const bf16* a1 = A + (long long)(m0 + r0 + 64) * lda + kc;
  const bf16* b0 = B + (long long)(n0 + r0) * ldb + kc;
  const bf16* b1 = B + (long long)(n0 + r0 + 64) * ldb + kc;
  bf16x8 pa0 = *(const bf16x8*)a0, pa1 = *(const bf16x8*)a1;
  bf16x8 pb0 = *(const bf16x8*)b0, pb1 = *(const bf16x8*)b1;
  // 32x32x16 fragments: lane l holds row (col) l % 32, K elements (l / 32) * 8 .. + 7
  const int fr = lane & 31, fk = (lane >> 5) * 8;
  for (int k0 = 0; k0 < K; k0 += 32) {
    __syncthreads();
    *(bf16x8*)(As + r0 * LD + kc) = pa0;
    *(bf16x8*)(As + (r0 + 64) * LD + kc) = pa1;
    *(bf16x8*)(Bs + r0 * LD + kc) = pb0;
    *(bf16x8*)(Bs + (r0 + 64) * LD + kc) = pb1;
    __syncthreads();
    if (k0 + 32 < K) {  // next tiles in flight during this step's products
      pa0 = *(const bf16x8*)(a0 + k0 + 32);
      pa1 = *(const bf16x8*)(a1 + k0 + 32);
      pb0 = *(const bf16x8*)(b0 + k0 + 32);
      pb1 = *(const bf16x8*)(b1 + k0 + 32);
    }
#pragma unroll
    for (int ks = 0; ks < 32; ks += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8*)(As + (wm + i * 32 + fr) * LD + ks + fk);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8*)(Bs + (wn + j * 32 + fr) * LD + ks + fk);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // lane l holds rows (r / 4) * 8 + (l / 32) * 4 + r % 4 (r = 0..15) of column l % 32
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + j * 32 + (lane & 31);
      const float bn = bias[n];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const long long o = (long long)m * ldc + n;
        const float c = acc[i][j][r] + bn;
        if (EPI == EPI_RELU_BF16)
          Cb[o] = (bf16)fmaxf(c, 0.f);
        else
          Cf[o] = c;
      }
    }
}

// Whole forward pass of 128 rows per workgroup.  The activations (128 x 256
// BF16, 64 KB) stay in LDS through the five layers.  The transposed weights
// (N x K per layer) are staged in LDS in slices of 64 K values, shared by the
// four waves; all slices of a layer are requested at its start and staged in
// turn.  Products use v_mfma_f32_32x32x16_bf16.  Row r of the activations
// keeps its 16-byte chunk c at position c ^ (r % 32), so that the 32 rows of an
// A fragment read distinct banks; weight-slice rows are padded to 144 bytes.
struct MlpArgs {
  const bf16* W[NL];    // transposed weights of each layer (NOUT x KIN)
  const float* b[NL];   // biases
};

constexpr int MLP_KS = 64;           // K values per weight slice
constexpr int MLP_LDW = MLP_KS + 8;  // LDS row of a weight slice (BF16)
// dynamic LDS: activations, then two weight slices of up to 256 rows
constexpr size_t MLP_LDS = (size_t)128 * 256 * 2 + (size_t)2 * 256 * MLP_LDW * 2;

__device__ __forceinline__ bf16* mlp_row(bf16* act, int row, int chunk) {
  return act + row * 256 + ((chunk ^ (row & 31)) << 3);
}

// slice s of W (NN x K) into registers: 16-byte chunks q = t + 256 j
template <int K, int NN>
__device__ __forceinline__ void mlp_fetch(const bf16* __restrict__ W, int s, int t, bf16x8* v) {
  constexpr int KS = K < MLP_KS ? K : MLP_KS, CPR = KS / 8, TOT = NN * CPR;
#pragma unroll
  for (int j = 0; j < (TOT + 255) / 256; ++j) {
    const int q = t + 256 * j;
    if (q < TOT) v[j] = *(const bf16x8*)(W + (long long)(q / CPR) * K + s * KS + (q % CPR) * 8);
  }
}
template <int K, int NN>
__device__ __forceinline__ void mlp_stage(bf16* wb, int t, const bf16x8* v) {
  constexpr int KS = K < MLP_KS ? K : MLP_KS, CPR = KS / 8, TOT = NN * CPR;
#pragma unroll
  for (int j = 0; j < (TOT + 255) / 256; ++j) {
    const int q = t + 256 * j;
    if (q < TOT) *(bf16x8*)(wb + (q / CPR) * MLP_LDW + (q % CPR) * 8) = v[j];
  }
}

// hidden layer: act (128 x K) -> relu(act W^T + b) (128 x 256), in place;
// wave w computes columns [64 w, 64 w + 64) of all 128 rows
template <int K>
__device__ __forceinline__ void mlp_hidden(bf16* act, bf16* wbuf, const bf16* __restrict__ W,
                                           const float* __restrict__ bias, int t) {
  constexpr int KS = K < MLP_KS ? K : MLP_KS, NS = K / KS;
  const int lane = t & 63, w = t >> 6, fr = lane & 31, fk = lane >> 5;
  f32x16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  // every slice of the layer requested at once (one wave per SIMD leaves the
  // registers for it); each is staged when its turn comes
  bf16x8 v[NS][8];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) mlp_fetch<K, 256>(W, sl, t, v[sl]);
  mlp_stage<K, 256>(wbuf, t, v[0]);
  __syncthreads();
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const bf16* wb = wbuf + (sl & 1) * 256 * MLP_LDW;
#pragma unroll
    for (int ks = 0; ks < KS; ks += 16) {
      const bf16x8 b0 = *(const bf16x8*)(wb + (64 * w + fr) * MLP_LDW + ks + fk * 8);
      const bf16x8 b1 = *(const bf16x8*)(wb + (64 * w + 32 + fr) * MLP_LDW + ks + fk * 8);
      const int ch = ((sl * KS + ks) >> 3) + fk;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bf16x8 a = *(const bf16x8*)mlp_row(act, 32 * i + fr, ch);
        acc[i][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc[i][0], 0, 0, 0);
        acc[i][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc[i][1], 0, 0, 0);
      }
    }
    __syncthreads();  // every wave is done with this slice (and, last, with act)
    if (sl + 1 < NS) {
      mlp_stage<K, 256>(wbuf + ((sl + 1) & 1) * 256 * MLP_LDW, t, v[sl + 1]);
      __syncthreads();
    }
  }
  // lane l holds rows (r / 4) * 8 + (l / 32) * 4 + r % 4 of column l % 32
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = 64 * w + 32 * j + fr;
    const float bn = bias[n];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * i + (r >> 2) * 8 + fk * 4 + (r & 3);
        mlp_row(act, row, n >> 3)[n & 7] = (bf16)fmaxf(acc[i][j][r] + bn, 0.f);
      }
  }
  __syncthreads();
}

// X: n x 6 FP32 rows, y: n x 51 FP32 rows; rows from n on are computed on zero
// inputs and not written
__global__ __launch_bounds__(256) void k_mlp(const float* __restrict__ X, int n, MlpArgs a,
                                             float* __restrict__ y) {
  extern __shared__ __attribute__((aligned(16))) bf16 mlp_lds[];
  bf16* act = mlp_lds;
  bf16* wbuf = mlp_lds + 128 * 256;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.x * 128;
  // inputs padded to 32 features: 128 rows of 4 chunks, the features in chunk 0
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int q = t + 256 * j, row = q >> 2, ch = q & 3;
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (bf16)0.f;
    if (ch == 0 && m0 + row < n) {
      const float* x = X + (long long)(m0 + row) * SRG_IN;
#pragma unroll
      for (int e = 0; e < SRG_IN; ++e) v[e] = (bf16)x[e];
    }
    *(bf16x8*)mlp_row(act, row, ch) = v;
  }
  __syncthreads();
  mlp_hidden<32>(act, wbuf, a.W[0], a.b[0], t);
  mlp_hidden<256>(act, wbuf, a.W[1], a.b[1], t);
  mlp_hidden<256>(act, wbuf, a.W[2], a.b[2], t);
  mlp_hidden<256>(act, wbuf, a.W[3], a.b[3], t);
  // output layer: 64 padded columns; wave w takes rows [32 w, 32 w + 32)
  const int fr = lane & 31, fk = lane >> 5;
  f32x16 acc[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
  constexpr int NS4 = 256 / MLP_KS;
  bf16x8 v[NS4][8];
#pragma unroll
  for (int sl = 0; sl < NS4; ++sl) mlp_fetch<256, 64>(a.W[4], sl, t, v[sl]);
  mlp_stage<256, 64>(wbuf, t, v[0]);
  __syncthreads();
#pragma unroll
  for (int sl = 0; sl < NS4; ++sl) {
    const bf16* wb = wbuf + (sl & 1) * 256 * MLP_LDW;
#pragma unroll
    for (int ks = 0; ks < MLP_KS; ks += 16) {
      const bf16x8 b0 = *(const bf16x8*)(wb + fr * MLP_LDW + ks + fk * 8);
      const bf16x8 b1 = *(const bf16x8*)(wb + (32 + fr) * MLP_LDW + ks + fk * 8);
      const bf16x8 av =
          *(const bf16x8*)mlp_row(act, 32 * w + fr, ((sl * MLP_KS + ks) >> 3) + fk);
      acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, b1, acc[1], 0, 0, 0);
    }
    __syncthreads();
    if (sl + 1 < NS4) {
      mlp_stage<256, 64>(wbuf + ((sl + 1) & 1) * 256 * MLP_LDW, t, v[sl + 1]);
      __syncthreads();
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = 32 * j + fr;
    if (col >= SRG_OUT) continue;
    const float bn = a.b[4][col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + 32 * w + (r >> 2) * 8 + fk * 4 + (r & 3);
      if (row < n) y[(long long)row * SRG_OUT + col] = acc[j][r] + bn;
    }
  }
}

// rows of the training set picked by the permutation, as padded BF16 inputs
__global__ void k_gather(const bf16* __restrict__ Xall, const int* __restrict__ perm, int off,
                         int B, bf16* __restrict__ Xb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * 4) return;
  const int r = t >> 2, c = (t & 3) * 8;
  *(bf16x8*)(Xb + (long long)r * 32 + c) = *(const bf16x8*)(Xall + (long long)perm[off + r] * 32 + c);
}

// loss and its gradient dL/dy (B x 64, BF16, zero in the padding); loss sum in
// acc[0] (atomic).  Sample r of the batch is training row perm[off + r] (perm
// null: row r of lab/traj).
__global__ void k_loss(const float* __restrict__ Y, const int* __restrict__ perm, int off, int B,
                       const int* __restrict__ lab, const float* __restrict__ traj, float w_traj,
                       bf16* __restrict__ dY, float* __restrict__ acc) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (r < B) {
    const int row = perm ? perm[off + r] : r;
    const float* y = Y + (long long)r * 64;
    const float mx = fmaxf(y[0], fmaxf(y[1], y[2]));
    float e[NCLS], se = 0.f;
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
      e[c] = __expf(y[c] - mx);
      se += e[c];
    }
    const int lb = lab[row];
    bf16* d = dY + (long long)r * 64;
    const float invB = 1.0f / (float)B;
#pragma unroll
    for (int c = 0; c < NCLS; ++c) {
      const float p = e[c] / se;
      d[c] = (bf16)((p - (c == lb ? 1.f : 0.f)) * invB);
    }
    l = -(y[lb] - mx - __logf(se));
    const float* tr = traj + (long long)row * NTRAJ;
    const float s = 2.f * w_traj * invB / (float)NTRAJ;
    float se2 = 0.f;
    for (int j = 0; j < NTRAJ; ++j) {
      const float df = y[NCLS + j] - tr[j];
      se2 += df * df;
      d[NCLS + j] = (bf16)(s * df);
    }
    for (int j = NCLS + NTRAJ; j < 64; ++j) d[j] = (bf16)0.f;
    l = (l + w_traj * se2 / (float)NTRAJ) * invB;
  }
  // wave sum, one atomic per wave
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(acc, l);
}

// column sums of a BF16 matrix (bias gradient).  A workgroup takes 64 columns;
// its 16 waves take interleaved groups of 8 rows (eight loads in flight per
// lane), then the 16 partial sums of a column are added in a fixed order.
constexpr int COLSUM_WAVES = 16;
__global__ __launch_bounds__(64 * COLSUM_WAVES) void k_colsum(const bf16* __restrict__ D, int M,
                                                              int N, int ld,
                                                              float* __restrict__ out) {
  __shared__ float part[COLSUM_WAVES][64];
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  float s = 0.f;
  if (n < N) {
    for (int m0 = 8 * w; m0 < M; m0 += 8 * COLSUM_WAVES) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = m0 + u < M ? (float)D[(long long)(m0 + u) * ld + n] : 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
  }
  part[w][c] = s;
  __syncthreads();
  if (w == 0 && n < N) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < COLSUM_WAVES; ++q) t += part[q][c];
    out[n] = t;
  }
}

// Adam on the whole parameter vector; refreshes the BF16 copy
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, bf16* __restrict__ pb, long long n, float lr,
                       float bc1, float bc2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
  p[i] = pi;
  pb[i] = (bf16)pi;
}

// BF16 copy of a weight matrix W (K x N, FP32) stored transposed (N x K), the
// layout the forward product stages without scattering
__global__ void k_transpose_bf16(const float* __restrict__ W, int K, int N, bf16* __restrict__ Wt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * N) return;
  const int n = t / K, k = t - n * K;
  Wt[t] = (bf16)W[(long long)k * N + n];
}

__global__ void k_to_bf16(const float* __restrict__ p, bf16* __restrict__ pb, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = (bf16)p[i];
}

}  // namespace srg

using namespace srg;

namespace {
size_t aup(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t w_off[NL], b_off[NL], n_par;  // offsets (elements) in the padded vector
  size_t t_off[NL], n_wt;              // transposed weight copies (N x K per layer)
  size_t off_p, off_g, off_m, off_v, off_pb, off_pbt, off_xall, off_lab, off_traj, off_perm, off_xb,
      off_act[NL], off_y, off_dy, off_dz[2], off_acc, off_xin, off_yout, total;
};

Layout make_layout(int max_batch, int max_train) {
  Layout L{};
  size_t e = 0;
  for (int l = 0; l < NL; ++l) {
    L.w_off[l] = e;
    e += (size_t)KIN[l] * NOUT[l];
    L.b_off[l] = e;
    e += NOUT[l];
  }
  L.n_par = e;
  size_t t = 0;
  for (int l = 0; l < NL; ++l) {
    L.t_off[l] = t;
    t += (size_t)KIN[l] * NOUT[l];
  }
  L.n_wt = t;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = aup(o + std::max<size_t>(bytes, 1));
    return r;
  };
  L.off_p = take(4 * e);
  L.off_g = take(4 * e);
  L.off_m = take(4 * e);
  L.off_v = take(4 * e);
  L.off_pb = take(2 * e);
  L.off_pbt = take(2 * t);
  L.off_xall = take(2 * 32 * (size_t)max_train);
  L.off_lab = take(4 * (size_t)max_train);
  L.off_traj = take(4 * NTRAJ * (size_t)max_train);
  L.off_perm = take(4 * (size_t)max_train);
  L.off_xb = take(2 * 32 * (size_t)max_batch);
  for (int l = 0; l < NL; ++l) L.off_act[l] = take(2 * 256 * (size_t)max_batch);  // act[0] unused
  L.off_y = take(4 * 64 * (size_t)max_batch);
  L.off_dy = take(2 * 64 * (size_t)max_batch);
  L.off_dz[0] = take(2 * 256 * (size_t)max_batch);
  L.off_dz[1] = take(2 * 256 * (size_t)max_batch);
  L.off_acc = take(64);
  L.off_xin = take(4 * SRG_IN * (size_t)max_batch);
  L.off_yout = take(4 * SRG_OUT * (size_t)max_batch);
  L.total = o;
  return L;
}

uint16_t host_bf16(float f) {  // round to nearest even
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
}  // namespace

struct srg_ctx {
  hipStream_t stream;
  char* ws;
  Layout L;
  int max_batch, max_train, n_train = 0;
  int step = 0;  // Adam step count
  int err = 0;
  char msg[256];
  float* p() { return (float*)(ws + L.off_p); }
  float* g() { return (float*)(ws + L.off_g); }
  bf16* pb() { return (bf16*)(ws + L.off_pb); }
  bf16* pbt() { return (bf16*)(ws + L.off_pbt); }
  bf16* act(int l) { return (bf16*)(ws + L.off_act[l]); }
};

static int srg_err(srg_ctx* c, int code, const char* fmt, ...) {
  if (c && c->err == 0) {
    c->err = code;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->msg, sizeof c->msg, fmt, ap);
    va_end(ap);
  }
  return code;
}

#define SCHK(ctx, call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return srg_err((ctx), LBM_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

static int refresh_transposed(srg_ctx* c);

template <bool TA, bool TB, int EPI>
static hipError_t gemm(hipStream_t st, int M, int N, int K, const bf16* A, int lda, const bf16* B,
                       int ldb, const float* bias, const bf16* act, int ldact, bf16* Cb, float* Cf,
                       int ldc) {
  const dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, bias,
                     act, ldact, Cb, Cf, ldc);
  return hipGetLastError();
}

// inference over n rows of FP32 inputs X (n x 6) to y (n x 51), both on the
// device: the whole pass in one kernel, the activations in LDS
static int infer(srg_ctx* c, const float* X, int n, float* y) {
  MlpArgs a;
  for (int l = 0; l < NL; ++l) {
    a.W[l] = c->pbt() + c->L.t_off[l];
    a.b[l] = c->p() + c->L.b_off[l];
  }
  static bool lds_set = false;  // above 64 KB of LDS needs the attribute once
  if (!lds_set) {
    SCHK(c, hipFuncSetAttribute((const void*)k_mlp, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)MLP_LDS));
    lds_set = true;
  }
  hipLaunchKernelGGL(k_mlp, dim3((n + 127) / 128), dim3(256), MLP_LDS, c->stream, X, n, a, y);
  SCHK(c, hipGetLastError());
  return LBM_OK;
}

// training forward over B rows of packed inputs Xb: output Y and the
// activations act[1..4] that the backward pass reads
static int forward(srg_ctx* c, const bf16* Xb, int B) {
  hipStream_t st = c->stream;
  const float* p = c->p();
  const bf16* in = Xb;
  int ld_in = 32;
  for (int l = 0; l < NL - 1; ++l) {
    if (B % 128 == 0 && NOUT[l] % 128 == 0) {
      hipLaunchKernelGGL((k_gemm_big<EPI_RELU_BF16>), dim3(NOUT[l] / 128, B / 128), dim3(256), 0,
                         st, B, NOUT[l], KIN[l], in, ld_in, c->pbt() + c->L.t_off[l], KIN[l],
                         p + c->L.b_off[l], c->act(l + 1), nullptr, 256);
      SCHK(c, hipGetLastError());
    } else {
      SCHK(c, (gemm<false, true, EPI_RELU_BF16>(st, B, NOUT[l], KIN[l], in, ld_in,
                                                c->pbt() + c->L.t_off[l], KIN[l],
                                                p + c->L.b_off[l], nullptr, 0, c->act(l + 1),
                                                nullptr, 256)));
    }
    in = c->act(l + 1);
    ld_in = 256;
  }
  SCHK(c, (gemm<false, true, EPI_LINEAR_F32>(st, B, 64, 256, in, 256, c->pbt() + c->L.t_off[4],
                                             256, p + c->L.b_off[4], nullptr, 0, nullptr,
                                             (float*)(c->ws + c->L.off_y), 64)));
  return LBM_OK;
}

// loss gradient dY is in place; backward through all layers into the gradient vector
static int backward(srg_ctx* c, const bf16* Xb, int B) {
  hipStream_t st = c->stream;
  const bf16* pb = c->pb();
  float* g = c->g();
  const bf16* dz = (const bf16*)(c->ws + c->L.off_dy);
  int ld_dz = 64;
  int which = 0;
  for (int l = NL - 1; l >= 0; --l) {
    const bf16* a_in = l == 0 ? Xb : c->act(l);
    const int ld_in = l == 0 ? 32 : 256;
    // dW_l = a_in^T dz  (KIN x NOUT)
    SCHK(c, (gemm<true, false, EPI_F32>(st, KIN[l], NOUT[l], B, a_in, ld_in, dz, ld_dz, nullptr,
                                        nullptr, 0, nullptr, g + c->L.w_off[l], NOUT[l])));
    hipLaunchKernelGGL(k_colsum, dim3((NOUT[l] + 63) / 64), dim3(64 * COLSUM_WAVES), 0, st, dz, B,
                       NOUT[l], ld_dz, g + c->L.b_off[l]);
    SCHK(c, hipGetLastError());
    if (l > 0) {
      // dz_{l-1} = (dz W_l^T) * relu'(a_in)
      bf16* nd = (bf16*)(c->ws + c->L.off_dz[which]);
      SCHK(c, (gemm<false, true, EPI_DRELU_BF16>(st, B, 256, NOUT[l], dz, ld_dz, pb + c->L.w_off[l],
                                                 NOUT[l], nullptr, a_in, 256, nd, nullptr, 256)));
      dz = nd;
      ld_dz = 256;
      which ^= 1;
    }
  }
  return LBM_OK;
}

extern "C" {

size_t srg_workspace_bytes(int32_t max_batch, int32_t max_train) {
  if (max_batch < 64 || max_batch % 64 != 0 || max_train < 0) return 0;
  return make_layout(max_batch, max_train).total;
}

int srg_create(void* dev_workspace, size_t ws_bytes, int32_t max_batch, int32_t max_train,
               void* hip_stream, srg_ctx** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  const size_t need = srg_workspace_bytes(max_batch, max_train);
  if (need == 0 || !dev_workspace) return LBM_EINVAL;
  if (ws_bytes < need) return LBM_ENOMEM;
  if (((uintptr_t)dev_workspace) % ALIGN != 0) return LBM_EINVAL;
  srg_ctx* c = new (std::nothrow) srg_ctx();
  if (!c) return LBM_ENOMEM;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)dev_workspace;
  c->L = make_layout(max_batch, max_train);
  c->max_batch = max_batch;
  c->max_train = max_train;
  c->msg[0] = 0;
  *out = c;
  // zero parameters, gradients, moments (padding stays zero forever)
  SCHK(c, hipMemsetAsync(c->ws, 0, c->L.off_xall, c->stream));
  SCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int srg_set_params(srg_ctx* c, const float* params) {
  if (!c || !params) return LBM_EINVAL;
  if (c->err) return LBM_ESTATE;
  std::vector<float> pad(c->L.n_par, 0.f);
  size_t k = 0;
  for (int l = 0; l < NL; ++l) {
    for (int i = 0; i < KREAL[l]; ++i)
      for (int j = 0; j < NREAL[l]; ++j) pad[c->L.w_off[l] + (size_t)i * NOUT[l] + j] = params[k++];
    for (int j = 0; j < NREAL[l]; ++j) pad[c->L.b_off[l] + j] = params[k++];
  }
  const size_t nb = 4 * c->L.n_par;
  SCHK(c, hipMemcpyAsync(c->p(), pad.data(), nb, hipMemcpyHostToDevice, c->stream));
  SCHK(c, hipMemsetAsync(c->ws + c->L.off_m, 0, nb, c->stream));
  SCHK(c, hipMemsetAsync(c->ws + c->L.off_v, 0, nb, c->stream));
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((c->L.n_par + 255) / 256)), dim3(256), 0, c->stream,
                     c->p(), c->pb(), (long long)c->L.n_par);
  SCHK(c, hipGetLastError());
  if (int rc = refresh_transposed(c)) return rc;
  c->step = 0;
  SCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

static void unpad(const srg_ctx* c, const std::vector<float>& pad, float* out) {
  size_t k = 0;
  for (int l = 0; l < NL; ++l) {
    for (int i = 0; i < KREAL[l]; ++i)
      for (int j = 0; j < NREAL[l]; ++j) out[k++] = pad[c->L.w_off[l] + (size_t)i * NOUT[l] + j];
    for (int j = 0; j < NREAL[l]; ++j) out[k++] = pad[c->L.b_off[l] + j];
  }
}

int srg_get_params(srg_ctx* c, float* params) {
  if (!c || !params) return LBM_EINVAL;
  if (c->err) return LBM_ESTATE;
  std::vector<float> pad(c->L.n_par);
  SCHK(c, hipMemcpyAsync(pad.data(), c->p(), 4 * c->L.n_par, hipMemcpyDeviceToHost, c->stream));
  SCHK(c, hipStreamSynchronize(c->stream));
  unpad(c, pad, params);
  return LBM_OK;
}

static int upload_set(srg_ctx* c, const float* X, const int32_t* label, const float* traj, int n,
                      size_t off_x, size_t off_lab, size_t off_traj) {
  std::vector<uint16_t> xb((size_t)n * 32, 0);
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < SRG_IN; ++j) xb[(size_t)r * 32 + j] = host_bf16(X[(size_t)r * SRG_IN + j]);
  SCHK(c, hipMemcpyAsync(c->ws + off_x, xb.data(), 2 * xb.size(), hipMemcpyHostToDevice, c->stream));
  if (label)
    SCHK(c, hipMemcpyAsync(c->ws + off_lab, label, 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
  if (traj)
    SCHK(c, hipMemcpyAsync(c->ws + off_traj, traj, 4 * (size_t)NTRAJ * n, hipMemcpyHostToDevice,
                           c->stream));
  SCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int srg_set_train(srg_ctx* c, const float* X, const int32_t* label, const float* traj, int32_t n) {
  if (!c || !X || !label || !traj || n < 1) return LBM_EINVAL;
  if (c->err) return LBM_ESTATE;
  if (n > c->max_train) return srg_err(c, LBM_ERANGE, "training set larger than max_train");
  for (int i = 0; i < n; ++i)
    if (label[i] < 0 || label[i] >= NCLS) return srg_err(c, LBM_EINVAL, "label out of range");
  int rc = upload_set(c, X, label, traj, n, c->L.off_xall, c->L.off_lab, c->L.off_traj);
  if (rc) return rc;
  c->n_train = n;
  return LBM_OK;
}

static int refresh_transposed(srg_ctx* c) {
  for (int l = 0; l < NL; ++l) {
    const int n = KIN[l] * NOUT[l];
    hipLaunchKernelGGL(k_transpose_bf16, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                       c->p() + c->L.w_off[l], KIN[l], NOUT[l], c->pbt() + c->L.t_off[l]);
  }
  SCHK(c, hipGetLastError());
  return LBM_OK;
}

static int adam(srg_ctx* c, float lr) {
  ++c->step;
  const float bc1 = 1.f - powf(0.9f, (float)c->step), bc2 = 1.f - powf(0.999f, (float)c->step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((c->L.n_par + 255) / 256)), dim3(256), 0, c->stream,
                     c->p(), c->g(), (float*)(c->ws + c->L.off_m), (float*)(c->ws + c->L.off_v),
                     c->pb(), (long long)c->L.n_par, lr, bc1, bc2);
  SCHK(c, hipGetLastError());
  return refresh_transposed(c);
}

int srg_train(srg_ctx* c, int32_t epochs, int32_t batch, float lr, float w_traj, uint64_t seed,
              float* epoch_loss) {
  if (!c) return LBM_EINVAL;
  if (c->err) return LBM_ESTATE;
  if (epochs < 0 || batch < 64 || batch % 64 != 0 || batch > c->max_batch || batch > c->n_train)
    return srg_err(c, LBM_EINVAL, "batch must be a multiple of 64, <= max_batch and the set size");
  const int n = c->n_train, nb = n / batch;
  std::mt19937_64 rng(seed);
  std::vector<int> perm(n);
  float* acc = (float*)(c->ws + c->L.off_acc);
  bf16* Xb = (bf16*)(c->ws + c->L.off_xb);
  int* dperm = (int*)(c->ws + c->L.off_perm);
  for (int e = 0; e < epochs; ++e) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    std::shuffle(perm.begin(), perm.end(), rng);
    SCHK(c, hipMemcpyAsync(dperm, perm.data(), 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    SCHK(c, hipMemsetAsync(acc, 0, 4, c->stream));
    for (int b = 0; b < nb; ++b) {
      hipLaunchKernelGGL(k_gather, dim3((batch * 4 + 255) / 256), dim3(256), 0, c->stream,
                         (const bf16*)(c->ws + c->L.off_xall), dperm, b * batch, batch, Xb);
      SCHK(c, hipGetLastError());
      int rc = forward(c, Xb, batch);
      if (rc) return rc;
      hipLaunchKernelGGL(k_loss, dim3((batch + 255) / 256), dim3(256), 0, c->stream,
                         (const float*)(c->ws + c->L.off_y), dperm, b * batch, batch,
                         (const int*)(c->ws + c->L.off_lab), (const float*)(c->ws + c->L.off_traj),
                         w_traj, (bf16*)(c->ws + c->L.off_dy), acc);
      SCHK(c, hipGetLastError());
      rc = backward(c, Xb, batch);
      if (rc) return rc;
      rc = adam(c, lr);
      if (rc) return rc;
    }
    float s = 0.f;
    SCHK(c, hipMemcpyAsync(&s, acc, 4, hipMemcpyDeviceToHost, c->stream));
    SCHK(c, hipStreamSynchronize(c->stream));
    if (epoch_loss) epoch_loss[e] = nb > 0 ? s / nb : 0.f;
  }
  return LBM_OK;
}

int srg_gradients(srg_ctx* c, const float* X, const int32_t* label, const float* traj, int32_t n,
                  float w_traj, float* grads, float* loss) {
  if (!c || !X || !label || !traj || !grads) return LBM_EINVAL;
  if (c->err) return LBM_ESTATE;
  if (n < 64 || n % 64 != 0 || n > c->max_batch)
    return srg_err(c, LBM_EINVAL, "n must be a multiple of 64 and <= max_batch");
  for (int i = 0; i < n; ++i)
    if (label[i] < 0 || label[i] >= NCLS) return srg_err(c, LBM_EINVAL, "label out of range");
  // the batch goes through the training-set buffers' batch slots: inputs in
  // Xb, labels and trajectories in the (batch-sized) prefix of dedicated rows
  std::vector<uint16_t> xb((size_t)n * 32, 0);
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < SRG_IN; ++j) xb[(size_t)r * 32 + j] = host_bf16(X[(size_t)r * SRG_IN + j]);
  bf16* Xb = (bf16*)(c->ws + c->L.off_xb);
  SCHK(c, hipMemcpyAsync(Xb, xb.data(), 2 * xb.size(), hipMemcpyHostToDevice, c->stream));
  // labels and trajectories staged in the FP32 output buffer region of the
  // inference path (sized max_batch x 51 floats >= n x 49)
  int* dlab = (int*)(c->ws + c->L.off_yout);
  float* dtr = (float*)(c->ws + c->L.off_yout) + n;
  SCHK(c, hipMemcpyAsync(dlab, label, 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
  SCHK(c, hipMemcpyAsync(dtr, traj, 4 * (size_t)NTRAJ * n, hipMemcpyHostToDevice, c->stream));
  float* acc = (float*)(c->ws + c->L.off_acc);
  SCHK(c, hipMemsetAsync(acc, 0, 4, c->stream));
  int rc = forward(c, Xb, n);
  if (rc) return rc;
  hipLaunchKernelGGL(k_loss, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                     (const float*)(c->ws + c->L.off_y), (const int*)nullptr, 0, n, dlab, dtr, w_traj,
                     (bf16*)(c->ws + c->L.off_dy), acc);
  SCHK(c, hipGetLastError());
  rc = backward(c, Xb, n);
  if (rc) return rc;
  std::vector<float> pad(c->L.n_par);
  SCHK(c, hipMemcpyAsync(pad.data(), c->g(), 4 * c->L.n_par, hipMemcpyDeviceToHost, c->stream));
  float s = 0.f;
  SCHK(c, hipMemcpyAsync(&s, acc, 4, hipMemcpyDeviceToHost, c->stream));
  SCHK(c, hipStreamSynchronize(c->stream));
  unpad(c, pad, grads);
  if (loss) *loss = s;
  return LBM_OK;
}

int srg_predict(srg_ctx* c, const float* X, int32_t n, float* y, int32_t src_is_device,
                int32_t dst_is_device) {
  if (!c || !X || !y || n < 1) return LBM_EINVAL;
  if (c->err) return LBM_ESTATE;
  float* xin = (float*)(c->ws + c->L.off_xin);
  float* yout = (float*)(c->ws + c->L.off_yout);
  for (int r0 = 0; r0 < n; r0 += c->max_batch) {
    const int m = std::min(c->max_batch, n - r0);
    const float* src = X + (size_t)r0 * SRG_IN;
    if (!src_is_device) {
      SCHK(c, hipMemcpyAsync(xin, src, 4 * (size_t)SRG_IN * m, hipMemcpyHostToDevice, c->stream));
      src = xin;
    }
    float* dst = dst_is_device ? y + (size_t)r0 * SRG_OUT : yout;
    int rc = infer(c, src, m, dst);
    if (rc) return rc;
    if (!dst_is_device) {
      SCHK(c, hipMemcpyAsync(y + (size_t)r0 * SRG_OUT, yout, 4 * (size_t)SRG_OUT * m,
                             hipMemcpyDeviceToHost, c->stream));
      SCHK(c, hipStreamSynchronize(c->stream));
    }
  }
  if (!src_is_device) SCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int srg_sync(srg_ctx* c) {
  if (!c) return LBM_EINVAL;
  if (c->err) return LBM_ESTATE;
  SCHK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

void srg_destroy(srg_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* srg_last_error(const srg_ctx* c) {
  if (!c || c->err == 0) return nullptr;
  return c->msg;
}

}  // extern "C"
