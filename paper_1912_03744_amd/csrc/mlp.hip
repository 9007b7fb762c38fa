// mlp.hip -- the learned surrogate: a GELU multilayer perceptron trained and
// evaluated with bf16 matrix cores (v_mfma_f32_32x32x16_bf16) and fp32
// accumulation, fp32 master weights and Adam.
//
// Network: x (n0 features) -> h_l = gelu(h_{l-1} W_l + b_l) for the hidden
// layers -> y = h_L W_out + b_out.  gelu(u) = u Phi(u) (erf form).  Hidden
// activations are stored in bf16 (the next product's operand), the output
// and all pre-activations in fp32.  Loss: mean squared error over batch and
// outputs.  Weights W_l are [n_in x n_out] row-major; the flat parameter
// vector holds, layer by layer, W_l then b_l.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "common.hpp"

namespace adi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 64, BN = 64, KT = 32, LDP = KT + 8;  // tile sizes; padded LDS rows (bf16)
constexpr int MAX_LAYERS = 8;
constexpr int KPAD = 64;                                 // input features padded to a whole tile

// EPI_INFER: the hidden epilogue without the fp32 pre-activation (inference
// only, nothing kept for a backward pass).
enum Epi { EPI_HIDDEN = 0, EPI_OUTPUT = 1, EPI_DGELU = 2, EPI_PARTIAL = 3, EPI_INFER = 4 };

struct GemmArgs {
  const __bf16* A;  // [M][K] (a_kmajor) or [K][M]
  long lda;
  const __bf16* B;  // [N][K] (b_kmajor) or [K][N]
  long ldb;
  int M, N, K, Ks;  // K per split (grid.z splits)
  const float* bias;
  const float* U;   // pre-activations for EPI_DGELU
  float* out_f32;
  __bf16* out_bf16;
  long ldo;
  long split_stride;
};

// erf by the rational approximation of Abramowitz and Stegun, Handbook of
// Mathematical Functions, formula 7.1.26 (|error| <= 1.5e-7, far below the
// bf16 rounding of the activations it feeds): for x >= 0,
// erf x = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2), t = 1/(1 + p x),
// odd in x.
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * ax);
  const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float r = 1.0f - poly * __expf(-ax * ax);
  return copysignf(r, x);
}
__device__ __forceinline__ float gelu_f(float u) { return 0.5f * u * (1.0f + erf_as(u * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float u) {
  return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) + u * 0.39894228040143268f * expf(-0.5f * u * u);
}

// C[m][n] = sum_k A[m][k] B[k][n] over this block's K range, 64 x 64 tile per
// workgroup, one 32 x 32 bf16 MFMA accumulator per wave.
template <bool AK, bool BK, int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[BM][LDP];  // [m][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][LDP];  // [n][k]
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * g.Ks;
  const int kend = min(g.K, kbeg + g.Ks);
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  floatx16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;

  for (int k0 = kbeg; k0 < kend; k0 += KT) {
    // stage A (64 x 32) and B (32 x 64) tiles: 256 threads x 8 bf16 each
    if (AK) {
      const int row = t >> 2, kq = (t & 3) * 8;
      *(bf16x8*)&As[row][kq] = *(const bf16x8*)(g.A + (long)(m0 + row) * g.lda + k0 + kq);
    } else {
      const int kr = t >> 3, mq = (t & 7) * 8;
      const bf16x8 v = *(const bf16x8*)(g.A + (long)(k0 + kr) * g.lda + m0 + mq);
#pragma unroll
      for (int j = 0; j < 8; ++j) As[mq + j][kr] = v[j];
    }
    if (BK) {
      const int row = t >> 2, kq = (t & 3) * 8;
      *(bf16x8*)&Bs[row][kq] = *(const bf16x8*)(g.B + (long)(n0 + row) * g.ldb + k0 + kq);
    } else {
      const int kr = t >> 3, nq = (t & 7) * 8;
      const bf16x8 v = *(const bf16x8*)(g.B + (long)(k0 + kr) * g.ldb + n0 + nq);
#pragma unroll
      for (int j = 0; j < 8; ++j) Bs[nq + j][kr] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KT; kk += 16) {
      const bf16x8 a = *(const bf16x8*)&As[wm + (lane & 31)][kk + 8 * (lane >> 5)];
      const bf16x8 b = *(const bf16x8*)&Bs[wn + (lane & 31)][kk + 8 * (lane >> 5)];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }

  // accumulator i of lane l: row 8*(i/4) + 4*(l/32) + i%4, column l%32
  const int n = n0 + wn + (lane & 31);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    const long o = (long)m * g.ldo + n;
    const float v = acc[i];
    if constexpr (EPI == EPI_HIDDEN || EPI == EPI_INFER) {
      const float u = v + g.bias[n];
      if constexpr (EPI == EPI_HIDDEN) g.out_f32[o] = u;
      g.out_bf16[o] = (__bf16)gelu_f(u);
    } else if constexpr (EPI == EPI_OUTPUT) {
      g.out_f32[o] = v + g.bias[n];
    } else if constexpr (EPI == EPI_DGELU) {
      const float d = v * gelu_grad_f(g.U[o]);
      g.out_f32[o] = d;
      g.out_bf16[o] = (__bf16)d;
    } else {
      g.out_f32[(long)blockIdx.z * g.split_stride + o] = v;
    }
  }
}

// One forward layer out = epilogue(A W + b) for a whole batch, with the
// layer's weights resident in LDS: the workgroups stay for the whole batch
// (one per compute unit), each first copies W^T (ND rows of KD bf16, rows
// padded by 8 so that the 32 lanes reading one 16-byte column piece of 32
// rows hit different banks), then takes row tiles of 64 NWAVE rows; each
// wave multiplies its 64 rows (two 32-row A fragments per 16-wide k step,
// held in registers for the whole K) with every 32-column block of W^T,
// reusing each W fragment for both row halves: 2 ND/32 accumulators of
// 32 x 32 fp32.  The k steps run in the same order as in k_gemm, so each
// output element sees the same sequence of products and sums.
template <int KD, int ND, int EPI>
__global__ void __launch_bounds__(256) k_layer(const __bf16* __restrict__ A, const __bf16* __restrict__ Wt,
                                               const float* __restrict__ bias, long B, float* out_f32,
                                               __bf16* out_bf16) {
  constexpr int NWAVE = 4, ROWS = 64 * NWAVE, LDW = KD + 8, NB = ND / 32, KS = KD / 16;
  __shared__ __attribute__((aligned(16))) __bf16 W[ND * LDW];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  // W^T into LDS: ND x KD bf16 in 16-byte pieces
  // unrolled: the copy's global loads all in flight, not one latency each
#pragma unroll 16
  for (int q = t; q < ND * KD / 8; q += 256) {
    const int n = q / (KD / 8), k8 = q % (KD / 8);
    *(bf16x8*)&W[n * LDW + 8 * k8] = *(const bf16x8*)(Wt + (long)n * KD + 8 * k8);
  }
  __syncthreads();
  const int half = lane >> 5, lr = lane & 31;
  for (long tile = blockIdx.x; tile * ROWS < B; tile += gridDim.x) {
    const long m0 = tile * ROWS + wave * 64;
    // the wave's A fragments: rows m0 + lr (first half) and m0 + 32 + lr
    bf16x8 a0[KS], a1[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const long r0 = m0 + lr, r1 = m0 + 32 + lr;
      bf16x8 z;
#pragma unroll
      for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
      a0[k] = r0 < B ? *(const bf16x8*)(A + r0 * KD + 16 * k + 8 * half) : z;
      a1[k] = r1 < B ? *(const bf16x8*)(A + r1 * KD + 16 * k + 8 * half) : z;
    }
    floatx16 acc0[NB], acc1[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        acc0[nb][i] = 0.0f;
        acc1[nb][i] = 0.0f;
      }
#pragma unroll
    for (int k = 0; k < KS; ++k)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const bf16x8 b = *(const bf16x8*)&W[(nb * 32 + lr) * LDW + 16 * k + 8 * half];
        acc0[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0[k], b, acc0[nb], 0, 0, 0);
        acc1[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[k], b, acc1[nb], 0, 0, 0);
      }
    // epilogue: accumulator i of lane l holds row 8 (i/4) + 4 (l/32) + i%4,
    // column l%32 of its 32 x 32 block (32 lanes store 32 consecutive
    // columns of a row: 64-byte runs in bf16; packing 4 values per lane
    // along the accumulator index instead, by swapping the operands, scatters
    // 8-byte pieces over 32 rows and was measured twice as slow)
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int n = nb * 32 + lr;
        const float bn = bias[n];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const long m = m0 + 32 * hb + 8 * (i >> 2) + 4 * half + (i & 3);
          if (m >= B) continue;
          const float v = hb ? acc1[nb][i] : acc0[nb][i];
          const long o = m * ND + n;
          const float u = v + bn;
          if constexpr (EPI == EPI_OUTPUT) {
            out_f32[o] = u;
          } else {
            if constexpr (EPI == EPI_HIDDEN) out_f32[o] = u;
            out_bf16[o] = (__bf16)gelu_f(u);
          }
        }
      }
  }
}

// The whole inference forward pass of a network whose hidden layers are 256
// wide (input padded to KPAD = 64, output NOUT), in one kernel: each
// workgroup of FUSED_WAVES waves takes tiles of 256 rows (32 per wave) and
// keeps their activations on the CU from the input to the output.  The wave
// encodes its rows' inputs straight into its A fragments; per layer the
// workgroup copies W^T into LDS, each wave multiplies its 32 rows with
// every 32-column block of W^T (the fragments, k order and epilogue
// arithmetic of k_layer), and for a hidden layer writes bias + GELU as bf16
// into LDS (the weights' space, no longer needed), from where it reads its A
// fragments of the next layer; the output layer stores bias + product as
// fp32.  Activations never go to HBM: per tile only the inputs are read and
// the outputs written.  32 rows per wave (one A fragment per k step, 8
// accumulators) leave room for two waves per SIMD, which hide the latency
// of the epilogue: 64 rows per wave at one wave per SIMD took 1.6x as long.
struct FusedArgs {
  const float* x;
  int nin;
  long B;
  const float* shift;
  const float* scale;
  const __bf16* Wt[MAX_LAYERS];
  const float* bias[MAX_LAYERS];
  int nl;
  float* y;
};

constexpr int FUSED_WAVES = 8;
constexpr int FUSED_ROWS = 32 * FUSED_WAVES;  // rows per tile
constexpr int FUSED_LDA = 256 + 8;            // padded LDS rows (bf16): W^T and activations

// One layer of k_mlp_fused for the wave's rows m0 .. m0 + 31 (A fragments
// a: row m0 + lr, k step k in a[k]; the first KD/16 used).
template <int KD, int ND, bool LAST>
__device__ __forceinline__ void fused_layer(const FusedArgs& f, int l, long m0, __bf16* lds, bf16x8 (&a)[16]) {
  constexpr int LDW = KD + 8, NB = ND / 32, KS = KD / 16;
  static_assert(ND * LDW <= FUSED_ROWS * FUSED_LDA, "W^T fits the LDS space");
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, half = lane >> 5, lr = lane & 31;
  const __bf16* __restrict__ Wt = f.Wt[l];
  const float* __restrict__ bias = f.bias[l];
  __syncthreads();  // every wave is done with the LDS space
  // unrolled: the copy's loads in flight together, not one latency each
#pragma unroll 4
  for (int q = t; q < ND * KD / 8; q += 64 * FUSED_WAVES) {
    const int n = q / (KD / 8), k8 = q % (KD / 8);
    *(bf16x8*)&lds[n * LDW + 8 * k8] = *(const bf16x8*)(Wt + (long)n * KD + 8 * k8);
  }
  __syncthreads();
  floatx16 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[nb][i] = 0.0f;
#pragma unroll
  for (int k = 0; k < KS; ++k)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const bf16x8 b = *(const bf16x8*)&lds[(nb * 32 + lr) * LDW + 16 * k + 8 * half];
      acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[k], b, acc[nb], 0, 0, 0);
    }
  // accumulator i of lane l: row 8 (i/4) + 4 (l/32) + i%4, column l%32
  if constexpr (LAST) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int n = nb * 32 + lr;
      const float bn = bias[n];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const long m = m0 + 8 * (i >> 2) + 4 * half + (i & 3);
        if (m < f.B) f.y[m * ND + n] = acc[nb][i] + bn;
      }
    }
  } else {
    static_assert(ND == 256, "hidden layers are 256 wide");
    __syncthreads();  // every wave has read its W^T fragments
    __bf16* act = lds + (size_t)wave * 32 * FUSED_LDA;  // the wave's 32 rows
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int n = nb * 32 + lr;
      const float bn = bias[n];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = 8 * (i >> 2) + 4 * half + (i & 3);
        act[r * FUSED_LDA + n] = (__bf16)gelu_f(acc[nb][i] + bn);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = *(const bf16x8*)&act[lr * FUSED_LDA + 16 * k + 8 * half];
  }
}

template <int NOUT>
__global__ void __launch_bounds__(64 * FUSED_WAVES, 2) k_mlp_fused(FusedArgs f) {
  __shared__ __attribute__((aligned(16))) __bf16 lds[FUSED_ROWS * FUSED_LDA];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, half = lane >> 5, lr = lane & 31;
  for (long tile = blockIdx.x; tile * FUSED_ROWS < f.B; tile += gridDim.x) {
    const long m0 = tile * FUSED_ROWS + wave * 32;
    // encoded inputs as A fragments (k_encode's arithmetic): features
    // 16 k + 8 half + e of row m0 + lr, 0 past nin
    bf16x8 a[16];
    const long r = m0 + lr;
#pragma unroll
    for (int k = 0; k < KPAD / 16; ++k)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = 16 * k + 8 * half + e;
        a[k][e] = (__bf16)(c < f.nin && r < f.B ? (f.x[r * f.nin + c] - f.shift[c]) * f.scale[c] : 0.0f);
      }
    fused_layer<KPAD, 256, false>(f, 0, m0, lds, a);
    for (int l = 1; l < f.nl - 1; ++l) fused_layer<256, 256, false>(f, l, m0, lds, a);
    fused_layer<256, NOUT, true>(f, f.nl - 1, m0, lds, a);
  }
}

// x (B x nin fp32) -> (x - shift) * scale as bf16, zero-padded to KPAD
// columns: one row per thread, written as KPAD/8 16-byte pieces.
__global__ void k_encode(const float* __restrict__ x, int nin, long B, const float* shift, const float* scale,
                         __bf16* __restrict__ out) {
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < B; r += (long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int p = 0; p < KPAD / 8; ++p) {
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = 8 * p + e;
        v[e] = (__bf16)(c < nin ? (x[r * nin + c] - shift[c]) * scale[c] : 0.0f);
      }
      *(bf16x8*)(out + r * KPAD + 8 * p) = v;
    }
  }
}

// Mean squared error: dY = 2 (Y - T) / (B * nout), per-row sums of squares
// (reduced in a fixed order by k_sum_rows).  One wave per row, lane j on
// columns j, j + 64, ... (coalesced); the lanes' partial sums are added by a
// butterfly in a fixed order.
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ Y, const float* __restrict__ T, long B,
                                              int nout, float* dY, __bf16* dYb, float* rowsq) {
  const int lane = threadIdx.x & 63;
  const float c = 2.0f / (float)((double)B * nout);
  const long first = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6;
  const long stride = ((long)gridDim.x * blockDim.x) >> 6;
  for (long r = first; r < B; r += stride) {
    double s = 0.0;
    for (int j = lane; j < nout; j += 64) {
      const long e = r * nout + j;
      const float d = Y[e] - T[e];
      s += (double)d * d;
      dY[e] = c * d;
      dYb[e] = (__bf16)(c * d);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) rowsq[r] = (float)s;
  }
}

__global__ void __launch_bounds__(256) k_sum_rows(const float* v, long n, double denom, float* out) {
  __shared__ double s[256];
  double a = 0.0;
  for (long i = threadIdx.x; i < n; i += blockDim.x) a += v[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(s[0] / denom);
}

// Column sums of D (B x N fp32) in two passes, each in a fixed order: block
// (x, s) sums rows [s R, s R + R) of 64 columns (four row phases, combined
// in order) into part[s][c]; k_colsum_final adds the slices (below).
__global__ void __launch_bounds__(256) k_colsum_part(const float* __restrict__ D, long B, int N, long R,
                                                     float* __restrict__ part) {
  __shared__ float sm[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
  const long r0 = blockIdx.y * R, r1 = r0 + R < B ? r0 + R : B;
  float a = 0.0f;
  if (c < N)
    for (long r = r0 + ph; r < r1; r += 4) a += D[r * N + c];
  sm[ph][threadIdx.x & 63] = a;
  __syncthreads();
  if (ph == 0 && c < N)
    part[(long)blockIdx.y * N + c] = ((sm[0][threadIdx.x] + sm[1][threadIdx.x]) + sm[2][threadIdx.x]) +
                                     sm[3][threadIdx.x];
}

// One wave per column: lane q adds slices q, q + 64, ... in order, then the
// lanes' sums are combined by a butterfly (lane 0's order is fixed).
__global__ void __launch_bounds__(256) k_colsum_final(const float* __restrict__ part, int S, int N,
                                                      float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int c = (int)((blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6);
  if (c >= N) return;  // whole waves: c is the same in every lane of a wave
  float a = 0.0f;
  for (int q = lane; q < S; q += 64) a += part[(long)q * N + c];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) out[c] = a;
}

// Rows per slice of the column sums: at least 64, at most COLSUM_SLICES
// slices.
constexpr int COLSUM_SLICES = 256;
inline long colsum_rows(long B) {
  const long R = (B + COLSUM_SLICES - 1) / COLSUM_SLICES;
  return std::max(64L, (R + 3) / 4 * 4);
}

// Sum the split-K partial products (fixed order) into the gradient of W,
// keeping the first `rows` rows (the real input features of layer 1).
__global__ void k_reduce_splits(const float* __restrict__ part, int splits, long stride, int rows, int N,
                                float* out) {
  const long n = (long)rows * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    float a = 0.0f;
    for (int s = 0; s < splits; ++s) a += part[s * stride + e];
    out[e] = a;
  }
}

// Adam with bias correction on fp32 master parameters.
__global__ void k_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// bf16 operand copies of one layer's weights: W as [kin_pad][nout] and its
// transpose [nout][kin_pad]; rows past kin are zero.
__global__ void k_refresh(const float* __restrict__ W, int kin, int kin_pad, int nout, __bf16* Wb, __bf16* Wtb) {
  const long n = (long)kin_pad * nout;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / nout), j = (int)(e % nout);
    const __bf16 v = (__bf16)(i < kin ? W[(long)i * nout + j] : 0.0f);
    Wb[e] = v;
    Wtb[(long)j * kin_pad + i] = v;
  }
}

}  // namespace adi

// Work area of adi_mlp_forward_noalloc: the encoded input and two ping-pong
// hidden activations (bf16), for callers that cannot allocate.  Every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol): it uses the device address obtained once per device with
// hipGetSymbolAddress (noalloc_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[ADI_MLP_NOALLOC_SCRATCH_BYTES];

using namespace adi;

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device `dev`, looked up once per
// device (called with that device current).
adi_status noalloc_scratch_setup(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(ADI_EUNSUPPORTED, "device %d beyond %d", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return ADI_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(ADI_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
  g_scratch_ptr[dev] = ptr;
  return ADI_OK;
}

void* noalloc_scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (dev >= 0 && dev < MAX_DEVICES) ? g_scratch_ptr[dev] : nullptr;
}

}  // namespace

struct adi_mlp_s {
  int device = 0;
  int cus = 256;              // compute units of the device
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int nl = 0;                 // number of weight layers
  int width[MAX_LAYERS + 1];  // width[0] = inputs, width[nl] = outputs
  int kin_pad[MAX_LAYERS];    // padded input width of each layer
  long woff[MAX_LAYERS], boff[MAX_LAYERS], nparams = 0;
  float *P = nullptr, *Gr = nullptr, *Mm = nullptr, *Vv = nullptr;
  __bf16 *Wb[MAX_LAYERS] = {}, *Wtb[MAX_LAYERS] = {};
  float *shift = nullptr, *scale = nullptr;
  // activations for `cap` rows
  long cap = 0;
  __bf16* X = nullptr;
  __bf16* H[MAX_LAYERS] = {};
  float* U[MAX_LAYERS] = {};
  float* Y = nullptr;
  float* dYf = nullptr;
  __bf16* dYb = nullptr;
  float *dUf = nullptr, *dUf2 = nullptr;
  __bf16 *dUb = nullptr, *dUb2 = nullptr;
  float* rowsq = nullptr;
  float* colpart = nullptr;  // slices of the bias-gradient column sums
  float* part = nullptr;
  long part_cap = 0;
  float* loss = nullptr;
  long step = 0;
  float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
};

namespace {

adi_status mlp_handle(adi_mlp m) {
  if (!m) return fail(ADI_EINVAL, "null network handle");
  ADI_HIP(hipSetDevice(m->device));
  return ADI_OK;
}

template <bool AK, bool BK, int EPI>
adi_status gemm(adi_mlp mm, const GemmArgs& g, int splits) {
  if (g.M % BM || g.N % BN || g.K % KT || g.Ks % KT)
    return fail(ADI_EINVAL, "internal: gemm shape %dx%dx%d not tiled", g.M, g.N, g.K);
  hipLaunchKernelGGL((k_gemm<AK, BK, EPI>), dim3(g.M / BM, g.N / BN, splits), dim3(256), 0, mm->stream, g);
  ADI_CHECK_LAUNCH();
  return ADI_OK;
}

void free_acts(adi_mlp m) {
  dev_free(m->X);
  m->X = nullptr;
  for (int l = 0; l < MAX_LAYERS; ++l) {
    dev_free(m->H[l]);
    dev_free(m->U[l]);
    m->H[l] = nullptr;
    m->U[l] = nullptr;
  }
  void* b[] = {m->Y, m->dYf, m->dYb, m->dUf, m->dUf2, m->dUb, m->dUb2, m->rowsq, m->colpart};
  for (void* p : b) dev_free(p);
  m->Y = m->dYf = m->dUf = m->dUf2 = m->rowsq = m->colpart = nullptr;
  m->dYb = m->dUb = m->dUb2 = nullptr;
  m->cap = 0;
}

adi_status ensure_acts(adi_mlp m, long B) {
  if (B <= m->cap) return ADI_OK;
  ADI_HIP(hipStreamSynchronize(m->stream));
  free_acts(m);
  long cap = ((B + 1023) / 1024) * 1024;
  int wmax = 0;
  for (int l = 1; l <= m->nl; ++l) wmax = std::max(wmax, m->width[l]);
  ADI_TRY(dev_alloc((void**)&m->X, 2 * cap * KPAD, m->stream));
  for (int l = 0; l < m->nl - 1; ++l) {
    ADI_TRY(dev_alloc((void**)&m->H[l], 2 * cap * m->width[l + 1], m->stream));
    ADI_TRY(dev_alloc((void**)&m->U[l], 4 * cap * m->width[l + 1], m->stream));
  }
  const int nout = m->width[m->nl];
  ADI_TRY(dev_alloc((void**)&m->Y, 4 * cap * nout, m->stream));
  ADI_TRY(dev_alloc((void**)&m->dYf, 4 * cap * nout, m->stream));
  ADI_TRY(dev_alloc((void**)&m->dYb, 2 * cap * nout, m->stream));
  ADI_TRY(dev_alloc((void**)&m->dUf, 4 * cap * wmax, m->stream));
  ADI_TRY(dev_alloc((void**)&m->dUf2, 4 * cap * wmax, m->stream));
  ADI_TRY(dev_alloc((void**)&m->dUb, 2 * cap * wmax, m->stream));
  ADI_TRY(dev_alloc((void**)&m->dUb2, 2 * cap * wmax, m->stream));
  ADI_TRY(dev_alloc((void**)&m->rowsq, 4 * cap, m->stream));
  ADI_TRY(dev_alloc((void**)&m->colpart, 4L * COLSUM_SLICES * wmax, m->stream));
  m->cap = cap;
  return ADI_OK;
}

adi_status refresh_weights(adi_mlp m) {
  for (int l = 0; l < m->nl; ++l) {
    const long n = (long)m->kin_pad[l] * m->width[l + 1];
    hipLaunchKernelGGL(k_refresh, dim3((int)std::min<long>((n + 255) / 256, 1024)), dim3(256), 0, m->stream,
                       m->P + m->woff[l], m->width[l], m->kin_pad[l], m->width[l + 1], m->Wb[l], m->Wtb[l]);
    ADI_CHECK_LAUNCH();
  }
  return ADI_OK;
}

adi_status check_batch(adi_mlp m, long B) {
  if (B < 1 || B > (1L << 26)) return fail(ADI_EINVAL, "batch must be in [1, 2^26]");
  if (B % BM) return fail(ADI_EINVAL, "batch must be a multiple of %d", BM);
  (void)m;
  return ADI_OK;
}

adi_status layer_forward(adi_mlp m, int l, int epi, const __bf16* in, long B, float* of, __bf16* ob);

// Inference-only forward pass: encoded input in X, hidden activations of
// layer l in H[l] (no pre-activations kept), output straight into y.  The
// same products and epilogue arithmetic as forward().
adi_status forward_infer(adi_mlp m, const float* x, long B, __bf16* X, __bf16* const* H, float* y) {
  // the whole pass in one kernel when every CU gets a tile of 256 rows
  // and the network is 64 (padded input) -> 256 x (nl - 1) -> 64 | 128 | 256
  bool fused = B >= 256L * m->cus && m->nl >= 2 && m->kin_pad[0] == KPAD;
  for (int l = 1; l < m->nl; ++l) fused = fused && m->width[l] == 256;
  const int nout = m->width[m->nl];
  fused = fused && (nout == 64 || nout == 128 || nout == 256);
  if (fused) {
    FusedArgs f{};
    f.x = x;
    f.nin = m->width[0];
    f.B = B;
    f.shift = m->shift;
    f.scale = m->scale;
    for (int l = 0; l < m->nl; ++l) {
      f.Wt[l] = m->Wtb[l];
      f.bias[l] = m->P + m->boff[l];
    }
    f.nl = m->nl;
    f.y = y;
    const int grid = (int)std::min<long>(m->cus, (B + FUSED_ROWS - 1) / FUSED_ROWS);
    const dim3 block(64 * FUSED_WAVES);
    if (nout == 64) hipLaunchKernelGGL(k_mlp_fused<64>, dim3(grid), block, 0, m->stream, f);
    else if (nout == 128) hipLaunchKernelGGL(k_mlp_fused<128>, dim3(grid), block, 0, m->stream, f);
    else hipLaunchKernelGGL(k_mlp_fused<256>, dim3(grid), block, 0, m->stream, f);
    ADI_CHECK_LAUNCH();
    return ADI_OK;
  }
  hipLaunchKernelGGL(k_encode, dim3((int)std::min<long>((B + 255) / 256, 8192)), dim3(256), 0, m->stream,
                     x, m->width[0], B, m->shift, m->scale, X);
  ADI_CHECK_LAUNCH();
  const __bf16* in = X;
  for (int l = 0; l < m->nl; ++l) {
    if (l < m->nl - 1) {
      ADI_TRY(layer_forward(m, l, EPI_INFER, in, B, nullptr, H[l]));
      in = H[l];
    } else {
      ADI_TRY(layer_forward(m, l, EPI_OUTPUT, in, B, y, nullptr));
    }
  }
  return ADI_OK;
}

adi_status forward(adi_mlp m, const float* x, long B) {
  hipLaunchKernelGGL(k_encode, dim3((int)std::min<long>((B + 255) / 256, 8192)), dim3(256), 0, m->stream,
                     x, m->width[0], B, m->shift, m->scale, m->X);
  ADI_CHECK_LAUNCH();
  const __bf16* in = m->X;
  for (int l = 0; l < m->nl; ++l) {
    if (l < m->nl - 1) {
      ADI_TRY(layer_forward(m, l, EPI_HIDDEN, in, B, m->U[l], m->H[l]));
      in = m->H[l];
    } else {
      ADI_TRY(layer_forward(m, l, EPI_OUTPUT, in, B, m->Y, nullptr));
    }
  }
  return ADI_OK;
}

// Loss, gradients of all parameters into m->Gr.
adi_status backward(adi_mlp m, const float* target, long B) {
  const int nout = m->width[m->nl];
  hipLaunchKernelGGL(k_loss, dim3((int)std::min<long>((B + 3) / 4, 4096)), dim3(256), 0, m->stream, m->Y,
                     target, B, nout, m->dYf, m->dYb, m->rowsq);
  ADI_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, m->stream, m->rowsq, B, (double)B * nout, m->loss);
  ADI_CHECK_LAUNCH();
  // split-K over the batch for the weight gradients: ~256 rows per split
  const int splits = (int)std::max<long>(1, std::min<long>(64, B / 256));
  const long Ks = ((B / splits + KT - 1) / KT) * KT;
  const int nsplit = (int)((B + Ks - 1) / Ks);
  long need = 0;
  for (int l = 0; l < m->nl; ++l) need = std::max(need, (long)nsplit * m->kin_pad[l] * m->width[l + 1]);
  if (need > m->part_cap) {
    ADI_HIP(hipStreamSynchronize(m->stream));
    dev_free(m->part);
    m->part = nullptr;
    ADI_TRY(dev_alloc((void**)&m->part, 4 * need, m->stream));
    m->part_cap = need;
  }
  const float* dF = m->dYf;     // fp32 gradient w.r.t. this layer's pre-activation
  const __bf16* dB = m->dYb;    // same in bf16
  for (int l = m->nl - 1; l >= 0; --l) {
    const int kin = m->kin_pad[l], no = m->width[l + 1];
    // dW_l = H_{l-1}^T dU_l (split over the batch), db_l = column sums
    GemmArgs w{};
    w.A = l > 0 ? m->H[l - 1] : m->X;
    w.lda = kin;
    w.B = dB;
    w.ldb = no;
    w.M = kin;
    w.N = no;
    w.K = (int)B;
    w.Ks = (int)Ks;
    w.out_f32 = m->part;
    w.ldo = no;
    w.split_stride = (long)kin * no;
    ADI_TRY((gemm<false, false, EPI_PARTIAL>(m, w, nsplit)));
    const long nw = (long)m->width[l] * no;
    hipLaunchKernelGGL(k_reduce_splits, dim3((int)std::min<long>((nw + 255) / 256, 2048)), dim3(256), 0,
                       m->stream, m->part, nsplit, (long)kin * no, m->width[l], no, m->Gr + m->woff[l]);
    ADI_CHECK_LAUNCH();
    const long R = colsum_rows(B);
    const int S = (int)((B + R - 1) / R);
    hipLaunchKernelGGL(k_colsum_part, dim3((no + 63) / 64, S), dim3(256), 0, m->stream, dF, B, no, R, m->colpart);
    ADI_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_colsum_final, dim3((no + 3) / 4), dim3(256), 0, m->stream, m->colpart, S, no,
                       m->Gr + m->boff[l]);
    ADI_CHECK_LAUNCH();
    if (l == 0) break;
    // dU_{l-1} = (dU_l W_l^T) * gelu'(U_{l-1})
    GemmArgs d{};
    d.A = dB;
    d.lda = no;
    d.B = m->Wb[l];  // [kin][no]: the transposed operand in [n][k] form
    d.ldb = no;
    d.M = (int)B;
    d.N = kin;
    d.K = d.Ks = no;
    d.U = m->U[l - 1];
    float* of = (dF == m->dUf) ? m->dUf2 : m->dUf;
    __bf16* ob = (dB == m->dUb) ? m->dUb2 : m->dUb;
    d.out_f32 = of;
    d.out_bf16 = ob;
    d.ldo = kin;
    ADI_TRY((gemm<true, true, EPI_DGELU>(m, d, 1)));
    dF = of;
    dB = ob;
  }
  return ADI_OK;
}

// One forward layer through k_layer when its (padded) input and output
// widths are ones it is built for, else through k_gemm.  epi: EPI_HIDDEN,
// EPI_INFER or EPI_OUTPUT.
template <int KD, int ND>
adi_status launch_layer(adi_mlp m, int epi, const __bf16* A, const __bf16* Wt, const float* bias, long B,
                        float* of, __bf16* ob) {
  const int grid = (int)std::min<long>(m->cus, (B + 255) / 256);
  if (epi == EPI_HIDDEN)
    hipLaunchKernelGGL((k_layer<KD, ND, EPI_HIDDEN>), dim3(grid), dim3(256), 0, m->stream, A, Wt, bias, B, of, ob);
  else if (epi == EPI_INFER)
    hipLaunchKernelGGL((k_layer<KD, ND, EPI_INFER>), dim3(grid), dim3(256), 0, m->stream, A, Wt, bias, B, of, ob);
  else
    hipLaunchKernelGGL((k_layer<KD, ND, EPI_OUTPUT>), dim3(grid), dim3(256), 0, m->stream, A, Wt, bias, B, of, ob);
  ADI_CHECK_LAUNCH();
  return ADI_OK;
}

// One layer: the weight-resident kernel when the batch gives every CU at
// least one workgroup of 256 rows (each workgroup first loads the whole
// layer's weights into LDS), else the tiled GEMM (64 x 64 output tiles, as
// many as the batch has).
adi_status layer_forward(adi_mlp m, int l, int epi, const __bf16* in, long B, float* of, __bf16* ob) {
  const int kd = m->kin_pad[l], nd = m->width[l + 1];
  const float* bias = m->P + m->boff[l];
  const bool resident = B >= 256L * m->cus;
  if (resident && kd == 64 && nd == 256) return launch_layer<64, 256>(m, epi, in, m->Wtb[l], bias, B, of, ob);
  if (resident && kd == 256 && nd == 256) return launch_layer<256, 256>(m, epi, in, m->Wtb[l], bias, B, of, ob);
  if (resident && kd == 256 && nd == 64) return launch_layer<256, 64>(m, epi, in, m->Wtb[l], bias, B, of, ob);
  if (resident && kd == 256 && nd == 128) return launch_layer<256, 128>(m, epi, in, m->Wtb[l], bias, B, of, ob);
  if (resident && kd == 64 && nd == 64) return launch_layer<64, 64>(m, epi, in, m->Wtb[l], bias, B, of, ob);
  GemmArgs g{};
  g.A = in;
  g.lda = kd;
  g.B = m->Wtb[l];
  g.ldb = kd;
  g.M = (int)B;
  g.N = nd;
  g.K = g.Ks = kd;
  g.bias = bias;
  g.ldo = nd;
  g.out_f32 = of;
  g.out_bf16 = ob;
  if (epi == EPI_HIDDEN) return gemm<true, true, EPI_HIDDEN>(m, g, 1);
  if (epi == EPI_INFER) return gemm<true, true, EPI_INFER>(m, g, 1);
  return gemm<true, true, EPI_OUTPUT>(m, g, 1);
}

}  // namespace

extern "C" {

adi_status adi_mlp_create(const int32_t* widths, int32_t nwidths, uint64_t seed, void* hip_stream,
                          adi_mlp* out) {
  if (!out) return fail(ADI_EINVAL, "null output handle");
  *out = nullptr;
  if (!widths || nwidths < 2 || nwidths > MAX_LAYERS + 1) return fail(ADI_EINVAL, "need 2..%d widths", MAX_LAYERS + 1);
  if (widths[0] < 1 || widths[0] > KPAD) return fail(ADI_EINVAL, "input width must be in [1, %d]", KPAD);
  for (int l = 1; l < nwidths; ++l)
    if (widths[l] < BN || widths[l] % BN || widths[l] > 4096)
      return fail(ADI_EINVAL, "layer widths must be multiples of %d (got %d)", BN, widths[l]);
  adi_mlp m = new (std::nothrow) adi_mlp_s();
  if (!m) return fail(ADI_ENOMEM, "host allocation failed");
  auto cleanup = [&](adi_status s) {
    adi_mlp_destroy(m);
    return s;
  };
  m->nl = nwidths - 1;
  for (int l = 0; l < nwidths; ++l) m->width[l] = widths[l];
  long off = 0;
  for (int l = 0; l < m->nl; ++l) {
    m->kin_pad[l] = l == 0 ? KPAD : widths[l];
    m->woff[l] = off;
    off += (long)widths[l] * widths[l + 1];
    m->boff[l] = off;
    off += widths[l + 1];
  }
  m->nparams = off;
  hipError_t e = hipGetDevice(&m->device);
  if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)));
  adi_status st = noalloc_scratch_setup(m->device);
  if (st != ADI_OK) return cleanup(st);
  e = hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, m->device);
  if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "device attribute: %s", hipGetErrorString(e)));
  m->stream = (hipStream_t)hip_stream;
  if (!m->stream) {
    e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e)));
    m->own_stream = true;
  }
  float** f32[] = {&m->P, &m->Gr, &m->Mm, &m->Vv};
  for (float** p : f32)
    if ((st = dev_alloc((void**)p, 4 * m->nparams, m->stream)) != ADI_OK) return cleanup(st);
  for (int l = 0; l < m->nl; ++l) {
    const long n = (long)m->kin_pad[l] * widths[l + 1];
    if ((st = dev_alloc((void**)&m->Wb[l], 2 * n, m->stream)) != ADI_OK) return cleanup(st);
    if ((st = dev_alloc((void**)&m->Wtb[l], 2 * n, m->stream)) != ADI_OK) return cleanup(st);
  }
  if ((st = dev_alloc((void**)&m->shift, 4 * KPAD, m->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&m->scale, 4 * KPAD, m->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&m->loss, 256, m->stream)) != ADI_OK) return cleanup(st);
  // He-normal weights, zero biases (host generator, seeded)
  std::vector<float> h(m->nparams, 0.0f);
  std::mt19937_64 rng(seed);
  for (int l = 0; l < m->nl; ++l) {
    std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / widths[l]));
    for (long i = 0; i < (long)widths[l] * widths[l + 1]; ++i) h[m->woff[l] + i] = (float)nd(rng);
  }
  std::vector<float> one(KPAD, 1.0f);
  e = hipMemcpyAsync(m->P, h.data(), 4 * m->nparams, hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m->scale, one.data(), 4 * KPAD, hipMemcpyHostToDevice, m->stream);
  if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "upload: %s", hipGetErrorString(e)));
  if ((st = refresh_weights(m)) != ADI_OK) return cleanup(st);
  e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "sync: %s", hipGetErrorString(e)));
  *out = m;
  return ADI_OK;
}

adi_status adi_mlp_num_params(adi_mlp m, int64_t* n) {
  ADI_TRY(mlp_handle(m));
  if (!n) return fail(ADI_EINVAL, "null output");
  *n = m->nparams;
  return ADI_OK;
}

adi_status adi_mlp_set_scaling(adi_mlp m, const float* shift, const float* scale) {
  ADI_TRY(mlp_handle(m));
  if (!shift || !scale) return fail(ADI_EINVAL, "null scaling array");
  std::vector<float> s(KPAD, 0.0f), c(KPAD, 1.0f);
  for (int i = 0; i < m->width[0]; ++i) {
    if (!is_fin(shift[i]) || !is_fin(scale[i])) return fail(ADI_ENONFINITE, "scaling %d is not finite", i);
    s[i] = shift[i];
    c[i] = scale[i];
  }
  ADI_HIP(hipMemcpyAsync(m->shift, s.data(), 4 * KPAD, hipMemcpyHostToDevice, m->stream));
  ADI_HIP(hipMemcpyAsync(m->scale, c.data(), 4 * KPAD, hipMemcpyHostToDevice, m->stream));
  ADI_HIP(hipStreamSynchronize(m->stream));
  return ADI_OK;
}

adi_status adi_mlp_get_params(adi_mlp m, float* host_out, int64_t count) {
  ADI_TRY(mlp_handle(m));
  if (!host_out || count != m->nparams) return fail(ADI_EINVAL, "need %ld parameters", m->nparams);
  ADI_HIP(hipMemcpyAsync(host_out, m->P, 4 * m->nparams, hipMemcpyDeviceToHost, m->stream));
  ADI_HIP(hipStreamSynchronize(m->stream));
  return ADI_OK;
}

adi_status adi_mlp_set_params(adi_mlp m, const float* host_in, int64_t count) {
  ADI_TRY(mlp_handle(m));
  if (!host_in || count != m->nparams) return fail(ADI_EINVAL, "need %ld parameters", m->nparams);
  for (long i = 0; i < m->nparams; ++i)
    if (!is_fin(host_in[i])) return fail(ADI_ENONFINITE, "parameter %ld is not finite", i);
  ADI_HIP(hipMemcpyAsync(m->P, host_in, 4 * m->nparams, hipMemcpyHostToDevice, m->stream));
  ADI_TRY(refresh_weights(m));
  ADI_HIP(hipStreamSynchronize(m->stream));
  m->step = 0;
  ADI_HIP(hipMemsetAsync(m->Mm, 0, 4 * m->nparams, m->stream));
  ADI_HIP(hipMemsetAsync(m->Vv, 0, 4 * m->nparams, m->stream));
  ADI_HIP(hipStreamSynchronize(m->stream));
  return ADI_OK;
}

adi_status adi_mlp_forward(adi_mlp m, const float* dev_x, int64_t batch, float* dev_y) {
  ADI_TRY(mlp_handle(m));
  if (!dev_x || !dev_y) return fail(ADI_EINVAL, "null device buffer");
  ADI_TRY(check_batch(m, batch));
  ADI_TRY(ensure_acts(m, batch));
  // inference only: no pre-activations kept, the output straight into dev_y
  ADI_TRY(forward_infer(m, dev_x, batch, m->X, m->H, dev_y));
  return ADI_OK;
}

adi_status adi_mlp_forward_noalloc(adi_mlp m, const float* dev_x, int64_t batch, float* dev_y) {
  ADI_TRY(mlp_handle(m));
  if (!dev_x || !dev_y) return fail(ADI_EINVAL, "null device buffer");
  ADI_TRY(check_batch(m, batch));
  int wmax = 0;
  for (int l = 1; l < m->nl; ++l) wmax = std::max(wmax, m->width[l]);
  // X: batch x KPAD, H0 and H1: batch x wmax (bf16); batch is a multiple of
  // 64 and the widths multiples of 64, so every part starts 256-byte aligned
  const long xb = 2L * batch * KPAD, hb = 2L * batch * wmax;
  const long per_row = 2L * (KPAD + 2L * wmax);
  if (xb + 2 * hb > (long)ADI_MLP_NOALLOC_SCRATCH_BYTES)
    return fail(ADI_EINVAL, "batch %ld needs %ld bytes of work area, more than the %ld available (at most %ld rows "
                "for this network)", (long)batch, xb + 2 * hb, (long)ADI_MLP_NOALLOC_SCRATCH_BYTES,
                (long)ADI_MLP_NOALLOC_SCRATCH_BYTES / per_row / BM * BM);
  unsigned char* base = (unsigned char*)noalloc_scratch_ptr(m->device);
  if (!base) return fail(ADI_EDEVICE, "work area of device %d was not set up", m->device);
  __bf16* H[MAX_LAYERS];
  for (int l = 0; l < MAX_LAYERS; ++l) H[l] = (__bf16*)(base + xb + (l & 1) * hb);
  return forward_infer(m, dev_x, batch, (__bf16*)base, H, dev_y);
}

adi_status adi_mlp_sync(adi_mlp m) {
  ADI_TRY(mlp_handle(m));
  ADI_HIP(hipStreamSynchronize(m->stream));
  return ADI_OK;
}

adi_status adi_mlp_gradients(adi_mlp m, const float* dev_x, const float* dev_t, int64_t batch, float* host_grads,
                             float* loss_out) {
  ADI_TRY(mlp_handle(m));
  if (!dev_x || !dev_t) return fail(ADI_EINVAL, "null device buffer");
  ADI_TRY(check_batch(m, batch));
  ADI_TRY(ensure_acts(m, batch));
  ADI_TRY(forward(m, dev_x, batch));
  ADI_TRY(backward(m, dev_t, batch));
  if (host_grads) ADI_HIP(hipMemcpyAsync(host_grads, m->Gr, 4 * m->nparams, hipMemcpyDeviceToHost, m->stream));
  if (loss_out) ADI_HIP(hipMemcpyAsync(loss_out, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
  ADI_HIP(hipStreamSynchronize(m->stream));
  return ADI_OK;
}

adi_status adi_mlp_train_step(adi_mlp m, const float* dev_x, const float* dev_t, int64_t batch, float lr,
                              float* loss_out) {
  ADI_TRY(mlp_handle(m));
  if (!dev_x || !dev_t) return fail(ADI_EINVAL, "null device buffer");
  if (!(lr >= 0.0f) || !is_fin(lr)) return fail(ADI_EINVAL, "learning rate must be >= 0");
  ADI_TRY(check_batch(m, batch));
  ADI_TRY(ensure_acts(m, batch));
  ADI_TRY(forward(m, dev_x, batch));
  ADI_TRY(backward(m, dev_t, batch));
  m->step += 1;
  const float c1 = 1.0f - std::pow(m->b1, (float)m->step), c2 = 1.0f - std::pow(m->b2, (float)m->step);
  hipLaunchKernelGGL(k_adam, dim3((int)std::min<long>((m->nparams + 255) / 256, 2048)), dim3(256), 0, m->stream,
                     m->P, m->Gr, m->Mm, m->Vv, m->nparams, lr, m->b1, m->b2, m->eps, c1, c2);
  ADI_CHECK_LAUNCH();
  ADI_TRY(refresh_weights(m));
  if (loss_out) {
    ADI_HIP(hipMemcpyAsync(loss_out, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
    ADI_HIP(hipStreamSynchronize(m->stream));
  }
  return ADI_OK;
}

void adi_mlp_destroy(adi_mlp m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  free_acts(m);
  void* b[] = {m->P, m->Gr, m->Mm, m->Vv, m->shift, m->scale, m->part, m->loss};
  for (void* p : b) dev_free(p);
  for (int l = 0; l < MAX_LAYERS; ++l) {
    dev_free(m->Wb[l]);
    dev_free(m->Wtb[l]);
  }
  if (m->own_stream) (void)hipStreamDestroy(m->stream);
  delete m;
}

}  // extern "C"
