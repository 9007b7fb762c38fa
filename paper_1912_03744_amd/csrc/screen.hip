// screen.hip -- device reductions of the surrogate-screened design sweep:
// the ensemble's outputs decoded into each design's predicted profile, its
// peak, the members' disagreement and the maximum-principle check, and the
// selection of the k largest values, so that the predictions of a sweep
// never leave the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace adi {
namespace {

constexpr int SCREEN_NPTS = 64;  // profile points: one per lane of a wave

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// One wave per design, lane k on profile point k.  pred: [members][n][nout]
// fp32, outputs 0..63 the profile's shape, 64..nout-1 its standardised log
// scale (their mean is used).  A member's profile is y_k = exp(mu + sd *
// scale) * shape_k; the ensemble's is the mean over the members.
__global__ void __launch_bounds__(256) k_screen(const float* __restrict__ pred, int members, long n, int nout,
                                                double mu, double sd, double floor_, const double* __restrict__ qt,
                                                double* __restrict__ peak, double* __restrict__ dis,
                                                uint8_t* __restrict__ bound_ok) {
  const int lane = threadIdx.x & 63;
  const long first = (blockIdx.x * (long)blockDim.x + threadIdx.x) >> 6;
  const long stride = (gridDim.x * (long)blockDim.x) >> 6;
  const int nsc = nout - SCREEN_NPTS;
  for (long d = first; d < n; d += stride) {
    double ysum = 0.0, y0 = 0.0, ylast = 0.0;
    for (int m = 0; m < members; ++m) {
      const float* row = pred + ((long)m * n + d) * nout;
      double sc = 0.0;
      for (int c = SCREEN_NPTS + lane; c < nout; c += SCREEN_NPTS) sc += (double)row[c];
      sc = wave_sum(sc) / nsc;
      const double y = exp(mu + sd * sc) * (double)row[lane];
      ysum += y;
      if (m == 0) y0 = y;
      if (m == members - 1) ylast = y;
    }
    const double ybar = ysum / members;
    const double ymax = wave_max(ybar);
    const double dmax = wave_max(fabs(y0 - ylast));
    const bool bad = __any(!(ybar <= 1.0 + 1e-3));
    if (lane == 0) {
      peak[d] = ymax * (qt ? qt[d] : 1.0);
      dis[d] = dmax / fmax(ymax, floor_);
      bound_ok[d] = bad ? 0 : 1;
    }
  }
}

// Order-preserving 64-bit key of a double (NaN below every number, -0 and
// +0 equal).
__device__ __forceinline__ unsigned long long order_key(double x) {
  if (x != x) return 0ull;
  if (x == 0.0) x = 0.0;
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}

constexpr int TOPK_BLOCK = 1024;

// Histogram of the digit at `shift` (8 bits) over the keys whose higher
// digits equal `prefix` (under `mask`).
__global__ void __launch_bounds__(256) k_digit_hist(const double* __restrict__ v, long n, unsigned long long prefix,
                                                    unsigned long long mask, int shift, unsigned* __restrict__ hist) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const unsigned long long k = order_key(v[i]);
    if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

// Rank of each lane's flag among the block's flagged elements before it
// (index order) and the block's total.  Every lane of the block calls it.
__device__ __forceinline__ unsigned block_rank(bool flag, unsigned* wtot, unsigned* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long ball = __ballot(flag);
  const unsigned before = __popcll(ball & ((1ull << lane) - 1ull));
  if (lane == 0) wtot[w] = __popcll(ball);
  __syncthreads();
  unsigned off = 0, sum = 0;
  for (int q = 0; q < TOPK_BLOCK / 64; ++q) {
    if (q < w) off += wtot[q];
    sum += wtot[q];
  }
  __syncthreads();
  *total = sum;
  return off + before;
}

// Per block of TOPK_BLOCK elements: how many keys lie above `kth` and how
// many equal it.
__global__ void __launch_bounds__(TOPK_BLOCK) k_topk_count(const double* __restrict__ v, long n,
                                                           unsigned long long kth, unsigned* __restrict__ cnt) {
  __shared__ unsigned wtot[TOPK_BLOCK / 64];
  const long i = blockIdx.x * (long)TOPK_BLOCK + threadIdx.x;
  const unsigned long long k = i < n ? order_key(v[i]) : 0ull;
  unsigned tg, te;
  block_rank(i < n && k > kth, wtot, &tg);
  block_rank(i < n && k == kth, wtot, &te);
  if (threadIdx.x == 0) {
    cnt[2 * blockIdx.x] = tg;
    cnt[2 * blockIdx.x + 1] = te;
  }
}

// Write the indices of the keys above `kth` (from out[0], index order) and
// of the first `ties` keys equal to it (from out[n_gt], index order); off:
// per block, the exclusive prefix counts of both kinds.
__global__ void __launch_bounds__(TOPK_BLOCK) k_topk_write(const double* __restrict__ v, long n,
                                                           unsigned long long kth, const long* __restrict__ off,
                                                           long n_gt, long ties, int64_t* __restrict__ out) {
  __shared__ unsigned wtot[TOPK_BLOCK / 64];
  const long i = blockIdx.x * (long)TOPK_BLOCK + threadIdx.x;
  const unsigned long long k = i < n ? order_key(v[i]) : 0ull;
  const bool gt = i < n && k > kth, eq = i < n && k == kth;
  unsigned tot;
  const unsigned rg = block_rank(gt, wtot, &tot);
  const unsigned re = block_rank(eq, wtot, &tot);
  if (gt) out[off[2 * blockIdx.x] + rg] = i;
  if (eq) {
    const long r = off[2 * blockIdx.x + 1] + re;
    if (r < ties) out[n_gt + r] = i;
  }
}

}  // namespace
}  // namespace adi

using namespace adi;

extern "C" {

adi_status adi_screen_profiles(const float* dev_pred, int32_t members, int64_t n, int32_t nout, double mu,
                               double sd, double floor_, const double* dev_qt, double* dev_peak, double* dev_dis,
                               uint8_t* dev_bound_ok, void* hip_stream) {
  if (members < 1) return fail(ADI_EINVAL, "members must be >= 1");
  if (n < 0) return fail(ADI_EINVAL, "n must be >= 0");
  if (nout <= SCREEN_NPTS || nout > 4096) return fail(ADI_EINVAL, "nout must be in (64, 4096]");
  if (!is_fin(mu) || !is_fin(sd) || !(floor_ > 0.0) || !is_fin(floor_))
    return fail(ADI_EINVAL, "mu, sd must be finite and floor > 0");
  if (n == 0) return ADI_OK;
  if (!dev_pred || !dev_peak || !dev_dis || !dev_bound_ok) return fail(ADI_EINVAL, "null device buffer");
  hipStream_t st = (hipStream_t)hip_stream;
  const long waves = std::min<long>(n, 1L << 16);
  hipLaunchKernelGGL(k_screen, dim3((int)((waves + 3) / 4)), dim3(256), 0, st, dev_pred, (int)members, (long)n,
                     (int)nout, mu, sd, floor_, dev_qt, dev_peak, dev_dis, dev_bound_ok);
  ADI_CHECK_LAUNCH();
  return ADI_OK;
}

adi_status adi_top_k(const double* dev_vals, int64_t n, int32_t k, int64_t* dev_idx, void* hip_stream) {
  if (n < 1 || n > (1LL << 40)) return fail(ADI_EINVAL, "n must be in [1, 2^40]");
  if (k < 1 || k > n) return fail(ADI_EINVAL, "k must be in [1, n]");
  if (!dev_vals || !dev_idx) return fail(ADI_EINVAL, "null device buffer");
  hipStream_t st = (hipStream_t)hip_stream;
  const long nblk = (n + TOPK_BLOCK - 1) / TOPK_BLOCK;
  unsigned* hist = nullptr;
  unsigned* cnt = nullptr;
  long* off = nullptr;
  adi_status s = dev_alloc((void**)&hist, 256 * sizeof(unsigned), st);
  if (s == ADI_OK) s = dev_alloc((void**)&cnt, 2 * nblk * sizeof(unsigned), st);
  if (s == ADI_OK) s = dev_alloc((void**)&off, 2 * nblk * sizeof(long), st);
  auto done = [&](adi_status r) {
    (void)hipStreamSynchronize(st);
    dev_free(hist);
    dev_free(cnt);
    dev_free(off);
    return r;
  };
  if (s != ADI_OK) return done(s);
  // radix selection of the k-th largest key, 8 bits at a time
  unsigned long long prefix = 0, mask = 0;
  long remaining = k;
  unsigned h[256];
  const int hist_blocks = (int)std::min<long>((n + 255) / 256, 2048);
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipError_t e = hipMemsetAsync(hist, 0, 256 * sizeof(unsigned), st);
    if (e != hipSuccess) return done(fail(ADI_EDEVICE, "clearing the histogram: %s", hipGetErrorString(e)));
    hipLaunchKernelGGL(k_digit_hist, dim3(hist_blocks), dim3(256), 0, st, dev_vals, (long)n, prefix, mask, shift,
                       hist);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, hist, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return done(fail(ADI_EDEVICE, "digit histogram: %s", hipGetErrorString(e)));
    int dg = 255;
    for (; dg > 0 && (long)h[dg] < remaining; --dg) remaining -= h[dg];
    prefix |= (unsigned long long)dg << shift;
    mask |= 255ull << shift;
  }
  // `remaining` of the keys equal to the k-th are taken, k - remaining lie above it
  const long n_gt = k - remaining;
  hipLaunchKernelGGL(k_topk_count, dim3((unsigned)nblk), dim3(TOPK_BLOCK), 0, st, dev_vals, (long)n, prefix, cnt);
  hipError_t e = hipGetLastError();
  std::vector<unsigned> c(2 * nblk);
  std::vector<long> o(2 * nblk);
  if (e == hipSuccess) e = hipMemcpyAsync(c.data(), cnt, c.size() * sizeof(unsigned), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return done(fail(ADI_EDEVICE, "selection counts: %s", hipGetErrorString(e)));
  long sg = 0, se = 0;
  for (long b = 0; b < nblk; ++b) {
    o[2 * b] = sg;
    o[2 * b + 1] = se;
    sg += c[2 * b];
    se += c[2 * b + 1];
  }
  if (sg != n_gt || se < remaining) return done(fail(ADI_EDEVICE, "inconsistent selection counts"));
  e = hipMemcpyAsync(off, o.data(), o.size() * sizeof(long), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_topk_write, dim3((unsigned)nblk), dim3(TOPK_BLOCK), 0, st, dev_vals, (long)n, prefix, off,
                       n_gt, remaining, dev_idx);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return done(fail(ADI_EDEVICE, "selection: %s", hipGetErrorString(e)));
  return done(ADI_OK);
}

}  // extern "C"
