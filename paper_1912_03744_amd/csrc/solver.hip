// solver.hip -- single-instance ADI solver: kernels and the adi_* problem ABI.
//
// Each time step is two sweeps (r lines, then z lines); each sweep reads the
// right-hand side of its half step, solves every line with the partition
// solver of device.hpp and writes the right-hand side of the next half step
// (and, when asked, the solution).  Per step the field moves through HBM
// exactly twice: 8 B read + 8 B written per active cell per half step.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <unordered_map>
#include <mutex>

#include "common.hpp"
#include "device.hpp"
#include "strip.hpp"
#include "resident.hpp"
#include "problem_core.hpp"

namespace adi {

// ------------------------------------------------------------- errors ----

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
  char buf[768];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

// Device allocations: hipMalloc / hipFree, or the caller's allocator
// (adi_set_allocator).  Every block from the caller's allocator is recorded
// with the free function that owns it, so a later change of allocator still
// returns it to the right one.
namespace {
struct HookOwner {
  adi_free_fn free_fn;
  void* ctx;
};
std::mutex g_alloc_mu;
adi_alloc_fn g_alloc_fn = nullptr;
adi_free_fn g_free_fn = nullptr;
void* g_alloc_ctx = nullptr;
std::unordered_map<void*, HookOwner>& hooked_blocks() {
  static std::unordered_map<void*, HookOwner> m;
  return m;
}
}  // namespace

adi_status dev_alloc(void** p, size_t bytes, hipStream_t stream) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  adi_alloc_fn al;
  adi_free_fn fr;
  void* ctx;
  {
    std::lock_guard<std::mutex> g(g_alloc_mu);
    al = g_alloc_fn;
    fr = g_free_fn;
    ctx = g_alloc_ctx;
  }
  if (al) {
    void* q = al(bytes, ctx);
    if (!q) return fail(ADI_ENOMEM, "allocator hook returned no memory for %zu bytes", bytes);
    if ((uintptr_t)q % 256 != 0) {
      fr(q, ctx);
      return fail(ADI_EINVAL, "allocator hook returned a block not aligned to 256 bytes");
    }
    {
      std::lock_guard<std::mutex> g(g_alloc_mu);
      hooked_blocks()[q] = {fr, ctx};
    }
    *p = q;
  } else {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      *p = nullptr;
      return fail(e == hipErrorOutOfMemory ? ADI_ENOMEM : ADI_EDEVICE, "hipMalloc(%zu) failed: %s",
                  bytes, hipGetErrorString(e));
    }
  }
  hipError_t e = hipMemsetAsync(*p, 0, bytes, stream);
  if (e != hipSuccess) return fail(ADI_EDEVICE, "hipMemsetAsync failed: %s", hipGetErrorString(e));
  return ADI_OK;
}

void dev_free(void* p) {
  if (!p) return;
  HookOwner o{nullptr, nullptr};
  {
    std::lock_guard<std::mutex> g(g_alloc_mu);
    auto it = hooked_blocks().find(p);
    if (it != hooked_blocks().end()) {
      o = it->second;
      hooked_blocks().erase(it);
    }
  }
  if (o.free_fn) {
    // like hipFree: no work of the library still uses the block when the
    // caller's allocator gets it back
    (void)hipDeviceSynchronize();
    o.free_fn(p, o.ctx);
  } else {
    (void)hipFree(p);
  }
}

// ------------------------------------------------------------ kernels ----

__global__ void k_geometry(Params P, const double* rfi, const double* zfi, Geom g, int* ranges) {
  build_geometry(P, rfi, zfi, g, ranges);
}

// Tables of one direction.
struct DirTabs {
  LineTab* tabs;
  double *pos, *chk, *eng, *xc, *work;
  int ncls, n, G, M;
  int paired;  // tables in the paired layout (read by the strip-layout sweeps)
};

// One workgroup per line class: r bands first, then z column classes.
__global__ void __launch_bounds__(256) k_assemble(Params P, Geom g, DirTabs r, DirTabs z) {
  const bool isr = (int)blockIdx.x < r.ncls;
  const DirTabs D = isr ? r : z;
  const int dir = isr ? 0 : 1;
  const int cls = isr ? blockIdx.x : blockIdx.x - r.ncls;
  const long GM = (long)D.G * D.M;
  double* pos = D.pos + cls * P_NFIELDS * GM;
  double* chk = D.chk + (long)cls * C_NFIELDS * D.G;
  double* eng = D.eng + (long)cls * 2 * D.n;
  double* xc = D.xc + (long)cls * D.n;
  double* work = D.work + cls * assemble_work(D.G, D.M);
  assemble_class(P, g, dir, cls, D.G, D.M, pos, chk, eng, xc, work, D.paired != 0);
  if (threadIdx.x == 0) {
    // cells outside the domain form one contiguous run of a line
    int lo = D.n, hi = D.n, cnt = 0;
    for (int p = 0; p < D.n; ++p) {
      const int m = dir == 0 ? region_of(cls, g.kap[p]) : region_of(g.bet[p], cls);
      if (m == MASKED) {
        if (cnt == 0) lo = p;
        hi = p + 1;
        ++cnt;
      }
    }
    if (cnt != hi - lo) lo = hi = D.n;  // not contiguous: skip nothing
    LineTab t;
    t.pos = pos;
    t.chk = chk;
    t.n = D.n;
    t.G = D.G;
    t.M = D.M;
    t.skip_lo = cnt ? lo : D.n;
    t.skip_hi = cnt ? hi : D.n;
    D.tabs[cls] = t;
  }
}

// Right-hand side of the first r half step from a field T: the z-direction
// output operator applied to T plus the r boundary constant.  Every element
// of the buffer is written: cells outside the domain and padding get exactly
// 0, which the strip sweeps rely on.  strip = 0: rows layout (nr*nz
// elements); else strip layout with `total` elements.
__global__ void k_init_rhs(const double* __restrict__ T, double* __restrict__ d, Geom g,
                           DirTabs z, const double* __restrict__ rxc, int nr, int nz, long strip, long total) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int i, j;
    if (strip) {
      const long s = e / strip, rem = e - s * strip;
      j = (int)(rem >> 2);
      i = (int)(4 * s + (rem & 3));
    } else {
      i = (int)(e % nr);
      j = (int)(e / nr);
    }
    double o = 0.0;
    if (i < nr && j < nz) {
      const int kap = g.kap[i], bet = g.bet[j];
      if (region_of(bet, kap) != MASKED) {
        const long c = (long)j * nr + i;
        const long GM = (long)z.G * z.M;
        const double* pos = z.pos + kap * P_NFIELDS * GM;
        const long ix = (long)(j % z.M) * z.G + j / z.M;
        o = pos[pos_at(P_OD, GM, ix, z.paired != 0)] * T[c] + pos[pos_at(P_OC, GM, ix, z.paired != 0)] + rxc[(long)bet * nr + i];
        if (j > 0) o += pos[pos_at(P_OL, GM, ix, z.paired != 0)] * T[c - nr];
        if (j < nz - 1) o += pos[pos_at(P_OU, GM, ix, z.paired != 0)] * T[c + nr];
      }
    }
    d[e] = o;
  }
}

// NGW line groups per workgroup, WPL waves per group.  The grid has one
// workgroup per NGW line groups.  Lines along contiguous memory (r) and
// across it (z) are separate instantiations.
template <int M, int LPW, int WPL, int R, int NGW>
__global__ void __launch_bounds__(64 * WPL * NGW) k_sweep(SweepArgs a) {
  __shared__ double lds[NGW][WPL > 1 ? WPL * LPW * (R + 1) : 1];
  const int wave = threadIdx.x >> 6;
  const int gw = wave / WPL;
  const int wv = wave % WPL;
  const int group = xcd_block(blockIdx.x, gridDim.x) * NGW + gw;
  if (a.pos_stride == 1)
    solve_group<M, LPW, WPL, R, true>(a, group, lds[gw], group < a.ngroups, wv);
  else
    solve_group<M, LPW, WPL, R, false>(a, group, lds[gw], group < a.ngroups, wv);
}

// Energy and boundary flows of a field, one workgroup per row, fixed-order
// tree in LDS.  part[j*4 + {0,1,2,3}] = E, B_r, B_z, P of row j.
__global__ void __launch_bounds__(256) k_energy_rows(const double* __restrict__ T, Params P, Geom g,
                                                     DirTabs r, DirTabs z, double* part) {
  __shared__ double s[4][256];
  const int j = blockIdx.x;
  const int nr = P.nr;
  double e = 0.0, br = 0.0, bz = 0.0, pw = 0.0;
  const int bet = g.bet[j];
  for (int i = threadIdx.x; i < nr; i += blockDim.x) {
    const int kap = g.kap[i];
    const int m = region_of(bet, kap);
    if (m == MASKED) continue;
    const double t = T[(long)j * nr + i];
    const double vr = g.rc[i] * g.dr[i];
    const double V = vr * g.dz[j];
    e += P.rhoc[m] * t * V;
    pw += P.q[m] * V;
    const double* er = r.eng + (long)bet * 2 * r.n;
    br += g.dz[j] * (er[i] * t - er[r.n + i]);
    const double* ez = z.eng + (long)kap * 2 * z.n;
    bz += vr * (ez[j] * t - ez[z.n + j]);
  }
  s[0][threadIdx.x] = e;
  s[1][threadIdx.x] = br;
  s[2][threadIdx.x] = bz;
  s[3][threadIdx.x] = pw;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[(long)j * 4 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_energy_final(const double* __restrict__ part, int nrows, double* out) {
  __shared__ double s[4][256];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < nrows; j += blockDim.x)
    for (int q = 0; q < 4; ++q) acc[q] += part[(long)j * 4 + q];
  for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

// Energy identity of one step from the reductions of T^n, the intermediate
// field and T^{n+1}.  state: [0] largest relative residual, [1] non-finite
// flag, [2] violation flag, [3] number of checks.
__global__ void k_check(const double* e0, const double* em, const double* e1, double ta, int scheme,
                        double tol, double* state) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double P = e0[3];
  double rhs, scale;
  if (scheme == ADI_PR) {
    rhs = ta * (2.0 * P - 2.0 * em[1] - e0[2] - e1[2]);
    scale = fabs(e0[0]) + fabs(e1[0]) + ta * (2.0 * fabs(P) + 2.0 * fabs(em[1]) + fabs(e0[2]) + fabs(e1[2]));
  } else {
    rhs = ta * (P - em[1] - e1[2]);
    scale = fabs(e0[0]) + fabs(e1[0]) + ta * (fabs(P) + fabs(em[1]) + fabs(e1[2]));
  }
  const double lhs = e1[0] - e0[0];
  const double rel = scale > 0.0 ? fabs(lhs - rhs) / scale : fabs(lhs - rhs);
  const bool fin = isfinite(lhs) && isfinite(rhs) && isfinite(rel);
  if (!fin) state[1] = 1.0;
  else {
    state[0] = fmax(state[0], rel);
    if (rel > tol) state[2] = 1.0;
  }
  state[3] += 1.0;
}

__global__ void k_region_map(Geom g, int nr, int nz, uint8_t* out) {
  const long n = (long)nr * nz;
  for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n; c += (long)gridDim.x * blockDim.x)
    out[c] = (uint8_t)region_of(g.bet[c / nr], g.kap[c % nr]);
}

// Set T = T0 on active cells (when fill) and 0 outside the domain.
__global__ void k_set_field(double* T, Geom g, int nr, int nz, int fill, double T0) {
  const long n = (long)nr * nz;
  for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n; c += (long)gridDim.x * blockDim.x) {
    if (region_of(g.bet[c / nr], g.kap[c % nr]) == MASKED) T[c] = 0.0;
    else if (fill) T[c] = T0;
  }
}

// Linear resampling of one row at r_k = (k+0.5)*rmax/npts.
__global__ void k_profile(const double* __restrict__ T, Geom g, int nr, int row, double rmax, int npts,
                          double* out) {
  const double* v = T + (long)row * nr;
  for (int kk = blockIdx.x * blockDim.x + threadIdx.x; kk < npts; kk += gridDim.x * blockDim.x) {
    const double r = (kk + 0.5) * rmax / npts;
    double o;
    if (r <= g.rc[0]) o = v[0];
    else if (r >= g.rc[nr - 1]) o = v[nr - 1];
    else {
      int lo = 0, hi = nr - 1;  // rc[lo] <= r < rc[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g.rc[mid] <= r) lo = mid; else hi = mid;
      }
      o = v[lo] + (v[lo + 1] - v[lo]) * (r - g.rc[lo]) / (g.rc[lo + 1] - g.rc[lo]);
    }
    out[kk] = o;
  }
}

__global__ void k_clear(double* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

// ------------------------------------------------------- sweep variants ----

using SweepFn = void (*)(SweepArgs);
struct Variant {
  int M, LPW, WPL, R, NGW;
  SweepFn fn;
};

// Compiled launch shapes: cells per chunk M, lines per wave slot group LPW
// (lanes split into LPW slots x 64/LPW chunks), waves per line WPL, lines
// per lane R, line groups per workgroup NGW.  A line of n cells runs on any
// shape with (64/LPW)*WPL*M >= n.
#define ADI_V(m, lpw, wpl, r, ngw) {m, lpw, wpl, r, ngw, k_sweep<m, lpw, wpl, r, ngw>}
static const Variant kVariants[] = {
    // contiguous lines (r)
    ADI_V(4, 1, 4, 2, 1), ADI_V(4, 1, 4, 4, 1), ADI_V(4, 1, 4, 8, 1), ADI_V(8, 1, 2, 4, 1),
    ADI_V(8, 1, 2, 8, 1), ADI_V(16, 1, 1, 2, 4), ADI_V(4, 2, 4, 4, 1), ADI_V(8, 1, 2, 2, 2),
    // strided lines (z)
    ADI_V(10, 4, 16, 1, 1), ADI_V(10, 4, 16, 2, 1), ADI_V(5, 2, 16, 4, 1), ADI_V(5, 2, 16, 2, 1),
    ADI_V(5, 1, 8, 8, 1), ADI_V(5, 1, 8, 4, 1), ADI_V(10, 1, 4, 4, 1), ADI_V(10, 2, 8, 4, 1),
    ADI_V(20, 8, 16, 1, 1), ADI_V(10, 8, 8, 2, 1), ADI_V(5, 4, 16, 2, 1),
    // small lines (tests, single layout, batch sizes)
    ADI_V(3, 1, 1, 1, 4), ADI_V(6, 2, 1, 1, 4), ADI_V(3, 2, 1, 2, 4), ADI_V(4, 4, 1, 2, 4),
    ADI_V(8, 4, 1, 1, 4), ADI_V(12, 4, 1, 1, 4), ADI_V(6, 4, 2, 1, 2), ADI_V(4, 16, 1, 1, 4),
    ADI_V(8, 16, 1, 2, 4), ADI_V(10, 8, 2, 1, 2), ADI_V(5, 8, 4, 2, 1), ADI_V(10, 16, 4, 1, 1),
    ADI_V(15, 16, 8, 1, 1), ADI_V(8, 16, 4, 2, 1), ADI_V(12, 16, 2, 1, 2),
    // long lines (up to 8192 cells)
    ADI_V(8, 1, 4, 2, 1), ADI_V(16, 1, 4, 1, 1), ADI_V(12, 4, 16, 1, 1), ADI_V(6, 2, 16, 2, 1),
    ADI_V(32, 4, 16, 1, 1),
};
#undef ADI_V
static const int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

static int find_variant(int M, int LPW, int WPL, int R, int NGW) {
  for (int v = 0; v < kNumVariants; ++v) {
    const Variant& V = kVariants[v];
    if (V.M == M && V.LPW == LPW && V.WPL == WPL && V.R == R && V.NGW == NGW) return v;
  }
  return -1;
}

// Strip-layout kernels: r sweeps take 4 cells per chunk and NW waves (lines
// up to 256*NW cells); z sweeps take M cells per chunk and NW waves (lines up
// to 64*NW*M cells, LDS 8*64*NW*(4M+2) bytes).
using StripFn = void (*)(StripArgs);
struct StripVariant {
  int dir, M, NW;
  StripFn fn;
};
#define ADI_SR(nw) {0, 4, nw, k_sweep_rs<nw>}
#define ADI_SZ(m, nw) {1, m, nw, k_sweep_zs<m, nw>}
static const StripVariant kStrip[] = {
    ADI_SR(1), ADI_SR(2), ADI_SR(4), ADI_SR(8),
    ADI_SZ(3, 1), ADI_SZ(5, 1), ADI_SZ(8, 1), ADI_SZ(5, 2), ADI_SZ(8, 2), ADI_SZ(5, 4), ADI_SZ(10, 4),
    ADI_SZ(4, 8), ADI_SZ(5, 8), ADI_SZ(3, 16),
};
#undef ADI_SR
#undef ADI_SZ
static const int kNumStrip = sizeof(kStrip) / sizeof(kStrip[0]);

static int find_strip(int dir, int M, int NW) {
  for (int v = 0; v < kNumStrip; ++v)
    if (kStrip[v].dir == dir && kStrip[v].M == M && kStrip[v].NW == NW) return v;
  return -1;
}

}  // namespace adi

using namespace adi;

// ------------------------------------------------------------ problem ----

namespace {

struct Launch {
  int M = 0, LPW = 0, WPL = 0, R = 1, NGW = 1;  // shape
  int G = 0, variant = -1;
  int layout = ADI_LAYOUT_ROWS;  // kernel family; variant indexes kVariants or kStrip
};

struct DirState {
  Launch L;
  int n = 0, nlines = 0, ncls = 0;
  LineTab* tabs = nullptr;
  LineTab htabs[MAX_CLS] = {};  // host copy (the strip kernels take them by value)
  double *pos = nullptr, *chk = nullptr, *eng = nullptr, *xc = nullptr, *work = nullptr;
  DirTabs view() const {
    DirTabs d;
    d.tabs = tabs; d.pos = pos; d.chk = chk; d.eng = eng; d.xc = xc; d.work = work;
    d.ncls = ncls; d.n = n; d.G = L.G; d.M = L.M;
    d.paired = L.layout == ADI_LAYOUT_STRIPS;  // the strip sweeps read pairs
    return d;
  }
};

adi_status validate_strip_launch(int dir, int n, int chunk, int lpw, int wpl, int r, int ngw, Launch* out) {
  const int v = lpw == 1 && r == 4 && ngw == 1 ? find_strip(dir, chunk, wpl) : -1;
  if (v < 0)
    return fail(ADI_EUNSUPPORTED, "no strip-layout %s kernel for chunk %d, %d lines/wave, %d waves, %d lines/lane, "
                "%d groups/block", dir == 0 ? "r" : "z", chunk, lpw, wpl, r, ngw);
  const int G = 64 * wpl;
  if ((long)G * chunk < n)
    return fail(ADI_EINVAL, "%d chunks of %d cells do not cover a line of %d", G, chunk, n);
  out->M = chunk; out->LPW = 1; out->WPL = wpl; out->R = 4; out->NGW = 1;
  out->G = G; out->variant = v; out->layout = ADI_LAYOUT_STRIPS;
  return ADI_OK;
}

// Strip-layout default: least padding, then the most waves up to 8.
bool default_strip_launch(int dir, int n, Launch* out) {
  int best = -1;
  double best_score = -1e300;
  for (int v = 0; v < kNumStrip; ++v) {
    const StripVariant& V = kStrip[v];
    if (V.dir != dir) continue;
    const long cover = 64L * V.NW * V.M;
    if (cover < n) continue;
    const double score = -8.0 * std::log2((double)cover / n) - std::fabs(std::log2(V.NW / 8.0));
    if (score > best_score) best_score = score, best = v;
  }
  if (best < 0) return false;
  Launch L;
  L.M = kStrip[best].M; L.LPW = 1; L.WPL = kStrip[best].NW; L.R = 4; L.NGW = 1;
  L.G = 64 * L.WPL; L.variant = best; L.layout = ADI_LAYOUT_STRIPS;
  *out = L;
  return true;
}

adi_status validate_launch(int n, int chunk, int lpw, int wpl, int r, int ngw, Launch* out) {
  const int v = find_variant(chunk, lpw, wpl, r, ngw);
  if (v < 0)
    return fail(ADI_EUNSUPPORTED, "no kernel for chunk %d, %d lines/wave, %d waves/line, %d lines/lane, "
                "%d groups/block", chunk, lpw, wpl, r, ngw);
  const int G = (64 / lpw) * wpl;
  if ((long)G * chunk < n)
    return fail(ADI_EINVAL, "%d chunks of %d cells do not cover a line of %d", G, chunk, n);
  out->M = chunk; out->LPW = lpw; out->WPL = wpl; out->R = r; out->NGW = ngw;
  out->G = G; out->variant = v;
  return ADI_OK;
}

// Default launch shape: lines along contiguous memory use one line per wave
// group; strided lines put 16 adjacent lines side by side in a wave so every
// load instruction reads whole 128-byte rows.
Launch default_launch(int dir, int n, int nlines) {
  Launch best;
  double best_score = -1e300;
  for (int v = 0; v < kNumVariants; ++v) {
    const Variant& V = kVariants[v];
    const int G = (64 / V.LPW) * V.WPL;
    if ((long)G * V.M < n) continue;
    const double pad = (double)G * V.M / n;                     // >= 1
    const double lines = (double)V.LPW * V.R * V.NGW;            // lines per workgroup pass
    double score = -8.0 * std::log2(pad);                       // wasted padded cells
    score -= 1.0 * std::fabs(std::log2((double)V.M * V.R / 16.0));  // ~16 cells per lane
    score -= 2.0 * std::max(0.0, std::log2(lines / std::max(1, nlines / 64)));  // keep >= 64 groups
    if (dir == 1) score += 1.0 * std::log2((double)V.LPW * V.R);   // adjacent columns per row
    if (score > best_score) {
      best_score = score;
      Launch L;
      L.M = V.M; L.LPW = V.LPW; L.WPL = V.WPL; L.R = V.R; L.NGW = V.NGW; L.G = G; L.variant = v;
      best = L;
    }
  }
  return best;
}

}  // namespace

struct adi_problem_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  adi_scheme scheme = ADI_PR;
  Params P{};
  std::vector<double> h_rf, h_zf;
  double *d_rfi = nullptr, *d_zfi = nullptr;
  Geom g{};
  void* geom_mem = nullptr;
  bool geom_built = false;
  bool has_mat = false, has_src = false;
  DirState r, z;
  void* tab_mem = nullptr;
  bool tabs_valid = false;
  double tabs_dt = 0.0;
  bool rhs_valid = false;
  double *T = nullptr, *dA = nullptr, *dB = nullptr, *mid = nullptr;
  int layout = ADI_LAYOUT_ROWS;  // layout of dA / dB (and of mid when a z sweep writes it)
  long strip = 0;                // doubles per strip in the strip layout
  double *part = nullptr, *eout = nullptr, *state = nullptr, *prof = nullptr;
  uint8_t* dmap = nullptr;
  int* dranges = nullptr;
  int ranges[17] = {0};
  int check_every = 0;
  double check_tol = 1e-9;
  int64_t steps = 0;
  double time = 0.0;
  double E0 = 0.0;
  bool E0_valid = false;
  std::vector<uint8_t> hmap;
  int graph_steps = 0;
  // captured segments: (steps, check-first) -> executable graph
  struct Seg {
    int steps;
    bool check;
    hipGraphExec_t exec;
  };
  std::vector<Seg> graphs;
  // extension state (the nonlinear path) and its destructor
  void* ext = nullptr;
  void (*ext_destroy)(void*) = nullptr;
};

namespace {

adi_status check_handle(adi_problem p) {
  if (!p) return fail(ADI_EINVAL, "null problem handle");
  ADI_HIP(hipSetDevice(p->device));
  return ADI_OK;
}

void drop_graphs(adi_problem p) {
  for (auto& s : p->graphs) (void)hipGraphExecDestroy(s.exec);
  p->graphs.clear();
}

adi_status build_geometry_once(adi_problem p) {
  if (p->geom_built) return ADI_OK;
  hipLaunchKernelGGL(k_geometry, dim3(1), dim3(256), 0, p->stream, p->P, p->d_rfi, p->d_zfi, p->g,
                     p->dranges);
  ADI_CHECK_LAUNCH();
  ADI_HIP(hipMemcpyAsync(p->ranges, p->dranges, sizeof p->ranges, hipMemcpyDeviceToHost, p->stream));
  ADI_HIP(hipStreamSynchronize(p->stream));
  if (p->ranges[16]) return fail(ADI_EINVAL, "a line class is not one contiguous range of lines");
  p->geom_built = true;
  return ADI_OK;
}

adi_status alloc_tables(adi_problem p) {
  dev_free(p->tab_mem);
  p->tab_mem = nullptr;
  DirState* ds[2] = {&p->r, &p->z};
  size_t bytes = 0;
  auto add = [&](size_t b) { size_t o = bytes; bytes += (b + 255) & ~size_t(255); return o; };
  size_t off[2][6];
  for (int d = 0; d < 2; ++d) {
    DirState& D = *ds[d];
    const long GM = (long)D.L.G * D.L.M;
    off[d][0] = add(sizeof(LineTab) * D.ncls);
    off[d][1] = add(sizeof(double) * D.ncls * P_NFIELDS * GM);
    off[d][2] = add(sizeof(double) * D.ncls * C_NFIELDS * D.L.G);
    off[d][3] = add(sizeof(double) * D.ncls * 2 * D.n);
    off[d][4] = add(sizeof(double) * D.ncls * D.n);
    off[d][5] = add(sizeof(double) * D.ncls * assemble_work(D.L.G, D.L.M));
  }
  ADI_TRY(dev_alloc(&p->tab_mem, bytes, p->stream));
  char* b = (char*)p->tab_mem;
  for (int d = 0; d < 2; ++d) {
    DirState& D = *ds[d];
    D.tabs = (LineTab*)(b + off[d][0]);
    D.pos = (double*)(b + off[d][1]);
    D.chk = (double*)(b + off[d][2]);
    D.eng = (double*)(b + off[d][3]);
    D.xc = (double*)(b + off[d][4]);
    D.work = (double*)(b + off[d][5]);
  }
  return ADI_OK;
}

adi_status ensure_tables(adi_problem p, double dt) {
  if (!p->has_mat || !p->has_src)
    return fail(ADI_ESTATE, "set_materials and set_sources must be called before stepping");
  if (p->tabs_valid && p->tabs_dt == dt) return ADI_OK;
  ADI_TRY(build_geometry_once(p));
  if (!p->tab_mem) ADI_TRY(alloc_tables(p));
  p->P.ta = p->scheme == ADI_PR ? 0.5 * dt : dt;
  p->P.theta = p->scheme == ADI_PR ? 1.0 : 0.0;
  hipLaunchKernelGGL(k_assemble, dim3(p->r.ncls + p->z.ncls), dim3(256), 0, p->stream, p->P, p->g,
                     p->r.view(), p->z.view());
  ADI_CHECK_LAUNCH();
  for (DirState* D : {&p->r, &p->z})
    ADI_HIP(hipMemcpyAsync(D->htabs, D->tabs, sizeof(LineTab) * D->ncls, hipMemcpyDeviceToHost, p->stream));
  ADI_HIP(hipStreamSynchronize(p->stream));
  p->tabs_valid = true;
  p->tabs_dt = dt;
  p->rhs_valid = false;
  drop_graphs(p);
  return ADI_OK;
}

adi_status launch_init_rhs(adi_problem p) {
  const long n = (long)p->P.nr * p->P.nz;
  const int blocks = (int)std::min<long>((n + 255) / 256, 4096);
  const bool strips = p->layout == ADI_LAYOUT_STRIPS;
  const long total = strips ? (long)((p->P.nr + 3) / 4) * p->strip : n;
  hipLaunchKernelGGL(k_init_rhs, dim3(blocks), dim3(256), 0, p->stream, p->T, p->dA, p->g, p->z.view(),
                     p->r.xc, p->P.nr, p->P.nz, strips ? p->strip : 0L, total);
  ADI_CHECK_LAUNCH();
  p->rhs_valid = true;
  return ADI_OK;
}

// Launch a sweep kernel taking one argument struct; with events, they take
// the kernel's own start and end times (no separate event packets).
template <class Args>
void launch_args(const void* fn, int grid, int threads, hipStream_t stream, Args& a, hipEvent_t e0, hipEvent_t e1) {
  void* args[] = {&a};
  if (e0 || e1)
    (void)hipExtLaunchKernel(fn, dim3(grid), dim3(threads), args, 0, stream, e0, e1, 0);
  else
    (void)hipLaunchKernel(fn, dim3(grid), dim3(threads), args, 0, stream);
}

adi_status launch_strip_sweep(adi_problem p, int dir, const double* din, double* dout, double* xout,
                              hipEvent_t e0, hipEvent_t e1) {
  const DirState& D = dir == 0 ? p->r : p->z;
  const DirState& X = dir == 0 ? p->z : p->r;
  StripArgs a;
  a.din = din;
  a.dout = dout;
  a.xout = xout;
  for (int c = 0; c < MAX_CLS; ++c) a.tabs[c] = D.htabs[c < D.ncls ? c : 0];
  bool ambient = false;
  for (int c = 0; c < 4; ++c) ambient = ambient || p->P.tinf[c] != 0.0;
  a.xc = ambient ? X.xc : nullptr;  // the crossing constants vanish with zero ambient temperatures
  a.strip = p->strip;
  a.nr = p->P.nr;
  a.nz = p->P.nz;
  const int grid = strip_setup(a, p->ranges, dir, D.nlines, D.ncls, X.ncls, p->P.theta);
  const StripVariant& V = kStrip[D.L.variant];
  launch_args((const void*)V.fn, grid, 64 * V.NW, p->stream, a, e0, e1);
  ADI_CHECK_LAUNCH();
  return ADI_OK;
}

adi_status launch_sweep(adi_problem p, int dir, const double* din, double* dout, double* xout,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const DirState& D = dir == 0 ? p->r : p->z;
  if (D.L.layout == ADI_LAYOUT_STRIPS) return launch_strip_sweep(p, dir, din, dout, xout, e0, e1);
  SweepArgs a;
  a.din = din;
  a.dout = dout;
  a.xout = xout;
  a.tabs = D.tabs;
  a.pos_xclass = dir == 0 ? p->g.kap : p->g.bet;
  a.xc = dir == 0 ? p->z.xc : p->r.xc;  // r sweep adds b_z, z sweep adds b_r
  a.line_stride = dir == 0 ? p->P.nr : 1;
  a.pos_stride = dir == 0 ? 1 : p->P.nr;
  a.nlines = D.nlines;
  a.ncls = D.ncls;
  const int per_group = D.L.LPW * D.L.R;
  int g0 = 0;
  for (int c = 0; c < D.ncls; ++c) {
    const int* rg = p->ranges + (dir * MAX_CLS + c) * 2;
    a.cls_l0[c] = rg[0];
    a.cls_l1[c] = rg[1];
    a.cls_g0[c] = g0;
    g0 += (rg[1] - rg[0] + per_group - 1) / per_group;
  }
  for (int c = D.ncls; c < MAX_CLS; ++c) a.cls_l0[c] = a.cls_l1[c] = 0, a.cls_g0[c] = g0;
  a.cls_g0[MAX_CLS] = g0;
  a.cls_g0[D.ncls] = g0;
  a.ngroups = g0;
  const Variant& V = kVariants[D.L.variant];
  const int threads = 64 * D.L.WPL * D.L.NGW;
  const int blocks = std::max(1, (a.ngroups + D.L.NGW - 1) / D.L.NGW);
  launch_args((const void*)V.fn, blocks, threads, p->stream, a, e0, e1);
  ADI_CHECK_LAUNCH();
  return ADI_OK;
}

adi_status launch_energy(adi_problem p, const double* T, double* out4) {
  hipLaunchKernelGGL(k_energy_rows, dim3(p->P.nz), dim3(256), 0, p->stream, T, p->P, p->g, p->r.view(),
                     p->z.view(), p->part);
  ADI_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, p->stream, p->part, p->P.nz, out4);
  ADI_CHECK_LAUNCH();
  return ADI_OK;
}

bool is_check_step(const adi_problem p, int64_t global_step) {
  return p->check_every > 0 && global_step % p->check_every == 0;
}

// Enqueue one step.  write_T: the z sweep also stores the solution in T.
// The LDS-resident kernel runs grids whose lines split into chunks of at
// most 16 cells over its waves and whose right-hand side and tables fit in
// the 160 KB of LDS of one compute unit.
bool resident_fits(int nr, int nz) {
  return resident_shape_ok(nr, nz) && resident_lds_doubles(nr, nz) * 8 <= 160L * 1024;
}

// n steps of the LDS-resident kernel (launches of at most 2^20 steps) from
// the carried right-hand side in rhs (rows layout), which it leaves carried
// again; T (if not null) receives the field after the last step.  e0 / e1:
// start and end events of the first and last launch (null: none).
adi_status launch_resident(adi_problem p, double* rhs, double* T, int64_t n, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr) {
  // the kernel takes more than the default 64 KB of dynamic LDS: raise its
  // limit once per device
  static std::atomic<uint64_t> attr_set{0};
  const uint64_t bit = p->device < 64 ? 1ull << p->device : 0;
  if (!bit || !(attr_set.load() & bit)) {
    ADI_HIP(hipFuncSetAttribute((const void*)k_resident, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr_set.fetch_or(bit);
  }
  const size_t lds = sizeof(double) * resident_lds_doubles(p->P.nr, p->P.nz);
  bool ambient = false;
  for (int c = 0; c < 4; ++c) ambient = ambient || p->P.tinf[c] != 0.0;
  for (int64_t done = 0; done < n;) {
    const int k = (int)std::min<int64_t>(n - done, 1 << 20);
    ResArgs a;
    a.P = p->P;
    a.g = p->g;
    a.rhs = rhs;
    a.T = T;
    a.xcr = ambient ? p->r.xc : nullptr;  // the z sweep adds b_r
    a.xcz = ambient ? p->z.xc : nullptr;  // the r sweep adds b_z
    a.nsteps = k;
    a.write_T = T && done + k == n;
    void* args[] = {&a};
    hipEvent_t s0 = done == 0 ? e0 : nullptr, s1 = done + k == n ? e1 : nullptr;
    if (s0 || s1)
      (void)hipExtLaunchKernel((const void*)k_resident, dim3(1), dim3(RES_THREADS), args, lds, p->stream, s0, s1, 0);
    else
      (void)hipLaunchKernel((const void*)k_resident, dim3(1), dim3(RES_THREADS), args, lds, p->stream);
    ADI_CHECK_LAUNCH();
    done += k;
  }
  return ADI_OK;
}

adi_status enqueue_step(adi_problem p, bool check, bool write_T) {
  if (check) ADI_TRY(launch_energy(p, p->T, p->eout));
  ADI_TRY(launch_sweep(p, 0, p->dA, p->dB, check ? p->mid : nullptr));
  if (check) ADI_TRY(launch_energy(p, p->mid, p->eout + 4));
  ADI_TRY(launch_sweep(p, 1, p->dB, p->dA, (check || write_T) ? p->T : nullptr));
  if (check) {
    ADI_TRY(launch_energy(p, p->T, p->eout + 8));
    hipLaunchKernelGGL(k_check, dim3(1), dim3(64), 0, p->stream, p->eout, p->eout + 4, p->eout + 8,
                       p->P.ta, (int)p->scheme, p->check_tol, p->state);
    ADI_CHECK_LAUNCH();
  }
  return ADI_OK;
}

// Enqueue `n` steps starting at global step s0, with plain launches.
adi_status enqueue_steps(adi_problem p, int64_t s0, int64_t n) {
  for (int64_t s = 0; s < n; ++s) {
    const int64_t gs = s0 + s;
    const bool check = is_check_step(p, gs);
    const bool write_T = s == n - 1 || is_check_step(p, gs + 1);
    ADI_TRY(enqueue_step(p, check, write_T));
  }
  return ADI_OK;
}

// A captured segment of `n` steps; the first step may carry the check and
// the last always writes T.
adi_status get_graph(adi_problem p, int n, bool check, hipGraphExec_t* out) {
  for (auto& s : p->graphs)
    if (s.steps == n && s.check == check) {
      *out = s.exec;
      return ADI_OK;
    }
  hipGraph_t graph = nullptr;
  ADI_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
  adi_status st = ADI_OK;
  for (int s = 0; s < n && st == ADI_OK; ++s) st = enqueue_step(p, check && s == 0, s == n - 1);
  hipError_t e = hipStreamEndCapture(p->stream, &graph);
  if (st != ADI_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(ADI_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(ADI_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  p->graphs.push_back({n, check, exec});
  *out = exec;
  return ADI_OK;
}

// Captured segments of K steps and of every power of two below K, with and
// without the check in their first step (the latter only when checks run):
// any run of steps between checks is then a sequence of whole segments
// (largest first), so every call of adi_step replays graphs, whatever its
// step count.  All of them are captured at once, on the first call after
// the tables or the check pattern change.
adi_status ensure_graph_family(adi_problem p) {
  if (!p->graphs.empty()) return ADI_OK;
  const int K = p->graph_steps;
  for (int c = 0; c < (p->check_every > 0 ? 2 : 1); ++c) {
    for (int n = 1; n < K; n *= 2) {
      hipGraphExec_t ex;
      ADI_TRY(get_graph(p, n, c == 1, &ex));
    }
    hipGraphExec_t ex;
    ADI_TRY(get_graph(p, K, c == 1, &ex));
  }
  return ADI_OK;
}

adi_status sync_and_check(adi_problem p) {
  ADI_HIP(hipStreamSynchronize(p->stream));
  double st[4];
  ADI_HIP(hipMemcpy(st, p->state, sizeof st, hipMemcpyDeviceToHost));
  if (st[1] != 0.0) return fail(ADI_ENONFINITE, "non-finite energy in a periodic check");
  if (st[2] != 0.0)
    return fail(ADI_EBALANCE, "energy identity violated: relative residual %.3e > %.3e", st[0], p->check_tol);
  return ADI_OK;
}

adi_status host_map(adi_problem p) {
  if (!p->hmap.empty()) return ADI_OK;
  ADI_TRY(build_geometry_once(p));
  const long n = (long)p->P.nr * p->P.nz;
  hipLaunchKernelGGL(k_region_map, dim3((int)std::min<long>((n + 255) / 256, 4096)), dim3(256), 0,
                     p->stream, p->g, p->P.nr, p->P.nz, p->dmap);
  ADI_CHECK_LAUNCH();
  p->hmap.resize(n);
  ADI_HIP(hipMemcpyAsync(p->hmap.data(), p->dmap, n, hipMemcpyDeviceToHost, p->stream));
  ADI_HIP(hipStreamSynchronize(p->stream));
  return ADI_OK;
}

adi_status validate_geometry(const adi_geometry* g) {
  if (!g) return fail(ADI_EINVAL, "null geometry");
  const double v[] = {g->r0, g->r1, g->r2, g->rmax, g->z0, g->zmax, g->ztop};
  for (double x : v)
    if (!is_fin(x)) return fail(ADI_EINVAL, "geometry values must be finite");
  if (!(0.0 < g->r0 && g->r0 <= g->r1 && g->r1 <= g->r2 && g->r2 <= g->rmax))
    return fail(ADI_EINVAL, "need 0 < r0 <= r1 <= r2 <= rmax");
  if (!(0.0 < g->z0 && g->z0 <= g->zmax && g->zmax <= g->ztop))
    return fail(ADI_EINVAL, "need 0 < z0 <= zmax <= ztop");
  if (g->nr < 1 || g->nz < 1) return fail(ADI_EINVAL, "nr and nz must be >= 1");
  if ((long long)g->nr * g->nz >= (1LL << 31)) return fail(ADI_EINVAL, "nr*nz must be < 2^31");
  auto check_faces = [](const double* f, int n, double len, const char* name) -> adi_status {
    if (!f) return ADI_OK;
    if (f[0] != 0.0 || f[n] != len) return fail(ADI_EINVAL, "%s must run from 0 to the domain end", name);
    for (int i = 0; i < n; ++i)
      if (!(f[i + 1] > f[i]) || !is_fin(f[i + 1])) return fail(ADI_EINVAL, "%s must increase", name);
    return ADI_OK;
  };
  ADI_TRY(check_faces(g->r_faces, g->nr, g->rmax, "r_faces"));
  ADI_TRY(check_faces(g->z_faces, g->nz, g->ztop, "z_faces"));
  return ADI_OK;
}

adi_status validate_bc(const adi_bc* bc) {
  if (!bc) return fail(ADI_EINVAL, "null boundary conditions");
  for (int c = 0; c < 4; ++c) {
    if (!(bc->h[c] >= 0.0) || bc->h[c] != bc->h[c]) return fail(ADI_EINVAL, "h[%d] must be >= 0", c);
    if (!is_fin(bc->t_inf[c])) return fail(ADI_EINVAL, "t_inf[%d] must be finite", c);
  }
  return ADI_OK;
}

// The resident layout's timing: nlaunch steps in one launch on a copy of
// the carried right-hand side (in mid); the time per step.
adi_status time_resident(adi_problem p, int32_t nlaunch, float* ms_step, float* ms_zero) {
  hipEvent_t e[2] = {nullptr, nullptr};
  adi_status st = ADI_OK;
  for (auto& x : e)
    if (hipEventCreate(&x) != hipSuccess) {
      x = nullptr;
      st = fail(ADI_EDEVICE, "hipEventCreate failed");
    }
  if (st == ADI_OK && hipMemcpyAsync(p->mid, p->dA, sizeof(double) * p->P.nr * p->P.nz, hipMemcpyDeviceToDevice,
                                     p->stream) != hipSuccess)
    st = fail(ADI_EDEVICE, "copy of the carried right-hand side failed");
  if (st == ADI_OK) st = launch_resident(p, p->mid, nullptr, nlaunch, e[0], e[1]);
  hipError_t err = hipStreamSynchronize(p->stream);
  float ms = 0.f;
  if (st == ADI_OK && err == hipSuccess) err = hipEventElapsedTime(&ms, e[0], e[1]);
  for (auto& x : e)
    if (x) (void)hipEventDestroy(x);
  if (st != ADI_OK) return st;
  if (err != hipSuccess) return fail(ADI_EDEVICE, "event timing: %s", hipGetErrorString(err));
  if (ms_step) *ms_step = ms / nlaunch;
  if (ms_zero) *ms_zero = 0.f;
  return ADI_OK;
}

}  // namespace

// ------------------------------------------------------------------ ABI --

namespace adi {

adi_status problem_core(adi_problem p, ProblemCore* out) {
  ADI_TRY(check_handle(p));
  if (!out) return fail(ADI_EINVAL, "null output");
  ADI_TRY(build_geometry_once(p));
  out->device = p->device;
  out->stream = p->stream;
  out->P = p->P;
  out->g = p->g;
  out->T = p->T;
  out->time = p->time;
  return ADI_OK;
}

void problem_field_advanced(adi_problem p, double time, int64_t steps) {
  p->rhs_valid = false;
  p->time = time;
  p->steps += steps;
}

void* problem_ext(adi_problem p) { return p ? p->ext : nullptr; }

void problem_set_ext(adi_problem p, void* ext, void (*destroy)(void*)) {
  if (p->ext && p->ext_destroy && p->ext != ext) p->ext_destroy(p->ext);
  p->ext = ext;
  p->ext_destroy = destroy;
}

}  // namespace adi

extern "C" {

const char* adi_status_string(adi_status s) {
  switch (s) {
    case ADI_OK: return "ok";
    case ADI_EINVAL: return "invalid argument";
    case ADI_ENOMEM: return "out of memory";
    case ADI_EDEVICE: return "device error";
    case ADI_ESTATE: return "invalid state";
    case ADI_ENONFINITE: return "non-finite value";
    case ADI_EBALANCE: return "energy balance violated";
    case ADI_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* adi_last_error(void) { return g_error.c_str(); }

adi_status adi_set_allocator(adi_alloc_fn alloc, adi_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(ADI_EINVAL, "allocator and free function must both be given or both be null");
  std::lock_guard<std::mutex> g(g_alloc_mu);
  g_alloc_fn = alloc;
  g_free_fn = free_fn;
  g_alloc_ctx = ctx;
  return ADI_OK;
}

const char* adi_version(void) { return "adi-mi355x 0.1 (gfx950)"; }

adi_status adi_create_problem(const adi_geometry* g, const adi_bc* bc, adi_scheme scheme, void* hip_stream,
                              adi_problem* out) {
  if (!out) return fail(ADI_EINVAL, "null output handle");
  *out = nullptr;
  ADI_TRY(validate_geometry(g));
  ADI_TRY(validate_bc(bc));
  if (scheme != ADI_PR && scheme != ADI_LOD_BE) return fail(ADI_EINVAL, "unknown scheme %d", (int)scheme);
  adi_problem p = new (std::nothrow) adi_problem_s();
  if (!p) return fail(ADI_ENOMEM, "host allocation failed");
  auto cleanup = [&](adi_status s) {
    adi_destroy(p);
    return s;
  };
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)));
  p->stream = (hipStream_t)hip_stream;
  if (!p->stream) {
    // a stream of our own (default priority) so that steps can be captured
    e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e)));
    p->own_stream = true;
  }
  p->scheme = scheme;
  Params& P = p->P;
  P.r0 = g->r0; P.r1 = g->r1; P.r2 = g->r2; P.rmax = g->rmax;
  P.z0 = g->z0; P.zmax = g->zmax; P.ztop = g->ztop;
  P.nr = g->nr; P.nz = g->nz;
  for (int c = 0; c < 4; ++c) { P.h[c] = bc->h[c]; P.tinf[c] = bc->t_inf[c]; }
  const int nr = g->nr, nz = g->nz;
  const long n = (long)nr * nz;
  adi_status st;
  if (g->r_faces) {
    p->h_rf.assign(g->r_faces, g->r_faces + nr + 1);
    if ((st = dev_alloc((void**)&p->d_rfi, sizeof(double) * (nr + 1), p->stream)) != ADI_OK) return cleanup(st);
    e = hipMemcpyAsync(p->d_rfi, p->h_rf.data(), sizeof(double) * (nr + 1), hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "copy r_faces: %s", hipGetErrorString(e)));
  }
  if (g->z_faces) {
    p->h_zf.assign(g->z_faces, g->z_faces + nz + 1);
    if ((st = dev_alloc((void**)&p->d_zfi, sizeof(double) * (nz + 1), p->stream)) != ADI_OK) return cleanup(st);
    e = hipMemcpyAsync(p->d_zfi, p->h_zf.data(), sizeof(double) * (nz + 1), hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "copy z_faces: %s", hipGetErrorString(e)));
  }
  // geometry arrays in one allocation
  const size_t gbytes = sizeof(double) * (3 * (nr + 1) + 3 * (nz + 1)) + (nr + nz) + 64;
  if ((st = dev_alloc(&p->geom_mem, gbytes, p->stream)) != ADI_OK) return cleanup(st);
  double* gd = (double*)p->geom_mem;
  p->g.rf = gd; gd += nr + 1;
  p->g.rc = gd; gd += nr + 1;
  p->g.dr = gd; gd += nr + 1;
  p->g.zf = gd; gd += nz + 1;
  p->g.zc = gd; gd += nz + 1;
  p->g.dz = gd; gd += nz + 1;
  p->g.kap = (uint8_t*)gd;
  p->g.bet = p->g.kap + nr;
  // field and work buffers
  // dA, dB and mid also hold the strip layout: ceil(nr/4) strips, each of
  // 4*ceil(nz/4) rows of 4 doubles
  p->strip = strip_stride(nz);
  const long nbuf = std::max(n, (long)((nr + 3) / 4) * p->strip);
  double** bufs[] = {&p->T, &p->dA, &p->dB, &p->mid};
  for (double** b : bufs)
    if ((st = dev_alloc((void**)b, sizeof(double) * (b == &p->T ? n : nbuf), p->stream)) != ADI_OK)
      return cleanup(st);
  if ((st = dev_alloc((void**)&p->part, sizeof(double) * 4 * nz, p->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&p->eout, sizeof(double) * 16, p->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&p->state, sizeof(double) * 8, p->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&p->prof, sizeof(double) * 4096, p->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&p->dmap, n, p->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&p->dranges, sizeof p->ranges, p->stream)) != ADI_OK) return cleanup(st);
  // line classes: r lines by row band (3), z lines by column class (4)
  p->r.n = nr; p->r.nlines = nz; p->r.ncls = 3;
  p->z.n = nz; p->z.nlines = nr; p->z.ncls = 4;
  p->r.L = default_launch(0, nr, nz);
  p->z.L = default_launch(1, nz, nr);
  if (p->r.L.variant < 0 || p->z.L.variant < 0)
    return cleanup(fail(ADI_EUNSUPPORTED, "no line-solver kernel covers lines of %d / %d cells", nr, nz));
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "stream sync: %s", hipGetErrorString(e)));
  *out = p;
  return ADI_OK;
}

adi_status adi_set_materials(adi_problem p, const double k[5], const double rho_c[5]) {
  ADI_TRY(check_handle(p));
  if (!k || !rho_c) return fail(ADI_EINVAL, "null material array");
  for (int m = 0; m < 5; ++m) {
    if (!(k[m] > 0.0) || !is_fin(k[m])) return fail(ADI_EINVAL, "k[%d] must be > 0 and finite", m);
    if (!(rho_c[m] > 0.0) || !is_fin(rho_c[m])) return fail(ADI_EINVAL, "rho_c[%d] must be > 0 and finite", m);
  }
  for (int m = 0; m < 5; ++m) { p->P.k[m] = k[m]; p->P.rhoc[m] = rho_c[m]; }
  p->has_mat = true;
  p->tabs_valid = false;
  return ADI_OK;
}

adi_status adi_set_sources(adi_problem p, const double q[5]) {
  ADI_TRY(check_handle(p));
  if (!q) return fail(ADI_EINVAL, "null source array");
  for (int m = 0; m < 5; ++m)
    if (!is_fin(q[m])) return fail(ADI_ENONFINITE, "q[%d] is not finite", m);
  for (int m = 0; m < 5; ++m) p->P.q[m] = q[m];
  p->has_src = true;
  p->tabs_valid = false;
  return ADI_OK;
}

adi_status adi_set_field(adi_problem p, const double* host_T, double T0) {
  ADI_TRY(check_handle(p));
  const long n = (long)p->P.nr * p->P.nz;
  if (!host_T && !is_fin(T0)) return fail(ADI_ENONFINITE, "T0 is not finite");
  ADI_TRY(host_map(p));
  if (host_T) {
    for (long c = 0; c < n; ++c)
      if (p->hmap[c] != MASKED && !is_fin(host_T[c]))
        return fail(ADI_ENONFINITE, "field value %ld is not finite", c);
    ADI_HIP(hipMemcpyAsync(p->T, host_T, sizeof(double) * n, hipMemcpyHostToDevice, p->stream));
  }
  hipLaunchKernelGGL(k_set_field, dim3((int)std::min<long>((n + 255) / 256, 4096)), dim3(256), 0, p->stream,
                     p->T, p->g, p->P.nr, p->P.nz, host_T ? 0 : 1, T0);
  ADI_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, p->stream, p->state, 8);
  ADI_CHECK_LAUNCH();
  ADI_HIP(hipStreamSynchronize(p->stream));
  p->rhs_valid = false;
  p->steps = 0;
  p->time = 0.0;
  p->E0_valid = false;
  return ADI_OK;
}

adi_status adi_set_check(adi_problem p, int32_t every, double tol) {
  ADI_TRY(check_handle(p));
  if (every < 0) return fail(ADI_EINVAL, "check interval must be >= 0");
  if (!(tol > 0.0)) return fail(ADI_EINVAL, "check tolerance must be > 0");
  p->check_every = every;
  p->check_tol = tol;
  drop_graphs(p);
  return ADI_OK;
}

adi_status adi_set_graph_steps(adi_problem p, int32_t steps) {
  ADI_TRY(check_handle(p));
  if (steps < 0 || steps > 4096) return fail(ADI_EINVAL, "graph steps must be in [0, 4096]");
  p->graph_steps = steps;
  drop_graphs(p);
  return ADI_OK;
}

adi_status adi_step(adi_problem p, double dt, int64_t nsteps) {
  ADI_TRY(check_handle(p));
  if (!(dt > 0.0) || !is_fin(dt)) return fail(ADI_EINVAL, "dt must be > 0 and finite");
  if (nsteps < 0) return fail(ADI_EINVAL, "nsteps must be >= 0");
  if (!p->has_mat || !p->has_src)
    return fail(ADI_ESTATE, "set_materials and set_sources must be called before stepping");
  if (nsteps == 0) return ADI_OK;
  ADI_TRY(ensure_tables(p, dt));
  if (!p->E0_valid) {
    ADI_TRY(launch_energy(p, p->T, p->eout + 12));
    double e[4];
    ADI_HIP(hipMemcpyAsync(e, p->eout + 12, sizeof e, hipMemcpyDeviceToHost, p->stream));
    ADI_HIP(hipStreamSynchronize(p->stream));
    p->E0 = e[0];
    p->E0_valid = true;
  }
  if (!p->rhs_valid) ADI_TRY(launch_init_rhs(p));
  int64_t s = 0;
  const int K = p->graph_steps;
  if (p->layout == ADI_LAYOUT_RESIDENT) {
    // every run of steps between checks in one launch; a check step on the
    // rows kernels
    while (s < nsteps) {
      const int64_t gs = p->steps + s;
      int64_t seg = nsteps - s;
      if (p->check_every > 0) {
        const int64_t to_next = p->check_every - (gs % p->check_every);
        seg = std::min<int64_t>(seg, is_check_step(p, gs) ? p->check_every : to_next);
      }
      int64_t left = seg;
      if (is_check_step(p, gs)) {
        ADI_TRY(enqueue_step(p, true, seg == 1));
        left -= 1;
      }
      if (left > 0) ADI_TRY(launch_resident(p, p->dA, p->T, left));
      s += seg;
    }
    p->steps += nsteps;
    p->time += dt * (double)nsteps;
    return ADI_OK;
  }
  while (s < nsteps) {
    const int64_t gs = p->steps + s;
    const int64_t left = nsteps - s;
    // a segment never crosses a check step except at its start, and ends
    // where the next check begins so that T is written before the check
    int64_t seg = left;
    if (p->check_every > 0) {
      const int64_t to_next = p->check_every - (gs % p->check_every);
      seg = std::min<int64_t>(seg, is_check_step(p, gs) ? p->check_every : to_next);
    }
    const bool check = is_check_step(p, gs);
    if (K > 0) {
      ADI_TRY(ensure_graph_family(p));
      for (int64_t done = 0; done < seg;) {
        const int64_t rem = seg - done;
        int n = K;
        if (rem < K) {
          n = 1;
          while (2 * (int64_t)n <= rem) n *= 2;
        }
        hipGraphExec_t ex;
        ADI_TRY(get_graph(p, n, check && done == 0, &ex));
        ADI_HIP(hipGraphLaunch(ex, p->stream));
        done += n;
      }
      s += seg;
      continue;
    }
    ADI_TRY(enqueue_steps(p, gs, seg));
    s += seg;
  }
  p->steps += nsteps;
  p->time += dt * (double)nsteps;
  return ADI_OK;
}

adi_status adi_read_field(adi_problem p, double* host_out, size_t count) {
  ADI_TRY(check_handle(p));
  const size_t n = (size_t)p->P.nr * p->P.nz;
  if (!host_out) return fail(ADI_EINVAL, "null output buffer");
  if (count != n) return fail(ADI_EINVAL, "count %zu != nz*nr = %zu", count, n);
  ADI_TRY(host_map(p));
  ADI_HIP(hipMemcpyAsync(host_out, p->T, sizeof(double) * n, hipMemcpyDeviceToHost, p->stream));
  adi_status st = sync_and_check(p);
  for (size_t c = 0; c < n; ++c)
    if (p->hmap[c] == MASKED) host_out[c] = NAN;
  return st;
}

adi_status adi_read_field_device(adi_problem p, void* dev_out) {
  ADI_TRY(check_handle(p));
  if (!dev_out) return fail(ADI_EINVAL, "null device buffer");
  ADI_HIP(hipMemcpyAsync(dev_out, p->T, sizeof(double) * p->P.nr * p->P.nz, hipMemcpyDeviceToDevice,
                         p->stream));
  return ADI_OK;
}

adi_status adi_read_region_map(adi_problem p, uint8_t* host_out, size_t count) {
  ADI_TRY(check_handle(p));
  const size_t n = (size_t)p->P.nr * p->P.nz;
  if (!host_out) return fail(ADI_EINVAL, "null output buffer");
  if (count != n) return fail(ADI_EINVAL, "count %zu != nz*nr = %zu", count, n);
  ADI_TRY(host_map(p));
  memcpy(host_out, p->hmap.data(), n);
  return ADI_OK;
}

adi_status adi_read_profile(adi_problem p, int32_t which, int32_t npts, double* host_out) {
  ADI_TRY(check_handle(p));
  if (!host_out) return fail(ADI_EINVAL, "null output buffer");
  if (npts < 1 || npts > 4096) return fail(ADI_EINVAL, "npts must be in [1, 4096]");
  if (which != 0 && which != 1) return fail(ADI_EINVAL, "which must be 0 (top) or 1 (contact)");
  ADI_TRY(host_map(p));
  const int nr = p->P.nr, nz = p->P.nz;
  int row = -1;
  if (which == 0) row = nz - 1;
  else
    for (int j = 0; j < nz; ++j)
      if (p->hmap[(size_t)j * nr] == 4) { row = j; break; }
  if (row < 0) return fail(ADI_EINVAL, "the grid has no terminal row");
  for (int i = 0; i < nr; ++i)
    if (p->hmap[(size_t)row * nr + i] == MASKED) return fail(ADI_EINVAL, "profile row leaves the domain");
  hipLaunchKernelGGL(k_profile, dim3(1), dim3(256), 0, p->stream, p->T, p->g, nr, row, p->P.rmax, npts, p->prof);
  ADI_CHECK_LAUNCH();
  ADI_HIP(hipMemcpyAsync(host_out, p->prof, sizeof(double) * npts, hipMemcpyDeviceToHost, p->stream));
  return sync_and_check(p);
}

adi_status adi_energy(adi_problem p, adi_energy_report* out) {
  ADI_TRY(check_handle(p));
  if (!out) return fail(ADI_EINVAL, "null report");
  if (!p->has_mat || !p->has_src) return fail(ADI_ESTATE, "materials and sources are not set");
  if (!p->tab_mem) ADI_TRY(ensure_tables(p, p->tabs_dt > 0 ? p->tabs_dt : 1.0));
  else if (!p->tabs_valid) ADI_TRY(ensure_tables(p, p->tabs_dt));
  ADI_TRY(launch_energy(p, p->T, p->eout + 12));
  double e[4], st[4];
  ADI_HIP(hipMemcpyAsync(e, p->eout + 12, sizeof e, hipMemcpyDeviceToHost, p->stream));
  ADI_HIP(hipMemcpyAsync(st, p->state, sizeof st, hipMemcpyDeviceToHost, p->stream));
  adi_status s = sync_and_check(p);
  out->E = e[0];
  out->E0 = p->E0_valid ? p->E0 : e[0];
  out->source_power = e[3];
  out->boundary_flow = e[1] + e[2];
  out->residual = st[0];
  out->checks = (int64_t)st[3];
  out->steps = p->steps;
  out->time = p->time;
  if (s == ADI_OK && !is_fin(e[0])) return fail(ADI_ENONFINITE, "field holds non-finite values");
  return s;
}

adi_status adi_time_sweeps(adi_problem p, double dt, int32_t nlaunch, float* ms_r, float* ms_z) {
  ADI_TRY(check_handle(p));
  if (nlaunch < 1) return fail(ADI_EINVAL, "nlaunch must be >= 1");
  if (!(dt > 0.0)) return fail(ADI_EINVAL, "dt must be > 0");
  ADI_TRY(ensure_tables(p, dt));
  if (!p->rhs_valid) ADI_TRY(launch_init_rhs(p));
  if (p->layout == ADI_LAYOUT_RESIDENT) return time_resident(p, nlaunch, ms_r, ms_z);
  // Half steps alternate as in a time step, so every sweep reads what the
  // other direction has just written: r sweeps read the last z output (dA
  // first) and write dB, z sweeps read dB and write mid; the carried state
  // (dA, T) is untouched.  Every launch carries its own start and end events.
  const size_t ne = 4 * (size_t)nlaunch;
  std::vector<hipEvent_t> ev(ne, nullptr);
  adi_status st = ADI_OK;
  for (auto& x : ev)
    if (hipEventCreate(&x) != hipSuccess) {
      x = nullptr;
      st = fail(ADI_EDEVICE, "hipEventCreate failed");
      break;
    }
  for (int i = 0; i < nlaunch && st == ADI_OK; ++i) {
    st = launch_sweep(p, 0, i == 0 ? p->dA : p->mid, p->dB, nullptr, ev[4 * i], ev[4 * i + 1]);
    if (st == ADI_OK) st = launch_sweep(p, 1, p->dB, p->mid, nullptr, ev[4 * i + 2], ev[4 * i + 3]);
  }
  hipError_t e = hipStreamSynchronize(p->stream);
  float a = 0.f, b = 0.f;
  for (int i = 0; i < nlaunch && st == ADI_OK && e == hipSuccess; ++i) {
    float x = 0.f, y = 0.f;
    e = hipEventElapsedTime(&x, ev[4 * i], ev[4 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&y, ev[4 * i + 2], ev[4 * i + 3]);
    a += x;
    b += y;
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  if (st != ADI_OK) return st;
  if (e != hipSuccess) return fail(ADI_EDEVICE, "event timing: %s", hipGetErrorString(e));
  if (ms_r) *ms_r = a / nlaunch;
  if (ms_z) *ms_z = b / nlaunch;
  return ADI_OK;
}

adi_status adi_set_launch(adi_problem p, int32_t dir, int32_t chunk, int32_t lines_per_wave,
                          int32_t waves_per_line, int32_t lines_per_lane, int32_t groups_per_block) {
  ADI_TRY(check_handle(p));
  if (dir != 0 && dir != 1) return fail(ADI_EINVAL, "dir must be 0 (r) or 1 (z)");
  DirState& D = dir == 0 ? p->r : p->z;
  Launch L;
  if (p->layout == ADI_LAYOUT_STRIPS)
    ADI_TRY(validate_strip_launch(dir, D.n, chunk, lines_per_wave, waves_per_line, lines_per_lane,
                                  groups_per_block, &L));
  else
    ADI_TRY(validate_launch(D.n, chunk, lines_per_wave, waves_per_line, lines_per_lane, groups_per_block, &L));
  const bool shape_change = L.G != D.L.G || L.M != D.L.M;
  D.L = L;
  if (shape_change) {
    // tables depend on the chunking: rebuild them (and re-derive the carried
    // right-hand side from T) before the next step
    ADI_HIP(hipStreamSynchronize(p->stream));
    dev_free(p->tab_mem);
    p->tab_mem = nullptr;
    p->tabs_valid = false;
  }
  drop_graphs(p);
  return ADI_OK;
}

adi_status adi_sync(adi_problem p) {
  ADI_TRY(check_handle(p));
  ADI_HIP(hipStreamSynchronize(p->stream));
  return ADI_OK;
}

adi_status adi_set_layout(adi_problem p, int32_t layout) {
  ADI_TRY(check_handle(p));
  if (layout != ADI_LAYOUT_ROWS && layout != ADI_LAYOUT_STRIPS && layout != ADI_LAYOUT_RESIDENT)
    return fail(ADI_EINVAL, "unknown layout %d", (int)layout);
  if (layout == p->layout) return ADI_OK;
  if (layout == ADI_LAYOUT_RESIDENT && !resident_fits(p->P.nr, p->P.nz))
    return fail(ADI_EUNSUPPORTED, "grid %dx%d does not fit the LDS-resident kernel", p->P.nr, p->P.nz);
  Launch Lr, Lz;
  if (layout == ADI_LAYOUT_STRIPS) {
    if (!default_strip_launch(0, p->P.nr, &Lr) || !default_strip_launch(1, p->P.nz, &Lz))
      return fail(ADI_EUNSUPPORTED, "grid %dx%d exceeds the strip-layout kernels (nr <= 2048, nz <= 3072)",
                  p->P.nr, p->P.nz);
  } else {
    Lr = default_launch(0, p->P.nr, p->P.nz);
    Lz = default_launch(1, p->P.nz, p->P.nr);
  }
  // the carried right-hand side is re-derived from T in the new layout
  ADI_HIP(hipStreamSynchronize(p->stream));
  p->r.L = Lr;
  p->z.L = Lz;
  p->layout = layout;
  dev_free(p->tab_mem);
  p->tab_mem = nullptr;
  p->tabs_valid = false;
  p->rhs_valid = false;
  drop_graphs(p);
  return ADI_OK;
}

adi_status adi_get_layout(adi_problem p, int32_t* layout) {
  ADI_TRY(check_handle(p));
  if (!layout) return fail(ADI_EINVAL, "null output");
  *layout = p->layout;
  return ADI_OK;
}

adi_status adi_layout_shapes(int32_t layout, int32_t dir, int32_t* out, int32_t max_shapes, int32_t* count) {
  if (!count) return fail(ADI_EINVAL, "null count");
  if (max_shapes > 0 && !out) return fail(ADI_EINVAL, "null output array");
  if (dir != 0 && dir != 1) return fail(ADI_EINVAL, "dir must be 0 (r) or 1 (z)");
  if (layout == ADI_LAYOUT_ROWS) return adi_launch_shapes(out, max_shapes, count);
  if (layout == ADI_LAYOUT_RESIDENT) {
    *count = 0;  // one fixed launch shape
    return ADI_OK;
  }
  if (layout != ADI_LAYOUT_STRIPS) return fail(ADI_EINVAL, "unknown layout %d", (int)layout);
  int c = 0;
  for (int v = 0; v < kNumStrip; ++v) {
    if (kStrip[v].dir != dir) continue;
    if (c < max_shapes) {
      const int32_t f[5] = {kStrip[v].M, 1, kStrip[v].NW, 4, 1};
      for (int q = 0; q < 5; ++q) out[5 * c + q] = f[q];
    }
    ++c;
  }
  *count = c;
  return ADI_OK;
}

adi_status adi_get_launch(adi_problem p, int32_t dir, int32_t* chunk, int32_t* lines_per_wave,
                          int32_t* waves_per_line, int32_t* lines_per_lane, int32_t* groups_per_block) {
  ADI_TRY(check_handle(p));
  if (dir != 0 && dir != 1) return fail(ADI_EINVAL, "dir must be 0 (r) or 1 (z)");
  const Launch& L = (dir == 0 ? p->r : p->z).L;
  if (chunk) *chunk = L.M;
  if (lines_per_wave) *lines_per_wave = L.LPW;
  if (waves_per_line) *waves_per_line = L.WPL;
  if (lines_per_lane) *lines_per_lane = L.R;
  if (groups_per_block) *groups_per_block = L.NGW;
  return ADI_OK;
}

adi_status adi_launch_shapes(int32_t* out, int32_t max_shapes, int32_t* count) {
  if (!count) return fail(ADI_EINVAL, "null count");
  if (max_shapes > 0 && !out) return fail(ADI_EINVAL, "null output array");
  for (int v = 0; v < kNumVariants && v < max_shapes; ++v) {
    const Variant& V = kVariants[v];
    const int32_t f[5] = {V.M, V.LPW, V.WPL, V.R, V.NGW};
    for (int q = 0; q < 5; ++q) out[5 * v + q] = f[q];
  }
  *count = kNumVariants;
  return ADI_OK;
}

void adi_destroy(adi_problem p) {
  if (!p) return;
  (void)hipSetDevice(p->device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  drop_graphs(p);
  if (p->ext && p->ext_destroy) p->ext_destroy(p->ext);
  p->ext = nullptr;
  void* bufs[] = {p->d_rfi, p->d_zfi, p->geom_mem, p->tab_mem, p->T, p->dA, p->dB, p->mid,
                  p->part, p->eout, p->state, p->prof, p->dmap, p->dranges};
  for (void* b : bufs) dev_free(b);
  if (p->own_stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

}  // extern "C"
