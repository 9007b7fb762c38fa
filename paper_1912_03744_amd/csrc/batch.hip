// batch.hip -- ragged batch of independent instances in one persistent launch.
//
// Every instance of a design sweep is a complete problem (own geometry,
// materials, grid size up to 192 x 480).  One persistent kernel advances all
// of them: each workgroup takes the next instance from an atomic queue
// (largest grids first), builds its geometry and factor tables in a private
// scratch area, runs the whole time loop (r sweep, workgroup barrier, z
// sweep, barrier) with the line solver of device.hpp, records the outer
// terminal-face profile every `snapshot_every` steps, writes the final field
// and takes the next instance.  No grid-wide synchronisation is needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "batch.hpp"

namespace adi {

__device__ void fill_sweep_args(SweepArgs& s, int dir, const Params& P, const Geom& g, const int* ranges,
                                const LineTab* tabs, const double* xc_other, int lines_per_group) {
  s.tabs = tabs;
  s.pos_xclass = dir == 0 ? g.kap : g.bet;
  s.xc = xc_other;
  s.line_stride = dir == 0 ? P.nr : 1;
  s.pos_stride = dir == 0 ? 1 : P.nr;
  s.nlines = dir == 0 ? P.nz : P.nr;
  s.ncls = dir == 0 ? 3 : 4;
  int g0 = 0;
  for (int c = 0; c < MAX_CLS; ++c) {
    const int l0 = c < s.ncls ? ranges[(dir * MAX_CLS + c) * 2] : 0;
    const int l1 = c < s.ncls ? ranges[(dir * MAX_CLS + c) * 2 + 1] : 0;
    s.cls_l0[c] = l0;
    s.cls_l1[c] = l1;
    s.cls_g0[c] = g0;
    g0 += (l1 - l0 + lines_per_group - 1) / lines_per_group;
  }
  s.cls_g0[MAX_CLS] = g0;
  s.ngroups = g0;
}

template <int M, int LPW, int R, bool CONTIG, int NW>
__device__ __forceinline__ void batch_sweep(const SweepArgs& s) {
  const int wave = threadIdx.x >> 6;
  for (int grp = wave; grp < s.ngroups; grp += NW) solve_group<M, LPW, 1, R, CONTIG>(s, grp, nullptr, true, 0);
}

template <int R, int NW>
__device__ void sweep_r(int rs, const SweepArgs& s) {
  switch (rs) {
    case 0: batch_sweep<kBR_M[0], kBR_LPW, R, true, NW>(s); break;
    case 1: batch_sweep<kBR_M[1], kBR_LPW, R, true, NW>(s); break;
    case 2: batch_sweep<kBR_M[2], kBR_LPW, R, true, NW>(s); break;
    default: batch_sweep<kBR_M[3], kBR_LPW, R, true, NW>(s); break;
  }
}
template <int R, int NW>
__device__ void sweep_z(int zs, const SweepArgs& s) {
  switch (zs) {
    case 0: batch_sweep<kBZ_M[0], kBZ_LPW, R, false, NW>(s); break;
    case 1: batch_sweep<kBZ_M[1], kBZ_LPW, R, false, NW>(s); break;
    case 2: batch_sweep<kBZ_M[2], kBZ_LPW, R, false, NW>(s); break;
    default: batch_sweep<kBZ_M[3], kBZ_LPW, R, false, NW>(s); break;
  }
}

template <int R, int NW>
__global__ void __launch_bounds__(64 * NW) k_batch(BatchArgs a) {
  __shared__ int s_next;
  char* ws = a.scratch + (long)blockIdx.x * a.lay.stride;
  const BatchLayout& Ly = a.lay;
  double* dA = (double*)(ws + Ly.dA);
  double* dB = (double*)(ws + Ly.dB);
  int* ranges = (int*)(ws + Ly.ranges);
  LineTab* rtabs = (LineTab*)(ws + Ly.rtabs);
  LineTab* ztabs = (LineTab*)(ws + Ly.ztabs);
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(a.queue, 1);
    __syncthreads();
    const int q = s_next;
    __syncthreads();
    if (q >= a.ninst) break;  // every wave of the workgroup leaves together
    const int idx = a.order[q];
    const BatchInst I = a.inst[idx];
    const Params& P = I.P;
    const int nr = P.nr, nz = P.nz;
    const int Mr = kBR_M[I.rs], Mz = kBZ_M[I.zs];

    // geometry
    Geom g;
    double* gd = (double*)(ws + Ly.geo);
    g.rf = gd; g.rc = gd + (kMaxNr + 1); g.dr = gd + 2 * (kMaxNr + 1);
    g.zf = gd + 3 * (kMaxNr + 1); g.zc = g.zf + (kMaxNz + 1); g.dz = g.zf + 2 * (kMaxNz + 1);
    g.kap = (uint8_t*)(ws + Ly.kap);
    g.bet = (uint8_t*)(ws + Ly.bet);
    build_geometry(P, nullptr, nullptr, g, ranges);

    // factor tables of the 3 row bands and 4 column classes
    double* rpos = (double*)(ws + Ly.rpos);
    double* rchk = (double*)(ws + Ly.rchk);
    double* reng = (double*)(ws + Ly.reng);
    double* rxc = (double*)(ws + Ly.rxc);
    double* zpos = (double*)(ws + Ly.zpos);
    double* zchk = (double*)(ws + Ly.zchk);
    double* zeng = (double*)(ws + Ly.zeng);
    double* zxc = (double*)(ws + Ly.zxc);
    double* work = (double*)(ws + Ly.work);
    for (int c = 0; c < 3; ++c) {
      assemble_class(P, g, 0, c, kBR_G, Mr, rpos + c * P_NFIELDS * kBR_G * Mr, rchk + c * C_NFIELDS * kBR_G,
                     reng + c * 2 * nr, rxc + c * nr, work, false);
      if (threadIdx.x == 0) {
        LineTab t;
        t.pos = rpos + c * P_NFIELDS * kBR_G * Mr;
        t.chk = rchk + c * C_NFIELDS * kBR_G;
        t.n = nr; t.G = kBR_G; t.M = Mr;
        skip_range(0, c, ranges, nr, &t.skip_lo, &t.skip_hi);
        rtabs[c] = t;
      }
    }
    for (int c = 0; c < 4; ++c) {
      assemble_class(P, g, 1, c, kBZ_G, Mz, zpos + c * P_NFIELDS * kBZ_G * Mz, zchk + c * C_NFIELDS * kBZ_G,
                     zeng + c * 2 * nz, zxc + c * nz, work, false);
      if (threadIdx.x == 0) {
        LineTab t;
        t.pos = zpos + c * P_NFIELDS * kBZ_G * Mz;
        t.chk = zchk + c * C_NFIELDS * kBZ_G;
        t.n = nz; t.G = kBZ_G; t.M = Mz;
        skip_range(1, c, ranges, nz, &t.skip_lo, &t.skip_hi);
        ztabs[c] = t;
      }
    }
    __syncthreads();

    // right-hand side of the first r half step from the uniform field T0
    bool any_xc = false;
    for (int c = 0; c < 4; ++c) any_xc = any_xc || P.tinf[c] != 0.0;
    const long ncell = (long)nr * nz;
    for (long cidx = threadIdx.x; cidx < ncell; cidx += blockDim.x) {
      const int i = (int)(cidx % nr), j = (int)(cidx / nr);
      const int kap = g.kap[i], bet = g.bet[j];
      if (region_of(bet, kap) == MASKED) continue;
      const int GM = kBZ_G * Mz;
      const double* pz = zpos + kap * P_NFIELDS * GM;
      const int ix = (j % Mz) * kBZ_G + j / Mz;
      dA[cidx] = (pz[pos_at(P_OD, GM, ix, false)] + pz[pos_at(P_OL, GM, ix, false)] + pz[pos_at(P_OU, GM, ix, false)]) * I.T0 + pz[pos_at(P_OC, GM, ix, false)] +
                 rxc[bet * nr + i];
    }
    __syncthreads();

    SweepArgs sr, sz;
    fill_sweep_args(sr, 0, P, g, ranges, rtabs, any_xc ? zxc : nullptr, kBR_LPW * R);
    fill_sweep_args(sz, 1, P, g, ranges, ztabs, any_xc ? rxc : nullptr, kBZ_LPW * R);
    sr.din = dA; sr.dout = dB; sr.xout = nullptr;
    sz.din = dB; sz.dout = dA;
    double* Ti = a.T + I.toff;
    int snap = 0;
    for (int st = 1; st <= a.nsteps; ++st) {
      const bool take = a.snap_every > 0 && st % a.snap_every == 0 && snap < a.nsnap;
      sweep_r<R, NW>(I.rs, sr);
      __syncthreads();
      sz.xout = (take || st == a.nsteps) ? Ti : nullptr;
      sweep_z<R, NW>(I.zs, sz);
      __syncthreads();
      if (take) {
        // outer terminal-face profile from the top row
        const double* row = Ti + (long)(nz - 1) * nr;
        for (int kk = threadIdx.x; kk < a.npts; kk += blockDim.x) {
          const double r = (kk + 0.5) * P.rmax / a.npts;
          double o;
          if (r <= g.rc[0]) o = row[0];
          else if (r >= g.rc[nr - 1]) o = row[nr - 1];
          else {
            int lo = 0, hi = nr - 1;
            while (hi - lo > 1) {
              const int mid = (lo + hi) >> 1;
              if (g.rc[mid] <= r) lo = mid; else hi = mid;
            }
            o = row[lo] + (row[lo + 1] - row[lo]) * (r - g.rc[lo]) / (g.rc[lo + 1] - g.rc[lo]);
          }
          a.prof[((long)idx * a.nsnap + snap) * a.npts + kk] = o;
        }
        ++snap;
      }
    }
    __syncthreads();
  }
}

__global__ void k_reset_queue(int* q) {
  if (threadIdx.x == 0) q[0] = 0;
}

using BatchFn = void (*)(BatchArgs);
struct BatchVariant {
  int R, NW;
  BatchFn fn;
};
// R = 1, 2: rows-layout line solver; R = 4: the strip-layout kernel
// (4 lines per lane, one wave per block of lines); R = 4 with one wave per
// workgroup: batched sweep launches (no persistent kernel).
static const BatchVariant kBatchVariants[] = {
    {1, 4, k_batch<1, 4>}, {2, 4, k_batch<2, 4>}, {1, 8, k_batch<1, 8>}, {2, 8, k_batch<2, 8>},
    {4, 4, k_batch_s<4>},  {4, 8, k_batch_s<8>},  {4, 1, nullptr},
};
static const int kNumBatchVariants = sizeof(kBatchVariants) / sizeof(kBatchVariants[0]);

static int shape_index(const int* cover_m, int G, int n) {
  for (int s = 0; s < 4; ++s)
    if (G * cover_m[s] >= n) return s;
  return -1;
}


}  // namespace adi

using namespace adi;

struct adi_batch_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  adi_scheme scheme = ADI_PR;
  int n = 0;
  std::vector<BatchInst> hinst;
  BatchInst* dinst = nullptr;
  int* dorder = nullptr;
  int* queue = nullptr;
  double* T = nullptr;
  long total_cells = 0, maxcells = 0;  // arena size (aligned), largest instance
  long cells = 0, active = 0;           // cells, cells inside the domain
  long maxstrip = 0;                    // largest right-hand side in the strip layout (doubles)
  double* prof = nullptr;
  long prof_cap = 0;           // doubles
  double* prof_out = nullptr;  // where the last step wrote its snapshots (prof or the caller's buffer)
  int nsnap = 0, npts = 64;
  char* scratch = nullptr;
  BatchLayout lay{};
  int nblocks = 0;
  int variant = 1;
  int blocks_per_cu = 2;
  bool has_mat = false;
  int64_t steps = 0;
  // batched sweep launches: per-instance scratch areas and right-hand sides,
  // sweep arguments, workgroup maps (r: all instances; z: per chunk shape)
  BatchLayout slay{};
  char* saux = nullptr;
  double* srhs = nullptr;
  long* srhs_off = nullptr;
  StripArgs* sargs = nullptr;
  int* smap = nullptr;
  int nmap_r[3] = {0, 0, 0}, rmap_off[3] = {0, 0, 0};  // r: slots of 16, 32, 64 tiles
  int nmap_z[4] = {0, 0, 0, 0}, zmap_off[4] = {0, 0, 0, 0};
  int zvar[4] = {0, 0, 0, 0};  // candidate shape of each z class
};

namespace {

adi_status batch_handle(adi_batch b) {
  if (!b) return fail(ADI_EINVAL, "null batch handle");
  ADI_HIP(hipSetDevice(b->device));
  return ADI_OK;
}

adi_status ensure_scratch(adi_batch b) {
  int cus = 0;
  ADI_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
  const int want = std::max(1, std::min(b->n, cus * b->blocks_per_cu));
  if (b->scratch && b->nblocks == want) return ADI_OK;
  if (b->scratch) {
    ADI_HIP(hipStreamSynchronize(b->stream));
    dev_free(b->scratch);
    b->scratch = nullptr;
  }
  ADI_TRY(dev_alloc((void**)&b->scratch, (size_t)b->lay.stride * want, b->stream));
  b->nblocks = want;
  return ADI_OK;
}

// Buffers of the batched sweep launches (allocated on first use).
adi_status ensure_sweep(adi_batch b) {
  if (b->saux) return ADI_OK;
  b->slay = batch_layout(0, 0);  // scratch areas without right-hand sides
  const BSweepPlan plan = bsweep_plan(b->hinst.data(), b->n);
  const std::vector<long>& off = plan.off;
  const std::vector<int>& map = plan.map;
  const long total = plan.total;
  for (int w = 0; w < 3; ++w) b->nmap_r[w] = plan.nmap_r[w], b->rmap_off[w] = plan.rmap_off[w];
  for (int c = 0; c < 4; ++c) b->nmap_z[c] = plan.nmap_z[c], b->zmap_off[c] = plan.zmap_off[c];
  ADI_TRY(dev_alloc((void**)&b->saux, (size_t)b->slay.stride * b->n, b->stream));
  ADI_TRY(dev_alloc((void**)&b->srhs, sizeof(double) * total, b->stream));
  ADI_TRY(dev_alloc((void**)&b->srhs_off, sizeof(long) * b->n, b->stream));
  ADI_TRY(dev_alloc((void**)&b->sargs, sizeof(StripArgs) * 3 * b->n, b->stream));
  ADI_TRY(dev_alloc((void**)&b->smap, sizeof(int) * map.size(), b->stream));
  ADI_HIP(hipMemcpyAsync(b->srhs_off, off.data(), sizeof(long) * b->n, hipMemcpyHostToDevice, b->stream));
  ADI_HIP(hipMemcpyAsync(b->smap, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice, b->stream));
  ADI_HIP(hipStreamSynchronize(b->stream));
  return ADI_OK;
}

// Steps st0 .. st1 (1-based, inclusive) of the time loop as batched sweep
// launches on the batch's stream (being captured by the caller): the
// instance prologues first when st0 is 1, then per step one r launch per row
// slot width and one z launch per z shape (the last of the nsteps steps and
// snapshot steps write the field), and the profile launch at snapshots.
void launch_sweeps(adi_batch b, int64_t st0, int64_t st1, int64_t nsteps, int snapshot_every, int nsnap,
                   int npts) {
  BSweepArgs a;
  a.inst = b->dinst;
  a.aux = b->saux;
  a.lay = b->slay;
  a.rhs = b->srhs;
  a.rhs_off = b->srhs_off;
  a.args = b->sargs;
  a.n = b->n;
  a.T = b->T;
  a.prof = b->prof_out;
  a.npts = npts;
  a.map = b->smap;
  for (int c = 0; c < 4; ++c) a.zvar[c] = b->zvar[c];
  if (st0 == 1) hipLaunchKernelGGL(k_bsetup, dim3(b->n), dim3(256), 0, b->stream, a);
  for (int64_t st = st0; st <= st1; ++st) {
    const int64_t snap = snapshot_every > 0 ? st / snapshot_every - 1 : -1;  // index if st is a snapshot step
    const bool take = snapshot_every > 0 && st % snapshot_every == 0 && snap < nsnap;
    const int write_T = (take || st == nsteps) ? 1 : 0;
    for (int w = 0; w < 3; ++w) {
      if (!b->nmap_r[w]) continue;
      a.map = b->smap + b->rmap_off[w];
      if (w == 0) hipLaunchKernelGGL(k_bsweep_r<16>, dim3(b->nmap_r[w]), dim3(64), 0, b->stream, a);
      else if (w == 1) hipLaunchKernelGGL(k_bsweep_r<32>, dim3(b->nmap_r[w]), dim3(64), 0, b->stream, a);
      else hipLaunchKernelGGL(k_bsweep_r<64>, dim3(b->nmap_r[w]), dim3(64), 0, b->stream, a);
    }
    for (int c = 0; c < 4; ++c) {
      if (!b->nmap_z[c]) continue;
      a.map = b->smap + b->zmap_off[c];
      bwz_dispatch(c, b->zvar[c], [&](auto m, auto nw) {
        constexpr int M = decltype(m)::value, NW = decltype(nw)::value;
        hipLaunchKernelGGL((k_bsweep_z<M, NW>), dim3(b->nmap_z[c]), dim3(64 * NW), 0, b->stream, a, write_T);
      });
    }
    if (take) hipLaunchKernelGGL(k_bprofile, dim3(b->n), dim3(64), 0, b->stream, a, (int)snap, nsnap);
  }
}

// Capture whatever `enqueue` puts on the batch's stream into a graph and
// launch it (the graph is released once it has run).
template <class F>
adi_status launch_captured(adi_batch b, F enqueue) {
  hipGraph_t graph = nullptr;
  ADI_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  enqueue();
  hipError_t e = hipStreamEndCapture(b->stream, &graph);
  if (e != hipSuccess) return fail(ADI_EDEVICE, "capture of the batch launch: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(ADI_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  e = hipGraphLaunch(exec, b->stream);
  (void)hipGraphExecDestroy(exec);
  if (e != hipSuccess) return fail(ADI_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
  return ADI_OK;
}

// Steps per captured graph of the batched sweep launches (about 8 launches
// per step): bounds the graph's size for any number of steps.
constexpr int64_t kSweepGraphSteps = 256;

}  // namespace

extern "C" {

adi_status adi_create_batch(int32_t n, const adi_geometry* geoms, const adi_bc* bcs, adi_scheme scheme,
                            void* hip_stream, adi_batch* out) {
  if (!out) return fail(ADI_EINVAL, "null output handle");
  *out = nullptr;
  if (n < 1) return fail(ADI_EINVAL, "batch size must be >= 1");
  if (!geoms || !bcs) return fail(ADI_EINVAL, "null geometry or boundary array");
  if (scheme != ADI_PR && scheme != ADI_LOD_BE) return fail(ADI_EINVAL, "unknown scheme %d", (int)scheme);
  adi_batch b = new (std::nothrow) adi_batch_s();
  if (!b) return fail(ADI_ENOMEM, "host allocation failed");
  auto cleanup = [&](adi_status s) {
    adi_batch_destroy(b);
    return s;
  };
  b->n = n;
  b->scheme = scheme;
  b->hinst.resize(n);
  long off = 0;
  for (int i = 0; i < n; ++i) {
    const adi_geometry& g = geoms[i];
    const adi_bc& bc = bcs[i];
    const double v[] = {g.r0, g.r1, g.r2, g.rmax, g.z0, g.zmax, g.ztop};
    for (double x : v)
      if (!is_fin(x)) return cleanup(fail(ADI_EINVAL, "instance %d: geometry values must be finite", i));
    if (!(0.0 < g.r0 && g.r0 <= g.r1 && g.r1 <= g.r2 && g.r2 <= g.rmax) ||
        !(0.0 < g.z0 && g.z0 <= g.zmax && g.zmax <= g.ztop))
      return cleanup(fail(ADI_EINVAL, "instance %d: layers out of order", i));
    if (g.r_faces || g.z_faces)
      return cleanup(fail(ADI_EUNSUPPORTED, "instance %d: batches use uniform grids", i));
    if (g.nr < 3 || g.nz < 3 || g.nr > kMaxNr || g.nz > kMaxNz)
      return cleanup(fail(ADI_EUNSUPPORTED, "instance %d: grid %dx%d outside 3..%d x 3..%d", i, g.nr, g.nz,
                          kMaxNr, kMaxNz));
    for (int c = 0; c < 4; ++c)
      if (!(bc.h[c] >= 0.0) || !is_fin(bc.t_inf[c]))
        return cleanup(fail(ADI_EINVAL, "instance %d: invalid boundary film %d", i, c));
    BatchInst& I = b->hinst[i];
    memset(&I, 0, sizeof I);
    Params& P = I.P;
    P.r0 = g.r0; P.r1 = g.r1; P.r2 = g.r2; P.rmax = g.rmax;
    P.z0 = g.z0; P.zmax = g.zmax; P.ztop = g.ztop;
    P.nr = g.nr; P.nz = g.nz;
    for (int c = 0; c < 4; ++c) { P.h[c] = bc.h[c]; P.tinf[c] = bc.t_inf[c]; }
    I.rs = shape_index(kBR_M, kBR_G, g.nr);
    I.zs = shape_index(kBZ_M, kBZ_G, g.nz);
    I.zss = batch_strip_zshape(g.nz);
    b->maxstrip = std::max(b->maxstrip, batch_strip_doubles(g.nr, g.nz));
    I.toff = off;
    off += ((long)g.nr * g.nz + 31) & ~31L;  // 256-byte aligned fields (16-byte vector stores)
    b->maxcells = std::max(b->maxcells, (long)g.nr * g.nz);
    // cells outside the domain: columns with centre r >= r0 times rows with
    // z0 <= centre z < zmax (centres evaluated as on the device)
    long ncol = 0, nrow = 0;
    for (int ii = 0; ii < g.nr; ++ii) ncol += (ii + 0.5) * g.rmax / g.nr >= g.r0;
    for (int jj = 0; jj < g.nz; ++jj) {
      const double zc = (jj + 0.5) * g.ztop / g.nz;
      nrow += zc >= g.z0 && zc < g.zmax;
    }
    b->cells += (long)g.nr * g.nz;
    b->active += (long)g.nr * g.nz - ncol * nrow;
  }
  b->total_cells = off;
  b->lay = batch_layout(b->maxcells, b->maxstrip);
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)));
  b->stream = (hipStream_t)hip_stream;
  if (!b->stream) {
    e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e)));
    b->own_stream = true;
  }
  // longest instances first (every instance runs the same number of steps)
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (long)b->hinst[x].P.nr * b->hinst[x].P.nz > (long)b->hinst[y].P.nr * b->hinst[y].P.nz;
  });
  adi_status st;
  if ((st = dev_alloc((void**)&b->dinst, sizeof(BatchInst) * n, b->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&b->dorder, sizeof(int) * n, b->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&b->queue, 256, b->stream)) != ADI_OK) return cleanup(st);
  if ((st = dev_alloc((void**)&b->T, sizeof(double) * b->total_cells, b->stream)) != ADI_OK) return cleanup(st);
  e = hipMemcpyAsync(b->dorder, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return cleanup(fail(ADI_EDEVICE, "upload order: %s", hipGetErrorString(e)));
  *out = b;
  return ADI_OK;
}

adi_status adi_batch_set_materials(adi_batch b, const double* k, const double* rho_c, const double* q) {
  ADI_TRY(batch_handle(b));
  if (!k || !rho_c || !q) return fail(ADI_EINVAL, "null material array");
  for (int i = 0; i < b->n; ++i)
    for (int m = 0; m < 5; ++m) {
      const double kk = k[5 * i + m], rc = rho_c[5 * i + m], qq = q[5 * i + m];
      if (!(kk > 0.0) || !is_fin(kk)) return fail(ADI_EINVAL, "instance %d: k[%d] must be > 0", i, m);
      if (!(rc > 0.0) || !is_fin(rc)) return fail(ADI_EINVAL, "instance %d: rho_c[%d] must be > 0", i, m);
      if (!is_fin(qq)) return fail(ADI_ENONFINITE, "instance %d: q[%d] is not finite", i, m);
    }
  for (int i = 0; i < b->n; ++i)
    for (int m = 0; m < 5; ++m) {
      b->hinst[i].P.k[m] = k[5 * i + m];
      b->hinst[i].P.rhoc[m] = rho_c[5 * i + m];
      b->hinst[i].P.q[m] = q[5 * i + m];
    }
  b->has_mat = true;
  return ADI_OK;
}

adi_status adi_batch_set_initial(adi_batch b, const double* T0) {
  ADI_TRY(batch_handle(b));
  for (int i = 0; i < b->n; ++i) {
    const double v = T0 ? T0[i] : 0.0;
    if (!is_fin(v)) return fail(ADI_ENONFINITE, "instance %d: T0 is not finite", i);
    b->hinst[i].T0 = v;
  }
  return ADI_OK;
}

adi_status adi_batch_set_launch(adi_batch b, int32_t lines_per_lane, int32_t waves_per_block,
                                int32_t blocks_per_cu) {
  ADI_TRY(batch_handle(b));
  int v = -1;
  for (int i = 0; i < kNumBatchVariants; ++i)
    if (kBatchVariants[i].R == lines_per_lane && kBatchVariants[i].NW == waves_per_block) v = i;
  if (v < 0) return fail(ADI_EUNSUPPORTED, "no batch kernel with %d lines/lane and %d waves/block", lines_per_lane,
                         waves_per_block);
  if (blocks_per_cu < 1 || blocks_per_cu > 8) return fail(ADI_EINVAL, "blocks_per_cu must be in [1, 8]");
  b->variant = v;
  b->blocks_per_cu = blocks_per_cu;
  return ADI_OK;
}

adi_status adi_batch_zshape_info(int32_t zclass, int32_t variant, int32_t* waves, int32_t* cells,
                                 int32_t* max_rows) {
  if (!waves || !cells || !max_rows) return fail(ADI_EINVAL, "null output");
  if (zclass < 0 || zclass > 3) return fail(ADI_EINVAL, "z class %d outside 0..3", zclass);
  if (!bwz_valid(zclass, variant)) return fail(ADI_EINVAL, "z class %d has no shape %d", zclass, variant);
  *waves = kBWZ_W[zclass][variant];
  *cells = kBWZ_CM[zclass][variant];
  *max_rows = kBS_G * kBSZ_M[zclass];
  return ADI_OK;
}

adi_status adi_batch_set_zshape(adi_batch b, int32_t zclass, int32_t variant) {
  ADI_TRY(batch_handle(b));
  if (zclass < 0 || zclass > 3) return fail(ADI_EINVAL, "z class %d outside 0..3", zclass);
  if (!bwz_valid(zclass, variant)) return fail(ADI_EINVAL, "z class %d has no shape %d", zclass, variant);
  b->zvar[zclass] = variant;
  return ADI_OK;
}

adi_status adi_batch_step(adi_batch b, double dt, int64_t nsteps, int32_t snapshot_every, int32_t npts,
                          double* dev_profiles) {
  ADI_TRY(batch_handle(b));
  if (!b->has_mat) return fail(ADI_ESTATE, "adi_batch_set_materials must be called before stepping");
  if (!(dt > 0.0) || !is_fin(dt)) return fail(ADI_EINVAL, "dt must be > 0 and finite");
  if (nsteps < 1 || nsteps > (1 << 30)) return fail(ADI_EINVAL, "nsteps must be in [1, 2^30]");
  if (snapshot_every < 0) return fail(ADI_EINVAL, "snapshot_every must be >= 0");
  if (npts < 1 || npts > 4096) return fail(ADI_EINVAL, "npts must be in [1, 4096]");
  const int nsnap = snapshot_every > 0 ? (int)(nsteps / snapshot_every) : 0;
  const long need = (long)b->n * std::max(nsnap, 1) * npts;
  if (!dev_profiles && need > b->prof_cap) {
    ADI_HIP(hipStreamSynchronize(b->stream));
    dev_free(b->prof);
    b->prof = nullptr;
    ADI_TRY(dev_alloc((void**)&b->prof, sizeof(double) * need, b->stream));
    b->prof_cap = need;
  }
  b->nsnap = nsnap;
  b->npts = npts;
  b->prof_out = dev_profiles ? dev_profiles : b->prof;
  for (auto& I : b->hinst) {
    I.P.ta = b->scheme == ADI_PR ? 0.5 * dt : dt;
    I.P.theta = b->scheme == ADI_PR ? 1.0 : 0.0;
  }
  ADI_HIP(hipMemcpyAsync(b->dinst, b->hinst.data(), sizeof(BatchInst) * b->n, hipMemcpyHostToDevice, b->stream));
  const BatchVariant& V = kBatchVariants[b->variant];
  if (!V.fn) ADI_TRY(ensure_sweep(b));
  else ADI_TRY(ensure_scratch(b));
  BatchArgs a;
  a.inst = b->dinst;
  a.order = b->dorder;
  a.ninst = b->n;
  a.queue = b->queue;
  a.T = b->T;
  a.prof = b->prof_out;
  a.nsnap = nsnap;
  a.npts = npts;
  a.snap_every = snapshot_every;
  a.nsteps = (int)nsteps;
  a.scratch = b->scratch;
  a.lay = b->lay;
  if (V.fn) {
    // queue reset + persistent kernel, captured into one graph and launched
    ADI_TRY(launch_captured(b, [&] {
      hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, b->stream, b->queue);
      hipLaunchKernelGGL(V.fn, dim3(b->nblocks), dim3(64 * V.NW), 0, b->stream, a);
    }));
  } else {
    // batched sweep launches, captured kSweepGraphSteps steps at a time
    for (int64_t st0 = 1; st0 <= nsteps; st0 += kSweepGraphSteps) {
      const int64_t st1 = std::min(nsteps, st0 + kSweepGraphSteps - 1);
      ADI_TRY(launch_captured(b, [&] { launch_sweeps(b, st0, st1, nsteps, snapshot_every, nsnap, npts); }));
    }
  }
  b->steps = nsteps;
  return ADI_OK;
}

adi_status adi_batch_sync(adi_batch b) {
  ADI_TRY(batch_handle(b));
  ADI_HIP(hipStreamSynchronize(b->stream));
  return ADI_OK;
}

adi_status adi_batch_read_profiles(adi_batch b, int32_t npts, double* host_out, size_t count) {
  ADI_TRY(batch_handle(b));
  if (!host_out) return fail(ADI_EINVAL, "null output buffer");
  if (npts != b->npts) return fail(ADI_EINVAL, "npts %d != %d, the points per profile of the last step", npts, b->npts);
  const size_t n = (size_t)b->n * b->nsnap * b->npts;
  if (count != n) return fail(ADI_EINVAL, "count %zu != n*nsnap*npts = %zu", count, n);
  if (n) ADI_HIP(hipMemcpyAsync(host_out, b->prof_out, sizeof(double) * n, hipMemcpyDefault, b->stream));
  ADI_HIP(hipStreamSynchronize(b->stream));
  return ADI_OK;
}

adi_status adi_batch_read_field(adi_batch b, int32_t i, double* host_out, size_t count) {
  ADI_TRY(batch_handle(b));
  if (i < 0 || i >= b->n) return fail(ADI_EINVAL, "instance %d out of range", i);
  if (!host_out) return fail(ADI_EINVAL, "null output buffer");
  const size_t n = (size_t)b->hinst[i].P.nr * b->hinst[i].P.nz;
  if (count != n) return fail(ADI_EINVAL, "count %zu != nz*nr = %zu", count, n);
  ADI_HIP(hipMemcpyAsync(host_out, b->T + b->hinst[i].toff, sizeof(double) * n, hipMemcpyDeviceToHost,
                         b->stream));
  ADI_HIP(hipStreamSynchronize(b->stream));
  return ADI_OK;
}

adi_status adi_batch_info(adi_batch b, int64_t* total_cells, int32_t* nsnap, int32_t* workgroups) {
  ADI_TRY(batch_handle(b));
  if (total_cells) *total_cells = b->total_cells;
  if (nsnap) *nsnap = b->nsnap;
  if (workgroups)
    *workgroups = kBatchVariants[b->variant].fn ? b->nblocks : b->nmap_r[0] + b->nmap_r[1] + b->nmap_r[2];
  return ADI_OK;
}

adi_status adi_batch_active_cells(adi_batch b, int64_t* active) {
  ADI_TRY(batch_handle(b));
  if (!active) return fail(ADI_EINVAL, "null output");
  *active = b->active;
  return ADI_OK;
}

adi_status adi_batch_time(adi_batch b, double dt, int64_t nsteps, int32_t reps, float* ms_out) {
  ADI_TRY(batch_handle(b));
  if (reps < 1) return fail(ADI_EINVAL, "reps must be >= 1");
  if (!ms_out) return fail(ADI_EINVAL, "null output");
  hipEvent_t ev[2];
  for (auto& x : ev) ADI_HIP(hipEventCreate(&x));
  adi_status st = ADI_OK;
  (void)hipEventRecord(ev[0], b->stream);
  for (int i = 0; i < reps && st == ADI_OK; ++i) st = adi_batch_step(b, dt, nsteps, 0, 64, nullptr);
  (void)hipEventRecord(ev[1], b->stream);
  hipError_t e = hipEventSynchronize(ev[1]);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  for (auto& x : ev) (void)hipEventDestroy(x);
  if (st != ADI_OK) return st;
  if (e != hipSuccess) return fail(ADI_EDEVICE, "event timing: %s", hipGetErrorString(e));
  *ms_out = ms / reps;
  return ADI_OK;
}

void adi_batch_destroy(adi_batch b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  void* bufs[] = {b->dinst, b->dorder, b->queue, b->T, b->prof, b->scratch, b->saux, b->srhs, b->srhs_off,
                  b->sargs, b->smap};
  for (void* p : bufs) dev_free(p);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
