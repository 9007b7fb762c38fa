// batch.hpp -- ragged batch: instance descriptors, scratch layout and the
// persistent kernel on the strip-layout line solver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "device.hpp"
#include "strip.hpp"

namespace adi {

// Compiled line shapes of the batch kernel (one wave per line group):
// r lines use 4 lines x 16 chunks per wave, z lines 2 lines x 32 chunks.
constexpr int kBR_LPW = 4, kBR_G = 16;
constexpr int kBZ_LPW = 2, kBZ_G = 32;
constexpr int kBR_M[4] = {4, 6, 8, 12};   // r lines up to 64, 96, 128, 192 cells
constexpr int kBZ_M[4] = {5, 8, 10, 15};  // z lines up to 160, 256, 320, 480 cells
constexpr int kMaxNr = 192, kMaxNz = 480;

struct BatchInst {
  Params P;
  long toff;   // offset of the instance's field in the arena (doubles)
  int rs, zs;  // shape index of its r and z lines (rows-layout kernels)
  int zss;     // shape index of its z lines for the strip-layout kernel
  double T0;   // uniform initial temperature
};

// Byte offsets inside one workgroup's scratch area.
struct BatchLayout {
  long dA, dB, geo, kap, bet, ranges, rtabs, rpos, rchk, reng, rxc, ztabs, zpos, zchk, zeng, zxc, work;
  long stride;
};

struct BatchArgs {
  const BatchInst* inst;
  const int* order;
  int ninst;
  int* queue;
  double* T;
  double* prof;
  int nsnap, npts, snap_every;
  int nsteps;
  char* scratch;
  BatchLayout lay;
};

__device__ __forceinline__ void skip_range(int dir, int cls, const int* ranges, int n, int* lo, int* hi) {
  // masked cells of an r line in band 1: columns of classes 1..3, i.e. from
  // the end of column class 0; of a z line of class >= 1: rows of band 1
  *lo = *hi = n;
  if (dir == 0 && cls == 1) {
    const int i0 = ranges[(1 * MAX_CLS + 0) * 2 + 1];
    if (i0 < n) { *lo = i0; *hi = n; }
  } else if (dir == 1 && cls >= 1) {
    const int a = ranges[(0 * MAX_CLS + 1) * 2], b = ranges[(0 * MAX_CLS + 1) * 2 + 1];
    if (b > a) { *lo = a; *hi = b; }
  }
}

// Strip-layout batch kernel: one wave per block of 4 lines.  r lines: 64
// chunks of 4 cells (up to 256 cells); z lines: 64 chunks of kBSZ_M[zss]
// cells (up to 192, 256, 320, 512 rows).
constexpr int kBSR_M = 4;
constexpr int kBSZ_M[4] = {3, 4, 5, 8};
constexpr int kBS_G = 64;
// z lines of the batched sweep launches: candidate shapes of each z shape
// class (lines up to 192, 256, 320, 512 rows), as waves of 64 chunks and
// cells per chunk; every candidate covers its class's longest lines, the
// first is the default and the autotuner picks one per class (0 = unused).
constexpr int kBWZ_NV = 3;
constexpr int kBWZ_W[4][kBWZ_NV] = {{1, 2, 0}, {1, 2, 0}, {1, 2, 0}, {2, 1, 3}};
constexpr int kBWZ_CM[4][kBWZ_NV] = {{3, 3, 0}, {4, 3, 0}, {5, 3, 0}, {4, 8, 3}};

__host__ __device__ constexpr bool bwz_valid(int c, int v) {
  return c >= 0 && c < 4 && v >= 0 && v < kBWZ_NV && kBWZ_W[c][v] > 0;
}

// Calls f(integral_constant<M>, integral_constant<NW>) with the compiled
// shape of candidate v of z class c (the default when v is not a candidate).
template <class F>
inline void bwz_dispatch(int c, int v, F&& f) {
  using std::integral_constant;
  if (!bwz_valid(c, v)) v = 0;
  switch (c * kBWZ_NV + v) {
    case 0: f(integral_constant<int, 3>{}, integral_constant<int, 1>{}); break;
    case 1: f(integral_constant<int, 3>{}, integral_constant<int, 2>{}); break;
    case 3: f(integral_constant<int, 4>{}, integral_constant<int, 1>{}); break;
    case 4: f(integral_constant<int, 3>{}, integral_constant<int, 2>{}); break;
    case 6: f(integral_constant<int, 5>{}, integral_constant<int, 1>{}); break;
    case 7: f(integral_constant<int, 3>{}, integral_constant<int, 2>{}); break;
    case 9: f(integral_constant<int, 4>{}, integral_constant<int, 2>{}); break;
    case 10: f(integral_constant<int, 8>{}, integral_constant<int, 1>{}); break;
    default: f(integral_constant<int, 3>{}, integral_constant<int, 3>{}); break;
  }
}

__host__ __device__ inline int batch_strip_zshape(int nz) {
  for (int s = 0; s < 4; ++s)
    if (kBS_G * kBSZ_M[s] >= nz) return s;
  return -1;
}

// Doubles of one right-hand side of an nr x nz instance in the strip layout.
__host__ __device__ inline long batch_strip_doubles(int nr, int nz) {
  return (long)((nr + 3) / 4) * 16L * ((nz + 3) / 4);
}

// The geometry of an instance in its scratch area (fixed-size arrays).
__device__ __forceinline__ Geom batch_geom(char* ws, const BatchLayout& Ly) {
  Geom g;
  double* gd = (double*)(ws + Ly.geo);
  g.rf = gd; g.rc = gd + (kMaxNr + 1); g.dr = gd + 2 * (kMaxNr + 1);
  g.zf = gd + 3 * (kMaxNr + 1); g.zc = g.zf + (kMaxNz + 1); g.dz = g.zf + 2 * (kMaxNz + 1);
  g.kap = (uint8_t*)(ws + Ly.kap);
  g.bet = (uint8_t*)(ws + Ly.bet);
  return g;
}

// Prologue of an instance on the strip-layout batch paths, by a whole
// workgroup: geometry and line-class tables (r lines 64 chunks of 4 cells,
// z lines Gz chunks of Mz cells) in the scratch area ws, the first
// r half step's right-hand side (from the uniform field T0; strip layout,
// exact zeros outside the domain and in the padding) into dA, and the sweep
// arguments (r: dA -> dB, z: dB -> dA, no solution output), written by
// thread 0 into ar and az.  Ends with a workgroup barrier.
__device__ void batch_strip_prologue(const BatchInst& I, char* ws, const BatchLayout& Ly, double* dA, double* dB,
                                     StripArgs* ar, StripArgs* az, int Gz, int Mz) {
  const Params& P = I.P;
  const int nr = P.nr, nz = P.nz;
  int* ranges = (int*)(ws + Ly.ranges);
  Geom g = batch_geom(ws, Ly);
  build_geometry(P, nullptr, nullptr, g, ranges);

  double* rpos = (double*)(ws + Ly.rpos);
  double* rchk = (double*)(ws + Ly.rchk);
  double* reng = (double*)(ws + Ly.reng);
  double* rxc = (double*)(ws + Ly.rxc);
  double* zpos = (double*)(ws + Ly.zpos);
  double* zchk = (double*)(ws + Ly.zchk);
  double* zeng = (double*)(ws + Ly.zeng);
  double* zxc = (double*)(ws + Ly.zxc);
  double* work = (double*)(ws + Ly.work);
  const long rGM = (long)kBS_G * kBSR_M, zGM = (long)Gz * Mz;
  for (int c = 0; c < 3; ++c)
    assemble_class(P, g, 0, c, kBS_G, kBSR_M, rpos + c * P_NFIELDS * rGM, rchk + c * C_NFIELDS * kBS_G,
                   reng + c * 2 * nr, rxc + c * nr, work, false);
  for (int c = 0; c < 4; ++c)
    assemble_class(P, g, 1, c, Gz, Mz, zpos + c * P_NFIELDS * zGM, zchk + c * C_NFIELDS * Gz,
                   zeng + c * 2 * nz, zxc + c * nz, work, false);
  // sweep arguments (uniform across the workgroup; read on use)
  if (threadIdx.x == 0) {
    bool ambient = false;
    for (int c = 0; c < 4; ++c) ambient = ambient || P.tinf[c] != 0.0;
    for (int c = 0; c < MAX_CLS; ++c) {
      LineTab t;
      const int cr = c < 3 ? c : 0;
      t.pos = rpos + cr * P_NFIELDS * rGM;
      t.chk = rchk + cr * C_NFIELDS * kBS_G;
      t.n = nr; t.G = kBS_G; t.M = kBSR_M;
      skip_range(0, cr, ranges, nr, &t.skip_lo, &t.skip_hi);
      ar->tabs[c] = t;
      t.pos = zpos + c * P_NFIELDS * zGM;
      t.chk = zchk + c * C_NFIELDS * Gz;
      t.n = nz; t.G = Gz; t.M = Mz;
      skip_range(1, c, ranges, nz, &t.skip_lo, &t.skip_hi);
      az->tabs[c] = t;
    }
    ar->strip = az->strip = 16L * ((nz + 3) / 4);
    ar->nr = az->nr = nr;
    ar->nz = az->nz = nz;
    ar->xc = ambient ? zxc : nullptr;  // the r sweep adds b_z, the z sweep b_r
    az->xc = ambient ? rxc : nullptr;
    ar->nlines = nz;
    az->nlines = nr;
    strip_class_ends(ranges, 0, 3, ar->line_end);
    strip_class_ends(ranges, 1, 4, ar->pos_end);
    ar->nxcls = 4;
    strip_class_ends(ranges, 1, 4, az->line_end);
    strip_class_ends(ranges, 0, 3, az->pos_end);
    az->nxcls = 3;
    ar->nblocks = az->nblocks = 0;
    ar->nmix = az->nmix = 0;
    ar->theta = az->theta = P.theta;
    ar->din = dA; ar->dout = dB; ar->xout = nullptr;
    az->din = dB; az->dout = dA; az->xout = nullptr;
  }
  const long sstrip = 16L * ((nz + 3) / 4);

  // right-hand side of the first r half step from the uniform field T0
  const long nbuf = batch_strip_doubles(nr, nz);
  for (long e = threadIdx.x; e < nbuf; e += blockDim.x) {
    const long s = e / sstrip, rem = e - s * sstrip;
    const int j = (int)(rem >> 2), i = (int)(4 * s + (rem & 3));
    double o = 0.0;
    if (i < nr && j < nz) {
      const int kap = g.kap[i], bet = g.bet[j];
      if (region_of(bet, kap) != MASKED) {
        const double* pz = zpos + kap * P_NFIELDS * zGM;
        const long ix = (long)(j % Mz) * Gz + j / Mz;
        o = (pz[pos_at(P_OD, zGM, ix, false)] + pz[pos_at(P_OL, zGM, ix, false)] * (j > 0) + pz[pos_at(P_OU, zGM, ix, false)] * (j < nz - 1)) * I.T0 +
            pz[pos_at(P_OC, zGM, ix, false)] + rxc[bet * nr + i];
      }
    }
    dA[e] = o;
  }
  __syncthreads();
}

// Outer terminal-face profile of an instance (linear interpolation of its
// top row at npts points r = (k + 1/2) rmax / npts), by a whole workgroup.
__device__ void batch_profile(const Params& P, const Geom& g, const double* Ti, double* out, int npts) {
  const int nr = P.nr, nz = P.nz;
  const double* row = Ti + (long)(nz - 1) * nr;
  for (int kk = threadIdx.x; kk < npts; kk += blockDim.x) {
    const double r = (kk + 0.5) * P.rmax / npts;
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
    out[kk] = o;
  }
}

// The persistent batch kernel on the strip-layout line solver.  Each
// workgroup pops the next instance from the queue, runs its prologue
// (geometry, tables, first right-hand side) in its scratch and runs the
// time loop: every wave takes whole blocks of 4 lines (r row groups, then z
// strips) and solves them alone (DPP scans inside the wave, no workgroup
// barrier inside a sweep); the workgroup synchronises between sweeps.
template <int NW>
__global__ void __launch_bounds__(64 * NW) k_batch_s(BatchArgs a) {
  __shared__ __align__(16) double lbuf[NW][64 * 4 * 8];  // per wave: a z strip or 64 r tiles
  __shared__ double lcarry[NW][strip_carry(1)];          // unused: one wave per line
  __shared__ StripArgs s_args[2];  // r sweep, z sweep
  __shared__ int s_next;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  char* ws = a.scratch + (long)blockIdx.x * a.lay.stride;
  const BatchLayout& Ly = a.lay;
  double* dA = (double*)(ws + Ly.dA);
  double* dB = (double*)(ws + Ly.dB);
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
    batch_strip_prologue(I, ws, Ly, dA, dB, &s_args[0], &s_args[1], kBS_G, kBSZ_M[I.zss]);
    const Geom g = batch_geom(ws, Ly);

    double* Ti = a.T + I.toff;
    const int nrg = (nz + 3) / 4, nstrips = (nr + 3) / 4;
    int snap = 0;
    for (int st = 1; st <= a.nsteps; ++st) {
      const bool take = a.snap_every > 0 && st % a.snap_every == 0 && snap < a.nsnap;
      for (int J = wave; J < nrg; J += NW) strip_r_body<1>(s_args[0], J, lane, lbuf[wave], lcarry[wave]);
      if (threadIdx.x == 0) s_args[1].xout = (take || st == a.nsteps) ? Ti : nullptr;
      __syncthreads();
      for (int s = wave; s < nstrips; s += NW) {
        switch (I.zss) {
          case 0: strip_z_body<kBSZ_M[0], 1>(s_args[1], s, lane, lbuf[wave], lcarry[wave]); break;
          case 1: strip_z_body<kBSZ_M[1], 1>(s_args[1], s, lane, lbuf[wave], lcarry[wave]); break;
          case 2: strip_z_body<kBSZ_M[2], 1>(s_args[1], s, lane, lbuf[wave], lcarry[wave]); break;
          default: strip_z_body<kBSZ_M[3], 1>(s_args[1], s, lane, lbuf[wave], lcarry[wave]); break;
        }
      }
      __syncthreads();
      if (take) {
        batch_profile(P, g, Ti, a.prof + ((long)idx * a.nsnap + snap) * a.npts, a.npts);
        ++snap;
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------- batched sweep launches ---
//
// The other way to run the batch: every half step is one launch over all
// instances (r), or over the instances of one z chunk shape (z), with one
// single-wave workgroup per block of 4 lines.  Hundreds of thousands of
// independent workgroups per launch keep every CU busy with workgroups in
// different phases (loading, solving, storing), unlike the persistent
// kernel, where each workgroup steps one instance alone.  Each instance
// keeps its own strip-layout right-hand sides and scratch area.

// Arguments of the batched-sweep kernels.
struct BSweepArgs {
  const BatchInst* inst;
  char* aux;           // scratch areas, one per instance (stride lay.stride)
  BatchLayout lay;
  double* rhs;         // right-hand sides: instance i at rhs_off[i] (dA), + its strip size (dB)
  const long* rhs_off;
  StripArgs* args;     // [3][n]: r sweep, z sweep, z sweep writing the field
  const int* map;      // workgroup -> 256 * instance + block of 4 lines
  int n;
  double* T;
  double* prof;
  int npts;
  int zvar[4];         // candidate shape of each z class
};

// One workgroup per instance: prologue into its own scratch area and
// right-hand sides.
__global__ void __launch_bounds__(256) k_bsetup(BSweepArgs a) {
  const int i = blockIdx.x;
  const BatchInst I = a.inst[i];
  double* dA = a.rhs + a.rhs_off[i];
  double* dB = dA + batch_strip_doubles(I.P.nr, I.P.nz);
  batch_strip_prologue(I, a.aux + (long)i * a.lay.stride, a.lay, dA, dB, &a.args[i], &a.args[a.n + i],
                       64 * kBWZ_W[I.zss][a.zvar[I.zss]], kBWZ_CM[I.zss][a.zvar[I.zss]]);
  if (threadIdx.x == 0) {
    a.args[2 * a.n + i] = a.args[a.n + i];
    a.args[2 * a.n + i].xout = a.T + I.toff;
  }
}

// r half step of the instances whose rows fit CPW tiles (4*CPW cells):
// workgroup -> (instance, first of 64/CPW consecutive row groups).
template <int CPW>
__global__ void __launch_bounds__(64) k_bsweep_r(BSweepArgs a) {
  __shared__ __align__(16) double buf[64 * 18];
  __shared__ double carry[strip_carry(1)];
  const int e = a.map[xcd_block(blockIdx.x, gridDim.x)];
  strip_r_slots<CPW>(a.args[e >> 8], e & 255, buf, carry);
}

// Tile slot width of the batched r sweep of an instance with nr columns.
__host__ __device__ inline int bsweep_r_cpw(int nr) {
  const int tiles = (nr + 3) / 4;
  return tiles <= 16 ? 16 : (tiles <= 32 ? 32 : 64);
}

// z half step of the instances of one z shape (NW waves of chunks of M
// cells): workgroup -> (instance, strip); the solution goes to the
// instance's field when `snap` is set.
template <int M, int NW>
__global__ void __launch_bounds__(64 * NW) k_bsweep_z(BSweepArgs a, int snap) {
  __shared__ __align__(16) double buf[64 * NW * 4 * M];
  __shared__ double carry[strip_carry(NW)];
  const int e = a.map[xcd_block(blockIdx.x, gridDim.x)];
  strip_z_body<M, NW>(a.args[(snap ? 2 : 1) * a.n + (e >> 8)], e & 255, threadIdx.x, buf, carry);
}

// Terminal-face profiles of every instance (snapshot `snap` of nsnap).
__global__ void __launch_bounds__(64) k_bprofile(BSweepArgs a, int snap, int nsnap) {
  const int i = blockIdx.x;
  const BatchInst I = a.inst[i];
  const Geom g = batch_geom(a.aux + (long)i * a.lay.stride, a.lay);
  batch_profile(I.P, g, a.T + I.toff, a.prof + ((long)i * nsnap + snap) * a.npts, a.npts);
}

// Scratch layout of one workgroup (persistent kernels) or one instance
// (batched sweeps, maxcells = maxstrip = 0: no right-hand sides).
inline BatchLayout batch_layout(long maxcells, long maxstrip) {
  BatchLayout L{};
  long off = 0;
  auto put = [&](long bytes) {
    const long o = off;
    off += (bytes + 255) & ~255L;
    return o;
  };
  // tables sized for both kernel families (rows layout, strip layout)
  const long rGM = std::max((long)kBR_G * kBR_M[3], (long)kBS_G * kBSR_M);
  long zGM = std::max((long)kBZ_G * kBZ_M[3], (long)kBS_G * kBSZ_M[3]);
  long zG = std::max(kBZ_G, kBS_G);
  for (int c = 0; c < 4; ++c)
    for (int v = 0; v < kBWZ_NV; ++v) {
      zGM = std::max(zGM, 64L * kBWZ_W[c][v] * kBWZ_CM[c][v]);
      zG = std::max(zG, 64L * kBWZ_W[c][v]);
    }
  const long rG = std::max(kBR_G, kBS_G);
  L.dA = put(8 * std::max(maxcells, maxstrip));
  L.dB = put(8 * std::max(maxcells, maxstrip));
  L.geo = put(8 * (3 * (kMaxNr + 1) + 3 * (kMaxNz + 1)));
  L.kap = put(kMaxNr);
  L.bet = put(kMaxNz);
  L.ranges = put(4 * 17);
  L.rtabs = put(sizeof(LineTab) * 3);
  L.rpos = put(8 * 3 * P_NFIELDS * rGM);
  L.rchk = put(8 * 3 * C_NFIELDS * rG);
  L.reng = put(8 * 3 * 2 * kMaxNr);
  L.rxc = put(8 * 3 * kMaxNr);
  L.ztabs = put(sizeof(LineTab) * 4);
  L.zpos = put(8 * 4 * P_NFIELDS * zGM);
  L.zchk = put(8 * 4 * C_NFIELDS * zG);
  L.zeng = put(8 * 4 * 2 * kMaxNz);
  L.zxc = put(8 * 4 * kMaxNz);
  long work = std::max(std::max(assemble_work(kBR_G, kBR_M[3]), assemble_work(kBZ_G, kBZ_M[3])),
                       std::max(assemble_work(kBS_G, kBSR_M), assemble_work(kBS_G, kBSZ_M[3])));
  for (int c = 0; c < 4; ++c)
    for (int v = 0; v < kBWZ_NV; ++v)
      if (bwz_valid(c, v)) work = std::max(work, assemble_work(64 * kBWZ_W[c][v], kBWZ_CM[c][v]));
  L.work = put(8 * work);
  L.stride = off;
  return L;
}

// Host plan of the batched sweep launches: each instance's right-hand sides
// (two strip-layout buffers, 256-byte aligned) in one arena, and the
// workgroup maps (256 * instance + first block of 4 lines): r launches by
// row slot width (16, 32, 64 tiles), z launches by z shape.
struct BSweepPlan {
  std::vector<long> off;  // doubles
  long total = 0;
  std::vector<int> map;
  int nmap_r[3] = {0, 0, 0}, rmap_off[3] = {0, 0, 0};
  int nmap_z[4] = {0, 0, 0, 0}, zmap_off[4] = {0, 0, 0, 0};
};

inline BSweepPlan bsweep_plan(const BatchInst* inst, int n) {
  BSweepPlan p;
  p.off.resize(n);
  for (int i = 0; i < n; ++i) {
    p.off[i] = p.total;
    p.total += (2 * batch_strip_doubles(inst[i].P.nr, inst[i].P.nz) + 31) & ~31L;
  }
  for (int w = 0; w < 3; ++w) {
    const int cpw = 16 << w, per = 64 / cpw;
    p.rmap_off[w] = (int)p.map.size();
    for (int i = 0; i < n; ++i)
      if (bsweep_r_cpw(inst[i].P.nr) == cpw)
        for (int J = 0; J < (inst[i].P.nz + 3) / 4; J += per) p.map.push_back(256 * i + J);
    p.nmap_r[w] = (int)p.map.size() - p.rmap_off[w];
  }
  for (int c = 0; c < 4; ++c) {
    p.zmap_off[c] = (int)p.map.size();
    for (int i = 0; i < n; ++i)
      if (inst[i].zss == c)
        for (int q = 0; q < (inst[i].P.nr + 3) / 4; ++q) p.map.push_back(256 * i + q);
    p.nmap_z[c] = (int)p.map.size() - p.zmap_off[c];
  }
  return p;
}

}  // namespace adi
