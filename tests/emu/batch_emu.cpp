// CPU emulation of the batched sweep launches of the ragged batch (test
// infrastructure).  Reads a batch from argv[1] (text: "n scheme dt nsteps",
// then per instance its geometry, grid, films, materials and T0), runs the
// library's instance set-up kernel and, per step, its r launches (every row
// slot width) and z launches (every z shape) over all instances, with the
// library's own host plan of workgroup maps, and writes the final fields
// (each nz*nr doubles, r fastest, in instance order) to argv[2].  argv[3..6]:
// the z shape of each z class (default 0).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hip/hip_runtime.h"
#include "device.hpp"
#include "strip.hpp"
#include "batch.hpp"

using namespace adi;

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  FILE* f = fopen(argv[1], "r");
  if (!f) return 2;
  int n = 0, scheme = 0, nsteps = 0, ok = 1;
  double dt = 0.0;
  ok &= fscanf(f, "%d %d %lf %d", &n, &scheme, &dt, &nsteps) == 4;
  if (!ok || n < 1) return 2;
  std::vector<BatchInst> inst(n);
  long toff = 0;
  for (int i = 0; i < n && ok; ++i) {
    BatchInst& I = inst[i];
    memset(&I, 0, sizeof I);
    Params& P = I.P;
    ok &= fscanf(f, "%lf %lf %lf %lf %lf %lf %lf %d %d", &P.r0, &P.r1, &P.r2, &P.rmax, &P.z0, &P.zmax, &P.ztop,
                 &P.nr, &P.nz) == 9;
    for (int c = 0; c < 4; ++c) ok &= fscanf(f, "%lf", &P.h[c]) == 1;
    for (int c = 0; c < 4; ++c) ok &= fscanf(f, "%lf", &P.tinf[c]) == 1;
    for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.k[c]) == 1;
    for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.rhoc[c]) == 1;
    for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.q[c]) == 1;
    ok &= fscanf(f, "%lf", &I.T0) == 1;
    if (P.nr < 3 || P.nz < 3 || P.nr > kMaxNr || P.nz > kMaxNz) ok = 0;
    P.ta = scheme == 0 ? 0.5 * dt : dt;
    P.theta = scheme == 0 ? 1.0 : 0.0;
    I.zss = batch_strip_zshape(P.nz);
    I.toff = toff;
    toff += ((long)P.nr * P.nz + 31) & ~31L;
  }
  fclose(f);
  if (!ok) return 2;
  const BatchLayout lay = batch_layout(0, 0);
  const BSweepPlan plan = bsweep_plan(inst.data(), n);
  std::vector<double> aux(lay.stride / 8 * n + 32, 0.0), rhs(plan.total, 0.0), T(toff, 0.0);
  std::vector<StripArgs> args(3 * n);
  BSweepArgs a;
  a.inst = inst.data();
  a.aux = (char*)aux.data();
  a.lay = lay;
  a.rhs = rhs.data();
  a.rhs_off = plan.off.data();
  a.args = args.data();
  a.map = plan.map.data();
  a.n = n;
  a.T = T.data();
  a.prof = nullptr;
  a.npts = 64;
  for (int c = 0; c < 4; ++c) {
    a.zvar[c] = argc > 3 + c ? atoi(argv[3 + c]) : 0;
    if (!bwz_valid(c, a.zvar[c])) return 2;
  }
  emu_launch(n, 256, [&] { k_bsetup(a); });
  for (int st = 1; st <= nsteps; ++st) {
    for (int w = 0; w < 3; ++w) {
      if (!plan.nmap_r[w]) continue;
      a.map = plan.map.data() + plan.rmap_off[w];
      if (w == 0) emu_launch(plan.nmap_r[w], 64, [&] { k_bsweep_r<16>(a); });
      else if (w == 1) emu_launch(plan.nmap_r[w], 64, [&] { k_bsweep_r<32>(a); });
      else emu_launch(plan.nmap_r[w], 64, [&] { k_bsweep_r<64>(a); });
    }
    const int snap = st == nsteps ? 1 : 0;
    for (int c = 0; c < 4; ++c) {
      if (!plan.nmap_z[c]) continue;
      a.map = plan.map.data() + plan.zmap_off[c];
      bwz_dispatch(c, a.zvar[c], [&](auto m, auto nw) {
        constexpr int M = decltype(m)::value, NW = decltype(nw)::value;
        emu_launch(plan.nmap_z[c], 64 * NW, [&] { k_bsweep_z<M, NW>(a, snap); });
      });
    }
  }
  FILE* o = fopen(argv[2], "wb");
  if (!o) return 2;
  for (int i = 0; i < n; ++i) fwrite(T.data() + inst[i].toff, 8, (size_t)inst[i].P.nr * inst[i].P.nz, o);
  fclose(o);
  return 0;
}
