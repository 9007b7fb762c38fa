// CPU emulation of the LDS-resident time loop (test infrastructure).  Reads
// a problem from argv[1] (text, the format of strip_emu.cpp without the
// launch shape), builds the geometry with the library's device code, forms
// the first right-hand side as the library's init kernel does, runs the
// library's resident kernel for nsteps steps in launches of at most `chunk`
// steps (the carried right-hand side passes from one launch to the next) and
// writes the final field (nz*nr doubles, r fastest) to argv[2].
#include <cstdio>
#include <vector>

#include "hip/hip_runtime.h"
#include "device.hpp"
#include "resident.hpp"

using namespace adi;

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  FILE* f = fopen(argv[1], "r");
  if (!f) return 2;
  Params P{};
  double dt, T0;
  int nsteps, scheme, chunk, ok = 1;
  ok &= fscanf(f, "%lf %lf %lf %lf %lf %lf %lf %d %d", &P.r0, &P.r1, &P.r2, &P.rmax, &P.z0, &P.zmax, &P.ztop,
               &P.nr, &P.nz) == 9;
  for (int c = 0; c < 4; ++c) ok &= fscanf(f, "%lf", &P.h[c]) == 1;
  for (int c = 0; c < 4; ++c) ok &= fscanf(f, "%lf", &P.tinf[c]) == 1;
  for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.k[c]) == 1;
  for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.rhoc[c]) == 1;
  for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.q[c]) == 1;
  ok &= fscanf(f, "%lf %d %d %d %lf", &dt, &nsteps, &scheme, &chunk, &T0) == 5;
  fclose(f);
  if (!ok || chunk < 1) return 2;
  const int nr = P.nr, nz = P.nz;
  if (!resident_shape_ok(nr, nz)) return 3;
  P.ta = scheme == 0 ? 0.5 * dt : dt;
  P.theta = scheme == 0 ? 1.0 : 0.0;
  std::vector<double> geo(3 * (nr + 1) + 3 * (nz + 1));
  std::vector<uint8_t> kap(nr), bet(nz);
  Geom g;
  g.rf = geo.data(); g.rc = g.rf + nr + 1; g.dr = g.rc + nr + 1;
  g.zf = g.dr + nr + 1; g.zc = g.zf + nz + 1; g.dz = g.zc + nz + 1;
  g.kap = kap.data(); g.bet = bet.data();
  int ranges[17];
  emu_launch(1, 64, [&] { build_geometry(P, nullptr, nullptr, g, ranges); });
  // boundary constants of each direction and class, and the first
  // right-hand side (z output operator on the start field plus b_r)
  std::vector<double> xr(3L * nr), xz(4L * nz), T((long)nr * nz, 0.0), d((long)nr * nz, 0.0);
  emu_launch(1, 64, [&] {
    if (threadIdx.x != 0) return;
    for (int c = 0; c < 3; ++c)
      for (int i = 0; i < nr; ++i) xr[(long)c * nr + i] = row_coef(P, g, 0, c, i).bconst;
    for (int c = 0; c < 4; ++c)
      for (int j = 0; j < nz; ++j) xz[(long)c * nz + j] = row_coef(P, g, 1, c, j).bconst;
    for (int j = 0; j < nz; ++j)
      for (int i = 0; i < nr; ++i)
        if (region_of(g.bet[j], g.kap[i]) != MASKED) T[(long)j * nr + i] = T0;
    for (int j = 0; j < nz; ++j)
      for (int i = 0; i < nr; ++i) {
        const long c = (long)j * nr + i;
        if (region_of(g.bet[j], g.kap[i]) == MASKED) continue;
        const RowCoef R = row_coef(P, g, 1, g.kap[i], j);
        double o = R.od * T[c] + R.oc + xr[(long)g.bet[j] * nr + i];
        if (j > 0) o += R.ol * T[c - nr];
        if (j < nz - 1) o += R.ou * T[c + nr];
        d[c] = o;
      }
  });
  bool ambient = false;
  for (int c = 0; c < 4; ++c) ambient = ambient || P.tinf[c] != 0.0;
  const size_t lds = sizeof(double) * resident_lds_doubles(nr, nz);
  for (int done = 0; done < nsteps;) {
    const int k = std::min(chunk, nsteps - done);
    ResArgs a;
    a.P = P;
    a.g = g;
    a.rhs = d.data();
    a.T = T.data();
    a.xcr = ambient ? xr.data() : nullptr;
    a.xcz = ambient ? xz.data() : nullptr;
    a.nsteps = k;
    a.write_T = done + k == nsteps;
    emu_launch(1, RES_THREADS, [&] { k_resident(a); }, lds);
    done += k;
  }
  FILE* o = fopen(argv[2], "wb");
  if (!o) return 2;
  fwrite(T.data(), 8, T.size(), o);
  fclose(o);
  return 0;
}
