// CPU emulation of the strip-layout ADI sweeps (test infrastructure).
// Reads a problem from argv[1] (text), builds geometry and line-class tables
// with the library's device code, runs the library's r and z strip kernels
// for nsteps steps from a uniform start and writes the final field (nz*nr
// doubles, r fastest) to argv[2].  The workload and launch shape come from
// the problem file; the host-side launch arguments use strip_setup, as the
// library does.
#include <cstdio>
#include <vector>

#include "hip/hip_runtime.h"
#include "device.hpp"
#include "strip.hpp"

using namespace adi;

template <int NWR, int MZ, int NWZ>
int run(Params P, double dt, int nsteps, int scheme, double T0, const char* out) {
  const int nr = P.nr, nz = P.nz;
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
  struct Dir {
    int ncls, n, G, M;
    std::vector<double> pos, chk, eng, xc, work;
    std::vector<LineTab> tabs;
  };
  Dir D[2] = {{3, nr, 64 * NWR, 4, {}, {}, {}, {}, {}, {}}, {4, nz, 64 * NWZ, MZ, {}, {}, {}, {}, {}, {}}};
  for (int d = 0; d < 2; ++d) {
    Dir& X = D[d];
    const long GM = (long)X.G * X.M;
    X.pos.assign(X.ncls * P_NFIELDS * GM, 0.0);
    X.chk.assign(X.ncls * C_NFIELDS * X.G, 0.0);
    X.eng.assign(X.ncls * 2 * X.n, 0.0);
    X.xc.assign(X.ncls * X.n, 0.0);
    X.work.assign(X.ncls * assemble_work(X.G, X.M), 0.0);
    X.tabs.resize(MAX_CLS);
    for (int c = 0; c < X.ncls; ++c) {
      double* pos = X.pos.data() + c * P_NFIELDS * GM;
      double* chk = X.chk.data() + (long)c * C_NFIELDS * X.G;
      emu_launch(1, 64, [&] {
        assemble_class(P, g, d, c, X.G, X.M, pos, chk, X.eng.data() + (long)c * 2 * X.n,
                       X.xc.data() + (long)c * X.n, X.work.data() + c * assemble_work(X.G, X.M), true);
      });
      // the run of cells outside the domain along a line of this class
      int lo = X.n, hi = X.n, cnt = 0;
      for (int p = 0; p < X.n; ++p) {
        const int m = d == 0 ? region_of(c, g.kap[p]) : region_of(g.bet[p], c);
        if (m == MASKED) {
          if (cnt == 0) lo = p;
          hi = p + 1;
          ++cnt;
        }
      }
      if (cnt != hi - lo) lo = hi = X.n;
      X.tabs[c] = {pos, chk, X.n, X.G, X.M, cnt ? lo : X.n, cnt ? hi : X.n};
    }
    for (int c = X.ncls; c < MAX_CLS; ++c) X.tabs[c] = X.tabs[0];
  }
  const long strip = strip_stride(nz);
  const long nbuf = (long)((nr + 3) / 4) * strip;
  std::vector<double> T((long)nr * nz, 0.0), dA(nbuf, 0.0), dB(nbuf, 0.0);
  for (int j = 0; j < nz; ++j)
    for (int i = 0; i < nr; ++i)
      if (region_of(g.bet[j], g.kap[i]) != MASKED) T[(long)j * nr + i] = T0;
  {  // right-hand side of the first r half step, as the library's init kernel
    Dir& Z = D[1];
    const long GM = (long)Z.G * Z.M;
    for (int j = 0; j < nz; ++j)
      for (int i = 0; i < nr; ++i) {
        const long c = (long)j * nr + i;
        const int kp = g.kap[i], bt = g.bet[j];
        if (region_of(bt, kp) == MASKED) continue;
        const double* pos = Z.pos.data() + kp * P_NFIELDS * GM;
        const long ix = (long)(j % Z.M) * Z.G + j / Z.M;
        double o = pos[pos_at(P_OD, GM, ix, true)] * T[c] + pos[pos_at(P_OC, GM, ix, true)] + D[0].xc[(long)bt * nr + i];
        if (j > 0) o += pos[pos_at(P_OL, GM, ix, true)] * T[c - nr];
        if (j < nz - 1) o += pos[pos_at(P_OU, GM, ix, true)] * T[c + nr];
        dA[(long)(i >> 2) * strip + 4L * j + (i & 3)] = o;
      }
  }
  bool ambient = false;
  for (int c = 0; c < 4; ++c) ambient = ambient || P.tinf[c] != 0.0;
  auto args = [&](int dir, const double* din, double* dout, double* xout, int* grid) {
    StripArgs a{};
    a.din = din; a.dout = dout; a.xout = xout;
    for (int c = 0; c < MAX_CLS; ++c) a.tabs[c] = D[dir].tabs[c];
    a.xc = ambient ? D[1 - dir].xc.data() : nullptr;
    a.strip = strip; a.nr = nr; a.nz = nz;
    *grid = strip_setup(a, ranges, dir, dir == 0 ? nz : nr, D[dir].ncls, D[1 - dir].ncls, P.theta);
    return a;
  };
  for (int s = 0; s < nsteps; ++s) {
    int gr, gz;
    const StripArgs a = args(0, dA.data(), dB.data(), nullptr, &gr);
    emu_launch(gr, 64 * NWR, [&] { k_sweep_rs<NWR>(a); });
    const StripArgs b = args(1, dB.data(), dA.data(), s == nsteps - 1 ? T.data() : nullptr, &gz);
    emu_launch(gz, 64 * NWZ, [&] { k_sweep_zs<MZ, NWZ>(b); });
  }
  FILE* f = fopen(out, "wb");
  if (!f) return 2;
  fwrite(T.data(), 8, T.size(), f);
  fclose(f);
  return 0;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  FILE* f = fopen(argv[1], "r");
  if (!f) return 2;
  Params P{};
  double dt, T0;
  int nsteps, scheme, nwr, mz, nwz, ok = 1;
  ok &= fscanf(f, "%lf %lf %lf %lf %lf %lf %lf %d %d", &P.r0, &P.r1, &P.r2, &P.rmax, &P.z0, &P.zmax, &P.ztop,
               &P.nr, &P.nz) == 9;
  for (int c = 0; c < 4; ++c) ok &= fscanf(f, "%lf", &P.h[c]) == 1;
  for (int c = 0; c < 4; ++c) ok &= fscanf(f, "%lf", &P.tinf[c]) == 1;
  for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.k[c]) == 1;
  for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.rhoc[c]) == 1;
  for (int c = 0; c < 5; ++c) ok &= fscanf(f, "%lf", &P.q[c]) == 1;
  ok &= fscanf(f, "%lf %d %d %d %d %d %lf", &dt, &nsteps, &scheme, &nwr, &mz, &nwz, &T0) == 7;
  fclose(f);
  if (!ok) return 2;
  if (nwr == 1 && mz == 3 && nwz == 1) return run<1, 3, 1>(P, dt, nsteps, scheme, T0, argv[2]);
  if (nwr == 1 && mz == 5 && nwz == 1) return run<1, 5, 1>(P, dt, nsteps, scheme, T0, argv[2]);
  if (nwr == 1 && mz == 5 && nwz == 2) return run<1, 5, 2>(P, dt, nsteps, scheme, T0, argv[2]);
  if (nwr == 2 && mz == 5 && nwz == 2) return run<2, 5, 2>(P, dt, nsteps, scheme, T0, argv[2]);
  fprintf(stderr, "launch shape not instantiated\n");
  return 3;
}
