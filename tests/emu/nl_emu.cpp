// CPU emulation of the nonlinear path's persistent kernel (test
// infrastructure).  Reads a problem from argv[1] (text, see below), builds
// its geometry with the library's own device routine, runs the library's
// step-set-up and persistent kernels with every workgroup resident on a host
// thread (as the cooperative launch does), and writes to argv[2]: status,
// t, steps, rejected, solves_r, solves_z, min_margin, last solves and
// changes of the last attempt, the log rows, then the final field (nz*nr
// doubles, r fastest).
//
// Input: nr nz grid_blocks mode(0 run, 1 one attempt)
//        r0 r1 r2 rmax z0 zmax ztop
//        has_faces [nr+1 r faces, nz+1 z faces]
//        h[4] t_inf[4]  lam[20] cap[20] src[20]
//        kind t_per t_src t_trs xi zeta
//        eps iter_max tau_min div_trs div_src ptol
//        t0 t_end_or_tau max_steps log_cap
//        field (nz*nr)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hip/hip_runtime.h"
#include "device.hpp"
#include "nonlinear.hpp"

using namespace adi;
using namespace adi::nl;

static bool rd(FILE* f, double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (fscanf(f, "%lf", &x[i]) != 1) return false;
  return true;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  FILE* f = fopen(argv[1], "r");
  if (!f) return 2;
  int nr, nz, grid, mode, has_faces;
  if (fscanf(f, "%d %d %d %d", &nr, &nz, &grid, &mode) != 4) return 2;
  Params P;
  memset(&P, 0, sizeof P);
  P.nr = nr;
  P.nz = nz;
  double geo[7];
  if (!rd(f, geo, 7) || fscanf(f, "%d", &has_faces) != 1) return 2;
  P.r0 = geo[0]; P.r1 = geo[1]; P.r2 = geo[2]; P.rmax = geo[3]; P.z0 = geo[4]; P.zmax = geo[5]; P.ztop = geo[6];
  std::vector<double> rfi, zfi;
  if (has_faces) {
    rfi.resize(nr + 1);
    zfi.resize(nz + 1);
    if (!rd(f, rfi.data(), nr + 1) || !rd(f, zfi.data(), nz + 1)) return 2;
  }
  if (!rd(f, P.h, 4) || !rd(f, P.tinf, 4)) return 2;
  Laws L;
  if (!rd(f, &L.lam[0][0], 20) || !rd(f, &L.cap[0][0], 20) || !rd(f, &L.src[0][0], 20)) return 2;
  Pulse pu;
  double pp[5];
  if (fscanf(f, "%d", &pu.kind) != 1 || !rd(f, pp, 5)) return 2;
  pu.tper = pp[0]; pu.tsrc = pp[1]; pu.ttrs = pp[2]; pu.xi = pp[3]; pu.zeta = pp[4];
  double ctl6[6], run4[4];
  int iter_max;
  if (!rd(f, ctl6, 1) || fscanf(f, "%d", &iter_max) != 1 || !rd(f, ctl6 + 1, 4) || !rd(f, run4, 4)) return 2;
  const long n = (long)nr * nz;
  std::vector<double> F0(n), F1(n, 0.0), F2(n, 0.0), F3(n, 0.0), E(n, 0.0), prev(n, 0.0);
  if (!rd(f, F0.data(), (int)n)) return 2;
  fclose(f);

  // geometry with the library's routine
  std::vector<double> rf(nr + 1), rc(nr + 1), dr(nr + 1), zf(nz + 1), zc(nz + 1), dz(nz + 1);
  std::vector<uint8_t> kap(nr), bet(nz);
  std::vector<int> ranges(17);
  Geom g;
  g.rf = rf.data(); g.rc = rc.data(); g.dr = dr.data();
  g.zf = zf.data(); g.zc = zc.data(); g.dz = dz.data();
  g.kap = kap.data(); g.bet = bet.data();
  const double* rfp = has_faces ? rfi.data() : nullptr;
  const double* zfp = has_faces ? zfi.data() : nullptr;
  emu_launch(1, 64, [&]() { build_geometry(P, rfp, zfp, g, ranges.data()); });

  auto chunk = [](int len, int lanes, int& M, int& G) {
    M = std::max(3, (len + lanes - 1) / lanes);
    G = (len + M - 1) / M;
  };
  Ctl c;
  memset(&c, 0, sizeof c);
  const long long log_cap = (long long)run4[3];
  std::vector<double> log(4 * (size_t)std::max(1LL, log_cap), 0.0);
  Args a;
  memset(&a, 0, sizeof a);
  a.P = P;
  a.g = g;
  a.L = L;
  a.pulse = pu;
  a.F[0] = F0.data(); a.F[1] = F1.data(); a.F[2] = F2.data(); a.F[3] = F3.data();
  a.E = E.data();
  a.prev = prev.data();
  a.ctl = &c;
  a.log = log_cap > 0 ? log.data() : nullptr;
  a.log_cap = log_cap;
  a.eps = ctl6[0]; a.iter_max = iter_max; a.tau_min = ctl6[1]; a.div_trs = ctl6[2]; a.div_src = ctl6[3];
  a.ptol = ctl6[4];
  a.guard = 1e-9 * pu.ttrs / a.div_trs;
  const char* polls = getenv("ADI_NL_WAIT_POLLS");
  a.spin_limit = polls ? std::max(0LL, atoll(polls)) : SPIN_LIMIT;
  chunk(nr, 64 * NW, a.Mr, a.Gr);
  chunk(nz, 64, a.Mz, a.Gz);
  a.wz = 1;
  if (a.Mz > 16 || getenv("NL_EMU_WZ_BLOCK")) {
    a.wz = NW;
    chunk(nz, 64 * NW, a.Mz, a.Gz);
  }
  const size_t lds = sizeof(double) * nl_lds_doubles(a.Mr, a.Mz, a.wz);
  c.t = run4[0];
  c.min_margin = INFINITY;
  c.max_steps = (long long)run4[2];
  c.status = RUNNING;
  if (mode == 1) {
    c.t_end = INFINITY;
    c.tau = run4[1];
    c.max_steps = 1;
    a.single = 1;
    a.attempts = 1;
  } else {
    c.t_end = run4[1];
    a.single = 0;
    a.attempts = 64;
    if (a.ptol > 0.0) prev = F0;
    emu_launch(1, 64, [&]() { k_nl_begin(a); });
  }
  for (int launches = 0; launches < 100000; ++launches) {
    emu_launch_grid(grid, 64 * NW, [&]() { k_nl_run(a); }, lds);
    if (c.status != RUNNING || c.abort) break;
  }
  const double* out = a.F[c.cur];
  FILE* o = fopen(argv[2], "w");
  if (!o) return 2;
  fprintf(o, "%d %.17g %lld %lld %lld %lld %.17g %d %d %.17g %.17g %d\n", c.abort ? FAIL_WAIT : c.status, c.t,
          c.steps, c.rejected, c.solves_r, c.solves_z, c.min_margin, c.last_it[0], c.last_it[1], c.last_chg[0],
          c.last_chg[1], c.accepted);
  const long long rows = std::min(c.steps, log_cap);
  for (long long r = 0; r < rows; ++r)
    fprintf(o, "%.17g %.17g %.17g %.17g\n", log[4 * r], log[4 * r + 1], log[4 * r + 2], log[4 * r + 3]);
  for (long e = 0; e < n; ++e) fprintf(o, "%.17g\n", out[e]);
  fclose(o);
  return 0;
}
