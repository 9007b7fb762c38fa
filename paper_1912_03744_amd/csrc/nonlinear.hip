// nonlinear.hip -- host side of the nonlinear method path (adi_set_laws,
// adi_set_pulse, adi_set_iteration, adi_set_step_rule, adi_nl_step,
// adi_nl_run): the run state kept with a problem, the cooperative launches
// of the persistent kernel of nonlinear.hpp and the reports.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "nonlinear.hpp"
#include "problem_core.hpp"

namespace adi {
namespace nl {

// ---------------------------------------------------------------- host --

struct State {
  int device = 0;
  long n = 0;
  double* buf = nullptr;     // F[1..3], E, prev: 5 fields
  Ctl* ctl = nullptr;
  double* dlog = nullptr;
  long long log_cap = 0;
  Laws laws{};
  bool has_laws = false;
  Pulse pulse{0, 0.1, 0.01, 1e-4, 4.0, 2.0};
  double eps = 1e-6, tau_min = 1e-12, ptol = 0.0, div_trs = 1000.0, div_src = 100.0;
  int iter_max = 10;
  int grid = 0;
  size_t lds = 0;
  int Mr = 0, Gr = 0, Mz = 0, Gz = 0, wz = 1;
};

void destroy_state(void* v) {
  State* s = (State*)v;
  if (!s) return;
  dev_free(s->buf);
  dev_free(s->ctl);
  dev_free(s->dlog);
  delete s;
}

// Chunks of a line of n cells over `lanes` lanes: M cells each (at least 3),
// G chunks.
void chunking(int n, int lanes, int& M, int& G) {
  M = std::max(MIN_M, (n + lanes - 1) / lanes);
  G = (n + M - 1) / M;
}

adi_status get_state(adi_problem p, ProblemCore& core, State** out) {
  ADI_TRY(problem_core(p, &core));
  State* s = (State*)problem_ext(p);
  if (!s) {
    const int nr = core.P.nr, nz = core.P.nz;
    // r lines: a workgroup of NW waves each; z lines: one wave each, or a
    // workgroup when the line is long
    int Mr, Gr, Mz, Gz, wz = 1;
    chunking(nr, 64 * NW, Mr, Gr);
    chunking(nz, 64, Mz, Gz);
    if (Mz > 16) {
      wz = NW;
      chunking(nz, 64 * NW, Mz, Gz);
    }
    if (Mr > MAX_M || Mz > MAX_M)
      return fail(ADI_EUNSUPPORTED, "the nonlinear path takes lines of at most %d cells (grid %d x %d)", 64 * MAX_M, nr,
                  nz);
    if ((long)nr * nz >= (1L << 28))
      return fail(ADI_EUNSUPPORTED, "the nonlinear path takes fields of fewer than 2^28 cells (32-bit byte offsets)");
    s = new (std::nothrow) State();
    if (!s) return fail(ADI_ENOMEM, "host allocation failed");
    s->device = core.device;
    s->n = (long)nr * nz;
    s->Mr = Mr; s->Gr = Gr; s->Mz = Mz; s->Gz = Gz; s->wz = wz;
    adi_status st = dev_alloc((void**)&s->buf, sizeof(double) * 5 * s->n, core.stream);
    if (st == ADI_OK) st = dev_alloc((void**)&s->ctl, sizeof(Ctl), core.stream);
    if (st != ADI_OK) {
      destroy_state(s);
      return st;
    }
    s->lds = sizeof(double) * nl_lds_doubles(Mr, Mz, wz);
    hipError_t e = hipFuncSetAttribute((const void*)k_nl_run, hipFuncAttributeMaxDynamicSharedMemorySize, (int)s->lds);
    int per_cu = 0, cus = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_nl_run, 64 * NW, s->lds);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, core.device);
    if (e != hipSuccess || per_cu < 1) {
      destroy_state(s);
      return fail(ADI_EDEVICE, "occupancy of the nonlinear kernel: %s (%d per CU)", hipGetErrorString(e), per_cu);
    }
    // every workgroup resident (cooperative launch); no more workgroups than
    // the lines need
    s->grid = std::min(per_cu * cus, std::max(nz, wz == 1 ? (nr + NW - 1) / NW : nr));
    problem_set_ext(p, s, destroy_state);
  }
  *out = s;
  return ADI_OK;
}

Args make_args(const ProblemCore& core, const State* s) {
  Args a{};
  a.P = core.P;
  a.g = core.g;
  a.L = s->laws;
  a.pulse = s->pulse;
  a.F[0] = core.T;
  for (int q = 1; q < 4; ++q) a.F[q] = s->buf + (long)(q - 1) * s->n;
  a.E = s->buf + 3 * s->n;
  a.prev = s->buf + 4 * s->n;
  a.ctl = s->ctl;
  a.eps = s->eps;
  a.tau_min = s->tau_min;
  a.ptol = s->ptol;
  a.div_trs = s->div_trs;
  a.div_src = s->div_src;
  a.guard = 1e-9 * s->pulse.ttrs / s->div_trs;
  a.iter_max = s->iter_max;
  a.Mr = s->Mr; a.Gr = s->Gr; a.Mz = s->Mz; a.Gz = s->Gz; a.wz = s->wz;
  // ADI_NL_WAIT_POLLS lowers the bound of every grid-wide wait, so that the
  // abort path can be exercised from the host (every wave still exits).
  const char* polls = getenv("ADI_NL_WAIT_POLLS");
  a.spin_limit = polls ? std::max(0LL, atoll(polls)) : SPIN_LIMIT;
  return a;
}

adi_status launch_run(const ProblemCore& core, const State* s, Args& a) {
  void* args[] = {&a};
  ADI_HIP(hipLaunchCooperativeKernel((const void*)k_nl_run, dim3(s->grid), dim3(64 * NW), args, (unsigned)s->lds,
                                     core.stream));
  return ADI_OK;
}

// After a run: the field back in F[0] (the problem's own buffer).
adi_status settle(const ProblemCore& core, const State* s, const Ctl& h) {
  if (h.cur != 0) {
    const double* src = s->buf + (long)(h.cur - 1) * s->n;
    hipLaunchKernelGGL(k_nl_copy, dim3((int)std::min<long>((s->n + 255) / 256, 4096)), dim3(256), 0, core.stream, src,
                       core.T, s->n);
    ADI_CHECK_LAUNCH();
  }
  ADI_HIP(hipStreamSynchronize(core.stream));
  return ADI_OK;
}

adi_status read_ctl(const ProblemCore& core, const State* s, Ctl* h) {
  ADI_HIP(hipMemcpyAsync(h, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, core.stream));
  ADI_HIP(hipStreamSynchronize(core.stream));
  return ADI_OK;
}

adi_status start_ctl(const ProblemCore& core, const State* s, double t, double t_end, double tau, long long max_steps) {
  Ctl h;
  std::memset(&h, 0, sizeof h);
  h.t = t;
  h.t_end = t_end;
  h.tau = tau;
  h.min_margin = INFINITY;
  h.max_steps = max_steps;
  h.cur = 0;
  h.status = RUNNING;
  ADI_HIP(hipMemcpyAsync(s->ctl, &h, sizeof h, hipMemcpyHostToDevice, core.stream));
  return ADI_OK;
}

adi_status check_ready(const State* s) {
  if (!s->has_laws) return fail(ADI_ESTATE, "adi_set_laws must be called before a nonlinear step");
  return ADI_OK;
}

}  // namespace nl
}  // namespace adi

using namespace adi;
using namespace adi::nl;

extern "C" {

adi_status adi_set_laws(adi_problem p, const double lam[20], const double cap[20], const double src[20]) {
  ProblemCore core;
  State* s;
  ADI_TRY(get_state(p, core, &s));
  if (!lam || !cap || !src) return fail(ADI_EINVAL, "null law array");
  for (int q = 0; q < 20; ++q)
    if (!is_fin(lam[q]) || !is_fin(cap[q]) || !is_fin(src[q]))
      return fail(ADI_ENONFINITE, "law coefficient %d is not finite", q);
  for (int m = 0; m < 5; ++m)
    for (int q = 0; q < 4; ++q) {
      s->laws.lam[m][q] = lam[4 * m + q];
      s->laws.cap[m][q] = cap[4 * m + q];
      s->laws.src[m][q] = src[4 * m + q];
    }
  s->has_laws = true;
  return ADI_OK;
}

adi_status adi_set_pulse(adi_problem p, int32_t kind, const double params[5]) {
  ProblemCore core;
  State* s;
  ADI_TRY(get_state(p, core, &s));
  if (kind < 0 || kind > 2) return fail(ADI_EINVAL, "pulse kind must be 0, 1 or 2");
  if (!params) {
    if (kind != 0) return fail(ADI_EINVAL, "null pulse parameters");
    s->pulse.kind = 0;
    return ADI_OK;
  }
  const double tper = params[0], tsrc = params[1], ttrs = params[2];
  if (!(tsrc > 0.0) || !is_fin(tsrc) || !(ttrs > 0.0) || !is_fin(ttrs))
    return fail(ADI_EINVAL, "t_src and t_trs must be > 0 and finite");
  if (kind != 0 && (!(tper > 0.0) || !is_fin(tper) || !(tsrc <= tper) || !(tsrc + ttrs <= tper) ||
                    !(ttrs <= tsrc) || !is_fin(params[3]) || !is_fin(params[4]) || !(params[4] > 0.0)))
    return fail(ADI_EINVAL, "pulse needs 0 < t_trs <= t_src, t_src + t_trs <= t_per, finite xi and zeta > 0");
  s->pulse = Pulse{kind, params[0], params[1], params[2], params[3], params[4]};
  return ADI_OK;
}

adi_status adi_set_iteration(adi_problem p, double eps, int32_t iter_max, double tau_min) {
  ProblemCore core;
  State* s;
  ADI_TRY(get_state(p, core, &s));
  if (!(eps > 0.0) || !is_fin(eps)) return fail(ADI_EINVAL, "eps must be > 0 and finite");
  if (iter_max < 1 || iter_max > ITER_CAP) return fail(ADI_EINVAL, "iter_max must be in [1, %d]", ITER_CAP);
  if (!(tau_min > 0.0) || !is_fin(tau_min)) return fail(ADI_EINVAL, "tau_min must be > 0 and finite");
  s->eps = eps;
  s->iter_max = iter_max;
  s->tau_min = tau_min;
  return ADI_OK;
}

adi_status adi_set_step_rule(adi_problem p, double tau_trs_div, double tau_src_div, double periodic_tol) {
  ProblemCore core;
  State* s;
  ADI_TRY(get_state(p, core, &s));
  if (!(tau_trs_div >= 1.0) || !is_fin(tau_trs_div) || !(tau_src_div >= 1.0) || !is_fin(tau_src_div))
    return fail(ADI_EINVAL, "step divisors must be >= 1 and finite");
  if (!(periodic_tol >= 0.0) || !is_fin(periodic_tol)) return fail(ADI_EINVAL, "periodic tolerance must be >= 0");
  s->div_trs = tau_trs_div;
  s->div_src = tau_src_div;
  s->ptol = periodic_tol;
  return ADI_OK;
}

adi_status adi_nl_step(adi_problem p, double tau, int32_t* accepted, int32_t solves[2], double changes[2]) {
  ProblemCore core;
  State* s;
  ADI_TRY(get_state(p, core, &s));
  ADI_TRY(check_ready(s));
  if (!(tau > 0.0) || !is_fin(tau)) return fail(ADI_EINVAL, "tau must be > 0 and finite");
  ADI_TRY(start_ctl(core, s, core.time, INFINITY, tau, 1));
  Args a = make_args(core, s);
  a.single = 1;
  a.attempts = 1;
  ADI_TRY(launch_run(core, s, a));
  Ctl h;
  ADI_TRY(read_ctl(core, s, &h));
  if (h.status == FAIL_WAIT || h.abort) return fail(ADI_EDEVICE, "a grid-wide wait of the nonlinear kernel ran out");
  ADI_TRY(settle(core, s, h));
  if (accepted) *accepted = h.accepted;
  if (solves) {
    solves[0] = h.last_it[0];
    solves[1] = h.last_it[1];
  }
  if (changes) {
    changes[0] = h.last_chg[0];
    changes[1] = h.last_chg[1];
  }
  if (h.accepted) problem_field_advanced(p, h.t, 1);
  return ADI_OK;
}

adi_status adi_nl_run(adi_problem p, double t_end, int64_t max_steps, double* host_log, int64_t log_cap,
                      adi_nl_report* out) {
  ProblemCore core;
  State* s;
  ADI_TRY(get_state(p, core, &s));
  ADI_TRY(check_ready(s));
  if (!is_fin(t_end)) return fail(ADI_EINVAL, "t_end must be finite");
  if (max_steps < 0) return fail(ADI_EINVAL, "max_steps must be >= 0");
  if (log_cap < 0 || (log_cap > 0 && !host_log)) return fail(ADI_EINVAL, "log needs a host buffer of log_cap rows");
  if (log_cap > s->log_cap) {
    dev_free(s->dlog);
    s->dlog = nullptr;
    s->log_cap = 0;
    ADI_TRY(dev_alloc((void**)&s->dlog, sizeof(double) * 4 * log_cap, core.stream));
    s->log_cap = log_cap;
  }
  ADI_TRY(start_ctl(core, s, core.time, t_end, 0.0, max_steps));
  Args a = make_args(core, s);
  a.log = log_cap > 0 ? s->dlog : nullptr;
  a.log_cap = log_cap;
  a.single = 0;
  a.attempts = 4096;
  const long n = s->n;
  if (s->ptol > 0.0) {
    hipLaunchKernelGGL(k_nl_copy, dim3((int)std::min<long>((n + 255) / 256, 4096)), dim3(256), 0, core.stream, core.T,
                       a.prev, n);
    ADI_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_nl_begin, dim3(1), dim3(64), 0, core.stream, a);
  ADI_CHECK_LAUNCH();
  Ctl h;
  for (;;) {
    ADI_TRY(launch_run(core, s, a));
    ADI_TRY(read_ctl(core, s, &h));
    if (h.status != RUNNING || h.abort) break;
  }
  if (h.status == FAIL_WAIT || h.abort) return fail(ADI_EDEVICE, "a grid-wide wait of the nonlinear kernel ran out");
  ADI_TRY(settle(core, s, h));
  if (h.steps > 0) problem_field_advanced(p, h.t, h.steps);
  if (log_cap > 0) {
    const long rows = (long)std::min<long long>(h.steps, log_cap);
    if (rows > 0) ADI_HIP(hipMemcpy(host_log, s->dlog, sizeof(double) * 4 * rows, hipMemcpyDeviceToHost));
  }
  if (out) {
    out->t = h.t;
    out->steps = h.steps;
    out->rejected = h.rejected;
    out->solves_r = h.solves_r;
    out->solves_z = h.solves_z;
    out->periodic = h.status == END_PERIODIC;
    out->min_margin = h.min_margin;
  }
  if (h.status == FAIL_TAU) return fail(ADI_EINVAL, "step halving went below tau_min at t = %.17g", h.t);
  return ADI_OK;
}

}  // extern "C"
