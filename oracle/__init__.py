"""CPU FP64 oracle for the axisymmetric ADI heat solver (arXiv 1912.03744).

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or calls
anything in this package; only the test suite, the smoke check and the
CPU-baseline leg of the benchmark do.  The oracle shares no code with the HIP
implementation: the solver lives in ``adi_oracle.c`` (plain C, FP64, Thomas per
line, Sec. 3 eq. 7-11 and the Thomas solve at the end of Sec. 3), the network
in ``mlp.py`` (numpy FP64).

This module is the ctypes glue for ``adi_oracle.c``: argument marshalling only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adi_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_LIB = None

MASKED = 255

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile ``adi_oracle.c`` into ``liboracle.so`` with gcc (FP64, no FMA
    contraction; OpenMP only for the threaded timing entry point)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp",
             "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_SO)
        lib.or_create.restype = ctypes.c_void_p
        lib.or_create.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
                                  _dp, _dp, _dp]
        lib.or_free.argtypes = [ctypes.c_void_p]
        lib.or_grid.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        lib.or_region_map.argtypes = [ctypes.c_void_p, _u8p]
        lib.or_coeffs.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        lib.or_apply.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        lib.or_thomas.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.or_step.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                ctypes.c_long, _dp, _dp]
        lib.or_step_omp.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_long, _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        lib.or_energy.argtypes = [ctypes.c_void_p, _dp, _dp]
        lib.or_profile.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int, ctypes.c_int, _dp]
        lib.or_nl_set_laws.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        lib.or_nl_apply.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        lib.or_pulse.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
        lib.or_pulse.restype = ctypes.c_double
        lib.or_nl_step.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                   _dp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp]
        _lp = ctypes.POINTER(ctypes.c_long)
        lib.or_nl_run.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp,
                                  ctypes.c_int, ctypes.c_long, _lp, _dp, ctypes.c_long, _dp]
        for f in ("or_coeffs", "or_step", "or_step_omp", "or_profile", "or_nl_step", "or_nl_run"):
            getattr(lib, f).restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


_COEFF = {"Lr_w": 0, "Lr_c": 1, "Lr_e": 2, "br": 3, "Lz_s": 4, "Lz_c": 5,
          "Lz_n": 6, "bz": 7, "C": 8, "Q": 9, "V": 10, "Bw_r": 11, "Bt_r": 12,
          "Bw_z": 13, "Bt_z": 14}

SCHEMES = {"pr": 0, "lod": 1}


def thomas(a, b, c, d):
    """Solve one tridiagonal system with the oracle's Thomas routine."""
    a, b, c, d = (_f64(v) for v in (a, b, c, d))
    n = b.size
    x, cp, dp = np.empty(n), np.empty(n), np.empty(n)
    _lib().or_thomas(n, _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(x), _ptr(cp), _ptr(dp))
    return x


class Problem:
    """One assembled problem on the oracle side.

    geom: (r0, r1, r2, rmax, z0, zmax, ztop); bc: (h[0..3], t_inf[0..3]);
    k, rhoc, q: five values each, regions 0 cooler .. 4 terminal.
    """

    def __init__(self, geom, nr, nz, h, t_inf, k, rhoc, q, r_faces=None, z_faces=None):
        self.nr, self.nz = int(nr), int(nz)
        self._keep = [_f64(geom, 7), _f64(list(h) + list(t_inf), 8), _f64(k, 5),
                      _f64(rhoc, 5), _f64(q, 5),
                      None if r_faces is None else _f64(r_faces, self.nr + 1),
                      None if z_faces is None else _f64(z_faces, self.nz + 1)]
        g, bc, kk, rc, qq, rf, zf = self._keep
        self._h = _lib().or_create(_ptr(g), self.nr, self.nz, _ptr(rf), _ptr(zf),
                                   _ptr(bc), _ptr(kk), _ptr(rc), _ptr(qq))
        if not self._h:
            raise ValueError("oracle rejected the problem")

    @classmethod
    def from_spec(cls, s):
        """Build from any object with the workload-spec attributes."""
        return cls((s.r0, s.r1, s.r2, s.rmax, s.z0, s.zmax, s.ztop), s.nr, s.nz,
                   s.h, s.t_inf, s.k, s.rhoc, s.q,
                   getattr(s, "r_faces", None), getattr(s, "z_faces", None))

    def __del__(self):
        if getattr(self, "_h", None):
            _lib().or_free(self._h)
            self._h = None

    @property
    def shape(self):
        return (self.nz, self.nr)

    def grid(self):
        rf, zf = np.empty(self.nr + 1), np.empty(self.nz + 1)
        rc, zc = np.empty(self.nr), np.empty(self.nz)
        _lib().or_grid(self._h, _ptr(rf), _ptr(zf), _ptr(rc), _ptr(zc))
        return rf, zf, rc, zc

    def region_map(self):
        out = np.empty(self.shape, dtype=np.uint8)
        _lib().or_region_map(self._h, out.ctypes.data_as(_u8p))
        return out

    def active(self):
        return self.region_map() != MASKED

    def coeffs(self, name):
        out = np.empty(self.shape)
        if _lib().or_coeffs(self._h, _COEFF[name], _ptr(out)) != 0:
            raise ValueError(name)
        return out

    def apply(self, T):
        """Return (A_r T, A_z T) with boundary constants included."""
        T = _f64(T, self.nr * self.nz)
        ar, az = np.empty(self.shape), np.empty(self.shape)
        _lib().or_apply(self._h, _ptr(T), _ptr(ar), _ptr(az))
        return ar, az

    def step(self, T, scheme, dt, nsteps):
        """Advance a copy of T; returns (T_new, T_half_of_last_step)."""
        T = _f64(T, self.nr * self.nz).reshape(self.shape).copy()
        mid = np.zeros(self.shape)
        rc = _lib().or_step(self._h, SCHEMES[scheme], float(dt), int(nsteps), _ptr(T), _ptr(mid))
        if rc != 0:
            raise ValueError("or_step failed: %d" % rc)
        return T, mid

    def step_threads(self, T, scheme, dt, nsteps, threads):
        """The same steps with the line solves of each half step shared among
        `threads` OpenMP threads (the paper's CPU parallelisation); the result
        is bit-identical to step().  Returns (T_new, threads that ran)."""
        T = _f64(T, self.nr * self.nz).reshape(self.shape).copy()
        used = ctypes.c_int(0)
        rc = _lib().or_step_omp(self._h, SCHEMES[scheme], float(dt), int(nsteps), _ptr(T),
                                int(threads), ctypes.byref(used))
        if rc != 0:
            raise ValueError("or_step_omp failed: %d" % rc)
        return T, used.value

    def energy(self, T):
        T = _f64(T, self.nr * self.nz)
        out = np.empty(4)
        _lib().or_energy(self._h, _ptr(T), _ptr(out))
        return {"E": out[0], "Br": out[1], "Bz": out[2], "P": out[3]}

    def profile(self, T, which=0, npts=64):
        T = _f64(T, self.nr * self.nz)
        out = np.empty(npts)
        if _lib().or_profile(self._h, _ptr(T), int(which), int(npts), _ptr(out)) != 0:
            raise ValueError("profile row has masked cells")
        return out

    def initial(self, T0):
        """Uniform field T0 on active cells, 0 on masked cells."""
        return np.where(self.active(), float(T0), 0.0)


# ------------------------------------------------------------ nonlinear --
# The simple (Picard) iteration of eq. 12-14, the pulsed source of eq. 2-4
# and the adaptive step of Sec. 3-4 (adi_oracle.c, section "Nonlinear path").

PULSES = {"const": 0, "rect": 1, "erf": 2}


def pulse(kind, t, t_per=0.1, t_src=0.01, t_trs=1e-4, xi=4.0, zeta=2.0):
    """Normalised source p(t): 'const' (1), 'rect' (eq. 3) or 'erf' (eq. 4)."""
    pp = _f64([t_per, t_src, t_trs, xi, zeta], 5)
    return _lib().or_pulse(PULSES[kind], float(t), _ptr(pp))


class NonlinearProblem(Problem):
    """A problem with temperature-dependent laws: lam, cap, src are 5 x 4
    polynomial coefficients (region-major, c0 + c1 T + c2 T^2 + c3 T^3) of
    the conductivity, the volumetric heat capacity and the source amplitude."""

    def set_laws(self, lam, cap, src):
        self._laws = [_f64(lam, 20), _f64(cap, 20), _f64(src, 20)]
        _lib().or_nl_set_laws(self._h, *(_ptr(a) for a in self._laws))

    def set_constant_laws(self, k, rhoc, q):
        """Laws equal to the linear problem's constants."""
        z = np.zeros((5, 3))
        self.set_laws(np.column_stack([k, z]), np.column_stack([rhoc, z]), np.column_stack([q, z]))

    def nl_apply(self, F, T):
        """(A_r T, A_z T) with the laws evaluated on the field F."""
        F = _f64(F, self.nr * self.nz)
        T = _f64(T, self.nr * self.nz)
        ar, az = np.empty(self.shape), np.empty(self.shape)
        _lib().or_nl_apply(self._h, _ptr(F), _ptr(T), _ptr(ar), _ptr(az))
        return ar, az

    def nl_step(self, T, tau, t, kind="const", pulse_args=(0.1, 0.01, 1e-4, 4.0, 2.0), eps=1e-10,
                iter_max=10):
        """One step by eq. 12 and 14.  Returns (accepted, T_new, solves,
        last_changes); T_new is T itself when the step failed."""
        T = _f64(T, self.nr * self.nz).reshape(self.shape).copy()
        pp = _f64(pulse_args, 5)
        it = (ctypes.c_int * 2)()
        chg = np.zeros(2)
        ok = _lib().or_nl_step(self._h, _ptr(T), float(tau), float(t), PULSES[kind], _ptr(pp), float(eps),
                               int(iter_max), it, _ptr(chg))
        if ok < 0:
            raise MemoryError("or_nl_step")
        return bool(ok), T, (it[0], it[1]), chg

    def nl_run(self, T, t0, t_end, kind="erf", pulse_args=(0.1, 0.01, 1e-4, 4.0, 2.0), eps=1e-6,
               iter_max=10, tau_min=1e-12, periodic_tol=0.0, tau_trs_div=1000.0, tau_src_div=100.0,
               max_steps=1 << 40, log_cap=0):
        """The adaptive loop of Sec. 4.  Returns a dict with the field, the
        final time, the counts and (log_cap > 0) the per-step log rows
        (t_before, tau, solves_r, solves_z)."""
        T = _f64(T, self.nr * self.nz).reshape(self.shape).copy()
        pp = _f64(pulse_args, 5)
        ctl = _f64([eps, tau_min, periodic_tol, tau_trs_div, tau_src_div], 5)
        t = np.array([float(t0)])
        counts = (ctypes.c_long * 5)()
        log = np.zeros((max(log_cap, 1), 4))
        margin = np.zeros(1)
        rc = _lib().or_nl_run(self._h, _ptr(T), _ptr(t), float(t_end), PULSES[kind], _ptr(pp), _ptr(ctl),
                              int(iter_max), int(max_steps), counts, _ptr(log) if log_cap else None,
                              int(log_cap), _ptr(margin))
        if rc != 0:
            raise ValueError("or_nl_run failed: %d" % rc)
        steps = counts[0]
        return {"T": T, "t": float(t[0]), "steps": steps, "rejected": counts[1], "solves_r": counts[2],
                "solves_z": counts[3], "periodic": bool(counts[4]), "min_margin": float(margin[0]),
                "log": log[:min(steps, log_cap)] if log_cap else None}
