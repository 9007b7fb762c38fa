"""ctypes binding of libadi.so (include/adi.h): argument marshalling only.

Every step of the method runs in the HIP kernels of the library; this module
converts Python values to the C ABI and raises on error codes.  The library
must have been built (``python -m paper_1912_03744_amd.build``); loading
fails loudly otherwise.  torch is imported first so that the library binds
to the HIP runtime torch already uses (one runtime per process, so torch
streams and device pointers can be passed in).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # torch provides device memory and streams to callers; load its HIP runtime first
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadi.so")

ADI_OK, ADI_EINVAL, ADI_ENOMEM, ADI_EDEVICE, ADI_ESTATE = 0, -1, -2, -3, -4
ADI_ENONFINITE, ADI_EBALANCE, ADI_EUNSUPPORTED = -5, -6, -7
SCHEMES = {"pr": 0, "lod": 1}
LAYOUTS = {"rows": 0, "strips": 1, "resident": 2}


class AdiError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (%d): %s" % (_STATUS.get(status, "?"), status, message))
        self.status = status


_STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "ENONFINITE",
           -6: "EBALANCE", -7: "EUNSUPPORTED"}


class Geometry(ctypes.Structure):
    _fields_ = [("r0", ctypes.c_double), ("r1", ctypes.c_double), ("r2", ctypes.c_double),
                ("rmax", ctypes.c_double), ("z0", ctypes.c_double), ("zmax", ctypes.c_double),
                ("ztop", ctypes.c_double), ("nr", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("r_faces", ctypes.POINTER(ctypes.c_double)),
                ("z_faces", ctypes.POINTER(ctypes.c_double))]


class BC(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double * 4), ("t_inf", ctypes.c_double * 4)]


class NlReport(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("steps", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("solves_r", ctypes.c_int64), ("solves_z", ctypes.c_int64), ("periodic", ctypes.c_int32),
                ("min_margin", ctypes.c_double)]


class EnergyReport(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("E0", ctypes.c_double), ("source_power", ctypes.c_double),
                ("boundary_flow", ctypes.c_double), ("residual", ctypes.c_double),
                ("time", ctypes.c_double), ("steps", ctypes.c_int64), ("checks", ctypes.c_int64)]


_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p

# name -> argtypes (restype adi_status = int unless listed otherwise)
# device-memory hook of adi_set_allocator
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_SIGS = {
    "adi_set_allocator": [ALLOC_FN, FREE_FN, ctypes.c_void_p],
    "adi_create_problem": [ctypes.POINTER(Geometry), ctypes.POINTER(BC), ctypes.c_int, _vp,
                           ctypes.POINTER(_vp)],
    "adi_set_materials": [_vp, _dp, _dp],
    "adi_set_sources": [_vp, _dp],
    "adi_set_field": [_vp, _dp, ctypes.c_double],
    "adi_step": [_vp, ctypes.c_double, ctypes.c_int64],
    "adi_set_check": [_vp, ctypes.c_int32, ctypes.c_double],
    "adi_read_field": [_vp, _dp, ctypes.c_size_t],
    "adi_read_field_device": [_vp, _vp],
    "adi_read_region_map": [_vp, ctypes.POINTER(ctypes.c_uint8), ctypes.c_size_t],
    "adi_read_profile": [_vp, ctypes.c_int32, ctypes.c_int32, _dp],
    "adi_energy": [_vp, ctypes.POINTER(EnergyReport)],
    "adi_time_sweeps": [_vp, ctypes.c_double, ctypes.c_int32, _fp, _fp],
    "adi_set_launch": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                       ctypes.c_int32, ctypes.c_int32],
    "adi_get_launch": [_vp, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p],
    "adi_set_graph_steps": [_vp, ctypes.c_int32],
    "adi_launch_shapes": [_i32p, ctypes.c_int32, _i32p],
    "adi_layout_shapes": [ctypes.c_int32, ctypes.c_int32, _i32p, ctypes.c_int32, _i32p],
    "adi_set_layout": [_vp, ctypes.c_int32],
    "adi_sync": [_vp],
    "adi_set_laws": [_vp, _dp, _dp, _dp],
    "adi_set_pulse": [_vp, ctypes.c_int32, _dp],
    "adi_set_iteration": [_vp, ctypes.c_double, ctypes.c_int32, ctypes.c_double],
    "adi_set_step_rule": [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "adi_nl_step": [_vp, ctypes.c_double, _i32p, _i32p, _dp],
    "adi_nl_run": [_vp, ctypes.c_double, ctypes.c_int64, _dp, ctypes.c_int64, ctypes.POINTER(NlReport)],
    "adi_mlp_sync": [_vp],
    "adi_get_layout": [_vp, _i32p],
    "adi_destroy": [_vp],
    "adi_create_batch": [ctypes.c_int32, ctypes.POINTER(Geometry), ctypes.POINTER(BC), ctypes.c_int,
                         _vp, ctypes.POINTER(_vp)],
    "adi_batch_set_materials": [_vp, _dp, _dp, _dp],
    "adi_batch_set_initial": [_vp, _dp],
    "adi_batch_set_launch": [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
    "adi_batch_zshape_info": [ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p],
    "adi_batch_set_zshape": [_vp, ctypes.c_int32, ctypes.c_int32],
    "adi_batch_step": [_vp, ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _vp],
    "adi_batch_sync": [_vp],
    "adi_batch_read_profiles": [_vp, ctypes.c_int32, _dp, ctypes.c_size_t],
    "adi_batch_read_field": [_vp, ctypes.c_int32, _dp, ctypes.c_size_t],
    "adi_batch_info": [_vp, ctypes.POINTER(ctypes.c_int64), _i32p, _i32p],
    "adi_batch_active_cells": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "adi_batch_time": [_vp, ctypes.c_double, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)],
    "adi_batch_destroy": [_vp],
    "adi_mlp_create": [_i32p, ctypes.c_int32, ctypes.c_uint64, _vp, ctypes.POINTER(_vp)],
    "adi_mlp_num_params": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "adi_mlp_set_scaling": [_vp, _fp, _fp],
    "adi_mlp_get_params": [_vp, _fp, ctypes.c_int64],
    "adi_mlp_set_params": [_vp, _fp, ctypes.c_int64],
    "adi_mlp_forward": [_vp, _vp, ctypes.c_int64, _vp],
    "adi_mlp_forward_noalloc": [_vp, _vp, ctypes.c_int64, _vp],
    "adi_mlp_gradients": [_vp, _vp, _vp, ctypes.c_int64, _fp, _fp],
    "adi_mlp_train_step": [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_float, _fp],
    "adi_mlp_destroy": [_vp],
    "adi_screen_profiles": [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, _vp, _vp, _vp, _vp, _vp],
    "adi_top_k": [_vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp],
    "adi_status_string": [ctypes.c_int],
    "adi_last_error": [],
    "adi_version": [],
}
_RESTYPE = {"adi_destroy": None, "adi_batch_destroy": None, "adi_mlp_destroy": None, "adi_status_string": ctypes.c_char_p,
            "adi_last_error": ctypes.c_char_p, "adi_version": ctypes.c_char_p}

_LIB = None
_HOOKS = []  # every installed allocator callback: blocks keep their free function


def lib():
    """Load libadi.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libadi.so is not built: run `python -m paper_1912_03744_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _RESTYPE.get(name, ctypes.c_int)
        _LIB = L
    return _LIB


def set_allocator(alloc=None, free=None):
    """Route the library's device allocations through alloc(nbytes) -> device
    pointer (int; 0 when out of memory) and free(ptr) (adi_set_allocator);
    set_allocator() restores hipMalloc / hipFree.  Blocks allocated under a
    hook go back to that hook's free function whenever they are released."""
    if (alloc is None) != (free is None):
        raise ValueError("give both alloc and free, or neither")
    if alloc is None:
        check(lib().adi_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return
    a = ALLOC_FN(lambda nbytes, ctx: int(alloc(int(nbytes))) or None)
    f = FREE_FN(lambda ptr, ctx: free(int(ptr)))
    _HOOKS.append((a, f))
    check(lib().adi_set_allocator(a, f, None))


def use_torch_allocator():
    """Take the library's device memory from PyTorch's caching allocator
    (blocks on the current device, tied to torch's current stream)."""
    import torch
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n), torch.cuda.caching_allocator_delete)


def exported_symbols():
    return list(_SIGS)


def check(status):
    if status != ADI_OK:
        raise AdiError(status, lib().adi_last_error().decode())
    return status


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _torch_stream_sync():
    torch.cuda.current_stream().synchronize()


def current_stream():
    """The current torch stream as a hipStream_t, or None (the library then
    uses a stream of its own) when torch has no GPU or is on its default
    stream, which cannot be captured into a graph."""
    if torch is not None and torch.cuda.is_available():
        s = torch.cuda.current_stream().cuda_stream
        return ctypes.c_void_p(s) if s else None
    return None


class Problem:
    """One single-instance problem on the GPU (adi_create_problem ...)."""

    def __init__(self, geom, nr, nz, h, t_inf, scheme="pr", r_faces=None, z_faces=None, stream=None):
        r0, r1, r2, rmax, z0, zmax, ztop = (float(x) for x in geom)
        self.nr, self.nz = int(nr), int(nz)
        self._rf = None if r_faces is None else _f64(r_faces, self.nr + 1)
        self._zf = None if z_faces is None else _f64(z_faces, self.nz + 1)
        g = Geometry(r0, r1, r2, rmax, z0, zmax, ztop, self.nr, self.nz,
                     _ptr(self._rf), _ptr(self._zf))
        bc = BC((ctypes.c_double * 4)(*[float(x) for x in h]),
                (ctypes.c_double * 4)(*[float(x) for x in t_inf]))
        h_ = _vp()
        st = stream if stream is not None else current_stream()
        check(lib().adi_create_problem(ctypes.byref(g), ctypes.byref(bc), SCHEMES[scheme], st,
                                       ctypes.byref(h_)))
        self._h = h_
        # on a stream of its own the library is not ordered with torch's work
        self._own_stream = st is None
        self._destroy = lib().adi_destroy
        self.scheme = scheme

    @classmethod
    def from_spec(cls, s, stream=None):
        p = cls(s.geom, s.nr, s.nz, s.h, s.t_inf, s.scheme, s.r_faces, s.z_faces, stream)
        p.set_materials(s.k, s.rhoc)
        p.set_sources(s.q)
        p.set_field(None, s.T0)
        return p

    def close(self):
        # the destroy function is looked up while the module is alive: at
        # interpreter shutdown module globals may already be gone
        h, destroy = getattr(self, "_h", None), getattr(self, "_destroy", None)
        if h and destroy is not None:
            destroy(h)
        self._h = None

    __del__ = close

    @property
    def shape(self):
        return (self.nz, self.nr)

    def set_materials(self, k, rhoc):
        check(lib().adi_set_materials(self._h, _ptr(_f64(k, 5)), _ptr(_f64(rhoc, 5))))

    def set_sources(self, q):
        check(lib().adi_set_sources(self._h, _ptr(_f64(q, 5))))

    def set_field(self, T=None, T0=0.0):
        a = None if T is None else _f64(T, self.nr * self.nz)
        check(lib().adi_set_field(self._h, _ptr(a), float(T0)))

    def step(self, dt, nsteps):
        check(lib().adi_step(self._h, float(dt), int(nsteps)))

    def set_check(self, every, tol=1e-9):
        check(lib().adi_set_check(self._h, int(every), float(tol)))

    def set_graph_steps(self, steps):
        check(lib().adi_set_graph_steps(self._h, int(steps)))

    def read_field(self):
        out = np.empty(self.shape)
        check(lib().adi_read_field(self._h, _ptr(out), out.size))
        return out

    def read_field_device(self, dev_ptr):
        """Copy T into device memory at dev_ptr (nz*nr doubles).  On the
        problem's stream; when that is a stream of the library's own, the
        call waits for torch's current stream first and for the copy after."""
        if self._own_stream:
            _torch_stream_sync()
        check(lib().adi_read_field_device(self._h, ctypes.c_void_p(dev_ptr)))
        if self._own_stream:
            check(lib().adi_sync(self._h))

    def region_map(self):
        out = np.empty(self.shape, dtype=np.uint8)
        check(lib().adi_read_region_map(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                        out.size))
        return out

    def profile(self, which=0, npts=64):
        out = np.empty(npts)
        check(lib().adi_read_profile(self._h, int(which), int(npts), _ptr(out)))
        return out

    def energy(self):
        r = EnergyReport()
        check(lib().adi_energy(self._h, ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in EnergyReport._fields_}

    def time_sweeps(self, dt, nlaunch):
        a, b = ctypes.c_float(), ctypes.c_float()
        check(lib().adi_time_sweeps(self._h, float(dt), int(nlaunch), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def set_launch(self, direction, chunk, lines_per_wave, waves_per_line, lines_per_lane=1,
                   groups_per_block=1):
        check(lib().adi_set_launch(self._h, int(direction), int(chunk), int(lines_per_wave),
                                   int(waves_per_line), int(lines_per_lane), int(groups_per_block)))

    def get_launch(self, direction):
        v = [ctypes.c_int32() for _ in range(5)]
        check(lib().adi_get_launch(self._h, int(direction), *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    # ---- nonlinear path (laws in T, simple iteration, pulsed source) ----
    PULSES = {"const": 0, "rect": 1, "erf": 2}

    def set_laws(self, lam, cap, src):
        """5 x 4 polynomial coefficients per law (region-major)."""
        self._laws = [_f64(lam, 20), _f64(cap, 20), _f64(src, 20)]
        check(lib().adi_set_laws(self._h, *(_ptr(a) for a in self._laws)))

    def set_pulse(self, kind, t_per=0.1, t_src=0.01, t_trs=1e-4, xi=4.0, zeta=2.0):
        pp = _f64([t_per, t_src, t_trs, xi, zeta], 5)
        check(lib().adi_set_pulse(self._h, self.PULSES[kind], _ptr(pp)))

    def set_iteration(self, eps=1e-6, iter_max=10, tau_min=1e-12):
        check(lib().adi_set_iteration(self._h, float(eps), int(iter_max), float(tau_min)))

    def set_step_rule(self, tau_trs_div=1000.0, tau_src_div=100.0, periodic_tol=0.0):
        check(lib().adi_set_step_rule(self._h, float(tau_trs_div), float(tau_src_div), float(periodic_tol)))

    def nl_step(self, tau):
        """One attempt of size tau: (accepted, (solves_r, solves_z), changes)."""
        acc = ctypes.c_int32()
        it = (ctypes.c_int32 * 2)()
        chg = np.zeros(2)
        check(lib().adi_nl_step(self._h, float(tau), ctypes.byref(acc), it, _ptr(chg)))
        return bool(acc.value), (it[0], it[1]), chg

    def nl_run(self, t_end, max_steps=1 << 62, log_cap=0):
        """The adaptive loop up to t_end; returns the report as a dict (and
        the per-step log rows when log_cap > 0)."""
        rep = NlReport()
        log = np.zeros((max(log_cap, 1), 4))
        check(lib().adi_nl_run(self._h, float(t_end), int(max_steps), _ptr(log) if log_cap else None,
                               int(log_cap), ctypes.byref(rep)))
        out = {k: getattr(rep, k) for k, _ in NlReport._fields_}
        out["periodic"] = bool(out["periodic"])
        if log_cap:
            out["log"] = log[:min(rep.steps, log_cap)]
        return out

    def set_layout(self, layout):
        """"rows", "strips" or "resident" (adi_set_layout); resets the launch
        shapes."""
        check(lib().adi_set_layout(self._h, LAYOUTS[layout]))

    def layout(self):
        v = ctypes.c_int32()
        check(lib().adi_get_layout(self._h, ctypes.byref(v)))
        return {b: a for a, b in LAYOUTS.items()}[v.value]


class Batch:
    """A ragged batch of independent instances (adi_create_batch ...)."""

    def __init__(self, specs, scheme="pr", stream=None):
        n = len(specs)
        geoms = (Geometry * n)()
        bcs = (BC * n)()
        for i, s in enumerate(specs):
            if s.r_faces is not None or s.z_faces is not None:
                raise ValueError("batches use uniform grids")
            geoms[i] = Geometry(*[float(x) for x in s.geom], int(s.nr), int(s.nz), None, None)
            bcs[i] = BC((ctypes.c_double * 4)(*[float(x) for x in s.h]),
                        (ctypes.c_double * 4)(*[float(x) for x in s.t_inf]))
        h = _vp()
        st = stream if stream is not None else current_stream()
        check(lib().adi_create_batch(n, geoms, bcs, SCHEMES[scheme], st, ctypes.byref(h)))
        self._h = h
        self._destroy = lib().adi_batch_destroy
        self.n = n
        self.shapes = [(int(s.nr), int(s.nz)) for s in specs]
        k = _f64([s.k for s in specs], 5 * n)
        rc = _f64([s.rhoc for s in specs], 5 * n)
        q = _f64([s.q for s in specs], 5 * n)
        check(lib().adi_batch_set_materials(self._h, _ptr(k), _ptr(rc), _ptr(q)))
        t0 = _f64([s.T0 for s in specs], n)
        check(lib().adi_batch_set_initial(self._h, _ptr(t0)))
        self._nsnap, self._npts = 0, 64

    def close(self):
        # the destroy function is looked up while the module is alive: at
        # interpreter shutdown module globals may already be gone
        h, destroy = getattr(self, "_h", None), getattr(self, "_destroy", None)
        if h and destroy is not None:
            destroy(h)
        self._h = None

    __del__ = close

    def set_launch(self, lines_per_lane, waves_per_block, blocks_per_cu):
        """(1|2, 4|8, bpc): persistent kernel on the rows layout; (4, 4|8,
        bpc): persistent kernel on the strip layout; (4, 1, 1): batched
        sweep launches (one launch per half step over all instances)."""
        check(lib().adi_batch_set_launch(self._h, int(lines_per_lane), int(waves_per_block),
                                         int(blocks_per_cu)))

    def set_zshape(self, zclass, variant):
        """Shape `variant` of batch_zshapes()[zclass] for the z lines of that
        class in the batched sweep launches (from the next step on)."""
        check(lib().adi_batch_set_zshape(self._h, int(zclass), int(variant)))

    def step(self, dt, nsteps, snapshot_every=0, npts=64, out=None):
        """Advance every instance from its initial field.  out: None, or a
        float64 CUDA tensor of n * (nsteps // snapshot_every) * npts elements
        that receives the profile snapshots on the device (it must stay alive
        until the batch's stream has finished the call)."""
        nsnap = int(nsteps) // int(snapshot_every) if snapshot_every else 0
        dev = None
        if out is not None:
            if not (out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()):
                raise ValueError("out must be a contiguous float64 CUDA tensor")
            if out.numel() < self.n * nsnap * int(npts):
                raise ValueError("out holds %d values, the snapshots need %d" % (out.numel(), self.n * nsnap * int(npts)))
            dev = ctypes.c_void_p(out.data_ptr())
            _torch_stream_sync()
        check(lib().adi_batch_step(self._h, float(dt), int(nsteps), int(snapshot_every), int(npts), dev))
        self._nsnap = nsnap
        self._npts = int(npts)

    def sync(self):
        check(lib().adi_batch_sync(self._h))

    def profiles(self):
        out = np.empty((self.n, self._nsnap, self._npts))
        check(lib().adi_batch_read_profiles(self._h, self._npts, _ptr(out), out.size))
        return out

    def field(self, i):
        nr, nz = self.shapes[i]
        out = np.empty((nz, nr))
        check(lib().adi_batch_read_field(self._h, int(i), _ptr(out), out.size))
        return out

    def info(self):
        tc, ns, wg = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().adi_batch_info(self._h, ctypes.byref(tc), ctypes.byref(ns), ctypes.byref(wg)))
        return {"total_cells": tc.value, "nsnap": ns.value, "workgroups": wg.value}

    def active_cells(self):
        a = ctypes.c_int64()
        check(lib().adi_batch_active_cells(self._h, ctypes.byref(a)))
        return a.value

    def cells(self):
        return sum(nr * nz for nr, nz in self.shapes)

    def time(self, dt, nsteps, reps=1):
        """Mean milliseconds of one adi_batch_step(dt, nsteps) call (HIP
        events on the batch's stream)."""
        ms = ctypes.c_float()
        check(lib().adi_batch_time(self._h, float(dt), int(nsteps), int(reps), ctypes.byref(ms)))
        return ms.value


def _f32(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


class MLP:
    """The surrogate network (adi_mlp_*).  Inputs/targets are torch cuda
    float32 tensors (device memory); parameters move as numpy float32."""

    def __init__(self, widths, seed=0, stream=None):
        w = (ctypes.c_int32 * len(widths))(*[int(x) for x in widths])
        h = _vp()
        st = stream if stream is not None else current_stream()
        check(lib().adi_mlp_create(w, len(widths), int(seed), st, ctypes.byref(h)))
        self._h = h
        # on a stream of its own the library is not ordered with torch's
        # work: calls that take torch tensors then synchronise both sides
        self._own_stream = st is None
        self._destroy = lib().adi_mlp_destroy
        self.widths = [int(x) for x in widths]
        n = ctypes.c_int64()
        check(lib().adi_mlp_num_params(self._h, ctypes.byref(n)))
        self.nparams = n.value

    def close(self):
        # the destroy function is looked up while the module is alive: at
        # interpreter shutdown module globals may already be gone
        h, destroy = getattr(self, "_h", None), getattr(self, "_destroy", None)
        if h and destroy is not None:
            destroy(h)
        self._h = None

    __del__ = close

    def set_scaling(self, shift, scale):
        n = self.widths[0]
        a, b = _f32(shift, n), _f32(scale, n)
        check(lib().adi_mlp_set_scaling(self._h, a.ctypes.data_as(_fp), b.ctypes.data_as(_fp)))

    def params(self):
        out = np.empty(self.nparams, dtype=np.float32)
        check(lib().adi_mlp_get_params(self._h, out.ctypes.data_as(_fp), self.nparams))
        return out

    def set_params(self, p):
        a = _f32(p, self.nparams)
        check(lib().adi_mlp_set_params(self._h, a.ctypes.data_as(_fp), self.nparams))

    def unflatten(self, flat):
        """[(W_l, b_l)] views of a flat parameter vector."""
        out, o = [], 0
        for a, b in zip(self.widths[:-1], self.widths[1:]):
            W = flat[o:o + a * b].reshape(a, b)
            o += a * b
            out.append((W, flat[o:o + b]))
            o += b
        return out

    def _before(self):
        if self._own_stream:
            _torch_stream_sync()

    def _after(self):
        if self._own_stream:
            check(lib().adi_mlp_sync(self._h))

    def forward(self, x, y):
        """x, y: contiguous torch float32 cuda tensors [B, n_in] / [B, n_out]."""
        self._before()
        check(lib().adi_mlp_forward(self._h, ctypes.c_void_p(x.data_ptr()), int(x.shape[0]),
                                    ctypes.c_void_p(y.data_ptr())))
        self._after()

    def forward_noalloc(self, x, y):
        """forward() through adi_mlp_forward_noalloc: the activations live in
        the library's fixed per-GPU work area, nothing is allocated."""
        self._before()
        check(lib().adi_mlp_forward_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), int(x.shape[0]),
                                            ctypes.c_void_p(y.data_ptr())))
        self._after()

    def gradients(self, x, t):
        g = np.empty(self.nparams, dtype=np.float32)
        loss = ctypes.c_float()
        self._before()
        check(lib().adi_mlp_gradients(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                      int(x.shape[0]), g.ctypes.data_as(_fp), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, x, t, lr, want_loss=False):
        loss = ctypes.c_float()
        self._before()
        check(lib().adi_mlp_train_step(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                       int(x.shape[0]), float(lr), ctypes.byref(loss) if want_loss else None))
        self._after()
        return loss.value if want_loss else None


def _stream_handle(stream):
    import torch
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def screen_profiles(pred, mu, sd, floor, qt=None, stream=None):
    """adi_screen_profiles on a contiguous float32 device tensor pred
    [members, n, nout]: returns device tensors (peak float64 [n],
    disagreement float64 [n], bound_ok uint8 [n]); qt: float64 device
    tensor [n] or None.  Asynchronous on `stream` (default: torch's current
    stream)."""
    import torch
    if pred.dtype != torch.float32 or not pred.is_contiguous() or pred.dim() != 3:
        raise ValueError("pred must be a contiguous float32 tensor [members, n, nout]")
    members, n, nout = pred.shape
    dev = pred.device
    peak = torch.empty(n, dtype=torch.float64, device=dev)
    dis = torch.empty(n, dtype=torch.float64, device=dev)
    ok = torch.empty(n, dtype=torch.uint8, device=dev)
    if qt is not None and (qt.dtype != torch.float64 or not qt.is_contiguous() or qt.numel() != n):
        raise ValueError("qt must be a contiguous float64 tensor of n values")
    check(lib().adi_screen_profiles(ctypes.c_void_p(pred.data_ptr()), int(members), int(n), int(nout), float(mu),
                                    float(sd), float(floor), ctypes.c_void_p(qt.data_ptr()) if qt is not None else None,
                                    ctypes.c_void_p(peak.data_ptr()), ctypes.c_void_p(dis.data_ptr()),
                                    ctypes.c_void_p(ok.data_ptr()), _stream_handle(stream)))
    return peak, dis, ok


def top_k(vals, k, stream=None):
    """adi_top_k on a contiguous float64 device tensor: int64 device tensor
    of the k largest values' indices (those above the k-th largest first,
    then its ties, each in ascending index order).  Synchronises."""
    import torch
    if vals.dtype != torch.float64 or not vals.is_contiguous():
        raise ValueError("vals must be a contiguous float64 tensor")
    idx = torch.empty(max(int(k), 1), dtype=torch.int64, device=vals.device)
    check(lib().adi_top_k(ctypes.c_void_p(vals.data_ptr()), int(vals.numel()), int(k),
                          ctypes.c_void_p(idx.data_ptr()), _stream_handle(stream)))
    return idx[:int(k)]


def launch_shapes():
    """Compiled (chunk, lines_per_wave, waves_per_line, lines_per_lane,
    groups_per_block) shapes."""
    n = ctypes.c_int32()
    check(lib().adi_launch_shapes(None, 0, ctypes.byref(n)))
    buf = (ctypes.c_int32 * (5 * n.value))()
    check(lib().adi_launch_shapes(buf, n.value, ctypes.byref(n)))
    return [tuple(buf[5 * i:5 * i + 5]) for i in range(n.value)]


def layout_shapes(layout, direction):
    """Compiled launch shapes of a layout ("rows" or "strips"; "resident" has
    one fixed shape and lists none) for one direction (0 = r, 1 = z)."""
    n = ctypes.c_int32()
    check(lib().adi_layout_shapes(LAYOUTS[layout], int(direction), None, 0, ctypes.byref(n)))
    buf = (ctypes.c_int32 * max(1, 5 * n.value))()
    check(lib().adi_layout_shapes(LAYOUTS[layout], int(direction), buf, n.value, ctypes.byref(n)))
    return [tuple(buf[5 * i:5 * i + 5]) for i in range(n.value)]


def batch_zshapes():
    """Per z class of the batched sweep launches (columns up to 192, 256,
    320, 512 rows): {"max_rows": rows, "shapes": [(waves, cells per chunk),
    ...]}, the first shape the default."""
    out = []
    for c in range(4):
        shapes, rows = [], 0
        w, m, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        v = 0
        while lib().adi_batch_zshape_info(c, v, ctypes.byref(w), ctypes.byref(m), ctypes.byref(r)) == 0:
            shapes.append((w.value, m.value))
            rows = r.value
            v += 1
        out.append({"max_rows": rows, "shapes": shapes})
    return out


def version():
    return lib().adi_version().decode()

