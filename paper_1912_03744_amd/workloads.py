"""Seeded synthetic workloads for the layered-cylinder heat problem.

This module only draws problem parameters (geometry, materials, sources,
boundary films, time step).  It holds none of the method's arithmetic, so both
the HIP path and the CPU oracle can be fed from it.

Geometry is the L-shaped quarter slice of Fig. 1 of Ayriyan & Busa (arXiv
1912.03744): cooler core r < r0 up to z = zmax, insulator [r0, r1), heater
[r1, r2), outer insulator [r2, rmax) up to z = z0, terminal slab
[zmax, ztop) over the whole radius; cells with r >= r0 and z0 <= z < zmax are
outside the domain.  The paper's physical material laws are not given in it,
so every workload here is synthetic, in dimensionless units.

Boundary-face classes: 0 bottom z = 0, 1 outer r = rmax, 2 top z = ztop,
3 faces against the cut-out (masked) cells.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

# grid sizes (nr, nz) of the ragged batch
BATCH_SIZES = ((64, 160), (96, 240), (128, 320), (192, 480))


@dataclasses.dataclass
class Spec:
    """One problem instance."""
    r0: float
    r1: float
    r2: float
    rmax: float
    z0: float
    zmax: float
    ztop: float
    nr: int
    nz: int
    h: Sequence[float]          # 4 face classes
    t_inf: Sequence[float]      # 4 face classes
    k: Sequence[float]          # 5 regions
    rhoc: Sequence[float]       # 5 regions
    q: Sequence[float]          # 5 regions
    scheme: str = "pr"          # "pr" (Peaceman-Rachford) or "lod" (LOD backward Euler)
    dt: float = 1e-3
    nsteps: int = 1
    T0: float = 0.0
    r_faces: Optional[np.ndarray] = None
    z_faces: Optional[np.ndarray] = None

    @property
    def geom(self):
        return (self.r0, self.r1, self.r2, self.rmax, self.z0, self.zmax, self.ztop)

    def replace(self, **kw) -> "Spec":
        return dataclasses.replace(self, **kw)


def single_layout(nr=64, nz=160, scheme="lod", dt=1e-3, nsteps=1000) -> Spec:
    """The fixed single instance: cooler r<2, insulator [2,3), heater [3,4),
    outer insulator [4,4.2) up to z = 8; cut-out 8 <= z < 10; terminal
    [10, 10.2).  k = (0.5, 0.05, 1.0, 0.05, 2.0), rho c = 1, Q = 1 in the
    heater, T0 = 0; Neumann at z = 0, Robin h = 0.1 (T_inf = 0) on the outer,
    top and cut-out faces."""
    return Spec(r0=2.0, r1=3.0, r2=4.0, rmax=4.2, z0=8.0, zmax=10.0, ztop=10.2,
                nr=nr, nz=nz, h=(0.0, 0.1, 0.1, 0.1), t_inf=(0.0, 0.0, 0.0, 0.0),
                k=(0.5, 0.05, 1.0, 0.05, 2.0), rhoc=(1.0,) * 5,
                q=(0.0, 0.0, 1.0, 0.0, 0.0), scheme=scheme, dt=dt, nsteps=nsteps)


def production(seed: int, nr=1024, nz=2560, scheme="pr", dt=1e-4, nsteps=10_000) -> Spec:
    """Same layout at production resolution with seeded materials: per region
    k = 10**U(-2, 1), rho c = U(0.5, 2); heater Q = U(0.5, 2).  Draw order:
    k[5], rho c[5], Q, from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = 10.0 ** rng.uniform(-2.0, 1.0, size=5)
    rhoc = rng.uniform(0.5, 2.0, size=5)
    q = rng.uniform(0.5, 2.0)
    base = single_layout(nr=nr, nz=nz, scheme=scheme, dt=dt, nsteps=nsteps)
    return base.replace(k=tuple(k), rhoc=tuple(rhoc), q=(0.0, 0.0, float(q), 0.0, 0.0))


def _centres(n, length):
    return (np.arange(n) + 0.5) * length / n


def _has_tie(s: Spec, tol=1e-12) -> bool:
    rc = _centres(s.nr, s.rmax)
    zc = _centres(s.nz, s.ztop)
    for x in (s.r0, s.r1, s.r2):
        if np.min(np.abs(rc - x)) < tol * s.rmax:
            return True
    for x in (s.z0, s.zmax):
        if np.min(np.abs(zc - x)) < tol * s.ztop:
            return True
    return False


def draw_design(rng: np.random.Generator) -> dict:
    """One design of the sweep, in a fixed draw order: r0, dr1, dr2, z0,
    log10 k[5], Q, log10 h."""
    r0 = rng.uniform(1.5, 2.5)
    r1 = r0 + rng.uniform(0.5, 1.5)
    r2 = r1 + rng.uniform(0.5, 1.5)
    z0 = rng.uniform(6.0, 9.0)
    logk = rng.uniform(-2.0, 1.0, size=5)
    q = rng.uniform(0.5, 2.0)
    logh = rng.uniform(-2.0, 0.0)
    return dict(r0=r0, r1=r1, r2=r2, z0=z0, logk=logk, q=q, logh=logh)


def design_spec(d: dict, nr: int, nz: int, scheme="pr", dt=1e-3, nsteps=2000) -> Spec:
    """Problem instance of one design: rmax = r2 + 0.2, zmax = z0 + 2,
    ztop = zmax + 0.2, rho c = 1, h on the outer, top and cut-out faces,
    Neumann at z = 0, T_inf = 0, T0 = 0."""
    h = 10.0 ** d["logh"]
    return Spec(r0=d["r0"], r1=d["r1"], r2=d["r2"], rmax=d["r2"] + 0.2,
                z0=d["z0"], zmax=d["z0"] + 2.0, ztop=d["z0"] + 2.2,
                nr=nr, nz=nz, h=(0.0, h, h, h), t_inf=(0.0,) * 4,
                k=tuple(10.0 ** np.asarray(d["logk"])), rhoc=(1.0,) * 5,
                q=(0.0, 0.0, float(d["q"]), 0.0, 0.0), scheme=scheme, dt=dt,
                nsteps=nsteps)


def ragged_batch(n: int, master_seed: int = 0, scheme="pr", dt=1e-3, nsteps=2000,
                 sizes=BATCH_SIZES) -> list:
    """n instances drawn one after the other from PCG64(master_seed): size
    index integers(len(sizes)), then the design draws.  An instance whose
    cell centre falls within 1e-12 of an interface is drawn again."""
    rng = np.random.Generator(np.random.PCG64(master_seed))
    out = []
    while len(out) < n:
        si = int(rng.integers(len(sizes)))
        d = draw_design(rng)
        s = design_spec(d, *sizes[si], scheme=scheme, dt=dt, nsteps=nsteps)
        if not _has_tie(s):
            out.append(s)
    return out


def design_matrix(n: int, seed: int) -> np.ndarray:
    """n designs as rows of 11 parameters (5 log10 k, Q, log10 h, r0, r1, r2,
    z0) drawn with draw_design from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.empty((n, 11))
    for i in range(n):
        d = draw_design(rng)
        X[i, :5] = d["logk"]
        X[i, 5] = d["q"]
        X[i, 6] = d["logh"]
        X[i, 7:] = (d["r0"], d["r1"], d["r2"], d["z0"])
    return X


def design_from_row(x) -> dict:
    x = np.asarray(x, dtype=np.float64)
    return dict(logk=x[:5], q=float(x[5]), logh=float(x[6]), r0=float(x[7]),
                r1=float(x[8]), r2=float(x[9]), z0=float(x[10]))


def layer_aligned_faces(bounds, counts):
    """Face coordinates uniform inside each layer: bounds = (x0, x1, ..., xL),
    counts = cells per layer.  Used for grids whose faces fall on the
    material interfaces, like the per-layer grid of Sec. 5."""
    faces = [bounds[0]]
    for a, b, n in zip(bounds[:-1], bounds[1:], counts):
        for i in range(1, n + 1):
            faces.append(a + (b - a) * i / n)
    f = np.array(faces, dtype=np.float64)
    f[-1] = bounds[-1]
    return f


# Sec. 5 case study: cell size, per-layer cell counts and source timing.
CASE_STUDY_GEOM = dict(r0=0.24, r1=0.245, r2=0.25, rmax=0.2501, z0=4.0, zmax=5.0)
CASE_STUDY_CELLS_R = (800, 200, 200, 10)   # core, insulator, heater, coating
CASE_STUDY_CELLS_Z = (80, 20)              # up to z0 (all layers), z0 to zmax (core only)
CASE_STUDY_PULSE = (0.1, 0.01, 1e-4, 4.0, 2.0)   # t_per, t_src, t_trs, xi, zeta
CASE_STUDY_T0 = 4.2


def case_study(scale_r=1.0, scale_z=1.0) -> Spec:
    """The cell of Sec. 5 on its per-layer grid: r faces uniform inside each
    layer (800, 200, 200, 10 cells; widths 3e-4, 2.5e-5, 2.5e-5, 1e-5), z
    faces uniform with 80 cells up to z0 and 20 from z0 to zmax (0.05 each),
    1210 x 100 cells.  No terminal slab (ztop = zmax): the terminal is the top
    face of the core, held at T0 = 4.2 (Dirichlet, eq. 6); every other face
    is insulated.  scale_r / scale_z shrink the cell counts of every layer
    (at least 2 cells each) for smaller test grids.  The materials here are
    placeholders: the nonlinear path takes its laws from case_study_laws."""
    g = CASE_STUDY_GEOM
    nrs = [max(2, int(round(c * scale_r))) for c in CASE_STUDY_CELLS_R]
    nzs = [max(2, int(round(c * scale_z))) for c in CASE_STUDY_CELLS_Z]
    rf = layer_aligned_faces((0.0, g["r0"], g["r1"], g["r2"], g["rmax"]), nrs)
    zf = layer_aligned_faces((0.0, g["z0"], g["zmax"]), nzs)
    return Spec(r0=g["r0"], r1=g["r1"], r2=g["r2"], rmax=g["rmax"], z0=g["z0"], zmax=g["zmax"], ztop=g["zmax"],
                nr=len(rf) - 1, nz=len(zf) - 1, h=(0.0, 0.0, float("inf"), 0.0),
                t_inf=(0.0, 0.0, CASE_STUDY_T0, 0.0), k=(40.0, 0.1, 1.0, 0.5, 1.0), rhoc=(1.0,) * 5,
                q=(0.0, 0.0, 1.0, 0.0, 0.0), scheme="pr", dt=1e-4, T0=CASE_STUDY_T0, r_faces=rf, z_faces=zf)


def case_study_laws():
    """Synthetic temperature laws for the case study (the paper does not
    publish its material data): per region (cooler, insulator, heater,
    coating, terminal) cubic polynomials in T of the conductivity, the
    volumetric heat capacity and the source amplitude, all positive and
    increasing over 4 <= T <= 60: a copper-like core conducting 100x better
    than the layers, capacities rising like a low-temperature solid's, and a
    heater whose resistive source rises 1 % per unit of T.  Returns (lam,
    cap, src) as 5 x 4 arrays (c0, c1, c2, c3)."""
    lam = np.array([[40.0, 0.4, 0.0, 0.0],
                    [0.1, 0.004, 0.0, 0.0],
                    [1.0, 0.02, 0.0, 0.0],
                    [0.5, 0.01, 0.0, 0.0],
                    [40.0, 0.4, 0.0, 0.0]])
    cap = np.array([[0.5, 0.0, 0.002, 2e-5],
                    [0.8, 0.0, 0.003, 2e-5],
                    [0.6, 0.0, 0.004, 3e-5],
                    [0.7, 0.0, 0.003, 2e-5],
                    [0.5, 0.0, 0.002, 2e-5]])
    src = np.zeros((5, 4))
    src[2] = (50000.0, 500.0, 0.0, 0.0)
    return lam, cap, src
