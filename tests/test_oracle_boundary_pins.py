"""Pins of the oracle's boundary branches against closed forms: the Dirichlet
limit h = infinity of the boundary film (eq. 6), the film on faces against
cells outside the domain (the cut-out of Fig. 1: the core's side face, the
outer layers' top face and the terminal's underside), and the row of the
contact-face profile.  Each closed form is a one-dimensional steady state
(series resistances, Sec. 2 eq. 1 with eq. 6) or a hand derivation from the
centre rule (eq. 7); none is computed by the oracle itself.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1912_03744_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def steady(P):
    """Steady state of the assembled operator on the active cells: the
    solution of (L_r + L_z) T = -(b_r + b_z + Q), by dense LU over the cells
    (probing the affine operators with unit vectors)."""
    n = P.nr * P.nz
    ar0, az0 = P.apply(np.zeros(n))
    b = (ar0 + az0).ravel()
    A = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        ar, az = P.apply(e)
        A[:, c] = (ar + az).ravel() - b
    act = P.active().ravel()
    T = np.full(n, np.nan)
    Q = P.coeffs("Q").ravel()
    T[act] = np.linalg.solve(A[np.ix_(act, act)], -(b + Q)[act])
    return T.reshape(P.shape)


# ------------------------------------------ Dirichlet limit (eq. 6) --

def test_dirichlet_top_face_linear_profile_exact():
    """A column of one material between a Robin bottom face (h0, T_a) and a
    Dirichlet top face (h = inf, T_b), no source: the heat flow is
    F = (T_a - T_b) / (1/h0 + Z/k) and T(z) = T_a - F/h0 - F z/k.  The
    cell-centred balance form with half-cell series resistances is exact on
    linear profiles, so any error in the Dirichlet conductance 2k/d shows up
    at rounding level."""
    k, h0, Ta, Tb, Z = 0.7, 0.45, 1.9, 0.3, 2.0
    for nz in (5, 16, 41):
        s = W.Spec(r0=1.0, r1=1.2, r2=1.4, rmax=1.5, z0=Z, zmax=Z, ztop=Z, nr=1, nz=nz,
                   h=(h0, 0.0, math.inf, 0.0), t_inf=(Ta, 0.0, Tb, 0.0),
                   k=(k,) * 5, rhoc=(1.0,) * 5, q=(0.0,) * 5)
        P = oracle.Problem.from_spec(s)
        assert P.region_map()[0, 0] == 0
        T = steady(P)[:, 0]
        _, _, _, zc = P.grid()
        F = (Ta - Tb) / (1.0 / h0 + Z / k)
        exact = Ta - F / h0 - F * zc / k
        assert np.max(np.abs(T - exact)) <= 1e-13 * max(abs(Ta), abs(Tb)), nz


def _radial_dirichlet(f, t_out=0.3):
    """Concentric layers, source in the core, Dirichlet (h = inf) at rmax:
    the series log-resistance steady state without the film term."""
    r0, r1, r2, rmax = 0.6, 0.9, 1.3, 1.5
    k = (2.0, 0.1, 1.2, 0.3, 1.0)
    Q = 1.7
    rf = W.layer_aligned_faces((0.0, r0, r1, r2, rmax), (6 * f, 4 * f, 5 * f, 3 * f))
    s = W.Spec(r0=r0, r1=r1, r2=r2, rmax=rmax, z0=1.0, zmax=1.0, ztop=1.0,
               nr=len(rf) - 1, nz=1, h=(0.0, math.inf, 0.0, 0.0), t_inf=(0.0, t_out, 0.0, 0.0),
               k=k, rhoc=(1.0,) * 5, q=(Q, 0.0, 0.0, 0.0, 0.0), r_faces=rf)
    P = oracle.Problem.from_spec(s)
    T = steady(P)[0]
    _, _, rc, _ = P.grid()
    phi = Q * r0 ** 2 / 2  # r q(r) outside the core
    rho = (r0, r1, r2, rmax)

    def shell(r, m):  # r in shell m (regions 1..3), temperature from rmax inwards
        v = t_out + phi * math.log(rho[m + 1] / r) / k[m + 1]
        for mm in range(m + 1, 3):
            v += phi * math.log(rho[mm + 1] / rho[mm]) / k[mm + 1]
        return v

    exact = np.empty_like(rc)
    for i, r in enumerate(rc):
        if r < r0:
            exact[i] = shell(r0, 0) + Q * (r0 ** 2 - r ** 2) / (4 * k[0])
        else:
            exact[i] = shell(r, 0 if r < r1 else (1 if r < r2 else 2))
    return np.max(np.abs(T - exact)) / np.max(np.abs(exact))


def test_dirichlet_outer_face_log_resistance_second_order():
    """Steady radial conduction through the layers with the outer face held
    at T_inf (h = inf): series logarithmic resistances with no film term.
    Second order on layer-aligned grids; a Dirichlet conductance that puts the
    boundary a whole cell (not half a cell) from the centre is first order."""
    errs = [_radial_dirichlet(f) for f in (1, 2, 4)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs
    assert errs[-1] < 2e-4, errs


# ------------------------- films against cells outside the domain (Fig. 1) --

def _core_side_face(f, h3=0.6, T3=0.3, h1=0.9, T1=5.0):
    """One row inside the cut-out band (z0 <= z_c < zmax): only the core's
    cells are in the domain, and the core's side face at r0 looks onto cells
    outside it (face class 3).  The outer face r = rmax belongs to a cell
    outside the domain, so class 1's film must not act."""
    r0, r1, r2, rmax = 1.0, 1.4, 1.7, 2.0
    k0, Q = 0.7, 1.3
    rf = W.layer_aligned_faces((0.0, r0, r1, r2, rmax), (8 * f, 3 * f, 3 * f, 2 * f))
    s = W.Spec(r0=r0, r1=r1, r2=r2, rmax=rmax, z0=0.2, zmax=1.8, ztop=2.0, nr=len(rf) - 1, nz=1,
               h=(0.0, h1, 0.0, h3), t_inf=(0.0, T1, 0.0, T3),
               k=(k0, 1.0, 1.0, 1.0, 1.0), rhoc=(1.0,) * 5, q=(Q, 0.0, 0.0, 0.0, 0.0), r_faces=rf)
    P = oracle.Problem.from_spec(s)
    m = P.region_map()[0]
    _, _, rc, _ = P.grid()
    assert np.all(m[rc < r0] == 0) and np.all(m[rc > r0] == oracle.MASKED)
    T = steady(P)[0]
    act = m != oracle.MASKED
    r = rc[act]
    exact = T3 + Q * r0 / (2 * h3) + Q * (r0 ** 2 - r ** 2) / (4 * k0)
    return np.max(np.abs(T[act] - exact)) / np.max(np.abs(exact))


def test_core_side_face_against_cutout_uses_class_3():
    """The core's side face inside the cut-out band carries class 3's film:
    steady state T(r) = T3 + Q r0/(2 h3) + Q (r0^2 - r^2)/(4 k0), second
    order in the radial cell width."""
    errs = [_core_side_face(f) for f in (1, 2, 4)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, errs
    assert errs[-1] < 1e-4, errs


def _column(nz_lo, nz_band, nz_top, h=(0.0, 0.0, 0.8, 0.55), t_inf=(0.0, 0.0, -0.4, 1.1)):
    """One column of the outer layers (nr = 1, centre in the heater): the
    rows below z0 are in the domain, the band z0 <= z < zmax is cut out, and
    the terminal slab above zmax is in the domain again.  Layer-aligned z
    faces put z0 and zmax on faces."""
    z0, zmax, ztop = 3.0, 5.0, 6.0
    zf = W.layer_aligned_faces((0.0, z0, zmax, ztop), (nz_lo, nz_band, nz_top))
    s = W.Spec(r0=0.2, r1=0.4, r2=0.8, rmax=1.0, z0=z0, zmax=zmax, ztop=ztop, nr=1, nz=len(zf) - 1,
               h=h, t_inf=t_inf, k=(1.0, 1.0, 0.9, 1.0, 1.7), rhoc=(1.0,) * 5, q=(0.0,) * 5,
               z_faces=zf)
    return oracle.Problem.from_spec(s), (z0, zmax, ztop)


@pytest.mark.parametrize("counts", [(6, 4, 3), (13, 7, 9)])
def test_terminal_underside_and_outer_top_face_use_class_3(counts):
    """In the column the terminal slab sits between the cut-out below it
    (class 3: h3, T3) and the top face (class 2: h2, T2); with no source its
    profile is linear with heat flow F = (T3 - T2)/(1/h3 + (ztop-zmax)/k4 +
    1/h2), exact on the cell-centred grid.  The outer layers below the
    cut-out are insulated at z = 0 and look onto the cut-out through class 3,
    so they settle at T3 exactly."""
    P, (z0, zmax, ztop) = _column(*counts)
    h2, h3 = 0.8, 0.55
    T2, T3 = -0.4, 1.1
    k4 = 1.7
    m = P.region_map()[:, 0]
    _, _, _, zc = P.grid()
    assert np.all(m[zc < z0] == 2) and np.all(m[zc > zmax] == 4)
    assert np.all(m[(zc > z0) & (zc < zmax)] == oracle.MASKED)
    T = steady(P)[:, 0]
    F = (T3 - T2) / (1.0 / h3 + (ztop - zmax) / k4 + 1.0 / h2)
    top = zc > zmax
    exact_top = T3 - F / h3 - F * (zc[top] - zmax) / k4
    assert np.max(np.abs(T[top] - exact_top)) <= 1e-13
    assert np.max(np.abs(T[zc < z0] - T3)) <= 1e-13


# ------------------------------------------ contact-face profile row --

def _golden_rows():
    rows = {}
    with open(os.path.join(GOLDEN, "contact_face_rows.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                nz, j = line.split("=")
                rows[int(nz)] = int(j)
    return rows


@pytest.mark.parametrize("nz", [160, 320, 40])
def test_contact_face_profile_row(nz):
    """which = 1 reads the first row of cells inside the terminal slab: on
    the single layout with nr = 64 the 64-point profile is that row itself,
    whose index is derived by hand in the golden file."""
    j = _golden_rows()[nz]
    s = W.single_layout(nr=64, nz=nz)
    P = oracle.Problem.from_spec(s)
    rng = np.random.default_rng(nz)
    T = np.where(P.active(), rng.normal(size=P.shape), 0.0)
    assert np.array_equal(P.profile(T, 1, 64), T[j])
    assert np.array_equal(P.profile(T, 0, 64), T[nz - 1])
