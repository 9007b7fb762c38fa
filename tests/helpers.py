"""Shared helpers for the GPU-vs-oracle tests: run the same seeded problem on
both sides and compare.  Imports both sides; neither side imports the other."""
import numpy as np

import oracle
from paper_1912_03744_amd import workloads as W


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def rel_inf(a, b, active):
    """max over active cells |a - b| / max over active cells |b| (the
    infinity-norm relative error used for every field comparison)."""
    d = np.max(np.abs(a[active] - b[active]))
    s = np.max(np.abs(b[active]))
    return d / s if s > 0 else d


def run_oracle(spec, nsteps, T0=None):
    P = oracle.Problem.from_spec(spec)
    T = P.initial(spec.T0) if T0 is None else T0
    out, mid = P.step(T, spec.scheme, spec.dt, nsteps)
    return P, out, mid


def run_gpu(spec, nsteps, launch=None, T0=None, graph_steps=0, check_every=0, tune=False, layout=None):
    from paper_1912_03744_amd import native
    p = native.Problem.from_spec(spec)
    if layout:
        p.set_layout(layout)
    if tune:
        from paper_1912_03744_amd import autotune
        autotune.apply(p, spec.dt, spec.scheme)
    if launch:
        for d, shape in launch.items():
            p.set_launch(d, *shape)
    if T0 is not None:
        p.set_field(T0)
    if graph_steps:
        p.set_graph_steps(graph_steps)
    if check_every:
        p.set_check(check_every)
    p.step(spec.dt, nsteps)
    return p, p.read_field()


def tiny_spec(nr=7, nz=12, scheme="pr", dt=0.05):
    """Every region, the cut-out, the terminal and all four boundary classes,
    with non-zero ambient temperatures and one Dirichlet class."""
    return W.Spec(r0=1.0, r1=1.6, r2=2.3, rmax=2.6, z0=3.1, zmax=4.4, ztop=5.0, nr=nr, nz=nz,
                  h=(0.3, 0.2, float("inf"), 0.15), t_inf=(0.4, -0.3, 0.25, 0.1),
                  k=(0.8, 0.07, 1.3, 0.2, 2.1), rhoc=(1.1, 0.6, 1.7, 0.9, 1.3),
                  q=(0.2, 0.0, 1.5, 0.3, 0.1), scheme=scheme, dt=dt, T0=0.3)
