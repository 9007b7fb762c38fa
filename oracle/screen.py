"""Plain definitions of the surrogate sweep's screening reductions (test
infrastructure, numpy in float64): the ensemble's decoded profile, its peak,
the members' disagreement, the maximum-principle check, and the indices of
the k largest values.  Only tests use this module."""
import numpy as np

NPTS = 64


def decode(pred, mu, sd):
    """Profiles [..., 64] from network outputs [..., nout]: the shape in
    outputs 0..63 times exp(mu + sd * mean of outputs 64..nout-1)."""
    P = np.asarray(pred, dtype=np.float64)
    scale = np.exp(mu + sd * P[..., NPTS:].mean(axis=-1))
    return scale[..., None] * P[..., :NPTS]


def screen(pred, mu, sd, floor, qt=None):
    """(peak, disagreement, bound_ok) of every design; pred [members, n,
    nout]."""
    y = decode(pred, mu, sd)
    ybar = y.mean(axis=0)
    ymax = ybar.max(axis=-1)
    peak = ymax * (1.0 if qt is None else np.asarray(qt, dtype=np.float64))
    dis = np.abs(y[0] - y[-1]).max(axis=-1) / np.maximum(ymax, floor)
    ok = np.all(ybar <= 1.0 + 1e-3, axis=-1)
    return peak, dis, ok


def top_k(vals, k):
    """Indices of the k largest values (NaN below every number; of equal
    values the lower indices first): those above the k-th largest value in
    ascending index order, then those equal to it in ascending index
    order."""
    v = np.asarray(vals, dtype=np.float64)
    nan = np.isnan(v)
    # rank: NaN last, then descending value, then ascending index (lexsort's
    # last key is the primary one)
    order = np.lexsort((np.arange(len(v)), -np.where(nan, 0.0, v), nan))
    chosen = order[:k]
    kth = chosen[-1]
    above = [i for i in sorted(chosen) if not _same(v[i], v[kth])]
    ties = [i for i in sorted(chosen) if _same(v[i], v[kth])]
    return np.array(above + ties, dtype=np.int64)


def _same(a, b):
    return (np.isnan(a) and np.isnan(b)) or a == b
