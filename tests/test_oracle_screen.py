"""Pins of the screening reductions' plain definitions (oracle/screen.py):
decoding against profiles built by hand, the disagreement and bound on
constructed ensembles, and the top-k selection against an exhaustive
ranking of every element."""
import numpy as np

from oracle import screen as O


def _encode(y, mu, sd, ncopies=64):
    m = y.max(axis=-1)
    z = (np.log(m) - mu) / sd
    return np.concatenate([y / m[..., None], np.repeat(z[..., None], ncopies, axis=-1)], axis=-1)


def test_decode_inverts_the_scale_and_shape_split():
    rng = np.random.default_rng(1)
    y = rng.uniform(0.0, 1.0, (3, 5, 64)) * 10.0 ** rng.uniform(-8, 0, (3, 5, 1))
    for ncopies in (64, 32):
        assert np.allclose(O.decode(_encode(y, -4.0, 3.0, ncopies), -4.0, 3.0), y, rtol=1e-13, atol=0)


def test_screen_on_constructed_ensembles():
    y = np.full((2, 3, 64), 0.25)
    y[1, 1, 7] = 0.5          # design 1: members differ at one point by 0.25
    y[:, 2, 3] = 1.5          # design 2: above the maximum-principle bound
    pred = _encode(y, 0.0, 1.0)
    peak, dis, ok = O.screen(pred, 0.0, 1.0, 1e-6, qt=np.array([2.0, 1.0, 1.0]))
    assert np.allclose(peak, [0.5, 0.375, 1.5], rtol=1e-14)
    assert np.allclose(dis, [0.0, 0.25 / 0.375, 0.0], rtol=1e-13, atol=1e-15)
    assert ok.tolist() == [True, True, False]


def test_top_k_against_exhaustive_ranking():
    rng = np.random.default_rng(2)
    for n in (1, 2, 7, 40):
        v = np.round(rng.normal(size=n), 1)   # many ties
        if n > 5:
            v[3] = np.nan
        for k in range(1, n + 1):
            # rank every element by (is NaN, -value, index), take the first k
            ranked = sorted(range(n), key=lambda i: (np.isnan(v[i]), 0.0 if np.isnan(v[i]) else -v[i], i))[:k]
            last = v[ranked[-1]]
            same = (lambda a: np.isnan(a) and np.isnan(last)) if np.isnan(last) else (lambda a: a == last)
            want = sorted(i for i in ranked if not same(v[i])) + sorted(i for i in ranked if same(v[i]))
            assert O.top_k(v, k).tolist() == want, (n, k)
