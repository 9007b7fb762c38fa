"""Host-side logic of the surrogate gate and target encoding (no GPU)."""
import numpy as np


def test_encode_decode_roundtrip_scale_and_shape():
    from paper_1912_03744_amd import surrogate as S
    rng = np.random.default_rng(0)
    Y = rng.uniform(0, 1, (5, 64)) * np.array([1.0, 1e-3, 1e-9, 0.5, 0.0])[:, None]
    mu, sd = S.fit_scale(Y[:4])
    Z = S.encode(Y, mu, sd)
    assert Z.shape == (5, 128)
    # the shape part peaks at exactly 1, the scale part holds one value per row
    assert np.allclose(Z[:4, :64].max(axis=1), 1.0)
    assert np.all(Z[:, 64:] == Z[:, 64:65])
    back = S.decode(Z, mu, sd)
    assert np.all(np.abs(back - Y) <= 1e-6 * Y.max(axis=1, keepdims=True) + 1e-300)
    # a cold profile decodes to (numerically) zero
    assert np.max(np.abs(back[4])) <= 1e-29
    # relative error is measured against the floor when the face is still cold
    e = S.rel_profile_error(np.full((1, 4), 2e-7), np.zeros((1, 4)))
    assert abs(e[0] - 0.2) < 1e-12


def test_gate_rejects_out_of_box_disagreement_and_bound():
    from paper_1912_03744_amd import surrogate as S
    mu, sd = -3.0, 2.0
    sur = S.Surrogate(nets=[], delta=0.01, mu=mu, sd=sd)
    D = np.tile((S.BOX_LO + S.BOX_HI) / 2, (4, 1))
    D[1, 0] = 5.0                       # k outside the training box
    P = np.stack([S.encode(np.full((4, 64), 0.5), mu, sd)] * 2)
    P[1, 2] = S.encode(np.full(64, 0.6), mu, sd)  # members disagree by ~18%
    P[:, 3] = S.encode(np.full(64, 1.5), mu, sd)  # violates the maximum-principle bound y <= 1
    ok = sur.gate(D, P)
    assert ok.tolist() == [True, False, False, False]
