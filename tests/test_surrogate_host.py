"""Host-side logic of the surrogate gate and target encoding (no GPU)."""
import numpy as np


def test_encode_decode_roundtrip_and_floor():
    from paper_1912_03744_amd import surrogate as S
    y = np.array([0.0, 1e-12, 1e-6, 1e-3, 0.5, 1.0])
    back = S.decode(S.encode(y))
    assert np.all(np.abs(back - y) <= 1e-6 * np.maximum(y, S.Y_FLOOR) + 1e-12)
    # relative error is measured against the floor when the face is still cold
    e = S.rel_profile_error(np.full((1, 4), 2e-7), np.zeros((1, 4)))
    assert abs(e[0] - 0.2) < 1e-12


def test_gate_rejects_out_of_box_disagreement_and_bound():
    from paper_1912_03744_amd import surrogate as S
    sur = S.Surrogate(nets=[], delta=0.01)
    D = np.tile((S.BOX_LO + S.BOX_HI) / 2, (4, 1))
    D[1, 0] = 5.0                       # k outside the training box
    P = np.stack([S.encode(np.full((4, 64), 0.5))] * 2)
    P[1, 2] = S.encode(np.full(64, 0.6))  # members disagree by ~18%
    P[:, 3] = S.encode(np.full(64, 1.5))  # violates the maximum-principle bound y <= 1
    ok = sur.gate(D, P)
    assert ok.tolist() == [True, False, False, False]
