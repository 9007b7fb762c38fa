"""GPU screening reductions of the surrogate sweep (adi_screen_profiles,
adi_top_k) against their plain definitions (oracle/screen.py): decoded
peaks, disagreements and bound flags of random ensembles (within 1e-13
relative: the device sums the scale outputs in another order), and the
top-k selection index for index, on ragged sizes, many ties, NaN and
signed zeros, up to the sweep's 2^20 designs and 10,486 selections."""
import numpy as np
import pytest

from helpers import gpu_available
from oracle import screen as O

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.mark.parametrize("members,n,nout", [(2, 5003, 128), (3, 64, 96), (1, 1, 65), (2, 1 << 16, 128)])
def test_screen_profiles_match_definition(members, n, nout):
    import torch
    from paper_1912_03744_amd import native
    rng = np.random.default_rng(n + nout)
    pred = rng.uniform(0.0, 1.0, (members, n, nout)).astype(np.float32)
    pred[..., 64:] = rng.normal(0.0, 1.0, (members, n, 1)) + rng.normal(0.0, 0.01, (members, n, nout - 64))
    pred[0, : n // 7, 5] = 3.0  # some profiles above the maximum-principle bound
    mu, sd, floor = -6.0, 2.5, 1e-6
    qt = rng.uniform(0.1, 4.0, n)
    peak, dis, ok = native.screen_profiles(torch.tensor(pred, device="cuda"), mu, sd, floor,
                                           torch.tensor(qt, device="cuda"))
    wp, wd, wo = O.screen(pred, mu, sd, floor, qt)
    assert np.allclose(peak.cpu().numpy(), wp, rtol=1e-13, atol=0)
    assert np.allclose(dis.cpu().numpy(), wd, rtol=1e-13, atol=1e-300)
    assert np.array_equal(ok.cpu().numpy().astype(bool), wo)
    peak1, _, _ = native.screen_profiles(torch.tensor(pred, device="cuda"), mu, sd, floor)
    assert np.allclose(peak1.cpu().numpy(), wp / qt, rtol=1e-13, atol=0)


@pytest.mark.parametrize("n,k", [(1, 1), (5, 3), (1023, 1023), (1025, 17), (100_003, 1000), (1 << 20, 10_486)])
def test_top_k_matches_definition(n, k):
    import torch
    from paper_1912_03744_amd import native
    rng = np.random.default_rng(n)
    v = np.round(rng.normal(size=n), 2)        # many ties
    if n > 10:
        v[rng.integers(0, n, 5)] = np.nan
        v[rng.integers(0, n, 5)] = -0.0
        v[rng.integers(0, n, 5)] = 0.0
    got = native.top_k(torch.tensor(v, device="cuda"), k).cpu().numpy()
    assert got.tolist() == O.top_k(v, k).tolist()


def test_top_k_all_equal_and_errors():
    import torch
    from paper_1912_03744_amd import native
    v = torch.full((3000,), 0.5, dtype=torch.float64, device="cuda")
    assert native.top_k(v, 7).cpu().numpy().tolist() == list(range(7))
    with pytest.raises(native.AdiError) as e:
        native.top_k(v, 3001)
    assert e.value.status == native.ADI_EINVAL
    with pytest.raises(native.AdiError):
        native.screen_profiles(torch.zeros(2, 10, 64, device="cuda"), 0.0, 1.0, 1e-6)
