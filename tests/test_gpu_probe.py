"""The blocked 0/1 contraction measurement (bn_zeta4_probe): both methods
compute the 4-bit upward zeta (Def. 1) of every 16-entry group exactly as a
direct sum over subsets does, so that their times compare like for like."""
import numpy as np
import pytest

import paper_1408_1664_amd as bn

pytestmark = pytest.mark.gpu


def _zeta4_direct(x):
    """t(g, T) = sum over S subset of T of x(g, S), written out per T."""
    g = x.reshape(-1, 16)
    out = np.zeros_like(g)
    for T in range(16):
        for S in range(16):
            if S & ~T == 0:
                out[:, T] += g[:, S]
    return out.reshape(-1)


@pytest.mark.parametrize("method", ["valu", "mfma"])
@pytest.mark.parametrize("groups", [16, 48, 4096 + 16])
def test_zeta4_probe_matches_direct_sum(method, groups):
    import torch

    rng = np.random.default_rng(groups)
    x = rng.random(16 * groups)
    xd = torch.from_numpy(x).cuda()
    yd = torch.full_like(xd, np.nan)
    print(f"zeta4 probe {method} groups={groups}", flush=True)
    ms = bn.zeta4_probe(xd, yd, method, reps=1)
    y = yd.cpu().numpy()
    want = _zeta4_direct(x)
    assert ms >= 0.0
    np.testing.assert_allclose(y, want, rtol=1e-14, atol=0.0)


def test_zeta4_probe_repeats():
    import torch

    x = np.random.default_rng(7).random(16 * 64)
    xd = torch.from_numpy(x).cuda()
    yv, ym = torch.empty_like(xd), torch.empty_like(xd)
    print("zeta4 probe reps=3", flush=True)
    bn.zeta4_probe(xd, yv, "valu", reps=3)
    bn.zeta4_probe(xd, ym, "mfma", reps=3)
    z = _zeta4_direct(x)
    # the register pass applies the transform three times in a row, the
    # matrix cores accumulate three equal products
    np.testing.assert_allclose(yv.cpu().numpy(), _zeta4_direct(_zeta4_direct(z)), rtol=1e-13)
    np.testing.assert_allclose(ym.cpu().numpy(), 3 * z, rtol=1e-14)
