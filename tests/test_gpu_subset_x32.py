"""GPU parity of the zeta transforms on FP32-scaled storage
(bn_subset_transform_x32) against the oracle's subset sums.

Inputs are m * 2^k with m an FP32 significand in [1, 2) and k spread over 600
binary orders around 2^1500, far outside FP64, plus zeros. The oracle sums the
same values with the common factor 2^1500 taken out (FP64 then holds every
term), and the expected binary logarithm of each output is that of the
oracle's sum plus 1500.

Tolerance. Each add aligns by an exact power of two and rounds to FP32, so an
output built through nbits rounds of additions of non-negative terms is off by
at most about nbits * 2^-24 relative; terms below 2^-64 of an output may be
dropped. The check is |log2 got - log2 want| <= (nbits + 2) * 2^-23, and an
output is 0 exactly when the oracle's is.
"""
import math

import numpy as np
import pytest

import paper_1408_1664_amd as bn
from oracle import oracle as O

pytestmark = pytest.mark.gpu
K0 = 1500          # common binary order of the inputs
BIAS = 200


def _inputs(nbits, seed, zero_frac=0.1):
    """(m, k, y): significands, binary orders, and y = m * 2^(k - K0) in FP64."""
    rng = np.random.default_rng(seed)
    size = 1 << nbits
    m = (1.0 + rng.random(size)).astype(np.float32)
    k = rng.integers(K0 - 300, K0 + 300, size)
    zero = rng.random(size) < zero_frac
    m[zero] = 0.0
    y = np.ldexp(m.astype(np.float64), (k - K0).astype(np.int64))
    return m, k, y


def _encode(m, k):
    """The storage form: b = e + 200 with e = floor((k + 32) / 64), f = m * 2^(k - 64 e)."""
    e = np.floor_divide(k + 32, 64)
    f = np.ldexp(m.astype(np.float64), (k - 64 * e).astype(np.int64)).astype(np.float32)
    b = (e + BIAS).astype(np.int64)
    assert b.min() >= 1 and b.max() <= 255
    b = np.where(m == 0, 0, b).astype(np.uint8)
    return f, b


def _log2_of(f, b):
    out = np.full(f.shape, -np.inf)
    nz = (b != 0) & (f > 0)
    out[nz] = np.log2(f[nz].astype(np.float64)) + 64.0 * (b[nz].astype(np.float64) - BIAS)
    return out


def _gpu(f, b, kind, d=-1, counts=None):
    import torch
    ft = torch.from_numpy(f).cuda()
    bt = torch.from_numpy(b).cuda()
    bn.subset_transform_x32(ft, bt, kind, d, counts)
    torch.cuda.synchronize()
    return ft.cpu().numpy(), bt.cpu().numpy()


def _check(got_log2, want_sum, nbits, what):
    want = np.full(want_sum.shape, -np.inf)
    pos = want_sum > 0
    want[pos] = np.log2(want_sum[pos]) + K0
    assert np.array_equal(np.isfinite(got_log2), pos), f"{what}: zero pattern differs"
    err = np.abs(got_log2[pos] - want[pos])
    tol = (nbits + 2) * 2.0 ** -23
    assert err.max() <= tol, f"{what}: max |dlog2| {err.max():.3e} > {tol:.3e}"
    return float(err.max())


@pytest.mark.parametrize("nbits", [1, 4, 12, 13, 16, 17])
def test_every_output_wide_range(nbits):
    m, k, y = _inputs(nbits, 40 + nbits)
    f, b = _encode(m, k)
    for kind, d in [("zeta_up", -1), ("zeta_up", 3), ("zeta_up", 0), ("zeta_down", -1)]:
        print(f"subset x32 nbits={nbits} kind={kind} d={d}", flush=True)
        gf, gb = _gpu(f, b, kind, d)
        err = _check(_log2_of(gf, gb), O.subset_sums(y, kind, d), nbits, f"{kind} d={d}")
        print(f"  max |dlog2| = {err:.3e}", flush=True)


@pytest.mark.parametrize("nbits", [20, 24])
def test_sampled_outputs(nbits):
    m, k, y = _inputs(nbits, 60 + nbits)
    f, b = _encode(m, k)
    rng = np.random.default_rng(nbits)
    for kind in ["zeta_up", "zeta_down"]:
        print(f"subset x32 sampled nbits={nbits} kind={kind}", flush=True)
        gf, gb = _gpu(f, b, kind)
        Ts = []
        for _ in range(512):
            cnt = int(rng.integers(0, 17))
            T = int(sum(1 << int(x) for x in rng.choice(nbits, cnt, replace=False)))
            Ts.append(T if kind == "zeta_up" else ((1 << nbits) - 1) ^ T)
        Ts = np.array(Ts, dtype=np.uint64)
        idx = Ts.astype(np.int64)
        _check(_log2_of(gf[idx], gb[idx]), O.subset_sums_at(y, kind, Ts), nbits, kind)


def test_full_size_2_30_closed_forms_and_counts():
    """2^30 entries (5 GiB in this form): all-ones input, whose outputs are
    integers FP32 holds exactly (upward 2^|T|, truncated upward
    sum_{j<=3} C(|T|, j), downward 2^(30-|T|)), on sampled subsets; no
    saturation or flush is counted."""
    import torch
    nbits = 30
    rng = np.random.default_rng(30)
    Ts = np.concatenate([rng.integers(0, 1 << nbits, 4096, dtype=np.int64),
                         np.array([0, (1 << nbits) - 1], dtype=np.int64)])
    pc = np.array([bin(int(T)).count("1") for T in Ts])
    idx = torch.from_numpy(Ts).cuda()
    f = torch.ones(1 << nbits, dtype=torch.float32, device="cuda")
    b = torch.full((1 << nbits,), BIAS, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    cases = [("zeta_up", -1, 2.0 ** pc),
             ("zeta_up", 3, np.array([sum(math.comb(int(p), j) for j in range(4)) for p in pc],
                                     dtype=float)),
             ("zeta_down", -1, 2.0 ** (nbits - pc))]
    for kind, d, want in cases:
        print(f"subset x32 2^30 kind={kind} d={d}", flush=True)
        f.fill_(1.0)
        b.fill_(BIAS)
        bn.subset_transform_x32(f, b, kind, d, cnt)
        torch.cuda.synchronize()
        got = _log2_of(f[idx].cpu().numpy(), b[idx].cpu().numpy())
        np.testing.assert_array_equal(got, np.log2(want))
    assert cnt.cpu().tolist() == [0, 0]
    del f, b
    torch.cuda.empty_cache()


def test_saturation_and_flush_counted():
    """Inputs at the top of the range overflow the byte and are clamped
    (counted in [0]); a transform of inputs at the bottom keeps them (no
    flush), since sums only grow."""
    import torch
    nbits = 12
    f = torch.full((1 << nbits,), 2.0 ** 31, dtype=torch.float32, device="cuda")
    b = torch.full((1 << nbits,), 255, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    print("subset x32 saturation", flush=True)
    bn.subset_transform_x32(f, b, "zeta_up", -1, cnt)
    torch.cuda.synchronize()
    c = cnt.cpu().tolist()
    bb = b.cpu().numpy()
    # entry T sums 2^|T| inputs of 2^31 * 2^(64 * 55): |T| >= 1 leaves the range
    assert bb[0] == 255 and np.all(bb[1:] == 255)
    assert c[0] == (1 << nbits) - 1 and c[1] == 0
    f.fill_(1.0)
    b.fill_(1)
    cnt.zero_()
    bn.subset_transform_x32(f, b, "zeta_down", -1, cnt)
    torch.cuda.synchronize()
    assert cnt.cpu().tolist() == [0, 0]
    got = _log2_of(f.cpu().numpy(), b.cpu().numpy())
    pc = np.array([bin(T).count("1") for T in range(1 << nbits)])
    np.testing.assert_array_equal(got, (nbits - pc) + 64.0 * (1 - BIAS))
