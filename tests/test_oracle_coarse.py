"""Pins of the coarse-grid transfers (oracle/coarse.py): identities at r = 1,
exactness on bilinear functions, the transpose relation between the two
transfers, and the masked warm start."""
import numpy as np
import pytest

from oracle import cnn as OC
from oracle import coarse as OK


def bilinear(H, W, r, coef):
    """A bilinear function sampled on the fine grid and on the coarse grid."""
    a, b, c, d = coef
    Hf, Wf = r * (H - 1) + 1, r * (W - 1) + 1
    yf, xf = np.meshgrid(np.arange(Hf) / r, np.arange(Wf) / r, indexing="ij")
    yc, xc = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    q = lambda y, x: a + b * x + c * y + d * x * y
    return q(yf, xf)[None], q(yc, xc)[None].astype(np.float64)


@pytest.mark.parametrize("r", [2, 3, 4, 8])
def test_restrict_and_prolong_reproduce_bilinear_functions(r):
    fine, coarse = bilinear(6, 5, r, (0.3, -1.2, 0.7, 2.5))
    assert np.allclose(OK.restrict(fine, r), coarse, rtol=0, atol=1e-13)
    assert np.allclose(OK.prolong(coarse, r), fine, rtol=0, atol=1e-13)


def test_r1_is_the_identity():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9))
    assert np.array_equal(OK.restrict(x, 1), x)
    assert np.array_equal(OK.prolong(x, 1), x)


@pytest.mark.parametrize("r,H,W", [(2, 5, 7), (3, 6, 4), (8, 5, 6)])
def test_restrict_is_the_scaled_transpose_of_prolong(r, H, W):
    # <R x, y> = <x, P y> / r^2 for coarse y vanishing on the coarse boundary
    # (R's interior rows are P's columns over r^2: the tent weights times
    # r^2 are the hat functions' values at the fine nodes)
    rng = np.random.default_rng(r)
    Hf, Wf = r * (H - 1) + 1, r * (W - 1) + 1
    x = rng.standard_normal((1, Hf, Wf))
    y = np.zeros((1, H, W))
    y[:, 1:-1, 1:-1] = rng.standard_normal((1, H - 2, W - 2))
    lhs = float((OK.restrict(x, r) * y).sum())
    rhs = float((x * OK.prolong(y, r)).sum()) / r ** 2
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_restrict_of_a_fine_delta_is_the_hat_function():
    # a unit value on one fine node reaches the coarse nodes whose tents cover it
    r, H, W = 4, 5, 5
    x = np.zeros((1, r * (H - 1) + 1, r * (W - 1) + 1))
    x[0, 6, 9] = 1.0   # fine (6, 9) = coarse (1.5, 2.25)
    got = OK.restrict(x, r)[0]
    want = np.zeros((H, W))
    for i, wy in ((1, 2 / 16), (2, 2 / 16)):
        for j, wx in ((2, 3 / 16), (3, 1 / 16)):
            want[i, j] = wy * wx
    assert np.allclose(got, want, rtol=0, atol=1e-16)


def test_boundary_coarse_nodes_are_injected():
    rng = np.random.default_rng(3)
    r = 3
    x = rng.standard_normal((2, 3 * 4 + 1, 3 * 5 + 1))
    c = OK.restrict(x, r)
    for sl in ((slice(None), 0, slice(None)), (slice(None), -1, slice(None)),
               (slice(None), slice(None), 0), (slice(None), slice(None), -1)):
        assert np.array_equal(c[sl], x[:, ::r, ::r][sl])


def test_warm_start_prolong_masks_and_reduces_to_the_fine_warm_start():
    rng = np.random.default_rng(4)
    B, H, W = 2, 6, 7
    s = rng.standard_normal((B, H, W))
    out = rng.standard_normal((B, H, W)).astype(np.float32)
    sn = np.abs(s).max(axis=(1, 2))
    mask = np.zeros((H, W), np.uint8)
    mask[1:-1, 1:-1] = 1
    u1 = OK.warm_start_prolong(s, sn, out, mask, 1)
    assert np.allclose(u1, OC.warm_start(s, sn, out, mask), rtol=0, atol=1e-15)
    r = 4
    Hf, Wf = r * (H - 1) + 1, r * (W - 1) + 1
    sf = rng.standard_normal((B, Hf, Wf))
    mf = (rng.random((Hf, Wf)) < 0.7).astype(np.uint8)
    u = OK.warm_start_prolong(sf, sn, out, mf, r)
    assert np.all(u[:, mf == 0] == 0)
    # at coarse nodes the interpolation is the coarse value itself
    on = np.zeros((Hf, Wf), bool)
    on[::r, ::r] = True
    sel = on & (mf == 1)
    want = sf + sn[:, None, None] * np.repeat(np.repeat(out.astype(np.float64), r, 1), r, 2)[:, :Hf, :Wf]
    assert np.allclose(u[:, sel], want[:, sel], rtol=0, atol=1e-14)


def test_shape_check():
    with pytest.raises(ValueError):
        OK.restrict(np.zeros((1, 10, 9)), 4)
