"""Pins of the oracle's 3x3x3 convolutions (CPU): a single-channel case equals
scipy.ndimage.correlate with zero boundary; conv3_dgrad is the transpose of
conv3 (dot-product identity); conv3_wgrad is the derivative of <conv3(x;w), dy>
with respect to w (the map is linear in w, so central differences are exact
up to rounding) and db the derivative with respect to b."""
import numpy as np
import scipy.ndimage as ndi

from paper_2512_21180_amd import workloads as W


def test_single_channel_matches_scipy(oracle):
    r = W.rng(1)
    x = r.standard_normal((1, 5, 7, 9))
    w = r.standard_normal((1, 1, 3, 3, 3))
    ref = ndi.correlate(x[0], w[0, 0], mode="constant", cval=0.0)
    got = oracle.conv3(x, w)[0]
    assert np.max(np.abs(got - ref)) < 1e-12


def test_dgrad_is_transpose(oracle):
    r = W.rng(2)
    x = r.standard_normal((3, 4, 6, 5))
    w = r.standard_normal((4, 3, 3, 3, 3))
    dy = r.standard_normal((4, 4, 6, 5))
    lhs = float(np.vdot(oracle.conv3(x, w), dy))
    rhs = float(np.vdot(x, oracle.conv3_dgrad(dy, w)))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_wgrad_is_weight_derivative(oracle):
    r = W.rng(3)
    x = r.standard_normal((2, 3, 4, 5))
    w = r.standard_normal((3, 2, 3, 3, 3))
    b = r.standard_normal(3)
    dy = r.standard_normal((3, 3, 4, 5))
    dw, db = oracle.conv3_wgrad(x, dy)
    f = lambda ww, bb: float(np.vdot(oracle.conv3(x, ww, bb), dy))
    for idx in [(0, 0, 0, 0, 0), (2, 1, 1, 2, 0), (1, 0, 2, 2, 2), (0, 1, 1, 1, 1)]:
        e = np.zeros_like(w)
        e[idx] = 0.5
        fd = (f(w + e, b) - f(w - e, b)) / 1.0
        assert abs(fd - dw[idx]) < 1e-9 * max(1.0, abs(fd))
    for c in range(3):
        e = np.zeros(3)
        e[c] = 0.5
        assert abs((f(w, b + e) - f(w, b - e)) - db[c]) < 1e-9 * max(1.0, abs(db[c]))
