"""Pins of the closure oracle (oracle/closure.py) against routes other than
itself: BF16 rounding on known values, the convolution against a circular
cross-correlation by FFT, the gradient against central finite differences,
and the first Adam step against its closed form.  CPU only."""
import numpy as np
import pytest

from oracle import closure as oc
from paper_1310_0998_amd import inputs


def test_bf16_rounding_known_values():
    one = 1.0
    assert oc.bf16(one) == 1.0
    assert oc.bf16(1.0 + 2.0 ** -8) == 1.0                       # tie -> even (1.0)
    assert oc.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6        # tie -> even (odd below)
    assert oc.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert oc.bf16(-3.140625) == -3.140625                        # 8 significant bits: exact
    assert oc.bf16(0.0) == 0.0
    assert oc.bf16(2.0 ** -130) == 2.0 ** -130                    # a power of two is exact
    x = np.random.default_rng(0).normal(size=1000)
    r = oc.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_conv_equals_fft_cross_correlation():
    rng = np.random.default_rng(1)
    B, M, ci, co = 2, 12, 3, 5
    X = rng.normal(size=(B, M, M, ci))
    W = rng.normal(size=(9, ci, co))
    b = rng.normal(size=co)
    Z = oc.conv(X, W, b)
    # Z[y, x] = sum_{dy, dx} X[y + dy, x + dx] K[dy, dx]: with the kernel placed at
    # (dy mod M, dx mod M), the DFT gives Z^ = X^ conj(K^)
    for o in range(co):
        for bb in range(B):
            acc = np.zeros((M, M))
            for c in range(ci):
                K = np.zeros((M, M))
                for tap in range(9):
                    dy, dx = tap // 3 - 1, tap % 3 - 1
                    K[dy % M, dx % M] = W[tap, c, o]
                acc += np.real(np.fft.ifft2(np.fft.fft2(X[bb, :, :, c]) * np.conj(np.fft.fft2(K))))
            assert np.allclose(Z[bb, :, :, o], acc + b[o], atol=1e-10)


@pytest.mark.parametrize("layers", [1, 3])
def test_gradient_matches_finite_differences(layers):
    rng = np.random.default_rng(2)
    c_in, width, M, B = 4, 16, 8, 2
    n = oc.param_count(c_in, width, layers)
    w = rng.normal(0.0, 0.3, size=n)
    u = rng.normal(size=(B, M, M, 2))
    cond = rng.normal(size=(B, c_in - 2))
    tgt = rng.normal(size=(B, M, M, 2))
    loss, g = oc.loss_and_gradient(w, u, cond, tgt, c_in, width, layers, bf16_ops=False)
    h = 1e-6
    for i in rng.choice(n, size=40, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        lp, _ = oc.loss_and_gradient(wp, u, cond, tgt, c_in, width, layers, bf16_ops=False)
        lm, _ = oc.loss_and_gradient(wm, u, cond, tgt, c_in, width, layers, bf16_ops=False)
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9), i


def test_zero_network_is_persistence():
    # all-zero parameters: pred = u exactly, the loss is the persistence error
    rng = np.random.default_rng(3)
    u = rng.normal(size=(1, 8, 8, 2))
    tgt = rng.normal(size=(1, 8, 8, 2))
    w = np.zeros(oc.param_count(4, 16, 2))
    pred, _ = oc.forward(w, u, np.zeros((1, 2)), 4, 16, 2)
    assert (pred == u).all()
    loss, _ = oc.loss_and_gradient(w, u, np.zeros((1, 2)), tgt, 4, 16, 2)
    assert loss == pytest.approx(((u - tgt) ** 2).mean(), rel=1e-14)


def test_adam_first_step_closed_form():
    # from zero moments the bias-corrected first step is lr g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w0 = np.array([1.0, 1.0, 1.0, 1.0])
    w, m, v = oc.adam(w0, np.zeros(4), np.zeros(4), g, 1, 0.01, 0.9, 0.999, 1e-8)
    assert w == pytest.approx(w0 - 0.01 * g / (np.abs(g) + 1e-8), rel=1e-12, abs=1e-15)


def test_init_recipe():
    w = inputs.closure_init(5, 4, 32, 4)
    assert w.dtype == np.float32 and len(w) == oc.param_count(4, 32, 4)
    assert (w == inputs.closure_init(5, 4, 32, 4)).all()
