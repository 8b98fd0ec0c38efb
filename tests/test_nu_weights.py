"""The polynomial tap weights compiled into the non-uniform FFT kernels
(csrc/nu_weights.h) are the ones gen_nu_weights.py fits, and they reproduce
the exponential-of-semicircle kernel: every tap within 1.5e-6 of psi at
offsets across [-1/2, 1/2], the mirrored taps equal, and the 7 weights
summing to the kernel's discrete partition of unity within the same bound.
A type-2 sum through them (one DFT of the deconvolved modes to the
oversampled grid, then 7 taps per frequency) stays within the kernel's own
aliasing error of the direct sum, as it does with exact psi values."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2311_13182_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_nu_weights", os.path.join(CSRC, "gen_nu_weights.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _weights(E, O, u):
    u2 = u * u
    w = np.zeros((7,) + np.shape(u))
    for t in range(4):
        e = np.polyval(E[t][::-1], u2)
        if t == 3:
            w[3] = e
        else:
            o = u * np.polyval(O[t][::-1], u2)
            w[t], w[6 - t] = e + o, e - o
    return w


def _device_coefficients(g):
    # the coefficients as the device sees them (single precision)
    E, O, _ = g.fit()
    return E.astype(np.float32).astype(np.float64), O.astype(np.float32).astype(np.float64)


def test_header_is_current():
    g = _gen()
    E, O, err = g.fit()
    with open(os.path.join(CSRC, "nu_weights.h")) as f:
        assert f.read() == g.header(E, O, err)


def test_weights_follow_the_kernel():
    g = _gen()
    E32, O32 = _device_coefficients(g)
    u = np.random.default_rng(3).uniform(-0.5, 0.5, 5000)
    w = _weights(E32, O32, u)
    exact = np.stack([g.psi(u + 3 - t) for t in range(7)])
    assert np.max(np.abs(w - exact)) < 1.5e-6
    assert np.allclose(_weights(E32, O32, -u)[::-1], w, atol=1e-12)
    # the taps of all grid points near x sum to sum_l psi(x - l) for any x
    assert np.max(np.abs(w.sum(axis=0) - exact.sum(axis=0))) < 1.5e-6


@pytest.mark.parametrize("S", [64, 256])
def test_type2_sum_through_the_weights(S):
    g = _gen()
    E32, O32 = _device_coefficients(g)
    M = 2 * S
    rng = np.random.default_rng(S)
    h = rng.standard_normal(S) + 1j * rng.standard_normal(S)
    sp = np.arange(S) - S // 2
    # Psi(k / M) = integral of psi(d) cos(2 pi k d / M) over the support
    d = np.linspace(-3.5, 3.5, 140001)
    Psi = (np.cos(2 * np.pi * np.outer(sp, d) / M) @ g.psi(d)) * (d[1] - d[0])
    L = np.arange(-M // 2 - 3, M // 2 + 4)
    rows = np.exp(2j * np.pi * np.outer(L, sp) / M) @ (h / Psi)
    gs = rng.uniform(-0.5, 0.5, 2000)
    direct = np.exp(2j * np.pi * np.outer(gs, sp)) @ h
    x = gs * M
    xr = np.rint(x)
    taps = rows[(xr + M // 2).astype(int)[:, None] + np.arange(7)]
    poly = np.sum(_weights(E32, O32, x - xr).T * taps, axis=1)
    exact = np.sum(np.stack([g.psi(x - xr + 3 - t) for t in range(7)]).T * taps, axis=1)
    h1 = np.sum(np.abs(h))
    assert np.max(np.abs(exact - direct)) / h1 < 5e-7   # the kernel's aliasing error
    assert np.max(np.abs(poly - direct)) / h1 < 5e-7
    assert np.max(np.abs(poly - exact)) / h1 < 2e-7
