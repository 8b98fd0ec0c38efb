"""The polynomial tap weights compiled into the non-uniform FFT kernels
(csrc/nu_weights.h) are the ones gen_nu_weights.py fits, and they reproduce
the exponential-of-semicircle kernel: every tap within 2e-7 of psi at offsets
across [-1/2, 1/2], the mirrored taps equal, and the 7 weights summing to the
kernel's discrete partition of unity within the same bound."""
import importlib.util
import os

import numpy as np

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


def test_header_is_current():
    g = _gen()
    E, O, err = g.fit()
    with open(os.path.join(CSRC, "nu_weights.h")) as f:
        assert f.read() == g.header(E, O, err)


def test_weights_follow_the_kernel():
    g = _gen()
    E, O, _ = g.fit()
    # the coefficients as the device sees them (single precision)
    E32, O32 = E.astype(np.float32).astype(np.float64), O.astype(np.float32).astype(np.float64)
    u = np.random.default_rng(3).uniform(-0.5, 0.5, 5000)
    w = _weights(E32, O32, u)
    exact = np.stack([g.psi(u + 3 - t) for t in range(7)])
    assert np.max(np.abs(w - exact)) < 2e-7
    assert np.allclose(_weights(E32, O32, -u)[::-1], w, atol=1e-12)
    # the taps of all grid points near x sum to sum_l psi(x - l) for any x
    assert np.max(np.abs(w.sum(axis=0) - exact.sum(axis=0))) < 2e-7
