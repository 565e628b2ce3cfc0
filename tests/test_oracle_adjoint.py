"""Pins of the oracle's reverse mode (noise -> delta_1 -> D-form orders).

The adjoint is checked only against the oracle's forward map, which has its
own pins, through identities the adjoint cannot satisfy by construction:
  * Euler's theorem: delta_n is homogeneous of degree n in the noise w (the
    linear field is linear in w and order n is a product of n first-order
    factors, Eq. 10), so for J = sum_n <g_n, delta_n> the gradient obeys
    <w, dJ/dw> = sum_n n <g_n, delta_n> exactly;
  * the directional derivative along any v, from the forward map alone: J(w + t v)
    is a polynomial of degree <= nmax <= 5 in t, and the seven-point central
    difference is exact for polynomials of degree <= 6, so it equals <v, dJ/dw>
    up to rounding, whatever the step;
  * order 1 alone is linear, so its adjoint is its transpose: <g, delta_1[v]> = <dJ/dw, v>.
A dropped term, a wrong sign, a missing factor 2 or an untransposed matrix in
any step changes one of these.
"""
import numpy as np
import pytest

import oracle

NS, GAMMA = 0.96, 0.21


def _setup(n=16, box=100.0, seed=1, nmax=4):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    g = rng.standard_normal((nmax, n, n, n))
    v = rng.standard_normal((n, n, n))
    return rng, w, g, v


def _J(w, g, box, amp, nmax, c1, c2, dz=1.0):
    d1 = oracle.noise_field(w, box, amp, NS, GAMMA, dz, c1)
    dd, _, _, _ = oracle.orders(d1, box, nmax, c1, c2, spectra=False)
    return sum(float((g[i] * dd[i]).sum()) for i in range(nmax)), dd


def _stencil(f, h):
    return (-f(-3 * h) + 9 * f(-2 * h) - 45 * f(-h) + 45 * f(h) - 9 * f(2 * h) + f(3 * h)) / (60 * h)


@pytest.mark.parametrize("nmax", [1, 2, 3, 5])
def test_euler_identity(nmax):
    n, box = 16, 100.0
    _, w, g, _ = _setup(n, box, 2, nmax)
    amp = oracle.sigma8_amp(0.8, NS, GAMMA)
    cut = oracle.cut_n2max_strict(n)
    gw = oracle.adjoint(w, box, amp, NS, GAMMA, 0.8, nmax, cut, cut, g)
    _, dd = _J(w, g, box, amp, nmax, cut, cut, 0.8)
    rhs = sum((i + 1) * float((g[i] * dd[i]).sum()) for i in range(nmax))
    assert abs(float((w * gw).sum()) - rhs) <= 1e-12 * sum(abs((i + 1) * float((g[i] * dd[i]).sum()))
                                                            for i in range(nmax))


@pytest.mark.parametrize("n,box,nmax,c1,c2", [(16, 100.0, 3, None, None), (16, 100.0, 5, None, None),
                                              (12, 90.0, 4, None, None), (16, 120.0, 4, 20, 14),
                                              (16, 80.0, 3, 40, 40)])
def test_directional_derivative(n, box, nmax, c1, c2):
    """Includes a radix-3 grid, W1 != W2 and a cut beyond the 2/3 rule (aliasing on)."""
    _, w, g, v = _setup(n, box, 3, nmax)
    amp = oracle.sigma8_amp(0.8, NS, GAMMA)
    c = oracle.cut_n2max_strict(n)
    c1 = c if c1 is None else c1
    c2 = c if c2 is None else c2
    gw = oracle.adjoint(w, box, amp, NS, GAMMA, 1.0, nmax, c1, c2, g)
    fd = _stencil(lambda t: _J(w + t * v, g, box, amp, nmax, c1, c2)[0], 0.25)
    got = float((v * gw).sum())
    assert abs(got - fd) <= 1e-11 * max(abs(fd), 1e-300), (got, fd)


def test_order_one_is_transpose():
    n, box = 16, 100.0
    _, w, g, v = _setup(n, box, 4, 1)
    amp = oracle.sigma8_amp(0.8, NS, GAMMA)
    cut = oracle.cut_n2max_strict(n)
    gw = oracle.adjoint(w, box, amp, NS, GAMMA, 1.3, 1, cut, cut, g)
    dv = oracle.noise_field(v, box, amp, NS, GAMMA, 1.3, cut)
    lhs, rhs = float((g[0] * dv).sum()), float((gw * v).sum())
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # the gradient does not depend on w at order 1
    gw2 = oracle.adjoint(2 * w + 1, box, amp, NS, GAMMA, 1.3, 1, cut, cut, g)
    assert np.array_equal(gw, gw2)


def test_noise_field_reproduces_seeded_linear_field():
    """noise_field(w) with w the generator's cells is the seeded linear field."""
    n, box = 16, 100.0
    amp = oracle.sigma8_amp(0.8, NS, GAMMA)
    cut = oracle.cut_n2max_strict(n)
    w = np.array([oracle.unit_gaussian(5, 2, c) for c in range(n ** 3)]).reshape(n, n, n)
    a = oracle.noise_field(w, box, amp, NS, GAMMA, 0.7, cut)
    b = oracle.linear_field(n, box, amp, NS, GAMMA, 0.7, cut, 5, 2)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))
