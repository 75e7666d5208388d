"""Pins of the oracle's kernels and quadrature rules against mathematics it does not use.

Kernels (Section 2.1, eq_potential, Eq_Ls): finite differences of the Green's functions,
the direct differences K = dGk - dG0 at moderate r, the kappa -> 0 limit.
Quadrature (Sections 2.2, 2.3): exactness on monomials of the unit right triangle,
int r^a s^b = a! b! / (a + b + 2)!, and a singular integral with a closed form.
"""
import math

import numpy as np
import pytest

from oracle import FOUR_PI
from oracle import kernels as K
from oracle import quadrature as Q


def _rand_unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_green_derivatives_match_finite_differences():
    rng = np.random.default_rng(11)
    kappa = 0.7
    for _ in range(20):
        x = rng.standard_normal(3)
        y = x + rng.standard_normal(3) * 0.8 + 0.3
        nx, ny = _rand_unit(rng, 2)
        h = 1e-4
        (g0y, g0x, g0xy), (gky, gkx, gkxy) = K.green_derivatives(x, nx, y, ny, kappa)
        # first normal derivatives (central differences)
        fd0y = (K.G0(x, y + h * ny) - K.G0(x, y - h * ny)) / (2 * h)
        fd0x = (K.G0(x + h * nx, y) - K.G0(x - h * nx, y)) / (2 * h)
        fdky = (K.Gk(x, y + h * ny, kappa) - K.Gk(x, y - h * ny, kappa)) / (2 * h)
        fdkx = (K.Gk(x + h * nx, y, kappa) - K.Gk(x - h * nx, y, kappa)) / (2 * h)
        for a, b in ((g0y, fd0y), (g0x, fd0x), (gky, fdky), (gkx, fdkx)):
            assert abs(a - b) <= 1e-6 * (abs(b) + 1e-3)

        # mixed second derivative
        def d_dy(G, xx):
            return (G(xx, y + h * ny) - G(xx, y - h * ny)) / (2 * h)

        g0 = lambda a, b: K.G0(a, b)
        gk = lambda a, b: K.Gk(a, b, kappa)
        fd0xy = (d_dy(g0, x + h * nx) - d_dy(g0, x - h * nx)) / (2 * h)
        fdkxy = (d_dy(gk, x + h * nx) - d_dy(gk, x - h * nx)) / (2 * h)
        assert abs(g0xy - fd0xy) <= 1e-5 * (abs(fd0xy) + 1e-2)
        assert abs(gkxy - fdkxy) <= 1e-5 * (abs(fdkxy) + 1e-2)


@pytest.mark.parametrize("kappa", [0.1257, 1.0, 3.0])
def test_kernels_equal_direct_differences(kappa):
    """K1..K4 from the cancellation-free form equal the printed differences (Eq_Ls)."""
    rng = np.random.default_rng(12)
    eps = 80.0
    x = rng.standard_normal((200, 3))
    y = x + _rand_unit(rng, 200) * rng.uniform(0.5, 5.0, size=(200, 1))
    nx, ny = _rand_unit(rng, 200), _rand_unit(rng, 200)
    K1, K2, K3, K4 = K.kernels(x, nx, y, ny, kappa, eps)
    (g0y, g0x, g0xy), (gky, gkx, gkxy) = K.green_derivatives(x, nx, y, ny, kappa)
    np.testing.assert_allclose(K1, K.G0(x, y) - K.Gk(x, y, kappa), rtol=1e-12)
    np.testing.assert_allclose(K2, eps * gky - g0y, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(K3, g0x - gkx / eps, rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(K4, gkxy - g0xy, rtol=1e-9, atol=1e-13)


def test_series_and_direct_forms_agree_at_the_switch():
    z = np.linspace(0.45, 0.55, 101)
    direct1 = 1.0 - np.exp(-z) * (1.0 + z)
    direct2 = 3.0 - np.exp(-z) * (3.0 + 3.0 * z + z * z)
    np.testing.assert_allclose(K.f1(z), direct1, rtol=1e-14)
    np.testing.assert_allclose(K.f2(z), direct2, rtol=1e-14)
    # leading Taylor terms at tiny z
    z = np.array([1e-6, 1e-4])
    np.testing.assert_allclose(K.f1(z), z * z / 2 - z ** 3 / 3 + z ** 4 / 8, rtol=1e-10)
    np.testing.assert_allclose(K.f2(z), z * z / 2 - z ** 4 / 8 + z ** 5 / 15, rtol=1e-10)


def test_kappa_zero_limit():
    """kappa = 0: K1 = K4 = 0, K2 = (eps-1) dG0/dny, K3 = (1-1/eps) dG0/dnx."""
    rng = np.random.default_rng(13)
    x = rng.standard_normal((50, 3))
    y = x + rng.standard_normal((50, 3))
    nx, ny = _rand_unit(rng, 50), _rand_unit(rng, 50)
    K1, K2, K3, K4 = K.kernels(x, nx, y, ny, 0.0, 80.0)
    (g0y, g0x, _), _ = K.green_derivatives(x, nx, y, ny, 0.0)
    assert np.all(K1 == 0.0) and np.all(K4 == 0.0)
    np.testing.assert_allclose(K2, 79.0 * g0y, rtol=1e-13)
    np.testing.assert_allclose(K3, (1 - 1 / 80.0) * g0x, rtol=1e-13)


def test_small_r_limit_of_k4():
    """As r -> 0, K4 ~ kappa^2 / (8 pi r) [(d^.nx)(d^.ny) - nx.ny] (weakly singular)."""
    kappa = 0.5
    nx = np.array([0.0, 0.0, 1.0])
    ny = np.array([0.0, 0.6, 0.8])
    dhat = np.array([0.6, 0.0, 0.8])
    for r in (1e-3, 1e-4):
        x = r * dhat
        _, _, _, K4 = K.kernels(x, nx, np.zeros(3), ny, kappa, 80.0)
        lead = kappa ** 2 / (8 * math.pi * r) * (np.dot(dhat, nx) * np.dot(dhat, ny) - np.dot(nx, ny))
        assert abs(K4 / lead - 1.0) < 5 * kappa * r + 1e-9


def _monomial(a, b):
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def test_gauss_radau_triangle_exact_to_degree_3():
    r, s, w = Q.gauss_radau_triangle()
    assert r.shape == (4,) and abs(w.sum() - 0.5) < 1e-16
    for a in range(4):
        for b in range(4 - a):
            assert abs(np.sum(w * r ** a * s ** b) - _monomial(a, b)) < 1e-16
    errs = [abs(np.sum(w * r ** a * s ** (4 - a)) - _monomial(a, 4 - a)) for a in range(5)]
    assert max(errs) > 1e-6          # degree 4 is not integrated exactly
    # the published node and weight values
    np.testing.assert_allclose(sorted(w), [0.0909793091] * 2 + [0.1590206909] * 2, atol=1e-10)
    assert np.all(np.isclose(r, s[[1, 0, 3, 2]]))      # symmetric under r <-> s


def test_gauss_legendre_01():
    x, w = Q.gauss_legendre_01(4)
    np.testing.assert_allclose(x, [0.0694318442, 0.3300094782, 0.6699905218, 0.9305681558], atol=1e-10)
    np.testing.assert_allclose(w, [(18 - 30 ** 0.5) / 72, (18 + 30 ** 0.5) / 72,
                                   (18 + 30 ** 0.5) / 72, (18 - 30 ** 0.5) / 72], rtol=1e-14)
    for k in range(8):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-15
    assert abs(np.sum(w * x ** 8) - 1.0 / 9) > 1e-8


def test_duffy_rule():
    r, s, w = Q.duffy_gauss_legendre(4)
    assert r.shape == (16,) and abs(w.sum() - 0.5) < 1e-15
    for a in range(7):
        for b in range(7 - a):
            assert abs(np.sum(w * r ** a * s ** b) - _monomial(a, b)) < 1e-15
    # int_T (r^2 + s^2)^(-1/2) = sqrt(2) ln(1 + sqrt(2)); the error falls as N_GL grows
    exact = math.sqrt(2.0) * math.log(1.0 + math.sqrt(2.0))
    errs = []
    for n in (2, 4, 8):
        r, s, w = Q.duffy_gauss_legendre(n)
        errs.append(abs(np.sum(w / np.sqrt(r * r + s * s)) - exact))
    assert errs[1] < errs[0] and errs[2] < errs[1] and errs[1] < 1e-3 * exact
