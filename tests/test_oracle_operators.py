"""Pins of the oracle's one-line finite-difference operators and of the
Theta scaling rule against closed forms (Sec. 2.1 and Sec. 3.3 of the paper).

D+, D- (eq. of the biased operators) come from cubic reconstructions, so they
are exact on cubics; D_c is their mean and is exact on quartics; the compact
D^2(K,Z) of the B matrix is exact whenever deg K + deg Z <= 5 and, for
constant K, is the textbook five-point fourth-order second derivative on the
half spacing.  Polynomial inputs make every one of these statements exact.
"""
import numpy as np
import pytest

import oracle as O

H = 0.137          # cell size; the lattice spacing is H/2
X0 = 0.41
OFF = np.arange(-2, 3) * H / 2


def poly(coefs):
    return np.polynomial.Polynomial(coefs)


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_biased_operators_exact_on_cubics(deg):
    rng = np.random.default_rng(deg)
    p = poly(rng.normal(size=deg + 1))
    z = p(X0 + OFF)
    d = p.deriv()(X0)
    assert O.op("dplus", z, H) == pytest.approx(d, abs=1e-12)
    assert O.op("dminus", z, H) == pytest.approx(d, abs=1e-12)
    assert O.op("dc", z, H) == pytest.approx(d, abs=1e-12)


def test_biased_operator_leading_errors():
    # on x^4 the biased operators err by +-dx^3/4 = +-dx^3 f''''/96
    p = poly([0, 0, 0, 0, 1])
    z = p(X0 + OFF)
    d = p.deriv()(X0)
    assert O.op("dplus", z, H) - d == pytest.approx(H ** 3 / 4, rel=1e-9)
    assert O.op("dminus", z, H) - d == pytest.approx(-H ** 3 / 4, rel=1e-9)
    # the central operator is exact on quartics, errs on x^5 by -dx^4/4
    assert O.op("dc", z, H) == pytest.approx(d, abs=1e-12)
    p5 = poly([0, 0, 0, 0, 0, 1])
    z5 = p5(X0 + OFF)
    assert O.op("dc", z5, H) - p5.deriv()(X0) == pytest.approx(-H ** 4 / 4, rel=1e-8)


def test_central_is_mean_and_dissipation_identity():
    rng = np.random.default_rng(7)
    for _ in range(20):
        z = rng.normal(size=5)
        dp, dm, dc = O.op("dplus", z, H), O.op("dminus", z, H), O.op("dc", z, H)
        assert dc == pytest.approx(0.5 * (dp + dm), abs=1e-12)
        # (3 dx)(D+ - D-) is the fourth difference (1,-4,6,-4,1)
        assert 3 * H * (dp - dm) == pytest.approx(z[0] - 4 * z[1] + 6 * z[2] - 4 * z[3] + z[4], abs=1e-12)


@pytest.mark.parametrize("dk,dz", [(0, 2), (0, 5), (1, 4), (2, 3), (3, 2), (4, 1), (5, 0), (2, 2), (1, 1)])
def test_compact_second_derivative_exact(dk, dz):
    rng = np.random.default_rng(10 * dk + dz)
    for _ in range(5):
        k = poly(rng.normal(size=dk + 1))
        z = poly(rng.normal(size=dz + 1))
        exact = (k * z.deriv()).deriv()(X0)
        val = O.op_d2(k(X0 + OFF), z(X0 + OFF), H)
        assert val == pytest.approx(exact, rel=1e-10, abs=1e-9)


def test_compact_second_derivative_not_exact_beyond_degree_five():
    k = poly([0, 0, 0, 1])
    z = poly([0, 0, 0, 1])
    exact = (k * z.deriv()).deriv()(X0)
    val = O.op_d2(k(X0 + OFF), z(X0 + OFF), H)
    assert abs(val - exact) > 1e-6


def test_compact_second_derivative_constant_k_is_textbook_stencil():
    rng = np.random.default_rng(3)
    h = H / 2
    for _ in range(10):
        z = rng.normal(size=5)
        kc = rng.uniform(0.5, 2.0)
        textbook = kc * (-z[0] + 16 * z[1] - 30 * z[2] + 16 * z[3] - z[4]) / (12 * h * h)
        assert O.op_d2(np.full(5, kc), z, H) == pytest.approx(textbook, rel=1e-11)


def test_compact_second_derivative_kills_constants():
    rng = np.random.default_rng(4)
    for _ in range(10):
        k = rng.normal(size=5)
        assert abs(O.op_d2(k, np.full(5, rng.normal()), H)) < 1e-10


def test_theta_rule():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        zL = rng.uniform(1e-14, 2.0)
        zH = rng.uniform(-3.0, 3.0)
        eps = min(1e-13, zL)
        th = O.theta(zL, zH, eps)
        assert 0.0 <= th <= 1.0
        for v in np.linspace(0.0, th, 7):
            assert (1 - v) * zL + v * zH >= eps * (1 - 1e-9) - 1e-15
        if zH >= eps:
            assert th == 1.0
        else:
            # the largest admissible blend: the segment reaches eps exactly
            assert (1 - th) * zL + th * zH == pytest.approx(eps, abs=1e-14)
