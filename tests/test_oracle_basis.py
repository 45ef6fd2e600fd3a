"""Pins of the oracle's polynomial bases and quadrature rules against closed forms.

Reference-element and basis readings: Sec. 3.1 (inner products) and Sec. 4.3
(hierarchical Dubiner basis)."""
import math

import numpy as np
import pytest
import scipy.special

from oracle import hdg_oracle as O


@pytest.mark.parametrize("n,a,b", [(0, 0, 0), (1, 0, 0), (4, 0, 0), (3, 3, 0), (5, 7, 0), (2, 11, 0)])
def test_jacobi_matches_scipy(n, a, b):
    x = np.linspace(-0.99, 0.99, 37)
    assert np.allclose(O.jacobi(n, a, b, x), scipy.special.eval_jacobi(n, a, b, x), rtol=1e-13, atol=1e-13)


def _exact_monomial(a, b):
    # integral over {xi, eta >= -1, xi + eta <= 0} of (1+xi)^a (1+eta)^b
    return 2.0 ** (a + b + 2) * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_triangle_rule_exact_to_2p_plus_2(p):
    xi, eta, w = O.triangle_rule(p)
    assert abs(w.sum() - 2.0) < 1e-14
    for a in range(2 * p + 3):
        for b in range(2 * p + 3 - a):
            q = np.sum(w * (1 + xi) ** a * (1 + eta) ** b)
            assert abs(q - _exact_monomial(a, b)) < 1e-13 * max(1.0, _exact_monomial(a, b))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_dubiner_orthonormal_and_complete(p):
    xi, eta, w = O.triangle_rule(p + 2)
    phi = O.dubiner(p, xi, eta)
    M = (phi * w) @ phi.T
    assert np.allclose(M, np.eye(O.n_modes(p)), atol=1e-13)
    # spans all polynomials of degree <= p: monomials are reproduced exactly
    mono = np.array([(1 + xi) ** a * (1 + eta) ** b for a in range(p + 1) for b in range(p + 1 - a)])
    coef = (mono * w) @ phi.T
    assert np.allclose(coef @ phi, mono, atol=1e-12)


@pytest.mark.parametrize("p", [2, 4])
def test_dubiner_hierarchical(p):
    """Modes of degree k are orthogonal to every polynomial of degree < k."""
    xi, eta, w = O.triangle_rule(p + 2)
    phi = O.dubiner(p, xi, eta)
    pairs = O.mode_pairs(p)
    for idx, (i, j) in enumerate(pairs):
        k = i + j
        for a in range(k):
            for b in range(k - a):
                assert abs(np.sum(w * phi[idx] * (1 + xi) ** a * (1 + eta) ** b)) < 1e-13
    # the lower modes are the basis of degree p-1
    assert np.allclose(O.dubiner(p - 1, xi, eta), phi[: O.n_modes(p - 1)], atol=1e-15)


@pytest.mark.parametrize("p", [1, 3, 5])
def test_dubiner_gradient_vs_finite_difference(p):
    rng = np.random.default_rng(0)
    u = rng.uniform(0.05, 0.9, 20)
    v = rng.uniform(0.05, 0.9, 20) * (1 - u)
    xi, eta = 2 * u - 1, 2 * v - 1
    g = O.dubiner_grad(p, xi, eta)
    h = 1e-6
    fx = (O.dubiner(p, xi + h, eta) - O.dubiner(p, xi - h, eta)) / (2 * h)
    fy = (O.dubiner(p, xi, eta + h) - O.dubiner(p, xi, eta - h)) / (2 * h)
    assert np.allclose(g[0], fx, atol=1e-7)
    assert np.allclose(g[1], fy, atol=1e-7)


@pytest.mark.parametrize("p", [0, 1, 3, 6])
def test_face_basis_orthonormal(p):
    s, w = O.gauss(p + 2)
    psi = O.legendre_face(p, s)
    assert np.allclose((psi * w) @ psi.T, np.eye(p + 1), atol=1e-14)
    # Gauss with n points integrates s^(2n-1) exactly
    for k in range(2 * (p + 2)):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * s ** k) - exact) < 1e-14
