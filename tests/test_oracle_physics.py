"""Pins of the oracle's physics (Sec. 2) against closed forms and special cases."""
import math

import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O

G = 1.4


def _state(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])


def test_euler_flux_hand_values():
    w = _state(2.0, 3.0, -1.0, 5.0)
    f = O.euler_flux(w, G)
    E = w[3]
    assert np.allclose(f[0], [6.0, 2 * 9 + 5, 2 * 3 * -1, 3 * (E + 5)])
    assert np.allclose(f[1], [-2.0, 2 * 3 * -1, 2 * 1 + 5, -1 * (E + 5)])


@pytest.mark.parametrize("theta", [0.0, 0.4, 2.0, 3.9])
def test_normal_jacobian_eigenvalues(theta):
    """The eigenvalues u_n - c, u_n, u_n, u_n + c fix the momentum flux rho v (x) v + p Id."""
    w = _state(1.3, 0.7, -0.2, 0.9)
    n = np.array([math.cos(theta), math.sin(theta)])
    ev = np.sort(np.linalg.eigvals(O.normal_flux_jacobian(w, n, G)).real)
    un = 0.7 * n[0] - 0.2 * n[1]
    c = math.sqrt(G * 0.9 / 1.3)
    assert np.allclose(ev, np.sort([un - c, un, un, un + c]), atol=1e-12)


def _phys(mu=0.01, pr=0.72):
    winf = hi.free_stream(0.5, 2.0)
    return O.Physics("ns", G, winf, 1.5, mu, pr)


def test_viscous_flux_shear_and_heat():
    ph = _phys()
    rho, u, v, p = 1.1, 0.3, -0.2, 0.8
    w = _state(rho, u, v, p)
    # pure shear du/dy = s (momentum gradient rho s), everything else uniform
    s = 0.7
    q = np.zeros((2, 4))
    q[1, 1] = rho * s
    q[1, 3] = rho * u * s          # dE/dy from the kinetic energy only
    fv = O.viscous_flux(w, q, ph)
    assert np.allclose(fv[0], [0, 0, ph.mu * s, v * ph.mu * s], atol=1e-15)
    assert np.allclose(fv[1], [0, ph.mu * s, 0, u * ph.mu * s], atol=1e-15)
    # heat conduction: velocity zero, internal energy gradient de/dx = t
    w0 = _state(rho, 0.0, 0.0, p)
    t = 0.3
    q = np.zeros((2, 4))
    q[0, 3] = rho * t
    fv = O.viscous_flux(w0, q, ph)
    assert np.allclose(fv[0], [0, 0, 0, ph.mu * G / ph.prandtl * t], atol=1e-15)
    assert np.allclose(fv[1], 0, atol=1e-15)
    # dilatation: du/dx = d, tau_xx = 4/3 mu d, tau_yy = -2/3 mu d
    d = 0.5
    q = np.zeros((2, 4))
    q[0, 1] = rho * d
    q[0, 3] = rho * u * d
    fv = O.viscous_flux(w, q, ph)
    assert np.allclose(fv[0][1], 4.0 / 3.0 * ph.mu * d)
    assert np.allclose(fv[1][2], -2.0 / 3.0 * ph.mu * d)


@pytest.mark.parametrize("mach,theta,nneg", [
    (0.5, 0.0, 1),              # subsonic outflow: one incoming characteristic
    (0.5, math.pi, 3),          # subsonic inflow: three incoming
    (1.5, 0.0, 0),              # supersonic outflow: all from the interior
    (1.5, math.pi, 4),          # supersonic inflow: all from the free stream
])
def test_farfield_projector_cases(mach, theta, nneg):
    winf = hi.free_stream(mach, 0.0)
    n = np.array([math.cos(theta), math.sin(theta)])
    P = O.farfield_projector(winf, n, G)
    A = O.normal_flux_jacobian(winf, n, G)
    assert np.allclose(P @ P, P, atol=1e-12)
    assert np.allclose(P @ A, A @ P, atol=1e-12)
    assert round(np.trace(P)) == 4 - nneg
    # the free stream is a fixed point of the boundary map
    wb = P @ winf + (np.eye(4) - P) @ winf
    assert np.allclose(wb, winf)


def test_farfield_tangential_flow_takes_interior_value():
    """u_n = 0: the repeated eigenvalue ties at zero and is taken from the interior."""
    winf = hi.free_stream(0.5, 0.0)
    P = O.farfield_projector(winf, np.array([0.0, 1.0]), G)
    assert round(np.trace(P)) == 3
