"""Pins of the oracle's shock capturing (Sec. 3.2): the artificial viscosity eps_K in closed
form for a linear state, its absence at the free stream, the volume term's structure in the
Newton matrix (eps_K held fixed) and its conservation."""
import math

import numpy as np

import hdg_inputs as hi
from oracle import hdg_oracle as O


def _project(mesh, e, fun):
    """L2 projection of fun(x, y) -> (4, Q) onto the element's basis, by the mass system."""
    g = mesh.geom(e)
    vals = fun(g.xq[:, 0], g.xq[:, 1])
    M = (g.phi * g.wq[None, :]) @ g.phi.T
    return np.linalg.solve(M, (g.phi * g.wq[None, :]) @ vals.T).T


def _one_triangle(eps0=0.2, degree=1):
    c = hi.Case(name="one", physics="euler", ng=1, xy=np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
                tri=np.array([[0, 1, 2]], dtype=np.int32), degree=np.array([degree], dtype=np.int8),
                mach=0.5, aoa_deg=0.0, amp=0.0, sc_eps0=eps0)
    c.W = np.zeros((1, 4, hi.n_modes(degree)))
    return c


def test_viscosity_closed_form_for_a_linear_density():
    """rho = 1 + s x at constant u = 0.5, v = 0, p = 1/gamma: div f_c = s (u, u^2, u v, u |v|^2 / 2),
    constant, so eps = eps_0 (h / p)^2 d with h = sqrt 2 (the hypotenuse) and p = 1."""
    c = _one_triangle()
    m = O.Mesh(c, O.make_physics(c))
    gam, u, s = 1.4, 0.5, 0.1
    p = 1.0 / gam

    def state(x, y):
        rho = 1.0 + s * x
        return np.stack([rho, rho * u, 0.0 * x, p / (gam - 1.0) + 0.5 * rho * u * u])
    W = _project(m, 0, state)
    d = s * (u + u * u + 0.0 + 0.5 * u ** 3)
    assert abs(d - 0.08125) < 1e-15
    assert abs(O.shock_viscosity(m, 0, W) - 0.2 * 2.0 * d) < 1e-14


def test_free_stream_has_no_viscosity():
    c = hi.make_case("euler", 3, [1, 2, 3], 0.5, 2.0, 0.0, seed=9, free_stream_only=True)
    c.sc_eps0 = 0.2
    m = O.Mesh(c, O.make_physics(c))
    for e in range(c.n_elements):
        n = hi.n_modes(int(c.degree[e]))
        assert O.shock_viscosity(m, e, c.W[e, :, :n]) < 1e-14


def test_volume_term_in_the_newton_matrix_and_conservation():
    """With eps_K held fixed, switching shock capturing on adds eps_K times the stiffness
    matrix to every field's diagonal block of A_K and nothing elsewhere; the term leaves the
    constant-mode rows (the element's conservation statement) unchanged."""
    c0 = hi.make_case("euler", 3, [1, 2, 3], 0.8, 1.25, 8e-2, seed=41)
    c1 = hi.make_case("euler", 3, [1, 2, 3], 0.8, 1.25, 8e-2, seed=41)
    c1.sc_eps0 = 0.2
    s0 = O.State(O.Mesh(c0, O.make_physics(c0)), c0.W, c0.lam)
    s1 = O.State(O.Mesh(c1, O.make_physics(c1)), c1.W, c1.lam)
    seen = 0.0
    for e in range(0, c0.n_elements, 2):
        b0, b1 = O.element_blocks(s0, e), O.element_blocks(s1, e)
        for name in ("B", "C", "D", "rl"):
            assert np.array_equal(getattr(b0, name), getattr(b1, name)), name
        n = hi.n_modes(int(c0.degree[e]))
        g = s1.mesh.geom(e)
        eps = O.shock_viscosity(s1.mesh, e, c1.W[e, :, :n])
        stiff = np.einsum("q,dnq,dmq->nm", g.wq, g.dphi, g.dphi)
        dA = b1.A - b0.A
        assert np.abs(dA - np.kron(np.eye(4), eps * stiff)).max() < 1e-12 * max(1.0, eps * np.abs(stiff).max())
        dr = b1.r - b0.r
        assert np.abs(dr.reshape(4, n)[:, 0]).max() < 1e-15          # constant-mode rows
        assert np.abs(dr + eps * (np.kron(np.eye(4), stiff) @ c1.W[e, :, :n].reshape(-1))).max() < 1e-14
        seen = max(seen, eps)
    assert seen > 1e-4       # the workload's state does switch the term on


def test_viscosity_scales_with_the_mesh_as_stated():
    """eps_K is proportional to h~^(2 - beta) for a fixed state: halving the triangle at fixed
    d(w) (a linear state) scales eps by 2^-(2 - beta) for beta = 0 and 1."""
    for beta, factor in ((0.0, 0.25), (1.0, 0.5)):
        vals = []
        for scale in (1.0, 0.5):
            c = _one_triangle()
            c.sc_beta = beta
            c.xy = c.xy * scale
            m = O.Mesh(c, O.make_physics(c))

            def state(x, y):
                rho = 1.0 + 0.1 * x
                return np.stack([rho, 0.5 * rho, 0.0 * x, 1.0 / 0.4 / 1.4 + 0.125 * rho])
            vals.append(O.shock_viscosity(m, 0, _project(m, 0, state)))
        assert abs(vals[1] / vals[0] - factor) < 1e-12


# ---- Navier-Stokes: the viscous form (Sec. 3.2), q_h in place of grad w_h

def _one_ns_triangle(eps0=0.2, degree=1):
    c = _one_triangle(eps0, degree)
    c.physics = "ns"
    c.reynolds = 100.0
    c.Q = np.zeros((1, 8, hi.n_modes(degree)))
    return c


def test_ns_viscosity_with_the_exact_gradient_equals_the_euler_form():
    """With q_h equal to the gradient of a linear state, the viscous form's eps(w, q) is the
    Euler eps(w, grad w): the closed form eps_0 (h/p)^2 d, d = 0.08125, of the test above."""
    c = _one_ns_triangle()
    m = O.Mesh(c, O.make_physics(c))
    gam, u, s = 1.4, 0.5, 0.1

    def state(x, y):
        rho = 1.0 + s * x
        return np.stack([rho, rho * u, 0.0 * x, 1.0 / gam / (gam - 1.0) + 0.5 * rho * u * u])

    def grad(x, y):          # rows 4 d + a: d/dx of (rho, rho u, rho v, E), then d/dy (zero)
        one = np.ones_like(x)
        return np.stack([s * one, s * u * one, 0 * one, 0.5 * u * u * s * one] + [0 * one] * 4)
    W, Q = _project(m, 0, state), _project(m, 0, grad)
    assert abs(O.shock_viscosity(m, 0, W, Q) - 0.2 * 2.0 * 0.08125) < 1e-14
    # a q_h that is not grad w_h changes it (the sensor reads q_h, not the state's gradient)
    assert abs(O.shock_viscosity(m, 0, W, 2.0 * Q) - 2.0 * 0.2 * 2.0 * 0.08125) < 1e-14


def test_ns_volume_term_in_the_newton_matrix_and_conservation():
    """Navier-Stokes, eps_K held fixed: switching the viscous form on adds eps_K (d_d phi_i, phi_j)
    to the (state row a, gradient column (d, a)) blocks of the local matrix and nothing else; the
    right-hand side changes by -eps_K (grad phi_i, q_h), which leaves the constant-mode rows (the
    element's conservation statement) unchanged."""
    kw = dict(seed=43, reynolds=200.0)
    c0 = hi.make_case("ns", 3, [1, 2], 0.8, 1.25, 8e-2, **kw)
    c1 = hi.make_case("ns", 3, [1, 2], 0.8, 1.25, 8e-2, **kw)
    c1.sc_eps0 = 0.2
    s0 = O.State(O.Mesh(c0, O.make_physics(c0)), c0.W, c0.lam, c0.Q)
    s1 = O.State(O.Mesh(c1, O.make_physics(c1)), c1.W, c1.lam, c1.Q)
    seen = 0.0
    for e in range(0, c0.n_elements, 2):
        b0, b1 = O.element_blocks(s0, e), O.element_blocks(s1, e)
        for name in ("B", "C", "D", "rl"):
            assert np.array_equal(getattr(b0, name), getattr(b1, name)), name
        n = hi.n_modes(int(c0.degree[e]))
        g = s1.mesh.geom(e)
        Qe, We = c1.Q[e, :, :n], c1.W[e, :, :n]
        eps = O.shock_viscosity(s1.mesh, e, We, Qe)
        expect = np.zeros_like(b1.A)
        for a in range(4):
            for d in range(2):
                blk = eps * np.einsum("q,nq,mq->nm", g.wq, g.dphi[d], g.phi)   # (d_d phi_i, phi_j)
                r0, c0_ = 8 * n + a * n, (4 * d + a) * n
                expect[r0: r0 + n, c0_: c0_ + n] = blk
        dA = b1.A - b0.A
        assert np.abs(dA - expect).max() < 1e-12 * max(1.0, np.abs(expect).max())
        dr = b1.r - b0.r
        assert np.abs(dr[: 8 * n]).max() == 0.0                      # gradient rows untouched
        dw = dr[8 * n:].reshape(4, n)
        assert np.abs(dw[:, 0]).max() < 1e-15                         # constant-mode rows
        grad_term = np.einsum("q,dnq,dkq->kn", g.wq, g.dphi, (Qe @ g.phi).reshape(2, 4, -1))
        assert np.abs(dw + eps * grad_term).max() < 1e-14
        seen = max(seen, eps)
    assert seen > 1e-4
