"""Pins of the oracle's backward-Euler pseudo-time term (Sec. 3.3): the local step dt_K,
the element mass matrix it divides, where the term enters the element system, the CFL
schedule (eq. cfl) and the relaxed Newton iteration it drives."""
import math

import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O


def _one_triangle(physics, cfl, reynolds=0.0):
    """The right triangle (0,0), (1,0), (0,1) at the constant free stream of Mach 0.5 along x
    (rho = 1, p = 1/gamma, so c = 1 and u = 0.5)."""
    c = hi.Case(name="one", physics=physics, ng=1, xy=np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
                tri=np.array([[0, 1, 2]], dtype=np.int32), degree=np.array([2], dtype=np.int8),
                mach=0.5, aoa_deg=0.0, amp=0.0, reynolds=reynolds, cfl=cfl)
    W = np.zeros((1, 4, hi.n_modes(2)))
    W[0, :, 0] = hi.SQRT2 * c.free_stream()      # constant field: leading coefficient sqrt(2) value
    c.W = W
    return c


def test_time_step_closed_form_euler():
    c = _one_triangle("euler", cfl=2.0)
    m = O.Mesh(c, O.make_physics(c))
    # edges: (0,0)-(1,0) length 1, normal (0,-1), v.n = 0; (1,0)-(0,1) length sqrt 2,
    # normal (1,1)/sqrt 2, v.n = 0.5/sqrt 2; (0,1)-(0,0) length 1, normal (-1,0), |v.n| = 0.5
    lam_c = (0.0 + 1.0) * 1.0 + (0.5 / math.sqrt(2.0) + 1.0) * math.sqrt(2.0) + (0.5 + 1.0) * 1.0
    assert abs(lam_c - (3.0 + math.sqrt(2.0))) < 1e-15
    dt = O.local_time_step(m, c.W[0, :, :6], 0)
    assert abs(dt - 2.0 * 0.5 / (3.0 + math.sqrt(2.0))) < 1e-15


def test_time_step_closed_form_navier_stokes():
    c = _one_triangle("ns", cfl=2.0, reynolds=100.0)
    phys = O.make_physics(c)
    assert abs(phys.mu - 0.5 / 100.0) < 1e-18          # rho |v| L / Re with L = 1
    m = O.Mesh(c, phys)
    # sum |e|^2 = 1 + 2 + 1 over |K| = 1/2: 8; lambda_v = mu gamma / (rho Pr) * 8
    lam_v = 0.005 * 1.4 / 0.72 * 8.0
    dt = O.local_time_step(m, c.W[0, :, :6], 0)
    assert abs(dt - 2.0 * 0.5 / (3.0 + math.sqrt(2.0) + 4.0 * lam_v)) < 1e-15


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_mass_matrix_is_det_j_identity(p):
    """The orthonormal basis makes the element mass matrix det J times the identity on any
    affine triangle (the shift is then a scalar on the diagonal)."""
    c = hi.make_case("euler", 3, p, 0.5, 2.0, 1e-2, seed=7, jitter=0.2)
    m = O.Mesh(c, O.make_physics(c))
    for e in (0, 5, 11):
        g = m.geom(e)
        mass = (g.phi * g.wq[None, :]) @ g.phi.T
        assert np.abs(mass - g.detJ * np.eye(mass.shape[0])).max() < 1e-13 * g.detJ


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_shift_enters_only_the_w_diagonal(physics):
    kw = dict(reynolds=200.0) if physics == "ns" else {}
    c0 = hi.make_case(physics, 3, [1, 2, 3], 0.5, 2.0, 2e-2, seed=21, **kw)
    c1 = hi.make_case(physics, 3, [1, 2, 3], 0.5, 2.0, 2e-2, seed=21, cfl=3.0, **kw)
    b0 = O.newton_step(c0, elements=None).blocks
    s1 = O.State(O.Mesh(c1, O.make_physics(c1)), c1.W, c1.lam, c1.Q)
    for e in range(0, c0.n_elements, 3):
        x0, x1 = b0[e], O.element_blocks(s1, e)
        for name in ("B", "C", "D", "r", "rl"):
            assert np.array_equal(getattr(x0, name), getattr(x1, name)), name
        dA = x1.A - x0.A
        npe = hi.n_modes(int(c0.degree[e]))
        w0 = 8 * npe if physics == "ns" else 0
        g = s1.mesh.geom(e)
        sig = g.detJ / O.local_time_step(s1.mesh, c1.W[e, :, :npe], e)
        assert sig > 0
        expect = np.zeros_like(dA)
        expect[w0:, w0:] = sig * np.eye(4 * npe)
        assert np.abs(dA - expect).max() < 1e-12 * sig


def test_small_cfl_local_solve_is_forward_euler():
    """As CFL -> 0 the element solve A^-1 r tends to dt_K M^-1 r = (dt_K / det J) r, an
    explicit Euler step of the element residual; the error is O(CFL)."""
    errs = []
    for cfl in (1e-4, 1e-6):
        c = hi.make_case("euler", 2, 2, 0.5, 2.0, 2e-2, seed=3, cfl=cfl)
        st = O.State(O.Mesh(c, O.make_physics(c)), c.W, c.lam, c.Q)
        b = O.element_blocks(st, 1)
        y = O.condense(b).y
        dt = O.local_time_step(st.mesh, c.W[1, :, :6], 1)
        ref = dt / st.mesh.geom(1).detJ * b.r
        errs.append(np.abs(y - ref).max() / np.abs(ref).max())
    assert errs[0] < 1e-2 and errs[1] < 1e-4
    assert errs[1] < 0.05 * errs[0]


def test_large_cfl_is_pure_newton():
    c0 = hi.make_case("euler", 3, [1, 2], 0.5, 2.0, 2e-2, seed=5)
    c1 = hi.make_case("euler", 3, [1, 2], 0.5, 2.0, 2e-2, seed=5, cfl=1e12)
    d0, d1 = O.newton_step(c0).dlam, O.newton_step(c1).dlam
    assert np.abs(d1 - d0).max() < 1e-8 * np.abs(d0).max()


def test_cfl_schedule_closed_form():
    """eq. cfl with the paper's constants c0 = 1e6, c1 = 1e3, n0 = 4."""
    ramp = [O.cfl_schedule(n, 0.0, 0.0, 1.0) for n in range(1, 5)]
    # c0 (3 s^2 - 2 s^3) at s = 1/4, 1/2, 3/4, 1
    assert ramp == [1e6 * (3 / 16 - 2 / 64), 5e5, 1e6 * (27 / 16 - 54 / 64), 1e6]
    assert ramp[0] == 156250.0 and ramp[2] == 843750.0
    # the smoothstep is symmetric about the middle of the ramp
    assert ramp[0] + ramp[2] == 1e6
    # growth: a residual reduced by the factor e multiplies the CFL by 1 + c1
    assert abs(O.cfl_schedule(5, 2.0, math.e, 1.0) - 2.0 * 1001.0) < 1e-12
    # a residual that grows leaves the CFL unchanged; a vanished one gives the Newton limit
    assert O.cfl_schedule(6, 3.0, 1.0, 2.0) == 3.0
    assert O.cfl_schedule(6, 3.0, 1.0, 0.0) == math.inf


def test_relaxed_iteration_has_the_newton_fixed_point():
    """The pseudo-time term changes the path, not the solution: a gently ramped iteration
    and the pure Newton iteration converge to the same discrete state."""
    c = hi.make_case("euler", 3, [1, 2], 0.5, 2.0, 2e-2, seed=8)
    relaxed = O.pseudo_transient(c, 14, c0=10.0, c1=1.0, n0=2)
    newton = O.pseudo_transient(c, 5, c0=1e14, c1=1.0, n0=1)
    assert relaxed.res[-1] < 1e-11 * relaxed.res[0]
    assert newton.res[-1] < 1e-11 * newton.res[0]
    # the relaxed path is genuinely different (slower) on the way
    assert relaxed.res[2] > 100 * newton.res[2]
    assert np.abs(relaxed.W - newton.W).max() < 1e-11
    assert np.abs(relaxed.lam - newton.lam).max() < 1e-11


def test_free_stream_is_a_fixed_point_of_the_iteration():
    c = hi.make_case("euler", 3, [1, 2, 3], 0.5, 2.0, 0.0, seed=9, free_stream_only=True)
    r = O.pseudo_transient(c, 2, c0=10.0, c1=1.0, n0=2)
    assert r.res[0] < 1e-13
    assert np.abs(r.W - c.W).max() < 1e-13 and np.abs(r.lam - c.lam).max() < 1e-13
