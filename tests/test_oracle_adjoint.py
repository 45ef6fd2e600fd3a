"""Pins of the oracle's adjoint (Sec. 4, eq. adjoint, eq. errest; Sec. 4.1): the hybridized
adjoint against the direct transposed solve, the transposed skeleton matrix, duality with
the primal Newton step, the adjoint-weighted residual and the enrichment to one degree more."""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O


def _case(physics):
    if physics == "ns":
        return hi.make_case("ns", 3, [1, 2], 0.5, 1.0, 2e-2, seed=31, reynolds=200.0)
    return hi.make_case("euler", 3, [1, 2, 3], 0.6, 1.5, 2e-2, seed=32)


def _functional(step, seed=4):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(b.A.shape[0]) for b in step.blocks]


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_hybridized_adjoint_equals_direct_transposed_solve(physics):
    step = O.newton_step(_case(physics))
    F = _functional(step)
    Ud, ld = O.adjoint_monolithic(step, F)
    Uh, lh, _ = O.adjoint_hybridized(step, F)
    assert O.relative_error(lh, ld) < 1e-11
    assert O.relative_error(np.concatenate(Uh), np.concatenate(Ud)) < 1e-11


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_condensed_adjoint_matrix_is_k_transposed(physics):
    """Condensing the transposed local blocks, D_K^T - B_K^T A_K^-T C_K^T summed over the
    elements, gives K^T: the adjoint reuses the primal skeleton matrix."""
    step = O.newton_step(_case(physics))
    m = step.mesh
    Kadj = np.zeros((m.n_skel, m.n_skel))
    for b in step.blocks:
        d = O.elem_dofs(m, b)
        if d.size:
            S = b.D.T - b.B.T @ np.linalg.solve(b.A.T, b.C.T)
            Kadj[np.ix_(d, d)] += S
    K = step.K.toarray()
    assert np.abs(Kadj - K.T).max() < 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_duality_with_the_newton_step(physics):
    """F~ . dU = z . [r; r_lam]: the adjoint and the primal Newton step are solves with the
    transposed and the original matrix, computed here by different routes."""
    step = O.newton_step(_case(physics))
    F = _functional(step, seed=9)
    Ut, lt = O.adjoint_monolithic(step, F)
    _, rhs, _ = O.global_jacobian(step)
    lhs = float(np.concatenate(F) @ np.concatenate(step.du))
    rhs_dot = float(np.concatenate(Ut + [lt]) @ rhs)
    assert abs(lhs - rhs_dot) < 1e-11 * (abs(lhs) + 1e-300)


def test_adjoint_weighted_residual_predicts_the_functional_change():
    """eq. errest in discrete form: -N_h(x; z) with the residual evaluated by the residual
    routine (not the Jacobian blocks) equals J'(x) dx for the Newton correction dx."""
    c = _case("euler")
    step = O.newton_step(c)
    F = _functional(step, seed=5)
    Ut, lt, _ = O.adjoint_hybridized(step, F)
    _, Rloc, Rsk = O.global_residual(c, c.W, c.lam)
    eta = -(sum(float(Ut[e] @ Rloc[e].reshape(-1)) for e in range(step.mesh.ne)) + float(lt @ Rsk))
    dJ = float(np.concatenate(F) @ np.concatenate(step.du))
    assert abs(eta - dJ) < 1e-10 * abs(dJ)
    ind = O.element_indicators(step, Ut)
    assert np.all(ind >= 0) and ind.shape == (step.mesh.ne,)


def test_enrichment_keeps_the_function_and_adds_test_functions():
    """The space of one degree more (Sec. 4): the padded state is the same function at any
    point (hierarchical basis), and the enriched residual has rows for the new test functions
    that the degree-p residual does not see."""
    c = hi.make_case("euler", 3, [1, 2], 0.5, 2.0, 2e-2, seed=33)
    ce = O.enrich(c)
    assert np.all(ce.degree == c.degree + 1)
    rng = np.random.default_rng(2)
    xi = rng.uniform(-1.0, 0.0, 40)
    eta = rng.uniform(-1.0, 0.0, 40)
    for e in range(c.n_elements):
        p = int(c.degree[e])
        v0 = c.W[e, :, : hi.n_modes(p)] @ O.dubiner(p, xi, eta)
        v1 = ce.W[e, :, : hi.n_modes(p + 1)] @ O.dubiner(p + 1, xi, eta)
        assert np.abs(v1 - v0).max() < 1e-13
    _, R0, _ = O.global_residual(c, c.W, c.lam)
    _, R1, _ = O.global_residual(ce, ce.W, ce.lam)
    for e in range(c.n_elements):
        n0 = hi.n_modes(int(c.degree[e]))
        new_rows = R1[e][:, n0:]
        assert np.abs(new_rows).max() > 1e-8          # tested against the new functions
        assert R1[e].shape[1] == hi.n_modes(int(c.degree[e]) + 1) and R0[e].shape[1] == n0


def test_doerfler_marking_hand_cases_and_brute_force():
    eta = np.array([3.0, 4.0, 0.0, 1.0, 2.0])             # eta_T^2 = 30
    assert list(np.flatnonzero(O.doerfler_mark(eta, 0.5))) == [1]           # 16 >= 0.25 * 30
    assert list(np.flatnonzero(O.doerfler_mark(eta, 0.05))) == [0, 1, 4]    # 16, 25, 29 >= 27.075
    assert not O.doerfler_mark(eta, 1.0).any()
    assert not O.doerfler_mark(np.zeros(4), 0.05).any()
    # ties go to the lower element id
    assert list(np.flatnonzero(O.doerfler_mark(np.array([1.0, 2.0, 2.0, 1.0]), 0.5))) == [1]
    # the smallest qualifying set, by exhaustive search over subsets
    import itertools
    rng = np.random.default_rng(7)
    for _ in range(20):
        e = rng.exponential(size=8)
        theta = rng.uniform(0.0, 0.9)
        need = (1 - theta) ** 2 * np.sum(e * e)
        best = min(k for k in range(9) for s in itertools.combinations(range(8), k)
                   if np.sum(e[list(s)] ** 2) >= need - 1e-15 * need)
        got = O.doerfler_mark(e, theta)
        assert got.sum() == best and np.sum(e[got] ** 2) >= need * (1 - 1e-15)


def test_smoothness_sensor_definition_cases():
    """A degree-(p-1) state has S = 0, a state made of degree-p modes only has S = 1, and in
    general S equals the energy of the degree-p coefficients over the total (orthonormal,
    hierarchical basis), although the oracle computes it from the projection's definition."""
    c = hi.make_case("euler", 3, [1, 2, 3], 0.5, 2.0, 5e-2, seed=12, jitter=0.2)
    rng = np.random.default_rng(3)
    for e in range(0, c.n_elements, 2):
        p = int(c.degree[e])
        n0, n1 = hi.n_modes(p - 1), hi.n_modes(p)
        W = np.zeros_like(c.W)
        W[e, :, :n0] = rng.standard_normal((4, n0))
        assert O.smoothness_sensor(c, W, e) < 1e-24
        W[:] = 0.0
        W[e, :, n0:n1] = rng.standard_normal((4, n1 - n0))
        assert abs(O.smoothness_sensor(c, W, e) - 1.0) < 1e-12
        W[e, :, :n1] = c.W[e, :, :n1]
        ref = np.sum(W[e, :, n0:n1] ** 2) / np.sum(W[e, :, :n1] ** 2)
        assert abs(O.smoothness_sensor(c, W, e) - ref) < 1e-12 * ref
