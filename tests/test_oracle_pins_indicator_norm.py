"""Pins of two oracle functions that the GPU path is compared with:

* element_indicators (Sec. 4, the element indicator with the skeleton adjoint dropped):
  eta_K = |z_K . R_K(x)|, z_K the element's adjoint unknowns and R_K its residual rows
  (Navier-Stokes: the gradient rows too).
* residual_norm (Sec. 3.3, the norm that eq. cfl reads): ||N_h(x)||_2 over every element
  row and every skeleton row, the skeleton rows summed over both neighbours.

Each pin computes the quantity along a route that shares no step with the function under
test: the element rows from the residual routine on real inputs (not the complex-step
blocks), the global estimate of eq. errest from the primal Newton step and the monolithic
adjoint, and the Euler skeleton rows from their closed form
R_e = -alpha int_e mu (2 lam - w+ - w-) (the trace fluxes f(lam).n of the two sides cancel).
The planted-mistake tests replace the function by a plausible wrong version and check that
the pin rejects it.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O


def _case(physics):
    if physics == "ns":
        return hi.make_case("ns", 2, [1, 2], 0.5, 1.0, 3e-2, seed=41, reynolds=100.0)
    return hi.make_case("euler", 2, [1, 2, 1, 3], 0.6, 1.5, 3e-2, seed=42)


def _functional(step, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(b.A.shape[0]) for b in step.blocks]


def _element_rows(case):
    """Per element the residual rows R_K in the element's unknown order (gradient rows first
    for Navier-Stokes), and the summed skeleton rows, from the residual routine."""
    _, Rloc, Rsk = O.global_residual(case, case.W, case.lam, case.Q)
    rows = []
    for r in Rloc:
        rows.append(np.concatenate([x.reshape(-1) for x in r]) if isinstance(r, tuple) else r.reshape(-1))
    return rows, Rsk


def _indicator_pin(case, indicator_fn):
    """Largest violation of the two indicator identities for `indicator_fn`:
    (i) eta_K = |z_K . R_K| with R_K from the residual routine, and
    (ii) sum_K z_K . R_K + Lam~ . R_lam = -J'(x) dx (eq. errest; dx the primal Newton step,
    z the adjoint of the monolithic transposed system), which fixes the signed values whose
    moduli (i) compares."""
    step = O.newton_step(case)
    F = _functional(step, seed=7)
    Ut, lt = O.adjoint_monolithic(step, F)
    eta = np.asarray(indicator_fn(step, Ut))
    rows, Rsk = _element_rows(case)
    signed = np.array([float(Ut[e] @ rows[e]) for e in range(step.mesh.ne)])
    scale = np.abs(signed).max()
    err_i = float(np.abs(eta - np.abs(signed)).max() / scale)
    dJ = float(np.concatenate(F) @ np.concatenate(step.du))
    err_ii = abs(signed.sum() + float(lt @ Rsk) + dJ) / abs(dJ)
    return max(err_i, err_ii)


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_element_indicators_pinned(physics):
    assert _indicator_pin(_case(physics), O.element_indicators) < 1e-10


# plausible mistakes in the indicator, each of which the pin must reject

def _ind_wrong_rows(step, Ut):
    # weights the adjoint of element K with the residual of the next element of its size
    ne = step.mesh.ne
    out = []
    for e in range(ne):
        n = step.blocks[e].r.size
        o = next(k % ne for k in range(e + 1, e + ne + 1) if step.blocks[k % ne].r.size == n)
        out.append(abs(float(Ut[e] @ (-step.blocks[o].r))))
    return np.array(out)


def _ind_reversed_modes(step, Ut):
    # pairs each adjoint entry with the residual row in reversed order
    return np.array([abs(float(Ut[e] @ (-b.r[::-1]))) for e, b in enumerate(step.blocks)])


def _ind_state_rows_only(step, Ut):
    # Navier-Stokes: drops the gradient rows (keeps the last 4 Np rows, the conserved fields)
    out = []
    for e, b in enumerate(step.blocks):
        n4 = b.A.shape[0] // 3
        out.append(abs(float(Ut[e][-n4:] @ (-b.r[-n4:]))))
    return np.array(out)


def _ind_with_skeleton(step, Ut):
    # adds the element's share of the skeleton adjoint term (the paper drops it)
    m = step.mesh
    F = _functional(step, seed=7)
    _, lt = O.adjoint_monolithic(step, F)
    out = []
    for e, b in enumerate(step.blocks):
        d = O.elem_dofs(m, b)
        v = float(Ut[e] @ (-b.r))
        if d.size:
            v += float(lt[d] @ (-b.rl))
        out.append(abs(v))
    return np.array(out)


@pytest.mark.parametrize("physics,mistake", [
    ("euler", _ind_wrong_rows), ("ns", _ind_wrong_rows), ("euler", _ind_reversed_modes),
    ("ns", _ind_state_rows_only), ("euler", _ind_with_skeleton), ("ns", _ind_with_skeleton)])
def test_element_indicator_pin_rejects_planted_mistakes(physics, mistake):
    assert _indicator_pin(_case(physics), mistake) > 1e-6


# ---------------------------------------------------------------------------
# residual norm
# ---------------------------------------------------------------------------

def _euler_skeleton_rows_closed_form(case):
    """R_e[a, k] = -alpha int_e psi_k (2 lam_a - w+_a - w-_a) ds for every interior face, the
    traces of both neighbours evaluated at the face's Gauss points (p_e + 2 of them) in the
    face's global parameterisation (from the lower to the higher vertex id)."""
    phys = O.make_physics(case)
    mesh = O.Mesh(case, phys)
    out = np.zeros(mesh.n_skel)
    xy = case.xy
    for f in range(mesh.nf):
        va, vb = (int(v) for v in mesh.face_vertices[f])
        pe = int(mesh.face_degree[f])
        s, wg = np.polynomial.legendre.leggauss(pe + 2)
        pts = 0.5 * (1 - s)[:, None] * xy[va] + 0.5 * (1 + s)[:, None] * xy[vb]
        half = 0.5 * np.linalg.norm(xy[vb] - xy[va])
        psi = np.stack([np.sqrt((2 * k + 1) / 2.0) * np.polynomial.legendre.Legendre.basis(k)(s)
                        for k in range(pe + 1)])            # (pe+1, g)
        lam = case.lam[f, :, : pe + 1] @ psi                # (4, g)
        wsum = np.zeros_like(lam)
        for e, _ in mesh.face_elems[f]:
            wsum += _element_state_at(case, int(e), pts)
        r = -phys.alpha * (psi * (wg * half)) @ (2.0 * lam - wsum).T   # (pe+1, 4)
        out[mesh.face_offset[f]: mesh.face_offset[f + 1]] = r.T.reshape(-1)
    return out


def _element_state_at(case, e, pts):
    """w_h of element e at physical points, from its Dubiner coefficients (affine map of the
    reference triangle {(-1,-1), (1,-1), (-1,1)})."""
    v = case.xy[case.tri[e]]
    J = np.column_stack([v[1] - v[0], v[2] - v[0]]) / 2.0
    ref = np.linalg.solve(J, (pts - v[0]).T) - 1.0          # (2, g)
    p = int(case.degree[e])
    phi = O.dubiner(p, ref[0], ref[1])                       # (Np, g)
    return case.W[e, :, : O.n_modes(p)] @ phi


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_residual_norm_equals_the_assembled_newton_right_hand_side(physics):
    """||N_h|| from residual_norm equals the norm of the right-hand side that global_jacobian
    assembles from the complex-step element blocks (element rows r_K, gradient rows included,
    and the skeleton rows summed with np.add.at), a second assembly route."""
    c = _case(physics)
    step = O.newton_step(c)
    _, rhs, _ = O.global_jacobian(step)
    assert abs(O.residual_norm(c, c.W, c.lam, c.Q) - np.linalg.norm(rhs)) < 1e-12 * np.linalg.norm(rhs)


def test_residual_norm_skeleton_rows_match_the_closed_form():
    """Euler: the skeleton part of ||N_h||^2 equals that of the closed-form rows, where the two
    neighbours' shares cancel in their flux part; the element part is the rest."""
    c = _case("euler")
    closed = _euler_skeleton_rows_closed_form(c)
    rows, Rsk = _element_rows(c)
    assert np.abs(Rsk - closed).max() < 1e-13 * max(1.0, np.abs(closed).max())
    total = np.sqrt(float(closed @ closed) + sum(float(r @ r) for r in rows))
    assert abs(O.residual_norm(c, c.W, c.lam) - total) < 1e-12 * total


def _norm_concatenated_shares(case, W, lam, Q=None, alpha=None):
    # concatenates the two neighbours' skeleton shares instead of summing them
    phys = O.make_physics(case, alpha)
    mesh = O.Mesh(case, phys)
    st = O.State(mesh, W, lam, Q)
    s = 0.0
    for e in range(mesh.ne):
        We, Qe, lams = st.elem_inputs(e)
        lb = [None if l is None else l[None] for l in lams]
        Rq, Rw, Rl = O.element_residual(mesh, e, We[None], None if Qe is None else Qe[None], lb)
        for x in ((Rw[0],) if Rq is None else (Rq[0], Rw[0])):
            s += float(np.sum(x * x))
        for lf in range(3):
            if mesh.elem_faces[e, lf] >= 0:
                s += float(np.sum(Rl[lf][0] ** 2))
    return float(np.sqrt(s))


def _norm_without_gradient_rows(case, W, lam, Q=None, alpha=None):
    # Navier-Stokes: omits the gradient rows
    _, Rloc, Rsk = O.global_residual(case, W, lam, Q, alpha)
    s = float(Rsk @ Rsk)
    for r in Rloc:
        x = r[1] if isinstance(r, tuple) else r
        s += float(np.sum(x * x))
    return float(np.sqrt(s))


@pytest.mark.parametrize("physics,mistake", [("euler", _norm_concatenated_shares), ("ns", _norm_concatenated_shares),
                                             ("ns", _norm_without_gradient_rows)])
def test_residual_norm_pin_rejects_planted_mistakes(physics, mistake):
    c = _case(physics)
    step = O.newton_step(c)
    _, rhs, _ = O.global_jacobian(step)
    ref = np.linalg.norm(rhs)
    assert abs(mistake(c, c.W, c.lam, c.Q) - ref) > 1e-6 * ref
