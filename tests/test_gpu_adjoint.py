"""GPU parity of the hybridized adjoint (Sec. 4.1): K^T, the adjoint right-hand side
E~ = -sum X_K^T F~_K, the local adjoint solves with the element indicators, and the whole
adjoint solve, against the oracle on the same seeded inputs (functional derivatives drawn
from a seeded generator)."""
import sys

import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(which):
    if which == "c1":
        return hi.config_case("c1")
    if which == "c1_enriched":          # the space of one degree more, as the paper solves the adjoint
        return O.enrich(hi.config_case("c1"))
    if which == "hp":
        return hi.make_case("euler", 4, [1, 2, 3, 4], 0.6, 1.5, 2e-2, seed=3)
    if which == "hp_shock":             # shock capturing and a pseudo-time step in the matrices
        c = hi.make_case("euler", 4, [1, 2, 3, 4], 0.8, 1.25, 8e-2, seed=43)
        c.sc_eps0 = 0.2
        c.cfl = 5.0
        return c
    if which == "ns14":
        return hi.make_case("ns", 3, [1, 2, 3, 4], 0.6, -2.0, 2e-2, seed=22, reynolds=500.0)
    return hi.make_case("ns", 3, [2, 3], 0.5, 1.0, 2e-2, seed=21, reynolds=200.0)


def _functional(step, case, seed=6):
    """Seeded F~ per element in the oracle's unknown order, and the same in the padded layouts."""
    rng = np.random.default_rng(seed)
    F = [rng.standard_normal(b.A.shape[0]) for b in step.blocks]
    npm = case.W.shape[2]
    fw = np.zeros((case.n_elements, 4, npm))
    fq = np.zeros((case.n_elements, 8, npm)) if case.physics == "ns" else None
    for e in range(case.n_elements):
        npe = hi.n_modes(int(case.degree[e]))
        if fq is not None:
            fq[e, :, :npe] = F[e][: 8 * npe].reshape(8, npe)
            fw[e, :, :npe] = F[e][8 * npe:].reshape(4, npe)
        else:
            fw[e, :, :npe] = F[e].reshape(4, npe)
    return F, fw, fq


def _setup(hdg, which):
    import torch
    case = _case(which)
    step = O.newton_step(case)
    F, fw, fq = _functional(step, case)
    plan = hdg.HDGPlan.from_case(case)
    dev = plan.device
    w = torch.tensor(case.W, dtype=torch.float64, device=dev)
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
    q = torch.tensor(case.Q, dtype=torch.float64, device=dev) if case.Q is not None else None
    fw_d = torch.tensor(fw, device=dev)
    fq_d = torch.tensor(fq, device=dev) if fq is not None else None
    plan.hdg_assemble_condense(w, lam, q=q)
    return case, step, F, plan, w, lam, q, fw_d, fq_d


@pytest.mark.parametrize("which", ["c1", "hp", "ns23"])
def test_transpose_and_adjoint_rhs_match_oracle(hdg, which):
    import torch
    _say(f"adjoint rhs {which}")
    case, step, F, plan, w, lam, q, fw, fq = _setup(hdg, which)
    kt = torch.empty_like(plan.bsr)
    plan.hdg_skeleton_transpose(kt)
    K = plan.skeleton_matrix_dense()
    assert np.array_equal(plan.skeleton_matrix_dense(kt), K.T)
    et = torch.empty(plan.n_skel, dtype=torch.float64, device=plan.device)
    plan.hdg_adjoint_rhs(fw, et, fq=fq)
    _, _, Et = O.adjoint_hybridized(step, F)
    assert O.relative_error(et.cpu().numpy(), Et) < 1e-12


@pytest.mark.parametrize("which", ["c1", "hp", "c1_enriched"])
def test_local_adjoint_matches_oracle(hdg, which):
    """Given the oracle's Lambda~, the transposed local solves and the indicators."""
    import torch
    _say(f"adjoint local {which}")
    case, step, F, plan, w, lam, q, fw, fq = _setup(hdg, which)
    Ut, lt, _ = O.adjoint_hybridized(step, F)
    lamt = torch.tensor(lt, device=plan.device)
    wt = torch.zeros_like(w)
    eta = torch.zeros(case.n_elements, dtype=torch.float64, device=plan.device)
    st = torch.zeros(case.n_elements, dtype=torch.int32, device=plan.device)
    plan.hdg_adjoint_local(w, lam, fw, lamt, wt, eta, elem_status=st)
    got = wt.cpu().numpy()
    for e in range(case.n_elements):
        npe = hi.n_modes(int(case.degree[e]))
        ref = Ut[e].reshape(4, npe)
        tol = 1e-12 + np.linalg.cond(step.blocks[e].A) * 1e-15
        assert O.relative_error(got[e, :, :npe], ref) < tol, (e, O.relative_error(got[e, :, :npe], ref))
    assert O.relative_error(eta.cpu().numpy(), O.element_indicators(step, Ut)) < 1e-11


@pytest.mark.parametrize("which", ["c1", "hp", "c1_enriched", "hp_shock"])
def test_adjoint_solve_matches_oracle(hdg, which):
    _say(f"adjoint solve {which}")
    case, step, F, plan, w, lam, q, fw, fq = _setup(hdg, which)
    lamt, wt, eta, it = plan.hdg_adjoint_solve(w, lam, fw, rtol=1e-13)
    _say(f"  gmres iterations on K^T: {it}")
    Ut, lt, _ = O.adjoint_hybridized(step, F)
    assert O.relative_error(lamt.cpu().numpy(), lt) < 1e-10
    got = wt.cpu().numpy()
    ref = np.zeros_like(got)
    for e in range(case.n_elements):
        npe = hi.n_modes(int(case.degree[e]))
        ref[e, :, :npe] = Ut[e].reshape(4, npe)
    assert O.relative_error(got, ref) < 1e-10
    assert O.relative_error(eta.cpu().numpy(), O.element_indicators(step, Ut)) < 1e-9


@pytest.mark.parametrize("which", ["ns23", "ns14"])
def test_navier_stokes_adjoint_matches_oracle(hdg, which):
    """Navier-Stokes: K^T Lambda~ = E~ through the same solver, then the local adjoint over
    all 12 Np element unknowns (gradient fields included) and the indicators; also the local
    solve alone from the oracle's Lambda~."""
    import torch
    _say(f"adjoint {which}")
    case, step, F, plan, w, lam, q, fw, fq = _setup(hdg, which)
    Ut, lt, _ = O.adjoint_hybridized(step, F)
    lamt, wt, eta, it, qt = plan.hdg_adjoint_solve(w, lam, fw, q=q, fq=fq, rtol=1e-13)
    _say(f"  gmres iterations on K^T: {it}")
    assert O.relative_error(lamt.cpu().numpy(), lt) < 1e-10
    npm = case.W.shape[2]
    rw, rq = np.zeros((case.n_elements, 4, npm)), np.zeros((case.n_elements, 8, npm))
    for e in range(case.n_elements):
        npe = hi.n_modes(int(case.degree[e]))
        rq[e, :, :npe] = Ut[e][: 8 * npe].reshape(8, npe)
        rw[e, :, :npe] = Ut[e][8 * npe:].reshape(4, npe)
    assert O.relative_error(wt.cpu().numpy(), rw) < 1e-10
    assert O.relative_error(qt.cpu().numpy(), rq) < 1e-10
    assert O.relative_error(eta.cpu().numpy(), O.element_indicators(step, Ut)) < 1e-9
    # the local solves alone, from the oracle's skeleton adjoint
    lt_d = torch.tensor(lt, device=plan.device)
    wt2, qt2 = torch.zeros_like(w), torch.zeros_like(q)
    eta2 = torch.zeros(case.n_elements, dtype=torch.float64, device=plan.device)
    st = torch.zeros(case.n_elements, dtype=torch.int32, device=plan.device)
    plan.hdg_adjoint_local(w, lam, fw, lt_d, wt2, eta2, q=q, fq=fq, qt=qt2, elem_status=st)
    assert O.relative_error(wt2.cpu().numpy(), rw) < 1e-11
    assert O.relative_error(qt2.cpu().numpy(), rq) < 1e-11
    assert O.relative_error(eta2.cpu().numpy(), O.element_indicators(step, Ut)) < 1e-10


@pytest.mark.parametrize("which", ["c1", "hp"])
def test_marking_and_sensor_match_oracle(hdg, which):
    """Doerfler marking and the smoothness sensor on seeded indicators: sensor values agree
    to rounding, the marked sets and the p/h flags exactly (ties included: the indicators are
    rounded so that many repeat)."""
    import torch
    _say(f"marking {which}")
    case = _case(which)
    plan = hdg.HDGPlan.from_case(case)
    w = torch.tensor(case.W, dtype=torch.float64, device=plan.device)
    S_ref = np.array([O.smoothness_sensor(case, case.W, e) for e in range(case.n_elements)])
    s_sorted = np.sort(S_ref)
    k = len(s_sorted) // 2
    eps_mid = float(np.sqrt(s_sorted[k - 1] * s_sorted[k]))   # between two sensor values: both flags occur
    rng = np.random.default_rng(11)
    for rounding in (None, 1):
        eta_h = rng.exponential(size=case.n_elements)
        if rounding is not None:
            eta_h = np.round(eta_h, rounding)
        eta = torch.tensor(eta_h, device=plan.device)
        for theta, eps in ((0.05, 1e-6), (0.3, eps_mid), (0.0, eps_mid), (1.0, eps_mid)):
            flag, S, m = plan.hdg_mark_elements(w, eta, theta=theta, eps_s=eps)
            ref, _ = O.adaptation_flags(case, case.W, eta_h, theta, eps)
            assert np.all(np.abs(S.cpu().numpy() - S_ref) <= 1e-13 + 1e-10 * S_ref)
            assert np.array_equal(flag.cpu().numpy(), ref), (theta, eps)
            assert m == int((ref > 0).sum())
