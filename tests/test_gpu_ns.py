"""GPU parity of the Navier-Stokes path (gradient unknowns eliminated on the device) against
the CPU oracle, which builds the full (q, w) local system by complex-step differentiation."""
import sys

import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-12
RESID_ROUNDING = 1e-13   # float64 rounding of a smooth-state residual, amplified by kappa(A_K)


def tol_resid(A) -> float:
    return TOL + np.linalg.cond(A) * RESID_ROUNDING


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return O.relative_error(a, b)


CASES = {
    "ns23": dict(physics="ns", ng=3, degrees=[2, 3], mach=0.5, aoa_deg=1.0, amp=2e-2, seed=21, reynolds=200.0),
    "ns14": dict(physics="ns", ng=3, degrees=[1, 2, 3, 4], mach=0.6, aoa_deg=-2.0, amp=2e-2, seed=22,
                 reynolds=500.0),
}


def _case(which):
    kw = dict(CASES[which])
    return hi.make_case(kw.pop("physics"), kw.pop("ng"), kw.pop("degrees"), kw.pop("mach"), kw.pop("aoa_deg"),
                        kw.pop("amp"), **kw)


def _state(plan, case):
    import torch
    w = torch.tensor(case.W, dtype=torch.float64, device=plan.device)
    q = torch.tensor(case.Q, dtype=torch.float64, device=plan.device)
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=plan.device)
    return w, q, lam


@pytest.mark.parametrize("which", list(CASES))
def test_ns_element_blocks_match_oracle(hdg, which):
    case = _case(which)
    _say(f"ns blocks {which}")
    plan = hdg.HDGPlan.from_case(case)
    w, q, lam = _state(plan, case)
    mesh = O.Mesh(case, O.make_physics(case))
    st = O.State(mesh, case.W, case.lam, case.Q)
    for e in range(case.n_elements):
        ob = O.element_blocks(st, e)
        gb = plan.debug_element_blocks(e, w, lam, q)
        for k, ref in (("A", ob.A), ("B", ob.B), ("C", ob.C), ("D", ob.D), ("r", ob.r), ("rl", ob.rl)):
            assert gb[k].shape == ref.shape, (e, k)
            if ref.size:
                assert rel(gb[k], ref) < TOL, (e, k, rel(gb[k], ref))


@pytest.mark.parametrize("which", list(CASES))
def test_ns_newton_step_matches_oracle(hdg, which):
    import torch
    case = _case(which)
    _say(f"ns newton step {which}")
    step = O.newton_step(case)
    plan = hdg.HDGPlan.from_case(case)
    w, q, lam = _state(plan, case)
    plan.hdg_assemble_condense(w, lam, q=q)
    torch.cuda.synchronize()
    for e in range(case.n_elements):
        X, y = plan.debug_local_solution(e)
        c = step.cond[e]
        assert rel(X, c.X) < TOL, (e, rel(X, c.X))
        assert rel(y, c.y) < tol_resid(step.blocks[e].A), (e, rel(y, c.y))
    K = plan.skeleton_matrix_dense()
    assert rel(K, step.K.toarray()) < TOL
    assert rel(plan.rhs.cpu().numpy(), step.E) < TOL
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    it, relres, _ = plan.hdg_skeleton_solve(dlam, rtol=1e-12, restart=30)
    x = dlam.cpu().numpy()
    _say(f"  gmres iters {it} relres {relres:.2e}")
    assert relres <= 1e-12
    assert np.linalg.norm(step.E - step.K @ x) / np.linalg.norm(step.E) <= 2e-12
    # back-substitution with the oracle's dLambda: both the gradient and the state updates
    dl = torch.tensor(step.dlam, dtype=torch.float64, device=plan.device)
    dw = torch.zeros_like(w)
    dq = torch.zeros_like(q)
    plan.hdg_back_substitute(dl, dw, dq)
    gw, gq = dw.cpu().numpy(), dq.cpu().numpy()
    rw, rq = np.zeros_like(gw), np.zeros_like(gq)
    for e in range(case.n_elements):
        rw[e], rq[e] = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(gw, rw) < 1e-11
    assert rel(gq, rq) < 1e-11


def test_ns_pseudo_time_step_matches_oracle(hdg):
    """The local pseudo-time term of Sec. 3.3 (with the viscous wave speed) at CFL 5."""
    import torch
    case = _case("ns23")
    case.cfl = 5.0
    _say("ns pseudo-time ns23")
    step = O.newton_step(case)
    plan = hdg.HDGPlan.from_case(case)
    w, q, lam = _state(plan, case)
    for e in range(0, case.n_elements, 3):
        gb = plan.debug_element_blocks(e, w, lam, q)
        assert rel(gb["A"], step.blocks[e].A) < TOL, (e, rel(gb["A"], step.blocks[e].A))
    plan.hdg_assemble_condense(w, lam, q=q)
    torch.cuda.synchronize()
    for e in range(case.n_elements):
        X, y = plan.debug_local_solution(e)
        c = step.cond[e]
        assert rel(X, c.X) < TOL, (e, rel(X, c.X))
        assert rel(y, c.y) < tol_resid(step.blocks[e].A), (e, rel(y, c.y))
    assert rel(plan.skeleton_matrix_dense(), step.K.toarray()) < TOL
    assert rel(plan.rhs.cpu().numpy(), step.E) < TOL
    dl = torch.tensor(step.dlam, dtype=torch.float64, device=plan.device)
    dw = torch.zeros_like(w)
    dq = torch.zeros_like(q)
    plan.hdg_back_substitute(dl, dw, dq)
    rw, rq = np.zeros_like(case.W), np.zeros_like(case.Q)
    for e in range(case.n_elements):
        rw[e], rq[e] = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(dw.cpu().numpy(), rw) < 1e-11
    assert rel(dq.cpu().numpy(), rq) < 1e-11


def test_ns_free_stream_gives_zero_rhs(hdg):
    case = hi.make_case("ns", 4, [1, 2, 3, 4], 0.5, 1.0, 0.0, seed=23, reynolds=100.0, free_stream_only=True)
    _say("ns free stream")
    plan = hdg.HDGPlan.from_case(case)
    w, q, lam = _state(plan, case)
    nrm = plan.hdg_assemble_condense(w, lam, q=q, want_norm=True)
    assert nrm < 1e-13


def test_c4_recipe_reduced_size_sampled(hdg):
    """The Navier-Stokes workload recipe (p in {2,3,4}, Re 5000, Pr 0.72) on a 24x24 mesh:
    sampled local solutions and the skeleton residual recomputed on the CPU."""
    import scipy.sparse as sp
    import torch
    case = hi.config_case("c4", ng=24)
    _say("c4 recipe 24x24")
    plan = hdg.HDGPlan.from_case(case)
    w, q, lam = _state(plan, case)
    plan.hdg_assemble_condense(w, lam, q=q)
    torch.cuda.synchronize()
    mesh = O.Mesh(case, O.make_physics(case))
    st = O.State(mesh, case.W, case.lam, case.Q)
    rng = np.random.default_rng(2)
    for e in rng.choice(case.n_elements, 9, replace=False):
        ob = O.element_blocks(st, int(e))
        oc = O.condense(ob)
        X, y = plan.debug_local_solution(int(e))
        assert rel(X, oc.X) < TOL
        assert rel(y, oc.y) < tol_resid(ob.A)
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    it, relres, _ = plan.hdg_skeleton_solve(dlam, rtol=1e-10, restart=30)
    _say(f"  c4-recipe gmres iters {it} relres {relres:.2e}")
    K = sp.csr_matrix(plan.skeleton_matrix_dense())
    E = plan.rhs.cpu().numpy()
    x = dlam.cpu().numpy()
    assert relres <= 1e-10 and np.linalg.norm(E - K @ x) / np.linalg.norm(E) <= 2e-10


def test_c4_full_size_sampled(hdg):
    """The 256x256 Navier-Stokes workload (p in {2, 3, 4}, 131072 elements) in the launch
    configuration the benchmark times: sampled local solutions (every degree, and elements on
    the far field) against the oracle, and sampled skeleton rows and right-hand side entries
    against the exact partial assembly from the two elements that share each face."""
    import torch
    case = hi.config_case("c4")
    _say("c4 full size")
    plan = hdg.HDGPlan.from_case(case)
    w, q, lam = _state(plan, case)
    plan.hdg_assemble_condense(w, lam, q=q)
    torch.cuda.synchronize()
    mesh = O.Mesh(case, O.make_physics(case))
    st = O.State(mesh, case.W, case.lam, case.Q)
    rng = np.random.default_rng(4)
    fid = {tuple(v): i for i, v in enumerate(plan.face_vertices)}
    owners = {}
    n_bnd = np.zeros(case.n_elements, dtype=np.int64)
    for e in range(case.n_elements):
        t = case.tri[e]
        for lf in range(3):
            key = tuple(sorted((int(t[lf]), int(t[(lf + 1) % 3]))))
            if key in fid:
                owners.setdefault(fid[key], []).append(e)
            else:
                n_bnd[e] += 1
    corner = np.flatnonzero(n_bnd == 2)
    edge = np.flatnonzero(n_bnd == 1)
    boundary = ([int(corner[0])] if corner.size else []) + [int(e) for e in rng.choice(edge, 2, replace=False)]
    sample = boundary + [int(e) for p in (2, 3, 4) for e in rng.choice(np.flatnonzero(case.degree == p), 2,
                                                                         replace=False)]
    cache = {}

    def cond(e):
        if e not in cache:
            ob = O.element_blocks(st, e)
            cache[e] = (ob, O.condense(ob))
        return cache[e]

    for e in sample:
        ob, oc = cond(e)
        X, y = plan.debug_local_solution(e)
        assert rel(X, oc.X) < TOL, (e, rel(X, oc.X))
        assert rel(y, oc.y) < tol_resid(ob.A), (e, rel(y, oc.y))
    # skeleton rows of sampled faces: only the face's two elements contribute
    rp, col, voff = plan.pattern()
    fo = plan.face_offset
    E_gpu = plan.rhs
    for f in rng.choice(len(plan.face_degree), 6, replace=False):
        f = int(f)
        f0, f1 = int(fo[f]), int(fo[f + 1])
        ref_rows = {}
        ref_E = np.zeros(f1 - f0)
        for e in owners[f]:
            ob, oc = cond(e)
            d = O.elem_dofs(mesh, ob)
            loc = np.flatnonzero((d >= f0) & (d < f1))
            for i in loc:
                for jj, gd in enumerate(d):
                    ref_rows[(int(d[i]) - f0, int(gd))] = ref_rows.get((int(d[i]) - f0, int(gd)), 0.0) + oc.S[i, jj]
                ref_E[int(d[i]) - f0] += oc.g[i]
        got = {}
        for k in range(rp[f], rp[f + 1]):
            g = int(col[k])
            g0, g1 = int(fo[g]), int(fo[g + 1])
            blk = plan.bsr[int(voff[k]): int(voff[k]) + (f1 - f0) * (g1 - g0)].cpu().numpy()
            blk = blk.reshape(g1 - g0, f1 - f0).T
            for i in range(f1 - f0):
                for j in range(g1 - g0):
                    got[(i, g0 + j)] = blk[i, j]
        keys = sorted(set(ref_rows) | set(got))
        a = np.array([got.get(k, 0.0) for k in keys])
        b = np.array([ref_rows.get(k, 0.0) for k in keys])
        assert rel(a, b) < TOL, (f, rel(a, b))
        e_got = E_gpu[f0:f1].cpu().numpy()
        assert rel(e_got, ref_E) < 1e-12 + max(np.linalg.cond(cond(e)[0].A) for e in owners[f]) * RESID_ROUNDING


@pytest.mark.parametrize("which,degree", [("ns23", 20), ("ns14", 20), ("ns14", 0)])
def test_ns_mixed_skeleton_solve_meets_gate(hdg, which, degree):
    """Mixed precision on Navier-Stokes: the float32 inner solve (with the float16 polynomial
    preconditioner, or plain block-Jacobi GMRES) inside float64 refinement reaches the 1e-10
    gate on the oracle's own K and E; forward error and the back-substituted update follow."""
    import torch
    case = _case(which)
    _say(f"ns mixed gate {which} degree {degree}")
    step = O.newton_step(case)
    plan = hdg.HDGPlan.from_case(case, precision="mixed")
    plan.hdg_set_poly_degree(degree)
    w, q, lam = _state(plan, case)
    plan.hdg_assemble_condense(w, lam, q=q)
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    it, relres, _ = plan.hdg_skeleton_solve(dlam, rtol=1e-10, restart=30)
    x = dlam.cpu().numpy()
    res_oracle = np.linalg.norm(step.E - step.K @ x) / np.linalg.norm(step.E)
    fwd = rel(x, step.dlam)
    _say(f"  iters {it} relres {relres:.3e} on oracle K {res_oracle:.3e} forward {fwd:.3e}")
    assert relres <= 1e-10
    assert res_oracle <= 2e-10
    assert fwd < 1e-6
    dw = torch.zeros_like(w)
    dq = torch.zeros_like(q)
    plan.hdg_back_substitute(dlam, dw, dq)
    ref_w = np.zeros_like(case.W)
    ref_q = np.zeros_like(case.Q)
    for e in range(case.n_elements):
        ref_w[e], ref_q[e] = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(dw.cpu().numpy(), ref_w) < 1e-6
    assert rel(dq.cpu().numpy(), ref_q) < 1e-6


def test_ns_shock_capturing_matches_oracle(hdg):
    """The viscous form of the shock capturing (Sec. 3.2, q_h in place of grad w_h) with a
    pseudo-time step: element blocks (inspection path), local solutions, K and E (condensation
    path), and the back-substitution."""
    import torch
    case = hi.make_case("ns", 3, [1, 2, 3], 0.8, 1.25, 8e-2, seed=43, reynolds=200.0)
    case.sc_eps0 = 0.2
    case.cfl = 5.0
    _say("ns shock capturing")
    step = O.newton_step(case)
    mesh = step.mesh
    eps = [O.shock_viscosity(mesh, e, case.W[e, :, :hi.n_modes(int(case.degree[e]))],
                             case.Q[e, :, :hi.n_modes(int(case.degree[e]))]) for e in range(case.n_elements)]
    _say(f"  eps_K max {max(eps):.3e}")
    assert max(eps) > 1e-4        # the term is switched on
    plan = hdg.HDGPlan.from_case(case)
    w, q, lam = _state(plan, case)
    for e in range(case.n_elements):
        gb = plan.debug_element_blocks(e, w, lam, q)
        for k, ref in (("A", step.blocks[e].A), ("r", step.blocks[e].r)):
            tol = TOL if k == "A" else tol_resid(step.blocks[e].A)
            assert rel(gb[k], ref) < tol, (e, k, rel(gb[k], ref))
    plan.hdg_assemble_condense(w, lam, q=q)
    torch.cuda.synchronize()
    for e in range(case.n_elements):
        X, y = plan.debug_local_solution(e)
        c = step.cond[e]
        assert rel(X, c.X) < TOL, (e, rel(X, c.X))
        assert rel(y, c.y) < tol_resid(step.blocks[e].A), (e, rel(y, c.y))
    assert rel(plan.skeleton_matrix_dense(), step.K.toarray()) < TOL
    assert rel(plan.rhs.cpu().numpy(), step.E) < TOL
    dl = torch.tensor(step.dlam, dtype=torch.float64, device=plan.device)
    dw = torch.zeros_like(w)
    dq = torch.zeros_like(q)
    plan.hdg_back_substitute(dl, dw, dq)
    rw, rq = np.zeros_like(case.W), np.zeros_like(case.Q)
    for e in range(case.n_elements):
        rw[e], rq[e] = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(dw.cpu().numpy(), rw) < 1e-11
    assert rel(dq.cpu().numpy(), rq) < 1e-11
