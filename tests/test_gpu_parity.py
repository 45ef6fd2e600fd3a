"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded
inputs. Tolerances follow the float64 gate: 1e-12 relative on blocks, local solutions,
skeleton matrix, right-hand side and back-substitution; the skeleton solve to a relative
residual of 1e-12 on the oracle's own K and E."""
import sys

import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-12
# The element residual of a smooth state is a sum with cancellation: evaluated in float64 it
# carries a relative rounding of up to ~4e-14 (measured against a long-double evaluation of
# the oracle on the 64x64 p=3 workload). Quantities driven by it (y_K = A_K^-1 r_K and the
# updates built from y_K) inherit that error times kappa(A_K), so their gate is
# 1e-12 + kappa(A_K) * 1e-13.
RESID_ROUNDING = 1e-13


def tol_resid(A) -> float:
    return TOL + np.linalg.cond(A) * RESID_ROUNDING


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return O.relative_error(a, b)


def _device_state(hdg, plan, case):
    import torch
    w = torch.tensor(case.W, dtype=torch.float64, device=plan.device).contiguous()
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=plan.device)
    return w, lam


def _tiny_hp(seed=3):
    return hi.make_case("euler", 4, [1, 2, 3, 4], 0.6, 1.5, 2e-2, seed=seed)


def _tiny_hp5(seed=4):
    """Degrees 3..5: exercises the LDS-resident kernel (degree 4, 5) and face degree 5."""
    return hi.make_case("euler", 3, [3, 4, 5], 0.8, 1.25, 5e-2, seed=seed)


def _case(which):
    if which == "c1":
        return hi.config_case("c1")
    return _tiny_hp() if which == "hp" else _tiny_hp5()


@pytest.mark.parametrize("which", ["c1", "hp", "hp5"])
def test_plan_faces_match_oracle(hdg, which):
    case = _case(which)
    _say(f"plan faces {which}")
    plan = hdg.HDGPlan.from_case(case)
    mesh = O.Mesh(case, O.make_physics(case))
    assert np.array_equal(plan.face_vertices, mesh.face_vertices)
    assert np.array_equal(plan.face_degree, mesh.face_degree)
    assert np.array_equal(plan.face_offset, mesh.face_offset)
    assert plan.sizes["n_boundary_faces"] == int((mesh.elem_faces < 0).sum())


@pytest.mark.parametrize("which", ["c1", "hp", "hp5"])
def test_element_blocks_match_oracle(hdg, which):
    case = _case(which)
    _say(f"element blocks {which}")
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    mesh = O.Mesh(case, O.make_physics(case))
    st = O.State(mesh, case.W, case.lam)
    elems = list(range(0, case.n_elements, max(1, case.n_elements // 12))) + [case.n_elements - 1]
    for e in elems:
        ob = O.element_blocks(st, e)
        gb = plan.debug_element_blocks(e, w, lam)
        for k, ref in (("A", ob.A), ("B", ob.B), ("C", ob.C), ("D", ob.D), ("r", ob.r), ("rl", ob.rl)):
            assert gb[k].shape == ref.shape, (e, k, gb[k].shape, ref.shape)
            if ref.size:
                assert rel(gb[k], ref) < TOL, (e, k, rel(gb[k], ref))


@pytest.fixture(scope="module")
def c1_oracle():
    case = hi.config_case("c1")
    return case, O.newton_step(case)


@pytest.mark.parametrize("which", ["c1", "hp", "hp5"])
def test_condensation_matches_oracle(hdg, which, c1_oracle):
    if which == "c1":
        case, step = c1_oracle
    else:
        case = _case(which)
        step = O.newton_step(case)
    _say(f"condense {which}")
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
    import torch
    torch.cuda.synchronize()
    for e in range(case.n_elements):
        X, y = plan.debug_local_solution(e)
        c = step.cond[e]
        assert rel(y, c.y) < TOL, (e, rel(y, c.y))
        if c.X.size:
            assert rel(X, c.X) < TOL, (e, rel(X, c.X))
    K = plan.skeleton_matrix_dense()
    Ko = step.K.toarray()
    assert rel(K, Ko) < TOL
    assert rel(plan.rhs.cpu().numpy(), step.E) < TOL


@pytest.mark.parametrize("which", ["c1", "hp", "hp5"])
def test_skeleton_solve_meets_fp64_gate(hdg, which, c1_oracle):
    import torch
    if which == "c1":
        case, step = c1_oracle
    else:
        case = _case(which)
        step = O.newton_step(case)
    _say(f"skeleton solve {which}")
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    it, relres, _ = plan.hdg_skeleton_solve(dlam, rtol=1e-12, restart=30)
    x = dlam.cpu().numpy()
    res_oracle = np.linalg.norm(step.E - step.K @ x) / np.linalg.norm(step.E)
    _say(f"  iters {it} relres {relres:.3e} on oracle K {res_oracle:.3e} forward {rel(x, step.dlam):.3e}")
    assert relres <= 1e-12
    assert res_oracle <= 2e-12
    assert rel(x, step.dlam) < 1e-9


@pytest.mark.parametrize("which", ["c1", "hp", "hp5"])
def test_back_substitution_matches_oracle(hdg, which, c1_oracle):
    """Given the oracle's dLambda, the reconstruction agrees to 1e-12."""
    import torch
    if which == "c1":
        case, step = c1_oracle
    else:
        case = _case(which)
        step = O.newton_step(case)
    _say(f"back substitute {which}")
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
    dl = torch.tensor(step.dlam, dtype=torch.float64, device=plan.device)
    dw = torch.zeros_like(w)
    plan.hdg_back_substitute(dl, dw)
    got = dw.cpu().numpy()
    ref = np.zeros_like(got)
    for e in range(case.n_elements):
        ref[e], _ = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(got, ref) < TOL


def test_newton_step_end_to_end_c1(hdg, c1_oracle):
    import torch
    case, step = c1_oracle
    _say("end to end c1")
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    plan.hdg_skeleton_solve(dlam, rtol=1e-13, restart=30)
    dw = torch.zeros_like(w)
    plan.hdg_back_substitute(dlam, dw)
    ref = np.zeros_like(case.W)
    for e in range(case.n_elements):
        ref[e], _ = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(dlam.cpu().numpy(), step.dlam) < 1e-10
    assert rel(dw.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("which", ["c1", "hp"])
def test_pseudo_time_step_matches_oracle(hdg, which):
    """The local pseudo-time term of Sec. 3.3 at CFL 5: element blocks, local solutions,
    skeleton system and the full Newton update agree with the oracle."""
    import torch
    case = _case(which)
    case.cfl = 5.0
    _say(f"pseudo-time {which}")
    step = O.newton_step(case)
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    for e in range(0, case.n_elements, max(1, case.n_elements // 8)):
        gb = plan.debug_element_blocks(e, w, lam)
        assert rel(gb["A"], step.blocks[e].A) < TOL, (e, rel(gb["A"], step.blocks[e].A))
    plan.hdg_assemble_condense(w, lam)
    torch.cuda.synchronize()
    for e in range(case.n_elements):
        X, y = plan.debug_local_solution(e)
        c = step.cond[e]
        assert rel(y, c.y) < TOL, (e, rel(y, c.y))
        if c.X.size:
            assert rel(X, c.X) < TOL, (e, rel(X, c.X))
    assert rel(plan.skeleton_matrix_dense(), step.K.toarray()) < TOL
    assert rel(plan.rhs.cpu().numpy(), step.E) < TOL
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    plan.hdg_skeleton_solve(dlam, rtol=1e-13, restart=30)
    dw = torch.zeros_like(w)
    plan.hdg_back_substitute(dlam, dw)
    ref = np.zeros_like(case.W)
    for e in range(case.n_elements):
        ref[e], _ = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(dlam.cpu().numpy(), step.dlam) < 1e-10
    assert rel(dw.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("which", ["hp", "hp5"])
def test_shock_capturing_matches_oracle(hdg, which):
    """Shock capturing of Sec. 3.2 (epsilon_0 = 0.2, beta = 0) on a strongly perturbed state:
    element blocks, condensation and the full Newton update agree with the oracle."""
    import torch
    case = (hi.make_case("euler", 4, [1, 2, 3, 4], 0.8, 1.25, 8e-2, seed=43) if which == "hp"
            else hi.make_case("euler", 3, [3, 4, 5], 0.8, 1.25, 8e-2, seed=44))
    case.sc_eps0 = 0.2
    _say(f"shock capturing {which}")
    step = O.newton_step(case)
    eps = [O.shock_viscosity(step.mesh, e, case.W[e, :, :hi.n_modes(int(case.degree[e]))])
           for e in range(case.n_elements)]
    assert max(eps) > 1e-4
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    for e in range(0, case.n_elements, max(1, case.n_elements // 10)):
        gb = plan.debug_element_blocks(e, w, lam)
        ob = step.blocks[e]
        assert rel(gb["A"], ob.A) < TOL, (e, rel(gb["A"], ob.A))
        assert rel(gb["r"], ob.r) < tol_resid(ob.A), (e, rel(gb["r"], ob.r))
    plan.hdg_assemble_condense(w, lam)
    torch.cuda.synchronize()
    for e in range(case.n_elements):
        X, y = plan.debug_local_solution(e)
        c = step.cond[e]
        assert rel(y, c.y) < tol_resid(step.blocks[e].A), (e, rel(y, c.y))
        if c.X.size:
            assert rel(X, c.X) < TOL, (e, rel(X, c.X))
    assert rel(plan.skeleton_matrix_dense(), step.K.toarray()) < TOL
    assert rel(plan.rhs.cpu().numpy(), step.E) < tol_resid(np.eye(2))
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    plan.hdg_skeleton_solve(dlam, rtol=1e-13, restart=30)
    dw = torch.zeros_like(w)
    plan.hdg_back_substitute(dlam, dw)
    ref = np.zeros_like(case.W)
    for e in range(case.n_elements):
        ref[e], _ = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(dlam.cpu().numpy(), step.dlam) < 1e-10
    assert rel(dw.cpu().numpy(), ref) < 1e-10


def test_shock_capturing_leaves_the_free_stream_steady(hdg):
    """The shock-capturing term vanishes at a uniform free stream (d(w) = 0 there), for Euler and
    for the viscous form of Navier-Stokes: E = 0 with the term switched on."""
    import torch
    for ph in ("euler", "ns"):
        case = hi.make_case(ph, 4, [1, 2, 3], 0.5, 2.0, 0.0, seed=9, free_stream_only=True,
                            reynolds=200.0 if ph == "ns" else 0.0)
        case.sc_eps0 = 0.2
        _say(f"shock capturing at the free stream ({ph})")
        plan = hdg.HDGPlan.from_case(case)
        w = torch.tensor(case.W, dtype=torch.float64, device=plan.device)
        lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=plan.device)
        q = torch.tensor(case.Q, dtype=torch.float64, device=plan.device) if case.Q is not None else None
        nrm = plan.hdg_assemble_condense(w, lam, q=q, want_norm=True)
        assert nrm < 1e-12, (ph, nrm)


def test_free_stream_gives_zero_rhs(hdg):
    """A uniform free stream is a discrete steady state: E = 0 and the local right-hand sides vanish."""
    import torch
    case = hi.make_case("euler", 6, [1, 2, 3, 4], 0.5, 2.0, 0.0, seed=9, free_stream_only=True)
    _say("free stream")
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    nrm = plan.hdg_assemble_condense(w, lam, want_norm=True)
    assert nrm < 1e-13
    for e in range(0, case.n_elements, 7):
        _, y = plan.debug_local_solution(e)
        assert np.abs(y).max() < 1e-13


def test_singular_element_is_reported(hdg):
    """A NaN in the state is reported as HDG_ERR_NONFINITE with the element id."""
    import torch
    case = hi.config_case("c1")
    _say("nonfinite state")
    plan = hdg.HDGPlan.from_case(case)
    W = case.W.copy()
    W[17, 2, 1] = np.nan
    w = torch.tensor(W, device=plan.device)
    lam = torch.tensor(plan.pack_lambda(case.lam), device=plan.device)
    status = torch.zeros(case.n_elements, dtype=torch.int32, device=plan.device)
    with pytest.raises(hdg.HdgError) as ei:
        plan.hdg_assemble_condense(w, lam, elem_status=status)
    assert ei.value.status in (3, 4)
    assert int(status[17].item()) in (3, 4)


def test_gmres_max_iter_returns_not_converged(hdg, c1_oracle):
    import torch
    case, step = c1_oracle
    _say("max_iter")
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    it, relres, st = plan.hdg_skeleton_solve(dlam, rtol=1e-12, restart=30, max_iter=5, raise_on_fail=False)
    assert st == 5 and it <= 5 and relres > 1e-12
    # the returned iterate is a real iterate: its residual equals the reported one
    x = dlam.cpu().numpy()
    K = plan.skeleton_matrix_dense()
    E = plan.rhs.cpu().numpy()
    assert abs(np.linalg.norm(E - K @ x) / np.linalg.norm(E) - relres) < 1e-10


def test_c2_full_size_sampled(hdg):
    """The 64x64 p=3 workload in the benchmark's launch configuration: sampled elements'
    local solutions and owned skeleton blocks against the oracle, the skeleton solve's
    residual recomputed on the CPU from the returned matrix."""
    import scipy.sparse as sp
    import torch
    case = hi.config_case("c2")
    _say("c2 full size")
    plan = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
    torch.cuda.synchronize()
    mesh = O.Mesh(case, O.make_physics(case))
    st = O.State(mesh, case.W, case.lam)
    rng = np.random.default_rng(0)
    sample = sorted(set(rng.choice(case.n_elements, 24, replace=False).tolist() + [0, case.n_elements - 1]))
    rp, col, voff = plan.pattern()
    vals = plan.bsr.cpu().numpy()
    for e in sample:
        ob = O.element_blocks(st, e)
        oc = O.condense(ob)
        X, y = plan.debug_local_solution(e)
        assert rel(X, oc.X) < TOL, (e, rel(X, oc.X))
        assert rel(y, oc.y) < tol_resid(ob.A), (e, rel(y, oc.y), tol_resid(ob.A))
        # off-diagonal blocks of S_e have e as their only contributor
        offs = np.concatenate([[0], np.cumsum(ob.fsizes)])
        for a, fa in enumerate(ob.faces):
            for b, fb in enumerate(ob.faces):
                if fa == fb:
                    continue
                blk = [k for k in range(rp[fa], rp[fa + 1]) if col[k] == fb][0]
                sa, sb = ob.fsizes[a], ob.fsizes[b]
                G = vals[voff[blk]: voff[blk] + sa * sb].reshape(sb, sa).T
                assert rel(G, oc.S[offs[a]:offs[a + 1], offs[b]:offs[b + 1]]) < TOL
    # skeleton solve at full size
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    it, relres, _ = plan.hdg_skeleton_solve(dlam, rtol=1e-12, restart=30)
    _say(f"  c2 gmres iters {it} relres {relres:.3e}")
    n = plan.n_skel
    rows, cols, data = [], [], []
    for f in range(len(plan.face_degree)):
        f0, f1 = plan.face_offset[f], plan.face_offset[f + 1]
        for k in range(rp[f], rp[f + 1]):
            g = col[k]
            g0, g1 = plan.face_offset[g], plan.face_offset[g + 1]
            blk = vals[voff[k]: voff[k] + (f1 - f0) * (g1 - g0)].reshape(g1 - g0, f1 - f0).T
            rr, cc = np.meshgrid(np.arange(f0, f1), np.arange(g0, g1), indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); data.append(blk.ravel())
    K = sp.csr_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    E = plan.rhs.cpu().numpy()
    x = dlam.cpu().numpy()
    cpu_res = np.linalg.norm(E - K @ x) / np.linalg.norm(E)
    assert relres <= 1e-12 and cpu_res <= 2e-12
    # back-substitution of sampled elements with the GPU's dLambda
    dw = torch.zeros_like(w)
    plan.hdg_back_substitute(dlam, dw)
    dwh = dw.cpu().numpy()
    for e in sample[:8]:
        ob = O.element_blocks(st, e)
        oc = O.condense(ob)
        d = O.elem_dofs(mesh, ob)
        ref = oc.y - oc.X @ x[d]
        assert rel(dwh[e, :, : ref.size // 4].reshape(-1), ref) < tol_resid(ob.A)


def test_graph_replays_match_direct_launches(hdg, c1_oracle):
    """The captured condensation sequence and GMRES cycles, replayed across several steps with
    eager work in between, give the same bits as direct launches (deterministic kernels; the
    kernel variants tuned by the first plan are reused by every later plan of the process)."""
    import os
    import torch
    case, step = c1_oracle
    _say("graph replays vs direct launches")
    os.environ["HDG_DISABLE_GRAPHS"] = "1"
    try:
        eager = hdg.HDGPlan.from_case(case)
    finally:
        del os.environ["HDG_DISABLE_GRAPHS"]
    graph = hdg.HDGPlan.from_case(case)
    w, lam = _device_state(hdg, eager, case)
    eager.hdg_assemble_condense(w, lam)
    ref = torch.zeros(eager.n_skel, dtype=torch.float64, device=eager.device)
    it_ref, rr_ref, _ = eager.hdg_skeleton_solve(ref, rtol=1e-12, restart=30)
    for rep in range(3):
        graph.hdg_assemble_condense(w, lam)
        torch.cuda.synchronize()
        assert torch.equal(graph.bsr, eager.bsr), rep
        assert torch.equal(graph.rhs, eager.rhs), rep
        assert torch.equal(graph.store, eager.store), rep
        got = torch.zeros_like(ref)
        it, rr, _ = graph.hdg_skeleton_solve(got, rtol=1e-12, restart=30)
        torch.cuda.synchronize()
        assert it == it_ref and rr == rr_ref, (rep, it, it_ref, rr, rr_ref)
        assert torch.equal(got, ref), rep


def test_c3_hp_full_size_sampled(hdg):
    """The 128x128 hp workload (degrees 1..5, 32768 elements): sampled local solutions against
    the oracle for every degree, and the skeleton solve's residual recomputed on the CPU."""
    import scipy.sparse as sp
    import torch
    case = hi.config_case("c3")
    _say("c3 full size")
    plan = hdg.HDGPlan.from_case(case)
    assert plan.sizes["n_buckets"] >= 10
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
    torch.cuda.synchronize()
    mesh = O.Mesh(case, O.make_physics(case))
    st = O.State(mesh, case.W, case.lam)
    rng = np.random.default_rng(1)
    sample = []
    for p in range(1, 6):
        idx = np.flatnonzero(case.degree == p)
        sample += rng.choice(idx, 3, replace=False).tolist()
    for e in sample:
        ob = O.element_blocks(st, e)
        oc = O.condense(ob)
        X, y = plan.debug_local_solution(e)
        assert rel(X, oc.X) < TOL, (e, case.degree[e], rel(X, oc.X))
        assert rel(y, oc.y) < tol_resid(ob.A), (e, case.degree[e], rel(y, oc.y))
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    it, relres, _ = plan.hdg_skeleton_solve(dlam, rtol=1e-10, restart=30)
    _say(f"  c3 gmres iters {it} relres {relres:.3e}")
    rp, col, voff = plan.pattern()
    vals = plan.bsr.cpu().numpy()
    n = plan.n_skel
    rows, cols, data = [], [], []
    for f in range(len(plan.face_degree)):
        f0, f1 = plan.face_offset[f], plan.face_offset[f + 1]
        for k in range(rp[f], rp[f + 1]):
            g = col[k]
            g0, g1 = plan.face_offset[g], plan.face_offset[g + 1]
            blk = vals[voff[k]: voff[k] + (f1 - f0) * (g1 - g0)].reshape(g1 - g0, f1 - f0).T
            rr, cc = np.meshgrid(np.arange(f0, f1), np.arange(g0, g1), indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); data.append(blk.ravel())
    K = sp.csr_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    E = plan.rhs.cpu().numpy()
    x = dlam.cpu().numpy()
    assert relres <= 1e-10 and np.linalg.norm(E - K @ x) / np.linalg.norm(E) <= 2e-10


@pytest.mark.parametrize("which", ["c1", "hp", "hp5"])
def test_mixed_mode_meets_gate(hdg, which, c1_oracle):
    """Mixed precision: the FP32 preconditioned matrix inside FP64 iterative refinement reaches
    the 1e-10 gate on the oracle's own K and E; the Newton update follows to the accuracy that
    the gate and the conditioning of K allow."""
    import torch
    if which == "c1":
        case, step = c1_oracle
    else:
        case = _case(which)
        step = O.newton_step(case)
    _say(f"mixed mode {which}")
    plan = hdg.HDGPlan.from_case(case, precision="mixed")
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
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
    plan.hdg_back_substitute(dlam, dw)
    gw = dw.cpu().numpy()
    ref = np.zeros_like(gw)
    for e in range(case.n_elements):
        ref[e], _ = O.unpack_local(step.mesh, e, step.du[e], case.W.shape[2])
    assert rel(gw, ref) < 1e-6


@pytest.mark.parametrize("precision,restart", [("fp64", 2), ("fp64", 32), ("mixed", 32)])
def test_gmres_restart_edges(hdg, c1_oracle, precision, restart):
    """Restart lengths at the ends of the supported range: with 2 nearly every column is the
    last of its cycle (rotated at the cycle's end); with 32 the basis is full and the second
    Gram-Schmidt pass is always taken. Both meet the gate on the oracle's K and E."""
    import torch
    case, step = c1_oracle
    _say(f"gmres restart {restart} {precision}")
    plan = hdg.HDGPlan.from_case(case, precision=precision)
    w, lam = _device_state(hdg, plan, case)
    plan.hdg_assemble_condense(w, lam)
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
    it, relres, _ = plan.hdg_skeleton_solve(dlam, rtol=1e-10, restart=restart, max_iter=400000)
    x = dlam.cpu().numpy()
    res_oracle = np.linalg.norm(step.E - step.K @ x) / np.linalg.norm(step.E)
    _say(f"  iters {it} relres {relres:.3e} on oracle K {res_oracle:.3e}")
    assert relres <= 1e-10
    assert res_oracle <= 2e-10
