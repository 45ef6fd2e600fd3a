"""GPU parity of the relaxed Newton iteration (Sec. 3.3, eq. cfl): the residual norm the
CFL schedule reads, the state update, and whole pseudo-transient runs against the oracle's
iteration on the same seeded inputs."""
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
    if which == "hp":
        return hi.make_case("euler", 4, [1, 2, 3, 4], 0.6, 1.5, 2e-2, seed=3)
    return hi.make_case("ns", 3, [2, 3], 0.5, 1.0, 2e-2, seed=21, reynolds=200.0)


def _state(plan, case):
    import torch
    w = torch.tensor(case.W, dtype=torch.float64, device=plan.device)
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=plan.device)
    q = torch.tensor(case.Q, dtype=torch.float64, device=plan.device) if case.Q is not None else None
    return w, lam, q


@pytest.mark.parametrize("which", ["c1", "hp", "ns23"])
def test_residual_norm_matches_oracle(hdg, which):
    case = _case(which)
    _say(f"residual norm {which}")
    plan = hdg.HDGPlan.from_case(case)
    w, lam, q = _state(plan, case)
    plan.hdg_assemble_condense(w, lam, q=q)
    got = plan.hdg_residual_norm()
    ref = O.residual_norm(case, case.W, case.lam, case.Q)
    assert abs(got - ref) <= 1e-12 * ref, (got, ref)
    # fixed-order reduction: the same bits again, also after a second assembly
    plan.hdg_assemble_condense(w, lam, q=q)
    assert plan.hdg_residual_norm() == got


def test_apply_update_adds_the_step(hdg):
    import torch
    case = _case("ns23")
    _say("apply update")
    plan = hdg.HDGPlan.from_case(case)
    w, lam, q = _state(plan, case)
    rng = np.random.default_rng(5)
    dw, dq, dl = (torch.tensor(rng.standard_normal(tuple(x.shape)), device=w.device) for x in (w, q, lam))
    ref = (w + dw, q + dq, lam + dl)
    plan.hdg_apply_update(w, lam, dw, dl, q=q, dq=dq)
    torch.cuda.synchronize()
    for got, r in zip((w, q, lam), ref):
        assert torch.equal(got, r)


@pytest.mark.parametrize("which", ["c1", "ns23"])
def test_pseudo_transient_matches_oracle(hdg, which):
    """Four relaxed Newton iterations with a gentle ramp (c0 = 10, c1 = 1, n0 = 2, so the
    pseudo-time term shapes every step): residual history, CFL history and final state."""
    case = _case(which)
    _say(f"pseudo-transient {which}")
    ref = O.pseudo_transient(case, 4, c0=10.0, c1=1.0, n0=2)
    plan = hdg.HDGPlan.from_case(case)
    w, lam, q = _state(plan, case)
    out = plan.hdg_pseudo_transient_solve(w, lam, q=q, c0=10.0, c1=1.0, n0=2, max_steps=4, rel_tol=0.0,
                                          gmres_rtol=1e-13)
    _say(f"  res {out['res_history']} cfl {out['cfl_history']} gmres {out['gmres_iters']}")
    assert out["steps"] == 4 and out["gmres_not_converged"] == 0
    assert np.abs(out["res_history"] - ref.res).max() <= 1e-9 * ref.res[0]
    assert np.abs(out["cfl_history"] / np.array(ref.cfl) - 1.0).max() <= 1e-8
    assert O.relative_error(w.cpu().numpy(), ref.W) < 1e-10
    lam_ref = plan.pack_lambda(ref.lam)
    assert O.relative_error(lam.cpu().numpy(), lam_ref) < 1e-10
    if q is not None:
        assert O.relative_error(q.cpu().numpy(), ref.Q) < 1e-9


def test_pseudo_transient_converges_with_the_paper_constants(hdg):
    """c0 = 1e6, c1 = 1e3, n0 = 4 on the 8x8 p=1 workload: the residual falls by ten orders
    of magnitude, monotonically, within a few iterations (mixed-precision skeleton solves)."""
    case = _case("c1")
    _say("pseudo-transient paper constants")
    plan = hdg.HDGPlan.from_case(case, precision="mixed")
    w, lam, q = _state(plan, case)
    out = plan.hdg_pseudo_transient_solve(w, lam, max_steps=10, rel_tol=1e-10, gmres_rtol=1e-10)
    _say(f"  res {out['res_history']} steps {out['steps']}")
    assert out["converged"] and out["steps"] <= 6
    h = out["res_history"]
    assert np.all(np.diff(h) < 0)
    assert h[-1] <= 1e-10 * h[0]
