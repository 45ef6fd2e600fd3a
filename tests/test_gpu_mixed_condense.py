"""The mixed-precision condensation (HDG_MIXED_CONDENSE): float32 elimination of the local
systems with float64 refinement of y_K. Against the CPU oracle: y_K and the condensed right-hand
side E (built from the refined y_K) meet the float64 gate of y_K; X_K and the skeleton matrix K
carry float32 accuracy (their errors are reported and only bounded loosely); the skeleton solve
meets 1e-10 on its own K; and the step agrees with the float64 step to float32 accuracy."""
import sys

import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O

pytestmark = pytest.mark.gpu

RESID_ROUNDING = 1e-13


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cases():
    return {"c1": hi.config_case("c1"),
            "hp4": hi.make_case("euler", 4, [1, 2, 3, 4], 0.6, 1.0, 2e-2, seed=31),
            "hp5": hi.make_case("euler", 4, [1, 2, 3, 4, 5], 0.8, 1.25, 5e-2, seed=32)}


def _bsr_to_csr(plan):
    import scipy.sparse as sp
    rp, col, voff = plan.pattern()
    vals = plan.bsr.cpu().numpy()
    rows, cols, data = [], [], []
    for f in range(len(plan.face_degree)):
        f0, f1 = plan.face_offset[f], plan.face_offset[f + 1]
        for k in range(rp[f], rp[f + 1]):
            g = col[k]
            g0, g1 = plan.face_offset[g], plan.face_offset[g + 1]
            blk = vals[voff[k]: voff[k] + (f1 - f0) * (g1 - g0)].reshape(g1 - g0, f1 - f0).T
            rr, cc = np.meshgrid(np.arange(f0, f1), np.arange(g0, g1), indexing="ij")
            rows.append(rr.ravel()); cols.append(cc.ravel()); data.append(blk.ravel())
    n = plan.n_skel
    return sp.csr_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


@pytest.mark.parametrize("which", ["c1", "hp4", "hp5"])
def test_mixed_condensation_against_oracle(hdg, which):
    import torch
    case = _cases()[which]
    _say(f"mixed condensation {which}")
    step = O.newton_step(case)
    plan = hdg.HDGPlan.from_case(case, precision="mixed_condense")
    dev = plan.device
    w = torch.tensor(case.W, dtype=torch.float64, device=dev)
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
    plan.hdg_assemble_condense(w, lam)
    torch.cuda.synchronize()
    worst_x, worst_y = 0.0, 0.0
    for e in range(case.n_elements):
        b, c = step.blocks[e], step.cond[e]
        X, y = plan.debug_local_solution(e)
        ex = O.relative_error(X, c.X) if c.X.size else 0.0
        ey = O.relative_error(y, c.y)
        kappa = np.linalg.cond(b.A)
        assert ey <= 1e-10 + kappa * RESID_ROUNDING, (e, int(case.degree[e]), ey, kappa)
        assert ex <= 1e-4, (e, ex)
        worst_x, worst_y = max(worst_x, ex), max(worst_y, ey)
    K = _bsr_to_csr(plan)
    E = plan.rhs.cpu().numpy()
    eK = abs(K - step.K).max() / abs(step.K).max()
    eE = O.relative_error(E, step.E)
    _say(f"  worst X {worst_x:.2e} y {worst_y:.2e}; K {eK:.2e}; E {eE:.2e}")
    assert eE <= 1e-10
    assert eK <= 1e-4
    # the skeleton solve meets the gate on the matrix this mode assembled
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=dev)
    it, relres, _ = plan.hdg_skeleton_solve(dlam, rtol=1e-10, restart=30)
    x = dlam.cpu().numpy()
    assert relres <= 1e-10
    assert np.linalg.norm(E - K @ x) / np.linalg.norm(E) <= 2e-10
    fwd = O.relative_error(x, step.dlam)
    _say(f"  iters {it} relres {relres:.2e} forward error vs the float64 step {fwd:.2e}")
    assert fwd <= 1e-3


def test_mixed_condensation_refused_for_navier_stokes(hdg):
    case = hi.make_case("ns", 3, 2, 0.5, 1.0, 1e-2, seed=33, reynolds=200.0)
    with pytest.raises(hdg.HdgError):
        hdg.HDGPlan.from_case(case, precision="mixed_condense")
