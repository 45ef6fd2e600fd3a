"""Every kernel variant of the float64 Euler condensation against the oracle.

The first call on a plan times four variants per bucket shape and keeps the fastest, so the
parity tests only see the variants that won on their inputs. Here each variant is forced in
turn (hdg_debug_condense_variant): the register-resident and the blocked matrix-core
Gauss-Jordan elimination, each at a 128- and a 256-VGPR budget, with and without shock
capturing (Sec. 3.2). Each must reproduce the oracle's local solutions X_K, y_K, the skeleton
matrix K and right-hand side E (Sec. 3.4, eq. hybridsystem) to the float64 gate."""
import sys

import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-12
RESID_ROUNDING = 1e-13   # the element residual's float64 rounding (relative), as in the parity tests


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(which, sc):
    if which == "hp":
        case = hi.make_case("euler", 4, [1, 2, 3, 4], 0.8, 1.25, 8e-2 if sc else 2e-2, seed=43 if sc else 3)
    else:
        case = hi.make_case("euler", 3, [3, 4, 5], 0.8, 1.25, 8e-2 if sc else 5e-2, seed=44 if sc else 4)
    if sc:
        case.sc_eps0 = 0.2
    return case


@pytest.mark.parametrize("sc", [False, True], ids=["plain", "shock"])
@pytest.mark.parametrize("which", ["hp", "hp5"])
def test_every_condensation_variant_matches_oracle(hdg, which, sc):
    import torch
    case = _case(which, sc)
    step = O.newton_step(case)
    Ko = step.K.toarray()
    plan = hdg.HDGPlan.from_case(case)
    w = torch.tensor(case.W, dtype=torch.float64, device=plan.device).contiguous()
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=plan.device)
    for variant in (0, 1, 2, 3, -1):
        _say(f"condense {which} {'shock capturing' if sc else 'plain'} variant {variant}")
        plan.debug_condense_variant(variant)
        plan.bsr.fill_(float("nan"))
        plan.rhs.fill_(float("nan"))
        for rep in range(2):   # the first call launches directly, the second replays the captured graph
            plan.hdg_assemble_condense(w, lam)
            torch.cuda.synchronize()
        for e in range(case.n_elements):
            X, y = plan.debug_local_solution(e)
            c = step.cond[e]
            ty = TOL + np.linalg.cond(step.blocks[e].A) * RESID_ROUNDING
            assert O.relative_error(y, c.y) < ty, (variant, e, O.relative_error(y, c.y))
            if c.X.size:
                assert O.relative_error(X, c.X) < TOL, (variant, e, O.relative_error(X, c.X))
        assert O.relative_error(plan.skeleton_matrix_dense(), Ko) < TOL, variant
        assert O.relative_error(plan.rhs.cpu().numpy(), step.E) < TOL + 2 * RESID_ROUNDING, variant


def test_forced_variant_is_rejected_outside_its_range(hdg):
    plan = hdg.HDGPlan.from_case(hi.config_case("c1"), allocate=False)
    for bad in (-2, 4):
        with pytest.raises(hdg.HdgError):
            plan.debug_condense_variant(bad)
