"""The allocation-free marking entry point (hdg_mark_elements_noalloc, static device scratch)
against hdg_mark_elements (caller's workspace): same flags, sensor and count, bit for bit, on two
calls in a row, the second on a smaller mesh (the static scratch keeps the first call's
contents)."""
import numpy as np
import pytest

import hdg_inputs as hi

pytestmark = pytest.mark.gpu


def _marking_inputs(hdg, name, ng, seed):
    import torch
    case = hi.config_case(name, ng)
    plan = hdg.HDGPlan.from_case(case)
    w = torch.tensor(case.W, dtype=torch.float64, device=plan.device)
    eta = torch.tensor(np.random.default_rng(seed).exponential(size=case.n_elements), device=plan.device)
    return case, plan, w, eta


def test_noalloc_marking_matches_workspace_marking(hdg):
    import torch
    big = _marking_inputs(hdg, "c3", 48, 11)       # hp degrees 1..5, 4608 elements
    small = _marking_inputs(hdg, "c2", 12, 12)     # p = 3, 288 elements
    got = []
    for case, plan, w, eta in (big, small):
        flag = torch.full((case.n_elements,), -1, dtype=torch.int32, device=plan.device)
        sensor = torch.full((case.n_elements,), -1.0, dtype=torch.float64, device=plan.device)
        m = plan.hdg_mark_elements_noalloc(w, eta, flag, sensor, theta=0.05, eps_s=1e-6)
        flag2 = torch.full_like(flag, -1)
        m2 = plan.hdg_mark_elements_noalloc(w, eta, flag2, None, theta=0.3, eps_s=1e-3)
        torch.cuda.synchronize()
        got.append((flag.cpu().numpy(), sensor.cpu().numpy(), m, flag2.cpu().numpy(), m2))
    for (case, plan, w, eta), (flag, sensor, m, flag2, m2) in zip((big, small), got):
        ref_flag, ref_sensor, ref_m = plan.hdg_mark_elements(w, eta, theta=0.05, eps_s=1e-6)
        ref_flag2, _, ref_m2 = plan.hdg_mark_elements(w, eta, theta=0.3, eps_s=1e-3)
        torch.cuda.synchronize()
        assert m == ref_m and m2 == ref_m2
        assert 0 < m < case.n_elements
        assert np.array_equal(flag, ref_flag.cpu().numpy())
        assert np.array_equal(flag2, ref_flag2.cpu().numpy())
        assert np.array_equal(sensor.view(np.int64), ref_sensor.cpu().numpy().view(np.int64))
