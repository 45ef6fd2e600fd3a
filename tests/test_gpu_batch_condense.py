"""Batched condensation of several cases (hdg_assemble_condense_batch): the elements of every
Euler plan share one launch per bucket shape, and the outputs are bit-identical to each plan's
own hdg_assemble_condense. Plans that cannot join (Navier-Stokes, the mixed-precision condensation,
a first call) are condensed one by one inside the same call."""
import numpy as np
import pytest

import hdg_inputs as hi

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[batch] {msg}", flush=True)


def _state(plan, case, torch):
    dev = plan.device
    w = torch.tensor(case.W, dtype=torch.float64, device=dev)
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
    q = torch.tensor(case.Q, dtype=torch.float64, device=dev) if case.Q is not None else None
    return w, lam, q


def _outputs(plan):
    return plan.bsr.cpu().numpy().copy(), plan.rhs.cpu().numpy().copy(), plan.store.cpu().numpy().copy()


def _reference(hdg, cases, precisions, torch):
    plans, states, refs = [], [], []
    for case, prec in zip(cases, precisions):
        plan = hdg.HDGPlan.from_case(case, precision=prec)
        w, lam, q = _state(plan, case, torch)
        plan.hdg_assemble_condense(w, lam, q=q)     # first call: picks the kernel variants
        plan.hdg_assemble_condense(w, lam, q=q)
        torch.cuda.synchronize()
        plans.append(plan)
        states.append((w, lam, q))
        refs.append(_outputs(plan))
    return plans, states, refs


def _clobber(plans):
    for p in plans:
        p.bsr.fill_(float("nan"))
        p.rhs.fill_(float("nan"))
        p.store.fill_(255)


def test_batch_matches_single_plan_calls(hdg):
    import torch
    cases = [hi.make_case("euler", 6, [1, 2, 3], 0.5, 1.0, 1e-2, seed=11),
             hi.make_case("euler", 8, [2, 3], 0.7, -1.5, 1e-2, seed=12),
             hi.config_case("c1"),
             hi.make_case("ns", 4, [2, 3], 0.5, 1.0, 1e-2, seed=13, reynolds=100.0),
             hi.make_case("euler", 5, [1, 2], 0.6, 0.0, 1e-2, seed=14)]
    precisions = ["fp64", "mixed", "fp64", "mixed", "mixed_condense"]
    _say("5 plans: 3 joinable Euler, 1 Navier-Stokes, 1 mixed-precision condensation")
    plans, states, refs = _reference(hdg, cases, precisions, torch)
    for rep in range(2):
        _clobber(plans)
        torch.cuda.synchronize()
        joined = hdg.hdg_assemble_condense_batch(plans, [s[0] for s in states], [s[1] for s in states],
                                                 qs=[s[2] for s in states])
        torch.cuda.synchronize()
        assert joined == 3, joined
        for k, p in enumerate(plans):
            got = _outputs(p)
            for name, a, b in zip(("bsr", "rhs", "store"), got, refs[k]):
                assert np.array_equal(a, b), (rep, k, name)


def test_batch_splits_groups_of_more_than_eight(hdg):
    import torch
    cases = [hi.make_case("euler", 4 + (k % 3), [2], 0.5, 0.5 * k, 1e-2, seed=20 + k) for k in range(11)]
    _say("11 Euler plans of one bucket shape (two launches per shape)")
    plans, states, refs = _reference(hdg, cases, ["fp64"] * len(cases), torch)
    _clobber(plans)
    joined = hdg.hdg_assemble_condense_batch(plans, [s[0] for s in states], [s[1] for s in states])
    torch.cuda.synchronize()
    assert joined == len(cases)
    for k, p in enumerate(plans):
        for a, b in zip(_outputs(p), refs[k]):
            assert np.array_equal(a, b), k


def test_batch_rejects_a_repeated_plan(hdg):
    import torch
    case = hi.config_case("c1")
    plan = hdg.HDGPlan.from_case(case)
    w, lam, _ = _state(plan, case, torch)
    with pytest.raises(hdg.HdgError):
        hdg.hdg_assemble_condense_batch([plan, plan], [w, w], [lam, lam])
    assert hdg.hdg_assemble_condense_batch([], [], []) == 0


def test_new_plan_of_known_shapes_joins_on_its_first_call(hdg):
    """Serving builds a plan per request: a plan whose bucket shapes the process has already tuned
    takes the kept variants and joins the batch on its very first call, with the same bits."""
    import torch
    case_a = hi.make_case("euler", 6, [1, 2, 3], 0.5, 1.0, 1e-2, seed=31)
    case_b = hi.make_case("euler", 7, [2, 3], 0.6, 2.0, 1e-2, seed=32)
    plans, states, refs = _reference(hdg, [case_a, case_b], ["fp64", "fp64"], torch)
    fresh = [hdg.HDGPlan.from_case(c) for c in (case_a, case_b)]
    st = [_state(p, c, torch) for p, c in zip(fresh, (case_a, case_b))]
    _say("two fresh plans of tuned shapes")
    joined = hdg.hdg_assemble_condense_batch(fresh, [s[0] for s in st], [s[1] for s in st])
    torch.cuda.synchronize()
    assert joined == 2
    for k, p in enumerate(fresh):
        for a, b in zip(_outputs(p), refs[k]):
            assert np.array_equal(a, b), k
