"""One plan serving several streams: full Newton steps (assemble + condense, skeleton solve,
back-substitution) issued concurrently from two host threads, each on its own HIP stream with
its own buffers, give the same bits as the same steps run one after the other."""
import ctypes as C
import threading

import numpy as np
import pytest

import hdg_inputs as hi

pytestmark = pytest.mark.gpu


def _buffers(plan, torch):
    sz = plan.sizes
    dev = plan.device
    return dict(bsr=torch.empty(max(1, sz["bsr_values"]), dtype=torch.float64, device=dev),
                rhs=torch.empty(max(1, plan.n_skel), dtype=torch.float64, device=dev),
                store=torch.empty(max(1, sz["local_store_bytes"]), dtype=torch.uint8, device=dev),
                ws=torch.empty(max(1, sz["workspace_bytes"]), dtype=torch.uint8, device=dev))


def _step(plan, torch, buf, w, lam, stream, out):
    from paper_1308_3995_amd._lib import check
    vp = lambda t: C.c_void_p(t.data_ptr())
    s = C.c_void_p(stream.cuda_stream)
    lib = plan.lib
    with torch.cuda.stream(stream):
        dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=plan.device)
        dw = torch.zeros_like(w)
    check(lib.hdg_assemble_condense(plan.handle, vp(w), None, vp(lam), vp(buf["bsr"]), vp(buf["rhs"]),
                                    vp(buf["store"]), vp(buf["ws"]), None, None, s))
    it, rr = C.c_int32(0), C.c_double(0.0)
    check(lib.hdg_skeleton_solve(plan.handle, vp(buf["bsr"]), vp(buf["rhs"]), vp(dlam), 1e-10, 30, 100000,
                                 vp(buf["ws"]), s, C.byref(it), C.byref(rr)))
    check(lib.hdg_back_substitute(plan.handle, vp(buf["store"]), vp(dlam), vp(dw), None, vp(buf["ws"]), s))
    stream.synchronize()
    out.append((dlam.cpu().numpy(), dw.cpu().numpy(), it.value))


def test_one_plan_two_streams_bitwise(hdg):
    import torch
    case = hi.config_case("c3", 20)          # hp degrees 1..5, 800 elements
    plan = hdg.HDGPlan.from_case(case, precision="mixed", allocate=False)
    dev = plan.device
    w = torch.tensor(case.W, dtype=torch.float64, device=dev)
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
    bufs = [_buffers(plan, torch), _buffers(plan, torch)]
    streams = [torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)]
    torch.cuda.synchronize()
    seq = [[], []]
    for k in range(2):
        _step(plan, torch, bufs[k], w, lam, streams[k], seq[k])
    assert np.array_equal(seq[0][0][0], seq[1][0][0]) and np.array_equal(seq[0][0][1], seq[1][0][1])
    for rep in range(3):
        con = [[], []]
        th = [threading.Thread(target=_step, args=(plan, torch, bufs[k], w, lam, streams[k], con[k]))
              for k in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for k in range(2):
            assert len(con[k]) == 1, (rep, k)
            assert con[k][0][2] == seq[k][0][2]
            assert np.array_equal(con[k][0][0], seq[k][0][0]), (rep, k)
            assert np.array_equal(con[k][0][1], seq[k][0][1]), (rep, k)
