"""Continuous-batching request loop for Newton-step solves of independent HDG cases.

Requests arrive on their own clock (seconds after the start of `run`). Preparation threads
build each arrived request's plan (host tables and device constants) off the admission path.
A request is admitted, in arrival order, as soon as its plan is ready, a slot is free and its
device footprint (skeleton matrix, local store, workspace and state, from hdg_plan_sizes)
fits in the HBM budget next to the cases already on the device. Each admitted case keeps its plan, state and
matrices resident and runs one full Newton step (hdg_assemble_condense,
hdg_skeleton_solve, hdg_back_substitute) on its own HIP stream from its own host thread,
so the kernels of concurrent cases overlap on the GPU; the condensations of concurrent Euler
cases are gathered into batched calls (one launch per bucket shape over all of their elements).
When a case finishes, its slot and memory are released and waiting requests are admitted. Latency is completion minus
arrival. All device work is deterministic (fixed-order reductions), so a case's result
does not depend on what else is running.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

# status of a request whose failure was not reported by the library (host-side exception)
STATUS_HOST_FAILURE = -1


@dataclass
class ServeRequest:
    index: int
    arrival_s: float
    case: object                      # hdg_inputs.Case (or anything HDGPlan.from_case accepts)
    rtol: float = 1e-10


@dataclass
class ServeResult:
    index: int
    arrival_s: float
    admitted_s: float
    done_s: float
    elements: int
    skel_dofs: int
    gmres_iters: int
    relres: float
    status: int
    footprint_bytes: int
    dw: Optional[np.ndarray] = None
    dlam: Optional[np.ndarray] = None
    phases: dict = field(default_factory=dict)   # seconds per phase: queue, condense, solve, back_substitute

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


@dataclass
class ServeStats:
    results: List[ServeResult] = field(default_factory=list)
    wall_s: float = 0.0
    max_concurrent: int = 0
    max_bytes_in_use: int = 0
    condense_batches: dict = field(default_factory=dict)   # batched condensation calls and their cases

    def summary(self) -> dict:
        # latency percentiles over every request, failed ones included (a failure is a
        # response too); the completed-only figures are reported beside them
        ok = [r for r in self.results if r.status == 0]
        lat_all = np.array([r.latency_s for r in self.results]) if self.results else np.zeros(1)
        lat_ok = np.array([r.latency_s for r in ok]) if ok else np.zeros(1)
        ne = sum(r.elements for r in ok)
        nd = sum(r.skel_dofs for r in ok)
        failed = {}
        for r in self.results:
            if r.status != 0:
                failed[r.status] = failed.get(r.status, 0) + 1
        phase = {}
        for name in ("queue", "condense", "solve", "back_substitute"):
            v = np.array([r.phases.get(name, 0.0) for r in self.results]) if self.results else np.zeros(1)
            phase[name] = {"p50_s": float(np.percentile(v, 50)), "p99_s": float(np.percentile(v, 99))}
        return {"requests": len(self.results), "completed": len(ok),
                "failed_by_status": {int(k): v for k, v in sorted(failed.items())},
                "p50_latency_s": float(np.percentile(lat_all, 50)), "p99_latency_s": float(np.percentile(lat_all, 99)),
                "p50_latency_completed_s": float(np.percentile(lat_ok, 50)),
                "p99_latency_completed_s": float(np.percentile(lat_ok, 99)),
                "phase_latency": phase,
                "elements_per_s": ne / self.wall_s if self.wall_s > 0 else 0.0,
                "skeleton_dof_per_s": nd / self.wall_s if self.wall_s > 0 else 0.0,
                "wall_s": self.wall_s, "max_concurrent": self.max_concurrent,
                "max_bytes_in_use": self.max_bytes_in_use, "condense_batches": self.condense_batches}


class _CondenseBatcher:
    """Issues the condensation of admitted Euler cases as batched library calls
    (hdg_assemble_condense_batch) on a stream of its own: a case hands over its plan and state
    and waits; the batcher takes every pending case (up to max_items), makes its stream wait for
    their inputs, condenses them with one call (one launch per bucket shape for all of them) and
    records an event that each case's stream then waits for. The outputs are bit-identical to the
    case's own hdg_assemble_condense. If a batched call fails, its cases are condensed one by one so
    that a failure stays with its own case."""

    def __init__(self, device: int, max_items: int = 8):
        import torch
        self.stream = torch.cuda.Stream(device=device)
        self.max_items = max_items
        self.calls = 0          # batched library calls
        self.cases = 0          # cases that went through the batcher
        self.joined = 0         # cases condensed together (the rest one by one within a call)
        self._cv = threading.Condition()
        self._pending = []
        self._stop = False
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()

    def condense(self, plan, w, lam, case_stream):
        import torch
        ready = torch.cuda.Event()
        ready.record(case_stream)
        item = {"plan": plan, "w": w, "lam": lam, "ready": ready, "done": threading.Event(), "event": None,
                "error": None}
        with self._cv:
            self._pending.append(item)
            self._cv.notify()
        item["done"].wait()
        if item["error"] is not None:
            raise item["error"]
        case_stream.wait_event(item["event"])

    def _loop(self):
        import torch
        from . import hdg_assemble_condense_batch
        while True:
            with self._cv:
                while not self._pending and not self._stop:
                    self._cv.wait()
                if not self._pending:
                    return
                batch, self._pending = self._pending[: self.max_items], self._pending[self.max_items:]
            for it in batch:
                self.stream.wait_event(it["ready"])
            try:
                self.joined += hdg_assemble_condense_batch([it["plan"] for it in batch], [it["w"] for it in batch],
                                                           [it["lam"] for it in batch], stream=self.stream)
            except Exception:
                for it in batch:     # isolate the failing case
                    try:
                        it["plan"].hdg_assemble_condense(it["w"], it["lam"], stream=self.stream)
                    except Exception as exc:
                        it["error"] = exc
            ev = torch.cuda.Event()
            ev.record(self.stream)
            self.calls += 1
            self.cases += len(batch)
            for it in batch:
                it["event"] = ev
                it["done"].set()

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        self._thread.join()


class ServingEngine:
    def __init__(self, max_slots: int = 8, hbm_budget_bytes: Optional[int] = None, precision: str = "mixed",
                 restart: int = 20, max_iter: int = 20000, keep_results: bool = False, device: int = 0,
                 prep_threads: int = 2, poly_degree: Optional[int] = None, batch_condense: bool = True):
        import torch
        self.max_slots = max_slots
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(device)
            hbm_budget_bytes = int(free * 0.8)
        self.budget = int(hbm_budget_bytes)
        self.precision = precision
        self.restart = restart
        self.max_iter = max_iter   # GMRES iterations per request before it is reported NOT_CONVERGED
        self.keep = keep_results
        self.device = device
        self.prep_threads = prep_threads   # host threads building plans ahead of admission
        self.poly_degree = poly_degree     # None: the library's default polynomial preconditioner
        self.batch_condense = batch_condense   # Euler condensations of concurrent cases share launches
        self._batcher = None
        self._lock = threading.Lock()
        self._cv = threading.Condition(self._lock)
        self._in_use = 0
        self._active = 0

    @staticmethod
    def footprint(sizes: dict, npmax: int, n_elements: int, ns: bool) -> int:
        state = n_elements * npmax * 8 * (12 if ns else 4) * 2      # state + update
        return int(sizes["bsr_values"] * 8 + sizes["local_store_bytes"] + sizes["workspace_bytes"]
                   + sizes["n_skel_dof"] * 8 * 3 + state)

    def _solve(self, req: ServeRequest, plan, t0: float, admitted: float, fp: int) -> ServeResult:
        import torch
        from . import _lib
        case = req.case
        dev = plan.device
        phases = {"queue": admitted - req.arrival_s}
        status = 0
        it, rr = 0, float("nan")
        dw_h = dl_h = None
        try:
            stream = torch.cuda.Stream(device=self.device)
            plan.allocate()
            with torch.cuda.stream(stream):
                w = torch.tensor(case.W, dtype=torch.float64, device=dev)
                q = torch.tensor(case.Q, dtype=torch.float64, device=dev) if case.Q is not None else None
                lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
                dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=dev)
                dw = torch.zeros_like(w)
                dq = torch.zeros_like(q) if q is not None else None
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                ev[0].record(stream)
                if self._batcher is not None and q is None:
                    self._batcher.condense(plan, w, lam, stream)
                else:
                    plan.hdg_assemble_condense(w, lam, q=q, stream=stream)
                ev[1].record(stream)
                it, rr, status = plan.hdg_skeleton_solve(dlam, rtol=req.rtol, restart=self.restart,
                                                         max_iter=self.max_iter, stream=stream, raise_on_fail=False)
                ev[2].record(stream)
                plan.hdg_back_substitute(dlam, dw, dq, stream=stream)
                ev[3].record(stream)
                stream.synchronize()
                phases = {"queue": admitted - req.arrival_s,
                          "condense": ev[0].elapsed_time(ev[1]) * 1e-3,
                          "solve": ev[1].elapsed_time(ev[2]) * 1e-3,
                          "back_substitute": ev[2].elapsed_time(ev[3]) * 1e-3}
                if self.keep:
                    dw_h = dw.cpu().numpy()
                    dl_h = dlam.cpu().numpy()
        except _lib.HdgError as e:      # a failed request is isolated: its slot is freed
            status = e.status
        except Exception:               # e.g. a device allocation of the request's buffers failed
            status = STATUS_HOST_FAILURE
        done = time.perf_counter() - t0
        return ServeResult(req.index, req.arrival_s, admitted, done, plan.ne, plan.n_skel, it, rr, status, fp,
                           dw_h, dl_h, phases)

    def run(self, requests: List[ServeRequest], on_result: Optional[Callable[[ServeResult], None]] = None
            ) -> ServeStats:
        from . import HDGPlan
        pending = sorted(requests, key=lambda r: r.arrival_s)
        stats = ServeStats()
        t0 = time.perf_counter()
        futures = []

        def finish(res: ServeResult, fp: int, plan):
            with self._cv:
                self._in_use -= fp
                self._active -= 1
                stats.results.append(res)
                self._cv.notify_all()
            del plan
            if on_result:
                on_result(res)

        def prepare(req):
            # host-side plan (mesh tables, buckets, device constants) and its footprint, built on
            # a preparation thread once the request has arrived
            now = time.perf_counter() - t0
            if req.arrival_s > now:
                time.sleep(req.arrival_s - now)
            plan = HDGPlan.from_case(req.case, precision=self.precision, device=self.device, allocate=False)
            if self.poly_degree is not None:
                plan.hdg_set_poly_degree(self.poly_degree)
            return plan, self.footprint(plan.sizes, plan.npmax, plan.ne, plan.physics == "ns")

        self._batcher = _CondenseBatcher(self.device, self.max_slots) if self.batch_condense else None
        with ThreadPoolExecutor(max_workers=self.max_slots) as pool, \
                ThreadPoolExecutor(max_workers=self.prep_threads) as prep:
            prepared = [prep.submit(prepare, r) for r in pending]
            i = 0
            while i < len(pending):
                req = pending[i]
                try:
                    plan, fp = prepared[i].result()
                except Exception as exc:     # the plan could not be built: the request fails alone
                    from . import _lib
                    status = exc.status if isinstance(exc, _lib.HdgError) else STATUS_HOST_FAILURE
                    now = time.perf_counter() - t0
                    res = ServeResult(req.index, req.arrival_s, now, now, 0, 0, 0, float("nan"), status, 0)
                    with self._cv:
                        stats.results.append(res)
                    if on_result:
                        on_result(res)
                    prepared[i] = None
                    i += 1
                    continue
                prepared[i] = None
                with self._cv:
                    while self._active >= self.max_slots or (self._active > 0 and self._in_use + fp > self.budget):
                        self._cv.wait(timeout=0.05)
                    self._in_use += fp
                    self._active += 1
                    stats.max_concurrent = max(stats.max_concurrent, self._active)
                    stats.max_bytes_in_use = max(stats.max_bytes_in_use, self._in_use)
                admitted = time.perf_counter() - t0

                def job(req=req, plan=plan, admitted=admitted, fp=fp):
                    res = None
                    try:
                        res = self._solve(req, plan, t0, admitted, fp)
                    finally:
                        # the slot and its memory are released whatever happened to the request
                        if res is None:
                            res = ServeResult(req.index, req.arrival_s, admitted, time.perf_counter() - t0,
                                              plan.ne, plan.n_skel, 0, float("nan"), STATUS_HOST_FAILURE, fp)
                        finish(res, fp, plan)
                    return res

                futures.append(pool.submit(job))
                i += 1
            for f in futures:
                f.result()
        stats.wall_s = time.perf_counter() - t0
        if self._batcher is not None:
            self._batcher.close()
            stats.condense_batches = {"calls": self._batcher.calls, "cases": self._batcher.cases,
                                      "condensed_together": self._batcher.joined}
            self._batcher = None
        stats.results.sort(key=lambda r: r.index)
        return stats


def stream_requests(n_requests: int, rate_per_s: float, seed: int = 1313, ne_range=(2000, 64000),
                    degrees=(1, 2, 3, 4), rtol: float = 1e-10, cfl: float = 0.0) -> List[ServeRequest]:
    """The serving workload: Poisson arrivals, log-uniform mesh sizes, Euler or NS with
    probability 1/2, p uniform in `degrees`, Mach ~ U(0.3, 0.9), alpha ~ U(-3, 3) deg. cfl > 0
    makes every request a relaxed Newton step (the pseudo-time term of Sec. 3.3 at that CFL)."""
    import hdg_inputs as hi
    out = []
    for r in hi.serving_stream(n_requests, rate_per_s, seed, ne_range, degrees):
        c = r.case()
        c.cfl = cfl
        out.append(ServeRequest(r.index, r.arrival_s, c, rtol))
    return out
