"""Benchmark of one implicit-HDG Newton step on one MI355X.

Workload: 2-D Euler, uniform p = 3 on a jittered 64 x 64 unit-square mesh split into
8192 triangles (local blocks 40 x 40, 3 faces x 4 nodes x 4 fields), Mach 0.5,
alpha 2 deg free stream plus a seeded perturbation of amplitude 1e-2; synthetic,
seeded inputs resident in HBM before timing starts.

A step is the whole hot path: assemble + condense (hdg_assemble_condense), block-Jacobi
GMRES on the skeleton (hdg_skeleton_solve) to a relative residual of 1e-10, and
back-substitution (hdg_back_substitute). Both precision modes are timed; the reported
`value` is condensed elements per second of full Newton steps of the mixed mode.
Beside the step: assemble + condense alone on three workloads (`condensation`), and with shock
capturing on the transonic hp and the Navier-Stokes workloads (`condensation_shock_capturing`), the
relaxed Newton iteration with the pseudo-time CFL schedule run to convergence
(`pseudo_transient`), the hybridized adjoint at one degree more with the marking decisions
(`adjoint`), a sample of the serving stream (`serving`) and the CPU oracle (`cpu_baseline`).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_worker_init(name: str):
    """Each oracle worker process runs its BLAS on one thread (fail loudly if that cannot be set)
    and builds the workload's oracle state before any timing."""
    from threadpoolctl import threadpool_limits, threadpool_info
    threadpool_limits(limits=1)
    for info in threadpool_info():
        if info.get("num_threads", 1) != 1:
            raise RuntimeError(f"could not limit {info.get('internal_api')} to one thread")
    _oracle_state(name)


_ORACLE_STATE = {}


def _oracle_state(name: str):
    """The oracle's mesh and state of a workload, built once per worker process."""
    if name not in _ORACLE_STATE:
        import hdg_inputs as hi
        from oracle import hdg_oracle as O
        case = hi.config_case(name)
        mesh = O.Mesh(case, O.make_physics(case))
        _ORACLE_STATE[name] = O.State(mesh, case.W, case.lam, case.Q)
    return _ORACLE_STATE[name]


def _oracle_condense(args):
    """Oracle blocks (complex-step) and condensation of a list of elements of a workload; returns
    the seconds spent (the state is built beforehand, outside the timing)."""
    name, elems = args
    from oracle import hdg_oracle as O
    st = _oracle_state(name)
    t0 = time.perf_counter()
    for e in elems:
        O.condense(O.element_blocks(st, int(e)))
    return time.perf_counter() - t0


def cpu_baseline(multi_elements: int = 1024, single_elements: int = 48, lu_ng: int = 16):
    """The CPU oracle, untouched, on the 64x64 p=3 workload (same seeds as the GPU step): the
    per-element path (complex-step Jacobian blocks, LU condensation) over a seeded sample of the
    mesh's elements spread over every core by multiprocessing with BLAS on one thread per
    process, the same on one core, and SuperLU on the skeleton system of the same recipe at
    lu_ng x lu_ng (the 64x64 skeleton needs every element's blocks), timed separately."""
    import multiprocessing as mp
    import hdg_inputs as hi
    from oracle import hdg_oracle as O
    # the host's CPU share: the affinity mask, at most 16 processes (one GPU's share of the box)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(avail, 16))
    case = hi.config_case("c2")
    rng = np.random.default_rng(1308)
    sample = np.sort(rng.choice(case.n_elements, size=min(multi_elements, case.n_elements), replace=False))
    chunks = [("c2", sample[i::cores]) for i in range(cores)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_oracle_worker_init, initargs=("c2",)) as pool:
        # every worker has imported the oracle and built the workload's state (initializer)
        pool.map(_oracle_condense, [("c2", [])] * cores, chunksize=1)
        t0 = time.perf_counter()
        pool.map(_oracle_condense, chunks, chunksize=1)
        t_multi = time.perf_counter() - t0
    with ctx.Pool(1, initializer=_oracle_worker_init, initargs=("c2",)) as pool:
        t_single = pool.map(_oracle_condense, [("c2", sample[:single_elements])])[0]
    rate_multi = len(sample) / t_multi
    rate_single = single_elements / t_single
    # SuperLU on the skeleton system of the same recipe at lu_ng x lu_ng
    small = hi.config_case("c2", ng=lu_ng)
    mesh = O.Mesh(small, O.make_physics(small))
    st = O.State(mesh, small.W, small.lam, small.Q)
    blocks = [O.element_blocks(st, e) for e in range(mesh.ne)]
    cond = [O.condense(b) for b in blocks]
    K, E = O.assemble_skeleton(mesh, blocks, cond)
    import scipy.sparse.linalg as spla
    t0 = time.perf_counter()
    spla.splu(K.tocsc()).solve(E)
    t_lu = time.perf_counter() - t0
    return {"value": rate_multi, "unit": "elements/s", "cores": cores, "kind": "oracle",
            "sample": (f"64x64 p=3 workload, same seeds: oracle assemble + condense (complex-step blocks, LU, "
                       f"Schur) of {len(sample)} seeded elements of the 8192 in {t_multi:.2f} s over {cores} "
                       f"processes with BLAS on one thread each; the skeleton solve is not included (it only "
                       f"adds time); one core: {rate_single:.1f} elements/s ({single_elements} elements); "
                       f"SuperLU on the {lu_ng}x{lu_ng} skeleton ({K.shape[0]} dofs) {t_lu:.3f} s"),
            "single_core_elements_per_s": rate_single, "superlu_seconds": t_lu, "superlu_dofs": int(K.shape[0]),
            "superlu_mesh": f"{lu_ng}x{lu_ng}", "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
            "cpu_affinity": avail}


def measured_traffic(kernel_source: str, summary: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary,
    or None when the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        fields = dict(line.split(None, 1) for line in open(os.path.join(ROOT, summary))
                      if line.strip() and not line.startswith("#"))
        cur = hashlib.sha256(open(os.path.join(ROOT, kernel_source), "rb").read()).hexdigest()
        if fields.get("skeleton_hip_sha256", "").strip() != cur:
            return None
        return float(fields["traffic_per_launch_MB"]) * 1e6
    except (OSError, KeyError, ValueError):
        return None


def condensation_work(case):
    """Algorithmic flops and HBM bytes of assembling and condensing every element once.

    Per element with n = 4 N_p state unknowns and f skeleton unknowns on its interior faces
    (f = sum of 4 (p_e + 1), no padding): LU-equivalent factorisation 2n^3/3, the solves for
    the f + 1 right-hand sides 2n^2 (f + 1), the Schur complement C_K X_K with C_K's actual
    structure (Euler: the field-diagonal trace mass, N_p entries per row; Navier-Stokes: dense
    after the gradient elimination, plus that elimination 2 (n + f)(n + f + 1) 2 N_p and the
    gradient rows of the local solutions 2 (8 N_p)(f + 1) N_p). The quadrature contractions of
    the assembly are not counted. Bytes: state in (W, and Q for Navier-Stokes), lambda in, 100 B
    of geometry, S_K, g_K, X_K, y_K out, all float64.
    """
    import hdg_inputs as hi
    tri, deg = case.tri, case.degree.astype(np.int64)
    ne = tri.shape[0]
    e = np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], axis=0), axis=1)
    _, inv, cnt = np.unique(e, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    owner = np.tile(np.arange(ne), 3)
    pe = np.zeros(cnt.shape[0], dtype=np.int64)
    np.maximum.at(pe, inv, deg[owner])
    interior = cnt[inv] == 2
    f = np.zeros(ne, dtype=np.float64)
    np.add.at(f, owner[interior], 4.0 * (pe[inv][interior] + 1))
    npm = np.array([hi.n_modes(int(p)) for p in deg], dtype=np.float64)
    n = 4.0 * npm
    flops = 2.0 * n ** 3 / 3.0 + 2.0 * n ** 2 * (f + 1.0)
    out_rows = n
    if case.physics == "ns":
        nq = 8.0 * npm
        flops += 2.0 * n * f * (f + 1.0) + 2.0 * (n + f) * (n + f + 1.0) * 2.0 * npm + 2.0 * nq * (f + 1.0) * npm
        bytes_in = (n + nq) * 8.0
        out_rows = n + nq
    else:
        flops += 2.0 * npm * f * (f + 1.0)
        bytes_in = n * 8.0
    nbytes = bytes_in + f * 8.0 + 100.0 + (f * f + f + out_rows * (f + 1.0)) * 8.0
    return float(flops.sum()), float(nbytes.sum())


def measured_copy_peak(reps: int = 5) -> float:
    """HBM bandwidth a plain device copy reaches (1 GiB read + 1 GiB written), best of `reps`:
    the measured peak beside the published 8 TB/s."""
    import torch
    n = (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del x, y
    return 2.0 * n * 8 / (best * 1e-3) / 1e9


def measured_fp64_peak(n: int = 8192, reps: int = 3, dtype: str = "float64") -> float:
    """Rate (TFLOP/s) a plain library GEMM of n x n reaches, best of `reps`: the measured FP64 peak
    beside the published 78.6 TFLOP/s (dtype "float32": the FP32 rate, TF32 off, beside 157.3)."""
    import torch
    dt = getattr(torch, dtype)
    torch.backends.cuda.matmul.allow_tf32 = False
    a = torch.rand(n, n, dtype=dt, device="cuda")
    b = torch.rand(n, n, dtype=dt, device="cuda")
    c = a @ b
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c = a @ b
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b, c
    return 2.0 * n ** 3 / (best * 1e-3) / 1e12


def condensation_report(names, warmup: int = 5, reps: int = 30, sc_eps0: float = 0.0,
                        fp64_measured: float = 0.0, hbm_measured: float = 0.0, precision: str = "fp64"):
    """Assemble + condense time of each named workload (float64 path, or the mixed-precision
    condensation with precision="mixed_condense"), with its roofline:
    `warmup` untimed calls, then the median and p99 of `reps` individually timed calls.
    sc_eps0 > 0 switches shock capturing on (Euler workloads; its extra work is not counted
    in the roofline's algorithmic figures)."""
    import torch
    import hdg_inputs as hi
    import paper_1308_3995_amd as hdg
    out = {}
    for name in names:
        case = hi.config_case(name)
        case.sc_eps0 = sc_eps0
        try:
            plan = hdg.HDGPlan.from_case(case, precision=precision)
        except hdg.HdgError as exc:
            out[name] = {"workload": f"{case.physics} {case.ng}x{case.ng}", "precision": precision,
                         "not_built": str(exc)}
            log(f"[bench] condensation {name} ({precision}): {exc}")
            continue
        dev = plan.device
        w = torch.tensor(case.W, dtype=torch.float64, device=dev)
        q = torch.tensor(case.Q, dtype=torch.float64, device=dev) if case.Q is not None else None
        lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
        for _ in range(warmup):
            plan.hdg_assemble_condense(w, lam, q=q)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.hdg_assemble_condense(w, lam, q=q)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        p99 = float(np.percentile(ts, 99))
        fl, by = condensation_work(case)
        t_f = fl / (FP64_PEAK_TFLOPS * 1e12)
        t_b = by / (HBM_PEAK_GBS * 1e9)
        out[name] = {"workload": f"{case.physics} {case.ng}x{case.ng}, degrees {sorted(set(case.degree.tolist()))}",
                     "precision": precision, "elements": case.n_elements, "ms": ms, "ms_p99": p99, "reps": reps,
                     "elements_per_s": case.n_elements / (ms * 1e-3),
                     "algorithmic_gflop": fl / 1e9, "algorithmic_gb": by / 1e9,
                     "achieved_tflops": fl / (ms * 1e-3) / 1e12, "achieved_gbs": by / (ms * 1e-3) / 1e9,
                     "bound": "fp64" if t_f >= t_b else "hbm", "roofline_frac": max(t_f, t_b) / (ms * 1e-3)}
        if fp64_measured > 0 and hbm_measured > 0:
            # the same fraction against the peaks measured on this GPU (a DGEMM, a device copy)
            out[name]["roofline_frac_of_measured"] = max(fl / (fp64_measured * 1e12),
                                                         by / (hbm_measured * 1e9)) / (ms * 1e-3)
        tag = f" with shock capturing (eps_0 {sc_eps0:g})" if sc_eps0 > 0 else ""
        if sc_eps0 > 0:
            out[name]["shock_capturing_eps0"] = sc_eps0
        log(f"[bench] condensation {name}{tag} ({precision}): {ms:.3f} ms, {case.n_elements / ms / 1e3:.2f} M elements/s, "
            f"roofline {out[name]['roofline_frac']:.3f} ({out[name]['bound']})")
        del plan
        torch.cuda.synchronize()
    return out


def full_step_report(name: str, mode: str, rtol: float, restart: int, cfl: float = 0.0, reps: int = 5,
                     warmup: int = 1, max_iter: int = 200000):
    """One full Newton step (assemble + condense, skeleton solve to rtol, back-substitution) of a
    named workload, `warmup` untimed then the median of `reps` HIP-event-timed steps; cfl > 0
    adds the pseudo-time term of Sec. 3.3 (a relaxed Newton step)."""
    import torch
    import hdg_inputs as hi
    import paper_1308_3995_amd as hdg
    case = hi.config_case(name)
    case.cfl = cfl
    plan = hdg.HDGPlan.from_case(case, precision=mode)
    dev = plan.device
    w = torch.tensor(case.W, dtype=torch.float64, device=dev)
    q = torch.tensor(case.Q, dtype=torch.float64, device=dev) if case.Q is not None else None
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
    dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=dev)
    dw = torch.zeros_like(w)
    dq = torch.zeros_like(q) if q is not None else None
    ts, its, rrs, sts = [], [], [], []
    for r in range(warmup + reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.hdg_assemble_condense(w, lam, q=q)
        it, rr, st = plan.hdg_skeleton_solve(dlam, rtol=rtol, restart=restart, max_iter=max_iter,
                                             raise_on_fail=False)
        plan.hdg_back_substitute(dlam, dw, dq)
        e1.record()
        torch.cuda.synchronize()
        if r >= warmup:
            ts.append(e0.elapsed_time(e1))
            its.append(it)
            rrs.append(rr)
            sts.append(st)
    ms = float(np.median(ts))
    ok = all(st == 0 for st in sts)
    out = {"workload": f"{case.physics} {case.ng}x{case.ng}, degrees {sorted(set(case.degree.tolist()))}"
                       + (f", pseudo-time CFL {cfl:g}" if cfl > 0 else ", pure Newton"),
           "precision": mode, "elements": case.n_elements, "skeleton_dofs": plan.n_skel, "ms": ms,
           "reps": len(ts), "gmres_iters": its[-1], "relres": rrs[-1], "status": sts[-1], "converged": ok}
    if ok:
        out["elements_per_s"] = case.n_elements / (ms * 1e-3)
        out["skeleton_dof_per_s"] = plan.n_skel / (ms * 1e-3)
    log(f"[bench] full step {name} {mode}{' cfl %g' % cfl if cfl > 0 else ''}: {ms:.1f} ms, {its[-1]} GMRES "
        f"iterations, relres {rrs[-1]:.2e}, status {sts[-1]}")
    del plan
    torch.cuda.synchronize()
    return out


def newton_loop_report(name: str, rtol: float, restart: int, max_steps: int = 12):
    """The relaxed Newton iteration (pseudo-time, CFL schedule with the paper's constants) from
    the workload's perturbed state to a residual reduction of 1e-10, mixed-precision skeleton
    solves; host-timed around the library call, which synchronises."""
    import torch
    import hdg_inputs as hi
    import paper_1308_3995_amd as hdg
    case = hi.config_case(name)
    plan = hdg.HDGPlan.from_case(case, precision="mixed")
    dev = torch.device("cuda", 0)
    w = torch.tensor(case.W, dtype=torch.float64, device=dev)
    lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
    q = torch.tensor(case.Q, dtype=torch.float64, device=dev) if case.Q is not None else None
    plan.hdg_assemble_condense(w, lam, q=q)   # kernel-variant tuning happens on a plan's first call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = plan.hdg_pseudo_transient_solve(w, lam, q=q, c0=1e6, c1=1e3, n0=4, max_steps=max_steps, rel_tol=1e-10,
                                        gmres_rtol=rtol, restart=restart)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    log(f"[bench] pseudo-transient {name}: {r['steps']} Newton steps in {sec:.3f} s, converged {r['converged']}, "
        f"residual {r['res0']:.3e} -> {r['res']:.3e}")
    return {"workload": f"{name}: {case.physics} {case.ng}x{case.ng}, degrees {sorted(set(case.degree.tolist()))}, "
                        f"from the perturbed state to ||N_h|| reduced 1e-10; CFL schedule c0=1e6, c1=1e3, n0=4; "
                        f"mixed precision, GMRES({restart}) to {rtol:g} per step",
            "steps": r["steps"], "converged": r["converged"], "seconds": sec,
            "ms_per_newton_step": sec / max(1, r["steps"]) * 1e3, "gmres_iters": r["gmres_iters"],
            "gmres_not_converged": r["gmres_not_converged"],
            "res_history": [float(x) for x in r["res_history"]], "cfl_history": [float(x) for x in r["cfl_history"]]}


def adjoint_report(name: str, rtol: float, restart: int, reps: int = 3):
    """The hybridized adjoint in the space of one degree more, as the paper solves it, for the
    total mass J(w) = integral of rho (F~ has one entry per element: sqrt(2) det J on the
    constant density mode), followed by the marking decisions (theta = 0.05, eps_S = 1e-6) on
    the primal state with the adjoint's indicators. Timed with HIP events around the whole
    sequence, median of `reps` after one warm-up."""
    import torch
    import hdg_inputs as hi
    import paper_1308_3995_amd as hdg
    case = hi.config_case(name)
    p1 = int(case.degree.max()) + 1
    npm = hi.n_modes(p1)
    W = np.zeros((case.n_elements, 4, npm))
    for e in range(case.n_elements):
        n = hi.n_modes(int(case.degree[e]))
        W[e, :, :n] = case.W[e, :, :n]
    plan = hdg.HDGPlan(case.xy, case.tri, (case.degree + 1).astype(np.int8), physics=case.physics,
                       mach=case.mach, aoa_deg=case.aoa_deg, precision="fp64")
    dev = torch.device("cuda", 0)
    fdeg = plan.face_degree
    lam = np.zeros(plan.n_skel)
    for f in range(len(fdeg)):     # the faces' coefficients up to their primal degree, zero above
        o, pf = plan.face_offset[f], int(fdeg[f])
        for a in range(4):
            lam[o + a * (pf + 1): o + a * (pf + 1) + pf] = case.lam[f, a, :pf]
    v = case.xy[case.tri]
    area = 0.5 * np.abs((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1]) -
                        (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1]))
    fw = np.zeros_like(W)
    fw[:, 0, 0] = np.sqrt(2.0) * area / 2.0
    w_d = torch.tensor(W, device=dev)
    lam_d = torch.tensor(lam, device=dev)
    fw_d = torch.tensor(fw, device=dev)
    primal = hdg.HDGPlan.from_case(case, precision="fp64", allocate=False)
    primal.allocate()
    w_p = torch.tensor(case.W, device=dev)
    ts = []
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lamt, wt, eta, it = plan.hdg_adjoint_solve(w_d, lam_d, fw_d, rtol=rtol, restart=restart)
        flag, S, m = primal.hdg_mark_elements(w_p, eta, theta=0.05, eps_s=1e-6)
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    fl = flag.cpu().numpy()
    log(f"[bench] adjoint {name} at p+1: {ms:.1f} ms, {it} GMRES iterations on K^T, {m} elements marked "
        f"({int((fl == 1).sum())} p, {int((fl == 2).sum())} h)")
    return {"workload": f"{name} state in the space of one degree more ({case.n_elements} elements, degrees "
                        f"{sorted(set((case.degree + 1).tolist()))}, {plan.n_skel} skeleton dofs); J = total mass; "
                        f"assemble + condense, K^T, E~, GMRES({restart}) on K^T to {rtol:g}, local adjoint solves "
                        f"and indicators, marking (theta 0.05, eps_S 1e-6)",
            "ms": ms, "gmres_iters": it, "marked": m, "p_enrich": int((fl == 1).sum()),
            "h_refine": int((fl == 2).sum()), "elements_per_s": case.n_elements / (ms * 1e-3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--restart", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--poly-degree", type=int, default=30,
                    help="degree of the GMRES polynomial preconditioner (0: plain block-Jacobi GMRES)")
    ap.add_argument("--poly-fp32", action="store_true",
                    help="mixed mode: the polynomial's products read the float32 matrix, not a float16 copy")
    ap.add_argument("--modes", default="fp64,mixed")
    ap.add_argument("--serving-requests", type=int, default=512,
                    help="requests of the Poisson serving stream to run (0 = skip; 512 = the full stream)")
    ap.add_argument("--serving-slots", type=int, default=16)
    ap.add_argument("--serving-cfl", type=float, default=10.0,
                    help="pseudo-time CFL of every serving request (0: pure Newton steps)")
    ap.add_argument("--serving-newton-requests", type=int, default=128,
                    help="requests of the same stream also served as pure Newton steps (0 = skip)")
    ap.add_argument("--full-steps", default="c2:mixed_condense:0,c3:mixed:0,c3:fp64:0,c3:mixed_condense:0,"
                                            "c4:mixed:100,c4:fp64:100,c4:mixed:0",
                    help="full Newton steps beside the headline: workload:precision:cfl, comma separated")
    ap.add_argument("--serving-max-iter", type=int, default=20000,
                    help="GMRES iterations per serving request before it counts as not converged")
    ap.add_argument("--condense-configs", default="c2,c3,c4",
                    help="workloads whose assemble + condense time is reported beside the step ('' = none)")
    ap.add_argument("--shock-configs", default="c3,c4",
                    help="workloads whose assemble + condense is also timed with shock capturing on ('' = none)")
    ap.add_argument("--newton-loop", default="c2",
                    help="workload of the pseudo-transient Newton iteration report ('' = none)")
    ap.add_argument("--adjoint", default="c2",
                    help="workload of the adjoint + marking report, solved at one degree more ('' = none)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--condense-only", action="store_true",
                    help="only run the condensation reports of --condense-configs, float64 and the mixed-precision "
                         "tier (a short run for kernel counters; prints them as one JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        n = (1 << 30) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}))
        return
    if args.condense_only:
        names = [c for c in args.condense_configs.split(",") if c]
        print(json.dumps({"condensation": condensation_report(names, warmup=1, reps=2),
                          "condensation_mixed": condensation_report(names, warmup=1, reps=2,
                                                                    precision="mixed_condense")}))
        return
    import hdg_inputs as hi
    import paper_1308_3995_amd as hdg

    hdg.load()
    case = hi.config_case("c2")
    dev = torch.device("cuda", 0)
    results = {}
    for mode in args.modes.split(","):
        log(f"[bench] mode {mode}: plan")
        plan = hdg.HDGPlan.from_case(case, precision=mode)
        plan.hdg_set_poly_degree(args.poly_degree, fp16_matrix=not args.poly_fp32)
        w = torch.tensor(case.W, dtype=torch.float64, device=dev).contiguous()
        lam = torch.tensor(plan.pack_lambda(case.lam), dtype=torch.float64, device=dev)
        dlam = torch.zeros(plan.n_skel, dtype=torch.float64, device=dev)
        dw = torch.zeros_like(w)
        stream = torch.cuda.current_stream()

        def step():
            plan.hdg_assemble_condense(w, lam)
            it, rr, _ = plan.hdg_skeleton_solve(dlam, rtol=args.rtol, restart=args.restart)
            plan.hdg_back_substitute(dlam, dw)
            return it, rr

        for i in range(args.warmup):
            it, rr = step()
            log(f"[bench] mode {mode}: warmup {i} gmres iters {it} relres {rr:.2e}")
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        iters = []
        ev[0].record(stream)
        for i in range(args.steps):
            it, rr = step()
            iters.append((it, rr))
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
        ms_step = ev[0].elapsed_time(ev[-1]) / args.steps
        ms_med, ms_p99 = float(np.median(per_step)), float(np.percentile(per_step, 99))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        # the same step once more with every launch of the dominant kernel bracketed by HIP
        # events on its stream (direct launches: events are not recorded inside graph replays)
        plan.hdg_kernel_timing(0, reset=True)
        plan.hdg_kernel_timing(1, reset=True)
        plan.hdg_set_kernel_timing(True)
        step()
        torch.cuda.synchronize()
        plan.hdg_set_kernel_timing(False)
        kt = [plan.hdg_kernel_timing(k, reset=True) for k in (0, 1)]
        kdom = 0 if kt[0][1] >= kt[1][1] else 1
        k_launches, k_ms, k_bytes = kt[kdom]
        log(f"[bench] mode {mode}: {ms_step:.3f} ms/step (median {ms_med:.3f}, p99 {ms_p99:.3f}), "
            f"gmres iters {iters[-1][0]}, relres {iters[-1][1]:.2e}")
        # condensation alone
        reps = max(5, args.steps)
        e0.record(stream)
        for _ in range(reps):
            plan.hdg_assemble_condense(w, lam)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_cond = e0.elapsed_time(e1) / reps
        log(f"[bench] mode {mode}: assemble+condense {ms_cond:.3f} ms")
        results[mode] = dict(ms_step=ms_step, ms_median=ms_med, ms_p99=ms_p99, ms_condense=ms_cond,
                             gmres_iters=iters[-1][0],
                             relres=iters[-1][1], n_skel=plan.n_skel, k_launches=k_launches, k_ms=k_ms,
                             k_bytes=k_bytes, k_dominant=kdom, k_all=kt)
        for k, nm in ((0, "poly SpMV"), (1, "SpMV+dots")):
            nl, tms, tb = kt[k]
            log(f"[bench] mode {mode}: {nm} kernel {nl} launches, {tms:.2f} ms, "
                f"{tms / max(1, nl) * 1e3:.2f} us avg, {tb / max(tms, 1e-12) / 1e6:.0f} GB/s algorithmic")
        del plan
        torch.cuda.synchronize()

    ne = case.n_elements
    main_mode = "mixed" if "mixed" in results else list(results)[0]
    r = results[main_mode]
    out = {
        "metric": "condensed elements/s + skeleton DOF/s, mixed vs FP64 at 1e-10; p50/p99 latency",
        "value": ne / (r["ms_step"] / 1e3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_mode == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": "2-D Euler HDG, uniform p=3, 64x64 jittered unit square (8192 triangles), "
                               "Mach 0.5, alpha 2 deg, perturbation 1e-2; one Newton step, block-Jacobi GMRES(30) "
                               "with a degree-20 GMRES polynomial preconditioner to 1e-10",
                   "elements": ne, "skeleton_dofs": r["n_skel"], "precision": main_mode},
        "modes": {m: {"ms_per_step": v["ms_step"], "ms_per_step_median": v["ms_median"],
                      "ms_per_step_p99": v["ms_p99"], "elements_per_s": ne / (v["ms_step"] / 1e3),
                      "skeleton_dof_per_s": v["n_skel"] / (v["ms_step"] / 1e3),
                      "condense_ms": v["ms_condense"], "condensed_elements_per_s": ne / (v["ms_condense"] / 1e3),
                      "gmres_iters": v["gmres_iters"], "relres": v["relres"]} for m, v in results.items()},
    }
    kl, kms, kb = r["k_launches"], r["k_ms"], r["k_bytes"]
    copy_peak = measured_copy_peak()
    log(f"[bench] device copy reaches {copy_peak:.0f} GB/s (published peak {HBM_PEAK_GBS:.0f})")
    achieved = kb / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    kdom = r["k_dominant"]
    kname = ({"mixed": "k_poly_op<__half>", "fp64": "k_poly_op<double>"}[main_mode] +
             " (float16 / float64 preconditioned skeleton SpMV of one polynomial-preconditioner factor, its vector "
             "work fused)") if kdom == 0 else "k_spmv_dots (preconditioned skeleton SpMV fused with the Gram-Schmidt dots)"
    summary = ("profiles/k_poly_op_c2_euler_p3_mixed_hbm_traffic.txt" if kdom == 0
               else "profiles/k_spmv_dots_c2_euler_p3_mixed_hbm_traffic.txt")
    out["roofline"] = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": (measured_traffic("paper_1308_3995_amd/csrc/skeleton.hip", summary)
                                   if main_mode == "mixed" else None),
                       "traffic_unit": "bytes/launch",
                       "peak_measured_copy": copy_peak, "frac_of_measured": achieved / copy_peak,
                       "launches": kl, "avg_launch_us": kms / max(1, kl) * 1e3,
                       "bytes_per_launch": kb / max(1, kl),
                       "other_kernel": {"name": "k_spmv_dots" if kdom == 0 else "k_poly_op",
                                        "launches": r["k_all"][1 - kdom][0], "ms": r["k_all"][1 - kdom][1],
                                        "bytes": r["k_all"][1 - kdom][2]}}
    if args.condense_configs:
        fp64_meas = measured_fp64_peak()
        log(f"[bench] library DGEMM reaches {fp64_meas:.1f} TFLOP/s (published FP64 peak {FP64_PEAK_TFLOPS})")
        fp32_meas = measured_fp64_peak(dtype="float32")
        log(f"[bench] library SGEMM reaches {fp32_meas:.1f} TFLOP/s (published FP32 peak 157.3)")
        out["measured_peaks"] = {"hbm_copy_gbs": copy_peak, "fp64_dgemm_tflops": fp64_meas,
                                 "fp32_sgemm_tflops": fp32_meas}
        out["condensation"] = condensation_report([c for c in args.condense_configs.split(",") if c],
                                                  fp64_measured=fp64_meas, hbm_measured=copy_peak)
        out["condensation_mixed"] = condensation_report([c for c in args.condense_configs.split(",") if c],
                                                        fp64_measured=fp64_meas, hbm_measured=copy_peak,
                                                        precision="mixed_condense")
        for k, v in out["condensation_mixed"].items():
            if "ms" in v and k in out["condensation"]:
                v["speedup_over_fp64"] = out["condensation"][k]["ms"] / v["ms"]
    if args.shock_configs:
        out["condensation_shock_capturing"] = condensation_report(
            [c for c in args.shock_configs.split(",") if c], sc_eps0=0.2)
    if args.full_steps:
        out["full_steps"] = {}
        for spec in [x for x in args.full_steps.split(",") if x]:
            name, mode, cfl = spec.split(":")
            cfl = float(cfl)
            # a pure Newton step that stalls is reported with its status after a bounded solve
            rep = full_step_report(name, mode, args.rtol, args.restart, cfl=cfl,
                                   reps=1 if cfl == 0 and name == "c4" else 5,
                                   warmup=0 if cfl == 0 and name == "c4" else 1,
                                   max_iter=20000 if cfl == 0 and name == "c4" else 200000)
            out["full_steps"][f"{name}_{mode}_" + (f"cfl{cfl:g}" if cfl > 0 else "newton")] = rep
    if args.newton_loop:
        out["pseudo_transient"] = newton_loop_report(args.newton_loop, args.rtol, args.restart)
    if args.adjoint:
        out["adjoint"] = adjoint_report(args.adjoint, args.rtol, args.restart)
    if args.serving_requests > 0:
        from paper_1308_3995_amd.serving import ServingEngine, stream_requests

        def serve(n, cfl, key):
            log(f"[bench] serving ({key}): generating {n} requests")
            reqs = stream_requests(512, 200.0, rtol=args.rtol, cfl=cfl)[:n]
            eng = ServingEngine(max_slots=args.serving_slots, precision="mixed", restart=args.restart,
                                max_iter=args.serving_max_iter)
            st = eng.run(reqs, on_result=lambda r: log(f"[bench] serving ({key}): request {r.index} done, "
                                                       f"latency {r.latency_s:.3f} s, {r.elements} elements, "
                                                       f"{r.gmres_iters} GMRES iterations, status {r.status}"))
            sm = st.summary()
            step = (f"relaxed Newton steps (pseudo-time CFL {cfl:g}, Sec. 3.3)" if cfl > 0
                    else "pure Newton steps")
            sm["workload"] = (f"first {n} of 512 Poisson requests at 200/s (seed 1313): 2k-64k triangles "
                              f"log-uniform, p in 1..4, Euler or NS, Mach U(0.3,0.9), alpha U(-3,3) deg; {step}; "
                              f"mixed precision, GMRES({args.restart}) to {args.rtol:g} within "
                              f"{args.serving_max_iter} iterations; {args.serving_slots} slots; latencies over "
                              f"every request (failed ones included), completed-only figures beside them")
            log(f"[bench] serving ({key}): p50 {sm['p50_latency_s']:.3f} s, p99 {sm['p99_latency_s']:.3f} s, "
                f"{sm['elements_per_s']:.0f} elements/s, failed {sm['failed_by_status']}")
            return sm

        out["serving"] = serve(args.serving_requests, args.serving_cfl, "relaxed")
        if args.serving_newton_requests > 0:
            out["serving_pure_newton"] = serve(args.serving_newton_requests, 0.0, "pure Newton")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
