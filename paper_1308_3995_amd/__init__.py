"""MI355X (gfx950) hot path of one implicit hybridized-DG Newton step for the 2-D
compressible Euler and Navier-Stokes equations (arXiv:1308.3995).

The numerical work runs in libhdg.so (hand-written HIP); this package marshals
arguments to its C ABI and uses PyTorch only for device memory and streams. The
method names mirror the C entry points of include/hdg.h.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional

import numpy as np

from ._lib import (HDG_EULER, HDG_FP64, HDG_MIXED, HDG_MIXED_CONDENSE, HDG_NS, HdgError, HdgParams,  # noqa: F401
                   HdgSizes, check, load)

__all__ = ["load", "HDGPlan", "HdgError", "HDG_FP64", "HDG_MIXED", "hdg_assemble_condense_batch"]


def _vp(t) -> Optional[C.c_void_p]:
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class HDGPlan:
    """A mesh plan plus the device buffers of one Newton step.

    Buffers (torch tensors on the plan's device): `bsr` (skeleton matrix values, float64),
    `rhs` (E), `store` (local solutions X_K, y_K), `ws` (workspace)."""

    def __init__(self, xy, tri, degree, physics: str = "euler", mach: float = 0.5, aoa_deg: float = 0.0,
                 reynolds: float = 0.0, prandtl: float = 0.72, gamma: float = 1.4, precision: str = "fp64",
                 alpha: float = 0.0, device: int = 0, allocate: bool = True, cfl: float = 0.0,
                 sc_eps0: float = 0.0, sc_beta: float = 0.0):
        import torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        deg = np.ascontiguousarray(degree, dtype=np.int8)
        self.physics = physics
        self.precision = precision
        prec = {"fp64": HDG_FP64, "mixed": HDG_MIXED, "mixed_condense": HDG_MIXED_CONDENSE}[precision]
        prm = HdgParams(HDG_NS if physics == "ns" else HDG_EULER, prec,
                        gamma, mach, math.radians(aoa_deg), reynolds, prandtl, alpha, cfl, sc_eps0, sc_beta)
        h = C.c_void_p()
        check(self.lib.hdg_plan_create(C.byref(h), xy.ctypes.data, xy.shape[0], tri.ctypes.data, tri.shape[0],
                                       deg.ctypes.data, C.byref(prm), device))
        self.handle = h
        sz = HdgSizes()
        check(self.lib.hdg_plan_sizes(h, C.byref(sz)))
        self.sizes = {f: getattr(sz, f) for f, _ in HdgSizes._fields_}
        nf = sz.n_faces
        self.face_vertices = np.zeros((nf, 2), dtype=np.int32)
        self.face_offset = np.zeros(nf + 1, dtype=np.int64)
        self.face_degree = np.zeros(nf, dtype=np.int32)
        check(self.lib.hdg_plan_faces(h, self.face_vertices.ctypes.data, self.face_offset.ctypes.data,
                                      self.face_degree.ctypes.data))
        self.n_skel = int(sz.n_skel_dof)
        self.npmax = int(sz.np_max)
        self.ne = int(sz.n_elements)
        self.bsr = self.rhs = self.store = self.ws = None
        if allocate:
            self.allocate()

    def allocate(self):
        """Device buffers of one Newton step (skeleton matrix, right-hand side, local store, workspace)."""
        import torch
        if self.bsr is not None:
            return
        sz = self.sizes
        f64 = dict(dtype=torch.float64, device=self.device)
        self.bsr = torch.empty(max(1, sz["bsr_values"]), **f64)
        self.rhs = torch.empty(max(1, self.n_skel), **f64)
        self.store = torch.empty(max(1, (sz["local_store_bytes"] + 7) // 8), **f64)
        self.ws = torch.empty(max(1, sz["workspace_bytes"]), dtype=torch.uint8, device=self.device)

    @classmethod
    def from_case(cls, case, precision: str = "fp64", device: int = 0, alpha: float = 0.0,
                  allocate: bool = True) -> "HDGPlan":
        return cls(case.xy, case.tri, case.degree, physics=case.physics, mach=case.mach, aoa_deg=case.aoa_deg,
                   reynolds=case.reynolds, prandtl=case.prandtl, gamma=case.gamma, precision=precision,
                   alpha=alpha, device=device, allocate=allocate, cfl=getattr(case, "cfl", 0.0),
                   sc_eps0=getattr(case, "sc_eps0", 0.0), sc_beta=getattr(case, "sc_beta", 0.0))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.hdg_plan_destroy(h)
            self.handle = None

    # ---- layout helpers (host-side marshalling)
    def pack_lambda(self, lam_padded: np.ndarray) -> np.ndarray:
        """Compact skeleton vector from a (n_faces, 4, >= p_f + 1) array in canonical face order."""
        out = np.empty(self.n_skel)
        for f in range(len(self.face_degree)):
            pe = self.face_degree[f]
            out[self.face_offset[f]: self.face_offset[f + 1]] = lam_padded[f, :, : pe + 1].reshape(-1)
        return out

    def pattern(self):
        nb = self.sizes["bsr_blocks"]
        rp = np.zeros(len(self.face_degree) + 1, dtype=np.int64)
        col = np.zeros(nb, dtype=np.int32)
        voff = np.zeros(nb, dtype=np.int64)
        check(self.lib.hdg_plan_pattern(self.handle, rp.ctypes.data, col.ctypes.data, voff.ctypes.data))
        return rp, col, voff

    # ---- the three calls of the hot path
    def hdg_assemble_condense(self, w, lam, q=None, elem_status=None, want_norm: bool = False, stream=None):
        nrm = C.c_double(0.0)
        check(self.lib.hdg_assemble_condense(self.handle, _vp(w), _vp(q), _vp(lam), _vp(self.bsr), _vp(self.rhs),
                                             _vp(self.store), _vp(self.ws), _vp(elem_status),
                                             C.byref(nrm) if want_norm else None, _stream(stream)))
        return nrm.value if want_norm else None

    def hdg_skeleton_solve(self, dlam, rtol: float = 1e-12, restart: int = 20, max_iter: int = 200000,
                           stream=None, raise_on_fail: bool = True):
        it = C.c_int32(0)
        rr = C.c_double(0.0)
        st = self.lib.hdg_skeleton_solve(self.handle, _vp(self.bsr), _vp(self.rhs), _vp(dlam), rtol, restart,
                                         max_iter, _vp(self.ws), _stream(stream), C.byref(it), C.byref(rr))
        if raise_on_fail:
            check(st)
        return it.value, rr.value, st

    def hdg_back_substitute(self, dlam, dw, dq=None, stream=None):
        check(self.lib.hdg_back_substitute(self.handle, _vp(self.store), _vp(dlam), _vp(dw), _vp(dq), _vp(self.ws),
                                           _stream(stream)))

    # ---- the relaxed Newton iteration (pseudo-time continuation)
    def hdg_set_cfl(self, cfl: float):
        check(self.lib.hdg_set_cfl(self.handle, cfl))

    def hdg_residual_norm(self, stream=None) -> float:
        """||N_h||_2 at the state of the last hdg_assemble_condense (synchronises)."""
        r = C.c_double(0.0)
        check(self.lib.hdg_residual_norm(self.handle, _vp(self.ws), None, C.byref(r), _stream(stream)))
        return r.value

    def hdg_apply_update(self, w, lam, dw, dlam, q=None, dq=None, stream=None):
        check(self.lib.hdg_apply_update(self.handle, _vp(w), _vp(q), _vp(lam), _vp(dw), _vp(dq), _vp(dlam),
                                        _stream(stream)))

    def hdg_cfl_schedule(self, n: int, cfl_prev: float, res_prev: float, res: float, c0: float = 1e6,
                         c1: float = 1e3, n0: int = 4) -> float:
        return self.lib.hdg_cfl_schedule(n, cfl_prev, res_prev, res, c0, c1, n0)

    def hdg_pseudo_transient_solve(self, w, lam, q=None, c0: float = 1e6, c1: float = 1e3, n0: int = 4,
                                   max_steps: int = 20, rel_tol: float = 1e-10, abs_tol: float = 0.0,
                                   gmres_rtol: float = 1e-8, restart: int = 20, max_iter: int = 200000,
                                   stream=None) -> dict:
        """Relaxed Newton iteration of the state (w, lam[, q]) in place; returns the report and
        the residual and CFL histories."""
        import torch
        from ._lib import HdgNewtonOpts, HdgNewtonReport
        dlam = torch.zeros(max(1, self.n_skel), dtype=torch.float64, device=self.device)
        dw = torch.zeros_like(w)
        dq = torch.zeros_like(q) if q is not None else None
        opts = HdgNewtonOpts(c0, c1, n0, max_steps, rel_tol, abs_tol, gmres_rtol, restart, max_iter)
        rep = HdgNewtonReport()
        res = np.zeros(max_steps + 1)
        cfl = np.zeros(max(1, max_steps))
        check(self.lib.hdg_pseudo_transient_solve(self.handle, _vp(w), _vp(q), _vp(lam), _vp(self.bsr),
                                                  _vp(self.rhs), _vp(self.store), _vp(dlam), _vp(dw), _vp(dq),
                                                  _vp(self.ws), C.byref(opts), C.byref(rep), res.ctypes.data,
                                                  cfl.ctypes.data, _stream(stream)))
        n = rep.steps
        return dict(steps=n, converged=bool(rep.converged), gmres_iters=int(rep.gmres_iters),
                    gmres_not_converged=int(rep.gmres_not_converged), res0=rep.res0, res=rep.res,
                    res_history=res[: n + 1].copy(), cfl_history=cfl[:n].copy())

    # ---- hybridized adjoint
    def hdg_skeleton_transpose(self, kt, stream=None):
        """K^T of the last assembly into kt (same pattern and length as the skeleton matrix)."""
        check(self.lib.hdg_skeleton_transpose(self.handle, _vp(self.bsr), _vp(kt), _stream(stream)))

    def hdg_adjoint_rhs(self, fw, etilde, fq=None, stream=None):
        check(self.lib.hdg_adjoint_rhs(self.handle, _vp(self.store), _vp(fw), _vp(fq), _vp(etilde), _vp(self.ws),
                                       _stream(stream)))

    def hdg_adjoint_local(self, w, lam, fw, lamt, wt, eta, q=None, fq=None, qt=None, elem_status=None,
                          stream=None):
        check(self.lib.hdg_adjoint_local(self.handle, _vp(w), _vp(q), _vp(lam), _vp(fw), _vp(fq), _vp(lamt),
                                         _vp(wt), _vp(qt), _vp(eta), _vp(self.ws), _vp(elem_status),
                                         _stream(stream)))

    def hdg_adjoint_solve(self, w, lam, fw, q=None, fq=None, rtol: float = 1e-12, restart: int = 20,
                          max_iter: int = 200000, stream=None):
        """The whole hybridized adjoint at the state (w, lam[, q]) for the functional derivative
        (fw[, fq]): returns (Lambda~, W~, eta, gmres iterations), and Q~ as a fifth entry for
        Navier-Stokes."""
        import torch
        self.hdg_assemble_condense(w, lam, q=q, stream=stream)
        kt = torch.empty_like(self.bsr)
        self.hdg_skeleton_transpose(kt, stream=stream)
        et = torch.empty(max(1, self.n_skel), dtype=torch.float64, device=self.device)
        self.hdg_adjoint_rhs(fw, et, fq=fq, stream=stream)
        lamt = torch.zeros_like(et)
        it = C.c_int32(0)
        rr = C.c_double(0.0)
        check(self.lib.hdg_skeleton_solve(self.handle, _vp(kt), _vp(et), _vp(lamt), rtol, restart, max_iter,
                                          _vp(self.ws), _stream(stream), C.byref(it), C.byref(rr)))
        wt = torch.zeros_like(w)
        qt = torch.zeros_like(q) if q is not None else None
        eta = torch.zeros(self.ne, dtype=torch.float64, device=self.device)
        self.hdg_adjoint_local(w, lam, fw, lamt, wt, eta, q=q, fq=fq, qt=qt, stream=stream)
        if q is not None:
            return lamt, wt, eta, it.value, qt
        return lamt, wt, eta, it.value

    # ---- adaptation decisions
    def hdg_mark_elements(self, w, eta, theta: float = 0.05, eps_s: float = 1e-6, stream=None):
        """Doerfler marking and the smoothness sensor: returns (flag, sensor, n_marked); flag is
        0 (unmarked), 1 (p-enrichment) or 2 (mesh refinement)."""
        import torch
        flag = torch.zeros(max(1, self.ne), dtype=torch.int32, device=self.device)
        sensor = torch.zeros(max(1, self.ne), dtype=torch.float64, device=self.device)
        m = C.c_int32(0)
        check(self.lib.hdg_mark_elements(self.handle, _vp(w), _vp(eta), theta, eps_s, _vp(flag), _vp(sensor),
                                         C.byref(m), _vp(self.ws), _stream(stream)))
        return flag[: self.ne], sensor[: self.ne], m.value

    def hdg_mark_elements_noalloc(self, w, eta, flag, sensor=None, theta: float = 0.05, eps_s: float = 1e-6,
                                  stream=None):
        """hdg_mark_elements on the library's static device scratch (no workspace, nothing
        allocated): fills the caller's flag (and sensor, if given) tensors, returns n_marked."""
        m = C.c_int32(0)
        check(self.lib.hdg_mark_elements_noalloc(self.handle, _vp(w), _vp(eta), theta, eps_s, _vp(flag),
                                                 _vp(sensor), C.byref(m), _stream(stream)))
        return m.value

    # ---- skeleton-solver options and kernel timing (benchmarks)
    def hdg_set_poly_degree(self, degree: int, fp16_matrix: bool = True):
        """Degree of the GMRES polynomial preconditioner (0 or 1: plain block-Jacobi GMRES) and, in
        the mixed mode, whether its products read a float16 copy of the preconditioned matrix."""
        check(self.lib.hdg_set_poly_degree(self.handle, int(degree), 1 if fp16_matrix else 0))

    def hdg_set_kernel_timing(self, enable: bool):
        check(self.lib.hdg_set_kernel_timing(self.handle, 1 if enable else 0))

    def hdg_kernel_timing(self, kernel: int = 0, reset: bool = True):
        """(launches, total ms, algorithmic bytes) of kernel 0 (the polynomial preconditioner's
        SpMV) or 1 (the SpMV fused with the Gram-Schmidt dots)."""
        n, ms, by = C.c_int64(0), C.c_double(0.0), C.c_double(0.0)
        check(self.lib.hdg_kernel_timing(self.handle, int(kernel), C.byref(n), C.byref(ms), C.byref(by),
                                         1 if reset else 0))
        return n.value, ms.value, by.value

    # ---- inspection (tests)
    def debug_element_blocks(self, element: int, w, lam, q=None):
        n = self.sizes["n_fields"] * 21
        f = 72
        bufs = {k: np.zeros(s) for k, s in (("A", n * n), ("B", n * f), ("C", f * n), ("D", f * f), ("r", n),
                                            ("rl", f))}
        no, fo = C.c_int32(0), C.c_int32(0)
        check(self.lib.hdg_debug_element_blocks(self.handle, element, _vp(w), _vp(q), _vp(lam),
                                                *[bufs[k].ctypes.data for k in ("A", "B", "C", "D", "r", "rl")],
                                                C.byref(no), C.byref(fo)))
        n, f = no.value, fo.value
        return dict(A=bufs["A"][: n * n].reshape(n, n).T, B=bufs["B"][: n * f].reshape(f, n).T,
                    C=bufs["C"][: f * n].reshape(n, f).T, D=bufs["D"][: f * f].reshape(f, f).T,
                    r=bufs["r"][:n].copy(), rl=bufs["rl"][:f].copy())

    def debug_local_solution(self, element: int):
        n = self.sizes["n_fields"] * 21
        X = np.zeros(n * 72)
        y = np.zeros(n)
        no, fo = C.c_int32(0), C.c_int32(0)
        check(self.lib.hdg_debug_local_solution(self.handle, _vp(self.store), element, X.ctypes.data, y.ctypes.data,
                                                C.byref(no), C.byref(fo)))
        n, f = no.value, fo.value
        return X[: n * f].reshape(f, n).T, y[:n].copy()

    def debug_condense_variant(self, variant: int):
        """Force condensation kernel variant 0..3 on every float64 Euler bucket (-1: the timed choice)."""
        check(self.lib.hdg_debug_condense_variant(self.handle, int(variant)))

    def skeleton_matrix_dense(self, values=None) -> np.ndarray:
        """Dense copy of the assembled skeleton matrix, or of other values in its block pattern
        (small meshes only)."""
        rp, col, voff = self.pattern()
        vals = (self.bsr if values is None else values).cpu().numpy()
        K = np.zeros((self.n_skel, self.n_skel))
        for f in range(len(self.face_degree)):
            sf = self.face_offset[f + 1] - self.face_offset[f]
            for b in range(rp[f], rp[f + 1]):
                g = col[b]
                sg = self.face_offset[g + 1] - self.face_offset[g]
                blk = vals[voff[b]: voff[b] + sf * sg].reshape(sg, sf).T
                K[self.face_offset[f]: self.face_offset[f + 1], self.face_offset[g]: self.face_offset[g + 1]] = blk
        return K


def hessenberg_eigenvalues(h):
    """Eigenvalues of a real upper Hessenberg matrix by the library's host QR iteration
    (inspection entry for tests; no device work)."""
    lib = load()
    h = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
    n = h.shape[0]
    wr, wi = np.zeros(n), np.zeros(n)
    check(lib.hdg_debug_hessenberg_eigenvalues(n, h.ctypes.data, wr.ctypes.data, wi.ctypes.data))
    return wr + 1j * wi


def hdg_assemble_condense_batch(plans, ws, lams, qs=None, stream=None) -> int:
    """hdg_assemble_condense_batch over several plans (each with its own state w, lam and, for
    Navier-Stokes, q; outputs in each plan's buffers). Returns the number of plans condensed
    together."""
    n = len(plans)
    if not (len(ws) == len(lams) == n) or (qs is not None and len(qs) != n):
        raise ValueError("hdg_assemble_condense_batch: one state per plan")
    arr = C.c_void_p * max(1, n)
    def ptrs(ts):
        return arr(*[None if t is None else t.data_ptr() for t in ts])
    out = C.c_int32(0)
    lib = load()
    check(lib.hdg_assemble_condense_batch(
        n, arr(*[p.handle.value for p in plans]), ptrs(ws),
        ptrs(qs) if qs is not None else None, ptrs(lams), ptrs([p.bsr for p in plans]),
        ptrs([p.rhs for p in plans]), ptrs([p.store for p in plans]), ptrs([p.ws for p in plans]),
        C.byref(out), _stream(stream)))
    return out.value
