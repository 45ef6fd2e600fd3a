"""Plain, slow, CPU FP64 oracle for one implicit-HDG Newton step.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

What it computes, in the paper's order (Woopen, Balan, May, Schuetz, 2013):
  * Sec. 2: Euler convective flux and equation of state, Navier-Stokes viscous
    flux with constant viscosity, far-field characteristic boundary state;
  * Sec. 3.2, eq. hdg_ls1..hdg_cont: the HDG residual N_h, element by element
    (local solver rows tested by tau and phi, skeleton rows tested by mu), with
    the Lax-Friedrichs-type trace flux f^(lam) . n - alpha (lam - w) and the
    adjoint-consistent boundary term built on w_bnd(w);
  * Sec. 3.3, eq. linearsystem: the Newton Jacobian, obtained here by
    complex-step differentiation of the element-local residual map (independent
    of any hand-derived Jacobian);
  * Sec. 3.2, optional shock capturing: the volume term (grad phi, eps_K grad w_h)
    with the element viscosity eps_K from the L1 norm of the strong residual;
  * Sec. 3.3, optional backward-Euler pseudo-time term: the element mass
    matrix over a local step dt_K (CFL number times |K| over the element's
    convective and viscous wave-speed sums at its mean state) added to the
    conserved-variable block of A_K; CFL = 0 gives the pure Newton step;
  * Sec. 3.3, eq. cfl: the CFL schedule (smooth ramp, then growth by the
    residual reduction) and the relaxed Newton iteration it drives, with the
    residual norm ||N_h||_2 over every element and skeleton row;
  * Sec. 4, eq. adjoint and Sec. 4.1: the adjoint of the Newton matrix, solved
    directly and in hybridized form (K^T Lam~ = E~ and the transposed local
    solves), the element indicators with the skeleton adjoint dropped, the
    enrichment to one degree more, Doerfler marking and the smoothness sensor
    that picks p-enrichment or mesh refinement;
  * Sec. 3.4, eq. ls/cons/hybridsystem: static condensation
    S_K = D_K - C_K A_K^-1 B_K, g_K = r_lam,K - C_K A_K^-1 r_K, summed into the
    skeleton system K dLam = E, solved directly, then the element-wise
    reconstruction dU_K = A_K^-1 (r_K - B_K dLam_K);
  * a monolithic solve of the un-condensed Newton system for cross-checks.

Readings of points the paper leaves open (identical on the GPU side, which is
written separately):
  * basis: orthonormal Dubiner basis on the reference triangle
    {(-1,-1),(1,-1),(-1,1)}, hierarchical order (degree k = 0..p, inside a
    degree by the second collapsed index j ascending); orthonormal Legendre
    basis on faces, parameterised from the lower to the higher global vertex id;
  * quadrature: collapsed Gauss-Legendre with (p_K+2)^2 points on elements,
    p_e+2 Gauss points on interior faces, p_K+2 on boundary faces;
  * momentum flux rho v (x) v + p Id (the printed formula drops rho);
  * alpha a constant scalar per case, default |v_inf| + c_inf;
  * far-field state w_b = P+ w + (I - P+) w_inf with P+ the spectral projector
    of f_c'(w_inf).n onto eigenvalues >= 0 (frozen at the free stream);
  * boundary term of the gradient equation with a minus sign, like the interior
    trace term, so that q = grad w is reproduced; q_bnd = q_h;
  * constant viscosity mu = rho_inf |v_inf| L / Re, heat flux (mu gamma/Pr) grad e.
  * shock capturing (Euler): h_K the element's longest edge, h~ = h_K / p_K;
    the strong residual div f_c(w_h) by the chain rule at the volume points;
    eps_K held fixed in the Newton matrix (evaluated at the current state);
  * pseudo-time step: dt_K = CFL |K| / (lambda_c + 4 lambda_v) with
    lambda_c = sum_e (|v.n| + c)|e| and lambda_v = (mu gamma / (rho Pr))
    sum_e |e|^2 / |K|, both at the integral mean of w_h over K (the paper
    names the step's ingredients but prints no formula for it);
  * unknown order inside an element: Navier-Stokes gradient fields (4d + a)
    first, then the 4 conserved fields; within a field the hierarchical modes.
    Skeleton unknowns per face: field-major, then the Legendre mode.

Parity pins live in tests/test_oracle_*.py.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

CSTEP = 1e-30  # complex-step size


# ---------------------------------------------------------------------------
# Polynomials and quadrature
# ---------------------------------------------------------------------------

def jacobi(n: int, a: float, b: float, x):
    """Jacobi polynomial P_n^{(a,b)}(x) by the three-term recurrence (complex-safe)."""
    x = np.asarray(x)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = 0.5 * (a - b + (a + b + 2.0) * x)
    for k in range(2, n + 1):
        c1 = 2.0 * k * (k + a + b) * (2.0 * k + a + b - 2.0)
        c2 = (2.0 * k + a + b - 1.0) * (a * a - b * b)
        c3 = (2.0 * k + a + b - 2.0) * (2.0 * k + a + b - 1.0) * (2.0 * k + a + b)
        c4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * (2.0 * k + a + b)
        p0, p1 = p1, ((c2 + c3 * x) * p1 - c4 * p0) / c1
    return p1


def n_modes(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def mode_pairs(p: int):
    """Hierarchical (i, j) pairs of the Dubiner basis: degree k = i + j ascending, then j."""
    out = []
    for k in range(p + 1):
        for j in range(k + 1):
            out.append((k - j, j))
    return out


def dubiner(p: int, xi, eta):
    """Orthonormal Dubiner basis on the reference triangle, shape (Np, npts).

    phi_ij = c_ij P_i(a) ((1-b)/2)^i P_j^{(2i+1,0)}(b), with the collapsed
    coordinates a = 2(1+xi)/(1-eta) - 1, b = eta and c_ij chosen so that the
    functions are orthonormal over the triangle of area 2."""
    xi = np.asarray(xi)
    eta = np.asarray(eta)
    a = 2.0 * (1.0 + xi) / (1.0 - eta) - 1.0
    b = eta
    out = []
    for (i, j) in mode_pairs(p):
        c = math.sqrt((2 * i + 1) * (i + j + 1) / 2.0)
        out.append(c * jacobi(i, 0.0, 0.0, a) * ((1.0 - b) / 2.0) ** i * jacobi(j, 2.0 * i + 1.0, 0.0, b))
    return np.array(out)


def dubiner_grad(p: int, xi, eta):
    """Reference gradients (2, Np, npts) by complex-step differentiation of `dubiner`."""
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    gx = dubiner(p, xi + 1j * CSTEP, eta.astype(complex)).imag / CSTEP
    gy = dubiner(p, xi.astype(complex), eta + 1j * CSTEP).imag / CSTEP
    return np.array([gx, gy])


def legendre_face(p: int, s):
    """Orthonormal Legendre basis on [-1, 1], shape (p+1, npts)."""
    s = np.asarray(s)
    return np.array([math.sqrt((2 * k + 1) / 2.0) * jacobi(k, 0.0, 0.0, s) for k in range(p + 1)])


def gauss(n: int):
    return np.polynomial.legendre.leggauss(n)


def triangle_rule(p: int):
    """Collapsed (Duffy) Gauss rule with (p+2)^2 points on the reference triangle."""
    x, w = gauss(p + 2)
    A, Bv = np.meshgrid(x, x, indexing="ij")
    WA, WB = np.meshgrid(w, w, indexing="ij")
    xi = (1.0 + A) * (1.0 - Bv) / 2.0 - 1.0
    eta = Bv
    wt = WA * WB * (1.0 - Bv) / 2.0
    return xi.ravel(), eta.ravel(), wt.ravel()


# ---------------------------------------------------------------------------
# Physics (Sec. 2)
# ---------------------------------------------------------------------------

@dataclass
class Physics:
    kind: str          # "euler" or "ns"
    gamma: float
    winf: np.ndarray
    alpha: float
    mu: float = 0.0
    prandtl: float = 0.72
    cfl: float = 0.0   # pseudo-time CFL number (Sec. 3.3); 0 = pure Newton
    sc_eps0: float = 0.0   # shock-capturing factor epsilon_0 (Sec. 3.2); 0 = off
    sc_beta: float = 0.0   # shock-capturing exponent beta


def make_physics(case, alpha: Optional[float] = None) -> Physics:
    winf = case.free_stream()
    speed = math.hypot(winf[1], winf[2]) / winf[0]
    pinf = (case.gamma - 1.0) * (winf[3] - 0.5 * (winf[1] ** 2 + winf[2] ** 2) / winf[0])
    cinf = math.sqrt(case.gamma * pinf / winf[0])
    if alpha is None:
        alpha = speed + cinf
    mu = 0.0
    if case.physics == "ns":
        mu = winf[0] * speed * 1.0 / case.reynolds
    return Physics(case.physics, case.gamma, winf, alpha, mu, case.prandtl, getattr(case, "cfl", 0.0),
                   getattr(case, "sc_eps0", 0.0), getattr(case, "sc_beta", 0.0))


def euler_flux(w, gamma):
    """Convective flux (2, ..., 4) of w (..., 4); momentum flux rho v (x) v + p Id."""
    rho, mx, my, E = w[..., 0], w[..., 1], w[..., 2], w[..., 3]
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * (mx * u + my * v))
    fx = np.stack([mx, mx * u + p, my * u, u * (E + p)], axis=-1)
    fy = np.stack([my, mx * v, my * v + p, v * (E + p)], axis=-1)
    return np.stack([fx, fy], axis=0)


def viscous_flux(w, q, phys: Physics):
    """Viscous flux (2, ..., 4) of state w (..., 4) and gradient q (..., 2, 4).

    Newtonian stress with constant mu; heat flux k grad T = (mu gamma / Pr) grad e,
    e = E/rho - |v|^2/2 (the ideal-gas temperature relation of Sec. 2.2)."""
    mu, gamma, pr = phys.mu, phys.gamma, phys.prandtl
    rho, mx, my, E = w[..., 0], w[..., 1], w[..., 2], w[..., 3]
    u, v = mx / rho, my / rho
    qx, qy = q[..., 0, :], q[..., 1, :]
    ux = (qx[..., 1] - u * qx[..., 0]) / rho
    uy = (qy[..., 1] - u * qy[..., 0]) / rho
    vx = (qx[..., 2] - v * qx[..., 0]) / rho
    vy = (qy[..., 2] - v * qy[..., 0]) / rho
    Er = E / rho
    ex = (qx[..., 3] - Er * qx[..., 0]) / rho - (u * ux + v * vx)
    ey = (qy[..., 3] - Er * qy[..., 0]) / rho - (u * uy + v * vy)
    div = ux + vy
    txx = mu * (2.0 * ux - 2.0 / 3.0 * div)
    tyy = mu * (2.0 * vy - 2.0 / 3.0 * div)
    txy = mu * (uy + vx)
    kap = mu * gamma / pr
    z = np.zeros_like(rho)
    fx = np.stack([z, txx, txy, u * txx + v * txy + kap * ex], axis=-1)
    fy = np.stack([z, txy, tyy, u * txy + v * tyy + kap * ey], axis=-1)
    return np.stack([fx, fy], axis=0)


def normal_flux_jacobian(w, n, gamma):
    """d(f_c(w) . n)/dw (4x4) by complex step."""
    J = np.zeros((4, 4))
    for b in range(4):
        wc = np.asarray(w, dtype=complex).copy()
        wc[b] += 1j * CSTEP
        f = euler_flux(wc, gamma)
        J[:, b] = (f[0] * n[0] + f[1] * n[1]).imag / CSTEP
    return J


def farfield_projector(winf, n, gamma):
    """Spectral projector of f_c'(w_inf).n onto its eigenvalues >= 0.

    The eigenvalues are u_n - c, u_n (twice) and u_n + c; the projector onto
    each eigenspace is the Frobenius covariant prod_{k != j} (A - mu_k)/(mu_j - mu_k)."""
    A = normal_flux_jacobian(winf, n, gamma)
    rho = winf[0]
    un = (winf[1] * n[0] + winf[2] * n[1]) / rho
    p = (gamma - 1.0) * (winf[3] - 0.5 * (winf[1] ** 2 + winf[2] ** 2) / rho)
    c = math.sqrt(gamma * p / rho)
    mus = []
    for m in (un - c, un, un + c):
        if all(abs(m - o) > 1e-12 for o in mus):
            mus.append(m)
    P = np.zeros((4, 4))
    for j, mj in enumerate(mus):
        if mj < 0.0:
            continue
        Pj = np.eye(4)
        for k, mk in enumerate(mus):
            if k != j:
                Pj = Pj @ (A - mk * np.eye(4)) / (mj - mk)
        P += Pj
    return P


# ---------------------------------------------------------------------------
# Mesh bookkeeping (Sec. 3.1)
# ---------------------------------------------------------------------------

@dataclass
class FaceSide:
    lf: int                 # local face id (v_lf, v_lf+1)
    face: int               # interior face id in canonical order, or -1 on the boundary
    normal: np.ndarray      # outward unit normal of the element
    length: float
    s: np.ndarray           # Gauss points on [-1,1], global orientation
    wq: np.ndarray          # weights times |e|/2
    phi: np.ndarray         # element basis at the face points, (Np, Qe)
    psi: Optional[np.ndarray]   # face basis (pe+1, Qe) for interior faces
    pe: int
    Pplus: Optional[np.ndarray]  # far-field projector on boundary faces


@dataclass
class ElementGeom:
    p: int
    detJ: float
    wq: np.ndarray          # volume weights times det J
    phi: np.ndarray         # (Np, Q)
    dphi: np.ndarray        # physical gradients (2, Np, Q)
    sides: List[FaceSide]
    xq: np.ndarray          # physical volume points (Q, 2)


class Mesh:
    """Faces, face degrees (p_e = max of the neighbours, Sec. 3.1), skeleton offsets and
    per-element geometry and basis tables."""

    def __init__(self, case, phys: Physics):
        self.case = case
        self.phys = phys
        xy, tri, deg = case.xy, case.tri, case.degree.astype(int)
        self.ne = tri.shape[0]
        edges: Dict[tuple, list] = {}
        for e in range(self.ne):
            for lf in range(3):
                a, b = int(tri[e, lf]), int(tri[e, (lf + 1) % 3])
                edges.setdefault((min(a, b), max(a, b)), []).append((e, lf))
        interior = sorted(k for k, v in edges.items() if len(v) == 2)
        self.face_vertices = np.array(interior, dtype=np.int32).reshape(-1, 2)
        self.nf = len(interior)
        self.face_index = {k: i for i, k in enumerate(interior)}
        self.face_elems = [edges[k] for k in interior]
        self.face_degree = np.array([max(deg[e] for (e, _) in edges[k]) for k in interior], dtype=int)
        sizes = 4 * (self.face_degree + 1)
        self.face_offset = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n_skel = int(self.face_offset[-1])
        self.elem_faces = np.full((self.ne, 3), -1, dtype=int)
        for e in range(self.ne):
            for lf in range(3):
                a, b = int(tri[e, lf]), int(tri[e, (lf + 1) % 3])
                self.elem_faces[e, lf] = self.face_index.get((min(a, b), max(a, b)), -1)
        self.m_loc = 12 if phys.kind == "ns" else 4
        self.elem_ndof = np.array([self.m_loc * n_modes(deg[e]) for e in range(self.ne)])
        self.elem_offset = np.concatenate([[0], np.cumsum(self.elem_ndof)]).astype(np.int64)
        self._geom: Dict[int, ElementGeom] = {}

    def geom(self, e: int) -> ElementGeom:
        if e in self._geom:
            return self._geom[e]
        xy, tri = self.case.xy, self.case.tri
        p = int(self.case.degree[e])
        v = xy[tri[e]]
        M = np.column_stack([v[1] - v[0], v[2] - v[0]])        # x = v0 + M [(1+xi)/2, (1+eta)/2]
        J = M / 2.0
        detJ = float(np.linalg.det(J))
        Jinv = np.linalg.inv(J)
        xi, eta, wt = triangle_rule(p)
        phi = dubiner(p, xi, eta)
        gref = dubiner_grad(p, xi, eta)
        dphi = np.einsum("rd,rnq->dnq", Jinv, gref)            # grad_x = J^-T grad_xi
        xq = (v[0][None, :] + (M @ np.stack([(1 + xi) / 2, (1 + eta) / 2])).T)
        sides = []
        Minv = np.linalg.inv(M)
        for lf in range(3):
            ia, ib = int(tri[e, lf]), int(tri[e, (lf + 1) % 3])
            t = xy[ib] - xy[ia]
            length = float(np.hypot(t[0], t[1]))
            normal = np.array([t[1], -t[0]]) / length
            fid = self.elem_faces[e, lf]
            if fid >= 0:
                pe = int(self.face_degree[fid])
                nq = pe + 2
            else:
                pe = p
                nq = p + 2
            s, ws = gauss(nq)
            A, Bv = (ia, ib) if ia < ib else (ib, ia)
            pts = xy[A][None, :] * ((1 - s) / 2)[:, None] + xy[Bv][None, :] * ((1 + s) / 2)[:, None]
            ref = (Minv @ (pts - v[0][None, :]).T) * 2.0 - 1.0    # reference coordinates
            fphi = dubiner(p, ref[0], ref[1])
            psi = legendre_face(pe, s) if fid >= 0 else None
            Pp = None if fid >= 0 else farfield_projector(self.phys.winf, normal, self.phys.gamma)
            sides.append(FaceSide(lf, fid, normal, length, s, ws * length / 2.0, fphi, psi, pe, Pp))
        g = ElementGeom(p, detJ, wt * detJ, phi, dphi, sides, xq)
        self._geom[e] = g
        return g

    def elem_lambda_size(self, e: int) -> int:
        return sum(4 * (self.face_degree[f] + 1) for f in self.elem_faces[e] if f >= 0)


# ---------------------------------------------------------------------------
# Element-local residual (eq. hdg_ls1 .. hdg_cont), batched and complex-safe
# ---------------------------------------------------------------------------

def shock_viscosity(mesh: Mesh, e: int, W: np.ndarray, Q: Optional[np.ndarray] = None) -> float:
    """Artificial viscosity of Sec. 3.2 (shock capturing): eps_K = eps_0 h~^(2 - beta) / |K|
    int_K d(w), with d(w) = sum over the components of |div f_c(w)| (the strong convective
    residual, by the chain rule from the flux Jacobians and the gradient of w_h) and
    h~ = h_K / p_K, h_K the element's longest edge. W: (4, Np) real coefficients. With Q
    ((8, Np) real coefficients of q_h, row 4 d + a = d w_a / d x_d; Navier-Stokes) the gradient
    in the strong residual is q_h, the viscous form of Sec. 3.2."""
    phys = mesh.phys
    if phys.sc_eps0 <= 0.0:
        return 0.0
    g = mesh.geom(e)
    wq = W @ g.phi                                   # (4, Q)
    if Q is None:
        gw = np.einsum("an,dnq->dqa", W, g.dphi)     # (2, Q, 4) physical gradient
    else:
        gw = (Q @ g.phi).T.reshape(-1, 2, 4).transpose(1, 0, 2)   # (2, Q, 4): q_h at the points
    d = np.zeros(wq.shape[1])
    for q in range(wq.shape[1]):
        div = (normal_flux_jacobian(wq[:, q], (1.0, 0.0), phys.gamma) @ gw[0, q]
               + normal_flux_jacobian(wq[:, q], (0.0, 1.0), phys.gamma) @ gw[1, q])
        d[q] = np.sum(np.abs(div))
    area = float(np.sum(g.wq))
    h = max(sd.length for sd in g.sides)
    ht = h / int(mesh.case.degree[e])
    return phys.sc_eps0 * ht ** (2.0 - phys.sc_beta) / area * float(g.wq @ d)


def element_residual(mesh: Mesh, e: int, W, Q, lam_faces):
    """Residual of element e.

    W (B, 4, Np), Q (B, 8, Np) or None, lam_faces: list over the element's local faces of
    (B, 4, pe+1) arrays (None on boundary faces). Returns (Rq or None, Rw, Rlam list)
    with Rlam[lf] = element e's share of the skeleton row of that face."""
    phys = mesh.phys
    g = mesh.geom(e)
    ns = phys.kind == "ns"
    Bn = W.shape[0]
    wq = np.einsum("ban,nq->bqa", W, g.phi)                           # (B, Q, 4)
    if ns:
        qq = np.einsum("ban,nq->bqa", Q, g.phi).reshape(Bn, -1, 2, 4)  # (B, Q, 2, 4)
    F = euler_flux(wq, phys.gamma)                                   # (2, B, Q, 4)
    if ns:
        F = F - viscous_flux(wq, qq, phys)
    # volume term: -(grad phi_i, F)
    Rw = -np.einsum("q,dnq,dbqa->ban", g.wq, g.dphi, F)
    if phys.sc_eps0 > 0.0:
        # shock capturing, volume term only: (grad phi_i, eps grad w_h); Navier-Stokes takes the
        # viscous form (grad phi_i, eps q_h) with eps from q_h as well. eps is evaluated at the
        # real part of the state: the Newton matrix holds it fixed (the paper leaves the
        # linearisation of the non-smooth |.| open)
        if ns:
            eps = shock_viscosity(mesh, e, np.asarray(W[0]).real, np.asarray(Q[0]).real)
            Rw = Rw + eps * np.einsum("q,dnq,bqda->ban", g.wq, g.dphi, qq)
        else:
            eps = shock_viscosity(mesh, e, np.asarray(W[0]).real)
            gw = np.einsum("ban,dnq->bdqa", W, g.dphi)
            Rw = Rw + eps * np.einsum("q,dnq,bdqa->ban", g.wq, g.dphi, gw)
    Rq = None
    if ns:
        # (tau, q) + (div tau, w)
        Rq = np.einsum("q,nq,bqk->bkn", g.wq, g.phi, qq.reshape(Bn, -1, 8))
        Rq = Rq + np.einsum("q,dnq,bqa->bdan", g.wq, g.dphi, wq).reshape(Bn, 8, -1)
    Rlam = []
    for side in g.sides:
        n = side.normal
        wt = np.einsum("ban,ng->bga", W, side.phi)                     # trace of w
        if ns:
            qt = np.einsum("bkn,ng->bgk", Q, side.phi).reshape(Bn, -1, 2, 4)
        if side.face >= 0:
            lam = np.einsum("bak,kg->bga", lam_faces[side.lf], side.psi)
            Fl = euler_flux(lam, phys.gamma)
            if ns:
                Fl = Fl - viscous_flux(lam, qt, phys)
            fhat = Fl[0] * n[0] + Fl[1] * n[1] - phys.alpha * (lam - wt)
            Rw = Rw + np.einsum("g,ng,bga->ban", side.wq, side.phi, fhat)
            Rlam.append(np.einsum("g,kg,bga->bak", side.wq, side.psi, fhat))
            trace_state = lam
        else:
            # far-field state: interior characteristics from w, incoming ones from w_inf
            wb = np.einsum("ac,bgc->bga", side.Pplus, wt) + ((np.eye(4) - side.Pplus) @ phys.winf)[None, None, :]
            Fb = euler_flux(wb, phys.gamma)
            if ns:
                Fb = Fb - viscous_flux(wb, qt, phys)
            fb = Fb[0] * n[0] + Fb[1] * n[1]
            Rw = Rw + np.einsum("g,ng,bga->ban", side.wq, side.phi, fb)
            Rlam.append(None)
            trace_state = wb
        if ns:
            # -<tau . n, lam> on interior faces, -<tau . n, w_b> on boundary faces
            Rq = Rq - np.einsum("g,ng,d,bga->bdan", side.wq, side.phi, n, trace_state).reshape(Bn, 8, -1)
    return Rq, Rw, Rlam


# ---------------------------------------------------------------------------
# Newton blocks by complex step, condensation, skeleton system (Sec. 3.3-3.4)
# ---------------------------------------------------------------------------

@dataclass
class ElementBlocks:
    A: np.ndarray   # n x n   local-local
    B: np.ndarray   # n x f   local-face
    C: np.ndarray   # f x n   face-local (element's share of the skeleton rows)
    D: np.ndarray   # f x f   face-face (element's share)
    r: np.ndarray   # n       -R_local
    rl: np.ndarray  # f       -R_lambda share
    faces: list     # interior face ids in local-face order
    fsizes: list


class State:
    """Views of the global state in the oracle's own layout."""

    def __init__(self, mesh: Mesh, W: np.ndarray, lam: np.ndarray, Q: Optional[np.ndarray] = None):
        self.mesh = mesh
        self.W = W
        self.Q = Q
        self.lam = lam   # (Nf, 4, >= pe+1) padded

    def elem_inputs(self, e):
        m = self.mesh
        npe = n_modes(int(m.case.degree[e]))
        W = self.W[e, :, :npe]
        Q = self.Q[e, :, :npe] if self.Q is not None else None
        lams = []
        for lf in range(3):
            f = m.elem_faces[e, lf]
            lams.append(None if f < 0 else self.lam[f, :, : m.face_degree[f] + 1])
        return W, Q, lams


def pack_local(W, Q):
    """Element unknown vector: [Q fields (4d+a) major, W fields] each mode-minor."""
    if Q is None:
        return W.reshape(-1)
    return np.concatenate([Q.reshape(-1), W.reshape(-1)])


def local_time_step(mesh: Mesh, W: np.ndarray, e: int) -> float:
    """Local pseudo-time step of Sec. 3.3: dt_K = CFL |K| / (lambda_c + 4 lambda_v), with
    lambda_c = sum over the element's edges of (|v.n| + c)|e| and lambda_v =
    (mu gamma / (rho Pr)) sum |e|^2 / |K| (Navier-Stokes only), both at the element-mean state
    (the integral mean of w_h over K). W: (4, Np) coefficients of the element."""
    phys = mesh.phys
    g = mesh.geom(e)
    area = float(np.sum(g.wq))
    wbar = (W @ g.phi) @ g.wq / area
    rho, u, v = wbar[0], wbar[1] / wbar[0], wbar[2] / wbar[0]
    p = (phys.gamma - 1.0) * (wbar[3] - 0.5 * rho * (u * u + v * v))
    c = math.sqrt(phys.gamma * p / rho)
    lam_c = sum((abs(u * sd.normal[0] + v * sd.normal[1]) + c) * sd.length for sd in g.sides)
    lam_v = 0.0
    if phys.kind == "ns":
        lam_v = phys.mu * phys.gamma / (rho * phys.prandtl) * sum(sd.length ** 2 for sd in g.sides) / area
    return phys.cfl * area / (lam_c + 4.0 * lam_v)


def pseudo_time_block(mesh: Mesh, W: np.ndarray, e: int) -> np.ndarray:
    """The term (phi_i, dw/dt_K) of the backward-Euler pseudo-time step (Sec. 3.3): the element
    mass matrix, by quadrature, over dt_K, for each of the 4 conserved fields (4 Np square)."""
    g = mesh.geom(e)
    mass = (g.phi * g.wq[None, :]) @ g.phi.T
    return np.kron(np.eye(4), mass) / local_time_step(mesh, W, e)


def element_blocks(state: State, e: int) -> ElementBlocks:
    m = state.mesh
    ns = m.phys.kind == "ns"
    W, Q, lams = state.elem_inputs(e)
    npe = W.shape[1]
    u0 = pack_local(W, Q)
    n = u0.size
    faces = [(lf, m.elem_faces[e, lf]) for lf in range(3) if m.elem_faces[e, lf] >= 0]
    fsizes = [lams[lf].size for lf, _ in faces]
    f = int(sum(fsizes))
    z0 = np.concatenate([u0] + [lams[lf].reshape(-1) for lf, _ in faces])
    nb = n + f + 1
    Z = np.tile(z0.astype(complex), (nb, 1))
    Z[np.arange(n + f), np.arange(n + f)] += 1j * CSTEP
    # unpack the batch
    if ns:
        Qb = Z[:, : 8 * npe].reshape(nb, 8, npe)
        Wb = Z[:, 8 * npe: 12 * npe].reshape(nb, 4, npe)
    else:
        Qb = None
        Wb = Z[:, :n].reshape(nb, 4, npe)
    lb = [None, None, None]
    off = n
    for (lf, fid), sz in zip(faces, fsizes):
        lb[lf] = Z[:, off: off + sz].reshape(nb, 4, sz // 4)
        off += sz
    Rq, Rw, Rl = element_residual(m, e, Wb, Qb, lb)
    Rloc = Rw.reshape(nb, -1) if not ns else np.concatenate([Rq.reshape(nb, -1), Rw.reshape(nb, -1)], axis=1)
    Rlam = np.concatenate([Rl[lf].reshape(nb, -1) for lf, _ in faces], axis=1) if faces else np.zeros((nb, 0))
    Jloc = (Rloc[: n + f].imag / CSTEP).T      # (n, n+f)
    Jlam = (Rlam[: n + f].imag / CSTEP).T      # (f, n+f)
    A = Jloc[:, :n].copy()
    if m.phys.cfl > 0.0:
        # pseudo-time: left-hand side only, on the conserved-variable rows and columns
        w0 = 8 * npe if ns else 0
        A[w0:, w0:] += pseudo_time_block(m, W, e)
    return ElementBlocks(A=A, B=Jloc[:, n:], C=Jlam[:, :n], D=Jlam[:, n:],
                         r=-Rloc[-1].real, rl=-Rlam[-1].real,
                         faces=[fid for _, fid in faces], fsizes=fsizes)


@dataclass
class Condensed:
    X: np.ndarray
    y: np.ndarray
    S: np.ndarray
    g: np.ndarray


def condense(b: ElementBlocks) -> Condensed:
    """LU with partial pivoting of A_K, local solves and the element Schur complement."""
    lu = scipy.linalg.lu_factor(b.A)
    X = scipy.linalg.lu_solve(lu, b.B) if b.B.size else np.zeros((b.A.shape[0], 0))
    y = scipy.linalg.lu_solve(lu, b.r)
    return Condensed(X=X, y=y, S=b.D - b.C @ X, g=b.rl - b.C @ y)


def elem_dofs(mesh: Mesh, b: ElementBlocks) -> np.ndarray:
    return np.concatenate([np.arange(mesh.face_offset[f], mesh.face_offset[f + 1]) for f in b.faces]) \
        if b.faces else np.zeros(0, dtype=np.int64)


def assemble_skeleton(mesh: Mesh, blocks: List[ElementBlocks], cond: List[Condensed]):
    """Sum the element Schur complements into the skeleton matrix K and right-hand side E."""
    rows, cols, vals = [], [], []
    E = np.zeros(mesh.n_skel)
    for b, c in zip(blocks, cond):
        d = elem_dofs(mesh, b)
        if d.size == 0:
            continue
        rr, cc = np.meshgrid(d, d, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(c.S.ravel())
        np.add.at(E, d, c.g)
    K = scipy.sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(mesh.n_skel, mesh.n_skel)).tocsr()
    K.sum_duplicates()
    return K, E


def solve_skeleton(K, E):
    if K.shape[0] <= 20000:
        return np.linalg.solve(K.toarray(), E)
    return scipy.sparse.linalg.splu(K.tocsc()).solve(E)


def back_substitute(mesh: Mesh, b: ElementBlocks, c: Condensed, dlam: np.ndarray) -> np.ndarray:
    d = elem_dofs(mesh, b)
    return c.y - c.X @ dlam[d] if d.size else c.y.copy()


def pack_skeleton(mesh: Mesh, lam: np.ndarray) -> np.ndarray:
    """Compact skeleton vector from a padded (Nf, 4, P+1) array."""
    return np.concatenate([lam[f, :, : mesh.face_degree[f] + 1].reshape(-1) for f in range(mesh.nf)])


def unpack_local(mesh: Mesh, e: int, u: np.ndarray, npm: int):
    """Split an element vector into padded (W (4, npm), Q (8, npm) or None)."""
    npe = n_modes(int(mesh.case.degree[e]))
    W = np.zeros((4, npm))
    if mesh.phys.kind == "ns":
        Q = np.zeros((8, npm))
        Q[:, :npe] = u[: 8 * npe].reshape(8, npe)
        W[:, :npe] = u[8 * npe:].reshape(4, npe)
        return W, Q
    W[:, :npe] = u.reshape(4, npe)
    return W, None


@dataclass
class NewtonStep:
    mesh: Mesh
    blocks: List[ElementBlocks]
    cond: List[Condensed]
    K: object
    E: np.ndarray
    dlam: np.ndarray
    du: List[np.ndarray]


def newton_step(case, alpha: Optional[float] = None, elements=None) -> NewtonStep:
    """One full Newton step: blocks, condensation, skeleton solve, reconstruction."""
    phys = make_physics(case, alpha)
    mesh = Mesh(case, phys)
    st = State(mesh, case.W, case.lam, case.Q)
    blocks = [element_blocks(st, e) for e in range(mesh.ne)]
    cond = [condense(b) for b in blocks]
    K, E = assemble_skeleton(mesh, blocks, cond)
    dlam = solve_skeleton(K, E)
    du = [back_substitute(mesh, b, c, dlam) for b, c in zip(blocks, cond)]
    return NewtonStep(mesh, blocks, cond, K, E, dlam, du)


def global_jacobian(step: NewtonStep):
    """The un-condensed Newton matrix [[A, B], [C, D]] over all element unknowns (first) and
    skeleton unknowns, and its right-hand side [r; r_lam]."""
    mesh = step.mesh
    nloc = int(mesh.elem_offset[-1])
    N = nloc + mesh.n_skel
    rows, cols, vals = [], [], []
    rhs = np.zeros(N)
    for e, b in enumerate(step.blocks):
        lo = np.arange(mesh.elem_offset[e], mesh.elem_offset[e + 1])
        sk = nloc + elem_dofs(mesh, b)
        for (R, C_, M) in ((lo, lo, b.A), (lo, sk, b.B), (sk, lo, b.C), (sk, sk, b.D)):
            if M.size == 0:
                continue
            rr, cc = np.meshgrid(R, C_, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(M.ravel())
        rhs[lo] += b.r
        np.add.at(rhs, sk, b.rl)
    J = scipy.sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(N, N)).tocsc()
    return J, rhs, nloc


def monolithic_solve(step: NewtonStep):
    """Solve the un-condensed Newton system [[A, B], [C, D]] [dU; dLam] = [r; r_lam] directly."""
    mesh = step.mesh
    J, rhs, nloc = global_jacobian(step)
    x = scipy.sparse.linalg.spsolve(J, rhs)
    du = [x[mesh.elem_offset[e]: mesh.elem_offset[e + 1]] for e in range(mesh.ne)]
    return du, x[nloc:]


# ---------------------------------------------------------------------------
# Adjoint (Sec. 4): eq. adjoint in matrix form and its hybridized form (Sec. 4.1)
# ---------------------------------------------------------------------------

def adjoint_monolithic(step: NewtonStep, F: List[np.ndarray]):
    """The transposed Newton matrix [[A, B], [C, D]]^T [U~; Lam~] = [F~; 0], solved directly:
    the functional depends on the element unknowns only, so its skeleton part is zero.
    F: per element, the functional derivative in the element's unknown order."""
    mesh = step.mesh
    J, _, nloc = global_jacobian(step)
    rhs = np.zeros(J.shape[0])
    rhs[:nloc] = np.concatenate(F)
    z = scipy.sparse.linalg.spsolve(J.T.tocsc(), rhs)
    Ut = [z[mesh.elem_offset[e]: mesh.elem_offset[e + 1]] for e in range(mesh.ne)]
    return Ut, z[nloc:]


def adjoint_hybridized(step: NewtonStep, F: List[np.ndarray]):
    """Static condensation of the adjoint system: K^T Lam~ = E~ with
    E~ = -sum_K B_K^T A_K^-T F~_K = -sum_K X_K^T F~_K (X_K = A_K^-1 B_K), then the local
    adjoint solves U~_K = A_K^-T (F~_K - C_K^T Lam~_K)."""
    mesh = step.mesh
    Et = np.zeros(mesh.n_skel)
    for e, (b, c) in enumerate(zip(step.blocks, step.cond)):
        d = elem_dofs(mesh, b)
        if d.size:
            np.add.at(Et, d, -(c.X.T @ F[e]))
    lamt = solve_skeleton(step.K.T.tocsr(), Et)
    Ut = []
    for e, b in enumerate(step.blocks):
        d = elem_dofs(mesh, b)
        rhs = F[e] - (b.C.T @ lamt[d] if d.size else 0.0)
        Ut.append(scipy.linalg.solve(b.A.T, rhs))
    return Ut, lamt, Et


def element_indicators(step: NewtonStep, Ut: List[np.ndarray]) -> np.ndarray:
    """eta_K = |N_h(x_h; q~, w~, 0) restricted to K| (Sec. 4): the element's residual rows
    R_K = -r_K weighted by its adjoint, the skeleton adjoint dropped."""
    return np.array([abs(float(Ut[e] @ (-b.r))) for e, b in enumerate(step.blocks)])


def smoothness_sensor(case, W: np.ndarray, e: int) -> float:
    """S_K = (w - w*, w - w*)_K / (w, w)_K (Sec. 4), by its definition: w* is the L2 projection
    of w onto the polynomials of degree p_K - 1, found from the projection's normal equations
    by quadrature; the inner product sums the four conserved fields."""
    m = Mesh(case, make_physics(case))
    g = m.geom(e)
    p = int(case.degree[e])
    wq = W[e, :, : n_modes(p)] @ g.phi                    # (4, Q) at the quadrature points
    low = g.phi[: n_modes(p - 1)]                          # a basis of degree p - 1 at the points
    M = (low * g.wq[None, :]) @ low.T
    c = np.linalg.solve(M, (low * g.wq[None, :]) @ wq.T)  # (Np(p-1), 4)
    d = wq - c.T @ low
    return float(np.sum(d * d * g.wq[None, :]) / np.sum(wq * wq * g.wq[None, :]))


def doerfler_mark(eta: np.ndarray, theta: float) -> np.ndarray:
    """The smallest set M with eta_M >= (1 - theta) eta_T, eta_M^2 = sum over M of eta_K^2
    (Sec. 4): the elements by decreasing eta_K, ties by increasing id, up to the first whose
    partial sum of eta_K^2 reaches (1 - theta)^2 eta_T^2. Returns a boolean mask."""
    eta = np.asarray(eta, dtype=np.float64)
    order = np.argsort(-eta, kind="stable")
    cum = np.cumsum(eta[order] ** 2)
    marked = np.zeros(eta.size, dtype=bool)
    if eta.size == 0:
        return marked
    target = (1.0 - theta) ** 2 * cum[-1]
    if not target > 0.0:
        return marked
    m = int(np.argmax(cum >= target)) + 1
    marked[order[:m]] = True
    return marked


def adaptation_flags(case, W, eta, theta: float = 0.05, eps_s: float = 1e-6):
    """Per element: 0 unmarked, 1 marked for p-enrichment (S_K < eps_S), 2 marked for mesh
    refinement; and the sensor values."""
    S = np.array([smoothness_sensor(case, W, e) for e in range(case.n_elements)])
    marked = doerfler_mark(eta, theta)
    flags = np.where(marked, np.where(S < eps_s, 1, 2), 0).astype(np.int32)
    return flags, S


def enrich(case):
    """The case in the space of one degree more (Sec. 4): every element degree raised by one,
    the state padded with zero coefficients past each element's (face's) own degree (the
    bases are hierarchical, so the padded state is the same function)."""
    import dataclasses
    p1 = int(case.degree.max()) + 1
    npm = n_modes(p1)
    fdeg = Mesh(case, make_physics(case)).face_degree

    def pad_elems(a):
        if a is None:
            return None
        out = np.zeros(a.shape[:-1] + (npm,))
        for e in range(a.shape[0]):
            n = n_modes(int(case.degree[e]))     # modes past the element's degree carry no meaning
            out[e, :, :n] = a[e, :, :n]
        return out

    lam = np.zeros(case.lam.shape[:-1] + (p1 + 1,))
    for f in range(lam.shape[0]):
        lam[f, :, : fdeg[f] + 1] = case.lam[f, :, : fdeg[f] + 1]
    return dataclasses.replace(case, degree=(case.degree + 1).astype(case.degree.dtype), W=pad_elems(case.W),
                               Q=pad_elems(case.Q), lam=lam)


def global_residual(case, W, lam, Q=None, alpha: Optional[float] = None):
    """Assembled residual: per-element local rows and the summed skeleton rows (real inputs)."""
    phys = make_physics(case, alpha)
    mesh = Mesh(case, phys)
    st = State(mesh, W, lam, Q)
    Rloc = []
    Rsk = np.zeros(mesh.n_skel)
    for e in range(mesh.ne):
        We, Qe, lams = st.elem_inputs(e)
        lb = [None if l is None else l[None] for l in lams]
        Rq, Rw, Rl = element_residual(mesh, e, We[None], None if Qe is None else Qe[None], lb)
        Rloc.append(Rw[0] if Rq is None else (Rq[0], Rw[0]))
        for lf in range(3):
            f = mesh.elem_faces[e, lf]
            if f >= 0:
                Rsk[mesh.face_offset[f]: mesh.face_offset[f + 1]] += Rl[lf][0].reshape(-1)
    return mesh, Rloc, Rsk


def residual_norm(case, W, lam, Q=None, alpha: Optional[float] = None) -> float:
    """||N_h(x)||_2 over every residual row: the element rows of each K (Navier-Stokes: the
    gradient rows and the conserved-variable rows) and the summed skeleton rows (Sec. 3.3)."""
    _, Rloc, Rsk = global_residual(case, W, lam, Q, alpha)
    s = float(Rsk @ Rsk)
    for r in Rloc:
        for x in (r if isinstance(r, tuple) else (r,)):
            s += float(np.sum(x * x))
    return math.sqrt(s)


def cfl_schedule(n: int, cfl_prev: float, res_prev: float, res: float,
                 c0: float = 1e6, c1: float = 1e3, n0: int = 4) -> float:
    """eq. cfl: for the first n0 iterations a smooth ramp c0 (3 s^2 - 2 s^3), s = n / n0
    (iterations counted from 1); afterwards the previous CFL grows by the factor
    1 + c1 max(0, log(||N^(n-1)|| / ||N^n||)). The paper's values: c0 = 1e6, c1 = 1e3, n0 = 4."""
    if n <= n0:
        s = n / n0
        return c0 * (3.0 * s * s - 2.0 * s * s * s)
    if res == 0.0:
        return math.inf   # the residual vanished: the pure Newton limit
    return cfl_prev * (1.0 + c1 * max(0.0, math.log(res_prev / res)))


@dataclass
class PseudoTransient:
    W: np.ndarray
    lam: np.ndarray
    Q: Optional[np.ndarray]
    res: List[float]     # ||N_h|| at x_1 .. x_(steps+1)
    cfl: List[float]     # CFL_1 .. CFL_steps


def pseudo_transient(case, steps: int, c0: float = 1e6, c1: float = 1e3, n0: int = 4,
                     alpha: Optional[float] = None) -> PseudoTransient:
    """The relaxed Newton iteration of Sec. 3.3: at iterate x_n, ||N_h(x_n)|| sets CFL_n by
    eq. cfl, one Newton step with the local pseudo-time term of that CFL gives dx, and
    x_(n+1) = x_n + dx. `steps` iterations from the case's state; nothing stops early."""
    import dataclasses
    W = case.W.copy()
    lam = case.lam.copy()
    Q = None if case.Q is None else case.Q.copy()
    res = [residual_norm(case, W, lam, Q, alpha)]
    cfls: List[float] = []
    cfl = 0.0
    for n in range(1, steps + 1):
        cfl = cfl_schedule(n, cfl, res[-2] if n > 1 else 0.0, res[-1], c0, c1, n0)
        cfls.append(cfl)
        cur = dataclasses.replace(case, W=W, lam=lam, Q=Q, cfl=cfl)
        step = newton_step(cur, alpha)
        m = step.mesh
        for e in range(m.ne):
            dW, dQ = unpack_local(m, e, step.du[e], W.shape[2])
            W[e] += dW
            if Q is not None:
                Q[e] += dQ
        for f in range(m.nf):
            pf = m.face_degree[f]
            lam[f, :, : pf + 1] += step.dlam[m.face_offset[f]: m.face_offset[f + 1]].reshape(4, pf + 1)
        res.append(residual_norm(cur, W, lam, Q, alpha))
    return PseudoTransient(W, lam, Q, res, cfls)


def relative_error(x, ref) -> float:
    x = np.asarray(x).ravel()
    ref = np.asarray(ref).ravel()
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (nr if nr > 0 else 1.0))
