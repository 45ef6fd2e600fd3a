"""Pins of the oracle's residual, Jacobian, condensation and reconstruction
(Sec. 3.2 eq. hdg_ls1..hdg_cont, Sec. 3.3 eq. linearsystem, Sec. 3.4 eq. ls/cons/hybridsystem)."""
import math

import numpy as np
import pytest

import hdg_inputs as hi
from oracle import hdg_oracle as O


def _tiny(physics="euler", ng=3, degrees=(1, 2, 3), amp=2e-2, seed=11, **kw):
    return hi.make_case(physics, ng, list(degrees), 0.5, 2.0, amp, seed=seed,
                        reynolds=200.0 if physics == "ns" else 0.0, **kw)


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_free_stream_preservation(physics):
    c = _tiny(physics, ng=4, degrees=(1, 2, 3, 4), amp=0.0, free_stream_only=True)
    mesh, Rloc, Rsk = O.global_residual(c, c.W, c.lam, c.Q)
    worst = 0.0
    for r in Rloc:
        for x in (r if isinstance(r, tuple) else (r,)):
            worst = max(worst, np.abs(x).max())
    assert worst < 1e-13
    assert np.abs(Rsk).max() < 1e-13


def test_mesh_counts_and_face_degrees():
    c = _tiny(ng=5)
    m = O.Mesh(c, O.make_physics(c))
    assert m.ne == 50 and m.nf == 3 * 25 - 2 * 5
    assert (m.elem_faces < 0).sum() == 4 * 5
    for f, elems in enumerate(m.face_elems):
        assert m.face_degree[f] == max(c.degree[e] for e, _ in elems)
    assert np.array_equal(m.face_vertices, hi.interior_faces(c.tri))


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_jacobian_blocks_vs_central_differences(physics):
    c = _tiny(physics, ng=2, degrees=(1, 2))
    ph = O.make_physics(c)
    mesh = O.Mesh(c, ph)
    st = O.State(mesh, c.W, c.lam, c.Q)
    for e in range(mesh.ne):
        b = O.element_blocks(st, e)
        W, Q, lams = st.elem_inputs(e)
        z0 = np.concatenate([O.pack_local(W, Q)] + [lams[lf].reshape(-1) for lf in range(3) if lams[lf] is not None])
        n = b.A.shape[0]

        def resid(z):
            npe = W.shape[1]
            if physics == "ns":
                Qz, Wz = z[: 8 * npe].reshape(1, 8, npe), z[8 * npe: 12 * npe].reshape(1, 4, npe)
            else:
                Qz, Wz = None, z[:n].reshape(1, 4, npe)
            lb, off = [None] * 3, n
            for lf in range(3):
                if lams[lf] is not None:
                    sz = lams[lf].size
                    lb[lf] = z[off: off + sz].reshape(1, 4, sz // 4)
                    off += sz
            Rq, Rw, Rl = O.element_residual(mesh, e, Wz, Qz, lb)
            loc = Rw.reshape(-1) if Rq is None else np.concatenate([Rq.reshape(-1), Rw.reshape(-1)])
            lam = [Rl[lf].reshape(-1) for lf in range(3) if Rl[lf] is not None]
            return np.concatenate([loc] + lam)

        J = np.vstack([np.hstack([b.A, b.B]), np.hstack([b.C, b.D])])
        Jfd = np.zeros_like(J)
        for j in range(z0.size):
            h = np.finfo(float).eps ** (1 / 3) * max(1.0, abs(z0[j]))
            zp, zm = z0.copy(), z0.copy()
            zp[j] += h
            zm[j] -= h
            Jfd[:, j] = (resid(zp) - resid(zm)) / (2 * h)
        assert np.abs(J - Jfd).max() < 1e-6 * max(1.0, np.abs(J).max())
        assert np.allclose(-resid(z0), np.concatenate([b.r, b.rl]), atol=1e-14)


@pytest.mark.parametrize("name,kw", [
    ("c1", None),
    ("hp-euler", dict(physics="euler", ng=3, degrees=(1, 2, 3, 4, 5))),
    ("ns", dict(physics="ns", ng=3, degrees=(2, 3))),
])
def test_condensation_equals_monolithic_solve(name, kw):
    c = hi.config_case("c1") if kw is None else _tiny(**kw)
    step = O.newton_step(c)
    du_m, dl_m = O.monolithic_solve(step)
    assert O.relative_error(step.dlam, dl_m) < 1e-11
    assert O.relative_error(np.concatenate(step.du), np.concatenate(du_m)) < 1e-11


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_conservation_identity(physics):
    """Testing every element row with 1 and every skeleton row with 1 leaves only the
    boundary flux: sum_K R_K[1] - sum_e R_e[1] = sum over boundary faces of the flux."""
    c = _tiny(physics, ng=3, degrees=(1, 2, 3))
    ph = O.make_physics(c)
    mesh, Rloc, Rsk = O.global_residual(c, c.W, c.lam, c.Q)
    s2 = math.sqrt(2.0)
    tot = np.zeros(4)
    for r in Rloc:
        rw = r[1] if isinstance(r, tuple) else r
        tot += s2 * rw[:, 0]
    for f in range(mesh.nf):
        pe = mesh.face_degree[f]
        tot -= s2 * Rsk[mesh.face_offset[f]: mesh.face_offset[f + 1]].reshape(4, pe + 1)[:, 0]
    # boundary flux computed directly at the boundary quadrature points
    bflux = np.zeros(4)
    for e in range(mesh.ne):
        g = mesh.geom(e)
        npe = g.phi.shape[0]
        for side in g.sides:
            if side.face >= 0:
                continue
            wt = (c.W[e, :, :npe] @ side.phi).T
            wb = wt @ side.Pplus.T + (np.eye(4) - side.Pplus) @ ph.winf
            F = O.euler_flux(wb, ph.gamma)
            if physics == "ns":
                qt = (c.Q[e, :, :npe] @ side.phi).T.reshape(-1, 2, 4)
                F = F - O.viscous_flux(wb, qt, ph)
            bflux += (side.wq[:, None] * (F[0] * side.normal[0] + F[1] * side.normal[1])).sum(0)
    assert np.allclose(tot, bflux, atol=1e-13)


def test_euler_skeleton_row_closed_form():
    """With opposite normals the convective parts cancel: R_e = -alpha int mu (2 lam - w+ - w-)."""
    c = _tiny("euler", ng=3, degrees=(1, 2, 3))
    ph = O.make_physics(c)
    mesh, Rloc, Rsk = O.global_residual(c, c.W, c.lam)
    for f in range(mesh.nf):
        pe = mesh.face_degree[f]
        (e0, lf0), (e1, lf1) = mesh.face_elems[f]
        s0, s1 = mesh.geom(e0).sides[lf0], mesh.geom(e1).sides[lf1]
        lam = (c.lam[f, :, : pe + 1] @ s0.psi).T
        w0 = (c.W[e0, :, : s0.phi.shape[0]] @ s0.phi).T
        w1 = (c.W[e1, :, : s1.phi.shape[0]] @ s1.phi).T
        ref = -ph.alpha * np.einsum("g,kg,ga->ak", s0.wq, s0.psi, 2 * lam - w0 - w1)
        got = Rsk[mesh.face_offset[f]: mesh.face_offset[f + 1]].reshape(4, pe + 1)
        assert np.allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("physics", ["euler", "ns"])
def test_rotational_invariance(physics):
    """Rotating mesh, free stream and momentum coefficients by theta rotates the residual."""
    c = _tiny(physics, ng=3, degrees=(1, 2, 3))
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    c2 = hi.Case(**{k: getattr(c, k) for k in ("name", "physics", "ng", "tri", "degree", "mach", "amp",
                                                "reynolds", "prandtl", "gamma", "face_vertices")},
                 xy=c.xy @ R.T, aoa_deg=c.aoa_deg + math.degrees(th))

    def rot_w(W):
        W2 = W.copy()
        W2[:, 1:3] = np.einsum("ij,ejn->ein", R, W[:, 1:3])
        return W2
    W2, lam2 = rot_w(c.W), rot_w(c.lam)
    Q2 = None
    if physics == "ns":
        # q[4d + a]: rotate the direction index d and the momentum field index a
        Q = c.Q.reshape(c.Q.shape[0], 2, 4, -1)
        Qd = np.einsum("ij,ejan->eian", R, Q)
        Qd[:, :, 1:3] = np.einsum("ij,edjn->edin", R, Qd[:, :, 1:3])
        Q2 = Qd.reshape(c.Q.shape)
    _, R1, S1 = O.global_residual(c, c.W, c.lam, c.Q)
    _, R2, S2 = O.global_residual(c2, W2, lam2, Q2)
    for a, b in zip(R1, R2):
        ra = a[1] if isinstance(a, tuple) else a
        rb = b[1] if isinstance(b, tuple) else b
        assert np.allclose(rot_w(ra[None])[0], rb, atol=1e-12)
    m = O.Mesh(c, O.make_physics(c))
    for f in range(m.nf):
        pe = m.face_degree[f]
        a = S1[m.face_offset[f]: m.face_offset[f + 1]].reshape(1, 4, pe + 1)
        b = S2[m.face_offset[f]: m.face_offset[f + 1]].reshape(4, pe + 1)
        assert np.allclose(rot_w(a)[0], b, atol=1e-12)


def test_ns_gradient_equation_reproduces_linear_gradient():
    """For w linear in x, lam its exact trace and q = grad w, the gradient rows vanish
    on elements without boundary faces (eq. hdg_ls1)."""
    c = _tiny("ns", ng=3, degrees=(1, 2), amp=0.0, free_stream_only=True)
    ph = O.make_physics(c)
    mesh = O.Mesh(c, ph)
    Gm = np.array([[0.1, -0.2], [0.05, 0.3], [-0.1, 0.2], [0.4, 0.1]])   # d w_a / d x_d
    w0 = ph.winf

    def field(x):
        return w0[None, :] + x @ Gm.T

    npm = c.W.shape[2]
    W = np.zeros_like(c.W)
    Q = np.zeros_like(c.Q)
    for e in range(mesh.ne):
        g = mesh.geom(e)
        vals = field(g.xq)                      # (Q, 4)
        proj = (g.phi * g.wq) @ vals / g.detJ   # orthonormal basis: mass = det J * I
        W[e, :, : g.phi.shape[0]] = proj.T
        Q[e, :, 0] = math.sqrt(2.0) * Gm.T.reshape(-1)
    lam = np.zeros_like(c.lam)
    for f in range(mesh.nf):
        (e0, lf0), _ = mesh.face_elems[f]
        s = mesh.geom(e0).sides[lf0]
        a, b = mesh.face_vertices[f]
        pts = c.xy[a][None] * ((1 - s.s) / 2)[:, None] + c.xy[b][None] * ((1 + s.s) / 2)[:, None]
        vals = field(pts)
        lam[f, :, : s.pe + 1] = ((s.psi * (s.wq / (s.length / 2))) @ vals).T
    _, Rloc, _ = O.global_residual(c, W, lam, Q)
    checked = 0
    for e in range(mesh.ne):
        if (mesh.elem_faces[e] < 0).any():
            continue
        assert np.abs(Rloc[e][0]).max() < 1e-13
        checked += 1
    assert checked > 0


def test_newton_converges_quadratically():
    """Two oracle Newton steps on a small smooth case: ||R|| drops quadratically."""
    c = _tiny("euler", ng=3, degrees=(2,), amp=1e-2)
    norms = []
    W, lam = c.W.copy(), c.lam.copy()
    for it in range(3):
        c.W, c.lam = W, lam
        mesh, Rloc, Rsk = O.global_residual(c, W, lam)
        norms.append(math.sqrt(sum(np.sum(r ** 2) for r in Rloc) + np.sum(Rsk ** 2)))
        if it == 2:
            break
        step = O.newton_step(c)
        for e in range(mesh.ne):
            dW, _ = O.unpack_local(mesh, e, step.du[e], W.shape[2])
            W = W.copy()
            W[e] += dW
        lam = lam.copy()
        for f in range(mesh.nf):
            pe = mesh.face_degree[f]
            lam[f, :, : pe + 1] += step.dlam[mesh.face_offset[f]: mesh.face_offset[f + 1]].reshape(4, pe + 1)
    assert norms[1] < norms[0] * 0.1
    assert norms[2] < max(10.0 * norms[1] ** 2 / norms[0], 1e-12)


def test_skeleton_block_pattern():
    """One diagonal and at most 2d = 4 off-diagonal blocks per skeleton row (Sec. 3.4)."""
    c = _tiny("euler", ng=4, degrees=(1, 2, 3))
    step = O.newton_step(c)
    m = step.mesh
    K = step.K.tocsr()
    for f in range(m.nf):
        rows = K[m.face_offset[f]: m.face_offset[f + 1]]
        cols = np.unique(rows.indices)
        blocks = set(np.searchsorted(m.face_offset, cols, side="right") - 1)
        assert f in blocks and len(blocks) <= 5
        nb = sum(1 for e, _ in m.face_elems[f] for g in m.elem_faces[e] if g >= 0 and g != f)
        assert len(blocks) == 1 + nb


def test_skeleton_operator_dissipative_spectrum():
    """Block-Jacobi-preconditioned skeleton operator of the c1 case: all eigenvalues in the
    right half plane (the alpha term is dissipative)."""
    step = O.newton_step(hi.config_case("c1"))
    K = step.K.toarray()
    m = step.mesh
    P = np.zeros_like(K)
    for f in range(m.nf):
        a, b = m.face_offset[f], m.face_offset[f + 1]
        P[a:b, a:b] = np.linalg.inv(K[a:b, a:b])
    assert np.linalg.eigvals(K @ P).real.min() > 0
