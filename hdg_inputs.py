"""Seeded synthetic workloads for one implicit-HDG Newton step.

This module is shared by the CPU oracle and the GPU harness. It holds no
discretisation arithmetic: it builds meshes, degree maps, flow parameters and
state coefficient arrays, nothing else.

Workload recipe (stands in for the airfoil meshes of Sec. 5, which are not
available):
  * unit square, ng x ng quads, each split along its (i,j)-(i+1,j+1) diagonal
    into two counter-clockwise triangles; interior vertices jittered by
    independent U(-0.1h, 0.1h) in x and y, boundary vertices fixed;
  * far-field boundary on all four sides;
  * non-dimensional free stream rho = 1, p = 1/gamma (sound speed 1),
    v = Ma (cos a, sin a);
  * a smooth sine perturbation of amplitude `amp` in density and both momenta.

State representation. Unknowns are coefficients of hierarchical orthonormal
bases (Sec. 4.3 names a hierarchical Dubiner basis): on the reference triangle
of area 2 the constant mode is 1/sqrt(2), on the reference edge [-1,1] the
constant Legendre mode is 1/sqrt(2). A constant field c therefore has the
leading coefficient sqrt(2) c and no other. The generator sets the leading
coefficient from the smooth field at the element centroid (face midpoint for
traces) and fills the higher modes with seeded uniform noise that decays by a
factor 2 per polynomial degree. Arrays are padded to the largest degree in the
case; modes beyond an element's (face's) own degree are ignored by both sides.

Layouts (all float64, C order):
  W[e, a, i]        element e, field a in (rho, rho u, rho v, E), mode i < Np(pmax)
  Q[e, 4d + a, i]   Navier-Stokes gradient unknowns q = grad w, direction d
  lam[f, a, k]      interior face f in canonical order, mode k <= pmax
Canonical interior-face order: faces sorted by (lower vertex id, higher vertex id).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

GAMMA = 1.4
SQRT2 = math.sqrt(2.0)


def n_modes(p: int) -> int:
    """Dimension of the polynomials of total degree <= p on a triangle."""
    return (p + 1) * (p + 2) // 2


def mode_degree(i: int) -> int:
    """Total degree of hierarchical mode i (modes are grouped by degree)."""
    k = 0
    while n_modes(k) <= i:
        k += 1
    return k


@dataclass
class Case:
    name: str
    physics: str                    # "euler" or "ns"
    ng: int
    xy: np.ndarray                  # (Nv, 2) float64
    tri: np.ndarray                 # (Ne, 3) int32, counter-clockwise
    degree: np.ndarray              # (Ne,) int8, polynomial degree per element
    mach: float
    aoa_deg: float
    amp: float
    reynolds: float = 0.0
    prandtl: float = 0.72
    gamma: float = GAMMA
    cfl: float = 0.0                # pseudo-time CFL number; 0 = pure Newton
    sc_eps0: float = 0.0            # shock-capturing factor epsilon_0; 0 = off
    sc_beta: float = 0.0            # shock-capturing exponent beta
    W: Optional[np.ndarray] = None
    Q: Optional[np.ndarray] = None
    lam: Optional[np.ndarray] = None
    face_vertices: Optional[np.ndarray] = None   # (Nf, 2) int32, canonical interior faces
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_elements(self) -> int:
        return int(self.tri.shape[0])

    @property
    def pmax(self) -> int:
        return int(self.degree.max())

    def free_stream(self) -> np.ndarray:
        return free_stream(self.mach, self.aoa_deg, self.gamma)


def free_stream(mach: float, aoa_deg: float, gamma: float = GAMMA) -> np.ndarray:
    a = math.radians(aoa_deg)
    u, v = mach * math.cos(a), mach * math.sin(a)
    p = 1.0 / gamma
    return np.array([1.0, u, v, p / (gamma - 1.0) + 0.5 * (u * u + v * v)])


def square_mesh(ng: int, rng: Optional[np.random.Generator], jitter: float = 0.1):
    """Jittered ng x ng unit-square mesh split into 2 ng^2 counter-clockwise triangles."""
    h = 1.0 / ng
    ii, jj = np.meshgrid(np.arange(ng + 1), np.arange(ng + 1), indexing="xy")
    xy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1).astype(np.float64)
    if rng is not None and jitter > 0:
        d = rng.uniform(-jitter * h, jitter * h, size=xy.shape)
        inner = (ii.ravel() > 0) & (ii.ravel() < ng) & (jj.ravel() > 0) & (jj.ravel() < ng)
        xy[inner] += d[inner]
    vid = lambda i, j: j * (ng + 1) + i
    tris = []
    for j in range(ng):
        for i in range(ng):
            v00, v10, v11, v01 = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris.append((v00, v10, v11))
            tris.append((v00, v11, v01))
    return xy, np.asarray(tris, dtype=np.int32)


def interior_faces(tri: np.ndarray) -> np.ndarray:
    """Edges shared by two triangles, as sorted vertex pairs in canonical order."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]], axis=0)
    e = np.sort(e, axis=1)
    uniq, counts = np.unique(e, axis=0, return_counts=True)
    return uniq[counts == 2].astype(np.int32)


class SineField:
    """Free stream plus A s_c sin(2 pi (k1 x + f1)) sin(2 pi (k2 y + f2)) in rho, rho u, rho v."""

    def __init__(self, winf: np.ndarray, amp: float, rng: np.random.Generator):
        self.winf = winf
        speed = math.hypot(winf[1], winf[2]) / winf[0]
        self.scale = np.array([1.0, speed, speed, 0.0]) * amp
        self.k = rng.integers(1, 4, size=(3, 2))
        self.phi = rng.uniform(0.0, 1.0, size=(3, 2))

    def value(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        out = np.broadcast_to(self.winf, x.shape + (4,)).copy()
        for c in range(3):
            sx = np.sin(2 * np.pi * (self.k[c, 0] * x + self.phi[c, 0]))
            sy = np.sin(2 * np.pi * (self.k[c, 1] * y + self.phi[c, 1]))
            out[..., c] += self.scale[c] * sx * sy
        return out

    def gradient(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        """(..., 2, 4): d/dx and d/dy of each field."""
        g = np.zeros(x.shape + (2, 4))
        for c in range(3):
            ax = 2 * np.pi * (self.k[c, 0] * x + self.phi[c, 0])
            ay = 2 * np.pi * (self.k[c, 1] * y + self.phi[c, 1])
            g[..., 0, c] = self.scale[c] * 2 * np.pi * self.k[c, 0] * np.cos(ax) * np.sin(ay)
            g[..., 1, c] = self.scale[c] * 2 * np.pi * self.k[c, 1] * np.sin(ax) * np.cos(ay)
        return g


def _decay(npm: int) -> np.ndarray:
    return np.array([0.5 ** mode_degree(i) for i in range(npm)])


def fill_state(case: Case, rng: np.random.Generator, free_stream_only: bool = False) -> Case:
    """Fill W, lam (and Q for Navier-Stokes) with the seeded recipe above."""
    winf = case.free_stream()
    pmax = case.pmax
    npm = n_modes(pmax)
    ne = case.n_elements
    fv = interior_faces(case.tri)
    case.face_vertices = fv
    amp = 0.0 if free_stream_only else case.amp
    fld = SineField(winf, amp, rng)
    cen = case.xy[case.tri].mean(axis=1)
    mid = case.xy[fv].mean(axis=1)

    W = np.zeros((ne, 4, npm))
    W[:, :, 0] = SQRT2 * fld.value(cen[:, 0], cen[:, 1])
    noise = rng.uniform(-1.0, 1.0, size=(ne, 4, npm))
    W[:, :, 1:] = (SQRT2 * noise * fld.scale[None, :, None] * _decay(npm)[None, None, :])[:, :, 1:]
    case.W = W

    lam = np.zeros((fv.shape[0], 4, pmax + 1))
    lam[:, :, 0] = SQRT2 * fld.value(mid[:, 0], mid[:, 1])
    noise = rng.uniform(-1.0, 1.0, size=(fv.shape[0], 4, pmax + 1))
    ldec = 0.5 ** np.arange(pmax + 1)
    lam[:, :, 1:] = (SQRT2 * noise * fld.scale[None, :, None] * ldec[None, None, :])[:, :, 1:]
    case.lam = lam

    if case.physics == "ns":
        Q = np.zeros((ne, 8, npm))
        g = fld.gradient(cen[:, 0], cen[:, 1])          # (ne, 2, 4)
        Q[:, :, 0] = SQRT2 * g.reshape(ne, 8)
        noise = rng.uniform(-1.0, 1.0, size=(ne, 8, npm))
        qs = np.tile(fld.scale, 2)
        Q[:, :, 1:] = (SQRT2 * noise * qs[None, :, None] * _decay(npm)[None, None, :])[:, :, 1:]
        case.Q = Q
    else:
        case.Q = None
    return case


def _rngs(seed: int, n: int = 3):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def make_case(physics: str, ng: int, degrees, mach: float, aoa_deg: float, amp: float,
              seed: int, reynolds: float = 0.0, prandtl: float = 0.72, name: str = "custom",
              degree_weights=None, jitter: float = 0.1, free_stream_only: bool = False,
              cfl: float = 0.0) -> Case:
    """Build a case. `degrees` is an int (uniform) or a list of allowed degrees
    drawn per element with `degree_weights` (uniform if None)."""
    r_jit, r_deg, r_state = _rngs(seed)
    xy, tri = square_mesh(ng, r_jit, jitter)
    ne = tri.shape[0]
    if isinstance(degrees, (int, np.integer)):
        deg = np.full(ne, int(degrees), dtype=np.int8)
    else:
        choices = np.asarray(list(degrees), dtype=np.int64)
        deg = r_deg.choice(choices, size=ne, p=degree_weights).astype(np.int8)
    case = Case(name=name, physics=physics, ng=ng, xy=xy, tri=tri, degree=deg, mach=mach,
                aoa_deg=aoa_deg, amp=amp, reynolds=reynolds, prandtl=prandtl, seed=seed, cfl=cfl)
    return fill_state(case, r_state, free_stream_only)


# The five workloads. Index c seeds the generator with 1308 + c.
CONFIGS = {
    "c1": dict(physics="euler", ng=8, degrees=1, mach=0.5, aoa_deg=2.0, amp=1e-2),
    "c2": dict(physics="euler", ng=64, degrees=3, mach=0.5, aoa_deg=2.0, amp=1e-2),
    "c3": dict(physics="euler", ng=128, degrees=[1, 2, 3, 4, 5], mach=0.8, aoa_deg=1.25, amp=5e-2,
               degree_weights=[0.3, 0.3, 0.2, 0.1, 0.1]),
    "c4": dict(physics="ns", ng=256, degrees=[2, 3, 4], mach=0.5, aoa_deg=1.0, amp=1e-2,
               reynolds=5000.0, prandtl=0.72),
}
CONFIG_INDEX = {"c1": 0, "c2": 1, "c3": 2, "c4": 3, "c5": 4}


def config_case(name: str, ng: Optional[int] = None) -> Case:
    """One of the named workloads; `ng` overrides the grid size (same recipe, smaller mesh)."""
    kw = dict(CONFIGS[name])
    if ng is not None:
        kw["ng"] = ng
    return make_case(name=name, seed=1308 + CONFIG_INDEX[name], **kw)


@dataclass
class Request:
    index: int
    arrival_s: float
    physics: str
    ng: int
    degree: int
    mach: float
    aoa_deg: float
    seed: int

    def case(self) -> Case:
        return make_case(self.physics, self.ng, self.degree, self.mach, self.aoa_deg, 1e-2,
                         seed=self.seed, reynolds=5000.0 if self.physics == "ns" else 0.0,
                         name=f"req{self.index}")


def serving_stream(n_requests: int = 512, rate_per_s: float = 200.0, seed: int = 1313,
                   ne_range=(2000, 64000), degrees=(1, 2, 3, 4)):
    """Poisson arrivals; mesh size log-uniform in elements; Euler or NS with probability 1/2."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_requests))
    out = []
    for r in range(n_requests):
        ne = math.exp(rng.uniform(math.log(ne_range[0]), math.log(ne_range[1])))
        ng = max(2, int(round(math.sqrt(ne / 2.0))))
        out.append(Request(index=r, arrival_s=float(t[r]),
                           physics="ns" if rng.uniform() < 0.5 else "euler", ng=ng,
                           degree=int(rng.choice(np.asarray(degrees))),
                           mach=float(rng.uniform(0.3, 0.9)), aoa_deg=float(rng.uniform(-3.0, 3.0)),
                           seed=int(seed * 1000 + r)))
    return out
