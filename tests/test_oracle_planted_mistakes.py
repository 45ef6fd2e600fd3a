"""The oracle's pins reject plausible mistakes planted in the oracle itself.

Each case rewrites one expression of an oracle function in memory (the function is recompiled
from its own source with the change and installed in the oracle module for this test only) and
runs the pin that has to catch it. A pin that still passed would let that mistake through into
every parity comparison.
"""
import inspect
import textwrap

import pytest

from oracle import hdg_oracle as O
import test_oracle_discretization as PD
import test_oracle_physics as PP
import test_oracle_shock as PS


def _planted(func, edits):
    """func recompiled from its source with every (old, new) substitution applied."""
    src = textwrap.dedent(inspect.getsource(func))
    for old, new in edits:
        assert old in src, f"{func.__name__}: {old!r} not found"
        src = src.replace(old, new)
    namespace = dict(vars(O))
    exec(compile(src, f"<planted {func.__name__}>", "exec"), namespace)
    return namespace[func.__name__]


CASES = [
    # Sec. 2.1: the momentum flux printed as p Id + v (x) v (the density dropped)
    ("momentum flux without rho", "euler_flux",
     [("mx * u + p", "u * u + p"), ("my * v + p", "v * v + p")],
     lambda: PP.test_normal_jacobian_eigenvalues(0.4)),
    # Sec. 2.2: the 2/3 of the Newtonian stress's dilatation term
    ("stress with 1/3 div v", "viscous_flux",
     [("2.0 / 3.0 * div", "1.0 / 3.0 * div")],
     PP.test_viscous_flux_shear_and_heat),
    # far-field projector: the eigenvalue test that keeps u_n = 0 characteristics from the interior
    ("projector drops zero eigenvalues", "farfield_projector",
     [("if mj < 0.0:", "if mj <= 0.0:")],
     PP.test_farfield_tangential_flow_takes_interior_value),
    # Sec. 3.2: the sign of the stabilisation alpha (lam - w) in the trace flux
    ("alpha term with + sign", "element_residual",
     [("- phys.alpha * (lam - wt)", "+ phys.alpha * (lam - wt)")],
     PD.test_euler_skeleton_row_closed_form),
    # eq. hdg_ls1: the sign of the face term <tau . n, lam> of the gradient equation
    ("gradient face term with + sign", "element_residual",
     [('Rq = Rq - np.einsum("g,ng,d,bga->bdan"', 'Rq = Rq + np.einsum("g,ng,d,bga->bdan"')],
     PD.test_ns_gradient_equation_reproduces_linear_gradient),
    # Sec. 3.1: the orientation of the outward face normal
    ("inward face normals", "element_residual",
     [("n = side.normal", "n = -side.normal")],
     lambda: PD.test_free_stream_preservation("euler")),
    # Sec. 3.2, viscous form: the Navier-Stokes sensor reading grad w_h instead of q_h
    ("sensor ignores q_h", "shock_viscosity",
     [("if Q is None:", "if True:")],
     PS.test_ns_viscosity_with_the_exact_gradient_equals_the_euler_form),
]


@pytest.mark.parametrize("label,name,edits,pin", CASES, ids=[c[0] for c in CASES])
def test_pin_rejects_planted_mistake(monkeypatch, label, name, edits, pin):
    monkeypatch.setattr(O, name, _planted(getattr(O, name), edits))
    with pytest.raises(AssertionError):
        pin()


@pytest.mark.parametrize("label,name,edits,pin", CASES, ids=[c[0] for c in CASES])
def test_pin_passes_on_the_unchanged_oracle(label, name, edits, pin):
    # the same pin on the oracle as committed (the planted cases above are not vacuous)
    pin()
