"""Host-side checks of the C-ABI library (no GPU): it loads and exports every symbol the
header declares, and the header and binding agree."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdg.h")
LIB = os.path.join(ROOT, "paper_1308_3995_amd", "libhdg.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hdg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("hdg_plan_create", "hdg_assemble_condense", "hdg_skeleton_solve", "hdg_back_substitute",
              "hdg_plan_destroy", "hdg_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_declared_symbol():
    from paper_1308_3995_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_error_string_starts_empty_and_plan_rejects_null():
    from paper_1308_3995_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.hdg_plan_create(ctypes.byref(h), None, 0, None, 0, None, None, 0)
    assert st == 1
    assert b"null" in lib.hdg_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_cfl_schedule_matches_the_oracle():
    """The library's eq. cfl (host arithmetic) against the oracle's, over the ramp, growth,
    a growing residual and a vanished one."""
    import math
    from oracle import hdg_oracle as O
    from paper_1308_3995_amd import _lib
    lib = _lib.load()
    cases = [(n, 0.0, 0.0, 1.0, 1e6, 1e3, 4) for n in range(1, 5)]
    cases += [(5, 1e6, 3.0e-2, 1.0e-3, 1e6, 1e3, 4), (7, 12.5, 1.0, 2.0, 10.0, 1.0, 2),
              (3, 21.5, 1.7e-3, 6.0e-4, 10.0, 1.0, 2), (9, 4.0, 1.0, 0.0, 1e6, 1e3, 4),
              (2, 0.0, 0.0, 1.0, 10.0, 1.0, 3)]
    for n, cp, rp, r, c0, c1, n0 in cases:
        got = lib.hdg_cfl_schedule(n, cp, rp, r, c0, c1, n0)
        ref = O.cfl_schedule(n, cp, rp, r, c0, c1, n0)
        if math.isinf(ref):
            assert math.isinf(got)
        else:
            assert abs(got - ref) <= 1e-15 * abs(ref), (n, got, ref)
    assert lib.hdg_set_cfl(None, 1.0) == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_hessenberg_eigenvalues_match_numpy():
    """The host QR iteration behind the polynomial preconditioner's roots against LAPACK (numpy)
    on random upper Hessenberg matrices: real and complex spectra, a split (zero subdiagonal),
    wide scaling, and the 1x1 and 2x2 cases."""
    import numpy as np
    import scipy.linalg
    from scipy.optimize import linear_sum_assignment
    import paper_1308_3995_amd as hdg
    rng = np.random.default_rng(7)
    worst = 0.0
    for trial in range(400):
        n = int(rng.integers(1, 41))
        A = rng.standard_normal((n, n)) * 10.0 ** rng.uniform(-3, 3)
        H = scipy.linalg.hessenberg(A)
        if trial % 5 == 0 and n > 3:
            H[n // 2, n // 2 - 1] = 0.0
        ev = hdg.hessenberg_eigenvalues(H)
        ref = np.linalg.eigvals(H)
        C = np.abs(ev[:, None] - ref[None, :])
        r, c = linear_sum_assignment(C)
        worst = max(worst, C[r, c].max() / np.abs(ref).max())
        # conjugate pairs: +imaginary part first
        for k in range(n - 1):
            if ev[k].imag > 0:
                assert ev[k + 1] == np.conj(ev[k])
    assert worst < 1e-11, worst
    # a rotation block [[0, -1], [1, 0]]: eigenvalues +-i
    ev = hdg.hessenberg_eigenvalues(np.array([[0.0, -1.0], [1.0, 0.0]]))
    assert np.allclose(sorted(ev, key=lambda z: z.imag), [-1j, 1j], atol=1e-15)
