"""CPU checks of the boundary: the built library loads and exports every
function the public header declares (no compute calls without a GPU), and
the binding's declarations match the header."""
import ctypes
import os
import re

import pytest

from paper_2307_13222_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hphi_mi355.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hphi_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_calls():
    names = header_functions()
    for must in ["hphi_init", "hphi_basis_spin", "hphi_basis_hubbard", "hphi_ham_spin",
                 "hphi_ham_hubbard", "hphi_mult", "hphi_lanczos", "hphi_ctpq", "hphi_sqw",
                 "hphi_time_evolve"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2307_13222_amd import build
        build.build(verbose=False)
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert set(header_functions()) <= set(_lib.SIGNATURES)


def test_version_and_last_error_without_gpu():
    L = _lib.lib()
    assert b"gfx950" in L.hphi_version()
    assert L.hphi_last_error() is not None


def test_tridiag_host_routine_matches_lapack():
    # host-only entry point: Sturm bisection + inverse iteration vs LAPACK
    import numpy as np
    import scipy.linalg
    from paper_2307_13222_amd import api
    rng = np.random.default_rng(1)
    for n in (1, 2, 7, 60, 300):
        a = rng.normal(size=n)
        b = np.concatenate([[0.0], rng.normal(size=n - 1)])
        k = min(n, 4)
        ev, vec = api.tridiag_lowest(a, b, k, want_vector=True)
        ref, U = scipy.linalg.eigh_tridiagonal(a, b[1:])
        scale = max(1.0, np.abs(ref).max())
        assert np.allclose(ev, ref[:k], atol=8 * np.finfo(float).eps * scale * max(1, n) ** 0.5)
        u0 = U[:, 0] * np.sign(U[np.argmax(np.abs(U[:, 0])), 0])
        if n == 1 or ref[1] - ref[0] > 1e-6:
            assert np.allclose(vec, u0, atol=1e-9)


def test_tridiag_lanczos_like_spectrum():
    # a T_k from the oracle's own Lanczos, with near-degenerate ghost values
    import numpy as np
    from oracle import core as O
    from paper_2307_13222_amd import api, workloads as W
    m = W.heisenberg_chain(12)
    s = O.basis_list(12, 6)
    r = O.lanczos(lambda v: O.spin_hv(m, s, v), O.splitmix_uniform(1, 0, len(s)), 200)
    ev = api.tridiag_lowest(r["alpha"], r["beta"], 3)
    ref = O.tridiag_lowest(r["alpha"], r["beta"], 3)
    assert np.allclose(ev, ref, atol=1e-12)


def test_invalid_arguments_fail_cleanly():
    import numpy as np
    from paper_2307_13222_amd import api
    with pytest.raises(api.HphiError):
        api.tridiag_lowest(np.zeros(3), np.zeros(3), 5)
