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


STRUCTS = {
    "SpinBond": "hphi_spin_bond", "Hop": "hphi_hop", "XyzBond": "hphi_xyz_bond", "PairTerm": "hphi_pair_term",
    "HubFrames": "hphi_hub_frames", "LanczosOpts": "hphi_lanczos_opts", "LanczosInfo": "hphi_lanczos_info",
    "BatchItem": "hphi_batch_item", "CtpqOpts": "hphi_ctpq_opts", "TevolOpts": "hphi_tevol_opts",
    "LobpcgOpts": "hphi_lobpcg_opts", "LobpcgInfo": "hphi_lobpcg_info", "Schedule": "hphi_schedule",
    "SqwOpts": "hphi_sqw_opts", "SqwInfo": "hphi_sqw_info",
}


def test_binding_structs_match_header_layout(tmp_path):
    # sizeof and every field's offset, from the header compiled by gcc
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for py, c in STRUCTS.items():
        lines.append(f'printf("{py} size %zu\\n", sizeof({c}));')
        for f, _ in getattr(_lib, py)._fields_:
            lines.append(f'printf("{py} {f} %zu\\n", offsetof({c}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in out:
        if not line:
            continue
        py, f, val = line.split()
        cls = getattr(_lib, py)
        got = ctypes.sizeof(cls) if f == "size" else getattr(cls, f).offset
        assert got == int(val), (py, f, got, val)
    # every header field is in the binding (same count)
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for py, c in STRUCTS.items():
        body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + c + r"\s*;", text).group(1)
        decl = [d.strip() for d in body.replace("\n", " ").split(";") if d.strip()]
        n = sum(len(d.split(",")) for d in decl)
        assert n == len(getattr(_lib, py)._fields_), (c, n)
