"""Host C/C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The library's host pieces (rank-table construction, the FP64 tridiagonal
  eigensolver and the one-user guard of a Hamiltonian) are built with g++
  and both sanitizers by tests/native/host_check.cpp and run: tables against
  enumeration for every (N, n, split) with N <= 16, the tridiagonal solver
  against LAPACK, the guard's thread and stream rules against a fake device.
* The oracle's C part is rebuilt with both sanitizers, loaded into a child
  Python with the sanitizer runtime preloaded, and its H*v and ranking
  functions must give the same numbers as the regular build.
"""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")

needs_gxx = pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(f"{ROCM}/include/hip"),
                               reason="g++ and the ROCm headers are needed")


@pytest.fixture(scope="module")
def host_check(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("san") / "host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g"] + SAN + [
        "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
        os.path.join(ROOT, "tests", "native", "host_check.cpp"),
        os.path.join(ROOT, "paper_2307_13222_amd", "csrc", "host.cpp"),
        f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


@needs_gxx
def test_rank_tables_sanitized(host_check):
    r = subprocess.run([host_check, "tables"], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("tables ok")


@needs_gxx
def test_guard_sanitized(host_check):
    r = subprocess.run([host_check, "guard"], capture_output=True, text=True, env=ENV, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "guard ok" in r.stdout


@needs_gxx
@pytest.mark.parametrize("n,k,seed", [(1, 1, 0), (2, 2, 1), (7, 3, 2), (60, 5, 3), (300, 4, 4)])
def test_tridiag_sanitized_vs_lapack(host_check, n, k, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-2, 2, n)
    b = np.concatenate([[0.0], rng.uniform(0.1, 1.0, n - 1)])
    inp = f"{n} {k}\n" + " ".join(repr(float(x)) for x in a) + "\n" + " ".join(repr(float(x)) for x in b) + "\n"
    r = subprocess.run([host_check, "tridiag"], input=inp, capture_output=True, text=True, env=ENV, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    vals = np.array([float(x) for x in r.stdout.split()])
    ev, vec = vals[:k], vals[k:]
    ref_ev, ref_vec = scipy.linalg.eigh_tridiagonal(a, b[1:], select="i", select_range=(0, k - 1))
    tnorm = np.max(np.abs(a)) + 2 * np.max(np.abs(b))
    assert np.max(np.abs(ev - ref_ev)) <= 8 * np.finfo(float).eps * tnorm * max(1, np.log2(n))
    v0 = ref_vec[:, 0]
    assert min(np.max(np.abs(vec - v0)), np.max(np.abs(vec + v0))) < 1e-8


ORACLE_CHILD = r"""
import sys, numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import core as O
from paper_2307_13222_amd import workloads as W
out = {}
s = O.basis_list(14, 7)
out["rank"] = O.rank_combinadic(s)
out["search"] = O.rank_search(s, s[::7])
m = W.random_heisenberg(14, "ladder", 3)
v = W.random_vector(len(s), 1)
out["spin"] = O.spin_hv(m, s, v)
hm = W.hubbard_square(2, 3, 1.0, 4.0)
ups, dns = O.hubbard_basis(6, 3, 2)
vh = W.random_vector(len(ups) * len(dns), 2)
out["hub"] = O.hubbard_hv(hm, ups, dns, vh)
out["sm"] = O.splitmix_uniform(7, 3, 100)
np.savez(sys.argv[2], **out)
"""


@needs_gxx
def test_oracle_c_sanitized(tmp_path):
    src = os.path.join(ROOT, "oracle", "hphi_oracle.c")
    so = str(tmp_path / "libhphi_oracle_san.so")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fPIC", "-shared"] + SAN +
                   ["-o", so, src, "-lm"], check=True, capture_output=True)
    pre = " ".join(subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True).stdout.strip()
                   for n in ("libasan.so", "libubsan.so"))
    script = tmp_path / "child.py"
    script.write_text(ORACLE_CHILD)
    ref_out, san_out = str(tmp_path / "ref.npz"), str(tmp_path / "san.npz")
    subprocess.run([sys.executable, str(script), ROOT, ref_out], check=True, capture_output=True, timeout=300)
    env = dict(ENV, LD_PRELOAD=pre, HPHI_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, str(script), ROOT, san_out], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    a, b = np.load(ref_out), np.load(san_out)
    for k in a.files:
        assert np.array_equal(a[k], b[k]), k
