"""GPU: the spin product split by bond locality (schedule spin_split = 1:
bonds with an end in the low half of the sites and the fields first, then
the high-half bonds in slab order) against the oracle, for single real and
complex vectors and for blocks of 4 and 16 complex vectors in FP64 and
FP32, with fields, on chains, ladders and the XXZ + J2 ring; the caller's
epilogue through cTPQ and Lanczos against the one-pass product. Tolerances
as for the one-pass kernel: FP64 1e-12 of max|Hv|, FP32 3e-6."""
import sys

import numpy as np
import pytest

from oracle import core as O
from paper_2307_13222_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    from paper_2307_13222_amd import api as A
    return A


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


CASES = [("xxz_j2_16", 16, 0, (1, "f64")), ("ladder_14_field", 14, 2, (1, "c128")),
         ("chain_15", 15, 1, (4, "c128")), ("xxz_j2_16", 16, 0, (16, "c64")),
         ("xxz_j2_18", 18, 0, (16, "c64")), ("ladder_16", 16, 0, (4, "f32")), ("chain_13", 13, 3, (1, "f32"))]


def model(name, n):
    if name.startswith("xxz_j2"):
        return W.xxz_chain_j2(n)
    if name.startswith("ladder"):
        m = W.random_heisenberg(n, "ladder", n)
        if "field" in name:
            m.hz = np.random.default_rng(n).normal(size=n)
        return m
    return W.random_heisenberg(n, "chain", n)


@pytest.mark.parametrize("name,n,two_sz,shape", CASES, ids=[f"{c[0]}-{c[3]}" for c in CASES])
def test_split_mult_vs_oracle(api, ctx, name, n, two_sz, shape):
    import torch
    nvec, dt = shape
    say("split mult", name, shape)
    m = model(name, n)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, n, two_sz), m)
    h.set_schedule(spin_split=1)
    assert h.get_schedule()["spin_split"] == 1
    s = O.basis_list(n, O.sector_popcount_spin(n, two_sz))
    cplx = dt.startswith("c")
    v = W.random_vector(len(s), 7, np.complex128 if cplx else np.float64, nvec=nvec)
    if v.ndim == 1:
        v = v[:, None]
    tdt = {"c128": torch.complex128, "c64": torch.complex64, "f64": torch.float64, "f32": torch.float32}[dt]
    vt = dev(v).to(tdt)
    if nvec == 1:
        vt = vt[:, 0].contiguous()
    w = host(h.mult(vt)).reshape(len(s), nvec)
    ref = O.spin_hv(m, s, host(vt).reshape(len(s), nvec).astype(np.complex128 if cplx else np.float64))
    assert relmax(w, ref) < (1e-12 if dt in ("c128", "f64") else 3e-6)
    # the one-pass product: equal up to summation order
    h.set_schedule(spin_split=-1)
    w1 = host(h.mult(vt)).reshape(len(s), nvec)
    assert relmax(w, w1) < (1e-13 if dt in ("c128", "f64") else 2e-6)


def test_split_ctpq_and_lanczos(api, ctx):
    say("split ctpq / lanczos")
    m = W.xxz_chain_j2(16)
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 16, 0), m)
    s = O.basis_list(16, 8)
    phi0 = O.splitmix_complex_gaussian(3, len(s))
    phi = np.stack([phi0, O.splitmix_complex_gaussian(4, len(s))], axis=1)
    h.set_schedule(spin_split=1)
    g = api.ctpq(h, 2, 6, 0.02, 12, phi0=dev(phi))
    o = O.ctpq(lambda x: O.spin_hv(m, s, x), phi, 6, 0.02, 12)
    assert relmax(g["D"], o["D"]) < 1e-11 and relmax(g["E"], o["E"]) < 1e-11 and relmax(g["E2"], o["E2"]) < 1e-11
    # Lanczos with the split product takes its dots in a pass of their own:
    # the recurrence of the one-pass product up to summation order, and the
    # oracle's
    r = api.lanczos(h, 150, seed=1)
    h.set_schedule(spin_split=-1)
    r1 = api.lanczos(h, 150, seed=1)
    assert np.max(np.abs(r["alpha"][:30] - r1["alpha"][:30])) < 1e-11
    assert abs(r["energies"][0] - r1["energies"][0]) < 1e-10
    o = O.lanczos(lambda x: O.spin_hv(m, s, x), O.splitmix_uniform(1, 0, len(s)), 20)
    assert np.max(np.abs(r["alpha"][:20] - o["alpha"][:20])) < 1e-11


@pytest.mark.parametrize("n,dt", [(18, "f64"), (20, "f32")])
def test_split_implicit_basis(api, ctx, n, dt):
    # the implicit-basis kernel (the path of sectors without a stored state
    # list) with the split: product against the oracle and the one-pass
    # product, Lanczos coefficients against the oracle's recurrence
    import torch
    say("split implicit", n, dt)
    m = W.j1j2_square(n // 2, 2, 1.0, 0.5) if n == 20 else W.xxz_chain_j2(n)
    b = api.Basis.spin(ctx, n, 0)
    h = api.Hamiltonian.spin(b, m)
    h.set_schedule(spin_implicit=1, spin_split=1)
    s = O.basis_list(n, n // 2)
    v = W.random_vector(len(s), 9)
    tdt = torch.float64 if dt == "f64" else torch.float32
    w = host(h.mult(dev(v).to(tdt))).astype(np.float64)
    ref = O.spin_hv(m, s, host(dev(v).to(tdt)).astype(np.float64))
    tol = 1e-12 if dt == "f64" else 3e-6
    assert relmax(w, ref) < tol
    h.set_schedule(spin_split=-1)
    w1 = host(h.mult(dev(v).to(tdt))).astype(np.float64)
    assert relmax(w, w1) < (1e-13 if dt == "f64" else 2e-6)
    if dt == "f64":
        h.set_schedule(spin_split=1)
        r = api.lanczos(h, 40, seed=2)
        o = O.lanczos(lambda x: O.spin_hv(m, s, x), O.splitmix_uniform(2, 0, len(s)), 20)
        assert np.max(np.abs(r["alpha"][:20] - o["alpha"][:20])) < 1e-11
        assert np.max(np.abs(r["beta"][1:20] - o["beta"][1:20])) < 1e-11
