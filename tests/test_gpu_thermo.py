"""GPU: finite-temperature and spectral quantities from device results --
cTPQ thermodynamics with the bootstrap against exact canonical values of the
same sector, mTPQ energies against canonical energies at the mTPQ
temperatures, and the Lanczos continued fraction against direct solves."""
import math
import sys

import numpy as np
import pytest

from oracle import core as O
from paper_2307_13222_amd import thermo as T
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


@pytest.fixture(scope="module")
def chain12():
    m = W.heisenberg_chain(12)
    s = O.basis_list(12, 6)
    ev = np.linalg.eigvalsh(O.spin_sparse(m, s).toarray())
    return m, s, ev


def test_ctpq_thermodynamics_against_canonical(api, ctx, chain12):
    say("thermo ctpq")
    m, s, ev = chain12
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), m)
    r = api.ctpq(h, 16, 6, 0.02, 150, storage="c128", seed=5)
    th = T.tpq_thermo(r["beta"], r["D"], r["E"], r["E2"], len(s), 12, n_boot=200)
    ex = O.canonical_thermo(ev, r["beta"], 12)
    for key in ("E", "C", "S"):
        dev = np.abs(th[key] - ex[key])
        assert np.all(dev < 5 * th[key + "_err"] + 3e-3), (key, float(dev.max()))
    # infinite temperature: S = ln(d_H) / N exactly
    assert abs(th["S"][0] - math.log(len(s)) / 12) < 1e-12


def test_mtpq_energy_against_canonical(api, ctx, chain12):
    say("thermo mtpq")
    m, s, ev = chain12
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), m)
    r = T.mtpq(api, h, 8, 1.0, 300, 12, seed=9)
    beta = r["beta"]
    assert np.all(np.diff(beta, axis=0) > 0)
    # average over vectors at each step; compare with the canonical energy at
    # the vectors' mean temperature (the spread of beta_k is tiny here)
    bm = beta.mean(axis=1)
    assert np.max(beta.std(axis=1) / np.maximum(bm, 1e-12)) < 0.05
    ex = O.canonical_thermo(ev, bm, 12)["E"]
    assert np.max(np.abs(r["u"].mean(axis=1) - ex)) < 0.02


def test_lanczos_continued_fraction_against_direct(api, ctx, chain12):
    import torch
    say("thermo continued fraction")
    m, s, ev = chain12
    h = api.Hamiltonian.spin(api.Basis.spin(ctx, 12, 0), m)
    Hs = O.spin_sparse(m, s)
    e, U = np.linalg.eigh(Hs.toarray())
    psi = U[:, 0]
    b = O.szq_excitation(m, s, math.pi, psi)
    assert np.max(np.abs(b.imag)) < 1e-14        # q = pi: the phases are +-1
    bd = torch.from_numpy(np.ascontiguousarray(b.real)).cuda()
    z = e[0] + np.linspace(0.0, 4.0, 32) + 0.1j
    g = T.lanczos_spectrum(api, h, bd, 300, z)
    ref = O.dyn_corr_direct(Hs, b, z)
    assert np.max(np.abs(g["D"] - ref)) / np.max(np.abs(ref)) < 1e-8
    assert np.all(-g["D"].imag > 0)
