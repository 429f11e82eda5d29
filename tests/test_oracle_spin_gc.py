"""Pins of the oracle's SpinGC H*v (spin-1/2 on the full 2^N space, SpinGC
keyword of Sec. 4.1, Table "Keywords"): an independent Pauli Kronecker-
product construction, the transverse-field Ising ring's free-fermion
ground energy, and the S^z-conserving case against the sector oracle
(the full spectrum is the union of the sector spectra)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from oracle import core as O
from paper_2307_13222_amd import workloads as W

SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SY = np.array([[0.0, -1j], [1j, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])


def pauli_dense(m) -> np.ndarray:
    """H from Kronecker products of 2x2 Pauli matrices in the basis
    (down, up) = (bit 0, bit 1) of each site, highest site first, so the
    row index is the configuration."""
    n = m.n_sites
    # matrices in (bit 0 = down, bit 1 = up) order: swap the (up, down) ones
    P = np.array([[0.0, 1.0], [1.0, 0.0]])
    ops = {"x": P @ SX @ P, "y": P @ SY @ P, "z": P @ SZ @ P}

    def site_op(a, i):
        out = np.array([[1.0 + 0j]])
        for k in range(n - 1, -1, -1):
            out = np.kron(out, ops[a] if k == i else np.eye(2))
        return out

    H = np.zeros((1 << n, 1 << n), dtype=complex)
    for b in range(m.n_bonds):
        i, j = int(m.bi[b]), int(m.bj[b])
        for a, c in (("x", m.jx[b]), ("y", m.jy[b]), ("z", m.jz[b])):
            H += 0.25 * c * site_op(a, i) @ site_op(a, j)
    for i in range(n):
        H -= 0.5 * m.hx[i] * site_op("x", i) + 0.5 * m.hz[i] * site_op("z", i)
    return H


@pytest.mark.parametrize("n,lat,seed", [(3, "chain", 1), (6, "chain", 2), (6, "ladder", 3), (8, "ladder", 4)])
def test_spin_gc_matches_pauli_products(n, lat, seed):
    m = W.random_spin_gc(n, lat, seed)
    ref = pauli_dense(m)
    assert np.max(np.abs(ref.imag)) < 1e-14
    Hs = O.spin_gc_sparse(m).toarray()
    assert np.allclose(Hs, ref.real, atol=1e-14)
    v = W.random_vector(1 << n, seed)
    assert np.allclose(O.spin_gc_hv(m, v), ref.real @ v, atol=1e-13)
    vc = W.random_vector(1 << n, seed + 1, np.complex128)
    assert np.allclose(O.spin_gc_hv(m, vc), ref.real @ vc, atol=1e-13)
    part = O.spin_gc_hv_rows(m, v, 3, 5)
    assert np.allclose(part, (ref.real @ v)[3:8], atol=1e-13)


def tfim_ring_e0(n, j, g):
    # free fermions (Pfeuty): the ground state lies in the even-parity
    # sector with antiperiodic momenta k = pi (2 m + 1) / n
    ks = np.pi * (2 * np.arange(n) + 1) / n
    return -np.sum(np.sqrt(j * j + g * g - 2 * j * g * np.cos(ks)))


@pytest.mark.parametrize("n,g", [(8, 0.5), (10, 1.0), (12, 1.7), (12, 0.0)])
def test_tfim_ring_free_fermion_energy(n, g):
    m = W.tfim_chain(n, 1.0, g)
    e0 = sla.eigsh(O.spin_gc_sparse(m), k=1, which="SA", tol=1e-13)[0][0]
    assert abs(e0 - tfim_ring_e0(n, 1.0, g)) < 1e-10


def test_tfim_limits():
    # g = 0: classical Ising ring, two-fold degenerate -n J
    ev = np.linalg.eigvalsh(O.spin_gc_sparse(W.tfim_chain(6, 1.0, 0.0)).toarray())
    assert abs(ev[0] + 6) < 1e-13 and abs(ev[1] + 6) < 1e-13 and ev[2] > -6 + 1
    # J = 0: free spins in the field, -n g
    ev = np.linalg.eigvalsh(O.spin_gc_sparse(W.tfim_chain(6, 0.0, 0.8)).toarray())
    assert abs(ev[0] + 6 * 0.8) < 1e-13


@pytest.mark.parametrize("n,lat,seed", [(8, "chain", 5), (10, "ladder", 6)])
def test_sz_conserving_case_is_the_union_of_sectors(n, lat, seed):
    # jx = jy (XXZ) and hx = 0: the full spectrum is the union of the S^z
    # sector spectra of the sector oracle
    sm = W.random_heisenberg(n, lat, seed)
    rng = np.random.default_rng(seed)
    hz = rng.normal(size=n)
    gc = W.spin_gc(n, np.stack([sm.bi, sm.bj], 1), sm.jxy, sm.jxy, sm.jz, 0.0, hz)
    full = np.sort(np.linalg.eigvalsh(O.spin_gc_sparse(gc).toarray()))
    sm.hz = hz
    secs = []
    for k in range(n + 1):
        s = O.basis_list(n, k)
        secs.append(np.linalg.eigvalsh(O.spin_sparse(sm, s).toarray()))
    assert np.allclose(full, np.sort(np.concatenate(secs)), atol=1e-11)


def test_row_matches_sparse():
    m = W.random_spin_gc(7, "chain", 9)
    Hs = O.spin_gc_sparse(m)
    for x in (0, 5, 77, 127):
        cols, vals = O.spin_gc_row(m, x)
        dense = np.zeros(1 << 7)
        np.add.at(dense, cols, vals)
        assert np.allclose(dense, Hs.getrow(x).toarray()[0], atol=1e-15)
