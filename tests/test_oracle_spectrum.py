"""CPU pins of the oracle's coupling matrix and its extreme eigenvalues
(the reference for the device Lanczos estimate, mars_spectrum): closed-form
spectra of ferromagnetic lattices, rings and complete graphs, gauge
invariance, and agreement of the matrix with the oracle's own energy."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05124_amd import inputs as I


def _ferro(L):
    return I.lattice_instance(L, 0, ferro=True)


@pytest.mark.parametrize("L", [(6, 4), (4, 6, 8), (8, 8)])
def test_ferro_lattice_spectrum_closed_form(L):
    """Periodic ferromagnet: J is the adjacency matrix of the torus, whose
    eigenvalues are sums over axes of 2 cos(2 pi k_a / L_a)."""
    grids = np.meshgrid(*[2 * np.cos(2 * np.pi * np.arange(n) / n) for n in L], indexing="ij")
    expect = np.sort(sum(grids).ravel())
    got = np.linalg.eigvalsh(O.coupling_matrix(_ferro(L)))
    assert np.allclose(got, expect, atol=1e-10)
    lo, hi = O.spectrum(_ferro(L))
    assert abs(hi - 2 * len(L)) < 1e-10 and abs(lo + 2 * len(L)) < 1e-10


def _csr(N, edges):
    """Undirected edges (i, j, w), each listed once."""
    ei = np.array([e[0] for e in edges], dtype=np.int64)
    ej = np.array([e[1] for e in edges], dtype=np.int64)
    w = np.array([e[2] for e in edges], dtype=np.int8)
    return I.csr_from_edges(N, ei, ej, w)


def test_ring_and_complete_graph_closed_form():
    n = 10
    ring = _csr(n, [(i, (i + 1) % n, 1) for i in range(n)])
    assert np.allclose(np.linalg.eigvalsh(O.coupling_matrix(ring)),
                       np.sort(2 * np.cos(2 * np.pi * np.arange(n) / n)), atol=1e-12)
    k = 7
    kn = _csr(k, [(i, j, -1) for i in range(k) for j in range(i + 1, k)])
    lo, hi = O.spectrum(kn)  # -(11^T - I): eigenvalues -(k - 1) once, +1 (k - 1 times)
    assert abs(lo + (k - 1)) < 1e-12 and abs(hi - 1) < 1e-12
    two = I.DenseInstance(J=np.array([[0.0, 0.75], [0.75, 0.0]], dtype=np.float32))
    assert O.spectrum(two) == (-0.75, 0.75)


def test_gauge_invariance():
    """J'_ij = xi_i xi_j J_ij is similar to J (diagonal sign matrix), so a
    gauge-transformed ferromagnet has the ferromagnet's spectrum."""
    L = (8, 6)
    f = _ferro(L)
    xi = np.where(np.random.default_rng(4).random(f.N) < 0.5, -1, 1)
    g = I.LatticeInstance(L=L, bond=f.bond.copy())
    for i in range(f.N):
        for a, st in enumerate([1, L[0]]):
            xa = (i // st) % L[a]
            j = i + (((xa + 1) % L[a]) - xa) * st
            g.bond[a, i] = xi[i] * xi[j]
    assert np.allclose(np.linalg.eigvalsh(O.coupling_matrix(g)), np.linalg.eigvalsh(O.coupling_matrix(f)),
                       atol=1e-10)


@pytest.mark.parametrize("kind", ["lattice2", "lattice3", "csr", "dense"])
def test_matrix_matches_oracle_energy(kind):
    """-s^T J s (eq. (2) with h = 0, J zero on the diagonal) from the matrix
    equals the C oracle's energy for random spins."""
    inst = {"lattice2": lambda: I.lattice_instance((6, 4), 3),
            "lattice3": lambda: I.lattice_instance((4, 4, 6), 5),
            "csr": lambda: I.er_instance(60, 2, p=0.1, weights="pm1"),
            "dense": lambda: I.sk_instance(40, 6)}[kind]()
    M = O.coupling_matrix(inst)
    assert np.all(np.diag(M) == 0) and np.array_equal(M, M.T)
    S = np.where(np.random.default_rng(1).random((5, inst.N)) < 0.5, -1, 1).astype(np.int8)
    E = O.energy(inst, S)
    for r in range(5):
        s = S[r].astype(np.float64)
        assert math.isclose(-(s @ M @ s), E[r], rel_tol=1e-12, abs_tol=1e-9)
