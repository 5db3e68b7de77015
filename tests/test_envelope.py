"""The sparsity fact the envelope-aware factorisation rests on, pinned on the
CPU with the oracle's element matrices.

A Cholesky factor has no nonzero left of the first nonzero of its row in the
matrix (the envelope of a symmetric positive definite matrix is kept by its
factor).  The batched factorisation skips every 64x64 factor tile left of
its tile row's first nonzero tile and every product with such a tile; this
checks, on the local stiffness of a hexahedral box in interior-first order,
that those entries of an ordinary dense Cholesky factor are exactly zero,
and that the interior block of that order is banded.
"""
import numpy as np

from oracle import fem
from workloads import cube_mesh

TS = 64


def _local_stiffness(n_el):
    """Assembled stiffness of one floating box of n_el^3 Q1 elements, its DOFs
    ordered interior nodes first, then boundary nodes (each set in node
    order, three DOFs per node), plus the number of interior DOFs."""
    mesh = cube_mesh(n_el, 1)
    Ke, _ = fem.element_matrices(mesh)
    n = mesh.xyz.shape[0]
    K = np.zeros((3 * n, 3 * n))
    for e in range(mesh.n_elems):
        d = (3 * mesh.hex8[e][:, None] + np.arange(3)[None, :]).ravel()
        K[np.ix_(d, d)] += Ke[e]
    on_boundary = np.any((mesh.xyz < 1e-12) | (mesh.xyz > 1.0 - 1e-12), axis=1)
    nodes = np.concatenate([np.flatnonzero(~on_boundary), np.flatnonzero(on_boundary)])
    perm = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
    return K[np.ix_(perm, perm)], 3 * int((~on_boundary).sum())


def _first_nonzero(A):
    return np.array([np.flatnonzero(A[r, : r + 1])[0] for r in range(A.shape[0])])


def test_cholesky_keeps_the_envelope():
    K, n_ii = _local_stiffness(8)   # 729 nodes, 2187 DOFs, as a cube32_s4 subdomain
    A = K + np.eye(K.shape[0])      # positive definite, same envelope (the box floats)
    fnz = _first_nonzero(A)
    L = np.linalg.cholesky(A)
    for r in range(A.shape[0]):
        assert np.all(L[r, : fnz[r]] == 0.0), r
    # the tile form used by the schedule: factor tiles left of the tile row's
    # first nonzero tile are zero
    nt = -(-A.shape[0] // TS)
    for I in range(nt):
        rows = slice(I * TS, min((I + 1) * TS, A.shape[0]))
        first_tile = fnz[rows].min() // TS
        assert np.all(L[rows, : first_tile * TS] == 0.0), I
    # interior rows reach back at most one node layer and a node row of the
    # 7 x 7 interior cross-section: a band of 3 (7 * 7 + 7 + 1) DOFs
    band = (np.arange(n_ii) - fnz[:n_ii]).max()
    assert band <= 3 * (7 * 7 + 7 + 1) + 2, band


def test_envelope_skips_most_interior_products():
    """Share of the interior and Schur tile products of a dense left-looking
    tile Cholesky that involve a factor tile left of the envelope (the work
    the schedule drops) on the 8^3-element box."""
    K, n_ii = _local_stiffness(8)
    fnz = _first_nonzero(K + np.eye(K.shape[0]))
    nti = -(-n_ii // TS)
    nt = nti + -(-(K.shape[0] - n_ii) // TS)

    def tile_rows(I):
        return range(I * TS, min((I + 1) * TS, n_ii)) if I < nti else \
            range(n_ii + (I - nti) * TS, min(n_ii + (I - nti + 1) * TS, K.shape[0]))

    E = [min(fnz[r] for r in tile_rows(I)) // TS for I in range(nt)]
    dense = kept = 0
    for j in range(nti):                      # interior column steps, rows below
        for i in range(j, nt):
            dense += j
            if E[i] <= j:
                kept += max(0, j - max(E[i], E[j]))
    for J in range(nti, nt):                  # Schur update of the interface block
        for I in range(J, nt):
            dense += nti
            kept += max(0, nti - max(E[I], E[J]))
    assert kept < 0.5 * dense, (kept, dense)
