"""Pins of the oracle's other leaf solvers against dense linear algebra:
the diagonal leaf (one Jacobi sweep, exact for a diagonal block such as the
solid-species block of Sec. 3.2) and DD(0)-ILU(0) (contiguous subdomains, no
overlap, incomplete LU with zero fill inside each).

ILU(0) facts used: the product of the factors reproduces the matrix on its
own pattern; with no fill possible (a tridiagonal block) it is the exact LU
factorisation; its transposed solve is the adjoint of the forward one.
"""
import numpy as np
import scipy.sparse as sp

import oracle
import synth

from test_oracle_pins import poisson1d


def _dense(s):
    return sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n)).toarray()


def _single_field(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64), n


def test_diagonal_leaf_is_exact_on_a_diagonal_block():
    s = synth.make_system(4, 4, 6, 1, seed=31)
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n)).tocoo()
    f = s.field_of_row
    keep = ~((f[A.row] == 3) & (f[A.col] == 3) & (A.row != A.col))  # the species block made diagonal
    B = sp.csr_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)
    B.sort_indices()
    o = oracle.Oracle(B.indptr, B.indices, B.data, s.nf, f, s.tree, block_jacobi=1, field_leaf=[0, 0, 0, 1])
    ref = oracle.Oracle(B.indptr, B.indices, B.data, s.nf, f, s.tree, block_jacobi=1)
    r = np.random.default_rng(0).standard_normal(s.n)
    z, zr = o.apply(r), ref.apply(r)
    m = f == 3
    d = B.diagonal()[m]
    assert np.allclose(z[m], r[m] / d, rtol=1e-15, atol=0)
    assert np.array_equal(z[~m], zr[~m])
    assert np.allclose(o.apply(r, transpose=True)[m], r[m] / d, rtol=1e-15, atol=0)


def _leaf_operator(o, n, transpose=False):
    """Dense M^-1 of a block-Jacobi preconditioner, column by column."""
    Z = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        Z[:, j] = o.apply(e, transpose=transpose)
    return Z


def test_ilu0_reproduces_the_matrix_on_its_pattern():
    s = synth.make_system(5, 4, 0, 1, seed=32)  # 2D, 80 rows
    A = _dense(s)
    sub = 7
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, block_jacobi=1,
                      field_leaf=[2, 2, 2, 2], ilu_block=sub)
    M = np.linalg.inv(_leaf_operator(o, s.n))  # = blockdiag over fields and subdomains of L U
    perm = o.permutation()  # original row -> permuted position
    f = s.field_of_row
    lo = {g: int(perm[f == g].min()) for g in range(s.nf)}
    same_sub = np.zeros((s.n, s.n), bool)
    for i in range(s.n):
        for j in range(s.n):
            if f[i] == f[j]:
                same_sub[i, j] = (perm[i] - lo[f[i]]) // sub == (perm[j] - lo[f[j]]) // sub
    pat = (A != 0) & same_sub
    scale = np.abs(A).max()
    assert np.abs(M[pat] - A[pat]).max() <= 1e-12 * scale
    assert np.abs(M[~same_sub]).max() <= 1e-12 * scale  # nothing couples subdomains or fields


def test_ilu0_is_exact_lu_without_fill():
    A = poisson1d(40) + sp.diags(np.linspace(0.1, 1.0, 40))
    rp, ci, v, n = _single_field(A)
    fld = np.zeros(n, np.int32)
    r = np.random.default_rng(1).standard_normal(n)
    o = oracle.Oracle(rp, ci, v, 1, fld, [-1, 0, -2], field_leaf=[2], ilu_block=n)
    Ad = A.toarray()
    assert np.linalg.norm(o.apply(r) - np.linalg.solve(Ad, r)) <= 1e-12 * np.linalg.norm(r) * 10
    assert np.linalg.norm(o.apply(r, transpose=True) - np.linalg.solve(Ad.T, r)) <= 1e-12 * np.linalg.norm(r) * 10
    # two subdomains: the coupling between the halves is dropped
    o2 = oracle.Oracle(rp, ci, v, 1, fld, [-1, 0, -2], field_leaf=[2], ilu_block=n // 2)
    h = n // 2
    ref = np.concatenate([np.linalg.solve(Ad[:h, :h], r[:h]), np.linalg.solve(Ad[h:, h:], r[h:])])
    assert np.linalg.norm(o2.apply(r) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_ilu0_transpose_is_the_adjoint():
    s = synth.make_system(5, 4, 6, 1, seed=33)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, block_jacobi=1,
                      field_leaf=[2, 2, 2, 2], ilu_block=16)
    rng = np.random.default_rng(2)
    u, w = rng.standard_normal(s.n), rng.standard_normal(s.n)
    Mw = o.apply(w)
    assert abs(u @ Mw - o.apply(u, transpose=True) @ w) <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(Mw) * 10


def test_species_ilu_leaf_in_the_sweep_converges():
    """The paper's choice for the species block (DD(0)-ILU(0)) inside the
    block Gauss-Seidel sweep, SA-AMG elsewhere."""
    s = synth.make_system(6, 6, 8, 1, seed=34)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, coarse_max=40, field_leaf=[0, 0, 0, 2],
                      ilu_block=64, rtol=1e-10)
    A = _dense(s)
    for tr in (False, True):
        b = s.b if not tr else s.x_t
        r = o.solve(b, transpose=tr)
        M = A.T if tr else A
        assert r["status"] == 0
        assert np.linalg.norm(b - M @ r["x"]) <= 1e-10 * np.linalg.norm(b)
