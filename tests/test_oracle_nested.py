"""Pins of the oracle's block-Jacobi, nested (inner flexible GMRES per
outermost group) and per-field Chebyshev-degree modes against dense linear
algebra and closed forms.

Nested form (Sec. 3.2): the children of the outermost group are visited as in
the block Gauss-Seidel sweep, and each child's block is inverted by an inner
GMRES preconditioned by the child's own sweep.  With exact leaf solves and a
converged inner solve this is the block lower-triangular solve over the
groups; one inner step is the one-dimensional minimal-residual correction.
"""
import numpy as np
import scipy.sparse as sp

import oracle
import synth

TREE4 = [-1, -1, 0, 1, -2, -1, 2, 3, -2, -2]  # ((phi_s, phi_e), (p, c))
TREE6 = [-1, -1, 0, 1, -2, -1, 2, 3, 4, 5, -2, -2]


def _dense(s):
    return sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n)).toarray()


def _groups(s, tree):
    """Rows (original ordering) of each child of the root, and each field's rows."""
    f = s.field_of_row
    groups, cur, depth = [], None, 0
    for code in tree:
        if code == -1:
            depth += 1
            if depth == 2:
                cur = []
        elif code == -2:
            if depth == 2:
                groups.append(cur)
            depth -= 1
        elif depth == 1:
            groups.append([code])
        else:
            cur.append(code)
    return [np.flatnonzero(np.isin(f, g)) for g in groups], groups


def _within_group_lower(A, s, rows, fields):
    """Block lower-triangular part (in field order) of a group's diagonal block."""
    f = s.field_of_row[rows]
    pos = {fld: q for q, fld in enumerate(fields)}
    p = np.array([pos[x] for x in f])
    B = A[np.ix_(rows, rows)]
    return B * (p[:, None] >= p[None, :])


def test_block_jacobi_exact_leaves_is_block_diagonal_solve():
    s = synth.make_system(4, 4, 6, 1, seed=21)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, exact_leaves=1, block_jacobi=1)
    A = _dense(s)
    r = np.random.default_rng(0).standard_normal(s.n)
    for tr in (False, True):
        z = o.apply(r, transpose=tr)
        for f in range(s.nf):
            m = s.field_of_row == f
            B = A[np.ix_(m, m)]
            ref = np.linalg.solve(B.T if tr else B, r[m])
            assert np.linalg.norm(z[m] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_nested_exact_equals_group_block_triangular_solve():
    s = synth.make_system(4, 4, 6, 3, seed=22)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, TREE6, exact_leaves=1, nested=1,
                      inner_rtol=1e-14, inner_max_iters=200)
    A = _dense(s)
    (g1, g2), _ = _groups(s, TREE6)
    r = np.random.default_rng(1).standard_normal(s.n)
    # forward: groups in order, lower coupling
    z = o.apply(r)
    z1 = np.linalg.solve(A[np.ix_(g1, g1)], r[g1])
    z2 = np.linalg.solve(A[np.ix_(g2, g2)], r[g2] - A[np.ix_(g2, g1)] @ z1)
    assert np.linalg.norm(z[g1] - z1) <= 1e-10 * np.linalg.norm(z1)
    assert np.linalg.norm(z[g2] - z2) <= 1e-10 * np.linalg.norm(z2)
    # transpose: groups in reverse order with the couplings of A^T
    zt = o.apply(r, transpose=True)
    At = A.T
    y2 = np.linalg.solve(At[np.ix_(g2, g2)], r[g2])
    y1 = np.linalg.solve(At[np.ix_(g1, g1)], r[g1] - At[np.ix_(g1, g2)] @ y2)
    assert np.linalg.norm(zt[g2] - y2) <= 1e-10 * np.linalg.norm(y2)
    assert np.linalg.norm(zt[g1] - y1) <= 1e-10 * np.linalg.norm(y1)


def test_nested_exact_outer_converges_in_one_step():
    """Group-level block lower-triangular A: the nested preconditioner with
    exact inner solves is A^-1, so the outer GMRES stops after one step."""
    s = synth.make_system(4, 4, 6, 1, seed=23)
    (g1, g2), _ = _groups(s, TREE4)
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n)).tocoo()
    in1 = np.zeros(s.n, bool)
    in1[g1] = True
    keep = ~(in1[A.row] & ~in1[A.col])  # drop rows of group 1 x columns of group 2
    L = sp.csr_matrix((A.data[keep], (A.row[keep], A.col[keep])), shape=A.shape)
    L.sort_indices()
    o = oracle.Oracle(L.indptr, L.indices, L.data, s.nf, s.field_of_row, TREE4, exact_leaves=1, nested=1,
                      inner_rtol=1e-14, inner_max_iters=200, rtol=1e-10)
    b = L @ s.x_star
    r = o.solve(b)
    assert r["status"] == 0 and r["iters"] == 1
    assert np.linalg.norm(r["x"] - s.x_star) <= 1e-8 * np.linalg.norm(s.x_star)


def test_nested_one_inner_step_is_minimal_residual_correction():
    """One inner step from zero: y = alpha s with s = M_G t (the group's
    sweep) and alpha = (t . A_GG s) / ||A_GG s||^2."""
    s = synth.make_system(4, 4, 6, 1, seed=24)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, TREE4, exact_leaves=1, nested=1,
                      inner_rtol=0.0, inner_max_iters=1, inner_restart=1)
    A = _dense(s)
    (g1, g2), (f1, f2) = _groups(s, TREE4)
    r = np.random.default_rng(3).standard_normal(s.n)
    z = o.apply(r)
    t = r[g1]
    s1 = np.linalg.solve(_within_group_lower(A, s, g1, f1), t)
    As = A[np.ix_(g1, g1)] @ s1
    z1 = (t @ As) / (As @ As) * s1
    t2 = r[g2] - A[np.ix_(g2, g1)] @ z[g1]
    s2 = np.linalg.solve(_within_group_lower(A, s, g2, f2), t2)
    As2 = A[np.ix_(g2, g2)] @ s2
    z2 = (t2 @ As2) / (As2 @ As2) * s2
    assert np.linalg.norm(z[g1] - z1) <= 1e-12 * np.linalg.norm(z1)
    assert np.linalg.norm(z[g2] - z2) <= 1e-12 * np.linalg.norm(z2)


def test_nested_amg_converges_and_duality():
    """With V-cycle leaves and the paper's inner settings, the outer solve
    converges in far fewer steps than the single sweep; the nested operator
    is not linear, so only the forward/adjoint solves are checked."""
    s = synth.make_system(6, 6, 8, 1, seed=25)
    flat = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, TREE4, coarse_max=40, rtol=1e-10)
    nest = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, TREE4, coarse_max=40, rtol=1e-10,
                         nested=1, restart=5)
    A = _dense(s)
    a, b = flat.solve(s.b), nest.solve(s.b)
    assert a["status"] == 0 and b["status"] == 0
    assert b["iters"] < a["iters"]
    for r in (a, b):
        assert np.linalg.norm(s.b - A @ r["x"]) <= 1e-10 * np.linalg.norm(s.b)
    bt = nest.solve(s.x_t, transpose=True)
    assert bt["status"] == 0
    assert np.linalg.norm(s.x_t - A.T @ bt["x"]) <= 1e-10 * np.linalg.norm(s.x_t)


def test_field_chebyshev_degree():
    """A per-field degree changes only that field's V-cycle: with the
    couplings dropped, field 0's result equals a standalone hierarchy of its
    block smoothed with that degree."""
    s = synth.make_system(6, 6, 8, 1, seed=26)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, coarse_max=40, block_jacobi=1,
                      field_cheb_degree=[4])
    o2 = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, coarse_max=40, block_jacobi=1)
    r = np.random.default_rng(4).standard_normal(s.n)
    z, z2 = o.apply(r), o2.apply(r)
    m0 = s.field_of_row == 0
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    B = A[m0][:, m0].tocsr()
    B.sort_indices()
    h = oracle.Amg(B.indptr, B.indices, B.data, theta=0.04, salt=oracle.field_salt_base(0x2602, 0),
                   opts=oracle.options(coarse_max=40, cheb_degree=4))
    assert np.array_equal(z[m0], h.vcycle(r[m0]))
    assert np.array_equal(z[~m0], z2[~m0])
    assert not np.array_equal(z[m0], z2[m0])
