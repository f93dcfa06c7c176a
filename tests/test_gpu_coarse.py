"""GPU: the dense coarsest-level solve (blocked LU with partial pivoting and
the explicit inverse built from it) against its definition.

A single field whose size is at most coarse_max has a one-level hierarchy:
the preconditioner is the coarsest solve itself, so apply(r) must equal
A^-1 r (and the transposed apply A^-T r).  The reference is
numpy.linalg.solve.  Matrices are chosen to need row interchanges, to have
ties in the pivot search, to fill the blocked path's 2048-row limit and to
take the unblocked path above it; a singular matrix must be rejected.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_13079_amd as H
    H.load()  # must be built: no fallback
    return torch, torch.device("cuda:0")


def _sym_pattern(A):
    """A with explicit zeros added where only A^T has an entry (diagonal field
    blocks must be structurally symmetric)."""
    A = sp.coo_matrix(A)
    T = sp.coo_matrix((np.zeros(A.nnz), (A.col, A.row)), shape=A.shape)
    C = sp.coo_matrix((np.concatenate([A.data, T.data]), (np.concatenate([A.row, T.row]),
                                                          np.concatenate([A.col, T.col]))), shape=A.shape)
    return C.tocsr()  # duplicates are summed; explicit zeros are kept


def _one_field(A):
    A = _sym_pattern(A)
    A.sort_indices()
    n = A.shape[0]
    return synth.System(n=n, nf=1, rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32),
                        val=A.data.astype(np.float64), field_of_row=np.zeros(n, np.int32), tree=[-1, 0, -2])


def _pivoting(n, seed):
    """P (3 I + R) + 1e-3 I: small diagonal entries, every column needs an
    interchange; well conditioned."""
    rng = np.random.default_rng(seed)
    P = sp.csr_matrix((np.ones(n), (np.arange(n), rng.permutation(n))), shape=(n, n))
    R = sp.random(n, n, density=min(1.0, 6.0 / n), random_state=rng, format="csr")
    return (P @ (3.0 * sp.eye(n) + R) + 1e-3 * sp.eye(n)).tocsr()


def _ties(n, seed):
    """Entries of equal magnitude (+-1) with a 0.5 diagonal: the pivot search
    meets ties, broken by the first row."""
    rng = np.random.default_rng(seed)
    M = np.sign(rng.standard_normal((n, n))) * (rng.random((n, n)) < 0.05) + 0.5 * np.eye(n)
    return sp.csr_matrix(M)


CASES = {
    "n1": lambda: sp.csr_matrix(np.array([[2.5]])),
    "n17_pivoting": lambda: _pivoting(17, 1),
    "n640_ties": lambda: _ties(640, 2),
    "n1397_pivoting": lambda: _pivoting(1397, 3),
    "n2048_pivoting": lambda: _pivoting(2048, 4),
    "n2100_unblocked": lambda: _pivoting(2100, 5),
}


@pytest.mark.parametrize("case", list(CASES))
def test_coarsest_solve_is_exact_inverse(torch_dev, case):
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    A = CASES[case]()
    n = A.shape[0]
    s = _one_field(A)
    rp, ci, v, fl = (torch.from_numpy(a).to(dev) for a in (s.rowptr, s.col, s.val, s.field_of_row))
    g = H.Solver(rp, ci, v, fl, 1, s.tree, coarse_max=max(n, 16))
    g.set_precision(0)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(n)
    Ad = A.toarray()
    for tr in (False, True):
        z = g.apply(torch.from_numpy(r).to(dev), transpose=tr).cpu().numpy()
        ref = np.linalg.solve(Ad.T if tr else Ad, r)
        err = np.abs(z - ref).max() / np.abs(ref).max()
        assert err <= 1e-11, (case, tr, err)
    del g


def test_singular_coarsest_rejected(torch_dev):
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    n = 40
    M = np.eye(n)
    M[:2, :2] = 1.0  # rows 0 and 1 equal, diagonal present and nonzero
    s = _one_field(M)
    rp, ci, v, fl = (torch.from_numpy(a).to(dev) for a in (s.rowptr, s.col, s.val, s.field_of_row))
    with pytest.raises(H.HBGSError) as e:
        H.Solver(rp, ci, v, fl, 1, s.tree, coarse_max=n)
    assert e.value.code == -4


def test_singular_field_in_concurrent_setup(torch_dev):
    """Two uncoupled fields built by concurrent build threads, the second one
    singular: the worker's ESINGULAR reaches the caller, and a valid solver
    built afterwards on the same device works."""
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    n = 40
    good = sp.diags([-1.0, 2.5, -1.0], [-1, 0, 1], shape=(n, n)).toarray()
    bad = np.eye(n)
    bad[:2, :2] = 1.0
    M = np.zeros((2 * n, 2 * n))
    M[:n, :n] = good
    M[n:, n:] = bad
    A = sp.csr_matrix(M)
    A.sort_indices()
    fl = np.repeat(np.arange(2, dtype=np.int32), n)
    rp, ci, v, f = (torch.from_numpy(a).to(dev) for a in (A.indptr.astype(np.int32), A.indices.astype(np.int32),
                                                           A.data.astype(np.float64), fl))
    with pytest.raises(H.HBGSError) as e:
        H.Solver(rp, ci, v, f, 2, [-1, 0, 1, -2], coarse_max=64, setup_concurrent=1)
    assert e.value.code == -4
    s = _one_field(good)
    rp, ci, v, f = (torch.from_numpy(a).to(dev) for a in (s.rowptr, s.col, s.val, s.field_of_row))
    g = H.Solver(rp, ci, v, f, 1, s.tree, coarse_max=64)
    b = good @ np.ones(n)
    x, st, it, _ = g.solve(torch.from_numpy(b).to(dev))
    assert st == 0 and np.allclose(x.cpu().numpy(), 1.0, rtol=1e-8)
