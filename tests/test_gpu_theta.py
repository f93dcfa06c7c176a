"""GPU parity for large strength thresholds (the paper's theta grid on the
solid-phase potential reaches 0.64): rows whose filtered matrix row is zero
keep their tentative prolongator row, and a coarsening that stops above the
8000-row dense limit ends in a smoothed coarsest level.  Hierarchies bitwise,
applies per field (FP64 1e-13, FP32 1e-5) in both directions, against the
oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from parity_util import assert_fields_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_13079_amd as H
    H.load()
    return torch, torch.device("cuda:0")


def _single_field(A):
    A = A.tocsr()
    A.sort_indices()
    n = A.shape[0]
    return synth.System(n=n, nf=1, rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32), val=A.data,
                        field_of_row=np.zeros(n, np.int32), tree=[-1, 0, -2])


def _poisson1d(n):
    return sp.diags([-np.ones(n - 1), np.full(n, 2.0), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def _compare(torch_dev, s, expect_smoothed, **opt):
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    args = (torch.from_numpy(s.rowptr).to(dev), torch.from_numpy(s.col).to(dev), torch.from_numpy(s.val).to(dev),
            torch.from_numpy(s.field_of_row).to(dev), s.nf, s.tree)
    g = H.Solver(*args, **opt)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, **opt)
    st = g.stats()
    for f in range(s.nf):
        oa = o.amg(f)
        assert oa.levels == st["levels"][f]
        if f in expect_smoothed:
            assert oa.smoothed_coarsest, f
        for l in range(oa.levels):
            for w in ("A", "AT") if l + 1 == oa.levels else ("A", "P", "R", "AT"):
                gr, gc, gv, _ = g.get_level(f, l, w)
                orp, oc, ov, _ = oa.get(l, w)
                assert np.array_equal(gr, orp) and np.array_equal(gc, oc), (f, l, w)
                assert np.array_equal(gv.view(np.int64), ov.view(np.int64)), (f, l, w)
            if l + 1 < oa.levels:
                assert np.array_equal(g.aggregates(f, l)[0], oa.agg(l))
            assert g.level_scalars(f, l) == oa.scalars(l), (f, l)
    r = np.random.default_rng(5).standard_normal(s.n)
    for precision in (0, 1):
        g.set_precision(precision)
        o.set_precision(precision)
        for tr in (False, True):
            z = g.apply(torch.from_numpy(r).to(dev), transpose=tr).cpu().numpy()
            zo = o.apply(r, transpose=tr)
            assert_fields_close(z, zo, s.field_of_row, 1e-13 if precision == 0 else 1e-5, (precision, tr))
    return g, o


def test_fully_weak_level_is_one_smoothed_level(torch_dev):
    """1D Poisson of 9000 rows at theta = 0.64: every connection is weak,
    the coarsening stalls at the finest level above the dense limit, and the
    hierarchy is one smoothed level."""
    s = _single_field(_poisson1d(9000))
    g, _ = _compare(torch_dev, s, {0}, theta=[0.64])
    assert g.stats()["levels"] == [1]


def test_level_cap_above_dense_limit(torch_dev):
    """1D Poisson of 30000 rows with two levels at most: the ~10000-row second
    level is smoothed, not solved."""
    s = _single_field(_poisson1d(30000))
    g, _ = _compare(torch_dev, s, {0}, theta=[0.0], max_levels=2)
    assert g.stats()["levels"] == [2]


@pytest.mark.parametrize("theta", [0.16, 0.64])
def test_theta_grid_upper_points_1m(torch_dev, theta):
    """The 1M-DOF system with theta_phi_s = 0.16 and 0.64: the phi_s
    hierarchy (zero filtered rows, stalled coarsening) equals the oracle's,
    the whole apply matches, and the solve converges to 1e-8."""
    torch, dev = torch_dev
    s = synth.make_system(cfg=1)
    g, o = _compare(torch_dev, s, {0}, theta=[theta])
    g.set_precision(1)
    x, st, it, _ = g.solve(torch.from_numpy(s.b).to(dev))
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    res = np.linalg.norm(s.b - A @ x.cpu().numpy()) / np.linalg.norm(s.b)
    print(f"theta {theta}: levels {g.stats()['levels']}, {it} iterations, true residual {res:.2e}")
    assert st == 0 and res <= 1e-8
