"""GPU parity of the preconditioner variants against the CPU oracle, through
the C ABI: block Jacobi (couplings dropped), per-field Chebyshev degree,
the other leaf solvers (diagonal / DD(0)-ILU(0)), and the nested form of
Sec. 3.2 (an inner flexible GMRES per child of the outermost group,
preconditioned by that child's sweep).

Bars: block Jacobi, per-field degree and the leaves as the single sweep (FP64 apply
<= 1e-13, FP32 V-cycle <= 1e-5, same iteration counts within 2).  The
nested preconditioner is not a fixed linear operator once the inner solve
stops on a tolerance, so its parity is taken with the inner and outer step
counts locked (rtol = 0): then both sides apply the same operator and x
agrees to 1e-9; with the paper's settings (inner GMRES(30) to 1e-6, outer
restart 5) iteration counts agree within 1 and the true residual meets the
tolerance.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from parity_util import assert_fields_close
import synth

pytestmark = pytest.mark.gpu

TREE4 = [-1, -1, 0, 1, -2, -1, 2, 3, -2, -2]  # ((phi_s, phi_e), (p, c))
TREE6 = [-1, -1, 0, 1, -2, -1, 2, 3, 4, 5, -2, -2]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_13079_amd as H
    H.load()
    return torch, torch.device("cuda:0")


CASES = {
    "cfg0_cm64": dict(sys=dict(cfg=0), coarse_max=64),
    "ragged7x5x9_6f_cm40": dict(sys=dict(nx=7, ny=5, nz=9, nspecies=3, seed=11), coarse_max=40),
}


def _system(case):
    return synth.make_system(**CASES[case]["sys"])


def _pair(torch_dev, case, tree=None, **opt):
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    s = _system(case)
    tree = s.tree if tree is None else tree
    cm = CASES[case]["coarse_max"]
    g = H.Solver(torch.from_numpy(s.rowptr).to(dev), torch.from_numpy(s.col).to(dev),
                 torch.from_numpy(s.val).to(dev), torch.from_numpy(s.field_of_row).to(dev), s.nf, tree,
                 coarse_max=cm, **opt)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, tree, coarse_max=cm, **opt)
    return s, g, o


def _res(s, x, b, tr=False):
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    if tr:
        A = A.T.tocsr()
    return np.linalg.norm(b - A @ x) / np.linalg.norm(b)


def _tree(s):
    return TREE4 if s.nf == 4 else TREE6


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_block_jacobi(torch_dev, case, precision):
    torch, dev = torch_dev
    s, g, o = _pair(torch_dev, case, block_jacobi=1, precision=precision)
    r = np.random.default_rng(5).standard_normal(s.n)
    tol = 1e-13 if precision == 0 else 1e-5
    for tr in (False, True):
        z = g.apply(torch.from_numpy(r).to(dev), transpose=tr).cpu().numpy()
        zo = o.apply(r, transpose=tr)
        assert_fields_close(z, zo, s.field_of_row, tol, tr)
    x, st, it, _ = g.solve(torch.from_numpy(s.b).to(dev))
    ro = o.solve(s.b)
    assert st == 0 and ro["status"] == 0 and abs(it - ro["iters"]) <= 2
    assert _res(s, x.cpu().numpy(), s.b) <= 1e-8


@pytest.mark.parametrize("precision", [0, 1])
def test_field_chebyshev_degree(torch_dev, precision):
    torch, dev = torch_dev
    s, g, o = _pair(torch_dev, "ragged7x5x9_6f_cm40", field_cheb_degree=[4, 4], precision=precision)
    r = np.random.default_rng(6).standard_normal(s.n)
    tol = 1e-13 if precision == 0 else 1e-5
    for tr in (False, True):
        z = g.apply(torch.from_numpy(r).to(dev), transpose=tr).cpu().numpy()
        zo = o.apply(r, transpose=tr)
        assert_fields_close(z, zo, s.field_of_row, tol, tr)


@pytest.mark.parametrize("case", list(CASES))
def test_nested_locked_steps(torch_dev, case):
    """Inner and outer step counts fixed (rtol = 0): the nested operator is
    then the same on both sides, in both directions."""
    torch, dev = torch_dev
    s = _system(case)
    opt = dict(nested=1, inner_rtol=0.0, inner_max_iters=3, inner_restart=3, rtol=0.0, max_iters=4, restart=5)
    s, g, o = _pair(torch_dev, case, tree=_tree(s), **opt)
    r = np.random.default_rng(8).standard_normal(s.n)
    for tr in (False, True):
        z = g.apply(torch.from_numpy(r).to(dev), transpose=tr).cpu().numpy()
        zo = o.apply(r, transpose=tr)
        assert_fields_close(z, zo, s.field_of_row, 1e-10, tr)
        b = s.b if not tr else s.x_t
        x, st, it, _ = g.solve(torch.from_numpy(b).to(dev), transpose=tr)
        ro = o.solve(b, transpose=tr)
        assert st == 1 and ro["status"] == 1 and it == ro["iters"] == 4
        assert np.linalg.norm(x.cpu().numpy() - ro["x"]) <= 1e-9 * np.linalg.norm(ro["x"]), tr


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_nested_paper_settings(torch_dev, case, precision):
    """Outer flexible GMRES(5), inner GMRES(30) to 1e-6: a few outer steps,
    as many as the oracle's within 1, forward and adjoint."""
    torch, dev = torch_dev
    s = _system(case)
    s, g, o = _pair(torch_dev, case, tree=_tree(s), nested=1, restart=5, precision=precision)
    for tr in (False, True):
        b = s.b if not tr else s.x_t
        x, st, it, _ = g.solve(torch.from_numpy(b).to(dev), transpose=tr)
        ro = o.solve(b, transpose=tr)
        assert st == 0 and ro["status"] == 0
        assert abs(it - ro["iters"]) <= 1, (it, ro["iters"])
        assert it <= 6
        assert _res(s, x.cpu().numpy(), b, tr) <= 1e-8


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("leaf", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_leaf_solvers(torch_dev, case, leaf, precision):
    """Diagonal (Jacobi) and DD(0)-ILU(0) leaves on the species block(s),
    SA-AMG elsewhere: apply parity in both directions, and the solve."""
    torch, dev = torch_dev
    s = _system(case)
    leaves = [0, 0, 0] + [leaf] * (s.nf - 3)
    s, g, o = _pair(torch_dev, case, field_leaf=leaves, ilu_block=48, precision=precision)
    r = np.random.default_rng(9).standard_normal(s.n)
    tol = 1e-13 if precision == 0 else 1e-5
    for tr in (False, True):
        z = g.apply(torch.from_numpy(r).to(dev), transpose=tr).cpu().numpy()
        zo = o.apply(r, transpose=tr)
        assert_fields_close(z, zo, s.field_of_row, tol, tr)
    x, st, it, _ = g.solve(torch.from_numpy(s.b).to(dev))
    ro = o.solve(s.b)
    assert st == 0 and ro["status"] == 0 and abs(it - ro["iters"]) <= 2
    assert _res(s, x.cpu().numpy(), s.b) <= 1e-8


@pytest.mark.parametrize("case", list(CASES))
def test_nested_deferred_transpose(torch_dev, case):
    """The nested form with the adjoint's operators deferred
    (build_transpose = 0): transposed applies equal the eager build's."""
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    s = _system(case)
    cm = CASES[case]["coarse_max"]
    opt = dict(nested=1, inner_rtol=0.0, inner_max_iters=3, inner_restart=3, coarse_max=cm)
    args = (torch.from_numpy(s.rowptr).to(dev), torch.from_numpy(s.col).to(dev), torch.from_numpy(s.val).to(dev),
            torch.from_numpy(s.field_of_row).to(dev), s.nf, _tree(s))
    ge = H.Solver(*args, **opt)
    gl = H.Solver(*args, build_transpose=0, **opt)
    r = torch.from_numpy(np.random.default_rng(14).standard_normal(s.n)).to(dev)
    assert torch.equal(ge.apply(r), gl.apply(r))
    assert torch.equal(ge.apply(r, transpose=True), gl.apply(r, transpose=True))
