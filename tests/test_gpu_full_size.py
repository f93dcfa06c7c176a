"""GPU parity at the full workload sizes, through the C ABI, against the
oracle on the same seeded systems:

  * 4.2M DOF (4 fields, the benchmark's system), 5.3M DOF (6 fields, the
    differentiation system) and 50.3M DOF (6 fields, the largest one-GPU
    system): every field's whole hierarchy -- aggregates, A_l, P_l, R_l and
    A_l^T with their FP64 values, and the eigenvalue scalars -- equals the
    oracle's bitwise;
  * the whole-system preconditioner apply, forward and transposed, FP64 to
    1e-13 and the FP32 sweep to 1e-5 relative in every field;
  * 4.2M and 5.3M: iteration-locked solves (rtol = 0, 12 steps) give the
    oracle's x, and free solves reach a true residual of 1e-8 forward and
    adjoint;
  * 5.3M: the j0 gradient against finite differences and the tangent
    identity; 50.3M: a value update followed by forward and adjoint mixed
    solves.

Each section keeps one device solver and one oracle alive and drops them
before the next, larger system.
"""
import gc

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


_big = {}


def _workload(torch_dev, cfg):
    """(system, device solver, oracle) of config `cfg`, built once; the
    previous workload is dropped first."""
    if _big.get("cfg") != cfg:
        torch, dev = torch_dev
        import paper_2602_13079_amd as H
        _big.clear()
        gc.collect()
        torch.cuda.empty_cache()
        print(f"building the {cfg} workload (generator, device setup, oracle setup)", flush=True)
        s = synth.make_system(cfg=cfg, with_dj0=(cfg == 3))
        rp, ci, v, fl = (torch.from_numpy(a).to(dev) for a in (s.rowptr, s.col, s.val, s.field_of_row))
        g = H.Solver(rp, ci, v, fl, s.nf, s.tree)
        oracle.set_verbose(True)
        try:
            o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree)
        finally:
            oracle.set_verbose(False)
        _big.update(cfg=cfg, s=s, g=g, o=o, dev_csr=(rp, ci, v, fl))
        print(f"  {s.n} DOF, {s.nnz} nonzeros, levels {g.stats()['levels']}", flush=True)
    return _big["s"], _big["g"], _big["o"]


def _true_res(s, x, b, transpose=False):
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    if transpose:
        A = A.T.tocsr()
    return np.linalg.norm(b - A @ x) / np.linalg.norm(b)


def _check_field_hierarchy(g, o, f):
    oa = o.amg(f)
    assert oa.levels == g.stats()["levels"][f]
    for l in range(oa.levels):
        coarsest = l + 1 == oa.levels
        for w in (("A", "AT") if coarsest else ("A", "P", "R", "AT")):
            gr, gc_, gv, gn = g.get_level(f, l, w)
            orp, oc, ov, on = oa.get(l, w)
            assert gn == on, (f, l, w)
            assert np.array_equal(gr, orp), (f, l, w)
            assert np.array_equal(gc_, oc), (f, l, w)
            assert np.array_equal(gv.view(np.int64), ov.view(np.int64)), (f, l, w, np.abs(gv - ov).max())
        if not coarsest:
            agg, sc = g.aggregates(f, l)
            assert np.array_equal(agg, oa.agg(l)), (f, l)
            assert sc == oa.scalars(l), (f, l)
    return oa.levels


def _check_apply(torch_dev, s, g, o, precision, seed):
    torch, dev = torch_dev
    g.set_precision(precision)
    o.set_precision(precision)
    r = np.random.default_rng(seed).standard_normal(s.n)
    tol = 1e-13 if precision == 0 else 1e-5
    try:
        for tr in (False, True):
            z = g.apply(torch.from_numpy(r).to(dev), transpose=tr).cpu().numpy()
            zo = o.apply(r, transpose=tr)
            err = assert_fields_close(z, zo, s.field_of_row, tol, tr)
            print(f"apply precision {precision} transpose {tr}: per-field relative differences "
                  f"{[f'{e:.1e}' for e in err]}", flush=True)
    finally:
        g.set_precision(0)
        o.set_precision(0)


def _check_locked(torch_dev, s, g, precision, k=12):
    """rtol = 0: both sides take exactly k Arnoldi steps (FP64 x to 1e-12;
    mixed: both run FP32 sweeps whose sums are ordered differently, each
    apply within 1e-5 of the other, x to 1e-5)."""
    torch, dev = torch_dev
    g.set_precision(precision)
    g.set_tolerance(0.0, k)
    try:
        x, st, it, _ = g.solve(torch.from_numpy(s.b).to(dev))
    finally:
        g.set_tolerance(1e-8, 2000)
        g.set_precision(0)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, rtol=0.0, max_iters=k,
                      precision=precision)
    ro = o.solve(s.b)
    del o
    assert st == 1 and ro["status"] == 1 and it == ro["iters"] == k
    x = x.cpu().numpy()
    rel = np.linalg.norm(x - ro["x"]) / np.linalg.norm(ro["x"])
    print(f"locked solve precision {precision}: x relative difference {rel:.2e}", flush=True)
    assert rel <= (1e-12 if precision == 0 else 1e-5)


def _check_solve(torch_dev, s, g, precision):
    torch, dev = torch_dev
    g.set_precision(precision)
    try:
        x, st, it, _ = g.solve(torch.from_numpy(s.b).to(dev))
        assert st == 0 and 5 <= it <= 60
        res = _true_res(s, x.cpu().numpy(), s.b)
        lam, st2, it2, _ = g.solve(torch.from_numpy(s.x_t).to(dev), transpose=True)
        res2 = _true_res(s, lam.cpu().numpy(), s.x_t, transpose=True)
    finally:
        g.set_precision(0)
    print(f"solve precision {precision}: {it} steps, true residual {res:.2e}; adjoint {it2} steps, {res2:.2e}")
    assert res <= 1e-8
    assert st2 == 0 and res2 <= 1e-8


# ------------------------------------------------------------ 4.2M DOF (cfg 2)
@pytest.mark.parametrize("field", [0, 1, 2, 3])
def test_full_size_hierarchy_cfg2(torch_dev, field):
    s, g, o = _workload(torch_dev, 2)
    _check_field_hierarchy(g, o, field)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_apply_cfg2(torch_dev, precision):
    s, g, o = _workload(torch_dev, 2)
    _check_apply(torch_dev, s, g, o, precision, seed=11)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_solve_locked_cfg2(torch_dev, precision):
    s, g, o = _workload(torch_dev, 2)
    _check_locked(torch_dev, s, g, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_solve_cfg2(torch_dev, precision):
    """The benchmark's configuration: true residual (recomputed on the host
    in FP64) at 1e-8 for the forward and the adjoint system."""
    s, g, o = _workload(torch_dev, 2)
    _check_solve(torch_dev, s, g, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_operand_tiles_bitwise_cfg2(torch_dev, precision):
    """The benchmark's configuration: its finest and first coarse levels and
    its outer operator take the SpMV with the operand staged in LDS; the
    gathering form must give the same bits (the apply in both directions,
    an 8-step locked solve)."""
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    s, g, o = _workload(torch_dev, 2)
    r = torch.from_numpy(np.random.default_rng(12).standard_normal(s.n)).to(dev)
    b = torch.from_numpy(s.b).to(dev)
    g.set_precision(precision)
    g.set_tolerance(0.0, 8)
    out = {}
    try:
        for on in (True, False):
            H.debug_spmv_tiles(on)
            z = [g.apply(r, transpose=tr).cpu().numpy() for tr in (False, True)]
            x, st, it, hist = g.solve(b)
            out[on] = (z, x.cpu().numpy(), np.asarray(hist), it)
    finally:
        H.debug_spmv_tiles(True)
        g.set_tolerance(1e-8, 2000)
        g.set_precision(0)
    (za, xa, ha, ia), (zb, xb, hb, ib) = out[True], out[False]
    for tr in (0, 1):
        assert np.array_equal(za[tr].view(np.int64), zb[tr].view(np.int64)), tr
    assert ia == ib == 8
    assert np.array_equal(xa.view(np.int64), xb.view(np.int64))
    assert np.array_equal(ha.view(np.int64), hb.view(np.int64))


# ------------------------------------------------------------ 5.3M DOF (cfg 3)
@pytest.mark.parametrize("field", [0, 1, 2, 3, 4, 5])
def test_full_size_hierarchy_cfg3(torch_dev, field):
    s, g, o = _workload(torch_dev, 3)
    _check_field_hierarchy(g, o, field)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_apply_cfg3(torch_dev, precision):
    s, g, o = _workload(torch_dev, 3)
    _check_apply(torch_dev, s, g, o, precision, seed=13)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_solve_locked_cfg3(torch_dev, precision):
    s, g, o = _workload(torch_dev, 3)
    _check_locked(torch_dev, s, g, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_solve_cfg3(torch_dev, precision):
    s, g, o = _workload(torch_dev, 3)
    _check_solve(torch_dev, s, g, precision)


def test_config3_j0_gradient_fd(torch_dev):
    """5.3M-DOF 6-field system: dL/dj0 for L = 0.5 ||x - x_t||^2 from the
    mixed-precision forward and adjoint solves (CSR-value gradient mapped to
    per-cell j0) against
      * central finite differences, h = 1e-6 j0, in FP64 on 8 seeded
        electrode cells (to 1e-3); the perturbed solutions are written x0 + dx with
        A(j0 +- h) dx = (b - A x0) -+ h (dA/dj0) x0, so the difference of the
        two losses is formed without cancellation;
      * the tangent identity dL/dj0 = g^T dx with A dx = -(dA/dj0) x (FP64,
        to 1e-6).
    The perturbed systems are solved with the base preconditioner."""
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    s, _, _ = _workload(torch_dev, 3)
    rtol = 1e-10
    rp, ci, v, fl = _big["dev_csr"]
    g = H.Solver(rp, ci, v, fl, s.nf, s.tree, rtol=rtol, precision=1)
    val = torch.from_numpy(s.val).to(dev)
    b = torch.from_numpy(s.b).to(dev)
    xt = torch.from_numpy(s.x_t).to(dev)
    x, st, it, _ = g.solve(b)
    assert st == 0
    lam, st, it2, _ = g.solve(x - xt, transpose=True)
    assert st == 0
    gv = g.grad_values(lam, x)
    dcell = torch.from_numpy(s.dcell.astype(np.int64)).to(dev)
    dcoef = torch.from_numpy(s.dcoef).to(dev)
    m = dcell >= 0
    gj = torch.zeros(len(s.j0), dtype=torch.float64, device=dev).index_add_(0, dcell[m], gv[m] * dcoef[m])
    gj = gj.cpu().numpy()
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    x0 = x.cpu().numpy()
    r0 = s.b - A @ x0
    row = np.repeat(np.arange(s.n), np.diff(s.rowptr))
    g.set_precision(0)
    # the correction systems have right-hand sides ~h smaller than b; 1e-8 of
    # their own norm is the attainable target for cond(A) ~1e7 in FP64
    g.set_tolerance(1e-8, 400)
    errs = []
    for c in synth.fd_cells(s.seed, s.layer, 8):
        sel = s.dcell == c
        dAx = np.zeros(s.n)
        np.add.at(dAx, row[sel], s.dcoef[sel] * x0[s.col[sel]])
        h = 1e-6 * s.j0[c]
        dxs = []
        for sign in (1.0, -1.0):
            vv = s.val.copy()
            vv[sel] += sign * h * s.dcoef[sel]
            g.set_values(torch.from_numpy(vv).to(dev), rebuild=False)
            dx, st, _, _ = g.solve(torch.from_numpy(r0 - sign * h * dAx).to(dev))
            assert st == 0
            dxs.append(dx.cpu().numpy())
        dL = np.sum((dxs[0] - dxs[1]) * (x0 - s.x_t + 0.5 * (dxs[0] + dxs[1])))
        fd = dL / (2 * h)
        g.set_values(val, rebuild=False)
        g.set_tolerance(rtol, 2000)
        dx_t, st, _, _ = g.solve(torch.from_numpy(-dAx).to(dev))
        g.set_tolerance(1e-8, 400)
        tangent = float(np.dot(x0 - s.x_t, dx_t.cpu().numpy()))
        errs.append(abs(gj[c] - fd) / abs(fd))
        print(f"cell {c}: grad {gj[c]:.10e} fd {fd:.10e} tangent {tangent:.10e}")
        # FD: each perturbed pair is solved to 1e-8 of an h-sized right-hand
        # side (the FP64 floor is eps * cond(A) ~ 2e-9 here), which leaves up to
        # ~1e-3 relative noise in the difference; the tangent identity has no
        # such cancellation and pins the gradient to 1e-6.
        assert gj[c] == pytest.approx(fd, rel=1e-3), (c, gj[c], fd)
        assert gj[c] == pytest.approx(tangent, rel=1e-6), (c, gj[c], tangent)
    print(f"max relative error vs FD over 8 cells: {max(errs):.2e}")


# ----------------------------------------------------------- 50.3M DOF (cfg 4)
def test_full_size_hierarchy_cfg4(torch_dev):
    """All six fields' hierarchies of the 50.3M-DOF system (8.4M rows per
    field, 494.8M nonzeros in A) equal the oracle's bitwise."""
    s, g, o = _workload(torch_dev, 4)
    for f in range(s.nf):
        nl = _check_field_hierarchy(g, o, f)
        print(f"field {f}: {nl} levels bitwise equal", flush=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_apply_cfg4(torch_dev, precision):
    s, g, o = _workload(torch_dev, 4)
    _check_apply(torch_dev, s, g, o, precision, seed=17)


def test_full_size_cfg4_value_update_and_adjoint(torch_dev):
    """A value update (two gathers over every nonzero, more than 2^28 of
    them) followed by forward and adjoint mixed solves; the residuals are
    recomputed on the GPU from the caller's CSR and reach 1e-8."""
    torch, dev = torch_dev
    s, g, o = _workload(torch_dev, 4)
    _big["o"] = None  # the oracle is not needed here
    del o
    gc.collect()
    rp, ci, v, fl = _big["dev_csr"]
    g.set_precision(1)
    g.set_values(v)
    rows = torch.repeat_interleave(torch.arange(s.n, device=dev), rp[1:] - rp[:-1])
    cols = ci.long()

    def matvec(x, transpose=False):
        y = torch.zeros(s.n, dtype=torch.float64, device=dev)
        if transpose:
            return y.index_add_(0, cols, v * x[rows])
        return y.index_add_(0, rows, v * x[cols])

    try:
        for tr, b in ((False, s.b), (True, s.x_t)):
            bt = torch.from_numpy(b).to(dev)
            x, st, it, hist = g.solve(bt, transpose=tr)
            res = float(torch.linalg.norm(bt - matvec(x, tr)) / torch.linalg.norm(bt))
            print(f"50.3M mixed solve transpose {tr}: {it} steps, residual {res:.2e} (estimate {hist[-1]:.2e})")
            assert st == 0 and res <= 1e-8, (tr, st, it, res)
    finally:
        g.set_precision(0)
        _big.clear()
        gc.collect()
        torch.cuda.empty_cache()
