"""GPU parity where the operand-staging SpMV runs 128-row blocks with a
ragged last block.

A 67 x 61 x 63 grid (257,481 cells, 4 fields, 1,029,924 DOF): each field's
finest operator is one row block of 256 short of the launch rule's 1024
blocks, so it takes 128-row blocks, and neither its row count nor the outer
operator's is a multiple of 128.  The test first restates on the host the
row-block rule (the largest block size whose fullest block fits the LDS
staging, stopping at the first that gives 1024 blocks) and the operand-tile
rule (at most 48 spans of 64 consecutive columns per block), so that these
matrices are known to take the staged path with a partial last block in
both precisions.  It then holds the HIP path to the oracle (hierarchies
bitwise; the apply per field to 1e-13 in FP64 and 1e-5 in FP32, both
directions; FP64 solves to 1e-8 with x within 1e-9 of the oracle's when the
iteration counts agree) and the staged path to the gathering one (bitwise:
applies and a 6-step locked solve in both precisions).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from parity_util import assert_fields_close
import synth

pytestmark = pytest.mark.gpu

DIMS = (67, 61, 63)
CAP_F32, CAP_F64 = 16384 // 4, 16384 // 8  # LDS staging entries per block
TILE_W, TILE_MAX = 64, 48


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_13079_amd as H
    H.load()  # must be built: no fallback
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def pair(torch_dev):
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    s = synth.make_system(*DIMS, 1, seed=29)
    g = H.Solver(torch.from_numpy(s.rowptr).to(dev), torch.from_numpy(s.col).to(dev),
                 torch.from_numpy(s.val).to(dev), torch.from_numpy(s.field_of_row).to(dev), s.nf, s.tree)
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree)
    return s, g, o


def _row_block(rp, cap):
    n = len(rp) - 1
    rb = 0
    for r in (256, 128, 64, 32, 16, 8, 4):
        st = np.arange(0, n, r)
        if int((rp[np.minimum(st + r, n)].astype(np.int64) - rp[st]).max()) > cap:
            continue
        rb = r
        if (n + r - 1) // r >= 1024:
            break
    return rb


def _max_tiles(rp, ci, rb):
    n = len(rp) - 1
    most = 0
    for r0 in range(0, n, rb):
        c = ci[rp[r0]:rp[min(n, r0 + rb)]]
        most = max(most, len(np.unique(c // TILE_W)))
    return most


def test_regime_ragged_staged_blocks(pair):
    s, g, _ = pair
    rp, ci, _, _ = g.get_level(0, 0, "A")
    n = len(rp) - 1
    for cap in (CAP_F32, CAP_F64):
        assert _row_block(rp, cap) == 128, cap
    assert n % 128 != 0 and (n + 255) // 256 < 1024, n
    assert _max_tiles(rp, ci, 128) <= TILE_MAX
    # the outer operator, rows ordered field by field
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    order = np.lexsort((np.arange(s.n), s.field_of_row))
    Ap = A[order][:, order].tocsr()
    assert _row_block(Ap.indptr, CAP_F64) == 128 and s.n % 128 != 0
    assert _max_tiles(Ap.indptr, Ap.indices, 128) <= TILE_MAX


def test_hierarchy_bit_exact(pair):
    s, g, o = pair
    st = g.stats()
    for f in range(s.nf):
        oa = o.amg(f)
        assert oa.levels == st["levels"][f]
        for l in range(oa.levels):
            for w in ("A", "AT") if l + 1 == oa.levels else ("A", "AT", "P", "R"):
                gr, gc, gv, _ = g.get_level(f, l, w)
                orp, oc, ov, _ = oa.get(l, w)
                assert np.array_equal(gr, orp) and np.array_equal(gc, oc), (f, l, w)
                assert np.array_equal(gv.view(np.int64), ov.view(np.int64)), (f, l, w)


@pytest.mark.parametrize("precision", [0, 1])
def test_apply_parity(torch_dev, pair, precision):
    torch, dev = torch_dev
    s, g, o = pair
    g.set_precision(precision)
    o.set_precision(precision)
    try:
        r = np.random.default_rng(13).standard_normal(s.n)
        tol = 1e-13 if precision == 0 else 1e-5
        for tr in (False, True):
            z = g.apply(torch.from_numpy(r).to(dev), transpose=tr).cpu().numpy()
            assert_fields_close(z, o.apply(r, transpose=tr), s.field_of_row, tol, tr)
    finally:
        g.set_precision(0)
        o.set_precision(0)


@pytest.mark.parametrize("precision", [0, 1])
def test_staged_equals_gathered(torch_dev, pair, precision):
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    s, g, _ = pair
    r = torch.from_numpy(np.random.default_rng(14).standard_normal(s.n)).to(dev)
    b = torch.from_numpy(s.b).to(dev)
    g.set_precision(precision)
    g.set_tolerance(0.0, 6)
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
    assert ia == ib == 6
    assert np.array_equal(xa.view(np.int64), xb.view(np.int64))
    assert np.array_equal(ha.view(np.int64), hb.view(np.int64))


def test_solve_parity_fp64(torch_dev, pair):
    torch, dev = torch_dev
    s, g, o = pair
    A = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    for tr in (False, True):
        b = s.b if not tr else s.x_t
        x, st, it, _ = g.solve(torch.from_numpy(b).to(dev), transpose=tr)
        x = x.cpu().numpy()
        ro = o.solve(b, transpose=tr)
        assert st == 0 and ro["status"] == 0
        M = A.T if tr else A
        assert np.linalg.norm(b - M @ x) <= 1e-8 * np.linalg.norm(b)
        assert abs(it - ro["iters"]) <= 2
        if it == ro["iters"]:
            assert np.linalg.norm(x - ro["x"]) <= 1e-9 * np.linalg.norm(ro["x"])
