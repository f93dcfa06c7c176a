"""hbgs_apply_noalloc (the entry point that allocates nothing) against
hbgs_apply, through the C ABI: two calls in a row on one device, the second
on a smaller system, in both precisions and both directions (on small
systems, and on a 1M-DOF one whose passes stage their operand in LDS); then
the rejections (too many rows, the nested form, adjoint operators not
built)."""
import ctypes

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
    H.load()
    return torch, torch.device("cuda:0")


def _solver(torch, dev, s, **opt):
    import paper_2602_13079_amd as H
    args = (torch.from_numpy(s.rowptr).to(dev), torch.from_numpy(s.col).to(dev), torch.from_numpy(s.val).to(dev),
            torch.from_numpy(s.field_of_row).to(dev), s.nf, s.tree)
    return H.Solver(*args, **opt)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_apply_matches_apply(torch_dev, precision):
    torch, dev = torch_dev
    big = synth.make_system(cfg=0)                       # 4,096 rows, three-level hierarchies
    small = synth.make_system(7, 5, 9, 3, seed=11)       # 1,890 rows, 6 fields
    gb = _solver(torch, dev, big, coarse_max=64, precision=precision)
    gs = _solver(torch, dev, small, coarse_max=40, precision=precision)
    for tr in (False, True):
        for tag, g, s in (("4096 rows", gb, big), ("1890 rows", gs, small)):
            print(f"noalloc apply: precision {precision} transpose {tr} {tag}", flush=True)
            r = torch.from_numpy(np.random.default_rng(21 + s.n).standard_normal(s.n)).to(dev)
            z = torch.full_like(r, float("nan"))
            g.apply_noalloc(r, z, transpose=tr)
            torch.cuda.synchronize()
            ref = g.apply(r, transpose=tr)
            assert torch.equal(z, ref), (tag, tr)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_apply_matches_apply_staged(torch_dev, precision):
    """A 1M-DOF system (its finest passes stage their operand in LDS, 256-row
    blocks; its fields run on concurrent streams), then a smaller one."""
    torch, dev = torch_dev
    big = synth.make_system(cfg=1)                       # 1,048,576 rows
    small = synth.make_system(cfg=0)                     # 4,096 rows
    gb = _solver(torch, dev, big, precision=precision)
    gs = _solver(torch, dev, small, coarse_max=64, precision=precision)
    for tr in (False, True):
        for tag, g, s in (("1M rows", gb, big), ("4096 rows", gs, small)):
            print(f"noalloc apply: precision {precision} transpose {tr} {tag}", flush=True)
            r = torch.from_numpy(np.random.default_rng(31 + s.n).standard_normal(s.n)).to(dev)
            z = torch.full_like(r, float("nan"))
            g.apply_noalloc(r, z, transpose=tr)
            torch.cuda.synchronize()
            ref = g.apply(r, transpose=tr)
            assert torch.equal(z, ref), (tag, tr)


def test_noalloc_rejections(torch_dev):
    torch, dev = torch_dev
    import paper_2602_13079_amd as H
    s = synth.make_system(7, 5, 9, 3, seed=11)
    r = torch.from_numpy(np.random.default_rng(3).standard_normal(s.n)).to(dev)
    z = torch.empty_like(r)
    # adjoint operators deferred and not yet built
    gl = _solver(torch, dev, s, coarse_max=40, build_transpose=0)
    with pytest.raises(H.HBGSError) as e:
        gl.apply_noalloc(r, z, transpose=True)
    assert e.value.code == -1 and "adjoint" in str(e.value)
    gl.apply(r, transpose=True)  # builds them
    gl.apply_noalloc(r, z, transpose=True)
    torch.cuda.synchronize()
    assert torch.equal(z, gl.apply(r, transpose=True))
    # the nested form
    gn = _solver(torch, dev, s, coarse_max=40, nested=1)
    with pytest.raises(H.HBGSError) as e:
        gn.apply_noalloc(r, z)
    assert e.value.code == -1
    # more rows than the fixed buffer holds: a 1D Laplacian of 4,194,305 rows
    n = 4194305
    A = sp.diags([-np.ones(n - 1), np.full(n, 2.0), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    A.sort_indices()
    one = synth.System(n=n, nf=1, rowptr=A.indptr.astype(np.int32), col=A.indices.astype(np.int32), val=A.data,
                       field_of_row=np.zeros(n, np.int32), tree=[-1, 0, -2])
    gbig = _solver(torch, dev, one)
    rb = torch.ones(n, dtype=torch.float64, device=dev)
    zb = torch.empty_like(rb)
    with pytest.raises(H.HBGSError) as e:
        gbig.apply_noalloc(rb, zb)
    assert e.value.code == -1 and "4194304" in str(e.value)
