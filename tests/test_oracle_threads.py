"""The oracle's parallel loops (OpenMP, used for the CPU baseline timing)
leave every result bitwise unchanged: hierarchies, applies and solves with
one thread equal those with several."""
import numpy as np

import oracle
import synth


def _run(s, threads, **opt):
    oracle.set_threads(threads)
    assert oracle.get_threads() == threads
    o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, **opt)
    out = {}
    for f in range(s.nf):
        h = o.amg(f)
        for l in range(h.levels):
            for w in ("A", "P", "R", "AT") if l + 1 < h.levels else ("A", "AT"):
                out[(f, l, w)] = h.get(l, w)[:3]
            if l + 1 < h.levels:
                out[(f, l, "agg")] = h.agg(l)
                out[(f, l, "sc")] = np.array(list(h.scalars(l).values()))
    r = np.random.default_rng(4).standard_normal(s.n)
    for tr in (False, True):
        out[("apply", tr)] = o.apply(r, transpose=tr)
        ro = o.solve(s.b if not tr else s.x_t, transpose=tr)
        out[("x", tr)] = ro["x"]
        out[("hist", tr)] = ro["hist"]
    return out


def test_thread_count_does_not_change_results():
    s = synth.make_system(24, 24, 24, 1, seed=5)  # 13,824 rows per field: the loops run threaded
    try:
        for precision in (0, 1):
            a = _run(s, 1, coarse_max=500, precision=precision, max_iters=30)
            b = _run(s, 4, coarse_max=500, precision=precision, max_iters=30)
            assert a.keys() == b.keys()
            for k in a:
                for p, q in zip(a[k] if isinstance(a[k], tuple) else (a[k],),
                                b[k] if isinstance(b[k], tuple) else (b[k],)):
                    assert np.array_equal(np.asarray(p).view(np.uint8), np.asarray(q).view(np.uint8)), (precision, k)
    finally:
        oracle.set_threads(1)
