"""The CPU oracle and the input generator built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc), then driven through their Python bindings
in a child process over small systems: every setup path (hierarchies with
dense and smoothed coarsest levels, leaves, nested form, block Jacobi),
applies, solves in both directions and precisions, gradients and the pin
building blocks.  Any sanitizer report fails the test.

The HIP library's host code runs only with a GPU; it is exercised by the
GPU tests, not here."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-O1", "-g"]

DRIVER = textwrap.dedent("""
    import sys
    import numpy as np
    import scipy.sparse as sp
    sys.path.insert(0, ROOT)
    import oracle, synth
    oracle._LIB_PATH = ORACLE_SO
    synth._LIB_PATH = SYNTH_SO
    oracle.set_threads(2)
    for args, cm in (((None, None), 64), ((7, 5, 9, 3), 40)):
        s = synth.make_system(cfg=0) if args[0] is None else synth.make_system(*args, seed=11)
        for opt in (dict(), dict(block_jacobi=1), dict(field_cheb_degree=[4, 4]),
                    dict(field_leaf=[0, 0, 0] + [2] * (s.nf - 3), ilu_block=48),
                    dict(field_leaf=[0, 0, 0] + [1] * (s.nf - 3)), dict(theta=[0.64])):
            for precision in (0, 1):
                o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, s.tree, coarse_max=cm,
                                  precision=precision, **opt)
                r = np.random.default_rng(1).standard_normal(s.n)
                for tr in (False, True):
                    o.apply(r, transpose=tr)
                    res = o.solve(s.b if not tr else s.x_t, transpose=tr)
                    assert np.all(np.isfinite(res["x"]))
                o.grad_values(r, r)
                for f in range(s.nf):
                    h = o.amg(f)
                    for l in range(h.levels):
                        h.get(l, "A")
                        if l + 1 < h.levels:
                            h.get(l, "P"); h.agg(l); h.scalars(l)
        tree2 = [-1, -1, 0, 1, -2, -1] + list(range(2, s.nf)) + [-2, -2]
        o = oracle.Oracle(s.rowptr, s.col, s.val, s.nf, s.field_of_row, tree2, coarse_max=cm, nested=1, restart=5)
        o.solve(s.b)
        o.solve(s.x_t, transpose=True)
    # a coarsening that stops above the dense limit: one smoothed level
    A = sp.diags([-np.ones(8999), np.full(9000, 2.0), -np.ones(8999)], [-1, 0, 1], format="csr")
    h = oracle.Amg(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data, theta=0.64, salt=7)
    assert h.smoothed_coarsest
    h.vcycle(np.ones(9000)); h.vcycle(np.ones(9000), transpose=True)
    # building blocks of the pins
    B = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    rp, ci, v = s.rowptr, s.col, s.val
    st = oracle.strength(rp, ci, v, 0.04)
    oracle.aggregate(rp, ci, v, st, 3)
    oracle.filtered(rp, ci, v, st)
    oracle.power_estimate(rp, ci, v, B.diagonal(), 10, 5)
    oracle.spgemm((rp, ci, v, s.n), (rp, ci, v, s.n))
    oracle.lu_solve(rp, ci, v, s.b[:s.n])
    print("sanitized run ok")
""")


def _build(tmp):
    osrc = os.path.join(ROOT, "oracle", "hbgs_oracle.cpp")
    ssrc = os.path.join(ROOT, "synth", "synth.c")
    oso, sso = os.path.join(tmp, "liboracle_san.so"), os.path.join(tmp, "libsynth_san.so")
    subprocess.check_call(["g++", *SAN, "-std=c++17", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", oso, osrc])
    subprocess.check_call(["gcc", *SAN, "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", sso, ssrc,
                           "-lm"])
    return oso, sso


def test_oracle_and_generator_under_asan_ubsan(tmp_path):
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"]).decode().strip()
    if not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime")
    oso, sso = _build(str(tmp_path))
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    code = f"ROOT = {ROOT!r}\nORACLE_SO = {oso!r}\nSYNTH_SO = {sso!r}\n" + DRIVER
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
    report = p.stdout + p.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert p.returncode == 0 and "sanitized run ok" in p.stdout, report[-4000:]
