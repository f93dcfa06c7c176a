"""CPU checks of the C ABI: the built library loads and exports every entry
point that include/hbgs.h declares (no device calls)."""
import ctypes
import os
import re

import paper_2602_13079_amd as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hbgs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hbgs_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(H.LIB_PATH)
    names = _declared()
    assert "hbgs_setup" in names and "hbgs_solve" in names and "hbgs_apply" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(H.EXPORTS)


def test_options_defaults_and_struct_layout():
    o = H.default_options()
    assert (o.restart, o.max_iters, o.cheb_degree, o.coarse_max) == (50, 2000, 2, 2000)
    assert o.rtol == 1e-8 and o.theta[0] == 0.04 and o.theta[1] == 0.0
    assert abs(o.sa_damping - 4 / 3) < 1e-15
    assert o.build_transpose == 1 and o.use_graphs == 0 and o.setup_concurrent == 1


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against include/hbgs.h and compare every field offset
    with the Python mirror structures."""
    import subprocess
    fields = {"hbgs_options": H.Options, "hbgs_stats_t": H.Stats}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "hbgs.h"', "int main(void){"]
    for cname, py in fields.items():
        src.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            src.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    src.append("return 0;}")
    c = tmp_path / "probe.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    for line in out:
        if not line:
            continue
        cname, fname, val = line.split()
        py = fields[cname]
        got = ctypes.sizeof(py) if fname == "size" else getattr(py, fname).offset
        assert got == int(val), (cname, fname)


def test_last_error_is_a_string():
    assert isinstance(H.load().hbgs_last_error(), bytes)


def test_debug_knobs_reject_other_values():
    """The process-wide test knobs set host state only (no device call):
    values outside their documented range return HBGS_EINVAL with a message
    and change nothing; the defaults are accepted and restored."""
    lib = H.load()
    for fn, bad, default in ((lib.hbgs_debug_spmv_tiles, (2, -1), 1), (lib.hbgs_debug_spgemm_route, (4, -1), 0)):
        for v in bad:
            assert fn(v) == -1
            assert lib.hbgs_last_error()
        assert fn(default) == 0
