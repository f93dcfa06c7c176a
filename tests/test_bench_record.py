"""bench.py's HBM-traffic lookup: a PMC record counts only for its own kernel
class, on its own workload (same algorithmic bytes per launch), and only
while the solve kernels' source matches the hash it was taken from; and its
refusal of more than one GPU."""
import hashlib
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(tmp_path):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    src = tmp_path / "paper_2602_13079_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "solve_kernels.hip").write_text("// kernels\n")
    (tmp_path / "profiles").mkdir()
    b.ROOT = str(tmp_path)
    return b, hashlib.sha256(b"// kernels\n").hexdigest()


def _record(tmp_path, **kw):
    rec = dict(kind="spmv_outer", algorithmic_bytes_per_launch=1000, hbm_bytes_per_launch=1234.0)
    rec.update(kw)
    (tmp_path / "profiles" / "pmc_spmv_outer_x.md").write_text("# pmc\n```json\n" + json.dumps(rec) + "\n```\n")


def test_record_matches_kind_workload_and_source(tmp_path):
    b, digest = _bench(tmp_path)
    _record(tmp_path, solve_kernels_sha256=digest)
    assert b.measured_traffic("spmv_outer", 1000)[0] == 1234
    assert b.measured_traffic("spmv_outer", 2000)[0] is None  # another workload
    assert b.measured_traffic("spmv_resid", 1000)[0] is None  # another kernel class


def test_stale_record_is_ignored(tmp_path):
    b, _ = _bench(tmp_path)
    _record(tmp_path, solve_kernels_sha256="0" * 64)
    traffic, why = b.measured_traffic("spmv_outer", 1000)
    assert traffic is None and "stale" in why


def test_more_than_one_gpu_is_refused():
    """bench.py --gpus N (N > 1), or a launch with WORLD_SIZE > 1, exits with
    status 2 and a message before touching any device."""
    import subprocess
    import sys
    for args, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                           env={**os.environ, **env}, timeout=60)
        assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == "", (args, env, r.stderr)
