"""bench.py's command-line contract on the host: more than one GPU is
refused with a message (the library runs on one GPU), before anything
touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_profiled_traffic_only_for_the_profiled_workload(tmp_path):
    """A counter summary's HBM traffic goes only on the line of the workload
    it was measured on, and only while the kernel sources hash to the
    profiled ones (checked on a copy of the sources and a written summary)."""
    import hashlib
    import shutil
    b = _bench_module()
    names = ("cia_phase.hip", "plan.h", "fastmath.h", "wave.h")
    csrc = tmp_path / "paper_2203_16657_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in names:
        shutil.copy(os.path.join(ROOT, "paper_2203_16657_amd", "csrc", f), csrc / f)
    h = hashlib.sha256(b"".join((csrc / f).read_bytes() for f in names)).hexdigest()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "s.md").write_text(
        "Workload: text\ntraffic_bytes_per_launch (other kernel): 5\n"
        "traffic_bytes_per_launch: 1.5e+10\nworkload: ensemble_256\nsource_sha256: %s\n" % h)
    b.ROOT = str(tmp_path)
    assert b.profiled_traffic("ensemble_256", "s.md") == 1.5e10
    assert b.profiled_traffic("kuramoto_powerlaw_n1000000", "s.md") is None
    assert b.profiled_traffic("ensemble_256", "no_such_summary.md") is None
    with open(csrc / "wave.h", "a") as f:
        f.write("\n")
    assert b.profiled_traffic("ensemble_256", "s.md") is None
