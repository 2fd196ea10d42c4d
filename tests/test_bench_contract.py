"""Host-side checks of the benchmark's contract (no GPU): the one-GPU
limit, and the traffic figure it reports against the committed rocprofv3
summary it is read from."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_profiled_traffic_matches_the_counter_table():
    import bench
    text = open(bench.PROFILE).read()
    m = re.search(r"bytes_per_launch=(\d+)", text)
    assert m, "machine-readable traffic line missing"
    committed = int(m.group(1))
    # the traffic table's row of the linearization: FETCH_SIZE and
    # WRITE_SIZE in KiB per dispatch, scaled by the copy calibration
    row = [ln for ln in text.splitlines() if ln.startswith("| linearize (direct)")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    fetch_kib = float(cells[1].replace(" ", ""))
    write_kib = float(cells[3].replace(" ", ""))
    flat = " ".join(text.split())
    f_fetch = float(re.search(r"factor ([\d.]+) to bytes read", flat).group(1))
    f_write = float(re.search(r"factor ([\d.]+) to bytes written", flat).group(1))
    est = (fetch_kib * f_fetch + write_kib * f_write) * 1024.0
    assert abs(est - committed) <= 1e-5 * committed
    # reported only while the kernel sources hash to the recorded value
    got = bench.profiled_traffic("linearize")
    assert got in (None, committed)
    assert bench.profiled_traffic("rollout") is None
