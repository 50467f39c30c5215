"""CPU-side tests of bench.py's host logic: the one-GPU refusal, the algorithmic work
that the headline TFLOP/s divides by, and the source digest that guards the stored HBM
counters."""
import os
import subprocess
import sys

import torch

import paper_2308_01480_amd as ttr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_sweep_work_of_the_48x5_workload():
    # Mode shapes of the 48^5 workload (r = 20, p = 10, q = 3): a saturated 48 x 48^4
    # first mode, regular 960 x 110592 and 960 x 2304 modes, and a saturated 960 x 48
    # last unfolding.  Regular: m n (2 s + 4 s (q + 1) + 2 r); saturated: the short-side
    # Gram min(m,n)(min(m,n)+1)max(m,n) plus the carry 2 r m n.
    s, q, r = 30, 3, 20
    reg = 2 * s + 4 * s * (q + 1) + 2 * r
    expect = (48 * 49 * 48 ** 4 + 2 * r * 48 * 48 ** 4) + 960 * 110592 * reg + 960 * 2304 * reg + \
        (48 * 49 * 960 + 2 * r * 960 * 48)
    pl = ttr.plan([48] * 5, 20, 3, 10, torch.float32)
    flops, nbytes = bench.sweep_flops_bytes(pl, 4, 4)
    assert flops == expect == 85542147072
    # reads: 2 passes of the first mode, q + 3 of each regular mode, 2 of the last; the
    # carries written once (r n each)
    reads = 2 * 48 ** 5 + (q + 3) * 960 * 110592 + (q + 3) * 960 * 2304 + 2 * 960 * 48
    writes = r * 48 ** 4 + r * 110592 + r * 2304 + r * 48
    assert nbytes == 4 * (reads + writes)


def test_stored_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    kv = {}
    if os.path.exists(bench.TRAFFIC_FILE):
        with open(bench.TRAFFIC_FILE) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.strip().split("=", 1)
                    kv[k] = v
        current = kv["source_digest"] == bench.kernel_source_digest()
        assert bench.measured_traffic() == (float(kv["hbm_bytes_per_launch"]) if current else None)
    else:
        assert bench.measured_traffic() is None
    stored = tmp_path / "traffic.txt"
    stored.write_text("# test\nsource_digest=%s\nhbm_bytes_per_launch=123.0\n" % bench.kernel_source_digest())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stored))
    assert bench.measured_traffic() == 123.0
    changed = tmp_path / "kernel.hip"
    changed.write_text("// a different kernel source\n")
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", [str(changed)])
    assert bench.measured_traffic() is None


def test_sweep_work_of_the_256x4_workload():
    # 256^4, r = 32, p = 8, q = 4: three regular modes 256 x 256^3, 8192 x 65536, 8192 x 256
    s, q, r = 40, 4, 32
    reg = 2 * s + 4 * s * (q + 1) + 2 * r
    pl = ttr.plan([256] * 4, 32, 4, 8, torch.bfloat16)
    assert pl.kinds == ["regular"] * 3
    flops, _ = bench.sweep_flops_bytes(pl, 2, 4)
    assert flops == (256 * 256 ** 3 + 8192 * 65536 + 8192 * 256) * reg
