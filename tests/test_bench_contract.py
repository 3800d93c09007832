"""Host-side checks of the benchmark script: the one-GPU restriction and the
algorithmic byte counts its roofline divides by."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_per_unit():
    """38 S + 3 S_u per fluid node (19 reads and 19 writes of the storage
    type, the three velocity components) and the walker record read and
    written back (cell + 3 offsets)."""
    sys.path.insert(0, ROOT)
    import bench
    assert [bench.fluid_bytes_per_node(p) for p in ("fp64", "fp32", "fp16", "bf16")] == [328, 164, 88, 88]
    assert [bench.walker_bytes_per_step(p) for p in ("fp64", "fp32", "fp16", "bf16")] == [56, 32, 32, 32]
    from paper_2308_05007_amd import workloads as W
    # the headline launch: 256^3 periodic fluid nodes and 1e7 walkers in FP32
    cfg = W.config_oscillator(precision="fp32", n_walkers=10_000_000)
    assert bench.fluid_nodes(cfg) == 256 ** 3
    assert bench.fluid_nodes(cfg) * 164 + cfg["walkers"]["n"] * 32 == 3071463424
    # the cache-resident channel: 128 x 126 x 128 fluid nodes (two wall planes) and 1e6 walkers
    cfg = W.config_channel(precision="fp32")
    assert bench.fluid_nodes(cfg) == 128 * 126 * 128
    assert bench.fluid_nodes(cfg) * 164 + cfg["walkers"]["n"] * 32 == 370558976
