"""The benchmark's command-line contract and its reading of the committed counter
summary (CPU only)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_exit_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def _cfg(**kw):
    c = dict(bulk_block_x=256, bulk_store_solid=0, link_block=256, graph_steps=16, bulk_xcd=1,
             bulk_fused=0, bulk_rows=1)
    c.update(kw)
    return c


def test_bulk_kernel_names_follow_the_templates():
    assert bench.bulk_kernel_name(_cfg(), "compact", "f32") == \
        "void bulk_kernel<1, false, true, 256, false, true, 1, 0>"
    assert bench.bulk_kernel_name(_cfg(bulk_block_x=64, bulk_store_solid=1), "dense", "f16") == \
        "void bulk_kernel<2, false, true, 64, true, false, 1, 0>"
    assert bench.bulk_kernel_name(_cfg(bulk_rows=2), "compact", "bf16").endswith(", 2, 0>")
    assert bench.bulk_kernel_name(_cfg(), "compact", "f32", coll=1).endswith(", 1, 1>")
    assert bench.bulk_kernel_name(_cfg(bulk_fused=1), "compact", "f32") is None
    assert bench.bulk_kernel_name(_cfg(bulk_runs=1), "compact", "f32") == \
        "void bulk_run_kernel<1, true, 0, false, false>"
    assert bench.bulk_kernel_name(_cfg(bulk_runs=1), "compact", "bf16", coll=1) == \
        "void bulk_run_kernel<3, true, 1, false, false>"
    assert bench.bulk_kernel_name(_cfg(bulk_runs=1, bulk_fused=1), "compact", "f32") == \
        "void bulk_run_kernel<1, true, 0, true, false>"
    assert bench.bulk_kernel_name(_cfg(bulk_runs=2), "compact", "f32") == \
        "void bulk_run_kernel<1, true, 0, false, true>"
    assert bench.bulk_kernel_name(_cfg(bulk_runs=1), "dense", "f32") is None


def test_counter_traffic_reads_the_committed_summary():
    """A summary taken on the current kernel source gives, for a shape it holds, HBM
    bytes of the right magnitude (between the algorithmic bytes and twice them);
    another layout, another storage or the fused form give none, and so does every
    shape once the kernel source has changed since the counters were taken."""
    txt = open(bench.COUNTER_SUMMARY).read()
    if f"kernel_source_sha256_12: {bench.kernel_hash()}" not in txt:
        for rows in (1, 2):
            assert bench.counter_traffic("compact", _cfg(bulk_rows=rows)) is None
        return
    shapes = [line.split("|")[0][len("variant:"):].strip() for line in txt.splitlines()
              if line.startswith("variant:")]
    assert shapes
    found = 0
    for rows in (1, 2):
        name = bench.bulk_kernel_name(_cfg(bulk_rows=rows), "compact", "f32")
        t = bench.counter_traffic("compact", _cfg(bulk_rows=rows))
        if name in shapes:
            found += 1
            assert 758311472 < t < 2 * 758311472
        else:
            assert t is None
    assert found >= 1
    assert bench.counter_traffic("dense", _cfg()) is None
    assert bench.counter_traffic("compact", _cfg(), "f16") is None
    assert bench.counter_traffic("compact", _cfg(bulk_fused=1)) is None
