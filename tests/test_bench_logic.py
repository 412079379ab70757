"""Host logic of bench.py (no GPU): the one-GPU refusal, the committed-counter lookup (workload,
reconstruction and kernel-source hash must all match, else the roofline traffic is reported as
null), and the unit counts behind the algorithmic bytes of each kernel.
"""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counters(tmp_path, **over):
    js = {"workload": "torus3d_256x256x256", "recon": "plm", "kernel_source_sha256": bench.kernel_source_hash(),
          "per_launch": {"update": {"hbm_read_bytes": 1.0, "hbm_write_bytes": 2.0, "fp64_flop": 3.0}}}
    js.update(over)
    p = tmp_path / "c.json"
    p.write_text(json.dumps(js))
    return str(p)


def test_counters_are_used_only_for_the_profiled_workload_reconstruction_and_sources(tmp_path, monkeypatch):
    good = _counters(tmp_path)
    monkeypatch.setattr(bench, "COUNTERS", {"plm": good, "ppm": good})
    assert bench.profiled_counters("torus3d_256x256x256", "plm")["update"]["hbm_write_bytes"] == 2.0
    assert bench.profiled_counters("torus3d_128x64x64", "plm") is None
    assert bench.profiled_counters("torus3d_256x256x256", "ppm") is None
    stale = _counters(tmp_path, kernel_source_sha256="0" * 64)
    monkeypatch.setattr(bench, "COUNTERS", {"plm": stale, "ppm": stale})
    assert bench.profiled_counters("torus3d_256x256x256", "plm") is None
    monkeypatch.setattr(bench, "COUNTERS", {"plm": str(tmp_path / "missing.json"), "ppm": good})
    assert bench.profiled_counters("torus3d_256x256x256", "plm") is None


def test_committed_counter_files_name_their_workload_and_reconstruction():
    for recon, path in bench.COUNTERS.items():
        with open(path) as fh:
            js = json.load(fh)
        assert js["workload"] == "torus3d_256x256x256"
        assert js.get("recon", "plm") == recon
        assert set(js["per_launch"]) >= {"flux1", "flux2", "flux3", "update"}
        for v in js["per_launch"].values():
            assert v["hbm_read_bytes"] >= 0 and v["hbm_write_bytes"] >= 0


def test_unit_counts_per_launch():
    n1, n2, n3 = 256, 256, 256
    assert bench.units_per_launch("flux1", n1, n2, n3) == 257 * 258 * 256
    assert bench.units_per_launch("flux2", n1, n2, n3) == 258 * 257 * 256
    assert bench.units_per_launch("flux3", n1, n2, n3) == 258 * 258 * 256
    assert bench.units_per_launch("update", n1, n2, n3) == n1 * n2 * n3
    # ghost cells: two layers (PLM) or three (PPM) around the X1 x X2 interior, every phi
    for recon, g in (("plm", 2), ("ppm", 3)):
        ghosts = ((n1 + 2 * g) * (n2 + 2 * g) - n1 * n2) * n3
        assert bench.units_per_launch("bound", n1, n2, n3, recon) == ghosts


def test_step_roofline_inputs():
    """320 B per zone-update (stage 1 reads and writes the state, stage 2 also reads P^n) and the
    FP64 operation count of the committed op-counting oracle run, which must cover the benchmark
    torus's physics."""
    assert bench.ALG_BYTES_STAGE == (128.0, 192.0) and bench.ALG_BYTES_ZU == 320.0
    f = bench.oracle_flops_per_zu()
    assert f is not None and 3e3 < f < 2e4
    with open(bench.FLOP_COUNT) as fh:
        js = json.load(fh)
    d = js["per_zone_update"][bench.FLOP_KEY]
    assert d["total"] == sum(d[k] for k in ("add", "mul", "div", "sqrt", "pow", "other_libm"))
    assert "command" in js
