"""The benchmark's contract on the CPU: it refuses more than one GPU before
touching a device, its CPU leg reports the oracle in the agreed shape, and the
HBM traffic figure is read only from a counter summary that matches the
kernel sources, workload and schedule."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import synth  # noqa: E402
import paper_1206_1199_amd as otoo  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr + r.stdout


def test_cpu_baseline_shape():
    pos, m = synth.plummer(4096, seed=11)
    t = otoo.Tree(pos, m, n_crit=16)
    lists = t.walk(theta=0.5, g_max=64)
    _, p32, m32, cm = t.export(4)
    sample = synth.sample_idx(len(m), 64, seed=12)
    base, (acc, pot), direct = bench.cpu_baseline(p32, m32, lists, cm, 0.01, sample)
    assert base["kind"] == "oracle" and base["unit"] == "Ginteractions/s" and base["value"] > 0
    assert base["cores"] >= 1 and isinstance(base["sample"], str)
    assert base["one_core"]["cores"] == 1 and base["one_core"]["value"] > 0
    assert base["direct"]["value"] > 0 and acc.shape == (len(m), 3) and pot.shape == (len(m),)
    assert direct[0].shape == (64, 3)


def test_traffic_is_read_only_for_matching_sources(tmp_path, monkeypatch):
    h = hashlib.sha256()
    for f in ("paper_1206_1199_amd/csrc/otoo_force.hip", "paper_1206_1199_amd/csrc/otoo_internal.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    sched = {"group_mode": "chunk", "g_max": 64, "chunk": 2048, "blocks_per_cu": 8, "lpt": 1, "tile": 256}
    prof = tmp_path / "profiles"
    prof.mkdir()

    def write(sha, workload, schedule, name="k_force_plummer1m.md"):
        (prof / name).write_text(
            f"# summary\n\ntraffic_bytes_per_launch: 123456\nsource_sha256: {sha}\nworkload: {workload}\n"
            f"schedule: {json.dumps(schedule, sort_keys=True)}\n")

    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "paper_1206_1199_amd" / "csrc").mkdir(parents=True)
    for f in ("otoo_force.hip", "otoo_internal.h"):
        (tmp_path / "paper_1206_1199_amd" / "csrc" / f).write_bytes(
            open(os.path.join(ROOT, "paper_1206_1199_amd", "csrc", f), "rb").read())
    write(h.hexdigest()[:16], "W", sched)
    assert bench.measured_traffic("plummer1m", "plain", "W", sched) == 123456.0
    assert bench.measured_traffic("plummer1m", "plain", "other workload", sched) is None
    assert bench.measured_traffic("plummer1m", "plain", "W", dict(sched, chunk=4096)) is None
    assert bench.measured_traffic("plummer1m", "learned", "W", sched) is None     # no summary of that mode
    assert bench.measured_traffic("cube16m", "plain", "W", sched) is None         # nor of that workload
    write(h.hexdigest()[:16], "W", sched, name="k_force_cube16m_learned.md")
    assert bench.measured_traffic("cube16m", "learned", "W", sched) == 123456.0
    write("0" * 16, "W", sched)
    assert bench.measured_traffic("plummer1m", "plain", "W", sched) is None
