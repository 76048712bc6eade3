"""Host logic of the benchmark (no GPU): the measured-traffic record is used
only for the kernel sources it was taken on, the kernel and the tile size it
names, and the algorithmic per-neuron bytes follow the state each model
keeps."""
import hashlib
import json
import os

import bench


def fake_root(tmp_path, tile=None):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source")
    ent = {"kernel": "k_step_binned", "bytes_per_launch": 1234}
    if tile is not None:
        ent["tile_neurons"] = tile
    rec = {"kernel_sources": ["k.hip"],
           "kernel_sources_sha256": hashlib.sha256(b"kernel source").hexdigest(),
           "workloads": {"sweep": ent}}
    os.makedirs(tmp_path / "profiles")
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    return src


def test_traffic_record_matches_sources_kernel_and_tile(tmp_path, monkeypatch):
    src = fake_root(tmp_path, tile=4096)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("sweep", "k_step_binned", 4096) == 1234
    assert bench.measured_traffic("sweep", "k_step_binned", 2048) is None
    assert bench.measured_traffic("sweep", "k_step", 4096) is None
    assert bench.measured_traffic("adex", "k_step_binned", 4096) is None
    src.write_bytes(b"kernel source, edited")
    assert bench.measured_traffic("sweep", "k_step_binned", 4096) is None


def test_traffic_record_without_tile_size(tmp_path, monkeypatch):
    fake_root(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("sweep", "k_step_binned", 512) == 1234


def test_committed_traffic_record_is_well_formed():
    rec = json.load(open(os.path.join(os.path.dirname(bench.__file__), "profiles", "traffic.json")))
    for src in rec["kernel_sources"]:
        assert os.path.exists(os.path.join(os.path.dirname(bench.__file__), src))
    for w, ent in rec["workloads"].items():
        assert ent["kernel"] in ("k_step", "k_step_binned", "k_step_binned_runs")
        scaled = (ent["fetch_kib"] * 1.99975 + ent["write_kib"]) * 1024
        assert abs(ent["bytes_per_launch"] / scaled - 1) < 1e-4, w


def test_neuron_bytes_per_model():
    pops = [dict(model="lif_delta", ports=1, n=10), dict(model="lif_exp", ports=2, n=3),
            dict(model="aeif_cond_exp", ports=2, n=5), dict(model="aeif_cond_beta", ports=2, n=7)]
    spec = dict(populations=pops)
    binned = 10 * 20 + 3 * (16 + 16 + 4) + 5 * (24 + 16 + 4) + 7 * (24 + 32 + 4)
    assert bench.bytes_per_step_neurons(spec, "binned") == binned
    assert bench.bytes_per_step_neurons(spec, "direct") == binned + 8 * (10 * 1 + 3 * 2 + 5 * 2 + 7 * 2)


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr and r.stdout == ""
