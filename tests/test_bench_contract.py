"""Host-side parts of the benchmark contract (no GPU needed)."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def test_counter_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    b = _bench()
    rec_path = os.path.join(ROOT, "profiles", "element_kernel_C5_hbm_traffic.json")
    with open(rec_path) as fh:
        rec = json.load(fh)
    assert b.counter_traffic("C3") is None               # measured on C5 only
    t = b.counter_traffic("C5")
    assert t is None or abs(t - rec["traffic_bytes_per_launch"]) < 1.0
    # a record whose source hash does not match is ignored
    fake = dict(rec, source_sha256="0" * 64)
    (tmp_path / "profiles").mkdir()
    with open(tmp_path / "profiles" / "element_kernel_C5_hbm_traffic.json", "w") as fh:
        json.dump(fake, fh)
    for f in rec["source_files"]:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        with open(os.path.join(ROOT, f), "rb") as src, open(dst, "wb") as out:
            out.write(src.read())
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.counter_traffic("C5") is None


def test_blend_mask_takes_the_lowest_fraction_with_seeded_ties():
    import numpy as np
    b = _bench()
    ind = np.array([5.0, 1.0, 1.0, 1.0, 3.0, 0.5, 9.0, 1.0])
    m = b.blend_mask(ind, 0.25, seed=3)
    assert m.sum() == 2 and m[5]                     # the minimum, plus one of the tied 1.0 values
    assert np.array_equal(m, b.blend_mask(ind, 0.25, seed=3))
