"""Host-side pieces of bench.py's JSON line: the roofline figures of a stage
and the committed HBM-traffic record (no GPU needed)."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _prof(stage):
    return {stage: {"ms": 7.0, "launches": 2, "alg_ops": 2.3e11, "alg_bytes": 9.6e9, "units": 60000}}


def _record(tmp_path, name, src, extra=""):
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "profiles" / name).write_text(
        "source {}\nsource_sha256 {}\nfetch_kib 1000\nwrite_kib 3000\nfetch_scale 2.0\nwrite_scale 1.0\n{}".format(
            src.name, hashlib.sha256(src.read_bytes()).hexdigest(), extra))


def test_roofline_with_and_without_a_traffic_record(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernels\n")
    _record(tmp_path, "k_fft_reg_float_128_8_uneven_batch_traffic.txt", src, "alg_bytes 4096000\n")
    _record(tmp_path, "k_direct16_uneven_batch_traffic.txt", src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    r = bench.roofline_for("fft32_n128", _prof("fft32_n128"), "uneven_batch")
    assert r["kernel"] == "k_fft_reg<float, 128, 8>"
    assert r["traffic"] == 1024.0 * 5000 and r["traffic_alg_bytes"] == 4096000.0
    assert abs(r["traffic_ratio"] - 1.25) < 1e-12
    for stage in ("fft32_n64", "fft64_n64", "fft32_n512", "decode32_fft", "ntt_n64"):
        r = bench.roofline_for(stage, _prof(stage), "uneven_batch")
        assert r["traffic"] is None and "traffic_ratio" not in r, stage
        assert r["achieved"] > 0 and r["frac"] > 0
    # a record without algorithmic bytes (the direct window's): traffic only
    r = bench.roofline_for("direct16", _prof("direct16"), "uneven_batch")
    assert r["traffic"] == 1024.0 * 5000 and "traffic_ratio" not in r


def test_committed_records_parse():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.endswith("_traffic.txt"):
            rec = dict(line.split(None, 1) for line in open(os.path.join(ROOT, "profiles", name))
                       if line.strip() and not line.startswith("#"))
            assert os.path.exists(os.path.join(ROOT, rec["source"].strip())), name
            for key in ("source_sha256", "fetch_kib", "write_kib", "fetch_scale", "write_scale"):
                assert key in rec, (name, key)


def test_traffic_record_invalid_once_the_source_changes(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    (tmp_path / "profiles").mkdir()
    rec = tmp_path / "profiles" / "k_x_float_wl_traffic.txt"
    body = ("kernel k_x<float>\nworkload wl\nsource k.hip\nsource_sha256 {}\nfetch_kib 10\nwrite_kib 20\n"
            "fetch_scale 2.0\nwrite_scale 1.0\nalg_bytes 40000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec.write_text(body.format(hashlib.sha256(src.read_bytes()).hexdigest()))
    assert bench.measured_traffic("k_x<float>", "wl") == 1024.0 * 40
    assert bench.measured_traffic("k_x<float>", "wl", with_alg=True) == (1024.0 * 40, 40000.0)
    src.write_text("kernel source, edited\n")
    assert bench.measured_traffic("k_x<float>", "wl") is None
    assert bench.measured_traffic("k_x<float>", "wl", with_alg=True) == (None, None)
    assert bench.measured_traffic("k_y<float>", "wl", with_alg=True) == (None, None)   # no record
