"""Host-side pieces of bench.py: the one-GPU guard, launch-shape parsing,
kernel labels, the roofline arithmetic and the profile lookup that gates
the HBM-traffic figure on the kernel sources.  CPU only."""
import hashlib
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_shapes_and_kernel_labels():
    b = _bench()
    assert b.parse_shape("") is None
    assert b.parse_shape("256,4,1,128") == {"block": 256, "lanes": 4, "targets": 1, "xcd_group": 128}
    assert b.step_kernel_name({"lanes": 4, "targets": 1}, dim=3) == "k_pair<3, float, 4, 0, 4, false>"
    assert b.step_kernel_name({"lanes": 1, "targets": 2}, coincident=True) == "k_pair2<2, float, 4, 0, true>"
    assert b.step_kernel_name({"lanes": 4, "targets": 2}, dim=3) == "k_pair42<3, float, 4, 0, false>"
    assert b.step_kernel_name({"lanes": 4, "targets": 2}, dim=3, coincident=True) == "k_pair<3, float, 4, 0, 4, true>"


def test_roofline_arithmetic():
    b = _bench()
    r = b.roofline_alu(3, 1_000_000_000, 1.0, "k_pair<3, float, 4, 0, 4, false>", 10)
    assert abs(r["achieved"] - 39.0) < 1e-9  # 39 flops x 1e9 interactions per ms
    assert abs(r["frac"] - 39.0 / 157.3) < 1e-12
    assert r["traffic"] is None  # no profile given
    assert abs(r["valu_issue_frac"] - 36 * 1e9 / 1e-3 / (256 * 64 * 2.4e9)) < 1e-12


def test_profile_lookup_follows_the_kernel_sources(tmp_path):
    b = _bench()
    h = hashlib.sha256()
    for f in b.PAIR_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_09488_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    good = tmp_path / "good.md"
    good.write_text(f"traffic_bytes_per_launch: 1.5e8\nl2_hit_rate: 0.8\nkernel: k_x<1>\nsource_sha256: {h.hexdigest()}\n")
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 1.5e8\nkernel: k_x<1>\nsource_sha256: 00\n")
    assert b.pair_profile("k_x<1>", "traffic_bytes_per_launch", str(good)) == 1.5e8
    assert b.pair_profile("k_x<1>", "l2_hit_rate", str(good)) == 0.8
    assert b.pair_profile("k_y<1>", "traffic_bytes_per_launch", str(good)) is None  # another kernel
    assert b.pair_profile("k_x<1>", "traffic_bytes_per_launch", str(stale)) is None  # sources changed
    assert b.pair_profile("k_x<1>", "traffic_bytes_per_launch", str(tmp_path / "none.md")) is None
