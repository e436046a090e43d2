"""bench.py helpers on the CPU: the counter-measured traffic is reported only
while the kernel source still has the hash its summary records, and more than
one GPU is refused."""
import hashlib
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_needs_a_matching_hash(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel source v1\n")
    h = hashlib.sha256(b"kernel source v1\n").hexdigest()
    summary = tmp_path / "traffic.md"
    summary.write_text(f"text\n\ntraffic_bytes_per_launch: 123456\nkernel_source_sha256: {h}\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(summary))
    assert bench.counter_traffic() == 123456.0
    src.write_bytes(b"kernel source v2\n")              # the kernel changed
    assert bench.counter_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.counter_traffic() is None


def test_more_than_one_gpu_is_refused(bench, monkeypatch):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as ei:
        bench.main()
    assert ei.value.code == 2
