"""Host-side logic of bench.py (no GPU): the one-GPU guard, the headline
workload's configuration, and the HBM-traffic figure read from the committed
counter summary only while it matches the kernel sources and build options."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_headline_workload():
    w = bench.workload()
    assert (w["W"], w["H"]) == (1000, 1000)
    assert (w["M"], w["a"], w["Q"], w["r0"]) == pytest.approx((0.5, 0.24, 0.3, 20.0), abs=1e-6)
    assert w["dt"] == 0.005 and w["max_steps"] == 50000 and w["fd_eps"] == 1e-8


def test_traffic_is_read_only_for_the_current_sources(tmp_path, monkeypatch):
    text = open(bench.TRAFFIC_PROFILE).read()
    current = bench.kernel_hash() in text
    assert (bench.recorded_traffic(1) is not None) == current
    fresh = tmp_path / "fresh.md"
    fresh.write_text("kernel source hash: " + bench.kernel_hash() + "\nHBM bytes per launch: 2.5e7\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(fresh))
    assert bench.recorded_traffic(1) == 2.5e7
    stale = tmp_path / "traffic.md"
    stale.write_text(text.replace(bench.kernel_hash(), "0" * 16))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    assert bench.recorded_traffic(1) is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.recorded_traffic(1) is None


def test_kernel_hash_covers_the_build_options(monkeypatch):
    """The hash changes with the tracing kernel's hipcc options, not with the
    rest of the build script."""
    import importlib.util
    base = bench.kernel_hash()
    real = importlib.util.spec_from_file_location

    def patched(name, path, *a, **k):
        spec = real(name, path, *a, **k)
        if name == "_grtrace_build_opts":
            loader = spec.loader

            class L(type(loader)):
                def exec_module(self, module):
                    loader.exec_module(module)
                    module.FLAGS = module.FLAGS + ["-DX"]
            spec.loader = L(loader.name, loader.path)
        return spec
    monkeypatch.setattr(importlib.util, "spec_from_file_location", patched)
    assert bench.kernel_hash() != base


def test_executed_counters_are_read_only_for_the_current_sources(tmp_path, monkeypatch):
    fresh = tmp_path / "counters.md"
    fresh.write_text("kernel source hash: " + bench.kernel_hash() +
                     "\nexecuted FP64 fraction of peak: 0.5\nexecuted flop per ray-step: 800\n")
    monkeypatch.setattr(bench, "COUNTER_PROFILE", str(fresh))
    assert bench.recorded_executed()["frac"] == 0.5
    fresh.write_text(fresh.read_text().replace(bench.kernel_hash(), "0" * 16))
    assert bench.recorded_executed() is None


def test_kernel_hash_does_not_depend_on_the_checkout_location(monkeypatch):
    """Include directories are absolute paths of the checkout; moving the
    repository must not change the hash (the profiles stay valid)."""
    import importlib.util
    base = bench.kernel_hash()
    real = importlib.util.spec_from_file_location

    def patched(name, path, *a, **k):
        spec = real(name, path, *a, **k)
        if name == "_grtrace_build_opts":
            loader = spec.loader

            class L(type(loader)):
                def exec_module(self, module):
                    loader.exec_module(module)
                    module.FLAGS = [("-I/elsewhere" + f[2:]) if f.startswith("-I") else f
                                    for f in module.FLAGS]
            spec.loader = L(loader.name, loader.path)
        return spec
    monkeypatch.setattr(importlib.util, "spec_from_file_location", patched)
    assert bench.kernel_hash() == base
