"""Host logic of the benchmark and the sweep (no GPU): the counter figure is
used only for the kernel source it was taken on, --gpus N > 1 is refused
with a message, the sweep's instance list is seeded and shaped as stated,
and the growth-rate fit recovers a known exponential."""

import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_traffic_figure_follows_the_kernel_source(tmp_path, monkeypatch):
    import bench

    def write(h):
        d = tmp_path / "profiles"
        d.mkdir(exist_ok=True)
        (d / "collide_64x32_fp32_hbm_counters.md").write_text(
            "# counters\n\n| a | b |\n\n```\ntraffic_bytes_per_launch: 12345\n"
            f"source_hash: {h}\nnx: 64\nny: 32\nprecision: fp32\n```\n")

    current = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: current)
    assert bench.traffic_from_profiles(64, 32, "fp32") is None  # no summary
    write(current)
    assert bench.traffic_from_profiles(64, 32, "fp32") == 12345.0
    # another workload, or counters taken on another kernel source: no figure
    assert bench.traffic_from_profiles(64, 64, "fp32") is None
    write("0" * 16)
    assert bench.traffic_from_profiles(64, 32, "fp32") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_sweep_instances_are_seeded_and_shaped():
    from paper_1812_05711_amd.sweep import five_smooth_at_least, sweep_configs

    a, b = sweep_configs(), sweep_configs()
    assert a == b and len(a) == 64
    for c in a:
        assert 64 <= c["ny"] <= 256 and 100.0 <= c["T"] <= 250.0
        nx = c["nx"]
        assert nx == five_smooth_at_least(round(1.22 * c["ny"]))
        k = nx
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        assert k == 1
    assert len({c["instance_id"] for c in a}) == 64


def test_growth_rate_fit():
    from paper_1812_05711_amd.sweep import growth_rate

    t0 = 1000.0
    steps = np.arange(1, 41) * 50.0
    hist = np.zeros((44, 5))
    hist[:40, 0] = steps
    hist[:40, 4] = 3e-4 * np.exp(0.7 * steps / t0)
    hist[:40, 1] = 1.0  # another column, not used by the default fit
    assert abs(growth_rate(hist, t0) - 0.7) < 1e-9
    assert abs(growth_rate(hist, t0, col=1)) < 1e-12


def test_threshold_zero_crossing():
    from paper_1812_05711_amd import sweep

    assert sweep.zero_crossing([160.0, 162.0, 164.0], [-0.2, -0.1, 0.3]) == pytest.approx(162.5)
    assert sweep.zero_crossing([164.0, 160.0], [0.3, -0.1]) == pytest.approx(161.0)
    assert sweep.zero_crossing([160.0, 162.0], [-0.2, -0.1]) is None
    cfgs = sweep.threshold_configs(122, 100, [160.0, 165.0])
    assert [c["T"] for c in cfgs] == [160.0, 165.0] and all(c["init_mode"] == "eq29" for c in cfgs)


def test_growth_fit_quality_and_transient_flag():
    from paper_1812_05711_amd.sweep import growth_fit

    t0 = 1000.0
    steps = np.arange(1, 41) * 50.0  # 2 ionic times
    hist = np.zeros((40, 7))
    hist[:, 0] = steps
    hist[:, 4] = 3e-4 * np.exp(-0.4 * steps / t0)
    f = growth_fit(hist, t0)
    assert abs(f["rate"] + 0.4) < 1e-9 and abs(f["r2"] - 1.0) < 1e-12
    assert f["span"] == 2.0 and not f["transient"]
    short = growth_fit(hist, 4 * t0)  # the same rows cover half an ionic time
    assert short["transient"] and short["span"] == 0.5
    rng = np.random.default_rng(1)
    hist[:, 4] = np.exp(rng.standard_normal(40))
    assert growth_fit(hist, t0)["r2"] < 0.5
