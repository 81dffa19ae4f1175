"""Host checks of bench.py (no GPU): the command line's one-GPU limit, the roofline
arithmetic of the algorithmic models, and the profiles' source digest."""
import math
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "GPU" in r.stderr or "GPU" in r.stdout


def _plan_like():
    info = {"mid_Pw": [7, 7, 7], "mid_I": [280, 280, 274], "mid_Izs": 576, "rc": 3.25}
    sizes = {"mid_zband": [100, 384], "near_degree": 14}
    return info, sizes


def test_near_model_counts_pairs_within_rc():
    info, sizes = _plan_like()
    N, box = 10 ** 6, (100.0, 100.0, 100.0)
    m = bench.kernel_models(info, sizes, N, box, 4)
    pairs = N * 4.0 / 3.0 * math.pi * 3.25 ** 3 * (N / 1e6)
    assert m["near"]["flops"] == pytest.approx(pairs * bench.NEAR_FLOPS_PER_PAIR)
    assert m["near"]["bound"] == "alu"
    # the FFT passes are priced by bytes: the y pass reads and writes the half spectrum
    cg = 280 * 280 * (576 // 2 + 1) * 2 * 4
    assert m["fft_y_fwd"]["bytes"] == 2 * cg and m["fft_y_fwd"]["bound"] == "hbm"


def test_roofline_fraction_is_achieved_over_published_peak():
    alu = bench.roofline_of({"bound": "alu", "flops": 4.3e9, "bytes": 0}, 0.75e-3)
    assert alu["peak"] == 157.3 and alu["unit"] == "TFLOP/s"
    assert alu["achieved"] == pytest.approx(4.3e9 / 0.75e-3 / 1e12)
    assert alu["frac"] == pytest.approx(alu["achieved"] / 157.3)
    assert alu["frac_nonpacked"] == pytest.approx(alu["achieved"] / 78.6)
    f64 = bench.roofline_of({"bound": "alu", "flops": 4.3e9, "bytes": 0}, 1.4e-3, fp64=True)
    assert f64["peak"] == 78.6 and "frac_nonpacked" not in f64
    hbm = bench.roofline_of({"bound": "hbm", "flops": None, "bytes": 3.7e8}, 0.1e-3)
    assert hbm["unit"] == "GB/s" and hbm["peak"] == 8000.0
    assert hbm["frac"] == pytest.approx(3.7e8 / 0.1e-3 / 1e9 / 8000.0)


def test_spread_gather_hbm_uses_particles_and_grid_points():
    info, sizes = _plan_like()
    N = 10 ** 6
    r = bench.spread_gather_hbm(info, sizes, N, {"mid_spread": 0.4, "mid_gather": 0.2}, 4)
    Ng = 280 * 280 * 576
    assert r["algorithmic_bytes"] == N * 32 + 2 * Ng * 4
    assert r["achieved"] == pytest.approx(r["algorithmic_bytes"] / 0.6e-3 / 1e9)
    assert r["band"]["algorithmic_bytes"] == N * 32 + 2 * 280 * 280 * 284 * 4
    assert bench.spread_gather_hbm(info, sizes, N, {"mid_spread": 0.4}, 4) is None


def test_source_digest_ignores_comments_and_follows_code(tmp_path):
    src = os.path.join(ROOT, "paper_2412_04595_amd", "csrc")
    dst = tmp_path / "paper_2412_04595_amd" / "csrc"
    shutil.copytree(src, dst)
    old_root = bench.ROOT
    try:
        d_repo = bench.source_digest()
        bench.ROOT = str(tmp_path)
        d0 = bench.source_digest()
        assert d0 == d_repo
        f = dst / "k_misc.hip"
        text = f.read_text()
        f.write_text("// a new comment line\n" + text.replace("\n", "\n  ", 1) + "\n/* and a block\n comment */\n")
        assert bench.source_digest() == d0
        f.write_text(text + "\nnamespace { constexpr int kUnusedForTheDigest = 1; }\n")
        assert bench.source_digest() != d0
    finally:
        bench.ROOT = old_root
