"""Host-side checks of bench.py: the helpers the default run calls exist and
work without a GPU (the oracle baseline leg, the counter-summary parser)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_oracle_baseline_small(monkeypatch):
    """The oracle timing of the default run's baseline leg on a 64 x 64
    stand-in of its workload."""
    import oracle
    from paper_2108_04315_amd import synth
    monkeypatch.setattr(bench, "H", 64)
    monkeypatch.setattr(bench, "W", 64)
    monkeypatch.setattr(bench, "N_ITER", 4)
    s = bench.S
    shifts = synth.frame_shifts(s, 4, 0.05, 1)
    psf = synth.psf_taps(0.8)
    y = synth.add_poisson_noise(oracle.forward(synth.phantom(64, 64, 0), shifts, psf, s), 1e4, 2)
    x0 = synth.bicubic_upsample(y[0], s)
    out, x_o, tr = bench.oracle_baseline(y, x0, shifts, psf, n_one=1)
    assert out["kind"] == "oracle" and out["unit"] == "HR Mpixel/s"
    assert out["value"] > 0 and out["cores"] >= 1 and "4-pass" in out["sample"]
    assert out["single_thread"]["passes"] == 1 and len(tr) == 4 and x_o.shape == (64, 64)


def test_profile_values_follow_the_kernel_hash():
    """traffic / VALU figures are reported only for the kernel sources the
    committed summaries were taken on."""
    h = bench.kernel_source_hash()
    for path, tag, key in ((bench.TRAFFIC_SUMMARY, "traffic", "bytes_per_launch"),
                           (bench.SQ_SUMMARY, "valu", "insts_per_launch")):
        assert os.path.exists(path)
        for variant in (0, 1, 2):
            assert bench.profile_value(path, tag, key, "0" * 16, variant) is None
            v = bench.profile_value(path, tag, key, h, variant)
            assert v is None or (np.isfinite(v) and v > 0)
        assert bench.profile_value(path, tag, key, h, 7) is None


def test_profile_value_selects_the_variant(tmp_path):
    p = tmp_path / "summary.md"
    p.write_text("text\ntraffic: kernel_source_hash=abc variant=0 bytes_per_launch=10\n"
                 "traffic: kernel_source_hash=abc variant=2 bytes_per_launch=12\n"
                 "traffic: kernel_source_hash=old variant=1 bytes_per_launch=99\n")
    f = bench.profile_value
    assert f(str(p), "traffic", "bytes_per_launch", "abc", 0) == 10
    assert f(str(p), "traffic", "bytes_per_launch", "abc", 2) == 12
    assert f(str(p), "traffic", "bytes_per_launch", "abc", 1) is None
    assert f(str(p), "traffic", "bytes_per_launch", "old", 1) == 99
    assert f(str(p), "valu", "bytes_per_launch", "abc", 0) is None


def test_main_refuses_more_than_one_gpu(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    try:
        bench.main()
    except SystemExit as e:
        assert e.code not in (0, None)
    else:
        raise AssertionError("bench.py --gpus 2 must exit")
