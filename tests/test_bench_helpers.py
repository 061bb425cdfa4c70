"""Host-side helpers of bench.py: the algorithmic byte and op counts its
roofline figures divide by, and the rule that a committed per-launch traffic
figure is reported only while the kernel sources it was measured on are
unchanged."""
import hashlib
import os
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def cls(**kw):
    base = dict(fp64=0, n=60, n_inst=10, n_points=76800, method=3, epi_fused=1, degree=7,
                series_terms=0, fallback_points=0)
    base.update(kw)
    return SimpleNamespace(**base)


def test_spread_fft_bytes_counts_each_stream_once():
    strain, stat, K = 1000, 30, 30
    fused = cls()
    # fused cell runs: strain once, statistic, power rows written and read back
    assert bench.spread_fft_bytes([fused], strain, stat, K) == strain + stat * 4 + 2 * 10 * K * 4
    # a separate FFT kernel adds the grid written by the spreader and read back
    sep = cls(epi_fused=0)
    assert bench.spread_fft_bytes([sep], strain, stat, K) == strain + stat * 4 + 2 * 10 * K * 4 + 2 * 10 * 60 * 8
    # staged classes also read their point stream (8 B per sample in FP32, 16 in FP64)
    st = cls(method=1, epi_fused=0, fp64=1)
    assert bench.spread_fft_bytes([st], strain, stat, K) == (strain + stat * 4 + 2 * 10 * K * 4 +
                                                              2 * 10 * 60 * 16 + 76800 * 16)


def test_algorithmic_ops_per_sample():
    # series of degree 9 (series_terms sums the degrees; degree + 1 FMAs per
    # point) and moments of degree 7: 10 + 6 + 2 + 13 + 2 + (3 * 7 + 1) = 55
    # lane-operations per sample
    c = cls(n_points=1000, series_terms=9 * 1000)
    assert bench.algorithmic_ops([c]) == 1000 * 55
    # log1p/expm1 points cost 40 instead of the series
    c = cls(n_points=1000, series_terms=9 * 900, fallback_points=100)
    assert bench.algorithmic_ops([c]) == 900 * 10 + 100 * 40 + 1000 * 45


def test_committed_traffic_follows_the_sources(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "kernel.hip"
    src.write_text("kernel v1\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "k.md").write_text(
        "# summary\n\ntraffic_bytes_per_launch[nr::k<float>]: 123456\n"
        "valu_instructions_per_launch[nr::k<float>]: 789\n"
        f"source_sha256: {digest}\nsources: kernel.hip\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.committed_traffic("nr::k<float>") == 123456
    assert bench.committed_counter("nr::k<float>", "valu_instructions_per_launch") == 789
    assert bench.committed_traffic("nr::other<float>") is None
    src.write_text("kernel v2\n")                    # the kernel changed since the counters were taken
    assert bench.committed_traffic("nr::k<float>") is None
    assert bench.committed_counter("nr::k<float>", "valu_instructions_per_launch") is None


def test_committed_records_ignore_prose(tmp_path, monkeypatch):
    """Only lines that start with the record names count: prose that happens
    to contain "sources:" does not hide the record."""
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "kernel.hip"
    src.write_text("kernel\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "k.md").write_text(
        "# summary\n\nmeasured on the earlier sources: other.hip, not these\n\n"
        "valu_instructions_per_launch[w:nr::k<float>]: 42\n"
        f"source_sha256: {digest}\nsources: kernel.hip\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.committed_counter("w:nr::k<float>", "valu_instructions_per_launch") == 42


@pytest.mark.parametrize("key", ["nr::spread_runs_kernel<float, 7, false>", "gather_kernel<1, false>"])
def test_committed_profiles_name_their_sources(key):
    """Every committed traffic record names sources that exist, so the check
    above can run on it."""
    import glob
    import re
    found = False
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        txt = open(path).read()
        m = re.search(r"traffic_bytes_per_launch\[(.+?)\]: (\d+)", txt)
        if m and m.group(1) == key:
            found = True
            srcs = re.search(r"sources: (.+)", txt).group(1).split()
            assert srcs and all(os.path.exists(os.path.join(ROOT, s)) for s in srcs)
            assert re.search(r"source_sha256: [0-9a-f]{64}", txt)
    assert found
