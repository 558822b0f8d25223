"""Host-side logic of bench.py that needs no GPU: the provenance check of measured
counter lines (a profile's figures are used only while the kernel's sources hash to
the value recorded with them) and the refusal of more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tree(tmp_path, text):
    csrc = tmp_path / "paper_1004_0024_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.CELL_SOURCES:
        (csrc / name).write_text(f"// {name}\n")
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k.md").write_text(text)
    return csrc


def test_measured_line_used_only_while_sources_match(tmp_path, monkeypatch):
    csrc = _tree(tmp_path, "")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.sources_hash(bench.CELL_SOURCES)
    line = '{"hbm_bytes_per_launch": 1.5e6, "sources_sha256": "%s"}' % h
    (tmp_path / "profiles" / "k.md").write_text(f"# title\n\nmeasured: {line}\n\ntext\n")
    fig, why = bench.measured_counters("E", "k.md", bench.CELL_SOURCES)
    assert why is None and fig["hbm_bytes_per_launch"] == 1.5e6 and fig["source"] == os.path.join("profiles", "k.md")
    (csrc / "cells.hip").write_text("// changed\n")  # the kernel changed since the profile
    fig, why = bench.measured_counters("E", "k.md", bench.CELL_SOURCES)
    assert fig is None and why.startswith("stale:")
    (tmp_path / "profiles" / "k.md").write_text("# no figures\n")
    fig, why = bench.measured_counters("E", "k.md", bench.CELL_SOURCES)
    assert fig is None and "no measured line" in why
    fig, why = bench.measured_counters("E", "missing.md", bench.CELL_SOURCES)
    assert fig is None and why.startswith("no ")


def test_committed_profiles_carry_a_measured_line():
    for name, sources in (("sweep_kernel_B_counters.md", bench.SWEEP_SOURCES),
                          ("cell_propose_kernel_E.md", bench.CELL_SOURCES)):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "\nmeasured: {" in text, name
        fig, why = bench.measured_counters("B", name, sources)
        assert fig is not None or why.startswith("stale:"), why


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_side_by_side_shape_candidates():
    """Threads per walker that the side-by-side refinement tries for a bucket: the
    current count, the powers of two at and below S, and above 64 also S, ceil(S/2)
    and their multiples of 64, within 8..1,024."""
    from paper_1004_0024_amd.tune import _shape_candidates
    assert _shape_candidates({"S": 392, "tpw": 512}) == [196, 256, 392, 448, 512]
    assert _shape_candidates({"S": 288, "tpw": 256}) == [144, 192, 256, 288, 320, 512]
    assert _shape_candidates({"S": 32, "tpw": 64}) == [16, 32, 64]
    assert _shape_candidates({"S": 8, "tpw": 8}) == [8]
    assert _shape_candidates({"S": 2048, "tpw": 1024}) == [1024]
