"""Host logic of bench.py: the algorithmic byte and flop counts per cell that
its roofline line divides by, the committed traffic figure it reports only
for the kernel source the counters were taken on, and the one-GPU contract."""
import hashlib
import importlib.util
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_per_cell_counts_match_the_stated_figures():
    """FP32 tables, V = 4: 720 / 476 bytes and 11,056 / 6,348 flops per
    quadrilateral / triangle, the figures the kernel notes and the profile
    use.  Bytes by hand, in 4-byte values: S - 1 stencil indices, 2n Gauss
    points x 2 offsets, M candidates x 4 operator entries, 2n x M linear
    weights; then V FP64 state values of 8 bytes."""
    b = _bench()
    assert b.recon_bytes(4, 4, 4) == 4 * (12 + 16 + 48 + 96) + 32 == 720
    assert b.recon_bytes(3, 4, 4) == 4 * (9 + 12 + 36 + 54) + 32 == 476
    assert b.recon_flops(4, 4) == 11056
    assert b.recon_flops(3, 4) == 6348
    # FP64 tables double every table value but the stencil indices
    assert b.recon_bytes(4, 8, 4) == 4 * 12 + 8 * (16 + 48 + 96) + 32
    # the scalar equation reads one state value
    assert b.recon_bytes(3, 4, 1) == 476 - 24


def test_flop_count_scales_with_the_variables_as_the_formulas_do():
    """Per (Gauss point, candidate, variable) the count is the candidate value
    (3) and two signs of 11: the difference between V = 4 and V = 1 is the
    per-variable part only."""
    b = _bench()
    for nf, (S, M) in ((4, (13, 12)), (3, (10, 9))):
        G = 2 * nf
        per_var = (S - 1) + 9 * M + G * M * (3 + 2 * 11) + G * 6
        assert b.recon_flops(nf, 4) - b.recon_flops(nf, 1) == 3 * per_var


def test_committed_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    b = _bench()
    text = open(b.TRAFFIC_PROFILE).read()
    recorded = re.search(r"kernels.hip sha256: `([0-9a-f]{64})`", text).group(1)
    value = float(re.search(r"traffic bytes per pass: `(\d+)`", text).group(1))
    current = hashlib.sha256(open(b.KERNEL_SOURCE, "rb").read()).hexdigest()
    assert b.committed_traffic() == (value if current == recorded else None)
    other = tmp_path / "kernels.hip"
    other.write_bytes(open(b.KERNEL_SOURCE, "rb").read() + b"\n// changed\n")
    monkeypatch.setattr(b, "KERNEL_SOURCE", str(other))
    assert b.committed_traffic() is None
    monkeypatch.setattr(b, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert b.committed_traffic() is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
