"""Host logic of bench.py (CPU): the unit counts and the arithmetic behind the
roofline it reports.

The pair kernel's fraction of the issue peak divides its algorithmic work by
the number of (target, source) pairs within r_c, which bench.py takes from a
closed form for uniform density (expected_real_pairs).  Here that number is
checked against a brute-force count of real and first-image neighbours on the
benchmark's own seeded input, and the roofline block against its definition.
"""
import math
import os
import sys

import numpy as np
import pytest
from scipy.spatial import cKDTree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2405_06333_amd import inputs  # noqa: E402


def counted_pairs(w, n_targets, seed):
    """N times the mean number of sources within r_c of a sampled target:
    real charges (minimum image in x and y, the target itself excluded) plus
    the first-order images, i.e. sources within r_c of the target reflected
    in z = 0 and in z = H (Sec. 3.1; higher orders lie beyond r_c when
    H > r_c), the target's own image included."""
    assert w.H > w.r_c
    pos, _ = inputs.sample(w)
    # z is not periodic: a period of 4 H exceeds every distance that matters
    box = [w.Lx, w.Ly, 4.0 * w.H]
    tree = cKDTree(np.c_[pos[:, 0] % w.Lx, pos[:, 1] % w.Ly, pos[:, 2] + w.H], boxsize=box)
    rng = np.random.default_rng(seed)
    idx = rng.choice(w.N, n_targets, replace=False)
    t = pos[idx].copy()
    t[:, 0] %= w.Lx
    t[:, 1] %= w.Ly
    total = 0
    for zmap in (lambda z: z, lambda z: -z, lambda z: 2.0 * w.H - z):
        q = np.c_[t[:, 0], t[:, 1], zmap(t[:, 2]) + w.H]
        total += sum(len(x) for x in tree.query_ball_point(q, w.r_c * (1.0 - 1e-12)))
    total -= n_targets   # each target finds itself among the real sources
    return w.N * total / n_targets


def test_expected_real_pairs_matches_count():
    w = inputs.LARGE_MD
    expected = bench.expected_real_pairs(w)
    counted = counted_pairs(w, 4000, seed=11)
    # per-target counts vary by ~40 with height: the sample mean is good to ~0.5 %
    assert abs(counted - expected) <= 0.02 * expected, (counted, expected)
    # the closed form itself: 164 pairs per ion on this slab, images included
    assert 160 < expected / w.N < 168


def test_expected_real_pairs_of_the_replica_batch():
    """The 64-replica batch's pair count (the batch roofline's unit) is the sum
    of the replicas' closed forms; checked on every replica against the count
    over all of its ions (thin slabs, H = 10 < 2 r_c, where both faces cut
    most spheres)."""
    ws = inputs.replicas()
    expected = sum(bench.expected_real_pairs(w) for w in ws)
    counted = sum(counted_pairs(w, min(w.N, 2000), seed=12) for w in ws)
    assert abs(counted - expected) <= 0.005 * expected, (counted, expected)


def test_expected_real_pairs_is_not_the_full_sphere():
    """The slab's faces cut the spheres: fewer pairs than the unbounded
    4/3 pi r_c^3 rho; with the faces far away, the full sphere plus the few
    targets within r_c / 2 of a face that meet their own image."""
    w = inputs.LARGE_MD
    rho = w.N / (w.Lx * w.Ly * (w.H - 2 * w.margin))
    assert bench.expected_real_pairs(w) < rho * w.N * 4.0 / 3.0 * math.pi * w.r_c ** 3
    far = w.with_(H=1e6 * w.H)
    span = far.H - 2 * far.margin
    sphere = far.N / (far.Lx * far.Ly * span) * far.N * 4.0 / 3.0 * math.pi * far.r_c ** 3
    own = far.N * 2.0 * (0.5 * far.r_c - far.margin) / span
    assert bench.expected_real_pairs(far) == pytest.approx(sphere + own, rel=2e-4)


def test_roofline_block_definition():
    """frac = algorithmic slots per unit x units / duration / lane-slot peak,
    with the dominant kernel's duration from the breakdown or given live."""
    NP, pairs = 5.0e8, 1.638e8
    breakdown = {"sf_pass": (3.0, 10), "force_scatter": (2.0, 10), "real_pairs": (8.0, 10),
                 "cell_build": (1.0, 10)}
    roof, fr = bench.roofline_of(breakdown, "fp32", NP, pairs)
    assert roof["kernel"] == "real_pairs"
    want = bench.SLOTS_REAL * pairs / 0.8e-3 / bench.VALU_LANE_SLOTS
    assert roof["frac"] == pytest.approx(want, abs=1e-4)
    assert roof["peak"] == pytest.approx(256 * 64 * 2.4e9 / 1e12, rel=1e-3)
    assert fr["sf_pass"]["valu_frac"] == pytest.approx(bench.SLOTS_SF * NP / 0.3e-3 / bench.VALU_LANE_SLOTS,
                                                       abs=1e-4)
    # a live duration replaces the breakdown's
    roof2, _ = bench.roofline_of(breakdown, "fp32", NP, pairs, dom="real_pairs", t_dom=1.0e-3)
    assert roof2["frac"] == pytest.approx(bench.SLOTS_REAL * pairs / 1.0e-3 / bench.VALU_LANE_SLOTS, abs=1e-4)


def test_traffic_figure_only_for_the_sources_it_was_measured_on(tmp_path, monkeypatch):
    """roofline.traffic comes from the committed counter summary only while
    the pair kernel's sources hash to the value recorded with it."""
    good = tmp_path / "good.txt"
    good.write_text("bench_kernel: real_pairs\nsource_sha256: %s\ntraffic_bytes_per_launch: 1234\n"
                    % bench.kernel_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.measured_traffic("real_pairs") == 1234.0
    assert bench.measured_traffic("sf_pass") is None          # recorded for another kernel
    stale = tmp_path / "stale.txt"
    stale.write_text("bench_kernel: real_pairs\nsource_sha256: %s\ntraffic_bytes_per_launch: 1234\n" % ("0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic("real_pairs") is None       # other kernel sources
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("real_pairs") is None

