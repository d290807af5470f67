"""Byte accounting against the figures the paper prints."""

import math
import os

from paper_1611_02665_amd import accounting as A

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_byte_accounting.txt")


def _golden():
    tiles, facts = [], {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b = line.split()
        if a.isdigit():
            tiles.append((int(a), int(b)))
        else:
            facts[a] = int(b)
    return tiles, facts


def test_tile_working_set_matches_paper():
    tiles, _ = _golden()
    ng = 48**3
    for nb, mb in tiles:
        got = A.tile_working_set_bytes(ng, nb) / 1e6
        # the paper rounds to the megabyte ("roughly 28MB", "7MB")
        assert abs(got - mb) < 1.0, (nb, got, mb)


def test_per_position_traffic_matches_paper():
    _, facts = _golden()
    n = 2048
    assert A.bytes_per_eval("vgh", "f32") * n == (facts["reads_per_position_per_spline"] * 4
                                                  + facts["vgh_soa_writes_per_spline"] * 4) * n
    assert A.NOUT["vgh"] == facts["vgh_soa_writes_per_spline"]
    assert 1 + 3 + 9 == facts["vgh_aos_outputs_per_spline"]


def test_bytes_per_eval_table():
    assert A.bytes_per_eval("vgh", "f32") == 296
    assert A.bytes_per_eval("vgl", "f32") == 276
    assert A.bytes_per_eval("v", "f32") == 260
    assert A.bytes_per_eval("vgh", "f16") == 168
    assert A.bytes_per_eval("vgl", "bf16") == 148
    assert A.bytes_per_eval("v", "f16") == 132
    # roofline at 8 TB/s: 2.70e10 FP32 VGH evals/s
    assert abs(A.roofline_evals_per_s("vgh", "f32") - 2.7027e10) < 1e7


def test_unique_row_fraction():
    # 512 positions on the 51^3 padded grid: lambda = 0.247 -> 0.886
    f = A.unique_row_fraction(512, 51**3)
    assert abs(f - 0.886) < 0.002
    lam = 64 * 4096 / 51**3
    assert math.isclose(A.unique_row_fraction(4096, 51**3), (1 - math.exp(-lam)) / lam)
