"""The memory-ceiling probe (spline_stream_probe): every unit's written word
is the sum of its six read words, in every read pattern and launch shape.
The inputs are small integers, so the check is exact."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_02665_amd import binding as B  # noqa: E402


def _expected(src, units, flags, salt):
    """The probe's sums restated on the host (the random mode draws spans with
    the published SplitMix64 finaliser of (span * golden gamma + salt))."""
    w = src.reshape(-1, 4).astype(np.int64)
    i = np.arange(units, dtype=np.int64)
    if flags & (B.BSPL_PROBE_CHUNKED | B.BSPL_PROBE_RANDOM):
        span = i >> 6
        if flags & B.BSPL_PROBE_RANDOM:
            m = (1 << 64) - 1
            z = (span.astype(object) * 0x9E3779B97F4A7C15 + salt) & m
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
            z = z ^ (z >> 31)
            span = np.array([int(x) % (units >> 6) for x in z], dtype=np.int64)
        idx = [span * 384 + j * 64 + (i & 63) for j in range(6)]
    else:
        idx = [j * units + i for j in range(6)]
    return sum(w[k] for k in idx) & 0xFFFFFFFF


@pytest.mark.parametrize("flags", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("per_lane,grid", [(1, 0), (2, 0), (4, 0), (1, 7), (4, 3)])
def test_probe_sums(flags, per_lane, grid):
    units = 64 * 97
    rng = np.random.default_rng(flags * 10 + per_lane)
    src = rng.integers(0, 1 << 20, size=6 * units * 4, dtype=np.int64).astype(np.int32)
    s = torch.from_numpy(src).cuda()
    d = torch.full((units * 4,), -1, dtype=torch.int32, device="cuda")
    salt = 12345 + flags
    B.spline_stream_probe(s, d, units, per_lane, grid, flags, salt)
    torch.cuda.synchronize()
    got = d.cpu().numpy().astype(np.int64).reshape(-1, 4) & 0xFFFFFFFF
    want = _expected(src, units, flags, salt)
    assert np.array_equal(got, want)
