"""The C ABI used from plain C (tests/c_abi_demo.c, built by the build
step with gcc against libbspline.so and the HIP runtime, no Python or
PyTorch in the process): VGH at random positions against the oracle, and
inside the program a spline-blocked copy of the table and a batch plan over
both (graph replay and direct launches), byte for byte."""

import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEMO = os.path.join(os.path.dirname(__file__), "c_abi_demo")


def test_c_program_matches_oracle(tmp_path):
    if not os.path.exists(DEMO):
        pytest.fail("tests/c_abi_demo is not built (run the build step)")
    dims, n, npos = (11, 9, 13), 600, 64  # 600 splines: three blocks of 256
    coef = synth.coef_table(*dims, n, stream=160)
    pos = synth.positions(npos, stream=161) * 3 - 1
    coef.tofile(tmp_path / "coef.bin")
    np.ascontiguousarray(pos).tofile(tmp_path / "pos.bin")
    out_path = tmp_path / "out.bin"
    r = subprocess.run([DEMO, *map(str, dims), str(n), str(npos), str(tmp_path / "coef.bin"),
                        str(tmp_path / "pos.bin"), str(out_path)],
                       capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "spline-blocked table: identical outputs" in r.stdout
    assert "batch plan over both tables" in r.stdout
    out = np.fromfile(out_path, dtype=np.float32).astype(np.float64)
    v = out[:npos * n].reshape(npos, n)
    g = out[npos * n:npos * n * 4].reshape(npos, 3, n)
    h = out[npos * n * 4:].reshape(npos, 6, n)
    assert_close("vgh", {"v": v, "g": g, "h": h}, oracle.evaluate("vgh", coef, pos),
                 label="plain C")
