"""The C ABI end to end from a plain C program on the GPU (no PyTorch in the
process): tests/c/vgicp_example.c allocates with hipMalloc, voxelizes the
target, binds one factor, linearizes it and evaluates its overlap.  The
single-factor workload (2,000 x 2,000 points) is checked against the FP64
oracle: inliers and overlap hits exact, every block of H and b, the
elementwise metric and e within 1e-5."""

import os
import subprocess

import numpy as np
import pytest

import oracle
from synth import make_single_factor
from tests.gpu_helpers import TOL, factor_errors

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "tests", "c", "vgicp_example")


def test_plain_c_client_linearizes_one_factor(tmp_path):
    w = make_single_factor()
    (sx, sc), (tx, tc) = w.sources[0], w.targets[0]
    ns, nt = sx.shape[0], tx.shape[0]
    blob = b"".join([
        np.array([ns, nt], np.int64).tobytes(),
        np.array([w.resolution], np.float64).tobytes(),
        np.ascontiguousarray(w.poses, np.float64).tobytes(),
        np.ascontiguousarray(sx.T, np.float32).tobytes(), np.ascontiguousarray(sc, np.float32).tobytes(),
        np.ascontiguousarray(tx.T, np.float32).tobytes(), np.ascontiguousarray(tc, np.float32).tobytes(),
    ])
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    inp.write_bytes(blob)
    print("running", EXAMPLE, flush=True)
    r = subprocess.run([EXAMPLE, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = out.read_bytes()
    d = np.frombuffer(raw[:157 * 8], np.float64)
    inl, hits = np.frombuffer(raw[157 * 8:159 * 8], np.int64)
    ovl = np.frombuffer(raw[159 * 8:], np.float64)[0]
    H, b, e = d[:144].reshape(12, 12), d[144:156], d[156]
    vmap, _ = oracle.voxelize(tx, tc, w.resolution)
    ref = oracle.linearize_factor(sx, sc, vmap, w.poses[0], w.poses[1])
    assert inl == ref["inliers"] and hits == inl
    assert ovl == inl / ns
    errs = factor_errors(H, b, e, ref["H"], ref["b"], ref["e"])
    print("C client errors", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= TOL, errs
