"""Parity at full size (GPU): the 4,500-factor round of 1,000 corridor frames
(1.016e8 source points) in the launch configuration the bench times (tuned
tile, HIP graph replay on a side stream).

The oracle cannot linearize every factor in a test's time, so
  * a seeded sample of 40 factors is compared with the oracle (inliers and
    correspondences bit-exact, every block of H and b, the elementwise
    metric and e within 1e-5);
  * over all factors: the overlap hits equal the inliers bit for bit, the
    cost-only kernel gives the same e, H is exactly symmetric with no negative
    diagonal, e >= 0, and a factor without inliers is exactly zero;
  * repeated replays are bit-identical.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_helpers import assert_linearize_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    import bench
    return bench.build_workload("batched4500")


def test_batched4500_round(full):
    import torch
    from paper_2109_07073_amd import vgicp as vg
    w = full
    stream = torch.cuda.Stream()
    ctx = vg.Context(0, stream=stream)
    with torch.cuda.stream(stream):
        src, _ = vg.clouds_to_device(w.sources)
        tgt, _ = vg.clouds_to_device(w.targets)
        maps = [vg.voxelize(ctx, x, c, w.resolution) for (x, c) in tgt]
        fs = vg.FactorSet(ctx, src, maps, w.factors, w.poses.shape[0])
        poses = torch.from_numpy(np.ascontiguousarray(w.poses)).to("cuda")
        tile, _ = vg.tune_tiles(ctx, fs, poses)
        out = vg.linearize_factors(ctx, fs, poses)
        vg.linearize_factors(ctx, fs, poses, use_graph=True, out=out)
        first = {k: v.clone() for k, v in out.items()}
        for _ in range(3):
            vg.linearize_factors(ctx, fs, poses, use_graph=True, out=out)
        ev = vg.evaluate_errors(ctx, fs, poses)
        vg.evaluate_errors(ctx, fs, poses, use_graph=True, out=ev)
        ov = vg.overlap(ctx, fs, poses)
    stream.synchronize()
    print("tile", tile, "form", vg.form_of(fs), "factors", fs.n_factors, "tiles", fs.n_tiles)
    for k in out:
        assert torch.equal(first[k], out[k]), k
    H = out["H"].cpu().numpy()
    b = out["b"].cpu().numpy()
    e = out["e"].cpu().numpy()
    inl = out["inliers"].cpu().numpy()
    assert np.array_equal(ov["hits"].cpu().numpy(), inl)
    if vg.form_of(fs) == "source":   # the cost kernel sums as the source-frame form does
        assert np.array_equal(ev["e"].cpu().numpy(), e)
    else:
        assert np.allclose(ev["e"].cpu().numpy(), e, rtol=1e-6, atol=0.0)
    assert np.array_equal(ev["inliers"].cpu().numpy(), inl)
    assert np.array_equal(H, np.transpose(H, (0, 2, 1)))
    assert np.all(np.diagonal(H, axis1=1, axis2=2) >= 0) and np.all(e >= 0)
    zero = inl == 0
    assert not H[zero].any() and not b[zero].any() and not e[zero].any()
    assert inl.sum() > 0.3 * fs.total_points

    # a seeded sample against the oracle, with correspondences
    ids = np.sort(np.random.default_rng(11).choice(w.n_factors, 40, replace=False))
    with torch.cuda.stream(stream):
        outc = vg.linearize_factors(ctx, fs, poses, with_corr=True)
    stream.synchronize()
    corr = outc["corr"].cpu().numpy()
    offs = np.concatenate([[0], np.cumsum(fs.source_sizes)])
    vmaps = {}
    refs = {"H": [], "b": [], "e": [], "inliers": []}
    for f in ids:
        s, t, pi, pj = w.factors[f]
        if t not in vmaps:
            vmaps[t] = oracle.voxelize(*w.targets[t], w.resolution)[0]
        ref = oracle.linearize_factor(*w.sources[s], vmaps[t], w.poses[pi], w.poses[pj])
        assert inl[f] == ref["inliers"]
        assert np.array_equal(corr[offs[f]:offs[f + 1]], ref["corr"])
        for k in refs:
            refs[k].append(ref[k])
    refs = {k: np.array(v) for k, v in refs.items()}
    got = {"H": H[ids], "b": b[ids], "e": e[ids], "inliers": inl[ids]}
    worst = assert_linearize_parity(got, refs)
    print("sampled worst errors", {k: f"{v[0]:.2e}" for k, v in worst.items()})
