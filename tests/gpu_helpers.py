"""Helpers for the GPU parity tests: upload a synthetic workload through the
binding, run the library, run the oracle on the same inputs, compare."""

import numpy as np

import oracle

TOL = 1e-5      # relative Frobenius tolerance on H, b, e per factor (FP32 path vs FP64)


def rel_fro(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(got - ref)
    if den == 0.0:
        return float(num)
    return float(num / den)


class GpuWorkload:
    """Device copies of a synth.Workload plus its maps and factor set."""

    def __init__(self, vg, ctx, w, tile_points=0, factors=None):
        import torch
        self.vg, self.ctx, self.w = vg, ctx, w
        self.src = [vg.cloud_to_device(x, c) for (x, c) in w.sources]
        self.tgt = [vg.cloud_to_device(x, c) for (x, c) in w.targets]
        self.maps = [vg.voxelize(ctx, x, c, w.resolution) for (x, c) in self.tgt]
        self.factors = w.factors if factors is None else factors
        self.fs = vg.FactorSet(ctx, self.src, self.maps, self.factors, w.poses.shape[0], tile_points)
        self.poses = torch.from_numpy(np.ascontiguousarray(w.poses)).to("cuda")

    def linearize(self, **kw):
        out = self.vg.linearize_factors(self.ctx, self.fs, self.poses, **kw)
        self.ctx.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}

    def overlap(self):
        out = self.vg.overlap(self.ctx, self.fs, self.poses)
        self.ctx.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}

    def evaluate(self, **kw):
        out = self.vg.evaluate_errors(self.ctx, self.fs, self.poses, **kw)
        self.ctx.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}


def oracle_results(w, factors=None, with_corr=True):
    maps = oracle.build_maps(w.targets, w.resolution)
    f = w.factors if factors is None else factors
    return maps, oracle.linearize_workload(w.sources, maps, w.poses, f, with_corr=with_corr)


def assert_linearize_parity(got, ref, tol=TOL, factors=None):
    """Inliers bit-exact, H/b/e within `tol` relative Frobenius per factor."""
    F = ref["H"].shape[0]
    assert np.array_equal(got["inliers"], ref["inliers"]), \
        np.flatnonzero(got["inliers"] != ref["inliers"])[:10]
    worst = {"H": 0.0, "b": 0.0, "e": 0.0}
    for f in range(F):
        if ref["inliers"][f] == 0:
            assert not np.any(got["H"][f]) and not np.any(got["b"][f]) and got["e"][f] == 0.0
            continue
        for k in ("H", "b", "e"):
            worst[k] = max(worst[k], rel_fro(got[k][f], ref[k][f]))
    assert worst["H"] <= tol and worst["b"] <= tol and worst["e"] <= tol, worst
    return worst
