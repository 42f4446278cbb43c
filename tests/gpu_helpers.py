"""Helpers for the GPU parity tests: upload a synthetic workload through the
binding, run the library, run the oracle on the same inputs, compare."""

import numpy as np

import oracle

TOL = 1e-5      # relative tolerance on every block of H and b, and on e, per factor (FP32 path vs FP64)

# Tolerance of the opt-in all-FP32 fused covariance (fused="f32").  With
# covariances regularized to (1, 1, 1e-3), F' of a surface point has
# eigenvalues near (2, 2, 2e-3); forming it in FP32 perturbs its entries by
# about 2^-24 * |F'| ~ 1.2e-7, the small eigenvalue by ~6e-5 of itself, and so
# the weight along the normal by up to ~1e-4 relative, point by point.  Block
# and elementwise errors of a small factor reach a few 1e-5; 2e-4 bounds them.
FUSED32_TOL = 2e-4

# Elementwise tolerance of the plain FP32 accumulation (accum="f32"): a tile's
# 256 lane sums pass through a six-level FP32 DPP tree and an FP32 sum over 4
# waves, each level rounding at 2^-24 of the partial sum.  An entry whose
# terms cancel down to the metric's floor (1e-3 of the factor's largest entry)
# carries that rounding amplified up to 1e3 times: about sqrt(8) * 6e-8 * 1e3
# = 1.7e-4 at worst.  The compensated and FP64 accumulations stay at TOL.
ACC32_ELEM_TOL = 1e-4


def elem_tol_for(accum):
    """Elementwise tolerance for an accumulation variant (None: TOL)."""
    return ACC32_ELEM_TOL if accum == "f32" else None

# Sub-blocks of the 12x12 Hessian factor and the 12-vector b in the order
# [omega_i, rho_i, omega_j, rho_j]: each 6x6 block of H split into its
# rotation (w) and translation (r) parts.  The (w, w) blocks scale with |mu|^2
# (10^2 - 10^3 m^2 at 10 - 40 m), so a norm over the whole factor would hide
# an error confined to the (r, r) or cross blocks.
_W_I, _R_I, _W_J, _R_J = slice(0, 3), slice(3, 6), slice(6, 9), slice(9, 12)
H_BLOCKS = {
    "Hii_ww": (_W_I, _W_I), "Hii_wr": (_W_I, _R_I), "Hii_rr": (_R_I, _R_I),
    "Hij_ww": (_W_I, _W_J), "Hij_wr": (_W_I, _R_J), "Hij_rw": (_R_I, _W_J), "Hij_rr": (_R_I, _R_J),
    "Hjj_ww": (_W_J, _W_J), "Hjj_wr": (_W_J, _R_J), "Hjj_rr": (_R_J, _R_J),
}
B_BLOCKS = {"bi_w": _W_I, "bi_r": _R_I, "bj_w": _W_J, "bj_r": _R_J}
ELEM_FLOOR = 1e-3   # elementwise metric |d| / (|ref| + ELEM_FLOOR * max|ref|)


def rel_fro(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(got - ref)
    if den == 0.0:
        return float(num)
    return float(num / den)


def elementwise(got, ref):
    """max |got - ref| / (|ref| + ELEM_FLOOR * max|ref|) over the entries."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    if scale == 0.0:
        return float(np.abs(got - ref).max()) if got.size else 0.0
    return float((np.abs(got - ref) / (np.abs(ref) + ELEM_FLOOR * scale)).max())


def factor_errors(H, b, e, Hr, br, er):
    """Every error metric of one factor against its reference: relative
    Frobenius error of each H and b sub-block, the elementwise metric of H
    and of b, the whole-factor norms and the relative error of e."""
    out = {k: rel_fro(H[r, c], Hr[r, c]) for k, (r, c) in H_BLOCKS.items()}
    out.update({k: rel_fro(b[r], br[r]) for k, r in B_BLOCKS.items()})
    out["H_elem"] = elementwise(H, Hr)
    out["b_elem"] = elementwise(b, br)
    out["H"] = rel_fro(H, Hr)
    out["b"] = rel_fro(b, br)
    out["e"] = abs(float(e) - float(er)) / abs(float(er)) if er != 0 else abs(float(e))
    return out


def worst_errors(got, ref, factors=None):
    """Worst of every metric over the factors with inliers, and the factor
    where it occurs: {metric: (error, factor)}."""
    idx = range(ref["H"].shape[0]) if factors is None else factors
    worst = {}
    for f in idx:
        if ref["inliers"][f] == 0:
            continue
        errs = factor_errors(got["H"][f], got["b"][f], got["e"][f], ref["H"][f], ref["b"][f],
                             ref["e"][f])
        for k, v in errs.items():
            if k not in worst or v > worst[k][0]:
                worst[k] = (v, int(f))
    return worst


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


def assert_linearize_parity(got, ref, tol=TOL, factors=None, elem_tol=None):
    """Inliers bit-exact; factors without inliers exactly zero; every H and b
    sub-block, the elementwise metric and e within `tol` of the FP64 oracle
    per factor (the elementwise metric within `elem_tol` when given).
    Returns {metric: (worst error, factor)} and prints the worst block."""
    F = ref["H"].shape[0]
    idx = range(F) if factors is None else factors
    assert np.array_equal(np.asarray(got["inliers"])[list(idx)], np.asarray(ref["inliers"])[list(idx)]), \
        np.flatnonzero(np.asarray(got["inliers"])[list(idx)] != np.asarray(ref["inliers"])[list(idx)])[:10]
    for f in idx:
        if ref["inliers"][f] == 0:
            assert not np.any(got["H"][f]) and not np.any(got["b"][f]) and got["e"][f] == 0.0
    worst = worst_errors(got, ref, idx)
    if worst:
        k = max(worst, key=lambda m: worst[m][0])
        print(f"worst metric {k} = {worst[k][0]:.3e} (factor {worst[k][1]}); "
              f"H {worst['H'][0]:.2e}, b {worst['b'][0]:.2e}, e {worst['e'][0]:.2e}")
    lim = {k: (elem_tol if elem_tol is not None and k.endswith("_elem") else tol) for k in worst}
    bad = {k: v for k, v in worst.items() if not v[0] <= lim[k]}
    assert not bad, bad
    return worst
