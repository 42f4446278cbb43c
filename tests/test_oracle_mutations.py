"""Planted mistakes in the oracle (CPU only): every plausible slip in the
oracle's arithmetic must make at least one independent pin fail.  The
mistakes are patched into the oracle module for the duration of one test."""

import json
import os

import numpy as np
import pytest

import oracle
from oracle import vgicp_oracle as vo
from synth import make_tiny_workload
from tests.oracle_pins import (fd_hessian_factor, hom, icp_normal_equations,
                               null_space_basis, rel_err)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pins_hold() -> bool:
    """Run the pins on a tiny workload; False as soon as one fails."""
    w = make_tiny_workload(seed=11, n_src=300, n_tgt=500, resolution=0.5)
    xyz, cov = w.sources[0]
    pi, pj = w.poses[0], w.poses[1]
    try:
        vm, _ = oracle.voxelize(*w.targets[0], w.resolution)
        # voxel means against plain averaging of each group
        _, inv = oracle.voxelize(*w.targets[0], w.resolution)
        txyz = w.targets[0][0].astype(np.float64)
        for o in range(0, vm.n_voxels, 7):
            m = txyz[inv == o].mean(0)
            assert np.allclose(vm.mean[o], m, rtol=1e-6, atol=1e-6)
        # FP32 fused multiply-add: (1 + 2^-24) + 2^-80 lies just above the
        # midpoint of 1 and 1 + 2^-23, so it rounds up
        a, b = np.float32(24929 * 2.0 ** -12), np.float32(673 * 2.0 ** -12)
        assert vo.fma32(a, b, np.float32(2.0 ** -80)) == np.float32(1 + 2.0 ** -23)
        assert vo.fma32(a, b, np.float32(-(2.0 ** -80))) == np.float32(1.0)
        # correspondences against the exact motion and a box scan
        R, t = oracle.relative_pose(pi, pj)
        corr = oracle.lookup(vm, xyz, R, t)
        T = np.linalg.inv(hom(pj)) @ hom(pi)
        q64 = xyz.astype(np.float64) @ T[:3, :3].T + T[:3, 3]
        lo = vm.keys * w.resolution
        inside = np.all((q64[:, None] >= lo[None] - 1e-4) & (q64[:, None] < lo[None] + w.resolution + 1e-4), 2)
        assert all(inside[k, c] for k, c in enumerate(corr) if c >= 0)
        # finite differences
        fd = fd_hessian_factor(xyz, cov, vm, pi, pj)
        out = fd["oracle"]
        assert rel_err(out["H"], fd["H"]) < 1e-7 and rel_err(out["b"], fd["b"]) < 1e-7
        assert abs(out["e"] - fd["e"]) <= 1e-10 * abs(fd["e"])
        # gauge null space
        N = null_space_basis(pi, pj)
        assert np.linalg.norm(out["H"] @ N) <= 1e-9 * np.linalg.norm(out["H"]) * np.linalg.norm(N)
        # isotropic closed form
        s2, t2 = 0.5, 0.25
        cs = np.tile(np.array([s2, 0, 0, s2, 0, s2], np.float32), (xyz.shape[0], 1))
        ct = np.tile(np.array([t2, 0, 0, t2, 0, t2], np.float32), (w.targets[0][0].shape[0], 1))
        vmi, _ = oracle.voxelize(w.targets[0][0], ct, w.resolution)
        iso = oracle.linearize_factor(xyz, cs, vmi, pi, pj)
        H, b, e = icp_normal_equations(xyz, vmi, pi, pj, iso["corr"], 1 / (s2 + t2))
        assert rel_err(iso["H"], H) < 1e-10 and rel_err(iso["b"], b) < 1e-10
        # hand-derived single-point factors
        with open(os.path.join(GOLDEN, "single_point_factors.json")) as fh:
            for c in json.load(fh)["cases"]:
                eye6 = np.array([[1, 0, 0, 1, 0, 1]], np.float32)
                v1, _ = oracle.voxelize(np.array([c["target_point"]], np.float32), eye6, 1.0)
                o1 = oracle.linearize_factor(np.array([c["mu"]], np.float32), eye6, v1,
                                             np.array(c["pose_i"], float), np.array(c["pose_j"], float))
                assert o1["inliers"] == c["inliers"]
                assert np.allclose(o1["b"], c["b"], atol=1e-12)
    except (AssertionError, np.linalg.LinAlgError):
        return False
    return True


def test_unmodified_oracle_passes_its_pins():
    assert _pins_hold()


def _jac_R_transposed(R, mu, q):
    return _orig_jac(R.T, mu, q)


def _jac_B_sign(R, mu, q):
    A, B = _orig_jac(R, mu, q)
    B[:, :, :3] *= -1
    return A, B


def _jac_blocks_swapped(R, mu, q):
    A, B = _orig_jac(R, mu, q)
    return B, A


def _fused_drops_source_cov(S, C, R):
    return _orig_fused(S, 0 * C, R)


def _fused_wrong_congruence(S, C, R):
    return _orig_fused(S, C, R.T)


def _residual_sign(m, R, t, mu):
    e, q = _orig_res(m, R, t, mu)
    return -e, q


def _relpose_reversed(pi, pj):
    return _orig_rel(pj, pi)


def _relpose_transposed(pi, pj):
    R, t = _orig_rel(pi, pj)
    return R.T.copy(), t


def _voxelize_count_off_by_one(xyz, cov, r):
    vm, inv = _orig_vox(xyz, cov, r)
    txyz = np.asarray(xyz, np.float64)
    sums = np.zeros((vm.n_voxels, 3))
    np.add.at(sums, inv, txyz)
    vm.mean = (sums / (vm.count[:, None] + 1)).astype(np.float32)
    return vm, inv


def _fma32_two_roundings(a, b, c):
    a64, b64, c64 = (np.asarray(v, np.float32).astype(np.float64) for v in (a, b, c))
    return (a64 * b64 + c64).astype(np.float32)


_orig_jac = vo.jacobians
_orig_fused = vo.fused_information
_orig_res = vo.residuals
_orig_rel = vo.relative_pose
_orig_vox = vo.voxelize

MUTANTS = [
    ("jacobians", _jac_R_transposed),
    ("jacobians", _jac_B_sign),
    ("jacobians", _jac_blocks_swapped),
    ("fused_information", _fused_drops_source_cov),
    ("fused_information", _fused_wrong_congruence),
    ("residuals", _residual_sign),
    ("relative_pose", _relpose_reversed),
    ("relative_pose", _relpose_transposed),
    ("voxelize", _voxelize_count_off_by_one),
    ("fma32", _fma32_two_roundings),
]


@pytest.mark.parametrize("name,fn", MUTANTS, ids=[f.__name__ for _, f in MUTANTS])
def test_planted_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(vo, name, fn)
    if name in ("relative_pose", "voxelize"):
        monkeypatch.setattr(oracle, name, fn)
    assert not _pins_hold()


# ----------------------------------------------------------------- assembly

def _assembly_pins_hold() -> bool:
    from tests.oracle_pins import fd_global_system, global_null_space, small_pose_graph
    w = small_pose_graph(seed=6)
    maps = oracle.build_maps(w.targets, w.resolution)
    ref = oracle.linearize_workload(w.sources, maps, w.poses, w.factors)
    Hg, bg = oracle.assemble_system(ref["H"], ref["b"], w.factors, w.poses.shape[0])
    Hfd, bfd = fd_global_system(w)
    N = global_null_space(w.poses)
    return (rel_err(Hg, Hfd) < 1e-7 and rel_err(bg, bfd) < 1e-7
            and np.linalg.norm(Hg @ N) <= 1e-10 * np.linalg.norm(Hg) * np.linalg.norm(N))


def _asm_poses_swapped(H, b, factors, P):
    f = np.asarray(factors).copy()
    f[:, [2, 3]] = f[:, [3, 2]]
    return _orig_asm(H, b, f, P)


def _asm_cross_transposed(H, b, factors, P):
    H = np.array(H, copy=True)
    for k in range(H.shape[0]):
        H[k, :6, 6:] = H[k, :6, 6:].T.copy()
        H[k, 6:, :6] = H[k, 6:, :6].T.copy()
    return _orig_asm(H, b, factors, P)


def _asm_bj_sign(H, b, factors, P):
    b = np.array(b, copy=True)
    b[:, 6:] *= -1
    return _orig_asm(H, b, factors, P)


_orig_asm = vo.assemble_system

ASM_MUTANTS = [_asm_poses_swapped, _asm_cross_transposed, _asm_bj_sign]


def test_unmodified_assembly_passes_its_pins():
    assert _assembly_pins_hold()


@pytest.mark.parametrize("fn", ASM_MUTANTS, ids=[f.__name__ for f in ASM_MUTANTS])
def test_planted_assembly_mistake_is_caught(monkeypatch, fn):
    monkeypatch.setattr(vo, "assemble_system", fn)
    monkeypatch.setattr(oracle, "assemble_system", fn)
    assert not _assembly_pins_hold()


# ------------------------------------------- degenerate fused covariances (R9)

def _degenerate_pins_hold() -> bool:
    from synth import make_degenerate_workload
    from tests.oracle_pins import degenerate_pins
    try:
        degenerate_pins(make_degenerate_workload())
    except (AssertionError, np.linalg.LinAlgError):
        return False
    return True


_orig_pd = vo.positive_definite
_orig_lin = vo.linearize_factor


def _pd_without_third_minor(F):
    """Sylvester's criterion stopped at the 2x2 minor."""
    F = np.asarray(F, np.float64)
    with np.errstate(all="ignore"):
        return (F[:, 0, 0] > 0) & (F[:, 0, 0] * F[:, 1, 1] - F[:, 0, 1] ** 2 > 0)


def _fused_inverts_before_masking(S, C, R):
    """Every row inverted, the positive-definite mask applied only afterwards."""
    F = vo.fused_covariance(S, C, R)
    return np.linalg.inv(F), _orig_pd(F)


def _fused_pseudo_inverse_for_all(S, C, R):
    """Non-positive-definite rows weighted by a pseudo-inverse instead of
    being left out."""
    F = vo.fused_covariance(S, C, R)
    F = np.where(np.isfinite(F), F, 0.0)
    return np.linalg.pinv(F), np.ones(F.shape[0], dtype=bool)


def _lin_counts_only_weighted_hits(xyz, cov, vmap, pi, pj):
    """Inliers counted after the positive-definite test instead of before."""
    out = _orig_lin(xyz, cov, vmap, pi, pj)
    hit = out["corr"] >= 0
    if hit.any():
        Cs = vo._unpack_cov(np.asarray(cov, np.float32).reshape(-1, 6)[hit])
        Sv = vo._unpack_cov(vmap.cov[out["corr"][hit]])
        _, good = _orig_fused(Sv, Cs, out["R"])
        out["inliers"] = int(good.sum())
    return out


DEG_MUTANTS = [
    ("positive_definite", _pd_without_third_minor),
    ("fused_information", _fused_inverts_before_masking),
    ("fused_information", _fused_pseudo_inverse_for_all),
    ("linearize_factor", _lin_counts_only_weighted_hits),
]


def test_unmodified_oracle_passes_its_degenerate_pins():
    assert _degenerate_pins_hold()


@pytest.mark.parametrize("name,fn", DEG_MUTANTS, ids=[f.__name__ for _, f in DEG_MUTANTS])
def test_planted_degenerate_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(vo, name, fn)
    monkeypatch.setattr(oracle, name, fn)
    with np.errstate(all="ignore"):
        assert not _degenerate_pins_hold()
