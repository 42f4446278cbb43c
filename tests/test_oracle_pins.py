"""Pins of the FP64 oracle against facts fixed by the paper and by plain
mathematics (CPU only).

  * voxel keys: hand-derived table (tests/golden/voxel_keys.txt);
  * voxel map: brute-force grouping with exact rational arithmetic;
  * correspondences: linear scan over every voxel box; the FP32 fused
    multiply-add against exact rational arithmetic;
  * relative pose: 4x4 inverse;
  * H, b: central finite differences of the frozen residual;
    gradient of the frozen cost = 2 b;
  * structure: symmetry, positive semidefinite, six-dimensional gauge null
    space, b orthogonal to it, invariance under a common rigid motion;
  * isotropic covariances: point-to-point ICP normal equations;
  * single-point factors derived by hand (tests/golden/single_point_factors.json);
  * overlap: self overlap is 1, a far cloud 0, hits equal inliers;
  * hits whose fused covariance is not positive definite (zero, rank one or
    two, indefinite, NaN or infinite entries): inliers that add nothing,
    against the same factor without them and finite differences.
"""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import make_degenerate_workload, make_single_factor, make_tiny_workload, pose_rows
from tests.oracle_pins import (degenerate_pins, fd_cost_gradient, fd_hessian_factor, hom,
                               icp_normal_equations, null_space_basis,
                               rel_err, rows)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def cfg1():
    return make_single_factor()


@pytest.fixture(scope="module")
def tiny():
    return make_tiny_workload(seed=7, n_src=400, n_tgt=600, resolution=0.5)


# ----------------------------------------------------------------- voxel keys

def test_voxel_keys_golden():
    rows_ = []
    with open(os.path.join(GOLDEN, "voxel_keys.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                r, x, k = line.split()
                rows_.append((float(r), float(x), int(k)))
    for r, x, k in rows_:
        s = oracle.voxel_scale(r)
        got = oracle.voxel_keys(np.array([[x, 0.0, 0.0]], np.float32), s)[0, 0]
        assert got == k, (r, x, got, k)


def test_voxel_keys_reject_out_of_range_and_nonfinite():
    s = oracle.voxel_scale(0.5)
    with pytest.raises(OverflowError):
        oracle.voxel_keys(np.array([[6e5, 0, 0]], np.float32), s)
    with pytest.raises(FloatingPointError):
        oracle.voxel_keys(np.array([[np.nan, 0, 0]], np.float32), s)
    with pytest.raises(ValueError):
        oracle.voxel_scale(0.0)
    # the largest admissible key
    k = oracle.voxel_keys(np.array([[524287.5, -524288.0, 0]], np.float32), s)
    assert k[0, 0] == (1 << 20) - 1 and k[0, 1] == -(1 << 20)


@pytest.mark.parametrize("r", [0.25, 0.5, 1.0])
def test_voxelize_bruteforce_exact(tiny, r):
    xyz, cov = tiny.targets[0]
    # duplicate a few points so voxels with repeated points occur
    xyz = np.concatenate([xyz, xyz[:20]])
    cov = np.concatenate([cov, cov[:20]])
    vm, inv = oracle.voxelize(xyz, cov, r)
    groups = {}
    for i in range(xyz.shape[0]):
        key = tuple(math.floor(Fraction(float(v)) / Fraction(r)) for v in xyz[i])
        groups.setdefault(key, []).append(i)
    keys = sorted(groups)
    assert vm.n_voxels == len(keys)
    assert [tuple(k) for k in vm.keys.tolist()] == keys
    for o, key in enumerate(keys):
        idx = groups[key]
        assert vm.count[o] == len(idx)
        assert all(inv[i] == o for i in idx)
        for arr, got in ((xyz, vm.mean[o]), (cov, vm.cov[o])):
            exact = [sum(Fraction(float(arr[i, c])) for i in idx) / len(idx)
                     for c in range(arr.shape[1])]
            for c, ex in enumerate(exact):
                # the stored FP32 value is a rounding of the exact mean
                g = Fraction(float(got[c]))
                ulp = Fraction(float(np.spacing(np.float32(abs(float(ex))) or np.float32(1e-30))))
                assert abs(g - ex) <= ulp, (o, c, float(g), float(ex))


def test_voxelize_empty():
    vm, inv = oracle.voxelize(np.zeros((0, 3), np.float32), np.zeros((0, 6), np.float32), 0.5)
    assert vm.n_voxels == 0 and inv.shape == (0,)


# ------------------------------------------------------------ relative pose

def test_relative_pose_matches_matrix_inverse(tiny):
    pi, pj = tiny.poses[0], tiny.poses[1]
    R, t = oracle.relative_pose(pi, pj)
    T = np.linalg.inv(hom(pj)) @ hom(pi)
    assert np.abs(R - T[:3, :3]).max() < 1e-14
    assert np.abs(t - T[:3, 3]).max() < 1e-13


def test_relative_pose_equal_poses_is_exact_identity(tiny):
    R, t = oracle.relative_pose(tiny.poses[0], tiny.poses[0])
    assert np.array_equal(R, np.eye(3)) and np.array_equal(t, np.zeros(3))


# ---------------------------------------------------------- correspondences

def _rn32(x: Fraction) -> np.float32:
    """The float32 nearest to the rational x (ties to an even last bit),
    chosen among the neighbours of a first guess by exact comparison."""
    g = np.float32(float(x))
    cands = [np.nextafter(g, np.float32(-np.inf)), g, np.nextafter(g, np.float32(np.inf))]
    best = min(cands, key=lambda f: (abs(Fraction(float(f)) - x),
                                     int(np.array(f, np.float32).view(np.int32)) & 1))
    return np.float32(best)


def _fma_cases():
    """(a, b, c) float32 triples whose exact a*b + c lies on, or a hair off,
    a midpoint between two float32 values, where rounding the FP64 sum to
    FP32 (two roundings) goes the wrong way."""
    two = np.float32
    a, b = two(24929 * 2.0 ** -12), two(673 * 2.0 ** -12)   # a * b = 1 + 2^-24 exactly
    tiny = two(2.0 ** -80)
    return [(a, b, tiny), (a, b, -tiny), (a, b, two(0.0)),
            (-a, b, -tiny), (a, -b, tiny), (a, b, two(2.0 ** -60)),
            (two(3.0), two(1.0 / 3.0), two(-1.0))]


def test_fma32_rounds_once_on_midpoint_cases():
    """On sums that sit on or next to a float32 midpoint, fma32 equals the
    exact sum rounded once, where the FP64 sum rounded to FP32 does not."""
    wrong_twice = 0
    for a, b, c in _fma_cases():
        exact = Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))
        want = _rn32(exact)
        got = oracle.vgicp_oracle.fma32(a, b, c)
        assert got.view(np.int32) == np.array(want).view(np.int32), (a, b, c)
        twice = np.float32(np.float64(a) * np.float64(b) + np.float64(c))
        wrong_twice += int(twice != want)
    assert wrong_twice >= 2


def test_fma32_matches_exact_rounding_on_random_operands():
    rng = np.random.default_rng(5)
    n = 3000
    a = (rng.standard_normal(n) * 10.0 ** rng.integers(-3, 4, n)).astype(np.float32)
    b = (rng.standard_normal(n) * 10.0 ** rng.integers(-3, 4, n)).astype(np.float32)
    c = (-(a.astype(np.float64) * b) * (1 + rng.standard_normal(n) * 1e-6)).astype(np.float32)
    c[::3] = rng.standard_normal(c[::3].shape).astype(np.float32)
    got = oracle.vgicp_oracle.fma32(a, b, c)
    for k in range(n):
        exact = Fraction(float(a[k])) * Fraction(float(b[k])) + Fraction(float(c[k]))
        assert got[k].view(np.int32) == np.array(_rn32(exact)).view(np.int32), k


def test_lookup_coords_are_the_scaled_relative_motion(tiny):
    xyz = tiny.sources[0][0]
    R, t = oracle.relative_pose(tiny.poses[0], tiny.poses[1])
    s = oracle.voxel_scale(0.5)
    v = oracle.vgicp_oracle.lookup_coords_fp32(xyz, R, t, s)
    T = np.linalg.inv(hom(tiny.poses[1])) @ hom(tiny.poses[0])
    v64 = (xyz.astype(np.float64) @ T[:3, :3].T + T[:3, 3]) * float(s)
    scale = (np.abs(xyz).max() + np.abs(T[:3, 3]).max()) * float(s)
    assert np.abs(v - v64).max() < 8 * np.finfo(np.float32).eps * scale


def test_lookup_coords_identity_pose_are_the_voxelization_coords(tiny):
    """Under the identity the lookup coordinates are fl32(x * s), the
    coordinates voxelization takes its keys from, so every point finds its
    own voxel."""
    xyz, cov = tiny.targets[0]
    s = oracle.voxel_scale(0.5)
    v = oracle.vgicp_oracle.lookup_coords_fp32(xyz, np.eye(3), np.zeros(3), s)
    assert np.array_equal(v, (xyz.astype(np.float32) * s).astype(np.float32))
    vm, inv = oracle.voxelize(xyz, cov, 0.5)
    assert np.array_equal(oracle.lookup(vm, xyz, np.eye(3), np.zeros(3)), inv)


@pytest.mark.parametrize("r", [0.5, 1.0])
def test_lookup_linear_scan(tiny, r):
    src, tgt = tiny.sources[0][0], tiny.targets[0]
    vm, _ = oracle.voxelize(*tgt, r)
    R, t = oracle.relative_pose(tiny.poses[0], tiny.poses[1])
    corr = oracle.lookup(vm, src, R, t)
    v = oracle.vgicp_oracle.lookup_coords_fp32(src, R, t, vm.scale).astype(np.float64)
    lo = vm.keys.astype(np.float64)                    # (V, 3) voxel boxes, voxel units
    inside = np.all((v[:, None, :] >= lo[None]) & (v[:, None, :] < lo[None] + 1.0), axis=2)
    want = np.where(inside.any(1), inside.argmax(1), -1)
    assert inside.sum(1).max() <= 1
    assert np.array_equal(corr, want)
    assert (corr >= 0).sum() > 50


def test_lookup_far_and_out_of_range_keys_miss(tiny):
    src, tgt = tiny.sources[0][0], tiny.targets[0]
    vm, _ = oracle.voxelize(*tgt, 0.5)
    for shift in (1e4, 1e6, 1e30):
        pj = hom(tiny.poses[1])
        pj[0, 3] += shift
        R, t = oracle.relative_pose(tiny.poses[0], rows(pj))
        assert np.all(oracle.lookup(vm, src, R, t) == -1)


# --------------------------------------------------------- Hessian factor

def test_jacobians_hessian_and_b_match_finite_differences(tiny):
    xyz, cov = tiny.sources[0]
    vm, _ = oracle.voxelize(*tiny.targets[0], tiny.resolution)
    fd = fd_hessian_factor(xyz, cov, vm, tiny.poses[0], tiny.poses[1])
    out = fd["oracle"]
    assert out["inliers"] > 50
    assert rel_err(out["H"], fd["H"]) < 1e-7
    assert rel_err(out["b"], fd["b"]) < 1e-7
    assert abs(out["e"] - fd["e"]) <= 1e-12 * abs(fd["e"])
    # per-point Jacobians
    hit = out["corr"] >= 0
    R, t = out["R"], out["t"]
    mu = xyz[hit].astype(np.float64)
    A, B = oracle.vgicp_oracle.jacobians(R, mu, mu @ R.T + t)
    Jo = np.concatenate([A, B], 2)
    assert np.abs(Jo - fd["J"]).max() < 1e-6 * max(1.0, np.abs(Jo).max())


def test_frozen_cost_gradient_is_twice_b(tiny):
    xyz, cov = tiny.sources[0]
    vm, _ = oracle.voxelize(*tiny.targets[0], tiny.resolution)
    g, out = fd_cost_gradient(xyz, cov, vm, tiny.poses[0], tiny.poses[1])
    assert rel_err(g, 2 * out["b"]) < 1e-7


def test_hessian_structure(cfg1):
    vm, _ = oracle.voxelize(*cfg1.targets[0], cfg1.resolution)
    out = oracle.linearize_factor(*cfg1.sources[0], vm, cfg1.poses[0], cfg1.poses[1])
    H, b = out["H"], out["b"]
    nH = np.linalg.norm(H)
    assert np.abs(H - H.T).max() <= 1e-13 * nH
    ev = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert ev.min() >= -1e-10 * ev.max()
    N = null_space_basis(cfg1.poses[0], cfg1.poses[1])
    assert np.linalg.norm(H @ N) <= 1e-10 * nH * np.linalg.norm(N)
    assert np.abs(b @ N).max() <= 1e-10 * np.linalg.norm(b) * np.linalg.norm(N)
    # exactly six gauge directions: rank 6
    assert np.sum(ev > 1e-8 * ev.max()) == 6


def test_invariance_under_common_rigid_motion(cfg1):
    vm, _ = oracle.voxelize(*cfg1.targets[0], cfg1.resolution)
    base = oracle.linearize_factor(*cfg1.sources[0], vm, cfg1.poses[0], cfg1.poses[1])
    # a sign-flip rotation (180 degrees about z) keeps the relative pose bitwise
    G = np.diag([-1.0, -1.0, 1.0, 1.0])
    pi, pj = rows(G @ hom(cfg1.poses[0])), rows(G @ hom(cfg1.poses[1]))
    flip = oracle.linearize_factor(*cfg1.sources[0], vm, pi, pj)
    assert np.array_equal(flip["corr"], base["corr"])
    assert np.array_equal(flip["H"], base["H"]) and flip["e"] == base["e"]
    # a generic motion changes the relative pose only by rounding
    from tests.oracle_pins import so3_exp
    G = np.eye(4)
    G[:3, :3] = so3_exp(np.array([0.3, -0.2, 0.5]))
    G[:3, 3] = [3.0, -7.0, 1.5]
    pi, pj = rows(G @ hom(cfg1.poses[0])), rows(G @ hom(cfg1.poses[1]))
    gen = oracle.linearize_factor(*cfg1.sources[0], vm, pi, pj)
    assert np.array_equal(gen["corr"], base["corr"])
    assert rel_err(gen["H"], base["H"]) < 1e-12
    assert rel_err(gen["b"], base["b"]) < 1e-10
    assert abs(gen["e"] - base["e"]) < 1e-12 * base["e"]


def test_isotropic_covariances_reduce_to_icp_normal_equations(tiny):
    xyz, _ = tiny.sources[0]
    txyz, _ = tiny.targets[0]
    sig2, tau2 = 0.5, 0.25
    cov_s = np.tile(np.array([sig2, 0, 0, sig2, 0, sig2], np.float32), (xyz.shape[0], 1))
    cov_t = np.tile(np.array([tau2, 0, 0, tau2, 0, tau2], np.float32), (txyz.shape[0], 1))
    vm, _ = oracle.voxelize(txyz, cov_t, tiny.resolution)
    assert np.all(vm.cov[:, [0, 3, 5]] == tau2) and np.all(vm.cov[:, [1, 2, 4]] == 0)
    out = oracle.linearize_factor(xyz, cov_s, vm, tiny.poses[0], tiny.poses[1])
    H, b, e = icp_normal_equations(xyz, vm, tiny.poses[0], tiny.poses[1], out["corr"],
                                   1.0 / (sig2 + tau2))
    assert rel_err(out["H"], H) < 1e-12
    assert rel_err(out["b"], b) < 1e-12
    assert abs(out["e"] - e) < 1e-12 * e


def test_single_point_golden():
    with open(os.path.join(GOLDEN, "single_point_factors.json")) as fh:
        cases = json.load(fh)["cases"]
    eye6 = np.array([[1, 0, 0, 1, 0, 1]], np.float32)
    for c in cases:
        vm, _ = oracle.voxelize(np.array([c["target_point"]], np.float32), eye6, c["resolution"])
        out = oracle.linearize_factor(np.array([c["mu"]], np.float32), eye6, vm,
                                      np.array(c["pose_i"], float), np.array(c["pose_j"], float))
        assert out["inliers"] == c["inliers"], c["name"]
        assert np.allclose(out["b"], c["b"], atol=1e-15), c["name"]
        assert abs(out["e"] - c["e"]) < 1e-15, c["name"]
        if c["J_columns"] is None:
            assert np.all(out["H"] == 0)
        else:
            J = np.array(c["J_columns"], float).T           # (3, 12)
            assert np.allclose(out["H"], 0.5 * J.T @ J, atol=1e-15), c["name"]
            assert np.allclose(out["b"], 0.5 * J.T @ np.array(c["residual"]), atol=1e-15)


def test_empty_source_and_no_hits(tiny):
    vm, _ = oracle.voxelize(*tiny.targets[0], 0.5)
    out = oracle.linearize_factor(np.zeros((0, 3), np.float32), np.zeros((0, 6), np.float32),
                                  vm, tiny.poses[0], tiny.poses[1])
    assert out["inliers"] == 0 and out["e"] == 0.0 and not out["H"].any()
    assert oracle.overlap_factor(np.zeros((0, 3), np.float32), vm, tiny.poses[0],
                                 tiny.poses[1]) == (0, 0.0)


def test_degenerate_fused_covariance_hits_count_and_add_nothing():
    """Reading of Eq. (2) where the fused covariance C'_k + R C_k R^T has no
    inverse or is not positive definite: the hit counts as an inlier and
    adds nothing to H, b or e."""
    w = make_degenerate_workload()
    outs = degenerate_pins(w)
    assert all(np.all(np.isfinite(o["H"])) and np.all(np.isfinite(o["b"])) for o in outs)
    # every kind is present and its fused covariance really is degenerate
    assert set(w.meta["kinds"][1]) == {"regular", "zero", "rank1", "rank2", "indefinite",
                                       "nan", "inf", "neg_inf"}


def test_positive_definite_test_on_textbook_matrices():
    """Sylvester's criterion on matrices whose definiteness is known."""
    F = np.stack([np.eye(3), np.diag([1.0, 1.0, 0.0]), np.diag([1.0, -1.0, 1.0]),
                  np.zeros((3, 3)), np.full((3, 3), np.nan), np.diag([np.inf, 1.0, 1.0]),
                  np.array([[2.0, 1.0, 0.0], [1.0, 2.0, 1.0], [0.0, 1.0, 2.0]]),
                  np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]])])
    assert oracle.positive_definite(F).tolist() == [True, False, False, False, False, False,
                                                    True, False]
    Om, good = oracle.fused_information(F, np.zeros_like(F), np.eye(3))
    assert good.tolist() == oracle.positive_definite(F).tolist()
    assert np.allclose(Om[0], np.eye(3)) and not Om[1:6].any()


# ----------------------------------------------------------------- overlap

def test_overlap_self_far_and_hits_equal_inliers(cfg1):
    xyz, cov = cfg1.targets[0]
    vm, _ = oracle.voxelize(xyz, cov, cfg1.resolution)
    assert oracle.overlap_factor(xyz, vm, cfg1.poses[0], cfg1.poses[0]) == (xyz.shape[0], 1.0)
    far = hom(cfg1.poses[1])
    far[:3, 3] += [1e4, 0, 0]
    assert oracle.overlap_factor(xyz, vm, cfg1.poses[1], rows(far)) == (0, 0.0)
    sx, sc = cfg1.sources[0]
    hits, ov = oracle.overlap_factor(sx, vm, cfg1.poses[0], cfg1.poses[1])
    out = oracle.linearize_factor(sx, sc, vm, cfg1.poses[0], cfg1.poses[1])
    assert hits == out["inliers"] and ov == hits / sx.shape[0]


def test_keyframe_rules_on_hand_cases():
    """Sec. III-B / III-C thresholds on hand-picked overlaps, including
    equality with each threshold (strict rules do not fire on it)."""
    rules = dict(skip_above=0.95, close_below=0.10, max_frames=15)
    cases = [
        ((0, 0.0, 0.0), "start"), ((0, 1.0, 1.0), "start"),
        ((3, 0.951, 0.5), "skip"), ((3, 0.95, 0.5), "insert"), ((3, 0.95, 0.0999), "close"),
        ((3, 0.5, 0.10), "insert"), ((14, 0.5, 0.5), "insert"), ((15, 0.5, 0.5), "close"),
        ((15, 0.99, 0.01), "skip"), ((1, 0.2, 0.2), "insert"), ((1, 0.05, 0.05), "close"),
    ]
    for (n, ol, of), want in cases:
        assert oracle.submap_decision(n, ol, of, **rules) == want, (n, ol, of)
    assert oracle.factor_admitted(0.0251, 0.025) and not oracle.factor_admitted(0.025, 0.025)
    assert oracle.factor_admitted(0.05, 0.05, at_least=True)
    assert not oracle.factor_admitted(0.0499, 0.05, at_least=True)
    # an exact rate: 1 hit in 40 points is 0.025 in FP64, on the threshold
    assert 1 / 40 == 0.025 and not oracle.factor_admitted(1 / 40, 0.025)


def test_workload_driver_matches_per_factor():
    w = make_tiny_workload(seed=3, n_src=[50, 80, 0], n_tgt=[90, 60, 70], resolution=0.5, n_factors=3)
    maps = oracle.build_maps(w.targets, w.resolution)
    res = oracle.linearize_workload(w.sources, maps, w.poses, w.factors)
    for f, (s, t, pi, pj) in enumerate(w.factors):
        one = oracle.linearize_factor(*w.sources[s], maps[t], w.poses[pi], w.poses[pj])
        assert np.array_equal(res["H"][f], one["H"]) and res["inliers"][f] == one["inliers"]
    assert res["inliers"][2] == 0


# ----------------------------------------------------------------- assembly

def test_assembled_system_matches_global_finite_differences():
    from tests.oracle_pins import fd_global_system, global_null_space, small_pose_graph
    w = small_pose_graph()
    maps = oracle.build_maps(w.targets, w.resolution)
    ref = oracle.linearize_workload(w.sources, maps, w.poses, w.factors)
    assert np.all(ref["inliers"] > 30)
    P = w.poses.shape[0]
    Hg, bg = oracle.assemble_system(ref["H"], ref["b"], w.factors, P)
    Hfd, bfd = fd_global_system(w)
    assert rel_err(Hg, Hfd) < 1e-7
    assert rel_err(bg, bfd) < 1e-7
    # gauge: a common motion of all poses is free
    N = global_null_space(w.poses)
    assert np.linalg.norm(Hg @ N) <= 1e-10 * np.linalg.norm(Hg) * np.linalg.norm(N)
    assert np.abs(bg @ N).max() <= 1e-10 * np.linalg.norm(bg) * np.linalg.norm(N)
    # the factor on one pose (rows 5) adds nothing: its relative pose is fixed
    Hs, bs = oracle.assemble_system(ref["H"][5:6], ref["b"][5:6], w.factors[5:6], P)
    assert np.linalg.norm(ref["H"][5]) > 0
    assert np.abs(Hs).max() <= 1e-12 * np.linalg.norm(ref["H"][5])
    assert np.abs(bs).max() <= 1e-12 * np.linalg.norm(ref["b"][5]) + 1e-300
    # block read-out
    pairs = [(0, 1), (0, 3), (1, 2), (1, 3)]
    diag, bvec, off = oracle.system_blocks(Hg, bg, P, pairs)
    assert np.array_equal(off[0], Hg[0:6, 6:12]) and np.array_equal(diag[2], Hg[12:18, 12:18])
    assert np.array_equal(bvec[3], bg[18:24])
