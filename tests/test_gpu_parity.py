"""Parity of the HIP path with the FP64 oracle (GPU).

Integer outputs (voxel keys and counts, correspondences, inliers, overlap
hits) must be bit-exact; the FP32 voxel payload is compared bit-exactly too
(both sides sum in FP64 in point order and round once).  H, b and e must lie
within a relative 1e-5 of the FP64 oracle for every accumulation variant,
per factor and per block: each 6x6 block of H split into its rotation and
translation parts, b_i and b_j split likewise, and the elementwise error
|d| / (|ref| + 1e-3 max|ref|) of H and of b (1e-4 for the plain FP32
accumulation's elementwise error, whose wave tree rounds in FP32)."""

import numpy as np
import pytest

from synth import (Workload, make_degenerate_workload, make_scan_workload, make_single_factor,
                   make_tiny_workload, pose_rows)
from tests.gpu_helpers import (FUSED32_TOL, TOL, GpuWorkload, assert_linearize_parity,
                               elem_tol_for, oracle_results, rel_fro)
import oracle

pytestmark = pytest.mark.gpu

ACCS = ["mixed", "f32", "f32_comp", "f64"]


@pytest.fixture(scope="module")
def vg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2109_07073_amd import vgicp
    return vgicp


@pytest.fixture(scope="module")
def ctx(vg):
    return vg.Context(0)


@pytest.fixture(scope="module")
def cfg1():
    return make_single_factor()


@pytest.fixture(scope="module")
def ragged():
    sizes = [0, 1, 255, 256, 257, 4095, 4096, 4097, 9000, 513, 3]
    tgts = [50, 700, 1, 2000, 900, 3000, 0, 2500, 4000, 800, 10]
    return make_tiny_workload(seed=21, n_src=sizes, n_tgt=tgts, resolution=0.5,
                              n_factors=len(sizes), half=6.0, height=3.0)


@pytest.fixture(scope="module")
def scans():
    return make_scan_workload(cfg=2, n_frames=6, n_factors=8, n_target=20000, workers=4)


@pytest.fixture(scope="module")
def degenerate():
    return make_degenerate_workload()


@pytest.fixture(scope="module")
def scans40():
    """40 factors of the 100-frame, 500-factor scan workload (20,000 points each)."""
    w = make_scan_workload(cfg=2, n_frames=100, n_factors=500, n_target=20000, workers=8)
    w.factors = w.factors[::12][:40].copy()
    return w


# ------------------------------------------------------------------ voxelize

def _export_np(m):
    return {k: v.cpu().numpy() for k, v in m.export().items()}


@pytest.mark.parametrize("r", [0.5, 1.0, 0.3, 2.0])
def test_voxelize_bitexact(vg, ctx, ragged, r):
    for k in (1, 5, 8, 9):
        xyz, cov = ragged.targets[k]
        dx, dc = vg.cloud_to_device(xyz, cov)
        m = vg.voxelize(ctx, dx, dc, r)
        ref, _ = oracle.voxelize(xyz, cov, r)
        assert m.n_voxels == ref.n_voxels
        # brick table: the smallest power of two >= max(16, 8 * bricks), the
        # bricks being the distinct floor(key / 4); 32-byte records, an
        # occupancy bitset of min(cap, 2^16) bits (at least 32), plus 52 bytes
        # per voxel (36 bytes of statistics, 16 of key, ordinal and count)
        n_bricks = (np.unique(np.floor_divide(ref.keys, 4), axis=0).shape[0]
                    if ref.n_voxels else 0)
        cap = 16
        while cap < 8 * n_bricks:
            cap *= 2
        assert m.capacity == cap
        assert m.device_bytes == 32 * cap + max(32, min(cap, 1 << 16)) // 8 + 52 * m.n_voxels
        got = _export_np(m)
        assert np.array_equal(got["keys"], ref.keys.astype(np.int32))
        assert np.array_equal(got["count"], ref.count.astype(np.int32))
        assert np.array_equal(got["mean"].view(np.uint32), ref.mean.view(np.uint32))
        assert np.array_equal(got["cov"].view(np.uint32), ref.cov.view(np.uint32))


def test_voxelize_scan_frames_bitexact(vg, ctx, scans):
    for xyz, cov in scans.targets[:3]:
        m = vg.voxelize(ctx, *vg.cloud_to_device(xyz, cov), scans.resolution)
        ref, _ = oracle.voxelize(xyz, cov, scans.resolution)
        got = _export_np(m)
        assert np.array_equal(got["keys"], ref.keys.astype(np.int32))
        assert np.array_equal(got["count"], ref.count.astype(np.int32))
        assert np.array_equal(got["mean"].view(np.uint32), ref.mean.view(np.uint32))
        assert np.array_equal(got["cov"].view(np.uint32), ref.cov.view(np.uint32))


def test_voxelize_empty_and_single_point(vg, ctx):
    import torch
    z3 = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    z6 = torch.zeros((0, 6), dtype=torch.float32, device="cuda")
    m = vg.voxelize(ctx, z3, z6, 0.5)
    assert m.n_voxels == 0
    xyz = np.array([[0.25, -0.75, 3.5]], np.float32)
    cov = np.array([[1, 0, 0, 1, 0, 1]], np.float32)
    m = vg.voxelize(ctx, *vg.cloud_to_device(xyz, cov), 0.5)
    got = _export_np(m)
    assert m.n_voxels == 1 and got["keys"].tolist() == [[0, -2, 7]]
    assert np.array_equal(got["mean"], xyz) and got["count"].tolist() == [1]


def test_voxelize_rejects_nonfinite_and_out_of_range(vg, ctx):
    xyz = np.zeros((300, 3), np.float32)
    cov = np.tile(np.array([1, 0, 0, 1, 0, 1], np.float32), (300, 1))
    bad = xyz.copy()
    bad[123, 1] = np.nan
    with pytest.raises(vg.VgicpError) as ex:
        vg.voxelize(ctx, *vg.cloud_to_device(bad, cov), 0.5)
    assert ex.value.code == vg.ENONFINITE
    bad = xyz.copy()
    bad[7, 0] = 6e5        # key 1.2e6 >= 2^20 at r = 0.5
    with pytest.raises(vg.VgicpError) as ex:
        vg.voxelize(ctx, *vg.cloud_to_device(bad, cov), 0.5)
    assert ex.value.code == vg.ERANGE
    with pytest.raises(vg.VgicpError) as ex:
        vg.voxelize(ctx, *vg.cloud_to_device(xyz, cov), 0.0)
    assert ex.value.code == vg.EINVAL
    # covariances must be 8-byte aligned, as the interface states
    import torch
    dx, dc = vg.cloud_to_device(xyz, cov)
    buf = torch.zeros(6 * 300 + 1, dtype=torch.float32, device="cuda")
    shifted = buf[1:].view(300, 6)
    shifted.copy_(dc)
    with pytest.raises(vg.VgicpError) as ex:
        vg.voxelize(ctx, dx, shifted, 0.5)
    assert ex.value.code == vg.EINVAL
    with pytest.raises(vg.VgicpError) as ex:
        vg.FactorSet(ctx, [(dx, shifted)], [vg.voxelize(ctx, dx, dc, 0.5)], [(0, 0, 0, 0)], 1)
    assert ex.value.code == vg.EINVAL
    # the context stays usable
    m = vg.voxelize(ctx, *vg.cloud_to_device(xyz, cov), 0.5)
    assert m.n_voxels == 1


def test_clouds_above_the_size_limit_are_refused(vg, ctx):
    """Clouds of more than 2^26 points are refused by the host-side checks,
    before any device access (the counts here exceed the small buffers the
    pointers name, which nothing reads)."""
    import ctypes
    xyz = np.zeros((4, 3), np.float32)
    cov = np.tile(np.array([1, 0, 0, 1, 0, 1], np.float32), (4, 1))
    dx, dc = vg.cloud_to_device(xyz, cov)
    big = (1 << 26) + 1
    c = vg.CCloud(dx.data_ptr(), dc.data_ptr(), big)
    h = ctypes.c_void_p()
    rc = vg._lib.vgicp_voxelize(ctx.handle, ctypes.byref(c), ctypes.c_double(0.5), ctypes.byref(h))
    assert rc == vg.EINVAL and not h.value
    assert "2^26" in vg._lib.vgicp_last_error(ctx.handle).decode()
    m = vg.voxelize(ctx, dx, dc, 0.5)
    cl = (vg.CCloud * 1)(c)
    mp = (ctypes.c_void_p * 1)(m.handle)
    fac = (vg.CFactor * 1)(vg.CFactor(0, 0, 0, 0))
    fs = ctypes.c_void_p()
    rc = vg._lib.vgicp_factorset_create(ctx.handle, cl, 1, mp, 1, fac, 1, 1, 0, ctypes.byref(fs))
    assert rc == vg.EINVAL and not fs.value
    ctx.synchronize()


# ------------------------------------------------------ correspondences, H/b/e

@pytest.mark.parametrize("accum", ACCS)
def test_cfg1_single_factor(vg, ctx, cfg1, accum):
    g = GpuWorkload(vg, ctx, cfg1)
    got = g.linearize(accum=accum, with_corr=True)
    _, ref = oracle_results(cfg1)
    assert np.array_equal(got["corr"], ref["corr"][0].astype(np.int32))
    worst = assert_linearize_parity(got, ref, elem_tol=elem_tol_for(accum))
    print(f"cfg1 {accum}: worst relative error {worst}")
    H = got["H"][0]
    assert np.array_equal(H, H.T)


@pytest.mark.parametrize("tile", [0, 256, 1024])
@pytest.mark.parametrize("accum", ACCS)
def test_ragged_factors(vg, ctx, ragged, accum, tile):
    g = GpuWorkload(vg, ctx, ragged, tile_points=tile)
    got = g.linearize(accum=accum, with_corr=True)
    _, ref = oracle_results(ragged)
    assert np.array_equal(got["corr"], np.concatenate(ref["corr"]).astype(np.int32))
    assert_linearize_parity(got, ref, elem_tol=elem_tol_for(accum))
    assert got["inliers"][0] == 0 and got["inliers"][6] == 0   # empty source / empty map


@pytest.mark.parametrize("accum", ACCS)
def test_scan_factors(vg, ctx, scans, accum):
    g = GpuWorkload(vg, ctx, scans)
    got = g.linearize(accum=accum, with_corr=True)
    _, ref = oracle_results(scans)
    assert np.array_equal(got["corr"], np.concatenate(ref["corr"]).astype(np.int32))
    worst = assert_linearize_parity(got, ref, elem_tol=elem_tol_for(accum))
    print(f"scans {accum}: worst relative error {worst}")


@pytest.fixture(scope="module")
def scans40_ref(scans40):
    return oracle_results(scans40)[1]


@pytest.mark.parametrize("accum", ACCS)
def test_scan_factors_40_fp64_residual(vg, ctx, scans40, scans40_ref, accum):
    g = GpuWorkload(vg, ctx, scans40)
    got = g.linearize(accum=accum, resid="f64")
    worst = assert_linearize_parity(got, scans40_ref, elem_tol=elem_tol_for(accum))
    print(f"40 scan factors {accum}/f64-residual: worst relative error {worst}")


def test_plain_fp32_residual_is_the_looser_variant(vg, ctx, scans40, scans40_ref):
    """The plain FP32 residual keeps bit-exact counts; its error is bounded by
    the transform's rounding: |mu| up to 80 m gives about 1e-5 m per residual
    against residuals of 0.1 m or more, so blocks are checked at 1e-4 and the
    elementwise metric, where small entries of b cancel, at 1e-3."""
    g = GpuWorkload(vg, ctx, scans40)
    got = g.linearize(accum="f64", resid="f32")
    worst = assert_linearize_parity(got, scans40_ref, tol=1e-4, elem_tol=1e-3)
    print(f"40 scan factors f64/f32-residual: worst relative error {worst}")
    r64 = g.linearize(accum="f64", resid="f64")
    assert np.array_equal(r64["inliers"], got["inliers"])


def test_schedules_graph_and_repeats_are_bitwise_identical(vg, ctx, ragged):
    import torch
    g = GpuWorkload(vg, ctx, ragged)
    base = g.linearize()
    per = g.linearize(schedule="per_factor")
    again = g.linearize()
    for k in ("H", "b", "e", "inliers"):
        assert np.array_equal(base[k], per[k]), k
        assert np.array_equal(base[k], again[k]), k
    # graph replay on a side stream, with eager work between replays
    side = torch.cuda.Stream()
    gctx = vg.Context(0, stream=side)
    F = g.fs.n_factors
    out = {"H": torch.empty((F, 12, 12), dtype=torch.float64, device="cuda"),
           "b": torch.empty((F, 12), dtype=torch.float64, device="cuda"),
           "e": torch.empty((F,), dtype=torch.float64, device="cuda"),
           "inliers": torch.empty((F,), dtype=torch.int64, device="cuda")}
    fs2 = vg.FactorSet(gctx, g.src, g.maps, g.factors, g.poses.shape[0])
    for rep in range(4):
        for v in out.values():
            v.zero_()
        torch.cuda.synchronize()
        vg.linearize_factors(gctx, fs2, g.poses, use_graph=True, out=out)
        gctx.synchronize()
        for k in ("H", "b", "e", "inliers"):
            assert np.array_equal(out[k].cpu().numpy(), base[k]), (rep, k)
        _ = g.linearize(accum="f64")        # unrelated eager work between replays


@pytest.mark.parametrize("tile", [256, 1024])
def test_persistent_grids_give_the_same_bits(vg, ctx, ragged, scans, tile):
    """Linearize, evaluate and overlap on one workgroup per tile and on
    persistent grids (tiles walked by 8, 64 and 1,024 workgroups, so that a
    workgroup runs tiles of several factors and maps) write the same bits."""
    for w in (ragged, scans):
        g = GpuWorkload(vg, ctx, w, tile_points=tile)
        assert vg.grid(g.fs) == 0
        base = g.linearize(with_corr=True)
        ev0, ov0 = g.evaluate(), g.overlap()
        for blocks in (8, 64, 1024):
            vg.set_grid(ctx, g.fs, blocks)
            assert vg.grid(g.fs) == blocks
            got = g.linearize(with_corr=True)
            for k in base:
                assert np.array_equal(got[k], base[k]), (w.name, blocks, k)
            ev, ov = g.evaluate(), g.overlap()
            for k in ev0:
                assert np.array_equal(ev[k], ev0[k]), (w.name, blocks, k)
            for k in ov0:
                assert np.array_equal(ov[k], ov0[k]), (w.name, blocks, k)
        with pytest.raises(vg.VgicpError):
            vg.set_grid(ctx, g.fs, 12)


@pytest.mark.parametrize("tile", [256, 1024])
def test_interleaved_layout_gives_the_same_bits(vg, ctx, ragged, scans, tile):
    """The interleaved tile table (the factors that read one source copy side
    by side, tile by tile) writes the same bits as the grouped one, in the
    batched and per-factor schedules, on a persistent grid and in the pair
    form; the scan factors share source frames, the ragged ones do not."""
    for w in (ragged, scans):
        g = GpuWorkload(vg, ctx, w, tile_points=tile)
        assert vg.layout_of(g.fs) == "grouped"
        base = g.linearize(with_corr=True)
        pair = g.linearize(form="pair")
        ev0, ov0 = g.evaluate(), g.overlap()
        vg.set_layout(ctx, g.fs, "interleaved")
        assert vg.layout_of(g.fs) == "interleaved"
        for kw in ({}, {"schedule": "per_factor"}):
            got = g.linearize(with_corr=True, **kw)
            for k in base:
                assert np.array_equal(got[k], base[k]), (w.name, kw, k)
        got = g.linearize(form="pair", schedule="per_factor")
        for k in pair:
            assert np.array_equal(got[k], pair[k]), (w.name, k)
        ev, ov = g.evaluate(), g.overlap()
        for k in ev0:
            assert np.array_equal(ev[k], ev0[k]), (w.name, k)
        for k in ov0:
            assert np.array_equal(ov[k], ov0[k]), (w.name, k)
        vg.set_grid(ctx, g.fs, 64)
        got = g.linearize(with_corr=True)
        for k in base:
            assert np.array_equal(got[k], base[k]), (w.name, "grid 64", k)
        vg.set_layout(ctx, g.fs, "grouped")
        got = g.linearize(with_corr=True)
        for k in base:
            assert np.array_equal(got[k], base[k]), (w.name, "back to grouped", k)
        with pytest.raises(ValueError):
            vg.set_layout(ctx, g.fs, "diagonal")


@pytest.mark.parametrize("tile", [1024, 3072])
def test_balanced_layout(vg, ctx, ragged, degenerate, scans, tile):
    """The balanced tile table (one run of about equal points per XCD, the
    factors ending a run in quarter-size tiles, runs padded with empty tiles):
    correspondences, inliers, hits and the FP64/degenerate counters equal the
    grouped table's bit for bit, H, b, e match the oracle, and the batched and
    per-factor schedules, a persistent grid, the pair form and graph replays
    agree bit for bit within the layout."""
    import torch
    for w in (ragged, degenerate, scans):
        _, ref = oracle_results(w)
        g = GpuWorkload(vg, ctx, w, tile_points=tile)
        base = g.linearize(with_corr=True)
        chk0 = vg.check_inputs(ctx, g.fs)
        wide0 = vg.fp64_points(ctx, g.fs)
        ov0 = g.overlap()
        vg.set_layout(ctx, g.fs, "balanced")
        assert vg.layout_of(g.fs) == "balanced"
        assert g.fs.n_tiles % 8 == 0
        print(f"balanced {w.name}, tile {tile}: {g.fs.n_tiles} tiles", flush=True)
        got = g.linearize(with_corr=True)
        for k in ("corr", "inliers"):
            assert np.array_equal(got[k], base[k]), (w.name, k)
        assert vg.check_inputs(ctx, g.fs) == chk0
        assert vg.fp64_points(ctx, g.fs) == wide0
        assert_linearize_parity(got, ref)
        again = g.linearize(with_corr=True, schedule="per_factor")
        for k in got:
            assert np.array_equal(again[k], got[k]), (w.name, "per factor", k)
        # graph replays (on a context with its own stream)
        side = torch.cuda.Stream()
        gctx = vg.Context(0, stream=side)
        fs2 = vg.FactorSet(gctx, g.src, g.maps, g.factors, g.poses.shape[0], tile)
        vg.set_layout(gctx, fs2, "balanced")
        F = fs2.n_factors
        out = {"H": torch.empty((F, 12, 12), dtype=torch.float64, device="cuda"),
               "b": torch.empty((F, 12), dtype=torch.float64, device="cuda"),
               "e": torch.empty((F,), dtype=torch.float64, device="cuda"),
               "inliers": torch.empty((F,), dtype=torch.int64, device="cuda")}
        for rep in range(3):
            for v in out.values():
                v.zero_()
            torch.cuda.synchronize()
            vg.linearize_factors(gctx, fs2, g.poses, use_graph=True, out=out)
            gctx.synchronize()
            for k in out:
                assert np.array_equal(out[k].cpu().numpy(), got[k]), (w.name, "graph", rep, k)
        del fs2, gctx
        pair = g.linearize(form="pair")
        assert np.array_equal(pair["inliers"], base["inliers"])
        assert_linearize_parity(pair, ref)
        ev = g.evaluate()
        assert np.array_equal(ev["inliers"], base["inliers"])
        assert np.array_equal(ev["e"], got["e"])
        ov = g.overlap()
        for k in ov0:
            assert np.array_equal(ov[k], ov0[k]), (w.name, k)
        vg.set_grid(ctx, g.fs, 64)
        again = g.linearize(with_corr=True)
        for k in got:
            assert np.array_equal(again[k], got[k]), (w.name, "grid 64", k)
        assert np.array_equal(g.linearize(form="pair")["H"], pair["H"])
        vg.set_grid(ctx, g.fs, 0)
        vg.set_layout(ctx, g.fs, "grouped")
        back = g.linearize(with_corr=True)
        for k in base:
            assert np.array_equal(back[k], base[k]), (w.name, "back to grouped", k)
        del g
        torch.cuda.synchronize()


def test_tuner_picks_a_tile_and_a_grid(vg, ctx, scans):
    g = GpuWorkload(vg, ctx, scans)
    base = g.linearize()
    best, ms = vg.tune_tiles(ctx, g.fs, g.poses, candidates=[768, 2304])
    assert best in (768, 2304) and ms > 0
    assert vg.grid(g.fs) % 8 == 0
    assert vg.layout_of(g.fs) in ("grouped", "interleaved", "balanced")
    print(f"tuned: tile {best}, grid {vg.grid(g.fs)}, layout {vg.layout_of(g.fs)}, {ms:.4f} ms")
    got = g.linearize()
    assert np.array_equal(got["inliers"], base["inliers"])
    _, ref = oracle_results(scans)
    assert_linearize_parity(got, ref)


def test_graph_cache_stays_bounded(vg, ctx, ragged):
    """Graph replay with a new set of output tensors on every call captures
    a new graph each time; the factor set keeps at most 8 (least recently
    replayed dropped), and every replay still writes the direct result."""
    import torch
    g = GpuWorkload(vg, ctx, ragged)
    base = g.linearize()
    side = torch.cuda.Stream()
    gctx = vg.Context(0, stream=side)
    fs = vg.FactorSet(gctx, g.src, g.maps, g.factors, g.poses.shape[0])
    outs = []
    with torch.cuda.stream(side):
        for k in range(12):
            out = vg.linearize_factors(gctx, fs, g.poses)
            vg.linearize_factors(gctx, fs, g.poses, use_graph=True, out=out)
            outs.append(out)
            assert fs.graph_count() == min(k + 1, 8)
        vg.linearize_factors(gctx, fs, g.poses, use_graph=True, out=outs[0])
    gctx.synchronize()
    assert fs.graph_count() == 8
    for out in outs:
        for k in ("H", "b", "e", "inliers"):
            assert np.array_equal(out[k].cpu().numpy(), base[k]), k


def test_results_do_not_depend_on_the_batch(vg, ctx, ragged):
    g = GpuWorkload(vg, ctx, ragged)
    full = g.linearize()
    for f in (3, 8, 9):
        alone = GpuWorkload(vg, ctx, ragged, factors=ragged.factors[f:f + 1])
        one = alone.linearize()
        for k in ("H", "b", "e", "inliers"):
            assert np.array_equal(one[k][0], full[k][f]), (f, k)


@pytest.mark.parametrize("accum", ACCS)
def test_evaluate_matches_linearize_and_the_oracle(vg, ctx, scans, ragged, accum):
    """The cost-only kernel (Eq. (3) for trial steps): e within 1e-5 of the
    oracle's cost and inliers bit-exact, and bit-identical to the e of the
    linearization with the same accumulation, in both schedules."""
    for w in (scans, ragged):
        _, ref = oracle_results(w, with_corr=False)
        g = GpuWorkload(vg, ctx, w)
        lin = g.linearize(accum=accum)
        ev = g.evaluate(accum=accum)
        assert np.array_equal(ev["inliers"], ref["inliers"])
        worst = 0.0
        for f in range(w.n_factors):
            if ref["inliers"][f] == 0:
                assert ev["e"][f] == 0.0
            else:
                worst = max(worst, abs(ev["e"][f] - ref["e"][f]) / ref["e"][f])
        print(f"{w.name} evaluate {accum}: worst relative error of e {worst:.2e}")
        assert worst <= TOL
        assert np.array_equal(ev["inliers"], lin["inliers"])
        assert np.array_equal(ev["e"], lin["e"])
        per = g.evaluate(accum=accum, schedule="per_factor")
        assert np.array_equal(per["e"], lin["e"])


# --------------------------------------------- degenerate fused covariances

def _oracle_degenerate_hits(w):
    """Hits of every factor whose fused covariance the oracle finds not
    positive definite."""
    from oracle.vgicp_oracle import _unpack_cov
    maps = oracle.build_maps(w.targets, w.resolution)
    n = 0
    for s, t, pi, pj in w.factors:
        x, c = w.sources[s]
        R, tt = oracle.relative_pose(w.poses[pi], w.poses[pj])
        corr = oracle.lookup(maps[t], x, R, tt)
        hit = corr >= 0
        F = oracle.fused_covariance(_unpack_cov(maps[t].cov[corr[hit]]), _unpack_cov(c[hit]), R)
        n += int((~oracle.positive_definite(F)).sum())
    return n


@pytest.mark.parametrize("fused,kappa", [("f64", 0.0), ("f32", 0.0), ("f32", 1e4)])
@pytest.mark.parametrize("accum", ACCS)
def test_degenerate_fused_covariances(vg, ctx, degenerate, accum, fused, kappa):
    """Hits whose fused covariance is zero, rank one or two, indefinite or
    has NaN or infinite entries: counted as inliers (correspondences
    bit-exact), adding nothing; H, b, e match the oracle (the all-FP32 fused
    covariance within its own tolerance), a factor of such hits alone is
    exactly zero, and the cost-only kernel agrees."""
    w = degenerate
    _, ref = oracle_results(w, with_corr=True)
    g = GpuWorkload(vg, ctx, w)
    tol = TOL if fused == "f64" else FUSED32_TOL
    elem = elem_tol_for(accum) if fused == "f64" else None
    got = g.linearize(accum=accum, fused=fused, fp64_kappa=kappa, with_corr=True)
    assert np.array_equal(got["corr"], np.concatenate(ref["corr"]).astype(np.int32))
    assert got["inliers"][2] == len(w.meta["kinds"][2])
    assert not got["H"][2].any() and not got["b"][2].any() and got["e"][2] == 0.0
    assert all(np.all(np.isfinite(got[k])) for k in ("H", "b", "e"))
    assert_linearize_parity(got, ref, tol=tol, elem_tol=elem)
    # with and without the degenerate points (tiles and summation order differ)
    for k in ("H", "b", "e"):
        assert rel_fro(got[k][0], got[k][3]) <= TOL, k
    # the counts of bad inputs: non-finite covariances of the clouds the set
    # copied, and the hits the oracle finds degenerate (as inliers adding nothing)
    chk = vg.check_inputs(ctx, g.fs)
    n_nonfinite = sum(int((~np.isfinite(c)).any(axis=1).sum()) for _, c in w.sources)
    assert chk["nonfinite_points"] == 0 and chk["nonfinite_covs"] == n_nonfinite
    if fused == "f64":   # FP32 positive-definiteness tests may round the other way
        assert chk["degenerate_hits"] == _oracle_degenerate_hits(w)
    ev = g.evaluate(accum=accum, fused=fused, fp64_kappa=kappa)
    assert np.array_equal(ev["inliers"], ref["inliers"])
    assert np.array_equal(ev["e"], got["e"])


# ------------------------------------------------------------------ overlap

def test_overlap_bitexact(vg, ctx, scans, ragged):
    for w in (scans, ragged):
        g = GpuWorkload(vg, ctx, w)
        got = g.overlap()
        maps = oracle.build_maps(w.targets, w.resolution)
        hits, ov = oracle.overlap_workload(w.sources, maps, w.poses, w.factors)
        assert np.array_equal(got["hits"], hits)
        assert np.array_equal(got["overlap"], ov)
        lin = g.linearize()
        assert np.array_equal(lin["inliers"], got["hits"])


def test_self_overlap_is_one_and_far_is_zero(vg, ctx, scans):
    import torch
    from tests.oracle_pins import hom, rows
    xyz, cov = scans.targets[0]
    d = vg.cloud_to_device(xyz, cov)
    m = vg.voxelize(ctx, *d, scans.resolution)
    far = hom(scans.poses[0])
    far[:3, 3] += [1e4, 0, 0]
    poses = torch.from_numpy(np.stack([scans.poses[0], rows(far)])).to("cuda")
    fs = vg.FactorSet(ctx, [d], [m], [(0, 0, 0, 0), (0, 0, 0, 1)], 2)
    out = vg.overlap(ctx, fs, poses)
    ctx.synchronize()
    assert out["hits"].tolist() == [xyz.shape[0], 0]
    assert out["overlap"].tolist() == [1.0, 0.0]


def test_transforms_beyond_the_key_range_miss(vg, ctx, cfg1):
    """Source points carried near and past the edge of the key range
    (|key| >= 2^20 voxels) miss like the oracle's, partly in range and partly
    out; nothing is added for them."""
    from tests.oracle_pins import hom, rows
    w = cfg1
    poses = [w.poses[0], w.poses[1]]
    for shift in (1048560.0, 1048600.0, -1048590.0, 3.0e7):
        Ti = hom(w.poses[0])
        Ti[:3, 3] += [shift * w.resolution, 0.0, 0.0]
        poses.append(rows(Ti))
    poses = np.stack(poses)
    factors = np.array([[0, 0, k, 1] for k in range(len(poses)) if k != 1], np.int32)
    wf = Workload(name="edge", resolution=w.resolution, sources=w.sources, targets=w.targets,
                  poses=poses, factors=factors, meta={})
    _, ref = oracle_results(wf, with_corr=True)
    g = GpuWorkload(vg, ctx, wf)
    got = g.linearize(with_corr=True)
    assert_linearize_parity(got, ref)
    assert np.array_equal(got["corr"], np.concatenate(ref["corr"]))
    assert ref["inliers"][0] > 0 and np.all(ref["inliers"][1:] == 0)
    ov = g.overlap()
    assert np.array_equal(ov["hits"], ref["inliers"])


def test_non_finite_source_points_miss(vg, ctx, cfg1):
    """Source points with NaN or infinite coordinates are misses (corr -1,
    nothing added), like finite points carried far outside the key range:
    the oracle gets such far points in their place."""
    xyz, cov = cfg1.sources[0]
    bad = np.arange(0, xyz.shape[0], 17)
    vals = np.array([np.nan, np.inf, -np.inf], np.float32)
    xyz_bad = xyz.copy()
    for j, i in enumerate(bad):
        xyz_bad[i, j % 3] = vals[j % 3]
    xyz_far = xyz.copy()
    xyz_far[bad] = np.float32(1.0e7)
    w_bad = Workload(name="nan", resolution=cfg1.resolution, sources=[(xyz_bad, cov)],
                     targets=cfg1.targets, poses=cfg1.poses, factors=cfg1.factors, meta={})
    w_far = Workload(name="far", resolution=cfg1.resolution, sources=[(xyz_far, cov)],
                     targets=cfg1.targets, poses=cfg1.poses, factors=cfg1.factors, meta={})
    _, ref = oracle_results(w_far, with_corr=True)
    g = GpuWorkload(vg, ctx, w_bad)
    got = g.linearize(with_corr=True)
    assert np.all(got["corr"][bad] == -1)
    assert np.array_equal(got["corr"], ref["corr"][0])
    assert_linearize_parity(got, ref)
    assert np.all(np.isfinite(got["H"])) and np.all(np.isfinite(got["b"]))
    # the factor set counted the bad points when it copied the cloud
    chk = vg.check_inputs(ctx, g.fs)
    assert chk == {"nonfinite_points": bad.size, "nonfinite_covs": 0, "degenerate_hits": 0}


def test_automatic_tile_size(vg, ctx, cfg1, ragged):
    """Small factor sets get the smallest whole-phase tile (768 points); an
    explicit tile is kept; results do not depend on it beyond rounding."""
    g = GpuWorkload(vg, ctx, ragged)
    assert g.fs.tile_points == 768
    fs = vg.FactorSet(ctx, g.src, g.maps, ragged.factors, ragged.poses.shape[0], 4608)
    assert fs.tile_points == 4608
    a = g.linearize()
    b = vg.linearize_factors(ctx, fs, g.poses)
    ctx.synchronize()
    assert np.array_equal(a["inliers"], b["inliers"].cpu().numpy())
    for f in range(ragged.factors.shape[0]):
        if a["inliers"][f]:
            assert rel_fro(b["H"][f].cpu().numpy(), a["H"][f]) < TOL


def test_tile_autotuning_keeps_parity(vg, ctx, scans, ragged):
    """Tuning picks one of the candidates, rebuilds the tiles, drops captured
    graphs, and the factors still match the oracle (and the graph replay the
    direct launch) afterwards."""
    import torch
    _, ref = oracle_results(ragged, with_corr=False)
    g = GpuWorkload(vg, ctx, ragged)
    stream = torch.cuda.Stream()
    sctx = vg.Context(0, stream=stream)
    fs = vg.FactorSet(sctx, g.src, g.maps, ragged.factors, ragged.poses.shape[0])
    with torch.cuda.stream(stream):
        poses = g.poses.clone()
        before = vg.linearize_factors(sctx, fs, poses)
        vg.linearize_factors(sctx, fs, poses, use_graph=True, out=before)
        best, ms = vg.tune_tiles(sctx, fs, poses, candidates=[1536, 768, 2304])
        assert best in (1536, 768, 2304) and fs.tile_points == best and ms > 0
        direct = vg.linearize_factors(sctx, fs, poses)
        graph = vg.linearize_factors(sctx, fs, poses, use_graph=True, out=before)
    stream.synchronize()
    got = {k: v.cpu().numpy() for k, v in direct.items()}
    assert_linearize_parity(got, ref)
    for k in ("H", "b", "e", "inliers"):
        assert torch.equal(graph[k], direct[k]), k
    with pytest.raises(vg.VgicpError):
        vg.tune_tiles(sctx, fs, poses, candidates=[100])


def test_empty_factor_set_is_a_no_op(vg, ctx, cfg1):
    import torch
    g = GpuWorkload(vg, ctx, cfg1)
    fs = vg.FactorSet(ctx, g.src, g.maps, np.zeros((0, 4), np.int32), 2)
    out = vg.linearize_factors(ctx, fs, g.poses)
    assert out["H"].shape == (0, 12, 12)
    ctx.synchronize()


def test_bad_arguments_raise(vg, ctx, cfg1):
    import torch
    g = GpuWorkload(vg, ctx, cfg1)
    with pytest.raises(vg.VgicpError):
        vg.FactorSet(ctx, g.src, g.maps, [(0, 1, 0, 1)], 2)
    with pytest.raises(vg.VgicpError):
        vg.FactorSet(ctx, g.src, g.maps, [(0, 0, 0, 1)], 2, tile_points=100)
    with pytest.raises(ValueError):
        vg.linearize_factors(ctx, g.fs, g.poses.float())
    with pytest.raises(ValueError):
        vg.linearize_factors(ctx, g.fs, g.poses[:1])
    out = vg.linearize_factors(ctx, g.fs, g.poses)
    with pytest.raises(vg.VgicpError):       # graph replay needs a side stream
        vg.linearize_factors(ctx, g.fs, g.poses, use_graph=True, out=out)
    with pytest.raises(ValueError):          # and caller-owned outputs
        vg.linearize_factors(ctx, g.fs, g.poses, use_graph=True)
    bad = dict(out, e=out["e"].float())
    with pytest.raises(ValueError):
        vg.linearize_factors(ctx, g.fs, g.poses, out=bad)
    with pytest.raises(ValueError):
        vg.evaluate_errors(ctx, g.fs, g.poses, out={"e": out["e"], "inliers": out["e"]})
    with pytest.raises(ValueError):
        vg.overlap(ctx, g.fs, g.poses, out={"hits": out["inliers"], "overlap": out["e"][:0]})
    ctx.synchronize()


@pytest.mark.parametrize("n,extent,r", [(60000, 12.0, 0.25), (200000, 30.0, 0.3),
                                        (5000, 500.0, 0.5)])
def test_dense_volumes_every_point_finds_its_voxel(vg, ctx, n, extent, r):
    """Uniform random volumes (many occupied bricks packed together, so brick
    records collide and lookups probe): under the identity every point finds
    its own voxel, and under a random pose the correspondences equal the
    oracle's, bit for bit."""
    rng = np.random.default_rng(n)
    xyz = (rng.random((n, 3)) * extent - extent / 2).astype(np.float32)
    cov = np.tile(np.array([1, 0, 0, 1, 0, 1], np.float32), (n, 1))
    vmap, inv = oracle.voxelize(xyz, cov, r)
    eye = pose_rows(np.eye(4))[0]
    T = np.eye(4)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    th = 0.3
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    T[:3, :3] = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)
    T[:3, 3] = rng.normal(size=3)
    poses = np.stack([eye, pose_rows(T)[0]])
    w = Workload(name="dense", resolution=r, sources=[(xyz, cov)], targets=[(xyz, cov)],
                 poses=poses, factors=np.array([[0, 0, 0, 0], [0, 0, 1, 0]], np.int32), meta={})
    got = GpuWorkload(vg, ctx, w).linearize(with_corr=True)
    corr = got["corr"].reshape(2, n)
    assert np.array_equal(corr[0], inv.astype(np.int32))
    R, t = oracle.relative_pose(poses[1], poses[0])
    assert np.array_equal(corr[1], oracle.lookup(vmap, xyz, R, t).astype(np.int32))
    assert got["inliers"][0] == n


# ----------------------------------------------------- factor-set source copies

def test_factor_set_reads_the_caller_clouds_only_at_creation(vg, ctx, scans):
    """A factor set keeps its own (spatially ordered) copy of every source
    cloud: overwriting the caller's arrays afterwards changes no output."""
    import torch
    g = GpuWorkload(vg, ctx, scans)
    before = g.linearize(with_corr=True)
    for (x, c) in g.src:
        x.fill_(float("nan"))
        c.fill_(float("nan"))
    torch.cuda.synchronize()
    after = g.linearize(with_corr=True)
    for k in ("H", "b", "e", "inliers", "corr"):
        assert np.array_equal(before[k], after[k]), k


def test_point_order_changes_only_the_summation_order(vg, ctx, scans):
    """Shuffling the points of every source cloud leaves the correspondences
    (which follow their points) and the inlier counts identical, and H, b, e
    within the tolerance: the library orders each cloud itself."""
    rng = np.random.default_rng(5)
    perms = [rng.permutation(x.shape[0]) for (x, _) in scans.sources]
    shuffled = Workload(name="shuffled", resolution=scans.resolution,
                        sources=[(x[p], c[p]) for (x, c), p in zip(scans.sources, perms)],
                        targets=scans.targets, poses=scans.poses, factors=scans.factors, meta={})
    a = GpuWorkload(vg, ctx, scans).linearize(with_corr=True)
    b = GpuWorkload(vg, ctx, shuffled).linearize(with_corr=True)
    assert np.array_equal(a["inliers"], b["inliers"])
    off = 0
    for s in scans.factors[:, 0]:
        n = scans.sources[s][0].shape[0]
        assert np.array_equal(a["corr"][off:off + n][perms[s]], b["corr"][off:off + n])
        off += n
    for f in range(len(scans.factors)):
        if a["inliers"][f]:
            for k in ("H", "b", "e"):
                assert rel_fro(b[k][f], a[k][f]) <= TOL, (f, k)


def test_target_order_copies_keep_parity(vg, ctx, scans, ragged):
    """vgicp_factorset_reorder gives every factor its own copy of its source
    ordered by target voxel at the given poses: correspondences (in the
    caller's point order) and inliers are unchanged, H, b, e stay within the
    tolerance of the oracle at those poses and at poses moved afterwards, a
    source shared by several factors is ordered per factor, and graph replay
    after the reorder writes the direct result."""
    import torch
    from tests.oracle_pins import hom, rows
    for w in (scans, ragged):
        _, ref = oracle_results(w, with_corr=True)
        g = GpuWorkload(vg, ctx, w)
        before = g.linearize(with_corr=True)
        vg.reorder_by_target(ctx, g.fs, g.poses)
        after = g.linearize(with_corr=True)
        assert np.array_equal(after["corr"], before["corr"])
        assert np.array_equal(after["corr"], np.concatenate(ref["corr"]).astype(np.int32))
        assert_linearize_parity(after, ref)
        ov = g.overlap()
        assert np.array_equal(ov["hits"], ref["inliers"])
        # poses moved by 5 cm / 0.5 degrees after the reorder
        rng = np.random.default_rng(3)
        moved = np.array(w.poses, copy=True)
        for p in range(moved.shape[0]):
            T = hom(moved[p])
            a = rng.normal(size=3)
            a *= np.deg2rad(0.5) / np.linalg.norm(a)
            K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
            dT = np.eye(4)
            dT[:3, :3] = np.eye(3) + K + K @ K / 2
            u, _, vt = np.linalg.svd(dT[:3, :3])
            dT[:3, :3] = u @ vt
            dT[:3, 3] = rng.normal(size=3) * 0.05 / np.sqrt(3)
            moved[p] = rows(T @ dT)
        wm = Workload(name=w.name + "_moved", resolution=w.resolution, sources=w.sources,
                      targets=w.targets, poses=moved, factors=w.factors, meta={})
        _, refm = oracle_results(wm, with_corr=True)
        pm = torch.from_numpy(moved).to("cuda")
        out = vg.linearize_factors(ctx, g.fs, pm, with_corr=True)
        ctx.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        assert np.array_equal(got["corr"], np.concatenate(refm["corr"]).astype(np.int32))
        assert_linearize_parity(got, refm)
    # graph replay after a reorder on a side stream
    side = torch.cuda.Stream()
    gctx = vg.Context(0, stream=side)
    g = GpuWorkload(vg, ctx, scans)
    fs = vg.FactorSet(gctx, g.src, g.maps, g.factors, g.poses.shape[0])
    with torch.cuda.stream(side):
        out = vg.linearize_factors(gctx, fs, g.poses)
        vg.linearize_factors(gctx, fs, g.poses, use_graph=True, out=out)
        vg.reorder_by_target(gctx, fs, g.poses)
        assert fs.graph_count() == 0
        direct = vg.linearize_factors(gctx, fs, g.poses)
        vg.linearize_factors(gctx, fs, g.poses, use_graph=True, out=out)
    gctx.synchronize()
    for k in ("H", "b", "e", "inliers"):
        assert torch.equal(out[k], direct[k]), k
