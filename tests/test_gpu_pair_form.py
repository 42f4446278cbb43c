"""The pair form (Eqs. (5)-(6) term by term: 78 upper-triangle entries of the
12 x 12 H, 12 of b and the cost per correspondence, in the target frame)
against the FP64 oracle, to the same bar as the source-frame form: inliers
bit-exact, every H and b sub-block, the elementwise metric and e within a
relative 1e-5 per factor (the plain FP32 accumulation's elementwise metric
within its derived 1e-4)."""

import ctypes

import numpy as np
import pytest

from synth import make_degenerate_workload, make_scan_workload, make_single_factor, make_tiny_workload
from tests.gpu_helpers import (FUSED32_TOL, TOL, GpuWorkload, assert_linearize_parity,
                               elem_tol_for, oracle_results, rel_fro)

pytestmark = pytest.mark.gpu

PAIR_ACCS = ["mixed", "f32", "f32_comp"]


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
def scans_ref(scans):
    return oracle_results(scans, with_corr=False)[1]


@pytest.mark.parametrize("accum", PAIR_ACCS)
def test_pair_form_single_and_ragged_factors(vg, ctx, cfg1, ragged, accum):
    for w, tiles in ((cfg1, (0,)), (ragged, (0, 256, 1024))):
        _, ref = oracle_results(w, with_corr=False)
        for tile in tiles:
            print(f"pair form {accum}: {w.name}, tile {tile}", flush=True)
            g = GpuWorkload(vg, ctx, w, tile_points=tile)
            got = g.linearize(accum=accum, form="pair")
            worst = assert_linearize_parity(got, ref, elem_tol=elem_tol_for(accum))
            print(f"  worst {max(worst.items(), key=lambda kv: kv[1][0])}")
            for f in range(got["H"].shape[0]):
                assert np.array_equal(got["H"][f], got["H"][f].T), f


@pytest.mark.parametrize("accum", PAIR_ACCS)
def test_pair_form_scan_factors(vg, ctx, scans, scans_ref, accum):
    g = GpuWorkload(vg, ctx, scans)
    got = g.linearize(accum=accum, form="pair")
    worst = assert_linearize_parity(got, scans_ref, elem_tol=elem_tol_for(accum))
    print(f"pair form scans {accum}: worst {max(worst.items(), key=lambda kv: kv[1][0])}")
    src = g.linearize(accum=accum, form="source")
    for k in ("H", "b", "e"):
        for f in range(got[k].shape[0]):
            assert rel_fro(got[k][f], src[k][f]) <= 2 * TOL, (k, f)


def test_pair_form_precision_variants(vg, ctx, scans, scans_ref):
    g = GpuWorkload(vg, ctx, scans)
    got = g.linearize(form="pair", fused="f32")
    assert_linearize_parity(got, scans_ref, tol=FUSED32_TOL, elem_tol=FUSED32_TOL)
    got = g.linearize(form="pair", fused="f32", fp64_kappa=1e3)
    assert_linearize_parity(got, scans_ref, tol=FUSED32_TOL, elem_tol=FUSED32_TOL)
    # the plain FP32 residual: blocks at 1e-4, elementwise at 1e-3 (as for the
    # source-frame form)
    got = g.linearize(form="pair", resid="f32")
    assert_linearize_parity(got, scans_ref, tol=1e-4, elem_tol=1e-3)


def test_pair_form_degenerate_fused_covariances(vg, ctx):
    w = make_degenerate_workload()
    _, ref = oracle_results(w, with_corr=False)
    g = GpuWorkload(vg, ctx, w)
    got = g.linearize(form="pair")
    assert got["inliers"][2] == len(w.meta["kinds"][2])
    assert not got["H"][2].any() and not got["b"][2].any() and got["e"][2] == 0.0
    assert all(np.all(np.isfinite(got[k])) for k in ("H", "b", "e"))
    assert_linearize_parity(got, ref)
    src_chk = vg.check_inputs(ctx, g.fs)
    g.linearize(form="source")
    assert vg.check_inputs(ctx, g.fs) == src_chk


def test_pair_form_schedules_and_graphs_are_bitwise_identical(vg, ctx, ragged):
    import torch
    g = GpuWorkload(vg, ctx, ragged)
    base = g.linearize(form="pair")
    per = g.linearize(form="pair", schedule="per_factor")
    for k in ("H", "b", "e", "inliers"):
        assert np.array_equal(base[k], per[k]), k
    side = torch.cuda.Stream()
    gctx = vg.Context(0, stream=side)
    fs2 = vg.FactorSet(gctx, g.src, g.maps, g.factors, g.poses.shape[0])
    F = fs2.n_factors
    out = {"H": torch.empty((F, 12, 12), dtype=torch.float64, device="cuda"),
           "b": torch.empty((F, 12), dtype=torch.float64, device="cuda"),
           "e": torch.empty((F,), dtype=torch.float64, device="cuda"),
           "inliers": torch.empty((F,), dtype=torch.int64, device="cuda")}
    for rep in range(3):
        for v in out.values():
            v.zero_()
        torch.cuda.synchronize()
        vg.linearize_factors(gctx, fs2, g.poses, use_graph=True, out=out, form="pair")
        gctx.synchronize()
        for k in ("H", "b", "e", "inliers"):
            assert np.array_equal(out[k].cpu().numpy(), base[k]), (rep, k)
        _ = g.linearize(form="source")   # unrelated eager work between replays
    vg.set_grid(ctx, g.fs, 64)
    got = g.linearize(form="pair")
    for k in ("H", "b", "e", "inliers"):
        assert np.array_equal(got[k], base[k]), k


def test_tuner_chooses_a_form(vg, ctx, scans, scans_ref):
    g = GpuWorkload(vg, ctx, scans)
    assert vg.form_of(g.fs) == "source"
    best, ms = vg.tune_tiles(ctx, g.fs, g.poses, candidates=[768, 2304])
    form = vg.form_of(g.fs)
    print(f"tuned: tile {best}, grid {vg.grid(g.fs)}, form {form}, {ms:.4f} ms")
    assert form in ("source", "pair") and best in (768, 2304)
    src_ms = vg.time_kernel(ctx, g.fs, g.poses, reps=5, form="source")
    pair_ms = vg.time_kernel(ctx, g.fs, g.poses, reps=5, form="pair")
    print(f"kernel: source form {src_ms:.4f} ms, pair form {pair_ms:.4f} ms")
    assert src_ms > 0 and pair_ms > 0
    got = g.linearize()   # form "auto": the tuned form
    assert_linearize_parity(got, scans_ref)
    # tuning one form leaves the kept form as it was
    vg.tune_tiles(ctx, g.fs, g.poses, candidates=[768], form="source")
    assert vg.form_of(g.fs) == form
    # "auto" falls back to the source-frame form where the pair form does not apply
    got = g.linearize(with_corr=True)
    assert "corr" in got
    got = g.linearize(accum="f64")
    assert_linearize_parity(got, scans_ref)


def test_pair_form_rejections(vg, ctx, cfg1):
    import torch
    g = GpuWorkload(vg, ctx, cfg1)
    with pytest.raises(vg.VgicpError) as ei:
        g.linearize(form="pair", with_corr=True)
    assert ei.value.code == vg.EINVAL
    with pytest.raises(vg.VgicpError) as ei:
        g.linearize(form="pair", accum="f64")
    assert ei.value.code == vg.EINVAL
    with pytest.raises(ValueError):
        g.linearize(form="both")
    F = g.fs.n_factors
    out = {"H": torch.empty((F, 12, 12), dtype=torch.float64, device="cuda"),
           "b": torch.empty((F, 12), dtype=torch.float64, device="cuda"),
           "e": torch.empty((F,), dtype=torch.float64, device="cuda"),
           "inliers": torch.empty((F,), dtype=torch.int64, device="cuda")}
    o = vg._opts("mixed", "batched", False, form="pair")
    rc = vg._lib.vgicp_linearize_factors_noalloc(
        ctx.handle, g.fs.handle, g.poses.data_ptr(), ctypes.byref(o), out["H"].data_ptr(),
        out["b"].data_ptr(), out["e"].data_ptr(), out["inliers"].data_ptr(), None)
    assert rc == vg.EINVAL
    cfg = vg.CServerConfig(0, 16, 1 << 20, 16, 2, 0, 0, vg._opts("mixed", "batched", False,
                                                                form="pair"))
    h = ctypes.c_void_p()
    assert vg._lib.vgicp_server_create(0, ctypes.byref(cfg), ctypes.byref(h)) == vg.EINVAL
    assert not h.value
    ctx.synchronize()
