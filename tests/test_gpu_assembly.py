"""Assembly of the global linear system on the GPU against the FP64 oracle.

The per-factor H and b already carry the parity bound of the linearization
(relative 1e-5 per factor); a block of the global system is a sum of such
contributions, so its error is bounded by 1e-5 times the sum of the norms of
the contributions (triangle inequality), which is what the tests check.  The
pair list is host logic and must be exact; the device sums run in factor
order and must repeat bit for bit."""

import numpy as np
import pytest

import oracle
from synth import make_scan_workload
from tests.gpu_helpers import TOL, GpuWorkload, oracle_results
from tests.oracle_pins import small_pose_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2109_07073_amd import vgicp
    return vgicp


@pytest.fixture(scope="module")
def ctx(vg):
    return vg.Context(0)


def _expected_pairs(factors):
    return sorted({(min(i, j), max(i, j)) for (_, _, i, j) in factors if i != j})


def _contribution_norms(ref, factors, P, pairs):
    """Sum over contributing factors of the norm of each added block."""
    nd = np.zeros(P)
    nb = np.zeros(P)
    no = np.zeros(len(pairs))
    index = {p: k for k, p in enumerate(pairs)}
    for f, (_, _, i, j) in enumerate(factors):
        H, b = ref["H"][f], ref["b"][f]
        nd[i] += np.linalg.norm(H[:6, :6])
        nd[j] += np.linalg.norm(H[6:, 6:])
        nb[i] += np.linalg.norm(b[:6])
        nb[j] += np.linalg.norm(b[6:])
        if i == j:
            nd[i] += 2 * np.linalg.norm(H[:6, 6:])
        else:
            no[index[(min(i, j), max(i, j))]] += np.linalg.norm(H[:6, 6:])
    return nd, nb, no


def _check(vg, ctx, w, ref):
    import torch
    g = GpuWorkload(vg, ctx, w)
    P = w.poses.shape[0]
    pairs = _expected_pairs(w.factors)
    assert [tuple(p) for p in g.fs.pairs] == pairs
    lin = vg.linearize_factors(ctx, g.fs, g.poses)
    a1 = vg.assemble_system(ctx, g.fs, lin["H"], lin["b"])
    a2 = vg.assemble_system(ctx, g.fs, lin["H"], lin["b"])
    ctx.synchronize()
    got = {k: v.cpu().numpy() for k, v in a1.items()}
    for k in a1:
        assert torch.equal(a1[k], a2[k]), k
    Hg, bg = oracle.assemble_system(ref["H"], ref["b"], w.factors, P)
    diag, bvec, off = oracle.system_blocks(Hg, bg, P, pairs)
    nd, nb, no = _contribution_norms(ref, w.factors, P, pairs)
    worst = 0.0
    for p in range(P):
        err = np.linalg.norm(got["Hdiag"][p] - diag[p])
        assert err <= TOL * nd[p] + 1e-300, (p, err, nd[p])
        assert np.linalg.norm(got["bvec"][p] - bvec[p]) <= TOL * nb[p] + 1e-300, p
        worst = max(worst, err / max(nd[p], 1e-300))
    for k in range(len(pairs)):
        assert np.linalg.norm(got["Hoff"][k] - off[k]) <= TOL * no[k] + 1e-300, pairs[k]
    # untouched poses are exact zeros
    touched = set(w.factors[:, 2]) | set(w.factors[:, 3])
    for p in range(P):
        if p not in touched:
            assert not np.any(got["Hdiag"][p]) and not np.any(got["bvec"][p])
    return worst


def test_small_pose_graph(vg, ctx):
    w = small_pose_graph()
    _, ref = oracle_results(w, with_corr=False)
    _check(vg, ctx, w, ref)


def test_scan_pose_graph(vg, ctx):
    w = make_scan_workload(cfg=2, n_frames=30, n_factors=90, n_target=20000, workers=8)
    _, ref = oracle_results(w, with_corr=False)
    print("worst diag block error / bound", _check(vg, ctx, w, ref))


def test_without_offdiagonal_blocks_and_untouched_poses(vg, ctx):
    w = small_pose_graph()
    # two more poses that no factor touches
    w.poses = np.vstack([w.poses, w.poses[:2]])
    _, ref = oracle_results(w, with_corr=False)
    _check(vg, ctx, w, ref)
    g = GpuWorkload(vg, ctx, w)
    lin = vg.linearize_factors(ctx, g.fs, g.poses)
    full = vg.assemble_system(ctx, g.fs, lin["H"], lin["b"])
    part = vg.assemble_system(ctx, g.fs, lin["H"], lin["b"], with_offdiag=False)
    ctx.synchronize()
    assert "Hoff" not in part
    assert np.array_equal(full["Hdiag"].cpu().numpy(), part["Hdiag"].cpu().numpy())


def test_empty_factor_set(vg, ctx):
    import torch
    w = small_pose_graph()
    g = GpuWorkload(vg, ctx, w, factors=np.zeros((0, 4), np.int32))
    assert g.fs.pairs.shape == (0, 2)
    H = torch.empty((0, 12, 12), dtype=torch.float64, device="cuda")
    b = torch.empty((0, 12), dtype=torch.float64, device="cuda")
    out = vg.assemble_system(ctx, g.fs, H, b)
    ctx.synchronize()
    assert not out["Hdiag"].any() and not out["bvec"].any()
    with pytest.raises(ValueError):
        vg.assemble_system(ctx, g.fs, H[:, :6], b)


def test_fully_connected_local_graph(vg, ctx):
    """The local-mapping shape: every pair of 8 consecutive frames of a drive."""
    from synth import Workload, drive_positions, pose_rows, stream_scan_frames
    N = 8
    pos = drive_positions(6, 160)[120:120 + N]
    fr = list(stream_scan_frames(2, N, positions=pos, perturb=(0.02, 0.2), workers=1))
    clouds = [(x, c) for (_, _, x, c) in fr]
    w = Workload(name="local8", resolution=0.5, sources=clouds, targets=clouds,
                 poses=pose_rows([T for (_, T, _, _) in fr]),
                 factors=np.array([(a, b, a, b) for a in range(N) for b in range(a)], np.int32),
                 meta={})
    _, ref = oracle_results(w, with_corr=False)
    assert np.all(ref["inliers"] > 1000)
    _check(vg, ctx, w, ref)
