"""Serving (GPU): continuous batching over resident keyframes.

  * a request's results are bit-identical alone, in a mix with other requests,
    split across batches, and through the factor-set path;
  * requests submitted while batches run are merged and overlap on the device;
  * the memory budget refuses frames (EFULL) and frees them on removal;
  * requests from several host threads all complete.
"""

import threading

import numpy as np
import pytest

from synth import make_scan_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import torch
    assert torch.cuda.is_available()
    from paper_2109_07073_amd import vgicp
    return vgicp


@pytest.fixture(scope="module")
def scans():
    return make_scan_workload(cfg=2, n_frames=12, n_factors=40, n_target=20000, workers=8)


def _frames(srv, w):
    return [srv.add_frame(x, c, w.resolution) for (x, c) in w.targets]


def test_alone_mix_split_and_factorset_agree(vg, scans):
    import torch
    srv = vg.Server(max_batch_factors=7, inflight=2)
    ids = _frames(srv, scans)
    fac = scans.factors.copy()
    fac[:, 0] = [ids[s] for s in fac[:, 0]]
    fac[:, 1] = [ids[t] for t in fac[:, 1]]
    A, B, C = fac[:15], fac[15:30], fac[30:]
    alone = srv.submit("linearize", A, scans.poses).wait()
    # the same request in a mix (and split over several 7-factor batches)
    reqs = [srv.submit("linearize", X, scans.poses) for X in (B, A, C, A)]
    for r in reqs:
        r.wait()
    for mixed in (reqs[1], reqs[3]):
        for k in ("H", "b", "e", "inliers"):
            assert np.array_equal(getattr(mixed, k), getattr(alone, k)), k
    # the factor-set path computes the same bits
    ctx = vg.Context(0)
    dev = [vg.cloud_to_device(x, c) for (x, c) in scans.targets]
    maps = [vg.voxelize(ctx, x, c, scans.resolution) for (x, c) in dev]
    fs = vg.FactorSet(ctx, dev, maps, scans.factors[:15], scans.poses.shape[0])
    out = vg.linearize_factors(ctx, fs, torch.from_numpy(scans.poses).to("cuda"))
    ctx.synchronize()
    for k in ("H", "b", "e", "inliers"):
        assert np.array_equal(out[k].cpu().numpy(), getattr(alone, k)), k
    st = srv.stats()
    assert st["max_requests_per_batch"] >= 2 and st["batches"] >= 6
    print("server stats", st, "latency ms", [round(r.latency_ms, 3) for r in reqs])
    srv.close()


def test_evaluate_and_overlap_requests(vg, scans):
    import torch
    srv = vg.Server(inflight=3)
    ids = _frames(srv, scans)
    fac = scans.factors.copy()
    fac[:, 0] = [ids[s] for s in fac[:, 0]]
    fac[:, 1] = [ids[t] for t in fac[:, 1]]
    lin = srv.submit("linearize", fac, scans.poses)
    ev = srv.submit("evaluate", fac, scans.poses)
    ov = srv.submit("overlap", fac, scans.poses)
    for r in (lin, ev, ov):
        r.wait()
    assert np.array_equal(ev.e, lin.e) and np.array_equal(ev.inliers, lin.inliers)
    assert np.array_equal(ov.inliers, lin.inliers)
    n = np.array([scans.sources[s][0].shape[0] for s in scans.factors[:, 0]])
    assert np.array_equal(ov.overlap, ov.inliers / n)
    srv.close()


def test_memory_budget_admission(vg, scans):
    srv = vg.Server(memory_budget_bytes=1)
    with pytest.raises(vg.VgicpError) as ex:
        srv.add_frame(*scans.targets[0], scans.resolution)
    assert ex.value.code == vg.EFULL
    srv.close()
    probe = vg.Server()
    fid = probe.add_frame(*scans.targets[0], scans.resolution)
    one = probe.memory()[0]
    probe.close()
    srv = vg.Server(memory_budget_bytes=int(one * 2.5))
    a = srv.add_frame(*scans.targets[0], scans.resolution)
    b = srv.add_frame(*scans.targets[1], scans.resolution)
    with pytest.raises(vg.VgicpError) as ex:
        srv.add_frame(*scans.targets[2], scans.resolution)
    assert ex.value.code == vg.EFULL
    srv.remove_frame(a)
    c = srv.add_frame(*scans.targets[2], scans.resolution)
    assert srv.memory()[0] <= int(one * 2.5)
    # unknown frames and out-of-range poses are refused at submit
    with pytest.raises(vg.VgicpError):
        srv.submit("linearize", [(a, b, 0, 1)], scans.poses)
    with pytest.raises(vg.VgicpError):
        srv.submit("linearize", [(b, c, 0, 10**6)], scans.poses)
    r = srv.submit("overlap", [(b, c, 0, 1)], scans.poses).wait()
    assert r.inliers[0] >= 0
    srv.close()


def test_threads_submit_concurrently(vg, scans):
    srv = vg.Server(max_batch_factors=16, inflight=2)
    ids = _frames(srv, scans)
    fac = scans.factors.copy()
    fac[:, 0] = [ids[s] for s in fac[:, 0]]
    fac[:, 1] = [ids[t] for t in fac[:, 1]]
    ref = srv.submit("linearize", fac, scans.poses).wait()
    results = {}

    def client(k):
        rs = [srv.submit("linearize", fac[k::4], scans.poses) for _ in range(3)]
        results[k] = [r.wait() for r in rs]

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for k, rs in results.items():
        for r in rs:
            assert np.array_equal(r.H, ref.H[k::4]) and np.array_equal(r.e, ref.e[k::4])
    srv.close()
