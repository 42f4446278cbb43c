"""Serving (GPU): continuous batching over resident keyframes.

  * a request's results are bit-identical alone, in a mix with other requests,
    split across batches, and through the factor-set path;
  * requests submitted while batches run are merged and overlap on the device;
  * the memory budget refuses frames (EFULL) and frees them on removal;
  * requests from several host threads all complete;
  * linearize, evaluate and overlap results match the FP64 oracle alone,
    mixed and split across batches.
"""

import threading

import numpy as np
import pytest

import oracle
from synth import make_scan_workload
from tests.gpu_helpers import TOL, assert_linearize_parity

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
    with vg.Server(max_batch_factors=7, inflight=2) as srv:
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
        st = srv.stats()
    for mixed in (reqs[1], reqs[3]):
        for k in ("H", "b", "e", "inliers"):
            assert np.array_equal(getattr(mixed, k), getattr(alone, k)), k
    # the factor-set path computes the same bits with the server's tile size
    ctx = vg.Context(0)
    dev = [vg.cloud_to_device(x, c) for (x, c) in scans.targets]
    maps = [vg.voxelize(ctx, x, c, scans.resolution) for (x, c) in dev]
    fs = vg.FactorSet(ctx, dev, maps, scans.factors[:15], scans.poses.shape[0], tile_points=4608)
    out = vg.linearize_factors(ctx, fs, torch.from_numpy(scans.poses).to("cuda"))
    ctx.synchronize()
    for k in ("H", "b", "e", "inliers"):
        assert np.array_equal(out[k].cpu().numpy(), getattr(alone, k)), k
    print("server stats", st, "latency ms", [round(r.latency_ms, 3) for r in reqs])
    assert st["max_requests_per_batch"] >= 2 and st["batches"] >= 6


def test_requests_reuse_host_buffers(vg, scans):
    """A request submitted with out= writes into a finished request's arrays
    (an optimizer's next round) and gives the same bits; an unfinished or
    mismatched request is refused."""
    with vg.Server(max_batch_factors=9, inflight=2) as srv:
        ids = _frames(srv, scans)
        fac = scans.factors.copy()
        fac[:, 0] = [ids[s] for s in fac[:, 0]]
        fac[:, 1] = [ids[t] for t in fac[:, 1]]
        first = srv.submit("linearize", fac[:20], scans.poses).wait()
        ref = {k: getattr(first, k).copy() for k in ("H", "b", "e", "inliers")}
        for k in ("H", "b", "e"):
            getattr(first, k)[...] = np.nan
        again = srv.submit("linearize", fac[:20], scans.poses, out=first)
        with pytest.raises(ValueError):   # still in flight
            srv.submit("linearize", fac[:20], scans.poses, out=again)
        again.wait()
        assert again.H is first.H
        for k in ref:
            assert np.array_equal(getattr(again, k), ref[k]), k
        with pytest.raises(ValueError):   # another size
            srv.submit("linearize", fac[:19], scans.poses, out=again)
        with pytest.raises(ValueError):   # another kind
            srv.submit("evaluate", fac[:20], scans.poses, out=again)


def test_submit_many_matches_single_submits(vg, scans):
    """Requests queued together (vgicp_server_submit_many) give the bits of the
    same requests submitted one by one, share batches, reuse host buffers, and
    an invalid request queues none of them."""
    with vg.Server(max_batch_factors=64, inflight=2) as srv:
        ids = _frames(srv, scans)
        fac = scans.factors.copy()
        fac[:, 0] = [ids[s] for s in fac[:, 0]]
        fac[:, 1] = [ids[t] for t in fac[:, 1]]
        parts = [("linearize", fac[:12], scans.poses), ("linearize", fac[12:], scans.poses),
                 ("evaluate", fac, scans.poses), ("overlap", fac[:7], scans.poses)]
        single = [srv.submit(*p).wait() for p in parts]
        before = srv.stats()["batches"]
        many = [r.wait() for r in srv.submit_many(parts)]
        # the two linearize requests went out in one batch
        assert srv.stats()["batches"] - before <= 3
        for a, b in zip(single, many):
            for k in ("H", "b", "e", "inliers", "overlap"):
                x, y = getattr(a, k), getattr(b, k)
                assert (x is None) == (y is None), k
                if x is not None:
                    assert np.array_equal(x, y), (a.kind, k)
        # the next round reuses the first round's host arrays
        again = [r.wait() for r in srv.submit_many([p + (m,) for p, m in zip(parts, many)])]
        for a, b in zip(many, again):
            assert b.inliers is a.inliers
        # one request's arrays serve one request in flight
        with pytest.raises(ValueError):
            srv.submit_many([parts[0] + (again[0],), parts[0] + (again[0],)])
        # all or nothing: a bad frame id in the last request queues none
        bad = fac[:3].copy()
        bad[0, 0] = 10**6
        n_req = srv.stats()["requests"]
        with pytest.raises(vg.VgicpError) as ei:
            srv.submit_many([parts[0], ("linearize", bad, scans.poses)])
        assert ei.value.code == vg.EINVAL
        # a request queued by the failed call would complete before this one
        srv.submit(*parts[3]).wait()
        assert srv.stats()["requests"] == n_req + 1
        assert srv.submit_many([]) == []


def test_evaluate_and_overlap_requests(vg, scans):
    with vg.Server(inflight=3) as srv:
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


def test_memory_budget_admission(vg, scans):
    with vg.Server(memory_budget_bytes=1) as srv:
        with pytest.raises(vg.VgicpError) as ex:
            srv.add_frame(*scans.targets[0], scans.resolution)
        assert ex.value.code == vg.EFULL
        assert srv.memory()[0] == 0
    # frame sizes differ (the brick table size is a power of two): measure each
    size = []
    with vg.Server() as probe:
        for k in range(3):
            before = probe.memory()[0]
            probe.add_frame(*scans.targets[k], scans.resolution)
            size.append(probe.memory()[0] - before)
    budget = sum(size) - 1           # any two frames fit, all three do not
    with vg.Server(memory_budget_bytes=budget) as srv:
        a = srv.add_frame(*scans.targets[0], scans.resolution)
        b = srv.add_frame(*scans.targets[1], scans.resolution)
        assert srv.memory()[0] == size[0] + size[1]
        with pytest.raises(vg.VgicpError) as ex:
            srv.add_frame(*scans.targets[2], scans.resolution)
        assert ex.value.code == vg.EFULL
        assert srv.memory()[0] == size[0] + size[1]
        srv.remove_frame(a)
        with pytest.raises(vg.VgicpError):
            srv.submit("linearize", [(a, b, 0, 1)], scans.poses)   # removed frame
        c = srv.add_frame(*scans.targets[2], scans.resolution)     # may reuse a's id
        assert srv.memory()[0] == size[1] + size[2] <= budget
        # unknown frames and out-of-range poses are refused at submit
        with pytest.raises(vg.VgicpError):
            srv.submit("linearize", [(10**6, b, 0, 1)], scans.poses)
        with pytest.raises(vg.VgicpError):
            srv.submit("linearize", [(b, c, 0, 10**6)], scans.poses)
        r = srv.submit("overlap", [(b, c, 0, 1)], scans.poses).wait()
    assert r.inliers[0] >= 0


def test_threads_submit_concurrently(vg, scans):
    results = {}
    with vg.Server(max_batch_factors=16, inflight=2) as srv:
        ids = _frames(srv, scans)
        fac = scans.factors.copy()
        fac[:, 0] = [ids[s] for s in fac[:, 0]]
        fac[:, 1] = [ids[t] for t in fac[:, 1]]
        ref = srv.submit("linearize", fac, scans.poses).wait()

        def client(k):
            rs = [srv.submit("linearize", fac[k::4], scans.poses) for _ in range(3)]
            results[k] = [r.wait() for r in rs]

        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    assert sorted(results) == [0, 1, 2, 3]
    for k, rs in results.items():
        for r in rs:
            assert np.array_equal(r.H, ref.H[k::4]) and np.array_equal(r.e, ref.e[k::4])


def test_unwaited_requests_finish_before_close(vg, scans):
    """Requests nobody waits for still complete into their arrays before the
    server is freed; the binding keeps their arrays alive until then."""
    with vg.Server(max_batch_factors=5, inflight=2) as srv:
        ids = _frames(srv, scans)
        fac = scans.factors.copy()
        fac[:, 0] = [ids[s] for s in fac[:, 0]]
        fac[:, 1] = [ids[t] for t in fac[:, 1]]
        ref = srv.submit("linearize", fac, scans.poses).wait()
        reqs = [srv.submit("linearize", fac, scans.poses) for _ in range(3)]
    for r in reqs:
        assert np.array_equal(r.H, ref.H) and np.array_equal(r.inliers, ref.inliers)


def test_server_results_match_the_oracle(vg, scans):
    """Each request kind against the oracle (the server's frames are the
    workload's target clouds, used both as sources and as targets): alone,
    then the three kinds in flight together with a second linearize request
    over an overlapping range, every request split over 7-factor batches."""
    maps = oracle.build_maps(scans.targets, scans.resolution)
    ref = oracle.linearize_workload(scans.targets, maps, scans.poses, scans.factors)
    hits, rate = oracle.overlap_workload(scans.targets, maps, scans.poses, scans.factors)
    with vg.Server(max_batch_factors=7, inflight=2) as srv:
        ids = _frames(srv, scans)
        fac = scans.factors.copy()
        fac[:, 0] = [ids[s] for s in fac[:, 0]]
        fac[:, 1] = [ids[t] for t in fac[:, 1]]
        alone = {k: srv.submit(k, fac, scans.poses).wait()
                 for k in ("linearize", "evaluate", "overlap")}
        # the second linearize request queues right behind the first, so the
        # first's last batch (40 = 5 * 7 + 5 factors) takes two of its
        # factors: one batch serves both requests
        mixed = {"linearize": srv.submit("linearize", fac, scans.poses)}
        part = srv.submit("linearize", fac[10:25], scans.poses)
        mixed.update({k: srv.submit(k, fac, scans.poses) for k in ("evaluate", "overlap")})
        for r in list(mixed.values()) + [part]:
            r.wait()
        st = srv.stats()
    sub = {k: v[10:25] for k, v in ref.items()}
    for run in (alone, mixed):
        lin = run["linearize"]
        assert_linearize_parity({"H": lin.H, "b": lin.b, "e": lin.e, "inliers": lin.inliers}, ref)
        ev = run["evaluate"]
        assert np.array_equal(ev.inliers, ref["inliers"])
        for f in range(len(fac)):
            if ref["inliers"][f]:
                assert abs(ev.e[f] - ref["e"][f]) <= TOL * ref["e"][f], f
        ov = run["overlap"]
        assert np.array_equal(ov.inliers, hits) and np.array_equal(ov.overlap, rate)
    assert_linearize_parity({"H": part.H, "b": part.b, "e": part.e, "inliers": part.inliers}, sub)
    print("server stats", st)
    assert st["max_requests_per_batch"] >= 2
