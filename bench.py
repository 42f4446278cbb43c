"""Benchmark: VGICP factor linearization rounds on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload batched4500|scan500|single|serving|local]

A step is one linearization round: every factor of the batch is relinearized
at the current poses (relative pose, FP32 transform and voxel lookup, fused
covariance inverse, per-point Hessian/gradient/cost terms, atomic-free
per-factor reduction and expansion to the 12x12 Hessian factor).  The voxel
maps are built once per frame at ingest and the overlap of every pair once at
factor creation; both are timed in the same run and reported under "stages".

Prints ONE JSON line (see the keys below).  Everything is seeded synthetic
input; inputs are resident in HBM before timing starts.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s

WORKLOADS = {
    # 1,000 corridor frames, 4,500 factors, sources U{5,000..40,000}, r = 0.5 m
    "batched4500": dict(cfg=3, n_frames=1000, n_factors=4500, src_range=(5000, 40000)),
    # 100 frames of 20,000 points, 500 factors between frames within 20 m
    "scan500": dict(cfg=2, n_frames=100, n_factors=500, src_range=None),
    # one 2,000 x 2,000 factor on the room scene, r = 1.0 m
    "single": dict(cfg=1),
    # keyframes streamed into the continuous-batching server (see run_serving)
    "serving": dict(cfg=5),
    # local mapping: overlap-gated submaps of fully connected factor graphs (see run_local)
    "local": dict(cfg=6),
    # precision study: batched4500 plus 450 ill-conditioned factors (see run_precision)
    "precision": dict(cfg=4),
}


# Blocks of the 12x12 factor and the 12-vector b in the order [omega_i,
# rho_i, omega_j, rho_j]: each 6x6 block split into rotation (w) and
# translation (r) parts, so that an error confined to a small block is not
# hidden by the large (w, w) entries.
_BLK = {"w_i": slice(0, 3), "r_i": slice(3, 6), "w_j": slice(6, 9), "r_j": slice(9, 12)}
_H_BLOCKS = [("w_i", "w_i"), ("w_i", "r_i"), ("r_i", "r_i"), ("w_i", "w_j"), ("w_i", "r_j"),
             ("r_i", "w_j"), ("r_i", "r_j"), ("w_j", "w_j"), ("w_j", "r_j"), ("r_j", "r_j")]


def parity_metrics(H, b, e, Hr, br, er):
    """Relative errors of one factor against the FP64 oracle: whole-factor
    Frobenius norms of H and b, every H and b block, the elementwise metric
    |d| / (|ref| + 1e-3 max|ref|) of H and of b, and e."""
    def fro(g, r):
        d = np.linalg.norm(r)
        return float(np.linalg.norm(g - r) / d) if d > 0 else float(np.linalg.norm(g))

    def elem(g, r):
        m = np.abs(r).max()
        return float((np.abs(g - r) / (np.abs(r) + 1e-3 * m)).max()) if m > 0 else float(np.abs(g).max())
    out = {"H": fro(H, Hr), "b": fro(b, br), "e": abs(float(e) - er) / abs(er) if er else abs(float(e)),
           "H_elem": elem(H, Hr), "b_elem": elem(b, br)}
    for a, c in _H_BLOCKS:
        out[f"H_{a}{c}"] = fro(H[_BLK[a], _BLK[c]], Hr[_BLK[a], _BLK[c]])
    for a in _BLK:
        out[f"b_{a}"] = fro(b[_BLK[a]], br[_BLK[a]])
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name: str):
    from synth import make_scan_workload, make_single_factor
    spec = WORKLOADS[name]
    if name == "single":
        return make_single_factor()
    return make_scan_workload(cfg=spec["cfg"], n_frames=spec["n_frames"],
                              n_factors=spec["n_factors"], src_range=spec["src_range"])


def profiled_traffic(workload: str, tile_points: int | None = None, layout: str | None = None):
    """HBM bytes per linearize launch measured by rocprofv3 (FETCH_SIZE and
    WRITE_SIZE, scaled by a copy-kernel calibration) for this workload, from
    profiles/k_linearize_<workload>.md, or None when there is no profile, the
    kernel sources have changed since it was taken, or no figure was taken at
    this tile size and tile-table layout."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_linearize_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            key, _, val = line.strip().partition(": ")
            if key in ("traffic_bytes_per_launch", "source_sha256_16", "tile_points", "layout") or \
                    key.startswith("traffic_bytes_per_launch_at_"):
                fields[key] = val.strip()
    csrc = os.path.join(ROOT, "paper_2109_07073_amd", "csrc")
    h = hashlib.sha256()
    for f in ("linearize.hip", "voxelize.hip", "vgicp_internal.hpp", "reorder.hip"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    if fields.get("source_sha256_16") != h.hexdigest()[:16]:
        return None
    if layout is not None and fields.get("layout", "grouped") != layout:
        return None
    if tile_points is None or fields.get("tile_points") == str(tile_points):
        return float(fields["traffic_bytes_per_launch"])
    other = fields.get(f"traffic_bytes_per_launch_at_{tile_points}")
    return float(other) if other is not None else None


def measured_copy_gbs(nbytes=1 << 30, reps=10):
    """Device-to-device copy rate of a plain torch copy (read + write bytes per
    second), the practical HBM ceiling the roofline fraction is also quoted
    against."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    t1.synchronize()
    gbs = 2.0 * nbytes * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def distinct_voxels(fs_sizes, corr_t):
    """U_f: distinct target voxels touched per factor, from the per-point
    correspondence output (device tensor)."""
    import torch
    F = len(fs_sizes)
    fid = torch.repeat_interleave(torch.arange(F, device=corr_t.device),
                                  torch.as_tensor(fs_sizes, device=corr_t.device))
    hit = corr_t >= 0
    key = fid[hit].to(torch.int64) * (1 << 32) + corr_t[hit].to(torch.int64)
    u = torch.unique(key)
    return torch.bincount((u >> 32), minlength=F).cpu().numpy()


_CPU_W = None     # the workload, inherited by forked oracle workers


def _oracle_worker(args):
    """Linearize factors order[k::stride] with the oracle until the budget runs out."""
    import oracle
    k, stride, order, budget_s = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:       # pragma: no cover
        pass
    w = _CPU_W
    maps, outs = {}, []
    t0 = time.perf_counter()
    for f in order[k::stride]:
        s, tg, pi, pj = w.factors[f]
        if tg not in maps:
            maps[tg] = oracle.voxelize(*w.targets[tg], w.resolution)[0]
        o = oracle.linearize_factor(*w.sources[s], maps[tg], w.poses[pi], w.poses[pj])
        outs.append((int(f), {"H": o["H"], "b": o["b"], "e": o["e"], "inliers": o["inliers"]},
                     int(w.sources[s][0].shape[0])))
        if time.perf_counter() - t0 > budget_s:
            break
    return outs, time.perf_counter() - t0


def cpu_baseline(w, cpu_seconds: float = 24.0, workers: int = 1):
    """The FP64 oracle on a bounded sample of the workload's factors, over
    `workers` forked processes of one thread each (factors dealt round-robin
    from a seeded permutation; each process stops once it has used its share
    of `cpu_seconds`).  Must run before the process touches the GPU.  Returns
    (corr/s, processes, sample text, factor ids, outputs)."""
    workers = max(1, min(workers, w.n_factors))   # no process without a factor of its own
    budget_s = cpu_seconds / workers
    import multiprocessing as mp
    global _CPU_W
    _CPU_W = w
    order = np.random.default_rng(7).permutation(w.n_factors)
    jobs = [(k, workers, order, budget_s) for k in range(workers)]
    t0 = time.perf_counter()
    if workers == 1:
        res = [_oracle_worker(jobs[0])]
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    ids, outs, inl, pts = [], [], 0, 0
    busy = sum(t for _, t in res)
    for chunk, _ in res:
        for f, o, n in chunk:
            ids.append(f)
            outs.append(o)
            inl += int(o["inliers"])
            pts += n
    sample = (f"{len(ids)} of {w.n_factors} factors ({pts} source points, {inl} correspondences) "
              f"linearized by the FP64 numpy oracle, voxel maps included, {workers} processes "
              f"of 1 thread, {wall:.2f} s wall, {busy:.2f} s of CPU work")
    # one process runs in this one: its own clock leaves out the oracle's import
    return inl / (wall if workers > 1 else busy), workers, sample, ids, outs


def cpu_single_process(w, seconds: float = 3.0):
    """The same oracle in this one process (one thread), on the first factors
    of the same seeded order for about `seconds`: correspondences per second."""
    global _CPU_W
    _CPU_W = w
    order = np.random.default_rng(7).permutation(w.n_factors)
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):      # the worker's own one-thread limit ends here too
        outs, t = _oracle_worker((0, 1, order, seconds))
    return sum(int(o["inliers"]) for _, o, _ in outs) / t, len(outs)


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_all(w, workers: int):
    """The FP64 oracle over every factor of w (forked processes, no time
    budget), as {factor: outputs}.  Must run before the GPU is touched.
    Returns (outputs, correspondences per second, wall seconds)."""
    import multiprocessing as mp
    global _CPU_W
    _CPU_W = w
    order = np.arange(w.n_factors)
    jobs = [(k, workers, order, float("inf")) for k in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    outs = {f: o for chunk, _ in res for f, o, _ in chunk}
    corr = sum(int(o["inliers"]) for o in outs.values())
    return outs, corr / wall, wall


PRECISION_VARIANTS = [
    # (accumulation, residual, fused covariance, fp64_kappa); the first is the default
    ("mixed", "f64", "f64", 0.0), ("f32", "f64", "f64", 0.0), ("f32_comp", "f64", "f64", 0.0),
    ("f64", "f64", "f64", 0.0),
    ("f32", "f64", "f32", 0.0), ("f32", "f64", "f32", 1e3), ("f32", "f64", "f32", 1e4),
    ("f32", "f64", "f32", 1e5), ("f64", "f64", "f32", 1e4), ("f32", "f32", "f64", 0.0),
]


def run_precision(args):
    """Precision study at full size: the batched4500 round (k-NN covariances,
    spectrum 1, 1, 1e-3, at the perturbed pose estimates) and 450
    ill-conditioned factors (the first 450 pairs, analytic surface-normal
    covariances with spectrum 1, 1, 1e-6) at the estimates and at the ground
    truth.  For each accumulation / residual / fused-covariance / FP64-gate
    variant: max and p99 relative Frobenius error of H, b and e over the
    factors against the FP64 oracle (every factor), the worst block and
    elementwise error, the fraction of correspondences that formed the fused
    covariance in FP64, and the device time of a round (HIP graph replay)."""
    import copy
    from synth import make_scan_workload
    t_gen = time.perf_counter()
    w = make_scan_workload(cfg=3, n_frames=1000, n_factors=4500, src_range=(5000, 40000),
                           ill_eps=1e-6)
    ill = copy.copy(w)
    ill.sources = w.meta["ill"]["sources"]
    ill.targets = w.meta["ill"]["targets"]
    ill.factors = w.factors[:450].copy()
    ill.meta = {}
    ill_gt = copy.copy(ill)
    ill_gt.poses = w.meta["poses_gt"]
    sets = {"regular": w, "ill": ill, "ill_gt": ill_gt}
    log(f"[bench] precision workload generated in {time.perf_counter() - t_gen:.1f} s")
    workers = max(1, min(args.cpu_workers, os.cpu_count() or 1))
    refs, cpu_rate, cpu_wall = {}, {}, {}
    for name, ws in sets.items():
        refs[name], cpu_rate[name], cpu_wall[name] = oracle_all(ws, workers)
        log(f"[bench] oracle {name}: {ws.n_factors} factors in {cpu_wall[name]:.1f} s")

    import torch
    from paper_2109_07073_amd import vgicp as vg
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.Stream()
    ctx = vg.Context(0, stream=stream)
    steps = max(1, min(args.steps, 20))
    table, default_ms, default_corr = {}, None, None
    with torch.cuda.stream(stream):
        for name, ws in sets.items():
            src, _ = vg.clouds_to_device(ws.sources)
            tgt, _ = vg.clouds_to_device(ws.targets)
            used = sorted(set(int(t) for t in ws.factors[:, 1]))
            maps = [None] * len(tgt)
            for t in used:
                maps[t] = vg.voxelize(ctx, *tgt[t], ws.resolution)
            # unused targets get an empty map (no factor refers to them)
            empty = vg.voxelize(ctx, torch.zeros((3, 0), device="cuda"),
                                torch.zeros((0, 6), device="cuda"), ws.resolution)
            maps = [m if m is not None else empty for m in maps]
            fs = vg.FactorSet(ctx, src, maps, ws.factors, ws.poses.shape[0],
                              args.tile or 4608)
            poses = torch.from_numpy(np.ascontiguousarray(ws.poses)).to("cuda")
            ref = refs[name]
            F = ws.n_factors
            rH = np.stack([ref[f]["H"] for f in range(F)])
            rb = np.stack([ref[f]["b"] for f in range(F)])
            re_ = np.array([ref[f]["e"] for f in range(F)])
            rin = np.array([ref[f]["inliers"] for f in range(F)])
            for accum, resid, fused, kappa in PRECISION_VARIANTS:
                kw = dict(accum=accum, resid=resid, fused=fused, fp64_kappa=kappa)
                out = vg.linearize_factors(ctx, fs, poses, **kw)
                for _ in range(3):
                    vg.linearize_factors(ctx, fs, poses, use_graph=True, out=out, **kw)
                t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0.record(stream)
                for _ in range(steps):
                    vg.linearize_factors(ctx, fs, poses, use_graph=True, out=out, **kw)
                t1.record(stream)
                stream.synchronize()
                ms = t0.elapsed_time(t1) / steps
                n64 = vg.fp64_points(ctx, fs)
                H, b = out["H"].cpu().numpy(), out["b"].cpu().numpy()
                e, inl = out["e"].cpu().numpy(), out["inliers"].cpu().numpy()
                ok = rin > 0
                def rel(g, r):
                    num = np.linalg.norm((g - r).reshape(F, -1)[ok], axis=1)
                    den = np.linalg.norm(r.reshape(F, -1)[ok], axis=1)
                    return num / den
                errs = {"H": rel(H, rH), "b": rel(b, rb), "e": rel(e, re_)}
                blk = {}
                for f in np.flatnonzero(ok):
                    for k, v in parity_metrics(H[f], b[f], e[f], rH[f], rb[f], re_[f]).items():
                        if k not in ("H", "b", "e") and v > blk.get(k, (-1.0,))[0]:
                            blk[k] = (v, int(f))
                wk = max(blk, key=lambda k: blk[k][0]) if blk else None
                key = f"{accum}/{resid}/{fused}/{kappa:g}"
                table.setdefault(key, {})[name] = {
                    "max_rel_err": {k: float(v.max()) for k, v in errs.items()},
                    "p99_rel_err": {k: float(np.percentile(v, 99)) for k, v in errs.items()},
                    "worst_block": {"metric": wk, "err": blk[wk][0] if wk else None,
                                    "factor": blk[wk][1] if wk else None},
                    "inlier_mismatches": int((inl != rin).sum()),
                    "fp64_fraction": n64 / max(1, int(rin.sum())),
                    "ms_per_round": round(ms, 5),
                }
                if name == "regular" and (accum, resid, fused, kappa) == PRECISION_VARIANTS[0]:
                    default_ms, default_corr = ms, int(inl.sum())
                log(f"[bench] {name:8s} {key:18s} {ms:.3f} ms  max H {errs['H'].max():.2e} "
                    f"b {errs['b'].max():.2e} e {errs['e'].max():.2e}  worst block "
                    f"{wk} {blk[wk][0] if wk else 0:.2e}  FP64 {n64}")
            del fs, maps, src, tgt
    total_corr = sum(int(o["inliers"]) for r in refs.values() for o in r.values())
    total_wall = sum(cpu_wall.values())
    result = {
        "metric": "point correspondences linearized/sec (1 GPU); p50/p99 linearization-round latency",
        "value": default_corr / (default_ms * 1e-3),
        "unit": "correspondences/s",
        "n_gpus": 1, "steps": steps, "warmup": 3,
        "ms_per_step": round(default_ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "precision study: corridor_1000frames_4500factors_r0.5 plus the "
                               "first 450 pairs with surface-normal covariances (1, 1, 1e-6) "
                               "at the pose estimates and at the ground truth",
                   "factors": {k: v.n_factors for k, v in sets.items()},
                   "tile_points": args.tile or 4608, "seed": [210907073, 3]},
        "precision": table,
        "cpu_baseline": {"value": total_corr / total_wall, "unit": "correspondences/s",
                         "cores": workers, "kind": "oracle",
                         "sample": f"every factor of the three sets ({sum(len(r) for r in refs.values())} "
                                   f"factors, {total_corr} correspondences), {workers} processes "
                                   f"of 1 thread, {total_wall:.1f} s wall"},
    }
    print(json.dumps(result))


def run_serving(args):
    """Serving form: keyframes of 20,000 points arrive as a seeded Poisson
    stream (10 Hz, virtual clock) and are ingested into a continuous-batching
    server: voxel map, overlap against every resident keyframe, a factor for
    every pair with overlap >= 5 %.  Admission is by the server's memory
    budget: a refused keyframe evicts the oldest resident ones.  After each
    arrival, for each of 3 LM rounds, two optimizer requests are in flight
    together: a global window (every factor touching the newest `window`
    keyframes) and a local, fully connected graph over the newest 10
    keyframes.  Poses get a seeded 1 mm / 0.05 degree perturbation per round.
    Reported: correspondences linearized per second of round time, the
    p50/p99 round latency (both requests submitted until both outputs are in
    host memory) and the p50/p99 request latency."""
    from paper_2109_07073_amd import vgicp as vg
    from synth import random_perturbation, rng_for, stream_scan_frames

    n = args.keyframes
    resolution = 0.5
    rng = rng_for(5, 1)
    arrivals = np.cumsum(rng.exponential(0.1, size=n))
    # generated up front (before the GPU is used), so that no generator
    # process competes with the served rounds for the host's cores
    t_gen = time.perf_counter()
    frames = list(stream_scan_frames(5, n, workers=None))
    log(f"[serving] {n} keyframes generated in {time.perf_counter() - t_gen:.1f} s")
    srv = vg.Server(memory_budget_bytes=int(args.budget_gib * 2**30), max_batch_factors=16384,
                    max_batch_points=1 << 28, max_batch_poses=65536, inflight=2)
    poses = np.zeros((0, 12))
    resident = []
    adj = {}                              # keyframe id -> set of factors (src, tgt) touching it
    n_factors = 0
    n_paper_rule = 0                      # pairs the paper's rule (overlap > 2.5 %) would admit
    lat, corr_total, round_time, evictions, overlap_ms = [], 0, 0.0, 0, []
    round_ms, submit_ms = [], []
    by_size = []                          # (resident keyframes, round ms, correspondences)
    overlap_by_size = []                  # (resident keyframes, overlap request ms)
    t_start = time.perf_counter()

    def pose_rows(Ts):
        Ts = np.asarray(Ts).reshape(-1, 4, 4)
        return np.concatenate([Ts[:, :3, :3].reshape(-1, 9), Ts[:, :3, 3]], axis=1)

    def perturbed(P, ids):
        """Right-compose a seeded 1 mm / 0.05 degree motion onto poses `ids`."""
        ids = np.asarray(sorted(ids), dtype=np.int64)
        Q = P.copy()
        if ids.size == 0:
            return Q
        ax = rng.normal(size=(ids.size, 3))
        ax /= np.linalg.norm(ax, axis=1, keepdims=True)
        th = np.deg2rad(0.05)
        K = np.zeros((ids.size, 3, 3))
        K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -ax[:, 2], ax[:, 1], -ax[:, 0]
        K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = ax[:, 2], -ax[:, 1], ax[:, 0]
        dR = np.eye(3)[None] + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)
        dt = rng.normal(size=(ids.size, 3))
        dt *= 1e-3 / np.linalg.norm(dt, axis=1, keepdims=True)
        R = Q[ids, :9].reshape(-1, 3, 3)
        t = Q[ids, 9:]
        Q[ids, :9] = (R @ dR).reshape(-1, 9)
        Q[ids, 9:] = t + np.einsum("nij,nj->ni", R, dt)
        return Q

    for f, T, xyz, cov in frames:
        while True:
            try:
                fid = srv.add_frame(xyz, cov, resolution)
                break
            except vg.VgicpError as ex:
                if ex.code != vg.EFULL or not resident:
                    raise
                old = resident.pop(0)
                srv.remove_frame(old)
                for x in adj.pop(old, set()):
                    other = x[0] if x[1] == old else x[1]
                    adj.get(other, set()).discard(x)
                    n_factors -= 1
                evictions += 1
        if fid >= poses.shape[0]:
            poses = np.concatenate([poses, np.zeros((fid + 1 - poses.shape[0], 12))])
        poses[fid] = pose_rows(T)[0]
        adj[fid] = set()
        if resident:
            # overlap-gated factor creation in the library (vgicp_server_connect)
            t0 = time.perf_counter()
            con = srv.connect(fid, poses[fid], resident, poses[resident], threshold=0.05,
                              rule="at_least")
            overlap_ms.append((time.perf_counter() - t0) * 1e3)
            overlap_by_size.append((len(resident), overlap_ms[-1]))
            n_paper_rule += int((con["overlap"] > 0.025).sum())
            for old, adm in zip(resident, con["admitted"]):
                if adm:
                    adj[fid].add((fid, old))
                    adj[old].add((fid, old))
                    n_factors += 1
        resident.append(fid)
        glob = set()
        for w_id in resident[-args.window:]:
            glob |= adj[w_id]
        glob = sorted(glob)
        loc_ids = resident[-10:]
        loc = [(a, b) for ia, a in enumerate(loc_ids) for b in loc_ids[:ia]]
        # the optimizer's variables: the poses its factors touch, numbered
        # 0..U-1 in the requests (each request carries only those poses)
        used_ids = sorted({a for a, _ in glob} | {b for _, b in glob} | set(loc_ids))
        var = {k: n for n, k in enumerate(used_ids)}
        glob = np.asarray([(a, b, var[a], var[b]) for a, b in glob], np.int32).reshape(-1, 4)
        loc = np.asarray([(a, b, var[a], var[b]) for a, b in loc], np.int32).reshape(-1, 4)
        prev = {}   # each optimizer reuses its previous round's host buffers
        for _ in range(3):
            P = perturbed(poses, used_ids)[used_ids]
            t0 = time.perf_counter()
            # the two optimizers submit on their own (queued together with
            # submit_many they share one batch, and the round takes longer than
            # two batches overlapping on the server's two streams)
            reqs = {k: srv.submit("linearize", g, P, out=prev.get(k))
                    for k, g in (("glob", glob), ("loc", loc)) if len(g)}
            t1 = time.perf_counter()
            done = [r.wait() for r in reqs.values()]
            prev = reqs
            t2 = time.perf_counter()
            round_time += t2 - t0
            round_ms.append((t2 - t0) * 1e3)
            submit_ms.append((t1 - t0) * 1e3)
            corr_round = 0
            for r in done:
                lat.append(r.latency_ms)
                corr_round += int(r.inliers.sum())
            corr_total += corr_round
            by_size.append((len(resident), round_ms[-1], corr_round))
        if f % 200 == 0:
            log(f"[serving] keyframe {f}: resident {len(resident)}, factors {n_factors}, "
                f"global {len(glob)}, local {len(loc)}")
    wall = time.perf_counter() - t_start
    st = srv.stats()
    used, budget = srv.memory()
    srv.close()
    # latency and throughput against the number of resident keyframes
    bucket = 1000
    size_table = []
    for lo in range(0, n, bucket):
        rs = [(ms, c) for k, ms, c in by_size if lo < k <= lo + bucket]
        ovs = [ms for k, ms in overlap_by_size if lo < k <= lo + bucket]
        if not rs:
            continue
        ms_r = np.array([a for a, _ in rs])
        size_table.append({
            "resident_keyframes": f"{lo + 1}-{lo + bucket}",
            "round_p50_ms": round(float(np.percentile(ms_r, 50)), 4),
            "round_p99_ms": round(float(np.percentile(ms_r, 99)), 4),
            "correspondences_per_s": sum(c for _, c in rs) / (ms_r.sum() * 1e-3),
            "overlap_request_p50_ms": round(float(np.percentile(ovs, 50)), 4) if ovs else None,
            "overlap_request_p99_ms": round(float(np.percentile(ovs, 99)), 4) if ovs else None,
        })
    result = {
        "metric": "point correspondences linearized/sec (1 GPU); p50/p99 linearization-round latency",
        "value": corr_total / round_time,
        "unit": "correspondences/s",
        "n_gpus": 1,
        "steps": 3 * n,
        "warmup": 0,
        "ms_per_step": round(round_time * 1e3 / (3 * n), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving_corridor_{n}keyframes_r0.5", "keyframes": n,
                   "arrival_rate_hz": 10, "simulated_seconds": float(arrivals[-1]),
                   "overlap_threshold": 0.05, "global_window": args.window, "local_window": 10,
                   "memory_budget_bytes": budget, "seed": [210907073, 5]},
        "round_latency_ms": {"round_p50": float(np.percentile(round_ms, 50)),
                             "round_p99": float(np.percentile(round_ms, 99)),
                             "submit_p50": float(np.percentile(submit_ms, 50)),
                             "request_p50": float(np.percentile(lat, 50)),
                             "request_p99": float(np.percentile(lat, 99)),
                             "overlap_request_p50": float(np.percentile(overlap_ms, 50)),
                             "overlap_request_p99": float(np.percentile(overlap_ms, 99))},
        "serving": {"batches": st["batches"], "requests": st["requests"],
                    "max_requests_per_batch": st["max_requests_per_batch"],
                    "max_inflight_batches": st["max_inflight"], "evictions": evictions,
                    "resident_keyframes": len(resident), "factors_admitted": n_factors,
                    "pairs_over_2.5_percent": n_paper_rule,
                    "device_bytes_resident": used, "wall_s": round(wall, 2)},
        "by_map_size": size_table,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(result))


def _so3_exp(w):
    th = float(np.linalg.norm(w))
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th**2 * (K @ K)


def _rel_pose_errors(T_est, T_gt):
    """Translation (m) and rotation (deg) error of every consecutive relative pose."""
    et, er = [], []
    for a in range(len(T_est) - 1):
        E = np.linalg.inv(np.linalg.inv(T_gt[a]) @ T_gt[a + 1]) @ (np.linalg.inv(T_est[a]) @ T_est[a + 1])
        et.append(float(np.linalg.norm(E[:3, 3])))
        er.append(float(np.degrees(np.arccos(np.clip((np.trace(E[:3, :3]) - 1) / 2, -1, 1)))))
    return et, er


def run_local(args):
    """Local mapping (the paper's submap construction): frames of a 10 Hz
    scan stream from a vehicle that cruises and stops (initial poses 2 cm /
    0.2 degrees off the truth, as from odometry) are voxelized at r = 0.5 m; a frame whose overlap with the submap's last frame exceeds
    95 % is skipped (the sensor did not move), otherwise it joins the submap
    with a factor to every frame already in it (fully connected graph).  When
    the overlap between the newest and the first frame drops below 10 % or
    the submap holds more than 15 frames, the submap's poses are optimized
    by Levenberg-Marquardt: every iteration linearizes all factors, assembles
    the global system on the GPU, solves the small dense system on the host
    (first pose fixed) and evaluates the cost at the trial poses on the GPU;
    it stops after 10 iterations, a relative decrease below 1e-3 or three
    rejected steps in a row.
    Reported: correspondences linearized per second of linearization time,
    p50/p99 of the LM iteration (linearize + assemble + copy + solve +
    evaluate) and of the linearization alone, and the relative pose error
    against the ground truth before and after."""
    import torch

    from paper_2109_07073_amd import vgicp as vg
    from synth import drive_positions, pose_rows, stream_scan_frames

    n = args.frames
    r, th_max, th_min, n_max, max_iters = 0.5, 0.95, 0.10, 15, 10
    positions = drive_positions(6, n)
    # generated up front (before the GPU is used), so that no generator
    # process competes with the timed loop for the host's cores
    t_gen = time.perf_counter()
    frames = list(stream_scan_frames(2, n, positions=positions, with_truth=True,
                                     perturb=(0.02, 0.2)))
    log(f"[local] {n} frames generated in {time.perf_counter() - t_gen:.1f} s")
    ctx = vg.Context(0)
    sub = []                      # current submap: dicts of frame data
    stats = {"frames": 0, "skipped": 0, "submaps": 0, "factors": 0, "lm_iterations": 0,
             "accepted": 0}
    lin_ms, iter_ms, ov_ms, vox_ms, submap_ms, corr_lin = [], [], [], [], [], 0
    err_before, err_after, cost_ratio = [], [], []
    lin_time = 0.0

    def sync():
        ctx.synchronize()

    def optimize(frames):
        nonlocal lin_time, corr_lin
        N = len(frames)
        if N < 2:
            return
        t_sub = time.perf_counter()
        factors = np.array([(a, b, a, b) for a in range(N) for b in range(a)], dtype=np.int32)
        fs = vg.FactorSet(ctx, [f["dev"] for f in frames], [f["map"] for f in frames], factors, N)
        T = [f["T"].copy() for f in frames]
        P = torch.from_numpy(pose_rows(T)).to("cuda")
        lin = vg.linearize_factors(ctx, fs, P)
        ev = vg.evaluate_errors(ctx, fs, P)
        asm = None
        sync()
        e_cur = float(lin["e"].sum().item())
        e0, lam, rejects = e_cur, 1e-4, 0
        for it in range(max_iters):
            t0 = time.perf_counter()
            vg.linearize_factors(ctx, fs, P, out=lin)
            sync()
            t1 = time.perf_counter()
            asm = vg.assemble_system(ctx, fs, lin["H"], lin["b"], out=asm)
            Hd, bv, Ho = (asm["Hdiag"].cpu().numpy(), asm["bvec"].cpu().numpy(),
                          asm["Hoff"].cpu().numpy())
            inl = int(lin["inliers"].sum().item())
            A = np.zeros((6 * N, 6 * N))
            for p in range(N):
                A[6 * p:6 * p + 6, 6 * p:6 * p + 6] = Hd[p]
            for k, (p, q) in enumerate(fs.pairs):
                A[6 * p:6 * p + 6, 6 * q:6 * q + 6] = Ho[k]
                A[6 * q:6 * q + 6, 6 * p:6 * p + 6] = Ho[k].T
            g = bv.reshape(-1)
            A, g = A[6:, 6:], g[6:]                       # the first pose is held fixed
            A = A + lam * np.diag(np.diag(A))
            xi = np.linalg.solve(A, -g).reshape(-1, 6)
            T_try = [T[0]] + [T[p] @ np.block([[_so3_exp(xi[p - 1, :3]), xi[p - 1, 3:, None]],
                                                [np.zeros((1, 3)), np.ones((1, 1))]])
                              for p in range(1, N)]
            P_try = torch.from_numpy(pose_rows(T_try)).to("cuda")
            vg.evaluate_errors(ctx, fs, P_try, out=ev)
            e_try = float(ev["e"].sum().item())
            t2 = time.perf_counter()
            lin_ms.append((t1 - t0) * 1e3)
            iter_ms.append((t2 - t0) * 1e3)
            lin_time += t1 - t0
            corr_lin += inl
            stats["lm_iterations"] += 1
            if e_try < e_cur:
                stats["accepted"] += 1
                rel = (e_cur - e_try) / e_cur
                T, P, e_cur, lam, rejects = T_try, P_try, e_try, lam * 0.1, 0
                if rel < 1e-3:
                    break
            else:
                lam, rejects = lam * 10.0, rejects + 1
                if rejects == 3:
                    break
        submap_ms.append((time.perf_counter() - t_sub) * 1e3)
        cost_ratio.append(e_cur / e0 if e0 > 0 else 1.0)
        b_t, _ = _rel_pose_errors([f["T"] for f in frames], [f["gt"] for f in frames])
        a_t, _ = _rel_pose_errors(T, [f["gt"] for f in frames])
        err_before.extend(b_t)
        err_after.extend(a_t)
        stats["submaps"] += 1
        stats["factors"] += int(factors.shape[0])

    # load every kernel once (first launches pay for code-object loading)
    _, T0, _, x0, c0 = frames[0]
    d0 = vg.cloud_to_device(x0, c0)
    m0 = vg.voxelize(ctx, d0[0], d0[1], r)
    fs0 = vg.FactorSet(ctx, [d0, d0], [m0, m0], [(0, 1, 0, 1)], 2)
    P0 = torch.from_numpy(pose_rows([T0, T0])).to("cuda")
    l0 = vg.linearize_factors(ctx, fs0, P0)
    vg.assemble_system(ctx, fs0, l0["H"], l0["b"])
    vg.evaluate_errors(ctx, fs0, P0)
    vg.overlap(ctx, fs0, P0)
    sync()
    del fs0, m0, d0

    t_start = time.perf_counter()
    for f, T_est, T_gt, xyz, cov in frames:
        stats["frames"] += 1
        t0 = time.perf_counter()
        dev = vg.cloud_to_device(xyz, cov)
        vmap = vg.voxelize(ctx, dev[0], dev[1], r)
        sync()
        vox_ms.append((time.perf_counter() - t0) * 1e3)
        cur = {"dev": dev, "map": vmap, "T": T_est, "gt": T_gt}
        if sub:
            t0 = time.perf_counter()
            pair = [sub[-1], sub[0], cur]
            # the submap rules in the library (vgicp_submap_step)
            decision, _, _ = vg.submap_step(
                ctx, dev[0], pose_rows([T_est])[0], first=sub[0]["map"],
                first_pose=pose_rows([sub[0]["T"]])[0], last=sub[-1]["map"],
                last_pose=pose_rows([sub[-1]["T"]])[0], n_submap=len(sub), skip_above=th_max,
                close_below=th_min, max_frames=n_max)
            ov_ms.append((time.perf_counter() - t0) * 1e3)
            if decision == "skip":
                stats["skipped"] += 1
                continue
            sub.append(cur)
            if decision == "close":
                optimize(sub)
                sub = []
        else:
            sub.append(cur)
        if f % 200 == 0:
            log(f"[local] frame {f}: submaps {stats['submaps']}, skipped {stats['skipped']}")
    optimize(sub)
    wall = time.perf_counter() - t_start
    result = {
        "metric": "point correspondences linearized/sec (1 GPU); p50/p99 linearization-round latency",
        "value": corr_lin / lin_time if lin_time > 0 else 0.0,
        "unit": "correspondences/s",
        "n_gpus": 1,
        "steps": stats["lm_iterations"],
        "warmup": 0,
        "ms_per_step": round(float(np.mean(lin_ms)), 4) if lin_ms else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"local_mapping_corridor_{n}frames_r0.5", "frames": n,
                   "resolution_m": r, "th_max": th_max, "th_min": th_min, "n_max": n_max,
                   "lm_max_iterations": max_iters, "seed": [210907073, 2, 400, 6]},
        "round_latency_ms": {"linearize_p50": float(np.percentile(lin_ms, 50)),
                             "linearize_p99": float(np.percentile(lin_ms, 99)),
                             "lm_iteration_p50": float(np.percentile(iter_ms, 50)),
                             "lm_iteration_p99": float(np.percentile(iter_ms, 99)),
                             "overlap_check_p50": float(np.percentile(ov_ms, 50)),
                             "voxelize_p50": float(np.percentile(vox_ms, 50)),
                             "submap_p50": float(np.percentile(submap_ms, 50))},
        "local_mapping": dict(stats, wall_s=round(wall, 2),
                              rel_trans_err_before_m=float(np.mean(err_before)),
                              rel_trans_err_after_m=float(np.mean(err_after)),
                              cost_ratio_median=float(np.median(cost_ratio))),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(result))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30,
                    help="untimed rounds first (the GPU clocks ramp up over the first few)")
    ap.add_argument("--workload", default="batched4500", choices=sorted(WORKLOADS))
    ap.add_argument("--accum", default="mixed", choices=["mixed", "f32", "f32_comp", "f64"])
    ap.add_argument("--fused", default="f64", choices=["f64", "f32"],
                    help="precision of the fused covariance and its inverse")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--layout", default="auto",
                    choices=["auto", "grouped", "interleaved", "balanced"],
                    help="tile-table layout (auto: the tuner's choice, or grouped with --tile)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reorder", action="store_true",
                    help="keep the Morton-ordered source copies (no target-order copies)")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="oracle processes for the CPU baseline (capped by the host's CPUs)")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--keyframes", type=int, default=4000, help="serving: keyframes streamed")
    ap.add_argument("--frames", type=int, default=600, help="local: frames streamed (10 Hz)")
    ap.add_argument("--window", type=int, default=20, help="serving: global optimizer window")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serving: memory budget")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU "
                                   "sharding is a design note only", "n_gpus": args.gpus}))
        sys.exit(2)

    # Everything that forks worker processes (input generation, the CPU
    # baseline, the frame streams' pools) starts before the GPU is touched.
    if args.workload == "serving":
        run_serving(args)
        return
    if args.workload == "local":
        run_local(args)
        return
    if args.workload == "precision":
        run_precision(args)
        return
    t_gen = time.perf_counter()
    w = build_workload(args.workload)
    log(f"[bench] workload {w.name}: {w.n_factors} factors, {w.source_points()} source points, "
        f"generated in {time.perf_counter() - t_gen:.1f} s")
    # two 50,000-point scans 1 m apart for the single-pair overlap latency
    from synth import stream_scan_frames
    pair = [(x, c, T) for (_, T, x, c) in stream_scan_frames(2, 2, n_points=50000, workers=1)]
    cpu_run = None
    if not args.no_cpu_baseline:
        cpu_run = cpu_baseline(w, workers=max(1, min(args.cpu_workers, os.cpu_count() or 1)))
        log(f"[bench] cpu baseline: {cpu_run[2]}")
        cpu_single = cpu_single_process(w)
        log(f"[bench] cpu baseline, one process: {cpu_single[0] / 1e6:.2f} M corr/s "
            f"({cpu_single[1]} factors)")

    import torch
    from paper_2109_07073_amd import vgicp as vg

    assert torch.cuda.is_available(), "bench.py needs a GPU"

    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    ctx = vg.Context(0, stream=stream)

    # ---- upload and ingest (voxel maps, once per frame)
    src, src_buf = vg.clouds_to_device(w.sources)
    tgt, tgt_buf = vg.clouds_to_device(w.targets)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    maps = [vg.voxelize(ctx, x, c, w.resolution) for (x, c) in tgt]
    ctx.synchronize()
    t_vox = time.perf_counter() - t0
    n_vox = int(sum(m.n_voxels for m in maps))
    map_bytes = int(sum(m.device_bytes for m in maps))
    t0 = time.perf_counter()
    fs = vg.FactorSet(ctx, src, maps, w.factors, w.poses.shape[0], args.tile)
    t_fs = time.perf_counter() - t0     # includes the Morton-ordered source copies
    poses = torch.from_numpy(np.ascontiguousarray(w.poses)).to("cuda")
    # per-factor source copies in the order of the target voxels at these poses
    # (an optimizer reorders once per optimization; the poses move little
    # between its rounds)
    t_reorder = None
    if not args.no_reorder:
        t0 = time.perf_counter()
        vg.reorder_by_target(ctx, fs, poses)
        t_reorder = time.perf_counter() - t0
    tuned = None
    if args.layout != "auto":
        vg.set_layout(ctx, fs, args.layout)
    if not args.tile:      # measure the candidate tile sizes and keep the fastest
        best, best_ms = vg.tune_tiles(ctx, fs, poses, accum=args.accum, fused=args.fused)
        tuned = {"tile_points": best, "round_ms": round(best_ms, 4)}
        log(f"[bench] tile autotuned: {best} points ({best_ms:.3f} ms per round)")
    F = fs.n_factors
    log(f"[bench] {len(maps)} voxel maps ({n_vox} voxels, {map_bytes / 2**20:.1f} MiB) in "
        f"{t_vox * 1e3:.1f} ms; {fs.n_tiles} tiles")

    # ---- overlap of every pair (factor creation)
    ov = vg.overlap(ctx, fs, poses)
    ctx.synchronize()
    ov_reps = 5
    t0 = time.perf_counter()
    for _ in range(ov_reps):
        vg.overlap(ctx, fs, poses, out=ov)
    ctx.synchronize()
    t_ov = (time.perf_counter() - t0) / ov_reps

    # ---- one overlap check between two 50,000-point scans (factor creation)
    pair_dev = [vg.cloud_to_device(x, c) for (x, c, _) in pair]
    pair_maps = [vg.voxelize(ctx, x, c, w.resolution) for (x, c) in pair_dev]
    pair_fs = vg.FactorSet(ctx, pair_dev, pair_maps, [(1, 0, 1, 0)], 2)
    from synth import pose_rows
    pair_poses = torch.from_numpy(pose_rows([T for (_, _, T) in pair])).to("cuda")
    pov = vg.overlap(ctx, pair_fs, pair_poses)
    for _ in range(20):
        vg.overlap(ctx, pair_fs, pair_poses, out=pov)
    torch.cuda.synchronize()
    pair_dev_ms, pair_host_ms = [], []
    for _ in range(100):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        h0 = time.perf_counter()
        a.record(stream)
        vg.overlap(ctx, pair_fs, pair_poses, out=pov)
        b.record(stream)
        stream.synchronize()
        pair_host_ms.append((time.perf_counter() - h0) * 1e3)
        pair_dev_ms.append(a.elapsed_time(b))
    pair_overlap = float(pov["overlap"].cpu()[0])

    # ---- outputs, correspondences, distinct voxels
    out = vg.linearize_factors(ctx, fs, poses, accum=args.accum, fused=args.fused, with_corr=True)
    ctx.synchronize()
    inliers = out["inliers"].cpu().numpy()
    assert np.array_equal(inliers, ov["hits"].cpu().numpy()), "overlap hits differ from inliers"
    U = distinct_voxels(fs.source_sizes, out["corr"])
    del out["corr"]
    n_corr = int(inliers.sum())
    n_pts = int(fs.total_points)

    # ---- round latency: device time (events) and host-visible (incl. D2H),
    # over at least 100 rounds, after untimed rounds that capture and
    # instantiate the round's graph and bring the clocks up (the first of them
    # run long)
    for _ in range(max(args.warmup, 20)):
        vg.linearize_factors(ctx, fs, poses, accum=args.accum, fused=args.fused, use_graph=True, out=out)
    torch.cuda.synchronize()
    dev_ms, host_ms = [], []
    host_H = torch.empty((F, 12, 12), dtype=torch.float64, pin_memory=True)
    for _ in range(max(args.steps, 100)):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        h0 = time.perf_counter()
        a.record(stream)
        vg.linearize_factors(ctx, fs, poses, accum=args.accum, fused=args.fused, use_graph=True, out=out)
        b.record(stream)
        host_H.copy_(out["H"], non_blocking=True)
        stream.synchronize()
        host_ms.append((time.perf_counter() - h0) * 1e3)
        dev_ms.append(a.elapsed_time(b))

    # ---- warmup + timed rounds (graph replay of [linearize, reduce]), right
    # after the latency rounds so that the GPU clocks are up when timing starts
    for _ in range(args.warmup):
        vg.linearize_factors(ctx, fs, poses, accum=args.accum, fused=args.fused, use_graph=True, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        vg.linearize_factors(ctx, fs, poses, accum=args.accum, fused=args.fused, use_graph=True, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps

    # ---- kernel timing for the roofline: the linearize kernel launched
    # args.steps times back to back between one pair of HIP events on its
    # stream; the reduce kernel bracketed by events per launch
    k_ms = vg.time_kernel(ctx, fs, poses, "linearize", reps=args.steps, accum=args.accum,
                          fused=args.fused)
    form = vg.form_of(fs)
    # both forms of the per-correspondence terms, whichever the tuner kept
    form_ms = {f"{f}_kernel_ms": round(vg.time_kernel(ctx, fs, poses, "linearize",
                                                      reps=args.steps, accum=args.accum,
                                                      fused=args.fused, form=f), 5)
               for f in ("source", "pair")} if args.accum != "f64" else None
    ctx.reset_timing()
    ctx.set_timing(True)
    for _ in range(min(args.steps, 20)):
        vg.linearize_factors(ctx, fs, poses, accum=args.accum, fused=args.fused, out=out)
    red_ms, red_n = ctx.read_timing("reduce")
    ctx.set_timing(False)
    sizes = fs.source_sizes
    # bytes one linearize launch must move: every source point's xyz (12 B),
    # the covariance of the points that hit a voxel (24 B; misses never read
    # theirs), each distinct target voxel touched once (8 B key + 36 B mean and
    # covariance) and 91 FP64 outputs per factor
    needed_bytes = float(12 * sizes.sum() + 24 * n_corr + 44 * U.sum() + 91 * 8 * F)
    # the same with the covariance of every source point charged (36 B per point)
    all_cov_bytes = float(36 * sizes.sum() + 44 * U.sum() + 91 * 8 * F)
    achieved = needed_bytes / (k_ms * 1e-3) / 1e9
    traffic = (profiled_traffic(args.workload, fs.tile_points, vg.layout_of(fs))
               if (args.accum, args.fused, form) == ("mixed", "f64", "source") else None)
    copy_gbs = measured_copy_gbs()

    # ---- plain per-factor launches on the same factors
    plain = None
    if args.plain_steps > 0 and args.workload != "single":
        vg.linearize_factors(ctx, fs, poses, accum=args.accum, fused=args.fused, schedule="per_factor", out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            vg.linearize_factors(ctx, fs, poses, accum=args.accum, fused=args.fused, schedule="per_factor", out=out)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) * 1e3 / args.plain_steps
        plain = {"ms_per_step": round(pms, 4), "value": n_corr / (pms * 1e-3),
                 "launches_per_step": 2 * F}

    # ---- error-only round (cost evaluation for trial steps)
    ev = vg.evaluate_errors(ctx, fs, poses, accum=args.accum, fused=args.fused)
    vg.evaluate_errors(ctx, fs, poses, accum=args.accum, fused=args.fused, use_graph=True, out=ev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        vg.evaluate_errors(ctx, fs, poses, accum=args.accum, fused=args.fused, use_graph=True, out=ev)
    torch.cuda.synchronize()
    ev_ms = (time.perf_counter() - t0) * 1e3 / args.steps

    # ---- CPU oracle baseline and a parity spot check on the same factors
    cpu = None
    spot = None
    if cpu_run is not None:
        rate, cores, sample, ids, outs = cpu_run
        cpu = {"value": rate, "unit": "correspondences/s", "cores": cores, "kind": "oracle",
               "sample": sample, "single_process_value": cpu_single[0],
               "single_process_factors": cpu_single[1], "host_cpu": host_cpu_model(),
               "host_logical_cpus": os.cpu_count()}
        Hg, bg, eg = out["H"].cpu().numpy(), out["b"].cpu().numpy(), out["e"].cpu().numpy()
        errs = {}
        for f, o in zip(ids, outs):
            assert int(inliers[f]) == o["inliers"]
            if o["inliers"] == 0:
                continue
            for k, v in parity_metrics(Hg[f], bg[f], eg[f], o["H"], o["b"], o["e"]).items():
                errs[k] = max(errs.get(k, 0.0), v)
        worst = max(errs, key=errs.get) if errs else None
        spot = {"factors": len(ids), "max_rel_err": {k: errs[k] for k in ("H", "b", "e")},
                "worst_block": {"metric": worst, "err": errs.get(worst)},
                "max_elementwise": {"H": errs.get("H_elem"), "b": errs.get("b_elem")},
                "within_1e-5": bool(errs) and max(errs.values()) <= 1e-5}

    result = {
        "metric": "point correspondences linearized/sec (1 GPU); p50/p99 linearization-round latency",
        "value": n_corr / (ms_per_step * 1e-3),
        "unit": "correspondences/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "factors": F,
            "source_points_per_round": n_pts,
            "correspondences_per_round": n_corr,
            "resolution_m": w.resolution,
            "accumulation": args.accum,
            "fused_covariance": args.fused,
            "schedule": "batched, HIP graph replay" + (", autotuned tile" if tuned else ""),
            "tile_points": int(fs.tile_points),
            "grid_blocks": vg.grid(fs),
            "form": form,
            "layout": vg.layout_of(fs),
            "source_order": "Morton cells" if args.no_reorder else "target voxel order",
            "seed": w.meta.get("seed"),
        },
        "round_latency_ms": {
            "device_p50": float(np.percentile(dev_ms, 50)),
            "device_p99": float(np.percentile(dev_ms, 99)),
            "host_visible_p50": float(np.percentile(host_ms, 50)),
            "host_visible_p99": float(np.percentile(host_ms, 99)),
        },
        "source_points_per_s": n_pts / (ms_per_step * 1e-3),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
            "kernel": "k_linearize" if form == "source" else "k_linearize_pair",
            "kernel_ms": round(k_ms, 5),
            "bytes_per_launch": needed_bytes,
            "bytes_model": "12 B per source point + 24 B per correspondence + 44 B per "
                           "distinct voxel touched + 91 x 8 B per factor",
            "all_cov_bytes_per_launch": all_cov_bytes,
            "all_cov_frac": round(all_cov_bytes / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic_frac": (round(traffic / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                             if traffic else None),
            "reduce_kernel_ms": round(red_ms / max(red_n, 1), 5),
            "copy_GBs": round(copy_gbs, 1),
            "frac_vs_copy": round(achieved / copy_gbs, 4),
        },
        "forms": form_ms,
        "stages": {
            "voxelize_all_maps_ms": round(t_vox * 1e3, 3),
            "factorset_create_ms": round(t_fs * 1e3, 3),
            "target_order_copies_ms": round(t_reorder * 1e3, 3) if t_reorder is not None else None,
            "maps": len(maps),
            "overlap_all_pairs_ms": round(t_ov * 1e3, 4),
            "overlap_one_pair_50k_ms": {"device_p50": float(np.percentile(pair_dev_ms, 50)),
                                        "host_visible_p50": float(np.percentile(pair_host_ms, 50)),
                                        "overlap": round(pair_overlap, 4)},
            "evaluate_round_ms": round(ev_ms, 4),
            "distinct_voxels_touched": int(U.sum()),
        },
        "plain_per_factor": plain,
        "cpu_baseline": cpu,
        "parity_spot_check": spot,
    }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
