"""Synthetic LiDAR-shaped workloads for VGICP factor linearization.

Everything here is input generation: scenes, ray-cast scans, k-NN covariances
(the per-point preprocessing the paper runs once per cloud, Sec. III), poses
and factor lists.  The clouds are handed unchanged to both the FP64 oracle and
the HIP path.

Layout conventions (host side, numpy):
  xyz  float32 (n, 3)   frame-local coordinates
  cov  float32 (n, 6)   symmetric covariance as xx, xy, xz, yy, yz, zz
  pose float64 (12,)    sensor-to-world: R row-major (9 values) then t (3)
Seeds are np.random.default_rng([210907073, cfg, ...]).
"""

from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

SEED_BASE = 210907073


def rng_for(cfg: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(cfg), *[int(e) for e in extra]])


# --------------------------------------------------------------------------
# small rigid-motion helpers used only to place scenes and perturb poses
# --------------------------------------------------------------------------

def _rodrigues(axis: np.ndarray, angle: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def _unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def random_perturbation(rng: np.random.Generator, trans: float = 0.1,
                        rot_deg: float = 2.0) -> np.ndarray:
    """4x4 rigid motion: `trans` metres along a random direction and
    `rot_deg` degrees about a random axis."""
    T = np.eye(4)
    T[:3, :3] = _rodrigues(_unit(rng), np.deg2rad(rot_deg))
    T[:3, 3] = trans * _unit(rng)
    return T


def pose_rows(Ts) -> np.ndarray:
    """Stack 4x4 poses into the (n, 12) float64 layout: R row-major, then t."""
    Ts = np.asarray(Ts, dtype=np.float64).reshape(-1, 4, 4)
    out = np.empty((Ts.shape[0], 12), dtype=np.float64)
    out[:, :9] = Ts[:, :3, :3].reshape(-1, 9)
    out[:, 9:] = Ts[:, :3, 3]
    return out


# --------------------------------------------------------------------------
# covariances (paper Sec. III preprocessing: per-point covariance from k
# neighbours; regularisation to a plane-like spectrum)
# --------------------------------------------------------------------------

def _sym6(C: np.ndarray) -> np.ndarray:
    return np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2],
                     C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]], axis=1)


def knn_covariances(xyz: np.ndarray, k: int, eps: float = 1e-3) -> np.ndarray:
    """k-NN covariances (the point itself included), eigenvalues replaced by
    (eps, 1, 1) so every covariance is a regularised plane.  FP64 in, FP64
    (n, 6) out."""
    xyz = np.asarray(xyz, dtype=np.float64)
    n = xyz.shape[0]
    if n == 0:
        return np.zeros((0, 6))
    kk = min(k, n)
    _, nb = cKDTree(xyz).query(xyz, k=kk)
    nb = nb.reshape(n, kk)
    P = xyz[nb]                                   # (n, k, 3)
    P = P - P.mean(axis=1, keepdims=True)
    C = np.matmul(P.transpose(0, 2, 1), P) / max(kk - 1, 1)
    _, V = np.linalg.eigh(C)                     # ascending eigenvalues
    lam = np.array([eps, 1.0, 1.0])
    Creg = np.einsum("nij,j,nkj->nik", V, lam, V)
    return _sym6(Creg)


def normal_covariances(normals: np.ndarray, eps: float) -> np.ndarray:
    """Plane covariance from an analytic unit normal: eigenvalue eps along the
    normal, 1 in the tangent plane.  FP64 (n, 6)."""
    nrm = np.asarray(normals, dtype=np.float64)
    nrm = nrm / np.linalg.norm(nrm, axis=1, keepdims=True)
    C = np.eye(3)[None] - (1.0 - eps) * np.einsum("ni,nj->nij", nrm, nrm)
    return _sym6(C)


# --------------------------------------------------------------------------
# workload container
# --------------------------------------------------------------------------

@dataclass
class Workload:
    """A batch of VGICP factors.

    sources[k] / targets[k] are (xyz float32 (n,3), cov float32 (n,6)).
    factors rows are (source index, target index, pose_i, pose_j): the source
    cloud lives in frame pose_i and is matched against the voxel map of the
    target cloud, which lives in frame pose_j.
    """
    name: str
    resolution: float
    sources: list
    targets: list
    poses: np.ndarray           # (n_poses, 12) float64
    factors: np.ndarray         # (n_factors, 4) int32
    meta: dict = field(default_factory=dict)

    @property
    def n_factors(self) -> int:
        return int(self.factors.shape[0])

    def source_points(self) -> int:
        return int(sum(self.sources[s][0].shape[0] for s in self.factors[:, 0]))


def _f32_cloud(xyz, cov):
    return (np.ascontiguousarray(xyz, dtype=np.float32),
            np.ascontiguousarray(cov, dtype=np.float32))


# --------------------------------------------------------------------------
# single-factor room scene (ground plane plus four walls)
# --------------------------------------------------------------------------

def room_points(rng: np.random.Generator, n: int, half: float = 20.0,
                height: float = 5.0, noise: float = 0.02):
    """Points sampled uniformly by area on z=0 over [-half, half]^2 and on the
    walls x=+-half, y=+-half (0 <= z <= height), plus N(0, noise^2) per axis.
    Returns xyz (n,3) and analytic normals (n,3), FP64."""
    a_ground = (2 * half) ** 2
    a_wall = 2 * half * height
    p = np.array([a_ground, a_wall, a_wall, a_wall, a_wall])
    which = rng.choice(5, size=n, p=p / p.sum())
    xyz = np.empty((n, 3))
    nrm = np.zeros((n, 3))
    u = rng.uniform(-half, half, size=n)
    v = rng.uniform(-half, half, size=n)
    z = rng.uniform(0.0, height, size=n)
    g = which == 0
    xyz[g] = np.stack([u[g], v[g], np.zeros(g.sum())], 1)
    nrm[g, 2] = 1.0
    for w, (ax, sgn) in enumerate([(0, 1.0), (0, -1.0), (1, 1.0), (1, -1.0)], start=1):
        m = which == w
        pts = np.empty((m.sum(), 3))
        pts[:, ax] = sgn * half
        pts[:, 1 - ax] = u[m]
        pts[:, 2] = z[m]
        xyz[m] = pts
        nrm[m, ax] = -sgn
    xyz += rng.normal(0.0, noise, size=xyz.shape)
    return xyz, nrm


def make_single_factor(seed_cfg: int = 1, n: int = 2000, k: int = 10,
                       resolution: float = 1.0, trans: float = 0.1,
                       rot_deg: float = 2.0) -> Workload:
    """One factor on the room scene: source and target drawn independently,
    target pose identity, source pose estimate perturbed from its true
    identity pose."""
    rng = rng_for(seed_cfg)
    src_xyz, _ = room_points(rng, n)
    tgt_xyz, _ = room_points(rng, n)
    src_cov = knn_covariances(src_xyz, k)
    tgt_cov = knn_covariances(tgt_xyz, k)
    T_i = random_perturbation(rng, trans, rot_deg)
    T_j = np.eye(4)
    return Workload(
        name=f"room_single_factor_{n}pts_r{resolution:g}",
        resolution=resolution,
        sources=[_f32_cloud(src_xyz, src_cov)],
        targets=[_f32_cloud(tgt_xyz, tgt_cov)],
        poses=pose_rows([T_i, T_j]),
        factors=np.array([[0, 0, 0, 1]], dtype=np.int32),
        meta={"seed": [SEED_BASE, seed_cfg], "k": k},
    )


def make_tiny_workload(seed: int, n_src: int, n_tgt: int, resolution: float,
                       n_factors: int = 1, trans: float = 0.1,
                       rot_deg: float = 2.0, half: float = 3.0,
                       height: float = 2.0, k: int = 10,
                       cov_eps: float = 1e-3) -> Workload:
    """Small room-scene factors for parity and edge-case tests.  Each factor
    has its own source cloud, target cloud and pose pair."""
    rng = rng_for(100, seed)
    sources, targets, poses, factors = [], [], [], []
    for f in range(n_factors):
        ns = n_src[f] if hasattr(n_src, "__len__") else n_src
        nt = n_tgt[f] if hasattr(n_tgt, "__len__") else n_tgt
        sx, _ = room_points(rng, ns, half=half, height=height)
        tx, _ = room_points(rng, nt, half=half, height=height)
        sources.append(_f32_cloud(sx, knn_covariances(sx, k, cov_eps)))
        targets.append(_f32_cloud(tx, knn_covariances(tx, k, cov_eps)))
        Tj = random_perturbation(rng, 1.0, 30.0)
        Ti = Tj @ random_perturbation(rng, trans, rot_deg)
        poses += [Ti, Tj]
        factors.append([f, f, 2 * f, 2 * f + 1])
    return Workload(
        name=f"tiny_{seed}", resolution=resolution, sources=sources,
        targets=targets, poses=pose_rows(poses),
        factors=np.array(factors, dtype=np.int32).reshape(-1, 4),
        meta={"seed": [SEED_BASE, 100, seed]})


# --------------------------------------------------------------------------
# hits with degenerate covariances
# --------------------------------------------------------------------------

# Point covariances (xx, xy, xz, yy, yz, zz) of the degenerate kinds.
DEGENERATE_COVS = {
    "zero": [0.0, 0.0, 0.0, 0.0, 0.0, 0.0],
    "rank1": [1.0, 0.0, 0.0, 0.0, 0.0, 0.0],
    "rank2": [1.0, 0.0, 0.0, 1.0, 0.0, 0.0],
    "indefinite": [-3.0, 0.0, 0.0, -3.0, 0.0, -3.0],
    "nan": [1.0, np.nan, 0.0, 1.0, 0.0, 1.0],
    "inf": [np.inf, 0.0, 0.0, 1.0, 0.0, 1.0],
    "neg_inf": [1.0, 0.0, 0.0, 1.0, 0.0, -np.inf],
}


def make_degenerate_workload(seed: int = 0, n_regular: int = 400, n_target: int = 600,
                             per_kind: int = 6, resolution: float = 0.5) -> Workload:
    """Factors whose sources mix regular points with points of degenerate
    covariance placed where the target has points, so that they fall in
    target voxels.

    The target is a small room scene (k-NN covariances) plus eight pads of
    three points each with zero covariance, centred in 0.5 m cells at
    x = 5.25 ... 12.25 m on the x axis (cells that hold no other point).
    Degenerate source points are copies of target points carried into the
    source frame: "zero", "rank1" and "rank2" ones at the pads (where the
    voxel covariance is zero, so the fused covariance is 0 or singular),
    "indefinite", "nan", "inf" and "neg_inf" ones at regular target points.

    factor 0: regular + zero/indefinite/nan/inf/neg_inf, relative pose of
              0.1 m and 2 degrees on top of a random target pose
    factor 1: regular + every kind, relative pose exactly a 90 degree turn
              about z with no translation (target pose I), so that the
              rank-deficient covariances stay exactly singular
    factor 2: factor 0's degenerate points alone
    factor 3: factor 0's regular points alone
    meta["kinds"][f] lists the kind of every source point of factor f
    ("regular" or a key of DEGENERATE_COVS)."""
    rng = rng_for(101, seed)
    half, height = 3.0, 2.0
    tx, _ = room_points(rng, n_target, half=half, height=height)
    tcov = knn_covariances(tx, 10, 1e-3)
    pads = np.array([[5.25 + k, 0.25, 0.25] for k in range(8)])
    pad_pts = np.repeat(pads, 3, axis=0) + rng.uniform(-0.1, 0.1, size=(24, 3))
    tgt_xyz = np.concatenate([tx, pad_pts]).astype(np.float32)
    tgt_cov = np.concatenate([tcov, np.zeros((24, 6))]).astype(np.float32)

    def carried(x, T):
        """Points given in the target frame, expressed in a source frame whose
        relative pose to the target is T (source -> target)."""
        R, t = T[:3, :3], T[:3, 3]
        return (np.asarray(x, np.float64) - t) @ R

    def source(T, kinds_wanted, with_regular=True):
        pts, covs, kinds = [], [], []
        if with_regular:
            rx, _ = room_points(rng, n_regular, half=half, height=height)
            pts.append(carried(rx, T))
            covs.append(knn_covariances(pts[-1], 10, 1e-3))
            kinds += ["regular"] * n_regular
        for kind in kinds_wanted:
            if kind in ("zero", "rank1", "rank2"):
                at = pad_pts[rng.choice(24, size=per_kind, replace=False)]
            else:
                at = tx[rng.choice(n_target, size=per_kind, replace=False)]
            pts.append(carried(at, T))
            covs.append(np.tile(np.array(DEGENERATE_COVS[kind]), (per_kind, 1)))
            kinds += [kind] * per_kind
        return np.concatenate(pts), np.concatenate(covs), kinds

    Tj0 = random_perturbation(rng, 1.0, 30.0)
    Trel0 = random_perturbation(rng, 0.1, 2.0)
    Ti0 = Tj0 @ Trel0
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    Trel1 = np.eye(4)
    Trel1[:3, :3] = Rz
    generic = ["zero", "indefinite", "nan", "inf", "neg_inf"]
    s0x, s0c, k0 = source(Trel0, generic)
    s1x, s1c, k1 = source(Trel1, list(DEGENERATE_COVS))
    deg = np.array([k != "regular" for k in k0])
    sources = [(s0x, s0c), (s1x, s1c), (s0x[deg], s0c[deg]), (s0x[~deg], s0c[~deg])]
    kinds = [k0, k1, [k for k in k0 if k != "regular"], ["regular"] * int((~deg).sum())]
    poses = pose_rows([Ti0, Tj0, Trel1, np.eye(4)])
    factors = np.array([[0, 0, 0, 1], [1, 0, 2, 3], [2, 0, 0, 1], [3, 0, 0, 1]], dtype=np.int32)
    return Workload(
        name=f"degenerate_{seed}", resolution=resolution,
        sources=[_f32_cloud(x, c) for (x, c) in sources],
        targets=[(tgt_xyz, tgt_cov)], poses=poses, factors=factors,
        meta={"seed": [SEED_BASE, 101, seed], "kinds": kinds})


# --------------------------------------------------------------------------
# urban corridor scene and HDL-64-like ring scans
# --------------------------------------------------------------------------

class Corridor:
    """Procedural corridor: ground z=0, facades as vertical quads at 8-12 m
    lateral offset from a smooth random centreline, and poles."""

    def __init__(self, rng: np.random.Generator, length: float,
                 continuous: bool = False):
        ds = 0.25
        s = np.arange(-100.0, length + 100.0 + ds, ds)
        amp = np.deg2rad(rng.uniform(4.0, 10.0, size=3))
        lam = rng.uniform(120.0, 600.0, size=3)
        phase = rng.uniform(0, 2 * np.pi, size=3)
        heading = np.sum(amp[None] * np.sin(2 * np.pi * s[:, None] / lam[None] + phase[None]), axis=1)
        dxy = np.stack([np.cos(heading), np.sin(heading)], 1) * ds
        pos = np.cumsum(dxy, axis=0)
        pos -= pos[np.searchsorted(s, 0.0)]
        self.s, self.heading, self.pos = s, heading, pos

        walls = []    # rows: ax, ay, bx, by, height
        for side in (1.0, -1.0):
            cur = s[0]
            while cur < s[-1] - 1.0:
                seg = rng.uniform(5.0, 15.0)
                off = side * rng.uniform(8.0, 12.0)
                h = rng.uniform(10.0, 30.0)
                gap = (not continuous) and rng.uniform() < 0.15
                if not gap:
                    a = self._at(cur, off)
                    b = self._at(min(cur + seg, s[-1]), off)
                    walls.append([a[0], a[1], b[0], b[1], h])
                cur += seg
        self.walls = np.array(walls)

        poles = []    # rows: cx, cy, radius, height
        cur = s[0]
        while cur < s[-1]:
            cur += rng.uniform(10.0, 25.0)
            side = 1.0 if rng.uniform() < 0.5 else -1.0
            c = self._at(min(cur, s[-1]), side * 6.5)
            poles.append([c[0], c[1], 0.15, 6.0])
        self.poles = np.array(poles)

    def _at(self, s_val: float, lateral: float) -> np.ndarray:
        i = int(np.clip(np.searchsorted(self.s, s_val), 0, len(self.s) - 1))
        h = self.heading[i]
        nrm = np.array([-np.sin(h), np.cos(h)])
        return self.pos[i] + lateral * nrm

    def sensor_pose(self, s_val: float, height: float = 1.8) -> np.ndarray:
        i = int(np.clip(np.searchsorted(self.s, s_val), 0, len(self.s) - 1))
        T = np.eye(4)
        T[:3, :3] = _rodrigues(np.array([0.0, 0.0, 1.0]), self.heading[i])
        T[:2, 3] = self.pos[i]
        T[2, 3] = height
        return T


def raycast_scan(scene: Corridor, T: np.ndarray, rng: np.random.Generator,
                 rings: int = 64, azimuths: int = 1024, el_min: float = -25.0,
                 el_max: float = 2.0, max_range: float = 80.0,
                 noise: float = 0.02):
    """Ring scan from sensor pose T.  Returns sensor-frame points and normals
    (FP64) of valid returns in ring-major order (ring, then azimuth)."""
    el = np.deg2rad(np.linspace(el_min, el_max, rings))
    az = 2 * np.pi * np.arange(azimuths) / azimuths
    ce, se = np.cos(el)[:, None], np.sin(el)[:, None]
    d_s = np.stack([np.broadcast_to(ce * np.cos(az)[None], (rings, azimuths)),
                    np.broadcast_to(ce * np.sin(az)[None], (rings, azimuths)),
                    np.broadcast_to(se, (rings, azimuths))], -1).reshape(-1, 3)
    R, o = T[:3, :3], T[:3, 3]
    d = d_s @ R.T
    nray = d.shape[0]
    best = np.full(nray, np.inf)
    nrm = np.zeros((nray, 3))

    # ground
    down = d[:, 2] < -1e-9
    tg = np.where(down, -o[2] / np.where(down, d[:, 2], -1.0), np.inf)
    upd = tg < best
    best[upd] = tg[upd]
    nrm[upd] = [0.0, 0.0, 1.0]

    d2 = d[:, :2]
    o2 = o[:2]
    # facades near the sensor
    W = scene.walls
    mid = 0.5 * (W[:, :2] + W[:, 2:4])
    near = np.linalg.norm(mid - o2[None], axis=1) < max_range + 20.0
    W = W[near]
    if W.shape[0]:
        A, B, H = W[:, :2], W[:, 2:4], W[:, 4]
        E = B - A                                     # (w, 2)
        AO = A - o2[None]                             # (w, 2)
        den = d2[:, 0:1] * E[None, :, 1] - d2[:, 1:2] * E[None, :, 0]
        den_safe = np.where(np.abs(den) > 1e-12, den, 1.0)
        t = (AO[None, :, 0] * E[None, :, 1] - AO[None, :, 1] * E[None, :, 0]) / den_safe
        u = (AO[None, :, 0] * d2[:, 1:2] - AO[None, :, 1] * d2[:, 0:1]) / den_safe
        z = o[2] + t * d[:, 2:3]
        ok = (np.abs(den) > 1e-12) & (u >= 0) & (u <= 1) & (t > 0) & (z >= 0) & (z <= H[None])
        t = np.where(ok, t, np.inf)
        wi = np.argmin(t, axis=1)
        tw = t[np.arange(nray), wi]
        upd = tw < best
        best[upd] = tw[upd]
        En = E[wi[upd]]
        nn = np.stack([-En[:, 1], En[:, 0], np.zeros(upd.sum())], 1)
        nn /= np.linalg.norm(nn, axis=1, keepdims=True)
        nrm[upd] = nn
    # poles
    P = scene.poles
    near = np.linalg.norm(P[:, :2] - o2[None], axis=1) < max_range + 1.0
    P = P[near]
    if P.shape[0]:
        C, rad, H = P[:, :2], P[:, 2], P[:, 3]
        OC = o2[None] - C                              # (p, 2)
        a = np.sum(d2 * d2, axis=1)[:, None]
        b = 2.0 * (d2 @ OC.T)
        c = np.sum(OC * OC, axis=1)[None] - rad[None] ** 2
        disc = b * b - 4 * a * c
        ok = (disc >= 0) & (a > 1e-12)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t = (-b - sq) / (2 * np.where(a > 1e-12, a, 1.0))
        z = o[2] + t * d[:, 2:3]
        ok &= (t > 0) & (z >= 0) & (z <= H[None])
        t = np.where(ok, t, np.inf)
        pi = np.argmin(t, axis=1)
        tp = t[np.arange(nray), pi]
        upd = tp < best
        best[upd] = tp[upd]
        hit = o2[None] + tp[upd, None] * d2[upd]
        nn = np.concatenate([hit - C[pi[upd]], np.zeros((upd.sum(), 1))], 1)
        nn /= np.linalg.norm(nn, axis=1, keepdims=True)
        nrm[upd] = nn

    valid = best <= max_range
    rng_m = best[valid] + rng.normal(0.0, noise, size=valid.sum())
    pts = d_s[valid] * rng_m[:, None]
    nrm_s = nrm[valid] @ R                           # world -> sensor frame
    return pts, nrm_s


def _scan_frame(args):
    """Worker: one frame's full valid scan with k-NN covariances (and the
    analytic-normal covariances when asked)."""
    scene, T, seed, k, ill_eps = args
    rng = np.random.default_rng(seed)
    pts, nrm = raycast_scan(scene, T, rng)
    cov = knn_covariances(pts, k)
    ill = normal_covariances(nrm, ill_eps) if ill_eps else None
    return pts, cov, ill


def _pool_map(fn, jobs, workers):
    if workers <= 1 or len(jobs) <= 1:
        return [fn(j) for j in jobs]
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, jobs, chunksize=max(1, len(jobs) // (4 * workers))))


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def make_scan_workload(cfg: int, n_frames: int, n_factors: int,
                       n_target: int = 20000, src_range=None,
                       resolution: float = 0.5, k: int = 20,
                       pair_radius: float = 20.0, ill_eps: float = 0.0,
                       workers: int | None = None) -> Workload:
    """Corridor ring-scan workload.

    Frames sit at 1 m spacing along the corridor.  Target clouds are each
    frame's random `n_target`-point subsample.  If `src_range` is None the
    source of factor (i, j) is frame i's target subsample; otherwise factor f
    draws its own subsample of n_f ~ U{src_range} points from frame i's full
    valid scan (seed f).  Covariances come from the full scan.  With
    `ill_eps` > 0 every cloud also carries analytic-normal covariances with
    spectrum (ill_eps, 1, 1) in meta["ill"].  Pose estimates are ground truth
    composed with a 0.1 m / 2 degree perturbation per frame.
    """
    rng = rng_for(cfg)
    scene = Corridor(rng, float(n_frames), continuous=src_range is not None)
    T_gt = [scene.sensor_pose(float(f)) for f in range(n_frames)]
    T_est = [T @ random_perturbation(rng) for T in T_gt]
    seeds = rng.integers(0, 2**63 - 1, size=n_frames)
    jobs = [(scene, T_gt[f], int(seeds[f]), k, ill_eps) for f in range(n_frames)]
    frames = _pool_map(_scan_frame, jobs, workers or default_workers())

    need = n_target if src_range is None else max(n_target, src_range[1])
    targets, ill_targets, full = [], [], []
    for f, (pts, cov, ill) in enumerate(frames):
        if pts.shape[0] < need:
            raise RuntimeError(f"frame {f} has only {pts.shape[0]} returns (< {need})")
        sel = np.sort(rng.choice(pts.shape[0], n_target, replace=False))
        targets.append(_f32_cloud(pts[sel], cov[sel]))
        if ill is not None:
            ill_targets.append(_f32_cloud(pts[sel], ill[sel]))
        full.append((pts, cov, ill))

    pos = np.array([T[:3, 3] for T in T_gt])
    cand = [(i, j) for i in range(n_frames) for j in range(i)
            if np.linalg.norm(pos[i] - pos[j]) <= pair_radius]
    order = rng.permutation(len(cand))
    if n_factors > len(cand):
        raise RuntimeError(f"only {len(cand)} candidate pairs for {n_factors} factors")
    pairs = [cand[o] for o in order[:n_factors]]

    sources, ill_sources, factors = [], [], []
    for f, (i, j) in enumerate(pairs):
        if src_range is None:
            factors.append([i, j, i, j])
        else:
            frng = rng_for(cfg, 1, f)
            pts, cov, ill = full[i]
            nf = int(frng.integers(src_range[0], src_range[1] + 1))
            sel = np.sort(frng.choice(pts.shape[0], nf, replace=False))
            sources.append(_f32_cloud(pts[sel], cov[sel]))
            if ill is not None:
                ill_sources.append(_f32_cloud(pts[sel], ill[sel]))
            factors.append([f, j, i, j])
    if src_range is None:
        sources = targets
        ill_sources = ill_targets
    meta = {"seed": [SEED_BASE, cfg], "k": k, "n_frames": n_frames,
            "valid_returns_mean": float(np.mean([p[0].shape[0] for p in frames])),
            "poses_gt": pose_rows(T_gt)}
    if ill_eps:
        meta["ill"] = {"sources": ill_sources, "targets": ill_targets, "eps": ill_eps}
    return Workload(
        name=f"corridor_{n_frames}frames_{n_factors}factors_r{resolution:g}",
        resolution=resolution, sources=sources, targets=targets,
        poses=pose_rows(T_est), factors=np.array(factors, dtype=np.int32),
        meta=meta)


def _scan_frame_subsampled(args):
    """Worker: one frame's scan, k-NN covariances on the full scan, then a
    random subsample of n_points kept in scan order (FP32)."""
    scene, T, seed, k, n_points = args
    rng = np.random.default_rng(seed)
    pts, _ = raycast_scan(scene, T, rng)
    cov = knn_covariances(pts, k)
    if pts.shape[0] < n_points:
        raise RuntimeError(f"frame has only {pts.shape[0]} returns (< {n_points})")
    sel = np.sort(rng.choice(pts.shape[0], n_points, replace=False))
    return _f32_cloud(pts[sel], cov[sel])


def drive_positions(seed: int, n_frames: int, dt: float = 0.1, v_max: float = 12.0):
    """Arc-length positions of a 10 Hz sensor on a vehicle that cruises at
    2-12 m/s and stops now and then (stops last 1-4 s), seeded."""
    rng = rng_for(400, seed)
    s, v, out = 0.0, 0.0, []
    target, stop_left = rng.uniform(2.0, v_max), 0
    for _ in range(n_frames):
        if stop_left > 0:
            stop_left -= 1
            v = 0.0
        else:
            if rng.random() < 0.01:
                stop_left = int(rng.integers(10, 41))
            if rng.random() < 0.05:
                target = rng.uniform(2.0, v_max)
            v += float(np.clip(target - v, -3.0 * dt, 2.0 * dt))
        s += v * dt
        out.append(s)
    return np.array(out)


def stream_scan_frames(cfg: int, n_frames: int, n_points: int = 20000, k: int = 20,
                       workers: int | None = None, spacing: float = 1.0,
                       positions=None, with_truth: bool = False,
                       perturb=(0.1, 2.0)):
    """Yield (index, estimated pose 4x4, xyz float32 (n,3), cov float32 (n,6))
    for keyframes `spacing` metres apart along a corridor (or at the given
    arc-length `positions`), generated in a process pool and returned in
    order (memory stays bounded by the pool).  Each estimate is the truth
    composed with a random (translation m, rotation deg) = `perturb` motion.
    With `with_truth` the ground truth pose follows the estimate:
    (index, T_est, T_gt, xyz, cov)."""
    rng = rng_for(cfg)
    if positions is None:
        positions = np.arange(n_frames) * float(spacing)
    positions = np.asarray(positions, dtype=np.float64)
    assert positions.shape == (n_frames,)
    scene = Corridor(rng, float(positions.max(initial=0.0)) + 1.0, continuous=False)
    T_gt = [scene.sensor_pose(float(s)) for s in positions]
    T_est = [T @ random_perturbation(rng, *perturb) for T in T_gt]
    seeds = rng.integers(0, 2**63 - 1, size=n_frames)
    # a sensor at rest sees the same returns again
    for f in range(1, n_frames):
        if positions[f] == positions[f - 1]:
            seeds[f] = seeds[f - 1]
    jobs = [(scene, T_gt[f], int(seeds[f]), k, n_points) for f in range(n_frames)]
    w = workers or default_workers()
    if w <= 1:
        for f, job in enumerate(jobs):
            xyz, cov = _scan_frame_subsampled(job)
            yield (f, T_est[f], T_gt[f], xyz, cov) if with_truth else (f, T_est[f], xyz, cov)
        return
    with ProcessPoolExecutor(max_workers=w) as ex:
        for f, (xyz, cov) in enumerate(ex.map(_scan_frame_subsampled, jobs, chunksize=4)):
            yield (f, T_est[f], T_gt[f], xyz, cov) if with_truth else (f, T_est[f], xyz, cov)
