"""Plain FP64 CPU oracle for VGICP matching-cost factors.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the library.  It is deliberately slow and
literal: every continuous quantity is computed in FP64 straight from the
paper's definitions, with no blocking, fusion or algebraic shortcut.

Paper: Koide et al., "Globally Consistent 3D LiDAR Mapping with
GPU-accelerated GICP Matching Cost Factors", IEEE RA-L 2021.

  voxelize          Sec. III-A, VGICP data association (voxel mean and the
                    aggregated point covariances per voxel)
  relative_pose     Sec. III-A, Eq. (3): relative pose between the pair
  lookup            Sec. III-A, Eq. (3): corresponding voxel of each point
  fma32             exact FP32 fused multiply-add (rounding to odd)
  linearize_factor  Sec. III-A, Eqs. (2)-(6): error, Hessian factor, b
  evaluate_factor   Sec. III-A, Eq. (3): the matching cost alone
  overlap_factor    Sec. III-B, Eqs. (7)-(8): voxel overlap rate
  factor_admitted   Sec. III-C: overlap-gated factor creation
  submap_decision   Sec. III-B: skip / insert / close of a local submap
  assemble_system   Sec. III-D: the factors' Hessians summed into the
                    global linear system over all poses

Readings where the paper is silent (each one is also a line of the design
notes):
  * the source cloud is mapped into the target frame by T_j^-1 T_i, the
    pose that carries P_i's points into the frame of P_j's voxel map;
  * poses are sensor-to-world, perturbed on the right, T <- T Exp(xi) with
    xi = (omega, rho), and the 12-vector order is [xi_i; xi_j];
  * the voxel key of a point is floor(fl32(x * fl32(1/r))) per axis in FP32,
    keys lie in [-2^20, 2^20); the voxel mean is fl32 of the FP64 mean of
    the points and the voxel covariance fl32 of the FP64 mean of the point
    covariances;
  * the correspondence of a point is decided in FP32: its coordinates in
    voxel units are three fused multiply-adds per axis with the rotation and
    translation scaled by fl32(1/r) and rounded to FP32 (lookup_coords_fp32),
    and its key is their floor; the residual and weights are then FP64;
  * only the single voxel holding the transformed point is used; points in
    no voxel contribute nothing and are not inliers;
  * e is the plain sum of d^T Omega d (no 1/2), b = sum J^T Omega e with
    e_k = mu'_k - T mu_k, Omega and the correspondences frozen at the
    linearization point;
  * a hit whose fused covariance is not positive definite contributes
    nothing to H, b, e but is still counted as an inlier;
  * an empty source cloud has overlap 0.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

KEY_LIMIT = 1 << 20          # voxel keys lie in [-KEY_LIMIT, KEY_LIMIT)


# --------------------------------------------------------------------------
# small linear-algebra helpers (FP64)
# --------------------------------------------------------------------------

def _unpack_cov(c6: np.ndarray) -> np.ndarray:
    """(n, 6) xx, xy, xz, yy, yz, zz -> (n, 3, 3) symmetric, FP64."""
    c = np.asarray(c6, dtype=np.float64)
    out = np.empty(c.shape[:-1] + (3, 3))
    out[..., 0, 0] = c[..., 0]
    out[..., 0, 1] = out[..., 1, 0] = c[..., 1]
    out[..., 0, 2] = out[..., 2, 0] = c[..., 2]
    out[..., 1, 1] = c[..., 3]
    out[..., 1, 2] = out[..., 2, 1] = c[..., 4]
    out[..., 2, 2] = c[..., 5]
    return out


def _skew(v: np.ndarray) -> np.ndarray:
    """[v]x for (n, 3) vectors: [v]x w = v cross w."""
    n = v.shape[0]
    S = np.zeros((n, 3, 3))
    S[:, 0, 1] = -v[:, 2]
    S[:, 0, 2] = v[:, 1]
    S[:, 1, 0] = v[:, 2]
    S[:, 1, 2] = -v[:, 0]
    S[:, 2, 0] = -v[:, 1]
    S[:, 2, 1] = v[:, 0]
    return S


def _pose_matrix(pose12) -> tuple[np.ndarray, np.ndarray]:
    p = np.asarray(pose12, dtype=np.float64).reshape(12)
    return p[:9].reshape(3, 3), p[9:].copy()


# --------------------------------------------------------------------------
# voxel map (Sec. III-A, VGICP voxel data association)
# --------------------------------------------------------------------------

@dataclass
class VoxelMap:
    """keys (V, 3) int64 in lexicographic (kx, ky, kz) order; the voxel
    ordinal is the row index.  mean (V, 3) and cov (V, 6) are float32,
    count (V,) int64.  scale is fl32(1 / resolution)."""
    keys: np.ndarray
    mean: np.ndarray
    cov: np.ndarray
    count: np.ndarray
    scale: np.float32
    resolution: float

    @property
    def n_voxels(self) -> int:
        return int(self.keys.shape[0])


def voxel_scale(resolution: float) -> np.float32:
    """fl32(1 / r), the reciprocal taken in FP64 and rounded once."""
    r = float(resolution)
    if not (np.isfinite(r) and r > 0.0):
        raise ValueError("resolution must be finite and > 0")
    return np.float32(1.0 / r)


def _scaled_fl32(xyz32: np.ndarray, s: np.float32) -> np.ndarray:
    x = np.asarray(xyz32, dtype=np.float32)
    return (x * np.float32(s)).astype(np.float32)      # one FP32 rounding


def voxel_keys(xyz32: np.ndarray, s: np.float32) -> np.ndarray:
    """Integer voxel key per point: floor(fl32(x * s)) per axis.  Raises on
    non-finite coordinates and on keys outside [-2^20, 2^20)."""
    v = _scaled_fl32(xyz32, s)
    if not np.all(np.isfinite(v)):
        raise FloatingPointError("non-finite point coordinate")
    k = np.floor(v.astype(np.float64))
    if np.any(k < -KEY_LIMIT) or np.any(k >= KEY_LIMIT):
        raise OverflowError("voxel key outside [-2^20, 2^20)")
    return k.astype(np.int64).reshape(-1, 3)


def voxelize(xyz32: np.ndarray, cov32: np.ndarray, resolution: float):
    """Voxel map of a cloud at resolution r.

    Each voxel holds the points whose key equals its key; its mean is the
    FP64 mean of their positions and its covariance the FP64 mean of their
    covariances (the VGICP aggregation of point distributions), both
    accumulated in point order and rounded once to FP32.
    Returns (VoxelMap, ordinal of each point)."""
    s = voxel_scale(resolution)
    xyz32 = np.asarray(xyz32, dtype=np.float32).reshape(-1, 3)
    cov32 = np.asarray(cov32, dtype=np.float32).reshape(-1, 6)
    if xyz32.shape[0] != cov32.shape[0]:
        raise ValueError("xyz and cov lengths differ")
    if xyz32.shape[0] == 0:
        empty = VoxelMap(np.zeros((0, 3), np.int64), np.zeros((0, 3), np.float32),
                         np.zeros((0, 6), np.float32), np.zeros(0, np.int64), s,
                         float(resolution))
        return empty, np.zeros(0, np.int64)
    keys = voxel_keys(xyz32, s)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    V = uniq.shape[0]
    count = np.bincount(inv, minlength=V).astype(np.int64)
    sum_mu = np.zeros((V, 3))
    sum_cov = np.zeros((V, 6))
    np.add.at(sum_mu, inv, xyz32.astype(np.float64))     # sequential, point order
    np.add.at(sum_cov, inv, cov32.astype(np.float64))
    mean = (sum_mu / count[:, None]).astype(np.float32)
    cov = (sum_cov / count[:, None]).astype(np.float32)
    return VoxelMap(uniq.astype(np.int64), mean, cov, count, s, float(resolution)), inv


# --------------------------------------------------------------------------
# relative pose and correspondence (Sec. III-A, Eq. (3))
# --------------------------------------------------------------------------

def relative_pose(pose_i, pose_j) -> tuple[np.ndarray, np.ndarray]:
    """T_j^-1 T_i in FP64 with a fixed evaluation order:
        R[r][c] = (Rj[0][r] Ri[0][c] + Rj[1][r] Ri[1][c]) + Rj[2][r] Ri[2][c]
        d = t_i - t_j,  t[r] = (Rj[0][r] d0 + Rj[1][r] d1) + Rj[2][r] d2
    and exactly (I, 0) when the two poses are bitwise equal."""
    pi = np.asarray(pose_i, dtype=np.float64).reshape(12)
    pj = np.asarray(pose_j, dtype=np.float64).reshape(12)
    if np.array_equal(pi.view(np.uint64), pj.view(np.uint64)):
        return np.eye(3), np.zeros(3)
    Ri, ti = _pose_matrix(pi)
    Rj, tj = _pose_matrix(pj)
    R = np.empty((3, 3))
    for r in range(3):
        for c in range(3):
            R[r, c] = (Rj[0, r] * Ri[0, c] + Rj[1, r] * Ri[1, c]) + Rj[2, r] * Ri[2, c]
    d = ti - tj
    t = np.empty(3)
    for r in range(3):
        t[r] = (Rj[0, r] * d[0] + Rj[1, r] * d[1]) + Rj[2, r] * d[2]
    return R, t


def fma32(a, b, c) -> np.ndarray:
    """FP32 fused multiply-add: a * b + c for float32 operands, rounded once
    to FP32 (round to nearest, ties to even).

    The product of two float32 values is exact in FP64.  Knuth's two-sum
    splits the FP64 sum into its rounding s and the exact error err
    (a * b + c = s + err); s is then rounded to odd (replaced by its neighbour
    towards err, which has an odd last bit, when err != 0 and s's last bit is
    even), and one FP64 -> FP32 rounding of that is the correctly rounded
    result: rounding to odd with at least two spare bits followed by rounding
    to nearest equals one rounding to nearest (Boldo and Melquiond, "Emulation
    of FMA and correctly rounded sums: proved algorithms using rounding to
    odd", IEEE Trans. Computers 57(4), 2008).  Non-finite values pass through."""
    a64 = np.asarray(a, dtype=np.float32).astype(np.float64)
    b64 = np.asarray(b, dtype=np.float32).astype(np.float64)
    c64 = np.asarray(c, dtype=np.float32).astype(np.float64)
    with np.errstate(invalid="ignore", over="ignore"):
        p = a64 * b64
        s = np.asarray(p + c64, dtype=np.float64)
        bp = s - p
        err = (p - (s - bp)) + (c64 - bp)
        even = (s.view(np.int64) & 1) == 0
        fix = np.isfinite(s) & (err != 0) & even
        s = np.where(fix, np.nextafter(s, np.where(err > 0, np.inf, -np.inf)), s)
        return s.astype(np.float32)


def lookup_coords_fp32(xyz32: np.ndarray, R: np.ndarray, t: np.ndarray, s) -> np.ndarray:
    """The FP32 coordinates, in voxel units, that decide correspondences
    (Sec. III-A, Eq. (3): the voxel holding T_j^-1 T_i mu):
        v_r = fma(S[r][2], z, fma(S[r][1], y, fma(S[r][0], x, u[r])))
    with S = fl32(s R) and u = fl32(s t) (FP64 products, one rounding each),
    every fma rounded once to FP32, and s = fl32(1/r) the map's scale."""
    S = (np.float64(s) * np.asarray(R, dtype=np.float64)).astype(np.float32)
    with np.errstate(over="ignore"):
        u = (np.float64(s) * np.asarray(t, dtype=np.float64)).astype(np.float32)
    p = np.asarray(xyz32, dtype=np.float32).reshape(-1, 3)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    v = np.empty_like(p)
    for r in range(3):
        v[:, r] = fma32(S[r, 2], z, fma32(S[r, 1], y, fma32(S[r, 0], x, u[r])))
    return v


def _packed(keys: np.ndarray) -> np.ndarray:
    k = np.asarray(keys, dtype=np.int64) + KEY_LIMIT
    return (k[:, 0] << 42) | (k[:, 1] << 21) | k[:, 2]


def lookup(vmap: VoxelMap, xyz32: np.ndarray, R: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Ordinal of the voxel of `vmap` containing each transformed point, or
    -1 when that voxel is empty or its key is outside the key range."""
    v = lookup_coords_fp32(xyz32, R, t, vmap.scale)
    ok = np.all(np.isfinite(v), axis=1)
    kf = np.floor(np.where(np.isfinite(v), v, 0.0).astype(np.float64))
    ok &= np.all((kf >= -KEY_LIMIT) & (kf < KEY_LIMIT), axis=1)
    corr = np.full(v.shape[0], -1, dtype=np.int64)
    if vmap.n_voxels == 0 or not ok.any():
        return corr
    table = _packed(vmap.keys)                      # sorted because keys are
    want = _packed(kf[ok].astype(np.int64))
    pos = np.searchsorted(table, want)
    pos_c = np.minimum(pos, table.shape[0] - 1)
    found = table[pos_c] == want
    idx = np.flatnonzero(ok)
    corr[idx[found]] = pos_c[found]
    return corr


# --------------------------------------------------------------------------
# per-correspondence terms (Sec. III-A, Eqs. (2), (4)-(6))
# --------------------------------------------------------------------------

def fused_covariance(Sigma_v: np.ndarray, C_k: np.ndarray, R: np.ndarray) -> np.ndarray:
    """F_k = C'_k + R C_k R^T for (n, 3, 3) stacks, FP64 (Eq. (2))."""
    return Sigma_v + np.einsum("ab,nbc,dc->nad", R, C_k, R)


def positive_definite(F: np.ndarray) -> np.ndarray:
    """Rows of an (n, 3, 3) stack that are positive definite: every entry
    finite and the three leading principal minors positive (Sylvester's
    criterion)."""
    F = np.asarray(F, dtype=np.float64)
    ok = np.all(np.isfinite(F), axis=(1, 2))
    out = np.zeros(F.shape[0], dtype=bool)
    if ok.any():
        G = F[ok]
        d1 = G[:, 0, 0]
        d2 = G[:, 0, 0] * G[:, 1, 1] - G[:, 0, 1] * G[:, 1, 0]
        d3 = np.linalg.det(G)
        out[ok] = (d1 > 0) & (d2 > 0) & (d3 > 0)
    return out


def fused_information(Sigma_v: np.ndarray, C_k: np.ndarray, R: np.ndarray) -> tuple:
    """Omega_k = (C'_k + R C_k R^T)^-1 for (n, 3, 3) stacks, FP64 (Eq. (2)).

    Returns (Omega, good).  Only rows whose fused covariance is positive
    definite are inverted; the others (singular, indefinite or non-finite:
    Eq. (2) defines no weight for them) get Omega = 0 and good = False."""
    F = fused_covariance(Sigma_v, C_k, R)
    good = positive_definite(F)
    Omega = np.zeros_like(F)
    if good.any():
        Omega[good] = np.linalg.inv(F[good])
    return Omega, good


def residuals(m_v: np.ndarray, R: np.ndarray, t: np.ndarray, mu: np.ndarray) -> tuple:
    """q_k = R mu_k + t and e_k = mu'_k - q_k, FP64."""
    q = mu @ R.T + t[None]
    return m_v - q, q


def jacobians(R: np.ndarray, mu: np.ndarray, q: np.ndarray) -> tuple:
    """A_k = d e_k / d xi_i = [R [mu]x, -R] and B_k = d e_k / d xi_j =
    [-[q]x, I] under right perturbations with xi = (omega, rho)."""
    n = mu.shape[0]
    A = np.empty((n, 3, 6))
    A[:, :, :3] = np.einsum("ab,nbc->nac", R, _skew(mu))
    A[:, :, 3:] = -R[None]
    B = np.empty((n, 3, 6))
    B[:, :, :3] = -_skew(q)
    B[:, :, 3:] = np.eye(3)[None]
    return A, B


def linearize_factor(src_xyz32, src_cov32, vmap: VoxelMap, pose_i, pose_j):
    """Hessian factor of one matching-cost factor e^M(P_i, P_j, T_i, T_j).

    Returns dict with H (12, 12) = [[H_ii, H_ij], [H_ij^T, H_jj]], b (12,) =
    [b_i; b_j], e (the cost, Eq. (3)), inliers and corr (per-point voxel
    ordinal or -1)."""
    R, t = relative_pose(pose_i, pose_j)
    xyz32 = np.asarray(src_xyz32, dtype=np.float32).reshape(-1, 3)
    corr = lookup(vmap, xyz32, R, t)
    hit = corr >= 0
    H = np.zeros((12, 12))
    b = np.zeros(12)
    e = 0.0
    inliers = int(hit.sum())
    if inliers:
        mu = xyz32[hit].astype(np.float64)
        C_k = _unpack_cov(np.asarray(src_cov32, dtype=np.float32).reshape(-1, 6)[hit])
        m_v = vmap.mean[corr[hit]].astype(np.float64)
        S_v = _unpack_cov(vmap.cov[corr[hit]])
        res, q = residuals(m_v, R, t, mu)
        Omega, good = fused_information(S_v, C_k, R)
        A, B = jacobians(R, mu, q)
        J = np.concatenate([A, B], axis=2)[good]          # (n, 3, 12)
        Om = Omega[good]
        r = res[good]
        JtO = np.einsum("nai,nab->nib", J, Om)             # J^T Omega
        H = np.einsum("nib,nbj->ij", JtO, J)
        b = np.einsum("nib,nb->i", JtO, r)
        e = float(np.einsum("na,nab,nb->", r, Om, r))
    return {"H": H, "b": b, "e": e, "inliers": inliers, "corr": corr, "R": R, "t": t}


def evaluate_factor(src_xyz32, src_cov32, vmap: VoxelMap, pose_i, pose_j):
    """The matching cost e^M (Eq. (3)) and inlier count without the Hessian
    factor."""
    out = linearize_factor(src_xyz32, src_cov32, vmap, pose_i, pose_j)
    return {"e": out["e"], "inliers": out["inliers"]}


# --------------------------------------------------------------------------
# overlap (Sec. III-B, Eqs. (7)-(8))
# --------------------------------------------------------------------------

def overlap_factor(src_xyz32, vmap: VoxelMap, pose_i, pose_j):
    """hits = number of source points falling in a voxel of the target map
    under T_j^-1 T_i; overlap = hits / N (0 for an empty source)."""
    R, t = relative_pose(pose_i, pose_j)
    corr = lookup(vmap, src_xyz32, R, t)
    hits = int((corr >= 0).sum())
    n = int(np.asarray(src_xyz32).reshape(-1, 3).shape[0])
    return hits, (hits / n if n else 0.0)


# --------------------------------------------------------------------------
# keyframe control by overlap (Sec. III-B local mapping, Sec. III-C global)
# --------------------------------------------------------------------------

def factor_admitted(overlap: float, threshold: float, at_least: bool = False) -> bool:
    """Sec. III-C: a matching-cost factor is created for a keyframe pair whose
    overlap rate is larger than th^G_min.  at_least=True is the variant that
    also admits an overlap equal to the threshold."""
    return overlap >= threshold if at_least else overlap > threshold


def submap_decision(n_submap: int, overlap_last: float, overlap_first: float,
                    skip_above: float, close_below: float, max_frames: int) -> str:
    """Sec. III-B, for a frame arriving at a submap of n_submap frames, given
    its overlap with the submap's last frame and with its first frame:
      * an empty submap: the frame starts it ("start");
      * overlap with the last frame above th^L_max: the sensor has not moved
        and the frame is skipped ("skip");
      * otherwise the frame is inserted; the submap is then closed when the
        overlap between its first and newest (this) frame is below th^L_min
        or it holds more than N^L_max frames ("close"), else it stays open
        ("insert")."""
    if n_submap == 0:
        return "start"
    if overlap_last > skip_above:
        return "skip"
    if overlap_first < close_below or n_submap + 1 > max_frames:
        return "close"
    return "insert"


# --------------------------------------------------------------------------
# batch drivers over a factor list
# --------------------------------------------------------------------------

def build_maps(targets, resolution: float):
    return [voxelize(x, c, resolution)[0] for (x, c) in targets]


def linearize_workload(sources, maps, poses, factors, with_corr: bool = False):
    """Loop linearize_factor over (src, tgt, pose_i, pose_j) rows."""
    factors = np.asarray(factors).reshape(-1, 4)
    F = factors.shape[0]
    H = np.zeros((F, 12, 12))
    b = np.zeros((F, 12))
    e = np.zeros(F)
    inl = np.zeros(F, dtype=np.int64)
    corr = []
    for f, (s, tg, pi, pj) in enumerate(factors):
        out = linearize_factor(sources[s][0], sources[s][1], maps[tg], poses[pi], poses[pj])
        H[f], b[f], e[f], inl[f] = out["H"], out["b"], out["e"], out["inliers"]
        if with_corr:
            corr.append(out["corr"])
    res = {"H": H, "b": b, "e": e, "inliers": inl}
    if with_corr:
        res["corr"] = corr
    return res


def overlap_workload(sources, maps, poses, factors):
    factors = np.asarray(factors).reshape(-1, 4)
    hits = np.zeros(factors.shape[0], dtype=np.int64)
    ov = np.zeros(factors.shape[0])
    for f, (s, tg, pi, pj) in enumerate(factors):
        hits[f], ov[f] = overlap_factor(sources[s][0], maps[tg], poses[pi], poses[pj])
    return hits, ov


# --------------------------------------------------------------------------
# assembly of the global linear system (Sec. III-D)
# --------------------------------------------------------------------------

def assemble_system(H, b, factors, n_poses: int):
    """Global Gauss-Newton system over all poses, 6 unknowns (omega, rho) per
    pose.  Factor f with poses (i, j) maps the global perturbation to its own
    12-vector through the selection S_f = [E_i; E_j] (E_p picks pose p's six
    unknowns), so it adds S_f^T H_f S_f to the global matrix and S_f^T b_f to
    the global vector.  Returns the dense (6P, 6P) matrix and (6P,) vector."""
    factors = np.asarray(factors).reshape(-1, 4)
    P6 = 6 * int(n_poses)
    Hg = np.zeros((P6, P6))
    bg = np.zeros(P6)
    for f, (_, _, pi, pj) in enumerate(factors):
        S = np.zeros((12, P6))
        S[0:6, 6 * pi:6 * pi + 6] += np.eye(6)
        S[6:12, 6 * pj:6 * pj + 6] += np.eye(6)
        Hg += S.T @ np.asarray(H[f], np.float64) @ S
        bg += S.T @ np.asarray(b[f], np.float64)
    return Hg, bg


def system_blocks(Hg, bg, n_poses: int, pairs):
    """Diagonal 6x6 blocks, per-pose b and the (p, q) blocks of the listed
    pose pairs, read out of the dense system."""
    P = int(n_poses)
    diag = np.stack([Hg[6 * p:6 * p + 6, 6 * p:6 * p + 6] for p in range(P)]) if P else np.zeros((0, 6, 6))
    bvec = bg.reshape(P, 6)
    off = np.stack([Hg[6 * p:6 * p + 6, 6 * q:6 * q + 6] for (p, q) in pairs]) if len(pairs) else np.zeros((0, 6, 6))
    return diag, bvec, off
