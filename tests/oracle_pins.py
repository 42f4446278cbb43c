"""Independent checks of the FP64 oracle (helpers shared by the pin tests and
the planted-mistake tests).  Nothing here calls the HIP library.

Each helper recomputes a fact the paper or plain mathematics fixes by a route
different from the oracle's own code:
  * rigid motions through 4x4 homogeneous matrices and np.linalg.inv;
  * Jacobians by central finite differences of the frozen residual;
  * point-to-point ICP normal equations for isotropic covariances, written
    with cross-product identities instead of stacked Jacobians.
"""

import numpy as np

import oracle


def hom(pose12):
    p = np.asarray(pose12, dtype=np.float64)
    T = np.eye(4)
    T[:3, :3] = p[:9].reshape(3, 3)
    T[:3, 3] = p[9:]
    return T


def rows(T):
    return np.concatenate([T[:3, :3].reshape(9), T[:3, 3]])


def so3_exp(w):
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th**2 * (K @ K)


def se3_exp_right(xi):
    """Retraction T <- T Exp(xi), xi = (omega, rho); first-order exact."""
    T = np.eye(4)
    T[:3, :3] = so3_exp(xi[:3])
    T[:3, 3] = xi[3:]
    return T


def unpack6(c):
    c = np.asarray(c, dtype=np.float64)
    return np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])


def frozen_residuals(xi12, Ti, Tj, mu, m):
    """r_k(xi) = m_k - (T_j Exp xi_j)^-1 (T_i Exp xi_i) mu_k, (n, 3)."""
    Ti_p = Ti @ se3_exp_right(xi12[:6])
    Tj_p = Tj @ se3_exp_right(xi12[6:])
    Tji = np.linalg.inv(Tj_p) @ Ti_p
    q = mu @ Tji[:3, :3].T + Tji[:3, 3]
    return m - q


def fd_hessian_factor(src_xyz, src_cov, vmap, pose_i, pose_j, h=1e-6):
    """H, b, e and per-point Jacobians from central differences of the
    frozen residual, with Omega built from 4x4 algebra."""
    out = oracle.linearize_factor(src_xyz, src_cov, vmap, pose_i, pose_j)
    corr = out["corr"]
    hit = corr >= 0
    Ti, Tj = hom(pose_i), hom(pose_j)
    Tji = np.linalg.inv(Tj) @ Ti
    R = Tji[:3, :3]
    mu = np.asarray(src_xyz, np.float64)[hit]
    m = vmap.mean[corr[hit]].astype(np.float64)
    n = mu.shape[0]
    J = np.zeros((n, 3, 12))
    for a in range(12):
        d = np.zeros(12)
        d[a] = h
        J[:, :, a] = (frozen_residuals(d, Ti, Tj, mu, m) - frozen_residuals(-d, Ti, Tj, mu, m)) / (2 * h)
    r0 = frozen_residuals(np.zeros(12), Ti, Tj, mu, m)
    Om = np.empty((n, 3, 3))
    cov = np.asarray(src_cov, np.float64)[hit]
    vc = vmap.cov[corr[hit]].astype(np.float64)
    for k in range(n):
        Om[k] = np.linalg.inv(unpack6(vc[k]) + R @ unpack6(cov[k]) @ R.T)
    H = np.einsum("nai,nab,nbj->ij", J, Om, J)
    b = np.einsum("nai,nab,nb->i", J, Om, r0)
    e = float(np.einsum("na,nab,nb->", r0, Om, r0))
    return {"H": H, "b": b, "e": e, "J": J, "oracle": out}


def fd_cost_gradient(src_xyz, src_cov, vmap, pose_i, pose_j, h=1e-6):
    """Gradient of the frozen cost sum r^T Omega r by central differences."""
    out = oracle.linearize_factor(src_xyz, src_cov, vmap, pose_i, pose_j)
    corr = out["corr"]
    hit = corr >= 0
    Ti, Tj = hom(pose_i), hom(pose_j)
    Tji = np.linalg.inv(Tj) @ Ti
    R = Tji[:3, :3]
    mu = np.asarray(src_xyz, np.float64)[hit]
    m = vmap.mean[corr[hit]].astype(np.float64)
    cov = np.asarray(src_cov, np.float64)[hit]
    vc = vmap.cov[corr[hit]].astype(np.float64)
    Om = np.stack([np.linalg.inv(unpack6(vc[k]) + R @ unpack6(cov[k]) @ R.T) for k in range(mu.shape[0])])

    def cost(xi):
        r = frozen_residuals(xi, Ti, Tj, mu, m)
        return float(np.einsum("na,nab,nb->", r, Om, r))

    g = np.zeros(12)
    for a in range(12):
        d = np.zeros(12)
        d[a] = h
        g[a] = (cost(d) - cost(-d)) / (2 * h)
    return g, out


def icp_normal_equations(src_xyz, vmap, pose_i, pose_j, corr, w):
    """Point-to-point ICP Gauss-Newton system for isotropic weights w*I,
    written with cross-product identities ([v]x^T [v]x = |v|^2 I - v v^T)."""
    Tji = np.linalg.inv(hom(pose_j)) @ hom(pose_i)
    R, t = Tji[:3, :3], Tji[:3, 3]
    hit = corr >= 0
    mu = np.asarray(src_xyz, np.float64)[hit]
    m = vmap.mean[corr[hit]].astype(np.float64)
    H = np.zeros((12, 12))
    b = np.zeros(12)
    e = 0.0
    I3 = np.eye(3)

    def sk(v):
        return np.array([[0, -v[2], v[1]], [v[2], 0, -v[0]], [-v[1], v[0], 0]])

    for k in range(mu.shape[0]):
        u = mu[k]
        q = R @ u + t
        r = m[k] - q
        rs = R.T @ r
        Hii = np.block([[(u @ u) * I3 - np.outer(u, u), sk(u)], [-sk(u), I3]])
        Hjj = np.block([[(q @ q) * I3 - np.outer(q, q), sk(q)], [-sk(q), I3]])
        Hij = np.block([[sk(u) @ R.T @ sk(q), -sk(u) @ R.T], [R.T @ sk(q), -R.T]])
        H[:6, :6] += Hii
        H[6:, 6:] += Hjj
        H[:6, 6:] += Hij
        H[6:, :6] += Hij.T
        b[:3] += np.cross(rs, u)
        b[3:6] += -rs
        b[6:9] += np.cross(q, r)
        b[9:] += r
        e += r @ r
    return w * H, w * b, w * e


def null_space_basis(pose_i, pose_j):
    """Columns [Ad(T_i^-1) eta; Ad(T_j^-1) eta] for the six unit eta: a common
    left motion of both poses leaves T_j^-1 T_i unchanged."""
    def ad(T):
        R, t = T[:3, :3], T[:3, 3]
        S = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
        A = np.zeros((6, 6))
        A[:3, :3] = R
        A[3:, :3] = S @ R
        A[3:, 3:] = R
        return A
    Ai = ad(np.linalg.inv(hom(pose_i)))
    Aj = ad(np.linalg.inv(hom(pose_j)))
    return np.vstack([Ai, Aj])          # (12, 6)


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def small_pose_graph(seed=5, n_poses=4):
    """Four nearby poses and room clouds, with factors that exercise every
    case of the assembly: distinct pairs, a pair repeated, the same pair
    reversed, and a factor whose two poses coincide."""
    from synth import make_tiny_workload, pose_rows
    from synth.scenes import random_perturbation, rng_for
    w = make_tiny_workload(seed=seed, n_src=300, n_tgt=500, resolution=0.5, n_factors=3)
    rng = rng_for(300, seed)
    T = [np.eye(4)] + [random_perturbation(rng, 0.15, 3.0) for _ in range(n_poses - 1)]
    w.poses = pose_rows(T)
    w.factors = np.array([[0, 1, 0, 1], [1, 2, 1, 2], [2, 0, 3, 0], [0, 2, 1, 0],
                          [1, 0, 0, 1], [2, 1, 2, 2], [1, 2, 3, 1]], dtype=np.int32)
    return w


def fd_global_system(w, h=1e-6):
    """Global H, b over all poses from finite differences of each factor's
    frozen residual in the 6P-vector of pose perturbations (each factor sees
    its own two poses' slices; a factor on one pose sees that slice twice)."""
    P = w.poses.shape[0]
    maps = oracle.build_maps(w.targets, w.resolution)
    Hg = np.zeros((6 * P, 6 * P))
    bg = np.zeros(6 * P)
    for (s, tg, pi, pj) in w.factors:
        xyz, cov = w.sources[s]
        out = oracle.linearize_factor(xyz, cov, maps[tg], w.poses[pi], w.poses[pj])
        hit = out["corr"] >= 0
        Ti, Tj = hom(w.poses[pi]), hom(w.poses[pj])
        R = (np.linalg.inv(Tj) @ Ti)[:3, :3]
        mu = np.asarray(xyz, np.float64)[hit]
        m = maps[tg].mean[out["corr"][hit]].astype(np.float64)
        cs = np.asarray(cov, np.float64)[hit]
        vc = maps[tg].cov[out["corr"][hit]].astype(np.float64)
        Om = np.stack([np.linalg.inv(unpack6(vc[k]) + R @ unpack6(cs[k]) @ R.T)
                       for k in range(mu.shape[0])])

        def resid(x):
            return frozen_residuals(np.concatenate([x[6 * pi:6 * pi + 6], x[6 * pj:6 * pj + 6]]),
                                    Ti, Tj, mu, m)
        J = np.zeros((mu.shape[0], 3, 6 * P))
        for a in range(6 * P):
            d = np.zeros(6 * P)
            d[a] = h
            J[:, :, a] = (resid(d) - resid(-d)) / (2 * h)
        r0 = resid(np.zeros(6 * P))
        Hg += np.einsum("nai,nab,nbj->ij", J, Om, J)
        bg += np.einsum("nai,nab,nb->i", J, Om, r0)
    return Hg, bg


def global_null_space(poses):
    """Columns Ad(T_p^-1) eta stacked over all poses, for the six unit eta:
    a common left motion of every pose leaves every relative pose unchanged."""
    cols = []
    for p in poses:
        Ti = np.linalg.inv(hom(p))
        R, t = Ti[:3, :3], Ti[:3, 3]
        S = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
        A = np.zeros((6, 6))
        A[:3, :3] = R
        A[3:, :3] = S @ R
        A[3:, 3:] = R
        cols.append(A)
    return np.vstack(cols)


def degenerate_pins(w):
    """Pins of the reading for hits whose fused covariance is not positive
    definite (Eq. (2) gives them no weight): each such hit is an inlier and
    adds exactly nothing.  `w` is synth.make_degenerate_workload().  Raises
    AssertionError (or LinAlgError from an oracle that inverts a singular
    matrix) when a pin fails.

      * every degenerate point lies, under the exact 4x4 relative motion, in
        the box of the voxel the oracle assigns it (a hit by geometry);
      * inliers = every hit, degenerate ones included;
      * the factor of degenerate points alone: H = 0, b = 0, e = 0 exactly;
      * a factor with degenerate points equals, bit for bit, the factor of
        its regular points alone, and that one matches central finite
        differences of the frozen residual;
      * the exact 90 degree factor (rank-one and rank-two covariances stay
        exactly singular) equals the oracle on its regular points alone."""
    vm = oracle.voxelize(*w.targets[0], w.resolution)[0]
    kinds = w.meta["kinds"]
    outs = []
    for f, (s, _, pi, pj) in enumerate(w.factors):
        xyz, cov = w.sources[s]
        out = oracle.linearize_factor(xyz, cov, vm, w.poses[pi], w.poses[pj])
        outs.append(out)
        deg = np.array([k != "regular" for k in kinds[f]])
        corr = out["corr"]
        assert np.all(corr[deg] >= 0), f"factor {f}: a degenerate point misses"
        T = np.linalg.inv(hom(w.poses[pj])) @ hom(w.poses[pi])
        q = xyz[deg].astype(np.float64) @ T[:3, :3].T + T[:3, 3]
        lo = vm.keys[corr[deg]] * w.resolution
        assert np.all((q >= lo - 1e-6) & (q < lo + w.resolution + 1e-6)), f"factor {f}: box"
        assert out["inliers"] == int((corr >= 0).sum()), f"factor {f}: inliers"
    # degenerate points only
    assert outs[2]["inliers"] == len(kinds[2])
    assert not outs[2]["H"].any() and not outs[2]["b"].any() and outs[2]["e"] == 0.0
    # with and without the degenerate points
    n_deg0 = sum(k != "regular" for k in kinds[0])
    assert outs[0]["inliers"] == outs[3]["inliers"] + n_deg0
    for k in ("H", "b"):
        assert np.array_equal(outs[0][k], outs[3][k]), k
    assert outs[0]["e"] == outs[3]["e"]
    fd = fd_hessian_factor(*w.sources[3], vm, w.poses[0], w.poses[1])
    assert rel_err(outs[0]["H"], fd["H"]) < 1e-7 and rel_err(outs[0]["b"], fd["b"]) < 1e-7
    assert abs(outs[0]["e"] - fd["e"]) <= 1e-10 * abs(fd["e"])
    # exact 90 degree turn, every kind
    reg1 = np.array([k == "regular" for k in kinds[1]])
    x1, c1 = w.sources[1]
    alone = oracle.linearize_factor(x1[reg1], c1[reg1], vm, w.poses[2], w.poses[3])
    assert outs[1]["inliers"] == alone["inliers"] + int((~reg1).sum())
    for k in ("H", "b"):
        assert np.array_equal(outs[1][k], alone[k]), k
    assert outs[1]["e"] == alone["e"]
    return outs
