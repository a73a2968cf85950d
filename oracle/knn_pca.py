"""kNN-PCA surfel ellipsoids in FP64 (test infrastructure only).

The paper estimates each point's ellipsoid with a network (Section 3.2); its closest analytic
relatives are local-covariance splat shapes (Section 2.1) and CPU normal estimation
(Section 4.2). The renderer's plain path, its fallback and the judge of the learned estimator's
PSNR gap is this classical estimate:

1. neighbours: the k points nearest to p_i (the point itself included), ordered by
   (squared distance, index) so ties break by index;
2. mu = mean of the neighbours; C = (1/k) sum (p_j - mu)(p_j - mu)^T;
3. eigen-decomposition C = E diag(l1 >= l2 >= l3) E^T;
4. scales s1 = kappa sqrt(l1), s2 = kappa sqrt(l2), s3 = max(kappa sqrt(l3), floor * s2);
5. normal n = the eigenvector of l3, oriented so n . (p_i - cloud centroid) >= 0;
6. rotation R = [e1 e2 n] (columns), with e2 negated if det R < 0; quaternion (w,x,y,z) of R
   with w >= 0.

Step 1 uses exact brute force for small clouds and a k-d tree (a library primitive) followed by an
exact FP64 re-ranking for large ones. Step 3 uses ``numpy.linalg.eigh``.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation


def knn_bruteforce(points: np.ndarray, k: int = 16) -> np.ndarray:
    """O(N^2) exact kNN, ties by index. points (3, n); returns (n, k) int64."""
    p = np.asarray(points, np.float64).T
    n = p.shape[0]
    out = np.zeros((n, k), np.int64)
    idx = np.arange(n)
    for i in range(n):
        d2 = ((p - p[i]) ** 2).sum(axis=1)
        order = np.lexsort((idx, d2))
        out[i] = order[:k]
    return out


def knn(points: np.ndarray, k: int = 16, brute_max: int = 4000, workers: int = -1) -> np.ndarray:
    """Exact kNN with ties broken by index. points (3, n); returns (n, k) int64 and the squared
    distance gap between the k-th and (k+1)-th neighbour (for near-tie detection)."""
    p = np.ascontiguousarray(np.asarray(points, np.float64).T)
    n = p.shape[0]
    if n <= brute_max:
        nb = knn_bruteforce(points, min(k + 1, n))
        d2 = ((p[nb] - p[:, None, :]) ** 2).sum(axis=2)
        gap = d2[:, k] - d2[:, k - 1] if nb.shape[1] > k else np.full(n, np.inf)
        return nb[:, :k], gap
    tree = cKDTree(p)
    kk = min(n, 2 * k + 8)
    while True:
        _, cand = tree.query(p, k=kk, workers=workers)
        d2 = ((p[cand] - p[:, None, :]) ** 2).sum(axis=2)
        # the candidate set is complete when the (k+1)-th exact distance is below the largest one
        order = np.lexsort((cand, d2), axis=1)
        cand = np.take_along_axis(cand, order, axis=1)
        d2 = np.take_along_axis(d2, order, axis=1)
        ok = d2[:, k] < d2[:, -1] if kk > k + 1 else np.ones(n, bool)
        if ok.all() or kk >= n:
            gap = d2[:, k] - d2[:, k - 1]
            return cand[:, :k], gap
        kk = min(n, 2 * kk)


def knn_pca(points: np.ndarray, k: int = 16, kappa: float = 1.0, floor: float = 0.1,
            neighbours: np.ndarray | None = None) -> dict:
    """Surfel ellipsoids of every point: quat (4,n), scale (3,n), normal (3,n), cov (n,3,3) of the
    ellipsoid, and the neighbourhood eigenvalues (n,3) descending. FP64."""
    p = np.asarray(points, np.float64)
    n = p.shape[1]
    if neighbours is None:
        neighbours, _ = knn(p, k)
    P = p.T[neighbours]                                    # (n, k, 3)
    mu = P.mean(axis=1, keepdims=True)
    D = P - mu
    Cn = np.einsum("nki,nkj->nij", D, D) / k
    lam, vec = np.linalg.eigh(Cn)                          # ascending
    lam = lam[:, ::-1]
    vec = vec[:, :, ::-1]
    lam_c = np.clip(lam, 0.0, None)
    s1 = kappa * np.sqrt(lam_c[:, 0])
    s2 = kappa * np.sqrt(lam_c[:, 1])
    s3 = np.maximum(kappa * np.sqrt(lam_c[:, 2]), floor * s2)
    centroid = p.mean(axis=1)
    nrm = vec[:, :, 2].copy()
    flip = np.einsum("ni,ni->n", nrm, p.T - centroid) < 0
    nrm[flip] *= -1
    e1 = vec[:, :, 0]
    e2 = vec[:, :, 1].copy()
    R = np.stack([e1, e2, nrm], axis=2)                    # columns
    neg = np.linalg.det(R) < 0
    e2[neg] *= -1
    R = np.stack([e1, e2, nrm], axis=2)
    q_xyzw = Rotation.from_matrix(R).as_quat()
    q = np.stack([q_xyzw[:, 3], q_xyzw[:, 0], q_xyzw[:, 1], q_xyzw[:, 2]])
    q[:, q[0] < 0] *= -1
    scale = np.stack([s1, s2, s3])
    cov = np.einsum("nij,nj,nkj->nik", R, scale.T ** 2, R)
    return dict(quat=q, scale=scale, normal=nrm.T.copy(), cov=cov, eig=lam, neighbours=neighbours)
