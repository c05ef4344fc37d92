"""Least-squares rotation on an inlier set (Sec. 4.2, the stacked system Q q = 0).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's CPU
leg, never by the product path.  float64 numpy, written from the paper:

* Lemma (Sec. 4.2): q lies on correspondence i's circle iff q is orthogonal
  to q_{i,b3} and q_{i,b4}, the two unit normals of the hyperplanes whose
  intersection with S^3 is the circle.  Stacking [q_{i,b3}, q_{i,b4}]^T over
  the inliers gives Q (2m x 4); the least-squares rotation is the eigenvector
  of Q^T Q with the smallest eigenvalue.
* q_{i,b3}, q_{i,b4} are an orthonormal basis of the orthogonal complement of
  the circle's plane, which is the -1 eigenspace of M_i (App. A: eigenvalues
  (1, 1, -1, -1), the circle spans the +1 eigenspace).  The Gram sum
  q_b3 q_b3^T + q_b4 q_b4^T of an orthonormal basis is the orthogonal
  projector onto the subspace, here (I - M_i) / 2, whatever basis is chosen;
  so Q^T Q = sum_i (I - M_i) / 2.
* M_i is written out from q^T M q = b^T R(q) a (App. A):
  M_00 = a.b, M_0k = M_k0 = (a x b)_m, M_kk = 2 a_m b_m - a.b,
  M_kl = a_m b_n + a_n b_m (k = m + 1, l = n + 1, m != n).

Readings (where the paper is silent): the unit vectors are the rule's step 1
(the oracle's float32 normalisation, as the vote uses); the eigenvector's sign
is canonicalised like a vote sample (w >= 0, ties by the first nonzero
component); the system is ill-posed, and the input rotation is kept, when the
two smallest eigenvalues of Q^T Q are within 1e-6 * max(1, m) of each other
(one correspondence, or all of them parallel); the refined rotation is the
float64 eigenvector rounded to float32 per component; the refined inlier set
is the rule's rescoring (|L_i q|^2 <= T2 in float32) of the refined rotation.
"""
from __future__ import annotations

import numpy as np

GAP_REL = 1e-6


def m_matrices(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """M_i (App. A) for unit a, b given as float64 [3, m] arrays: [m, 4, 4]."""
    m = a.shape[1]
    dot = a[0] * b[0] + a[1] * b[1] + a[2] * b[2]
    cr = np.stack([a[1] * b[2] - a[2] * b[1],
                   a[2] * b[0] - a[0] * b[2],
                   a[0] * b[1] - a[1] * b[0]])
    M = np.zeros((m, 4, 4))
    M[:, 0, 0] = dot
    for k in range(3):
        M[:, 0, k + 1] = M[:, k + 1, 0] = cr[k]
        M[:, k + 1, k + 1] = 2.0 * a[k] * b[k] - dot
        for l in range(k + 1, 3):
            M[:, k + 1, l + 1] = M[:, l + 1, k + 1] = a[k] * b[l] + a[l] * b[k]
    return M


def qtq(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Q^T Q = sum_i (I - M_i) / 2 over the given unit pairs (float64 [3, m])."""
    M = m_matrices(a, b)
    return (a.shape[1] * np.eye(4) - M.sum(axis=0)) / 2.0


def canonical(q: np.ndarray) -> np.ndarray:
    q = np.asarray(q, np.float64)
    for c in q:
        if c != 0.0:
            return q if c > 0.0 else -q
    return q


def solve_qtq(A: np.ndarray, m: int):
    """Smallest-eigenvalue eigenvector of Q^T Q (canonical sign), or None when
    the two smallest eigenvalues are within GAP_REL * max(1, m)."""
    w, V = np.linalg.eigh(A)
    if m == 0 or w[1] - w[0] <= GAP_REL * max(1.0, float(m)):
        return None
    return canonical(V[:, 0])


def refine_once(orc, x, y, mask):
    """One least-squares solve on the correspondences with mask[i] set.
    Returns (q64 or None, m) with m the number of usable masked pairs."""
    a, b, ok = orc.normalise_pairs(x, y)
    use = ok & (np.asarray(mask) != 0)
    a64 = a[:, use].astype(np.float64)
    b64 = b[:, use].astype(np.float64)
    m = int(use.sum())
    if m == 0:
        return None, 0
    return solve_qtq(qtq(a64, b64), m), m


def refine(orc, x, y, eps_rad: float, mask, q_in, iterations: int = 1) -> dict:
    """`iterations` rounds of: least squares on the current inlier set, then
    rescoring of the refined rotation (which gives the next inlier set).
    A round whose system is ill-posed keeps the current rotation."""
    T2 = orc.residual_bound(eps_rad)
    q = np.asarray(q_in, np.float32).copy()
    mask = np.asarray(mask).astype(np.uint8)
    count = int(mask.sum())
    q64 = None
    for _ in range(iterations):
        q64, _m = refine_once(orc, x, y, mask)
        if q64 is not None:
            q = q64.astype(np.float32)
        count, mask = orc.rescore(x, y, q, T2, want_mask=True)
    return dict(q=q, q64=q64, count=count, mask=mask)
