"""Rigid pose (R, t) from point correspondences by pairwise decoupling
(Sec. 4.5: the pairwise constraint, the length check of Sec. 4.5.1 and the
translation vote of Sec. 4.5.2).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's CPU
leg, never by the product path.  Plain numpy in binary32 (numpy rounds every
float32 operation on its own and never fuses a multiply with an add), over the
C oracle's rotation solve and ``oracle/refine.py``.

What is computed, in the paper's order:

1. Pairs.  For two correspondences i != j of one rigid motion,
   R (x_i - x_j) = y_i - y_j: the differences m = x_i - x_j, n = y_i - y_j
   are a rotation-only correspondence.  (i, j) and (j, i) give (-m, -n), the
   same constraint, so the pairs are i < j, listed row by row (i ascending,
   then j ascending).
2. Length check.  A rotation keeps lengths, so a pair with
   | |m| - |n| | > mu is an outlier and is dropped; a pair with a zero
   difference constrains no rotation and is dropped as well.  Lengths are
   sqrt((c0*c0 + c1*c1) + c2*c2) in binary32.
3. Rotation.  The rotation vote (Alg. 1 with top-K rescoring) on the kept
   pairs, optionally followed by least-squares rounds (Sec. 4.2) on the pairs'
   inlier set.
4. Translation.  With R* fixed every correspondence gives a candidate
   t_i = y_i - R* x_i; the candidates vote in a grid of cubic cells over the
   domain [t_min, t_min + cells * step)^3 (Sec. 5.4.1: [-5, 5]^3, step 0.025),
   and t* is the centre of the cell holding the most candidates.
5. Inliers.  A correspondence is an inlier of (R*, t*) iff
   |t_i - t*| <= tau.

Readings where the paper is silent: R(q) is the homogeneous form of the
unit-quaternion rotation matrix, evaluated in binary32 in the order written in
``rotation_matrix``; (R x)_r = (R_r0*x0 + R_r1*x1) + R_r2*x2 and
t_r = y_r - (R x)_r; the cell of a candidate is floor((t_r - t_min) / step)
per axis (correctly rounded binary32 division), a candidate outside the domain
(or not finite) does not vote; cell index (c_z * cells + c_y) * cells + c_x;
ties between cells go to the lowest index; the centre is
t_min + ((float)c + 0.5) * step; the inlier test is
(e0*e0 + e1*e1) + e2*e2 <= f32(tau^2) with e = t_i - t* (tau the binary32
parameter, squared in binary64 and rounded once); with no vote at all,
t* = 0 and no correspondence is an inlier.
"""
from __future__ import annotations

import numpy as np

from . import refine as RF

F = np.float32


def pairs(x, y, mu: float):
    """Steps 1-2.  Returns (m [3, P], n [3, P], i [P], j [P]) in row order."""
    x = np.ascontiguousarray(x, F)
    y = np.ascontiguousarray(y, F)
    mu = F(mu)
    N = x.shape[1]
    ms, ns, ii, jj = [], [], [], []
    with np.errstate(over="ignore", invalid="ignore"):
        _pair_rows(x, y, mu, N, ms, ns, ii, jj)
    if not ms:
        z = np.zeros((3, 0), F)
        return z, z.copy(), np.zeros(0, np.int32), np.zeros(0, np.int32)
    return (np.ascontiguousarray(np.concatenate(ms, axis=1)),
            np.ascontiguousarray(np.concatenate(ns, axis=1)),
            np.concatenate(ii), np.concatenate(jj))


def pairs_of_row(x, y, mu, i: int):
    """Row i of steps 1-2: the kept j > i, with their m and n (binary32)."""
    m = x[:, i:i + 1] - x[:, i + 1:]
    d = y[:, i:i + 1] - y[:, i + 1:]
    lm = np.sqrt((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2])
    ln = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
    keep = (lm > 0) & (ln > 0) & (np.abs(lm - ln) <= mu)
    k = np.nonzero(keep)[0]
    return (k + i + 1).astype(np.int32), m[:, k], d[:, k]


def _pair_rows(x, y, mu, N, ms, ns, ii, jj):
    for i in range(N - 1):
        j, m, d = pairs_of_row(x, y, mu, i)
        if len(j):
            ms.append(m)
            ns.append(d)
            ii.append(np.full(len(j), i, np.int32))
            jj.append(j)


def rotation_matrix(q):
    """R(q) for a unit quaternion (w, x, y, z), binary32, homogeneous form."""
    w, x, y, z = (F(c) for c in q)
    ww, xx, yy, zz = w * w, x * x, y * y, z * z
    xy, xz, yz = x * y, x * z, y * z
    wx, wy, wz = w * x, w * y, w * z
    two = F(2)
    return np.array([
        [(ww + xx) - (yy + zz), two * (xy - wz), two * (xz + wy)],
        [two * (xy + wz), (ww + yy) - (xx + zz), two * (yz - wx)],
        [two * (xz - wy), two * (yz + wx), (ww + zz) - (xx + yy)],
    ], F)


def candidates(x, y, R):
    """t_i = y_i - R x_i, binary32 [3, N]."""
    x = np.ascontiguousarray(x, F)
    y = np.ascontiguousarray(y, F)
    R = np.asarray(R, F)
    t = np.empty_like(y)
    with np.errstate(over="ignore", invalid="ignore"):
        for r in range(3):
            rx = (R[r, 0] * x[0] + R[r, 1] * x[1]) + R[r, 2] * x[2]
            t[r] = y[r] - rx
    return t


def cells(t, t_min: float, step: float, ncell: int):
    """Cell index of every candidate, -1 outside the domain."""
    t_min, step = F(t_min), F(step)
    with np.errstate(invalid="ignore", over="ignore"):
        u = (t - t_min) / step
        ok = np.all((u >= 0) & (u < F(ncell)), axis=0)
    c = np.where(ok[None, :], np.floor(np.where(ok[None, :], u, 0)), 0).astype(np.int64)
    key = (c[2] * ncell + c[1]) * ncell + c[0]
    return np.where(ok, key, -1)


def centre(key: int, t_min: float, step: float, ncell: int):
    c = (key % ncell, (key // ncell) % ncell, key // (ncell * ncell))
    return np.array([F(t_min) + (F(ci) + F(0.5)) * F(step) for ci in c], F)


def translation(x, y, q, t_min: float, step: float, ncell: int, tau: float) -> dict:
    """Steps 4-5 for a given rotation q."""
    t = candidates(x, y, rotation_matrix(q))
    key = cells(t, t_min, step, ncell)
    valid = key[key >= 0]
    if len(valid) == 0:
        n = x.shape[1]
        return dict(t=np.zeros(3, F), votes=0, key=-1, inliers=0, mask=np.zeros(n, bool))
    ks, cnt = np.unique(valid, return_counts=True)
    best = int(np.argmax(cnt))           # first maximum: the lowest key among ties
    ts = centre(int(ks[best]), t_min, step, ncell)
    tf = float(F(tau))                   # the binary32 parameter, squared in binary64
    T2 = F(tf * tf)
    e = t - ts[:, None]
    with np.errstate(invalid="ignore", over="ignore"):
        d2 = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]
        mask = d2 <= T2
    return dict(t=ts, votes=int(cnt[best]), key=int(ks[best]), inliers=int(mask.sum()), mask=mask)


def solve_rigid(orc, x, y, mu: float, G: int, J: int, eps_rad: float, K: int, refine_rounds: int,
                t_min: float, step: float, ncell: int, tau: float, nthreads: int = 1) -> dict:
    """Steps 1-5.  refine_rounds least-squares rounds follow the vote (the
    result at a fixed point does not depend on further rounds)."""
    m, n, pi, pj = pairs(x, y, mu)
    P = m.shape[1]
    if P:
        s = orc.solve(m, n, G, J, eps_rad, K, nthreads)
        q, rot_count, rot_mask = s["q"], s["count"], s["mask"]
    else:
        s = None
        q, rot_count, rot_mask = np.float32([1, 0, 0, 0]), 0, np.zeros(0, bool)
    if refine_rounds and P:
        r = RF.refine(orc, m, n, eps_rad, rot_mask, q, iterations=refine_rounds)
        q, rot_count, rot_mask = r["q"], r["count"], r["mask"].astype(bool)
    tr = translation(x, y, q, t_min, step, ncell, tau)
    return dict(pairs=P, pair_i=pi, pair_j=pj, m=m, n=n, solve=s, q=np.asarray(q, F),
                rot_count=int(rot_count), rot_mask=rot_mask, **tr)
