"""Several rotations from one vote (the paper's multiple-rotation variant:
Alg. 1 returning several high peaks instead of one; Sec. 4.4's multiple
rotation motions, whose inlier circles meet in one cluster point each).

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the product
path.  Written from the paper plus the readings below; uses the C oracle for
the vote, the candidates, their decode and the rule's rescoring.

Readings (the paper says only "return multiple possible high peaks"):
* candidates are the solve's K best cells (count desc, index asc), decoded to
  their centres, each with its exact inlier set (|L_i q|^2 <= T2);
* models are picked greedily: the candidate with the most inliers not yet
  claimed by an earlier model (ties to the earlier candidate) becomes the next
  model if that number reaches min_inliers; its unclaimed inliers are
  labelled with it;
* a picked model suppresses every candidate that is the same rotation to
  within sep: |q_a . q_b| >= f32(cos(sep / 2)) (rotation angle <= sep), the
  dot product in float32 as ((a_w b_w + a_x b_x) + a_y b_y) + a_z b_z;
* at most max_models models; labels are 0 for unclaimed correspondences and
  m + 1 for model m.
"""
from __future__ import annotations

import math

import numpy as np


def sep_cos(sep_rad: float) -> np.float32:
    return np.float32(math.cos(0.5 * float(sep_rad)))


def dot32(a, b) -> np.float32:
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    s = a[0] * b[0]
    s = np.float32(s + a[1] * b[1])
    s = np.float32(s + a[2] * b[2])
    s = np.float32(s + a[3] * b[3])
    return s


def candidates(orc, x, y, G: int, J: int, eps_rad: float, K: int, nthreads: int = 1):
    """The solve's candidates: cell indices, votes, decoded centres and inlier sets."""
    o = orc.solve(x, y, G, J, eps_rad, K, nthreads=nthreads)
    T2 = orc.residual_bound(eps_rad)
    qs, sets = [], []
    for idx in o["top_idx"]:
        q = orc.decode(int(idx), G)
        qs.append(q)
        sets.append(orc.rescore(x, y, q, T2, want_mask=True)[1].astype(bool))
    return o, qs, sets


def select(qs, sets, n: int, max_models: int, sep_rad: float, min_inliers: int):
    """Greedy exclusive selection over candidates (qs, inlier sets)."""
    C = sep_cos(sep_rad)
    K = len(qs)
    claimed = np.zeros(n, bool)
    labels = np.zeros(n, np.uint8)
    suppressed = np.zeros(K, bool)
    models = []
    for m in range(max_models):
        best, best_cnt = -1, -1
        for k in range(K):
            if suppressed[k]:
                continue
            c = int((sets[k] & ~claimed).sum())
            if c > best_cnt:
                best, best_cnt = k, c
        if best < 0 or best_cnt < min_inliers:
            break
        new = sets[best] & ~claimed
        labels[new] = m + 1
        claimed |= new
        models.append(dict(q=np.asarray(qs[best], np.float32), count=best_cnt, cand=best))
        for k in range(K):
            if k == best or abs(dot32(qs[k], qs[best])) >= C:
                suppressed[k] = True
    return models, labels


def solve_multi(orc, x, y, G: int, J: int, eps_rad: float, K: int, max_models: int,
                sep_rad: float, min_inliers: int, nthreads: int = 1) -> dict:
    o, qs, sets = candidates(orc, x, y, G, J, eps_rad, K, nthreads)
    models, labels = select(qs, sets, x.shape[1], max_models, sep_rad, min_inliers)
    return dict(models=models, labels=labels, solve=o, cand_q=qs)
