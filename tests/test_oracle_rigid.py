"""CPU: pins of the oracle's rigid-pose front end (oracle/rigid.py, Sec. 4.5).

* pairs against a pure-Python double loop in float64 (pairs away from the
  threshold), row order, each difference the single rounding of the exact one;
* noise-free rigid motion: every inlier pair passes a tight length check;
  swapping x and y keeps the same pairs; a permutation of the correspondences
  maps the pair set;
* R(q) against scipy's rotation matrix; orthonormality;
* the translation vote against a Counter over cells computed in float64 on
  candidates placed away from cell faces, with planted ties;
* exact motion: with the true rotation every inlier votes for the true cell;
* empty, single, coincident and out-of-domain inputs;
* a synthetic 6-DoF scene end to end (Sec. 5.4.1);
* planted mistakes in the pairs and the translation, each caught.
"""
import collections
import math

import numpy as np
import pytest

import oracle
from oracle import rigid as RG
from paper_2506_11547_amd import datagen

F = np.float32


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


# ---------------------------------------------------------------- pairs

def brute_pairs(x, y, mu, margin):
    """float64 double loop; returns (kept set, set of pairs within margin of mu)."""
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    n = x.shape[1]
    kept, near = set(), set()
    for i in range(n):
        for j in range(i + 1, n):
            lm = math.sqrt(sum((x[c, i] - x[c, j]) ** 2 for c in range(3)))
            ln = math.sqrt(sum((y[c, i] - y[c, j]) ** 2 for c in range(3)))
            d = abs(lm - ln)
            if abs(d - mu) < margin or lm < margin or ln < margin:
                near.add((i, j))
            elif d <= mu:
                kept.add((i, j))
    return kept, near


def check_pairs(pairs_fn, x, y, mu):
    m, n, pi, pj = pairs_fn(x, y, mu)
    got = list(zip(pi.tolist(), pj.tolist()))
    assert got == sorted(got) and all(i < j for i, j in got)          # row order
    kept, near = brute_pairs(x, y, mu, 1e-5)
    assert set(got) - near == kept
    # each difference is the single rounding of the exact one
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    assert np.array_equal(m, (x64[:, pi] - x64[:, pj]).astype(F))
    assert np.array_equal(n, (y64[:, pi] - y64[:, pj]).astype(F))
    return got


def test_pairs_brute_force():
    inst = datagen.make_rigid_instance(60, 0.5, 0.01, 11)
    got = check_pairs(RG.pairs, inst.x, inst.y, 0.05)
    assert 30 < len(got) < 60 * 59 // 2


def test_pairs_noise_free_inliers_all_kept():
    inst = datagen.make_rigid_instance(80, 0.5, 0.0, 12)
    _, _, pi, pj = RG.pairs(inst.x, inst.y, 1e-5)
    got = set(zip(pi.tolist(), pj.tolist()))
    idx = np.nonzero(inst.inlier)[0]
    want = {(int(a), int(b)) for k, a in enumerate(idx) for b in idx[k + 1:]}
    assert want <= got
    assert len(got - want) <= 3      # an outlier pair passes 1e-5 only by chance


def test_pairs_swap_and_permutation():
    inst = datagen.make_rigid_instance(70, 0.6, 0.01, 13)
    m, n, pi, pj = RG.pairs(inst.x, inst.y, 0.04)
    m2, n2, qi, qj = RG.pairs(inst.y, inst.x, 0.04)
    assert np.array_equal(pi, qi) and np.array_equal(pj, qj)
    assert np.array_equal(m, n2) and np.array_equal(n, m2)
    p = np.random.default_rng(1).permutation(inst.n)
    _, _, ri, rj = RG.pairs(inst.x[:, p], inst.y[:, p], 0.04)
    mapped = {tuple(sorted((int(p[a]), int(p[b])))) for a, b in zip(ri, rj)}
    assert mapped == set(zip(pi.tolist(), pj.tolist()))


def test_pairs_degenerate():
    z = np.zeros((3, 0), F)
    assert RG.pairs(z, z, 0.1)[0].shape == (3, 0)
    one = np.ones((3, 1), F)
    assert RG.pairs(one, one, 0.1)[2].size == 0
    same = np.ones((3, 5), F)            # coincident points: zero differences
    assert RG.pairs(same, same, 0.1)[2].size == 0
    bad = np.array([[0, 1, np.nan], [0, 0, 0], [0, 0, 0]], F)
    _, _, pi, pj = RG.pairs(bad, bad, 0.1)
    assert list(zip(pi, pj)) == [(0, 1)]


# ---------------------------------------------------------------- rotation matrix

def test_rotation_matrix_against_scipy():
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(3)
    for _ in range(200):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R = RG.rotation_matrix(q.astype(F)).astype(np.float64)
        S = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert np.max(np.abs(R - S)) < 2e-6
        assert np.max(np.abs(R @ R.T - np.eye(3))) < 2e-6
    assert np.array_equal(RG.rotation_matrix(F([1, 0, 0, 0])), np.eye(3, dtype=F))


# ---------------------------------------------------------------- translation

T_MIN, STEP, NC = -5.0, 0.025, 400


def planted_candidates(seed):
    """x random, q = identity (R = I exactly), y = x + t with t placed at
    cell coordinates c + 0.5 + U(-0.3, 0.3): clusters of 40, 40 (a tie),
    15 and 60 scattered candidates."""
    rng = np.random.default_rng(seed)
    cl = [np.array([10, 200, 300]), np.array([9, 200, 300]), np.array([50, 60, 70])]
    sizes = [40, 40, 15]
    cs = [np.repeat(c[None, :], s, axis=0) for c, s in zip(cl, sizes)]
    cs.append(rng.integers(0, NC, size=(60, 3)))
    c = np.concatenate(cs)
    u = c + 0.5 + rng.uniform(-0.3, 0.3, size=c.shape)
    t = T_MIN + u * STEP
    x = rng.uniform(-1, 1, size=c.shape)
    perm = rng.permutation(len(c))
    return (np.ascontiguousarray(x[perm].T.astype(F)),
            np.ascontiguousarray((x + t)[perm].T.astype(F)))


def check_translation(translation_fn, x, y, q, tau):
    r = translation_fn(x, y, F(q), T_MIN, STEP, NC, tau)
    # float64 cells and a Counter, for candidates away from every cell face
    R = datagen.quat_to_matrix(np.float64(F(q)))
    t = y.astype(np.float64) - R @ x.astype(np.float64)
    u = (t - T_MIN) / STEP
    near = np.any(np.abs(u - np.round(u)) <= 1e-3, axis=0)
    inside = np.all((u >= 0) & (u < NC), axis=0) & ~near
    c = np.floor(u[:, inside]).astype(np.int64)
    cnt = collections.Counter(((c[2] * NC + c[1]) * NC + c[0]).tolist())
    best = max(cnt.values())
    key = min(k for k, v in cnt.items() if v == best)
    if not near.any():
        assert r["votes"] == best and r["key"] == key
    else:   # candidates on a cell face may fall either way
        second = max([v for k, v in cnt.items() if k != key], default=0)
        assert best <= r["votes"] <= best + int(near.sum())
        assert second + int(near.sum()) < best and r["key"] == key
    cc = np.array([key % NC, (key // NC) % NC, key // (NC * NC)])
    assert np.max(np.abs(r["t"] - (T_MIN + (cc + 0.5) * STEP))) < 1e-6
    d = np.linalg.norm(t - r["t"].astype(np.float64)[:, None], axis=0)
    far = np.abs(d - tau) > 1e-5
    assert np.array_equal(r["mask"][far], (d <= tau)[far])
    assert r["inliers"] == int(r["mask"].sum())
    return r


def test_translation_vote_against_counter():
    x, y = planted_candidates(4)
    r = check_translation(RG.translation, x, y, [1, 0, 0, 0], 0.02)
    assert r["votes"] == 40                              # the tie went to the lower key
    assert r["key"] == (300 * NC + 200) * NC + 9


def test_translation_exact_motion():
    inst = datagen.make_rigid_instance(300, 0.6, 0.0, 21)
    u = (inst.t_gt - T_MIN) / STEP
    assert np.all(np.abs(u - np.round(u)) > 1e-3)        # t_gt away from cell faces
    q = F(inst.q_gt)
    r = RG.translation(inst.x, inst.y, q, T_MIN, STEP, NC, 0.03)
    assert r["votes"] >= int(inst.inlier.sum())
    assert np.max(np.abs(r["t"] - inst.t_gt)) <= STEP / 2 + 1e-6
    assert np.all(r["mask"][inst.inlier])
    assert r["inliers"] <= int(inst.inlier.sum()) + 2
    check_translation(RG.translation, inst.x, inst.y, q, 0.03)


def test_translation_degenerate():
    x = np.zeros((3, 4), F)
    y = np.full((3, 4), 7.0, F)                          # every candidate outside [-5, 5)
    r = RG.translation(x, y, F([1, 0, 0, 0]), T_MIN, STEP, NC, 0.1)
    assert r["votes"] == 0 and r["inliers"] == 0 and not r["mask"].any()
    assert np.array_equal(r["t"], np.zeros(3, F))
    y[0, 2] = np.nan
    y[:, 3] = 0.0
    r = RG.translation(x, y, F([1, 0, 0, 0]), T_MIN, STEP, NC, 0.1)
    assert r["votes"] == 1 and r["mask"].tolist() == [False, False, False, True]


# ---------------------------------------------------------------- end to end

def test_rigid_scene_end_to_end(orc):
    inst = datagen.make_rigid_instance(400, 0.7, 0.01, 5)
    eps = float(F(math.radians(3.0)))
    r = RG.solve_rigid(orc, inst.x, inst.y, 0.05, 64, 512, eps, 16, 8, T_MIN, STEP, NC, 0.06,
                       nthreads=oracle.threads())
    assert r["pairs"] > 0
    assert datagen.rotation_error_deg(np.float64(r["q"]), inst.q_gt) < 1.0
    assert np.linalg.norm(np.float64(r["t"]) - inst.t_gt) < 0.04
    tp = int((r["mask"] & inst.inlier).sum())
    assert tp >= 0.9 * inst.inlier.sum() and tp >= 0.9 * r["inliers"]
    # the pairs' inlier set is mostly pairs of two true inliers
    both = inst.inlier[r["pair_i"]] & inst.inlier[r["pair_j"]]
    assert (both[r["rot_mask"]]).mean() > 0.9


# ---------------------------------------------------------------- planted mistakes

def pairs_both_orders(x, y, mu):
    m, n, pi, pj = RG.pairs(x, y, mu)
    k = np.lexsort((np.concatenate([pj, pi]), np.concatenate([pi, pj])))
    return (np.concatenate([m, -m], axis=1)[:, k], np.concatenate([n, -n], axis=1)[:, k],
            np.concatenate([pi, pj])[k], np.concatenate([pj, pi])[k])


def pairs_squared_lengths(x, y, mu):
    x = np.asarray(x, F)
    y = np.asarray(y, F)
    out = [[], [], [], []]
    for i in range(x.shape[1] - 1):
        m = x[:, i:i + 1] - x[:, i + 1:]
        d = y[:, i:i + 1] - y[:, i + 1:]
        lm2 = (m[0] * m[0] + m[1] * m[1]) + m[2] * m[2]
        ln2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        k = np.nonzero((lm2 > 0) & (ln2 > 0) & (np.abs(lm2 - ln2) <= F(mu)))[0]
        out[0].append(m[:, k])
        out[1].append(d[:, k])
        out[2].append(np.full(len(k), i, np.int32))
        out[3].append((k + i + 1).astype(np.int32))
    return (np.concatenate(out[0], axis=1), np.concatenate(out[1], axis=1),
            np.concatenate(out[2]), np.concatenate(out[3]))


def translation_plus(x, y, q, t_min, step, nc, tau):
    """t = y + R x."""
    return RG.translation(x, -np.asarray(y), q, t_min, step, nc, tau) | {}


def translation_transposed(x, y, q, t_min, step, nc, tau):
    """R^T instead of R (the conjugate quaternion)."""
    qc = np.asarray(q, F).copy()
    qc[1:] = -qc[1:]
    return RG.translation(x, y, qc, t_min, step, nc, tau)


def translation_high_tie(x, y, q, t_min, step, nc, tau):
    t = RG.candidates(x, y, RG.rotation_matrix(q))
    key = RG.cells(t, t_min, step, nc)
    ks, cnt = np.unique(key[key >= 0], return_counts=True)
    best = len(cnt) - 1 - int(np.argmax(cnt[::-1]))     # ties to the highest key
    r = RG.translation(x, y, q, t_min, step, nc, tau)
    r.update(key=int(ks[best]), votes=int(cnt[best]), t=RG.centre(int(ks[best]), t_min, step, nc))
    return r


def translation_corner(x, y, q, t_min, step, nc, tau):
    """The cell's lower corner instead of its centre."""
    r = RG.translation(x, y, q, t_min, step, nc, tau)
    r["t"] = r["t"] - F(0.5) * F(step)
    return r


@pytest.mark.parametrize("mutant", [pairs_both_orders, pairs_squared_lengths])
def test_planted_pair_mistakes_are_caught(mutant):
    inst = datagen.make_rigid_instance(60, 0.5, 0.01, 11)
    with pytest.raises(AssertionError):
        check_pairs(mutant, inst.x, inst.y, 0.05)


@pytest.mark.parametrize("mutant", [translation_plus, translation_transposed, translation_high_tie,
                                    translation_corner])
def test_planted_translation_mistakes_are_caught(mutant):
    x, y = planted_candidates(4)
    inst = datagen.make_rigid_instance(300, 0.6, 0.0, 21)
    caught = 0
    for xx, yy, q in ((x, y, [1, 0, 0, 0]), (inst.x, inst.y, inst.q_gt)):
        try:
            r = check_translation(mutant, xx, yy, q, 0.03)
            if q is not inst.q_gt:
                assert r["votes"] == 40 and r["key"] == (300 * NC + 200) * NC + 9
            else:
                assert r["votes"] >= int(inst.inlier.sum())
        except AssertionError:
            caught += 1
    assert caught > 0
