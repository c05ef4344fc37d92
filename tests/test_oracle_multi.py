"""CPU: pins of the oracle's multiple-rotation extraction (oracle/multi.py).

* one model is the single solve's winner (the paper's variant reduces to Alg. 1);
* a hand-built candidate set with overlapping inlier sets and known angles
  against the selection rule worked out by hand;
* several rotations in one scene (the paper's multiple-rotation experiment,
  synthetic): every rotation found within the quantisation bound, the labels
  agree with the ground-truth models;
* relabelling under a permutation of the correspondences;
* planted mistakes in the selection, each caught.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import multi as MM
from paper_2506_11547_amd import datagen


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def qz(angle):
    """Unit quaternion of a rotation about z."""
    return np.float32([math.cos(angle / 2), 0.0, 0.0, math.sin(angle / 2)])


def test_one_model_is_the_solve_winner(orc):
    w, inst = datagen.make_workload("small")
    eps = float(np.float32(math.radians(w.eps_deg)))
    r = MM.solve_multi(orc, inst.x, inst.y, w.grid, w.samples, eps, w.topk, 1, 0.1, 1)
    o = r["solve"]
    assert len(r["models"]) == 1
    m = r["models"][0]
    assert m["cand"] == o["winner"] and m["count"] == o["count"]
    assert np.array_equal(m["q"].view(np.uint32), o["q"].view(np.uint32))
    assert np.array_equal(r["labels"] == 1, o["mask"].astype(bool))


def hand_built():
    """Five candidates with known angles about z and overlapping inlier sets."""
    n = 19
    S = np.zeros((5, n), bool)
    S[0, [0, 1, 2, 3, 4, 5, 14, 15]] = True            # 8
    S[1, [0, 1, 2, 11, 12]] = True                     # 5, 3 deg from candidate 0
    S[2, [6, 7, 8, 9]] = True                          # 4
    S[3, [4, 5, 6, 7, 8, 9, 10, 16, 17, 18]] = True    # 10
    S[4, [10, 13]] = True                              # 2
    qs = [qz(math.radians(a)) for a in (40.0, 43.0, 120.0, 200.0, 300.0)]
    return qs, list(S), n


def test_hand_built_selection():
    qs, S, n = hand_built()
    models, labels = MM.select(qs, S, n, 5, math.radians(5.0), 2)
    # pick 1: candidate 3 (10); nothing else within 5 deg of it
    # pick 2: unclaimed 0:{0,1,2,3,14,15}=6, 1:{0,1,2,11,12}=5, 2:0, 4:{13}=1 -> 0;
    #         candidate 1 (3 deg away) is suppressed with it
    # pick 3: 2:0, 4:1 < min_inliers 2 -> stop
    assert [m["cand"] for m in models] == [3, 0]
    assert [m["count"] for m in models] == [10, 6]
    assert labels.tolist() == [2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 2, 2, 1, 1, 1]
    # zero separation: candidate 1 stays eligible and takes {11, 12}; then {13}
    models, labels = MM.select(qs, S, n, 5, 0.0, 1)
    assert [m["cand"] for m in models] == [3, 0, 1, 4]
    assert [m["count"] for m in models] == [10, 6, 2, 1]
    # the model cap
    models, _ = MM.select(qs, S, n, 1, 0.0, 1)
    assert [m["cand"] for m in models] == [3]


@pytest.mark.parametrize("models,per_model", [(2, 1000), (3, 1000), (4, 2000)])
def test_several_rotations_in_one_scene(orc, models, per_model):
    inst = datagen.make_multi_instance(models, per_model, per_model // 2, 0.01, 100 + models)
    G, J, K = 64, 540, 64
    eps = float(np.float32(math.radians(2.0)))
    r = MM.solve_multi(orc, inst.x, inst.y, G, J, eps, K, models + 2, math.radians(10.0), 50,
                       nthreads=oracle.threads())
    found = r["models"]
    assert len(found) == models
    bound = math.degrees(4 * math.sqrt(3) / G) + 2.0
    used = set()
    for mi, m in enumerate(found):
        errs = [datagen.rotation_error_deg(m["q"].astype(np.float64), q) for q in inst.q_gt]
        j = int(np.argmin(errs))
        assert errs[j] < bound and j not in used
        used.add(j)
        lab = r["labels"] == (mi + 1)
        # most of the label set is that model's inliers
        assert (inst.model[lab] == j).mean() > 0.95


def test_permutation_relabels(orc):
    inst = datagen.make_multi_instance(2, 600, 200, 0.01, 5)
    eps = float(np.float32(math.radians(2.0)))
    a = MM.solve_multi(orc, inst.x, inst.y, 48, 384, eps, 32, 4, math.radians(10.0), 20)
    p = np.random.default_rng(0).permutation(inst.x.shape[1])
    b = MM.solve_multi(orc, inst.x[:, p], inst.y[:, p], 48, 384, eps, 32, 4, math.radians(10.0), 20)
    assert [(m["cand"], m["count"]) for m in a["models"]] == \
        [(m["cand"], m["count"]) for m in b["models"]]
    assert np.array_equal(a["labels"][p], b["labels"])


def _select_total_counts(qs, sets, n, max_models, sep_rad, min_inliers):
    """Mistake: total instead of exclusive counts, no suppression."""
    order = sorted(range(len(qs)), key=lambda k: (-int(sets[k].sum()), k))
    labels = np.zeros(n, np.uint8)
    models = []
    for m, k in enumerate(order[:max_models]):
        if int(sets[k].sum()) < min_inliers:
            break
        labels[sets[k] & (labels == 0)] = m + 1
        models.append(dict(q=np.asarray(qs[k], np.float32), count=int(sets[k].sum()), cand=k))
    return models, labels


def _select_no_suppression(qs, sets, n, max_models, sep_rad, min_inliers):
    """Mistake: exclusive counts but no suppression of nearby candidates."""
    claimed = np.zeros(n, bool)
    labels = np.zeros(n, np.uint8)
    taken = set()
    models = []
    for m in range(max_models):
        cnt = [(-1 if k in taken else int((sets[k] & ~claimed).sum())) for k in range(len(qs))]
        best = int(np.argmax(cnt))
        if cnt[best] < min_inliers:
            break
        labels[sets[best] & ~claimed] = m + 1
        claimed |= sets[best]
        taken.add(best)
        models.append(dict(q=np.asarray(qs[best], np.float32), count=cnt[best], cand=best))
    return models, labels


@pytest.mark.parametrize("mutant", [_select_total_counts, _select_no_suppression])
def test_planted_mistakes_are_caught(mutant):
    qs, S, n = hand_built()
    models, labels = mutant(qs, S, n, 5, math.radians(5.0), 2)
    assert [m["cand"] for m in models] != [3, 0] or \
        labels.tolist() != [2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0, 2, 2, 1, 1, 1]
