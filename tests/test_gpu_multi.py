"""GPU: several rotations from one vote (rot_vote_solve_multi) against the
oracle (oracle/multi.py), bit for bit: the candidates, the chosen models
(candidate, claimed count, rotation bits) and every label."""
import math

import numpy as np
import pytest

import oracle
from oracle import multi as MM
from paper_2506_11547_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rv():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2506_11547_amd import rotvote
    return rotvote


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_both(rv, orc, x, y, G, J, eps_deg, K, M, sep_deg, min_inl, strategy="auto"):
    with rv.Solver(max_n=max(1, x.shape[1]), max_grid=G, topk=K, samples_per_circle=J,
                   strategy=strategy) as s:
        q, cnt, lab = s.solve_multi(dev(x), dev(y), G, eps_deg, M, sep_deg, min_inl)
        top = s.topk()
        lab = lab.cpu().numpy()
    eps = rv.eps_deg_to_rad(eps_deg)
    r = MM.solve_multi(orc, x, y, G, J, eps, K, M, float(np.float32(math.radians(sep_deg))),
                       min_inl, nthreads=oracle.threads())
    return q, cnt, lab, top, r


def check(q, cnt, lab, top, r):
    o = r["solve"]
    assert top["idx"] == o["top_idx"].tolist()
    assert top["votes"] == o["top_counts"].tolist()
    assert top["inliers"] == o["cand_counts"].tolist()
    models = r["models"]
    assert len(q) == len(models)
    for k, m in enumerate(models):
        assert np.array_equal(np.float32(q[k]).view(np.uint32), m["q"].view(np.uint32)), k
        assert cnt[k] == m["count"], k
    if models:
        assert top["winner"] == models[0]["cand"]
    assert np.array_equal(lab, r["labels"])


@pytest.mark.parametrize("models,per_model,G,J", [(2, 1000, 64, 540), (3, 1500, 64, 540),
                                                  (5, 1000, 96, 540), (9, 1000, 128, 540),
                                                  (4, 1000, 200, 540), (3, 1000, 300, 540)])
def test_scene_with_several_rotations(rv, orc, models, per_model, G, J):
    inst = datagen.make_multi_instance(models, per_model, per_model, 0.01, 200 + models)
    q, cnt, lab, top, r = run_both(rv, orc, inst.x, inst.y, G, J, 2.0, 64, models + 3, 10.0, 50)
    check(q, cnt, lab, top, r)
    # every rotation of the scene is found (within the quantisation bound)
    bound = math.degrees(4 * math.sqrt(3) / G) + 2.0
    for qg in inst.q_gt:
        assert min(datagen.rotation_error_deg(np.array(qm), qg) for qm in q) < bound


def test_one_model_equals_single_solve(rv, orc):
    w, inst = datagen.make_workload("small")
    q, cnt, lab, top, r = run_both(rv, orc, inst.x, inst.y, w.grid, w.samples, w.eps_deg, w.topk,
                                   1, 5.0, 1)
    check(q, cnt, lab, top, r)
    with rv.Solver(max_n=inst.n, max_grid=w.grid, topk=w.topk, samples_per_circle=w.samples) as s:
        q1, c1, m1 = s.solve(dev(inst.x), dev(inst.y), w.grid, w.eps_deg)
    assert q[0] == q1 and cnt[0] == c1
    assert np.array_equal(lab == 1, m1.cpu().numpy())


@pytest.mark.parametrize("sep,min_inl,M", [(0.0, 1, 16), (180.0, 1, 16), (10.0, 10**9, 4),
                                           (3.0, 5, 64)])
def test_selection_parameters(rv, orc, sep, min_inl, M):
    inst = datagen.make_multi_instance(3, 800, 400, 0.01, 9)
    q, cnt, lab, top, r = run_both(rv, orc, inst.x, inst.y, 48, 384, 2.0, 64, M, sep, min_inl)
    check(q, cnt, lab, top, r)
    if sep == 180.0:
        assert len(q) == 1
    if min_inl == 10**9:
        assert len(q) == 0 and not lab.any()


@pytest.mark.parametrize("strategy", ["global", "brick"])
def test_strategies_and_degenerate_inputs(rv, orc, strategy):
    inst = datagen.make_multi_instance(2, 500, 300, 0.01, 21)
    x, y = inst.x.copy(), inst.y.copy()
    x[:, :40] = 0
    y[2, 40:50] = np.inf
    q, cnt, lab, top, r = run_both(rv, orc, x, y, 80, 320, 2.0, 32, 6, 10.0, 20, strategy)
    check(q, cnt, lab, top, r)


def test_empty_and_unusable(rv):
    with rv.Solver(max_n=64, max_grid=16, topk=8) as s:
        e = torch.empty(3, 0, dtype=torch.float32, device="cuda")
        assert s.solve_multi(e, e, 16, 1.0, 4, 5.0, 1)[:2] == ([], [])
        z = torch.zeros(3, 64, dtype=torch.float32, device="cuda")
        q, c, lab = s.solve_multi(z, z, 16, 1.0, 4, 5.0, 1)
        assert q == [] and c == [] and not lab.cpu().numpy().any()


def test_multi_error_conventions(rv):
    with rv.Solver(max_n=100, max_grid=16, topk=8) as s:
        x = torch.randn(3, 50, device="cuda")
        lab = torch.empty(50, dtype=torch.uint8, device="cuda")
        for M, sep, mi in [(0, 0.1, 1), (9, 0.1, 1), (2, -0.1, 1), (2, 3.2, 1), (2, 0.1, 0)]:
            with pytest.raises(rv.RotVoteError) as e:
                s.solve_multi_raw(x.data_ptr(), x.data_ptr(), 50, 16, 0.01, M, sep, mi,
                                  lab.data_ptr())
            assert e.value.status == rv.RV_EINVAL
