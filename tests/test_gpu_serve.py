"""GPU: the request server (rot_vote_server_*).

Every result is identical alone and in the mix: a mixed burst of requests
(batchable small ones, large ones, three grids, some with refinement) goes
through a server with several workers and batching; each reply and mask must
equal, bit for bit, a standalone rot_vote_solve (+ rot_vote_refine) of the same
request, and the batched small ones the CPU oracle as well.  Then admission:
queue backpressure, the HBM budget, waits and errors.
"""
import numpy as np
import pytest

import oracle
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


def mixed_requests(seed=0):
    r = np.random.default_rng(seed)
    reqs = []
    specs = ([(64, int(n), 0) for n in r.integers(50, 3000, 24)] +      # batchable
             [(64, 40000, 0), (64, 70000, 0)] +                         # G 64, too big to fuse
             [(128, int(n), 0) for n in r.integers(1000, 60000, 4)] +
             [(256, 200000, 0), (256, 400000, 3), (128, 30000, 4), (64, 2000, 2)])
    for k, (G, n, refine) in enumerate(specs):
        inst = datagen.make_instance(n, float(r.uniform(0.5, 0.95)), 1.0, 500 + k)
        reqs.append(dict(G=G, x=dev(inst.x), y=dev(inst.y), xh=inst.x, yh=inst.y,
                         mask=torch.empty(n, dtype=torch.uint8, device="cuda"), refine=refine))
    return reqs


def test_each_result_identical_alone_and_in_the_mix(rv, orc):
    reqs = mixed_requests()
    eps_deg = 1.5
    with rv.Server(workers=3, max_n=1 << 20, max_grid=256, topk=16, max_batch=16,
                   batch_max_n=65536) as srv:
        # the largest first: they hold the workers while the small ones queue up
        order = sorted(range(len(reqs)), key=lambda k: -reqs[k]["x"].shape[1] * reqs[k]["G"])
        tickets = {k: srv.submit(reqs[k]["x"], reqs[k]["y"], reqs[k]["G"], eps_deg,
                                 reqs[k]["mask"], reqs[k]["refine"]) for k in order}
        replies = [srv.wait(tickets[k]) for k in range(len(reqs))]
        assert srv.stats()["queued"] == 0 and srv.stats()["in_flight"] == 0
    torch.cuda.synchronize()
    assert all(r["status"] == 0 for r in replies)
    assert max(r["batched"] for r in replies) > 1          # batching happened
    assert len({r["worker"] for r in replies}) > 1          # several workers served
    with rv.Solver(max_n=1 << 20, max_grid=256, topk=16) as s:
        for q, r in zip(reqs, replies):
            m = torch.empty_like(q["mask"])
            q1, c1, _ = s.solve(q["x"], q["y"], q["G"], eps_deg, mask=m.view(torch.bool))
            if q["refine"]:
                q1, c1, ran = s.refine(q["x"], q["y"], q1, m, eps_deg, max_rounds=q["refine"])
                assert ran == r["refine_rounds_run"]
            assert r["q"] == q1 and r["count"] == c1
            assert torch.equal(m, q["mask"])
            assert r["t_submit"] <= r["t_start"] <= r["t_end"]
    # the fused small requests against the oracle as well
    eps = rv.eps_deg_to_rad(eps_deg)
    for q, r in zip(reqs, replies):
        if r["batched"] > 1:
            o = orc.solve(q["xh"], q["yh"], q["G"], 8 * q["G"], eps, 16)
            assert np.array_equal(np.float32(r["q"]).view(np.uint32), o["q"].view(np.uint32))
            assert r["count"] == o["count"]
            assert np.array_equal(q["mask"].cpu().numpy(), o["mask"])


def test_queue_backpressure_and_waits(rv):
    inst = datagen.make_instance(300000, 0.9, 1.0, 3)
    x, y = dev(inst.x), dev(inst.y)
    masks = [torch.empty(inst.n, dtype=torch.uint8, device="cuda") for _ in range(12)]
    with rv.Server(workers=1, max_n=inst.n, max_grid=256, max_batch=0, max_queue=2) as srv:
        tickets, refused = [], 0
        for m in masks:
            try:
                tickets.append(srv.submit(x, y, 256, 1.0, m))
            except rv.RotVoteError as e:
                assert e.status == rv.RV_EAGAIN
                refused += 1
        assert refused > 0 and len(tickets) >= 2
        counts = set()
        try:
            counts.add(srv.wait(tickets[-1], timeout_ms=0)["count"])
            tickets.pop()  # already done and collected
        except rv.RotVoteError as e:
            assert e.status == rv.RV_ETIMEDOUT
        for t in tickets:
            counts.add(srv.wait(t)["count"])
        assert len(counts) == 1
        with pytest.raises(rv.RotVoteError) as e:
            srv.wait(tickets[0])  # collected already
        assert e.value.status == rv.RV_EINVAL


def test_hbm_budget_admission(rv):
    with rv.Server(workers=1, max_n=1 << 18, max_grid=128, max_batch=8) as one:
        per = one.stats()["device_bytes"]
    assert per > 0
    with pytest.raises(rv.RotVoteError) as e:
        rv.Server(workers=2, max_n=1 << 18, max_grid=128, max_batch=8, hbm_budget=per // 2)
    assert e.value.status == rv.RV_ENOMEM
    with rv.Server(workers=4, max_n=1 << 18, max_grid=128, max_batch=8,
                   hbm_budget=int(per * 2.5)) as srv:
        st = srv.stats()
        assert st["workers"] == 2 and st["device_bytes"] <= per * 2.5


def test_request_errors(rv):
    with rv.Server(workers=1, max_n=1000, max_grid=64) as srv:
        x = torch.randn(3, 100, device="cuda")
        m = torch.empty(100, dtype=torch.uint8, device="cuda")
        for n, G, eps in [(1001, 16, 0.01), (100, 65, 0.01), (100, 0, 0.01), (100, 16, 0.0),
                          (-1, 16, 0.01)]:
            with pytest.raises(rv.RotVoteError) as e:
                srv.submit_raw(x.data_ptr(), x.data_ptr(), n, G, eps, m.data_ptr())
            assert e.value.status == rv.RV_EINVAL
        # an empty request is served
        e0 = torch.empty(3, 0, device="cuda")
        t = srv.submit(e0, e0, 16, 1.0, torch.empty(0, dtype=torch.uint8, device="cuda"))
        r = srv.wait(t)
        assert r["status"] == 0 and r["count"] == 0 and r["q"] == [1.0, 0.0, 0.0, 0.0]
