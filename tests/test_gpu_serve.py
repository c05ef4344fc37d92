"""GPU: the request server (rot_vote_server_*).

Every result is identical alone and in the mix: a mixed burst of requests
(batchable small ones, large ones, three grids, some with refinement) goes
through a server with several workers and batching; each reply and mask must
equal, bit for bit, a standalone rot_vote_solve (+ rot_vote_refine) of the same
request, and the batched small ones the CPU oracle as well.  Then admission
by each request's scratch bytes (blocking when the arena is full, admitting
many small requests at once), ordering after the producer's stream, queue
backpressure, waits and errors.
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


def standalone(rv, reqs, eps_deg):
    """Each request solved alone on a handle of its own: (q, count, mask)."""
    out = []
    with rv.Solver(max_n=1 << 20, max_grid=256, topk=16) as s:
        for q in reqs:
            m = torch.empty_like(q["mask"])
            q1, c1, _ = s.solve(q["x"], q["y"], q["G"], eps_deg, mask=m.view(torch.bool))
            out.append((q1, c1, m))
    return out


def make_requests(specs, seed):
    r = np.random.default_rng(seed)
    reqs = []
    for k, (G, n) in enumerate(specs):
        inst = datagen.make_instance(n, float(r.uniform(0.8, 0.99)), 1.0, seed * 1000 + k)
        reqs.append(dict(G=G, x=dev(inst.x), y=dev(inst.y),
                         mask=torch.empty(n, dtype=torch.uint8, device="cuda")))
    return reqs


def overlap_max(replies):
    """The most requests whose [t_start, t_end] intervals overlap at one time."""
    ev = sorted([(r["t_start"], 1) for r in replies] + [(r["t_end"], -1) for r in replies],
                key=lambda e: (e[0], e[1]))
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def test_admission_blocks_by_bytes(rv):
    """The arena holds two large requests' footprints and a half: with eight
    lanes free, only two of four queued large requests are admitted at once;
    the others wait for memory, not for a lane.  Results equal standalone solves."""
    reqs = make_requests([(256, 300000)] * 4, 7)
    eps_deg = 1.5
    with rv.Server(workers=8, max_n=1 << 20, max_grid=256, topk=16, max_batch=0,
                   hbm_budget=1) as probe:
        big = probe.request_bytes(300000, 256)
    budget = 2 * big + big // 2
    with rv.Server(workers=8, max_n=1 << 20, max_grid=256, topk=16, max_batch=0,
                   hbm_budget=budget) as srv:
        mem = srv.memory()
        assert mem["arena_bytes"] >= budget and mem["in_use"] == 0
        srv.pause()
        tickets = [srv.submit(q["x"], q["y"], q["G"], eps_deg, q["mask"]) for q in reqs]
        assert srv.stats()["queued"] == 4 and srv.stats()["in_flight"] == 0
        srv.pause(False)
        replies = [srv.wait(t) for t in tickets]
        mem = srv.memory()
    assert mem["peak_in_flight"] == 2
    assert 2 * big <= mem["peak_in_use"] <= budget and mem["in_use"] == 0
    assert overlap_max(replies) <= 2
    assert all(r["scratch_bytes"] == big and r["status"] == 0 for r in replies)
    for (q1, c1, m1), r, q in zip(standalone(rv, reqs, eps_deg), replies, reqs):
        assert r["q"] == q1 and r["count"] == c1 and torch.equal(m1, q["mask"])


def test_admission_by_bytes_not_by_count(rv):
    """In the same arena (room for two large requests) eight small ones (1 MiB
    grids) are admitted at once, one per free lane; then one large request and
    six small ones: the large one is admitted, then the small ones while their
    bytes fit.  Every result equals a standalone solve."""
    with rv.Server(workers=8, max_n=1 << 20, max_grid=256, topk=16, max_batch=0,
                   hbm_budget=1) as probe:
        big = probe.request_bytes(300000, 256)
        small = probe.request_bytes(3000, 64)
    assert small == 64 ** 3 * 4  # the global strategy's footprint is its grid
    eps_deg = 1.5
    smalls = make_requests([(64, 3000)] * 8, 8)
    with rv.Server(workers=8, max_n=1 << 20, max_grid=256, topk=16, max_batch=0,
                   hbm_budget=2 * big + big // 2) as srv:
        srv.pause()
        tickets = [srv.submit(q["x"], q["y"], q["G"], eps_deg, q["mask"]) for q in smalls]
        srv.pause(False)
        replies = [srv.wait(t) for t in tickets]
        assert srv.memory()["peak_in_flight"] == 8
    for (q1, c1, m1), r, q in zip(standalone(rv, smalls, eps_deg), replies, smalls):
        assert r["q"] == q1 and r["count"] == c1 and torch.equal(m1, q["mask"])
    mix = make_requests([(256, 300000)] + [(128, 20000)] * 6, 9)
    with rv.Server(workers=8, max_n=1 << 20, max_grid=256, topk=16, max_batch=0,
                   hbm_budget=1) as probe:
        mid = probe.request_bytes(20000, 128)
    budget = big + 3 * mid + mid // 2
    with rv.Server(workers=8, max_n=1 << 20, max_grid=256, topk=16, max_batch=0,
                   hbm_budget=budget) as srv:
        srv.pause()
        tickets = [srv.submit(q["x"], q["y"], q["G"], eps_deg, q["mask"]) for q in mix]
        srv.pause(False)
        replies = [srv.wait(t) for t in tickets]
        mem = srv.memory()
    assert mem["peak_in_flight"] >= 4 and mem["peak_in_use"] <= budget
    assert [r["scratch_bytes"] for r in replies] == [big] + [mid] * 6
    for (q1, c1, m1), r, q in zip(standalone(rv, mix, eps_deg), replies, mix):
        assert r["q"] == q1 and r["count"] == c1 and torch.equal(m1, q["mask"])


def test_request_beyond_the_arena_is_refused(rv):
    with rv.Server(workers=2, max_n=1 << 20, max_grid=256, max_batch=0,
                   hbm_budget=16 << 20) as srv:
        x = torch.randn(3, 1000, device="cuda")
        m = torch.empty(1000, dtype=torch.uint8, device="cuda")
        with pytest.raises(rv.RotVoteError) as e:
            srv.submit(x, x, 256, 1.0, m)  # a 64 MiB grid
        assert e.value.status == rv.RV_ENOMEM
        r = srv.wait(srv.submit(x, x, 64, 1.0, m))  # 1 MiB: admitted
        assert r["status"] == 0


def test_request_waits_for_its_producer_stream(rv):
    """x is written on torch's current stream behind a long GPU spin; the
    request is submitted at once, and its lane (another stream) must wait for
    that write: the result equals a standalone solve of the final data."""
    inst = datagen.make_instance(50000, 0.9, 1.0, 41)
    src_x, src_y = dev(inst.x), dev(inst.y)
    x = torch.full_like(src_x, float("nan"))
    y = torch.full_like(src_y, float("nan"))
    mask = torch.empty(inst.n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    with rv.Server(workers=2, max_n=1 << 17, max_grid=128, max_batch=0) as srv:
        torch.cuda._sleep(200_000_000)  # on the current stream
        x.copy_(src_x)
        y.copy_(src_y)
        r = srv.wait(srv.submit(x, y, 128, 1.5, mask))
    (q1, c1, m1), = standalone(rv, [dict(G=128, x=src_x, y=src_y, mask=mask)], 1.5)
    assert r["status"] == 0 and r["count"] > 0
    assert r["q"] == q1 and r["count"] == c1 and torch.equal(m1, mask)


def test_request_errors(rv):
    with rv.Server(workers=1, max_n=1000, max_grid=64) as srv:
        x = torch.randn(3, 100, device="cuda")
        m = torch.empty(100, dtype=torch.uint8, device="cuda")
        for n, G, eps in [(1001, 16, 0.01), (100, 65, 0.01), (100, 0, 0.01), (100, 16, 0.0),
                          (-1, 16, 0.01)]:
            with pytest.raises(rv.RotVoteError) as e:
                srv.submit_raw(x.data_ptr(), x.data_ptr(), n, G, eps, m.data_ptr())
            assert e.value.status == rv.RV_EINVAL
        r = rv.Request(x.data_ptr(), x.data_ptr(), 100, 16, 0.01, m.data_ptr(), 0, 4, None)
        t = __import__("ctypes").c_uint64()
        assert srv._lib.rot_vote_server_submit(srv._h, __import__("ctypes").byref(r),
                                               __import__("ctypes").byref(t)) == rv.RV_EINVAL
        # an empty request is served
        e0 = torch.empty(3, 0, device="cuda")
        t = srv.submit(e0, e0, 16, 1.0, torch.empty(0, dtype=torch.uint8, device="cuda"))
        r = srv.wait(t)
        assert r["status"] == 0 and r["count"] == 0 and r["q"] == [1.0, 0.0, 0.0, 0.0]
