"""GPU: rot_vote_solve_async (the solve enqueued without waiting, result
written to a device rv_result) against rot_vote_solve and the oracle: the
same rotation bits, count, winner and mask; several solves in flight on one
stream; n = 0; argument errors; and the call captured into a HIP graph,
replayed on new inputs with eager work between the replays, every replay
checked against an eager solve.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same_q(a, b):
    return np.array_equal(np.float32(a).view(np.uint32), np.float32(b).view(np.uint32))


def instance(n, seed, outliers=0.8):
    inst = datagen.make_instance(n, outliers, 0.5, seed, radii=(0.5, 2.0))
    return inst.x, inst.y


@pytest.mark.parametrize("strategy", ["auto", "global", "brick"])
@pytest.mark.parametrize("n,G", [(1000, 64), (20000, 128), (5000, 300)])
def test_async_matches_sync_and_oracle(rv, strategy, n, G):
    xh, yh = instance(n, 11 + G)
    x, y = dev(xh), dev(yh)
    eps = 1.0
    with rv.Solver(max_n=n, max_grid=G, topk=16, strategy=strategy) as s:
        q, cnt, m = s.solve(x, y, G, eps)
        m = m.clone()
        top_sync = s.topk()
        res, ma = s.solve_async(x, y, G, eps)
        torch.cuda.synchronize()
        r = rv.decode_result(res)
        assert same_q(r["q"], q) and r["count"] == cnt
        assert torch.equal(ma, m)
        top = s.topk()   # describes the asynchronous solve
        assert top == top_sync and r["winner"] == top["winner"]
        assert r["n_cand"] == len(top["votes"])
    if n <= 5000:
        o = oracle.get().solve(xh, yh, G, 8 * G, rv.eps_deg_to_rad(eps), 16)
        assert np.array_equal(np.float32(r["q"]).view(np.uint32), o["q"].view(np.uint32))
        assert r["count"] == o["count"]
        assert np.array_equal(ma.cpu().numpy(), o["mask"])


def test_several_solves_in_flight(rv):
    """Three instances enqueued back to back on one stream (shared scratch,
    ordered by the stream), results into rows of one tensor, no wait between."""
    inst = [instance(3000, 1), instance(800, 2, 0.5), instance(12000, 3, 0.95)]
    G, eps = 128, 1.5
    with rv.Solver(max_n=12000, max_grid=G, topk=16) as s:
        ref = []
        for xh, yh in inst:
            q, c, m = s.solve(dev(xh), dev(yh), G, eps)
            ref.append((q, c, m.clone()))
        xs = [(dev(xh), dev(yh)) for xh, yh in inst]
        res = torch.empty(len(inst), rv.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        masks = []
        for rep in range(2):
            for k in (range(len(inst)) if rep == 0 else reversed(range(len(inst)))):
                _, mk = s.solve_async(xs[k][0], xs[k][1], G, eps, result=res[k])
                masks.append((k, mk))
            torch.cuda.synchronize()
            for k in range(len(inst)):
                r = rv.decode_result(res[k])
                assert same_q(r["q"], ref[k][0]) and r["count"] == ref[k][1], (rep, k)
            for k, mk in masks:
                assert torch.equal(mk, ref[k][2]), (rep, k)
            masks.clear()


def test_async_empty_input(rv):
    with rv.Solver(max_n=100, max_grid=64) as s:
        z = torch.zeros(3, 0, dtype=torch.float32, device="cuda")
        res = torch.full((rv.RESULT_BYTES,), 7, dtype=torch.uint8, device="cuda")
        s.solve_async(z, z, 64, 1.0, result=res)
        torch.cuda.synchronize()
        r = rv.decode_result(res)
        assert r == {"q": [1.0, 0.0, 0.0, 0.0], "count": 0, "winner": -1, "n_cand": 0}


def test_async_argument_errors(rv):
    with rv.Solver(max_n=100, max_grid=64) as s:
        x = torch.randn(3, 100, device="cuda")
        mask = torch.empty(100, dtype=torch.uint8, device="cuda")
        buf = torch.zeros(2 * rv.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        host = torch.zeros(rv.RESULT_BYTES, dtype=torch.uint8)
        for rptr, G in [(buf.data_ptr() + 4, 64),          # misaligned
                        (host.data_ptr(), 64),             # host memory
                        (0, 64),                           # NULL
                        (buf.data_ptr(), 65)]:             # grid beyond max_grid
            with pytest.raises(rv.RotVoteError) as e:
                s.solve_async_raw(x.data_ptr(), x.data_ptr(), 100, G, 0.01, rptr, mask.data_ptr())
            assert e.value.status == rv.RV_EINVAL
        assert int(buf.sum()) == 0   # nothing was written


@pytest.mark.parametrize("mode", ["relaxed", "global"])
@pytest.mark.parametrize("G", [64, 256])
def test_async_solve_in_a_graph(rv, G, mode):
    """Captured once, replayed on three new inputs copied into the captured
    buffers; eager solves and synchronisations between the replays."""
    n = 4000
    inputs = [instance(n, 40 + k, 0.9) for k in range(3)]
    eps = 1.5
    stream = torch.cuda.Stream()
    xb = torch.empty(3, n, dtype=torch.float32, device="cuda")
    yb = torch.empty_like(xb)
    res = torch.zeros(rv.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    mask = torch.zeros(n, dtype=torch.bool, device="cuda")
    with rv.Solver(max_n=n, max_grid=G, topk=16, stream=stream) as s, \
            rv.Solver(max_n=n, max_grid=G, topk=16) as eager:
        xb.copy_(dev(inputs[0][0]))
        yb.copy_(dev(inputs[0][1]))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            s.solve_async(xb, yb, G, eps, result=res, mask=mask)   # uploads the table
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream, capture_error_mode=mode):
            s.solve_async(xb, yb, G, eps, result=res, mask=mask)
        torch.cuda.synchronize()
        for rep in range(2):
            for xh, yh in inputs:
                xb.copy_(dev(xh))
                yb.copy_(dev(yh))
                res.zero_()
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                q, c, m = eager.solve(dev(xh), dev(yh), G, eps)
                r = rv.decode_result(res)
                assert same_q(r["q"], q) and r["count"] == c, rep
                assert torch.equal(mask, m), rep
        del g


def test_async_stage_timings(rv):
    """With timing events the stage times of an asynchronous solve are read
    after waiting for its last event (no explicit synchronisation)."""
    xh, yh = instance(20000, 5)
    x, y = dev(xh), dev(yh)
    with rv.Solver(max_n=20000, max_grid=128, topk=16, timing=True) as s:
        q, c, _ = s.solve(x, y, 128, 1.0)
        res, _ = s.solve_async(x, y, 128, 1.0)
        t = s.timings()
        assert set(t) == set(rv.STAGE_NAMES) and all(v >= 0.0 for v in t.values())
        assert t["vote"] > 0.0
        r = rv.decode_result(res)
        assert same_q(r["q"], q) and r["count"] == c
