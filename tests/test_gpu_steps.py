"""GPU: each device step of the rule against the oracle's step, bit for bit,
and the rounding of the primitive operations the rule relies on."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def probe():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2506_11547_amd.rotvote import Probe
    return Probe()


@pytest.fixture(scope="module")
def orc():
    return oracle.get()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def test_fast_reciprocal_exact_on_1_2(probe):
    """The chart's reciprocal is only ever taken of 1 + |w| in [1, 2]: every
    binary32 value there gets IEEE 1/d from the refined hardware reciprocal."""
    d = np.arange(0x3F800000, 0x40000001, dtype=np.uint32).view(np.float32)
    fast = probe.recip(dev(d), fast=True).cpu().numpy()
    ieee = probe.recip(dev(d), fast=False).cpu().numpy()
    ref = (np.float32(1.0) / d).astype(np.float32)
    assert np.array_equal(bits(ieee), bits(ref))
    assert np.array_equal(bits(fast), bits(ref))


def test_division_and_sqrt_correctly_rounded(probe):
    r = np.random.default_rng(0)
    a = np.concatenate([r.normal(size=1 << 20), r.uniform(0, 1e-38, 1 << 16),
                        10.0 ** r.uniform(-30, 30, 1 << 18)]).astype(np.float32)
    a = np.abs(a)
    b = np.concatenate([r.normal(size=a.size - (1 << 16)), r.uniform(1e-39, 1e-37, 1 << 16)])
    b = b.astype(np.float32)
    b[b == 0] = 1.0
    q, s = probe.div_sqrt(dev(a), dev(b))
    with np.errstate(all="ignore"):
        assert np.array_equal(bits(q.cpu().numpy()), bits((a / b).astype(np.float32)))
        assert np.array_equal(bits(s.cpu().numpy()), bits(np.sqrt(a).astype(np.float32)))


def _hard_pairs(n, seed):
    r = np.random.default_rng(seed)
    x = r.normal(size=(3, n)) * 10 ** r.uniform(-3, 3, size=n)
    y = r.normal(size=(3, n))
    k = n // 8
    y[:, :k] = x[:, :k]                                  # a = b
    y[:, k:2 * k] = -x[:, k:2 * k] * 3                   # a = -b
    y[:, 2 * k:3 * k] = x[:, 2 * k:3 * k] + 1e-4 * r.normal(size=(3, k))
    e = np.eye(3)
    for t in range(9):
        x[:, 3 * k + t] = e[t % 3]
        y[:, 3 * k + t] = (-1) ** t * e[t // 3]
    x[:, 4 * k] = 0
    y[:, 4 * k + 1] = np.nan
    x[:, 4 * k + 2] = np.inf
    y[:, 4 * k + 3] = 1e30
    x[:, 4 * k + 4] = 1e-30
    x[:, 4 * k + 5] = [3e-39, 0, 0]                      # subnormal direction
    return x.astype(np.float32), y.astype(np.float32)


def test_basis_matches_oracle(probe, orc):
    x, y = _hard_pairs(20000, 1)
    u, v, ok = probe.basis(dev(x), dev(y))
    u, v, ok = u.cpu().numpy(), v.cpu().numpy(), ok.cpu().numpy()
    for i in range(x.shape[1]):
        oka, a = orc.normalise(x[:, i])
        okb, b = orc.normalise(y[:, i])
        assert bool(ok[i]) == (oka and okb), i
        if not ok[i]:
            continue
        uo, vo, _ = orc.circle_basis(a, b)
        assert np.array_equal(bits(u[i]), bits(uo)), i
        assert np.array_equal(bits(v[i]), bits(vo)), i


@pytest.mark.parametrize("fast", [False, True])
@pytest.mark.parametrize("G", [1, 2, 3, 7, 64, 128, 255, 256, 360])
def test_cells_match_oracle(probe, orc, G, fast):
    r = np.random.default_rng(G)
    q = r.normal(size=(20000, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[:500, 0] = 0.0                                       # equator
    q[500:1000, 0] = -0.0
    q[1000:1100, :2] = 0.0
    q[1100:1200, 0] = -0.0
    q[1100:1200, 1:3] = 0.0
    q[1100:1200, 3] = -1.0
    q[1200:1300] = [1, 0, 0, 0]
    q = q.astype(np.float32)
    got = probe.cells(dev(q), G, fast).cpu().numpy()
    ref = np.array([orc.cell_of(qq, G)[0] for qq in q], np.int32)
    assert np.array_equal(got, ref)
    neg = probe.cells(dev(-q), G, fast).cpu().numpy()
    assert np.array_equal(neg, ref)


@pytest.mark.parametrize("G", [1, 4, 7, 64, 256])
def test_decode_matches_oracle(probe, orc, G):
    n = min(G ** 3, 50000)
    idx = np.random.default_rng(G).choice(G ** 3, size=n, replace=False).astype(np.int32)
    got = probe.decode(dev(idx), G).cpu().numpy()
    ref = np.stack([orc.decode(i, G) for i in idx])
    assert np.array_equal(bits(got), bits(ref))


def test_residual_matches_oracle(probe, orc):
    x, y = _hard_pairs(20000, 2)
    r = np.random.default_rng(3)
    for _ in range(4):
        q = r.normal(size=4)
        q = (q / np.linalg.norm(q)).astype(np.float32)
        got = probe.residual(dev(x), dev(y), dev(q)).cpu().numpy()
        ref = np.array([orc.residual(x[:, i], y[:, i], q) for i in range(x.shape[1])], np.float32)
        assert np.array_equal(bits(got), bits(ref))

