"""GPU: the ceiling micro-benchmarks of the probe library (measurement hooks
of the benchmark).  Each one checks its own result on the host (the LDS and
device atomics are summed back, the copy's last element is read); here the
rates must be positive and plausible against the published figures of one
MI355X, and invalid arguments must be refused.
"""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALU_PEAK = 256 * 64 * 2.4e9   # 32-bit lane operations/s, one per lane per clock
HBM_PEAK = 8e12


@pytest.fixture(scope="module")
def probe():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2506_11547_amd import rotvote
    return rotvote.Probe()


def test_valu_ceiling_near_issue_peak(probe):
    r = probe.ceiling_valu(blocks=4096, iters=2048)
    assert 0.3 * ALU_PEAK < r < 1.1 * ALU_PEAK, r / ALU_PEAK


@pytest.mark.parametrize("random", [True, False])
def test_lds_atomic_ceiling(probe, random):
    r = probe.ceiling_lds_atomic(random, blocks=512, iters=256)
    assert r > 1e11, r


@pytest.mark.parametrize("contiguous", [False, True])
@pytest.mark.parametrize("mib", [1, 64])
def test_global_atomic_ceiling(probe, mib, contiguous):
    r = probe.ceiling_global_atomic(mib << 18, blocks=1024, iters=64, contiguous=contiguous)
    assert r > 1e9, r


def test_copy_ceiling_below_hbm_peak(probe):
    r = probe.ceiling_copy(1 << 30)
    assert 0.5e12 < r < 1.05 * HBM_PEAK, r


def test_read_ceiling_below_hbm_peak(probe):
    r = probe.ceiling_read(1 << 30)
    assert 0.5e12 < r < 1.05 * HBM_PEAK, r


def test_invalid_arguments_refused(probe):
    with pytest.raises(RuntimeError):
        probe.ceiling_global_atomic(3000)          # not a power of two
    with pytest.raises(RuntimeError):
        probe.ceiling_copy(100)                    # not a multiple of 16
    with pytest.raises(RuntimeError):
        probe.ceiling_read(100)                    # not a multiple of 16
    with pytest.raises(RuntimeError):
        probe.ceiling_valu(blocks=0)
