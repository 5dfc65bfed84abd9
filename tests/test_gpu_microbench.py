"""The roof micro-benchmarks run, count their operations as documented, and
reject bad arguments."""
import pytest

from paper_2401_05345_amd import gsr
from gpu_util import say

pytestmark = pytest.mark.gpu

MIB = 1 << 20
THREADS, ITERS = 8192 * 256, 64


@pytest.fixture(scope="module")
def renderer(gsr):
    import torch
    r = gsr.Renderer(0)
    yield r
    torch.cuda.synchronize()
    r.close()


@pytest.mark.parametrize("kind,ops", [
    (gsr.GSR_MB_COPY, 8 * MIB),
    (gsr.GSR_MB_ATOMIC_F32_DISTINCT, THREADS * ITERS),
    (gsr.GSR_MB_ATOMIC_F64_DISTINCT, THREADS * ITERS),
    (gsr.GSR_MB_ATOMIC_F32_SAME_ADDRESS, THREADS * ITERS),
    (gsr.GSR_MB_ATOMIC_F32_ONE_LANE, THREADS // 64 * ITERS),
    (gsr.GSR_MB_ATOMIC_F64_NINE_LANES, THREADS // 64 * ITERS * 9),
    (gsr.GSR_MB_WRITE, 8 * MIB),
    (gsr.GSR_MB_READ, 8 * MIB - 16),
    (gsr.GSR_MB_COPY_NT, 8 * MIB),
    (gsr.GSR_MB_GATHER48, 131072 * 48),
])
def test_microbench_runs_and_counts(renderer, kind, ops):
    say(f"[gpu] microbench kind {kind}")
    ms, n = gsr.gsr_microbench(renderer.ctx, kind, 8 * MIB, reps=3)
    assert n == ops
    assert 0.0 < ms < 1000.0


def test_microbench_rejects_bad_arguments(renderer):
    for kind, nbytes, reps in [(10, 8 * MIB, 3), (-1, 8 * MIB, 3), (0, 3 * MIB, 3), (0, MIB // 2, 3),
                               (0, 8 << 30, 3), (0, 8 * MIB, 0), (0, 8 * MIB, 101)]:
        with pytest.raises(gsr.GsrError) as e:
            gsr.gsr_microbench(renderer.ctx, kind, nbytes, reps)
        assert e.value.status == gsr.GSR_EINVAL
