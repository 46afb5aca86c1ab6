"""The FMA-rate probe that the bench quotes measured peaks from (libsymprobe.so, a
benchmark helper outside the libsym ABI): it runs, its output is finite, and the rate it
implies lies below the data-sheet vector peak of the precision (FP32 157.3 TFLOP/s
counting packed FMA, which the library is compiled not to emit; FP64 78.6)."""
import pytest
import torch

from gpu_util import device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,spec", [(torch.float32, 157.3), (torch.float64, 78.6)])
def test_fma_probe_rate(dtype, spec):
    import bench

    device()
    rate = bench.fma_rate(torch, dtype, iters=2048, reps=3)
    print(f"  {dtype}: {rate:.1f} TFLOP/s")
    assert 1.0 < rate <= 1.05 * spec
