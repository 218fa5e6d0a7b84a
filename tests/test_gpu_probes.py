"""Roofline probes (paper_1305_2353_amd/probes.py, libctp_probe.so) on the
GPU: the measured peaks are plausible against MI355X's datasheet figures
(FP64 matrix 78.6, FP32 matrix 157.3, BF16 2500 TFLOP/s dense; HBM 8 TB/s):
at least 60% of each, at most 105%."""

import pytest

from gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu

DATASHEET = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16"])
def test_mfma_probe_near_datasheet(dtype):
    from paper_1305_2353_amd import probes
    print("case: mfma probe", dtype, flush=True)
    tf = probes.mfma_peak(dtype, grid=1024, iters=1024)
    print(f"{dtype}: {tf:.1f} TFLOP/s", flush=True)
    assert 0.6 * DATASHEET[dtype] <= tf <= 1.05 * DATASHEET[dtype]


def test_copy_probe_near_datasheet():
    from paper_1305_2353_amd import probes
    print("case: copy probe", flush=True)
    gbs = probes.copy_bandwidth(1 << 30)
    print(f"copy: {gbs:.0f} GB/s", flush=True)
    # a plain stream copy reaches 0.59-0.62 of the datasheet figure on these
    # machines (1 GiB here, 2 GiB in the benchmark's probe section); the test
    # checks that the probe measures a sane rate, not a particular machine
    assert 0.5 * 8000.0 <= gbs <= 1.05 * 8000.0
