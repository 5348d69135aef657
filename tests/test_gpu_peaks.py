"""Machine-limit microbenchmarks: the measured rates are positive and no
higher than the published MI355X figures allow (a miscounted operation
per instruction or byte per launch shows up as a rate above them)."""

import pytest

torch = pytest.importorskip("torch")

from paper_1901_04289_amd import arbgpu

pytestmark = pytest.mark.gpu

# Published dense figures at 2.4 GHz on 256 compute units.
PUBLISHED = {"int8_mfma_tops": 5000.0, "fp64_mfma_tflops": 78.6, "hbm_copy_gbs": 8000.0, "hbm_read_gbs": 8000.0}


def test_probe_peaks_within_published_limits():
    ctx = arbgpu.Context(0)
    try:
        buf = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        pk = ctx.probe_peaks(buf)
        print(pk, flush=True)
        for k, lim in PUBLISHED.items():
            assert 0.05 * lim < pk[k] <= 1.02 * lim, (k, pk[k])
        # 32-bit multiplies: no faster than the vector FP32 rate (32 lanes per
        # cycle per SIMD, 4 SIMDs per compute unit, 2.4 GHz)
        lane_cycles = pk["compute_units"] * 4 * 32 * 2.4   # G lane-ops/s
        for k in ("mad_u64_u32_gops", "mul_hi_u32_gops"):
            assert 0.0 < pk[k] <= 1.02 * lane_cycles, (k, pk[k])
        assert 500.0 < pk["clock_mhz"] <= 2500.0
        assert pk["compute_units"] == 256
    finally:
        ctx.close()
