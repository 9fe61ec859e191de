"""The chip-rate probes the benchmark reports beside its rooflines: every
rate positive and below what the chip's units allow (two wave64 FP32 VALU
instructions per CU per cycle, a transcendental at a quarter of that, the
2.5 PFLOP/s dense BF16 peak at 2.4 GHz, 8 TB/s of HBM), and the shader
clock in a plausible range."""
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu


def test_probe_rates_are_within_the_chip_limits(gpu_lib):
    from paper_2508_04929_amd import probe
    announce("chip-rate probes")
    r = probe.measure(copy_mib=256)
    for name in ("fma", "exp", "lds", "mfma"):
        assert 0.5 < r[name]["clock_ghz"] < 2.6, (name, r[name]["clock_ghz"])
        assert r[name]["per_cu_per_cycle"] > 0
    assert r["fma"]["per_cu_per_cycle"] <= 2.05
    assert r["exp"]["per_cu_per_cycle"] <= 0.55
    assert r["mfma"]["tflops_bf16"] <= 2.5e3 * 1.02
    assert 0 < r["copy"]["gb_per_s"] <= 8000 * 1.02
