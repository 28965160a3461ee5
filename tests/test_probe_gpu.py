"""Peak probes (FMA issue, LDS reads) run and give rates in a plausible range
of the published MI355X figures: FMA issue at 50-110 % of 256 CUs x 64 lanes
x 2.4 GHz, LDS reads of at least 32 bytes per CU and clock."""
import pytest

pytestmark = pytest.mark.gpu


def test_probes_measure_plausible_rates():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import bench
    r = bench.measure_peaks()
    print(r, flush=True)
    assert 0.5 <= r["valu_fma"]["frac_of_published"] <= 1.1, r
    assert r["lds_read"]["per_cu_bytes_per_clock"] >= 32, r
    assert r["hbm_copy"]["measured"] > 1.0, r
