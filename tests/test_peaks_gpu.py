"""Peak probes: each sustained rate must lie between a tenth of the unit's
published MI355X peak and 10% above it (clocks may run a little above the
nominal 2.4 GHz; a probe far above the peak would mean its work accounting
is wrong), and a short buffer is refused before any launch."""
from __future__ import annotations

import pytest

from gpu_harness import log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# published dense peaks: fp4 10.1 PFLOP/s and int8 5.0 POP/s (2 ops per MAC),
# 32-bit VALU 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, HBM3E 8 TB/s
PUBLISHED = {"fp4": 10.1e15 / 2, "i8": 5.0e15 / 2, "valu": 256 * 4 * 16 * 2.4e9, "hbm": 8.0e12}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1707_00516_amd.torch_api import Context
    c = Context(0)
    yield c
    c.sync()
    c.close()


def test_peak_probes_within_published_peaks(ctx):
    from paper_1707_00516_amd import (FID_PROBE_HBM_COPY, FID_PROBE_MFMA_FP4, FID_PROBE_MFMA_I8,
                                      FID_PROBE_VALU, fid_peak_probe)
    buf = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")  # 1 GiB copied: well past the caches
    for name, probe in (("fp4", FID_PROBE_MFMA_FP4), ("i8", FID_PROBE_MFMA_I8), ("valu", FID_PROBE_VALU),
                        ("hbm", FID_PROBE_HBM_COPY)):
        log(f"peak probe {name}")
        rate, ms = fid_peak_probe(ctx.handle, probe, buf.data_ptr(), buf.numel())
        log(f"peak probe {name}: {rate:.3e} per s, {ms:.3f} ms")
        assert ms > 0
        assert 0.1 * PUBLISHED[name] < rate <= 1.10 * PUBLISHED[name], (name, rate)


def test_peak_probe_rejects_short_buffer(ctx):
    from paper_1707_00516_amd import FID_EINVAL, FID_PROBE_VALU, FidError, fid_peak_probe
    buf = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(FidError) as e:
        fid_peak_probe(ctx.handle, FID_PROBE_VALU, buf.data_ptr(), buf.numel())
    assert e.value.status == FID_EINVAL
    with pytest.raises(FidError):
        fid_peak_probe(ctx.handle, 9, buf.data_ptr(), buf.numel())
