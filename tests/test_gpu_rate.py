"""Sustained-rate probes: each measured ceiling is positive and below the
published MI355X peak of its kind (with 5 % margin for clock reporting).
Invalid requests are tested on the host, in the C-ABI host tests."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)
import paper_2410_02314_amd as dl  # noqa: E402

PUBLISHED = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0, "hbm_copy": 8000.0}


@pytest.mark.parametrize("kind", ["fp32", "bf16", "fp8", "hbm_copy"])
def test_rate_below_published_peak(kind):
    v = dl.measure_rate(kind, 256 << 20, 2)
    assert 0.2 * PUBLISHED[kind] < v < 1.05 * PUBLISHED[kind], v

