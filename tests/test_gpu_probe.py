"""The streaming-read probe (fbc_probe_read): a positive rate below the HBM peak on a
device buffer, and the same buffer read twice gives rates within a factor of two."""
import pytest

pytestmark = pytest.mark.gpu


def test_read_probe_reports_a_plausible_rate():
    import torch
    from paper_2105_08798_amd import probe_read
    buf = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")     # 1 GiB
    a = probe_read(buf, 1024, reps=3)
    b = probe_read(buf, 2048, reps=3)
    assert 100.0 < a < 8000.0 * 1.05 and 100.0 < b < 8000.0 * 1.05, (a, b)
    assert 0.5 < a / b < 2.0, (a, b)
