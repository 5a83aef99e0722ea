"""Host-side checks of the Python binding (CPU only): a buffer that is not a contiguous
tensor of the problem's device, dtype and size is refused before any library call."""
import pytest
import torch

from paper_2308_01957_amd import apx


def test_check_buffer_accepts_the_exact_buffer():
    t = torch.zeros(12, dtype=torch.float32)
    assert apx.check_buffer(t, torch.device("cpu"), torch.float32, 12, "data") is t


@pytest.mark.parametrize("bad, why", [
    (lambda: torch.zeros(12, dtype=torch.float64), "dtype"),
    (lambda: torch.zeros(11, dtype=torch.float32), "elements"),
    (lambda: torch.zeros(24, dtype=torch.float32)[::2], "contiguous"),
    (lambda: [0.0] * 12, "torch tensor"),
])
def test_check_buffer_refuses_before_launch(bad, why):
    with pytest.raises(apx.ApxError) as e:
        apx.check_buffer(bad(), torch.device("cpu"), torch.float32, 12, "data")
    assert e.value.status == apx.APX_E_INVALID and why in str(e.value)


def test_check_buffer_refuses_another_device():
    with pytest.raises(apx.ApxError, match="on cpu"):
        apx.check_buffer(torch.zeros(4), torch.device("cuda", 0), torch.float32, 4, "weight")
