"""The energy meter fails loudly where the GPU's energy accumulator cannot be
read (no driver in a CPU-only container), instead of estimating."""
import pytest

from paper_2402_09222_amd import energy


def test_meter_fails_loudly_without_gpu():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(RuntimeError):
        energy.EnergyMeter(0)
