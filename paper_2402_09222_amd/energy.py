"""Board energy of the GPU the lookups run on.

The paper tunes not only for run time but for energy (power x run time) and
for the energy-delay product (energy x run time), section 7, reading node
power counters around each evaluation.  On an MI355X the board keeps an
energy accumulator that AMD SMI exposes; `EnergyMeter.joules()` reads it, so
the energy of a timed region is the difference of two readings taken after
the device has finished the region's work.

Fails loudly (RuntimeError) where the accumulator cannot be read; nothing
here estimates energy any other way.
"""
from __future__ import annotations


class EnergyMeter:
    """Energy accumulator of one GPU (torch device index `device`)."""

    def __init__(self, device: int = 0):
        try:
            import amdsmi
        except ImportError as e:  # pragma: no cover - depends on the image
            raise RuntimeError("AMD SMI (amdsmi) is not importable") from e
        self._smi = amdsmi
        try:
            amdsmi.amdsmi_init(amdsmi.AmdSmiInitFlags.INIT_AMD_GPUS)
            handles = amdsmi.amdsmi_get_processor_handles()
            if not handles:
                raise RuntimeError("AMD SMI reports no GPU")
            self.handle = handles[0] if len(handles) == 1 else self._match(
                handles, device)
            self.joules()  # fail now, not inside a timed region
        except amdsmi.AmdSmiException as e:
            raise RuntimeError(f"GPU energy accumulator unreadable: {e}") from e

    def _match(self, handles, device):
        import torch
        props = torch.cuda.get_device_properties(device)
        bus = getattr(props, "pci_bus_id", None)
        if bus is None:
            raise RuntimeError("cannot tell which GPU the torch device is")
        for h in handles:
            bdf = self._smi.amdsmi_get_gpu_device_bdf(h)  # "dddd:bb:dd.f"
            if int(bdf.split(":")[1], 16) == bus:
                return h
        raise RuntimeError(f"no AMD SMI GPU on PCI bus {bus:#x}")

    def joules(self) -> float:
        """The accumulator in joules (monotone while the process runs)."""
        e = self._smi.amdsmi_get_energy_count(self.handle)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6

    def close(self):
        try:
            self._smi.amdsmi_shut_down()
        except Exception:
            pass


def measure(fn, meter: EnergyMeter, min_seconds: float = 0.25,
            max_calls: int = 100000):
    """Runs fn() repeatedly for at least min_seconds of device time (the
    accumulator advances in coarse steps) and returns (seconds per call,
    joules per call).  fn must enqueue device work on torch's current
    stream."""
    import time

    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    one = max(time.perf_counter() - t0, 1e-6)
    calls = int(min(max_calls, max(3, min_seconds / one)))
    torch.cuda.synchronize()
    j0 = meter.joules()
    t0 = time.perf_counter()
    for _ in range(calls):
        fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    j1 = meter.joules()
    return dt / calls, (j1 - j0) / calls
