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
            depth: int = 4):
    """Board power while fn() runs back to back, and the energy of one call.

    The accumulator advances in steps at the firmware's update period, so a
    window between two arbitrary readings is off by up to one step.  Here
    the device is kept busy (up to `depth` calls queued) and the accumulator
    is polled while waiting; the window runs from one observed step to the
    first step after at least min_seconds, and power = energy difference /
    time between those two steps (the accumulator's own timestamps when
    they advance with it, else the host clock at detection).  The time of a
    call is measured on its own (synchronised wall time over several calls),
    and joules per call = power x seconds per call.

    fn must enqueue device work on torch's current stream.  Returns
    (seconds per call, joules per call, watts); measure.last holds the
    window's length and the accumulator steps inside it."""
    import time

    import torch
    fn()
    torch.cuda.synchronize()
    # seconds per call
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    one = max(time.perf_counter() - t0, 1e-6)
    reps = int(max(3, min(1000, 0.05 / one)))
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps

    def reading():
        e = meter._smi.amdsmi_get_energy_count(meter.handle)
        return (e["energy_accumulator"] * e["counter_resolution"] * 1e-6,
                e["timestamp"], time.perf_counter())

    events = []
    marks = []  # readings just after the accumulator stepped
    steps = 0   # accumulator steps seen inside the window
    last = reading()
    deadline = None
    limit = time.perf_counter() + 20.0 * max(min_seconds, 10 * one) + 5.0
    while True:
        ev = torch.cuda.Event()
        fn()
        ev.record()
        events.append(ev)
        while len(events) >= depth and not events[0].query():
            r = reading()
            if r[0] != last[0]:
                if marks:
                    steps += 1
                if len(marks) == 0 or (deadline and r[2] >= deadline):
                    marks.append(r)
                    if len(marks) == 1:
                        deadline = r[2] + min_seconds
                last = r
        while len(events) >= depth and events[0].query():
            events.pop(0)
        if len(marks) >= 2:
            break
        if time.perf_counter() > limit:
            torch.cuda.synchronize()
            raise RuntimeError("the energy accumulator did not advance")
    torch.cuda.synchronize()
    (e0, ts0, h0), (e1, ts1, h1) = marks[0], marks[1]
    dt = h1 - h0
    if ts1 > ts0:
        # the accumulator's timestamp: pick the power of ten that matches
        # the host clock
        import math
        unit = 10.0 ** round(math.log10((ts1 - ts0) / dt))
        if abs((ts1 - ts0) / unit - dt) < 0.2 * dt:
            dt = (ts1 - ts0) / unit
    watts = (e1 - e0) / dt
    measure.last = {"window_s": dt, "steps": steps}
    return sec, watts * sec, watts
