"""GPU energy over a timed region, from the device's accumulated-energy counter and
sampled socket power (AMD SMI). Measurement only; nothing here touches the GPU's
settings.

    meter = EnergyMeter()          # the device torch calls cuda:0
    meter.start(); ...; rec = meter.stop()
    rec["joules"], rec["avg_power_w"], rec["samples"]

If the SMI library is missing or refuses the queries, `EnergyMeter.available` is
False and `stop()` returns None fields with the reason.
"""
from __future__ import annotations

import threading
import time


def joules_from_counter(acc0: int, acc1: int, resolution_uj: float, bits: int = 64) -> float:
    """Energy between two readings of a wrapping accumulator counting in units of
    `resolution_uj` microjoules."""
    d = (acc1 - acc0) % (1 << bits)
    return d * resolution_uj * 1e-6


def mean_power(samples) -> float | None:
    """Time-weighted mean of (t_seconds, watts) samples (trapezoid rule); the plain
    mean when all samples share one time."""
    s = sorted(samples)
    if not s:
        return None
    if len(s) == 1 or s[-1][0] == s[0][0]:
        return sum(w for _, w in s) / len(s)
    area = sum((t1 - t0) * (w0 + w1) / 2 for (t0, w0), (t1, w1) in zip(s, s[1:]))
    return area / (s[-1][0] - s[0][0])


class EnergyMeter:
    def __init__(self, torch_device: int = 0, period_s: float = 0.02):
        self.period = period_s
        self.available = False
        self.reason = None
        self._h = None
        self._smi = None
        try:
            import amdsmi
            import torch
            amdsmi.amdsmi_init()
            self._smi = amdsmi
            props = torch.cuda.get_device_properties(torch_device)
            want = (getattr(props, "pci_domain_id", 0), getattr(props, "pci_bus_id", None),
                    getattr(props, "pci_device_id", None))
            handles = amdsmi.amdsmi_get_processor_handles()
            pick = None
            for h in handles:
                bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)  # "dddd:bb:dd.f"
                dom, bus, rest = bdf.split(":")
                dev = rest.split(".")[0]
                if want[1] is not None and (int(dom, 16), int(bus, 16), int(dev, 16)) == want:
                    pick = h
                    break
            if pick is None and len(handles) == 1:
                pick = handles[0]
            if pick is None:
                raise RuntimeError(f"no SMI device matches PCI {want}")
            self._h = pick
            self._read_counter()
            self.available = True
        except Exception as e:  # noqa: BLE001 - any SMI failure just disables the meter
            self.reason = f"{type(e).__name__}: {e}"

    def _read_counter(self):
        r = self._smi.amdsmi_get_energy_count(self._h)
        return r["energy_accumulator"], r["counter_resolution"]

    def _read_power(self):
        p = self._smi.amdsmi_get_power_info(self._h)
        w = p.get("current_socket_power")
        if not isinstance(w, (int, float)) or w in (0, "N/A"):
            w = p.get("average_socket_power")
        return float(w) if isinstance(w, (int, float)) else None

    def _sample(self):
        while not self._stop.is_set():
            try:
                w = self._read_power()
                if w is not None:
                    self._samples.append((time.perf_counter(), w))
            except Exception:  # noqa: BLE001
                pass
            self._stop.wait(self.period)

    def start(self):
        if not self.available:
            return
        self._samples = []
        self._stop = threading.Event()
        self._t0 = time.perf_counter()
        self._acc0, self._res = self._read_counter()
        self._thr = threading.Thread(target=self._sample, daemon=True)
        self._thr.start()

    def close(self):
        if self._smi is not None:
            try:
                self._smi.amdsmi_shut_down()
            except Exception:  # noqa: BLE001
                pass
            self._smi = None
            self.available = False

    def stop(self):
        if not self.available:
            return {"joules": None, "avg_power_w": None, "samples": 0, "reason": self.reason}
        acc1, res = self._read_counter()
        t1 = time.perf_counter()
        self._stop.set()
        self._thr.join()
        joules = joules_from_counter(self._acc0, acc1, res)
        return {"joules": joules, "seconds": t1 - self._t0,
                "avg_power_w": joules / (t1 - self._t0) if t1 > self._t0 else None,
                "sampled_power_w": mean_power(self._samples), "samples": len(self._samples),
                "counter_resolution_uj": res}
