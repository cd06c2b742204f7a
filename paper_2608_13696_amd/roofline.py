"""Instruction roofline arithmetic (Section 2.2, Table 2 of the paper).

The paper's instruction throughput is N_SM x N_SMSP-per-SM x measured clock,
in warp instructions per second; its ridge is that throughput divided by the
DRAM sector rate (bandwidth / 32 B sectors). On CDNA4 the analogue of an SMSP
issue slot is one VALU wave64 instruction per CU per clock, so the VALU issue
ceiling is N_CU x 1 x clock.
"""
from __future__ import annotations

from dataclasses import dataclass

SECTOR_BYTES = 32


def inst_throughput(n_units: int, issue_per_unit: int, clock_hz: float) -> float:
    """Instructions per second with every unit issuing every clock."""
    return float(n_units) * float(issue_per_unit) * float(clock_hz)


def ridge_per_sector(inst_per_s: float, bytes_per_s: float, sector_bytes: int = SECTOR_BYTES) -> float:
    """Instructions per DRAM sector at which the two rooflines meet."""
    return inst_per_s / (bytes_per_s / sector_bytes)


def ridge_per_byte(inst_per_s: float, bytes_per_s: float) -> float:
    return inst_per_s / bytes_per_s


@dataclass(frozen=True)
class Device:
    name: str
    n_units: int
    issue_per_unit: int
    clock_hz: float
    hbm_bytes_per_s: float

    @property
    def inst_per_s(self) -> float:
        return inst_throughput(self.n_units, self.issue_per_unit, self.clock_hz)

    @property
    def ridge_sector(self) -> float:
        return ridge_per_sector(self.inst_per_s, self.hbm_bytes_per_s)

    @property
    def ridge_byte(self) -> float:
        return ridge_per_byte(self.inst_per_s, self.hbm_bytes_per_s)

    def attainable_inst_per_s(self, inst_per_byte: float) -> float:
        """Roofline: min(issue ceiling, intensity x bandwidth)."""
        return min(self.inst_per_s, inst_per_byte * self.hbm_bytes_per_s)


# The two GPUs of Table 2 (clock is the measured SM clock).
L4 = Device("L4", 58, 4, 1.78e9, 300e9)
GH200 = Device("GH200", 132, 4, 1.96e9, 4022e9)

# MI355X vendor figures: 256 CUs, 2.4 GHz peak engine clock, 8 TB/s HBM3E.
MI355X_HBM_PEAK = 8.0e12
MI355X = Device("MI355X", 256, 1, 2.4e9, MI355X_HBM_PEAK)


def mi355x(clock_hz: float | None = None) -> Device:
    """MI355X roofline at a measured clock (defaults to the 2.4 GHz peak)."""
    return Device("MI355X", 256, 1, clock_hz or 2.4e9, MI355X_HBM_PEAK)


def fractions(bytes_moved: float, valu_wave_insts: float, seconds: float, dev: Device = MI355X) -> dict:
    """HBM and VALU fractions of one kernel or pipeline, and the binding one."""
    hbm = bytes_moved / seconds / dev.hbm_bytes_per_s if seconds > 0 else 0.0
    valu = valu_wave_insts / seconds / dev.inst_per_s if seconds > 0 else 0.0
    return {"hbm_frac": hbm, "valu_frac": valu, "binding": "hbm" if hbm >= valu else "valu",
            "binding_frac": max(hbm, valu),
            "intensity_inst_per_byte": (valu_wave_insts / bytes_moved) if bytes_moved > 0 else 0.0}
