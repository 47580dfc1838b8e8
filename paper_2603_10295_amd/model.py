"""Host-side accounting: memory footprint and operation counts of the path.

Counts are in complex multiply-adds (cMAC); one cMAC is 8 real flops.  The
paper's own counts are Eq. (8) (single loop) and Eq. (11) (nested loop); the
nested-loop form implemented here differs in two places:

* the band rotation of one (k, q) pair costs 2 Nw^3 Nm cMAC (two Nw x Nw
  matrix products per mode), not the 2 Nb^2 Nm printed in Eqs. (8) and (11);
* the mode rotation is applied once per q to g(Re, q), where it costs
  Ne Nw^2 Nm^2, instead of once per (k, q) pair.
"""
from __future__ import annotations

import dataclasses


def g_bytes(nw: int, nm: int, ne: int, np_: int, elem_bytes: int = 16) -> int:
    """Size of g(Re,Rp): 16 Nb^2 Nm Ne Np bytes for complex128 (Table 3)."""
    return elem_bytes * nw * nw * nm * ne * np_


def single_loop_cmul(nw, nm, ne, np_, nk, nq) -> float:
    """Eq. (8) as printed (complex multiplications)."""
    return (nw * nw * nm * ne * np_ + nw * nw * nm * ne + 2 * nw * nw * nm + nw * nw * nm * nm) * nk * nq


def nested_loop_cmul(nw, nm, ne, np_, nk, nq) -> float:
    """Eq. (11) as printed (complex multiplications)."""
    return nw * nw * nm * ne * np_ * nq + (nw * nw * nm * ne + 2 * nw * nw * nm + nw * nw * nm * nm) * nk * nq


def nested_over_single(nw, nm, ne, np_, nk) -> float:
    """Eq. (12): T_NL / T_SL ~ 1/Nk + (1 + 2/Ne + Nm/Ne) / Np."""
    return 1.0 / nk + (1.0 + 2.0 / ne + nm / ne) / np_


@dataclasses.dataclass
class StageCounts:
    """Algorithmic cMAC of each stage of one interpolation call."""
    rp: float          # Eq. (9): Nq Ne Np Nw^2 Nm
    modes: float       # u(q) applied to g(Re,q): Nq Ne Nw^2 Nm^2
    re: float          # Eq. (10) Re sum: Nk Nq Ne Nw^2 Nm
    rot: float         # V(k+q)^dagger g V(k): Nk Nq 2 Nw^3 Nm
    hkq: float         # H(k+q) interpolation when k+q is not on the k grid: Nk Nq Nh Nw^2
    elems: float       # outputs: Nk Nq Nw^2 Nm

    @property
    def gemm(self) -> float:
        """cMAC of the two phase GEMMs (Eqs. (9) and (10))."""
        return self.rp + self.re

    @property
    def total(self) -> float:
        return self.rp + self.modes + self.re + self.rot + self.hkq


def stage_counts(nw: int, nm: int, ne: int, np_: int, nk: int, nq: int, nh: int = 0,
                 kq_on_grid: bool = True) -> StageCounts:
    e = nw * nw * nm
    return StageCounts(
        rp=float(nq) * ne * np_ * e,
        modes=float(nq) * ne * nw * nw * nm * nm,
        re=float(nk) * nq * ne * e,
        rot=float(nk) * nq * 2 * nw ** 3 * nm,
        hkq=0.0 if kq_on_grid else float(nk) * nq * nh * nw * nw,
        elems=float(nk) * nq * e,
    )


# MI355X published peaks (dense)
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
