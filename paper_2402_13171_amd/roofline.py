"""Roofline arithmetic of the lattice-Boltzmann update (Sec. 4.3 of the paper:
machine balance, code balance, "lightspeed" and the bandwidth-bound maximum
performance P_max = b_S / n_b)."""
from __future__ import annotations

Q = 27
HBM_PEAK_BPS = 8.0e12          # MI355X HBM3E, published peak
FP32_VALU_PEAK = 157.3e12      # MI355X FP32 vector, published peak


def bytes_per_lup(storage_bytes: int, force_components: int = 0,
                  force_bytes: int = 4) -> int:
    """Algorithmic bytes per lattice update: every population read once and
    written once, plus an optional force vector read."""
    return 2 * Q * storage_bytes + force_components * force_bytes


def p_max_lups(bandwidth_bps: float, n_b: float) -> float:
    """Bandwidth-bound maximum update rate (lattice updates per second)."""
    return bandwidth_bps / n_b


def lightspeed(bandwidth_bps: float, n_f: float, peak_flops: float, n_b: float) -> float:
    """l = min(1, B_m / B_c) with machine balance B_m = b_S / P_peak and code
    balance B_c = n_b / n_f; l < 1 means the kernel is memory bound."""
    return min(1.0, (bandwidth_bps / peak_flops) / (n_b / n_f))


def fraction_of_pmax(measured_lups: float, bandwidth_bps: float, n_b: float) -> float:
    return measured_lups / p_max_lups(bandwidth_bps, n_b)


def achieved_bandwidth(lups: float, n_b: float) -> float:
    """Algorithmic bytes per second at a given update rate."""
    return lups * n_b
