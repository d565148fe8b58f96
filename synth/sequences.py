"""Excitation trains (flip angles alpha_t, RF phases) of the synthetic workloads."""
from __future__ import annotations

import numpy as np

from . import rng


def fisp_train(L: int) -> np.ndarray:
    """alpha_t = 10 + 50 |sin(pi t / 125)| degrees, t = 1..L (64x64 FISP workload)."""
    t = np.arange(1, L + 1, dtype=np.float64)
    return 10.0 + 50.0 * np.abs(np.sin(np.pi * t / 125.0))


def halfsine_train(L: int, seed: int, period: int = 250, gap: int = 50,
                   peaks=(60.0, 30.0), noise_std: float = 5.0) -> np.ndarray:
    """The pseudo-random IR-bSSFP flip-angle pattern of the phantom experiment
    (Section "Numerical Brainweb phantom", its footnote): half-sine lobes of
    ``period`` TRs whose peaks alternate 60/30 degrees, each followed by
    ``gap`` TRs without excitation, plus zero-mean uniform noise of standard
    deviation ``noise_std`` degrees on the lobes, truncated to L."""
    cyc = period + gap
    t0 = np.arange(L)
    c = t0 // cyc
    u = t0 % cyc + 1                       # 1..cyc within a cycle
    amp = np.where(c % 2 == 0, peaks[0], peaks[1])
    lobe = u <= period
    alpha = np.where(lobe, amp * np.sin(np.pi * u / period), 0.0)
    half_width = noise_std * np.sqrt(3.0)  # U(-a, a) has std a / sqrt(3)
    noise = rng.uniform(seed, "fa-noise", L, -half_width, half_width)
    return np.where(lobe, alpha + noise, 0.0)


def alternating_phase(L: int) -> np.ndarray:
    """RF phase 0, pi, 0, pi, ... (balanced SSFP phase cycling)."""
    return np.pi * (np.arange(L) % 2).astype(np.float64)
