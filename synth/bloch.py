"""Discrete-time Bloch responses B(Theta; TR, TE, alpha) of eq. fingerprints.

Two sequences are simulated in FP64, vectorised over parameter sets:

* IR-FISP by the extended phase graph (EPG) formalism (Weigel, "Extended
  phase graphs: dephasing, RF pulses, and echoes - pure and simple",
  JMRI 2015).  Each TR: RF pulse (phase 0) -> relaxation over TE -> read F+_0
  -> relaxation over TR-TE -> one unit of gradient dephasing.  With RF phase 0
  the echo F+_0 is purely imaginary; the atom is its imaginary part (real).
* IR-bSSFP as a single isochromat with off-resonance df: RF pulse about an
  axis at phase phi_t in the transverse plane -> free precession and
  relaxation over TE -> read (Mx + i My) * exp(-i phi_t) -> free precession
  and relaxation over TR-TE.  B1 multiplies every flip angle.

Both start from an ideal inversion (Mz = -1) followed by relaxation over TI.
Units: times in ms, off-resonance in Hz, flip angles in degrees.

Rotation convention (shared by both): a pulse of angle a about +x maps
My' = My cos a - Mz sin a and Mz' = My sin a + Mz cos a; free precession
multiplies Mx + i My by exp(-i 2 pi df t).
"""
from __future__ import annotations

import numpy as np


def _relax_factors(tau, T1, T2):
    return np.exp(-tau / T1), np.exp(-tau / T2)


def fisp_epg(T1, T2, alpha_deg, TR: float, TE: float, TI: float,
             return_mz_end: bool = False):
    """IR-FISP fingerprints by EPG.

    T1, T2: arrays [d] (ms).  alpha_deg: [L] flip angles.
    Returns atoms [d][L] (real, FP64) and, if asked, Z_0 at the end of each
    TR (the longitudinal magnetisation, [d][L]).
    """
    T1 = np.atleast_1d(np.asarray(T1, dtype=np.float64))
    T2 = np.atleast_1d(np.asarray(T2, dtype=np.float64))
    alpha = np.deg2rad(np.asarray(alpha_deg, dtype=np.float64))
    d, L = T1.size, alpha.size
    K = L + 1
    Fp = np.zeros((d, K), dtype=np.complex128)
    Fm = np.zeros((d, K), dtype=np.complex128)
    Zs = np.zeros((d, K), dtype=np.complex128)
    # ideal inversion, then recovery over TI
    e1, _ = _relax_factors(TI, T1, T2)
    Zs[:, 0] = -1.0 * e1 + (1.0 - e1)
    e1_te, e2_te = _relax_factors(TE, T1, T2)
    e1_rest, e2_rest = _relax_factors(TR - TE, T1, T2)
    out = np.zeros((d, L), dtype=np.float64)
    mz_end = np.zeros((d, L), dtype=np.float64) if return_mz_end else None
    max_imag_re = 0.0
    for t in range(L):
        a = alpha[t]
        c2, s2 = np.cos(a / 2) ** 2, np.sin(a / 2) ** 2
        sa, ca = np.sin(a), np.cos(a)
        Fp, Fm, Zs = (c2 * Fp + s2 * Fm - 1j * sa * Zs,
                      s2 * Fp + c2 * Fm + 1j * sa * Zs,
                      -0.5j * sa * Fp + 0.5j * sa * Fm + ca * Zs)
        # relaxation over TE
        Fp *= e2_te[:, None]
        Fm *= e2_te[:, None]
        Zs[:, 1:] *= e1_te[:, None]
        Zs[:, 0] = Zs[:, 0] * e1_te + (1.0 - e1_te)
        echo = Fp[:, 0]
        max_imag_re = max(max_imag_re, float(np.max(np.abs(echo.real))))
        out[:, t] = echo.imag
        # relaxation over the rest of the TR
        Fp *= e2_rest[:, None]
        Fm *= e2_rest[:, None]
        Zs[:, 1:] *= e1_rest[:, None]
        Zs[:, 0] = Zs[:, 0] * e1_rest + (1.0 - e1_rest)
        if return_mz_end:
            mz_end[:, t] = Zs[:, 0].real
        # one unit of dephasing: F+ orders move up, F- orders move down
        Fp = np.concatenate([np.zeros((d, 1), dtype=np.complex128), Fp[:, :-1]], axis=1)
        Fm = np.concatenate([Fm[:, 1:], np.zeros((d, 1), dtype=np.complex128)], axis=1)
        Fp[:, 0] = np.conj(Fm[:, 0])
    fisp_epg.last_max_abs_real = max_imag_re
    if return_mz_end:
        return out, mz_end
    return out


def bssfp(T1, T2, df, alpha_deg, phase_rad, TR: float, TE: float, TI: float,
          B1=None, return_state: bool = False):
    """IR-bSSFP fingerprints of a single isochromat.

    T1, T2, df (and B1): arrays [d].  alpha_deg, phase_rad: [L].
    Returns complex atoms [d][L] (FP64).
    """
    T1 = np.atleast_1d(np.asarray(T1, dtype=np.float64))
    T2 = np.atleast_1d(np.asarray(T2, dtype=np.float64))
    df = np.atleast_1d(np.asarray(df, dtype=np.float64))
    d = T1.size
    B1 = np.ones(d) if B1 is None else np.atleast_1d(np.asarray(B1, dtype=np.float64))
    alpha = np.deg2rad(np.asarray(alpha_deg, dtype=np.float64))
    phase = np.asarray(phase_rad, dtype=np.float64)
    L = alpha.size
    m = np.zeros(d, dtype=np.complex128)      # Mx + i My
    e1_ti, _ = _relax_factors(TI, T1, T2)
    mz = -1.0 * e1_ti + (1.0 - e1_ti)
    e1_te, e2_te = _relax_factors(TE, T1, T2)
    e1_rest, e2_rest = _relax_factors(TR - TE, T1, T2)
    p_te = np.exp(-2j * np.pi * df * TE * 1e-3)
    p_rest = np.exp(-2j * np.pi * df * (TR - TE) * 1e-3)
    out = np.zeros((d, L), dtype=np.complex128)
    for t in range(L):
        a = B1 * alpha[t]
        rot = np.exp(-1j * phase[t])
        # move to the pulse frame, rotate about x, move back
        mr = m * rot
        mx, my = mr.real, mr.imag
        ca, sa = np.cos(a), np.sin(a)
        my2 = my * ca - mz * sa
        mz = my * sa + mz * ca
        m = (mx + 1j * my2) * np.conj(rot)
        # free precession and relaxation over TE
        m = m * p_te * e2_te
        mz = mz * e1_te + (1.0 - e1_te)
        out[:, t] = m * rot
        # rest of the TR
        m = m * p_rest * e2_rest
        mz = mz * e1_rest + (1.0 - e1_rest)
    if return_state:
        return out, (m, mz)
    return out


def _bssfp_rows(p, alpha_deg, phase_rad, TR, TE, TI, has_b1):
    if has_b1:
        return bssfp(p[:, 0], p[:, 1], p[:, 3], alpha_deg, phase_rad, TR, TE, TI, B1=p[:, 2])
    return bssfp(p[:, 0], p[:, 1], p[:, 2], alpha_deg, phase_rad, TR, TE, TI)


def _bssfp_chunk_job(args):
    p, alpha_deg, phase_rad, TR, TE, TI, has_b1, dtype = args
    return _bssfp_rows(p, alpha_deg, phase_rad, TR, TE, TI, has_b1).astype(dtype)


def bssfp_chunked(params: np.ndarray, alpha_deg, phase_rad, TR, TE, TI,
                  has_b1: bool = False, chunk: int = 65536, dtype=np.complex128, workers: int = 1):
    """bssfp over a params table [d][P] (T1, T2, [B1,] df), in atom chunks;
    workers > 1 computes the chunks in forked processes (the same values: each
    atom's recursion is independent of the chunking)."""
    d = params.shape[0]
    L = len(alpha_deg)
    out = np.empty((d, L), dtype=dtype)
    starts = list(range(0, d, chunk))
    if workers > 1 and len(starts) > 1:
        import multiprocessing
        jobs = [(params[s:s + chunk], alpha_deg, phase_rad, TR, TE, TI, has_b1, dtype) for s in starts]
        with multiprocessing.get_context("fork").Pool(min(workers, len(starts))) as pool:
            for s, rows in zip(starts, pool.imap(_bssfp_chunk_job, jobs)):
                out[s:s + chunk] = rows
        return out
    for s in starts:
        out[s:s + chunk] = _bssfp_rows(params[s:s + chunk], alpha_deg, phase_rad, TR, TE, TI, has_b1)
    return out
