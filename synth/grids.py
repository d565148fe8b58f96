"""Parameter grids of the fingerprint dictionary (the discretised parameter
space of Section "Bloch dynamic model", eq. fingerprints).

Atoms are enumerated row-major over the grid with the LAST parameter varying
fastest, so a grid point (i_0, ..., i_{P-1}) has atom index
sum_k i_k * prod_{l>k} N_l.  The optional T2 < T1 filter drops physically
implausible pairs (the in-vivo grid of Section "In-vivo data" only reaches
its printed atom count with it); a filtered grid is no longer a box, so the
learned-proposal path needs the unfiltered grid.
"""
from __future__ import annotations

import numpy as np


def log_grid(tmin: float, tmax: float, n: int) -> np.ndarray:
    """n points geometrically spaced from tmin to tmax inclusive."""
    if n == 1:
        return np.array([float(tmin)])
    k = np.arange(n, dtype=np.float64)
    return tmin * (tmax / tmin) ** (k / (n - 1))


def lin_grid(a: float, b: float, n: int) -> np.ndarray:
    """n points linearly spaced from a to b inclusive."""
    return np.linspace(float(a), float(b), int(n))


def colon(a: float, step: float, b: float) -> np.ndarray:
    """The range a:step:b of the paper's grid notation (b included if hit)."""
    n = int(np.floor((b - a) / step + 1e-9)) + 1
    return a + step * np.arange(n, dtype=np.float64)


def brainweb_axes():
    """T1, T2, B0 axes of the phantom experiment's dictionary (Section
    "Numerical Brainweb phantom"), in ms, ms and Hz."""
    t1 = np.concatenate([colon(100, 40, 2000), colon(2200, 200, 6000)])
    t2 = np.concatenate([colon(20, 2, 100), colon(110, 4, 200), colon(220, 20, 600)])
    b0 = np.concatenate([colon(-250, 40, -190), colon(-50, 2, 50), colon(190, 40, 250)])
    return t1, t2, b0


def invivo_axes():
    """T1, T2, B0 axes of the in-vivo dictionary (Section "In-vivo data")."""
    t1 = np.concatenate([colon(100, 20, 2000), colon(2300, 300, 5000)])
    t2 = np.concatenate([colon(20, 5, 100), colon(110, 10, 200), colon(300, 200, 1900)])
    b0 = np.concatenate([colon(-250, 20, -190), colon(-50, 1, 50), colon(190, 20, 250)])
    return t1, t2, b0


def product_grid(axes, t2_lt_t1: bool = False, t1_axis: int = 0, t2_axis: int = 1,
                 inclusive: bool = False) -> np.ndarray:
    """All combinations of the axes, row-major (last axis fastest).

    Returns params[d][P].  With ``t2_lt_t1`` the rows with T2 >= T1 (or
    T2 > T1 when ``inclusive``) are removed, keeping the order.
    """
    mesh = np.meshgrid(*[np.asarray(a, dtype=np.float64) for a in axes], indexing="ij")
    params = np.stack([m.reshape(-1) for m in mesh], axis=1)
    if t2_lt_t1:
        t1 = params[:, t1_axis]
        t2 = params[:, t2_axis]
        keep = (t2 <= t1) if inclusive else (t2 < t1)
        params = params[keep]
    return params


def grid_index(sub: np.ndarray, dims) -> np.ndarray:
    """Row-major atom index of integer grid coordinates sub[..., P]."""
    sub = np.asarray(sub, dtype=np.int64)
    idx = np.zeros(sub.shape[:-1], dtype=np.int64)
    for k, n in enumerate(dims):
        idx = idx * int(n) + sub[..., k]
    return idx


def grid_sub(idx: np.ndarray, dims) -> np.ndarray:
    """Inverse of grid_index: integer grid coordinates of atom indices."""
    idx = np.asarray(idx, dtype=np.int64)
    out = np.zeros(idx.shape + (len(dims),), dtype=np.int64)
    rem = idx.copy()
    for k in range(len(dims) - 1, -1, -1):
        out[..., k] = rem % int(dims[k])
        rem //= int(dims[k])
    return out
