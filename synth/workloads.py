"""Seeded synthetic workloads standing in for the paper's datasets.

The phantom and in-vivo data of the paper's experiments are not available;
these generators produce inputs with the same shapes, sequences and
sampling structure (recipes listed per function).  All randomness comes from
``synth.rng`` keyed by (seed, purpose tag).

Conventions shared with the library:
* images are frame-major complex arrays [S][L][ny][nx] (slice, frame, row,
  column); voxel v = s*ny*nx + y*nx + x;
* k-space indices are flat ky*nx + kx in unshifted FFT order (frequency 0
  at index 0, negative frequencies wrapped to the top);
* the sampling pattern is CSR over (slice, frame) pairs in order s*L + t:
  samples of pair p are idx[off[p]:off[p+1]], unique within the pair.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import bloch, grids, rng, sequences


# ----------------------------------------------------------------------------
# dictionaries
# ----------------------------------------------------------------------------
@dataclass
class Dictionary:
    atoms: np.ndarray            # [d][L] float64 (real) or complex128
    params: np.ndarray           # [d][P] float64: T1, T2[, B1][, df]
    grid_dims: tuple | None      # per-parameter sizes (None if filtered)
    axes: list                   # per-parameter grid values
    names: tuple                 # parameter names
    seq: dict = field(default_factory=dict)

    @property
    def d(self):
        return self.atoms.shape[0]

    @property
    def L(self):
        return self.atoms.shape[1]

    @property
    def is_complex(self):
        return np.iscomplexobj(self.atoms)


def fisp_dictionary(L: int = 100, n_t1: int = 40, n_t2: int = 50,
                    t1_range=(100.0, 4000.0), t2_range=(10.0, 600.0),
                    t2_lt_t1: bool = False, TR=10.0, TE=5.0, TI=10.0) -> Dictionary:
    """Real IR-FISP dictionary on a log-spaced (T1, T2) grid (64x64 workload:
    L=100, 40 x 50 = 2,000 atoms)."""
    t1 = grids.log_grid(*t1_range, n_t1)
    t2 = grids.log_grid(*t2_range, n_t2)
    params = grids.product_grid([t1, t2], t2_lt_t1=t2_lt_t1)
    alpha = sequences.fisp_train(L)
    atoms = bloch.fisp_epg(params[:, 0], params[:, 1], alpha, TR, TE, TI)
    dims = None if t2_lt_t1 else (n_t1, n_t2)
    return Dictionary(atoms, params, dims, [t1, t2], ("T1", "T2"),
                      dict(kind="fisp", alpha=alpha, TR=TR, TE=TE, TI=TI))


def bssfp_dictionary(L: int = 500, n_t1: int = 60, n_t2: int = 60, n_df: int = 28,
                     t1_range=(100.0, 4000.0), t2_range=(10.0, 600.0),
                     df_range=(-40.0, 40.0), b1_axis=None, seed: int = 2,
                     t2_lt_t1: bool = False, TR=10.0, TE=5.0, TI=10.0,
                     dtype=np.complex128, workers: int = 1) -> Dictionary:
    """Complex IR-bSSFP dictionary on T1 x T2 [x B1] x df (256x256 workload:
    L=500, 60 x 60 x 28 = 100,800 atoms)."""
    t1 = grids.log_grid(*t1_range, n_t1)
    t2 = grids.log_grid(*t2_range, n_t2)
    df = grids.lin_grid(*df_range, n_df)
    axes = [t1, t2] + ([np.asarray(b1_axis, dtype=np.float64)] if b1_axis is not None else []) + [df]
    names = ("T1", "T2") + (("B1",) if b1_axis is not None else ()) + ("df",)
    params = grids.product_grid(axes, t2_lt_t1=t2_lt_t1)
    alpha = sequences.halfsine_train(L, seed)
    phase = sequences.alternating_phase(L)
    atoms = bloch.bssfp_chunked(params, alpha, phase, TR, TE, TI,
                                has_b1=b1_axis is not None, dtype=dtype, workers=workers)
    dims = None if t2_lt_t1 else tuple(len(a) for a in axes)
    return Dictionary(atoms, params, dims, axes, names,
                      dict(kind="bssfp", alpha=alpha, phase=phase, TR=TR, TE=TE, TI=TI))


# ----------------------------------------------------------------------------
# voxel sets and phantoms
# ----------------------------------------------------------------------------
def random_voxels(D: Dictionary, n: int, seed: int = 2, pd_range=(0.3, 1.0),
                  snr_db_range=(20.0, 40.0)):
    """Voxels drawn as random atoms scaled by PD plus complex Gaussian noise at
    a per-voxel SNR (standalone matched-filter workload).

    Returns (Z [n][L] complex128, true_idx [n], pd [n], snr_db [n]).
    Per-voxel noise: E|xi|^2 per entry = (||x_v||^2 / L) 10^(-SNR/10).
    """
    j = rng.randint(seed, "vox-atom", n, D.d)
    pd = rng.uniform(seed, "vox-pd", n, *pd_range)
    snr = rng.uniform(seed, "vox-snr", n, *snr_db_range)
    x = pd[:, None] * D.atoms[j]
    sig2 = np.sum(np.abs(x) ** 2, axis=1) / D.L * 10.0 ** (-snr / 10.0)
    noise = rng.complex_gaussian(seed, "vox-noise", (n, D.L), sig2[:, None])
    return x + noise, j, pd, snr


@dataclass
class Phantom:
    X0: np.ndarray          # [S][L][ny][nx] complex128 ground-truth image
    idx: np.ndarray         # [n] generating atom index (-1: background)
    pd: np.ndarray          # [n] proton density (0: background)
    params: np.ndarray      # [n][P] true parameters (NaN: background)
    S: int
    ny: int
    nx: int


def _to_frame_major(vox: np.ndarray, S: int, ny: int, nx: int) -> np.ndarray:
    L = vox.shape[1]
    return np.ascontiguousarray(vox.reshape(S, ny, nx, L).transpose(0, 3, 1, 2))


def disc_phantom(D: Dictionary, seed: int = 1, size: int = 64, radius: float = 28.0,
                 classes=((800.0, 50.0), (1200.0, 80.0), (1800.0, 150.0), (4000.0, 2000.0)),
                 pd_range=(0.5, 1.0), snap: bool = True) -> Phantom:
    """Disc phantom with four angular-quadrant tissue classes (64x64 workload).

    With ``snap`` each class takes the grid atom nearest (log distance) to its
    (T1, T2), so noiseless voxels lie exactly in cone(D); otherwise the
    signatures are simulated at the true, off-grid parameters.
    """
    yy, xx = np.mgrid[0:size, 0:size].astype(np.float64)
    cy = cx = (size - 1) / 2.0
    r = np.hypot(yy - cy, xx - cx)
    ang = np.arctan2(yy - cy, xx - cx)
    quad = ((ang + np.pi) // (np.pi / 2)).astype(np.int64) % 4
    inside = r <= radius
    n = size * size
    pd = np.zeros(n)
    pd_all = rng.uniform(seed, "phantom-pd", n, *pd_range)
    pd[inside.reshape(-1)] = pd_all[inside.reshape(-1)]
    idx = np.full(n, -1, dtype=np.int64)
    params = np.full((n, 2), np.nan)
    vox = np.zeros((n, D.L), dtype=np.complex128)
    cls = np.asarray(classes, dtype=np.float64)
    for c in range(len(cls)):
        sel = (inside & (quad == c)).reshape(-1)
        if snap:
            dist = (np.log(D.params[:, 0] / cls[c, 0]) ** 2 + np.log(D.params[:, 1] / cls[c, 1]) ** 2)
            j = int(np.argmin(dist))
            idx[sel] = j
            params[sel] = D.params[j, :2]
            sig = D.atoms[j]
        else:
            params[sel] = cls[c]
            sig = bloch.fisp_epg([cls[c, 0]], [cls[c, 1]], D.seq["alpha"], D.seq["TR"],
                                 D.seq["TE"], D.seq["TI"])[0]
        vox[sel] = pd[sel, None] * sig[None, :]
    return Phantom(_to_frame_major(vox, 1, size, size), idx, pd, params, 1, size, size)


def _smooth_field(seed: int, tag: str, S: int, ny: int, nx: int, width: float) -> np.ndarray:
    """Gaussian-filtered white noise, [S][ny][nx], zero mean, unit std."""
    g = rng.normal(seed, tag, S * ny * nx).reshape(S, ny, nx)
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (np.pi * width) ** 2 * (kx ** 2 + ky ** 2))
    f = np.real(np.fft.ifft2(np.fft.fft2(g) * filt))
    f -= f.mean(axis=(1, 2), keepdims=True)
    f /= f.std(axis=(1, 2), keepdims=True) + 1e-30
    return f


def smooth_phantom(D: Dictionary, seed: int = 4, S: int = 8, size: int = 256,
                   n_tissue: int = 6, pd_range=(0.3, 1.0), dtype=np.complex128) -> Phantom:
    """Multi-slice phantom on grid atoms (multi-slice IPG workloads).

    Per slice: an elliptical head region split into ``n_tissue`` smooth random
    regions, each with one (T1, T2[, B1]) grid point; a smooth linear df ramp
    across the slice snapped to the df grid; a smooth PD in pd_range.
    Background voxels are zero.
    """
    dims = D.grid_dims
    assert dims is not None, "smooth_phantom needs an unfiltered grid"
    P = len(dims)
    n_sl = size * size
    n = S * n_sl
    # tissue labels: argmax of n_tissue smooth fields
    fields = np.stack([_smooth_field(seed, f"label{k}", S, size, size, size / 12.0)
                       for k in range(n_tissue)], axis=0)
    label = np.argmax(fields, axis=0).reshape(-1)
    yy, xx = np.mgrid[0:size, 0:size].astype(np.float64)
    c = (size - 1) / 2.0
    head = (((yy - c) / (0.45 * size)) ** 2 + ((xx - c) / (0.38 * size)) ** 2 <= 1.0).reshape(-1)
    head = np.tile(head, S)
    # per-tissue grid coordinates for every axis but the last (df)
    tis = np.stack([rng.randint(seed, f"tissue-axis{k}", n_tissue, dims[k]) for k in range(P - 1)], axis=1)
    # df: smooth ramp over the slice, snapped to the df grid
    ramp_dir = rng.uniform(seed, "ramp-dir", S, 0.0, 2.0 * np.pi)
    ramp = (np.cos(ramp_dir)[:, None, None] * (xx - c)[None] + np.sin(ramp_dir)[:, None, None] * (yy - c)[None])
    ramp = ramp / (np.abs(ramp).max(axis=(1, 2), keepdims=True) + 1e-30)
    df_sub = np.clip(np.rint((ramp.reshape(-1) + 1.0) / 2.0 * (dims[-1] - 1)), 0, dims[-1] - 1).astype(np.int64)
    sub = np.concatenate([tis[label], df_sub[:, None]], axis=1)
    idx = grids.grid_index(sub, dims)
    pdf = _smooth_field(seed, "pd", S, size, size, size / 16.0).reshape(-1)
    pd = pd_range[0] + (pd_range[1] - pd_range[0]) * (0.5 + 0.5 * np.tanh(pdf))
    pd = np.where(head, pd, 0.0)
    idx = np.where(head, idx, -1)
    params = np.where(head[:, None], D.params[np.maximum(idx, 0)], np.nan)
    vox = np.zeros((n, D.L), dtype=dtype)
    sel = head
    vox[sel] = pd[sel, None] * D.atoms[idx[sel]]
    return Phantom(_to_frame_major(vox, S, size, size), idx, pd, params, S, size, size)


# ----------------------------------------------------------------------------
# sampling patterns
# ----------------------------------------------------------------------------
@dataclass
class Sampling:
    off: np.ndarray     # [S*L+1] int64 CSR offsets
    idx: np.ndarray     # [M] int32 flat ky*nx+kx (FFT order)
    dcf: np.ndarray | None  # [M] float64 weights or None
    S: int
    L: int
    ny: int
    nx: int

    @property
    def M(self):
        return int(self.off[-1])


def _csr(rows, S, L, ny, nx, dcf=None) -> Sampling:
    off = np.zeros(S * L + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return Sampling(off, idx, dcf, S, L, ny, nx)


def random_lines(seed: int, S: int, L: int, ny: int, nx: int, nlines) -> Sampling:
    """Per (slice, frame): ``nlines`` ky lines drawn uniformly without
    replacement (random Cartesian EPI).  ``nlines`` may be a per-slice list."""
    nl = np.broadcast_to(np.asarray(nlines), (S,))
    rows = []
    for s in range(S):
        for t in range(L):
            perm = rng.permutation(seed, f"lines-s{s}-t{t}", ny)[: int(nl[s])]
            ky = np.sort(perm)
            rows.append((ky[:, None] * nx + np.arange(nx)[None, :]).reshape(-1))
    return _csr(rows, S, L, ny, nx)


def shifted_epi(S: int, L: int, ny: int, nx: int, shots: int = 16) -> Sampling:
    """Multi-shot EPI: ``shots`` uniformly spaced ky lines per frame, shifted
    by one line per frame (the phantom experiment's sampling)."""
    step = ny // shots
    rows = []
    for _s in range(S):
        for t in range(L):
            ky = (np.arange(shots) * step + t) % ny
            ky = np.sort(ky)
            rows.append((ky[:, None] * nx + np.arange(nx)[None, :]).reshape(-1))
    return _csr(rows, S, L, ny, nx)


def _spiral_points(ny: int, nx: int, npts: int, theta: float, turns: float = 8.0,
                   power: float = 2.0) -> np.ndarray:
    """Grid points (centred ky, kx) along a variable-density spiral arm
    k(u) = kmax u^power exp(i(2 pi turns u + theta)), rasterised and
    de-duplicated, then ``npts`` taken evenly along the arm."""
    kmax = min(ny, nx) / 2.0 - 1.0
    u = np.linspace(0.0, 1.0, 200000)
    r = kmax * u ** power
    ph = 2.0 * np.pi * turns * u + theta
    kx = np.rint(r * np.cos(ph)).astype(np.int64)
    ky = np.rint(r * np.sin(ph)).astype(np.int64)
    key = ky * 4 * nx + kx
    _, first = np.unique(key, return_index=True)
    order = np.sort(first)
    pts = np.stack([ky[order], kx[order]], axis=1)
    if len(pts) > npts:
        pick = np.unique(np.rint(np.linspace(0, len(pts) - 1, npts)).astype(np.int64))
        pts = pts[pick]
    return pts


def spiral_sampling(S: int, L: int, ny: int, nx: int, frac: float = 0.05,
                    rot_deg: float = 7.5, with_dcf: bool = True) -> Sampling:
    """Variable-density spiral-like sampling rasterised onto the Cartesian
    grid, one arm per frame rotated by rot_deg per frame (the in-vivo
    readout's rotation), about ``frac`` of k-space per frame, with discrete
    Voronoi density compensation (cell areas within the spiral's disc,
    normalised to mean 1 per frame)."""
    npts = int(round(frac * ny * nx))
    rows, wts = [], []
    yy, xx = np.mgrid[0:ny, 0:nx]
    cy = ((yy + ny // 2) % ny) - ny // 2      # centred coordinate of each FFT-order cell
    cx = ((xx + nx // 2) % nx) - nx // 2
    cells = np.stack([cy.reshape(-1), cx.reshape(-1)], axis=1).astype(np.float64)
    kmax = min(ny, nx) / 2.0 - 1.0
    in_disc = np.hypot(cells[:, 0], cells[:, 1]) <= kmax + 0.5
    for _s in range(S):
        for t in range(L):
            pts = _spiral_points(ny, nx, npts, np.deg2rad(rot_deg) * t)
            flat = (pts[:, 0] % ny) * nx + (pts[:, 1] % nx)
            rows.append(flat)
            if with_dcf:
                c = cells[in_disc]
                d2 = ((c[:, None, :] - pts[None, :, :].astype(np.float64)) ** 2).sum(-1)
                owner = np.argmin(d2, axis=1)
                area = np.bincount(owner, minlength=len(pts)).astype(np.float64)
                area = np.maximum(area, 1.0)
                wts.append(area / area.mean())
    smp = _csr(rows, S, L, ny, nx)
    if with_dcf:
        smp.dcf = np.concatenate(wts)
    return smp


# ----------------------------------------------------------------------------
# measurements
# ----------------------------------------------------------------------------
def pd_phase_map(seed: int, S: int, ny: int, nx: int, max_ramp: float = 2.0) -> np.ndarray:
    """A smooth PD phase map [S][ny][nx] (radians): a seeded constant plus a
    linear ramp of at most ``max_ramp`` radians across the field of view in
    each direction, per slice (complex-PD phantoms: X0 * exp(1j * map))."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    out = np.empty((S, ny, nx))
    for s in range(S):
        u = rng.uniform(seed, f"pdphase-s{s}", 3)
        out[s] = (2.0 * np.pi * (u[0] - 0.5) + max_ramp * (u[1] - 0.5) * 2.0 * yy / ny
                  + max_ramp * (u[2] - 0.5) * 2.0 * xx / nx)
    return out


def coil_maps(seed: int, S: int, c: int, ny: int, nx: int) -> np.ndarray:
    """Smooth synthetic receive-coil sensitivities [S][c][ny][nx] complex128:
    coil q sits on a ring around the field of view (angle 2 pi q / c plus a
    seeded jitter, per slice), with a Gaussian magnitude profile of width
    0.45 FOV and a smooth phase (constant + linear ramp); the maps are
    normalised to unit sum of squares at every pixel (sum_q |S_q|^2 = 1)."""
    yy, xx = np.mgrid[0:ny, 0:nx]
    y = (yy - ny / 2.0) / ny
    x = (xx - nx / 2.0) / nx
    out = np.empty((S, c, ny, nx), dtype=np.complex128)
    for s in range(S):
        u = rng.uniform(seed, f"coils-s{s}", 4 * c).reshape(c, 4)
        for q in range(c):
            ang = 2.0 * np.pi * q / c + 0.3 * (u[q, 0] - 0.5)
            cy, cx = 0.6 * np.sin(ang), 0.6 * np.cos(ang)
            mag = np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2.0 * 0.45 ** 2))
            ph = 2.0 * np.pi * u[q, 1] + 2.0 * (u[q, 2] - 0.5) * y + 2.0 * (u[q, 3] - 0.5) * x
            out[s, q] = mag * np.exp(1j * ph)
        out[s] /= np.sqrt(np.sum(np.abs(out[s]) ** 2, axis=0, keepdims=True))
    return out


@dataclass
class Trajectory:
    """Non-Cartesian sampling: per (slice, frame) pair p the samples
    off[p]..off[p+1] at k-space coordinates coords [M][2] = (ky, kx) in
    cycles per pixel (FP32 values, in [-0.5, 0.5)), with density
    compensation weights dcf [M]."""
    off: np.ndarray
    coords: np.ndarray
    dcf: np.ndarray | None
    S: int
    L: int
    ny: int
    nx: int

    @property
    def M(self):
        return int(self.off[-1])


def _voronoi_areas(pts: np.ndarray, rmax: float) -> np.ndarray:
    """Area of each point's Voronoi cell within the disc of radius rmax
    (bounded by a ring of guard points; vertices outside the disc are pulled
    onto its boundary, an approximate clipping), for density compensation."""
    from scipy.spatial import Voronoi
    ng = 64
    ang = 2.0 * np.pi * np.arange(ng) / ng
    guard = 1.5 * rmax * np.stack([np.sin(ang), np.cos(ang)], axis=1)
    vor = Voronoi(np.concatenate([pts, guard]))
    areas = np.empty(len(pts))
    for i in range(len(pts)):
        reg = vor.regions[vor.point_region[i]]
        poly = vor.vertices[reg]
        # clip the polygon to the disc by pulling vertices outside it onto the circle
        rad = np.hypot(poly[:, 0], poly[:, 1])
        poly = np.where((rad > rmax)[:, None], poly * (rmax / np.maximum(rad, 1e-300))[:, None], poly)
        x, y = poly[:, 1], poly[:, 0]
        areas[i] = 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))
    return areas


def spiral_trajectory(S: int, L: int, ny: int, nx: int, frac: float = 0.05, rot_deg: float = 7.5,
                      turns: float = 8.0, power: float = 2.0, with_dcf: bool = True) -> Trajectory:
    """Variable-density spiral readouts off the Cartesian grid: one arm per
    frame, k(u) = 0.5 u^power exp(i (2 pi turns u + theta_t)) cycles per pixel
    (denser near the centre), theta_t rotating by rot_deg per frame (the
    in-vivo readout's rotation), round(frac * ny * nx) points per arm evenly in
    u (the first one at the centre), coordinates rounded to FP32; Voronoi
    density compensation (cell areas within the sampled disc) normalised to
    mean 1 per frame."""
    npts = max(2, int(round(frac * ny * nx)))
    u = np.linspace(0.0, 1.0, npts, endpoint=False) + 0.5 / npts
    r = 0.5 * u ** power
    rows, wts = [], []
    for _s in range(S):
        for t in range(L):
            ph = 2.0 * np.pi * turns * u + np.deg2rad(rot_deg) * t
            k = np.stack([r * np.sin(ph), r * np.cos(ph)], axis=1).astype(np.float32)
            k = np.where(k >= 0.5, np.float32(-0.5), k)       # keep [-0.5, 0.5)
            rows.append(k)
            if with_dcf:
                a = _voronoi_areas(k.astype(np.float64), 0.5)
                wts.append(a / a.mean())
    off = np.zeros(S * L + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r_) for r_ in rows])
    coords = np.concatenate(rows).astype(np.float32)
    dcf = np.concatenate(wts) if with_dcf else None
    return Trajectory(off, coords, dcf, S, L, ny, nx)


def simulate_kspace_nc(X0: np.ndarray, tr: Trajectory, snr_db, seed: int, smaps=None):
    """Y = P_Omega F S X0 + xi for non-Cartesian coordinates, F the exact
    non-uniform DFT y(k) = (ny nx)^(-1/2) sum_r x_r exp(-2 pi i k . r) over
    pixels r = (ry, rx) in [0, ny) x [0, nx) (on grid frequencies k = kappa/n
    it is the unitary DFT).  Noise as in simulate_kspace.  Returns [M] or
    [c][M]."""
    S, L, ny, nx = X0.shape
    c = 1 if smaps is None else smaps.shape[1]
    Y = np.empty((c, tr.M), dtype=np.complex128)
    for s in range(S):
        for t in range(L):
            p = s * L + t
            k = tr.coords[tr.off[p]:tr.off[p + 1]].astype(np.float64)
            # exp(-2 pi i (ky ry + kx rx)) evaluated as the product of its two factors
            ey = np.exp(-2j * np.pi * k[:, 0:1] * np.arange(ny)[None, :])
            ex = np.exp(-2j * np.pi * k[:, 1:2] * np.arange(nx)[None, :])
            for q in range(c):
                img = X0[s, t] if smaps is None else smaps[s, q] * X0[s, t]
                Y[q, tr.off[p]:tr.off[p + 1]] = np.sum((ey @ img) * ex, axis=1) / np.sqrt(ny * nx)
    if snr_db is not None and np.isfinite(snr_db):
        sig2 = np.sum(np.abs(Y) ** 2) / max(c * tr.M, 1) * 10.0 ** (-snr_db / 10.0)
        Y = Y + (rng.complex_gaussian(seed, "kspace-noise", (tr.M,), sig2)[None] if c == 1
                 else rng.complex_gaussian(seed, "kspace-noise-coils", (c, tr.M), sig2))
    return Y[0] if smaps is None else Y


def simulate_kspace(X0: np.ndarray, smp: Sampling, snr_db: float, seed: int, smaps=None):
    """Y = P_Omega F S X0 + xi (eq. forward; S = I without coil maps), F the
    unitary 2-D DFT per frame.  Noise: circular complex Gaussian with
    per-sample variance (||P_Omega F S X0||^2 / (c M)) 10^(-SNR/10).
    Returns complex128 [M], or [c][M] (coil-major) with maps [S][c][ny][nx]."""
    S, L, ny, nx = X0.shape
    c = 1 if smaps is None else smaps.shape[1]
    Y = np.empty((c, smp.M), dtype=np.complex128)
    for q in range(c):
        for s in range(S):
            img = X0[s] if smaps is None else smaps[s, q][None] * X0[s]
            k = np.fft.fft2(img, norm="ortho").reshape(L, ny * nx)
            for t in range(L):
                p = s * L + t
                Y[q, smp.off[p]:smp.off[p + 1]] = k[t, smp.idx[smp.off[p]:smp.off[p + 1]]]
    if snr_db is not None and np.isfinite(snr_db):
        sig2 = np.sum(np.abs(Y) ** 2) / max(c * smp.M, 1) * 10.0 ** (-snr_db / 10.0)
        Y = Y + (rng.complex_gaussian(seed, "kspace-noise", (smp.M,), sig2)[None] if c == 1
                 else rng.complex_gaussian(seed, "kspace-noise-coils", (c, smp.M), sig2))
    return Y[0] if smaps is None else Y
