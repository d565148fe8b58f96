"""Projected gradient (BLIP / inexact IPG) reconstruction, FP64.

Test infrastructure only.

Follows eq. blip (with the DCF weighting of eq. blip_dcf) and Algorithm 2:
    Z     = X^k - mu_k A^H diag(w) (A X^k - Y)
    X'    = P(Z)                                   (exact matched filter)
    accept  iff  mu_k < ||X' - X^k||^2 / ||A(X' - X^k)||_W^2     (eq. steprule)
    else    mu_k <- mu_k / zeta and project again (the gradient is unchanged)
with A = P_Omega F S (eq. forward; S = I for one coil, else the coil
sensitivity maps, with the samples of every coil in Y), X^0 = 0, mu_k reset to the initial mu at every new k (Algorithm 2 sets
mu_k = mu for every k before any shrinkage), stop after max_iter accepted
iterations or when the relative decrease of the objective
f = ||Y - A X||_W^2 falls below rel_tol (Section "Numerical experiments",
computational cost paragraph).  With w = 1 the weighted norms are the plain
ones.  Edge readings: Delta X = 0 accepts and stops (fixed point);
||A Delta X|| = 0 with Delta X != 0 accepts.  The optional non-expansive
safeguard keeps X^k_v where it is closer to Z_v than the projection
(footnote to eq. nonexpansive); the optional kappa rescaling multiplies X^1
and mu by ||Y|| / ||A X^1|| after the first iteration.
"""
from __future__ import annotations

import numpy as np

from . import covertree, fourier, mf, nudft, phase, subspace


class NoConvergence(RuntimeError):
    pass


def _weighted_sq(r: np.ndarray, w) -> float:
    a = np.abs(r) ** 2
    return float(np.sum(a if w is None else np.asarray(w, dtype=np.float64) * a))


def project(Z: np.ndarray, atoms: np.ndarray, warm_idx=None, X_prev=None,
            nonexpansive: bool = False, u=None, tree=None, eps: float = 0.0):
    """Cone projection of a frame-major image Z [S][L][ny][nx]; with a phase
    vector u, the phase-aligned projection (atoms are then the aligned ones);
    with a cover tree (built from covertree.atom_rows(atoms)), CoverBLIP's
    projection: Algorithm 1 at inaccuracy eps, warm-started at warm_idx."""
    S, L, ny, nx = Z.shape
    Zv = fourier.frame_to_voxel(Z)
    if tree is not None:
        if u is not None:
            raise ValueError("the tree projection of a phase-aligned dictionary is not defined here")
        res = covertree.tree_mf(Zv, atoms, tree, eps, warm_idx=warm_idx)
    else:
        res = (mf.exact_mf(Zv, atoms, warm_idx=warm_idx, want_X=True) if u is None
               else phase.project_aligned(Zv, atoms, u, warm_idx=warm_idx))
    Xv = res["X"]
    if nonexpansive and X_prev is not None:
        Xp = fourier.frame_to_voxel(X_prev)
        keep = np.sum(np.abs(Xp - Zv) ** 2, axis=1) < np.sum(np.abs(Xv - Zv) ** 2, axis=1)
        Xv = np.where(keep[:, None], Xp, Xv)
        res["kept_previous"] = keep
    return fourier.voxel_to_frame(Xv, S, ny, nx), res


def op_forward(X, off, idx, V=None, smaps=None, coords=None):
    """A X, or with a temporal subspace V (eq. CS1) A(expand(X)); with coil
    maps smaps [S][c][ny][nx] the samples are coil-major [c][M]; with
    non-Cartesian coordinates (idx unused) F is the non-uniform DFT."""
    Xf = X if V is None else subspace.expand(X, V)
    if coords is not None:
        return nudft.forward(Xf, off, coords) if smaps is None else nudft.forward_coils(Xf, off, coords, smaps)
    return fourier.forward(Xf, off, idx) if smaps is None else fourier.forward_coils(Xf, off, idx, smaps)


def op_adjoint(R, off, idx, S, L, ny, nx, V=None, smaps=None, coords=None):
    """A^H R over L frames (coils combined with conj(S_q) when smaps is
    given), compressed by V^H when V is given."""
    Lf = L if V is None else V.shape[0]
    if coords is not None:
        G = (nudft.adjoint(R, off, coords, S, Lf, ny, nx) if smaps is None
             else nudft.adjoint_coils(R, off, coords, S, Lf, ny, nx, smaps))
    else:
        G = (fourier.adjoint(R, off, idx, S, Lf, ny, nx) if smaps is None
             else fourier.adjoint_coils(R, off, idx, S, Lf, ny, nx, smaps))
    return G if V is None else subspace.compress(G, V)


def gradient(X, Y, off, idx, w, V=None, smaps=None, coords=None):
    """A^H W (A X - Y) and the residual; with V: the compressed gradient of
    eq. gradupdate, compress(A^H W (A expand(X) - Y)).  The weights w [M]
    apply to every coil's samples."""
    S, L, ny, nx = X.shape
    R = op_forward(X, off, idx, V, smaps, coords) - Y
    WR = R if w is None else np.asarray(w, dtype=np.float64) * R
    return op_adjoint(WR, off, idx, S, L, ny, nx, V, smaps, coords), R


def ipg_step(Y, off, idx, atoms, X, mu: float, w=None, warm_idx=None,
             nonexpansive: bool = False, V=None, smaps=None, u=None, coords=None, tree=None,
             eps: float = 0.0):
    """One projected-gradient step at a fixed mu.  Returns (X', projection
    result, stats) with stats = dx2, adx2 (weighted), f_old, f_new.  With a
    temporal subspace V, X has s compressed frames, atoms are the compressed
    atoms and dx2 is the compressed norm (the compressed step rule).  With
    coil maps, Y is [c][M].  With a phase vector u the projection is the
    phase-aligned one (complex PD) over aligned atoms; with a cover tree it
    is CoverBLIP's (Algorithm 1 at inaccuracy eps, warm-started at warm_idx)."""
    Y = np.asarray(Y, dtype=np.complex128)
    X = np.asarray(X, dtype=np.complex128)
    G, R = gradient(X, Y, off, idx, w, V, smaps, coords)
    Z = X - mu * G
    Xn, res = project(Z, atoms, warm_idx=warm_idx, X_prev=X, nonexpansive=nonexpansive, u=u, tree=tree,
                      eps=eps)
    dX = Xn - X
    AdX = op_forward(dX, off, idx, V, smaps, coords)
    stats = dict(dx2=float(np.sum(np.abs(dX) ** 2)), adx2=_weighted_sq(AdX, w),
                 f_old=_weighted_sq(R, w),
                 f_new=_weighted_sq(op_forward(Xn, off, idx, V, smaps, coords) - Y, w))
    res["Z"] = Z
    return Xn, res, stats


def ipg_solve(Y, off, idx, dims, atoms, mu0: float, zeta: float = 2.0,
              adaptive: bool = True, max_iter: int = 50, rel_tol: float = 1e-6,
              max_shrinks: int = 30, X0=None, w=None, kappa: bool = False,
              nonexpansive: bool = False, V=None, smaps=None, u=None, coords=None, tree=None,
              eps: float = 0.0):
    """Full reconstruction; dims = (S, L, ny, nx) (L = s compressed frames
    when a temporal subspace V is given).  With a cover tree the projection
    is CoverBLIP's: Algorithm 1 at inaccuracy eps, warm-started at the
    previous iterate's atoms (the root at the first iteration).  Returns (X,
    idx, gamma, history) where history lists per accepted iteration: f
    (objective after the step), mu, shrinks, dx2, adx2 (and, with a tree,
    evals: distance evaluations of the accepted projection)."""
    S, L, ny, nx = dims
    Y = np.asarray(Y, dtype=np.complex128)
    X = np.zeros(dims, dtype=np.complex128) if X0 is None else np.asarray(X0, dtype=np.complex128).copy()
    warm = None
    gamma = np.zeros(S * ny * nx)
    f = _weighted_sq(op_forward(X, off, idx, V, smaps, coords) - Y, w)
    hist = []
    mu_init = float(mu0)
    for k in range(max_iter):
        G, _ = gradient(X, Y, off, idx, w, V, smaps, coords)
        mu = mu_init
        shrinks = 0
        while True:
            Z = X - mu * G
            Xn, res = project(Z, atoms, warm_idx=warm, X_prev=X, nonexpansive=nonexpansive, u=u, tree=tree,
                              eps=eps)
            dX = Xn - X
            dx2 = float(np.sum(np.abs(dX) ** 2))
            adx2 = _weighted_sq(op_forward(dX, off, idx, V, smaps, coords), w)
            if (not adaptive) or dx2 == 0.0 or adx2 == 0.0 or mu < dx2 / adx2:
                break
            mu /= zeta
            shrinks += 1
            if shrinks > max_shrinks:
                raise NoConvergence(f"step size not accepted after {max_shrinks} shrinks")
        X = Xn
        warm = res["idx"]
        gamma = res["gamma"]
        if kappa and k == 0:
            kap = np.sqrt(_weighted_sq(Y, None)) / max(np.sqrt(_weighted_sq(op_forward(X, off, idx, V, smaps, coords), None)),
                                                       1e-300)
            X = X * kap
            gamma = gamma * kap
            mu_init *= kap
        f_new = _weighted_sq(op_forward(X, off, idx, V, smaps, coords) - Y, w)
        hist.append(dict(f=f_new, mu=mu, shrinks=shrinks, dx2=dx2, adx2=adx2))
        if tree is not None:
            hist[-1]["evals"] = int(np.sum(res["evals"]))
        if dx2 == 0.0:
            break
        if rel_tol and f > 0 and (f - f_new) / f < rel_tol:
            f = f_new
            break
        f = f_new
    return X, warm, gamma, hist
