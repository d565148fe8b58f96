"""Exact local matched filter around a proposed grid cell, with fallback.

Test infrastructure only.

For a voxel Z_v and a proposed cell c (one grid index per parameter of a
product-grid dictionary, atoms row-major with the last parameter fastest),
the candidate set is the box prod_p [c_p - r, c_p + r] clipped to the grid.
The local answer is the exact matched filter (eq. exactP / exactPs) over that
box: the lowest-index maximiser of Re<Z_v, D_j>/||D_j||.  With recentre
rounds, a best atom lying on a box face that is not a grid edge moves the
box centre to that atom and the box search repeats.  If the winning
normalised correlation is below the threshold, the exhaustive matched filter
over the whole dictionary is used instead (fallback).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import mf


def box_atoms(cell, dims, r):
    """Row-major atom indices of the clipped box around ``cell`` (ascending)."""
    ranges = [range(max(0, int(c) - r), min(int(n) - 1, int(c) + r) + 1) for c, n in zip(cell, dims)]
    idx = []
    for sub in itertools.product(*ranges):
        j = 0
        for s, n in zip(sub, dims):
            j = j * int(n) + s
        idx.append(j)
    return np.asarray(idx, dtype=np.int64)


def _sub(j, dims):
    out = []
    for n in reversed(dims):
        out.append(j % int(n))
        j //= int(n)
    return list(reversed(out))


def local_match(Z, atoms, dims, cells, r=3, threshold=0.98, recentre=0, warm=None):
    """Returns dict(idx, score, corr, fallback [bool], rounds [int]) per voxel.

    warm (optional, [n] atom indices): the previous iterate's atom competes
    with the box's best under the same order (higher score, then lower
    index) before the fallback test, so the projection is never worse than
    the warm start (the non-expansive safeguard of the inexact projection)."""
    Z = np.asarray(Z).astype(np.complex128)
    n = Z.shape[0]
    nrm = mf.atom_norms(atoms)
    znorm = np.sqrt(np.sum(np.abs(Z) ** 2, axis=1))
    idx = np.zeros(n, dtype=np.int64)
    score = np.zeros(n)
    rounds = np.zeros(n, dtype=np.int64)
    for v in range(n):
        cell = [int(c) for c in cells[v]]
        for rd in range(recentre + 1):
            cand = box_atoms(cell, dims, r)
            c = mf.correlations(Z[v:v + 1], atoms[cand], nrm[cand])[0]
            k = int(np.argmax(c))                      # first maximiser: lowest index
            j, s = int(cand[k]), float(c[k])
            idx[v], score[v] = j, s
            sub = _sub(j, dims)
            face = any((sub[p] == cell[p] - r and sub[p] > 0) or (sub[p] == cell[p] + r and sub[p] < int(dims[p]) - 1)
                       for p in range(len(dims)))
            if not face or rd == recentre:
                break
            cell = sub
            rounds[v] = rd + 1
        if warm is not None and znorm[v] > 0 and 0 <= int(warm[v]) < atoms.shape[0]:
            w = int(warm[v])
            cw = float(mf.correlations(Z[v:v + 1], atoms[w:w + 1], nrm[w:w + 1])[0, 0])
            if cw > score[v] or (cw == score[v] and w < idx[v]):
                idx[v], score[v] = w, cw
    corr = np.where(znorm > 0, score / np.where(znorm > 0, znorm, 1.0), 0.0)
    fb = corr < threshold
    if np.any(fb):
        ex = mf.exact_mf(Z[fb], atoms)
        idx[fb] = ex["idx"]
        score[fb] = ex["score"]
        corr[fb] = ex["corr"]
    return dict(idx=idx, score=score, corr=corr, fallback=fb, rounds=rounds)
