"""Cover tree and its (1+eps)-approximate nearest-neighbour search, FP64.

Test infrastructure only.

Construction (the paper gives none, Table 1 only states costs): greedy
nested nets on the normalised, de-duplicated atoms.  Root S_0 = {atom 0},
sigma = max_j ||D_0 - D_j||.  Level i+1 (radius r = sigma 2^-(i+1)) starts
from S_i and scans the remaining atoms in increasing index, adding an atom
when its distance to every node already in S_{i+1} exceeds r.  A new node's
parent is its nearest node in S_i (ties: lower index).  A maximal
sigma 2^-i separated set covers within sigma 2^-i, so nesting, covering
(||p - q|| <= sigma 2^-i for q in S_{i+1}, parent p in S_i) and separation
(> sigma 2^-i inside S_i) of Section "Cover trees" hold by construction.
Levels continue until every atom is a node.  Each node q of level i stores
maxdist(q) = max over its descendants q' (q's subtree below level i,
itself included) of ||q - q'||.

Search: Algorithm 1, verbatim apart from the notation: Q_0 = {root}; q_c
the warm start (root if none); d_min = ||p - q_c||; while i < i_max and
sigma 2^(-i+1) (1 + 1/eps) > d_min: Q = children of Q_i (a node is its own
child, whose distance is reused, not recomputed); q* = argmin over Q (ties:
lower index); update q_c, d_min if ||p - q*|| < d_min; Q_{i+1} = {q in Q :
||p - q|| <= d_min + maxdist(q)}.  With eps = 0 the loop runs to i_max.
"""
from __future__ import annotations

import numpy as np


def _dist(a, B):
    d = B - a[None, :]
    return np.sqrt(np.sum(np.abs(d) ** 2, axis=1))


class CoverTree:
    def __init__(self, X, levels, parent, sigma, rep):
        self.X = X                # unique normalised atoms [u][K] (FP64)
        self.levels = levels      # list of sorted unique-atom index arrays S_0 ... S_imax
        self.parent = parent      # parent[i][q] for q in S_i (i >= 1): node of S_{i-1}
        self.sigma = sigma
        self.rep = rep            # unique index -> lowest dictionary index
        self.maxdist = None

    @property
    def imax(self):
        return len(self.levels) - 1

    def children(self, i, q):
        """Children of node q of level i: nodes of level i+1 whose parent is q
        (q itself among them), in increasing index."""
        if not hasattr(self, "_kids"):
            self._kids = {}
        if i not in self._kids:          # grouped once per level (bookkeeping only)
            g = {}
            for c, p in self.parent[i + 1].items():
                g.setdefault(p, []).append(c)
            self._kids[i] = {p: sorted(cs) for p, cs in g.items()}
        return self._kids[i].get(q, [])


def unique_atoms(atoms_hat):
    """De-duplicate (exactly equal rows merge into the lowest index)."""
    rows = np.ascontiguousarray(atoms_hat)
    seen = {}
    rep = []
    keep = []
    for j in range(rows.shape[0]):
        key = rows[j].tobytes()
        if key in seen:
            continue
        seen[key] = len(rep)
        rep.append(j)
        keep.append(j)
    return rows[keep], np.asarray(rep, dtype=np.int64)


def build(atoms_hat):
    """Greedy nested nets (definition above) on normalised atoms [d][K]."""
    X, rep = unique_atoms(np.asarray(atoms_hat))
    u = X.shape[0]
    d0 = _dist(X[0], X)
    sigma = float(d0.max())
    levels = [np.array([0])]
    parent = [dict()]
    inS = np.zeros(u, dtype=bool)
    inS[0] = True
    i = 0
    while not inS.all():
        r = sigma * 2.0 ** -(i + 1)
        prev = levels[i]
        nodes = list(prev)
        new = []
        for a in range(u):
            if inS[a]:
                continue
            if np.min(_dist(X[a], X[nodes])) > r:
                nodes.append(a)
                new.append(a)
        par = {int(q): int(q) for q in prev}       # self-children
        for a in new:
            dp = _dist(X[a], X[prev])
            par[a] = int(prev[int(np.argmin(dp))])  # first minimiser: lowest index (prev sorted)
            inS[a] = True
        levels.append(np.array(sorted(nodes)))
        parent.append(par)
        i += 1
        if sigma == 0.0:
            break
    t = CoverTree(X, levels, parent, sigma, rep)
    t.maxdist = _maxdist(t)
    return t


def _maxdist(t):
    """maxdist[i][q]: max distance from node q of level i to its subtree."""
    imax = t.imax
    md = [dict() for _ in range(imax + 1)]
    # subtree members of (q, i): every atom whose ancestor at level i is q
    anc = {int(a): int(a) for a in t.levels[imax]}      # ancestor at the current level
    for i in range(imax, -1, -1):
        groups = {}
        for a, q in anc.items():
            groups.setdefault(q, []).append(a)
        for q, mem in groups.items():
            md[i][q] = float(np.max(_dist(t.X[q], t.X[mem])))
        if i > 0:
            anc = {a: t.parent[i][q] for a, q in anc.items()}
    return md


def check_invariants(t, rtol=1e-12):
    """Nesting, covering and separation of Section "Cover trees", and the
    maxdist bound of eq. maxdistbound."""
    s = t.sigma
    for i in range(1, t.imax + 1):
        assert set(t.levels[i - 1]).issubset(set(t.levels[i]))                 # nesting
        for q, p in t.parent[i].items():
            assert np.linalg.norm(t.X[q] - t.X[p]) <= s * 2.0 ** -(i - 1) * (1 + rtol)   # covering
    for i in range(t.imax + 1):
        L = t.levels[i]
        for k, q in enumerate(L):
            if k + 1 < len(L):
                assert np.min(_dist(t.X[q], t.X[L[k + 1:]])) > s * 2.0 ** -i * (1 - rtol)  # separation
        for q in L:
            assert t.maxdist[i][int(q)] < s * 2.0 ** (-i + 1) * (1 + rtol) + 1e-300   # eq. maxdistbound
    return True


def search(t, p, eps, q_init=None):
    """Algorithm 1.  p: query (unit norm, as the normalised gradient update);
    q_init: unique-atom index of the warm start.  Returns (unique index of
    q_c, d_min, distance evaluations)."""
    p = np.asarray(p)
    root = int(t.levels[0][0])
    evals = 0
    qc = root if q_init is None else int(q_init)
    dmin = float(np.linalg.norm(p - t.X[qc]))
    evals += 1
    Qi = {root: float(np.linalg.norm(p - t.X[root]))}
    evals += 1
    i = 0
    inv_eps = np.inf if eps == 0 else 1.0 / eps
    while i < t.imax and t.sigma * 2.0 ** (-i + 1) * (1.0 + inv_eps) > dmin:
        Q = {}
        for q, dq in Qi.items():
            for c in t.children(i, q):
                if c == q:
                    Q[c] = dq                       # self-child: distance reused
                else:
                    Q[c] = float(np.linalg.norm(p - t.X[c]))
                    evals += 1
        qstar = min(Q, key=lambda c: (Q[c], c))
        if Q[qstar] < dmin:
            dmin = Q[qstar]
            qc = qstar
        Qi = {c: dc for c, dc in Q.items() if dc <= dmin + t.maxdist[i + 1][c]}
        i += 1
    return qc, dmin, evals


def atom_rows(atoms):
    """Normalised atoms as the real rows the tree is built on: (Re, Im)
    interleaved per frame for complex atoms, the atoms themselves for real
    ones."""
    a = np.asarray(atoms)
    a = a / np.linalg.norm(a, axis=1, keepdims=True)
    if np.iscomplexobj(a):
        b = np.empty((a.shape[0], 2 * a.shape[1]))
        b[:, 0::2], b[:, 1::2] = a.real, a.imag
        return b
    return a.astype(np.float64)


def query_rows(Z, complex_atoms):
    """Z_v / ||Z_v|| in the atoms' row layout (the real part for real atoms,
    whose score Re<Z, D_j> only sees it); rows with ||Z_v|| = 0 stay zero."""
    Z = np.asarray(Z).astype(np.complex128)
    if complex_atoms:
        q = np.empty((Z.shape[0], 2 * Z.shape[1]))
        q[:, 0::2], q[:, 1::2] = Z.real, Z.imag
    else:
        q = Z.real.copy()
    nz = np.linalg.norm(Z, axis=1)
    return q / np.where(nz > 0, nz, 1.0)[:, None]


def tree_mf(Z, atoms, t, eps, warm_idx=None):
    """The cone projection of Algorithm 2 with the exact argmax replaced by
    Algorithm 1 (Section "CoverBLIP algorithm"): per voxel, the
    (1+eps)-approximate nearest normalised atom to Z_v / ||Z_v|| (on the
    unit sphere the nearest atom is the one of largest Re<Z_v, Dhat_j>),
    warm-started at the atom of the previous estimate (the root when there is
    none).  t must be built from atom_rows(atoms).  The PD and X follow as
    for the exact filter: gamma = max(Re<Z_v, D_j>, 0) / ||D_j||^2,
    X_v = gamma D_j; a zero voxel keeps its warm index (0 without one) and
    gets gamma = 0.  Returns the keys of mf.exact_mf (idx, gamma, score, X)
    and evals (distance evaluations per voxel)."""
    Z = np.asarray(Z).astype(np.complex128)
    a = np.asarray(atoms)
    rows = atom_rows(a)
    uniq = {}
    for u, j in enumerate(t.rep):                # dictionary index -> unique node
        uniq[rows[j].tobytes()] = u
    node_of = np.array([uniq[rows[j].tobytes()] for j in range(rows.shape[0])])
    nrm = np.linalg.norm(a, axis=1)
    P = query_rows(Z, np.iscomplexobj(a))
    n = Z.shape[0]
    idx = np.zeros(n, dtype=np.int64)
    evals = np.zeros(n, dtype=np.int64)
    znorm = np.linalg.norm(Z, axis=1)
    for v in range(n):
        w = None if warm_idx is None else int(np.asarray(warm_idx)[v])
        if znorm[v] == 0.0:
            idx[v] = 0 if w is None else w
            continue
        qc, _, ev = search(t, P[v], eps, q_init=None if w is None else int(node_of[w]))
        idx[v] = int(t.rep[qc])
        evals[v] = ev
    score = np.real(np.sum(Z * np.conj(a[idx]), axis=1)) / nrm[idx]
    score = np.where(znorm == 0.0, 0.0, score)
    gamma = np.maximum(score, 0.0) / nrm[idx]
    X = gamma[:, None] * a[idx].astype(np.complex128)
    return dict(idx=idx, gamma=gamma, score=score, X=X, evals=evals, znorm=znorm)
