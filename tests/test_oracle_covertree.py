"""Pins of the cover-tree oracle: a hand-worked tree, the cover-tree
invariants (nesting, covering, separation, eq. maxdistbound), exact search
at eps = 0 against brute force, the (1+eps) bound of Definition 3.1, and the
non-expansive warm start of Algorithm 2."""
import numpy as np
import pytest

from oracle import covertree as ct
from oracle import mf
from synth import rng, workloads


def test_hand_worked_tree():
    # points on a line: 0, 4, 1, 2 (rows of length 1)
    X = np.array([[0.0], [4.0], [1.0], [2.0]])
    t = ct.build(X)
    assert t.sigma == 4.0
    assert [list(l) for l in t.levels] == [[0], [0, 1], [0, 1, 3], [0, 1, 2, 3]]
    # atom 3 (x=2) is 2 from both 0 and 4: the tie goes to the lower index
    assert t.parent[2][3] == 0 and t.parent[3][2] == 0
    assert t.maxdist[0][0] == 4.0 and t.maxdist[1][1] == 0.0 and t.maxdist[1][0] == 2.0
    ct.check_invariants(t)


def _clustered(seed, n, dim):
    c = rng.normal(seed, "c", 8 * dim).reshape(8, dim)
    lab = rng.randint(seed, "l", n, 8)
    x = c[lab] + 0.15 * rng.normal(seed, "x", n * dim).reshape(n, dim)
    return x / np.linalg.norm(x, axis=1, keepdims=True)


@pytest.mark.parametrize("kind", ["clustered", "fisp", "bssfp"])
def test_invariants_and_search(kind):
    if kind == "clustered":
        X = _clustered(1, 300, 8)
    elif kind == "fisp":
        D = workloads.fisp_dictionary(L=40, n_t1=12, n_t2=14)
        X = D.atoms / np.linalg.norm(D.atoms, axis=1, keepdims=True)
    else:
        D = workloads.bssfp_dictionary(L=30, n_t1=8, n_t2=8, n_df=5, seed=2)
        A = D.atoms / np.linalg.norm(D.atoms, axis=1, keepdims=True)
        X = np.concatenate([A.real, A.imag], axis=1)      # the real 2L form
    t = ct.build(X)
    ct.check_invariants(t)
    assert len(t.levels[-1]) == len(t.rep)
    # queries: noisy points, normalised (as Algorithm 2 feeds Z_v/||Z_v||)
    q = X[rng.randint(2, "q", 60, X.shape[0])] + 0.05 * rng.normal(2, "n", 60 * X.shape[1]).reshape(60, -1)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    for v in range(60):
        dist = np.linalg.norm(t.X - q[v], axis=1)
        best = dist.min()
        j0, d0, e0 = ct.search(t, q[v], 0.0)
        assert abs(d0 - best) <= 1e-14 and dist[j0] <= best + 1e-14   # eps = 0: exact NN
        for eps in (0.1, 0.4, 1.6):
            j, dd, e = ct.search(t, q[v], eps)
            assert dd <= (1 + eps) * best * (1 + 1e-12)             # Definition 3.1
            assert e <= e0 + 2
            w = int(rng.randint(3, f"w{v}", 1, len(t.rep))[0])
            jw, dw, _ = ct.search(t, q[v], eps, q_init=w)
            assert dw <= np.linalg.norm(q[v] - t.X[w])              # non-expansive warm start


def test_duplicates_merge_to_lowest_index():
    X = _clustered(4, 50, 6)
    Xd = np.concatenate([X, X[7:8], X[3:4]], axis=0)
    t = ct.build(Xd)
    assert len(t.rep) == 50 and t.rep[7] == 7 and t.rep[3] == 3
    ct.check_invariants(t)


def test_eps0_search_equals_matched_filter():
    """With unit-norm queries and atoms, the nearest atom is the matched
    filter's argmax (eq. exactP)."""
    D = workloads.bssfp_dictionary(L=30, n_t1=8, n_t2=8, n_df=5, seed=2)
    A = D.atoms / np.linalg.norm(D.atoms, axis=1, keepdims=True)
    X = np.concatenate([A.real, A.imag], axis=1)
    t = ct.build(X)
    Z, j, pd, snr = workloads.random_voxels(D, 40, seed=6, snr_db_range=(10.0, 30.0))
    ref = mf.exact_mf(Z, D.atoms)
    for v in range(40):
        p = np.concatenate([Z[v].real, Z[v].imag]) / np.linalg.norm(Z[v])
        ju, _, _ = ct.search(t, p, 0.0)
        assert t.rep[ju] == ref["idx"][v]
