"""Pins of the oracle's global-local numbering and direct stiffness summation
(paper section 4.2.1, distinct global-local node numbering after Fischer
1991): permutation and counting invariants, and Q Q^T checked against a
sparse Boolean scatter matrix built independently from the node positions."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as orc
from seminputs import uniform

MESHES = [(1, 2, 2, 2), (2, 3, 2, 1), (3, 2, 3, 4), (4, 1, 1, 1), (7, 2, 2, 2),
          (5, 3, 1, 2)]


@pytest.mark.parametrize("N,ex,ey,ez", MESHES)
def test_maps_are_consistent_permutations(N, ex, ey, ez):
    l2g, perm, offsets, mult, bmask = orc.maps(N, ex, ey, ez, 1)
    n1 = N + 1
    nL = ex * ey * ez * n1 ** 3
    nG = (ex * N + 1) * (ey * N + 1) * (ez * N + 1)
    assert offsets.shape[0] == nG + 1 and offsets[0] == 0 and offsets[-1] == nL
    assert np.all(np.diff(offsets) >= 1)               # every global node used
    np.testing.assert_array_equal(np.sort(perm), np.arange(nL))
    g_sorted = l2g[perm]
    assert np.all(np.diff(g_sorted) >= 0)               # sorted by g
    same = np.diff(g_sorted) == 0
    assert np.all(np.diff(perm)[same] > 0)              # ties ascending in l
    np.testing.assert_array_equal(
        g_sorted, np.repeat(np.arange(nG), np.diff(offsets)))
    np.testing.assert_array_equal(mult, np.diff(offsets)[l2g])
    # multiplicities: corner 8, edge 4, face 2, interior 1 copies
    assert mult.max() == min(8, 2 ** sum(d > 1 for d in (ex, ey, ez)))


@pytest.mark.parametrize("N,ex,ey,ez", MESHES)
def test_l2g_matches_node_positions(N, ex, ey, ez):
    """Two local nodes share a global id exactly when they sit at the same
    point of the (affine) mesh; the id of a point is its lexicographic rank
    on the (ex N + 1) x (ey N + 1) x (ez N + 1) lattice."""
    l2g, *_ = orc.maps(N, ex, ey, ez, 1)
    X = orc.coords(N, ex, ey, ez, orc.MAP_AFFINE)
    G = np.array([ex * N + 1, ey * N + 1, ez * N + 1])
    # lattice position of every node: round the coordinate to the GLL lattice
    xi, _ = orc.gll(N)
    lat = []
    for d, Ed in enumerate((ex, ey, ez)):
        pts = np.unique(np.concatenate([e / Ed + (xi + 1) / (2 * Ed)
                                        for e in range(Ed)]).round(12))
        assert pts.shape[0] == G[d]
        lat.append(np.searchsorted(pts, X[d].round(12)))
    g_ref = lat[0] + G[0] * (lat[1] + G[1] * lat[2])
    np.testing.assert_array_equal(l2g, g_ref)


@pytest.mark.parametrize("N,ex,ey,ez", MESHES)
def test_dirichlet_mask_marks_outer_faces(N, ex, ey, ez):
    l2g, perm, offsets, mult, bmask = orc.maps(N, ex, ey, ez, 1)
    X = orc.coords(N, ex, ey, ez, orc.MAP_AFFINE)
    onb = np.any((np.abs(X) < 1e-12) | (np.abs(X - 1) < 1e-12), axis=0)
    np.testing.assert_array_equal(bmask.astype(bool), onb)
    nG = offsets.shape[0] - 1
    nb = len(np.unique(l2g[bmask.astype(bool)]))
    Gd = [ex * N + 1, ey * N + 1, ez * N + 1]
    assert nb == nG - max(0, Gd[0] - 2) * max(0, Gd[1] - 2) * max(0, Gd[2] - 2)
    _, _, _, _, bm0 = orc.maps(N, ex, ey, ez, 0)
    assert bm0.sum() == 0


@pytest.mark.parametrize("N,ex,ey,ez", MESHES)
def test_gs_equals_boolean_scatter(N, ex, ey, ez):
    m = orc.mesh(N, ex, ey, ez, orc.MAP_SINE_CYCLIC, dirichlet=1)
    Q = sp.csr_matrix((np.ones(m.nL), (np.arange(m.nL), m.l2g)),
                      shape=(m.nL, m.nG))
    v = uniform(m.nL, seed=3)
    keep = 1.0 - m.bmask
    ref = keep * (Q @ (Q.T @ v))
    out = orc.gs(m, v)
    np.testing.assert_allclose(out, ref, rtol=1e-15, atol=1e-15)
    # masked entries exactly zero
    assert np.all(out[m.bmask.astype(bool)] == 0.0)


@pytest.mark.parametrize("N,ex,ey,ez", MESHES)
def test_gs_invariants(N, ex, ey, ez):
    m = orc.mesh(N, ex, ey, ez, orc.MAP_AFFINE, dirichlet=0)
    v = uniform(m.nL, seed=4)
    out = orc.gs(m, v)
    # continuity: every copy of a global node holds the same value
    g0 = orc.to_global(m, out)
    np.testing.assert_array_equal(out, g0[m.l2g])
    # conservation: sum over unique nodes of Q^T v equals sum over copies
    assert abs(g0.sum() - v.sum()) < 1e-12 * np.abs(v).sum()
    # Q Q^T of a continuous vector is mult o v
    c = orc.to_local(m, uniform(m.nG, seed=5))
    np.testing.assert_allclose(orc.gs(m, c), m.mult * c, rtol=1e-15)


def test_gs_summation_order_is_ascending_local_index():
    """Bit-level pin of the summation order: with values whose sum depends
    on the order, each global node must hold ((0 + v_l0) + v_l1) + ... over
    its copies in ascending local index."""
    m = orc.mesh(2, 2, 2, 2, orc.MAP_AFFINE, dirichlet=0)
    rng = np.random.default_rng(0)
    v = rng.choice([1e16, -1e16, 1.0, 3.0, -7.0], size=m.nL)
    out = orc.gs(m, v)
    for g in range(m.nG):
        ls = np.flatnonzero(m.l2g == g)      # ascending
        s = 0.0
        for l in ls:
            s = s + v[l]
        assert out[ls[0]] == s
