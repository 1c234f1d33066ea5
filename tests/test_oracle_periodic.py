"""Oracle pins for periodic meshes (the screened equation of section 4.2,
equation semPDE, is positive definite with alpha > 0 also without Dirichlet
faces, which allows periodic boxes).  A periodic direction identifies the
faces at 0 and 1 of the unit cube; the distinct global-local numbering of
section 4.2.1 then has E_d N coordinates in that direction.

Pinned against what does not come from the numbering itself:
  - node counts and copy multiplicities in closed form;
  - at N = 1 on an affine box the assembled operator is h times the
    7-point Laplacian stencil in every row, with the neighbours wrapped
    around the periodic directions (and the plain stencil where a direction
    has Dirichlet faces);
  - constants are annihilated on a curved, fully periodic mesh (alpha = 0,
    variable kappa);
  - shifting a field by one element commutes with the assembled operator
    on a fully periodic affine box;
  - the screened manufactured solution u = sin 2 pi x sin 2 pi y sin 2 pi z
    (f = (12 pi^2 + alpha) u) converges spectrally in N on a curved
    periodic mesh."""
import numpy as np
import pytest

from oracle import oracle as orc
from seminputs import grf_features


def _dense_global(m):
    A = np.zeros((m.nG, m.nG))
    e = np.zeros(m.nG)
    for g in range(m.nG):
        e[g] = 1.0
        A[:, g] = orc.apply_global(m, e)
        e[g] = 0.0
    return A


@pytest.mark.parametrize("per", [1, 2, 4, 3, 7])
@pytest.mark.parametrize("N,dims", [(3, (2, 3, 1)), (2, (1, 2, 2)), (4, (3, 1, 2))])
def test_counts_and_multiplicities(per, N, dims):
    ex, ey, ez = dims
    l2g, perm, off, mult, bmask = orc.maps(N, ex, ey, ez, 1, per)
    G = [e * N + (0 if per & (1 << d) else 1) for d, e in enumerate(dims)]
    assert off.shape[0] - 1 == G[0] * G[1] * G[2]
    n1 = N + 1
    q = np.arange(n1 ** 3)
    idx = [q % n1, (q // n1) % n1, q // (n1 * n1)]
    # a copy count 2 per direction whose index is on a face shared with a
    # neighbour (interior faces; both faces of a periodic direction)
    for e in range(ex * ey * ez):
        ec = [e % ex, (e // ex) % ey, e // (ex * ey)]
        want = np.ones(n1 ** 3, np.int64)
        for d in range(3):
            i, E = idx[d], dims[d]
            shared = np.zeros(n1 ** 3, bool)
            if per & (1 << d):
                shared = (i == 0) | (i == N)
            else:
                shared = ((i == 0) & (ec[d] > 0)) | ((i == N) & (ec[d] < E - 1))
            want *= np.where(shared, 2, 1)
        np.testing.assert_array_equal(mult[e * n1 ** 3:(e + 1) * n1 ** 3], want)
    # no Dirichlet node in a periodic direction: a fully periodic box has none
    if per == 7:
        assert not bmask.any()
    # perm lists the copies of each global node in ascending local index
    for g in range(off.shape[0] - 1):
        seg = perm[off[g]:off[g + 1]]
        assert np.all(np.diff(seg) > 0) and np.all(l2g[seg] == g)


@pytest.mark.parametrize("per,dirichlet", [(7, 0), (1, 1), (6, 1)])
def test_n1_is_h_times_wrapped_seven_point_stencil(per, dirichlet):
    n = 4
    m = orc.mesh(1, n, n, n, orc.MAP_AFFINE, dirichlet=dirichlet, periodic=per)
    A = _dense_global(m)
    h = 1.0 / n
    G = [n if per & (1 << d) else n + 1 for d in range(3)]
    assert m.nG == G[0] * G[1] * G[2]
    gmask = np.zeros(m.nG, bool)
    gmask[m.l2g[m.bmask.astype(bool)]] = True
    checked = 0
    for gz in range(G[2]):
        for gy in range(G[1]):
            for gx in range(G[0]):
                g = gx + G[0] * (gy + G[1] * gz)
                if gmask[g]:
                    continue
                c = (gx, gy, gz)
                # rows next to a Dirichlet face have masked neighbours:
                # check rows whose six neighbours all exist and are free
                nbs = []
                ok = True
                for d in range(3):
                    for s in (-1, 1):
                        cc = list(c)
                        cc[d] += s
                        if per & (1 << d):
                            cc[d] %= G[d]
                        elif not 0 <= cc[d] < G[d]:
                            ok = False
                            continue
                        nbs.append(cc[0] + G[0] * (cc[1] + G[1] * cc[2]))
                if not ok or any(gmask[q] for q in nbs):
                    continue
                row = A[g].copy()
                assert abs(row[g] - 6 * h) < 1e-14
                for q in nbs:
                    assert abs(row[q] + h) < 1e-14, (c, q)
                    row[q] = 0.0
                row[g] = 0.0
                assert np.max(np.abs(row)) < 1e-14
                checked += 1
    # every row whose neighbours are all free: all G_d coordinates of a
    # periodic direction, 2 .. G_d - 3 of one with Dirichlet faces
    want = 1
    for d in range(3):
        want *= G[d] if per & (1 << d) else (G[d] - 4 if dirichlet else G[d] - 2)
    assert checked == want


def test_constants_in_the_null_space_when_fully_periodic():
    kap = grf_features(seed=3, M=32, ell=0.3, sigma=0.5)
    m = orc.mesh(4, 2, 3, 2, orc.MAP_SINE_CYCLIC, dirichlet=0, kappa_params=kap,
                 periodic=7)
    one = np.ones(m.nG)
    Au = orc.apply_global(m, one)
    scale = np.max(np.abs(orc.apply_global(m, np.random.default_rng(0).uniform(-1, 1, m.nG))))
    assert np.max(np.abs(Au)) <= 1e-13 * scale
    # with only x periodic and Dirichlet faces elsewhere, constants are not
    # in the null space
    m2 = orc.mesh(4, 2, 3, 2, orc.MAP_SINE_CYCLIC, dirichlet=1, kappa_params=kap,
                  periodic=1)
    assert np.max(np.abs(orc.apply_global(m2, np.ones(m2.nG)))) > 1e-3 * scale


def test_shift_by_one_element_commutes_with_the_operator():
    N, n = 3, 3
    m = orc.mesh(N, n, n, n, orc.MAP_AFFINE, dirichlet=0, periodic=7)
    G = n * N
    u = np.random.default_rng(4).uniform(-1, 1, m.nG).reshape(G, G, G)  # [z][y][x]
    for axis in (0, 1, 2):
        su = np.roll(u, N, axis=axis)
        Asu = orc.apply_global(m, su.reshape(-1)).reshape(G, G, G)
        sAu = np.roll(orc.apply_global(m, u.reshape(-1)).reshape(G, G, G), N, axis=axis)
        assert np.max(np.abs(Asu - sAu)) <= 1e-12 * np.max(np.abs(sAu))


@pytest.mark.parametrize("mapping,rate,final", [(orc.MAP_AFFINE, 0.01, 1e-6),
                                                 (orc.MAP_SINE_X, 0.1, 1e-4)])
def test_screened_periodic_manufactured_solution_converges(mapping, rate, final):
    """Nodal error of the FP64 PCG solution at N = 3, 5, 7 on a 2^3 fully
    periodic mesh (measured: affine 5.7e-3, 2.9e-5, 1.3e-7; mapped 1.6e-2,
    9.3e-4, 4.9e-5): an error in the periodic numbering leaves an O(1)
    error."""
    alpha = 1.0
    errs = []
    for N in (3, 5, 7):
        m = orc.mesh(N, 2, 2, 2, mapping, dirichlet=0, alpha=alpha, periodic=7)
        X = m.X
        ue = np.sin(2 * np.pi * X[0]) * np.sin(2 * np.pi * X[1]) * np.sin(2 * np.pi * X[2])
        f = (12 * np.pi ** 2 + alpha) * ue
        b = orc.to_global(m, orc.rhs_local(m, f))
        x, st, it, _ = orc.pcg(m, b, 1e-13, 5000)
        assert st == 0
        err = np.max(np.abs(x - orc.to_global(m, ue)))
        errs.append(err)
    assert errs[1] < rate * errs[0] and errs[2] < rate * errs[1]
    assert errs[2] < final
