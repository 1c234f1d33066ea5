"""GPU parity of the DG shallow-water volume term (paper section 4.3) through
the C ABI (include/dg.h) against the FP64 oracle (oracle/dg.py).

The matrix cores accumulate the products in their own order, so the bar is
componentwise: |rhs_gpu - rhs_oracle| <= 1e-13 (|Drw| |Fr| + |Dsw| |Fs| +
max|Drw| sum|Fr| + max|Dsw| sum|Fs| + g |h| (|rx| |Dr| + |sx| |Ds|) |B|
(and the same with ry, sy)) at every node (Fr = rx F + ry G, Fs = sx F +
sy G; sums over the element's nodes): the sizes of the terms the rounding
acts on.  Each side builds its matrices itself; entries that vanish in exact
arithmetic carry rounding of ~1e-16 max|D| on each side (measured agreement
of the two constructions: 2e-16 to 1.7e-14 of max|D|, N = 1..8), hence the
max|D| terms; the bathymetry gradient is likewise formed from B by each
side in its own order.  Setup arrays against the oracle:
affine factors and node coordinates to 1e-14 relative, weak derivative
matrices and the bathymetry gradient to 1e-12 of their scale.  Meshes: 70
elements (a ragged last workgroup of 64 elements) for every order 1..8, and
the example's 212,800 elements at N = 8 and N = 3."""
import numpy as np
import pytest

from oracle import dg
from seminputs import tri_mesh

from gpu_util import to_dev, to_host, torch

pytestmark = pytest.mark.gpu

G_GRAV = 9.81


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


def _state(X, Y):
    """Smooth positive depth, momenta and bathymetry at the nodes."""
    B = 0.3 * np.exp(-((X - 0.4) ** 2 + (Y - 0.6) ** 2) / 0.05) + 0.1 * X * Y
    h = 2.0 + 0.3 * np.sin(2 * np.pi * X) * np.cos(np.pi * Y) - B
    hu = 0.2 * np.cos(3 * X + Y) * h
    hv = -0.1 * np.sin(X - 2 * Y) * h
    return B, np.stack([h, hu, hv], axis=1)


def _setup(sem, N, nx, ny, seed=1):
    vx, vy, etov = tri_mesh(nx, ny, seed=seed)
    ops = dg.reference_operators(N)
    geo = dg.geometric_factors(vx, vy, etov)
    X, Y = dg.physical_nodes(ops, vx, vy, etov)
    B, Q = _state(X, Y)
    h = sem.dg_setup(N, vx, vy, etov, bathymetry=B, g=G_GRAV)
    return h, ops, geo, X, Y, B, Q


def _bound(ops, geo, Q, B):
    rx, sx, ry, sy, _ = geo
    F, G = dg.fluxes(Q, G_GRAV)
    Fr = np.abs(rx[:, None, None] * F) + np.abs(ry[:, None, None] * G)
    Fs = np.abs(sx[:, None, None] * F) + np.abs(sy[:, None, None] * G)
    b = Fr @ np.abs(ops["Drw"]).T + Fs @ np.abs(ops["Dsw"]).T
    b += (np.max(np.abs(ops["Drw"])) * Fr.sum(axis=2, keepdims=True)
          + np.max(np.abs(ops["Dsw"])) * Fs.sum(axis=2, keepdims=True))
    aBr, aBs = np.abs(B) @ np.abs(ops["Dr"]).T, np.abs(B) @ np.abs(ops["Ds"]).T
    gh = G_GRAV * np.abs(Q[:, 0])
    b[:, 1] += gh * (np.abs(rx)[:, None] * aBr + np.abs(sx)[:, None] * aBs)
    b[:, 2] += gh * (np.abs(ry)[:, None] * aBr + np.abs(sy)[:, None] * aBs)
    return b


@pytest.mark.parametrize("N", range(1, 9))
def test_setup_arrays_match_oracle(sem, N):
    t = torch()
    h, ops, geo, X, Y, B, Q = _setup(sem, N, 7, 5)
    try:
        Np, E = sem.dg_query(h)
        assert Np == dg.num_nodes(N) and E == 70
        def ex(which, n):
            buf = t.empty(n, dtype=t.float64, device="cuda")
            sem.dg_export(h, which, buf)
            t.cuda.synchronize()
            return to_host(buf)
        rx, sx, ry, sy, _ = geo
        g4 = ex(sem.DG_ARR_GEO, 4 * E).reshape(E, 4)
        ref = np.stack([rx, sx, ry, sy], axis=1)
        assert np.max(np.abs(g4 - ref)) <= 1e-14 * np.max(np.abs(ref))
        np.testing.assert_allclose(ex(sem.DG_ARR_X, E * Np).reshape(E, Np), X, rtol=0, atol=1e-15)
        np.testing.assert_allclose(ex(sem.DG_ARR_Y, E * Np).reshape(E, Np), Y, rtol=0, atol=1e-15)
        for which, key in ((sem.DG_ARR_DRW, "Drw"), (sem.DG_ARR_DSW, "Dsw")):
            got = ex(which, Np * Np).reshape(Np, Np)
            assert np.max(np.abs(got - ops[key])) <= 1e-12 * np.max(np.abs(ops[key])), key
        Bx, By = dg.bathymetry_gradient(ops, geo, B)
        dB = ex(sem.DG_ARR_DB, E * 2 * Np).reshape(E, 2, Np)
        scale = max(np.max(np.abs(Bx)), np.max(np.abs(By)))
        assert np.max(np.abs(dB[:, 0] - Bx)) <= 1e-12 * scale
        assert np.max(np.abs(dB[:, 1] - By)) <= 1e-12 * scale
    finally:
        sem.dg_destroy(h)


def _check_volume(sem, h, ops, geo, B, Q):
    t = torch()
    Bx, By = dg.bathymetry_gradient(ops, geo, B)
    ref = dg.volume_rhs(ops, geo, Q, Bx, By, G_GRAV)
    dQ = to_dev(Q)
    drhs = t.empty_like(dQ)
    sem.dg_volume(h, dQ, drhs)
    t.cuda.synchronize()
    got = to_host(drhs)
    bound = _bound(ops, geo, Q, B) + 1e-300
    ratio = np.max(np.abs(got - ref) / bound)
    # the blocked layout gives the same bits; padding is neither read (NaN
    # state there) nor written (sentinel kept)
    E, _, Np = Q.shape
    nb = (E + 15) // 16
    Qb = np.full((nb * 16, 3, Np), np.nan)
    Qb[:E] = Q
    Qb = np.ascontiguousarray(Qb.reshape(nb, 16, 3, Np).transpose(0, 2, 3, 1))
    dQb = to_dev(Qb)
    drb = to_dev(np.full_like(Qb, 7.25))
    sem.dg_volume_blocked(h, dQb, drb)
    t.cuda.synchronize()
    gb = to_host(drb).transpose(0, 3, 1, 2).reshape(nb * 16, 3, Np)
    assert np.array_equal(gb[:E].view(np.uint64), got.view(np.uint64))
    assert np.all(gb[E:] == 7.25)
    return ratio, np.max(np.abs(got - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("N", range(1, 9))
def test_volume_term_matches_oracle(sem, N):
    print(f"[gpu] dg volume N={N} 70 elements", flush=True)
    h, ops, geo, X, Y, B, Q = _setup(sem, N, 7, 5)
    try:
        ratio, rel = _check_volume(sem, h, ops, geo, B, Q)
        print(f"[dg N={N}] error / componentwise bound {ratio:.2e}, max-norm rel {rel:.2e}")
        assert ratio <= 1e-13
    finally:
        sem.dg_destroy(h)


@pytest.mark.parametrize("N", [8, 3])
def test_volume_term_example_size(sem, N):
    """The example's 212,800 triangles (266 x 400 cells), every element."""
    print(f"[gpu] dg volume N={N} 212800 elements", flush=True)
    h, ops, geo, X, Y, B, Q = _setup(sem, N, 266, 400, seed=0)
    try:
        ratio, rel = _check_volume(sem, h, ops, geo, B, Q)
        print(f"[dg N={N} 212800] error / bound {ratio:.2e}, rel {rel:.2e}")
        assert ratio <= 1e-13
    finally:
        sem.dg_destroy(h)


def test_flat_bottom_and_errors(sem):
    t = torch()
    vx, vy, etov = tri_mesh(3, 2, seed=4)
    N = 4
    ops = dg.reference_operators(N)
    geo = dg.geometric_factors(vx, vy, etov)
    X, Y = dg.physical_nodes(ops, vx, vy, etov)
    _, Q = _state(X, Y)
    h = sem.dg_setup(N, vx, vy, etov, bathymetry=None, g=G_GRAV)
    try:
        zero = np.zeros_like(X)
        ratio, _ = _check_volume(sem, h, ops, geo, zero, Q)
        assert ratio <= 1e-13
        dQ = to_dev(Q)
        with pytest.raises(sem.SemError) as ei:
            sem.dg_volume(h, dQ, dQ)
        assert ei.value.code == sem.SEM_ERR_ARG
        with pytest.raises(sem.SemError) as ei:
            sem.dg_volume_blocked(h, dQ, dQ)
        assert ei.value.code == sem.SEM_ERR_ARG
    finally:
        sem.dg_destroy(h)
    bad = etov.copy()
    bad[0, 1], bad[0, 2] = bad[0, 2], bad[0, 1]  # clockwise
    for kw in ({"N": 0, "etov": etov}, {"N": 9, "etov": etov}, {"N": 3, "etov": bad},
               {"N": 3, "etov": np.where(etov == 0, 10 ** 6, etov)}):
        with pytest.raises(sem.SemError) as ei:
            sem.dg_setup(kw["N"], vx, vy, kw["etov"], g=G_GRAV)
        assert ei.value.code == sem.SEM_ERR_ARG
