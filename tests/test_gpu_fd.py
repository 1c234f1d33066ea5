"""GPU parity of the finite-difference wave step (paper section 4.1) through
the C ABI (include/fd2d.h) against the FP64 oracle (oracle/fd.py).

The kernel multiplies and adds in the oracle's order without fused
multiply-add, and its weights are correctly rounded like the oracle's exact
rationals, so the bar is bit-exactness: weights, single steps for every
stencil radius on ragged grids (strips and row chunks with partial last
ones, grids smaller than the stencil), multi-step runs of even and odd
length, the in-place update of the older level, and sampled rows at the
benchmark size (8192 x 8192)."""
import numpy as np
import pytest

from oracle import fd

from gpu_util import to_dev, to_host, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("r", range(1, 8))
def test_weights_bit_exact(sem, r):
    np.testing.assert_array_equal(_bits(sem.fd2d_weights(r)), _bits(fd.weights(r)))


GRIDS = [(300, 77), (513, 130), (256, 64), (260, 9), (7, 5), (3, 2), (1, 1),
         (1000, 1)]


@pytest.mark.parametrize("nx,ny", GRIDS)
@pytest.mark.parametrize("r", [1, 4, 7])
def test_step_bit_exact(sem, nx, ny, r):
    print(f"[gpu] fd2d step {nx}x{ny} r={r}", flush=True)
    t = torch()
    rng = np.random.default_rng(nx * 1000 + ny + r)
    uc, up = rng.uniform(-1, 1, (ny, nx)), rng.uniform(-1, 1, (ny, nx))
    dx = 2.0 / nx
    dt = 0.3 * dx
    ref = fd.step(uc, up, r, dt, dx)
    duc, dup = to_dev(uc), to_dev(up)
    dn = t.empty_like(duc)
    sem.fd2d_step(duc, dup, dn, r, dt, dx)
    t.cuda.synchronize()
    np.testing.assert_array_equal(_bits(to_host(dn)), _bits(ref))
    # the older level may be overwritten in place
    sem.fd2d_step(duc, dup, dup, r, dt, dx)
    t.cuda.synchronize()
    np.testing.assert_array_equal(_bits(to_host(dup)), _bits(ref))


@pytest.mark.parametrize("r", [2, 3, 5, 6])
def test_step_every_radius(sem, r):
    t = torch()
    nx, ny = 300, 77
    rng = np.random.default_rng(40 + r)
    uc, up = rng.uniform(-1, 1, (ny, nx)), rng.uniform(-1, 1, (ny, nx))
    dx = 2.0 / nx
    dt = 0.2 * dx
    dn = t.empty((ny, nx), dtype=t.float64, device="cuda")
    sem.fd2d_step(to_dev(uc), to_dev(up), dn, r, dt, dx)
    t.cuda.synchronize()
    np.testing.assert_array_equal(_bits(to_host(dn)), _bits(fd.step(uc, up, r, dt, dx)))


@pytest.mark.parametrize("nsteps", [12, 7, 0])
def test_run_bit_exact_and_roles(sem, nsteps):
    t = torch()
    nx, ny, r = 333, 70, 3
    dx = 2.0 / nx
    dt = 0.25 * dx
    x = -1.0 + dx * np.arange(nx)
    y = -1.0 + dx * np.arange(ny)
    X, Y = np.meshgrid(x, y)
    u0 = np.exp(-20 * (X ** 2 + Y ** 2))
    u1 = u0.copy()
    ra, rb = fd.run(u0, u1, r, dt, dx, nsteps)  # (level K-1, level K)
    da, db = to_dev(u0), to_dev(u1)
    sem.fd2d_run(da, db, r, dt, dx, nsteps)
    t.cuda.synchronize()
    older, newer = (da, db) if nsteps % 2 == 0 else (db, da)
    np.testing.assert_array_equal(_bits(to_host(newer)), _bits(rb))
    np.testing.assert_array_equal(_bits(to_host(older)), _bits(ra))


def test_benchmark_size_sampled_rows(sem):
    """8192 x 8192, r = 7 (the largest stencil): one step on the device,
    sampled rows (first and last rows and columns wrap) against the oracle
    applied to the band of 2r + 1 rows around each."""
    print("[gpu] fd2d 8192^2 r=7", flush=True)
    t = torch()
    n, r = 8192, 7
    g = t.Generator(device="cuda")
    g.manual_seed(3)
    duc = t.rand((n, n), dtype=t.float64, device="cuda", generator=g) * 2 - 1
    dup = t.rand((n, n), dtype=t.float64, device="cuda", generator=g) * 2 - 1
    dn = t.empty_like(duc)
    dx = 2.0 / n
    dt = 0.25 * dx
    sem.fd2d_step(duc, dup, dn, r, dt, dx)
    t.cuda.synchronize()
    rows = [0, 1, 6, 7, 63, 64, 4095, 8100, 8184, 8191]
    for j in rows:
        band_idx = t.tensor([(j + k) % n for k in range(-r, r + 1)], device="cuda")
        band = to_host(duc.index_select(0, band_idx))
        prev = to_host(dup[j:j + 1]).repeat(2 * r + 1, axis=0)
        ref = fd.step(band, prev, r, dt, dx)[r]
        np.testing.assert_array_equal(_bits(to_host(dn[j])), _bits(ref))


def test_argument_errors(sem):
    t = torch()
    a = t.zeros((4, 4), dtype=t.float64, device="cuda")
    b = t.zeros_like(a)
    c = t.zeros_like(a)
    for kw in ({"r": 0}, {"r": 8}):
        with pytest.raises(sem.SemError) as ei:
            sem.fd2d_step(a, b, c, kw["r"], 0.1, 0.5)
        assert ei.value.code == sem.SEM_ERR_ARG
    with pytest.raises(sem.SemError) as ei:
        sem.fd2d_step(a, b, a, 2, 0.1, 0.5)
    assert ei.value.code == sem.SEM_ERR_ARG
    with pytest.raises(sem.SemError) as ei:
        sem.fd2d_step(a, b, c, 2, 0.1, 0.0)
    assert ei.value.code == sem.SEM_ERR_ARG
    with pytest.raises(sem.SemError) as ei:
        sem.fd2d_run(a, a, 2, 0.1, 0.5, 3)
    assert ei.value.code == sem.SEM_ERR_ARG
    with pytest.raises(sem.SemError) as ei:
        sem.fd2d_run(a, b, 2, 0.1, 0.5, -1)
    assert ei.value.code == sem.SEM_ERR_ARG
    with pytest.raises(sem.SemError) as ei:
        sem.fd2d_weights(9)
    assert ei.value.code == sem.SEM_ERR_ARG
