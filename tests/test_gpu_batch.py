"""Batched uneven solves (persistent launches over (solve, tile) work items,
one captured graph per CG step) against individual solves and the oracle.

A solve must give the same bits alone or inside a batch (every reduction has
a fixed per-solve partition and order), and its solution must match the
oracle's PCG solution as in the single-solve tests."""
import os

import numpy as np
import pytest

from oracle import oracle as orc
from seminputs import batch_configs, fourier_modes

from gpu_util import to_host, torch

pytestmark = pytest.mark.gpu

# small uneven batch: (n, N) cubic grids, orders from {3, 5, 7}
SMALL = [(2, 3), (3, 5), (2, 7), (4, 3), (3, 7), (2, 5)]


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


@pytest.fixture(scope="module")
def batch(sem):
    t = torch()
    hs, bs = [], []
    for q, (n, N) in enumerate(SMALL):
        h = sem.sem_setup(N, n, n, n, mapping=sem.SEM_MAP_SINE_CYCLIC)
        _, nL, _ = sem.sem_query(h)
        b = t.empty(nL, dtype=t.float64, device="cuda")
        sem.sem_rhs(h, b, sem.SEM_SRC_FOURIER, fourier_modes(seed=1000 + q))
        hs.append(h)
        bs.append(b)
    t.cuda.synchronize()
    bt = sem.sem_batch_create(hs)
    yield hs, bs, bt
    sem.sem_batch_destroy(bt)
    for h in hs:
        sem.sem_destroy(h)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_batch_equals_individual_solves_bitwise(sem, batch, prec):
    print(f"[gpu] batch vs individual, inner {prec}", flush=True)
    t = torch()
    hs, bs, bt = batch
    p = {"fp64": sem.SEM_FP64, "fp32": sem.SEM_FP32, "bf16": sem.SEM_BF16}[prec]
    kw = dict(rtol=1e-10, maxit=4000, inner_prec=p, inner_rtol=1e-2,
              check_every=8)
    xs = [t.zeros_like(b) for b in bs]
    code, stats = sem.sem_batch_pcg_solve(bt, bs, xs, **kw)
    t.cuda.synchronize()
    assert code == 0
    for q, (h, b) in enumerate(zip(hs, bs)):
        x1 = t.zeros_like(b)
        st1 = sem.sem_pcg_solve(h, b, x1, **kw)
        t.cuda.synchronize()
        assert stats[q]["iters"] == st1["iters"], (q, stats[q], st1)
        assert stats[q]["outer_iters"] == st1["outer_iters"]
        assert stats[q]["final_rel_res"] <= 1e-10
        assert t.equal(xs[q], x1), q


def test_batch_matches_oracle(sem, batch):
    print("[gpu] batch vs oracle", flush=True)
    t = torch()
    hs, bs, bt = batch
    xs = [t.zeros_like(b) for b in bs]
    code, stats = sem.sem_batch_pcg_solve(bt, bs, xs, rtol=1e-10, maxit=4000,
                                          inner_prec=sem.SEM_FP32,
                                          inner_rtol=1e-2, check_every=8)
    t.cuda.synchronize()
    assert code == 0
    for q in (0, 1, 4):
        n, N = SMALL[q]
        m = orc.mesh(N, n, n, n, orc.MAP_SINE_CYCLIC)
        k, a, phi = fourier_modes(seed=1000 + q)
        bo = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
        xo, so, _, _ = orc.pcg(m, bo, 1e-12, 5000)
        xg = orc.to_global(m, to_host(xs[q]))
        rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
        print(f"[batch solve {q} n={n} N={N}] iters {stats[q]['iters']} "
              f"outer {stats[q]['outer_iters']} rel err {rel:.2e}")
        assert rel <= 1e-7


def test_autotuner_and_cache(sem, batch, tmp_path):
    hs, bs, bt = batch
    path = str(tmp_path / "tune.json")
    os.environ["SEM_AUTOTUNE_CACHE"] = path
    try:
        b1, g1, us1 = sem.sem_batch_tune(bt, sem.SEM_FP32)
        assert b1 in (64, 128, 256) and g1 in (0, 4, 8, 16, 32) and us1 > 0
        text = open(path).read()
        assert "prec1" in text and f"[{b1}, {g1}]" in text
        b2, g2, us2 = sem.sem_batch_tune(bt, sem.SEM_FP32)
        assert (b2, g2, us2) == (b1, g1, -1.0)
    finally:
        del os.environ["SEM_AUTOTUNE_CACHE"]
    # solves still converge with the tuned launch shape
    t = torch()
    xs = [t.zeros_like(b) for b in bs]
    code, stats = sem.sem_batch_pcg_solve(bt, bs, xs, rtol=1e-9, maxit=4000,
                                          inner_prec=sem.SEM_FP32)
    assert code == 0 and all(s["final_rel_res"] <= 1e-9 for s in stats)


def test_unsupported_order_mix_rejected(sem):
    h1 = sem.sem_setup(2, 2, 2, 2)
    h2 = sem.sem_setup(3, 2, 2, 2)
    try:
        with pytest.raises(sem.SemError) as ei:
            sem.sem_batch_create([h1, h2])
        assert ei.value.code == sem.SEM_ERR_ARG
        with pytest.raises(sem.SemError):
            sem.sem_batch_create([h1, h1])
    finally:
        sem.sem_destroy(h1)
        sem.sem_destroy(h2)


def test_batch_config_generator_is_uneven():
    cfg = batch_configs(256, seed=0)
    ns = [n for n, _ in cfg]
    Ns = [N for _, N in cfg]
    assert min(ns) >= 6 and max(ns) <= 24 and set(Ns) == {3, 5, 7}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_order8_block_holds_an_element(sem, prec, tmp_path):
    """N = 8 has 81 (i, j) columns per element, one thread each: a batch of
    order-8 solves never runs the batched operator with 64-thread
    workgroups, whether from its defaults, the tuner's candidates or a
    cache entry that asks for them; its solves equal the single solves bit
    for bit and agree with the oracle."""
    print(f"[gpu] batch of order-8 solves, inner {prec}", flush=True)
    t = torch()
    p = {"fp64": sem.SEM_FP64, "fp32": sem.SEM_FP32}[prec]
    sizes = [(2, 2, 2), (3, 2, 2)]
    hs, bs = [], []
    for q, (ex, ey, ez) in enumerate(sizes):
        h = sem.sem_setup(8, ex, ey, ez, mapping=sem.SEM_MAP_SINE_CYCLIC)
        _, nL, _ = sem.sem_query(h)
        b = t.empty(nL, dtype=t.float64, device="cuda")
        sem.sem_rhs(h, b, sem.SEM_SRC_FOURIER, fourier_modes(seed=1100 + q))
        hs.append(h)
        bs.append(b)
    bt = sem.sem_batch_create(hs)
    path = str(tmp_path / "tune8.json")
    os.environ["SEM_AUTOTUNE_CACHE"] = path
    try:
        kw = dict(rtol=1e-10, maxit=4000, inner_prec=p, inner_rtol=1e-2,
                  check_every=8)
        # defaults first, then a cache entry rewritten to 64 threads
        for stage in ("default", "cache64"):
            if stage == "cache64":
                b1, g1, _ = sem.sem_batch_tune(bt, p)
                assert b1 >= 128
                text = open(path).read().replace(f"[{b1}, {g1}]", "[64, 0]")
                open(path, "w").write(text)
                b2, g2, us2 = sem.sem_batch_tune(bt, p)
                assert b2 >= 128 and us2 > 0, (b2, g2, us2)
            xs = [t.zeros_like(b) for b in bs]
            code, stats = sem.sem_batch_pcg_solve(bt, bs, xs, **kw)
            t.cuda.synchronize()
            assert code == 0, stats
            for q, (h, b) in enumerate(zip(hs, bs)):
                x1 = t.zeros_like(b)
                st1 = sem.sem_pcg_solve(h, b, x1, **kw)
                t.cuda.synchronize()
                assert stats[q]["iters"] == st1["iters"], (stage, q)
                assert t.equal(xs[q], x1), (stage, q)
        for q, (ex, ey, ez) in enumerate(sizes):
            m = orc.mesh(8, ex, ey, ez, orc.MAP_SINE_CYCLIC)
            k, a, phi = fourier_modes(seed=1100 + q)
            bo = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
            xo, _, _, _ = orc.pcg(m, bo, 1e-12, 5000)
            rel = (np.linalg.norm(orc.to_global(m, to_host(xs[q])) - xo)
                   / np.linalg.norm(xo))
            print(f"[batch N=8 solve {q}] rel err {rel:.2e}")
            assert rel <= 1e-7
    finally:
        del os.environ["SEM_AUTOTUNE_CACHE"]
        sem.sem_batch_destroy(bt)
        for h in hs:
            sem.sem_destroy(h)


@pytest.mark.parametrize("N", [5, 8])
def test_matrix_core_batch_equals_individual_solves_bitwise(sem, N):
    """A batch of one order around the matrix-core inner operator (the
    batched persistent kernel) gives the bits of the same solves run alone
    (the single-solve kernel): both store the element energies in one fixed
    order, and the update kernels share their per-chunk code."""
    print(f"[gpu] matrix-core batch vs individual, N = {N}", flush=True)
    t = torch()
    hs, bs = [], []
    for q, n in enumerate((2, 3, 2)):
        h = sem.sem_setup(N, n, n + q % 2, n, mapping=sem.SEM_MAP_SINE_CYCLIC)
        _, nL, _ = sem.sem_query(h)
        b = t.empty(nL, dtype=t.float64, device="cuda")
        sem.sem_rhs(h, b, sem.SEM_SRC_FOURIER, fourier_modes(seed=1200 + q))
        hs.append(h)
        bs.append(b)
    bt = sem.sem_batch_create(hs)
    try:
        kw = dict(rtol=1e-10, maxit=4000, inner_prec=sem.SEM_BF16_MFMA, inner_rtol=1e-2,
                  check_every=8)
        xs = [t.zeros_like(b) for b in bs]
        code, stats = sem.sem_batch_pcg_solve(bt, bs, xs, **kw)
        t.cuda.synchronize()
        assert code == 0
        for q, (h, b) in enumerate(zip(hs, bs)):
            x1 = t.zeros_like(b)
            st1 = sem.sem_pcg_solve(h, b, x1, **kw)
            t.cuda.synchronize()
            assert stats[q]["iters"] == st1["iters"], (q, stats[q], st1)
            assert stats[q]["outer_iters"] == st1["outer_iters"]
            assert stats[q]["final_rel_res"] <= 1e-10
            assert t.equal(xs[q], x1), q
    finally:
        sem.sem_batch_destroy(bt)
        for h in hs:
            sem.sem_destroy(h)
