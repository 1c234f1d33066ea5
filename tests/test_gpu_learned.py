"""GPU kernels of the learned coarse correction against the FP64 oracle, and
learned flexible-CG solves with their fallback.

Bars: forward and gradient with the same BF16-rounded weights and inputs as
the oracle differ only by FP32 accumulation and BF16 rounding of the hidden
activations: relative error <= 1e-2 and cosine >= 0.999; one Adam step
matches the oracle to 1e-6 relative; a checkpoint round-trips exactly and a
truncated or altered one is rejected; learned solves reach the FP64 true
residual tolerance, with Jacobi-PCG taking over when the network is broken."""
import numpy as np
import pytest

from oracle import mlp
from oracle import oracle as orc
from seminputs import fourier_modes, grf_features, normal

from gpu_util import bf16_round, to_dev, to_host, torch

pytestmark = pytest.mark.gpu

N = 5
N3 = (N + 1) ** 3
NIN = N3 + 8


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


def _bf16_theta(params, n_in, n_out):
    """Weights rounded to BF16 as the forward layers see them; biases FP32."""
    W1, b1, W2, b2, W3, b3 = mlp.unpack(params.astype(np.float64), n_in, 128,
                                        n_out)
    r = lambda a: bf16_round(a)[0].reshape(a.shape)
    return mlp.pack([r(W1), b1, r(W2), b2, r(W3), b3])


def _inputs(B, ldx, seed):
    x = normal((B, ldx), seed=seed)
    x[:, NIN:] = 0.0
    xb, u16 = bf16_round(x)
    return xb.reshape(B, ldx), u16.reshape(B, ldx)


def _cos(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("nout", [8, N3])
def test_forward_matches_oracle(sem, nout):
    t = torch()
    net = sem.sem_mlp_create(NIN, 128, nout, seed=3)
    try:
        info = sem.sem_mlp_info(net)
        ldx = info["n_in_padded"]
        B = 150  # several 64-row workgroups and a ragged tail
        xb, u16 = _inputs(B, ldx, seed=1)
        params = sem.sem_mlp_get_params(net)
        params[128 * NIN:128 * NIN + 128] = normal(128, seed=5) * 0.1  # biases
        sem.sem_mlp_set_params(net, params)
        Y = t.empty((B, nout), dtype=t.float32, device="cuda")
        sem.sem_mlp_forward(net, to_dev(u16.view(np.int16), t.int16), ldx, B, Y)
        t.cuda.synchronize()
        ref = mlp.forward(_bf16_theta(params, NIN, nout), xb[:, :NIN], NIN, 128,
                          nout)
        got = to_host(Y).astype(np.float64)
        rel = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"[mlp fwd] rel {rel:.2e} cos {_cos(got.ravel(), ref.ravel()):.6f}")
        assert rel <= 1e-2 and _cos(got.ravel(), ref.ravel()) >= 0.999
    finally:
        sem.sem_mlp_destroy(net)


@pytest.mark.parametrize("nout", [8, N3])
def test_gradient_and_adam_match_oracle(sem, nout):
    t = torch()
    net = sem.sem_mlp_create(NIN, 128, nout, seed=4)
    try:
        ldx = sem.sem_mlp_info(net)["n_in_padded"]
        B = 96
        xb, u16 = _inputs(B, ldx, seed=2)
        T = normal((B, N3), seed=3).astype(np.float32)
        params = sem.sem_mlp_get_params(net)
        grad = t.empty(params.size, dtype=t.float32, device="cuda")
        Xd = to_dev(u16.view(np.int16), t.int16)
        loss = sem.sem_mlp_loss_grad(net, Xd, ldx, to_dev(T, t.float32), B, N, grad)
        t.cuda.synchronize()
        xi, _ = orc.gll(N)
        P = mlp.prolongation(xi) if nout == 8 else np.eye(N3)
        lref, gref = mlp.loss_and_grad(_bf16_theta(params, NIN, nout),
                                       xb[:, :NIN], T.astype(np.float64), P, NIN,
                                       128, nout)
        g = to_host(grad).astype(np.float64)
        rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
        print(f"[mlp grad] loss {loss:.6e} vs {lref:.6e}; grad rel {rel:.2e} "
              f"cos {_cos(g, gref):.6f}")
        assert abs(loss - lref) <= 1e-2 * lref
        assert rel <= 1e-2 and _cos(g, gref) >= 0.999
        # one Adam step on the GPU gradient
        sem.sem_mlp_adam(net, grad, lr=1e-3)
        t.cuda.synchronize()
        new = sem.sem_mlp_get_params(net).astype(np.float64)
        th_ref, _, _ = mlp.adam_step(params.astype(np.float64), g,
                                     np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
        err = np.max(np.abs(new - th_ref)) / np.max(np.abs(th_ref))
        print(f"[adam] rel err {err:.2e}")
        assert err <= 1e-6
        assert sem.sem_mlp_info(net)["adam_steps"] == 1
    finally:
        sem.sem_mlp_destroy(net)


def test_checkpoint_roundtrip_and_rejection(sem, tmp_path):
    net = sem.sem_mlp_create(NIN, 128, N3, seed=5)
    path = tmp_path / "net.ckpt"
    try:
        sem.sem_mlp_set_damping(net, 0.15, -0.05)
        sem.sem_mlp_save(net, path)
        net2 = sem.sem_mlp_load(path)
        try:
            np.testing.assert_array_equal(sem.sem_mlp_get_params(net),
                                          sem.sem_mlp_get_params(net2))
            assert sem.sem_mlp_get_damping(net2) == (0.15, -0.05)
        finally:
            sem.sem_mlp_destroy(net2)
        raw = path.read_bytes()
        bad = tmp_path / "truncated.ckpt"
        bad.write_bytes(raw[: len(raw) // 2])
        with pytest.raises(sem.SemError) as ei:
            sem.sem_mlp_load(bad)
        assert ei.value.code == sem.SEM_ERR_ARG
        flipped = bytearray(raw)
        flipped[len(raw) // 3] ^= 0x40
        bad.write_bytes(bytes(flipped))
        with pytest.raises(sem.SemError):
            sem.sem_mlp_load(bad)
    finally:
        sem.sem_mlp_destroy(net)


# ---------------------------------------------------------------------------
# learned solves on a variable-coefficient problem
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def problem(sem):
    t = torch()
    kap = grf_features(seed=7, M=512, ell=0.1, sigma=1.0)
    h = sem.sem_setup(N, 6, 6, 6, mapping=sem.SEM_MAP_AFFINE, kappa=kap)
    _, nL, _ = sem.sem_query(h)

    def rhs(seed):
        b = t.empty(nL, dtype=t.float64, device="cuda")
        sem.sem_rhs(h, b, sem.SEM_SRC_FOURIER, fourier_modes(seed=seed))
        return b

    train = [rhs(100 + q) for q in range(4)]
    test = [rhs(900 + q) for q in range(2)]
    net = sem.sem_mlp_create(NIN, 128, N3, seed=11)
    untrained = sem.sem_mlp_create(NIN, 128, N3, seed=11)
    print("[gpu] training the correction network", flush=True)
    rep = sem.sem_learn_train(h, net, train, n_pairs=4000, snapshot_every=8,
                              max_snapshots=32, epochs=20, batch=256, lr=1e-3,
                              solve_rtol=1e-11, seed=1)
    print(f"[train] {rep}", flush=True)
    t.cuda.synchronize()
    # the ablation uses the trained network's damping and progress judge
    sem.sem_mlp_set_damping(untrained, *sem.sem_mlp_get_damping(net))
    yield h, net, untrained, test, nL, rep
    sem.sem_learn_attach(h, None)
    sem.sem_mlp_destroy(net)
    sem.sem_mlp_destroy(untrained)
    sem.sem_destroy(h)


def _solve(sem, h, b, **kw):
    t = torch()
    x = t.zeros_like(b)
    st = sem.sem_pcg_solve(h, b, x, raise_on_fail=False, **kw)
    t.cuda.synchronize()
    return x, st


def test_training_reduces_loss(problem):
    h, net, untrained, test, nL, rep = problem
    assert rep["pairs"] == 4000 and rep["snapshots"] > 0
    assert rep["last_loss"] < rep["first_loss"]
    assert rep["jacobi_rate"] < 0
    assert rep["damping"] in (0.0, 0.2, 0.15, 0.1, 0.05)
    if rep["damping"] > 0:
        assert rep["val_iters_learned"] < rep["val_iters_jacobi"]


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_learned_gain_report(sem, problem, inner):
    h, net, untrained, test, nL, rep = problem
    prec = sem.SEM_FP64 if inner == "fp64" else sem.SEM_FP32
    kw = dict(rtol=1e-8, maxit=20000, inner_prec=prec, inner_rtol=1e-3,
              check_every=8)
    for b in test:
        xj, sj = _solve(sem, h, b, pc=sem.SEM_PC_JACOBI, **kw)
        sem.sem_learn_attach(h, untrained)
        xu, su = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        sem.sem_learn_attach(h, net)
        xt, stt = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        print(f"[gain {inner}] jacobi {sj['iters']} it {sj['seconds']*1e3:.1f} ms | "
              f"untrained {su['iters']} it fb={su['fell_back']} | "
              f"trained {stt['iters']} it fb={stt['fell_back']} "
              f"{stt['seconds']*1e3:.1f} ms")
        for st in (sj, su, stt):
            assert st["status"] == 0 and st["final_rel_res"] <= 1e-8
        # validated damping and the progress judge keep the trained solve
        # within a small margin of Jacobi-PCG
        assert stt["iters"] <= 1.3 * sj["iters"] + 10
        ref = to_host(xj)
        for x in (xu, xt):
            assert np.linalg.norm(to_host(x) - ref) <= 1e-6 * np.linalg.norm(ref)


def test_fallback_on_broken_networks(sem, problem):
    h, net, untrained, test, nL, rep = problem
    b = test[0]
    kw = dict(rtol=1e-8, maxit=20000, inner_prec=sem.SEM_FP64, check_every=8)
    _, sj = _solve(sem, h, b, pc=sem.SEM_PC_JACOBI, **kw)
    good = sem.sem_mlp_get_params(net)
    broken = sem.sem_mlp_create(NIN, 128, N3, seed=0)
    try:
        sem.sem_learn_attach(h, broken)
        # NaN output bias (a NaN in the first layer is cut off by the ReLU):
        # breakdown detected, Jacobi-PCG takes over
        p = good.copy()
        p[-5:] = np.nan
        sem.sem_mlp_set_params(broken, p)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        assert st["status"] == 0 and st["fell_back"] == 1
        assert st["final_rel_res"] <= 1e-8
        # zero weights: the correction vanishes and flexible CG is Jacobi-PCG
        sem.sem_mlp_set_params(broken, np.zeros_like(good))
        sem.sem_mlp_set_damping(broken, 1.0, 0.0)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        assert st["status"] == 0 and st["fell_back"] == 0
        assert abs(st["iters"] - sj["iters"]) <= 3
        # sign-flipped output layer: still converges (with or without fallback)
        q = good.copy()
        n3w = 128 * NIN + 128 + 128 * 128 + 128
        q[n3w:] = -q[n3w:]
        sem.sem_mlp_set_params(broken, q)
        sem.sem_mlp_set_damping(broken, 1.0, 0.0)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, **kw)
        assert st["status"] == 0 and st["final_rel_res"] <= 1e-8
        # mixed precision with NaN weights
        sem.sem_mlp_set_params(broken, p)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, rtol=1e-8, maxit=20000,
                       inner_prec=sem.SEM_FP32, inner_rtol=1e-3, check_every=8)
        assert st["status"] == 0 and st["fell_back"] == 1
        # an iteration budget that cannot be met ends cleanly
        sem.sem_learn_attach(h, net)
        _, st = _solve(sem, h, b, pc=sem.SEM_PC_LEARNED, rtol=1e-8, maxit=2,
                       inner_prec=sem.SEM_FP64, check_every=1)
        assert st["status"] == sem.SEM_ERR_NOT_CONVERGED
    finally:
        sem.sem_learn_attach(h, net)
        sem.sem_mlp_destroy(broken)


def test_learned_needs_attached_network(sem):
    t = torch()
    h = sem.sem_setup(3, 2, 2, 2)
    try:
        _, nL, _ = sem.sem_query(h)
        b = t.ones(nL, dtype=t.float64, device="cuda")
        x = t.zeros_like(b)
        with pytest.raises(sem.SemError) as ei:
            sem.sem_pcg_solve(h, b, x, pc=sem.SEM_PC_LEARNED)
        assert ei.value.code == sem.SEM_ERR_STATE
        wrong = sem.sem_mlp_create(100, 128, 64 + 0)
        try:
            with pytest.raises(sem.SemError):
                sem.sem_learn_attach(h, wrong)
        finally:
            sem.sem_mlp_destroy(wrong)
    finally:
        sem.sem_destroy(h)


def test_learned_precond_apply_matches_oracle(sem, problem):
    """z = dinv r + averaged correction: the GPU pipeline (features, BF16
    MFMA network, scaling, averaging over copies) against the oracle's
    composition with the same BF16-rounded weights and inputs."""
    t = torch()
    h, net, untrained, test, nL, rep = problem
    kap = grf_features(seed=7, M=512, ell=0.1, sigma=1.0)
    m = orc.mesh(N, 6, 6, 6, orc.MAP_AFFINE, 1, kap)
    damping, rate = sem.sem_mlp_get_damping(net)
    sem.sem_mlp_set_damping(net, 0.1, rate)
    sem.sem_learn_attach(h, net)
    try:
        params = sem.sem_mlp_get_params(net)
        theta = _bf16_theta(params, NIN, N3)
        n1, E = N + 1, m.E
        kv = np.array([[m.kappa[e * N3 + (v & 1) * N + n1 * ((v >> 1) & 1) * N
                                + n1 * n1 * (v >> 2) * N] for v in range(8)]
                       for e in range(E)])
        lk = np.log(kv)
        kfeat = lk - lk.mean(1, keepdims=True)
        invkh = 1.0 / (kv.mean(1) * (1.0 / 6))
        dinv = orc.jacobi_dinv_global(m)
        gmask = np.zeros(m.nG, bool)
        gmask[m.l2g[m.bmask.astype(bool)]] = True
        rg = normal(m.nG, seed=8)
        rg[gmask] = 0.0
        R = rg[m.l2g].reshape(E, N3)
        s = np.linalg.norm(R, axis=1)
        X = bf16_round(np.concatenate([R / s[:, None], kfeat], 1))[0].reshape(E, NIN)
        cL = 0.1 * (s * invkh)[:, None] * mlp.forward(theta, X, NIN, 128, N3)
        c = np.zeros(m.nG)
        np.add.at(c, m.l2g, cL.reshape(-1))
        c = np.where(gmask, 0.0, c / np.diff(m.offsets))
        rL = to_dev(orc.to_local(m, rg))
        z = t.empty_like(rL)
        sem.sem_precond_apply(h, sem.SEM_PC_LEARNED, sem.SEM_FP64, rL, z)
        t.cuda.synchronize()
        cg = orc.to_global(m, to_host(z)) - dinv * rg
        rel = np.linalg.norm(cg - c) / np.linalg.norm(c)
        print(f"[learned precond] correction rel {rel:.2e} cos {_cos(cg, c):.6f}")
        assert rel <= 1e-2 and _cos(cg, c) >= 0.999
    finally:
        sem.sem_mlp_set_damping(net, damping, rate)
