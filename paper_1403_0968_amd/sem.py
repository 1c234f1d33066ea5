"""ctypes binding of libsem.so (argument marshalling only).

The functions carry the names of the C ABI in ``include/sem.h``.  Vectors are
torch tensors on the GPU (``tensor.data_ptr()`` is passed); PyTorch provides
device memory and streams only -- every step of the computation runs in the
library's HIP kernels.  Loading fails loudly when ``libsem.so`` has not been
built (``python -m paper_1403_0968_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsem.so")

SEM_OK, SEM_ERR_ARG, SEM_ERR_HIP, SEM_ERR_OOM = 0, 1, 2, 3
SEM_ERR_NOT_CONVERGED, SEM_ERR_BREAKDOWN, SEM_ERR_STATE = 4, 5, 6
SEM_FP64, SEM_FP32, SEM_BF16, SEM_BF16_PLAIN_D, SEM_BF16_MFMA = 0, 1, 2, 3, 4
SEM_PC_NONE, SEM_PC_JACOBI, SEM_PC_LEARNED = 0, 1, 2
SEM_MAP_AFFINE, SEM_MAP_SINE_X, SEM_MAP_SINE_CYCLIC = 0, 1, 2
SEM_SRC_FOURIER, SEM_SRC_SINE = 0, 1
(SEM_ARR_L2G, SEM_ARR_PERM, SEM_ARR_OFFSETS, SEM_ARR_MULT, SEM_ARR_MASK,
 SEM_ARR_COORDS, SEM_ARR_GEOM, SEM_ARR_MASS, SEM_ARR_DIAG,
 SEM_ARR_DINV, SEM_ARR_HMASS) = range(11)

EXPORTED = ["sem_setup", "sem_destroy", "sem_query", "sem_export", "sem_ax",
            "sem_gs", "sem_rhs", "sem_precond_apply", "sem_pcg_solve",
            "sem_pcg_solve_noalloc",
            "sem_batch_create", "sem_batch_destroy", "sem_batch_tune",
            "sem_batch_pcg_solve", "sem_mlp_create", "sem_mlp_destroy",
            "sem_mlp_info", "sem_mlp_get_params", "sem_mlp_set_params",
            "sem_mlp_set_precision", "sem_mlp_get_precision",
            "sem_mlp_forward", "sem_mlp_adam", "sem_mlp_set_damping",
            "sem_mlp_get_damping", "sem_mlp_save", "sem_mlp_load",
            "sem_learn_attach", "sem_learn_attach_exact", "sem_learn_train",
            "sem_learn_coarse_exact", "sem_mlp_loss_grad_factor",
            "fd2d_weights", "fd2d_step", "fd2d_run", "dg_reference_nodes",
            "dg_setup", "dg_destroy", "dg_query", "dg_export", "dg_volume",
            "dg_volume_blocked",
            "sem_last_error"]


class sem_mesh_desc(C.Structure):
    _fields_ = [("N", C.c_int32), ("ex", C.c_int32), ("ey", C.c_int32),
                ("ez", C.c_int32), ("dirichlet", C.c_int32),
                ("mapping", C.c_int32), ("alpha", C.c_double),
                ("kappa_nfeat", C.c_int32),
                ("kappa_omega", C.POINTER(C.c_double)),
                ("kappa_b", C.POINTER(C.c_double)),
                ("kappa_sigma", C.c_double),
                ("alpha_nodal", C.POINTER(C.c_double)),
                ("periodic", C.c_int32)]


class sem_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nmodes", C.c_int32),
                ("k", C.POINTER(C.c_double)), ("a", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double))]


class sem_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("pc", C.c_int32),
                ("inner_prec", C.c_int32), ("inner_rtol", C.c_double),
                ("check_every", C.c_int32), ("use_graph", C.c_int32)]


class sem_train_opts(C.Structure):
    _fields_ = [("n_pairs", C.c_int32), ("snapshot_every", C.c_int32),
                ("max_snapshots", C.c_int32), ("epochs", C.c_int32),
                ("batch", C.c_int32), ("reserved", C.c_int32),
                ("lr", C.c_double), ("solve_rtol", C.c_double),
                ("seed", C.c_uint64)]


class sem_train_report(C.Structure):
    _fields_ = [("pairs", C.c_int32), ("epochs", C.c_int32),
                ("snapshots", C.c_int32), ("reserved", C.c_int32),
                ("first_loss", C.c_double), ("last_loss", C.c_double),
                ("data_seconds", C.c_double), ("train_seconds", C.c_double),
                ("validate_seconds", C.c_double), ("damping", C.c_double),
                ("jacobi_rate", C.c_double), ("val_iters_jacobi", C.c_int32),
                ("val_iters_learned", C.c_int32), ("val_iters", C.c_int32 * 4)]


class sem_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32),
                ("status", C.c_int32), ("fell_back", C.c_int32),
                ("final_rel_res", C.c_double), ("seconds", C.c_double),
                ("outer_contraction", C.c_double)]


_lib = None


def lib():
    """Load libsem.so; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch's HIP runtime must be the process's only HIP runtime: importing
    # torch first makes the loader resolve libsem.so's libamdhip64.so.7 to the
    # copy torch already loaded, so torch streams and allocations are valid
    # handles for the library.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run python -m paper_1403_0968_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.sem_setup.argtypes = [C.POINTER(sem_mesh_desc), vp, C.POINTER(vp)]
    L.sem_destroy.argtypes = [vp]
    L.sem_query.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.sem_export.argtypes = [vp, i32, vp, i64, vp]
    L.sem_ax.argtypes = [vp, i32, vp, vp, vp]
    L.sem_gs.argtypes = [vp, i32, vp, vp]
    L.sem_rhs.argtypes = [vp, C.POINTER(sem_source), vp, vp]
    L.sem_precond_apply.argtypes = [vp, i32, i32, vp, vp, vp]
    L.sem_pcg_solve.argtypes = [vp, C.POINTER(sem_solve_opts), vp, vp,
                                C.POINTER(sem_solve_stats), vp]
    L.sem_pcg_solve_noalloc.argtypes = [vp, C.POINTER(sem_solve_opts), vp, vp,
                                C.POINTER(sem_solve_stats), vp]
    L.sem_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp)]
    L.sem_batch_destroy.argtypes = [vp]
    L.sem_batch_tune.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32),
                                 C.POINTER(C.c_double)]
    L.sem_batch_pcg_solve.argtypes = [vp, C.POINTER(sem_solve_opts),
                                      C.POINTER(vp), C.POINTER(vp),
                                      C.POINTER(sem_solve_stats), vp]
    L.sem_mlp_create.argtypes = [i32, i32, i32, C.c_uint64, C.POINTER(vp)]
    L.sem_mlp_destroy.argtypes = [vp]
    L.sem_mlp_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32),
                               C.POINTER(i32), C.POINTER(i32), C.POINTER(i64),
                               C.POINTER(i64)]
    L.sem_mlp_get_params.argtypes = [vp, vp, i64]
    L.sem_mlp_set_params.argtypes = [vp, vp, i64]
    L.sem_mlp_forward.argtypes = [vp, vp, i32, i32, vp, vp]
    L.sem_mlp_set_precision.argtypes = [vp, i32]
    L.sem_mlp_get_precision.argtypes = [vp, C.POINTER(i32)]
    L.sem_mlp_loss_grad_factor.argtypes = [vp, vp, i32, vp, i32, i32, vp,
                                           C.POINTER(C.c_double), vp]
    L.sem_learn_coarse_exact.argtypes = [vp, vp, C.POINTER(i32), vp]
    L.sem_mlp_adam.argtypes = [vp, vp, C.c_double, C.c_double, C.c_double,
                               C.c_double, vp]
    L.sem_mlp_set_damping.argtypes = [vp, C.c_double, C.c_double]
    L.sem_mlp_get_damping.argtypes = [vp, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
    L.sem_mlp_save.argtypes = [vp, C.c_char_p]
    L.sem_mlp_load.argtypes = [C.c_char_p, C.POINTER(vp)]
    L.sem_learn_attach.argtypes = [vp, vp]
    L.sem_learn_attach_exact.argtypes = [vp, C.c_double]
    L.sem_learn_train.argtypes = [vp, vp, C.POINTER(vp), i32,
                                  C.POINTER(sem_train_opts),
                                  C.POINTER(sem_train_report), vp]
    L.fd2d_weights.argtypes = [i32, C.POINTER(C.c_double)]
    L.fd2d_step.argtypes = [vp, vp, vp, C.c_int64, C.c_int64, i32, C.c_double,
                            C.c_double, vp]
    L.fd2d_run.argtypes = [vp, vp, C.c_int64, C.c_int64, i32, C.c_double,
                           C.c_double, i32, vp]
    L.dg_reference_nodes.argtypes = [i32, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
    L.dg_setup.argtypes = [i32, C.c_int64, C.POINTER(C.c_double),
                           C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_int32),
                           C.POINTER(C.c_double), C.c_double, vp, C.POINTER(vp)]
    L.dg_destroy.argtypes = [vp]
    L.dg_query.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    L.dg_export.argtypes = [vp, i32, vp, C.c_int64, vp]
    L.dg_volume.argtypes = [vp, vp, vp, vp]
    L.dg_volume_blocked.argtypes = [vp, vp, vp, vp]
    L.sem_last_error.argtypes = []
    L.sem_last_error.restype = C.c_char_p
    for name in EXPORTED[:-1]:
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


class SemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sem status {code}: {msg}")
        self.code = code


def _check(code):
    if code != SEM_OK:
        raise SemError(code, lib().sem_last_error().decode())
    return code


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(a):
    """Host double array (anything numpy accepts) -> (keepalive, pointer)."""
    import numpy as np
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr, arr.ctypes.data_as(C.POINTER(C.c_double))


# ----------------------------------------------------------------------------
# thin wrappers with the C names
# ----------------------------------------------------------------------------

def sem_setup(N, ex, ey, ez, mapping=SEM_MAP_AFFINE, dirichlet=1,
              kappa=None, stream=None, alpha=0.0, alpha_nodal=None, periodic=0):
    """kappa: None or (omega[M,3], b[M], sigma).  alpha: constant mass
    coefficient; alpha_nodal: host array of n_local values (replaces the
    constant).  periodic: bit 1 x, 2 y, 4 z.  Returns an opaque handle."""
    d = sem_mesh_desc()
    d.N, d.ex, d.ey, d.ez = N, ex, ey, ez
    d.dirichlet, d.mapping, d.alpha = int(dirichlet), int(mapping), float(alpha)
    d.periodic = int(periodic)
    keep = []
    if alpha_nodal is not None:
        al_a, al_p = _dptr(alpha_nodal)
        n_local = ex * ey * ez * (N + 1) ** 3
        if al_a.ndim != 1 or al_a.shape[0] != n_local:
            raise ValueError(f"alpha_nodal needs {n_local} values (n_local), "
                             f"got shape {al_a.shape}")
        keep.append(al_a)
        d.alpha_nodal = al_p
    if kappa is not None:
        om, b, sigma = kappa
        om_a, om_p = _dptr(om)
        b_a, b_p = _dptr(b)
        keep += [om_a, b_a]
        d.kappa_nfeat = int(b_a.shape[0])
        d.kappa_omega, d.kappa_b, d.kappa_sigma = om_p, b_p, float(sigma)
    h = C.c_void_p()
    _check(lib().sem_setup(C.byref(d), _stream(stream), C.byref(h)))
    return h


def sem_destroy(h):
    _check(lib().sem_destroy(h))


def sem_query(h):
    E, nL, nG = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().sem_query(h, C.byref(E), C.byref(nL), C.byref(nG)))
    return E.value, nL.value, nG.value


def sem_export(h, which, dst, stream=None):
    _check(lib().sem_export(h, int(which), _ptr(dst),
                            dst.numel() * dst.element_size(), _stream(stream)))


def sem_ax(h, prec, u, w, stream=None):
    _check(lib().sem_ax(h, int(prec), _ptr(u), _ptr(w), _stream(stream)))


def sem_gs(h, prec, v, stream=None):
    _check(lib().sem_gs(h, int(prec), _ptr(v), _stream(stream)))


def sem_rhs(h, b, kind=SEM_SRC_FOURIER, modes=None, stream=None):
    """modes: (k[nm,3], a[nm], phi[nm]) for SEM_SRC_FOURIER."""
    s = sem_source()
    s.kind = int(kind)
    keep = []
    if kind == SEM_SRC_FOURIER:
        k, a, phi = modes
        ka, kp = _dptr(k)
        aa, ap = _dptr(a)
        pa, pp = _dptr(phi)
        keep += [ka, aa, pa]
        s.nmodes = int(aa.shape[0])
        s.k, s.a, s.phi = kp, ap, pp
    _check(lib().sem_rhs(h, C.byref(s), _ptr(b), _stream(stream)))


def sem_precond_apply(h, pc, prec, r, z, stream=None):
    _check(lib().sem_precond_apply(h, int(pc), int(prec), _ptr(r), _ptr(z),
                                   _stream(stream)))


def sem_pcg_solve(h, b, x, rtol=1e-8, maxit=10000, pc=SEM_PC_JACOBI,
                  inner_prec=SEM_FP64, inner_rtol=1e-2, check_every=16,
                  use_graph=1, stream=None, raise_on_fail=True):
    o = sem_solve_opts()
    o.rtol, o.maxit, o.pc = float(rtol), int(maxit), int(pc)
    o.inner_prec, o.inner_rtol = int(inner_prec), float(inner_rtol)
    o.check_every, o.use_graph = int(check_every), int(use_graph)
    st = sem_solve_stats()
    code = lib().sem_pcg_solve(h, C.byref(o), _ptr(b), _ptr(x), C.byref(st),
                               _stream(stream))
    if raise_on_fail and code != SEM_OK:
        _check(code)
    return {"status": code, "iters": st.iters, "outer_iters": st.outer_iters,
            "fell_back": st.fell_back,
            "final_rel_res": st.final_rel_res, "seconds": st.seconds,
            "outer_contraction": st.outer_contraction}


def sem_pcg_solve_noalloc(h, b, x, rtol=1e-8, maxit=10000, pc=SEM_PC_JACOBI,
                          check_every=16, stream=None, raise_on_fail=True):
    """Plain FP64 PCG with no allocation inside the library (its buffers
    live in a fixed per-GPU array)."""
    o = _opts(rtol, maxit, pc, SEM_FP64, 1e-2, check_every, 0)
    st = sem_solve_stats()
    code = lib().sem_pcg_solve_noalloc(h, C.byref(o), _ptr(b), _ptr(x),
                                       C.byref(st), _stream(stream))
    if raise_on_fail and code != SEM_OK:
        _check(code)
    return {"status": code, "iters": st.iters, "outer_iters": st.outer_iters,
            "fell_back": st.fell_back,
            "final_rel_res": st.final_rel_res, "seconds": st.seconds,
            "outer_contraction": st.outer_contraction}


def _opts(rtol, maxit, pc, inner_prec, inner_rtol, check_every, use_graph):
    o = sem_solve_opts()
    o.rtol, o.maxit, o.pc = float(rtol), int(maxit), int(pc)
    o.inner_prec, o.inner_rtol = int(inner_prec), float(inner_rtol)
    o.check_every, o.use_graph = int(check_every), int(use_graph)
    return o


def sem_batch_create(handles):
    arr = (C.c_void_p * len(handles))(*[h.value for h in handles])
    b = C.c_void_p()
    _check(lib().sem_batch_create(arr, len(handles), C.byref(b)))
    return b


def sem_batch_destroy(b):
    _check(lib().sem_batch_destroy(b))


def sem_batch_tune(b, prec):
    bs, gm, us = C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().sem_batch_tune(b, int(prec), C.byref(bs), C.byref(gm),
                                C.byref(us)))
    return bs.value, gm.value, us.value


def sem_batch_pcg_solve(b, bs, xs, rtol=1e-8, maxit=10000, pc=SEM_PC_JACOBI,
                        inner_prec=SEM_FP64, inner_rtol=1e-2, check_every=16,
                        use_graph=1, stream=None, raise_on_fail=True):
    """bs, xs: lists of device FP64 E-vectors (one per solve)."""
    n = len(bs)
    o = _opts(rtol, maxit, pc, inner_prec, inner_rtol, check_every, use_graph)
    barr = (C.c_void_p * n)(*[t.data_ptr() for t in bs])
    xarr = (C.c_void_p * n)(*[t.data_ptr() for t in xs])
    st = (sem_solve_stats * n)()
    code = lib().sem_batch_pcg_solve(b, C.byref(o), barr, xarr, st,
                                     _stream(stream))
    if raise_on_fail and code != SEM_OK:
        _check(code)
    return code, [{"status": st[q].status, "iters": st[q].iters,
                   "fell_back": st[q].fell_back,
                   "outer_iters": st[q].outer_iters,
                   "final_rel_res": st[q].final_rel_res,
                   "seconds": st[q].seconds,
                   "outer_contraction": st[q].outer_contraction}
                  for q in range(n)]


# ----------------------------------------------------------------------------
# learned correction
# ----------------------------------------------------------------------------

def sem_mlp_create(n_in, n_hidden=128, n_out=8, seed=0):
    """n_out: 8 (trilinear vertex values) or (N+1)^3 (nodal values)."""
    net = C.c_void_p()
    _check(lib().sem_mlp_create(int(n_in), int(n_hidden), int(n_out),
                                int(seed), C.byref(net)))
    return net


def sem_mlp_destroy(net):
    _check(lib().sem_mlp_destroy(net))


def sem_mlp_info(net):
    a, b, c, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    e, f = C.c_int64(), C.c_int64()
    _check(lib().sem_mlp_info(net, C.byref(a), C.byref(b), C.byref(c),
                              C.byref(d), C.byref(e), C.byref(f)))
    return {"n_in": a.value, "n_hidden": b.value, "n_out": c.value,
            "n_in_padded": d.value, "n_params": e.value, "adam_steps": f.value}


def sem_mlp_get_params(net):
    import numpy as np
    n = sem_mlp_info(net)["n_params"]
    out = np.zeros(n, dtype=np.float32)
    _check(lib().sem_mlp_get_params(net, out.ctypes.data_as(C.c_void_p), n))
    return out


def sem_mlp_set_params(net, params):
    import numpy as np
    arr = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().sem_mlp_set_params(net, arr.ctypes.data_as(C.c_void_p),
                                    arr.shape[0]))


def sem_mlp_forward(net, X, ldx, B, Y, stream=None):
    _check(lib().sem_mlp_forward(net, _ptr(X), int(ldx), int(B), _ptr(Y),
                                 _stream(stream)))


def sem_mlp_set_precision(net, p):
    _check(lib().sem_mlp_set_precision(net, int(p)))


def sem_mlp_get_precision(net):
    p = C.c_int32()
    _check(lib().sem_mlp_get_precision(net, C.byref(p)))
    return p.value


def sem_mlp_loss_grad_factor(net, X, ldx, T, K, B, grad=None, stream=None):
    loss = C.c_double()
    _check(lib().sem_mlp_loss_grad_factor(net, _ptr(X), int(ldx), _ptr(T), int(K),
                                          int(B), _ptr(grad), C.byref(loss),
                                          _stream(stream)))
    return loss.value


def sem_learn_coarse_exact(h, M, stream=None):
    """M: device FP64 tensor of E*K*K values; returns K."""
    k = C.c_int32()
    _check(lib().sem_learn_coarse_exact(h, _ptr(M), C.byref(k), _stream(stream)))
    return k.value


def sem_mlp_adam(net, grad=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
    _check(lib().sem_mlp_adam(net, _ptr(grad), float(lr), float(beta1),
                              float(beta2), float(eps), _stream(stream)))


def sem_mlp_set_damping(net, damping, jacobi_rate=0.0):
    _check(lib().sem_mlp_set_damping(net, float(damping), float(jacobi_rate)))


def sem_mlp_get_damping(net):
    d, r = C.c_double(), C.c_double()
    _check(lib().sem_mlp_get_damping(net, C.byref(d), C.byref(r)))
    return d.value, r.value


def sem_mlp_save(net, path):
    _check(lib().sem_mlp_save(net, str(path).encode()))


def sem_mlp_load(path):
    net = C.c_void_p()
    _check(lib().sem_mlp_load(str(path).encode(), C.byref(net)))
    return net


def sem_learn_attach(h, net):
    _check(lib().sem_learn_attach(h, net))


def sem_learn_train(h, net, bs, n_pairs=20000, snapshot_every=16,
                    max_snapshots=64, epochs=20, batch=512, lr=1e-3,
                    solve_rtol=1e-12, seed=0, stream=None):
    o = sem_train_opts()
    o.n_pairs, o.snapshot_every, o.max_snapshots = n_pairs, snapshot_every, max_snapshots
    o.epochs, o.batch, o.lr, o.solve_rtol, o.seed = epochs, batch, lr, solve_rtol, seed
    rep = sem_train_report()
    arr = (C.c_void_p * len(bs))(*[t.data_ptr() for t in bs])
    _check(lib().sem_learn_train(h, net, arr, len(bs), C.byref(o), C.byref(rep),
                                 _stream(stream)))
    out = {k: getattr(rep, k) for k, _ in sem_train_report._fields_
           if k not in ("val_iters", "reserved")}
    out["val_iters"] = list(rep.val_iters)
    return out


def sem_learn_attach_exact(h, damping=1.0):
    _check(lib().sem_learn_attach_exact(h, float(damping)))


def sem_last_error():
    return lib().sem_last_error().decode()


# ----------------------------------------------------------------------------
# finite-difference wave step (include/fd2d.h)
# ----------------------------------------------------------------------------

def fd2d_weights(r):
    """Unit-spacing second-derivative weights of order 2r (numpy, 2r+1)."""
    import numpy as np
    w = (C.c_double * (2 * int(r) + 1))()
    _check(lib().fd2d_weights(int(r), w))
    return np.array(list(w))


def _grid_shape(t):
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError("fd2d grids are contiguous 2-D tensors [ny, nx]")
    return int(t.shape[1]), int(t.shape[0])


def fd2d_step(u_cur, u_prev, u_next, r, dt, dx, stream=None):
    """Tensors [ny, nx] float64 on the device; u_next may be u_prev."""
    nx, ny = _grid_shape(u_cur)
    for t in (u_prev, u_next):
        if tuple(t.shape) != tuple(u_cur.shape):
            raise ValueError("fd2d grids must have equal shapes")
    _check(lib().fd2d_step(_ptr(u_cur), _ptr(u_prev), _ptr(u_next), nx, ny,
                           int(r), float(dt), float(dx), _stream(stream)))


def fd2d_run(u_a, u_b, r, dt, dx, nsteps, stream=None):
    """In place on two levels (u_a older, u_b newer); after an odd number of
    steps u_a holds the newest level."""
    nx, ny = _grid_shape(u_a)
    if tuple(u_b.shape) != tuple(u_a.shape):
        raise ValueError("fd2d grids must have equal shapes")
    _check(lib().fd2d_run(_ptr(u_a), _ptr(u_b), nx, ny, int(r), float(dt),
                          float(dx), int(nsteps), _stream(stream)))


# ----------------------------------------------------------------------------
# DG shallow-water volume term (include/dg.h)
# ----------------------------------------------------------------------------

DG_ARR_X, DG_ARR_Y, DG_ARR_GEO, DG_ARR_DB, DG_ARR_DRW, DG_ARR_DSW = range(6)


def dg_reference_nodes(N):
    import numpy as np
    np_ = (N + 1) * (N + 2) // 2
    r, s = (C.c_double * np_)(), (C.c_double * np_)()
    _check(lib().dg_reference_nodes(int(N), r, s))
    return np.array(list(r)), np.array(list(s))


def dg_setup(N, vx, vy, etov, bathymetry=None, g=9.81, stream=None):
    """vx, vy: host vertex coordinates; etov: int [E][3] counterclockwise;
    bathymetry: host [E][Np] nodal B or None.  Returns a handle."""
    import numpy as np
    vx_a, vx_p = _dptr(vx)
    vy_a, vy_p = _dptr(vy)
    ev = np.ascontiguousarray(etov, dtype=np.int32)
    keep = [vx_a, vy_a, ev]
    b_p = None
    if bathymetry is not None:
        b_a, b_p = _dptr(bathymetry)
        np_ = (N + 1) * (N + 2) // 2
        if b_a.size != ev.shape[0] * np_:
            raise ValueError(f"bathymetry needs {ev.shape[0] * np_} nodal values")
        keep.append(b_a)
    h = C.c_void_p()
    _check(lib().dg_setup(int(N), int(vx_a.shape[0]), vx_p, vy_p,
                          int(ev.shape[0]),
                          ev.ctypes.data_as(C.POINTER(C.c_int32)), b_p,
                          float(g), _stream(stream), C.byref(h)))
    return h


def dg_destroy(h):
    _check(lib().dg_destroy(h))


def dg_query(h):
    n, e = C.c_int32(), C.c_int64()
    _check(lib().dg_query(h, C.byref(n), C.byref(e)))
    return n.value, e.value


def dg_export(h, which, dst, stream=None):
    _check(lib().dg_export(h, int(which), _ptr(dst),
                           dst.numel() * dst.element_size(), _stream(stream)))


def dg_volume(h, Q, rhs, stream=None):
    """Q, rhs: device float64 tensors [E][3][Np]."""
    _check(lib().dg_volume(h, _ptr(Q), _ptr(rhs), _stream(stream)))


def dg_volume_blocked(h, Q, rhs, stream=None):
    """Q, rhs: device float64 tensors [ceil(E/16)][3][Np][16] (blocks of 16
    elements, element fastest)."""
    _check(lib().dg_volume_blocked(h, _ptr(Q), _ptr(rhs), _stream(stream)))
