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
SEM_FP64, SEM_FP32, SEM_BF16 = 0, 1, 2
SEM_PC_NONE, SEM_PC_JACOBI = 0, 1
SEM_MAP_AFFINE, SEM_MAP_SINE_X, SEM_MAP_SINE_CYCLIC = 0, 1, 2
SEM_SRC_FOURIER, SEM_SRC_SINE = 0, 1
(SEM_ARR_L2G, SEM_ARR_PERM, SEM_ARR_OFFSETS, SEM_ARR_MULT, SEM_ARR_MASK,
 SEM_ARR_COORDS, SEM_ARR_GEOM, SEM_ARR_MASS, SEM_ARR_DIAG,
 SEM_ARR_DINV) = range(10)

EXPORTED = ["sem_setup", "sem_destroy", "sem_query", "sem_export", "sem_ax",
            "sem_gs", "sem_rhs", "sem_precond_apply", "sem_pcg_solve",
            "sem_batch_create", "sem_batch_destroy", "sem_batch_tune",
            "sem_batch_pcg_solve", "sem_last_error"]


class sem_mesh_desc(C.Structure):
    _fields_ = [("N", C.c_int32), ("ex", C.c_int32), ("ey", C.c_int32),
                ("ez", C.c_int32), ("dirichlet", C.c_int32),
                ("mapping", C.c_int32), ("alpha", C.c_double),
                ("kappa_nfeat", C.c_int32),
                ("kappa_omega", C.POINTER(C.c_double)),
                ("kappa_b", C.POINTER(C.c_double)),
                ("kappa_sigma", C.c_double)]


class sem_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nmodes", C.c_int32),
                ("k", C.POINTER(C.c_double)), ("a", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double))]


class sem_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("pc", C.c_int32),
                ("inner_prec", C.c_int32), ("inner_rtol", C.c_double),
                ("check_every", C.c_int32), ("use_graph", C.c_int32)]


class sem_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32),
                ("status", C.c_int32), ("reserved", C.c_int32),
                ("final_rel_res", C.c_double), ("seconds", C.c_double)]


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
    L.sem_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp)]
    L.sem_batch_destroy.argtypes = [vp]
    L.sem_batch_tune.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32),
                                 C.POINTER(C.c_double)]
    L.sem_batch_pcg_solve.argtypes = [vp, C.POINTER(sem_solve_opts),
                                      C.POINTER(vp), C.POINTER(vp),
                                      C.POINTER(sem_solve_stats), vp]
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
              kappa=None, stream=None):
    """kappa: None or (omega[M,3], b[M], sigma).  Returns an opaque handle."""
    d = sem_mesh_desc()
    d.N, d.ex, d.ey, d.ez = N, ex, ey, ez
    d.dirichlet, d.mapping, d.alpha = int(dirichlet), int(mapping), 0.0
    keep = []
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
            "final_rel_res": st.final_rel_res, "seconds": st.seconds}


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
                   "outer_iters": st[q].outer_iters,
                   "final_rel_res": st[q].final_rel_res,
                   "seconds": st[q].seconds} for q in range(n)]


def sem_last_error():
    return lib().sem_last_error().decode()
