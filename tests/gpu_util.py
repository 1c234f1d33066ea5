"""Helpers for the GPU tests: device tensors, exports, oracle meshes."""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc


def torch():
    import torch as t
    return t


def dev():
    return torch().device("cuda:0")


def to_dev(a, dtype=None):
    t = torch()
    dtype = dtype or t.float64
    return t.as_tensor(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def to_host(x):
    return x.detach().to("cpu").numpy()


def export(sem, h, which, n, dtype):
    t = torch()
    buf = t.empty(n, dtype=dtype, device=dev())
    sem.sem_export(h, which, buf)
    t.cuda.synchronize()
    return to_host(buf)


def bf16_round(a):
    """Round FP64 values to bfloat16 (via float32, round to nearest even)
    and return them as float64; bit patterns as uint16 in the second value."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    u16 = u.astype(np.uint16)
    back = (u16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return back, u16


class Pair:
    """A library handle and the oracle mesh for the same discretisation."""

    def __init__(self, sem, N, ex, ey, ez, mapping=0, dirichlet=1, kappa=None,
                 oracle=True, alpha=0.0, alpha_nodal=None, periodic=0):
        self.sem = sem
        self.N, self.ex, self.ey, self.ez = N, ex, ey, ez
        self.h = sem.sem_setup(N, ex, ey, ez, mapping=mapping,
                               dirichlet=dirichlet, kappa=kappa, alpha=alpha,
                               alpha_nodal=alpha_nodal, periodic=periodic)
        self.E, self.nL, self.nG = sem.sem_query(self.h)
        self.m = (orc.mesh(N, ex, ey, ez, mapping, dirichlet, kappa,
                           alpha=alpha, alpha_nodal=alpha_nodal, periodic=periodic)
                  if oracle else None)

    def close(self):
        if self.h is not None:
            self.sem.sem_destroy(self.h)
            self.h = None
