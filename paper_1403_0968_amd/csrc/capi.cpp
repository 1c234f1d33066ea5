// C ABI of libsem.so: argument validation, error codes, handle lifetime.
// No exception crosses this boundary.
#include <cstdio>
#include <cstring>
#include <new>

#include "sem_internal.h"

namespace sem {

static thread_local std::string g_last_error;

void fail(sem_status code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what, const char *file, int line) {
  if (e == hipSuccess) return;
  char buf[512];
  snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e),
           file, line);
  fail(e == hipErrorOutOfMemory ? SEM_ERR_OOM : SEM_ERR_HIP, buf);
}

DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}

void DevBuf::alloc(size_t nbytes) {
  if (p) {
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  if (nbytes == 0) nbytes = 256;
  SEM_HIP(hipMalloc(&p, nbytes));
  bytes = nbytes;
}

template <class F> static sem_status guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return SEM_OK;
  } catch (const Error &e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return SEM_ERR_OOM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return SEM_ERR_STATE;
  }
}

static hipStream_t strm(void *s) { return static_cast<hipStream_t>(s); }

static void need(bool ok, const char *msg) {
  if (!ok) fail(SEM_ERR_ARG, msg);
}

}  // namespace sem

using namespace sem;

extern "C" {

sem_status sem_setup(const sem_mesh_desc *d, void *stream, sem_handle **out) {
  if (out) *out = nullptr;
  sem_handle *h = nullptr;
  sem_status st = guarded([&] {
    need(d != nullptr && out != nullptr, "sem_setup: null argument");
    need(d->N >= 1 && d->N <= 8, "sem_setup: N must be in 1..8");
    need(d->ex >= 1 && d->ey >= 1 && d->ez >= 1, "sem_setup: element counts >= 1");
    need(d->mapping >= SEM_MAP_AFFINE && d->mapping <= SEM_MAP_SINE_CYCLIC,
         "sem_setup: unknown mapping");
    need(d->alpha == 0.0, "sem_setup: alpha must be 0 (mass term not supported)");
    need(d->kappa_nfeat >= 0, "sem_setup: kappa_nfeat must be >= 0");
    need(d->kappa_nfeat == 0 || (d->kappa_omega && d->kappa_b),
         "sem_setup: kappa features need omega and b");
    h = new sem_handle();
    device_setup(h, d, strm(stream));
  });
  if (st != SEM_OK) {
    if (h) {
      destroy_ws(h);
      delete h;
    }
    return st;
  }
  *out = h;
  return SEM_OK;
}

sem_status sem_destroy(sem_handle *h) {
  return guarded([&] {
    if (!h) return;
    (void)hipDeviceSynchronize();
    destroy_ws(h);
    delete h;
  });
}

sem_status sem_query(const sem_handle *h, int64_t *n_elements, int64_t *n_local,
                     int64_t *n_global) {
  return guarded([&] {
    need(h != nullptr, "sem_query: null handle");
    if (n_elements) *n_elements = h->E;
    if (n_local) *n_local = h->nL;
    if (n_global) *n_global = h->nG;
  });
}

sem_status sem_export(const sem_handle *h, int32_t which, void *dst,
                      int64_t dst_bytes, void *stream) {
  return guarded([&] {
    need(h != nullptr && dst != nullptr, "sem_export: null argument");
    const void *src = nullptr;
    int64_t n = 0;
    const int64_t nL = h->nL, nG = h->nG;
    const int64_t ngeo = h->E * 6 * (int64_t)h->n1 * h->n1 * h->n1;
    switch (which) {
      case SEM_ARR_L2G: src = h->l2g.p; n = nL * 4; break;
      case SEM_ARR_PERM: src = h->perm.p; n = nL * 4; break;
      case SEM_ARR_OFFSETS: src = h->offsets.p; n = (nG + 1) * 4; break;
      case SEM_ARR_MULT: src = h->mult.p; n = nL * 4; break;
      case SEM_ARR_MASK: src = h->bmask.p; n = nL; break;
      case SEM_ARR_COORDS: src = h->coords.p; n = 3 * nL * 8; break;
      case SEM_ARR_GEOM: src = h->G64.p; n = ngeo * 8; break;
      case SEM_ARR_MASS: src = h->mass.p; n = nL * 8; break;
      case SEM_ARR_DIAG: src = h->diag_L.p; n = nL * 8; break;
      case SEM_ARR_DINV: src = h->dinv_G.p; n = nG * 8; break;
      default: fail(SEM_ERR_ARG, "sem_export: unknown array");
    }
    need(dst_bytes >= n, "sem_export: destination too small");
    SEM_HIP(hipMemcpyAsync(dst, src, (size_t)n, hipMemcpyDeviceToDevice,
                           strm(stream)));
  });
}

sem_status sem_ax(sem_handle *h, int32_t p, const void *u_L, void *w_L,
                  void *stream) {
  return guarded([&] {
    need(h != nullptr && u_L != nullptr && w_L != nullptr, "sem_ax: null argument");
    need(u_L != w_L, "sem_ax: input and output must not alias");
    const void *G = nullptr, *D = nullptr;
    if (p == SEM_FP64) {
      G = h->G64.p;
      D = h->D64.p;
    } else if (p == SEM_FP32) {
      G = h->G32.p;
      D = h->D32.p;
    } else if (p == SEM_BF16) {
      G = h->G16.p;
      D = h->D32.p;
      need(reinterpret_cast<uintptr_t>(u_L) % 16 == 0,
           "sem_ax: BF16 input must be 16-byte aligned");
    } else {
      fail(SEM_ERR_ARG, "sem_ax: unknown precision");
    }
    launch_ax(h->N, p, h->E, D, G, u_L, w_L, strm(stream));
  });
}

sem_status sem_gs(sem_handle *h, int32_t p, void *v_L, void *stream) {
  return guarded([&] {
    need(h != nullptr && v_L != nullptr, "sem_gs: null argument");
    launch_gs(h, p, v_L, strm(stream));
  });
}

sem_status sem_rhs(sem_handle *h, const sem_source *src, double *b_L,
                   void *stream) {
  return guarded([&] {
    need(h != nullptr && src != nullptr && b_L != nullptr, "sem_rhs: null argument");
    launch_rhs(h, src, b_L, strm(stream));
  });
}

sem_status sem_precond_apply(sem_handle *h, int32_t pc, int32_t p,
                             const void *r_L, void *z_L, void *stream) {
  return guarded([&] {
    need(h != nullptr && r_L != nullptr && z_L != nullptr,
         "sem_precond_apply: null argument");
    launch_precond(h, pc, p, r_L, z_L, strm(stream));
  });
}

sem_status sem_pcg_solve(sem_handle *h, const sem_solve_opts *o,
                         const double *b_L, double *x_L, sem_solve_stats *st,
                         void *stream) {
  sem_status result = SEM_OK;
  sem_status g = guarded([&] {
    need(h != nullptr && o != nullptr && b_L != nullptr && x_L != nullptr,
         "sem_pcg_solve: null argument");
    need((const void *)b_L != (const void *)x_L, "sem_pcg_solve: b and x alias");
    result = pcg_solve(h, o, b_L, x_L, st, strm(stream));
  });
  if (g != SEM_OK) return g;
  if (result != SEM_OK)
    g_last_error = result == SEM_ERR_BREAKDOWN ? "sem_pcg_solve: breakdown"
                                               : "sem_pcg_solve: not converged";
  return result;
}

sem_status sem_batch_create(sem_handle *const *handles, int32_t n,
                            sem_batch **out) {
  if (out) *out = nullptr;
  return guarded([&] {
    need(handles != nullptr && out != nullptr && n >= 1,
         "sem_batch_create: need handles, n >= 1 and an output");
    *out = batch_create(handles, n);
  });
}

sem_status sem_batch_destroy(sem_batch *b) {
  return guarded([&] {
    if (!b) return;
    (void)hipDeviceSynchronize();
    batch_destroy(b);
  });
}

sem_status sem_batch_tune(sem_batch *b, int32_t p, int32_t *block_size,
                          int32_t *grid_mult, double *us) {
  return guarded([&] {
    need(b != nullptr, "sem_batch_tune: null batch");
    int bs = 0, gm = 0;
    double t = 0.0;
    batch_tune(b, p, &bs, &gm, &t);
    if (block_size) *block_size = bs;
    if (grid_mult) *grid_mult = gm;
    if (us) *us = t;
  });
}

sem_status sem_batch_pcg_solve(sem_batch *b, const sem_solve_opts *o,
                               const double *const *b_L, double *const *x_L,
                               sem_solve_stats *stats, void *stream) {
  sem_status result = SEM_OK;
  sem_status g = guarded([&] {
    need(b != nullptr && o != nullptr && b_L != nullptr && x_L != nullptr,
         "sem_batch_pcg_solve: null argument");
    result = batch_solve(b, o, b_L, x_L, stats, strm(stream));
  });
  if (g != SEM_OK) return g;
  if (result != SEM_OK)
    g_last_error = result == SEM_ERR_BREAKDOWN
                       ? "sem_batch_pcg_solve: breakdown in a solve"
                       : "sem_batch_pcg_solve: a solve did not converge";
  return result;
}

const char *sem_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
