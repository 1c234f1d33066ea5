// C ABI of libsem.so: argument validation, error codes, handle lifetime.
// No exception crosses this boundary.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>

#include "../../include/fd2d.h"
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
  if (p && own) (void)hipFree(p);
}

void DevBuf::alloc(size_t nbytes) {
  if (p) {
    if (own) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  own = true;
  if (nbytes == 0) nbytes = 256;
  SEM_HIP(hipMalloc(&p, nbytes));
  bytes = nbytes;
}

void DevBuf::view(void *q, size_t nbytes) {
  if (p && own) (void)hipFree(p);
  p = q;
  bytes = nbytes;
  own = false;
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
    need(std::isfinite(d->alpha) && d->alpha >= 0.0,
         "sem_setup: alpha must be finite and >= 0");
    need(d->kappa_nfeat >= 0, "sem_setup: kappa_nfeat must be >= 0");
    need(d->periodic >= 0 && d->periodic <= 7,
         "sem_setup: periodic takes the bits 1 (x), 2 (y), 4 (z)");
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
    learn_destroy(h);
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
      case SEM_ARR_HMASS:
        if (!h->has_mass) fail(SEM_ERR_STATE, "sem_export: the mesh has no mass term");
        src = h->H64.p;
        n = nL * 8;
        break;
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
    const void *G = nullptr, *D = nullptr, *H = nullptr;
    if (p == SEM_FP64) {
      G = h->G64.p;
      D = h->D64.p;
      H = h->H64.p;
    } else if (p == SEM_FP32) {
      G = h->G32.p;
      D = h->D32.p;
      H = h->H32.p;
    } else if (p == SEM_BF16) {
      G = h->G16.p;
      D = h->D32.p;
      H = h->H16.p;
      need(reinterpret_cast<uintptr_t>(u_L) % 16 == 0,
           "sem_ax: BF16 input must be 16-byte aligned");
    } else if (p == SEM_BF16_MFMA || p == SEM_BF16_PLAIN_D) {
      need(reinterpret_cast<uintptr_t>(u_L) % 16 == 0,
           "sem_ax: BF16 input must be 16-byte aligned");
      launch_ax_mfma(h->N, p == SEM_BF16_MFMA, h->E, h->D16hi.as<uint16_t>(),
                     h->D16lo.as<uint16_t>(), h->G16.as<uint16_t>(),
                     h->H16.as<uint16_t>(), (const uint16_t *)u_L, (float *)w_L,
                     strm(stream));
      return;
    } else {
      fail(SEM_ERR_ARG, "sem_ax: unknown precision");
    }
    launch_ax(h->N, p, h->E, D, G, h->has_mass ? H : nullptr, u_L, w_L,
              strm(stream));
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

sem_status sem_pcg_solve_noalloc(sem_handle *h, const sem_solve_opts *o,
                                 const double *b_L, double *x_L,
                                 sem_solve_stats *st, void *stream) {
  sem_status result = SEM_OK;
  sem_status g = guarded([&] {
    need(h != nullptr && o != nullptr && b_L != nullptr && x_L != nullptr,
         "sem_pcg_solve_noalloc: null argument");
    need((const void *)b_L != (const void *)x_L,
         "sem_pcg_solve_noalloc: b and x alias");
    result = pcg_solve_noalloc(h, o, b_L, x_L, st, strm(stream));
  });
  if (g != SEM_OK) return g;
  if (result != SEM_OK)
    g_last_error = result == SEM_ERR_BREAKDOWN ? "sem_pcg_solve_noalloc: breakdown"
                                               : "sem_pcg_solve_noalloc: not converged";
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

sem_status sem_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out,
                          uint64_t seed, sem_mlp **out) {
  if (out) *out = nullptr;
  return guarded([&] {
    need(out != nullptr, "sem_mlp_create: null output");
    *out = mlp_create(n_in, n_hidden, n_out, seed);
  });
}

sem_status sem_mlp_destroy(sem_mlp *net) {
  return guarded([&] {
    if (!net) return;
    (void)hipDeviceSynchronize();
    mlp_destroy(net);
  });
}

sem_status sem_mlp_info(const sem_mlp *net, int32_t *n_in, int32_t *n_hidden,
                        int32_t *n_out, int32_t *n_in_padded, int64_t *n_params,
                        int64_t *adam_steps) {
  return guarded([&] {
    need(net != nullptr, "sem_mlp_info: null network");
    int a = 0, b = 0, c = 0;
    int64_t np = 0, st = 0;
    mlp_info(net, &a, &b, &c, &np, &st);
    if (n_in) *n_in = a;
    if (n_hidden) *n_hidden = b;
    if (n_out) *n_out = c;
    if (n_in_padded) *n_in_padded = mlp_padded_inputs(net);
    if (n_params) *n_params = np;
    if (adam_steps) *adam_steps = st;
  });
}

sem_status sem_mlp_get_params(const sem_mlp *net, float *params, int64_t n) {
  return guarded([&] {
    need(net != nullptr && params != nullptr, "sem_mlp_get_params: null argument");
    mlp_get_params(net, params, n);
  });
}

sem_status sem_mlp_set_params(sem_mlp *net, const float *params, int64_t n) {
  return guarded([&] {
    need(net != nullptr && params != nullptr, "sem_mlp_set_params: null argument");
    mlp_set_params(net, params, n);
  });
}

sem_status sem_mlp_forward(sem_mlp *net, const uint16_t *X, int32_t ldx,
                           int32_t B, float *Y, void *stream) {
  return guarded([&] {
    need(net != nullptr && X != nullptr && Y != nullptr && B >= 0,
         "sem_mlp_forward: null argument or negative batch");
    int n_out = 0;
    mlp_info(net, nullptr, nullptr, &n_out, nullptr, nullptr);
    mlp_forward(net, X, ldx, B, Y, n_out, strm(stream));
  });
}

sem_status sem_mlp_set_precision(sem_mlp *net, int32_t p) {
  return guarded([&] {
    need(net != nullptr, "sem_mlp_set_precision: null network");
    need(p == SEM_BF16 || p == SEM_FP32,
         "sem_mlp_set_precision: SEM_BF16 or SEM_FP32");
    mlp_set_precision(net, p);
  });
}

sem_status sem_mlp_get_precision(const sem_mlp *net, int32_t *p) {
  return guarded([&] {
    need(net != nullptr && p != nullptr, "sem_mlp_get_precision: null argument");
    *p = mlp_precision(net);
  });
}

sem_status sem_mlp_loss_grad_factor(sem_mlp *net, const uint16_t *X,
                                    int32_t ldx, const float *T, int32_t K,
                                    int32_t B, float *grad, double *loss,
                                    void *stream) {
  return guarded([&] {
    need(net != nullptr && X != nullptr && T != nullptr && B >= 1,
         "sem_mlp_loss_grad_factor: null argument or empty batch");
    const double l = mlp_loss_grad_factor(net, X, ldx, T, K, B, true, strm(stream));
    if (loss) *loss = l;
    if (grad) {
      int64_t np = 0;
      mlp_info(net, nullptr, nullptr, nullptr, &np, nullptr);
      SEM_HIP(hipMemcpyAsync(grad, mlp_grad_ptr(net), np * 4,
                             hipMemcpyDeviceToDevice, strm(stream)));
    }
  });
}

sem_status sem_mlp_adam(sem_mlp *net, const float *grad, double lr,
                        double beta1, double beta2, double eps, void *stream) {
  return guarded([&] {
    need(net != nullptr, "sem_mlp_adam: null network");
    need(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0,
         "sem_mlp_adam: invalid hyper-parameters");
    mlp_adam(net, grad, lr, beta1, beta2, eps, strm(stream));
  });
}

sem_status sem_mlp_set_damping(sem_mlp *net, double damping, double jacobi_rate) {
  return guarded([&] {
    need(net != nullptr, "sem_mlp_set_damping: null network");
    need(std::isfinite(damping) && damping >= 0 && std::isfinite(jacobi_rate) &&
             jacobi_rate <= 0,
         "sem_mlp_set_damping: damping >= 0 and jacobi_rate <= 0 required");
    mlp_set_damping(net, damping, jacobi_rate);
  });
}

sem_status sem_mlp_get_damping(const sem_mlp *net, double *damping,
                               double *jacobi_rate) {
  return guarded([&] {
    need(net != nullptr, "sem_mlp_get_damping: null network");
    if (damping) *damping = mlp_damping(net);
    if (jacobi_rate) *jacobi_rate = mlp_ref_rate(net);
  });
}

sem_status sem_mlp_save(const sem_mlp *net, const char *path) {
  return guarded([&] {
    need(net != nullptr && path != nullptr, "sem_mlp_save: null argument");
    mlp_save(net, path);
  });
}

sem_status sem_mlp_load(const char *path, sem_mlp **out) {
  if (out) *out = nullptr;
  return guarded([&] {
    need(path != nullptr && out != nullptr, "sem_mlp_load: null argument");
    *out = mlp_load(path);
  });
}

sem_status sem_learn_attach(sem_handle *h, sem_mlp *net) {
  return guarded([&] {
    need(h != nullptr, "sem_learn_attach: null handle");
    learn_attach(h, net);
  });
}

sem_status sem_learn_train(sem_handle *h, sem_mlp *net, const double *const *b_L,
                           int32_t n_rhs, const sem_train_opts *opts,
                           sem_train_report *report, void *stream) {
  return guarded([&] {
    need(h != nullptr && net != nullptr && b_L != nullptr && opts != nullptr,
         "sem_learn_train: null argument");
    learn_train(h, net, b_L, n_rhs, opts, report, strm(stream));
  });
}

sem_status sem_learn_attach_exact(sem_handle *h, double damping) {
  return guarded([&] {
    need(h != nullptr, "sem_learn_attach_exact: null handle");
    need(std::isfinite(damping) && damping >= 0.0,
         "sem_learn_attach_exact: damping must be finite and >= 0");
    learn_attach_exact(h, damping);
  });
}

sem_status sem_learn_coarse_exact(sem_handle *h, double *M, int32_t *K,
                                  void *stream) {
  return guarded([&] {
    need(h != nullptr && M != nullptr, "sem_learn_coarse_exact: null argument");
    const int k = learn_coarse_exact(h, M, strm(stream));
    if (K) *K = k;
  });
}

sem_status fd2d_weights(int32_t r, double *w) {
  return guarded([&] {
    need(w != nullptr, "fd2d_weights: null output");
    fd2d_weights_host(r, w);
  });
}

static double fd2d_coefficient(double dt, double dx) {
  need(std::isfinite(dt) && std::isfinite(dx) && dx > 0.0,
       "fd2d: dt must be finite and dx finite and > 0");
  return (dt * dt) / (dx * dx);
}

sem_status fd2d_step(const double *u_cur, const double *u_prev, double *u_next,
                     int64_t nx, int64_t ny, int32_t r, double dt, double dx,
                     void *stream) {
  return guarded([&] {
    launch_fd2d(u_cur, u_prev, u_next, nx, ny, r, fd2d_coefficient(dt, dx),
                strm(stream));
  });
}

sem_status fd2d_run(double *u_a, double *u_b, int64_t nx, int64_t ny, int32_t r,
                    double dt, double dx, int32_t nsteps, void *stream) {
  return guarded([&] {
    need(nsteps >= 0, "fd2d_run: nsteps must be >= 0");
    need(u_a != u_b, "fd2d_run: the two levels must be distinct buffers");
    const double c = fd2d_coefficient(dt, dx);
    double *older = u_a, *newer = u_b;
    for (int32_t s = 0; s < nsteps; ++s) {
      launch_fd2d(newer, older, older, nx, ny, r, c, strm(stream));
      std::swap(older, newer);
    }
  });
}

sem_status dg_reference_nodes(int32_t N, double *r, double *s) {
  return guarded([&] {
    need(r != nullptr && s != nullptr, "dg_reference_nodes: null output");
    const DgRef R = make_dg_ref(N);
    for (int n = 0; n < R.Np; ++n) {
      r[n] = R.r[n];
      s[n] = R.s[n];
    }
  });
}

sem_status dg_setup(int32_t N, int64_t n_vertices, const double *vx,
                    const double *vy, int64_t n_elements, const int32_t *etov,
                    const double *bathymetry, double g, void *stream,
                    dg_handle **out) {
  if (out) *out = nullptr;
  dg_handle *h = nullptr;
  sem_status st = guarded([&] {
    need(out != nullptr && vx != nullptr && vy != nullptr, "dg_setup: null argument");
    need(n_vertices >= 3 && n_elements >= 0 && (n_elements == 0 || etov != nullptr),
         "dg_setup: need vertices and element connectivity");
    need(N >= 1 && N <= 8, "dg_setup: N must be in 1..8");
    need(std::isfinite(g), "dg_setup: g must be finite");
    need(n_elements < (int64_t)1 << 31, "dg_setup: too many elements");
    h = new dg_handle();
    h->N = N;
    h->E = n_elements;
    h->g = g;
    dg_device_setup(h, n_vertices, vx, vy, etov, bathymetry, strm(stream));
  });
  if (st != SEM_OK) {
    delete h;
    return st;
  }
  *out = h;
  return SEM_OK;
}

sem_status dg_destroy(dg_handle *h) {
  return guarded([&] {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
  });
}

sem_status dg_query(const dg_handle *h, int32_t *n_nodes, int64_t *n_elements) {
  return guarded([&] {
    need(h != nullptr, "dg_query: null handle");
    if (n_nodes) *n_nodes = h->Np;
    if (n_elements) *n_elements = h->E;
  });
}

sem_status dg_export(const dg_handle *h, int32_t which, void *dst,
                     int64_t dst_bytes, void *stream) {
  return guarded([&] {
    need(h != nullptr && dst != nullptr, "dg_export: null argument");
    const int64_t E = h->E, Np = h->Np;
    const void *src = nullptr;
    bool host = false;
    int64_t n = 0;
    switch (which) {
      case DG_ARR_X: src = h->X.p; n = E * Np * 8; break;
      case DG_ARR_Y: src = h->Y.p; n = E * Np * 8; break;
      case DG_ARR_GEO: src = h->geo.p; n = E * 4 * 8; break;
      case DG_ARR_DB: src = h->dB.p; n = E * 2 * Np * 8; break;
      case DG_ARR_DRW: src = h->ref.Drw.data(); n = Np * Np * 8; host = true; break;
      case DG_ARR_DSW: src = h->ref.Dsw.data(); n = Np * Np * 8; host = true; break;
      default: fail(SEM_ERR_ARG, "dg_export: unknown array");
    }
    need(dst_bytes >= n, "dg_export: destination too small");
    if (n == 0) return;
    SEM_HIP(hipMemcpyAsync(dst, src, (size_t)n,
                           host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           strm(stream)));
    if (host) SEM_HIP(hipStreamSynchronize(strm(stream)));
  });
}

sem_status dg_volume(dg_handle *h, const double *Q, double *rhs, void *stream) {
  return guarded([&] {
    need(h != nullptr && Q != nullptr && rhs != nullptr, "dg_volume: null argument");
    const size_t bytes = (size_t)h->E * 3 * h->Np * sizeof(double);
    const char *q0 = (const char *)Q, *r0 = (const char *)rhs;
    need(r0 + bytes <= q0 || q0 + bytes <= r0, "dg_volume: rhs must not overlap Q");
    launch_dg_volume(h, Q, rhs, false, strm(stream));
  });
}

sem_status dg_volume_blocked(dg_handle *h, const double *Q, double *rhs,
                             void *stream) {
  return guarded([&] {
    need(h != nullptr && Q != nullptr && rhs != nullptr,
         "dg_volume_blocked: null argument");
    const size_t bytes = (size_t)((h->E + 15) / 16) * 16 * 3 * h->Np * sizeof(double);
    const char *q0 = (const char *)Q, *r0 = (const char *)rhs;
    need(r0 + bytes <= q0 || q0 + bytes <= r0,
         "dg_volume_blocked: rhs must not overlap Q");
    launch_dg_volume(h, Q, rhs, true, strm(stream));
  });
}

const char *sem_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
