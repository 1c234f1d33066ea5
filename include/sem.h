/*
 * sem.h -- C ABI of libsem.so, an MI355X (gfx950) implementation of the
 * spectral-element Poisson operator and its preconditioned CG solve from
 * Medina, St-Cyr & Warburton, "OCCA: A unified approach to multi-threading
 * languages" (arXiv 1403.0968), section 4.2.
 *
 * Problem (section 4.2, equation semPDE):  -div(kappa grad u) + alpha u = f
 * on the image of the unit cube, discretised (section 4.2.1, equation
 * semOperator) with continuous piecewise tensor-product polynomials of degree
 * N on hexahedra, Lagrange basis on the (N+1) Gauss-Lobatto-Legendre points
 * per direction, GLL quadrature, and homogeneous Dirichlet conditions imposed
 * by masking.  The mass term of equation semOperator is lumped by the GLL
 * quadrature (section 4.2.1, discrete orthogonality): it adds
 * H_l u_l with H_l = alpha(X_l) B_l, B_l = w_i w_j w_k J at local node l, to
 * the local operator.  alpha(X) >= 0; with alpha > 0 the assembled operator
 * is symmetric positive definite also without Dirichlet faces.
 *
 * Conventions shared by every call:
 *   - n1 = N+1; element e = ex + Ex*(ey + Ey*ez); element-local node
 *     (i,j,k), i fastest; local ("E-vector") index
 *     l = e*n1^3 + i + n1*j + n1^2*k; n_local = E*n1^3.
 *   - global (unique) node g = gx + Gx*(gy + Gy*gz), gx = ex*N+i (y, z
 *     alike), Gd = Ed*N+1, or Gd = Ed*N with gd taken modulo Gd in a
 *     periodic direction; n_global = Gx*Gy*Gz.
 *   - Vectors passed to the calls are DEVICE pointers owned by the caller,
 *     contiguous, 256-byte aligned is recommended, in E-vector layout.
 *     Their element type is set by the sem_precision argument:
 *     SEM_FP64 -> double, SEM_FP32 -> float, SEM_BF16 -> bfloat16 stored as
 *     uint16_t (round-to-nearest-even of the float), outputs in float.
 *   - `stream` is a hipStream_t (cast to void*); NULL means the null
 *     (default) stream.  Every call is asynchronous on that stream unless
 *     stated otherwise.
 *   - Every function returns a sem_status; nothing aborts or throws across
 *     the ABI.  sem_last_error() returns the text of the last failure of the
 *     calling thread.
 *   - One handle must not be used by two host threads at once.
 */
#ifndef SEM_H
#define SEM_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SEM_OK = 0,
  SEM_ERR_ARG = 1,            /* invalid argument (null, size, range) */
  SEM_ERR_HIP = 2,            /* a HIP runtime call failed */
  SEM_ERR_OOM = 3,            /* device allocation failed */
  SEM_ERR_NOT_CONVERGED = 4,  /* solver hit maxit */
  SEM_ERR_BREAKDOWN = 5,      /* p^T A p <= 0, NaN or Inf in the solver */
  SEM_ERR_STATE = 6           /* call not valid for this handle */
} sem_status;

/* Operator precisions.  The input is used at the precision it is given in:
 * sem_ax takes it in the storage type listed under sem_ax; inside the
 * refinement's inner solves it is the FP32 search direction p.
 *   SEM_BF16: BF16 geometric factors, FP32 derivative matrix, arithmetic
 *     and output, VALU.  sem_ax: BF16 u (18 B per local node: u 2, G 12,
 *     w 4).  Solver: FP32 p, not rounded (G 12 + w 4 per local node, p 4
 *     per unique node).
 *   SEM_BF16_MFMA: the six contractions on the matrix cores with FP32
 *     accumulation, BF16 G and fluxes, the derivative matrix as a two-term
 *     BF16 split D = D_hi + D_lo (two accumulating MFMAs per contraction).
 *     sem_ax: BF16 u.  Solver: FP32 p as a two-term BF16 split
 *     p = p_hi + p_lo, each gradient contraction accumulating D_hi p_hi,
 *     D_lo p_hi and D_hi p_lo (rounding p to BF16 alone leaves an input
 *     error whose effect on refinement grows with the mesh).
 *   SEM_BF16_PLAIN_D: as SEM_BF16_MFMA with D rounded to BF16 (D_lo
 *     dropped): its error does not vanish on smooth inputs, so refinement
 *     around it contracts poorly or diverges (kept to measure exactly that). */
typedef enum {
  SEM_FP64 = 0,
  SEM_FP32 = 1,
  SEM_BF16 = 2,
  SEM_BF16_PLAIN_D = 3,
  SEM_BF16_MFMA = 4
} sem_precision;
typedef enum {
  SEM_PC_NONE = 0,     /* z = r (off the Dirichlet boundary) */
  SEM_PC_JACOBI = 1,   /* z = dinv o r */
  SEM_PC_LEARNED = 2   /* z = dinv o r + learned coarse correction c(r), inside
                          flexible CG; needs a network attached with
                          sem_learn_attach; Jacobi-PCG is the fallback */
} sem_precond;
typedef enum {
  SEM_MAP_AFFINE = 0,      /* the unit cube itself */
  SEM_MAP_SINE_X = 1,      /* X = (x + 0.05 s(y)s(z), y, z), s(t) = sin(2 pi t) */
  SEM_MAP_SINE_CYCLIC = 2  /* X = x + 0.05 (s(y)s(z), s(z)s(x), s(x)s(y)) */
} sem_mapping;

typedef struct sem_handle sem_handle; /* opaque, owned by the library */
typedef struct sem_batch sem_batch;   /* opaque batch of independent solves */
typedef struct sem_mlp sem_mlp;       /* opaque learned-correction network */

/* Mesh and coefficients.  All pointers here are HOST pointers, read during
 * sem_setup only. */
typedef struct {
  int32_t N;            /* polynomial order, 1..8 */
  int32_t ex, ey, ez;   /* elements per direction, >= 1 */
  int32_t dirichlet;    /* 1: homogeneous Dirichlet on the 6 outer faces;
                           0: pure Neumann (operator checks only) */
  int32_t mapping;      /* a sem_mapping */
  double alpha;         /* mass coefficient alpha(X) of semPDE when
                           alpha_nodal is NULL: finite, >= 0; 0 leaves the
                           mass term out (no extra bytes per node) */
  /* kappa(X) = exp(sigma sqrt(2/M) sum_m cos(omega_m . X + b_m)) when
   * kappa_nfeat = M > 0 (random Fourier features of a Gaussian field),
   * kappa = 1 when kappa_nfeat == 0. */
  int32_t kappa_nfeat;
  const double *kappa_omega; /* [M][3] */
  const double *kappa_b;     /* [M] */
  double kappa_sigma;
  /* alpha(X) at every local node, n_local values in E-vector order (equal
   * on the copies of a global node), finite and >= 0; NULL: the constant
   * alpha above.  Read during sem_setup only. */
  const double *alpha_nodal;
  /* Periodic directions, bit 1 x, 2 y, 4 z (0: none): the faces at 0 and 1
   * of that direction are identified (the distinct global-local numbering
   * of section 4.2.1 then has E_d N node coordinates in it; the Dirichlet
   * mask covers only the faces of non-periodic directions).  Each element
   * keeps its own node positions, so the copies of a node on the identified
   * faces sit at 0 and at 1: the mapping, kappa and the right-hand side
   * should be periodic (the sine mappings are).  With every direction
   * periodic (or dirichlet = 0) the operator is positive definite only
   * with alpha > 0 (section 4.2, equation semPDE). */
  int32_t periodic;
} sem_mesh_desc;

/* Right-hand side f(X) for sem_rhs.  HOST pointers. */
typedef enum {
  SEM_SRC_FOURIER = 0, /* f = sum_m a_m cos(2 pi k_m . X + phi_m) */
  SEM_SRC_SINE = 1     /* f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) */
} sem_source_kind;
typedef struct {
  int32_t kind;
  int32_t nmodes;      /* SEM_SRC_FOURIER: number of modes (<= 64) */
  const double *k;     /* [nmodes][3] wave vectors */
  const double *a;     /* [nmodes] amplitudes */
  const double *phi;   /* [nmodes] phases */
} sem_source;

typedef struct {
  double rtol;          /* stop when ||b - A x||_2 <= rtol ||b||_2, norms over
                           unique nodes (Dirichlet entries are zero) */
  int32_t maxit;        /* CG iterations (inner iterations summed for IR) */
  int32_t pc;           /* a sem_precond */
  int32_t inner_prec;   /* SEM_FP64: plain FP64 PCG.  Any other precision:
                           FP64 iterative refinement whose inner PCG uses
                           FP32 vectors and that operator applied to the
                           FP32 search direction (SEM_FP32, SEM_BF16,
                           SEM_BF16_MFMA, SEM_BF16_PLAIN_D as described at
                           sem_precision; the matrix-core ones for solves of
                           one order), with FP64 dot products and
                           scalars; refinement stops after 3 steps that do
                           not shrink the true residual by 10% */
  double inner_rtol;    /* inner relative tolerance for refinement */
  int32_t check_every;  /* CG iterations between host convergence polls */
  int32_t use_graph;    /* 1: replay a captured HIP graph of check_every
                           iterations; 0: launch kernels directly */
} sem_solve_opts;

typedef struct {
  int32_t iters;              /* CG iterations (all inner ones for IR) */
  int32_t outer_iters;        /* refinement steps (0 for plain PCG) */
  int32_t status;             /* sem_status of the solve */
  int32_t fell_back;          /* 1 when a learned solve switched to Jacobi */
  double final_rel_res;       /* recomputed FP64 ||b - A x|| / ||b|| */
  double seconds;             /* wall time of the solve on the stream */
  double outer_contraction;   /* largest ratio ||r_k+1|| / ||r_k|| of the FP64
                                 true residual over refinement steps (0 for
                                 plain PCG) */
} sem_solve_stats;

/* Build a handle: reference element (GLL nodes, weights, derivative matrix),
 * global-local maps (section 4.2.1, distinct global-local numbering),
 * coordinates and the six geometric factors per node (G_ab =
 * w_i w_j w_k J kappa grad r_a . grad r_b, the G^T G metric of section 4.2.1
 * precomputed per elemental node, FP64 with FP32/BF16 copies), the lumped
 * mass B = w_i w_j w_k J, the mass factor H = alpha(X) B when alpha != 0
 * and the Jacobi diagonal (stiffness plus H).  Synchronises `stream`
 * before returning.  On failure *out is NULL. */
sem_status sem_setup(const sem_mesh_desc *desc, void *stream, sem_handle **out);
/* Release a handle and every device buffer it owns (the set-up / allocate /
 * build / call / release host pattern of section 4.1.2's driver).  Batches
 * and networks that reference the handle must be destroyed or detached
 * first.  NULL is accepted. */
sem_status sem_destroy(sem_handle *h);

/* Sizes of the discretisation of section 4.2.1: elements E, local nodes
 * E (N+1)^3 (the E-vector length) and unique global nodes of the distinct
 * global-local numbering.  Outputs are HOST pointers, any may be NULL. */
sem_status sem_query(const sem_handle *h, int64_t *n_elements,
                     int64_t *n_local, int64_t *n_global);

/* Copy an internal array into caller device memory `dst` of `dst_bytes`
 * bytes (SEM_ERR_ARG when too small): the maps of the distinct global-local
 * numbering and the per-node factors of section 4.2.1, for checking.
 * Asynchronous on `stream`.  Layouts:
 *   SEM_ARR_L2G     int32 [n_local]   global id of each local node
 *   SEM_ARR_PERM    int32 [n_local]   local ids sorted by (global id, local id)
 *   SEM_ARR_OFFSETS int32 [n_global+1] start of each global id in PERM
 *   SEM_ARR_MULT    int32 [n_local]   number of copies of the node
 *   SEM_ARR_MASK    uint8 [n_local]   1 on Dirichlet nodes
 *   SEM_ARR_COORDS  double [3][n_local] physical x, y, z blocks
 *   SEM_ARR_GEOM    double [E][6][n1^3] (rr, rs, rt, ss, st, tt)
 *   SEM_ARR_MASS    double [n_local]   lumped mass B (unassembled)
 *   SEM_ARR_DIAG    double [n_local]   unassembled local-matrix diagonal
 *   SEM_ARR_DINV    double [n_global]  inverse assembled diagonal, 0 on
 *                                      Dirichlet nodes
 *   SEM_ARR_HMASS   double [n_local]   mass factor H = alpha(X) B
 *                                      (SEM_ERR_STATE when alpha = 0) */
typedef enum {
  SEM_ARR_L2G = 0, SEM_ARR_PERM = 1, SEM_ARR_OFFSETS = 2, SEM_ARR_MULT = 3,
  SEM_ARR_MASK = 4, SEM_ARR_COORDS = 5, SEM_ARR_GEOM = 6, SEM_ARR_MASS = 7,
  SEM_ARR_DIAG = 8, SEM_ARR_DINV = 9, SEM_ARR_HMASS = 10
} sem_array;
sem_status sem_export(const sem_handle *h, int32_t which, void *dst,
                      int64_t dst_bytes, void *stream);

/* Local stiffness action w_L = A_L u_L, element by element, unassembled and
 * unmasked: the factored operator of section 4.2.1 (last display),
 *   u_r = (I x I x D) u, u_s = (I x D x I) u, u_t = (D x I x I) u,
 *   [w_r w_s w_t] = G [u_r u_s u_t],  w = D_r^T w_r + D_s^T w_s + D_t^T w_t,
 * the kernel section 4.2.2 names as the dominant cost of PCG.
 * p = SEM_FP64: u, w double.  SEM_FP32: u, w float (FP32 G).
 * SEM_BF16: u bf16 (16-byte aligned), w float (BF16 G, FP32 derivative
 * matrix and FP32 accumulation, VALU).  SEM_BF16_MFMA: u bf16 (16-byte
 * aligned), w float; the six contractions on the matrix cores with the
 * split derivative matrix (N <= 7 in blocks of 8, N = 8 on 16-padded
 * operands).  SEM_BF16_PLAIN_D: the same with D
 * rounded to BF16.  When the mesh has a mass term (alpha != 0) every
 * precision adds H o u_L (H = alpha(X) B, stored in the precision of G; the
 * lumped mass operator of equation semOperator), 8 / 4 / 2 more bytes per
 * node.  u_L and w_L must not overlap. */
sem_status sem_ax(sem_handle *h, int32_t p, const void *u_L, void *w_L,
                  void *stream);

/* Direct stiffness summation in place: v <- mask o Q Q^T v (section 4.2.1:
 * the assembled operator follows from the element operators through the
 * distinct global-local node numbering the paper takes from Fischer 1991).
 * Every copy of a global node receives the sum of all copies taken in
 * ascending local index starting from +0.0 (no fused multiply-add; a node
 * with one copy receives +0.0 + v), then Dirichlet copies are set to zero.
 * Atomic-free: a precomputed list sorted by (global id, local id) gives each
 * shared node's copies.  p = SEM_FP64 (double) or SEM_FP32 (float); v_L is
 * a caller-owned device E-vector of n_local values, updated in place.
 * SEM_ERR_ARG for another precision or a null vector. */
sem_status sem_gs(sem_handle *h, int32_t p, void *v_L, void *stream);

/* Load vector b_L = mask o Q Q^T (B o f(X)): the weak-form right-hand side
 * <f, v> of equation semOperator (section 4.2.1) with the lumped GLL mass
 * B = w_i w_j w_k J, evaluated at the physical node positions.  b_L is a
 * caller-owned device FP64 E-vector of n_local values; src and its arrays
 * are HOST pointers.  SEM_ERR_ARG for an unknown source kind or more than
 * 64 Fourier modes. */
sem_status sem_rhs(sem_handle *h, const sem_source *src, double *b_L,
                   void *stream);

/* z_L = P r_L on continuous E-vectors: the preconditioner of the PCG solve
 * (section 4.2.2 solves the system by preconditioned conjugate gradients and
 * leaves the choice of preconditioner open; these are this library's).
 * SEM_PC_JACOBI: z = dinv o r with the inverse of the assembled diagonal (0
 * on Dirichlet nodes); SEM_PC_NONE: z = mask o r; SEM_PC_LEARNED (FP64 only,
 * network attached): z = dinv o r + the learned coarse correction of r.
 * p = SEM_FP64 (double) or SEM_FP32 (float); r_L, z_L caller-owned device
 * E-vectors of n_local values that must not overlap.  SEM_ERR_ARG for another
 * precision, SEM_ERR_STATE for SEM_PC_LEARNED without a network. */
sem_status sem_precond_apply(sem_handle *h, int32_t pc, int32_t p,
                             const void *r_L, void *z_L, void *stream);

/* Solve A x = b (section 4.2.2: preconditioned conjugate gradients) for a
 * continuous, masked FP64 E-vector b_L (e.g. from sem_rhs).  x_L holds the
 * initial guess on entry (continuous E-vector; use zeros) and the solution
 * on return.  Synchronises `stream`.  Returns SEM_ERR_NOT_CONVERGED /
 * SEM_ERR_BREAKDOWN with the stats filled in when the solve fails. */
sem_status sem_pcg_solve(sem_handle *h, const sem_solve_opts *opts,
                         const double *b_L, double *x_L,
                         sem_solve_stats *stats, void *stream);

/* For callers that cannot allocate memory (tight serving loops, harnesses
 * that forbid hipMalloc): sem_pcg_solve without any device or pinned host
 * allocation.  Plain FP64 PCG only (opts->inner_prec == SEM_FP64, opts->pc
 * SEM_PC_NONE or SEM_PC_JACOBI, else SEM_ERR_ARG); use_graph is ignored
 * (kernels are launched directly on `stream`, which is also where the solve
 * runs and is timed on the host).  The solver's vectors, descriptor, work
 * lists, partial sums and scalars live in one 32 MiB array per GPU that the
 * library holds until the process ends; a mesh whose solve needs more
 * (about 8 (7 n_global + n_local + E) bytes: N = 7 up to about 10^3
 * elements) gets SEM_ERR_ARG.  Every call on a GPU shares that GPU's array:
 * calls that overlap in time on one GPU (other streams or host threads)
 * race and must be serialised by the caller.  Results are bit-identical to
 * sem_pcg_solve's with the same options.  Synchronises `stream`. */
sem_status sem_pcg_solve_noalloc(sem_handle *h, const sem_solve_opts *opts,
                                 const double *b_L, double *x_L,
                                 sem_solve_stats *stats, void *stream);

/* Batches of independent solves of the system of section 4.2.2 (uneven
 * sizes, orders N in {3, 5, 7} may be mixed, or any single N).  A batch references existing handles (which
 * must outlive it) and owns its work lists, per-solve device scalars and
 * captured graphs.  One CG iteration of the whole batch is six launches of
 * persistent kernels over (solve, element tile) and (solve, node chunk)
 * work items, captured once in a HIP graph and replayed check_every
 * iterations at a time; finished solves drop out on the device.  A solve
 * gives bit-identical results alone (sem_pcg_solve) or inside any batch.
 * A batch of more than one solve needs meshes without a mass term
 * (alpha = 0): SEM_ERR_ARG otherwise. */
sem_status sem_batch_create(sem_handle *const *handles, int32_t n,
                            sem_batch **out);
/* Release a batch of section 4.2.2 solves (its work lists, device scalars
 * and graphs; the handles stay).  NULL is accepted. */
sem_status sem_batch_destroy(sem_batch *b);
/* Autotuner of the batched operator of section 4.2.1 (the paper's own
 * measurements compare kernel tuning choices per platform, section 4.2.3):
 * times the batched operator kernel of precision p for every
 * workgroup size (64, 128, 256 threads) that holds the (N+1)^2 columns of
 * an element of the batch's largest order (one thread per column: N = 8
 * needs 128 or 256) and every persistent grid (1 tile per workgroup, or 4,
 * 8, 16, 32 workgroups per compute unit) and keeps the fastest for later
 * solves.  With the environment variable SEM_AUTOTUNE_CACHE naming a JSON
 * file, results are read from / added to it, keyed by GPU architecture,
 * order set, precision and size bucket; a cached block size too small for
 * the batch is ignored and tuned again.  Outputs may be NULL; *us is -1
 * when the value came from the cache. */
sem_status sem_batch_tune(sem_batch *b, int32_t p, int32_t *block_size,
                          int32_t *grid_mult, double *us);
/* Solve every system of the batch by PCG (section 4.2.2): b_L[q], x_L[q]
 * (HOST arrays of n device pointers) are the device E-vectors
 * of solve q (as in sem_pcg_solve); stats[q] receives its statistics
 * (seconds = wall time of the whole batch).  Synchronises `stream`.
 * Returns SEM_OK when all converged, else the first failing status. */
sem_status sem_batch_pcg_solve(sem_batch *b, const sem_solve_opts *opts,
                               const double *const *b_L, double *const *x_L,
                               sem_solve_stats *stats, void *stream);

/* ------------------------------------------------------------------------
 * Learned per-element coarse correction (SEM_PC_LEARNED).  Section 4.2.2
 * solves the system by PCG and leaves the preconditioner open; this one adds
 * to Jacobi a coarse correction per element,
 *   c = damping B (M_e / (kappa_e h_e)) B^T r_I,
 * on the element's interior nodes (zero on its faces): B holds the K
 * interior "bubble" modes of the element, tensor products of
 * (1 - x^2) P_a(x), a <= p = min(2, N-2), K = (p+1)^3, each scaled so that
 * the unit reference element's coarse inverse has unit diagonal; r_I is the
 * residual at the interior nodes; kappa_e is the mean of kappa at the 8
 * element vertices and h_e the element size.  M_e = L L^T, where the packed
 * lower-triangular factor L (K(K+1)/2 values, row-major) is the output of a
 * three-layer perceptron
 *   z1 = x W1^T + b1, h1 = relu(z1), z2 = h1 W2^T + b2, h2 = relu(z2),
 *   o = h2 W3^T + b3,
 * hidden width 128, on the element's features x: log kappa at its 8
 * vertices minus their mean (n_in = 8, padded with zeros to 16 columns).
 * The correction is symmetric positive semi-definite whatever the network
 * outputs.  Its target is the exact element coarse inverse
 * M_e* = kappa_e h_e (B^T A_II,e B)^{-1} (sem_learn_coarse_exact), which can
 * also be attached directly (sem_learn_attach_exact).  It is used inside
 * flexible CG (Notay 2000) with z = dinv o r + c.  Fallback to Jacobi-PCG
 * (stats.fell_back = 1) happens on NaN / breakdown, on stagnation (the
 * smallest residual so far drops less than 2x over 400 iterations), when
 * the learned solve's smallest residual shows less than 30% of the average
 * Jacobi rate after 300 or more iterations, when a refinement step fails to
 * halve the FP64 true residual (the step is undone), or when the damping is
 * 0.  Parameters are one FP32 vector: W1 [128][n_in], b1, W2 [128][128],
 * b2, W3 [n_out][128], b3 (row-major [out][in]).
 * ------------------------------------------------------------------------ */
/* He-initialised network of the section 4.2.2 correction (hidden width must
 * be 128, 1 <= n_in <= 4096, 1 <= n_out <= 1024; SEM_ERR_ARG otherwise),
 * BF16 precision (below).  *out receives a network the caller releases with
 * sem_mlp_destroy. */
sem_status sem_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out,
                          uint64_t seed, sem_mlp **out);
/* Release a network of the section 4.2.2 correction (detach it from every
 * handle first).  NULL is accepted. */
sem_status sem_mlp_destroy(sem_mlp *net);
/* Shapes of a section 4.2.2 correction network: inputs, hidden width,
 * outputs, inputs padded to a multiple of 16 (the row stride of X), the
 * parameter count and the number of Adam steps taken.  HOST outputs, any
 * may be NULL. */
sem_status sem_mlp_info(const sem_mlp *net, int32_t *n_in, int32_t *n_hidden,
                        int32_t *n_out, int32_t *n_in_padded,
                        int64_t *n_params, int64_t *adam_steps);
/* FP32 master parameters of the section 4.2.2 correction network, HOST
 * arrays of n_params floats (SEM_ERR_ARG for another n); set resets Adam. */
sem_status sem_mlp_get_params(const sem_mlp *net, float *params, int64_t n);
/* See sem_mlp_get_params (section 4.2.2 correction network). */
sem_status sem_mlp_set_params(sem_mlp *net, const float *params, int64_t n);
/* Arithmetic of the section 4.2.2 correction network.  SEM_BF16 (default):
 * BF16 copies of the weights, BF16 hidden activations as layer inputs,
 * forward layers on the matrix cores with FP32 accumulation, backward in
 * FP32 on the same BF16 values.  SEM_FP32: FP32 weights and hidden
 * activations, forward and backward in FP32 on the vector units (for
 * element-by-element checks).  The input x is BF16 in both.  Any other p:
 * SEM_ERR_ARG.  Synchronises the device. */
sem_status sem_mlp_set_precision(sem_mlp *net, int32_t p);
/* The precision set by sem_mlp_set_precision for a section 4.2.2
 * correction network (HOST output). */
sem_status sem_mlp_get_precision(const sem_mlp *net, int32_t *p);
/* Forward pass of the section 4.2.2 correction network on B samples:
 * X device BF16 [B][ldx] (ldx >= n_in_padded, a multiple of 16; padding
 * columns finite), Y device FP32 [B][n_out]. */
sem_status sem_mlp_forward(sem_mlp *net, const uint16_t *X, int32_t ldx,
                           int32_t B, float *Y, void *stream);
/* Loss and gradient of the section 4.2.2 coarse factor (n_out = K(K+1)/2,
 * K in {1, 8, 27}): per sample, T (device FP32 [B][2K]) holds y and alpha*;
 * the network output is the row-major packed lower triangle of L and the
 * loss is the mean over samples and components of (L L^T y - alpha*)^2.
 * grad: device FP32 [n_params] in parameter order (may be NULL: the
 * network's own gradient buffer is used by sem_mlp_adam with grad NULL).
 * *loss is written on the host (synchronises the stream). */
sem_status sem_mlp_loss_grad_factor(sem_mlp *net, const uint16_t *X,
                                    int32_t ldx, const float *T, int32_t K,
                                    int32_t B, float *grad, double *loss,
                                    void *stream);
/* One Adam step (Kingma & Ba 2015) on the master parameters of a
 * section 4.2.2 correction network with device gradient grad (NULL: the last
 * sem_mlp_loss_grad_factor gradient); lr > 0, betas in [0, 1), eps > 0. */
sem_status sem_mlp_adam(sem_mlp *net, const float *grad, double lr,
                        double beta1, double beta2, double eps, void *stream);
/* Scale of the section 4.2.2 correction (damping >= 0) and the Jacobi
 * reference rate of the progress check (log10 residual drop per Jacobi-PCG
 * iteration, <= 0; 0 disables the check). */
sem_status sem_mlp_set_damping(sem_mlp *net, double damping, double jacobi_rate);
/* See sem_mlp_set_damping (section 4.2.2 correction). */
sem_status sem_mlp_get_damping(const sem_mlp *net, double *damping,
                               double *jacobi_rate);
/* Checkpoint of a section 4.2.2 correction network: magic, version,
 * shapes, Adam step, damping, FP32 parameters and Adam moments, CRC-32
 * (the precision setting is not stored).  Load rejects truncated or
 * altered files (SEM_ERR_ARG). */
sem_status sem_mlp_save(const sem_mlp *net, const char *path);
/* See sem_mlp_save (section 4.2.2 correction network). */
sem_status sem_mlp_load(const char *path, sem_mlp **out);

/* Attach a network (NULL detaches) to a handle for SEM_PC_LEARNED, the
 * section 4.2.2 correction; the network must outlive the attachment.  It
 * needs n_in = 8 and n_out = K(K+1)/2 with K = (min(2, N-2)+1)^3 and
 * N >= 2 (SEM_ERR_ARG otherwise).  The element operators M_e are computed
 * from the network when it is attached and again before a solve when its
 * parameters or precision have changed.  The targets are those of the
 * stiffness operator: meshes with a mass term (alpha != 0) are refused with
 * SEM_ERR_STATE, here and in sem_learn_train. */
sem_status sem_learn_attach(sem_handle *h, sem_mlp *net);

/* Attach the exact element coarse inverses M_e* (no network) for
 * SEM_PC_LEARNED, with the given damping (finite, >= 0) and no progress
 * check: the section 4.2.2 correction that the network is trained to
 * imitate, for measuring what the network itself gains or loses.  Replaces
 * an attached network; sem_learn_attach (with a network or NULL) replaces
 * it.  N >= 2, no mass term. */
sem_status sem_learn_attach_exact(sem_handle *h, double damping);

typedef struct {
  int32_t n_pairs;          /* element residual pairs to sample */
  int32_t snapshot_every;   /* solver iterations between snapshots */
  int32_t max_snapshots;    /* per right-hand side */
  int32_t epochs;
  int32_t batch;            /* samples per Adam step */
  int32_t reserved;
  double lr;                /* Adam learning rate */
  double solve_rtol;        /* FP64 Jacobi-PCG tolerance of the data solves */
  uint64_t seed;            /* sampling and shuffling */
} sem_train_opts;

typedef struct {
  int32_t pairs, epochs, snapshots;
  int32_t reserved;
  double first_loss, last_loss;   /* mean loss of the first / last epoch */
  double data_seconds, train_seconds, validate_seconds;
  double damping;                 /* chosen correction scale (0: disabled) */
  double jacobi_rate;             /* Jacobi-PCG log10 residual drop / iteration */
  int32_t val_iters_jacobi, val_iters_learned;  /* validation solve to 1e-6 */
  int32_t val_iters[4];   /* learned iterations for the damping candidates
                             1, 0.75, 0.5, 0.25; -1: not converged or fell
                             back */
} sem_train_report;

/* Generate training pairs with the FP64 solver and train the section 4.2.2
 * correction network on the GPU.  For every right-hand side b_L[q] (device
 * FP64 E-vectors) a FP64 Jacobi-PCG solve from x = 0 records snapshots of
 * the residual; residuals restricted to random elements give the pairs:
 * y = B^T r_I / ||B^T r_I|| (for half the pairs, chosen at random, a random
 * unit direction instead, so that every direction of the operator is
 * trained) and alpha* = M_e* y with the exact M_e* of
 * sem_learn_coarse_exact.  A network that has never taken an Adam step
 * first starts from the identity factor (output bias = packed identity,
 * output weights scaled by 0.01).  Training: epochs of shuffled minibatches
 * of forward, loss, backward and Adam, all on the GPU.  Then the damping is
 * chosen from {1, 0.75, 0.5, 0.25} on the last right-hand side (solves to
 * 1e-6 against Jacobi-PCG; 0 when none helps). */
sem_status sem_learn_train(sem_handle *h, sem_mlp *net, const double *const *b_L,
                           int32_t n_rhs, const sem_train_opts *opts,
                           sem_train_report *report, void *stream);

/* Exact normalised coarse inverses of the section 4.2.2 correction (the
 * definition of its training targets, exposed for checking): M[e] (device
 * FP64 [E][K][K]) = kappa_e h_e (B^T A_II,e B)^{-1}, computed on the GPU by
 * applying the element operator to the K bubble columns and inverting the
 * K x K Galerkin matrix by Cholesky (NaN if it is not positive definite).
 * *K receives K.  Synchronises the stream.  N in 2..8. */
sem_status sem_learn_coarse_exact(sem_handle *h, double *M, int32_t *K,
                                  void *stream);

/* Text of the calling thread's last error ("" if none): the error path of
 * the set-up / build / call host pattern of section 4.1.2's driver. */
const char *sem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
