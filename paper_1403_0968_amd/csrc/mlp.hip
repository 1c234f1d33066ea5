// Learned per-element coarse correction: a three-layer perceptron
//   z1 = x W1^T + b1, h1 = relu(z1); z2 = h1 W2^T + b2, h2 = relu(z2);
//   o = h2 W3^T + b3  (the packed factor of the element's coarse operator)
// trained on the GPU by the kernels of this file (forward, loss and
// backward, Adam of Kingma & Ba 2015).  The paper leaves the PCG
// preconditioner open (section 4.2.2); this network is one choice of it.
//
// Precision (per network): BF16 (the default) keeps FP32 master parameters
// and BF16 copies of the weights that feed the forward layers, which run on
// MFMA (v_mfma_f32_16x16x16_bf16, FP32 accumulation) with BF16 layer
// inputs; the backward pass is FP32 on VALU using the same BF16-rounded
// weights and layer inputs as the forward pass.  FP32 runs the forward
// layers on VALU with the FP32 master weights and FP32 hidden activations
// (the network input stays BF16), and the backward pass on the same values:
// it differs from an exact evaluation only by FP32 rounding, which makes
// element-by-element checks of every parameter block possible.
//
// MFMA tile (16x16x16): lane l holds A[l % 16][4 (l / 16) + 0..3] and
// B[4 (l / 16) + 0..3][l % 16] (4 BF16 values each); the result C[4 (l / 16) +
// q][l % 16] is accumulator slot q.  A forward layer Y = X W^T gives every
// wave a 16-row strip of X and all output columns.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <random>
#include <vector>

#include "common.h"
#include "sem_internal.h"

namespace sem {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// forward layer on MFMA
// ---------------------------------------------------------------------------
// Y = act(X W^T + b): X [M][ldx] BF16 (K columns used, K % 16 == 0),
// W [16 NT][K] BF16 (rows >= N are zero), b [N] FP32.  Writes columns < N of
// Yb (BF16, [M][ldyb]) and/or Yf (FP32, [M][ldyf]) when non-null.
// Output columns are split over blockIdx.y in slices of 16 NT; W must have
// at least 16 NT gridDim.y rows.
template <int NT, bool RELU>
__global__ void __launch_bounds__(256)
    k_dense_mfma(int M, int K, int N, const uint16_t *__restrict__ X, int ldx,
                 const uint16_t *__restrict__ W, const float *__restrict__ b,
                 uint16_t *__restrict__ Yb, int ldyb, float *__restrict__ Yf,
                 int ldyf) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + wave) * 16;
  const int cbase = blockIdx.y * 16 * NT;
  if (row0 >= M) return;  // whole wave; no barriers in this kernel
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ar = row0 + (l & 15);
  const int kq = 4 * (l >> 4);
  const bool arow = ar < M;
  for (int k0 = 0; k0 < K; k0 += 16) {
    s16x4 a = {0, 0, 0, 0};
    if (arow) a = *reinterpret_cast<const s16x4 *>(X + (size_t)ar * ldx + k0 + kq);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const s16x4 w = *reinterpret_cast<const s16x4 *>(
          W + (size_t)(cbase + 16 * t + (l & 15)) * K + k0 + kq);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, w, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = cbase + 16 * t + (l & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = row0 + 4 * (l >> 4) + q;
      if (row < M && col < N) {
        float v = acc[t][q] + b[col];
        if (RELU) v = fmaxf(v, 0.0f);
        if (Yb) Yb[(size_t)row * ldyb + col] = f32_to_bf16(v);
        if (Yf) Yf[(size_t)row * ldyf + col] = v;
      }
    }
  }
}

template <class T> __device__ inline float asf(T v);
template <> __device__ inline float asf<float>(float v) { return v; }
template <> __device__ inline float asf<uint16_t>(uint16_t v) {
  return bf16_to_f32(v);
}

// ---------------------------------------------------------------------------
// forward layer on VALU, FP32 weights (the FP32 precision of a network)
// ---------------------------------------------------------------------------
// Y[m][n] = act(sum_k X[m][k] W[n][k] + b[n]) for n < N, k < K: X [M][ldx]
// (BF16 or FP32), W FP32 [N][ldw], Y FP32 [M][ldy].  16 x 16 output tiles,
// 16-wide K slices through LDS; the sum runs over k in ascending order.
template <class TX, bool RELU>
__global__ void __launch_bounds__(256)
    k_dense_f32(int M, int K, int N, const TX *__restrict__ X, int ldx,
                const float *__restrict__ W, int ldw, const float *__restrict__ b,
                float *__restrict__ Y, int ldy) {
  __shared__ float sx[16][17], sw[16][17];
  const int tm = threadIdx.x / 16, tn = threadIdx.x % 16;
  const int m = blockIdx.x * 16 + tm, n = blockIdx.y * 16 + tn;
  float acc = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int r = threadIdx.x / 16, c = threadIdx.x % 16;
    const int mi = blockIdx.x * 16 + r, ni = blockIdx.y * 16 + r, kc = k0 + c;
    sx[r][c] = (mi < M && kc < K) ? asf<TX>(X[(size_t)mi * ldx + kc]) : 0.f;
    sw[r][c] = (ni < N && kc < K) ? W[(size_t)ni * ldw + kc] : 0.f;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += sx[tm][q] * sw[tn][q];
    __syncthreads();
  }
  if (m < M && n < N) {
    float v = acc + b[n];
    if (RELU) v = fmaxf(v, 0.0f);
    Y[(size_t)m * ldy + n] = v;
  }
}

// ---------------------------------------------------------------------------
// backward kernels (FP32)
// ---------------------------------------------------------------------------

// dW[n][k] = sum_b dY[b][n] X[b][k]  (n < N, k < Kv); dW row stride Kv
template <class TX>
__global__ void __launch_bounds__(256)
    k_grad_w(int B, int N, int Kv, const float *__restrict__ dY, int lddy,
             const TX *__restrict__ X, int ldx, float *__restrict__ dW) {
  __shared__ float sy[16][17], sx[16][17];
  const int tn = threadIdx.x / 16, tk = threadIdx.x % 16;
  const int n = blockIdx.x * 16 + tn, k = blockIdx.y * 16 + tk;
  float acc = 0.f;
  for (int b0 = 0; b0 < B; b0 += 16) {
    // load 16 samples: sy[bb][n-tile], sx[bb][k-tile]
    const int bb = threadIdx.x / 16, c = threadIdx.x % 16;
    const int bi = b0 + bb;
    const int nn = blockIdx.x * 16 + c, kk = blockIdx.y * 16 + c;
    sy[bb][c] = (bi < B && nn < N) ? dY[(size_t)bi * lddy + nn] : 0.f;
    sx[bb][c] = (bi < B && kk < Kv) ? asf<TX>(X[(size_t)bi * ldx + kk]) : 0.f;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += sy[q][tn] * sx[q][tk];
    __syncthreads();
  }
  if (n < N && k < Kv) dW[(size_t)n * Kv + k] = acc;
}

// db[n] = sum_b dY[b][n]
__global__ void k_grad_b(int B, int N, const float *__restrict__ dY, int lddy,
                         float *__restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float acc = 0.f;
  for (int b = 0; b < B; ++b) acc += dY[(size_t)b * lddy + n];
  db[n] = acc;
}

// dZ[b][k] = (sum_n dY[b][n] W[n][k]) * (H[b][k] > 0), W BF16 or FP32
// [>=N][ldw]
template <class TW>
__global__ void __launch_bounds__(256)
    k_grad_x(int B, int N, int K, const float *__restrict__ dY, int lddy,
             const TW *__restrict__ W, int ldw,
             const float *__restrict__ H, int ldh, float *__restrict__ dZ,
             int lddz) {
  __shared__ float sy[16][17], sw[16][17];
  const int tb = threadIdx.x / 16, tk = threadIdx.x % 16;
  const int b = blockIdx.x * 16 + tb, k = blockIdx.y * 16 + tk;
  float acc = 0.f;
  for (int n0 = 0; n0 < N; n0 += 16) {
    const int r = threadIdx.x / 16, c = threadIdx.x % 16;
    const int bi = blockIdx.x * 16 + r, ni = n0 + c;
    sy[r][c] = (bi < B && ni < N) ? dY[(size_t)bi * lddy + ni] : 0.f;
    const int nw = n0 + r, kw = blockIdx.y * 16 + c;
    sw[r][c] = (nw < N && kw < K) ? asf<TW>(W[(size_t)nw * ldw + kw]) : 0.f;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += sy[tb][q] * sw[q][tk];
    __syncthreads();
  }
  if (b < B && k < K)
    dZ[(size_t)b * lddz + k] = H[(size_t)b * ldh + k] > 0.f ? acc : 0.f;
}

// coarse-operator factor: the output is a lower-triangular K x K factor L
// (row-major packed); per sample, T holds y and alpha* (2K values) and the
// loss is the mean of (L L^T y - alpha*)^2; dL = g v^T + y (L^T g)^T with
// v = L^T y and g the loss gradient with respect to L L^T y.  One thread
// per sample.
template <int K>
__global__ void __launch_bounds__(64)
    k_loss_factor(int B, const float *__restrict__ O, int ldo,
                  const float *__restrict__ T, float *__restrict__ dO, int lddo,
                  double *__restrict__ lossp) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float *o = O + (size_t)b * ldo;
  const float *y = T + (size_t)b * 2 * K, *as = y + K;
  float v[K], g[K], w[K];
  for (int j = 0; j < K; ++j) v[j] = w[j] = 0.f;
  for (int i = 0, q = 0; i < K; ++i)
    for (int j = 0; j <= i; ++j, ++q) v[j] += o[q] * y[i];
  double loss = 0.0;
  const float sc = (float)(2.0 / ((double)B * K));
  for (int i = 0, q = 0; i < K; ++i) {
    float a = 0.f;
    for (int j = 0; j <= i; ++j) a += o[q + j] * v[j];
    q += i + 1;
    const float d = a - as[i];
    loss += (double)d * (double)d;
    g[i] = sc * d;
  }
  for (int i = 0, q = 0; i < K; ++i)
    for (int j = 0; j <= i; ++j, ++q) w[j] += o[q] * g[i];
  for (int i = 0, q = 0; i < K; ++i)
    for (int j = 0; j <= i; ++j, ++q) dO[(size_t)b * lddo + q] = g[i] * v[j] + y[i] * w[j];
  lossp[b] = loss;
}

__global__ void k_sum_losses(int B, const double *__restrict__ lossp, int nn,
                             double *out) {
  __shared__ double sm[4];
  double a = 0.0;
  for (int q = threadIdx.x; q < B; q += 256) a += lossp[q];
  const double s = block_sum<256>(a, sm);
  if (threadIdx.x == 0) out[0] = s / ((double)B * nn);
}

__global__ void k_adam(int64_t n, float *__restrict__ th, float *__restrict__ m,
                       float *__restrict__ v, const float *__restrict__ g,
                       float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  th[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// BF16 weights from the FP32 master: W1b [H][kin], W2b [H][H],
// W3b [w3rows][H] (rows >= n_out zero)
__global__ void k_refresh(int n_in, int kin, int H, int n_out, int w3rows,
                          const float *__restrict__ th, uint16_t *__restrict__ W1b,
                          uint16_t *__restrict__ W2b, uint16_t *__restrict__ W3b) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n1 = (int64_t)H * kin, n2 = (int64_t)H * H,
                n3 = (int64_t)w3rows * H;
  const float *W1 = th, *W2 = th + (int64_t)H * n_in + H,
              *W3 = W2 + (int64_t)H * H + H;
  if (q < n1) {
    const int r = (int)(q / kin), c = (int)(q % kin);
    W1b[q] = c < n_in ? f32_to_bf16(W1[(int64_t)r * n_in + c]) : 0;
  } else if (q < n1 + n2) {
    const int64_t p = q - n1;
    W2b[p] = f32_to_bf16(W2[p]);
  } else if (q < n1 + n2 + n3) {
    const int64_t p = q - n1 - n2;
    const int r = (int)(p / H), c = (int)(p % H);
    W3b[p] = r < n_out ? f32_to_bf16(W3[(int64_t)r * H + c]) : 0;
  }
}

}  // namespace sem

// ---------------------------------------------------------------------------
// the network object
// ---------------------------------------------------------------------------
struct sem_mlp {
  int n_in = 0, H = 0, n_out = 0, kin = 0;
  int prec = SEM_BF16;      // SEM_BF16 (MFMA, BF16 weights) or SEM_FP32 (VALU)
  int nt3 = 1, gy3 = 1, w3rows = 16;  // output layer: tiles per wave, grid.y
  int64_t np = 0, step = 0;
  uint64_t version = 1;     // changes whenever the parameters change
  double damping = 1.0;     // scale of the correction in the preconditioner
  double ref_rate = 0.0;    // Jacobi-PCG log10 residual drop per iteration
                            // on the training problem (0: unknown)
  sem::DevBuf th, m, v, grad, W1b, W2b, W3b;
  sem::DevBuf dev_damping;  // device copy of `damping` read by the correction
                            // kernels (captured graphs see its updates)
  // training scratch, sized for `cap` samples
  int cap = 0;
  sem::DevBuf h1b, h2b, h1f, h2f, of, dO, dz2, dz1, lossp, lossd;
  double *host_loss = nullptr;
  ~sem_mlp() {
    if (host_loss) (void)hipHostFree(host_loss);
  }
};

namespace sem {

void mlp_set_damping(sem_mlp *net, double d, double rate);

static int64_t mlp_np(int n_in, int H, int n_out) {
  return (int64_t)H * n_in + H + (int64_t)H * H + H + (int64_t)n_out * H + n_out;
}

void mlp_refresh(sem_mlp *net, hipStream_t s) {
  const int64_t n = (int64_t)net->H * net->kin + (int64_t)net->H * net->H +
                    (int64_t)net->w3rows * net->H;
  hipLaunchKernelGGL(k_refresh, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     net->n_in, net->kin, net->H, net->n_out, net->w3rows,
                     net->th.as<float>(),
                     net->W1b.as<uint16_t>(), net->W2b.as<uint16_t>(),
                     net->W3b.as<uint16_t>());
  SEM_HIP(hipGetLastError());
}

sem_mlp *mlp_create(int n_in, int H, int n_out, uint64_t seed) {
  if (n_in < 1 || n_in > 4096) fail(SEM_ERR_ARG, "mlp: n_in must be in 1..4096");
  if (H != 128) fail(SEM_ERR_ARG, "mlp: hidden width must be 128");
  if (n_out < 1 || n_out > 1024) fail(SEM_ERR_ARG, "mlp: n_out must be in 1..1024");
  sem_mlp *net = new sem_mlp();
  try {
    net->n_in = n_in;
    net->H = H;
    net->n_out = n_out;
    net->kin = (n_in + 15) / 16 * 16;
    if (n_out <= 16) {
      net->nt3 = 1;
      net->gy3 = 1;
      net->w3rows = 16;
    } else {
      net->nt3 = 8;
      net->gy3 = (n_out + 127) / 128;
      net->w3rows = 128 * net->gy3;
    }
    net->np = mlp_np(n_in, H, n_out);
    net->th.alloc(net->np * 4);
    net->m.alloc(net->np * 4);
    net->v.alloc(net->np * 4);
    net->grad.alloc(net->np * 4);
    net->W1b.alloc((size_t)H * net->kin * 2);
    net->W2b.alloc((size_t)H * H * 2);
    net->W3b.alloc((size_t)net->w3rows * H * 2);
    // He initialisation (normal, std sqrt(2 / fan_in)), zero biases
    std::vector<float> th(net->np, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    int64_t k = 0;
    auto fill = [&](int rows, int cols) {
      const double sd = std::sqrt(2.0 / cols);
      for (int64_t q = 0; q < (int64_t)rows * cols; ++q) th[k++] = (float)(nd(rng) * sd);
      k += rows;  // bias
    };
    fill(H, n_in);
    fill(H, H);
    fill(n_out, H);
    SEM_HIP(hipMemcpy(net->th.p, th.data(), net->np * 4, hipMemcpyHostToDevice));
    SEM_HIP(hipMemset(net->m.p, 0, net->np * 4));
    SEM_HIP(hipMemset(net->v.p, 0, net->np * 4));
    SEM_HIP(hipHostMalloc((void **)&net->host_loss, sizeof(double), 0));
    net->dev_damping.alloc(sizeof(float));
    mlp_set_damping(net, 1.0, 0.0);
    mlp_refresh(net, nullptr);
    SEM_HIP(hipDeviceSynchronize());
  } catch (...) {
    delete net;
    throw;
  }
  return net;
}

void mlp_set_params(sem_mlp *net, const float *host, int64_t n) {
  net->version += 1;
  if (n != net->np) fail(SEM_ERR_ARG, "mlp_set_params: wrong parameter count");
  SEM_HIP(hipMemcpy(net->th.p, host, n * 4, hipMemcpyHostToDevice));
  SEM_HIP(hipMemset(net->m.p, 0, n * 4));
  SEM_HIP(hipMemset(net->v.p, 0, n * 4));
  net->step = 0;
  mlp_refresh(net, nullptr);
  SEM_HIP(hipDeviceSynchronize());
}

void mlp_get_params(const sem_mlp *net, float *host, int64_t n) {
  if (n != net->np) fail(SEM_ERR_ARG, "mlp_get_params: wrong parameter count");
  SEM_HIP(hipDeviceSynchronize());
  SEM_HIP(hipMemcpy(host, net->th.p, n * 4, hipMemcpyDeviceToHost));
}

static void ensure_scratch(sem_mlp *net, int B) {
  if (B <= net->cap) return;
  const int H = net->H;
  net->h1b.alloc((size_t)B * H * 2);
  net->h2b.alloc((size_t)B * H * 2);
  net->h1f.alloc((size_t)B * H * 4);
  net->h2f.alloc((size_t)B * H * 4);
  const int wo = net->n_out > 16 ? net->n_out : 16;
  net->of.alloc((size_t)B * wo * 4);
  net->dO.alloc((size_t)B * wo * 4);
  net->dz2.alloc((size_t)B * H * 4);
  net->dz1.alloc((size_t)B * H * 4);
  net->lossp.alloc((size_t)B * 8);
  net->lossd.alloc(8);
  net->cap = B;
}

// forward of B samples X [B][ldx] BF16 (ldx >= kin, padding columns zero)
// into O [B][ldo] FP32 with the hidden activations in the given buffers:
// BF16 precision writes h1b, h2b (BF16 [B][H], the next layer's inputs) and,
// when non-null, their FP32 values h1f, h2f (for a backward pass); FP32
// precision writes h1f, h2f (FP32 [B][H]) only.
static void forward_into(sem_mlp *net, const uint16_t *X, int ldx, int B,
                         float *O, int ldo, uint16_t *h1b, uint16_t *h2b,
                         float *h1f, float *h2f, hipStream_t s) {
  if (ldx < net->kin || ldx % 16 != 0)
    fail(SEM_ERR_ARG, "mlp_forward: ldx must be >= padded n_in and a multiple of 16");
  const int H = net->H;
  const float *W1 = net->th.as<float>();
  const float *b1 = W1 + (int64_t)H * net->n_in;
  const float *W2 = b1 + H;
  const float *b2 = W2 + (int64_t)H * H;
  const float *W3 = b2 + H;
  const float *b3 = W3 + (int64_t)net->n_out * H;
  if (net->prec == SEM_FP32) {
    const unsigned gm = (unsigned)((B + 15) / 16);
    hipLaunchKernelGGL((k_dense_f32<uint16_t, true>), dim3(gm, H / 16), dim3(256),
                       0, s, B, net->n_in, H, X, ldx, W1, net->n_in, b1, h1f, H);
    hipLaunchKernelGGL((k_dense_f32<float, true>), dim3(gm, H / 16), dim3(256), 0,
                       s, B, H, H, (const float *)h1f, H, W2, H, b2, h2f, H);
    hipLaunchKernelGGL((k_dense_f32<float, false>),
                       dim3(gm, (unsigned)((net->n_out + 15) / 16)), dim3(256), 0,
                       s, B, H, net->n_out, (const float *)h2f, H, W3, H, b3, O,
                       ldo);
    SEM_HIP(hipGetLastError());
    return;
  }
  const unsigned grid = (unsigned)((B + 63) / 64);
  hipLaunchKernelGGL((k_dense_mfma<8, true>), dim3(grid), dim3(256), 0, s, B,
                     net->kin, H, X, ldx, net->W1b.as<uint16_t>(), b1, h1b, H,
                     h1f, H);
  hipLaunchKernelGGL((k_dense_mfma<8, true>), dim3(grid), dim3(256), 0, s, B, H,
                     H, h1b, H, net->W2b.as<uint16_t>(), b2, h2b, H, h2f, H);
  if (net->nt3 == 1)
    hipLaunchKernelGGL((k_dense_mfma<1, false>), dim3(grid), dim3(256), 0, s, B, H,
                       net->n_out, h2b, H, net->W3b.as<uint16_t>(), b3,
                       (uint16_t *)nullptr, 0, O, ldo);
  else
    hipLaunchKernelGGL((k_dense_mfma<8, false>), dim3(grid, net->gy3), dim3(256), 0,
                       s, B, H, net->n_out, h2b, H, net->W3b.as<uint16_t>(), b3,
                       (uint16_t *)nullptr, 0, O, ldo);
  SEM_HIP(hipGetLastError());
}

// forward with the hidden activations kept in the network's scratch (grown
// to B samples when needed) for a backward pass
void mlp_forward(sem_mlp *net, const uint16_t *X, int ldx, int B, float *O,
                 int ldo, hipStream_t s) {
  if (B <= 0) return;
  ensure_scratch(net, B);
  forward_into(net, X, ldx, B, O, ldo, net->h1b.as<uint16_t>(),
               net->h2b.as<uint16_t>(), net->h1f.as<float>(), net->h2f.as<float>(),
               s);
}

// backward pass from net->dO (written by a loss kernel) into net->grad
// (flat parameter order), on the weights and layer inputs the forward pass
// used; then the mean loss over B samples of `count` terms each
static double mlp_backward(sem_mlp *net, const uint16_t *X, int ldx, int B,
                           int count, bool host_loss, hipStream_t s) {
  const int H = net->H;
  const int wo = net->n_out > 16 ? net->n_out : 16;
  const bool f32 = net->prec == SEM_FP32;
  float *g = net->grad.as<float>();
  float *gW1 = g, *gb1 = gW1 + (int64_t)H * net->n_in, *gW2 = gb1 + H,
        *gb2 = gW2 + (int64_t)H * H, *gW3 = gb2 + H,
        *gb3 = gW3 + (int64_t)net->n_out * H;
  const float *W2 = net->th.as<float>() + (int64_t)H * net->n_in + H;
  const float *W3 = W2 + (int64_t)H * H + H;
  const float *dO = net->dO.as<float>(), *dz2 = net->dz2.as<float>(),
              *dz1 = net->dz1.as<float>();
  const float *h1f = net->h1f.as<float>(), *h2f = net->h2f.as<float>();
  // layer 3
  if (f32)
    hipLaunchKernelGGL((k_grad_w<float>), dim3((net->n_out + 15) / 16, H / 16),
                       dim3(256), 0, s, B, net->n_out, H, dO, wo, h2f, H, gW3);
  else
    hipLaunchKernelGGL((k_grad_w<uint16_t>), dim3((net->n_out + 15) / 16, H / 16),
                       dim3(256), 0, s, B, net->n_out, H, dO, wo,
                       (const uint16_t *)net->h2b.as<uint16_t>(), H, gW3);
  hipLaunchKernelGGL(k_grad_b, dim3((net->n_out + 127) / 128), dim3(128), 0, s, B,
                     net->n_out, dO, wo, gb3);
  if (f32)
    hipLaunchKernelGGL((k_grad_x<float>), dim3((B + 15) / 16, H / 16), dim3(256), 0,
                       s, B, net->n_out, H, dO, wo, W3, H, h2f, H,
                       net->dz2.as<float>(), H);
  else
    hipLaunchKernelGGL((k_grad_x<uint16_t>), dim3((B + 15) / 16, H / 16),
                       dim3(256), 0, s, B, net->n_out, H, dO, wo,
                       (const uint16_t *)net->W3b.as<uint16_t>(), H, h2f, H,
                       net->dz2.as<float>(), H);
  // layer 2
  if (f32)
    hipLaunchKernelGGL((k_grad_w<float>), dim3(H / 16, H / 16), dim3(256), 0, s, B,
                       H, H, dz2, H, h1f, H, gW2);
  else
    hipLaunchKernelGGL((k_grad_w<uint16_t>), dim3(H / 16, H / 16), dim3(256), 0, s,
                       B, H, H, dz2, H, (const uint16_t *)net->h1b.as<uint16_t>(),
                       H, gW2);
  hipLaunchKernelGGL(k_grad_b, dim3(1), dim3(128), 0, s, B, H, dz2, H, gb2);
  if (f32)
    hipLaunchKernelGGL((k_grad_x<float>), dim3((B + 15) / 16, H / 16), dim3(256), 0,
                       s, B, H, H, dz2, H, W2, H, h1f, H, net->dz1.as<float>(), H);
  else
    hipLaunchKernelGGL((k_grad_x<uint16_t>), dim3((B + 15) / 16, H / 16),
                       dim3(256), 0, s, B, H, H, dz2, H,
                       (const uint16_t *)net->W2b.as<uint16_t>(), H, h1f, H,
                       net->dz1.as<float>(), H);
  // layer 1 (the input X is BF16 in both precisions)
  hipLaunchKernelGGL((k_grad_w<uint16_t>),
                     dim3(H / 16, (net->n_in + 15) / 16), dim3(256), 0, s, B, H,
                     net->n_in, dz1, H, X, ldx, gW1);
  hipLaunchKernelGGL(k_grad_b, dim3(1), dim3(128), 0, s, B, H, dz1, H, gb1);
  hipLaunchKernelGGL(k_sum_losses, dim3(1), dim3(256), 0, s, B,
                     net->lossp.as<double>(), count, net->lossd.as<double>());
  SEM_HIP(hipGetLastError());
  if (!host_loss) return 0.0;
  SEM_HIP(hipMemcpyAsync(net->host_loss, net->lossd.p, sizeof(double),
                         hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  return *net->host_loss;
}

// loss and gradient of the coarse-operator factor (n_out = K(K+1)/2,
// K in {1, 8, 27}); T [B][2K] holds y and alpha* per sample
double mlp_loss_grad_factor(sem_mlp *net, const uint16_t *X, int ldx,
                            const float *T, int K, int B, bool host_loss,
                            hipStream_t s) {
  if (net->n_out != K * (K + 1) / 2 || (K != 1 && K != 8 && K != 27))
    fail(SEM_ERR_ARG, "mlp_loss_grad_factor: K must be 1, 8 or 27 and "
                      "n_out = K(K+1)/2");
  ensure_scratch(net, B);
  const int wo = net->n_out > 16 ? net->n_out : 16;
  mlp_forward(net, X, ldx, B, net->of.as<float>(), wo, s);
  const dim3 g((unsigned)((B + 63) / 64)), t(64);
  if (K == 1)
    hipLaunchKernelGGL(k_loss_factor<1>, g, t, 0, s, B, net->of.as<float>(), wo, T,
                       net->dO.as<float>(), wo, net->lossp.as<double>());
  else if (K == 8)
    hipLaunchKernelGGL(k_loss_factor<8>, g, t, 0, s, B, net->of.as<float>(), wo, T,
                       net->dO.as<float>(), wo, net->lossp.as<double>());
  else
    hipLaunchKernelGGL(k_loss_factor<27>, g, t, 0, s, B, net->of.as<float>(), wo, T,
                       net->dO.as<float>(), wo, net->lossp.as<double>());
  return mlp_backward(net, X, ldx, B, K, host_loss, s);
}

uint64_t mlp_version(const sem_mlp *net) { return net->version; }

void mlp_set_precision(sem_mlp *net, int prec) {
  if (prec != SEM_BF16 && prec != SEM_FP32)
    fail(SEM_ERR_ARG, "mlp_set_precision: SEM_BF16 or SEM_FP32");
  SEM_HIP(hipDeviceSynchronize());  // no forward pass may be in flight
  net->prec = prec;
  net->version += 1;  // outputs derived from the network must be recomputed
}

int mlp_precision(const sem_mlp *net) { return net->prec; }

void mlp_adam(sem_mlp *net, const float *grad, double lr, double b1, double b2,
              double eps, hipStream_t s) {
  net->version += 1;
  net->step += 1;
  const double c1 = 1.0 - std::pow(b1, (double)net->step);
  const double c2 = 1.0 - std::pow(b2, (double)net->step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((net->np + 255) / 256)), dim3(256), 0,
                     s, net->np, net->th.as<float>(), net->m.as<float>(),
                     net->v.as<float>(), grad ? grad : net->grad.as<float>(),
                     (float)lr, (float)b1, (float)b2, (float)eps, (float)c1,
                     (float)c2);
  SEM_HIP(hipGetLastError());
  mlp_refresh(net, s);
}

// ---------------------------------------------------------------------------
// checkpoint: header, FP32 master parameters, Adam moments, CRC-32 (IEEE
// 802.3 polynomial, reflected) of everything before it
// ---------------------------------------------------------------------------
static uint32_t crc32_update(uint32_t crc, const unsigned char *p, size_t n) {
  static uint32_t table[256];
  static bool init = false;
  if (!init) {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      table[i] = c;
    }
    init = true;
  }
  crc = ~crc;
  for (size_t q = 0; q < n; ++q) crc = table[(crc ^ p[q]) & 0xff] ^ (crc >> 8);
  return ~crc;
}

struct CkptHeader {
  char magic[8];  // "SEMMLP01"
  uint32_t version, n_in, H, n_out;
  uint64_t step, np;
  double damping, ref_rate;
};

void mlp_save(const sem_mlp *net, const char *path) {
  SEM_HIP(hipDeviceSynchronize());
  CkptHeader hd{};
  memcpy(hd.magic, "SEMMLP01", 8);
  hd.version = 2;
  hd.damping = net->damping;
  hd.ref_rate = net->ref_rate;
  hd.n_in = net->n_in;
  hd.H = net->H;
  hd.n_out = net->n_out;
  hd.step = (uint64_t)net->step;
  hd.np = (uint64_t)net->np;
  std::vector<float> buf(3 * net->np);
  SEM_HIP(hipMemcpy(buf.data(), net->th.p, net->np * 4, hipMemcpyDeviceToHost));
  SEM_HIP(hipMemcpy(buf.data() + net->np, net->m.p, net->np * 4,
                    hipMemcpyDeviceToHost));
  SEM_HIP(hipMemcpy(buf.data() + 2 * net->np, net->v.p, net->np * 4,
                    hipMemcpyDeviceToHost));
  uint32_t crc = crc32_update(0, (const unsigned char *)&hd, sizeof hd);
  crc = crc32_update(crc, (const unsigned char *)buf.data(), buf.size() * 4);
  std::ofstream f(path, std::ios::binary);
  if (!f) fail(SEM_ERR_ARG, "mlp_save: cannot open file");
  f.write((const char *)&hd, sizeof hd);
  f.write((const char *)buf.data(), buf.size() * 4);
  f.write((const char *)&crc, 4);
  if (!f) fail(SEM_ERR_ARG, "mlp_save: write failed");
}

sem_mlp *mlp_load(const char *path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) fail(SEM_ERR_ARG, "mlp_load: cannot open file");
  CkptHeader hd{};
  f.read((char *)&hd, sizeof hd);
  if (!f || memcmp(hd.magic, "SEMMLP01", 8) != 0 || hd.version != 2)
    fail(SEM_ERR_ARG, "mlp_load: not a network checkpoint");
  if (hd.H != 128 || hd.n_in < 1 || hd.n_in > 4096 || hd.n_out < 1 ||
      hd.n_out > 1024 || hd.np != (uint64_t)mlp_np(hd.n_in, hd.H, hd.n_out) ||
      !std::isfinite(hd.damping) || !std::isfinite(hd.ref_rate))
    fail(SEM_ERR_ARG, "mlp_load: inconsistent shapes");
  std::vector<float> buf(3 * hd.np);
  f.read((char *)buf.data(), buf.size() * 4);
  uint32_t crc_file = 0;
  f.read((char *)&crc_file, 4);
  if (!f) fail(SEM_ERR_ARG, "mlp_load: truncated checkpoint");
  uint32_t crc = crc32_update(0, (const unsigned char *)&hd, sizeof hd);
  crc = crc32_update(crc, (const unsigned char *)buf.data(), buf.size() * 4);
  if (crc != crc_file) fail(SEM_ERR_ARG, "mlp_load: checksum mismatch");
  sem_mlp *net = mlp_create(hd.n_in, hd.H, hd.n_out, 0);
  try {
    SEM_HIP(hipMemcpy(net->th.p, buf.data(), hd.np * 4, hipMemcpyHostToDevice));
    SEM_HIP(hipMemcpy(net->m.p, buf.data() + hd.np, hd.np * 4,
                      hipMemcpyHostToDevice));
    SEM_HIP(hipMemcpy(net->v.p, buf.data() + 2 * hd.np, hd.np * 4,
                      hipMemcpyHostToDevice));
    net->step = (int64_t)hd.step;
    mlp_set_damping(net, hd.damping, hd.ref_rate);
    mlp_refresh(net, nullptr);
    SEM_HIP(hipDeviceSynchronize());
  } catch (...) {
    delete net;
    throw;
  }
  return net;
}

void mlp_destroy(sem_mlp *net) { delete net; }

void mlp_info(const sem_mlp *net, int *n_in, int *H, int *n_out, int64_t *np,
              int64_t *step) {
  if (n_in) *n_in = net->n_in;
  if (H) *H = net->H;
  if (n_out) *n_out = net->n_out;
  if (np) *np = net->np;
  if (step) *step = net->step;
}

int mlp_padded_inputs(const sem_mlp *net) { return net->kin; }

const float *mlp_grad_ptr(const sem_mlp *net) { return net->grad.as<float>(); }

double mlp_damping(const sem_mlp *net) { return net->damping; }
double mlp_ref_rate(const sem_mlp *net) { return net->ref_rate; }
void mlp_set_damping(sem_mlp *net, double d, double rate) {
  net->damping = d;
  net->ref_rate = rate;
  const float f = (float)d;
  SEM_HIP(hipDeviceSynchronize());  // no solve may be reading it
  SEM_HIP(hipMemcpy(net->dev_damping.p, &f, sizeof f, hipMemcpyHostToDevice));
}

const float *mlp_damping_dev(const sem_mlp *net) {
  return net->dev_damping.as<float>();
}

}  // namespace sem
