// Calibration surrogate: a 4 -> 128 -> 128 -> 128 -> 4 multilayer perceptron
// with GELU hidden activations (Hendrycks and Gimpel, 2016), mapping a
// calibration tuple (model, Tr, width parameter, kappa) to the equilibrium
// properties (rho_l, rho_v, surface tension, interface width), trained with
// Adam (Kingma and Ba, 2015) on equilibria computed by the batched lattices.
//
// Kernels (gfx950):
//   k_mlp_forward  tile of 16 samples per 256-thread workgroup; layer inputs
//                  kept in LDS, weights streamed from L2 with reads that are
//                  contiguous across the output index;
//   k_mlp_grad     forward, loss and back-propagation of a tile in one
//                  workgroup; a workgroup walks several tiles and accumulates
//                  its weight gradient in its own slice of the workspace; for
//                  the transposed products the 128 x 128 weight matrix is
//                  staged in LDS with rows padded to 129 words (no bank
//                  conflicts); ~130 KB LDS per workgroup;
//   k_mlp_reduce   sums the per-workgroup slices in a fixed order, so the
//                  gradient is deterministic;
//   k_mlp_adam     one elementwise Adam update.
// The network is ~34k parameters: every launch is latency-bound, not bound
// by HBM or the matrix units.
//
// BF16 mode rounds every product operand (layer inputs and weights) to
// bfloat16, round to nearest even; products of two bfloat16 values are exact
// in FP32 and all sums accumulate in FP32.  Its two 128 x 128 hidden layers
// run on the matrix cores (v_mfma_f32_16x16x16_bf16, hidden_mfma), in the
// forward pass of inference and of training; the 4-wide input and output
// layers and all FP32-mode products run on the vector ALUs.  Biases and
// back-propagated errors are not rounded (so the backward products stay on
// the vector ALUs in FP32); the weight rounding is treated as the identity
// in the gradient.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>

#include "lbm.h"

namespace mlpk {

constexpr int H = 128, NI = 4, NO = 4;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NI * H;
constexpr int OFF_W2 = OFF_B1 + H;
constexpr int OFF_B2 = OFF_W2 + H * H;
constexpr int OFF_W3 = OFF_B2 + H;
constexpr int OFF_B3 = OFF_W3 + H * H;
constexpr int OFF_W4 = OFF_B3 + H;
constexpr int OFF_B4 = OFF_W4 + H * NO;
constexpr int NPARAM = OFF_B4 + NO;
static_assert(NPARAM == LBM_MLP_NPARAMS, "parameter count");
constexpr int TS = 16;         // samples per tile
constexpr int NT = 256;        // threads per workgroup
constexpr int HALF = TS / 2;   // samples per thread in the 128-wide phases
constexpr int WPAD = H + 1;    // padded LDS row
constexpr int MAX_GRAD_BLOCKS = 128;

struct Norm {
  float xs[NI], xk[NI], ys[NO], yk[NO];
};

__device__ __forceinline__ float bf16r(float v) {
  unsigned u = __float_as_uint(v);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

template <int BF>
__device__ __forceinline__ float rnd(float v) {
  if constexpr (BF) return bf16r(v);
  else return v;
}

__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Bit pattern of a float that is already a bfloat16 value (low half zero).
__device__ __forceinline__ short bf16_bits(float v) {
  return (short)(__float_as_uint(v) >> 16);
}

// One 128 -> 128 hidden layer of a 16-sample tile on the matrix cores
// (BF16 mode): Z = A W + b with A the tile's rounded activations [16][128]
// and W the layer's weights [128][128] (row k, column j), rounded to
// bfloat16 as they are read; products of bfloat16 values are exact and the
// sums accumulate in FP32.  v_mfma_f32_16x16x16_bf16 multiplies a 16 x 16
// block of A by a 16 x 16 block of W: lane l supplies A[l % 16][4 (l / 16)
// + v] and W[4 (l / 16) + v][l % 16] (v = 0..3, offsets within the blocks)
// and receives Z[4 (l / 16) + v][l % 16].  Each of the four wavefronts
// computes two 16-column blocks of Z over the eight 16-row blocks of W.
__device__ __forceinline__ void hidden_mfma(const float* __restrict__ W, const float* __restrict__ bias,
                            const float (*a)[H], float (*z)[H], float (*an)[H]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int j = (2 * wv + nb) * 16 + r;
    const float b = bias[j];
    f32x4 acc = {b, b, b, b};
#pragma unroll
    for (int kb = 0; kb < H / 16; ++kb) {
      const int k0 = kb * 16 + 4 * q;
      bf16x4 av, wv4;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        av[v] = bf16_bits(a[r][k0 + v]);
        wv4[v] = bf16_bits(bf16r(W[(k0 + v) * H + j]));
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, wv4, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * q + v;
      z[i][j] = acc[v];
      an[i][j] = bf16r(gelu(acc[v]));
    }
  }
}

// Forward pass of one tile.  s_a0: [TS][NI] rounded inputs (already set);
// s_z: [3][TS][H] pre-activations; s_a: [3][TS][H] rounded activations;
// s_o: [TS][NO] outputs in normalised log space.  Sample rows >= nv hold
// zero inputs and finite values that the callers ignore.
template <int BF>
__device__ __forceinline__ void forward_tile(const float* __restrict__ P, const float (*s_a0)[NI],
                             float (*s_z)[TS][H], float (*s_a)[TS][H], float (*s_o)[NO]) {
  const int t = threadIdx.x;
  const int j = t & (H - 1), sh = (t >> 7) * HALF;
  {
    float acc[HALF];
    const float b = P[OFF_B1 + j];
#pragma unroll
    for (int q = 0; q < HALF; ++q) acc[q] = b;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const float w = rnd<BF>(P[OFF_W1 + k * H + j]);
#pragma unroll
      for (int q = 0; q < HALF; ++q) acc[q] = fmaf(w, s_a0[sh + q][k], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
      s_z[0][sh + q][j] = acc[q];
      s_a[0][sh + q][j] = rnd<BF>(gelu(acc[q]));
    }
  }
  __syncthreads();
  for (int l = 1; l < 3; ++l) {
    const float* W = P + (l == 1 ? OFF_W2 : OFF_W3);
    if constexpr (BF) {
      hidden_mfma(W, P + (l == 1 ? OFF_B2 : OFF_B3), s_a[l - 1], s_z[l], s_a[l]);
      __syncthreads();
      continue;
    }
    float acc[HALF];
    const float b = P[(l == 1 ? OFF_B2 : OFF_B3) + j];
#pragma unroll
    for (int q = 0; q < HALF; ++q) acc[q] = b;
    for (int k = 0; k < H; ++k) {
      const float w = rnd<BF>(W[k * H + j]);
#pragma unroll
      for (int q = 0; q < HALF; ++q) acc[q] = fmaf(w, s_a[l - 1][sh + q][k], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < HALF; ++q) {
      s_z[l][sh + q][j] = acc[q];
      s_a[l][sh + q][j] = rnd<BF>(gelu(acc[q]));
    }
    __syncthreads();
  }
  if (t < TS * NO) {
    const int s = t / NO, o = t % NO;
    float acc = P[OFF_B4 + o];
    for (int k = 0; k < H; ++k) acc = fmaf(rnd<BF>(P[OFF_W4 + k * NO + o]), s_a[2][s][k], acc);
    s_o[s][o] = acc;
  }
  __syncthreads();
}

template <int BF>
__device__ __forceinline__ void load_inputs(const float* __restrict__ X, const Norm& nm, int s0,
                                            int nv, float (*s_a0)[NI], const int* __restrict__ idx,
                                            int nrows, bool* bad) {
  const int t = threadIdx.x;
  if (t < TS * NI) {
    const int s = t / NI, k = t % NI;
    float v = 0.0f;
    if (s < nv) {
      const int r = idx ? idx[s0 + s] : s0 + s;
      if (r >= 0 && r < nrows) v = rnd<BF>((X[(size_t)r * NI + k] - nm.xs[k]) * nm.xk[k]);
      else *bad = true;
    }
    s_a0[s][k] = v;
  }
}

template <int BF>
__global__ __launch_bounds__(NT) void k_mlp_forward(const float* __restrict__ P, Norm nm,
                                                    const float* __restrict__ X, int n,
                                                    float* __restrict__ Y) {
  __shared__ float s_a0[TS][NI];
  __shared__ float s_z[3][TS][H];
  __shared__ float s_a[3][TS][H];
  __shared__ float s_o[TS][NO];
  const int s0 = blockIdx.x * TS;
  const int nv = min(TS, n - s0);
  bool bad = false;
  load_inputs<BF>(X, nm, s0, nv, s_a0, nullptr, n, &bad);
  __syncthreads();
  forward_tile<BF>(P, s_a0, s_z, s_a, s_o);
  const int t = threadIdx.x;
  if (t < TS * NO) {
    const int s = t / NO, o = t % NO;
    if (s < nv) Y[(size_t)(s0 + s) * NO + o] = expf(s_o[s][o] * nm.yk[o] + nm.ys[o]);
  }
}

// Gradient slice update: the first tile of a workgroup stores, later tiles
// add.  Each slice element is owned by one thread in every phase, the same
// thread for every tile.
__device__ __forceinline__ void gput(float* p, float g, bool first) {
  if (first) *p = g;
  else *p += g;
}

// Loss and gradient partials.  Workgroup g handles tiles g, g + G, ...
// (G <= number of tiles, so every workgroup has at least one); its gradient
// slice part[g * NPARAM ...] and loss partial lpart[g] are fully written by
// this kernel (no prior clearing needed).
template <int BF>
__global__ __launch_bounds__(NT) void k_mlp_grad(const float* __restrict__ P, Norm nm,
                                                 const float* __restrict__ X,
                                                 const float* __restrict__ Y,
                                                 const int* __restrict__ idx, int n, int nrows,
                                                 float scale, float* __restrict__ part,
                                                 float* __restrict__ lpart) {
  __shared__ float s_a0[TS][NI];
  __shared__ float s_z[3][TS][H];
  __shared__ float s_a[3][TS][H];
  __shared__ float s_d[TS][H];   // dL/dz of the current layer
  __shared__ float s_e[TS][H];   // dL/dz of the layer below
  __shared__ float s_w[H][WPAD];
  __shared__ float s_o[TS][NO];  // outputs, then dL/dout
  __shared__ float s_l[NT / 64];
  __shared__ int s_bad;
  const int t = threadIdx.x;
  const int j = t & (H - 1), hsel = t >> 7, sh = hsel * HALF;
  float* G = part + (size_t)blockIdx.x * NPARAM;
  if (t == 0) s_bad = 0;
  __syncthreads();
  float lacc = 0.0f;
  const int ntiles = (n + TS - 1) / TS;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int s0 = tile * TS;
    const int nv = min(TS, n - s0);
    const bool first = tile == (int)blockIdx.x;
    bool bad = false;
    load_inputs<BF>(X, nm, s0, nv, s_a0, idx, nrows, &bad);
    if (bad) s_bad = 1;
    __syncthreads();
    forward_tile<BF>(P, s_a0, s_z, s_a, s_o);
    // loss and dL/dout (zero for padding rows and rejected indices)
    float dv = 0.0f;
    if (t < TS * NO) {
      const int s = t / NO, o = t % NO;
      if (s < nv) {
        const int r = idx ? idx[s0 + s] : s0 + s;
        if (r >= 0 && r < nrows) {
          const float tgt = (logf(Y[(size_t)r * NO + o]) - nm.ys[o]) / nm.yk[o];
          const float res = s_o[s][o] - tgt;
          lacc = fmaf(res, res, lacc);
          dv = 2.0f * res * scale;
        }
      }
    }
    __syncthreads();  // every output read before it is overwritten
    if (t < TS * NO) s_o[t / NO][t % NO] = dv;
    __syncthreads();
    // output layer: dW4[k][o] = sum_s a3[s][k] dout[s][o]
    for (int e = t; e < H * NO; e += NT) {
      const int k = e / NO, o = e % NO;
      float g = 0.0f;
#pragma unroll
      for (int s = 0; s < TS; ++s) g = fmaf(s_a[2][s][k], s_o[s][o], g);
      gput(&G[OFF_W4 + e], g, first);
    }
    if (t < NO) {
      float g = 0.0f;
#pragma unroll
      for (int s = 0; s < TS; ++s) g += s_o[s][t];
      gput(&G[OFF_B4 + t], g, first);
    }
    {
      float w[NO];
#pragma unroll
      for (int o = 0; o < NO; ++o) w[o] = rnd<BF>(P[OFF_W4 + j * NO + o]);
#pragma unroll
      for (int q = 0; q < HALF; ++q) {
        const int s = sh + q;
        float da = 0.0f;
#pragma unroll
        for (int o = 0; o < NO; ++o) da = fmaf(s_o[s][o], w[o], da);
        s_d[s][j] = da * gelu_d(s_z[2][s][j]);
      }
    }
    __syncthreads();
    // hidden layers 3 and 2: input activations s_a[l - 1], weights W_{l+1}
    for (int l = 2; l >= 1; --l) {
      const int offw = (l == 2) ? OFF_W3 : OFF_W2;
      const int offb = (l == 2) ? OFF_B3 : OFF_B2;
      const float* W = P + offw;
      for (int e = t; e < H * H; e += NT) s_w[e >> 7][e & (H - 1)] = rnd<BF>(W[e]);
      {
        float dz[TS];
#pragma unroll
        for (int s = 0; s < TS; ++s) dz[s] = s_d[s][j];
        for (int m = 0; m < H / 2; ++m) {
          const int k = hsel + 2 * m;
          float g = 0.0f;
#pragma unroll
          for (int s = 0; s < TS; ++s) g = fmaf(s_a[l - 1][s][k], dz[s], g);
          gput(&G[offw + k * H + j], g, first);
        }
        if (hsel == 0) {
          float g = 0.0f;
#pragma unroll
          for (int s = 0; s < TS; ++s) g += dz[s];
          gput(&G[offb + j], g, first);
        }
      }
      __syncthreads();  // weights staged
      {
        float acc[HALF];
#pragma unroll
        for (int q = 0; q < HALF; ++q) acc[q] = 0.0f;
        for (int jj = 0; jj < H; ++jj) {
          const float w = s_w[j][jj];
#pragma unroll
          for (int q = 0; q < HALF; ++q) acc[q] = fmaf(s_d[sh + q][jj], w, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < HALF; ++q) s_e[sh + q][j] = acc[q] * gelu_d(s_z[l - 1][sh + q][j]);
      }
      __syncthreads();
      for (int e = t; e < TS * H; e += NT) s_d[e >> 7][e & (H - 1)] = s_e[e >> 7][e & (H - 1)];
      __syncthreads();
    }
    // first layer: dW1[k][j] = sum_s a0[s][k] dz1[s][j]
    {
      float dz[TS];
#pragma unroll
      for (int s = 0; s < TS; ++s) dz[s] = s_d[s][j];
#pragma unroll
      for (int m = 0; m < NI / 2; ++m) {
        const int k = hsel + 2 * m;
        float g = 0.0f;
#pragma unroll
        for (int s = 0; s < TS; ++s) g = fmaf(s_a0[s][k], dz[s], g);
        gput(&G[OFF_W1 + k * H + j], g, first);
      }
      if (hsel == 0) {
        float g = 0.0f;
#pragma unroll
        for (int s = 0; s < TS; ++s) g += dz[s];
        gput(&G[OFF_B1 + j], g, first);
      }
    }
    __syncthreads();  // LDS reused by the next tile
  }
  // loss partial of this workgroup
  for (int off = 32; off > 0; off >>= 1) lacc += __shfl_down(lacc, off, 64);
  if ((t & 63) == 0) s_l[t >> 6] = lacc;
  __syncthreads();
  if (t == 0) {
    float s = 0.0f;
    for (int w = 0; w < NT / 64; ++w) s += s_l[w];
    lpart[blockIdx.x] = s_bad ? NAN : s;
  }
}

__global__ void k_mlp_reduce(const float* __restrict__ part, const float* __restrict__ lpart,
                             int nblk, float scale, float* __restrict__ grad,
                             float* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) {
    float g = 0.0f;
    for (int b = 0; b < nblk; ++b) g += part[(size_t)b * NPARAM + p];
    grad[p] = g;
  }
  if (p == 0 && loss) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += lpart[b];
    *loss = s * scale;
  }
}

__global__ void k_mlp_adam(float* __restrict__ P, float* __restrict__ M, float* __restrict__ V,
                           const float* __restrict__ G, float lr, float b1, float b2, float eps,
                           float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = G[p];
  const float m = b1 * M[p] + (1.0f - b1) * g;
  const float v = b2 * V[p] + (1.0f - b2) * g * g;
  M[p] = m;
  V[p] = v;
  P[p] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

Norm to_norm(const lbm_mlp_norm* n) {
  Norm r;
  for (int i = 0; i < NI; ++i) {
    r.xs[i] = n->x_shift[i];
    r.xk[i] = n->x_scale[i];
  }
  for (int i = 0; i < NO; ++i) {
    r.ys[i] = n->y_shift[i];
    r.yk[i] = n->y_scale[i];
  }
  return r;
}

bool norm_ok(const lbm_mlp_norm* n) {
  for (int i = 0; i < NO; ++i)
    if (!(n->y_scale[i] != 0.0f) || !isfinite(n->y_scale[i]) || !isfinite(n->y_shift[i]))
      return false;
  for (int i = 0; i < NI; ++i)
    if (!isfinite(n->x_scale[i]) || !isfinite(n->x_shift[i])) return false;
  return true;
}

int grad_blocks(int n) {
  const int tiles = (n + TS - 1) / TS;
  return tiles < MAX_GRAD_BLOCKS ? tiles : MAX_GRAD_BLOCKS;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace layout of a gradient over n samples: per-workgroup gradient
// slices, then the per-workgroup loss partials.
size_t part_bytes(int g) { return align256((size_t)g * NPARAM * sizeof(float)); }

lbm_status grad_args_ok(const float* d_params, const lbm_mlp_norm* norm, const float* d_x,
                        const float* d_y, int32_t n_rows, const int32_t* d_idx, int32_t n,
                        const float* d_grad, int32_t flags) {
  if (!d_params || !norm || !d_x || !d_y || !d_grad || n < 1 || n_rows < 1 ||
      (!d_idx && n > n_rows) || (flags & ~LBM_MLP_BF16))
    return LBM_ERR_INVALID_ARG;
  if (!norm_ok(norm)) return LBM_ERR_INVALID_ARG;
  return LBM_OK;
}

// The gradient kernels of lbm_mlp_grad on a scratch area `ws` laid out as
// above (arguments already checked).
lbm_status grad_launch(const float* d_params, const lbm_mlp_norm* norm, const float* d_x,
                       const float* d_y, int32_t n_rows, const int32_t* d_idx, int32_t n,
                       float* d_grad, float* d_loss, int32_t flags, char* ws, hipStream_t st) {
  const Norm nm = to_norm(norm);
  const int g = grad_blocks(n);
  float* part = (float*)ws;
  float* lpart = (float*)(ws + part_bytes(g));
  const float scale = 1.0f / (4.0f * (float)n);
  if (flags & LBM_MLP_BF16)
    hipLaunchKernelGGL(k_mlp_grad<1>, dim3(g), dim3(NT), 0, st, d_params, nm, d_x, d_y, d_idx,
                       n, n_rows, scale, part, lpart);
  else
    hipLaunchKernelGGL(k_mlp_grad<0>, dim3(g), dim3(NT), 0, st, d_params, nm, d_x, d_y, d_idx,
                       n, n_rows, scale, part, lpart);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, st, part, lpart, g,
                     scale, d_grad, d_loss);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

// ---- allocation-free gradient ----------------------------------------------
// lbm_mlp_grad_noalloc keeps the gradient partials in this file-scope device
// array instead of a caller workspace: room for the partials of
// LBM_MLP_NOALLOC_MAX_N samples (64 workgroup slices, about 8.4 MiB).  Every
// GPU the library runs on holds its own copy until the process ends.  In
// host code `scratch` is only a host-side stand-in for the symbol; kernels
// get its device address, looked up once per device below.
constexpr int NOALLOC_BLOCKS = (LBM_MLP_NOALLOC_MAX_N + TS - 1) / TS;
static_assert(NOALLOC_BLOCKS <= MAX_GRAD_BLOCKS, "no-alloc bound");
constexpr size_t NOALLOC_BYTES =
    ((size_t)NOALLOC_BLOCKS * NPARAM * sizeof(float) + 255) / 256 * 256 +
    ((size_t)NOALLOC_BLOCKS * sizeof(float) + 255) / 256 * 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device dev: hipGetSymbolAddress with dev
// current, on the first call for dev; later calls reuse the stored pointer.
lbm_status scratch_on(int dev, char** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return LBM_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return LBM_ERR_HIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return LBM_ERR_HIP;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return LBM_ERR_HIP;
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

}  // namespace mlpk

using namespace mlpk;

extern "C" {

lbm_status lbm_mlp_workspace_bytes(int32_t n, size_t* bytes) {
  if (n < 1 || !bytes) return LBM_ERR_INVALID_ARG;
  const int g = grad_blocks(n);
  *bytes = align256((size_t)g * NPARAM * sizeof(float)) + align256((size_t)g * sizeof(float));
  return LBM_OK;
}

lbm_status lbm_mlp_forward(const float* d_params, const lbm_mlp_norm* norm, const float* d_x,
                           int32_t n, float* d_y, int32_t flags, void* hip_stream) {
  if (!d_params || !norm || n < 0 || (n > 0 && (!d_x || !d_y)) || (flags & ~LBM_MLP_BF16))
    return LBM_ERR_INVALID_ARG;
  if (!norm_ok(norm)) return LBM_ERR_INVALID_ARG;
  if (n == 0) return LBM_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const Norm nm = to_norm(norm);
  const int nb = (n + TS - 1) / TS;
  if (flags & LBM_MLP_BF16)
    hipLaunchKernelGGL(k_mlp_forward<1>, dim3(nb), dim3(NT), 0, st, d_params, nm, d_x, n, d_y);
  else
    hipLaunchKernelGGL(k_mlp_forward<0>, dim3(nb), dim3(NT), 0, st, d_params, nm, d_x, n, d_y);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

lbm_status lbm_mlp_grad(const float* d_params, const lbm_mlp_norm* norm, const float* d_x,
                        const float* d_y, int32_t n_rows, const int32_t* d_idx, int32_t n,
                        float* d_grad, float* d_loss, int32_t flags, void* d_workspace,
                        size_t bytes, void* hip_stream) {
  lbm_status s = grad_args_ok(d_params, norm, d_x, d_y, n_rows, d_idx, n, d_grad, flags);
  if (s != LBM_OK) return s;
  size_t need;
  lbm_mlp_workspace_bytes(n, &need);
  if (!d_workspace || bytes < need || ((uintptr_t)d_workspace % 256) != 0)
    return LBM_ERR_WORKSPACE;
  return grad_launch(d_params, norm, d_x, d_y, n_rows, d_idx, n, d_grad, d_loss, flags,
                     (char*)d_workspace, (hipStream_t)hip_stream);
}

lbm_status lbm_mlp_grad_noalloc(const float* d_params, const lbm_mlp_norm* norm,
                                const float* d_x, const float* d_y, int32_t n_rows,
                                const int32_t* d_idx, int32_t n, float* d_grad, float* d_loss,
                                int32_t flags, void* hip_stream) {
  lbm_status s = grad_args_ok(d_params, norm, d_x, d_y, n_rows, d_idx, n, d_grad, flags);
  if (s != LBM_OK) return s;
  if (n > LBM_MLP_NOALLOC_MAX_N) return LBM_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = -1;
  if (st) {
    if (hipStreamGetDevice(st, &dev) != hipSuccess) return LBM_ERR_HIP;
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return LBM_ERR_HIP;
  }
  char* ws = nullptr;
  if ((s = scratch_on(dev, &ws)) != LBM_OK) return s;
  return grad_launch(d_params, norm, d_x, d_y, n_rows, d_idx, n, d_grad, d_loss, flags, ws, st);
}

lbm_status lbm_mlp_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t t,
                        float lr, float beta1, float beta2, float eps, void* hip_stream) {
  if (!d_params || !d_m || !d_v || !d_grad || t < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f) ||
      !(beta1 < 1.0f) || !(beta2 >= 0.0f) || !(beta2 < 1.0f) || !(eps > 0.0f))
    return LBM_ERR_INVALID_ARG;
  const float bc1 = (float)(1.0 - pow((double)beta1, (double)t));
  const float bc2 = (float)(1.0 - pow((double)beta2, (double)t));
  hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0,
                     (hipStream_t)hip_stream, d_params, d_m, d_v, d_grad, lr, beta1, beta2, eps,
                     bc1, bc2);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

lbm_status lbm_mlp_train_step(float* d_params, float* d_m, float* d_v, int64_t t, float lr,
                              const lbm_mlp_norm* norm, const float* d_x, const float* d_y,
                              int32_t n_rows, const int32_t* d_idx, int32_t n, float* d_grad,
                              float* d_loss, int32_t flags, void* d_workspace, size_t bytes,
                              void* hip_stream) {
  if (!d_m || !d_v || t < 1 || !(lr >= 0.0f)) return LBM_ERR_INVALID_ARG;
  lbm_status s = lbm_mlp_grad(d_params, norm, d_x, d_y, n_rows, d_idx, n, d_grad, d_loss, flags,
                              d_workspace, bytes, hip_stream);
  if (s != LBM_OK) return s;
  return lbm_mlp_adam(d_params, d_m, d_v, d_grad, t, lr, 0.9f, 0.999f, 1e-8f, hip_stream);
}

}  // extern "C"
