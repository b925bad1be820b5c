// Learned warm start: a small network trained on equilibria the method itself computes maps
// (voltage, permittivity ratio, contact angle) to the equilibrium phase field, used as the
// starting state of the equilibrium march (the march to the residual tolerance stays the
// judge).  Everything runs in the kernels below: the two small hidden layers in FP32, the
// large output layer (hidden units -> every grid value) and its two backward products on the
// matrix cores in BF16 with FP32 accumulation, FP32 master weights, Adam.
//
//   a1 = W1 p + b1, h1 = gelu(a1); a2 = W2 h1 + b2, h2 = gelu(a2); y = W3 h2 + b3
//   loss = mean over batch and outputs of (y - t)^2
//
// Layouts: weights in one FP32 blob [W1 (H1x3) | b1 | W2 (H2xH1) | b2 | W3 (NxH2) | b3 (N)],
// gradients, Adam moments likewise; W3 also as BF16 (row n contiguous); batch quantities
// sample-major, except dL/dy which is stored output-major [n][b] for the backward products.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <random>
#include <string>
#include <vector>

#include "../../include/pfd.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define WS_MAXB 32        // minibatch size the products are laid out for (smaller batches are zero-padded)
#define WS_H1 64
#define WS_H2 128
#define WS_CHUNK 1024     // output rows per work-group in the dL/dh2 product

namespace {

__device__ __forceinline__ uint16_t to_bf16(float f) {   // round to nearest, ties to even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float dgelu(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}
__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {      // 8 consecutive BF16 (16-byte aligned)
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// accumulator element j of lane group g holds row 4g + j, column lane % 16 (16x16 FP32 layout)

// ---- hidden layers, one work-group per sample (rows >= B are zero padding)
__global__ void k_ws_fwd_small(int B, const float* __restrict__ P, const int* __restrict__ idx,
                               const float* __restrict__ w, float* __restrict__ a1, float* __restrict__ h1,
                               float* __restrict__ a2, float* __restrict__ h2, uint16_t* __restrict__ h2b) {
  __shared__ float sh1[WS_H1];
  const int b = blockIdx.x, t = threadIdx.x;
  const float* W1 = w;
  const float* b1 = W1 + WS_H1 * 3;
  const float* W2 = b1 + WS_H1;
  const float* b2 = W2 + WS_H2 * WS_H1;
  if (b >= B) {
    if (t < WS_H2) {
      h2b[b * WS_H2 + t] = 0;
      h2[b * WS_H2 + t] = 0.0f;
    }
    return;
  }
  const float* p = P + 3 * (idx ? idx[b] : b);
  if (t < WS_H1) {
    const float a = b1[t] + W1[t * 3] * p[0] + W1[t * 3 + 1] * p[1] + W1[t * 3 + 2] * p[2];
    a1[b * WS_H1 + t] = a;
    const float h = gelu(a);
    h1[b * WS_H1 + t] = h;
    sh1[t] = h;
  }
  __syncthreads();
  if (t < WS_H2) {
    float a = b2[t];
    for (int j = 0; j < WS_H1; ++j) a += W2[t * WS_H1 + j] * sh1[j];
    a2[b * WS_H2 + t] = a;
    const float h = gelu(a);
    h2[b * WS_H2 + t] = h;
    h2b[b * WS_H2 + t] = to_bf16(h);
  }
}

// ---- output layer y = W3 h2 + b3 on the matrix cores; with targets also dL/dy and loss parts.
// A wave computes 16 output rows for every (padded) sample: K = H2 in four 32-wide steps.
__global__ void __launch_bounds__(256) k_ws_out(long N, int Bp, int B, const uint16_t* __restrict__ W3b,
                                                const uint16_t* __restrict__ h2b, const float* __restrict__ b3,
                                                const float* __restrict__ T, const int* __restrict__ idx,
                                                float* __restrict__ y, float* __restrict__ dy,
                                                uint16_t* __restrict__ dyb, double* __restrict__ part) {
  __shared__ double red[256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r16 = lane & 15, g = lane >> 4;
  const long n0 = ((long)blockIdx.x * 4 + w) * 16;
  const int nbt = Bp / 16;
  f32x4 acc[WS_MAXB / 16];
  for (int i = 0; i < WS_MAXB / 16; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const long na = n0 + r16 < N ? n0 + r16 : N - 1;     // clamped row (rows >= N never stored)
#pragma unroll
  for (int kk = 0; kk < WS_H2 / 32; ++kk) {
    const bf16x8 a = ld8(W3b + na * WS_H2 + 32 * kk + 8 * g);
    for (int bt = 0; bt < nbt; ++bt) {
      const bf16x8 bv = ld8(h2b + (16 * bt + r16) * WS_H2 + 32 * kk + 8 * g);
      acc[bt] = mma(a, bv, acc[bt]);
    }
  }
  double lsum = 0.0;
  for (int bt = 0; bt < nbt; ++bt) {
    const int b = 16 * bt + r16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long n = n0 + 4 * g + j;
      if (n >= N) continue;
      const float v = acc[bt][j] + b3[n];
      if (y && b < B) y[(long)b * N + n] = v;
      if (T) {
        float d = 0.0f;
        if (b < B) {
          const float dd = v - T[(long)(idx ? idx[b] : b) * N + n];
          lsum += (double)dd * dd;
          d = 2.0f * dd / ((float)B * (float)N);
        }
        dy[n * Bp + b] = d;
        dyb[n * Bp + b] = to_bf16(d);
      }
    }
  }
  if (!part) return;
  red[threadIdx.x] = lsum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---- dL/dW3 = dy^T h2 (K = batch) and dL/db3 = sum_b dy; a wave owns 16 output rows
__global__ void __launch_bounds__(256) k_ws_bwd_w3(long N, int Bp, const uint16_t* __restrict__ dyb,
                                                   const float* __restrict__ dy, const uint16_t* __restrict__ h2b,
                                                   float* __restrict__ gW3, float* __restrict__ gb3) {
  __shared__ __align__(16) uint16_t hT[WS_H2 * WS_MAXB];   // h2 transposed: [h][b]
  for (int i = threadIdx.x; i < WS_H2 * Bp; i += 256) {
    const int h = i / Bp, b = i - h * Bp;
    hT[h * Bp + b] = h2b[b * WS_H2 + h];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r16 = lane & 15, g = lane >> 4;
  const long n0 = ((long)blockIdx.x * 4 + w) * 16;
  const long na = n0 + r16 < N ? n0 + r16 : N - 1;
  f32x4 acc[WS_H2 / 16];
  for (int i = 0; i < WS_H2 / 16; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < Bp; k0 += 32) {
    const bf16x8 a = ld8(dyb + na * Bp + k0 + 8 * g);
#pragma unroll
    for (int ht = 0; ht < WS_H2 / 16; ++ht) {
      const bf16x8 bv = ld8(hT + (16 * ht + r16) * Bp + k0 + 8 * g);
      acc[ht] = mma(a, bv, acc[ht]);
    }
  }
#pragma unroll
  for (int ht = 0; ht < WS_H2 / 16; ++ht)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long n = n0 + 4 * g + j;
      if (n < N) gW3[n * WS_H2 + 16 * ht + r16] = acc[ht][j];
    }
  if (lane < 16) {
    const long n = n0 + lane;
    if (n < N) {
      float s = 0.0f;
      for (int b = 0; b < Bp; ++b) s += dy[n * Bp + b];
      gb3[n] = s;
    }
  }
}

// ---- dL/dh2 = dy W3 over all N outputs: each work-group sums WS_CHUNK rows (its four waves
// take a quarter each, reduced through LDS in a fixed order) into one partial [h][b]
__global__ void __launch_bounds__(256) k_ws_bwd_h2(long N, int Bp, const uint16_t* __restrict__ dyb,
                                                   const uint16_t* __restrict__ W3b, float* __restrict__ part) {
  __shared__ float red[3][WS_H2 / 16][WS_MAXB / 16][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r16 = lane & 15, g = lane >> 4;
  f32x4 acc[WS_H2 / 16][WS_MAXB / 16];
#pragma unroll
  for (int i = 0; i < WS_H2 / 16; ++i)
#pragma unroll
    for (int j = 0; j < WS_MAXB / 16; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const long c0 = (long)blockIdx.x * WS_CHUNK + (long)w * (WS_CHUNK / 4);
  for (long k0 = c0; k0 < c0 + WS_CHUNK / 4 && k0 < N; k0 += 32) {
    // A[h][n] = W3[n][h], B[n][b] = dy[n][b]; contraction index n = k0 + 8g + e
    bf16x8 av[WS_H2 / 16], bvv[WS_MAXB / 16];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      long n = k0 + 8 * g + e;
      const bool ok = n < N;
      n = ok ? n : N - 1;
#pragma unroll
      for (int ht = 0; ht < WS_H2 / 16; ++ht) av[ht][e] = __builtin_bit_cast(__bf16, W3b[n * WS_H2 + 16 * ht + r16]);
#pragma unroll
      for (int bt = 0; bt < WS_MAXB / 16; ++bt) {
        const uint16_t d = dyb[n * Bp + 16 * bt + r16];
        bvv[bt][e] = __builtin_bit_cast(__bf16, ok ? d : (uint16_t)0);
      }
    }
#pragma unroll
    for (int ht = 0; ht < WS_H2 / 16; ++ht)
#pragma unroll
      for (int bt = 0; bt < WS_MAXB / 16; ++bt) acc[ht][bt] = mma(av[ht], bvv[bt], acc[ht][bt]);
  }
  if (w > 0) {
#pragma unroll
    for (int ht = 0; ht < WS_H2 / 16; ++ht)
#pragma unroll
      for (int bt = 0; bt < WS_MAXB / 16; ++bt)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[w - 1][ht][bt][j][lane] = acc[ht][bt][j];
  }
  __syncthreads();
  if (w != 0) return;
  float* out = part + (long)blockIdx.x * WS_H2 * Bp;
#pragma unroll
  for (int ht = 0; ht < WS_H2 / 16; ++ht)
#pragma unroll
    for (int bt = 0; bt < WS_MAXB / 16; ++bt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float v = ((acc[ht][bt][j] + red[0][ht][bt][j][lane]) + red[1][ht][bt][j][lane]) +
                        red[2][ht][bt][j][lane];
        out[(16 * ht + 4 * g + j) * Bp + 16 * bt + r16] = v;
      }
}

// ---- sum the partials (fixed order), then the hidden layers' backward pass; one work-group
__global__ void __launch_bounds__(256) k_ws_bwd_small(int B, int Bp, int nparts, const float* __restrict__ part,
                                                      const float* __restrict__ P, const int* __restrict__ idx,
                                                      const float* __restrict__ w, const float* __restrict__ a1,
                                                      const float* __restrict__ h1, const float* __restrict__ a2,
                                                      float* __restrict__ grad) {
  __shared__ float da2[WS_MAXB][WS_H2];
  __shared__ float da1[WS_MAXB][WS_H1];
  const int t = threadIdx.x;
  const float* W2 = w + WS_H1 * 3 + WS_H1;
  float* gW1 = grad;
  float* gb1 = gW1 + WS_H1 * 3;
  float* gW2 = gb1 + WS_H1;
  float* gb2 = gW2 + WS_H2 * WS_H1;
  for (int i = t; i < B * WS_H2; i += 256) {
    const int b = i / WS_H2, h = i - b * WS_H2;
    float s = 0.0f;
    for (int q = 0; q < nparts; ++q) s += part[(long)q * WS_H2 * Bp + h * Bp + b];
    da2[b][h] = s * dgelu(a2[b * WS_H2 + h]);
  }
  __syncthreads();
  for (int i = t; i < WS_H2 * WS_H1; i += 256) {
    const int h = i / WS_H1, j = i - h * WS_H1;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += da2[b][h] * h1[b * WS_H1 + j];
    gW2[i] = s;
  }
  for (int h = t; h < WS_H2; h += 256) {
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += da2[b][h];
    gb2[h] = s;
  }
  for (int i = t; i < B * WS_H1; i += 256) {
    const int b = i / WS_H1, j = i - b * WS_H1;
    float s = 0.0f;
    for (int h = 0; h < WS_H2; ++h) s += W2[h * WS_H1 + j] * da2[b][h];
    da1[b][j] = s * dgelu(a1[b * WS_H1 + j]);
  }
  __syncthreads();
  for (int i = t; i < WS_H1 * 3; i += 256) {
    const int j = i / 3, c = i - j * 3;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += da1[b][j] * P[3 * (idx ? idx[b] : b) + c];
    gW1[i] = s;
  }
  for (int j = t; j < WS_H1; j += 256) {
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += da1[b][j];
    gb1[j] = s;
  }
}

// ---- Adam on every weight; refreshes the BF16 copy of W3
__global__ void k_ws_adam(long n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, float lr, float beta1, float beta2, float c1, float c2, float eps,
                          long o3, long n3, uint16_t* __restrict__ W3b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (i >= o3 && i < o3 + n3) W3b[i - o3] = to_bf16(wi);
  }
}

__global__ void k_ws_to_bf16(long n, const float* __restrict__ a, uint16_t* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = to_bf16(a[i]);
}

// b3 = mean of the training targets over the samples
__global__ void k_ws_mean(long N, long S, const float* __restrict__ T, float* __restrict__ b3) {
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (long q = 0; q < S; ++q) s += T[q * N + n];
    b3[n] = (float)(s / (double)S);
  }
}

// partial sums of weights * y and of the weights (mass projection)
__global__ void k_ws_wsum(long N, const float* __restrict__ y, const double* __restrict__ wt, double* __restrict__ part) {
  __shared__ double red[2][256];
  double s = 0.0, sw = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < N; i += (long)gridDim.x * 256) {
    s += wt[i] * (double)y[i];
    sw += wt[i];
  }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = sw;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}
__global__ void k_ws_shift(long N, const float* __restrict__ y, double c, double* __restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    out[i] = (double)y[i] + c;
}

}  // namespace

struct pfd_ws {
  pfd_ws_arch arch;
  hipStream_t stream = nullptr;
  std::string err;
  long N = 0, nw = 0, o3 = 0, nparts = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t* W3b = nullptr;
  float *a1 = nullptr, *h1 = nullptr, *a2 = nullptr, *h2 = nullptr;
  uint16_t* h2b = nullptr;
  float* y = nullptr;      // [Bp][N]
  float* dy = nullptr;     // [N][Bp]
  uint16_t* dyb = nullptr;
  float* part = nullptr;   // dL/dh2 partials
  double* lpart = nullptr; // loss partials
  double* wpart = nullptr; // weighted-sum partials
  int* idx = nullptr;
  float* pin = nullptr;    // inputs of one prediction
  long t = 0;              // Adam step count
};

static long ws_nweights(long N) { return WS_H1 * 3 + WS_H1 + WS_H2 * WS_H1 + WS_H2 + N * WS_H2 + N; }

namespace {
struct WsLayout {
  size_t bytes = 0;
  size_t off(size_t n, size_t align = 256) {
    bytes = (bytes + align - 1) / align * align;
    const size_t o = bytes;
    bytes += n;
    return o;
  }
};
}  // namespace

static pfd_status ws_layout(const pfd_ws_arch* a, WsLayout& L, size_t* offs) {
  if (!a || a->n_out < 16 || a->hidden1 != WS_H1 || a->hidden2 != WS_H2) return PFD_EINVAL;
  const long N = a->n_out, nw = ws_nweights(N), Bp = WS_MAXB;
  const long nparts = (N + WS_CHUNK - 1) / WS_CHUNK;
  const long nblk = (N + 63) / 64;
  size_t i = 0;
  offs[i++] = L.off(4 * nw);            // w
  offs[i++] = L.off(4 * nw);            // g
  offs[i++] = L.off(4 * nw);            // m
  offs[i++] = L.off(4 * nw);            // v
  offs[i++] = L.off(2 * N * WS_H2);     // W3b
  offs[i++] = L.off(4 * Bp * WS_H1);    // a1
  offs[i++] = L.off(4 * Bp * WS_H1);    // h1
  offs[i++] = L.off(4 * Bp * WS_H2);    // a2
  offs[i++] = L.off(4 * Bp * WS_H2);    // h2
  offs[i++] = L.off(2 * Bp * WS_H2);    // h2b
  offs[i++] = L.off(4 * Bp * N);        // y
  offs[i++] = L.off(4 * Bp * N);        // dy
  offs[i++] = L.off(2 * Bp * N);        // dyb
  offs[i++] = L.off(4 * nparts * WS_H2 * Bp);  // part
  offs[i++] = L.off(8 * nblk);          // lpart
  offs[i++] = L.off(8 * 1024);          // wpart
  offs[i++] = L.off(4 * Bp);            // idx
  offs[i++] = L.off(4 * 16);            // pin
  return PFD_OK;
}

extern "C" long pfd_ws_num_weights(const pfd_ws_arch* a) { return a ? ws_nweights(a->n_out) : 0; }

extern "C" pfd_status pfd_ws_workspace_query(const pfd_ws_arch* a, size_t* bytes) {
  WsLayout L;
  size_t offs[32];
  pfd_status s = ws_layout(a, L, offs);
  if (s) return s;
  if (bytes) *bytes = L.bytes + 256;
  return PFD_OK;
}

#define WCHK(x)                                                                \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      ws->err = std::string("HIP error: ") + hipGetErrorString(e_);            \
      return PFD_EHIP;                                                         \
    }                                                                          \
  } while (0)

extern "C" pfd_status pfd_ws_create(const pfd_ws_arch* a, void* dev, size_t bytes, void* stream, pfd_ws** out) {
  if (!out || !dev) return PFD_EINVAL;
  *out = nullptr;
  WsLayout L;
  size_t offs[32];
  pfd_status s = ws_layout(a, L, offs);
  if (s) return s;
  if (bytes < L.bytes || (reinterpret_cast<uintptr_t>(dev) & 255)) return PFD_ENOMEM;
  pfd_ws* ws = new pfd_ws;
  ws->arch = *a;
  ws->stream = (hipStream_t)stream;
  ws->N = a->n_out;
  ws->nw = ws_nweights(ws->N);
  ws->o3 = WS_H1 * 3 + WS_H1 + WS_H2 * WS_H1 + WS_H2;
  ws->nparts = (ws->N + WS_CHUNK - 1) / WS_CHUNK;
  char* base = static_cast<char*>(dev);
  size_t i = 0;
  ws->w = (float*)(base + offs[i++]);
  ws->g = (float*)(base + offs[i++]);
  ws->m = (float*)(base + offs[i++]);
  ws->v = (float*)(base + offs[i++]);
  ws->W3b = (uint16_t*)(base + offs[i++]);
  ws->a1 = (float*)(base + offs[i++]);
  ws->h1 = (float*)(base + offs[i++]);
  ws->a2 = (float*)(base + offs[i++]);
  ws->h2 = (float*)(base + offs[i++]);
  ws->h2b = (uint16_t*)(base + offs[i++]);
  ws->y = (float*)(base + offs[i++]);
  ws->dy = (float*)(base + offs[i++]);
  ws->dyb = (uint16_t*)(base + offs[i++]);
  ws->part = (float*)(base + offs[i++]);
  ws->lpart = (double*)(base + offs[i++]);
  ws->wpart = (double*)(base + offs[i++]);
  ws->idx = (int*)(base + offs[i++]);
  ws->pin = (float*)(base + offs[i++]);
  // initial weights from a seeded generator: N(0, 1/fan_in) for W1, W2; W3 small; biases 0
  std::vector<float> w0(ws->nw, 0.0f);
  std::mt19937_64 rng(a->seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  long o = 0;
  for (long k = 0; k < WS_H1 * 3; ++k) w0[o++] = (float)(nd(rng) / std::sqrt(3.0));
  o += WS_H1;
  for (long k = 0; k < WS_H2 * WS_H1; ++k) w0[o++] = (float)(nd(rng) / std::sqrt((double)WS_H1));
  o += WS_H2;
  for (long k = 0; k < ws->N * WS_H2; ++k) w0[o++] = (float)(0.01 * nd(rng) / std::sqrt((double)WS_H2));
  hipError_t e = hipMemcpyAsync(ws->w, w0.data(), 4 * ws->nw, hipMemcpyHostToDevice, ws->stream);
  if (!e) e = hipMemsetAsync(ws->m, 0, 4 * ws->nw, ws->stream);
  if (!e) e = hipMemsetAsync(ws->v, 0, 4 * ws->nw, ws->stream);
  if (!e) e = hipMemsetAsync(ws->g, 0, 4 * ws->nw, ws->stream);
  if (!e) e = hipStreamSynchronize(ws->stream);
  if (e) {
    delete ws;
    return PFD_EHIP;
  }
  hipLaunchKernelGGL(k_ws_to_bf16, dim3(1024), dim3(256), 0, ws->stream, ws->N * WS_H2, ws->w + ws->o3, ws->W3b);
  *out = ws;
  return PFD_OK;
}

extern "C" void pfd_ws_destroy(pfd_ws* ws) {
  if (!ws) return;
  (void)hipStreamSynchronize(ws->stream);
  delete ws;
}

extern "C" const char* pfd_ws_last_error(const pfd_ws* ws) { return ws ? ws->err.c_str() : ""; }

extern "C" pfd_status pfd_ws_set_weights(pfd_ws* ws, const float* host) {
  if (!ws || !host) return PFD_EINVAL;
  WCHK(hipMemcpyAsync(ws->w, host, 4 * ws->nw, hipMemcpyHostToDevice, ws->stream));
  hipLaunchKernelGGL(k_ws_to_bf16, dim3(1024), dim3(256), 0, ws->stream, ws->N * WS_H2, ws->w + ws->o3, ws->W3b);
  WCHK(hipStreamSynchronize(ws->stream));
  return PFD_OK;
}

extern "C" pfd_status pfd_ws_get_weights(pfd_ws* ws, float* host) {
  if (!ws || !host) return PFD_EINVAL;
  WCHK(hipMemcpyAsync(host, ws->w, 4 * ws->nw, hipMemcpyDeviceToHost, ws->stream));
  WCHK(hipStreamSynchronize(ws->stream));
  return PFD_OK;
}

extern "C" pfd_status pfd_ws_init_output_bias(pfd_ws* ws, const float* targets, long S) {
  if (!ws || !targets || S < 1) return PFD_EINVAL;
  hipLaunchKernelGGL(k_ws_mean, dim3(1024), dim3(256), 0, ws->stream, ws->N, S, targets, ws->w + ws->o3 + ws->N * WS_H2);
  WCHK(hipGetLastError());
  return PFD_OK;
}

// forward + backward on one minibatch: gradients in ws->g, loss to *loss (synchronises)
static pfd_status ws_grad(pfd_ws* ws, const float* P, const float* T, const int* idx_host, int B, double* loss) {
  if (B < 1 || B > WS_MAXB) { ws->err = "batch size must be in [1, 32]"; return PFD_EINVAL; }
  const int Bp = WS_MAXB;   // the K = 32 products need the full padded batch
  WCHK(hipMemcpyAsync(ws->idx, idx_host, sizeof(int) * B, hipMemcpyHostToDevice, ws->stream));
  hipLaunchKernelGGL(k_ws_fwd_small, dim3(Bp), dim3(WS_H2), 0, ws->stream, B, P, ws->idx, ws->w, ws->a1, ws->h1,
                     ws->a2, ws->h2, ws->h2b);
  const long nblk = (ws->N + 63) / 64;
  hipLaunchKernelGGL(k_ws_out, dim3(nblk), dim3(256), 0, ws->stream, ws->N, Bp, B, ws->W3b, ws->h2b,
                     ws->w + ws->o3 + ws->N * WS_H2, T, ws->idx, (float*)nullptr, ws->dy, ws->dyb, ws->lpart);
  hipLaunchKernelGGL(k_ws_bwd_w3, dim3(nblk), dim3(256), 0, ws->stream, ws->N, Bp, ws->dyb, ws->dy, ws->h2b,
                     ws->g + ws->o3, ws->g + ws->o3 + ws->N * WS_H2);
  hipLaunchKernelGGL(k_ws_bwd_h2, dim3(ws->nparts), dim3(256), 0, ws->stream, ws->N, Bp, ws->dyb, ws->W3b, ws->part);
  hipLaunchKernelGGL(k_ws_bwd_small, dim3(1), dim3(256), 0, ws->stream, B, Bp, (int)ws->nparts, ws->part, P, ws->idx,
                     ws->w, ws->a1, ws->h1, ws->a2, ws->g);
  WCHK(hipGetLastError());
  if (loss) {
    std::vector<double> lp(nblk);
    WCHK(hipMemcpyAsync(lp.data(), ws->lpart, 8 * nblk, hipMemcpyDeviceToHost, ws->stream));
    WCHK(hipStreamSynchronize(ws->stream));
    double s = 0.0;
    for (double x : lp) s += x;
    *loss = s / ((double)B * (double)ws->N);
  }
  return PFD_OK;
}

extern "C" pfd_status pfd_ws_gradients(pfd_ws* ws, const float* P, const float* T, const int* idx, int B,
                                       float* grad_host, double* loss) {
  if (!ws || !P || !T || !idx) return PFD_EINVAL;
  pfd_status s = ws_grad(ws, P, T, idx, B, loss);
  if (s) return s;
  if (grad_host) {
    WCHK(hipMemcpyAsync(grad_host, ws->g, 4 * ws->nw, hipMemcpyDeviceToHost, ws->stream));
    WCHK(hipStreamSynchronize(ws->stream));
  }
  return PFD_OK;
}

static pfd_status ws_adam(pfd_ws* ws, float lr) {
  ws->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)ws->t), c2 = 1.0f - std::pow(b2, (float)ws->t);
  hipLaunchKernelGGL(k_ws_adam, dim3(2048), dim3(256), 0, ws->stream, ws->nw, ws->w, ws->g, ws->m, ws->v, lr, b1, b2,
                     c1, c2, 1e-8f, ws->o3, ws->N * WS_H2, ws->W3b);
  WCHK(hipGetLastError());
  return PFD_OK;
}

extern "C" pfd_status pfd_ws_train_step(pfd_ws* ws, const float* P, const float* T, const int* idx, int B, float lr,
                                        double* loss) {
  if (!ws || !P || !T || !idx) return PFD_EINVAL;
  pfd_status s = ws_grad(ws, P, T, idx, B, loss);
  if (s) return s;
  return ws_adam(ws, lr);
}

extern "C" pfd_status pfd_ws_train(pfd_ws* ws, const float* P, const float* T, long S, int steps, int B, float lr,
                                   unsigned long long seed, double* loss_history) {
  if (!ws || !P || !T || S < 1 || steps < 0 || B < 1 || B > WS_MAXB || B > S) return PFD_EINVAL;
  if (S > 0x7fffffffL) return PFD_EINVAL;
  std::mt19937_64 rng(seed);
  std::vector<int> perm(S);
  for (long i = 0; i < S; ++i) perm[i] = (int)i;
  long pos = S;
  std::vector<int> idx(B);
  for (int it = 0; it < steps; ++it) {
    for (int b = 0; b < B; ++b) {
      if (pos >= S) {   // new epoch: reshuffle
        std::shuffle(perm.begin(), perm.end(), rng);
        pos = 0;
      }
      idx[b] = perm[pos++];
    }
    // cosine decay of the step size to 5% over the run
    const float lr_t = lr * (0.05f + 0.95f * 0.5f * (1.0f + std::cos(3.14159265f * (float)it / (float)steps)));
    double l = 0.0;
    pfd_status s = ws_grad(ws, P, T, idx.data(), B, loss_history ? &l : nullptr);
    if (s) return s;
    if (loss_history) loss_history[it] = l;
    s = ws_adam(ws, lr_t);
    if (s) return s;
  }
  WCHK(hipStreamSynchronize(ws->stream));
  return PFD_OK;
}

extern "C" pfd_status pfd_ws_predict(pfd_ws* ws, const float* p_host, const double* weights, double mass,
                                     double* out) {
  if (!ws || !p_host || !out) return PFD_EINVAL;
  const int zero = 0;
  WCHK(hipMemcpyAsync(ws->idx, &zero, sizeof(int), hipMemcpyHostToDevice, ws->stream));
  WCHK(hipMemcpyAsync(ws->pin, p_host, 3 * sizeof(float), hipMemcpyHostToDevice, ws->stream));
  hipLaunchKernelGGL(k_ws_fwd_small, dim3(WS_MAXB), dim3(WS_H2), 0, ws->stream, 1, (const float*)ws->pin, ws->idx,
                     ws->w, ws->a1, ws->h1, ws->a2, ws->h2, ws->h2b);
  const long nblk = (ws->N + 63) / 64;
  hipLaunchKernelGGL(k_ws_out, dim3(nblk), dim3(256), 0, ws->stream, ws->N, WS_MAXB, 1, ws->W3b, ws->h2b,
                     ws->w + ws->o3 + ws->N * WS_H2, (const float*)nullptr, ws->idx, ws->y, (float*)nullptr,
                     (uint16_t*)nullptr, (double*)nullptr);
  double c = 0.0;
  if (weights) {   // mass projection: shift so that sum(weights * out) = mass
    const int nb = 512;
    hipLaunchKernelGGL(k_ws_wsum, dim3(nb), dim3(256), 0, ws->stream, ws->N, ws->y, weights, ws->wpart);
    std::vector<double> h(2 * nb);
    WCHK(hipMemcpyAsync(h.data(), ws->wpart, 16 * nb, hipMemcpyDeviceToHost, ws->stream));
    WCHK(hipStreamSynchronize(ws->stream));
    double s = 0.0, sw = 0.0;
    for (int i = 0; i < nb; ++i) {
      s += h[2 * i];
      sw += h[2 * i + 1];
    }
    c = (mass - s) / sw;
  }
  hipLaunchKernelGGL(k_ws_shift, dim3(1024), dim3(256), 0, ws->stream, ws->N, ws->y, c, out);
  WCHK(hipGetLastError());
  WCHK(hipStreamSynchronize(ws->stream));
  return PFD_OK;
}
