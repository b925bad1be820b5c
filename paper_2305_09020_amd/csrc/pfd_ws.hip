// Learned warm start: a small network trained on equilibria the method itself computes maps
// (voltage, permittivity ratio, contact angle) to the equilibrium phase field, used as the
// starting state of the equilibrium march (the march to the residual tolerance still decides
// the result).  The network is a convolutional decoder onto the field's grid (nz x ny x nx values,
// z slowest):
//
//   a1 = W1 p + b1, h1 = gelu(a1)                      64 units   (FP32)
//   a2 = W2 h1 + b2, h2 = gelu(a2)                     128 units  (FP32)
//   x0 = W3 h2 + b3                                    16-channel latent grid Z0 x Y0 x X0
//   a_s = conv(up(x_{s-1}); K_s) + c_s, x_s = gelu(a_s)   s = 1, 2, 3: each axis doubled
//                                                      (nearest neighbour), 3x3x3 kernel
//   y = crop(sum_c wo[c] x_3[., c]) + bo               the corner nz x ny x nx
//   loss = mean over batch and outputs of (y - t)^2
//
// Z0 = ceil(nz / 8) and likewise Y0, X0.  A convolution neighbour outside the grid wraps
// around along an axis that is periodic with 8 Z0 = nz exactly and is zero along any other.
// The latent layer, the three convolutions and all their backward products run on the matrix
// cores with BF16 operands and FP32 accumulation (a convolution as an implicit GEMM: 16
// voxels x 16 channels per wave, the contraction over 27 taps x 16 channels in 14 steps of
// 32); the small layers, the 1x1 head, the reductions and Adam run in FP32 on the vector
// units; FP32 master weights.
//
// Layouts: activations channel-last [b][z][y][x][c]; weights in one FP32 blob [W1 (64x3) | b1
// | W2 (128x64) | b2 | W3 (L0x128) | b3 (L0) | K1 (27x16x16: tap, out, in) | c1 | K2 | c2 | K3
// | c3 | wo (16) | bo (nz ny nx)], L0 = 16 Z0 Y0 X0; gradients and Adam moments likewise.
// BF16 copies: W3 (row contiguous), each K as [28 taps][out][in] (tap 27 zero) and its
// flipped transpose [28][in][out] for the input-gradient convolution.
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
#define WS_C 16           // channels of the latent grid and of every convolution
#define WS_CHUNK 1024     // latent rows per work-group in the dL/dh2 product
#define WS_KLEN (27 * WS_C * WS_C + WS_C)   // one convolution's weights and bias
#define WS_WG_BLOCKS 256  // work-groups of the weight-gradient products (4 partials each)

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
// 16x16x32 fragments: lane l supplies A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16],
// e = 0..7; accumulator element j of lane l holds D[4 (l / 16) + j][l % 16]

// grid of one convolution: output dims, whether the input is the half-size grid doubled by
// nearest neighbour, and which axes wrap
struct ConvGeom {
  int Zo, Yo, Xo, up, wz, wy, wx;
};

// neighbour of (z, y, x) at tap t in the output grid, as an input-grid voxel index, or -1
__device__ __forceinline__ int nbr(const ConvGeom& g, int z, int y, int x, int t) {
  int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
  if (zz < 0 || zz >= g.Zo) {
    if (!g.wz) return -1;
    zz = zz < 0 ? zz + g.Zo : zz - g.Zo;
  }
  if (yy < 0 || yy >= g.Yo) {
    if (!g.wy) return -1;
    yy = yy < 0 ? yy + g.Yo : yy - g.Yo;
  }
  if (xx < 0 || xx >= g.Xo) {
    if (!g.wx) return -1;
    xx = xx < 0 ? xx + g.Xo : xx - g.Xo;
  }
  if (g.up) return ((zz >> 1) * (g.Yo >> 1) + (yy >> 1)) * (g.Xo >> 1) + (xx >> 1);
  return (zz * g.Yo + yy) * g.Xo + xx;
}

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

// ---- latent layer x0 = W3 h2 + b3 on the matrix cores, stored as BF16 [b][n] for the first
// convolution.  A wave computes 16 latent rows for every (padded) sample: K = H2 in four steps.
__global__ void __launch_bounds__(256) k_ws_lat(long N, int B, const uint16_t* __restrict__ W3b,
                                                const uint16_t* __restrict__ h2b, const float* __restrict__ b3,
                                                uint16_t* __restrict__ xb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r16 = lane & 15, g = lane >> 4;
  const long n0 = ((long)blockIdx.x * 4 + w) * 16;
  if (n0 >= N) return;
  f32x4 acc[WS_MAXB / 16];
  for (int i = 0; i < WS_MAXB / 16; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  const long na = n0 + r16 < N ? n0 + r16 : N - 1;     // clamped row (rows >= N never stored)
  const int nbt = (B + 15) / 16;
#pragma unroll
  for (int kk = 0; kk < WS_H2 / 32; ++kk) {
    const bf16x8 a = ld8(W3b + na * WS_H2 + 32 * kk + 8 * g);
    for (int bt = 0; bt < nbt; ++bt) {
      const bf16x8 bv = ld8(h2b + (16 * bt + r16) * WS_H2 + 32 * kk + 8 * g);
      acc[bt] = mma(a, bv, acc[bt]);
    }
  }
  for (int bt = 0; bt < nbt; ++bt) {
    const int b = 16 * bt + r16;
    if (b >= B) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long n = n0 + 4 * g + j;
      if (n < N) xb[(long)b * N + n] = to_bf16(acc[bt][j] + b3[n]);
    }
  }
}

// ---- 3x3x3 convolution, 16 -> 16 channels, as an implicit GEMM on the matrix cores: a wave
// owns 16 consecutive output voxels (flattened over the batch) x 16 output channels; step k of
// the contraction covers taps 2k and 2k+1 (tap 27 is zero) x 16 input channels.
// GRADIN = false: out = conv(in; w) + bias, stores the FP32 pre-activation and BF16 gelu of it.
// GRADIN = true: w is the flipped transpose and in holds dL/da; stores the FP32 sum only.
template <bool GRADIN>
__global__ void __launch_bounds__(256) k_ws_conv(int B, ConvGeom g, const uint16_t* __restrict__ in,
                                                 const uint16_t* __restrict__ w, const float* __restrict__ bias,
                                                 float* __restrict__ outf, uint16_t* __restrict__ outb) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r16 = lane & 15, grp = lane >> 4;
  const int V = g.Zo * g.Yo * g.Xo;
  const int Vi = g.up ? V >> 3 : V;
  const int tot = B * V;
  const int v0 = (blockIdx.x * 4 + wv) * 16;
  if (v0 >= tot) return;
  const int v = v0 + r16 < tot ? v0 + r16 : tot - 1;
  const int b = v / V;
  int r = v - b * V;
  const int z = r / (g.Yo * g.Xo);
  r -= z * g.Yo * g.Xo;
  const int y = r / g.Xo, x = r - y * g.Xo;
  const uint16_t* inb = in + (long)b * Vi * WS_C + (grp & 1) * 8;
  f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int k = 0; k < 14; ++k) {
    const int t = 2 * k + (grp >> 1);
    bf16x8 a = bf16x8{};
    if (t < 27) {
      const int q = nbr(g, z, y, x, t);
      if (q >= 0) a = ld8(inb + (long)q * WS_C);
    }
    const bf16x8 bw = ld8(w + (t * WS_C + r16) * WS_C + (grp & 1) * 8);
    acc = mma(a, bw, acc);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int vv = v0 + 4 * grp + j;
    if (vv >= tot) continue;
    const long o = (long)vv * WS_C + r16;
    if (GRADIN) {
      outf[o] = acc[j];
    } else {
      const float a = acc[j] + bias[r16];
      outf[o] = a;
      outb[o] = to_bf16(gelu(a));
    }
  }
}

// ---- weight gradient of a convolution: dK[t][co][ci] = sum over batch and voxels p of
// da[p][co] u[nbr(p, t)][ci] (u = the layer input, doubled if g.up), dc[co] = sum da[p][co].
// Contraction over voxels on the matrix cores (A = da^T, B = shifted u), 32 voxels per step;
// each wave keeps all 27 taps' 16x16 blocks and writes one partial of WS_KLEN floats.
__global__ void __launch_bounds__(256) k_ws_wgrad(int B, ConvGeom g, const uint16_t* __restrict__ da,
                                                  const uint16_t* __restrict__ in, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, r16 = lane & 15, grp = lane >> 4;
  const int V = g.Zo * g.Yo * g.Xo;
  const int Vi = g.up ? V >> 3 : V;
  const int tot = B * V;
  const int per = ((tot + gridDim.x - 1) / gridDim.x + 127) / 128 * 128;
  const int s0 = blockIdx.x * per;
  const int s1 = min(tot, s0 + per);
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;
  for (int c0 = s0 + 32 * wv; c0 < s1; c0 += 128) {
    bf16x8 a;
    int zs[8], ys[8], xs[8], bo[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int v = c0 + 8 * grp + e;
      const bool ok = v < s1;
      const uint16_t dv = ok ? da[(long)v * WS_C + r16] : (uint16_t)0;
      a[e] = __builtin_bit_cast(__bf16, dv);
      bsum += from_bf16(dv);
      const int vc = ok ? v : s0;
      const int b = vc / V;
      int r = vc - b * V;
      zs[e] = r / (g.Yo * g.Xo);
      r -= zs[e] * g.Yo * g.Xo;
      ys[e] = r / g.Xo;
      xs[e] = r - ys[e] * g.Xo;
      bo[e] = ok ? b * Vi : -1;
    }
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      bf16x8 bv;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int q = bo[e] >= 0 ? nbr(g, zs[e], ys[e], xs[e], t) : -1;
        const uint16_t u = q >= 0 ? in[(long)(bo[e] + q) * WS_C + r16] : (uint16_t)0;
        bv[e] = __builtin_bit_cast(__bf16, u);
      }
      acc[t] = mma(a, bv, acc[t]);
    }
  }
  float* out = part + (long)(blockIdx.x * 4 + wv) * WS_KLEN;
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) out[(t * WS_C + 4 * grp + j) * WS_C + r16] = acc[t][j];
  bsum += __shfl_xor(bsum, 16);
  bsum += __shfl_xor(bsum, 32);
  if (lane < 16) out[27 * WS_C * WS_C + r16] = bsum;
}

// out[i] = sum over q of part[q * len + i], in a fixed order
__global__ void k_ws_reduce(int nparts, int len, const float* __restrict__ part, float* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int q = 0; q < nparts; ++q) s += part[(long)q * len + i];
    out[i] = s;
  }
}

// ---- backward of the doubling: each coarse value sums its eight children in du (FP32);
// then dL/da = that * gelu'(a) as BF16 for a convolution layer, or, for the latent grid,
// dL/dx0 as FP32 and BF16 in row-major [n][Bp] for the latent layer's backward products
// (padded samples b >= B are written as zeros).
template <bool LAT>
__global__ void k_ws_down(int B, int Bp, int Zc, int Yc, int Xc, const float* __restrict__ du,
                          const float* __restrict__ a, uint16_t* __restrict__ da, float* __restrict__ dyl,
                          uint16_t* __restrict__ dybl) {
  const int Vc = Zc * Yc * Xc, Vf = Vc * 8;
  const int nb = LAT ? Bp : B;
  const long tot = (long)nb * Vc * WS_C;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % WS_C);
    const long vb = i / WS_C;
    int b, v;
    if (LAT) {   // thread order [n][b] so that the row-major stores are contiguous
      b = (int)(i % nb);
      const long n = i / nb;
      v = (int)(n / WS_C);
      const int cc = (int)(n % WS_C);
      float s = 0.0f;
      if (b < B) {
        const int z = v / (Yc * Xc), y = (v / Xc) % Yc, x = v % Xc;
        for (int dz = 0; dz < 2; ++dz)
          for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
              const int f = ((2 * z + dz) * (2 * Yc) + 2 * y + dy) * (2 * Xc) + 2 * x + dx;
              s += du[((long)b * Vf + f) * WS_C + cc];
            }
      }
      dyl[n * Bp + b] = s;
      dybl[n * Bp + b] = to_bf16(s);
    } else {
      b = (int)(vb / Vc);
      v = (int)(vb - (long)b * Vc);
      const int z = v / (Yc * Xc), y = (v / Xc) % Yc, x = v % Xc;
      float s = 0.0f;
      for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            const int f = ((2 * z + dz) * (2 * Yc) + 2 * y + dy) * (2 * Xc) + 2 * x + dx;
            s += du[((long)b * Vf + f) * WS_C + c];
          }
      da[i] = to_bf16(s * dgelu(a[i]));
    }
  }
}

// ---- output head, one thread per voxel of the last grid: y = sum_c wo[c] x3[c] + bo inside
// the nz x ny x nx corner.  With targets: the loss partials, dL/dy = 2 (y - t) / (B N),
// dL/dbo, dL/dwo partials, and dL/da3 = dL/dy wo gelu'(a3) as BF16 (zero outside the corner).
__global__ void __launch_bounds__(256) k_ws_head(int B, int nz, int ny, int nx, int Z3, int Y3, int X3,
                                                 const uint16_t* __restrict__ x3, const float* __restrict__ wo,
                                                 const float* __restrict__ bo, const float* __restrict__ T,
                                                 const int* __restrict__ idx, float* __restrict__ y,
                                                 const float* __restrict__ a3, uint16_t* __restrict__ da3,
                                                 float* __restrict__ gbo, float* __restrict__ gwo_part,
                                                 double* __restrict__ lpart) {
  __shared__ float red[WS_C][256];
  __shared__ double lred[256];
  const int V = Z3 * Y3 * X3;
  const long N = (long)nz * ny * nx;
  const int v = blockIdx.x * 256 + threadIdx.x;
  float gw[WS_C];
#pragma unroll
  for (int c = 0; c < WS_C; ++c) gw[c] = 0.0f;
  double ls = 0.0;
  if (v < V) {
    const int z = v / (Y3 * X3), yy = (v / X3) % Y3, x = v % X3;
    const bool in = z < nz && yy < ny && x < nx;
    const long n = ((long)z * ny + yy) * nx + x;
    float gb = 0.0f;
    for (int b = 0; b < B; ++b) {
      const long o = ((long)b * V + v) * WS_C;
      if (!in) {
        if (da3)
          for (int c = 0; c < WS_C; ++c) da3[o + c] = 0;
        continue;
      }
      float xv[WS_C];
      float s = bo[n];
#pragma unroll
      for (int c = 0; c < WS_C; ++c) {
        xv[c] = from_bf16(x3[o + c]);
        s += wo[c] * xv[c];
      }
      if (y) y[(long)b * N + n] = s;
      if (T) {
        const float d = s - T[(long)(idx ? idx[b] : b) * N + n];
        ls += (double)d * d;
        const float dy = 2.0f * d / ((float)B * (float)N);
        gb += dy;
#pragma unroll
        for (int c = 0; c < WS_C; ++c) {
          gw[c] += dy * xv[c];
          da3[o + c] = to_bf16(dy * wo[c] * dgelu(a3[o + c]));
        }
      }
    }
    if (T && in) gbo[n] = gb;
  }
  if (!T) return;
#pragma unroll
  for (int c = 0; c < WS_C; ++c) red[c][threadIdx.x] = gw[c];
  lred[threadIdx.x] = ls;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
#pragma unroll
      for (int c = 0; c < WS_C; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
      lred[threadIdx.x] += lred[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x < WS_C) gwo_part[blockIdx.x * WS_C + threadIdx.x] = red[threadIdx.x][0];
  if (threadIdx.x == 0) lpart[blockIdx.x] = lred[0];
}

// ---- dL/dW3 = dy^T h2 (K = batch) and dL/db3 = sum_b dy; a wave owns 16 latent rows
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

// ---- dL/dh2 = dy W3 over all latent rows: each work-group sums WS_CHUNK rows (its four waves
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

// BF16 copies of the three convolutions' weights: Kb[s][t][co][ci] and the flipped transpose
// Ktb[s][t][ci][co] = K_s[26 - t][co][ci]; tap 27 is zero in both
__global__ void k_ws_convw(const float* __restrict__ K1, uint16_t* __restrict__ Kb, uint16_t* __restrict__ Ktb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * 28 * WS_C * WS_C) return;
  const int s = i / (28 * WS_C * WS_C);
  const int r = i - s * 28 * WS_C * WS_C;
  const int t = r / (WS_C * WS_C), a = (r / WS_C) % WS_C, c = r % WS_C;
  const float* K = K1 + (long)s * WS_KLEN;
  Kb[i] = t < 27 ? to_bf16(K[(t * WS_C + a) * WS_C + c]) : (uint16_t)0;
  Ktb[i] = t < 27 ? to_bf16(K[((26 - t) * WS_C + c) * WS_C + a]) : (uint16_t)0;
}

__global__ void k_ws_to_bf16(long n, const float* __restrict__ a, uint16_t* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = to_bf16(a[i]);
}

// bo = mean of the training targets over the samples
__global__ void k_ws_mean(long N, long S, const float* __restrict__ T, float* __restrict__ bo) {
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (long q = 0; q < S; ++q) s += T[q * N + n];
    bo[n] = (float)(s / (double)S);
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
  int lat[3] = {0, 0, 0};     // latent grid Z0, Y0, X0
  int wrap[3] = {0, 0, 0};
  long N = 0, L0 = 0, nw = 0, nparts = 0, nhead = 0;
  long oW3 = 0, ob3 = 0, oK = 0, owo = 0, obo = 0;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  uint16_t *W3b = nullptr, *Kb = nullptr, *Ktb = nullptr;
  float *a1 = nullptr, *h1 = nullptr, *a2 = nullptr, *h2 = nullptr;
  uint16_t* h2b = nullptr;
  uint16_t* x0b = nullptr;              // latent [Bp][L0]
  float* a[3] = {nullptr, nullptr, nullptr};      // pre-activations of the three stages
  uint16_t* xb[3] = {nullptr, nullptr, nullptr};  // their gelu, BF16
  uint16_t* da[3] = {nullptr, nullptr, nullptr};  // dL/da, BF16
  float* du = nullptr;                  // input gradient of a convolution (largest stage)
  float* y = nullptr;                   // one prediction [N]
  float* dyl = nullptr;                 // dL/dx0 [L0][Bp]
  uint16_t* dybl = nullptr;
  float* part = nullptr;                // dL/dh2 partials
  float* wgp = nullptr;                 // weight-gradient partials
  float* hpart = nullptr;               // head dL/dwo partials
  double* lpart = nullptr;              // loss partials
  double* wpart = nullptr;              // weighted-sum partials
  int* idx = nullptr;
  float* pin = nullptr;                 // inputs of one prediction
  long t = 0;                           // Adam step count

  int dim(int s, int ax) const { return lat[ax] << s; }
  long vox(int s) const { return (long)dim(s, 0) * dim(s, 1) * dim(s, 2); }
};

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

struct WsDims {
  long N, L0, nw, V[4], nparts, nhead;
  int lat[3], wrap[3];
};

bool ws_dims(const pfd_ws_arch* a, WsDims& d) {
  if (!a || a->hidden1 != WS_H1 || a->hidden2 != WS_H2 || a->channels != WS_C) return false;
  if (a->nz < 1 || a->ny < 1 || a->nx < 1) return false;
  const int n[3] = {a->nz, a->ny, a->nx};
  const int per[3] = {a->periodic_z, a->periodic_y, a->periodic_x};
  for (int i = 0; i < 3; ++i) {
    if (n[i] > 4096) return false;
    d.lat[i] = (n[i] + 7) / 8;
    d.wrap[i] = per[i] && 8 * d.lat[i] == n[i];
  }
  d.N = (long)a->nz * a->ny * a->nx;
  if (d.N < 16) return false;
  d.V[0] = (long)d.lat[0] * d.lat[1] * d.lat[2];
  for (int s = 1; s <= 3; ++s) d.V[s] = d.V[0] << (3 * s);
  if ((long)WS_MAXB * d.V[3] * WS_C >= (1L << 31)) return false;   // kernels index voxels in 32 bits
  d.L0 = WS_C * d.V[0];
  d.nw = WS_H1 * 3 + WS_H1 + WS_H2 * WS_H1 + WS_H2 + d.L0 * WS_H2 + d.L0 + 3L * WS_KLEN + WS_C + d.N;
  d.nparts = (d.L0 + WS_CHUNK - 1) / WS_CHUNK;
  d.nhead = (d.V[3] + 255) / 256;
  return true;
}

pfd_status ws_layout(const pfd_ws_arch* a, WsLayout& L, size_t* offs, WsDims& d) {
  if (!ws_dims(a, d)) return PFD_EINVAL;
  const long Bp = WS_MAXB, nw = d.nw;
  size_t i = 0;
  offs[i++] = L.off(4 * nw);                    // w
  offs[i++] = L.off(4 * nw);                    // g
  offs[i++] = L.off(4 * nw);                    // m
  offs[i++] = L.off(4 * nw);                    // v
  offs[i++] = L.off(2 * d.L0 * WS_H2);          // W3b
  offs[i++] = L.off(2 * 3 * 28 * WS_C * WS_C);  // Kb
  offs[i++] = L.off(2 * 3 * 28 * WS_C * WS_C);  // Ktb
  offs[i++] = L.off(4 * Bp * WS_H1);            // a1
  offs[i++] = L.off(4 * Bp * WS_H1);            // h1
  offs[i++] = L.off(4 * Bp * WS_H2);            // a2
  offs[i++] = L.off(4 * Bp * WS_H2);            // h2
  offs[i++] = L.off(2 * Bp * WS_H2);            // h2b
  offs[i++] = L.off(2 * Bp * d.L0);             // x0b
  for (int s = 1; s <= 3; ++s) {
    offs[i++] = L.off(4 * Bp * d.V[s] * WS_C);  // a_s
    offs[i++] = L.off(2 * Bp * d.V[s] * WS_C);  // x_s
    offs[i++] = L.off(2 * Bp * d.V[s] * WS_C);  // da_s
  }
  offs[i++] = L.off(4 * Bp * d.V[3] * WS_C);    // du
  offs[i++] = L.off(4 * d.N);                   // y
  offs[i++] = L.off(4 * d.L0 * Bp);             // dyl
  offs[i++] = L.off(2 * d.L0 * Bp);             // dybl
  offs[i++] = L.off(4 * d.nparts * WS_H2 * Bp); // part
  offs[i++] = L.off(4L * 4 * WS_WG_BLOCKS * WS_KLEN);  // wgp
  offs[i++] = L.off(4 * d.nhead * WS_C);        // hpart
  offs[i++] = L.off(8 * d.nhead);               // lpart
  offs[i++] = L.off(8 * 1024);                  // wpart
  offs[i++] = L.off(4 * Bp);                    // idx
  offs[i++] = L.off(4 * 16);                    // pin
  return PFD_OK;
}
}  // namespace

extern "C" long pfd_ws_num_weights(const pfd_ws_arch* a) {
  WsDims d;
  return ws_dims(a, d) ? d.nw : 0;
}

extern "C" pfd_status pfd_ws_workspace_query(const pfd_ws_arch* a, size_t* bytes) {
  WsLayout L;
  WsDims d;
  size_t offs[48];
  pfd_status s = ws_layout(a, L, offs, d);
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

static void ws_refresh_bf16(pfd_ws* ws) {
  hipLaunchKernelGGL(k_ws_to_bf16, dim3(1024), dim3(256), 0, ws->stream, ws->L0 * WS_H2, ws->w + ws->oW3, ws->W3b);
  hipLaunchKernelGGL(k_ws_convw, dim3((3 * 28 * WS_C * WS_C + 255) / 256), dim3(256), 0, ws->stream,
                     (const float*)(ws->w + ws->oK), ws->Kb, ws->Ktb);
}

extern "C" pfd_status pfd_ws_create(const pfd_ws_arch* a, void* dev, size_t bytes, void* stream, pfd_ws** out) {
  if (!out || !dev) return PFD_EINVAL;
  *out = nullptr;
  WsLayout L;
  WsDims d;
  size_t offs[48];
  pfd_status s = ws_layout(a, L, offs, d);
  if (s) return s;
  if (bytes < L.bytes || (reinterpret_cast<uintptr_t>(dev) & 255)) return PFD_ENOMEM;
  pfd_ws* ws = new pfd_ws;
  ws->arch = *a;
  ws->stream = (hipStream_t)stream;
  for (int i = 0; i < 3; ++i) {
    ws->lat[i] = d.lat[i];
    ws->wrap[i] = d.wrap[i];
  }
  ws->N = d.N;
  ws->L0 = d.L0;
  ws->nw = d.nw;
  ws->nparts = d.nparts;
  ws->nhead = d.nhead;
  ws->oW3 = WS_H1 * 3 + WS_H1 + WS_H2 * WS_H1 + WS_H2;
  ws->ob3 = ws->oW3 + ws->L0 * WS_H2;
  ws->oK = ws->ob3 + ws->L0;
  ws->owo = ws->oK + 3L * WS_KLEN;
  ws->obo = ws->owo + WS_C;
  char* base = static_cast<char*>(dev);
  size_t i = 0;
  ws->w = (float*)(base + offs[i++]);
  ws->g = (float*)(base + offs[i++]);
  ws->m = (float*)(base + offs[i++]);
  ws->v = (float*)(base + offs[i++]);
  ws->W3b = (uint16_t*)(base + offs[i++]);
  ws->Kb = (uint16_t*)(base + offs[i++]);
  ws->Ktb = (uint16_t*)(base + offs[i++]);
  ws->a1 = (float*)(base + offs[i++]);
  ws->h1 = (float*)(base + offs[i++]);
  ws->a2 = (float*)(base + offs[i++]);
  ws->h2 = (float*)(base + offs[i++]);
  ws->h2b = (uint16_t*)(base + offs[i++]);
  ws->x0b = (uint16_t*)(base + offs[i++]);
  for (int st = 0; st < 3; ++st) {
    ws->a[st] = (float*)(base + offs[i++]);
    ws->xb[st] = (uint16_t*)(base + offs[i++]);
    ws->da[st] = (uint16_t*)(base + offs[i++]);
  }
  ws->du = (float*)(base + offs[i++]);
  ws->y = (float*)(base + offs[i++]);
  ws->dyl = (float*)(base + offs[i++]);
  ws->dybl = (uint16_t*)(base + offs[i++]);
  ws->part = (float*)(base + offs[i++]);
  ws->wgp = (float*)(base + offs[i++]);
  ws->hpart = (float*)(base + offs[i++]);
  ws->lpart = (double*)(base + offs[i++]);
  ws->wpart = (double*)(base + offs[i++]);
  ws->idx = (int*)(base + offs[i++]);
  ws->pin = (float*)(base + offs[i++]);
  // initial weights from a seeded generator: N(0, 1/fan_in) for W1, W2, W3 and the
  // convolutions (fan-in 27 x 16, times 2 for the gelu), wo small, biases 0
  std::vector<float> w0(ws->nw, 0.0f);
  std::mt19937_64 rng(a->seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  long o = 0;
  for (long k = 0; k < WS_H1 * 3; ++k) w0[o++] = (float)(nd(rng) / std::sqrt(3.0));
  o += WS_H1;
  for (long k = 0; k < WS_H2 * WS_H1; ++k) w0[o++] = (float)(nd(rng) / std::sqrt((double)WS_H1));
  o += WS_H2;
  for (long k = 0; k < ws->L0 * WS_H2; ++k) w0[o++] = (float)(nd(rng) / std::sqrt((double)WS_H2));
  o += ws->L0;
  for (int st = 0; st < 3; ++st) {
    for (long k = 0; k < 27 * WS_C * WS_C; ++k) w0[o++] = (float)(nd(rng) * std::sqrt(2.0 / (27.0 * WS_C)));
    o += WS_C;
  }
  for (int c = 0; c < WS_C; ++c) w0[o++] = (float)(0.01 * nd(rng));
  hipError_t e = hipMemcpyAsync(ws->w, w0.data(), 4 * ws->nw, hipMemcpyHostToDevice, ws->stream);
  if (!e) e = hipMemsetAsync(ws->m, 0, 4 * ws->nw, ws->stream);
  if (!e) e = hipMemsetAsync(ws->v, 0, 4 * ws->nw, ws->stream);
  if (!e) e = hipMemsetAsync(ws->g, 0, 4 * ws->nw, ws->stream);
  if (!e) e = hipStreamSynchronize(ws->stream);
  if (e) {
    delete ws;
    return PFD_EHIP;
  }
  ws_refresh_bf16(ws);
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
  ws_refresh_bf16(ws);
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
  hipLaunchKernelGGL(k_ws_mean, dim3(1024), dim3(256), 0, ws->stream, ws->N, S, targets, ws->w + ws->obo);
  WCHK(hipGetLastError());
  return PFD_OK;
}

static ConvGeom ws_geom(const pfd_ws* ws, int s, int up) {
  return ConvGeom{ws->dim(s, 0), ws->dim(s, 1), ws->dim(s, 2), up, ws->wrap[0], ws->wrap[1], ws->wrap[2]};
}

// forward pass of B samples (hidden layers, latent, three convolutions); inputs P[idx[b]]
static void ws_forward(pfd_ws* ws, const float* P, const int* idx_dev, int B) {
  hipLaunchKernelGGL(k_ws_fwd_small, dim3(WS_MAXB), dim3(WS_H2), 0, ws->stream, B, P, idx_dev, ws->w, ws->a1,
                     ws->h1, ws->a2, ws->h2, ws->h2b);
  hipLaunchKernelGGL(k_ws_lat, dim3((ws->L0 + 63) / 64), dim3(256), 0, ws->stream, ws->L0, B, ws->W3b, ws->h2b,
                     ws->w + ws->ob3, ws->x0b);
  for (int s = 1; s <= 3; ++s) {
    const long tot = (long)B * ws->vox(s);
    const uint16_t* in = s == 1 ? ws->x0b : ws->xb[s - 2];
    hipLaunchKernelGGL(k_ws_conv<false>, dim3((unsigned)((tot + 63) / 64)), dim3(256), 0, ws->stream, B,
                       ws_geom(ws, s, 1), in, ws->Kb + (s - 1) * 28 * WS_C * WS_C,
                       (const float*)(ws->w + ws->oK + (s - 1) * WS_KLEN + 27 * WS_C * WS_C), ws->a[s - 1],
                       ws->xb[s - 1]);
  }
}

// forward + backward on one minibatch: gradients in ws->g, loss to *loss (synchronises)
static pfd_status ws_grad(pfd_ws* ws, const float* P, const float* T, const int* idx_host, int B, double* loss) {
  if (B < 1 || B > WS_MAXB) { ws->err = "batch size must be in [1, 32]"; return PFD_EINVAL; }
  const int Bp = WS_MAXB;   // the K = 32 latent products need the full padded batch
  WCHK(hipMemcpyAsync(ws->idx, idx_host, sizeof(int) * B, hipMemcpyHostToDevice, ws->stream));
  ws_forward(ws, P, ws->idx, B);
  hipLaunchKernelGGL(k_ws_head, dim3((unsigned)ws->nhead), dim3(256), 0, ws->stream, B, ws->arch.nz, ws->arch.ny,
                     ws->arch.nx, ws->dim(3, 0), ws->dim(3, 1), ws->dim(3, 2), (const uint16_t*)ws->xb[2],
                     (const float*)(ws->w + ws->owo), (const float*)(ws->w + ws->obo), T, (const int*)ws->idx,
                     (float*)nullptr, (const float*)ws->a[2], ws->da[2], ws->g + ws->obo, ws->hpart, ws->lpart);
  hipLaunchKernelGGL(k_ws_reduce, dim3(1), dim3(64), 0, ws->stream, (int)ws->nhead, WS_C, (const float*)ws->hpart,
                     ws->g + ws->owo);
  for (int s = 3; s >= 1; --s) {
    const ConvGeom gf = ws_geom(ws, s, 1);
    const uint16_t* in = s == 1 ? ws->x0b : ws->xb[s - 2];
    const long tot = (long)B * ws->vox(s);
    const int nblk = (int)std::max(1L, std::min((long)WS_WG_BLOCKS, (tot + 511) / 512));
    hipLaunchKernelGGL(k_ws_wgrad, dim3(nblk), dim3(256), 0, ws->stream, B, gf, (const uint16_t*)ws->da[s - 1], in,
                       ws->wgp);
    hipLaunchKernelGGL(k_ws_reduce, dim3((WS_KLEN + 255) / 256), dim3(256), 0, ws->stream, 4 * nblk, WS_KLEN,
                       (const float*)ws->wgp, ws->g + ws->oK + (s - 1) * WS_KLEN);
    const ConvGeom gt = ws_geom(ws, s, 0);
    hipLaunchKernelGGL(k_ws_conv<true>, dim3((unsigned)((tot + 63) / 64)), dim3(256), 0, ws->stream, B, gt,
                       (const uint16_t*)ws->da[s - 1], (const uint16_t*)(ws->Ktb + (s - 1) * 28 * WS_C * WS_C),
                       (const float*)nullptr, ws->du, (uint16_t*)nullptr);
    const int Zc = ws->dim(s - 1, 0), Yc = ws->dim(s - 1, 1), Xc = ws->dim(s - 1, 2);
    if (s > 1)
      hipLaunchKernelGGL(k_ws_down<false>, dim3(2048), dim3(256), 0, ws->stream, B, Bp, Zc, Yc, Xc,
                         (const float*)ws->du, (const float*)ws->a[s - 2], ws->da[s - 2], (float*)nullptr,
                         (uint16_t*)nullptr);
    else
      hipLaunchKernelGGL(k_ws_down<true>, dim3(2048), dim3(256), 0, ws->stream, B, Bp, Zc, Yc, Xc,
                         (const float*)ws->du, (const float*)nullptr, (uint16_t*)nullptr, ws->dyl, ws->dybl);
  }
  const long nblk = (ws->L0 + 63) / 64;
  hipLaunchKernelGGL(k_ws_bwd_w3, dim3((unsigned)nblk), dim3(256), 0, ws->stream, ws->L0, Bp,
                     (const uint16_t*)ws->dybl, (const float*)ws->dyl, (const uint16_t*)ws->h2b, ws->g + ws->oW3,
                     ws->g + ws->ob3);
  hipLaunchKernelGGL(k_ws_bwd_h2, dim3((unsigned)ws->nparts), dim3(256), 0, ws->stream, ws->L0, Bp,
                     (const uint16_t*)ws->dybl, (const uint16_t*)ws->W3b, ws->part);
  hipLaunchKernelGGL(k_ws_bwd_small, dim3(1), dim3(256), 0, ws->stream, B, Bp, (int)ws->nparts,
                     (const float*)ws->part, P, (const int*)ws->idx, (const float*)ws->w, (const float*)ws->a1,
                     (const float*)ws->h1, (const float*)ws->a2, ws->g);
  WCHK(hipGetLastError());
  if (loss) {
    std::vector<double> lp(ws->nhead);
    WCHK(hipMemcpyAsync(lp.data(), ws->lpart, 8 * ws->nhead, hipMemcpyDeviceToHost, ws->stream));
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
                     c1, c2, 1e-8f, ws->oW3, ws->L0 * WS_H2, ws->W3b);
  hipLaunchKernelGGL(k_ws_convw, dim3((3 * 28 * WS_C * WS_C + 255) / 256), dim3(256), 0, ws->stream,
                     (const float*)(ws->w + ws->oK), ws->Kb, ws->Ktb);
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
  ws_forward(ws, ws->pin, ws->idx, 1);
  hipLaunchKernelGGL(k_ws_head, dim3((unsigned)ws->nhead), dim3(256), 0, ws->stream, 1, ws->arch.nz, ws->arch.ny,
                     ws->arch.nx, ws->dim(3, 0), ws->dim(3, 1), ws->dim(3, 2), (const uint16_t*)ws->xb[2],
                     (const float*)(ws->w + ws->owo), (const float*)(ws->w + ws->obo), (const float*)nullptr,
                     (const int*)nullptr, ws->y, (const float*)nullptr, (uint16_t*)nullptr, (float*)nullptr,
                     (float*)nullptr, (double*)nullptr);
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
