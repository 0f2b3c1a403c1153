// Warm-start network kernels: BF16 matrix-core convolutions (FP32
// accumulation) for gfx950, their gradients, and the small element-wise
// layers around them.
//
// Every convolution-like layer is one implicit GEMM
//     Y[o(p), co] = sum_t sum_ci X[g_t(p), ci] W[t][co][ci]
// over positions p: M = positions, N = output channels, K = taps x input
// channels, both operands K-contiguous (activations channels-last, weights
// [tap][cout][cin]), so every slab is staged with 16-byte loads and stores.
// A workgroup of four waves computes a 128 x 64 (or 256 x 32) output tile
// with v_mfma_f32_16x16x32_bf16, double-buffering its K slabs in LDS.  Operand lane layout of that instruction (lane l = 0..63,
// element e = 0..7): A[l % 16][8 (l / 16) + e], B[8 (l / 16) + e][l % 16];
// result element e of lane l is D[4 (l / 16) + e][l % 16].
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/pi_unet.h"

namespace pu {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __host__ inline float bf2f(uint16_t b) {
  union {
    uint32_t u;
    float f;
  } v;
  v.u = (uint32_t)b << 16;
  return v.f;
}

// round to nearest even; NaN stays NaN
__device__ __host__ inline uint16_t f2bf(float f) {
  union {
    uint32_t u;
    float f;
  } v;
  v.f = f;
  if ((v.u & 0x7f800000u) == 0x7f800000u && (v.u & 0x007fffffu)) return (uint16_t)((v.u >> 16) | 0x40);
  const uint32_t r = v.u + 0x7fffu + ((v.u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}

struct Tens {
  uint16_t *p;
  int n, d, h, w, c, ld, off;
};

__host__ inline Tens tens(const pu_tensor *t) {
  return Tens{(uint16_t *)t->ptr, t->n, t->d, t->h, t->w, t->c, t->ld, t->off};
}

struct ConvP {
  Tens x, y;
  const uint16_t *w;
  const float *bias;
  int taps, cin, cout;
  int md, mh, mw, sin, sout, ooz, ooy, oox;
  int relu, yfp32, acc;
  int64_t P;
  int8_t offs[27][3];
};

__device__ inline void decompose(int64_t p, int md, int mh, int mw, int &nb, int &z, int &y, int &x) {
  x = (int)(p % mw);
  int64_t t = p / mw;
  y = (int)(t % mh);
  t /= mh;
  z = (int)(t % md);
  nb = (int)(t / md);
}

__device__ inline bf16x8 lds8(const uint16_t *p) { return __builtin_bit_cast(bf16x8, *(const uint4 *)p); }

constexpr int kLdsRow = 40;  // 32 K values + 8 padding, 80-byte rows

// Y = act(X * W + b) over one BM-position x BN-channel tile, W given as
// [tap][cout][cin] so that both operands are K-contiguous in memory and in
// LDS.  Four waves; wave w computes rows [w BM/4, (w+1) BM/4) of the tile as
// (BM/64) x (BN/16) blocks of 16 x 16 (eight MFMAs per K step of 32 for
// both tile shapes: 128 x 64 for layers of 64 or more output channels,
// 256 x 32 for 32).  The K loop runs over (tap, 32-channel slab) steps with
// two LDS buffers: the global loads of step s + 1 are in flight while the
// MFMAs of step s run, then land in the other buffer; one barrier per step.
template <int BN>
__global__ __launch_bounds__(256) void k_conv(ConvP a) {
  constexpr int BM = 8192 / BN;          // 128 or 256 positions
  constexpr int RA = BM / 64;            // A rows staged per thread (16-byte chunks)
  constexpr int MI = BM / 64;            // 16-row blocks per wave
  constexpr int NJ = BN / 16;            // 16-column blocks
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM][kLdsRow];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN][kLdsRow];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  // A staging: rows tid/4 + 64 i, eight K values from kq
  const int kq = (tid & 3) * 8;
  int rz[RA], ry[RA], rx[RA], rb[RA];
  bool rin[RA];
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int64_t p = p0 + (tid >> 2) + 64 * i;
    rin[i] = p < a.P;
    rb[i] = rz[i] = ry[i] = rx[i] = 0;
    if (rin[i]) decompose(p, a.md, a.mh, a.mw, rb[i], rz[i], ry[i], rx[i]);
  }
  // B staging: channel row tid/4 (BN rows, all threads when BN = 64), eight K values from kq
  const int brow = tid >> 2;
  const bool bact = brow < BN;
  const bool xvec = (a.x.ld % 8 == 0) && (a.x.off % 8 == 0) && (a.cin % 8 == 0);
  const bool wvec = a.cin % 8 == 0;
  const int ksteps = (a.cin + 31) / 32;
  const int S = a.taps * ksteps;
  uint4 ra[RA], rbv;
  auto fetch = [&](int step) {
    const int t = step / ksteps, k0 = (step % ksteps) * 32 + kq;
#pragma unroll
    for (int i = 0; i < RA; ++i) {
      ra[i] = uint4{0u, 0u, 0u, 0u};
      const int iz = rz[i] * a.sin + a.offs[t][0], iy = ry[i] * a.sin + a.offs[t][1],
                ix = rx[i] * a.sin + a.offs[t][2];
      const bool v = rin[i] && iz >= 0 && iz < a.x.d && iy >= 0 && iy < a.x.h && ix >= 0 && ix < a.x.w && k0 < a.cin;
      if (v) {
        const int64_t xb = ((((int64_t)rb[i] * a.x.d + iz) * a.x.h + iy) * a.x.w + ix) * a.x.ld + a.x.off + k0;
        if (xvec) {
          ra[i] = *(const uint4 *)(a.x.p + xb);
        } else {
          uint16_t tmp[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) tmp[e] = (k0 + e < a.cin) ? a.x.p[xb + e] : (uint16_t)0;
          ra[i] = *(const uint4 *)tmp;
        }
      }
    }
    rbv = uint4{0u, 0u, 0u, 0u};
    if (bact && n0 + brow < a.cout && k0 < a.cin) {
      const uint16_t *wr = a.w + ((int64_t)t * a.cout + n0 + brow) * a.cin + k0;
      if (wvec) {
        rbv = *(const uint4 *)wr;
      } else {
        uint16_t tmp[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) tmp[e] = (k0 + e < a.cin) ? wr[e] : (uint16_t)0;
        rbv = *(const uint4 *)tmp;
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int i = 0; i < RA; ++i) *(uint4 *)&As[buf][(tid >> 2) + 64 * i][kq] = ra[i];
    if (bact) *(uint4 *)&Bs[buf][brow][kq] = rbv;
  };
  f4 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  fetch(0);
  stash(0);
  __syncthreads();
  for (int s = 0; s < S; ++s) {
    const int cur = s & 1;
    if (s + 1 < S) fetch(s + 1);
    bf16x8 bv[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) bv[j] = lds8(&Bs[cur][16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < MI; ++i) {
      const bf16x8 av = lds8(&As[cur][wave * (BM / 4) + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < NJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[j], acc[i][j], 0, 0, 0);
    }
    if (s + 1 < S) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = wave * (BM / 4) + 16 * i + 4 * (lane >> 4) + e, col = 16 * j + (lane & 15);
        const int64_t pp = p0 + row;
        const int co = n0 + col;
        if (pp >= a.P || co >= a.cout) continue;
        int b2, z2, y2, x2;
        decompose(pp, a.md, a.mh, a.mw, b2, z2, y2, x2);
        const int oz = z2 * a.sout + a.ooz, oy = y2 * a.sout + a.ooy, ox = x2 * a.sout + a.oox;
        const int64_t yi = ((((int64_t)b2 * a.y.d + oz) * a.y.h + oy) * a.y.w + ox) * a.y.ld + a.y.off + co;
        float val = acc[i][j][e] + (a.bias ? a.bias[co] : 0.f);
        if (a.relu) val = fmaxf(val, 0.f);
        if (a.yfp32) {
          float *yf = (float *)a.y.p;
          yf[yi] = a.acc ? yf[yi] + val : val;
        } else {
          a.y.p[yi] = f2bf(a.acc ? bf2f(a.y.p[yi]) + val : val);
        }
      }
}

struct WgP {
  Tens x, g;
  int taps, cin, cout;
  int md, mh, mw, sin, sout, ooz, ooy, oox;
  int64_t P, chunk;
  float *part;   // [nsplit][taps][cin][cout]
  float *bpart;  // [nsplit][cout] or NULL
  int8_t offs[27][3];
};

// Partial weight gradient over one chunk of positions for one (tap, 64-ci,
// 64-co) tile.
__global__ __launch_bounds__(256) void k_wgrad(WgP a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[64][kLdsRow];  // [ci][pos]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64][kLdsRow];  // [co][pos]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nct = (a.cout + 63) / 64;
  const int ci0 = (blockIdx.x / nct) * 64, co0 = (blockIdx.x % nct) * 64;
  const int t = blockIdx.y, split = blockIdx.z;
  const int64_t pbeg = (int64_t)split * a.chunk, pend = std::min<int64_t>(a.P, pbeg + a.chunk);
  const int pr = tid >> 3, q8 = (tid & 7) * 8;  // staging: position row, eight channels
  const bool xvec = (a.x.ld % 8 == 0) && (a.x.off % 8 == 0) && (a.cin % 8 == 0);
  const bool gvec = (a.g.ld % 8 == 0) && (a.g.off % 8 == 0) && (a.cout % 8 == 0);
  // gy does not depend on the tap: the (tap 0, first ci tile) blocks also sum it for the bias
  const bool do_bias = a.bpart && t == 0 && ci0 == 0;
  float bsum[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) bsum[e] = 0.f;
  f4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  for (int64_t pb = pbeg; pb < pend; pb += 32) {
    const int64_t p = pb + pr;
    uint16_t xa[8], ga[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) xa[e] = ga[e] = 0;
    if (p < pend) {
      int nb, mz, my, mx;
      decompose(p, a.md, a.mh, a.mw, nb, mz, my, mx);
      const int iz = mz * a.sin + a.offs[t][0], iy = my * a.sin + a.offs[t][1], ix = mx * a.sin + a.offs[t][2];
      if (iz >= 0 && iz < a.x.d && iy >= 0 && iy < a.x.h && ix >= 0 && ix < a.x.w && ci0 + q8 < a.cin) {
        const int64_t xb = ((((int64_t)nb * a.x.d + iz) * a.x.h + iy) * a.x.w + ix) * a.x.ld + a.x.off + ci0 + q8;
        if (xvec && ci0 + q8 + 8 <= a.cin) {
          *(uint4 *)xa = *(const uint4 *)(a.x.p + xb);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) xa[e] = (ci0 + q8 + e < a.cin) ? a.x.p[xb + e] : (uint16_t)0;
        }
      }
      const int oz = mz * a.sout + a.ooz, oy = my * a.sout + a.ooy, ox = mx * a.sout + a.oox;
      if (co0 + q8 < a.cout) {
        const int64_t gb = ((((int64_t)nb * a.g.d + oz) * a.g.h + oy) * a.g.w + ox) * a.g.ld + a.g.off + co0 + q8;
        if (gvec && co0 + q8 + 8 <= a.cout) {
          *(uint4 *)ga = *(const uint4 *)(a.g.p + gb);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) ga[e] = (co0 + q8 + e < a.cout) ? a.g.p[gb + e] : (uint16_t)0;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[q8 + e][pr] = xa[e];
      Bs[q8 + e][pr] = ga[e];
      bsum[e] += bf2f(ga[e]);
    }
    __syncthreads();
    const bf16x8 av8 = lds8(&As[16 * wave + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bf16x8 bv8 = lds8(&Bs[16 * j + (lane & 15)][8 * (lane >> 4)]);
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av8, bv8, acc[j], 0, 0, 0);
    }
    __syncthreads();
  }
  if (do_bias) {
    __shared__ float red[32][65];
#pragma unroll
    for (int e = 0; e < 8; ++e) red[pr][q8 + e] = bsum[e];
    __syncthreads();
    if (tid < 64 && co0 + tid < a.cout) {
      float s = 0.f;
      for (int k = 0; k < 32; ++k) s += red[k][tid];
      a.bpart[(int64_t)split * a.cout + co0 + tid] = s;
    }
  }
  float *out = a.part + ((int64_t)split * a.taps + t) * a.cin * a.cout;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ci = ci0 + 16 * wave + 4 * (lane >> 4) + e, co = co0 + 16 * j + (lane & 15);
      if (ci < a.cin && co < a.cout) out[(int64_t)ci * a.cout + co] = acc[j][e];
    }
  }
}

// Sum `nsplit` partial arrays of `count` floats in split order.
__global__ void k_sum_splits(const float *part, int64_t count, int nsplit, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float s = 0.f;
  for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * count + i];
  out[i] = s;
}

__global__ void k_transpose_taps(const uint16_t *w, uint16_t *wt, int taps, int cin, int cout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)cin * cout;
  if (i >= per * taps) return;
  const int64_t t = i / per, rem = i % per;
  const int ci = (int)(rem / cout), co = (int)(rem % cout);
  wt[t * per + (int64_t)co * cin + ci] = w[i];
}

__device__ inline int64_t elem(const Tens &t, int64_t cell, int c) { return cell * t.ld + t.off + c; }

__global__ void k_relu_bwd(Tens y, Tens g, int64_t cells) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cells * y.c) return;
  const int64_t cell = i / y.c;
  const int c = (int)(i % y.c);
  const int64_t gi = elem(g, cell, c);
  if (!(bf2f(y.p[elem(y, cell, c)]) > 0.f)) g.p[gi] = 0;
}

// y[n, z, y, x, c] = mean of x over the 2x2x2 block
__global__ void k_pool(Tens x, Tens y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cells = (int64_t)y.n * y.d * y.h * y.w;
  if (i >= cells * y.c) return;
  const int64_t cell = i / y.c;
  const int c = (int)(i % y.c);
  int nb, z, yy, xx;
  decompose(cell, y.d, y.h, y.w, nb, z, yy, xx);
  float s = 0.f;
  for (int q = 0; q < 8; ++q) {
    const int64_t src = (((int64_t)nb * x.d + 2 * z + (q >> 2)) * x.h + 2 * yy + ((q >> 1) & 1)) * x.w + 2 * xx + (q & 1);
    s += bf2f(x.p[elem(x, src, c)]);
  }
  y.p[elem(y, cell, c)] = f2bf(0.125f * s);
}

__global__ void k_pool_bwd(Tens gy, Tens gx, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cells = (int64_t)gx.n * gx.d * gx.h * gx.w;
  if (i >= cells * gx.c) return;
  const int64_t cell = i / gx.c;
  const int c = (int)(i % gx.c);
  int nb, z, yy, xx;
  decompose(cell, gx.d, gx.h, gx.w, nb, z, yy, xx);
  const int64_t src = (((int64_t)nb * gy.d + z / 2) * gy.h + yy / 2) * gy.w + xx / 2;
  float v = 0.125f * bf2f(gy.p[elem(gy, src, c)]);
  const int64_t di = elem(gx, cell, c);
  if (accumulate) v += bf2f(gx.p[di]);
  gx.p[di] = f2bf(v);
}

__global__ void k_head(Tens x, const float *w, const float *b, float *y, int64_t cells) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cells) return;
  float s = b[0];
  for (int c = 0; c < x.c; ++c) s += bf2f(x.p[elem(x, i, c)]) * w[c];
  y[i] = s;
}

__global__ void k_head_bwd_x(Tens gx, const float *w, const float *gy, int64_t cells) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cells * gx.c) return;
  const int64_t cell = i / gx.c;
  const int c = (int)(i % gx.c);
  gx.p[elem(gx, cell, c)] = f2bf(gy[cell] * w[c]);
}

// per-chunk partial sums of x[., c] * gy and of gy (last slot)
__global__ void k_head_bwd_w(Tens x, const float *gy, int64_t cells, int64_t chunk, float *part) {
  const int64_t beg = (int64_t)blockIdx.x * chunk, end = std::min<int64_t>(cells, beg + chunk);
  for (int c = threadIdx.x; c <= x.c; c += blockDim.x) {
    float s = 0.f;
    for (int64_t i = beg; i < end; ++i) s += (c < x.c ? bf2f(x.p[elem(x, i, c)]) : 1.f) * gy[i];
    part[(int64_t)blockIdx.x * (x.c + 1) + c] = s;
  }
}

__global__ void k_mse_part(const float *pred, const float *target, const uint8_t *mask, int64_t count, int64_t chunk,
                           float *part) {
  __shared__ float sd[256], sc[256];
  const int64_t beg = (int64_t)blockIdx.x * chunk, end = std::min<int64_t>(count, beg + chunk);
  float d2 = 0.f, cnt = 0.f;
  for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    if (mask && !mask[i]) continue;
    const float d = pred[i] - target[i];
    d2 += d * d;
    cnt += 1.f;
  }
  sd[threadIdx.x] = d2;
  sc[threadIdx.x] = cnt;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sd[threadIdx.x] += sd[threadIdx.x + s];
      sc[threadIdx.x] += sc[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd[0];
    part[2 * blockIdx.x + 1] = sc[0];
  }
}

__global__ void k_mse_finish(const float *part, int nchunk, float *loss, float *cnt_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.f, c = 0.f;
  for (int k = 0; k < nchunk; ++k) {
    s += part[2 * k];
    c += part[2 * k + 1];
  }
  *loss = c > 0.f ? s / c : 0.f;
  *cnt_out = c;
}

__global__ void k_mse_grad(const float *pred, const float *target, const uint8_t *mask, int64_t count,
                           const float *cnt, float *grad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float c = *cnt;
  grad[i] = (mask && !mask[i]) || c <= 0.f ? 0.f : 2.f * (pred[i] - target[i]) / c;
}

__global__ void k_rms_part(const float *gx, const float *gy, const float *gz, const uint8_t *mask, int64_t count,
                           int64_t chunk, float *part) {
  __shared__ float sd[256], sc[256];
  const int64_t beg = (int64_t)blockIdx.x * chunk, end = std::min<int64_t>(count, beg + chunk);
  float s = 0.f, cnt = 0.f;
  for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
    if (mask && !mask[i]) continue;
    const float z = gz ? gz[i] : 0.f;
    s += gx[i] * gx[i] + gy[i] * gy[i] + z * z;
    cnt += 1.f;
  }
  sd[threadIdx.x] = s;
  sc[threadIdx.x] = cnt;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      sd[threadIdx.x] += sd[threadIdx.x + k];
      sc[threadIdx.x] += sc[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd[0];
    part[2 * blockIdx.x + 1] = sc[0];
  }
}

__global__ void k_rms_finish(const float *part, int nchunk, float *rms) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.f, c = 0.f;
  for (int k = 0; k < nchunk; ++k) {
    s += part[2 * k];
    c += part[2 * k + 1];
  }
  *rms = c > 0.f ? sqrtf(s / c) : 0.f;
}

__global__ void k_adam(float *w, const float *g, float *m, float *v, uint16_t *wb, int64_t count, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = f2bf(wi);
}

// coarse cell (n = 0, z, y, x): averages of the data cells of its block
__global__ void k_prepare(const float *gx, const float *gy, const float *gz, const uint8_t *mask, int nx, int ny,
                          int nz, int f, int fz, float scale, Tens out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cells = (int64_t)out.d * out.h * out.w;
  if (i >= cells) return;
  const int cx = (int)(i % out.w), cy = (int)((i / out.w) % out.h), cz = (int)(i / ((int64_t)out.w * out.h));
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, cnt = 0.f;
  for (int dz = 0; dz < fz; ++dz)
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) {
        const int64_t c = ((int64_t)(cz * fz + dz) * ny + cy * f + dy) * nx + cx * f + dx;
        if (mask && !mask[c]) continue;
        s0 += gx[c];
        s1 += gy[c];
        if (gz) s2 += gz[c];
        cnt += 1.f;
      }
  const float inv = cnt > 0.f ? scale / cnt : 0.f;
  out.p[elem(out, i, 0)] = f2bf(s0 * inv);
  out.p[elem(out, i, 1)] = f2bf(s1 * inv);
  out.p[elem(out, i, 2)] = f2bf(s2 * inv);
  out.p[elem(out, i, 3)] = f2bf(cnt / (float)(f * f * fz));
}

// coarse cell (z, y, x): FP32 means of each gradient component over the data
// cells of its block (0 where the block holds none)
__global__ void k_block_mean(const float *gx, const float *gy, const float *gz, const uint8_t *mask, int nx, int ny,
                             int nz, int f, int fz, float *ox, float *oy, float *oz) {
  const int cnx = nx / f, cny = ny / f, cnz = nz / fz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)cnx * cny * cnz) return;
  const int cx = (int)(i % cnx), cy = (int)((i / cnx) % cny), cz = (int)(i / ((int64_t)cnx * cny));
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, cnt = 0.f;
  for (int dz = 0; dz < fz; ++dz)
    for (int dy = 0; dy < f; ++dy)
      for (int dx = 0; dx < f; ++dx) {
        const int64_t c = ((int64_t)(cz * fz + dz) * ny + cy * f + dy) * nx + cx * f + dx;
        if (mask && !mask[c]) continue;
        s0 += gx[c];
        s1 += gy[c];
        if (gz) s2 += gz[c];
        cnt += 1.f;
      }
  const float inv = cnt > 0.f ? 1.f / cnt : 0.f;
  ox[i] = s0 * inv;
  oy[i] = s1 * inv;
  if (oz) oz[i] = s2 * inv;
}

__device__ inline float lerp_idx(int fine, int f, int n, int &i0) {
  // cell-centred: fine centre (fine + 1/2) / f - 1/2 in coarse index units;
  // beyond the outermost coarse centres the line through the two outermost
  // ones continues (weight outside [0, 1]), so linear fields are exact up to
  // the grid's edge -- where the solver reads the start (the first cells of
  // the rays, [W^n])
  const float u = ((float)fine + 0.5f) / (float)f - 0.5f;
  i0 = min(max((int)floorf(u), 0), max(n - 2, 0));
  return n > 1 ? u - (float)i0 : 0.f;
}

__global__ void k_upsample(const float *coarse, int nx, int ny, int nz, int f, int fz, float scale, void *P,
                           int fp64, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cells = (int64_t)nx * ny * nz;
  if (i >= cells) return;
  const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
  const int cnx = nx / f, cny = ny / f, cnz = nz / fz;
  int x0, y0, z0;
  const float tx = lerp_idx(x, f, cnx, x0), ty = lerp_idx(y, f, cny, y0);
  const float tz = fz > 1 ? lerp_idx(z, fz, cnz, z0) : (z0 = z, 0.f);
  const int x1 = min(x0 + 1, cnx - 1), y1 = min(y0 + 1, cny - 1), z1 = min(z0 + 1, cnz - 1);
  auto at = [&](int zz, int yy, int xx) { return coarse[((int64_t)zz * cny + yy) * cnx + xx]; };
  const float c00 = at(z0, y0, x0) * (1 - tx) + at(z0, y0, x1) * tx;
  const float c01 = at(z0, y1, x0) * (1 - tx) + at(z0, y1, x1) * tx;
  const float c10 = at(z1, y0, x0) * (1 - tx) + at(z1, y0, x1) * tx;
  const float c11 = at(z1, y1, x0) * (1 - tx) + at(z1, y1, x1) * tx;
  const float v = scale * ((c00 * (1 - ty) + c01 * ty) * (1 - tz) + (c10 * (1 - ty) + c11 * ty) * tz);
  if (fp64)
    ((double *)P)[i] = (accumulate ? ((double *)P)[i] : 0.0) + (double)v;
  else
    ((float *)P)[i] = (accumulate ? ((float *)P)[i] : 0.f) + v;
}

inline unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

inline bool ok_tensor(const pu_tensor *t) {
  return t && t->ptr && t->n > 0 && t->d > 0 && t->h > 0 && t->w > 0 && t->c > 0 && t->off >= 0 &&
         t->ld >= t->off + t->c;
}

inline int64_t wgrad_chunk(int64_t P) { return std::max<int64_t>(2048, ((P + 255) / 256 + 31) / 32 * 32); }

}  // namespace pu

using namespace pu;

#define PU_LAUNCHED (hipGetLastError() == hipSuccess ? PI_OK : PI_ERR_DEVICE)

extern "C" pi_status pu_conv(const pu_tensor *x, const void *w, int32_t taps, const int8_t *offs, const float *bias,
                             const pu_tensor *y, int32_t md, int32_t mh, int32_t mw, int32_t sin, int32_t sout,
                             const int32_t oo[3], int32_t relu, int32_t y_fp32, int32_t accumulate, void *stream) {
  if (!ok_tensor(x) || !ok_tensor(y) || !w || !offs || taps < 1 || taps > 27 || md < 1 || mh < 1 || mw < 1 ||
      sin < 1 || sout < 1 || !oo || x->n != y->n)
    return PI_ERR_INVALID_ARG;
  // every output position must land inside y (inputs may fall outside x: zero)
  if ((md - 1) * sout + oo[0] >= y->d || (mh - 1) * sout + oo[1] >= y->h || (mw - 1) * sout + oo[2] >= y->w ||
      oo[0] < 0 || oo[1] < 0 || oo[2] < 0)
    return PI_ERR_INVALID_ARG;
  ConvP a;
  a.x = tens(x);
  a.y = tens(y);
  a.w = (const uint16_t *)w;
  a.bias = bias;
  a.taps = taps;
  a.cin = x->c;
  a.cout = y->c;
  a.md = md;
  a.mh = mh;
  a.mw = mw;
  a.sin = sin;
  a.sout = sout;
  a.ooz = oo[0];
  a.ooy = oo[1];
  a.oox = oo[2];
  a.relu = relu;
  a.yfp32 = y_fp32;
  a.acc = accumulate;
  a.P = (int64_t)x->n * md * mh * mw;
  for (int t = 0; t < taps; ++t)
    for (int k = 0; k < 3; ++k) a.offs[t][k] = offs[3 * t + k];
  // 32 output channels: a 256 x 32 tile wastes no MFMA columns
  if (a.cout <= 32) {
    k_conv<32><<<dim3(blocks(a.P, 256), 1), dim3(256), 0, (hipStream_t)stream>>>(a);
  } else {
    k_conv<64><<<dim3(blocks(a.P, 128), (a.cout + 63) / 64), dim3(256), 0, (hipStream_t)stream>>>(a);
  }
  return PU_LAUNCHED;
}

extern "C" size_t pu_wgrad_work_floats(int32_t taps, int32_t cin, int32_t cout, int64_t positions) {
  const int64_t chunk = wgrad_chunk(positions);
  const int64_t nsplit = (positions + chunk - 1) / chunk;
  return (size_t)(nsplit * ((int64_t)taps * cin * cout + cout));
}

extern "C" pi_status pu_conv_wgrad(const pu_tensor *x, const pu_tensor *gy, int32_t taps, const int8_t *offs,
                                   float *dw, float *db, int32_t md, int32_t mh, int32_t mw, int32_t sin,
                                   int32_t sout, const int32_t oo[3], float *work, void *stream) {
  if (!ok_tensor(x) || !ok_tensor(gy) || !dw || !offs || !work || taps < 1 || taps > 27 || x->n != gy->n || !oo)
    return PI_ERR_INVALID_ARG;
  if ((md - 1) * sout + oo[0] >= gy->d || (mh - 1) * sout + oo[1] >= gy->h || (mw - 1) * sout + oo[2] >= gy->w)
    return PI_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  WgP a;
  a.x = tens(x);
  a.g = tens(gy);
  a.taps = taps;
  a.cin = x->c;
  a.cout = gy->c;
  a.md = md;
  a.mh = mh;
  a.mw = mw;
  a.sin = sin;
  a.sout = sout;
  a.ooz = oo[0];
  a.ooy = oo[1];
  a.oox = oo[2];
  a.P = (int64_t)x->n * md * mh * mw;
  a.chunk = wgrad_chunk(a.P);
  const int nsplit = (int)((a.P + a.chunk - 1) / a.chunk);
  a.part = work;
  a.bpart = db ? work + (int64_t)nsplit * taps * a.cin * a.cout : nullptr;
  for (int t = 0; t < taps; ++t)
    for (int k = 0; k < 3; ++k) a.offs[t][k] = offs[3 * t + k];
  const int tiles = ((a.cin + 63) / 64) * ((a.cout + 63) / 64);
  k_wgrad<<<dim3(tiles, taps, nsplit), dim3(256), 0, s>>>(a);
  const int64_t count = (int64_t)taps * a.cin * a.cout;
  k_sum_splits<<<blocks(count), dim3(256), 0, s>>>(work, count, nsplit, dw);
  if (db) k_sum_splits<<<blocks(a.cout), dim3(256), 0, s>>>(a.bpart, a.cout, nsplit, db);
  return PU_LAUNCHED;
}

extern "C" pi_status pu_transpose_taps(const void *w, void *wt, int32_t taps, int32_t cin, int32_t cout,
                                       void *stream) {
  if (!w || !wt || taps < 1 || cin < 1 || cout < 1) return PI_ERR_INVALID_ARG;
  const int64_t n = (int64_t)taps * cin * cout;
  k_transpose_taps<<<blocks(n), dim3(256), 0, (hipStream_t)stream>>>((const uint16_t *)w, (uint16_t *)wt, taps, cin,
                                                                     cout);
  return PU_LAUNCHED;
}

static bool same_grid(const pu_tensor *a, const pu_tensor *b) {
  return a->n == b->n && a->d == b->d && a->h == b->h && a->w == b->w;
}

extern "C" pi_status pu_relu_backward(const pu_tensor *y, const pu_tensor *g, void *stream) {
  if (!ok_tensor(y) || !ok_tensor(g) || !same_grid(y, g) || y->c != g->c) return PI_ERR_INVALID_ARG;
  const int64_t cells = (int64_t)y->n * y->d * y->h * y->w;
  k_relu_bwd<<<blocks(cells * y->c), dim3(256), 0, (hipStream_t)stream>>>(tens(y), tens(g), cells);
  return PU_LAUNCHED;
}

extern "C" pi_status pu_pool(const pu_tensor *x, const pu_tensor *y, void *stream) {
  if (!ok_tensor(x) || !ok_tensor(y) || x->c != y->c || x->n != y->n || x->d != 2 * y->d || x->h != 2 * y->h ||
      x->w != 2 * y->w)
    return PI_ERR_INVALID_ARG;
  const int64_t cells = (int64_t)y->n * y->d * y->h * y->w;
  k_pool<<<blocks(cells * y->c), dim3(256), 0, (hipStream_t)stream>>>(tens(x), tens(y));
  return PU_LAUNCHED;
}

extern "C" pi_status pu_pool_backward(const pu_tensor *gy, const pu_tensor *gx, int32_t accumulate, void *stream) {
  if (!ok_tensor(gx) || !ok_tensor(gy) || gx->c != gy->c || gx->n != gy->n || gx->d != 2 * gy->d ||
      gx->h != 2 * gy->h || gx->w != 2 * gy->w)
    return PI_ERR_INVALID_ARG;
  const int64_t cells = (int64_t)gx->n * gx->d * gx->h * gx->w;
  k_pool_bwd<<<blocks(cells * gx->c), dim3(256), 0, (hipStream_t)stream>>>(tens(gy), tens(gx), accumulate);
  return PU_LAUNCHED;
}

extern "C" pi_status pu_head(const pu_tensor *x, const float *w, const float *b, float *y, void *stream) {
  if (!ok_tensor(x) || !w || !b || !y) return PI_ERR_INVALID_ARG;
  const int64_t cells = (int64_t)x->n * x->d * x->h * x->w;
  k_head<<<blocks(cells), dim3(256), 0, (hipStream_t)stream>>>(tens(x), w, b, y, cells);
  return PU_LAUNCHED;
}

extern "C" pi_status pu_head_backward(const pu_tensor *x, const float *w, const float *gy, const pu_tensor *gx,
                                      float *gw, float *gb, float *work, void *stream) {
  if (!ok_tensor(x) || !ok_tensor(gx) || !same_grid(x, gx) || x->c != gx->c || !w || !gy || !gw || !gb || !work)
    return PI_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int64_t cells = (int64_t)x->n * x->d * x->h * x->w;
  k_head_bwd_x<<<blocks(cells * x->c), dim3(256), 0, s>>>(tens(gx), w, gy, cells);
  const int64_t chunk = std::max<int64_t>(1024, (cells + 1023) / 1024);
  const int nch = (int)((cells + chunk - 1) / chunk);
  k_head_bwd_w<<<dim3(nch), dim3(64), 0, s>>>(tens(x), gy, cells, chunk, work);
  float *red = work + (int64_t)nch * (x->c + 1);
  k_sum_splits<<<1, dim3(256), 0, s>>>(work, x->c + 1, nch, red);
  if (hipMemcpyAsync(gw, red, x->c * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(gb, red + x->c, sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return PI_ERR_DEVICE;
  return PU_LAUNCHED;
}

extern "C" pi_status pu_mse(const float *pred, const float *target, const uint8_t *mask, int64_t count, float *loss,
                            float *grad, float *work, void *stream) {
  if (!pred || !target || count < 1 || !loss || !work) return PI_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int64_t chunk = std::max<int64_t>(4096, (count + 1023) / 1024);
  const int nch = (int)((count + chunk - 1) / chunk);
  k_mse_part<<<dim3(nch), dim3(256), 0, s>>>(pred, target, mask, count, chunk, work);
  k_mse_finish<<<1, 1, 0, s>>>(work, nch, loss, work + 2 * nch);
  if (grad) k_mse_grad<<<blocks(count), dim3(256), 0, s>>>(pred, target, mask, count, work + 2 * nch, grad);
  return PU_LAUNCHED;
}

extern "C" pi_status pu_adam(float *w, const float *g, float *m, float *v, void *wb, int64_t count, float lr,
                             float beta1, float beta2, float eps, int32_t step, void *stream) {
  if (!w || !g || !m || !v || count < 1 || step < 1) return PI_ERR_INVALID_ARG;
  const float c1 = 1.f / (1.f - powf(beta1, (float)step)), c2 = 1.f / (1.f - powf(beta2, (float)step));
  k_adam<<<blocks(count), dim3(256), 0, (hipStream_t)stream>>>(w, g, m, v, (uint16_t *)wb, count, lr, beta1, beta2,
                                                               eps, c1, c2);
  return PU_LAUNCHED;
}

extern "C" pi_status pu_prepare_input(const float *gx, const float *gy, const float *gz, const uint8_t *mask,
                                      const int64_t dims[3], int32_t factor, float scale, const pu_tensor *out,
                                      void *stream) {
  if (!gx || !gy || !dims || factor < 1 || !ok_tensor(out) || out->c != 4 || out->n != 1) return PI_ERR_INVALID_ARG;
  const int64_t nx = dims[0], ny = dims[1], nz = dims[2] > 0 ? dims[2] : 1;
  const int fz = gz ? factor : 1;
  if (nx % factor || ny % factor || nz % fz || out->w != nx / factor || out->h != ny / factor || out->d != nz / fz)
    return PI_ERR_INVALID_ARG;
  const int64_t cells = (int64_t)out->d * out->h * out->w;
  k_prepare<<<blocks(cells), dim3(256), 0, (hipStream_t)stream>>>(gx, gy, gz, mask, (int)nx, (int)ny, (int)nz, factor,
                                                                  fz, scale, tens(out));
  return PU_LAUNCHED;
}

extern "C" pi_status pu_block_mean(const float *gx, const float *gy, const float *gz, const uint8_t *mask,
                                   const int64_t dims[3], int32_t factor, float *ox, float *oy, float *oz,
                                   void *stream) {
  if (!gx || !gy || !dims || factor < 1 || !ox || !oy || (gz && !oz)) return PI_ERR_INVALID_ARG;
  const int64_t nx = dims[0], ny = dims[1], nz = dims[2] > 0 ? dims[2] : 1;
  const int fz = gz ? factor : 1;
  if (nx % factor || ny % factor || nz % fz) return PI_ERR_INVALID_ARG;
  const int64_t cells = (nx / factor) * (ny / factor) * (nz / fz);
  k_block_mean<<<blocks(cells), dim3(256), 0, (hipStream_t)stream>>>(gx, gy, gz, mask, (int)nx, (int)ny, (int)nz,
                                                                     factor, fz, ox, oy, gz ? oz : nullptr);
  return PU_LAUNCHED;
}

extern "C" pi_status pu_upsample_output(const float *coarse, const int64_t dims[3], int32_t factor, float scale,
                                        void *P, int32_t flags, void *stream) {
  if (!coarse || !dims || !P || factor < 1 || (flags & ~(PU_OUT_FP64 | PU_OUT_ADD))) return PI_ERR_INVALID_ARG;
  const int64_t nx = dims[0], ny = dims[1], nz = dims[2] > 0 ? dims[2] : 1;
  const int fz = nz > 1 ? factor : 1;
  if (nx % factor || ny % factor || nz % fz) return PI_ERR_INVALID_ARG;
  k_upsample<<<blocks(nx * ny * nz), dim3(256), 0, (hipStream_t)stream>>>(coarse, (int)nx, (int)ny, (int)nz, factor,
                                                                          fz, scale, P, (flags & PU_OUT_FP64) != 0,
                                                                          (flags & PU_OUT_ADD) != 0);
  return PU_LAUNCHED;
}

extern "C" pi_status pu_grad_rms(const float *gx, const float *gy, const float *gz, const uint8_t *mask,
                                 int64_t count, float *rms, float *work, void *stream) {
  if (!gx || !gy || count < 1 || !rms || !work) return PI_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int64_t chunk = std::max<int64_t>(4096, (count + 511) / 512);
  const int nch = (int)((count + chunk - 1) / chunk);
  k_rms_part<<<dim3(nch), dim3(256), 0, s>>>(gx, gy, gz, mask, count, chunk, work);
  k_rms_finish<<<1, 1, 0, s>>>(work, nch, rms);
  return PU_LAUNCHED;
}
