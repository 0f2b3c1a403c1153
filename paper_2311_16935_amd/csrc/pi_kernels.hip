// HIP kernels of the solve (gfx950).
//
// All kernels are memory-bound stencils or streaming updates; no matrix
// cores are involved.  Each kernel walks the block table described in
// pi_common.h.  A kernel that reduces writes one FP64 partial per block and
// nothing else crosses blocks inside a kernel: a small finalize kernel (one
// block per instance) then sums the partials in a fixed order and updates
// that instance's scalars.  The kernel boundary orders the two, so no fence
// or atomic counter sits on the hot path, and results are bitwise
// reproducible.
//
// Two ways of walking an instance's cells:
//  * stencil kernels march: a wave owns a strip of 64 * W consecutive cells
//    along x (W cells per lane, 16-byte loads when W = 4) and walks along the
//    slowest axis, fetching everything plane m+1 needs (operand, code words,
//    source, y neighbours, strip-edge values) while it computes plane m;
//  * point-wise kernels stream a contiguous range of cells per block,
//    16 bytes per lane per load, so each block reads long linear runs.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include "pi_common.h"
#include "pi_kernels.h"

namespace pi {

// Buffers reached through the instance record are generic pointers to the
// compiler, which would then emit flat accesses that wait on both the vector
// memory and LDS counters; every hot buffer is therefore cast to the global
// address space once.
#define PI_G __attribute__((address_space(1)))
template <typename T>
__device__ inline PI_G T *gp(void *p) {
  return (PI_G T *)p;
}
template <typename T>
__device__ inline const PI_G T *gp(const void *p) {
  return (const PI_G T *)p;
}

// ---------------------------------------------------------------------------
// short vectors: W consecutive cells of one array, moved with 16-byte (or,
// for two FP32 cells, 8-byte) accesses; the caller guarantees the alignment
// ---------------------------------------------------------------------------
template <typename V, int W>
struct Vec {
  V e[W];
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <int W, typename T>
__device__ inline Vec<T, W> ldv(const PI_G T *p, int64_t c) {
  Vec<T, W> v;
  if constexpr (W > 1 && W * sizeof(T) == 8) {
    const u32x2 u = *(const PI_G u32x2 *)(p + c);
    memcpy(&v.e[0], &u, 8);
  } else if constexpr (W * sizeof(T) < 16) {
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = p[c + k];
  } else {
    const PI_G u32x4 *q = (const PI_G u32x4 *)(p + c);
#pragma unroll
    for (int i = 0; i < (int)(W * sizeof(T) / 16); ++i) {
      const u32x4 u = q[i];
      memcpy(&v.e[i * (16 / sizeof(T))], &u, 16);
    }
  }
  return v;
}

template <int W, typename T>
__device__ inline void stv(PI_G T *p, int64_t c, const Vec<T, W> &v) {
  if constexpr (W > 1 && W * sizeof(T) == 8) {
    u32x2 u;
    memcpy(&u, &v.e[0], 8);
    *(PI_G u32x2 *)(p + c) = u;
  } else if constexpr (W * sizeof(T) < 16) {
#pragma unroll
    for (int k = 0; k < W; ++k) p[c + k] = v.e[k];
  } else {
    PI_G u32x4 *q = (PI_G u32x4 *)(p + c);
#pragma unroll
    for (int i = 0; i < (int)(W * sizeof(T) / 16); ++i) {
      u32x4 u;
      memcpy(&u, &v.e[i * (16 / sizeof(T))], 16);
      q[i] = u;
    }
  }
}

// Streams that one kernel writes (or reads at the cell only) and that the
// next kernel of the step reads again from memory: non-temporal, so they do
// not displace the neighbour rows that other waves are about to re-read
// from L2 (the CG passes always; the outer kernel where the autotuner
// measured it faster).
template <int W, typename T>
__device__ inline void stv_nt(PI_G T *p, int64_t c, const Vec<T, W> &v) {
  if constexpr (W * sizeof(T) >= 16) {
    PI_G u32x4 *q = (PI_G u32x4 *)(p + c);
#pragma unroll
    for (int i = 0; i < (int)(W * sizeof(T) / 16); ++i) {
      u32x4 u;
      memcpy(&u, &v.e[i * (16 / sizeof(T))], 16);
      __builtin_nontemporal_store(u, q + i);
    }
  } else {
    stv<W>(p, c, v);
  }
}
template <int W, typename T>
__device__ inline Vec<T, W> ldv_nt(const PI_G T *p, int64_t c) {
  if constexpr (W * sizeof(T) >= 16) {
    Vec<T, W> v;
    const PI_G u32x4 *q = (const PI_G u32x4 *)(p + c);
#pragma unroll
    for (int i = 0; i < (int)(W * sizeof(T) / 16); ++i) {
      const u32x4 u = __builtin_nontemporal_load(q + i);
      memcpy(&v.e[i * (16 / sizeof(T))], &u, 16);
    }
    return v;
  } else {
    return ldv<W>(p, c);
  }
}

template <typename V, int W>
__device__ inline Vec<V, W> vzero() {
  Vec<V, W> z;
#pragma unroll
  for (int k = 0; k < W; ++k) z.e[k] = V(0);
  return z;
}

// ---------------------------------------------------------------------------
// stencil work decomposition
// ---------------------------------------------------------------------------
// Everything a wave needs while it walks its segment, copied out of the
// instance record once: the compiler cannot keep fields of a global struct
// in registers across the kernel's own stores.
struct Walk {
  int64_t base;   // storage index of this lane's first cell at march position 0
  int64_t sm;     // stride of the march axis
  const PI_G uint32_t *code;
  int m0, m1;     // march range of this wave (uniform over the wave)
  int nm;         // length of the march axis
  int nx, ny, nz;
  int x;          // x of this lane's first cell
  int row;        // y of this wave's strip (3-D)
  bool act;       // lane owns cells inside the grid
};

template <int W>
__device__ inline Walk make_walk(const Inst &in, int lb) {
  Walk k;
  k.sm = in.sm;
  k.code = gp<uint32_t>(in.code);
  k.nm = in.nm;
  k.nx = in.nx;
  k.ny = in.ny;
  k.nz = in.nz;
  k.m0 = k.m1 = 0;
  k.x = k.row = 0;
  k.base = 0;
  k.act = false;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)lb * kWavesPerBlock + wave;
  if (w >= in.nwaves) return k;
  // strips are numbered x fastest, then y (3-D), then segment, so the four
  // waves of a block cover consecutive memory of one plane
  const int64_t xs = w % in.nxs;
  const int64_t t = w / in.nxs;
  const int64_t row = in.ndim == 3 ? t % in.rows : 0;
  const int64_t seg = in.ndim == 3 ? t / in.rows : t;
  k.x = (int)(xs * kWave * W + lane * W);
  k.m0 = (int)(seg * in.mseg);
  k.m1 = min(k.m0 + in.mseg, in.nm);
  k.act = k.x < in.nx;
  k.row = (int)row;
  // lanes past the end of a partial strip address the strip's last cells
  // (nx is a multiple of W), so that every load is in bounds without a
  // branch; they never store
  k.base = (int64_t)min(k.x, in.nx - W) + row * in.srow;
  return k;
}

__device__ inline int dstate(uint32_t code, int d, int bits) {
  return (int)((code >> (bits * d)) & ((1u << bits) - 1u));
}

// Counter code of a cell of a grid without missing data, from its
// coordinates: the same word the plan stores (face neighbour J = C + s e_a
// inside the grid; laterals of J with data along each remaining axis; far
// cell J + s e_a inside the grid), since every in-grid cell holds data.
template <int ND>
__device__ inline uint32_t code_at(int x, int y, int z, int nx, int ny, int nz) {
  const int c[3] = {x, y, z}, n[3] = {nx, ny, nz};
  int side[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) side[k] = (c[k] >= 1) + (c[k] + 1 < n[k]);
  const int bits = dir_bits(ND);
  uint32_t out = kValidBit;
#pragma unroll
  for (int d = 0; d < 2 * ND; ++d) {
    const int a = d >> 1, s = (d & 1) ? -1 : 1;
    const int j = c[a] + s, f = c[a] + 2 * s;
    if (j < 0 || j >= n[a]) continue;
    const int far = f >= 0 && f < n[a];
    const int l0 = a == 0 ? 1 : 0, l1 = a == 2 ? 1 : 2;
    const uint32_t state = ND == 3 ? 1u + side[l0] + 3u * side[l1] + 9u * far : 1u + side[l0] + 3u * far;
    out |= state << (bits * d);
  }
  return out;
}

// Code word of a cell whose face neighbours, their laterals and their far
// cells all hold data: every direction in its last state.
template <int ND>
__host__ __device__ constexpr uint32_t interior_code() {
  uint32_t c = kValidBit;
  for (int d = 0; d < 2 * ND; ++d) c |= (ND == 3 ? 18u : 6u) << ((ND == 3 ? 5 : 3) * d);
  return c;
}
template <int ND>
__host__ __device__ constexpr int interior_state() {
  return ND == 3 ? 18 : 6;
}

// What the stencil body sees at one cell: its operand value, the y
// neighbours (3-D only), the extra per-cell input and the code word.
// Neighbours outside the grid read as 0; internal vectors hold 0 in masked
// cells, and every neighbour value is used only through its counter state.
template <typename V, typename A>
struct Cell {
  V v, vN, vS;
  A aux;
  uint32_t code;
};

// One plane of a lane's W cells, fetched one plane ahead of its use.  vEdge
// is the x neighbour beyond the strip end (lane 0: west, lane 63: east).
template <typename V, typename A, int W>
struct Plane {
  Vec<V, W> v, vN, vS;
  Vec<A, W> aux;
  Vec<uint32_t, W> code;
  V vEdge;
};

// March one wave along its segment.
//   load(c)   -> Vec<V, W>  stencil operand at cells c .. c+W-1
//   load1(c)  -> V          stencil operand at one cell (strip edges)
//   aux(c)    -> Vec<A, W>  extra per-cell input
//   body(c, cell, vW, vE, vPrev, vNext) -> Out   one cell; x neighbours come
//             from the lane's own cells and adjacent lanes, march-axis
//             neighbours from registers
//   store(c, const Out (&)[W])
template <int ND, int W, bool GEN, typename V, typename A, typename Out, typename Load, typename Load1, typename Aux,
          typename Body, typename Store>
__device__ inline void march(const Walk &wk, Load load, Load1 load1, Aux aux, Body body, Store store) {
  if (wk.m1 <= wk.m0) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  const bool hasN = ND == 3 && wk.row + 1 < wk.ny, hasS = ND == 3 && wk.row > 0;
  const bool edgeW = lane == 0 && wk.x > 0, edgeE = lane == kWave - 1 && wk.x + W < wk.nx;
  const int64_t snx = wk.nx;
  // neighbour offsets resolved once; a neighbour that does not exist reads
  // the cell itself and is zeroed, so no load sits behind a branch
  const int64_t offN = hasN ? snx : 0, offS = hasS ? -snx : 0;
  const int64_t offE = edgeW ? -1 : edgeE ? W : 0;
  const bool hasEdge = edgeW || edgeE;
  const PI_G uint32_t *code = wk.code;
  // codes of an unmasked grid follow from (x, y, z): 3-D (x, row, m), 2-D (x, m, 0)
  auto codes = [&](int64_t c, int m) {
    if constexpr (GEN) {
      Vec<uint32_t, W> v;
      // cells two or more steps inside the grid on every axis have the
      // interior code (uniform over the wave except at the strip ends)
      const bool inner = m >= 2 && m + 2 < wk.nm && wk.x >= 2 && wk.x + W + 1 < wk.nx &&
                         (ND == 2 || (wk.row >= 2 && wk.row + 2 < wk.ny));
      if (inner) {
#pragma unroll
        for (int k = 0; k < W; ++k) v.e[k] = interior_code<ND>();
      } else {
#pragma unroll
        for (int k = 0; k < W; ++k)
          v.e[k] = ND == 3 ? code_at<3>(wk.x + k, wk.row, m, wk.nx, wk.ny, wk.nz)
                           : code_at<2>(wk.x + k, m, 0, wk.nx, wk.ny, 1);
      }
      return v;
    } else {
      return ldv<W>(code, c);
    }
  };
  auto fetch = [&](int64_t c, int m, Plane<V, A, W> &pl) {
    pl.v = load(c);
    pl.code = codes(c, m);
    pl.aux = aux(c);
    if (ND == 3) {
      const Vec<V, W> n = load(c + offN), s = load(c + offS);
#pragma unroll
      for (int k = 0; k < W; ++k) {
        pl.vN.e[k] = hasN ? n.e[k] : V(0);
        pl.vS.e[k] = hasS ? s.e[k] : V(0);
      }
    }
    const V e = load1(c + offE);
    pl.vEdge = hasEdge ? e : V(0);
  };
  const int64_t sm = wk.sm;
  int64_t c = wk.base + (int64_t)wk.m0 * sm;
  Vec<V, W> prev = wk.m0 > 0 ? load(c - sm) : vzero<V, W>();
  Plane<V, A, W> cur, nxt;
  fetch(c, wk.m0, cur);
  for (int m = wk.m0; m < wk.m1; ++m, c += sm) {
    // uniform over the wave: the whole next plane, or only its values when
    // it is the next segment's first plane, or nothing past the grid
    if (m + 1 < wk.m1)
      fetch(c + sm, m + 1, nxt);
    else
      nxt.v = m + 1 < wk.nm ? load(c + sm) : vzero<V, W>();
    V left = __shfl_up(cur.v.e[W - 1], 1, kWave);
    V right = __shfl_down(cur.v.e[0], 1, kWave);
    if (lane == 0) left = cur.vEdge;
    if (lane == kWave - 1) right = cur.vEdge;
    // lanes past the grid only serve the shuffles: they neither compute
    // (their cells duplicate a neighbour's, which would enter the sums) nor store
    if (wk.act) {
      Out o[W];
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const V vW = k == 0 ? left : cur.v.e[k > 0 ? k - 1 : 0];
        const V vE = k == W - 1 ? right : cur.v.e[k + 1 < W ? k + 1 : 0];
        Cell<V, A> cl;
        cl.v = cur.v.e[k];
        cl.vN = ND == 3 ? cur.vN.e[k] : V(0);
        cl.vS = ND == 3 ? cur.vS.e[k] : V(0);
        cl.aux = cur.aux.e[k];
        cl.code = cur.code.e[k];
        o[k] = body(c + k, cl, vW, vE, prev.e[k], nxt.v.e[k]);
      }
      store(c, o);
    }
    prev = cur.v;
    cur = nxt;
  }
}

// The loads of one plane as issued, before anything is computed from them.
template <typename LR, typename XR, typename L1R, int W>
struct RawPlane {
  LR v, vN, vS;
  XR x;
  L1R edge;
  Vec<uint32_t, W> code;
};

// march with the loads of plane m + 2 in flight while plane m is computed.
// march combines a plane's values as soon as they are loaded, so the wave
// waits for every load it has just issued before it computes; here the
// loaded values stay raw until their plane is consumed, and the copy of the
// raw buffer at the end of an iteration is the only wait, after the plane's
// arithmetic and stores have been issued.  It costs registers (the raw
// inputs of one more plane), so kernels whose occupancy it would lower keep
// march.
//   load(c)  -> LR   raw operand inputs at cells c .. c+W-1
//   load1(c) -> L1R  raw operand inputs at one cell (strip edges)
//   extra(c) -> XR   raw extra per-cell input
//   cookv(LR) -> Vec<V, W>, cook1(L1R) -> V, cooka(LR, XR) -> Vec<A, W>
// Planes past the segment are loaded at a clamped, in-bounds position and
// never used; the operand of the plane after the grid's last one reads 0.
template <int ND, int W, bool GEN, typename V, typename A, typename Out, typename Load, typename Load1,
          typename Extra, typename CookV, typename Cook1, typename CookA, typename Body, typename Store>
__device__ inline void march2(const Walk &wk, Load load, Load1 load1, Extra extra, CookV cookv, Cook1 cook1,
                              CookA cooka, Body body, Store store) {
  if (wk.m1 <= wk.m0) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  const bool hasN = ND == 3 && wk.row + 1 < wk.ny, hasS = ND == 3 && wk.row > 0;
  const bool edgeW = lane == 0 && wk.x > 0, edgeE = lane == kWave - 1 && wk.x + W < wk.nx;
  const int64_t snx = wk.nx;
  const int64_t offN = hasN ? snx : 0, offS = hasS ? -snx : 0;
  const int64_t offE = edgeW ? -1 : edgeE ? W : 0;
  const bool hasEdge = edgeW || edgeE;
  using LR = decltype(load(int64_t{}));
  using XR = decltype(extra(int64_t{}));
  using L1R = decltype(load1(int64_t{}));
  using RP = RawPlane<LR, XR, L1R, W>;
  const int jmax = min(wk.m1, wk.nm - 1);
  const int64_t sm = wk.sm;
  auto fetch = [&](int j, RP &rp) {
    const int64_t cj = wk.base + (int64_t)min(j, jmax) * sm;
    rp.v = load(cj);
    if constexpr (!GEN) rp.code = ldv<W>(wk.code, cj);
    rp.x = extra(cj);
    if constexpr (ND == 3) {
      rp.vN = load(cj + offN);
      rp.vS = load(cj + offS);
    }
    rp.edge = load1(cj + offE);
  };
  auto cook = [&](int j, const RP &rp, Plane<V, A, W> &pl) {
    const Vec<V, W> v = cookv(rp.v);
    const bool in = j < wk.nm;
#pragma unroll
    for (int k = 0; k < W; ++k) pl.v.e[k] = in ? v.e[k] : V(0);
    pl.aux = cooka(rp.v, rp.x);
    if constexpr (GEN) {
      const bool inner = j >= 2 && j + 2 < wk.nm && wk.x >= 2 && wk.x + W + 1 < wk.nx &&
                         (ND == 2 || (wk.row >= 2 && wk.row + 2 < wk.ny));
#pragma unroll
      for (int k = 0; k < W; ++k)
        pl.code.e[k] = inner ? interior_code<ND>()
                             : (ND == 3 ? code_at<3>(wk.x + k, wk.row, j, wk.nx, wk.ny, wk.nz)
                                        : code_at<2>(wk.x + k, j, 0, wk.nx, wk.ny, 1));
    } else {
      pl.code = rp.code;
    }
    if constexpr (ND == 3) {
      const Vec<V, W> n = cookv(rp.vN), s = cookv(rp.vS);
#pragma unroll
      for (int k = 0; k < W; ++k) {
        pl.vN.e[k] = hasN ? n.e[k] : V(0);
        pl.vS.e[k] = hasS ? s.e[k] : V(0);
      }
    }
    const V e = cook1(rp.edge);
    pl.vEdge = hasEdge ? e : V(0);
  };
  int64_t c = wk.base + (int64_t)wk.m0 * sm;
  Vec<V, W> prev = vzero<V, W>();
  if (wk.m0 > 0) prev = cookv(load(c - sm));
  RP ra, rb;
  fetch(wk.m0, ra);
  fetch(wk.m0 + 1, rb);
  Plane<V, A, W> cur, nxt;
  cook(wk.m0, ra, cur);
  for (int m = wk.m0; m < wk.m1; ++m, c += sm) {
    fetch(m + 2, ra);
    cook(m + 1, rb, nxt);
    V left = __shfl_up(cur.v.e[W - 1], 1, kWave);
    V right = __shfl_down(cur.v.e[0], 1, kWave);
    if (lane == 0) left = cur.vEdge;
    if (lane == kWave - 1) right = cur.vEdge;
    if (wk.act) {
      Out o[W];
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const V vW = k == 0 ? left : cur.v.e[k > 0 ? k - 1 : 0];
        const V vE = k == W - 1 ? right : cur.v.e[k + 1 < W ? k + 1 : 0];
        Cell<V, A> cl;
        cl.v = cur.v.e[k];
        cl.vN = ND == 3 ? cur.vN.e[k] : V(0);
        cl.vS = ND == 3 ? cur.vS.e[k] : V(0);
        cl.aux = cur.aux.e[k];
        cl.code = cur.code.e[k];
        o[k] = body(c + k, cl, vW, vE, prev.e[k], nxt.v.e[k]);
      }
      store(c, o);
    }
    prev = cur.v;
    cur = nxt;
    rb = ra;
  }
}

// ---------------------------------------------------------------------------
// point-wise work decomposition: block lb of an instance owns the cells
// [lb * per, (lb + 1) * per) with per a multiple of 1024
// ---------------------------------------------------------------------------
__device__ inline void linear_range(const Inst &in, int lb, int64_t &beg, int64_t &end) {
  const int64_t g = 1024;
  const int64_t per = ((in.ncell + in.nblocks - 1) / in.nblocks + g - 1) / g * g;
  beg = min(in.ncell, (int64_t)lb * per);
  end = min(in.ncell, beg + per);
}

// Stream [beg, end) with E cells per lane per access and U accesses in
// flight: f.load(c, u) / f.apply(c, u) for E cells at c, f.one(c) for a
// single cell at the ragged end of the array.
template <int E, int U, typename F>
__device__ inline void stream_linear(int64_t beg, int64_t end, F &f) {
  const int64_t step = (int64_t)kBlock * E;
  int64_t c = beg + (int64_t)threadIdx.x * E;
  for (; c + (U - 1) * step + E <= end; c += U * step) {
#pragma unroll
    for (int u = 0; u < U; ++u) f.load(c + u * step, u);
#pragma unroll
    for (int u = 0; u < U; ++u) f.apply(c + u * step, u);
  }
  for (; c + E <= end; c += step) {
    f.load(c, 0);
    f.apply(c, 0);
  }
  for (; c < end; ++c) f.one(c);  // at most E - 1 cells, last block only
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
template <int K>
__device__ inline void block_sum(double (&v)[K], double *lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, kWave);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[wave * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = ((lds[k] + lds[K + k]) + lds[2 * K + k]) + lds[3 * K + k];
  }
}

// Write this block's K partial sums into its slot (4 doubles per block).
template <int K>
__device__ inline void publish(const Inst &in, double *part, int lb, double (&v)[K]) {
  __shared__ double lds[kWavesPerBlock * 4];
  block_sum<K>(v, lds);
  if (threadIdx.x == 0) {
    double *slot = part + ((int64_t)in.part_base + lb) * 4;
#pragma unroll
    for (int k = 0; k < K; ++k) slot[k] = v[k];
  }
}

// The four sums (p.q, r.q, q.q, r.r) that the blocks of inner CG pass j of
// this instance wrote, added in a fixed order; every thread gets the totals.
// Pass j's partials sit in partial array 1 + (j & 1).
__device__ inline void cg_partials(const Inst &in, const double *part, int j, double (&s)[4]) {
  __shared__ double lds[kWavesPerBlock * 4];
  __shared__ double tot[4];
  const double2 *slots =
      reinterpret_cast<const double2 *>(part + ((int64_t)(1 + (j & 1)) * in.part_stride + in.part_base) * 4);
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = 0.0;
  for (int i = threadIdx.x; i < in.cg_slots; i += kBlock) {
    const double2 a = slots[2 * i], b = slots[2 * i + 1];
    s[0] += a.x;
    s[1] += a.y;
    s[2] += b.x;
    s[3] += b.y;
  }
  block_sum<4>(s, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) tot[k] = s[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = tot[k];
}

// From the sums of CG iteration j: alpha_j = r.r / p.q and, with
// |r_j - alpha_j q_j|^2 = r.r - 2 alpha_j r.q + alpha_j^2 q.q, beta_{j+1}.
// The fixed-point variant's inner solve stops once that residual is well
// below the tolerance (the FP64 outer step then confirms it), or once it is
// as small as the vector precision can resolve: beyond that only the
// residual's rounding-level constant part is left, which the singular
// operator cannot reduce (p.q -> 0 and alpha would blow up); the next outer
// step restarts from the FP64 residual.
struct CgScalars {
  double al, be;
  bool stop;
};
__device__ inline CgScalars cg_scalars(const Inst &in, const State *st, const double (&s)[4]) {
  const double pq = s[0], rq = s[1], qq = s[2], rr = s[3];
  const double al = pq != 0.0 ? rr / pq : 0.0;
  double rn = rr - 2.0 * al * rq + al * al * qq;
  if (!(rn > 0.0)) rn = 0.0;
  CgScalars c;
  c.al = al;
  c.be = rr != 0.0 ? rn / rr : 0.0;
  c.stop = in.inner_op != 0 && (rn <= 0.25 * in.tol * in.tol * st->normS2 || rn <= in.inner_floor * st->rr0);
  return c;
}

template <typename T>
__device__ inline void load_lut(const double (*src)[kStates], T (*dst)[kStates]) {
  for (int i = threadIdx.x; i < 6 * kStates; i += kBlock) dst[i / kStates][i % kStates] = (T)src[i / kStates][i % kStates];
  __syncthreads();
}

#define PI_PROLOGUE                                   \
  const BlockEnt e = tab[blockIdx.x];                 \
  if (e.inst < 0) return;                             \
  const Inst &in = insts[e.inst];                     \
  State *st = sts + e.inst;

// Skip conditions, evaluated identically by a kernel and by its finalize.
__device__ inline bool skip_outer(const State *st) { return st->done != 0; }
__device__ inline bool skip_inner(const Inst &in, const State *st) {
  return st->done != 0 || st->inner >= in.inner_iters;
}

// ---------------------------------------------------------------------------
// set-up: P^0 and the source vector
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts, double *part,
                                                 int warm) {
  PI_PROLOGUE
  int64_t beg, end;
  linear_range(in, e.lb, beg, end);
  const T *P0 = (const T *)in.P0;
  double *P = in.P[0];
  T *d = (T *)in.d;
  T *p0 = (T *)in.p[0], *p1 = (T *)in.p[1], *v = (T *)in.bs[1];
  T *q0 = (T *)in.q, *q1 = (T *)in.q1;
  const uint32_t *code = in.code;
  int bad = 0;
  for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
    // no correction before the first outer step, and finite search
    // directions and products for the first inner iteration (which scales
    // them by 0)
    d[c] = T(0);
    p0[c] = T(0);
    p1[c] = T(0);
    q0[c] = T(0);
    if (q1) q1[c] = T(0);
    if (v) v[c] = T(0);
    double x = 0.0;
    if (warm && (code[c] & kValidBit)) {
      x = (double)P0[c];
      if (!isfinite(x)) {
        bad = 1;
        x = 0.0;
      }
    }
    P[c] = x;
  }
  if (bad) atomicOr(&st->nonfinite, 1);
}

// S_C = - sum_j Delta_j (w_j^{n+1} + w_j^n) (f_j(J) + f_j(C)) / 2 over face
// neighbours J holding data (Eq. ExplicitEqn_FaceCrossing).  For such J the
// two counters add up to the face total (Eq. AE_Interior and the 3-D face
// integral), so w_j^{n+1} + w_j^n = a_j.  FP64 arithmetic and FP64 storage:
// the face terms cancel in pairs, so S sums to zero over every connected
// group; a float copy would not, and its constant part would put a floor of
// about 6e-8 / sqrt(cells) under the reachable residual.
template <typename T, int ND>
__global__ __launch_bounds__(kBlock) void k_source(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts, double *part) {
  PI_PROLOGUE
  int64_t beg, end;
  linear_range(in, e.lb, beg, end);
  const T *g[3] = {(const T *)in.g[0], (const T *)in.g[1], (const T *)in.g[2]};
  T *S = (T *)in.S;
  double *S64 = in.S64;
  const uint32_t *code = in.code;
  const int bits = dir_bits(ND);
  const int64_t off[6] = {1, -1, (int64_t)in.nx, -(int64_t)in.nx, ND == 3 ? (int64_t)in.nx * in.ny : 0,
                          ND == 3 ? -(int64_t)in.nx * in.ny : 0};
  double w[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) w[d] = -0.5 * in.dsig[d] * in.a[d];
  double acc[1] = {0.0};
  int bad = 0;
  for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
    const uint32_t cd = code[c];
    double s = 0.0;
    if (cd & kValidBit) {
      double own[3];
#pragma unroll
      for (int a = 0; a < ND; ++a) {
        own[a] = (double)g[a][c];
        if (!isfinite(own[a])) bad = 1;
      }
#pragma unroll
      for (int d = 0; d < 2 * ND; ++d) {
        if (dstate(cd, d, bits)) {
          const int a = d >> 1;
          const double nb = (double)g[a][c + off[d]];
          s += w[d] * (nb + own[a]);
        }
      }
    }
    S64[c] = s;
    if (S) S[c] = (T)s;
    acc[0] += s * s;
  }
  if (bad) atomicOr(&st->nonfinite, 1);
  publish<1>(in, part, e.lb, acc);
}

// ---------------------------------------------------------------------------
// outer step: P^{n+1} = P^n + delta, r = S - (M - N) P^{n+1}, eps_R
// ---------------------------------------------------------------------------
// The inner solve's correction as the outer kernel folds it in:
// delta = d + at * pt.  With CG, K = min(stop_at, inner_iters) passes ran;
// pass K - 1 left its search direction in p[K & 1] and its alpha in its
// partial sums (or, with a finalize kernel, in the state); the correction
// sum d was written by passes 1 .. K - 1, so it is read only when K >= 2
// (with K = 1 the buffer still holds the previous outer step's sum).
// BiCGStab adds every update into d itself.  Uniform over the launch.
template <typename T>
struct Pending {
  T at;
  const PI_G T *pt;
  bool use_d;
};
template <typename T>
__device__ inline Pending<T> pending(const Inst &in, const State *st, const double *part) {
  Pending<T> pd;
  pd.at = T(0);
  pd.pt = gp<T>(in.p[0]);
  pd.use_d = false;
  if (!st->have_delta) return pd;  // no inner solve yet
  if (in.bicg) {
    pd.use_d = st->dvalid != 0;
    return pd;
  }
  const int K = min(st->stop_at, in.inner_iters);
  pd.use_d = K >= 2;
  if (K >= 1) {
    double al;
    if (in.cg_inline) {
      double s[4];
      cg_partials(in, part, K - 1, s);
      al = s[0] != 0.0 ? s[3] / s[0] : 0.0;
    } else {
      al = st->alpha;
    }
    pd.at = (T)al;
    pd.pt = gp<T>(in.p[K & 1]);
  }
  return pd;
}

// (M - N) is applied as sum_j a_j (P_C - P_J) over face neighbours holding
// data: its off-diagonal entries are -(w_j^{n+1} + w_j^n) = -a_j and, since
// all counters of a data cell add up to A_tot, its diagonal 1 - w_C^n equals
// sum_j a_j.  With CG the last inner iteration's update is folded in here:
// delta = d + alpha p (the residual it would also update is recomputed from
// scratch anyway), which saves one pass over four vectors per outer step.
template <typename T, int ND, int W, bool GEN>
__global__ __launch_bounds__(kBlock) void k_outer(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts, double *part) {
  PI_PROLOGUE
  if (skip_outer(st)) return;
  const Walk wk = make_walk<W>(in, e.lb);
  const int cur = st->Pcur;
  const PI_G double *Pold = gp<double>(in.P[cur]);
  PI_G double *Pnew = gp<double>(in.P[cur ^ 1]);
  const Pending<T> pd = pending<T>(in, st, part);
  const T at = pd.at;
  const PI_G T *pt = pd.pt;
  const PI_G T *dl = gp<T>(in.d);
  const bool use_d = pd.use_d;
  const PI_G double *S = gp<double>(in.S64);
  PI_G T *res = gp<T>(in.res);
  const bool nt = in.nt_outer != 0;  // uniform over the launch
  const int bits = dir_bits(ND);
  double a[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) a[d] = in.a[d];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  struct Out {
    double p, r;
  };
  struct Aux {
    double S, d;
  };
  // delta is zero before the first outer step (set when the solve starts)
  auto delta = [&](int64_t c) {
    const Vec<T, W> d = use_d ? ldv<W>(dl, c) : vzero<T, W>(), p = ldv<W>(pt, c);
    Vec<T, W> v;
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = d.e[k] + at * p.e[k];
    return v;
  };
  auto load = [&](int64_t c) {
    const Vec<double, W> P = ldv<W>(Pold, c);
    const Vec<T, W> d = delta(c);
    Vec<double, W> v;
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = P.e[k] + (double)d.e[k];
    return v;
  };
  auto load1 = [&](int64_t c) -> double { return Pold[c] + (double)((use_d ? dl[c] : T(0)) + at * pt[c]); };
  auto aux = [&](int64_t c) {
    const Vec<double, W> s = nt ? ldv_nt<W>(S, c) : ldv<W>(S, c);
    const Vec<T, W> d = delta(c);
    Vec<Aux, W> x;
#pragma unroll
    for (int k = 0; k < W; ++k) x.e[k] = Aux{s.e[k], (double)d.e[k]};
    return x;
  };
  auto body = [&](int64_t, const Cell<double, Aux> &pl, double vW, double vE, double vP, double vN) -> Out {
    const uint32_t cd = pl.code;
    if (!(cd & kValidBit)) return Out{0.0, 0.0};
    const double vC = pl.v;
    // neighbours without data read as 0 and get weight 0: no branches
    const bool all = cd == interior_code<ND>();
    double w[6];
#pragma unroll
    for (int d = 0; d < 2 * ND; ++d) w[d] = (all || dstate(cd, d, bits)) ? a[d] : 0.0;
    double Lp = 0.0;
    Lp += w[DE] * (vC - vE);
    Lp += w[DW] * (vC - vW);
    if (ND == 3) {
      Lp += w[DN] * (vC - pl.vN);
      Lp += w[DS] * (vC - pl.vS);
      Lp += w[DF] * (vC - vN);
      Lp += w[DB] * (vC - vP);
    } else {
      Lp += w[DN] * (vC - vN);
      Lp += w[DS] * (vC - vP);
    }
    const double r = pl.aux.S - Lp;
    const double rt = (double)(T)r;
    acc[0] += r * r;
    acc[1] += rt * rt;
    acc[2] += pl.aux.d * pl.aux.d;
    acc[3] += vC * vC;
    return Out{vC, r};
  };
  auto store = [&](int64_t c, const Out (&o)[W]) {
    Vec<double, W> p;
    Vec<T, W> r;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      p.e[k] = o[k].p;
      r.e[k] = (T)o[k].r;
    }
    if (nt) {
      stv_nt<W>(Pnew, c, p);
      stv_nt<W>(res, c, r);
    } else {
      stv<W>(Pnew, c, p);
      stv<W>(res, c, r);
    }
  };
  march<ND, W, GEN, double, Aux, Out>(wk, load, load1, aux, body, store);
  publish<4>(in, part, e.lb, acc);
}

// ---------------------------------------------------------------------------
// inner conjugate gradient on M delta = r
// ---------------------------------------------------------------------------
// The inner operator [W^{n+1}]: s = v_C - sum_j w_j^{n+1} v_J over face
// neighbours J holding data, weights from the per-state LUT.  State 0 (no
// data) has weight 0 and such neighbours read as 0, so the sum needs no
// branches; a cell with the interior code takes the interior weights wi
// from registers instead of the LUT.
template <typename T, int ND>
__device__ inline T apply_m(const T (*lut)[kStates], const T *wi, uint32_t cd, int bits, T vC, T vW, T vE, T vN,
                            T vS, T vP, T vNx) {
  T w[6];
  if (cd == interior_code<ND>()) {
#pragma unroll
    for (int d = 0; d < 2 * ND; ++d) w[d] = wi[d];
  } else {
#pragma unroll
    for (int d = 0; d < 2 * ND; ++d) w[d] = lut[d][dstate(cd, d, bits)];
  }
  T s = vC;
  s -= w[DE] * vE;
  s -= w[DW] * vW;
  if (ND == 3) {
    s -= w[DN] * vN;
    s -= w[DS] * vS;
    s -= w[DF] * vNx;
    s -= w[DB] * vP;
  } else {
    s -= w[DN] * vNx;
    s -= w[DS] * vP;
  }
  return s;
}

// The fixed point's operator [W^{n+1}] - [W^n]: sum_j a_j (v_C - v_J) over
// face neighbours holding data (the PI_FIXED_POINT_CG variant's inner operator).
template <typename T, int ND>
__device__ inline T apply_l(const T *a, uint32_t cd, int bits, T vC, T vW, T vE, T vN, T vS, T vP, T vNx) {
  T w[6];
  const bool all = cd == interior_code<ND>();
#pragma unroll
  for (int d = 0; d < 2 * ND; ++d) w[d] = (all || dstate(cd, d, bits)) ? a[d] : T(0);
  T s = T(0);
  s += w[DE] * (vC - vE);
  s += w[DW] * (vC - vW);
  if (ND == 3) {
    s += w[DN] * (vC - vN);
    s += w[DS] * (vC - vS);
    s += w[DF] * (vC - vNx);
    s += w[DB] * (vC - vP);
  } else {
    s += w[DN] * (vC - vNx);
    s += w[DS] * (vC - vP);
  }
  return s;
}

// One inner CG iteration k in a single pass (one global reduction per
// iteration).  The update of iteration k-1 is folded in:
//   r_k = r_{k-1} - alpha_{k-1} q_{k-1},   delta_k = delta_{k-1} + alpha_{k-1} p_{k-1},
//   p_k = r_k + beta_k p_{k-1},            q_k = A p_k,
// with A = [W^{n+1}] (or the fixed point's operator for the variant).  The
// stencil needs p_k at the neighbours, so r, q and p are read there and
// written to the other buffer of each pair.  Pass 0 has p_0 = r_0 (the
// outer residual): it reads r alone and writes p and q.  Reductions: p.q,
// r.q, q.q, r.r into partial array 1 + (k & 1).  alpha_{k-1} and beta_k come
// from pass k-1's sums (cg_scalars): every block adds them up itself, or,
// for instances of many blocks, a finalize kernel did so into the state.
// Pass 0 has no update to fold (alpha, beta = 0) and pass 1 starts the
// correction from zero.  k is the pass's index in the outer step, the same
// for every instance of a launch.
template <typename T>
struct CgPass {
  const PI_G T *rold, *qold, *pold;
  PI_G T *rnew, *qnew, *pnew, *d;
  T al, be;
  bool rd_d, wr_d;
  bool skip;
};

__device__ inline bool rq_p0_is_r(const Inst &in) { return in.cg_rq && in.inner_op == 0 && in.inner_iters >= 2; }

template <typename T>
__device__ inline CgPass<T> cg_pass(const Inst &in, State *st, const double *part, int lb, int k) {
  CgPass<T> c;
  // passes after the inner solve stopped have nothing to do.  With a
  // finalize kernel, the stop at this pass was recorded before it started;
  // without one, this pass's first block records it while the others run,
  // so only earlier passes' stops are read here (the same value in every
  // thread of the launch), and this pass decides its own below
  c.skip = st->done != 0 || k >= in.inner_iters || st->stop_at < k || (!in.cg_inline && st->stop_at == k);
  if (c.skip) return c;
  double al = 0.0, be = 0.0;
  if (k > 0) {
    if (in.cg_inline) {
      double s[4];
      cg_partials(in, part, k - 1, s);
      const CgScalars cs = cg_scalars(in, st, s);
      if (cs.stop) {
        if (lb == 0 && threadIdx.x == 0) st->stop_at = k;
        c.skip = true;
        return c;
      }
      al = cs.al;
      be = cs.be;
    } else {
      al = st->alpha;
      be = st->beta;
    }
  }
  // buffers: pass 0 reads the outer residual (res) only, since p_0 = r_0,
  // and writes p and q; pass k >= 1 reads r from res/res1 by the parity of
  // k + 1 and writes the other, reads q and p by the parity of k and writes
  // the other
  const int o = k & 1;
  c.rold = gp<T>(k == 0 || o ? in.res : in.res1);
  c.rnew = gp<T>(o ? in.res1 : in.res);
  c.qold = gp<T>(o ? in.q1 : in.q);
  c.qnew = gp<T>(o ? in.q : in.q1);
  // p_0 = r_0: a plan whose later passes evaluate q again takes p_0 from
  // the residual in pass 1, so pass 0 stores neither p nor q (the paper's
  // iteration with at least two passes: its last pass, which the outer
  // kernel folds in, is then never pass 0)
  c.pold = gp<T>(k == 1 && rq_p0_is_r(in) ? in.res : in.p[o]);
  c.pnew = gp<T>(in.p[o ^ 1]);
  c.d = gp<T>(in.d);
  c.al = (T)al;
  c.be = (T)be;
  c.wr_d = k > 0;
  c.rd_d = k > 1;
  return c;
}

// partial array of CG pass k
__device__ inline double *cg_part(const Inst &in, double *part, int k) {
  return part + (int64_t)(1 + (k & 1)) * in.part_stride * 4;
}

template <typename T, int ND, int W, bool GEN, bool FIRST>
__device__ __forceinline__ void cg_step_body(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts, double *part,
                                             int kpass) {
  PI_PROLOGUE
  const CgPass<T> cg = cg_pass<T>(in, st, part, e.lb, kpass);
  if (cg.skip) return;
  __shared__ T lut[6][kStates];
  load_lut<T>(in.lut_np1, lut);
  T wi[6];  // interior weights, as the LUT holds them
#pragma unroll
  for (int d = 0; d < 6; ++d) wi[d] = (T)in.lut_np1[d][interior_state<ND>()];
  const Walk wk = make_walk<W>(in, e.lb);
  const int bits = dir_bits(ND);
  const bool opL = in.inner_op != 0;  // uniform over the launch
  T a[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) a[d] = (T)in.a[d];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  struct Aux {
    T r, d;
  };
  struct Out {
    T p, q, r, d;
  };
  auto load = [&](int64_t c) {
    const Vec<T, W> r = ldv<W>(cg.rold, c), q = ldv<W>(cg.qold, c), p = ldv<W>(cg.pold, c);
    Vec<T, W> v;
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = (r.e[k] - cg.al * q.e[k]) + cg.be * p.e[k];
    return v;
  };
  auto load1 = [&](int64_t c) -> T { return (cg.rold[c] - cg.al * cg.qold[c]) + cg.be * cg.pold[c]; };
  auto aux = [&](int64_t c) {
    const Vec<T, W> r = ldv<W>(cg.rold, c), q = ldv<W>(cg.qold, c), p = ldv<W>(cg.pold, c);
    const Vec<T, W> d = cg.rd_d ? ldv_nt<W>(cg.d, c) : vzero<T, W>();
    Vec<Aux, W> x;
#pragma unroll
    for (int k = 0; k < W; ++k) x.e[k] = Aux{r.e[k] - cg.al * q.e[k], d.e[k] + cg.al * p.e[k]};
    return x;
  };
  auto body = [&](int64_t, const Cell<T, Aux> &pl, T vW, T vE, T vP, T vN) -> Out {
    const uint32_t cd = pl.code;
    const T vC = pl.v;
    if (!(cd & kValidBit)) return Out{T(0), T(0), T(0), T(0)};
    const T s = opL ? apply_l<T, ND>(a, cd, bits, vC, vW, vE, pl.vN, pl.vS, vP, vN)
                    : apply_m<T, ND>(lut, wi, cd, bits, vC, vW, vE, pl.vN, pl.vS, vP, vN);
    const double r = (double)pl.aux.r, q = (double)s;
    acc[0] += (double)vC * q;
    acc[1] += r * q;
    acc[2] += q * q;
    acc[3] += r * r;
    return Out{vC, s, pl.aux.r, pl.aux.d};
  };
  auto store = [&](int64_t c, const Out (&o)[W]) {
    Vec<T, W> pv, qv, rv, dv;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      pv.e[k] = o[k].p;
      qv.e[k] = o[k].q;
      rv.e[k] = o[k].r;
      dv.e[k] = o[k].d;
    }
    stv_nt<W>(cg.pnew, c, pv);
    stv_nt<W>(cg.qnew, c, qv);
    stv_nt<W>(cg.rnew, c, rv);
    if (cg.wr_d) stv_nt<W>(cg.d, c, dv);
  };
  if constexpr (FIRST) {
    // p_0 = r_0: only the residual is read; p and q are written.  Few bytes
    // per cell, so the loads of two planes ahead stay in flight (march2).
    auto load0 = [&](int64_t c) { return ldv<W>(cg.rold, c); };
    auto load01 = [&](int64_t c) -> T { return cg.rold[c]; };
    struct None {};
    auto extra0 = [](int64_t) { return None{}; };
    auto cookv0 = [](const Vec<T, W> &v) { return v; };
    auto cook10 = [](T v) { return v; };
    auto cooka0 = [](const Vec<T, W> &r, None) {
      Vec<Aux, W> x;
#pragma unroll
      for (int k = 0; k < W; ++k) x.e[k] = Aux{r.e[k], T(0)};
      return x;
    };
    const bool keep = !rq_p0_is_r(in);  // uniform over the launch
    auto store0 = [&](int64_t c, const Out (&o)[W]) {
      Vec<T, W> pv, qv;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        pv.e[k] = o[k].p;
        qv.e[k] = o[k].q;
      }
      if (keep) {
        stv_nt<W>(cg.pnew, c, pv);
        stv_nt<W>(cg.qnew, c, qv);
      }
    };
    march2<ND, W, GEN, T, Aux, Out>(wk, load0, load01, extra0, cookv0, cook10, cooka0, body, store0);
  } else {
    march<ND, W, GEN, T, Aux, Out>(wk, load, load1, aux, body, store);
  }
  publish<4>(in, cg_part(in, part, kpass), e.lb, acc);
}

// pass 0 of an outer step and the passes after it, compiled apart so that
// each gets its own register allocation
template <typename T, int ND, int W, bool GEN>
__global__ __launch_bounds__(kBlock) void k_cg_first(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                     double *part, int kpass) {
  cg_step_body<T, ND, W, GEN, true>(tab, insts, sts, part, kpass);
}
template <typename T, int ND, int W, bool GEN>
__global__ __launch_bounds__(kBlock) void k_cg_step(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                    double *part, int kpass) {
  cg_step_body<T, ND, W, GEN, false>(tab, insts, sts, part, kpass);
}

// ---------------------------------------------------------------------------
// The inner CG pass without a stored q: 3-D grids without missing data, four
// cells per lane, FP32, rows of one wave strip or split over overlapping
// wave windows (rq_window).
//
// CG's state is r, p and the correction; q = A p is stored only so that the
// next pass can form r_k = r_{k-1} - alpha q_{k-1}.  Here q_{k-1} = A p_{k-1}
// is evaluated again where it is needed: p_k at the cell and at its six
// neighbours needs A p_{k-1} there, so p_{k-1} is read within two cells (rows
// y-2 .. y+2 of plane m, rows y-1 .. y+1 of planes m-1 .. m+1, row y of planes
// m-2 .. m+2; the rows off the wave's own come from L2) and r_{k-1} within
// one.  Per cell a pass reads r, p and d and writes r', p' and d: 24 bytes
// instead of 32.  A p_{k-1} is formed with the operator and operand values
// the previous pass used for q_{k-1}, in the same order, so r_k, p_k and the
// sums are those of the stored-q pass bit for bit.  The first pass of an
// outer step (k_cg_first) is unchanged.
//
// Work is split by where the counter codes are constant: the planes 3 ..
// nm-4 of rows 3 .. ny-4 of every wave strip, where every code a pass looks
// at depends on x alone, so each lane keeps the weights of its cells in
// registers (no table, no validity tests: rq_int_march), and the rest, the
// layers next to the y and march faces, as short wave tasks with per-cell
// codes and the weight table (rq_bnd_march) in blocks of their own.  One
// kernel does both (k_cg_rq).
// ---------------------------------------------------------------------------

// Per-direction weights of the operator at a cell of code cd, as apply_m
// ([W^{n+1}], from the state table) or apply_l (the fixed point's operator)
// take them.
template <typename T, bool OPL, class Lut>
__device__ inline void op_weights(Lut lut, const T *wi, const T *a, uint32_t cd, T (&w)[6]) {
  const bool all = cd == interior_code<3>();
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    if constexpr (OPL) w[d] = (all || dstate(cd, d, 5)) ? a[d] : T(0);
    else w[d] = all ? wi[d] : lut(d, dstate(cd, d, 5));
  }
}
// The stencil with given weights: the operations of apply_m / apply_l in
// their order.
template <typename T, bool OPL>
__device__ inline T op_w(const T (&w)[6], T vC, T vW, T vE, T vN, T vS, T vB, T vF) {
  if constexpr (OPL) {
    T s = T(0);
    s += w[DE] * (vC - vE);
    s += w[DW] * (vC - vW);
    s += w[DN] * (vC - vN);
    s += w[DS] * (vC - vS);
    s += w[DF] * (vC - vF);
    s += w[DB] * (vC - vB);
    return s;
  } else {
    T s = vC;
    s -= w[DE] * vE;
    s -= w[DW] * vW;
    s -= w[DN] * vN;
    s -= w[DS] * vS;
    s -= w[DF] * vF;
    s -= w[DB] * vB;
    return s;
  }
}

// x neighbours of a lane's W cells; beyond the wave's ends reads 0: the grid
// face where the window ends at one, else a cell the window does not own
// (rq_window keeps owned cells far enough inside)
template <typename T, int W>
__device__ inline void xnb0(const Vec<T, W> &v, int lane, T (&vW)[W], T (&vE)[W]) {
  T left = __shfl_up(v.e[W - 1], 1, kWave);
  T right = __shfl_down(v.e[0], 1, kWave);
  if (lane == 0) left = T(0);
  if (lane == kWave - 1) right = T(0);
#pragma unroll
  for (int k = 0; k < W; ++k) {
    vW[k] = k == 0 ? left : v.e[k > 0 ? k - 1 : 0];
    vE[k] = k == W - 1 ? right : v.e[k + 1 < W ? k + 1 : 0];
  }
}

// Class of coordinate c on an axis of n cells as the counter code sees it:
// min(c, 2) + 3 min(n - 1 - c, 2) (whether the cells one and two steps away
// on each side lie in the grid).  The code of a cell of a grid without
// missing data is a function of its three classes (729 of them).
__device__ inline int rq_cls(int c, int n) { return min(c, 2) + 3 * min(n - 1 - c, 2); }
// Fill the code table in LDS: entry cx + 9 cy + 81 cz is the code of a cell
// with those classes (a representative cell c = min(c, 2) on an axis of
// c + 1 + min(n - 1 - c, 2) cells has the same neighbours in the grid).
__device__ inline void rq_code_table(uint32_t *ctab) {
  for (int i = threadIdx.x; i < 729; i += kBlock) {
    const int cl[3] = {i % 9, (i / 9) % 9, i / 81};
    int c[3], n[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      c[ax] = cl[ax] % 3;
      n[ax] = c[ax] + 1 + cl[ax] / 3;
    }
    ctab[i] = code_at<3>(c[0], c[1], c[2], n[0], n[1], n[2]);
  }
  __syncthreads();
}

// The interior planes of a wave: [i0, i1), empty unless the
// row is at least three rows from both y faces.
__device__ inline void rq_split(const Walk &wk, int &i0, int &i1) {
  i0 = i1 = wk.m0;
  if (wk.row >= 3 && wk.row + 4 <= wk.ny) {
    const int a = max(wk.m0, 3), b = min(wk.m1, wk.nm - 3);
    if (a < b) {
      i0 = a;
      i1 = b;
    }
  }
}

template <int W, bool OPL>
__device__ inline void rq_int_march(const Inst &in, const CgPass<float> &cg, const Walk &wk, double (&acc)[4]) {
  using T = float;
  int i0, i1;
  rq_split(wk, i0, i1);
  if (i0 < i1) {  // uniform over the wave
    const int lane = threadIdx.x & 63;
    const T al = cg.al, be = cg.be;
    // weights of this lane's cells: their codes depend on x alone here
    T wc[W][6];
    {
      T wi[6], a[6];
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        wi[d] = (T)in.lut_np1[d][interior_state<3>()];
        a[d] = (T)in.a[d];
      }
      auto lut = [&](int d, int st) { return (T)in.lut_np1[d][st]; };
#pragma unroll
      for (int k = 0; k < W; ++k)
        op_weights<T, OPL>(lut, wi, a, code_at<3>(min(wk.x + k, wk.nx - 1), 3, 3, wk.nx, wk.ny, wk.nz), wc[k]);
    }
    auto opv = [&](const Vec<T, W> &v, const Vec<T, W> &vN, const Vec<T, W> &vS, const Vec<T, W> &vB,
                   const Vec<T, W> &vF) {
      T w[W], e[W];
      xnb0<T, W>(v, lane, w, e);
      Vec<T, W> o;
#pragma unroll
      for (int k = 0; k < W; ++k) o.e[k] = op_w<T, OPL>(wc[k], v.e[k], w[k], e[k], vN.e[k], vS.e[k], vB.e[k], vF.e[k]);
      return o;
    };
    const PI_G T *R = cg.rold, *Pp = cg.pold;
    const int64_t sm = wk.sm, sy = wk.nx;
    auto at = [&](int j) { return wk.base + (int64_t)j * sm; };
    // window at m = i0 (rows y-2 .. y+2 and planes i0-2 .. i0+2 are in the grid)
    Vec<T, W> P0a = ldv<W>(Pp, at(i0)), P0b = ldv<W>(Pp, at(i0 + 1));
    Vec<T, W> Pn0 = ldv<W>(Pp, at(i0 - 1) + sy), Pn1 = ldv<W>(Pp, at(i0) + sy);
    Vec<T, W> Ps0 = ldv<W>(Pp, at(i0 - 1) - sy), Ps1 = ldv<W>(Pp, at(i0) - sy);
    Vec<T, W> Um1, U0, rk0;
    {
      const Vec<T, W> Pm1 = ldv<W>(Pp, at(i0 - 1)), Pm2 = ldv<W>(Pp, at(i0 - 2));
      const Vec<T, W> Rm1 = ldv<W>(R, at(i0 - 1)), R0 = ldv<W>(R, at(i0));
      const Vec<T, W> Am1 = opv(Pm1, Pn0, Ps0, Pm2, P0a);
      const Vec<T, W> A0 = opv(P0a, Pn1, Ps1, Pm1, P0b);
#pragma unroll
      for (int k = 0; k < W; ++k) {
        Um1.e[k] = (Rm1.e[k] - al * Am1.e[k]) + be * Pm1.e[k];
        rk0.e[k] = R0.e[k] - al * A0.e[k];
        U0.e[k] = rk0.e[k] + be * P0a.e[k];
      }
    }
    // inputs of step m, fetched during step m - 1
    struct In {
      Vec<T, W> p2, pn1, ps1, pnn, pss, ry1, rn, rs, d;  // P(y, m+2), P(y+-1, m+1), P(y+-2, m), R(y, m+1), R(y+-1, m), d(y, m)
    };
    auto fetch = [&](int m, In &f) {
      const int64_t c0 = at(m), c1 = at(m + 1);
      f.p2 = ldv<W>(Pp, at(m + 2));
      f.pn1 = ldv<W>(Pp, c1 + sy);
      f.ps1 = ldv<W>(Pp, c1 - sy);
      f.pnn = ldv<W>(Pp, c0 + 2 * sy);
      f.pss = ldv<W>(Pp, c0 - 2 * sy);
      f.ry1 = ldv<W>(R, c1);
      f.rn = ldv<W>(R, c0 + sy);
      f.rs = ldv<W>(R, c0 - sy);
      f.d = cg.rd_d ? ldv_nt<W>(cg.d, c0) : vzero<T, W>();
    };
    In cur, nxt;
    fetch(i0, cur);
    for (int m = i0; m < i1; ++m) {
      if (m + 1 < i1) fetch(m + 1, nxt);  // uniform over the wave
      // A p_{k-1} where p_k is needed: (y, m+1), (y+1, m), (y-1, m)
      const Vec<T, W> Ay1 = opv(P0b, cur.pn1, cur.ps1, P0a, cur.p2);
      const Vec<T, W> An = opv(Pn1, cur.pnn, P0a, Pn0, cur.pn1);
      const Vec<T, W> As = opv(Ps1, P0a, cur.pss, Ps0, cur.ps1);
      Vec<T, W> U1, Un, Us, rk1;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        rk1.e[k] = cur.ry1.e[k] - al * Ay1.e[k];
        U1.e[k] = rk1.e[k] + be * P0b.e[k];
        Un.e[k] = (cur.rn.e[k] - al * An.e[k]) + be * Pn1.e[k];
        Us.e[k] = (cur.rs.e[k] - al * As.e[k]) + be * Ps1.e[k];
      }
      const Vec<T, W> q = opv(U0, Un, Us, Um1, U1);  // q_k = A p_k
      Vec<T, W> dv;
#pragma unroll
      for (int k = 0; k < W; ++k) dv.e[k] = cur.d.e[k] + al * P0a.e[k];
      if (wk.act) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const double r = (double)rk0.e[k], qd = (double)q.e[k];
          acc[0] += (double)U0.e[k] * qd;
          acc[1] += r * qd;
          acc[2] += qd * qd;
          acc[3] += r * r;
        }
        const int64_t c = at(m);
        stv_nt<W>(cg.pnew, c, U0);
        stv_nt<W>(cg.rnew, c, rk0);
        if (cg.wr_d) stv_nt<W>(cg.d, c, dv);
      }
      Um1 = U0;
      U0 = U1;
      rk0 = rk1;
      P0a = P0b;
      P0b = cur.p2;
      Pn0 = Pn1;
      Pn1 = cur.pn1;
      Ps0 = Ps1;
      Ps1 = cur.ps1;
      cur = nxt;
    }
  }
}

// The boundary layers: planes [a, b) of the wave, every operand and code
// checked.
template <int W, bool OPL>
__device__ inline void rq_bnd_march(const Inst &in, const CgPass<float> &cg, const Walk &wk, const float (*lut)[kStates],
                                    const uint32_t *ctab, const float *wi, const float *a, int a0, int a1,
                                    double (&acc)[4]) {
  using T = float;
  if (a0 >= a1) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  const T al = cg.al, be = cg.be;
  const int nm = wk.nm;
  const int64_t sm = wk.sm, sy = wk.nx;
  // rows y +- 1, y +- 2; a row outside the grid reads the wave's own row and is zeroed
  const bool hN1 = wk.row + 1 < wk.ny, hS1 = wk.row > 0, hN2 = wk.row + 2 < wk.ny, hS2 = wk.row > 1;
  const int64_t oN1 = hN1 ? sy : 0, oS1 = hS1 ? -sy : 0, oN2 = hN2 ? 2 * sy : 0, oS2 = hS2 ? -2 * sy : 0;
  const PI_G T *R = cg.rold, *Pp = cg.pold;
  const Vec<T, W> z = vzero<T, W>();
  // plane j, clamped into the grid; planes outside read as 0
  auto cj = [&](int j) { return wk.base + (int64_t)min(max(j, 0), nm - 1) * sm; };
  auto inp = [&](int j) { return j >= 0 && j < nm; };
  auto ldz = [&](const PI_G T *arr, int64_t c, bool ok) { return ok ? ldv<W>(arr, c) : z; };
  // codes from the class table: x class per cell (fixed), y class per row, z class per plane
  int cxk[W];
#pragma unroll
  for (int k = 0; k < W; ++k) cxk[k] = rq_cls(min(wk.x + k, wk.nx - 1), wk.nx);
  auto codes = [&](int j, int row) {
    const int cyz = 9 * rq_cls(min(max(row, 0), wk.ny - 1), wk.ny) + 81 * rq_cls(min(max(j, 0), nm - 1), nm);
    Vec<uint32_t, W> v;
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = ctab[cxk[k] + cyz];
    return v;
  };
  auto tl = [&](int d, int st) { return lut[d][st]; };
  auto opv = [&](const Vec<uint32_t, W> &cd, const Vec<T, W> &v, const Vec<T, W> &vN, const Vec<T, W> &vS,
                 const Vec<T, W> &vB, const Vec<T, W> &vF) {
    T w[W], e[W];
    xnb0<T, W>(v, lane, w, e);
    Vec<T, W> o;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      T wt[6];
      op_weights<T, OPL>(tl, wi, a, cd.e[k], wt);
      o.e[k] = op_w<T, OPL>(wt, v.e[k], w[k], e[k], vN.e[k], vS.e[k], vB.e[k], vF.e[k]);
    }
    return o;
  };
  // p_k = (r - al A p) + be p at in-grid cells, else 0; r_k likewise
  auto pk = [&](bool ok, const Vec<T, W> &r, const Vec<T, W> &Ap, const Vec<T, W> &p, Vec<T, W> &rk) {
    Vec<T, W> u;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      rk.e[k] = ok ? r.e[k] - al * Ap.e[k] : T(0);
      u.e[k] = ok ? rk.e[k] + be * p.e[k] : T(0);
    }
    return u;
  };
  Vec<T, W> P0a = ldz(Pp, cj(a0), true), P0b = ldz(Pp, cj(a0 + 1), inp(a0 + 1));
  Vec<T, W> Pn0 = ldz(Pp, cj(a0 - 1) + oN1, hN1 && inp(a0 - 1)), Pn1 = ldz(Pp, cj(a0) + oN1, hN1);
  Vec<T, W> Ps0 = ldz(Pp, cj(a0 - 1) + oS1, hS1 && inp(a0 - 1)), Ps1 = ldz(Pp, cj(a0) + oS1, hS1);
  Vec<T, W> Um1, U0, rk0, t;
  {
    const Vec<T, W> Pm1 = ldz(Pp, cj(a0 - 1), inp(a0 - 1)), Pm2 = ldz(Pp, cj(a0 - 2), inp(a0 - 2));
    const Vec<T, W> Am1 = opv(codes(a0 - 1, wk.row), Pm1, Pn0, Ps0, Pm2, P0a);
    Um1 = pk(inp(a0 - 1), ldz(R, cj(a0 - 1), inp(a0 - 1)), Am1, Pm1, t);
    const Vec<T, W> A0 = opv(codes(a0, wk.row), P0a, Pn1, Ps1, Pm1, P0b);
    U0 = pk(true, ldz(R, cj(a0), true), A0, P0a, rk0);
  }
  for (int m = a0; m < a1; ++m) {
    const int64_t c0 = cj(m), c1 = cj(m + 1);
    const Vec<T, W> P0c = ldz(Pp, cj(m + 2), inp(m + 2));
    const Vec<T, W> Pn2 = ldz(Pp, c1 + oN1, hN1 && inp(m + 1)), Ps2 = ldz(Pp, c1 + oS1, hS1 && inp(m + 1));
    const Vec<T, W> Pnn = ldz(Pp, c0 + oN2, hN2), Pss = ldz(Pp, c0 + oS2, hS2);
    Vec<T, W> rk1;
    const Vec<T, W> Ay1 = opv(codes(m + 1, wk.row), P0b, Pn2, Ps2, P0a, P0c);
    const Vec<T, W> U1 = pk(inp(m + 1), ldz(R, c1, inp(m + 1)), Ay1, P0b, rk1);
    const Vec<T, W> An = opv(codes(m, wk.row + 1), Pn1, Pnn, P0a, Pn0, Pn2);
    const Vec<T, W> Un = pk(hN1, ldz(R, c0 + oN1, hN1), An, Pn1, t);
    const Vec<T, W> As = opv(codes(m, wk.row - 1), Ps1, P0a, Pss, Ps0, Ps2);
    const Vec<T, W> Us = pk(hS1, ldz(R, c0 + oS1, hS1), As, Ps1, t);
    const Vec<T, W> q = opv(codes(m, wk.row), U0, Un, Us, Um1, U1);
    const Vec<T, W> d = cg.rd_d ? ldv_nt<W>(cg.d, c0) : z;
    Vec<T, W> dv;
#pragma unroll
    for (int k = 0; k < W; ++k) dv.e[k] = d.e[k] + al * P0a.e[k];
    if (wk.act) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const double r = (double)rk0.e[k], qd = (double)q.e[k];
        acc[0] += (double)U0.e[k] * qd;
        acc[1] += r * qd;
        acc[2] += qd * qd;
        acc[3] += r * r;
      }
      stv_nt<W>(cg.pnew, c0, U0);
      stv_nt<W>(cg.rnew, c0, rk0);
      if (cg.wr_d) stv_nt<W>(cg.d, c0, dv);
    }
    Um1 = U0;
    U0 = U1;
    rk0 = rk1;
    P0a = P0b;
    P0b = P0c;
    Pn0 = Pn1;
    Pn1 = Pn2;
    Ps0 = Ps1;
    Ps1 = Ps2;
  }
}

// Boundary-layer task t (rq_ntasks of them) -> wave strip, row and planes
// [a, b): the rows next to the y faces in chunks of kRqChunk planes, then for
// every other row the three planes next to each march face; false past the
// last.
__device__ inline bool rq_task(const Inst &in, int64_t t, int &xs, int &row, int &a, int &b) {
  const int ny = in.ny, nm = in.nm;
  xs = (int)(t % in.nxs);
  t /= in.nxs;
  const bool inner = ny >= 7 && nm >= 7;
  const int nbr = inner ? 6 : ny;
  const int nch = (nm + kRqChunk - 1) / kRqChunk;
  const int64_t nA = (int64_t)nbr * nch;
  if (t < nA) {
    const int i = (int)(t / nch), c = (int)(t % nch);
    row = inner ? (i < 3 ? i : ny - 6 + i) : i;
    a = c * kRqChunk;
    b = min(nm, a + kRqChunk);
    return true;
  }
  t -= nA;
  if (!inner || t >= 2 * (int64_t)(ny - 6)) return false;
  row = 3 + (int)(t / 2);
  a = (t % 2 == 0) ? 0 : nm - 3;
  b = a + 3;
  return true;
}

// Place a wave on its window of strip xs of row `row` (rq_window): lanes of
// a single-strip row past its end address the row's last cells and own
// nothing; in a split row every lane is inside the grid and owns its cells
// when they lie in the strip's owned range.
template <int W>
__device__ inline void rq_place(const Inst &in, int xs, int row, Walk &k) {
  int start, own0, own1;
  rq_window(in.nx, in.nxs, xs, start, own0, own1);
  k.x = start + (threadIdx.x & 63) * W;
  k.act = k.x >= own0 && k.x < own1;
  k.base = (int64_t)min(k.x, in.nx - W) + (int64_t)row * in.srow;
}

// A wave's view of a task: strip xs of row `row`, planes [m0, m1).
template <int W>
__device__ inline Walk rq_walk(const Inst &in, int xs, int row, int m0, int m1) {
  Walk k;
  k.sm = in.sm;
  k.code = gp<uint32_t>(in.code);
  k.nm = in.nm;
  k.nx = in.nx;
  k.ny = in.ny;
  k.nz = in.nz;
  k.m0 = m0;
  k.m1 = m1;
  k.row = row;
  rq_place<W>(in, xs, row, k);
  return k;
}

// The interior walk of block lb: the generic walk (make_walk) with the
// wave moved to its window.
template <int W>
__device__ inline Walk rq_iwalk(const Inst &in, int lb) {
  Walk k = make_walk<W>(in, lb);
  const int64_t w = (int64_t)lb * kWavesPerBlock + (threadIdx.x >> 6);
  if (w < in.nwaves && in.nxs > 1) rq_place<W>(in, (int)(w % in.nxs), k.row, k);
  return k;
}

// One CG pass.  Blocks 0 .. nblocks-1 of the instance march the interior
// planes of their strips and segments; the blocks after them (first in the
// launch's table, so dispatched first) take one boundary-layer task per wave.
template <int W, bool OPL>
__global__ __launch_bounds__(kBlock) void k_cg_rq(const BlockEnt *tab, const Inst *__restrict__ insts,
                                                 State *__restrict__ sts, double *part, int kpass) {
  using T = float;
  PI_PROLOGUE
  const CgPass<T> cg = cg_pass<T>(in, st, part, e.lb, kpass);
  if (cg.skip) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (e.lb < in.nblocks) {  // uniform over the block
    rq_int_march<W, OPL>(in, cg, rq_iwalk<W>(in, e.lb), acc);
  } else {
    __shared__ T lut[6][kStates];
    __shared__ uint32_t ctab[729];
    load_lut<T>(in.lut_np1, lut);
    rq_code_table(ctab);
    T wi[6], a[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      wi[d] = (T)in.lut_np1[d][interior_state<3>()];
      a[d] = (T)in.a[d];
    }
    int xs, row, a0, a1;
    const int64_t t = (int64_t)(e.lb - in.nblocks) * kWavesPerBlock + (threadIdx.x >> 6);
    if (rq_task(in, t, xs, row, a0, a1))  // uniform over the wave
      rq_bnd_march<W, OPL>(in, cg, rq_walk<W>(in, xs, row, a0, a1), lut, ctab, wi, a, a0, a1, acc);
  }
  publish<4>(in, cg_part(in, part, kpass), e.lb, acc);
}

// ---------------------------------------------------------------------------
// inner BiCGStab on M delta = r (shadow residual = the outer residual)
// ---------------------------------------------------------------------------
// phase 1: p <- r + beta (p - omega v) (p <- r first), v' <- M p (into q), rhat.v'
template <typename T, int ND, int W, bool GEN>
__global__ __launch_bounds__(kBlock) void k_bicg_spmv_p(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                        double *part) {
  PI_PROLOGUE
  if (skip_inner(in, st)) return;
  __shared__ T lut[6][kStates];
  load_lut<T>(in.lut_np1, lut);
  T wi[6];  // interior weights, as the LUT holds them
#pragma unroll
  for (int d = 0; d < 6; ++d) wi[d] = (T)in.lut_np1[d][interior_state<ND>()];
  const Walk wk = make_walk<W>(in, e.lb);
  const T beta = (T)st->beta, omega = (T)st->omega;
  const int pc = st->pcur;
  const PI_G T *pold = gp<T>(in.p[pc]);
  PI_G T *pnew = gp<T>(in.p[pc ^ 1]);
  const PI_G T *res = gp<T>(in.res);
  const PI_G T *v = gp<T>(in.bs[1]);
  const PI_G T *rhat = gp<T>(in.bs[0]);
  PI_G T *vnew = gp<T>(in.q);
  const int bits = dir_bits(ND);
  double acc[1] = {0.0};
  struct Out {
    T p, v;
  };
  auto load = [&](int64_t c) {
    const Vec<T, W> r = ldv<W>(res, c), p = ldv<W>(pold, c), vv = ldv<W>(v, c);
    Vec<T, W> o;
#pragma unroll
    for (int k = 0; k < W; ++k) o.e[k] = r.e[k] + beta * (p.e[k] - omega * vv.e[k]);
    return o;
  };
  auto load1 = [&](int64_t c) -> T { return res[c] + beta * (pold[c] - omega * v[c]); };
  auto aux = [&](int64_t c) { return ldv<W>(rhat, c); };
  auto body = [&](int64_t, const Cell<T, T> &pl, T vW, T vE, T vP, T vN) -> Out {
    const uint32_t cd = pl.code;
    const T vC = pl.v;
    if (!(cd & kValidBit)) return Out{T(0), T(0)};
    const T s = apply_m<T, ND>(lut, wi, cd, bits, vC, vW, vE, pl.vN, pl.vS, vP, vN);
    acc[0] += (double)pl.aux * (double)s;
    return Out{vC, s};
  };
  auto store = [&](int64_t c, const Out (&o)[W]) {
    Vec<T, W> pv, vv;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      pv.e[k] = o[k].p;
      vv.e[k] = o[k].v;
    }
    stv<W>(pnew, c, pv);
    stv<W>(vnew, c, vv);
  };
  march<ND, W, GEN, T, T, Out>(wk, load, load1, aux, body, store);
  publish<1>(in, part, e.lb, acc);
}

// phase 2: v <- v', s <- r - alpha v, t <- M s, t.s and t.t
template <typename T, int ND, int W, bool GEN>
__global__ __launch_bounds__(kBlock) void k_bicg_spmv_s(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                        double *part) {
  PI_PROLOGUE
  if (skip_inner(in, st)) return;
  __shared__ T lut[6][kStates];
  load_lut<T>(in.lut_np1, lut);
  T wi[6];  // interior weights, as the LUT holds them
#pragma unroll
  for (int d = 0; d < 6; ++d) wi[d] = (T)in.lut_np1[d][interior_state<ND>()];
  const Walk wk = make_walk<W>(in, e.lb);
  const T alpha = (T)st->alpha;
  const PI_G T *res = gp<T>(in.res);
  const PI_G T *vnew = gp<T>(in.q);
  PI_G T *v = gp<T>(in.bs[1]);
  PI_G T *s_out = gp<T>(in.bs[2]);
  PI_G T *t_out = gp<T>(in.bs[3]);
  const int bits = dir_bits(ND);
  double acc[2] = {0.0, 0.0};
  struct Out {
    T v, s, t;
  };
  auto load = [&](int64_t c) {
    const Vec<T, W> r = ldv<W>(res, c), vv = ldv<W>(vnew, c);
    Vec<T, W> o;
#pragma unroll
    for (int k = 0; k < W; ++k) o.e[k] = r.e[k] - alpha * vv.e[k];
    return o;
  };
  auto load1 = [&](int64_t c) -> T { return res[c] - alpha * vnew[c]; };
  auto aux = [&](int64_t c) { return ldv<W>(vnew, c); };
  auto body = [&](int64_t, const Cell<T, T> &pl, T vW, T vE, T vP, T vN) -> Out {
    const uint32_t cd = pl.code;
    const T vC = pl.v;
    const T vv = pl.aux;
    if (!(cd & kValidBit)) return Out{vv, T(0), T(0)};
    const T s = apply_m<T, ND>(lut, wi, cd, bits, vC, vW, vE, pl.vN, pl.vS, vP, vN);
    acc[0] += (double)s * (double)vC;
    acc[1] += (double)s * (double)s;
    return Out{vv, vC, s};
  };
  auto store = [&](int64_t c, const Out (&o)[W]) {
    Vec<T, W> a, b, d;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      a.e[k] = o[k].v;
      b.e[k] = o[k].s;
      d.e[k] = o[k].t;
    }
    stv<W>(v, c, a);
    stv<W>(s_out, c, b);
    stv<W>(t_out, c, d);
  };
  march<ND, W, GEN, T, T, Out>(wk, load, load1, aux, body, store);
  publish<2>(in, part, e.lb, acc);
}

// phase 3: delta <- delta + alpha p + omega s, r <- s - omega t, rhat.r
template <typename T>
struct BicgUpdate {
  static constexpr int E = 16 / sizeof(T);
  static constexpr int U = 1;
  const PI_G T *p, *s, *t, *rhat;
  PI_G T *res, *d;
  T alpha, omega;
  bool first;
  double acc;
  Vec<T, E> pv[U], sv[U], tv[U], hv[U], dv[U];
  __device__ void load(int64_t c, int u) {
    pv[u] = ldv<E>(p, c);
    sv[u] = ldv<E>(s, c);
    tv[u] = ldv<E>(t, c);
    hv[u] = ldv<E>(rhat, c);
    dv[u] = first ? vzero<T, E>() : ldv<E>(d, c);
  }
  __device__ void apply(int64_t c, int u) {
    Vec<T, E> dn, r;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      dn.e[k] = dv[u].e[k] + (alpha * pv[u].e[k] + omega * sv[u].e[k]);
      r.e[k] = sv[u].e[k] - omega * tv[u].e[k];
      acc += (double)hv[u].e[k] * (double)r.e[k];
    }
    stv<E>(d, c, dn);
    stv<E>(res, c, r);
  }
  __device__ void one(int64_t c) {
    d[c] = (first ? T(0) : d[c]) + (alpha * p[c] + omega * s[c]);
    const T r = s[c] - omega * t[c];
    res[c] = r;
    acc += (double)rhat[c] * (double)r;
  }
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_bicg_update(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                        double *part) {
  PI_PROLOGUE
  if (skip_inner(in, st)) return;
  int64_t beg, end;
  linear_range(in, e.lb, beg, end);
  BicgUpdate<T> f;
  f.p = gp<T>(in.p[st->pcur]);
  f.s = gp<T>(in.bs[2]);
  f.t = gp<T>(in.bs[3]);
  f.rhat = gp<T>(in.bs[0]);
  f.res = gp<T>(in.res);
  f.d = gp<T>(in.d);
  f.alpha = (T)st->alpha;
  f.omega = (T)st->omega;
  f.first = st->inner == 0;
  f.acc = 0.0;
  stream_linear<BicgUpdate<T>::E, BicgUpdate<T>::U>(beg, end, f);
  double acc[1] = {f.acc};
  publish<1>(in, part, e.lb, acc);
}

// copy of the outer residual used as BiCGStab's shadow vector
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy_res(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                     double *part) {
  PI_PROLOGUE
  if (skip_outer(st)) return;
  int64_t beg, end;
  linear_range(in, e.lb, beg, end);
  const T *res = (const T *)in.res;
  T *rhat = (T *)in.bs[0];
  for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) rhat[c] = res[c];
}

// ---------------------------------------------------------------------------
// gauge: remove the mean of P over every connected group of data cells
// ---------------------------------------------------------------------------
// Single group: fixed-order block partials.  Several groups: one block per
// segment of the group-sorted cell list (fixed order inside), then one thread
// per group sums its segments in order -- deterministic in both cases.
__global__ __launch_bounds__(kBlock) void k_gauge_sum(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                      double *part) {
  PI_PROLOGUE
  const double *P = in.P[st->Pcur];
  if (in.ncomp > 1) {
    __shared__ double lds[kWavesPerBlock * 4];
    for (int sg = e.lb; sg < in.nseg_g; sg += in.nblocks) {
      double v[1] = {0.0};
      for (int i = in.seg_begin[sg] + threadIdx.x; i < in.seg_begin[sg + 1]; i += kBlock) v[0] += P[in.comp_order[i]];
      block_sum<1>(v, lds);
      if (threadIdx.x == 0) in.seg_sum[sg] = v[0];
    }
    return;
  }
  int64_t beg, end;
  linear_range(in, e.lb, beg, end);
  const uint32_t *code = in.code;
  double acc[1] = {0.0};
  for (int64_t c = beg + threadIdx.x; c < end; c += kBlock)
    if (code[c] & kValidBit) acc[0] += P[c];
  publish<1>(in, part, e.lb, acc);
}

__global__ __launch_bounds__(kBlock) void k_gauge_groups(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                         double *part) {
  PI_PROLOGUE
  if (in.ncomp <= 1) return;
  for (int k = e.lb * kBlock + threadIdx.x; k < in.ncomp; k += in.nblocks * kBlock) {
    double s = 0.0;
    for (int sg = in.comp_seg[k]; sg < in.comp_seg[k + 1]; ++sg) s += in.seg_sum[sg];
    in.comp_sum[k] = s * in.comp_inv_count[k];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gauge_apply(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                        double *part) {
  PI_PROLOGUE
  int64_t beg, end;
  linear_range(in, e.lb, beg, end);
  const double *P = in.P[st->Pcur];
  const uint32_t *code = in.code;
  T *out = (T *)in.Pout;
  const bool zero = st->normS2 == 0.0;
  const double mean1 = st->red[0] * in.inv_nvalid;
  for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
    T v;
    if (code[c] & kValidBit) {
      if (zero) {
        v = T(0);
      } else if (in.ncomp > 1) {
        v = (T)(P[c] - in.comp_sum[in.label[c]]);
      } else {
        v = (T)(P[c] - mean1);
      }
    } else {
      v = (T)NAN;
    }
    out[c] = v;
  }
}

// ---------------------------------------------------------------------------
// finalize: one block per instance sums the partials of the kernel that just
// ran (fixed order) and updates the instance's scalars
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_finalize(const Inst *__restrict__ insts, State *__restrict__ sts, const double *part, int kind,
                                                    int kpass) {
  const Inst &in = insts[blockIdx.x];
  State *st = sts + blockIdx.x;
  switch (kind) {
    case K_SOURCE: break;
    case K_OUTER:
    case K_COPY_RES:
      if (skip_outer(st)) return;
      break;
    case K_GAUGE_SUM:
      if (in.ncomp > 1) return;
      break;
    case K_CG_STEP:
      // instances whose passes sum the partials themselves, and passes that
      // did not run
      if (in.cg_inline || st->done != 0 || kpass >= in.inner_iters || st->stop_at <= kpass) return;
      part += (int64_t)(1 + (kpass & 1)) * in.part_stride * 4;
      break;
    default:
      if (skip_inner(in, st)) return;
  }
  __shared__ double lds[kWavesPerBlock * 4];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  // slots are 32 bytes: load them as double2 pairs, several rounds in flight
  const double2 *slots = reinterpret_cast<const double2 *>(part + (int64_t)in.part_base * 4);
  const int nslots = kind == K_CG_STEP ? in.cg_slots : in.nblocks;
#pragma unroll 8
  for (int i = threadIdx.x; i < nslots; i += kBlock) {
    const double2 a = slots[2 * i], b = slots[2 * i + 1];
    s[0] += a.x;
    s[1] += a.y;
    s[2] += b.x;
    s[3] += b.y;
  }
  block_sum<4>(s, lds);
  if (threadIdx.x != 0) return;
  switch (kind) {
    case K_SOURCE:
      st->normS2 = s[0];
      if (st->nonfinite) {
        st->done = 1;
        st->status = 3;  // PI_ERR_NONFINITE
      }
      break;
    case K_OUTER: {
      const bool hd = st->have_delta != 0;
      // CG passes of the inner solve that just ended (BiCGStab counts its own)
      if (hd && !in.bicg) st->inner_total += min(st->stop_at, in.inner_iters);
      const double epsR = st->normS2 > 0.0 ? sqrt(s[0] / st->normS2) : 0.0;
      st->epsR = epsR;
      if (hd) st->epsP = s[3] > 0.0 ? sqrt(s[2] / s[3]) : 0.0;
      st->Pcur ^= 1;
      if (!isfinite(epsR)) {
        st->done = 1;
        st->status = 5;  // PI_ERR_DIVERGED
      } else if (epsR <= in.tol) {
        st->done = 1;
        st->status = 0;
      } else if (st->outer >= in.max_iter) {
        st->done = 1;
        st->status = 4;  // PI_ERR_NOT_CONVERGED
      } else {
        st->outer += 1;
        st->rr = s[1];
        st->rr0 = s[1];
        st->inner = 0;
        st->stop_at = kNoStop;
        st->dvalid = 0;
        st->first = 1;
        st->beta = 0.0;  // the first search direction is the residual itself
        st->have_delta = 1;
        // BiCGStab restarts with the new residual as its shadow vector
        st->rho = s[1];
        st->alpha = 1.0;
        st->omega = 1.0;
      }
      break;
    }
    case K_CG_STEP: {
      const CgScalars cs = cg_scalars(in, st, s);
      st->alpha = cs.al;
      st->beta = cs.be;
      if (cs.stop) st->stop_at = kpass + 1;
      break;
    }
    case K_BICG_P:
      st->alpha = s[0] != 0.0 ? st->rho / s[0] : 0.0;
      st->pcur ^= 1;
      st->first = 0;
      break;
    case K_BICG_S:
      st->omega = s[1] != 0.0 ? s[0] / s[1] : 0.0;
      break;
    case K_BICG_UPDATE: {
      const double rho_new = s[0];
      st->beta = (st->rho != 0.0 && st->omega != 0.0) ? (rho_new / st->rho) * (st->alpha / st->omega) : 0.0;
      st->rho = rho_new;
      st->dvalid = 1;  // every BiCGStab update writes the correction
      st->inner += 1;
      st->inner_total += 1;
      break;
    }
    case K_GAUGE_SUM:
      st->red[0] = s[0];
      break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// plain operator applies (pi_apply): y = M x, N x or (M - N) x
// ---------------------------------------------------------------------------
template <typename T, int ND, int W, bool GEN>
__global__ __launch_bounds__(kBlock) void k_apply(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts, double *part,
                                                  int op, const T *x_, T *y_) {
  PI_PROLOGUE
  const PI_G T *x = gp<T>(x_);
  PI_G T *y = gp<T>(y_);
  __shared__ T lut_a[6][kStates];
  __shared__ T lut_b[6][kStates];
  load_lut<T>(in.lut_np1, lut_a);
  load_lut<T>(in.lut_n, lut_b);
  T wi[6];  // interior weights of [W^{n+1}], as the LUT holds them
#pragma unroll
  for (int d = 0; d < 6; ++d) wi[d] = (T)in.lut_np1[d][interior_state<ND>()];
  const Walk wk = make_walk<W>(in, e.lb);
  T a[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) a[d] = (T)in.a[d];
  const int bits = dir_bits(ND);
  auto load = [&](int64_t c) { return ldv<W>(x, c); };
  auto load1 = [&](int64_t c) -> T { return x[c]; };
  struct None {};
  auto extra = [](int64_t) { return None{}; };
  auto cookv = [](const Vec<T, W> &v) { return v; };
  auto cook1 = [](T v) { return v; };
  auto cooka = [](const Vec<T, W> &, None) { return Vec<int, W>{}; };
  auto body = [&](int64_t, const Cell<T, int> &pl, T vW, T vE, T vP, T vN) -> T {
    const uint32_t cd = pl.code;
    const T vC = pl.v;
    if (!(cd & kValidBit)) return T(0);
    T nb[6];
    nb[DE] = vE;
    nb[DW] = vW;
    if (ND == 3) {
      nb[DN] = pl.vN;
      nb[DS] = pl.vS;
      nb[DF] = vN;
      nb[DB] = vP;
    } else {
      nb[DN] = vN;
      nb[DS] = vP;
    }
    T s;
    if (op == 0) {  // M = I - W^{n+1}, as the CG pass applies it
      s = apply_m<T, ND>(lut_a, wi, cd, bits, vC, vW, vE, pl.vN, pl.vS, vP, vN);
    } else if (op == 1) {  // N = W^n with diagonal w_C^n
      T wc = T(1);
      s = T(0);
      for (int d = 0; d < 2 * ND; ++d) {
        const int t = dstate(cd, d, bits);
        if (t) {
          s += lut_b[d][t] * nb[d];
          wc -= a[d];
        }
      }
      s += wc * vC;
    } else {  // M - N, as the variant's CG pass applies it
      s = apply_l<T, ND>(a, cd, bits, vC, vW, vE, pl.vN, pl.vS, vP, vN);
    }
    return s;
  };
  auto store = [&](int64_t c, const T (&o)[W]) {
    Vec<T, W> v;
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = o[k];
    stv<W>(y, c, v);
  };
  march2<ND, W, GEN, T, int, T>(wk, load, load1, extra, cookv, cook1, cooka, body, store);
}


// ---------------------------------------------------------------------------
// the 2-D cell-centred scheme: 9-point stencils over contiguous cell ranges
// ---------------------------------------------------------------------------
// The ring code of a cell tells which of the 24 cells within two steps hold
// data.  The source (once per solve) and pi_apply take contiguous cell
// ranges and read the 8 neighbours through L1/L2; the outer and CG kernels
// below march along y.

// offset of neighbour j in cells
__device__ inline int64_t cc_off(const Inst &in, int j) { return (int64_t)cc_dx(j) + (int64_t)cc_dy(j) * in.nx; }

// w_J^{n+1} (np1) and w_J^n (n) of the 8 neighbours from the ray pieces: a
// piece counts when J holds data, towards n+1 when K holds data as well
__device__ inline void cc_weights(const Inst &in, uint32_t cd, double (&np1)[8], double (&n)[8]) {
#pragma unroll
  for (int j = 0; j < 8; ++j) np1[j] = n[j] = 0.0;
  cc_pieces([&](int J, int jb, int kb, int maj, int mi) {
    const double m = in.cc_m[maj][mi];
    if ((cd >> jb) & 1u) {
      if ((cd >> kb) & 1u) np1[J] += m;
      else n[J] += m;
    }
  });
}

__device__ inline bool cc_has(uint32_t cd, int j) { return (cd >> cc_bit(cc_dx(j), cc_dy(j))) & 1u; }

// S_C = - sum_J Delta_J . (w_J^{n+1} + w_J^n) (f(J) + f(C)) / 2 over
// neighbours J with data (the sum of the two weights is the direction's
// total a_J), FP64
template <typename T>
__global__ __launch_bounds__(kBlock) void k_source_cc(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                     double *part) {
  PI_PROLOGUE
  int64_t beg, end;
  linear_range(in, e.lb, beg, end);
  const T *gx = (const T *)in.g[0], *gy = (const T *)in.g[1];
  T *S = (T *)in.S;
  double *S64 = in.S64;
  const uint32_t *code = in.code;
  double wx[8], wy[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    wx[j] = -0.5 * in.cc_a[j] * in.cc_step[j][0];
    wy[j] = -0.5 * in.cc_a[j] * in.cc_step[j][1];
  }
  double acc[1] = {0.0};
  int bad = 0;
  for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
    const uint32_t cd = code[c];
    double s = 0.0;
    if (cd & kValidBit) {
      const double fx = (double)gx[c], fy = (double)gy[c];
      if (!isfinite(fx) || !isfinite(fy)) bad = 1;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (!cc_has(cd, j)) continue;
        const int64_t q = c + cc_off(in, j);
        if (cc_dx(j) != 0) s += wx[j] * ((double)gx[q] + fx);
        if (cc_dy(j) != 0) s += wy[j] * ((double)gy[q] + fy);
      }
    }
    S64[c] = s;
    if (S) S[c] = (T)s;
    acc[0] += s * s;
  }
  if (bad) atomicOr(&st->nonfinite, 1);
  publish<1>(in, part, e.lb, acc);
}

// The outer and CG kernels march like the face-crossing ones: a wave owns 64
// consecutive cells of a row and walks its segment of rows.  Rows y-1, y,
// y+1 of the operand sit in registers; the x neighbours of all three rows
// come from adjacent lanes, and at the strip ends from one extra value per
// row (lane 0: west, lane 63: east).  Row y+1 is fetched before row y is
// computed.
template <int W, typename V>
struct CcRow {
  Vec<V, W> v;
  V edge;
};

// x neighbours of a row's W cells: inside the lane, from the adjacent
// lanes across lane boundaries, from the edge value at the strip ends.
// Selects, not conditional stores: written through references, edge cases
// merge into one store to a lane-chosen address, which puts the values in
// scratch memory.
template <int W, typename V>
__device__ inline void cc_sides(const CcRow<W, V> &r, int lane, V (&l)[W], V (&rt)[W]) {
  const V up = __shfl_up(r.v.e[W - 1], 1, kWave);
  const V dn = __shfl_down(r.v.e[0], 1, kWave);
  const V l0 = lane == 0 ? r.edge : up;
  const V rw = lane == kWave - 1 ? r.edge : dn;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    l[k] = k == 0 ? l0 : r.v.e[k > 0 ? k - 1 : 0];
    rt[k] = k == W - 1 ? rw : r.v.e[k + 1 < W ? k + 1 : 0];
  }
}

//   load(c) -> Vec<V, W>   operand at cells c .. c+W-1;  load1(c) -> V  one cell
//   aux(c)  -> Vec<A, W>   extra input of the cells, fetched with the operand one row ahead
//   body(c, code, centre, nb[8], aux) -> Out;  store(c, const Out (&)[W])
template <int W, typename V, typename A, typename Out, typename Load, typename Load1, typename Aux, typename Body,
          typename Store>
__device__ inline void march_cc(const Walk &wk, Load load, Load1 load1, Aux aux, Body body, Store store) {
  if (wk.m1 <= wk.m0) return;  // uniform over the wave
  const int lane = threadIdx.x & 63;
  const bool edgeW = lane == 0 && wk.x > 0, edgeE = lane == kWave - 1 && wk.x + W < wk.nx;
  // a neighbour that does not exist reads the cell itself and is zeroed
  const int64_t offE = edgeW ? -1 : edgeE ? W : 0;
  const bool hasEdge = edgeW || edgeE;
  const PI_G uint32_t *code = wk.code;
  auto fetch = [&](int64_t c) {
    CcRow<W, V> r;
    r.v = load(c);
    const V e = load1(c + offE);
    r.edge = hasEdge ? e : V(0);
    return r;
  };
  auto none = [] {
    CcRow<W, V> r;
    r.v = vzero<V, W>();
    r.edge = V(0);
    return r;
  };
  const int64_t sm = wk.sm;
  int64_t c = wk.base + (int64_t)wk.m0 * sm;
  CcRow<W, V> prev = wk.m0 > 0 ? fetch(c - sm) : none();
  CcRow<W, V> cur = fetch(c);
  Vec<uint32_t, W> cd = ldv<W>(code, c);
  Vec<A, W> ax = aux(c);
  for (int m = wk.m0; m < wk.m1; ++m, c += sm) {
    const bool more = m + 1 < wk.nm;  // uniform over the wave
    const bool own = m + 1 < wk.m1;   // the next row is this wave's too
    const CcRow<W, V> nxt = more ? fetch(c + sm) : none();
    Vec<uint32_t, W> cdn;
    Vec<A, W> axn;
    if (own) {
      cdn = ldv<W>(code, c + sm);
      axn = aux(c + sm);
    }
    V lp[W], rp[W], lc[W], rc[W], ln[W], rn[W];
    cc_sides<W, V>(prev, lane, lp, rp);
    cc_sides<W, V>(cur, lane, lc, rc);
    cc_sides<W, V>(nxt, lane, ln, rn);
    // lanes past the grid only serve the shuffles
    if (wk.act) {
      Out o[W];
#pragma unroll
      for (int k = 0; k < W; ++k) {
        V nb[8];
        nb[cc_dir(1, 0)] = rc[k];
        nb[cc_dir(-1, 0)] = lc[k];
        nb[cc_dir(0, 1)] = nxt.v.e[k];
        nb[cc_dir(0, -1)] = prev.v.e[k];
        nb[cc_dir(1, 1)] = rn[k];
        nb[cc_dir(-1, 1)] = ln[k];
        nb[cc_dir(1, -1)] = rp[k];
        nb[cc_dir(-1, -1)] = lp[k];
        o[k] = body(c + k, cd.e[k], cur.v.e[k], nb, ax.e[k]);
      }
      store(c, o);
    }
    prev = cur;
    cur = nxt;
    cd = cdn;
    ax = axn;
  }
}

// P' = P + delta (the pending last CG step folded in as in k_outer),
// r = S - (M - N) P' with (M - N) P' = sum_J a_J (P'_C - P'_J)
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_outer_cc(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                    double *part) {
  PI_PROLOGUE
  if (skip_outer(st)) return;
  const Walk wk = make_walk<W>(in, e.lb);
  const int cur = st->Pcur;
  const PI_G double *Pold = gp<double>(in.P[cur]);
  PI_G double *Pnew = gp<double>(in.P[cur ^ 1]);
  const Pending<T> pd = pending<T>(in, st, part);
  const T at = pd.at;
  const PI_G T *pt = pd.pt;
  const PI_G T *dl = gp<T>(in.d);
  const bool use_d = pd.use_d;
  const PI_G double *S = gp<double>(in.S64);
  PI_G T *res = gp<T>(in.res);
  double a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = in.cc_a[j];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  struct Out {
    double p, r;
  };
  struct Aux {
    double S, d;
  };
  auto delta = [&](int64_t c) {
    const Vec<T, W> d = use_d ? ldv<W>(dl, c) : vzero<T, W>(), p = ldv<W>(pt, c);
    Vec<T, W> v;
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = d.e[k] + at * p.e[k];
    return v;
  };
  auto load = [&](int64_t c) {
    const Vec<double, W> P = ldv<W>(Pold, c);
    const Vec<T, W> d = delta(c);
    Vec<double, W> v;
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = P.e[k] + (double)d.e[k];
    return v;
  };
  auto load1 = [&](int64_t c) -> double { return Pold[c] + (double)((use_d ? dl[c] : T(0)) + at * pt[c]); };
  auto aux = [&](int64_t c) {
    const Vec<double, W> s = ldv<W>(S, c);
    const Vec<T, W> d = delta(c);
    Vec<Aux, W> x;
#pragma unroll
    for (int k = 0; k < W; ++k) x.e[k] = Aux{s.e[k], (double)d.e[k]};
    return x;
  };
  auto body = [&](int64_t, uint32_t cd, double vC, const double (&nb)[8], const Aux &ax) -> Out {
    if (!(cd & kValidBit)) return Out{0.0, 0.0};
    double Lp = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (cc_has(cd, j)) Lp += a[j] * (vC - nb[j]);
    const double r = ax.S - Lp;
    const double rt = (double)(T)r;
    acc[0] += r * r;
    acc[1] += rt * rt;
    acc[2] += ax.d * ax.d;
    acc[3] += vC * vC;
    return Out{vC, r};
  };
  auto store = [&](int64_t c, const Out (&o)[W]) {
    Vec<double, W> p;
    Vec<T, W> r;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      p.e[k] = o[k].p;
      r.e[k] = (T)o[k].r;
    }
    stv<W>(Pnew, c, p);
    stv<W>(res, c, r);
  };
  march_cc<W, double, Aux, Out>(wk, load, load1, aux, body, store);
  publish<4>(in, part, e.lb, acc);
}

// One inner CG iteration with the previous one's update folded in, as
// k_cg_step, for the cell-centred scheme.
template <typename T, int W, bool FIRST>
__device__ __forceinline__ void cg_step_cc_body(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts, double *part,
                                                int kpass) {
  PI_PROLOGUE
  const CgPass<T> cg = cg_pass<T>(in, st, part, e.lb, kpass);
  if (cg.skip) return;
  const Walk wk = make_walk<W>(in, e.lb);
  const bool opL = in.inner_op != 0;
  T a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = (T)in.cc_a[j];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  struct Out {
    T p, q, r, d;
  };
  struct Aux {
    T r, d;
  };
  auto load = [&](int64_t c) {
    const Vec<T, W> r = ldv<W>(cg.rold, c), q = ldv<W>(cg.qold, c), p = ldv<W>(cg.pold, c);
    Vec<T, W> v;
#pragma unroll
    for (int k = 0; k < W; ++k) v.e[k] = (r.e[k] - cg.al * q.e[k]) + cg.be * p.e[k];
    return v;
  };
  auto load1 = [&](int64_t o) -> T { return (cg.rold[o] - cg.al * cg.qold[o]) + cg.be * cg.pold[o]; };
  auto aux = [&](int64_t c) {
    const Vec<T, W> r = ldv<W>(cg.rold, c), q = ldv<W>(cg.qold, c), p = ldv<W>(cg.pold, c);
    const Vec<T, W> d = cg.rd_d ? ldv<W>(cg.d, c) : vzero<T, W>();
    Vec<Aux, W> x;
#pragma unroll
    for (int k = 0; k < W; ++k) x.e[k] = Aux{r.e[k] - cg.al * q.e[k], d.e[k] + cg.al * p.e[k]};
    return x;
  };
  auto body = [&](int64_t, uint32_t cd, T pC, const T (&nb)[8], const Aux &ax) -> Out {
    if (!(cd & kValidBit)) return Out{T(0), T(0), T(0), T(0)};
    T s;
    if (opL) {
      s = T(0);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (cc_has(cd, j)) s += a[j] * (pC - nb[j]);
    } else if ((cd & kCcRing) == kCcRing) {
      s = pC;  // every cell within two steps holds data: w^{n+1} = a
#pragma unroll
      for (int j = 0; j < 8; ++j) s -= a[j] * nb[j];
    } else {
      double np1[8], wn[8];
      cc_weights(in, cd, np1, wn);
      s = pC;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (cc_has(cd, j)) s -= (T)np1[j] * nb[j];
    }
    const double r = (double)ax.r, q = (double)s;
    acc[0] += (double)pC * q;
    acc[1] += r * q;
    acc[2] += q * q;
    acc[3] += r * r;
    return Out{pC, s, ax.r, ax.d};
  };
  auto store = [&](int64_t c, const Out (&o)[W]) {
    Vec<T, W> pv, qv, rv, dv;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      pv.e[k] = o[k].p;
      qv.e[k] = o[k].q;
      rv.e[k] = o[k].r;
      dv.e[k] = o[k].d;
    }
    stv_nt<W>(cg.pnew, c, pv);
    stv_nt<W>(cg.qnew, c, qv);
    stv_nt<W>(cg.rnew, c, rv);
    if (cg.wr_d) stv_nt<W>(cg.d, c, dv);
  };
  if constexpr (FIRST) {
    // p_0 = r_0: only the residual is read; p and q are written
    auto load0 = [&](int64_t c) { return ldv<W>(cg.rold, c); };
    auto load01 = [&](int64_t o) -> T { return cg.rold[o]; };
    auto aux0 = [&](int64_t c) {
      const Vec<T, W> r = ldv<W>(cg.rold, c);
      Vec<Aux, W> x;
#pragma unroll
      for (int k = 0; k < W; ++k) x.e[k] = Aux{r.e[k], T(0)};
      return x;
    };
    auto store0 = [&](int64_t c, const Out (&o)[W]) {
      Vec<T, W> pv, qv;
#pragma unroll
      for (int k = 0; k < W; ++k) {
        pv.e[k] = o[k].p;
        qv.e[k] = o[k].q;
      }
      stv<W>(cg.pnew, c, pv);
      stv<W>(cg.qnew, c, qv);
    };
    march_cc<W, T, Aux, Out>(wk, load0, load01, aux0, body, store0);
  } else {
    march_cc<W, T, Aux, Out>(wk, load, load1, aux, body, store);
  }
  publish<4>(in, cg_part(in, part, kpass), e.lb, acc);
}

template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_cg_first_cc(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                       double *part, int kpass) {
  cg_step_cc_body<T, W, true>(tab, insts, sts, part, kpass);
}
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_cg_step_cc(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                      double *part, int kpass) {
  cg_step_cc_body<T, W, false>(tab, insts, sts, part, kpass);
}

// y = M x, N x or (M - N) x for pi_apply
template <typename T, int W>  // W: the plan's lane width; this kernel takes contiguous ranges
__global__ __launch_bounds__(kBlock) void k_apply_cc(const BlockEnt *tab, const Inst *__restrict__ insts, State *__restrict__ sts,
                                                    double *part, int op, const T *x, T *y) {
  PI_PROLOGUE
  int64_t beg, end;
  linear_range(in, e.lb, beg, end);
  const uint32_t *code = in.code;
  for (int64_t c = beg + threadIdx.x; c < end; c += kBlock) {
    const uint32_t cd = code[c];
    if (!(cd & kValidBit)) {
      y[c] = T(0);
      continue;
    }
    const T vC = x[c];
    double np1[8], wn[8];
    cc_weights(in, cd, np1, wn);
    T s;
    if (op == 0) {  // M = I - W^{n+1}
      s = vC;
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (cc_has(cd, j)) s -= (T)np1[j] * x[c + cc_off(in, j)];
    } else if (op == 1) {  // N = W^n, diagonal w_C^n = 1 - sum of a_J over neighbours with data
      double wc = 1.0;
      s = T(0);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (cc_has(cd, j)) {
          s += (T)wn[j] * x[c + cc_off(in, j)];
          wc -= in.cc_a[j];
        }
      s += (T)wc * vC;
    } else {  // M - N
      s = T(0);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (cc_has(cd, j)) s += (T)in.cc_a[j] * (vC - x[c + cc_off(in, j)]);
    }
    y[c] = s;
  }
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
#define PI_ARGS tab, insts, sts, part

// stencil kernels come in twelve shapes (see shape_of)
#define PI_MARCH8(KERN, ...)                                                              \
  do {                                                                                    \
    switch (shape) {                                                                      \
      case 0: KERN<T, 2, 1, false><<<grid, block, 0, s>>>(__VA_ARGS__); break;            \
      case 1: KERN<T, 3, 1, false><<<grid, block, 0, s>>>(__VA_ARGS__); break;            \
      case 2: KERN<T, 2, 4, false><<<grid, block, 0, s>>>(__VA_ARGS__); break;            \
      case 3: KERN<T, 3, 4, false><<<grid, block, 0, s>>>(__VA_ARGS__); break;            \
      case 4: KERN<T, 2, 2, false><<<grid, block, 0, s>>>(__VA_ARGS__); break;            \
      case 5: KERN<T, 3, 2, false><<<grid, block, 0, s>>>(__VA_ARGS__); break;            \
      case 6: KERN<T, 2, 1, true><<<grid, block, 0, s>>>(__VA_ARGS__); break;             \
      case 7: KERN<T, 3, 1, true><<<grid, block, 0, s>>>(__VA_ARGS__); break;             \
      case 8: KERN<T, 2, 4, true><<<grid, block, 0, s>>>(__VA_ARGS__); break;             \
      case 9: KERN<T, 3, 4, true><<<grid, block, 0, s>>>(__VA_ARGS__); break;             \
      case 10: KERN<T, 2, 2, true><<<grid, block, 0, s>>>(__VA_ARGS__); break;            \
      default: KERN<T, 3, 2, true><<<grid, block, 0, s>>>(__VA_ARGS__); break;            \
    }                                                                                     \
  } while (0)

// ... and the cell-centred scheme has kernels of its own (KERN_cc)
#define PI_MARCH(KERN, ...)                                                               \
  do {                                                                                    \
    if (shape == kShapeCC) KERN##_cc<T, 1><<<grid, block, 0, s>>>(__VA_ARGS__);           \
    else if (shape == kShapeCC4) KERN##_cc<T, 4><<<grid, block, 0, s>>>(__VA_ARGS__);     \
    else PI_MARCH8(KERN, __VA_ARGS__);                                                    \
  } while (0)

template <typename T>
static hipError_t launch_t(KernelId k, int shape, const LaunchArgs &la) {
  const int ndim = (shape == kShapeCC || shape == kShapeCC4) ? 2 : (shape % 2) ? 3 : 2;
  const dim3 grid(la.nblocks), block(kBlock);
  const BlockEnt *tab = la.tab;
  const Inst *insts = la.insts;
  State *sts = la.sts;
  double *part = la.part;
  hipStream_t s = la.stream;
  switch (k) {
    case K_INIT: k_init<T><<<grid, block, 0, s>>>(PI_ARGS, la.iarg); break;
    case K_SOURCE:
      if (shape == kShapeCC || shape == kShapeCC4) k_source_cc<T><<<grid, block, 0, s>>>(PI_ARGS);
      else if (ndim == 3) k_source<T, 3><<<grid, block, 0, s>>>(PI_ARGS);
      else k_source<T, 2><<<grid, block, 0, s>>>(PI_ARGS);
      break;
    case K_OUTER: PI_MARCH(k_outer, PI_ARGS); break;
    case K_CG_STEP:
      if (la.iarg == 0) PI_MARCH(k_cg_first, PI_ARGS, la.iarg);
      else PI_MARCH(k_cg_step, PI_ARGS, la.iarg);
      break;
    case K_BICG_P:
      if (shape == kShapeCC || shape == kShapeCC4) return hipErrorInvalidValue;  // CG only
      PI_MARCH8(k_bicg_spmv_p, PI_ARGS);
      break;
    case K_BICG_S:
      if (shape == kShapeCC || shape == kShapeCC4) return hipErrorInvalidValue;
      PI_MARCH8(k_bicg_spmv_s, PI_ARGS);
      break;
    case K_BICG_UPDATE: k_bicg_update<T><<<grid, block, 0, s>>>(PI_ARGS); break;
    case K_COPY_RES: k_copy_res<T><<<grid, block, 0, s>>>(PI_ARGS); break;
    case K_GAUGE_GROUPS: k_gauge_groups<<<grid, block, 0, s>>>(PI_ARGS); break;
    case K_GAUGE_SUM: k_gauge_sum<<<grid, block, 0, s>>>(PI_ARGS); break;
    case K_GAUGE_APPLY: k_gauge_apply<T><<<grid, block, 0, s>>>(PI_ARGS); break;
    case K_APPLY: PI_MARCH(k_apply, PI_ARGS, la.iarg, (const T *)la.x, (T *)la.y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch(KernelId k, bool fp64, int shape, const LaunchArgs &la) {
  if (la.nblocks <= 0) return hipSuccess;
  return fp64 ? launch_t<double>(k, shape, la) : launch_t<float>(k, shape, la);
}

hipError_t launch_cg_rq(bool opl, const LaunchArgs &la) {
  if (la.nblocks <= 0) return hipSuccess;
  const dim3 grid(la.nblocks), block(kBlock);
  const BlockEnt *tab = la.tab;
  const Inst *insts = la.insts;
  State *sts = la.sts;
  double *part = la.part;
  hipStream_t s = la.stream;
  if (opl)
    k_cg_rq<4, true><<<grid, block, 0, s>>>(PI_ARGS, la.iarg);
  else
    k_cg_rq<4, false><<<grid, block, 0, s>>>(PI_ARGS, la.iarg);
  return hipGetLastError();
}

bool reduces(KernelId k) {
  switch (k) {
    case K_SOURCE:
    case K_OUTER:
    case K_CG_STEP:
    case K_BICG_P:
    case K_BICG_S:
    case K_BICG_UPDATE:
    case K_GAUGE_SUM: return true;
    default: return false;
  }
}

hipError_t launch_finalize(KernelId k, const Inst *insts, State *sts, const double *part, int count, hipStream_t s,
                           int iarg) {
  if (count <= 0) return hipSuccess;
  k_finalize<<<dim3(count), dim3(kBlock), 0, s>>>(insts, sts, part, (int)k, iarg);
  return hipGetLastError();
}

}  // namespace pi
