// Velocity -> pressure-gradient source fields (declared in include/pi_flow.h).
//
// One lane per cell; each wave takes 64 consecutive cells of one grid row,
// so its loads are coalesced and its row, y and z are wave-uniform scalars.
// The neighbours of the difference stencils come from L1/L2.  Memory-bound
// in principle (every input read about once from HBM, every output written
// once), so the arithmetic is kept lean.  Inside the grid along an axis
// the central differences take the two neighbours directly; at the two ends
// of an axis a cell builds a table of up to four stencil points with the
// weights of the one-sided first and second differences and sums the
// weighted values.  Along y and z that choice is the same for a whole wave;
// along x only the waves holding a row end run both.  No divisions: the
// weights carry 1/(2h) and 1/h^2.  Arithmetic in FP64 on FP32 fields.
//
// Workgroups are dealt to the 8 XCDs round robin (workgroup b runs on XCD
// b mod 8).  The kernel renumbers them so that each XCD sweeps one
// contiguous eighth of the grid in order: the rows and planes a stencil
// needs around a cell were then fetched into that XCD's L2 by its own
// neighbouring workgroups shortly before.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "../../include/pi_flow.h"

namespace pf {

constexpr int kXcds = 8;
constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;

struct Grid {
  int n[3];          // cells along x, y, z (z = 1 in 2-D)
  int s[3];          // strides in cells
  double inv2h[3];   // 1 / (2 h)
  double invh2[3];   // 1 / h^2
  int nxc;           // 64-cell chunks per row
  int nrow;          // rows (ny * nz)
};

struct Args {
  Grid g;
  const float *u[3], *up[3], *un[3], *R[6];
  float *f[3];
  double rho, mu, inv2dt;
  double kT, T0, gas_R;
  int steady, has_R;
};

// Points and weights of the first (w1) and second (w2) difference along
// one axis at coordinate i of n cells with stride s:
//   inside             points c-s, c, c+s: w1 = (-1, 0, 1)/(2h),
//                      w2 = (1, -2, 1)/h^2
//   ends (n >= 3)      points c, c+-s, c+-2s, c+-3s (towards the inside):
//                      w1 = +-(-3, 4, -1, 0)/(2h),
//                      w2 = (2, -5, 4, -1)/h^2 (n >= 4) or the middle cell's
//                      three-point rule (1, -2, 1, 0)/h^2 (n = 3)
//   n = 2              points c, c+-s: w1 = +-(-1, 1)/h, w2 = 0
//   n = 1              all weights 0
// Unused points sit on c itself with weight 0.
struct Sten {
  int o[4];
  double w1[4], w2[4];
};

__device__ inline Sten stencil(const Grid &g, int k, int i) {
  const int n = g.n[k], s = g.s[k];
  const double a = g.inv2h[k], b = g.invh2[k];
  Sten t;
  const bool lo = i == 0, hi = i == n - 1;
  if (n >= 3 && !lo && !hi) {
    t.o[0] = -s, t.o[1] = 0, t.o[2] = s, t.o[3] = 0;
    t.w1[0] = -a, t.w1[1] = 0.0, t.w1[2] = a, t.w1[3] = 0.0;
    t.w2[0] = b, t.w2[1] = -2.0 * b, t.w2[2] = b, t.w2[3] = 0.0;
    return t;
  }
  const int d = lo ? s : -s;
  const double sg = lo ? 1.0 : -1.0;
  t.o[0] = 0, t.o[1] = n >= 2 ? d : 0, t.o[2] = n >= 3 ? 2 * d : 0, t.o[3] = n >= 4 ? 3 * d : 0;
  if (n >= 3) {
    t.w1[0] = -3.0 * sg * a, t.w1[1] = 4.0 * sg * a, t.w1[2] = -sg * a, t.w1[3] = 0.0;
    if (n >= 4) {
      t.w2[0] = 2.0 * b, t.w2[1] = -5.0 * b, t.w2[2] = 4.0 * b, t.w2[3] = -b;
    } else {
      t.w2[0] = b, t.w2[1] = -2.0 * b, t.w2[2] = b, t.w2[3] = 0.0;
    }
  } else {
    const double w = n == 2 ? 2.0 * sg * a : 0.0;  // 1/h on a 2-cell axis
    t.w1[0] = -w, t.w1[1] = w, t.w1[2] = 0.0, t.w1[3] = 0.0;
    t.w2[0] = 0.0, t.w2[1] = 0.0, t.w2[2] = 0.0, t.w2[3] = 0.0;
  }
  return t;
}

// field value at cell q; Off is the byte-offset type (32-bit when every
// field is below 4 GiB, which lets the loads use a scalar base plus a
// 32-bit vector offset)
template <typename Off>
__device__ inline double ld(const float *p, int64_t q) {
  return (double)*(const float *)((const char *)p + (Off)(q * 4));
}

// fields read or written once per cell (the snapshots before and after, the
// output): non-temporal, so that they do not push the neighbour rows and
// planes of u out of L2 before the next waves reuse them
template <typename Off>
__device__ inline double ld_once(const float *p, int64_t q) {
  return (double)__builtin_nontemporal_load((const float *)((const char *)p + (Off)(q * 4)));
}

// position of R_ij in the stress list: 2-D (uu, vv, uv), 3-D (uu, vv, ww, uv, uw, vw)
__device__ constexpr int sidx(int i, int j, int nd) {
  return i == j ? i : nd == 2 ? 2 : ((i < j ? i : j) == 0 ? ((i < j ? j : i) == 1 ? 3 : 4) : 5);
}

template <int ND, int MODEL, typename Off>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void k_flow(Args a) {
  const Grid &g = a.g;
  // hardware workgroup b -> logical block: XCD (b mod 8) takes the
  // contiguous range [xcd * per, (xcd + 1) * per) in increasing order
  const unsigned per = (gridDim.x + kXcds - 1) / kXcds;
  const unsigned blk = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
  const unsigned wv = __builtin_amdgcn_readfirstlane(blk * kWavesPerBlock + threadIdx.x / kWave);
  const int row = (int)(wv / (unsigned)g.nxc);
  if (row >= g.nrow) return;
  const int x = (int)(wv % (unsigned)g.nxc) * kWave + (int)(threadIdx.x % kWave);
  if (x >= g.n[0]) return;
  const int y = row % g.n[1], z = row / g.n[1];
  const int idx[3] = {x, y, z};
  const int64_t c = (int64_t)row * g.n[0] + x;
  constexpr int NP = MODEL == PI_FLOW_NS ? 4 : 3;  // second differences need the fourth point

  double out[3] = {0.0, 0.0, 0.0};
  if (MODEL == PI_FLOW_NS || MODEL == PI_FLOW_RANS) {
    double uc[3];
#pragma unroll
    for (int j = 0; j < ND; ++j) uc[j] = ld<Off>(a.u[j], c);
    double acc[3] = {0.0, 0.0, 0.0}, lap[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      double d1[3] = {0.0, 0.0, 0.0}, d1r[3] = {0.0, 0.0, 0.0};
      // along y and z the branch is wave-uniform; along x only the waves
      // holding a row end take both sides
      if (idx[j] >= 1 && idx[j] <= g.n[j] - 2) {
        const int s = g.s[j];
        const double ia = g.inv2h[j], ib = g.invh2[j];
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          const double vm = ld<Off>(a.u[i], c - s), vp = ld<Off>(a.u[i], c + s);
          d1[i] = (vp - vm) * ia;
          if (MODEL == PI_FLOW_NS) lap[i] = fma((vp - 2.0 * uc[i]) + vm, ib, lap[i]);
          if (MODEL == PI_FLOW_RANS && a.has_R) {
            const float *r = a.R[sidx(i, j, ND)];
            d1r[i] = (ld<Off>(r, c + s) - ld<Off>(r, c - s)) * ia;
          }
        }
      } else {
        const Sten t = stencil(g, j, idx[j]);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const int64_t q = c + t.o[k];
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            const double v = ld<Off>(a.u[i], q);
            d1[i] = fma(t.w1[k], v, d1[i]);
            if (MODEL == PI_FLOW_NS) lap[i] = fma(t.w2[k], v, lap[i]);
            if (MODEL == PI_FLOW_RANS && a.has_R)
              d1r[i] = fma(t.w1[k], ld<Off>(a.R[sidx(i, j, ND)], q), d1r[i]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < ND; ++i) acc[i] = fma(uc[j], d1[i], acc[i]) + d1r[i];
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      if (MODEL == PI_FLOW_NS) {
        if (!a.steady) acc[i] += (ld_once<Off>(a.un[i], c) - ld_once<Off>(a.up[i], c)) * a.inv2dt;
        out[i] = -a.rho * acc[i] + a.mu * lap[i];
      } else {
        out[i] = -a.rho * acc[i];
      }
    }
  } else {
    // compressible RANS: T from the adiabatic relation, W_ij = U_i U_j + R_ij;
    // div_i = dW_ij/dx_j and dT_j accumulated from the same stencil points
    double Uc[3], Wc[3][3];
#pragma unroll
    for (int j = 0; j < ND; ++j) Uc[j] = ld<Off>(a.u[j], c);
    double v2 = 0.0;
#pragma unroll
    for (int k = 0; k < ND; ++k) v2 += Uc[k] * Uc[k];
    const double T = a.T0 - a.kT * v2;
#pragma unroll
    for (int i = 0; i < ND; ++i)
#pragma unroll
      for (int j = 0; j < ND; ++j) Wc[i][j] = Uc[i] * Uc[j] + (a.has_R ? ld<Off>(a.R[sidx(i, j, ND)], c) : 0.0);
    double div[3] = {0.0, 0.0, 0.0}, dT[3] = {0.0, 0.0, 0.0};
    // T and W_i. (fixed j) at cell q, accumulated with weight w
    auto point = [&](int j, int64_t q, double w) {
      double U[3];
      double w2 = 0.0;
#pragma unroll
      for (int m = 0; m < ND; ++m) {
        U[m] = ld<Off>(a.u[m], q);
        w2 += U[m] * U[m];
      }
      dT[j] = fma(w, a.T0 - a.kT * w2, dT[j]);
#pragma unroll
      for (int i = 0; i < ND; ++i) {
        const double W = U[i] * U[j] + (a.has_R ? ld<Off>(a.R[sidx(i, j, ND)], q) : 0.0);
        div[i] = fma(w, W, div[i]);
      }
    };
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      if (idx[j] >= 1 && idx[j] <= g.n[j] - 2) {
        point(j, c - g.s[j], -g.inv2h[j]);
        point(j, c + g.s[j], g.inv2h[j]);
      } else {
        const Sten t = stencil(g, j, idx[j]);
#pragma unroll
        for (int k = 0; k < NP; ++k) point(j, c + t.o[k], t.w1[k]);
      }
    }
    const double RT = a.gas_R * T;
    double A[3][3], b[3];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      double corr = 0.0;
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        corr += Wc[i][j] / T * dT[j];
        A[i][j] = (i == j ? 1.0 : 0.0) + Wc[i][j] / RT;
      }
      b[i] = -(div[i] - corr) / RT;
    }
    if (ND == 2) {
      const double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
      out[0] = (A[1][1] * b[0] - A[0][1] * b[1]) / det;
      out[1] = (A[0][0] * b[1] - A[1][0] * b[0]) / det;
    } else {
      // Cramer's rule with the cofactors of A: x = adj(A) b / det
      const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
      const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
      const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
      const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
      const double c10 = A[0][2] * A[2][1] - A[0][1] * A[2][2];
      const double c11 = A[0][0] * A[2][2] - A[0][2] * A[2][0];
      const double c12 = A[0][1] * A[2][0] - A[0][0] * A[2][1];
      const double c20 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
      const double c21 = A[0][2] * A[1][0] - A[0][0] * A[1][2];
      const double c22 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
      out[0] = (c00 * b[0] + c10 * b[1] + c20 * b[2]) / det;
      out[1] = (c01 * b[0] + c11 * b[1] + c21 * b[2]) / det;
      out[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) / det;
    }
  }
#pragma unroll
  for (int i = 0; i < ND; ++i) __builtin_nontemporal_store((float)out[i], (float *)((char *)a.f[i] + (Off)(c * 4)));
}

}  // namespace pf

using namespace pf;

extern "C" pi_status pi_flow_source(int ndim, const int64_t dims[3], const double spacing[3], int model,
                                    const float *const *u, const float *const *u_prev,
                                    const float *const *u_next, const float *const *R,
                                    const pi_flow_params *prm, float *const *f, void *stream) {
  if ((ndim != 2 && ndim != 3) || !dims || !spacing || !u || !prm || !f) return PI_ERR_INVALID_ARG;
  if (model != PI_FLOW_NS && model != PI_FLOW_RANS && model != PI_FLOW_COMPRESSIBLE) return PI_ERR_INVALID_ARG;
  Args a = {};
  int64_t ncell = 1;
  for (int k = 0; k < 3; ++k) {
    const int64_t n = k < ndim ? dims[k] : 1;
    const double h = k < ndim ? spacing[k] : 1.0;
    if (n < 1 || !(h > 0.0) || !isfinite(h)) return PI_ERR_INVALID_ARG;
    a.g.n[k] = (int)n;
    a.g.inv2h[k] = 1.0 / (2.0 * h);
    a.g.invh2[k] = 1.0 / (h * h);
    ncell *= n;
    if (ncell >= (int64_t(1) << 31)) return PI_ERR_INVALID_ARG;
  }
  a.g.s[0] = 1;
  a.g.s[1] = a.g.n[0];
  a.g.s[2] = a.g.n[0] * a.g.n[1];
  a.g.nxc = (a.g.n[0] + kWave - 1) / kWave;
  a.g.nrow = a.g.n[1] * a.g.n[2];
  for (int k = 0; k < ndim; ++k) {
    if (!u[k] || !f[k]) return PI_ERR_INVALID_ARG;
    a.u[k] = u[k];
    a.f[k] = f[k];
  }
  a.rho = prm->rho;
  a.mu = prm->mu;
  a.steady = 1;
  if (model == PI_FLOW_NS && (u_prev || u_next)) {
    if (!u_prev || !u_next || !(prm->dt > 0.0)) return PI_ERR_INVALID_ARG;
    for (int k = 0; k < ndim; ++k) {
      if (!u_prev[k] || !u_next[k]) return PI_ERR_INVALID_ARG;
      a.up[k] = u_prev[k];
      a.un[k] = u_next[k];
    }
    a.steady = 0;
    a.inv2dt = 1.0 / (2.0 * prm->dt);
  }
  a.has_R = 0;
  if (model != PI_FLOW_NS && R) {
    const int nr = ndim == 2 ? 3 : 6;
    for (int k = 0; k < nr; ++k) {
      if (!R[k]) return PI_ERR_INVALID_ARG;
      a.R[k] = R[k];
    }
    a.has_R = 1;
  }
  if (model == PI_FLOW_COMPRESSIBLE) {
    if (!(prm->gas_R > 0.0) || !(prm->T_inf > 0.0) || !(prm->V_inf > 0.0) || !(prm->gamma > 1.0))
      return PI_ERR_INVALID_ARG;
    // T = T_inf (1 + (gamma - 1)/2 M^2 (1 - V^2 / V_inf^2)) = T0 - kT V^2
    const double q = 0.5 * (prm->gamma - 1.0) * prm->M_inf * prm->M_inf;
    a.T0 = prm->T_inf * (1.0 + q);
    a.kT = prm->T_inf * q / (prm->V_inf * prm->V_inf);
    a.gas_R = prm->gas_R;
  }
  // one wave per 64-cell row chunk, four waves per workgroup, a multiple of
  // 8 workgroups so that the XCD renumbering is a bijection; waves past the
  // last row exit at once
  const int64_t waves = (int64_t)a.g.nxc * a.g.nrow;
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  const unsigned nb = (unsigned)((blocks + kXcds - 1) / kXcds * kXcds);
  hipStream_t s = (hipStream_t)stream;
  const bool small = ncell <= (int64_t(1) << 30);  // every byte offset fits 32 bits
#define PF_GO(ND, M)                                                                              \
  do {                                                                                            \
    if (small) k_flow<ND, M, uint32_t><<<dim3(nb), dim3(kWave * kWavesPerBlock), 0, s>>>(a);      \
    else k_flow<ND, M, int64_t><<<dim3(nb), dim3(kWave * kWavesPerBlock), 0, s>>>(a);             \
  } while (0)
  if (ndim == 2) {
    if (model == PI_FLOW_NS) PF_GO(2, PI_FLOW_NS);
    else if (model == PI_FLOW_RANS) PF_GO(2, PI_FLOW_RANS);
    else PF_GO(2, PI_FLOW_COMPRESSIBLE);
  } else {
    if (model == PI_FLOW_NS) PF_GO(3, PI_FLOW_NS);
    else if (model == PI_FLOW_RANS) PF_GO(3, PI_FLOW_RANS);
    else PF_GO(3, PI_FLOW_COMPRESSIBLE);
  }
#undef PF_GO
  return hipGetLastError() == hipSuccess ? PI_OK : PI_ERR_DEVICE;
}
