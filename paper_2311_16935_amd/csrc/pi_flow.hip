// Velocity -> pressure-gradient source fields (declared in include/pi_flow.h).
//
// One thread per cell, x fastest so a wave reads consecutive cells; the
// neighbours of the difference stencils come from L1/L2.  Memory-bound:
// every input is read about once from HBM, every output written once.
// Arithmetic in FP64.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "../../include/pi_flow.h"

namespace pf {

struct Grid {
  int n[3];        // cells along x, y, z (z = 1 in 2-D)
  int64_t s[3];    // strides
  double h[3];     // spacing
  int64_t ncell;
};

struct Args {
  Grid g;
  const float *u[3], *up[3], *un[3], *R[6];
  float *f[3];
  double rho, mu, inv2dt;
  double gas_R, gamma, T_inf, M_inf, V_inf;
  int steady, has_R;
};

// first derivative along axis k of the cell field v(.) at cell c with
// coordinate i: central inside, second-order one-sided at the ends
template <typename V>
__device__ inline double d1(const Grid &g, int k, int64_t c, int i, V v) {
  const int n = g.n[k];
  const int64_t s = g.s[k];
  const double h = g.h[k];
  if (n == 1) return 0.0;
  if (n == 2) return i == 0 ? (v(c + s) - v(c)) / h : (v(c) - v(c - s)) / h;
  if (i == 0) return (-3.0 * v(c) + 4.0 * v(c + s) - v(c + 2 * s)) / (2.0 * h);
  if (i == n - 1) return (3.0 * v(c) - 4.0 * v(c - s) + v(c - 2 * s)) / (2.0 * h);
  return (v(c + s) - v(c - s)) / (2.0 * h);
}

// second derivative: three-point inside, four-point one-sided at the ends;
// with three cells the ends take the middle value, below three it is 0
template <typename V>
__device__ inline double d2(const Grid &g, int k, int64_t c, int i, V v) {
  const int n = g.n[k];
  const int64_t s = g.s[k];
  const double h2 = g.h[k] * g.h[k];
  if (n < 3) return 0.0;
  if (n == 3) {
    const int64_t m = c + (1 - i) * s;  // the middle cell
    return (v(m + s) - 2.0 * v(m) + v(m - s)) / h2;
  }
  if (i == 0) return (2.0 * v(c) - 5.0 * v(c + s) + 4.0 * v(c + 2 * s) - v(c + 3 * s)) / h2;
  if (i == n - 1) return (2.0 * v(c) - 5.0 * v(c - s) + 4.0 * v(c - 2 * s) - v(c - 3 * s)) / h2;
  return (v(c + s) - 2.0 * v(c) + v(c - s)) / h2;
}

// position of R_ij in the stress list: 2-D (uu, vv, uv), 3-D (uu, vv, ww, uv, uw, vw)
__device__ inline int sidx(int i, int j, int nd) {
  if (i == j) return i;
  const int a = i < j ? i : j, b = i < j ? j : i;
  if (nd == 2) return 2;
  return a == 0 ? (b == 1 ? 3 : 4) : 5;
}

template <int ND, int MODEL>
__global__ __launch_bounds__(256) void k_flow(Args a) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.g.ncell) return;
  const Grid &g = a.g;
  int idx[3];
  idx[0] = (int)(c % g.n[0]);
  idx[1] = (int)((c / g.n[0]) % g.n[1]);
  idx[2] = ND == 3 ? (int)(c / ((int64_t)g.n[0] * g.n[1])) : 0;
  double out[3] = {0.0, 0.0, 0.0};
  if (MODEL == PI_FLOW_NS || MODEL == PI_FLOW_RANS) {
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      const float *ui = a.u[i];
      auto vi = [&](int64_t q) { return (double)ui[q]; };
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < ND; ++j) acc += (double)a.u[j][c] * d1(g, j, c, idx[j], vi);
      if (MODEL == PI_FLOW_NS) {
        if (!a.steady) acc += ((double)a.un[i][c] - (double)a.up[i][c]) * a.inv2dt;
        double lap = 0.0;
#pragma unroll
        for (int j = 0; j < ND; ++j) lap += d2(g, j, c, idx[j], vi);
        out[i] = -a.rho * acc + a.mu * lap;
      } else {
        if (a.has_R) {
#pragma unroll
          for (int j = 0; j < ND; ++j) {
            const float *r = a.R[sidx(i, j, ND)];
            acc += d1(g, j, c, idx[j], [&](int64_t q) { return (double)r[q]; });
          }
        }
        out[i] = -a.rho * acc;
      }
    }
  } else {
    // compressible RANS: T from the adiabatic relation, W_ij = U_i U_j + R_ij
    const double kT = a.T_inf * 0.5 * (a.gamma - 1.0) * a.M_inf * a.M_inf / (a.V_inf * a.V_inf);
    const double T0 = a.T_inf * (1.0 + 0.5 * (a.gamma - 1.0) * a.M_inf * a.M_inf);
    auto T_at = [&](int64_t q) {
      double v2 = 0.0;
#pragma unroll
      for (int k = 0; k < ND; ++k) v2 += (double)a.u[k][q] * (double)a.u[k][q];
      return T0 - kT * v2;
    };
    auto W_at = [&](int i, int j, int64_t q) {
      double w = (double)a.u[i][q] * (double)a.u[j][q];
      if (a.has_R) w += (double)a.R[sidx(i, j, ND)][q];
      return w;
    };
    const double T = T_at(c);
    const double RT = a.gas_R * T;
    double dT[3];
#pragma unroll
    for (int j = 0; j < ND; ++j) dT[j] = d1(g, j, c, idx[j], T_at);
    double A[3][3], b[3];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      double div = 0.0, corr = 0.0;
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        div += d1(g, j, c, idx[j], [&](int64_t q) { return W_at(i, j, q); });
        const double w = W_at(i, j, c);
        corr += w / T * dT[j];
        A[i][j] = (i == j ? 1.0 : 0.0) + w / RT;
      }
      b[i] = -(div - corr) / RT;
    }
    if (ND == 2) {
      const double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
      out[0] = (A[1][1] * b[0] - A[0][1] * b[1]) / det;
      out[1] = (A[0][0] * b[1] - A[1][0] * b[0]) / det;
    } else {
      // Cramer's rule with the cofactors of A
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
      // x = adj(A) b / det, adj(A)_ij = cofactor_ji
      out[0] = (c00 * b[0] + c10 * b[1] + c20 * b[2]) / det;
      out[1] = (c01 * b[0] + c11 * b[1] + c21 * b[2]) / det;
      out[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) / det;
    }
  }
#pragma unroll
  for (int i = 0; i < ND; ++i) a.f[i][c] = (float)out[i];
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
    a.g.h[k] = h;
    ncell *= n;
    if (ncell >= (int64_t(1) << 31)) return PI_ERR_INVALID_ARG;
  }
  a.g.ncell = ncell;
  a.g.s[0] = 1;
  a.g.s[1] = a.g.n[0];
  a.g.s[2] = (int64_t)a.g.n[0] * a.g.n[1];
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
    a.gas_R = prm->gas_R;
    a.gamma = prm->gamma;
    a.T_inf = prm->T_inf;
    a.M_inf = prm->M_inf;
    a.V_inf = prm->V_inf;
  }
  const unsigned nb = (unsigned)((ncell + 255) / 256);
  hipStream_t s = (hipStream_t)stream;
#define PF_LAUNCH(ND, M) k_flow<ND, M><<<dim3(nb), dim3(256), 0, s>>>(a)
  if (ndim == 2) {
    if (model == PI_FLOW_NS) PF_LAUNCH(2, PI_FLOW_NS);
    else if (model == PI_FLOW_RANS) PF_LAUNCH(2, PI_FLOW_RANS);
    else PF_LAUNCH(2, PI_FLOW_COMPRESSIBLE);
  } else {
    if (model == PI_FLOW_NS) PF_LAUNCH(3, PI_FLOW_NS);
    else if (model == PI_FLOW_RANS) PF_LAUNCH(3, PI_FLOW_RANS);
    else PF_LAUNCH(3, PI_FLOW_COMPRESSIBLE);
  }
#undef PF_LAUNCH
  return hipGetLastError() == hipSuccess ? PI_OK : PI_ERR_DEVICE;
}
