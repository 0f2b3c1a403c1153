/*
 * pi_flow.h -- the velocity -> pressure-gradient stage of libpi.
 *
 * The pressure integration consumes a gradient ("source") field f.  In the
 * paper it comes from velocity measurements through the momentum equations:
 *   PI_FLOW_NS            incompressible Navier-Stokes (Eq. (1) of the
 *                         introduction): f = -rho (du/dt + (u . grad) u)
 *                         + mu lap u; du/dt from two snapshots 2 dt apart,
 *                         or 0 (steady) when they are not given.
 *   PI_FLOW_RANS          Reynolds-averaged, viscous terms dropped (Eq.
 *                         RANS_f): f_i = -rho (U_j dU_i/dx_j + dR_ij/dx_j).
 *   PI_FLOW_COMPRESSIBLE  compressible RANS of the supersonic double-fin
 *                         section (Eq. compressible-pressure), solved per
 *                         cell for f = grad ln(P / P_inf):
 *                         (delta_ij + W_ij / (R T)) f_j = -(1 / (R T))
 *                         (dW_ij/dx_j - W_ij / T dT/dx_j), W_ij = U_i U_j +
 *                         R_ij, T / T_inf = 1 + (gamma - 1)/2 M_inf^2 (1 -
 *                         V^2 / V_inf^2).
 * Derivatives are second-order central differences with second-order
 * one-sided differences at the grid ends (three-point second differences
 * inside, four-point one-sided ones at the ends for lap u).  Arithmetic is
 * FP64; inputs and outputs FP32.  Every cell must hold data (no mask).
 */
#ifndef PI_FLOW_H
#define PI_FLOW_H

#include <stddef.h>
#include <stdint.h>

#include "pi.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PI_FLOW_NS 0
#define PI_FLOW_RANS 1
#define PI_FLOW_COMPRESSIBLE 2

typedef struct pi_flow_params {
  double rho;    /* density (NS, RANS)                                     */
  double mu;     /* dynamic viscosity (NS)                                 */
  double dt;     /* NS: u_prev and u_next are snapshots at t - dt, t + dt  */
  double gas_R;  /* compressible: gas constant                            */
  double gamma;  /* compressible: ratio of specific heats                 */
  double T_inf;  /* compressible: T_inf of the temperature relation        */
  double M_inf;  /* compressible: free-stream Mach number                  */
  double V_inf;  /* compressible: free-stream speed                        */
} pi_flow_params;

/*
 * pi_flow_source -- f from velocity on an nx * ny (* nz) grid (storage order
 * x fastest, as the solver's).
 *   ndim, dims, spacing  as for pi_plan (dims and spacing host arrays).
 *   model   PI_FLOW_NS, PI_FLOW_RANS or PI_FLOW_COMPRESSIBLE.
 *   u       host array of ndim device pointers: velocity (NS) or mean
 *           velocity (RANS, compressible) components along x, y[, z].
 *   u_prev, u_next  NS only: host arrays of ndim device pointers to the
 *           snapshots before and after, or both NULL for a steady field.
 *   R       RANS / compressible: host array of device pointers to the
 *           Reynolds stresses (2-D: uu, vv, uv; 3-D: uu, vv, ww, uv, uw, vw),
 *           or NULL for none.
 *   prm     host pointer to the constants the model uses.
 *   f       host array of ndim device pointers receiving the components.
 * Inputs and outputs must not overlap.  PI_ERR_INVALID_ARG for bad sizes,
 * NULL pointers, spacing <= 0, a cell count of 2^31 or more, dt <= 0 with
 * snapshots, non-positive gas constants or temperatures.  Asynchronous on
 * `stream`.
 */
pi_status pi_flow_source(int ndim, const int64_t dims[3], const double spacing[3], int model,
                         const float *const *u, const float *const *u_prev, const float *const *u_next,
                         const float *const *R, const pi_flow_params *prm, float *const *f, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PI_FLOW_H */
