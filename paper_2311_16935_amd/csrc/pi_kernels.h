// Host-side entry to the solve kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "pi_common.h"

namespace pi {

enum KernelId {
  K_INIT,
  K_SOURCE,
  K_OUTER,
  K_CG_STEP,
  K_BICG_P,
  K_BICG_S,
  K_BICG_UPDATE,
  K_COPY_RES,
  K_GAUGE_SUM,
  K_GAUGE_GROUPS,
  K_GAUGE_APPLY,
  K_APPLY,
  K_COUNT
};

struct LaunchArgs {
  const BlockEnt *tab;
  const Inst *insts;
  State *sts;
  double *part;
  int nblocks;          // entries of tab (grid size)
  hipStream_t stream;
  int iarg;             // K_INIT: warm start flag; K_APPLY: operator; K_CG_STEP: pass index
  const void *x;        // K_APPLY input
  void *y;              // K_APPLY output
};

hipError_t launch(KernelId k, bool fp64, int shape, const LaunchArgs &la);

// Inner CG pass k >= 1 without a stored q (k_cg_rq) for
// one plan that qualifies (Inst.cg_rq): 3-D, no missing data, FP32, four
// cells per lane, rows of one wave strip or of as many overlapping windows
// as strips.  opl: the fixed point's operator.
hipError_t launch_cg_rq(bool opl, const LaunchArgs &la);

// Kernels that leave per-block partial sums, and the per-instance finalize
// (grid = count instances) that turns them into the instances' scalars.
bool reduces(KernelId k);
hipError_t launch_finalize(KernelId k, const Inst *insts, State *sts, const double *part, int count, hipStream_t s,
                           int iarg = 0);

// Plan-time kernel: packed per-cell counter codes from the device mask.
hipError_t launch_codes(int ndim, int nx, int ny, int nz, const uint8_t *mask, uint32_t *code, hipStream_t s);

}  // namespace pi
