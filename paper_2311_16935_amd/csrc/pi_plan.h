// Private plan object of libpi.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/pi.h"
#include "pi_common.h"

struct pi_plan_s {
  int ndim = 0;
  int64_t dims[3] = {1, 1, 1};
  double spacing[3] = {1, 1, 1};
  uint32_t flags = 0;
  bool fp64 = false;
  bool bicgstab = false;
  bool fixed_point = false;  // PI_FIXED_POINT_CG variant
  bool cc = false;           // PI_CELL_CENTERED scheme (2-D)
  int inner_iters = 4;
  int64_t ncell = 0;
  int64_t nvalid = 0;
  int32_t ncomp = 0;
  double c[3][3] = {};      // ray-count constants c_jk by axis
  double Atot = 0;
  double face[3] = {};      // per-face ray totals by axis
  size_t bytes = 0;         // device bytes held

  // device arrays owned by the plan
  uint32_t *code = nullptr;
  int32_t *label = nullptr;
  double *comp_inv = nullptr;
  double *comp_sum = nullptr;
  int32_t *comp_order = nullptr;
  int32_t *seg_begin = nullptr;
  int32_t *comp_seg = nullptr;
  double *seg_sum = nullptr;
  double *P[2] = {nullptr, nullptr};
  double *S64 = nullptr;
  void *res = nullptr, *q = nullptr, *d = nullptr, *res1 = nullptr, *q1 = nullptr;
  void *p[2] = {nullptr, nullptr};
  void *bs[4] = {nullptr, nullptr, nullptr, nullptr};

  // instance template (device pointers filled, per-solve fields empty)
  pi::Inst inst{};

  // single-instance launch state, reused by every call on this plan
  pi::Inst *d_inst = nullptr;
  pi::State *d_state = nullptr;
  pi::BlockEnt *d_tab = nullptr;
  double *d_part = nullptr;
  int ntab = 0;
  pi::BlockEnt *d_tab_rq = nullptr;  // CG passes of a cg_rq plan: boundary-layer blocks, then d_tab's
  int ntab_rq = 0;
  pi::State *h_state = nullptr;    // pinned mirror
  hipGraphExec_t graph = nullptr;  // cached outer-step graph
  int graph_key = -1;
  hipStream_t cap_stream = nullptr;
};

namespace pi {

// Allocation helper that records the bytes held by the plan.
hipError_t plan_alloc(pi_plan_s *p, void **ptr, size_t bytes);

// Geometry of the strip decomposition for one grid (fields of Inst).
void set_walk(Inst &in, int ndim, const int64_t dims[3], int mseg_override, int vw_override);

// Single-instance table and partial slots of a plan.
hipError_t plan_tables(pi_plan_s *p);

// Block table of a set of instances, XCD-aware.  With assign_parts the
// instances' partial-sum slots are numbered from part_base0 on (else their
// part_base is kept: a table rebuilt for a subset of a batch).
std::vector<BlockEnt> build_table(const std::vector<Inst *> &insts, int part_base0, int *part_total,
                                  bool assign_parts = true);

}  // namespace pi
