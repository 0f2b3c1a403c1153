// Shared host/device definitions of libpi.
//
// Work decomposition.  Stencil kernels cut a grid into "strips": 64 * W
// consecutive cells along x (one wavefront, W cells per lane; W = 4 when nx
// is a multiple of 4, else 1) at fixed y (3-D), which march along the
// slowest axis (z in 3-D, y in 2-D) over a segment of `mseg` planes/rows.
// The marching lane keeps the values of the previous and the next plane in
// registers, so the stencil reads each vector from HBM about once;
// x-neighbours come from the lane itself and adjacent lanes, y-neighbours in
// 3-D from L1/L2.  A block is four strips, consecutive in memory (x fastest,
// then y).  Point-wise kernels instead give
// block b of an instance a contiguous range of cells.  Every kernel of the
// solve walks a block table whose entries name (instance,
// block-within-instance), so one launch serves one grid or a whole batch of
// uneven grids; the table is ordered so that each instance's consecutive
// blocks sit on one XCD (hardware assigns workgroup i to XCD i mod 8), keeping
// plane-to-plane reuse inside one L2.
#pragma once

#include <stdint.h>

namespace pi {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kXcd = 8;
constexpr uint32_t kValidBit = 1u << 31;
constexpr int kStates = 20;      // per-direction counter states (3-D uses 0..18)
constexpr int kSegCells = 65536; // gauge segment length (cells)
constexpr int kShapes = 14;      // stencil launch shapes: (2-D, 3-D) x (1, 4, 2 cells per lane) x (codes
                                 // read, derived), and the 2-D cell-centred scheme with 1 or 4 cells per lane
constexpr int kShapeCC = 12;
// An instance of at most this many blocks runs its inner CG passes without a
// finalize kernel: every block of a pass re-sums the previous pass's partial
// sums (32 KB at this bound, from L2) to get alpha and beta.  Larger
// instances keep the finalize.  Measured per outer step at 1024 blocks: 1 %
// (256^3) to 4 % (2048^2) faster without it; at 2048 blocks 5-14 % slower.
constexpr int kInlineMaxBlocks = 1024;
constexpr int32_t kNoStop = 1 << 30;

// CG passes that evaluate q again (k_cg_rq): the layers next to the y faces
// (rows 0..2 and ny-3..ny-1, every plane, in chunks of kRqChunk planes) and
// next to the march faces (planes 0..2 and nm-3..nm-1 of the other rows) are
// wave tasks of blocks of their own, for every wave strip of the row; the
// rest is interior.  With ny or nm below 7 there is no interior and every
// row is a boundary row.
constexpr int kRqChunk = 3;
__host__ __device__ inline int64_t rq_ntasks(int ny, int nm, int nxs) {
  const bool inner = ny >= 7 && nm >= 7;
  const int64_t nA = (int64_t)(inner ? 6 : ny) * ((nm + kRqChunk - 1) / kRqChunk);
  return (nA + (inner ? 2 * (int64_t)(ny - 6) : 0)) * nxs;
}
// A row longer than one wave strip (64 lanes of four cells, kRqSpan cells)
// is split over overlapping wave windows: q_k at a cell needs p_{k-1} two
// cells away along x, which a window evaluates correctly only two cells or
// more inside its edges, so each window owns (stores and sums) the cells at
// least one lane (four cells) inside every edge that is not a grid face.
// The first window owns [0, kRqSpan - 4), the middle ones kRqSpan - 8 cells
// each, the last the rest; window xs starts four cells before its owned
// range, or at nx - kRqSpan where that is earlier.  Rows need nx % 4 == 0.
constexpr int kRqSpan = 256;
__host__ __device__ inline int rq_nstrips(int nx) {
  if (nx <= kRqSpan) return 1;
  const int rest = nx - 2 * (kRqSpan - 4);
  return 2 + (rest > 0 ? (rest + kRqSpan - 9) / (kRqSpan - 8) : 0);
}
__host__ __device__ inline void rq_window(int nx, int nxs, int xs, int &start, int &own0, int &own1) {
  if (nxs == 1) {
    start = own0 = 0;
    own1 = nx;
    return;
  }
  own0 = xs == 0 ? 0 : (kRqSpan - 4) + (kRqSpan - 8) * (xs - 1);
  own1 = xs == nxs - 1 ? nx : (kRqSpan - 4) + (kRqSpan - 8) * xs;
  start = xs == 0 ? 0 : (own0 - 4 < nx - kRqSpan ? own0 - 4 : nx - kRqSpan);
}
constexpr int kShapeCC4 = 13;

// Launch shape of an instance: (3-D) + 2 * (lane width: 0 for one cell, 1
// for four, 2 for two) + 6 * (no mask: counter codes derived from cell
// coordinates); the cell-centred scheme has shapes of its own.
__host__ __device__ inline int shape_of(int ndim, int vw, int gen, int cc) {
  if (cc) return vw == 4 ? kShapeCC4 : kShapeCC;
  return (ndim == 3 ? 1 : 0) + 2 * (vw == 4 ? 1 : vw == 2 ? 2 : 0) + (gen ? 6 : 0);
}

// Cell-centred scheme: the 8 neighbours J (E, W, N, S, NE, NW, SE, SW) and
// the bit of cell C + (dx, dy), |dx|, |dy| <= 2, in the 24-bit ring code of a
// data cell (bit 31 = data).
__host__ __device__ constexpr int cc_dir(int dx, int dy) {
  return dy == 0 ? (dx > 0 ? 0 : 1) : dx == 0 ? (dy > 0 ? 2 : 3) : dy > 0 ? (dx > 0 ? 4 : 5) : (dx > 0 ? 6 : 7);
}
__host__ __device__ constexpr int cc_dx(int j) { return (j == 0 || j == 4 || j == 6) ? 1 : (j == 1 || j == 5 || j == 7) ? -1 : 0; }
__host__ __device__ constexpr int cc_dy(int j) { return (j == 2 || j == 4 || j == 5) ? 1 : (j == 3 || j == 6 || j == 7) ? -1 : 0; }
__host__ __device__ constexpr int cc_bit(int dx, int dy) {
  return (dy + 2) * 5 + (dx + 2) < 12 ? (dy + 2) * 5 + (dx + 2) : (dy + 2) * 5 + (dx + 2) - 1;
}
constexpr uint32_t kCcRing = (1u << 24) - 1;

// The 32 kinds of ray piece of the cell-centred scheme, in a fixed order.
// Per major axis (rays less steep than the diagonal travel along x, steeper
// ones along y), travel sign and sign of the lateral slope, the rays through
// C fall into four pieces by the lateral offsets of the previous cell J and
// of the cell K before it (one and two steps back along the major axis):
//   0: J and K one lateral step back        (measure index 0)
//   1: J straight back, K one lateral step  (measure index 0)
//   2: J and K straight back                (measure index 1)
//   3: J one, K two lateral steps back      (measure index 2)
// f(J direction, bit of J, bit of K, major axis, measure index) is called
// for each.  The measures come from integrating the piece lengths, linear in
// tan(angle), over the angle (the plan's constants).
template <class F>
__host__ __device__ inline void cc_pieces(F &&f) {
#pragma unroll
  for (int maj = 0; maj < 2; ++maj)
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int pc = 0; pc < 4; ++pc) {
          const int sg = si ? -1 : 1, mu = mi ? -1 : 1;
          const int jM = -sg, jm = (pc == 0 || pc == 3) ? -mu : 0;
          const int kM = -2 * sg, km = pc == 2 ? 0 : pc == 3 ? -2 * mu : -mu;
          const int jx = maj ? jm : jM, jy = maj ? jM : jm;
          const int kx = maj ? km : kM, ky = maj ? kM : km;
          f(cc_dir(jx, jy), cc_bit(jx, jy), cc_bit(kx, ky), maj, pc == 3 ? 2 : pc == 2 ? 1 : 0);
        }
}

// Per-direction code layout: 3-D 5 bits (state = 1 + n1 + 3 n2 + 9 far for a
// face neighbour with data, 0 otherwise), 2-D 3 bits (state = 1 + n1 + 3 far).
// n1, n2 count the face neighbour's laterals with data along the first and
// second remaining axis (0..2); far is the neighbour's own far cell.
__host__ __device__ inline int dir_bits(int ndim) { return ndim == 3 ? 5 : 3; }

enum Dir { DE = 0, DW = 1, DN = 2, DS = 3, DF = 4, DB = 5 };

struct BlockEnt {
  int32_t inst;   // -1: padding entry, the block exits at once
  int32_t lb;     // block index inside the instance
};

// Per-instance description, device resident (read-only inside kernels).
struct Inst {
  int32_t ndim;
  int32_t nx, ny, nz;
  int64_t ncell;
  int32_t vw;       // cells per lane along x in stencil kernels (1, 2 or 4)
  int32_t gen;      // 1: every cell holds data, codes follow from coordinates
  int32_t nxs;      // strips of 64 * vw cells along x
  int32_t rows;     // strips stacked along y: ny in 3-D, 1 in 2-D
  int32_t nm;       // length of the marching axis
  int32_t mseg;     // marching segment length
  int32_t nseg;
  int32_t nblocks;  // blocks of this instance
  int64_t nwaves;
  int64_t sm;       // stride of the marching axis
  int64_t srow;     // stride between stacked strips (nx in 3-D, 0 in 2-D)
  int32_t part_base;// first slot of this instance in the partial-sum array
  int32_t part_stride; // slots of one partial-sum array; the CG passes use the
                       // two arrays after the first one, by pass parity
  int32_t bicg;     // inner solver is BiCGStab (else the single-pass CG)
  int32_t cg_inline;// the CG passes take alpha and beta from the previous
                    // pass's partials themselves (no finalize kernel)
  int32_t nt_outer; // the outer kernel streams S, P' and r non-temporally
                    // (chosen by the autotuner)
  int32_t cg_rq;    // the plan's CG passes evaluate q again instead of
                    // storing it (launch_cg_rq; 0 in batched launches)
  int32_t cg_slots; // partial-sum slots of a CG pass: nblocks, plus the
                    // boundary-layer blocks of k_cg_rq
  int32_t ncomp;    // connected groups of data cells
  int32_t inner_iters; // inner Krylov iterations per outer step
  int32_t inner_op; // operator of the inner solve: 0 [W^{n+1}], 1 [W^{n+1}] - [W^n]
  double inner_floor; // variant: stop the inner CG once r.r falls below this
                      // fraction of its value at the start of the inner solve
  double inv_nvalid;// 1 / data cells (gauge of a single group)
  double a[6];      // per-direction face total / A_tot
  double dsig[6];   // signed spacing Delta_j
  double lut_np1[6][kStates];  // w_j^{n+1} by direction and state
  double lut_n[6][kStates];    // w_j^{n}   by direction and state
  // cell-centred scheme (cc != 0): per-direction ray totals over A_tot,
  // displacement Delta_J = (dx_J h_x, dy_J h_y), and the measures over A_tot
  // of the three kinds of ray piece per major axis (see cc_weights)
  int32_t cc;
  double cc_a[8];
  double cc_step[8][2];
  double cc_m[2][3];
  const uint32_t *code;
  // connected groups (all NULL when ncomp == 1): data cells sorted by group,
  // cut into segments of at most kSegCells cells that never straddle groups
  const int32_t *label;        // group of each cell
  const double *comp_inv_count;// 1 / cells per group
  double *comp_sum;            // per-group mean, filled by the gauge kernels
  const int32_t *comp_order;   // data cells sorted by (group, index)
  const int32_t *seg_begin;    // [nseg_g + 1] bounds into comp_order
  const int32_t *comp_seg;     // [ncomp + 1] first segment of each group
  double *seg_sum;             // [nseg_g] per-segment sums
  int32_t nseg_g;
  // workspace, typed by the plan's precision (T)
  double *P[2];     // FP64 iterate, ping-pong
  double *S64;      // source vector, kept in FP64 so that it sums to zero
  void *S;          // optional copy of S in T (pi_source output), else NULL
  void *res;
  void *res1;       // CG: second residual buffer (ping-pong with res)
  void *p[2];       // search direction, ping-pong
  void *q;
  void *q1;         // CG: second M p buffer (ping-pong with q)
  void *d;          // correction accumulated by the inner solve
  void *bs[4];      // BiCGStab: rhat, v, s, t
  // per-solve user buffers
  const void *g[3];
  void *Pout;
  const void *P0;
  double tol;
  int64_t max_iter;
};

// Mutable scalars of one instance.
struct State {
  double normS2;
  double rr;        // CG: r.r of the current inner residual
  double rr0;       // CG: r.r at the start of the inner solve
  double alpha, beta;
  double rho, omega;// BiCGStab
  double epsR, epsP;
  double red[4];    // scratch for the last block's results
  int64_t outer;
  int64_t inner_total;
  int32_t inner;    // BiCGStab: inner iteration inside the current outer step
  int32_t first;    // BiCGStab: next search direction is the residual itself
  int32_t pcur;     // BiCGStab: current p buffer
  int32_t Pcur;     // current P buffer
  int32_t have_delta;
  int32_t done;
  int32_t status;   // pi_status
  int32_t nonfinite;
  int32_t stop_at;  // CG: first pass of the current outer step that did not
                    // run because the inner solve had converged (kNoStop if
                    // none); passes 0 .. min(stop_at, inner_iters) - 1 ran
  int32_t dvalid;   // BiCGStab: the correction buffer holds this outer step's
                    // sum (an update has run since the outer step began)
};

}  // namespace pi
