// Plan construction: argument checks, ray-count constants, packed counter
// codes, connected groups of data cells, and device workspace.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "pi_kernels.h"
#include "pi_plan.h"

namespace pi {

// ---------------------------------------------------------------------------
// counter codes (per cell, per face direction)
// ---------------------------------------------------------------------------
// For a data cell C and face direction j with neighbour J = C + s e_a:
// state 0 when J lies outside the grid or holds no data; otherwise
// 1 + n1 + 3 n2 + 9 far (3-D) or 1 + n1 + 3 far (2-D), where n1, n2 count the
// laterals J +- e_k with data along the first and second remaining axis, and
// far tells whether J + s e_a holds data.  These are exactly the b~ values
// that Eqs. AEnp1 / AEn / ANnp1 / ANn (and the 3-D A_N equations) read.
template <int ND>
__global__ __launch_bounds__(256) void k_codes(int nx, int ny, int nz, const uint8_t *mask, uint32_t *code) {
  const int64_t ncell = (int64_t)nx * ny * nz;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const int x = (int)(c % nx);
  const int y = (int)((c / nx) % ny);
  const int z = (int)(c / ((int64_t)nx * ny));
  const int n[3] = {nx, ny, nz};
  auto valid = [&](int px, int py, int pz) -> int {
    if (px < 0 || px >= nx || py < 0 || py >= ny || pz < 0 || pz >= nz) return 0;
    return mask[(int64_t)px + (int64_t)nx * ((int64_t)py + (int64_t)ny * pz)] != 0;
  };
  if (!valid(x, y, z)) {
    code[c] = 0u;
    return;
  }
  const int bits = dir_bits(ND);
  uint32_t out = kValidBit;
  for (int d = 0; d < 2 * ND; ++d) {
    const int a = d >> 1;
    const int s = (d & 1) ? -1 : 1;
    int J[3] = {x, y, z};
    J[a] += s;
    if (!valid(J[0], J[1], J[2])) continue;
    int cnt[2] = {0, 0};
    int li = 0;
    for (int k = 0; k < ND; ++k) {
      if (k == a) continue;
      int Lp[3] = {J[0], J[1], J[2]}, Lm[3] = {J[0], J[1], J[2]};
      Lp[k] += 1;
      Lm[k] -= 1;
      cnt[li++] = valid(Lp[0], Lp[1], Lp[2]) + valid(Lm[0], Lm[1], Lm[2]);
    }
    int Fr[3] = {J[0], J[1], J[2]};
    Fr[a] += s;
    const int far = valid(Fr[0], Fr[1], Fr[2]);
    (void)n;
    const uint32_t state = ND == 3 ? 1u + cnt[0] + 3u * cnt[1] + 9u * far : 1u + cnt[0] + 3u * far;
    out |= state << (bits * d);
  }
  code[c] = out;
}

hipError_t launch_codes(int ndim, int nx, int ny, int nz, const uint8_t *mask, uint32_t *code, hipStream_t s) {
  const int64_t ncell = (int64_t)nx * ny * nz;
  const int64_t nb = (ncell + 255) / 256;
  if (ndim == 3)
    k_codes<3><<<dim3((unsigned)nb), dim3(256), 0, s>>>(nx, ny, nz, mask, code);
  else
    k_codes<2><<<dim3((unsigned)nb), dim3(256), 0, s>>>(nx, ny, nz, mask, code);
  return hipGetLastError();
}

// Cell-centred scheme (2-D): bit 31 = data, bit cc_bit(dx, dy) = data at
// C + (dx, dy) for |dx|, |dy| <= 2; cells outside the grid hold no data.
__global__ __launch_bounds__(256) void k_codes_cc(int nx, int ny, const uint8_t *mask, uint32_t *code) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (int64_t)nx * ny) return;
  const int x = (int)(c % nx), y = (int)(c / nx);
  auto valid = [&](int px, int py) -> bool {
    return px >= 0 && px < nx && py >= 0 && py < ny && mask[(int64_t)px + (int64_t)nx * py] != 0;
  };
  if (!valid(x, y)) {
    code[c] = 0u;
    return;
  }
  uint32_t out = kValidBit;
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx)
      if ((dx != 0 || dy != 0) && valid(x + dx, y + dy)) out |= 1u << cc_bit(dx, dy);
  code[c] = out;
}

hipError_t launch_codes_cc(int nx, int ny, const uint8_t *mask, uint32_t *code) {
  const int64_t nb = ((int64_t)nx * ny + 255) / 256;
  k_codes_cc<<<dim3((unsigned)nb), dim3(256), 0, nullptr>>>(nx, ny, mask, code);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// quadrature for the anisotropic 3-D constants
// ---------------------------------------------------------------------------
// Gauss-Legendre nodes by Newton's method on the Legendre recurrence, used as
// a composite rule with interval halving until two levels agree.
struct GaussLegendre {
  std::vector<double> x, w;
  explicit GaussLegendre(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      double z = cos(M_PI * (i + 0.75) / (n + 0.5));
      double dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = 0.0;
        for (int j = 1; j <= n; ++j) {
          const double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        const double dz = p0 / dp;
        z -= dz;
        if (fabs(dz) < 1e-16) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
  template <class F>
  double rule(const F &f, double a, double b) const {
    const double h = 0.5 * (b - a), m = 0.5 * (a + b);
    double s = 0.0;
    for (size_t i = 0; i < x.size(); ++i) s += w[i] * f(m + h * x[i]);
    return s * h;
  }
  template <class F>
  double adapt(const F &f, double a, double b, double whole, double tol, int depth) const {
    const double m = 0.5 * (a + b);
    const double l = rule(f, a, m), r = rule(f, m, b);
    if (fabs(l + r - whole) <= tol || depth >= 48) return l + r;
    return adapt(f, a, m, l, 0.5 * tol, depth + 1) + adapt(f, m, b, r, 0.5 * tol, depth + 1);
  }
  template <class F>
  double integrate(const F &f, double a, double b, double tol = 1e-15) const {
    if (b <= a) return 0.0;
    return adapt(f, a, b, rule(f, a, b), tol, 0);
  }
};

// c_jj of Eq. FarFaceEquation; dj normal spacing, dl1/dl2 in-plane spacings.
static double far_face(const GaussLegendre &gl, double dj, double dl1, double dl2) {
  auto f = [&](double phi) {
    const double l1c = dl1 * cos(phi), l1s = dl1 * sin(phi);
    const double at = atan(dj / l1s);
    return M_PI * (dl2 * l1s - dj * l1c) + 2.0 * (dj * l1c * at - dl2 * l1s * at);
  };
  return gl.integrate(f, atan(dj / dl2), 0.5 * M_PI);
}

// c_jk (j != k) = I_A + I_B1 + I_B2 + I_C (Eqs. IAc, IB1c, IB2c, ICc).
static double dihedral(const GaussLegendre &gl, double dj, double dk, double dl) {
  const double dj2 = dj * dj, dk2 = dk * dk, dl2 = dl * dl;
  const double IA = 0.5 * dl2 * atanh(dj2 * dk2 / (2 * dl2 * dl2 + 2 * dl2 * dj2 + 2 * dl2 * dk2 + dj2 * dk2));
  const double phi0 = atan(dj / dl);
  auto b1 = [&](double phi) {
    const double kc = dk * cos(phi), ks = dk * sin(phi);
    return dl * ks * (atan(dl / kc) - dl * kc / (dl2 + kc * kc)) +
           kc * ks * (log(kc / sqrt(kc * kc + dl2)) + dl2 / (2.0 * (dl2 + kc * kc)));
  };
  auto b2 = [&](double phi) {
    const double kc = dk * cos(phi), ks = dk * sin(phi);
    return dl * ks * (atan(dj / ks) - dj * ks / (dj2 + ks * ks)) +
           kc * ks * (log(ks / sqrt(ks * ks + dj2)) + dj2 / (2.0 * (dj2 + ks * ks)));
  };
  auto ic = [&](double phi) {
    const double s = sin(phi);
    return 0.5 * dj * dk2 * s * (2.0 * dl * s - dj * cos(phi)) / (dj2 + dk2 * s * s);
  };
  return IA + gl.integrate(b1, 0.0, phi0) + gl.integrate(b2, phi0, 0.5 * M_PI) + gl.integrate(ic, phi0, 0.5 * M_PI);
}

static void constants(pi_plan_s *p) {
  const double dx = p->spacing[0], dy = p->spacing[1], dz = p->spacing[2];
  if (p->ndim == 2) {
    // Eq. cxx2D; A_tot of Eq. Atot2D; face totals 2 * (face length), Eq. AE_Interior
    const double dd = sqrt(dx * dx + dy * dy);
    p->c[0][0] = 2.0 * (dd - dx);
    p->c[1][1] = 2.0 * (dd - dy);
    p->c[0][1] = p->c[1][0] = dx + dy - dd;
    p->Atot = 4.0 * (dx + dy);
    p->face[0] = 2.0 * dy;
    p->face[1] = 2.0 * dx;
    return;
  }
  if (dx == dy && dy == dz) {
    // Eqs. ConstantFarFace and ConstantNearFaces
    const double r2 = sqrt(2.0), D2 = dx * dx;
    const double far = log(4.0 / 3.0) - r2 * atan(r2) + 0.5 * r2 * atan(10.0 * r2 / 23.0) + M_PI * (r2 - 1.0);
    const double nr = 0.5 * M_PI - 0.25 * log(4.0 / 3.0) - 0.25 * r2 * atan(10.0 * r2 / 23.0) - 0.5 * r2 * atan(r2);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) p->c[a][b] = (a == b ? far : nr) * D2;
  } else {
    const GaussLegendre gl(24);
    const double d[3] = {dx, dy, dz};
    for (int a = 0; a < 3; ++a) {
      const double l1 = d[(a + 1) % 3], l2 = d[(a + 2) % 3];
      p->c[a][a] = far_face(gl, d[a], l1, l2);
    }
    for (int a = 0; a < 3; ++a)
      for (int b = a + 1; b < 3; ++b) {
        const double l = d[3 - a - b];
        p->c[a][b] = p->c[b][a] = dihedral(gl, d[a], d[b], l);
      }
  }
  p->Atot = 2.0 * M_PI * (dx * dy + dx * dz + dy * dz);
  p->face[0] = M_PI * dy * dz;
  p->face[1] = M_PI * dx * dz;
  p->face[2] = M_PI * dx * dy;
}

// Per-(direction, state) weights w^{n+1} = A^{n+1} / A_tot and w^n = A^n / A_tot,
// decoding the state back into the lateral counts and the far flag.
static void fill_luts(pi_plan_s *p, Inst &in) {
  const int nd = p->ndim;
  for (int d = 0; d < 6; ++d) {
    for (int s = 0; s < kStates; ++s) {
      in.lut_np1[d][s] = 0.0;
      in.lut_n[d][s] = 0.0;
    }
    in.a[d] = 0.0;
    in.dsig[d] = 0.0;
  }
  for (int d = 0; d < 2 * nd; ++d) {
    const int a = d >> 1;
    const double sg = (d & 1) ? -1.0 : 1.0;
    int lat[2] = {-1, -1}, li = 0;
    for (int k = 0; k < nd; ++k)
      if (k != a) lat[li++] = k;
    const int nstates = nd == 3 ? 18 : 6;
    for (int s = 1; s <= nstates; ++s) {
      const int t = s - 1;
      int n1, n2, far;
      if (nd == 3) {
        n1 = t % 3;
        n2 = (t / 3) % 3;
        far = t / 9;
      } else {
        n1 = t % 3;
        n2 = 0;
        far = t / 3;
      }
      double Anp1 = p->c[a][lat[0]] * n1 + p->c[a][a] * far;
      double An = p->c[a][lat[0]] * (2 - n1) + p->c[a][a] * (1 - far);
      if (nd == 3) {
        Anp1 += p->c[a][lat[1]] * n2;
        An += p->c[a][lat[1]] * (2 - n2);
      }
      in.lut_np1[d][s] = Anp1 / p->Atot;
      in.lut_n[d][s] = An / p->Atot;
    }
    in.a[d] = p->face[a] / p->Atot;
    in.dsig[d] = sg * p->spacing[a];
  }
}

// Cell-centred constants.  Along major axis spacing hM (lateral hm), a ray
// at angle phi from the axis, 0 < phi < phi_d = atan(hm / hM), shifts
// laterally by tau = hM tan(phi) / hm cells per step; the rays through C
// cover lateral offsets of one cell with measure hm cos(phi) per unit offset
// and angle.  The four pieces (see cc_pieces) have lengths tau, tau,
// 1 - 2 tau, 0 for tau < 1/2 and 1 - tau, 1 - tau, 0, 2 tau - 1 above, so
// with phi_h = atan(hm / (2 hM)) their measures integrate to
//   m0 = hM (1 - cos phi_h) + hm (sin phi_d - sin phi_h) - hM (cos phi_h - cos phi_d)
//   m1 = hm sin phi_h - 2 hM (1 - cos phi_h)
//   m2 = 2 hM (cos phi_h - cos phi_d) - hm (sin phi_d - sin phi_h)
// All rays through a cell measure A_tot = 4 |(dx, dy)|.
static void fill_cc(pi_plan_s *p, Inst &in) {
  const double hx = p->spacing[0], hy = p->spacing[1];
  const double Atot = 4.0 * sqrt(hx * hx + hy * hy);
  for (int maj = 0; maj < 2; ++maj) {
    const double hM = maj ? hy : hx, hm = maj ? hx : hy;
    const double pd = atan2(hm, hM), ph = atan2(hm, 2.0 * hM);
    const double cd = cos(pd), sd = sin(pd), ch = cos(ph), sh = sin(ph);
    in.cc_m[maj][0] = (hM * (1.0 - ch) + hm * (sd - sh) - hM * (ch - cd)) / Atot;
    in.cc_m[maj][1] = (hm * sh - 2.0 * hM * (1.0 - ch)) / Atot;
    in.cc_m[maj][2] = (2.0 * hM * (ch - cd) - hm * (sd - sh)) / Atot;
  }
  // per-direction totals, summed in the kernels' order so that an interior
  // cell gets the same weights by either route
  for (int j = 0; j < 8; ++j) {
    in.cc_a[j] = 0.0;
    in.cc_step[j][0] = cc_dx(j) * hx;
    in.cc_step[j][1] = cc_dy(j) * hy;
  }
  cc_pieces([&](int J, int, int, int maj, int mi) { in.cc_a[J] += in.cc_m[maj][mi]; });
  p->Atot = Atot;
}

void set_walk(Inst &in, int ndim, const int64_t dims[3], int mseg_override, int vw_override) {
  in.ndim = ndim;
  in.nx = (int32_t)dims[0];
  in.ny = (int32_t)dims[1];
  in.nz = ndim == 3 ? (int32_t)dims[2] : 1;
  in.ncell = (int64_t)in.nx * in.ny * in.nz;
  // four (two) cells per lane, 16-byte (8-byte) accesses, need rows that
  // start aligned to them; the default is the widest allowed (two only for
  // the face-crossing scheme), the measured order at every size tried
  const bool can4 = in.nx % 4 == 0, can2 = in.nx % 2 == 0 && !in.cc;
  in.vw = vw_override == 1 ? 1 : vw_override == 2 ? 2 : (can4 ? 4 : can2 ? 2 : 1);
  const int strip = kWave * in.vw;
  in.nxs = (in.nx + strip - 1) / strip;
  int64_t strips;
  if (ndim == 3) {
    in.rows = in.ny;
    in.nm = in.nz;
    in.sm = (int64_t)in.nx * in.ny;
    in.srow = in.nx;
    strips = (int64_t)in.nxs * in.rows;
  } else {
    in.rows = 1;
    in.nm = in.ny;
    in.sm = in.nx;
    in.srow = 0;
    strips = in.nxs;
  }
  int mseg = mseg_override;
  if (mseg <= 0) {
    // about one occupancy round of waves (8 per SIMD on 256 CUs)
    const int64_t target_waves = 8192;
    const int64_t nseg_t = std::max<int64_t>(1, target_waves / std::max<int64_t>(1, strips));
    mseg = (int)std::max<int64_t>(4, (in.nm + nseg_t - 1) / nseg_t);
  }
  mseg = std::max(1, std::min(mseg, in.nm));
  in.mseg = mseg;
  in.nseg = (in.nm + mseg - 1) / mseg;
  in.nwaves = strips * in.nseg;
  in.nblocks = (int32_t)((in.nwaves + kWavesPerBlock - 1) / kWavesPerBlock);
}

std::vector<BlockEnt> build_table(const std::vector<Inst *> &insts, int part_base0, int *part_total,
                                  bool assign_parts) {
  std::vector<std::vector<BlockEnt>> q(kXcd);
  int base = part_base0;
  for (size_t i = 0; i < insts.size(); ++i) {
    Inst *in = insts[i];
    if (assign_parts) in->part_base = base;
    base += in->nblocks;
    const int B = in->nblocks;
    for (int k = 0; k < kXcd; ++k) {
      const int lo = (int)((int64_t)B * k / kXcd), hi = (int)((int64_t)B * (k + 1) / kXcd);
      for (int b = lo; b < hi; ++b) q[k].push_back(BlockEnt{(int32_t)i, b});
    }
  }
  size_t len = 0;
  for (auto &v : q) len = std::max(len, v.size());
  std::vector<BlockEnt> tab(len * kXcd, BlockEnt{-1, 0});
  for (int k = 0; k < kXcd; ++k)
    for (size_t j = 0; j < q[k].size(); ++j) tab[j * kXcd + k] = q[k][j];
  if (part_total) *part_total = base;
  return tab;
}

hipError_t plan_alloc(pi_plan_s *p, void **ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) return hipSuccess;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e == hipSuccess) p->bytes += bytes;
  return e;
}

// Union-find over adjacent data cells (host, once per plan): face neighbours,
// and diagonal ones for the cell-centred scheme.
static int32_t components(const pi_plan_s *p, const uint8_t *mask, std::vector<int32_t> &label,
                          std::vector<int64_t> &count) {
  const int64_t n = p->ncell;
  const int64_t nx = p->dims[0], ny = p->dims[1];
  std::vector<int32_t> parent(n);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int32_t a) {
    while (parent[a] != a) {
      parent[a] = parent[parent[a]];
      a = parent[a];
    }
    return a;
  };
  auto unite = [&](int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a != b) {
      if (a < b)
        parent[b] = a;
      else
        parent[a] = b;
    }
  };
  const int64_t sy = nx, sz = nx * ny;
  for (int64_t c = 0; c < n; ++c) {
    if (!mask[c]) continue;
    const int64_t x = c % nx, y = (c / nx) % ny, z = c / sz;
    if (x + 1 < nx && mask[c + 1]) unite((int32_t)c, (int32_t)(c + 1));
    if (y + 1 < ny && mask[c + sy]) unite((int32_t)c, (int32_t)(c + sy));
    if (p->cc && y + 1 < ny) {  // the cell-centred scheme couples diagonal neighbours
      if (x + 1 < nx && mask[c + sy + 1]) unite((int32_t)c, (int32_t)(c + sy + 1));
      if (x >= 1 && mask[c + sy - 1]) unite((int32_t)c, (int32_t)(c + sy - 1));
    }
    if (p->ndim == 3 && z + 1 < p->dims[2] && mask[c + sz]) unite((int32_t)c, (int32_t)(c + sz));
  }
  label.assign(n, -1);
  std::vector<int32_t> id(n, -1);
  int32_t k = 0;
  count.clear();
  for (int64_t c = 0; c < n; ++c) {
    if (!mask[c]) continue;
    const int32_t r = find((int32_t)c);
    if (id[r] < 0) {
      id[r] = k++;
      count.push_back(0);
    }
    label[c] = id[r];
    count[id[r]] += 1;
  }
  return k;
}

// (Re)build the single-instance block table and partial-sum slots for the
// plan's current strip decomposition.
hipError_t plan_tables(pi_plan_s *p) {
  if (p->d_tab) (void)hipFree(p->d_tab);
  if (p->d_tab_rq) (void)hipFree(p->d_tab_rq);
  if (p->d_part) (void)hipFree(p->d_part);
  p->d_tab = nullptr;
  p->d_tab_rq = nullptr;
  p->d_part = nullptr;
  p->ntab = 0;  // no table until the new one is in place
  p->ntab_rq = 0;
  std::vector<Inst *> one{&p->inst};
  int parts = 0;
  std::vector<BlockEnt> tab = build_table(one, 0, &parts);
  // three partial-sum arrays: the outer-step kernels', and one per parity
  // of the inner CG passes
  // CG passes without a stored q: 3-D, no missing data, FP32, four cells per
  // lane, and rows whose overlapping wave windows (rq_nstrips) are as many as
  // the plan's wave strips, so the interior blocks keep the plan's table.
  // Their boundary-layer blocks come first
  // in the CG passes' table (dispatched first, they run beside the interior
  // blocks) and have partial-sum slots of their own after the others.
  p->inst.cg_rq = (p->ndim == 3 && p->inst.gen && !p->fp64 && !p->bicgstab && !p->cc && p->inst.vw == 4 &&
                   p->inst.nxs == rq_nstrips(p->inst.nx))
                      ? 1
                      : 0;
  const int nbnd =
      p->inst.cg_rq ? (int)((rq_ntasks(p->inst.ny, p->inst.nm, p->inst.nxs) + kWavesPerBlock - 1) / kWavesPerBlock) : 0;
  p->inst.cg_slots = p->inst.nblocks + nbnd;
  p->inst.part_stride = std::max(parts, p->inst.cg_slots);
  p->inst.cg_inline = p->inst.cg_slots <= kInlineMaxBlocks ? 1 : 0;
  std::vector<BlockEnt> tab_rq;
  if (p->inst.cg_rq) {
    for (int j = 0; j < nbnd; ++j) tab_rq.push_back(BlockEnt{0, p->inst.nblocks + j});
    tab_rq.insert(tab_rq.end(), tab.begin(), tab.end());
  }
  hipError_t e = hipMalloc((void **)&p->d_tab, tab.size() * sizeof(BlockEnt));
  if (e == hipSuccess)
    e = hipMalloc((void **)&p->d_part, (size_t)std::max(p->inst.part_stride, 1) * 3 * 4 * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(p->d_tab, tab.data(), tab.size() * sizeof(BlockEnt), hipMemcpyHostToDevice);
  if (e == hipSuccess && !tab_rq.empty()) {
    e = hipMalloc((void **)&p->d_tab_rq, tab_rq.size() * sizeof(BlockEnt));
    if (e == hipSuccess)
      e = hipMemcpy(p->d_tab_rq, tab_rq.data(), tab_rq.size() * sizeof(BlockEnt), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    p->ntab = (int)tab.size();
    p->ntab_rq = (int)tab_rq.size();
  } else {
    if (p->d_tab) (void)hipFree(p->d_tab);
    if (p->d_tab_rq) (void)hipFree(p->d_tab_rq);
    if (p->d_part) (void)hipFree(p->d_part);
    p->d_tab = nullptr;
    p->d_tab_rq = nullptr;
    p->d_part = nullptr;
  }
  return e;
}

}  // namespace pi

using namespace pi;

#define PI_TRY(expr)                 \
  do {                               \
    if ((expr) != hipSuccess) {      \
      pi_plan_destroy(p);            \
      return PI_ERR_OOM;             \
    }                                \
  } while (0)

extern "C" pi_status pi_plan(int ndim, const int64_t dims[3], const double spacing[3], const uint8_t *mask,
                             uint32_t flags, pi_plan_t *out) {
  if (!out) return PI_ERR_INVALID_ARG;
  *out = nullptr;
  if ((ndim != 2 && ndim != 3) || !dims || !spacing) return PI_ERR_INVALID_ARG;
  if (flags & ~(PI_FP64 | PI_INNER_BICGSTAB | PI_FIXED_POINT_CG | PI_CELL_CENTERED)) return PI_ERR_INVALID_ARG;
  if ((flags & PI_FIXED_POINT_CG) && (flags & PI_INNER_BICGSTAB)) return PI_ERR_INVALID_ARG;
  if ((flags & PI_CELL_CENTERED) && (ndim != 2 || (flags & PI_INNER_BICGSTAB))) return PI_ERR_INVALID_ARG;
  int64_t ncell = 1;
  for (int a = 0; a < ndim; ++a) {
    if (dims[a] < 1 || dims[a] >= (int64_t(1) << 31)) return PI_ERR_INVALID_ARG;
    if (!(spacing[a] > 0.0) || !isfinite(spacing[a])) return PI_ERR_INVALID_ARG;
    ncell *= dims[a];
    if (ncell >= (int64_t(1) << 31)) return PI_ERR_INVALID_ARG;
  }
  pi_plan_s *p = new (std::nothrow) pi_plan_s();
  if (!p) return PI_ERR_OOM;
  p->ndim = ndim;
  for (int a = 0; a < 3; ++a) {
    p->dims[a] = a < ndim ? dims[a] : 1;
    p->spacing[a] = a < ndim ? spacing[a] : 1.0;
  }
  p->flags = flags;
  p->fp64 = (flags & PI_FP64) != 0;
  p->bicgstab = (flags & PI_INNER_BICGSTAB) != 0;
  p->fixed_point = (flags & PI_FIXED_POINT_CG) != 0;
  p->cc = (flags & PI_CELL_CENTERED) != 0;
  p->ncell = ncell;
  // inner iterations per outer step.  The outer step count falls towards its
  // exact-inner limit (about 16 times the longest side) as k grows, while an
  // outer step costs about k inner passes; measured on this GPU the best k
  // grows with log2 of the longest side L: 3-D 6 (L = 64), 8-12 (128),
  // 12 (256); 2-D 12 (512), 16-24 (2048).
  {
    int64_t L = 1;
    for (int a = 0; a < ndim; ++a) L = std::max<int64_t>(L, p->dims[a]);
    int lg = 0;
    while ((int64_t(1) << lg) < L) ++lg;
    p->inner_iters = ndim == 3 ? std::min(24, std::max(4, 3 * lg - 12)) : std::min(32, std::max(4, 4 * lg - 24));
    // the fixed-point variant restarts CG once per outer step and stops it
    // early once the tolerance is met: a restart length of a few times the
    // longest side lets one or two outer steps do
    if (p->fixed_point) p->inner_iters = (int)std::min<int64_t>(4096, std::max<int64_t>(32, 4 * L));
  }

  // data cells and their connected groups
  std::vector<uint8_t> ones;
  const uint8_t *m = mask;
  if (!m) {
    ones.assign(ncell, 1);
    m = ones.data();
  }
  int64_t nvalid = 0;
  for (int64_t c = 0; c < ncell; ++c) nvalid += m[c] != 0;
  if (nvalid == 0) {
    delete p;
    return PI_ERR_INVALID_ARG;
  }
  p->nvalid = nvalid;
  std::vector<int32_t> label;
  std::vector<int64_t> count;
  if (mask) {
    p->ncomp = components(p, m, label, count);
  } else {
    p->ncomp = 1;
  }

  constants(p);
  const size_t T = p->fp64 ? sizeof(double) : sizeof(float);
  const size_t N = (size_t)ncell;
  Inst &in = p->inst;
  memset(&in, 0, sizeof(in));
  in.cc = p->cc ? 1 : 0;
  set_walk(in, ndim, p->dims, 0, 0);
  in.gen = (mask || p->cc) ? 0 : 1;  // the cell-centred kernels always read codes
  in.inner_op = p->fixed_point ? 1 : 0;
  in.bicg = p->bicgstab ? 1 : 0;
  // relative r.r at which the variant's CG has reached the precision of its
  // vectors (about a relative residual of 1e-7 in FP32, 1e-13 in FP64)
  in.inner_floor = p->fixed_point ? (p->fp64 ? 1e-26 : 1e-14) : 0.0;
  fill_luts(p, in);
  if (p->cc) fill_cc(p, in);
  in.ncomp = p->ncomp;
  in.inv_nvalid = 1.0 / (double)nvalid;

  // counter codes from the mask
  uint8_t *d_mask = nullptr;
  if (hipMalloc((void **)&d_mask, N) != hipSuccess) {
    pi_plan_destroy(p);
    return PI_ERR_OOM;
  }
  PI_TRY(plan_alloc(p, (void **)&p->code, N * sizeof(uint32_t)));
  if (hipMemcpy(d_mask, m, N, hipMemcpyHostToDevice) != hipSuccess ||
      (p->cc ? launch_codes_cc((int)p->dims[0], (int)p->dims[1], d_mask, p->code)
             : launch_codes(ndim, (int)p->dims[0], (int)p->dims[1], (int)p->dims[2], d_mask, p->code, nullptr)) !=
          hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(d_mask);
    pi_plan_destroy(p);
    return PI_ERR_DEVICE;
  }
  (void)hipFree(d_mask);
  in.code = p->code;

  if (p->ncomp > 1) {
    std::vector<double> inv(p->ncomp);
    for (int32_t k = 0; k < p->ncomp; ++k) inv[k] = 1.0 / (double)count[k];
    PI_TRY(plan_alloc(p, (void **)&p->label, N * sizeof(int32_t)));
    PI_TRY(plan_alloc(p, (void **)&p->comp_inv, inv.size() * sizeof(double)));
    PI_TRY(plan_alloc(p, (void **)&p->comp_sum, inv.size() * sizeof(double)));
    if (hipMemcpy(p->label, label.data(), N * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->comp_inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      pi_plan_destroy(p);
      return PI_ERR_DEVICE;
    }
    // data cells sorted by group (counting sort keeps index order inside a
    // group), cut into segments that never straddle two groups
    std::vector<int32_t> first(p->ncomp + 1, 0);
    for (int32_t k = 0; k < p->ncomp; ++k) first[k + 1] = first[k] + (int32_t)count[k];
    std::vector<int32_t> order(nvalid), fill(first.begin(), first.end() - 1);
    for (int64_t c = 0; c < ncell; ++c)
      if (label[c] >= 0) order[fill[label[c]]++] = (int32_t)c;
    std::vector<int32_t> seg_begin, comp_seg(p->ncomp + 1, 0);
    for (int32_t k = 0; k < p->ncomp; ++k) {
      comp_seg[k] = (int32_t)seg_begin.size();
      for (int32_t b = first[k]; b < first[k + 1]; b += kSegCells) seg_begin.push_back(b);
    }
    comp_seg[p->ncomp] = (int32_t)seg_begin.size();
    const int32_t nseg = (int32_t)seg_begin.size();
    seg_begin.push_back((int32_t)nvalid);
    PI_TRY(plan_alloc(p, (void **)&p->comp_order, order.size() * sizeof(int32_t)));
    PI_TRY(plan_alloc(p, (void **)&p->seg_begin, seg_begin.size() * sizeof(int32_t)));
    PI_TRY(plan_alloc(p, (void **)&p->comp_seg, comp_seg.size() * sizeof(int32_t)));
    PI_TRY(plan_alloc(p, (void **)&p->seg_sum, (size_t)nseg * sizeof(double)));
    if (hipMemcpy(p->comp_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->seg_begin, seg_begin.data(), seg_begin.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->comp_seg, comp_seg.data(), comp_seg.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
            hipSuccess) {
      pi_plan_destroy(p);
      return PI_ERR_DEVICE;
    }
    in.label = p->label;
    in.comp_inv_count = p->comp_inv;
    in.comp_sum = p->comp_sum;
    in.comp_order = p->comp_order;
    in.seg_begin = p->seg_begin;
    in.comp_seg = p->comp_seg;
    in.seg_sum = p->seg_sum;
    in.nseg_g = nseg;
  }

  // workspace
  PI_TRY(plan_alloc(p, (void **)&p->P[0], N * sizeof(double)));
  PI_TRY(plan_alloc(p, (void **)&p->P[1], N * sizeof(double)));
  PI_TRY(plan_alloc(p, (void **)&p->S64, N * sizeof(double)));
  PI_TRY(plan_alloc(p, &p->res, N * T));
  PI_TRY(plan_alloc(p, &p->p[0], N * T));
  PI_TRY(plan_alloc(p, &p->p[1], N * T));
  PI_TRY(plan_alloc(p, &p->q, N * T));
  PI_TRY(plan_alloc(p, &p->d, N * T));
  if (!p->bicgstab) {  // CG ping-pongs its residual and M p
    PI_TRY(plan_alloc(p, &p->res1, N * T));
    PI_TRY(plan_alloc(p, &p->q1, N * T));
  }
  if (p->bicgstab)
    for (int i = 0; i < 4; ++i) PI_TRY(plan_alloc(p, &p->bs[i], N * T));
  in.P[0] = p->P[0];
  in.P[1] = p->P[1];
  in.S64 = p->S64;
  in.S = nullptr;
  in.res = p->res;
  in.p[0] = p->p[0];
  in.p[1] = p->p[1];
  in.q = p->q;
  in.q1 = p->q1;
  in.res1 = p->res1;
  in.d = p->d;
  for (int i = 0; i < 4; ++i) in.bs[i] = p->bs[i];

  // single-instance launch state
  if (plan_tables(p) != hipSuccess) {
    pi_plan_destroy(p);
    return PI_ERR_OOM;
  }
  PI_TRY(plan_alloc(p, (void **)&p->d_inst, sizeof(Inst)));
  PI_TRY(plan_alloc(p, (void **)&p->d_state, sizeof(State)));
  if (hipHostMalloc((void **)&p->h_state, 3 * sizeof(State), hipHostMallocDefault) != hipSuccess) {
    pi_plan_destroy(p);
    return PI_ERR_OOM;
  }
  if (hipMemcpy(p->d_inst, &in, sizeof(Inst), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(p->d_state, 0, sizeof(State)) != hipSuccess) {
    pi_plan_destroy(p);
    return PI_ERR_DEVICE;
  }
  *out = p;
  return PI_OK;
}

extern "C" void pi_plan_destroy(pi_plan_t p) {
  if (!p) return;
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  void *ptrs[] = {p->code, p->label, p->comp_inv, p->comp_sum, p->comp_order, p->seg_begin, p->comp_seg,
                  p->seg_sum, p->P[0], p->P[1], p->S64, p->res, p->q, p->res1, p->q1,
                  p->d, p->p[0], p->p[1], p->bs[0], p->bs[1], p->bs[2], p->bs[3], p->d_inst, p->d_state,
                  p->d_tab, p->d_tab_rq, p->d_part};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  if (p->h_state) (void)hipHostFree(p->h_state);
  delete p;
}

extern "C" size_t pi_workspace_bytes(pi_plan_t p) { return p ? p->bytes : 0; }

extern "C" pi_status pi_set_tile(pi_plan_t p, int32_t mseg, int32_t lane_cells) {
  if (!p || mseg < 0 || (lane_cells != 0 && lane_cells != 1 && lane_cells != 2 && lane_cells != 4))
    return PI_ERR_INVALID_ARG;
  if (lane_cells == 4 && p->dims[0] % 4 != 0) return PI_ERR_INVALID_ARG;
  // two cells per lane: face-crossing plans with an even row length
  if (lane_cells == 2 && (p->dims[0] % 2 != 0 || p->cc)) return PI_ERR_INVALID_ARG;
  // the captured outer-step graph holds the old table: drop it first, so
  // that no failure below leaves it pointing at freed memory
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  p->graph = nullptr;
  p->graph_key = -1;
  set_walk(p->inst, p->ndim, p->dims, mseg, lane_cells);
  if (plan_tables(p) != hipSuccess) return PI_ERR_OOM;
  if (hipMemcpy(p->d_inst, &p->inst, sizeof(Inst), hipMemcpyHostToDevice) != hipSuccess) return PI_ERR_DEVICE;
  return PI_OK;
}

extern "C" int32_t pi_get_tile(pi_plan_t p) { return p ? p->inst.mseg : 0; }

extern "C" int32_t pi_get_lane_cells(pi_plan_t p) { return p ? p->inst.vw : 0; }

extern "C" pi_status pi_set_inner_iters(pi_plan_t p, int32_t iters) {
  if (!p || iters < 1 || iters > 4096) return PI_ERR_INVALID_ARG;
  p->inner_iters = iters;
  return PI_OK;
}
