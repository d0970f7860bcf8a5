// vp_kernels.hpp -- HIP kernels (gfx950) of the metric semi-Lagrangian
// Vlasov-Poisson engine (Colombi & Alard, arXiv:1705.03750).
//
// Arithmetic is written operation by operation (fma only where written; the
// library is compiled with -ffp-contract=off) so that the FP64 path rounds
// exactly like a plain sequential evaluation of the same formulas.
//
// Data layout in device memory (all inside the caller's workspace):
//   F, C      padded [nv + 2*PV][pitch] arrays, pitch = nx + 2*PX, the grid
//             interior starting at (PV, PX).  F's padding is zero (data
//             outside the box); C carries mirror ghosts one site deep.
//   state     element state, SoA [12][E] doubles.
//   rec       per-element query record, AoS [E][12] doubles (96 B), rebuilt
//             after every drift: position, A = T^-1, -H/2 (xv terms doubled).
//   qm        lattice position Q_m of every element, [E][2] doubles.
//   cnt, lst  element lists of 8x8-site query blocks: every element whose
//             validity window holds a site of a block is listed in that
//             block.  Blocks of one 64-row group are shifted along x to
//             follow the drift of the elements since their last reset
//             (group_ox), so that they stay aligned with the element
//             lattice and a block meets few windows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vpk {

constexpr int PX = 16;  // x padding of F / C (values)
constexpr int PV = 2;   // v padding of F / C (rows)
constexpr int RS = 12;  // doubles per element query record (96 B)
constexpr int SPAN_LIMIT = 4096;  // max query blocks one element may enter

enum {
  R_X = 0, R_V, R_AXX, R_AXV, R_AVX, R_AVV,
  // -H/2 (the off-diagonal term doubled): the map's -A/2 factor moved onto
  // H, which scales every rounding step by an exact power of two
  R_HXXX, R_H2XXV, R_HXVV, R_HVXX, R_H2VXV, R_HVVV
};
enum {
  S_X = 0, S_V, S_TXX, S_TXV, S_TVX, S_TVV, S_HXXX, S_HXXV, S_HXVV, S_HVXX,
  S_HVXV, S_HVVV, NSTATE
};
enum { FLAG_NUMERIC = 1, FLAG_WIDE = 2 };
enum { MODE_DENSITY = 0, MODE_F = 1, MODE_ASSIGN = 2, MODE_DIAG = 3,
       MODE_EMAP = 4 };  // MODE_EMAP: the E_map maximum of MODE_DIAG alone
// Per-workgroup diagnostic partials of MODE_DIAG: sum v^2 f, sum f ln|f|,
// the largest E_map site value, sum |f|, sum f^2.
enum { DP_KIN = 0, DP_ENT, DP_EMAP, DP_L1, DP_L2, DPS };

struct KP {
  int nx, nv, sx, sv, mx, mv, E;
  int ox, ov, obx, obv, nbx, nbv, ngy, cap, pitch;
  double x_min, v_min, dx, dv, inv_dx, inv_dv, dxm, dvm, rx, rv;
  double G, dt, h, beta;
  int force_mode;
  double a0, a1, a2;
  double tau;  // time since the elements' last reset (query-block shift)
  // Variable time step (section 2.4), used when clk != nullptr: dt is then
  // the cap, and the step sizes, times and tau live in the device clock
  // below instead of the fields above.
  double cdyn;
  double *clk;
  int par;  // clock slot of the current step (step count & 1)
  // Periodic x (the plasma / periodic-gravity variant): period Lx, half
  // period hL, and nbl = nx / 8 query blocks per row, the first and the
  // last block column of a row group being one block split by the seam.
  int per, nbl;
  double Lx, hL, x_max;
  // rx == rv, a power of two: the query ranks candidates by the unscaled
  // squared offset, which is the scaled one divided by rx^2 exactly
  int r2;
  // query-block x shift of the row groups at list time tau (gox_set)
  long long goxA, goxB;
  // ceil(2^40 / nbx) when it splits every tile index exactly, else 0
  unsigned long long tdm;
};

// The drift at row group gy's central velocity since the elements' last
// reset, in sites, is (goxB + gy goxA) / 2^32 (32.32 fixed point; zero for
// a non-finite or huge drift).  Set wherever the list time is, so that the
// block lists and the queries that read them take the same geometry.
__host__ __device__ inline void gox_set(KP &p) {
  const double a = 64.0 * p.dv * p.tau * p.inv_dx;
  const double b =
      (p.v_min + ((double)(p.ov - 64 * p.obv + 32) + 0.5) * p.dv) * p.tau *
      p.inv_dx;
  if (fabs(a) * (double)(p.ngy + 1) + fabs(b) < 1.0e6) {
    p.goxA = llrint(a * 4294967296.0);
    p.goxB = llrint(b * 4294967296.0);
  } else {
    p.goxA = 0;
    p.goxB = 0;
  }
}

// Periodic x: a position moved out of [x_min, x_max) by a drift re-enters
// from the other side (one period at most; a sum that rounds onto x_max is
// put on x_min).
__device__ __forceinline__ double wrap_x(const KP &p, double x) {
  if (x < p.x_min) {
    x = x + p.Lx;
    if (x >= p.x_max) x = p.x_min;
  } else if (x >= p.x_max) {
    x = x - p.Lx;
    if (x < p.x_min) x = p.x_min;
  }
  return x;
}

// x offset of a site from an element, through the element's nearest image
// when x is periodic.
template <int PER>
__device__ __forceinline__ double image_dx(const KP &p, double d) {
  if (PER) {
    if (d > p.hL)
      d = d - p.Lx;
    else if (d < -p.hL)
      d = d + p.Lx;
  }
  return d;
}

// Block column whose list a reconstruction block reads: with periodic x the
// last column (the right part of the seam block) shares the first one's.
__device__ __forceinline__ int list_bx(const KP &p, int bx) {
  return (p.per && bx >= p.nbl) ? bx - p.nbl : bx;
}

// Device clock of a variable-step run: two slots of {dt, t, t_r, tau}, the
// slot of step n holding the step size and start time of step n, the time
// t_r of the elements' last reset and the list time tau of the last
// registration; and rho_max of the last density the field kernels saw.
// The element pass that completes step n reads slot n & 1 and writes slot
// (n + 1) & 1, so no launch reads a slot it writes.
enum { CK_DT = 0, CK_T, CK_TR, CK_TAU, CK_SLOT = 4, CK_RHO = 8,
       CK_DOUBLES = 16 };

// The step after a density with maximum rho_max: the largest dt <= cap that
// satisfies dt <= C_dyn / sqrt(rho_max) (section 2.4); the cap when no
// density is positive.  The cap is p.dt as the host set it.
__device__ __forceinline__ double next_dt(const KP &p, double rho_max) {
  if (!(rho_max > 0.0)) return p.dt;
  const double d = p.cdyn / sqrt(rho_max);
  return d < p.dt ? d : p.dt;
}

// List time of the current slot (kernels that read the block lists).
__device__ __forceinline__ void clock_tau(KP &p) {
  if (p.clk) {
    p.tau = p.clk[CK_SLOT * p.par + CK_TAU];
    gox_set(p);
  }
}

__device__ __forceinline__ double site_x(const KP &p, int i) {
  return p.x_min + ((double)i + 0.5) * p.dx;
}
__device__ __forceinline__ double site_v(const KP &p, int j) {
  return p.v_min + ((double)j + 0.5) * p.dv;
}
// query block of a site index along one axis (blocks of 8 sites whose
// boundaries sit o sites after a multiple of 8; a partial block 0 when o > 0)
__device__ __forceinline__ int blk(int i, int o, int ob) {
  return ((i - o) >> 3) + ob;
}

// Row group (64 rows, one reconstruction workgroup row) of a block row.
__device__ __forceinline__ int group_of_brow(const KP &p, int bv) {
  return p.obv + ((bv - p.obv) >> 3);
}

// x offset (0..7) of the query blocks of row group gy.  Elements drift by
// v tau along x since their last reset (when they sat on the lattice, at
// offset ox); the blocks of a row group move with the drift at the group's
// central velocity, rounded up, so that an element lattice displaced by a
// fraction of a site meets two blocks per axis instead of three.  Block bx
// of the group covers columns [o + 8 (bx - 1), o + 8 bx).  Only the work
// depends on this choice: lists and queries use the same geometry.
__device__ __forceinline__ int group_ox(const KP &p, int gy) {
  const long long x = p.goxB + (long long)gy * p.goxA;
  return (p.ox + (int)(-((-x) >> 32))) & 7;  // ceil(x / 2^32)
}

// Tile t of the reconstruction grid as (block column bx, row group gy).
__device__ __forceinline__ void tile_split(const KP &p, int t, int &bx,
                                           int &gy) {
  gy = p.tdm ? (int)(((unsigned long long)t * p.tdm) >> 40) : t / p.nbx;
  bx = t - gy * p.nbx;
}

// Workgroups are dealt to the 8 XCDs round-robin; give every XCD a
// contiguous range of the T logical tiles so that its L2 holds the element
// records and F_ini rows of one band of the grid.
__device__ __forceinline__ int xcd_tile(int bid, int T) {
  const int xcd = bid & 7, idx = bid >> 3;
  const int base = T >> 3, extra = T & 7;
  return xcd * base + min(xcd, extra) + idx;
}

// ------------------------------------------------------------- elements

// One element update kernel for every phase of the leapfrog (section 2.4):
//   kick     dual TSC of a, a', a'' at the element (section 2.5), kick of v,
//            T_v. and H_v from the half-step positions, corrector drift;
//   predict  predictor drift (when `drift`), then the per-element inverse
//            A = T^-1 (end of section 2.1) and the query record; when `reg`,
//            the element enters every query block its validity window can
//            reach.
// Applying the corrector and the next predictor in one pass keeps the two
// half drifts as two roundings, exactly as two separate passes would.
// cnt_zero (nb_zero counts consumed by the previous reconstruction) is
// cleared grid-wide; registration goes to the other count buffer.
struct ElemState {
  double x, v, txx, txv, tvx, tvv, hx0, hx1, hx2, hv0, hv1, hv2;
};

__device__ __forceinline__ void elem_load(const double *__restrict__ st,
                                          size_t E, int e, ElemState &s) {
  s.x = st[S_X * E + e];
  s.v = st[S_V * E + e];
  s.txx = st[S_TXX * E + e];
  s.txv = st[S_TXV * E + e];
  s.tvx = st[S_TVX * E + e];
  s.tvv = st[S_TVV * E + e];
  s.hx0 = st[S_HXXX * E + e];
  s.hx1 = st[S_HXXV * E + e];
  s.hx2 = st[S_HXVV * E + e];
  s.hv0 = st[S_HVXX * E + e];
  s.hv1 = st[S_HVXV * E + e];
  s.hv2 = st[S_HVVV * E + e];
}

__device__ __forceinline__ void elem_store(double *__restrict__ st, size_t E,
                                           int e, const ElemState &s) {
  st[S_X * E + e] = s.x;
  st[S_V * E + e] = s.v;
  st[S_TXX * E + e] = s.txx;
  st[S_TXV * E + e] = s.txv;
  st[S_TVX * E + e] = s.tvx;
  st[S_TVV * E + e] = s.tvv;
  st[S_HXXX * E + e] = s.hx0;
  st[S_HXXV * E + e] = s.hx1;
  st[S_HXVV * E + e] = s.hx2;
  st[S_HVXX * E + e] = s.hv0;
  st[S_HVXV * E + e] = s.hv1;
  st[S_HVVV * E + e] = s.hv2;
}

__device__ __forceinline__ void elem_drift(const KP &p, ElemState &s) {
  s.x = fma(p.h, s.v, s.x);
  if (p.per) s.x = wrap_x(p, s.x);
  s.txx = fma(p.h, s.tvx, s.txx);
  s.txv = fma(p.h, s.tvv, s.txv);
  s.hx0 = fma(p.h, s.hv0, s.hx0);
  s.hx1 = fma(p.h, s.hv1, s.hx1);
  s.hx2 = fma(p.h, s.hv2, s.hx2);
}

// Force tables a, a', a'' on the indices [-4, nx + 3] (array index q = i + 4)
struct AccTable {
  const double *acc;
  int n8;
  __device__ __forceinline__ void at(int q, double &a, double &da,
                                     double &d2a) const {
    a = acc[q];
    da = acc[n8 + q];
    d2a = acc[2 * n8 + q];
  }
};

// TSC cell of a position (section 2.5): u = (x - x_min)/dx - 1/2, clamped
// to [-3, nx + 2] (the force is constant beyond the grid, and a NaN
// position lands on -3), its nearest site floor(u + 1/2) (returned) and the
// offset w of u from it.
__device__ __forceinline__ double tsc_cell(const KP &p, double x, double &w) {
  double u = (x - p.x_min) * p.inv_dx - 0.5;
  if (!(u >= -3.0)) u = -3.0;
  if (u > (double)p.nx + 2.0) u = (double)p.nx + 2.0;
  const double fi = floor(u + 0.5);
  w = u - fi;
  return fi;
}

template <typename Acc>
__device__ __forceinline__ void elem_kick(const KP &p, const Acc &acc,
                                          ElemState &s) {
  double a, da, d2a;
  if (p.force_mode == 1) {
    a = fma(fma(p.a2, s.x, p.a1), s.x, p.a0);
    da = fma(2.0 * p.a2, s.x, p.a1);
    d2a = 2.0 * p.a2;
  } else {
    double w;
    const double fi = tsc_cell(p, s.x, w);
    const double tm = 0.5 - w, tp = 0.5 + w;
    const double w0 = 0.5 * (tm * tm), w1 = 0.75 - w * w, w2 = 0.5 * (tp * tp);
    const int idx = (int)fi + 4;
    double am, dam, d2am, a0, da0, d2a0, ap, dap, d2ap;
    acc.at(idx - 1, am, dam, d2am);
    acc.at(idx, a0, da0, d2a0);
    acc.at(idx + 1, ap, dap, d2ap);
    a = fma(w2, ap, fma(w1, a0, w0 * am));
    da = fma(w2, dap, fma(w1, da0, w0 * dam));
    d2a = fma(w2, d2ap, fma(w1, d2a0, w0 * d2am));
  }
  const double dt = p.dt, kdt = dt * da;
  s.v = fma(dt, a, s.v);
  s.tvx = fma(kdt, s.txx, s.tvx);
  s.tvv = fma(kdt, s.txv, s.tvv);
  s.hv0 = fma(dt, fma(da, s.hx0, d2a * (s.txx * s.txx)), s.hv0);
  s.hv1 = fma(dt, fma(da, s.hx1, d2a * (s.txx * s.txv)), s.hv1);
  s.hv2 = fma(dt, fma(da, s.hx2, d2a * (s.txv * s.txv)), s.hv2);
  elem_drift(p, s);
}

// Query record and block registration of one element.  A non-finite
// element or det T <= 0 raises FLAG_NUMERIC and is not registered.
//
// elem_record_box writes the record and returns the element's registration
// box: the query blocks whose 8x8 sites its validity window's bounding box
// touches (n = 0 when there is nothing to register).  reg_block tests one
// block of the box: a block is listed only if the validity window
// |l| < (dx_m, dv_m), l = A (P - P_m), can hold one of its sites, so sheared
// windows do not fill the lists of the blocks their bounding box merely
// touches.  l is linear in P: over the block's 8x8 rectangle of sites (a
// superset of its live sites at the grid edges) it ranges over l(centre) +-
// the sum of |A_ij| x half-width.  A block is skipped only when a component
// stays outside the window by more than a margin covering the rounding of l
// at the sites, relative to the magnitudes of the products A_ij dP_j (which
// may cancel), taken at the largest distance of a block site from the
// element, so that per block only l(centre) remains to compute.
struct RegBox {
  int n;              // blocks in the box, wxm per block row
  int wxm, b0v, ilo, ihi, ga;
  int opack;          // x offsets (0..7) of the row groups ga, ga + 1, ga + 2
                      // in bits 0-2, 3-5, 6-8
  double x, v, axx, axv, avx, avv, limx, limv;
};

// A box of at most 9 block rows lies in at most three row groups (a group
// is 8 block rows), whose x offsets the box carries; taller boxes (very
// sheared elements) compute the offset per block.
constexpr int REG_NEAR_ROWS = 9;

__device__ __forceinline__ RegBox elem_record_box(
    const KP &p, const ElemState &s, int e, double *__restrict__ rec,
    double *__restrict__ qm, int *__restrict__ flags, int reg) {
  RegBox B;
  B.n = 0;
  const double det = fma(s.txx, s.tvv, -(s.txv * s.tvx));
  const bool bad = !(det > 0.0) || !isfinite(det) || !isfinite(s.x) ||
                   !isfinite(s.v);
  const double inv = 1.0 / det;
  const double axx = s.tvv * inv, axv = -s.txv * inv, avx = -s.tvx * inv,
               avv = s.txx * inv;
  const int k = e % p.mx, l = e / p.mx;
  double *r = rec + (size_t)e * RS;
  r[R_X] = s.x;
  r[R_V] = s.v;
  r[R_AXX] = axx;
  r[R_AXV] = axv;
  r[R_AVX] = avx;
  r[R_AVV] = avv;
  r[R_HXXX] = -0.5 * s.hx0;
  r[R_H2XXV] = -s.hx1;
  r[R_HXVV] = -0.5 * s.hx2;
  r[R_HVXX] = -0.5 * s.hv0;
  r[R_H2VXV] = -s.hv1;
  r[R_HVVV] = -0.5 * s.hv2;
  qm[2 * (size_t)e] = site_x(p, p.sx * k + p.sx / 2);
  qm[2 * (size_t)e + 1] = site_v(p, p.sv * l + p.sv / 2);
  // Eulerian reach of the validity window |A dP| < dx_m: |dP_x| <=
  // |Txx| dx_m + |Txv| dv_m, in site units.  The relative margin covers the
  // rounding of l = A dP (it grows with the condition number of T), the
  // absolute one the rounding of site and element coordinates.
  const double tsum = fabs(s.txx) + fabs(s.txv) + fabs(s.tvx) + fabs(s.tvv);
  const double rel = 0x1p-20 + 0x1p-40 * (tsum * tsum) * fabs(inv);
  const double rxs = (fabs(s.txx) * p.dxm + fabs(s.txv) * p.dvm) * p.inv_dx *
                         (1.0 + rel) + 0x1p-20;
  const double rvs = (fabs(s.tvx) * p.dxm + fabs(s.tvv) * p.dvm) * p.inv_dv *
                         (1.0 + rel) + 0x1p-20;
  if (bad) {
    atomicOr(flags, FLAG_NUMERIC);
    return B;
  }
  if (!reg) return B;
  const double cx = (s.x - p.x_min) * p.inv_dx - 0.5;
  const double cv = (s.v - p.v_min) * p.inv_dv - 0.5;
  const double vlo = fmax(cv - rvs, -1.0), vhi = fmin(cv + rvs, (double)p.nv);
  const int jlo = max(0, (int)ceil(vlo)), jhi = min(p.nv - 1, (int)floor(vhi));
  int ilo, ihi;
  if (p.per) {
    // unwrapped columns around the element (cx in [-0.5, nx - 0.5)); a
    // window reaching half the period, or spanning more block columns than
    // a row has, is too wide for the nearest-image lists
    if (!(rxs < 0.5 * (double)p.nx - 2.0)) {
      atomicOr(flags, FLAG_WIDE);
      return B;
    }
    ilo = (int)ceil(cx - rxs);
    ihi = (int)floor(cx + rxs);
    if (ihi - ilo > p.nx - 24) {
      atomicOr(flags, FLAG_WIDE);
      return B;
    }
  } else {
    const double xlo = fmax(cx - rxs, -1.0), xhi = fmin(cx + rxs, (double)p.nx);
    ilo = max(0, (int)ceil(xlo));
    ihi = min(p.nx - 1, (int)floor(xhi));
  }
  if (ilo > ihi || jlo > jhi) return B;
  const int b0v = blk(jlo, p.ov, p.obv), b1v = blk(jhi, p.ov, p.obv);
  // blocks per row of the window's box, whatever the row group's x offset
  const int wxm = ((ihi - ilo) >> 3) + 2, wv = b1v - b0v + 1;
  if ((long long)wxm * (long long)wv > SPAN_LIMIT) {
    atomicOr(flags, FLAG_WIDE);
    return B;
  }
  const double hx = 3.5 * p.dx, hv = 3.5 * p.dv;
  const double mxm = (rxs + 8.0) * p.dx, mvm = (rvs + 8.0) * p.dv;
  B.limx =
      p.dxm + 0x1p-36 * (fabs(axx) * (mxm + 1.0) + fabs(axv) * (mvm + 1.0) +
                         p.dxm) + (fabs(axx) * hx + fabs(axv) * hv);
  B.limv =
      p.dvm + 0x1p-36 * (fabs(avx) * (mxm + 1.0) + fabs(avv) * (mvm + 1.0) +
                         p.dvm) + (fabs(avx) * hx + fabs(avv) * hv);
  B.ga = group_of_brow(p, b0v);
  B.opack = group_ox(p, B.ga) | (group_ox(p, B.ga + 1) << 3) |
            (group_ox(p, B.ga + 2) << 6);
  B.n = wxm * wv;
  B.wxm = wxm;
  B.b0v = b0v;
  B.ilo = ilo;
  B.ihi = ihi;
  B.x = s.x;
  B.v = s.v;
  B.axx = axx;
  B.axv = axv;
  B.avx = avx;
  B.avv = avv;
  return B;
}

// Block (row qr, column qc) of a registration box: its list index, or -1
// when the element's validity window cannot reach it; bvq and bxq receive
// its block row and (unwrapped) block column.
template <bool TALL>
__device__ __forceinline__ int reg_block(const KP &p, const RegBox &B, int qr,
                                         int qc, int &bvq, int &bxq) {
  bvq = B.b0v + qr;
  const int gy = group_of_brow(p, bvq);
  const int o = TALL ? group_ox(p, gy) : (B.opack >> (3 * (gy - B.ga))) & 7;
  bxq = blk(B.ilo, o, 1) + qc;
  const int i0 = o + 8 * (bxq - 1), j0 = p.ov + 8 * (bvq - p.obv);
  const double cx = (p.x_min + (double)(i0 + 4) * p.dx) - B.x;
  const double cv = (p.v_min + (double)(j0 + 4) * p.dv) - B.v;
  const double lxc = B.axx * cx + B.axv * cv, lvc = B.avx * cx + B.avv * cv;
  if (bxq <= blk(B.ihi, o, 1) && fabs(lxc) < B.limx && fabs(lvc) < B.limv)
    return bvq * p.nbx + (p.per ? ((bxq % p.nbl) + p.nbl) % p.nbl : bxq);
  return -1;
}

// Register blocks q0 .. nblk - 1 of a box with one global slot claim each:
// the claims are independent, so they are issued sixteen at a time and
// only then are the ids written (one atomic round trip per sixteen blocks).
template <bool TALL>
__device__ __forceinline__ void reg_claims(const KP &p, const RegBox &B,
                                           int q0, int e, int *__restrict__ cnt,
                                           int *__restrict__ lst) {
  constexpr int RB = 16;
  int qr = q0 / B.wxm, qc = q0 % B.wxm;
  for (int qb = q0; qb < B.n; qb += RB) {
    int bb[RB], slot[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      bb[k] = -1;
      if (qb + k < B.n) {
        int bvq, bxq;
        bb[k] = reg_block<TALL>(p, B, qr, qc, bvq, bxq);
        if (++qc == B.wxm) {
          qc = 0;
          ++qr;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < RB; ++k)
      slot[k] = (bb[k] >= 0) ? atomicAdd(&cnt[bb[k]], 1) : p.cap;
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (slot[k] < p.cap) lst[(size_t)bb[k] * p.cap + slot[k]] = e;
  }
}

__device__ __forceinline__ void reg_direct(const KP &p, const RegBox &B,
                                           int q0, int e, int *__restrict__ cnt,
                                           int *__restrict__ lst) {
  if (B.n / B.wxm > REG_NEAR_ROWS)
    reg_claims<true>(p, B, q0, e, cnt, lst);
  else
    reg_claims<false>(p, B, q0, e, cnt, lst);
}

// The element passes take elements in PATCH x PATCH lattice patches, one per
// 256-thread workgroup: the block lists an element registers into are mostly
// those of its neighbours in the same workgroup.
constexpr int PATCH = 16;

// Number of element patches of a run.
__host__ __device__ __forceinline__ int elem_patches(int mx, int mv) {
  return ((mx + PATCH - 1) / PATCH) * ((mv + PATCH - 1) / PATCH);
}

// Registration of a workgroup's elements through a table of block counters
// in LDS (RT block rows by RT block columns around the workgroup's element
// patch, rows from tr0 and columns from tc0).  Every claim of a block inside
// the table takes a rank among the workgroup's claims on it (LDS atomic);
// the first claimer of each block then takes the workgroup's slots of it
// with one device atomic (the base), and each claim writes its id at
// base + rank.  A claim outside the table, and the blocks of a box past the
// RB-th, take their slots one by one as in reg_claims.  The counts, and
// with them the readers' overflow test, are those of one atomic per claim;
// only the order of the ids within a list changes, which the query does not
// depend on (it ranks by distance, then id).  Every thread of the workgroup
// must call it: it holds two workgroup barriers.
constexpr int RT = 64;
// Element passes with fewer patches than this register directly: with a
// workgroup or so per CU the claims wait on the atomics' latency, which the
// table's barriers lengthen (measured: 256 patches slower with the table,
// 1024 and 4096 faster).
constexpr int ELEM_TABLE_MIN_PATCHES = 1024;

template <int RB, bool TALL>
__device__ __forceinline__ void reg_table_rank(const KP &p, const RegBox &B,
                                               int tr0, int tc0,
                                               int *__restrict__ rtab,
                                               int (&bb)[RB], int (&key)[RB],
                                               int (&loc)[RB]) {
  int qr = 0, qc = 0;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    bb[k] = -1;
    key[k] = -1;
    loc[k] = 0;
    if (k < B.n) {
      int bvq, bxq;
      bb[k] = reg_block<TALL>(p, B, qr, qc, bvq, bxq);
      if (++qc == B.wxm) {
        qc = 0;
        ++qr;
      }
      const unsigned r = (unsigned)(bvq - tr0), c = (unsigned)(bxq - tc0);
      if (bb[k] >= 0 && r < (unsigned)RT && c < (unsigned)RT) {
        key[k] = (int)(r * RT + c);
        loc[k] = atomicAdd(&rtab[key[k]], 1);
      }
    }
  }
}

template <int RB>
__device__ __forceinline__ void reg_table(const KP &p, const RegBox &B,
                                          int e, int tr0, int tc0,
                                          int *__restrict__ rtab,
                                          int *__restrict__ cnt,
                                          int *__restrict__ lst) {
  int bb[RB], key[RB], loc[RB], slot[RB];
  if (B.n > 0 && B.n / B.wxm > REG_NEAR_ROWS)
    reg_table_rank<RB, true>(p, B, tr0, tc0, rtab, bb, key, loc);
  else
    reg_table_rank<RB, false>(p, B, tr0, tc0, rtab, bb, key, loc);
  __syncthreads();
  // device atomics: one per block of the table (its first claimer), one
  // per claim outside it, all issued before any result is used
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    slot[k] = p.cap;
    if (bb[k] >= 0 && key[k] < 0)
      slot[k] = atomicAdd(&cnt[bb[k]], 1);
    else if (key[k] >= 0 && loc[k] == 0)
      slot[k] = atomicAdd(&cnt[bb[k]], rtab[key[k]]);
  }
#pragma unroll
  for (int k = 0; k < RB; ++k)
    if (key[k] >= 0 && loc[k] == 0) rtab[key[k]] = slot[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    if (bb[k] < 0) continue;
    const int sl = key[k] >= 0 ? rtab[key[k]] + loc[k] : slot[k];
    if (sl < p.cap) lst[(size_t)bb[k] * p.cap + sl] = e;
  }
  if (B.n > RB) reg_direct(p, B, RB, e, cnt, lst);
}

__device__ __forceinline__ void elem_record(
    const KP &p, const ElemState &s, int e, double *__restrict__ rec,
    double *__restrict__ qm, int *__restrict__ cnt, int *__restrict__ lst,
    int *__restrict__ flags, int reg) {
  const RegBox B = elem_record_box(p, s, e, rec, qm, flags, reg);
  if (B.n > 0) reg_direct(p, B, 0, e, cnt, lst);
}

// TAB false: thread gid takes element gid and registers every claim with
// its own device atomic (reg_direct).  TAB true: workgroup w takes lattice
// patch w and registers the first TABLE_RB blocks of each box through the
// workgroup's table (reg_table); the grid then covers every patch.
constexpr int TABLE_RB = 16;
template <bool TAB>
__global__ __launch_bounds__(256) void k_elem(
    KP p, double *__restrict__ st, const double *__restrict__ acc,
    double *__restrict__ rec, double *__restrict__ qm,
    int *__restrict__ cnt_zero, long long nb_zero,
    int *__restrict__ cnt_reg, int *__restrict__ lst, int *__restrict__ flags,
    int kick, int drift, int predict, int reg) {
  __shared__ int rtab[TAB ? RT * RT : 1];
  const int tid = threadIdx.x;
  const long long gid = (long long)blockIdx.x * blockDim.x + tid;
  const long long gsz = (long long)gridDim.x * blockDim.x;
  if (TAB && predict)
    for (int i = tid; i < RT * RT; i += 256) rtab[i] = 0;
  for (long long b = gid; b < nb_zero; b += gsz) cnt_zero[b] = 0;
  // this thread's element: gid, or (k, l) in lattice patch blockIdx.x
  const int npx = (p.mx + PATCH - 1) / PATCH;
  const int pat = blockIdx.x;
  const int ek = (pat % npx) * PATCH + tid % PATCH;
  const int el = (pat / npx) * PATCH + tid / PATCH;
  const bool has =
      TAB ? pat < elem_patches(p.mx, p.mv) && ek < p.mx && el < p.mv
          : gid < p.E;
  const int e = !has ? 0 : TAB ? el * p.mx + ek : (int)gid;
  // variable step: this step's dt from the clock; after a kick, the next
  // step's from the density the field kernel saw
  double t1 = 0.0, tr = 0.0, dtn = p.dt;
  if (p.clk) {
    const double *ck = p.clk + CK_SLOT * p.par;
    if (kick) dtn = next_dt(p, p.clk[CK_RHO]);  // p.dt is still the cap
    p.dt = ck[CK_DT];
    p.h = 0.5 * p.dt;
    t1 = ck[CK_T];
    tr = ck[CK_TR];
    if (kick) t1 = t1 + p.dt;
    const double hp = (predict && drift) ? 0.5 * (kick ? dtn : p.dt) : 0.0;
    p.tau = (t1 + hp) - tr;
    gox_set(p);
    if (gid == 0) {
      double *cw = p.clk + CK_SLOT * (kick ? p.par ^ 1 : p.par);
      if (kick) {
        cw[CK_DT] = dtn;
        cw[CK_T] = t1;
        cw[CK_TR] = tr;
      }
      cw[CK_TAU] = p.tau;
    }
  }
  const size_t E = (size_t)p.E;
  ElemState s;
  RegBox B;
  B.n = 0;
  if (has) {
    elem_load(st, E, e, s);
    if (kick) elem_kick(p, AccTable{acc, p.nx + 8}, s);
    if (p.clk && kick) p.h = 0.5 * dtn;
    if (predict && drift) elem_drift(p, s);
    if (kick || (predict && drift)) elem_store(st, E, e, s);
    if (predict) B = elem_record_box(p, s, e, rec, qm, flags, reg);
  }
  if (!predict) return;
  if (TAB) {
    // the registration table is centred on the patch's lattice sites
    const int tr0 =
        blk(p.sv * ((pat / npx) * PATCH + PATCH / 2), p.ov, p.obv) - RT / 2;
    const int tc0 =
        blk(p.sx * ((pat % npx) * PATCH + PATCH / 2), 0, 1) - RT / 2;
    reg_table<TABLE_RB>(p, B, e, tr0, tc0, rtab, cnt_reg, lst);
  } else if (B.n > 0) {
    reg_direct(p, B, 0, e, cnt_reg, lst);
  }
}

// New isotropic elements (P = Q_m, T = I, H = 0) and cleared block counts.
__global__ __launch_bounds__(256) void k_elem_reset(KP p,
                                                    double *__restrict__ st,
                                                    int *__restrict__ cnt,
                                                    long long nb) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long gsz = (long long)gridDim.x * blockDim.x;
  for (long long b = gid; b < nb; b += gsz) cnt[b] = 0;
  const int e = (int)gid;
  if (p.clk && gid == 0) {
    double *ck = p.clk + CK_SLOT * p.par;
    ck[CK_TR] = ck[CK_T];
  }
  if (e >= p.E) return;
  const size_t E = (size_t)p.E;
  const int k = e % p.mx, l = e / p.mx;
  for (int s = 0; s < NSTATE; ++s) st[s * E + e] = 0.0;
  st[S_X * E + e] = site_x(p, p.sx * k + p.sx / 2);
  st[S_V * E + e] = site_v(p, p.sv * l + p.sv / 2);
  st[S_TXX * E + e] = 1.0;
  st[S_TVV * E + e] = 1.0;
}

__global__ __launch_bounds__(256) void k_zero_i32(int *__restrict__ a,
                                                  long long n) {
  const long long gsz = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += gsz)
    a[i] = 0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *__restrict__ a, long long n,
                                              T val) {
  const long long gsz = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += gsz)
    a[i] = val;
}

// ------------------------------------------------------------- the query

// One candidate of the nearest-element query (sections 1 and 2.3): inverse
// map of eq. (QofP) with l = A dP, validity |l| < element spacing, squared
// Lagrangian distance of eq. (distdef) in element-spacing units; the best
// is the smallest (d^2, id).  r is the candidate's record.  With -H/2 in
// the record, dQ = l + A u' with u'_c = l^T (-H_c/2) l, which equals
// l - A u / 2 bit for bit (scaling by a power of two commutes with every
// rounding step).  With R2 (rx == rv == r, a power of two) d^2 is ranked
// as |dQ|^2 = d^2 / r^2: the same scaling argument makes the two orders
// (and their ties) identical.
template <int PER, bool R2, bool BF, typename R>
__device__ __forceinline__ void query_candidate(const KP &p, const R &r, int e,
                                                double xP, double vP,
                                                double &bd, int &best,
                                                double &bdqx, double &bdqv) {
  const double dx = image_dx<PER>(p, xP - r[R_X]), dv = vP - r[R_V];
  const double lx = fma(r[R_AXX], dx, r[R_AXV] * dv);
  const double lv = fma(r[R_AVX], dx, r[R_AVV] * dv);
  const bool valid = fabs(lx) < p.dxm && fabs(lv) < p.dvm;
  // BF: evaluated on every lane (a candidate is valid on some lane of the
  // block almost always), the validity folded into the update; else the
  // quadratic part runs under the validity mask (kernels held to few
  // registers keep their live ranges short that way)
  if (!BF && !valid) return;
  const double pxx = lx * lx, pxv = lx * lv, pvv = lv * lv;
  const double ux = fma(r[R_HXXX], pxx, fma(r[R_H2XXV], pxv, r[R_HXVV] * pvv));
  const double uv = fma(r[R_HVXX], pxx, fma(r[R_H2VXV], pxv, r[R_HVVV] * pvv));
  const double dqx = fma(r[R_AXX], ux, fma(r[R_AXV], uv, lx));
  const double dqv = fma(r[R_AVX], ux, fma(r[R_AVV], uv, lv));
  double d2;
  if (R2) {
    d2 = fma(dqx, dqx, dqv * dqv);
  } else {
    const double zx = dqx * p.rx, zv = dqv * p.rv;
    d2 = fma(zx, zx, zv * zv);
  }
  // (d2, id) order; an exact tie of d2 is rare, so the id comparison is
  // made only when some lane of the wavefront has one
  bool upd = valid && d2 < bd;
  const bool tie = valid && d2 == bd;
  if (__builtin_expect(__ballot(tie) != 0ull, 0)) upd = upd || (tie && e < best);
  if (upd) {
    bd = d2;
    best = e;
    bdqx = dqx;
    bdqv = dqv;
  }
}

// Same map without the validity test (neighbour predictions at remap).
template <int PER>
__device__ __forceinline__ void element_map(const KP &p,
                                            const double *__restrict__ r,
                                            double xP, double vP, double &dqx,
                                            double &dqv) {
  const double dx = image_dx<PER>(p, xP - r[R_X]), dv = vP - r[R_V];
  const double lx = fma(r[R_AXX], dx, r[R_AXV] * dv);
  const double lv = fma(r[R_AVX], dx, r[R_AVV] * dv);
  const double pxx = lx * lx, pxv = lx * lv, pvv = lv * lv;
  const double ux = fma(r[R_HXXX], pxx, fma(r[R_H2XXV], pxv, r[R_HXVV] * pvv));
  const double uv = fma(r[R_HVXX], pxx, fma(r[R_H2VXV], pxv, r[R_HVVV] * pvv));
  dqx = fma(r[R_AXX], ux, fma(r[R_AXV], uv, lx));
  dqv = fma(r[R_AVX], ux, fma(r[R_AVV], uv, lv));
}

// The map with its validity (the neighbour predictions of E_map).
template <int PER>
__device__ __forceinline__ bool element_map_valid(const KP &p,
                                                  const double *__restrict__ r,
                                                  double xP, double vP,
                                                  double &dqx, double &dqv) {
  const double dx = image_dx<PER>(p, xP - r[R_X]), dv = vP - r[R_V];
  const double lx = fma(r[R_AXX], dx, r[R_AXV] * dv);
  const double lv = fma(r[R_AVX], dx, r[R_AVV] * dv);
  element_map<PER>(p, r, xP, vP, dqx, dqv);
  return fabs(lx) < p.dxm && fabs(lv) < p.dvm;
}

struct Rec {
  double v[RS];
  __device__ __forceinline__ double operator[](int k) const { return v[k]; }
};

__device__ __forceinline__ void load_rec(const double *__restrict__ rec,
                                         int e, Rec &r) {
  const double *q = rec + (size_t)e * RS;
#pragma unroll
  for (int k = 0; k < RS; ++k) r.v[k] = q[k];
}

// Records staged per round in a wavefront's LDS area (QSTAGE * RS doubles).
typedef __attribute__((address_space(3))) void lds_void;
constexpr int QSTAGE = 20;
constexpr int RPIECES = RS / 2;  // 16-byte pieces per record

// First QSTAGE entries of a block's list, one per lane, requested before
// the count is known (the row has cap >= 16 slots; entries beyond the count
// are stale ids and are never used).
__device__ __forceinline__ int list_head(const KP &p, const int *L) {
  const int lane = threadIdx.x & 63;
  return (lane < min(p.cap, QSTAGE)) ? L[lane] : 0;
}

// Records c0 .. c0 + m - 1 of a block list (m <= QSTAGE) into a wave's LDS
// area: pieces lane and lane + 64 (QSTAGE * RPIECES <= 128), loaded straight
// into the area (a global-to-LDS load puts lane t's 16 bytes at the area's
// start + 16 t).  Only issues the loads; stage_wait completes them.  id0
// holds the list's first entries (lane-indexed), used for c0 == 0.
__device__ __forceinline__ void stage_issue(const double *__restrict__ rec,
                                            const int *__restrict__ L, int id0,
                                            int c0, int m, double *stage) {
  static_assert(QSTAGE * RPIECES <= 128, "two pieces per lane");
  const int lane = threadIdx.x & 63;
  const int myid = (lane < m) ? (c0 == 0 ? id0 : L[c0 + lane]) : 0;
  const int np = m * RPIECES;
  const int ta = lane, tb = lane + 64;
  const int ra = ta / RPIECES, rb = tb / RPIECES;
  const int ida = __shfl(myid, ra), idb = __shfl(myid, min(rb, 63));
  if (ta < np)
    __builtin_amdgcn_global_load_lds(
        rec + (size_t)ida * RS + 2 * (ta - ra * RPIECES), (lds_void *)stage,
        16, 0, 0);
  if (tb < np)
    __builtin_amdgcn_global_load_lds(
        rec + (size_t)idb * RS + 2 * (tb - rb * RPIECES),
        (lds_void *)(stage + 128), 16, 0, 0);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Every outstanding vector memory operation of the wave (the staging loads
// among them) complete, the area readable by all lanes.
__device__ __forceinline__ void stage_wait() {
  __builtin_amdgcn_s_waitcnt(0);
  wave_sync();
}

// The candidates of one staged round, unrolled: the record offsets are
// immediate and the ids scalar loads of the (uniform) list row.
template <int PER, bool R2, bool BF>
__device__ __forceinline__ void query_round(
    const KP &p, const int *__restrict__ L, int c0, int m, const double *stage,
    double xP, double vP, double &bd, int &best, double &dqx, double &dqv) {
#pragma unroll
  for (int k = 0; k < QSTAGE; ++k) {
    if (k < m) {
      const int e = L[c0 + k];
      Rec r;
#pragma unroll
      for (int q = 0; q < RS; ++q) r.v[q] = stage[k * RS + q];
      query_candidate<PER, R2, BF>(p, r, e, xP, vP, bd, best, dqx, dqv);
    }
  }
}

// Nearest element of (xP, vP) from the wave's block list, or from all
// elements when the list overflowed or an element was too wide to list.
// The list's records are brought into the wave's LDS area together, so the
// candidates cost one memory round trip per QSTAGE records instead of one
// each; the candidate loop then reads them as uniform LDS broadcasts.
// L is the block's list row, id0 its first entries (lane-indexed, loaded by
// the caller together with the count n).  With staged0, the caller has
// already issued and waited for the first round (stage_issue, stage_wait).
template <int PER, bool R2, bool BF>
__device__ __forceinline__ int query_block_r(
    const KP &p, const double *__restrict__ rec, const int *__restrict__ L,
    int id0, int n, bool scan_all, double xP, double vP, double &dqx,
    double &dqv, double *stage, bool staged0) {
  double bd = __builtin_inf();
  int best = -1;
  dqx = 0.0;
  dqv = 0.0;
  if (!scan_all) {
    for (int c0 = 0; c0 < n; c0 += QSTAGE) {
      const int m = min(QSTAGE, n - c0);
      if (!(staged0 && c0 == 0)) {
        stage_issue(rec, L, id0, c0, m, stage);
        stage_wait();
      }
      query_round<PER, R2, BF>(p, L, c0, m, stage, xP, vP, bd, best, dqx, dqv);
      wave_sync();
    }
  } else {
    for (int e = 0; e < p.E; ++e) {
      Rec r;
      load_rec(rec, e, r);
      query_candidate<PER, R2, BF>(p, r, e, xP, vP, bd, best, dqx, dqv);
    }
  }
  return best;
}

template <int PER, bool BF = false>
__device__ __forceinline__ int query_block(
    const KP &p, const double *__restrict__ rec, const int *__restrict__ L,
    int id0, int n, bool scan_all, double xP, double vP, double &dqx,
    double &dqv, double *stage, bool staged0 = false) {
  return p.r2 ? query_block_r<PER, true, BF>(p, rec, L, id0, n, scan_all, xP,
                                              vP, dqx, dqv, stage, staged0)
              : query_block_r<PER, false, BF>(p, rec, L, id0, n, scan_all, xP,
                                               vP, dqx, dqv, stage, staged0);
}

// ------------------------------------------------------- interpolations

// Periodic x: interpolation positions are clamped to [-12, nx + 11] sites
// (16 ghost columns of periodic copies hold every stencil point; only an
// element far outside its validity could reach beyond).
__device__ __forceinline__ double clamp_periodic(const KP &p, double sx) {
  if (sx < -12.0) return -12.0;
  if (sx > (double)p.nx + 11.0) return (double)p.nx + 11.0;
  return sx;
}

// Six-point second-order interpolation (section 2.2.1, eq. int1 with the
// Lagrange signs) of F at index-space position (sx, sv).  F points at the
// grid origin of a zero-padded array.
template <typename FT, int PER>
__device__ __forceinline__ FT int1(const KP &p, const FT *__restrict__ F,
                                   double sx, double sv) {
  if (PER) sx = clamp_periodic(p, sx);
  const double fin = floor(sx + 0.5), fjn = floor(sv + 0.5);
  if (!((PER || (fin >= -1.0 && fin <= (double)p.nx)) && fjn >= -1.0 &&
        fjn <= (double)p.nv))
    return (FT)0;
  const double fic = floor(sx), fjc = floor(sv);
  const int in = (int)fin, jn = (int)fjn, ic = (int)fic, jc = (int)fjc;
  const FT dqx = (FT)(sx - fin), dqv = (FT)(sv - fjn);
  const FT one = (FT)1, half = (FT)0.5;
  const FT w0 = (one - dqx * dqx) - dqv * dqv;
  const FT hx = half * dqx, hv = half * dqv;
  const FT wxp = hx * (one + dqx), wxm = hx * (one - dqx);
  const FT wvp = hv * (one + dqv), wvm = hv * (one - dqv);
  const FT wc = dqx * dqv;
  const long pt = p.pitch;
  const FT *n0 = F + (long)jn * pt + in;
  const FT *c0 = F + (long)jc * pt + ic;
  const FT cross = ((c0[pt + 1] + c0[0]) - c0[1]) - c0[pt];
  FT f = n0[0] * w0;
  f = fma(n0[1], wxp, f);
  f = fma(-n0[-1], wxm, f);
  f = fma(n0[pt], wvp, f);
  f = fma(-n0[-pt], wvm, f);
  f = fma(cross, wc, f);
  return f;
}

// Cubic B-spline weights at offset u in [0, 1].  In double precision the
// four weights, each times the rounded 1/6.  In single precision six times
// the weights: float(1/6) exceeds 1/6 by 3e-8, and that one rounding,
// shared by every weight of every site, would scale every resampled value
// (and the mass) by 1 + 6e-8 at each resampling; spline_eval applies the
// 1/36 of the two axes once instead, split into two floats so that the
// product rounds as the exact quotient would.
template <typename FT>
__device__ __forceinline__ void bspline_w(double ud, FT b[4]) {
  const FT u = (FT)ud;
  const FT t = (FT)1 - u;
  const FT u2 = u * u, u3 = u2 * u;
  if constexpr (sizeof(FT) == 8) {
    const FT sixth = (FT)(1.0 / 6.0);
    b[0] = ((t * t) * t) * sixth;
    b[1] = (((FT)3 * u3 - (FT)6 * u2) + (FT)4) * sixth;
    b[2] = ((((FT)-3 * u3 + (FT)3 * u2) + (FT)3 * u) + (FT)1) * sixth;
    b[3] = u3 * sixth;
  } else {
    b[0] = (t * t) * t;
    b[1] = ((FT)3 * u3 - (FT)6 * u2) + (FT)4;
    b[2] = (((FT)-3 * u3 + (FT)3 * u2) + (FT)3 * u) + (FT)1;
    b[3] = u3;
  }
}

// 1/36 as the sum of two floats (the normalisation of single-precision
// tensor weights in two axes).
constexpr float INV36_HI = (float)(1.0 / 36.0);
constexpr float INV36_LO = (float)(1.0 / 36.0 - (double)(float)(1.0 / 36.0));

// Cubic B-spline value (section 2.2.2) from coefficients C (padded, with
// mirror ghosts one site deep) at index-space position (sx, sv).
template <typename FT, int PER>
__device__ __forceinline__ FT spline_eval(const KP &p, const FT *__restrict__ C,
                                          double sx, double sv) {
  if (PER) sx = clamp_periodic(p, sx);
  if (!((PER || (sx >= 0.0 && sx <= (double)(p.nx - 1))) && sv >= 0.0 &&
        sv <= (double)(p.nv - 1)))
    return (FT)0;
  int i = (int)floor(sx), j = (int)floor(sv);
  if (!PER && i > p.nx - 2) i = p.nx - 2;
  if (j > p.nv - 2) j = p.nv - 2;
  FT bx[4], bv[4];
  bspline_w<FT>(sx - (double)i, bx);
  bspline_w<FT>(sv - (double)j, bv);
  const long pt = p.pitch;
  const FT *c = C + (long)(j - 1) * pt + (i - 1);
  FT f = (FT)0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const FT *cr = c + b * pt;
    FT row = bx[0] * cr[0];
    row = fma(bx[1], cr[1], row);
    row = fma(bx[2], cr[2], row);
    row = fma(bx[3], cr[3], row);
    f = (b == 0) ? bv[0] * row : fma(bv[b], row, f);
  }
  if constexpr (sizeof(FT) == 4) f = fmaf(f, INV36_HI, f * INV36_LO);
  return f;
}

// Monaghan kernel W (section 2.3.2).
__device__ __forceinline__ double W_kernel(double x) {
  if (x <= 1.0) {
    const double x2 = x * x;
    return fma(0.75 * x, x2, fma(-1.5, x2, 1.0));
  }
  if (x <= 2.0) {
    const double t = 2.0 - x;
    return ((0.25 * t) * t) * t;
  }
  return 0.0;
}

// ------------------------------------------------------------- the field

// Cumulative mass and force (section 2.5, eq. acccomp; a' as a centred
// difference over 2 dx).  M_left is summed in 64-site chunks, sequentially
// inside a chunk, and the chunk carries are added sequentially.  One
// workgroup of 256 threads handles 256 columns: it forms the column values
// (sum of the row-group partials in increasing group order, or rho given
// directly), the sequential prefix and total of each of its chunks; the
// last workgroup to finish adds the carries and writes M_left and a, a',
// a'' on the indices [-4, nx + 3] (plus optional copies on [0, nx)).
template <typename MP>
__device__ __forceinline__ double Ml_at(const MP &Ml, int nx, double Mtot,
                                        int i) {
  if (i < 0) return 0.0;
  if (i >= nx) return Mtot;
  return Ml[i];
}

constexpr int MCHUNK = 64;          // cumulative-mass chunk (sites)
constexpr int FIELD_CHUNKS = 2048;  // chunks: up to 131072 columns
constexpr int FIELD_WG = 256;       // columns per workgroup of k_field

// Sequential running sum of st[0, n) in place; returns the total.  Loads
// are batched ahead of the dependency chain.
__device__ __forceinline__ double seq_prefix(double *st, int n) {
  double s = 0.0;
  const int nb = n & ~15;
  for (int q0 = 0; q0 < nb; q0 += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = st[q0 + u];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      s += v[u];
      v[u] = s;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) st[q0 + u] = v[u];
  }
  for (int q = nb; q < n; ++q) {
    s += st[q];
    st[q] = s;
  }
  return s;
}

struct FieldArgs {
  const double *in;   // row-group partials [ngy][nx] or rho [nx]
  int ngy;            // number of row groups (partials), 0 when in is rho
  int in_is_rho;
  double *Mc;         // chunk-local prefix [nx]
  double *ctot;       // chunk totals [nch]
  int *fcnt;          // finished-chunk counter (zero between launches)
  double *Ml;         // cumulative mass [nx]
  double *acc;        // a, a', a'' on [-4, nx + 3]
  double *rho_out, *a_out, *da_out, *d2a_out;  // optional
  double *rmx;        // per-workgroup largest rho [nwg] (variable step)
  int tail;           // k_field publishes only; k_field_tail finishes
};

__device__ __forceinline__ double ld_coherent(const double *q) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<const unsigned long long *>(q), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT));
}

// Periodic x: M_right - M_left of eq. (acccomp) at site k in [0, nx)
// minus the uniform background's own, M_tot (2 k + 1) / nx.
template <typename MP>
__device__ __forceinline__ double periodic_B(const KP &p, const MP &M,
                                             double Mtot, int k) {
  const double bg = Mtot * ((double)(2 * k + 1) / (double)p.nx);
  const double Lm = (k >= 1) ? M[k - 1] : 0.0;
  return (bg - M[k]) - Lm;
}

// Mean of B over the ring, summed in the 64-site chunks of M_left (NT
// threads, the whole workgroup; sc holds nch + 1 LDS doubles, free again
// on return).
template <int NT>
__device__ __forceinline__ double periodic_mean(const KP &p, const double *M,
                                                double Mtot, double *sc) {
  const int nx = p.nx, tid = threadIdx.x;
  const int nch = (nx + MCHUNK - 1) / MCHUNK;
  for (int c = tid; c < nch; c += NT) {
    const int i1 = min(c * MCHUNK + MCHUNK, nx);
    double t = 0.0;
    for (int i = c * MCHUNK; i < i1; ++i) t += periodic_B(p, M, Mtot, i);
    sc[c] = t;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int c = 0; c < nch; ++c) t = t + sc[c];
    sc[nch] = t / (double)nx;
  }
  __syncthreads();
  const double r = sc[nch];
  __syncthreads();
  return r;
}

// a at any integer site i from M_left: eq. (acccomp) (constant beyond the
// grid), or with periodic x the force against the background, G (B - mean
// B) at i mod nx.
template <typename MP>
__device__ __forceinline__ double acc_site(const KP &p, const MP &M,
                                           double Mtot, double Bbar, int i) {
  if (p.per) {
    const int k = ((i % p.nx) + p.nx) % p.nx;
    return p.G * (periodic_B(p, M, Mtot, k) - Bbar);
  }
  return p.G * ((Mtot - Ml_at(M, p.nx, Mtot, i)) - Ml_at(M, p.nx, Mtot, i - 1));
}

// a, a', a'' at table index q (site i = q - 4) from M_left: a' as a centred
// difference over 2 dx, a'' the three-point second difference.
template <typename MP>
__device__ __forceinline__ void acc_from_mass(const KP &p, const MP &M,
                                              double Mtot, double Bbar, int q,
                                              double &a0, double &da,
                                              double &d2a) {
  const int i = q - 4;
  const double two_dx = 2.0 * p.dx, dx2 = p.dx * p.dx;
  const double am = acc_site(p, M, Mtot, Bbar, i - 1);
  a0 = acc_site(p, M, Mtot, Bbar, i);
  const double ap = acc_site(p, M, Mtot, Bbar, i + 1);
  da = (ap - am) / two_dx;
  d2a = ((ap + am) - 2.0 * a0) / dx2;
}

struct AccFromMass {
  const KP &p;
  const double *M;
  double Mtot, Bbar;
  __device__ __forceinline__ void at(int q, double &a, double &da,
                                     double &d2a) const {
    acc_from_mass(p, M, Mtot, Bbar, q, a, da, d2a);
  }
};

// The same force for one element without the whole M_left table (isolated
// x): the six cumulative masses M_left(i0 - 3 .. i0 + 2) that the dual TSC
// around site i0 needs, each the carry of its 64-site chunk plus the
// chunk's own prefix (mw, read beforehand), give a at i0 - 2 .. i0 + 2 and
// then a, a', a'' at i0 - 1 .. i0 + 1 with the operations of acc_site and
// acc_from_mass (the same values bit for bit).
struct AccWindow {
  const KP &p;
  double a[5];  // a at sites i0 - 2 .. i0 + 2
  int q0;       // table index i0 + 4 of site i0
  __device__ __forceinline__ AccWindow(const KP &p_, int i0,
                                       const double *car, const double *mw,
                                       double Mtot)
      : p(p_), q0(i0 + 4) {
    double m[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int j = i0 - 3 + d;
      m[d] = (j < 0) ? 0.0 : (j >= p.nx) ? Mtot : car[j / MCHUNK] + mw[d];
    }
#pragma unroll
    for (int d = 0; d < 5; ++d) a[d] = p.G * ((Mtot - m[d + 1]) - m[d]);
  }
  __device__ __forceinline__ void at(int q, double &a0, double &da,
                                     double &d2a) const {
    const int k = q - q0;  // -1, 0 or 1
    const double am = (k < 0) ? a[0] : (k == 0) ? a[1] : a[2];
    a0 = (k < 0) ? a[1] : (k == 0) ? a[2] : a[3];
    const double ap = (k < 0) ? a[2] : (k == 0) ? a[3] : a[4];
    const double two_dx = 2.0 * p.dx, dx2 = p.dx * p.dx;
    da = (ap - am) / two_dx;
    d2a = ((ap + am) - 2.0 * a0) / dx2;
  }
};

// Largest value over the 64 lanes of a wavefront (order-free: max is exact).
__device__ __forceinline__ double wave_max(double m) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  return m;
}

// LDS of one field workgroup
struct FieldLds {
  double stage[FIELD_WG];
  double car[FIELD_CHUNKS + 1];
  double red[FIELD_WG / 64];
  int last;
};

__device__ __forceinline__ void field_chunk(const KP &p, const FieldArgs &A,
                                            int c, FieldLds &L) {
  const int nx = p.nx, tid = threadIdx.x;
  const int nwg = (nx + FIELD_WG - 1) / FIELD_WG;
  const int nch = (nx + MCHUNK - 1) / MCHUNK;
  const int i0 = c * FIELD_WG, n = min(FIELD_WG, nx - i0);
  double m = 0.0;
  if (tid < n) {
    const int i = i0 + tid;
    double x;
    if (A.ngy > 0) {
      // increasing group order; loads issued 16 ahead of the additions
      x = 0.0;
      const double *col = A.in + i;
      int g = 0;
      for (; g + 16 <= A.ngy; g += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = col[(size_t)(g + u) * nx];
#pragma unroll
        for (int u = 0; u < 16; ++u) x += v[u];
      }
      for (; g < A.ngy; ++g) x += col[(size_t)g * nx];
    } else {
      x = A.in[i];
    }
    const double rho = A.in_is_rho ? x : p.dv * x;
    if (A.rho_out) A.rho_out[i] = rho;
    L.stage[tid] = p.dx * rho;
    m = fmax(m, rho);
  }
  if (p.clk) {
    m = wave_max(m);
    if ((tid & 63) == 0) L.red[tid >> 6] = m;
  }
  __syncthreads();
  if (tid * MCHUNK < n) {
    // this workgroup's chunk tid: sequential prefix and total
    const int q0 = tid * MCHUNK;
    A.ctot[i0 / MCHUNK + tid] = seq_prefix(L.stage + q0, min(MCHUNK, n - q0));
  }
  __syncthreads();
  // one wavefront publishes the chunk and takes the release/acquire count
  if (tid < 64) {
    for (int q = tid; q < n; q += 64) A.Mc[i0 + q] = L.stage[q];
    if (tid == 0) {
      if (p.clk) {
        double w = 0.0;
        for (int k = 0; k < FIELD_WG / 64; ++k) w = fmax(w, L.red[k]);
        A.rmx[c] = w;
      }
      const int old = __hip_atomic_fetch_add(A.fcnt, 1, __ATOMIC_ACQ_REL,
                                             __HIP_MEMORY_SCOPE_AGENT);
      L.last = (old == nwg - 1);
    }
  }
  __syncthreads();
  if (!L.last) return;
  if (A.tail) {
    // k_field_tail adds the carries and writes M_left and the force
    if (tid == 0)
      __hip_atomic_store(A.fcnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  // the last chunk: carries, M_left, force
  for (int k = tid; k < nch; k += FIELD_WG) L.car[k] = ld_coherent(A.ctot + k);
  if (p.clk && tid == 0) {
    double w = 0.0;
    for (int k = 0; k < nwg; ++k) w = fmax(w, ld_coherent(A.rmx + k));
    p.clk[CK_RHO] = w;
  }
  __syncthreads();
  if (tid == 0) {
    double carry = 0.0;
    for (int k = 0; k < nch; ++k) {
      const double t = L.car[k];
      L.car[k] = carry;
      carry = carry + t;
    }
  }
  __syncthreads();
  for (int i = tid; i < nx; i += FIELD_WG)
    A.Ml[i] = L.car[i / MCHUNK] + ld_coherent(A.Mc + i);
  __syncthreads();
  const double *Ml = A.Ml;
  const double Mtot = Ml[nx - 1];
  const double Bbar =
      p.per ? periodic_mean<FIELD_WG>(p, Ml, Mtot, L.car) : 0.0;
  const int n8 = nx + 8;
  for (int q = tid; q < n8; q += FIELD_WG) {
    const int i = q - 4;
    double a0, da, d2a;
    acc_from_mass(p, Ml, Mtot, Bbar, q, a0, da, d2a);
    A.acc[q] = a0;
    A.acc[n8 + q] = da;
    A.acc[2 * n8 + q] = d2a;
    if (A.a_out && i >= 0 && i < nx) {
      A.a_out[i] = a0;
      A.da_out[i] = da;
      A.d2a_out[i] = d2a;
    }
  }
  if (tid == 0)
    __hip_atomic_store(A.fcnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(FIELD_WG) void k_field(KP p, FieldArgs A) {
  __shared__ FieldLds L;
  field_chunk(p, A, blockIdx.x, L);
}

// M_left values of a window of columns held in LDS, indexed by column.
struct WinM {
  const double *w;
  int base;
  __device__ __forceinline__ double operator[](int i) const {
    return w[i - base];
  }
};

// Second launch of the field for grids without periodic x (after k_field
// with tail set): workgroup b adds the chunk carries (one sequential chain,
// the order of the single-workgroup form), writes M_left of its 256 columns
// and a, a', a'' at the table indices [256 b, 256 b + 256) (the last
// workgroup also the remaining indices up to nx + 8).  The M_left values
// its indices read, columns [256 b - 8, 256 b + 272), are formed in LDS from
// the published chunk prefixes with the same single addition, so no
// workgroup reads another's output.
constexpr int TAIL_HALO = 8;
__global__ __launch_bounds__(FIELD_WG) void k_field_tail(KP p, FieldArgs A) {
  __shared__ double car[FIELD_CHUNKS + 1];
  __shared__ double win[FIELD_WG + 3 * TAIL_HALO];
  const int nx = p.nx, tid = threadIdx.x, b = blockIdx.x;
  const int nch = (nx + MCHUNK - 1) / MCHUNK;
  const int n8 = nx + 8;
  const int q0 = b * FIELD_WG;
  const int q1 = (b == (int)gridDim.x - 1) ? n8 : min(n8, q0 + FIELD_WG);
  const int base = q0 - TAIL_HALO;
  const int nwin = (q1 - q0) + 2 * TAIL_HALO;
  for (int k = tid; k < nch; k += FIELD_WG) car[k] = A.ctot[k];
  if (p.clk && b == 0 && tid == 0) {
    double w = 0.0;
    const int nwg = (nx + FIELD_WG - 1) / FIELD_WG;
    for (int k = 0; k < nwg; ++k) w = fmax(w, A.rmx[k]);
    p.clk[CK_RHO] = w;
  }
  __syncthreads();
  if (tid == 0) {
    double carry = 0.0;
    for (int k = 0; k < nch; ++k) {
      const double t = car[k];
      car[k] = carry;
      carry = carry + t;
    }
  }
  __syncthreads();
  for (int u = tid; u < nwin; u += FIELD_WG) {
    const int i = base + u;
    if (i >= 0 && i < nx) win[u] = car[i / MCHUNK] + A.Mc[i];
  }
  const double Mtot = car[(nx - 1) / MCHUNK] + A.Mc[nx - 1];
  __syncthreads();
  const WinM M{win, base};
  for (int i = q0 + tid; i < min(q0 + FIELD_WG, nx); i += FIELD_WG)
    A.Ml[i] = M[i];
  for (int q = q0 + tid; q < q1; q += FIELD_WG) {
    const int i = q - 4;
    double a0, da, d2a;
    acc_from_mass(p, M, Mtot, 0.0, q, a0, da, d2a);
    A.acc[q] = a0;
    A.acc[n8 + q] = da;
    A.acc[2 * n8 + q] = d2a;
    if (A.a_out && i >= 0 && i < nx) {
      A.a_out[i] = a0;
      A.da_out[i] = da;
      A.d2a_out[i] = d2a;
    }
  }
}

// The same field in one workgroup for grids of at most FIELD1_MAX columns:
// no cross-workgroup hand-off, M_left stays in LDS.  Identical operations
// in identical order (column sums in increasing group order, 64-site chunk
// prefixes, sequential carries).
constexpr int FIELD1_MAX = 2048;

// M_left of every column into LDS M[0, nx) (NT threads, the whole
// workgroup); returns M_tot.  With a variable step (p.clk), also the
// largest rho (from 0) into rmax, red[] holding NT/64 LDS doubles.  `in` holds the row-group partials (ngy > 0)
// or rho (ngy == 0).
template <int NT>
__device__ __forceinline__ double mass_to_lds(const KP &p, const double *in,
                                              int ngy, int in_is_rho,
                                              double *rho_out, double *M,
                                              double *car, double *red,
                                              double &rmax) {
  constexpr int CPT = FIELD1_MAX / NT;  // columns per thread
  const int nx = p.nx, tid = threadIdx.x;
  const int nch = (nx + MCHUNK - 1) / MCHUNK;
  {
    double xs[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) xs[c] = 0.0;
    if (ngy > 0) {
      // increasing group order; loads 16 groups ahead of the additions
      for (int g0 = 0; g0 < ngy; g0 += 16) {
        double v[CPT][16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
#pragma unroll
          for (int c = 0; c < CPT; ++c) {
            const int i = tid + c * NT;
            v[c][u] = (g0 + u < ngy && i < nx)
                          ? in[(size_t)(g0 + u) * nx + i] : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          if (g0 + u < ngy) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) xs[c] += v[c][u];
          }
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int i = tid + c * NT;
        if (i < nx) xs[c] = in[i];
      }
    }
    double m = 0.0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int i = tid + c * NT;
      if (i < nx) {
        const double rho = in_is_rho ? xs[c] : p.dv * xs[c];
        if (rho_out) rho_out[i] = rho;
        M[i] = p.dx * rho;
        m = fmax(m, rho);
      }
    }
    if (p.clk) {
      m = wave_max(m);
      if ((tid & 63) == 0) red[tid >> 6] = m;
    }
  }
  __syncthreads();
  if (p.clk) {
    double m = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) m = fmax(m, red[w]);
    rmax = m;
  }
  if (tid < nch) {
    // sequential prefix of chunk tid
    const int q0 = tid * MCHUNK;
    car[tid] = seq_prefix(M + q0, min(MCHUNK, nx - q0));
  }
  __syncthreads();
  if (tid == 0) {
    double carry = 0.0;
    for (int k = 0; k < nch; ++k) {
      const double t = car[k];
      car[k] = carry;
      carry = carry + t;
    }
  }
  __syncthreads();
  for (int i = tid; i < nx; i += NT) M[i] = car[i / MCHUNK] + M[i];
  __syncthreads();
  return M[nx - 1];
}

__global__ __launch_bounds__(1024) void k_field1(KP p, FieldArgs A) {
  __shared__ double M[FIELD1_MAX];
  __shared__ double car[FIELD1_MAX / MCHUNK + 1];
  __shared__ double red[1024 / 64];
  const int nx = p.nx, tid = threadIdx.x;
  double rmax = 0.0;
  const double Mtot = mass_to_lds<1024>(p, A.in, A.ngy, A.in_is_rho,
                                        A.rho_out, M, car, red, rmax);
  const double Bbar = p.per ? periodic_mean<1024>(p, M, Mtot, car) : 0.0;
  if (p.clk && tid == 0) p.clk[CK_RHO] = rmax;
  for (int i = tid; i < nx; i += 1024) A.Ml[i] = M[i];
  const int n8 = nx + 8;
  for (int q = tid; q < n8; q += 1024) {
    double a0, da, d2a;
    acc_from_mass(p, M, Mtot, Bbar, q, a0, da, d2a);
    A.acc[q] = a0;
    A.acc[n8 + q] = da;
    A.acc[2 * n8 + q] = d2a;
    const int i = q - 4;
    if (A.a_out && i >= 0 && i < nx) {
      A.a_out[i] = a0;
      A.da_out[i] = da;
      A.d2a_out[i] = d2a;
    }
  }
}

// Clock of the element pass that completes a step (kick + corrector,
// optionally the next predictor).  Fixed step: returns dt and leaves p.
// Variable step: p.dt and p.h become this step's, p.tau the list time of
// the next predictor; returns the next step's dt (from rmax, the density's
// maximum); `writer` stores the next slot.
__device__ __forceinline__ double elem_clock(KP &p, double rmax, int predict,
                                             bool writer) {
  if (!p.clk) return p.dt;
  const double *ck = p.clk + CK_SLOT * p.par;
  const double dtn = next_dt(p, rmax);  // p.dt is still the cap
  p.dt = ck[CK_DT];
  p.h = 0.5 * p.dt;
  const double t1 = ck[CK_T] + p.dt, tr = ck[CK_TR];
  p.tau = (t1 + (predict ? 0.5 * dtn : 0.0)) - tr;
  gox_set(p);
  if (writer) {
    double *cw = p.clk + CK_SLOT * (p.par ^ 1);
    cw[CK_DT] = dtn;
    cw[CK_T] = t1;
    cw[CK_TR] = tr;
    cw[CK_TAU] = p.tau;
  }
  return dtn;
}

// Chunk c of the cumulative mass (one wavefront, one lane per column): the
// column sums of the reconstruction's row-group partials in increasing group
// order, rho, the chunk's sequential running sum of dx rho (Mc, the chunk's
// own prefix), its total (ctot) and, with the variable step, its largest
// density (cmax).  M holds MCHUNK doubles of LDS.
__device__ __forceinline__ void field_chunk_publish(
    const KP &p, const double *__restrict__ part, double *__restrict__ Mc,
    double *__restrict__ ctot, double *__restrict__ cmax, int c, double *M) {
  const int tid = threadIdx.x & 63, nx = p.nx;
  const int i0 = c * MCHUNK, n = min(MCHUNK, nx - i0);
  double m = 0.0;
  if (tid < n) {
    const int i = i0 + tid;
    double x = 0.0;
    // every row group's partial requested at once (one memory round trip
    // for grids up to 40 groups), then added in increasing group order
    for (int g0 = 0; g0 < p.ngy; g0 += 40) {
      double v[40];
#pragma unroll
      for (int u = 0; u < 40; ++u)
        v[u] = (g0 + u < p.ngy) ? part[(size_t)(g0 + u) * nx + i] : 0.0;
#pragma unroll
      for (int u = 0; u < 40; ++u)
        if (g0 + u < p.ngy) x += v[u];
    }
    const double rho = p.dv * x;
    M[tid] = p.dx * rho;
    m = fmax(m, rho);
  }
  if (p.clk) {
    // the chunk's largest density, published with the chunk
    m = wave_max(m);
    if (tid == 0) cmax[c] = m;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (tid == 0) ctot[c] = seq_prefix(M, n);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (tid < n) Mc[i0 + tid] = M[tid];
}

// The chunks of the cumulative mass as a launch of their own (one
// wavefront per chunk), for the element pass that follows it on the stream.
__global__ __launch_bounds__(64) void k_field_chunks(
    KP p, const double *__restrict__ part, double *__restrict__ Mc,
    double *__restrict__ ctot, double *__restrict__ cmax) {
  __shared__ double M[MCHUNK];
  field_chunk_publish(p, part, Mc, ctot, cmax, blockIdx.x, M);
}

// Field and element pass of a step (grids of at most FIELD1_MAX columns,
// self-consistent force), launched after k_field_chunks on the same stream:
// every workgroup adds the chunk totals sequentially into carries and takes
// M_left from the chunks (the whole table with periodic x, else the six
// values around each element's TSC cell), then kicks, corrects, predicts
// and registers its elements.  Every load the field needs is issued in one
// round trip together with the element state.
constexpr int ELEMC_WG = 256;
static_assert(PATCH * PATCH == ELEMC_WG, "one element per thread");

__global__ __launch_bounds__(ELEMC_WG) void k_elem_window(
    KP p, const double *__restrict__ Mc, const double *__restrict__ ctot,
    const double *__restrict__ cmax, double *__restrict__ st,
    double *__restrict__ rec, double *__restrict__ qm,
    int *__restrict__ cnt_zero, long long nb_zero, int *__restrict__ cnt_reg,
    int *__restrict__ lst, int *__restrict__ flags, int predict, int reg) {
  __shared__ double M[FIELD1_MAX];
  __shared__ double car[FIELD1_MAX / MCHUNK + 1];
  __shared__ double s_rmax, s_mtot;
  const int tid = threadIdx.x, nx = p.nx;
  const int nch = (nx + MCHUNK - 1) / MCHUNK;
  const long long gid = (long long)blockIdx.x * blockDim.x + tid;
  const long long gsz = (long long)gridDim.x * blockDim.x;
  // this thread's element: (k, l) in patch blockIdx.x
  const int npx = (p.mx + PATCH - 1) / PATCH;
  const int pat = blockIdx.x;
  const int ek = (pat % npx) * PATCH + tid % PATCH;
  const int el = (pat / npx) * PATCH + tid / PATCH;
  const bool has = pat < elem_patches(p.mx, p.mv) && ek < p.mx && el < p.mv;
  const int e = has ? el * p.mx + ek : 0;
  const size_t E = (size_t)p.E;
  ElemState s;
  if (has) elem_load(st, E, e, s);
  // one lane per chunk: the totals, the last prefix and the chunk maxima
  double ct = 0.0, cm = 0.0, mlast = 0.0;
  if (tid < nch) {
    ct = ctot[tid];
    if (p.clk) cm = cmax[tid];
  }
  if (tid == 0) mlast = Mc[nx - 1];
  // isolated x: the six chunk prefixes around the element's TSC cell
  double mw[6];
  int i0 = 0;
  if (has && !p.per) {
    double w;
    i0 = (int)tsc_cell(p, s.x, w);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int j = i0 - 3 + d;
      mw[d] = (j >= 0 && j < nx) ? Mc[j] : 0.0;
    }
  }
  // periodic x: the whole table (the mean of B needs every site)
  if (p.per)
    for (int i = tid; i < nx; i += ELEMC_WG) M[i] = Mc[i];
  // the counts of the lists the reconstruction has just used, for the next
  // element pass
  for (long long b = gid; b < nb_zero; b += gsz) cnt_zero[b] = 0;
  if (tid < 64) {
    if (tid < nch) car[tid] = ct;
    if (tid == 0) s_mtot = mlast;
    if (p.clk) {
      cm = wave_max(cm);
      if (tid == 0) s_rmax = cm;
    }
  }
  __syncthreads();
  if (tid == 0) {
    // exclusive carries, sequential in chunk order
    double carry = 0.0;
    for (int k = 0; k < nch; ++k) {
      const double t = car[k];
      car[k] = carry;
      carry = carry + t;
    }
    s_mtot = car[nch - 1] + s_mtot;
  }
  __syncthreads();
  double Mtot, Bbar = 0.0;
  if (p.per) {
    for (int i = tid; i < nx; i += ELEMC_WG) M[i] = car[i / MCHUNK] + M[i];
    __syncthreads();
    Mtot = M[nx - 1];
    Bbar = periodic_mean<ELEMC_WG>(p, M, Mtot, car);
  } else {
    Mtot = s_mtot;
  }
  const double dtn = elem_clock(p, p.clk ? s_rmax : 0.0, predict, gid == 0);
  if (has) {
    if (p.per)
      elem_kick(p, AccFromMass{p, M, Mtot, Bbar}, s);
    else {
      // the cell again, from the same x (equal to i0): the kick's own
      // tsc_cell then matches it at compile time, and the window's offsets
      // stay constants
      double w;
      const int ic = (int)tsc_cell(p, s.x, w);
      elem_kick(p, AccWindow(p, ic, car, mw, Mtot), s);
    }
    if (predict) {
      p.h = 0.5 * dtn;
      elem_drift(p, s);
    }
    elem_store(st, E, e, s);
  }
  if (!predict) return;
  RegBox B;
  B.n = 0;
  if (has) B = elem_record_box(p, s, e, rec, qm, flags, reg);
  if (B.n > 0) reg_direct(p, B, 0, e, cnt_reg, lst);
}

// ------------------------------------------------------- reconstruction

// Lattice neighbour column k of an element (k may be -1 or mx): -1 when
// there is none; with periodic x the columns wrap and the wrapped
// neighbour's Lagrangian position moves by one period (shift).
__device__ __forceinline__ int lattice_col(const KP &p, int k, double &shift) {
  shift = 0.0;
  if (k >= 0 && k < p.mx) return k;
  if (!p.per) return -1;
  if (k < 0) {
    shift = -p.Lx;
    return k + p.mx;
  }
  shift = p.Lx;
  return k - p.mx;
}

// One workgroup = 8 wavefronts stacked in v; one wavefront = one 8x8-site
// query block (lane -> site: x = lane & 7, v = lane >> 3).  The workgroup
// covers 8 columns x 64 rows, the row group of the fixed column-sum order.
// In the density modes each wavefront sums its 8-row strip per column
// (sequential over the rows), and each workgroup writes the 8 column
// partials of its row group (the strips in order); the field adds the
// groups in increasing order.  No workgroup waits on another, so the
// launch needs no device-scope synchronisation.
template <typename FT, int MODE, int PER, bool BF = false>
__device__ __forceinline__ void recon_tile(
    KP p, const double *__restrict__ rec, const double *__restrict__ qm,
    const int *__restrict__ cnt,
    const int *__restrict__ lst, const int *__restrict__ flags,
    const FT *__restrict__ F, double *__restrict__ part, FT *__restrict__ fout,
    int *__restrict__ aout, double *__restrict__ dpart,
    unsigned long long *__restrict__ ovf, const int bx, const int gy) {
  __shared__ double sf[512];
  __shared__ double sk[512];
  __shared__ __attribute__((aligned(16))) double qstage[8][QSTAGE * RS];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int bv = 8 * (gy - p.obv) + p.obv + w;
  const int c0 = group_ox(p, gy) + 8 * (bx - 1);
  const int i = c0 + (lane & 7);
  const int j = p.ov + 8 * (bv - p.obv) + (lane >> 3);
  const bool blk_ok = bv >= 0 && bv < p.nbv;
  const bool live = blk_ok && i >= 0 && i < p.nx && j >= 0 && j < p.nv;
  double f = 0.0, em = 0.0;
  int best = -1;
  if (blk_ok) {
    const int b = bv * p.nbx + (PER ? list_bx(p, bx) : bx);
    const int *L = lst + (size_t)b * p.cap;
    const int id0 = list_head(p, L);
    const int n = __builtin_amdgcn_readfirstlane(cnt[b]);
    const bool scan_all = (n > p.cap) || (flags[0] & FLAG_WIDE);
    if (scan_all && lane == 0 && n > p.cap) atomicAdd(ovf, 1ull);
    const double xP = site_x(p, i), vP = site_v(p, j);
    double dqx, dqv;
    best = query_block<PER, BF>(p, rec, L, id0, n, scan_all, xP, vP, dqx,
                                dqv, qstage[w]);
    if (live && best >= 0) {
      const double Qx = qm[2 * (size_t)best] + dqx;
      const double Qv = qm[2 * (size_t)best + 1] + dqv;
      const double sx = (Qx - p.x_min) * p.inv_dx - 0.5;
      const double sv = (Qv - p.v_min) * p.inv_dv - 0.5;
      const FT *F0 = F + (long)PV * p.pitch + PX;
      const FT fv = int1<FT, PER>(p, F0, sx, sv);
      f = (double)fv;
      if (MODE == MODE_F) fout[(size_t)j * p.nx + i] = fv;
    } else if (MODE == MODE_F && live) {
      fout[(size_t)j * p.nx + i] = (FT)0;
    }
    if (MODE == MODE_ASSIGN && live) aout[(size_t)j * p.nx + i] = best;
    if ((MODE == MODE_DIAG || MODE == MODE_EMAP) && live && best >= 0) {
      // E_map at this site: distance between the nearest element's
      // prediction of Q and those of its valid lattice neighbours
      const int l0 = best / p.mx, k0 = best - l0 * p.mx;
      const double qx0 = qm[2 * (size_t)best] + dqx;
      const double qv0 = qm[2 * (size_t)best + 1] + dqv;
      const int nk[4] = {-1, 1, 0, 0}, nl[4] = {0, 0, -1, 1};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double shift;
        const int k = lattice_col(p, k0 + nk[q], shift), l = l0 + nl[q];
        if (k < 0 || l < 0 || l >= p.mv) continue;
        const size_t m = (size_t)l * p.mx + k;
        double ex, ev;
        if (!element_map_valid<PER>(p, rec + m * RS, xP, vP, ex, ev)) continue;
        const double mx = ((qm[2 * m] + shift) + ex) - qx0;
        const double mv = (qm[2 * m + 1] + ev) - qv0;
        const double zx = mx * p.rx, zv = mv * p.rv;
        em = fmax(em, sqrt(fma(zx, zx, zv * zv)));
      }
    }
  }
  if (MODE == MODE_EMAP) {
    // the workgroup's largest site value, as MODE_DIAG writes it
    __shared__ double swm[8];
    const double wm = wave_max(em);
    if (lane == 0) swm[w] = wm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = swm[0];
#pragma unroll
      for (int k = 1; k < 8; ++k) m = fmax(m, swm[k]);
      dpart[DPS * ((size_t)gy * p.nbx + bx) + DP_EMAP] = m;
    }
    return;
  }
  if (MODE != MODE_DENSITY && MODE != MODE_DIAG) return;
  if (!live) f = 0.0;
  sf[threadIdx.x] = f;
  if (MODE == MODE_DIAG) {
    const double vj = live ? site_v(p, j) : 0.0;
    sk[threadIdx.x] = vj * vj * f;
  }
  // column partial of this wavefront's 8-row strip, sequential over the rows
  __shared__ double sp[64];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (lane < 8) {
    const double *col = sf + w * 64 + lane;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 8; ++r) s += col[r * 8];
    sp[w * 8 + lane] = s;
  }
  __syncthreads();
  if (MODE == MODE_DIAG) {
    // fixed-order tree sums of v^2 f, f ln|f|, |f| and f^2, and the largest
    // E_map site value, over the workgroup
    __shared__ double se[512], sm[512], s1[512], s2[512];
    se[threadIdx.x] = (f != 0.0) ? f * log(fabs(f)) : 0.0;
    sm[threadIdx.x] = em;
    s1[threadIdx.x] = fabs(f);
    s2[threadIdx.x] = f * f;
    __syncthreads();
    for (int s = 256; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        sk[threadIdx.x] += sk[threadIdx.x + s];
        se[threadIdx.x] += se[threadIdx.x + s];
        sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        s1[threadIdx.x] += s1[threadIdx.x + s];
        s2[threadIdx.x] += s2[threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const size_t wg = (size_t)gy * p.nbx + bx;
      dpart[DPS * wg + DP_KIN] = sk[0];
      dpart[DPS * wg + DP_ENT] = se[0];
      dpart[DPS * wg + DP_EMAP] = sm[0];
      dpart[DPS * wg + DP_L1] = s1[0];
      dpart[DPS * wg + DP_L2] = s2[0];
    }
  }
  if (w == 0 && lane < 8) {
    // column partial of this row group: the eight strip partials in order
    const int ic = c0 + lane;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += sp[k * 8 + lane];
    if (ic >= 0 && ic < p.nx) part[(size_t)gy * p.nx + ic] = s;
  }
}

template <typename FT, int MODE, int PER>
__global__ __launch_bounds__(512) void k_recon(
    KP p, const double *__restrict__ rec, const double *__restrict__ qm,
    const int *__restrict__ cnt,
    const int *__restrict__ lst, const int *__restrict__ flags,
    const FT *__restrict__ F, double *__restrict__ part, FT *__restrict__ fout,
    int *__restrict__ aout, double *__restrict__ dpart,
    unsigned long long *__restrict__ ovf) {
  const int t = xcd_tile(blockIdx.x, p.nbx * p.ngy);
  int bx, gy;
  tile_split(p, t, bx, gy);
  clock_tau(p);
  // branch-free candidates (as many registers as it takes; the batched
  // kernel, held to 64, keeps the masked form)
  recon_tile<FT, MODE, PER, true>(p, rec, qm, cnt, lst, flags, F, part, fout,
                                  aout, dpart, ovf, bx, gy);
}

// Resampling value at every site (section 2.3.2): nearest element, the
// beta-restricted neighbour set (diagonals dropped when an axis needs three
// values), W(2d)-weighted blend of their predictions Q_r, cubic B-spline of
// F_ini at Q_r; the outermost ring is zero.  Writes F (padded interior)
// when TO_F == 0, else f_out.
template <typename FT, int TO_F, int PER>
__device__ __forceinline__ void remap_tile(
    KP p, const double *__restrict__ rec, const double *__restrict__ qm,
    const int *__restrict__ cnt,
    const int *__restrict__ lst, const int *__restrict__ flags,
    const FT *__restrict__ C, FT *__restrict__ Fout,
    unsigned long long *__restrict__ ovf, const int bx, const int gy) {
  __shared__ __attribute__((aligned(16))) double qstage[8][QSTAGE * RS];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int bv = 8 * (gy - p.obv) + p.obv + w;
  if (bv < 0 || bv >= p.nbv) return;
  const int i = group_ox(p, gy) + 8 * (bx - 1) + (lane & 7);
  const int j = p.ov + 8 * (bv - p.obv) + (lane >> 3);
  const bool live = i >= 0 && i < p.nx && j >= 0 && j < p.nv;
  const int b = bv * p.nbx + (PER ? list_bx(p, bx) : bx);
  const int *L = lst + (size_t)b * p.cap;
  const int id0 = list_head(p, L);
  const int n = __builtin_amdgcn_readfirstlane(cnt[b]);
  const bool scan_all = (n > p.cap) || (flags[0] & FLAG_WIDE);
  if (scan_all && lane == 0 && n > p.cap) atomicAdd(ovf, 1ull);
  const double xP = site_x(p, i), vP = site_v(p, j);
  double dqx, dqv;
  const int best = query_block<PER>(p, rec, L, id0, n, scan_all, xP, vP, dqx,
                                    dqv, qstage[w]);
  if (!live) return;
  FT val = (FT)0;
  // zero edge rows (and columns, unless x is periodic)
  const bool ring = (j == 0 || j == p.nv - 1) ||
                    (!PER && (i == 0 || i == p.nx - 1));
  if (!ring && best >= 0) {
    const int l0 = best / p.mx, k0 = best - l0 * p.mx;
    const double zx = dqx * p.rx, zv = dqv * p.rv, beta = p.beta;
    const int xlo = (zx < beta) ? -1 : 0, xhi = (zx < -beta) ? 0 : 1;
    const int vlo = (zv < beta) ? -1 : 0, vhi = (zv < -beta) ? 0 : 1;
    const bool three = (xhi - xlo == 2) || (vhi - vlo == 2);
    // The beta-set in the order of the nested loops (v offset slowest), one
    // slot per trip so that a wavefront runs at most 4 or 5 neighbour maps
    // whatever its lanes' sets: without a three-valued axis the 4 corners;
    // with one, the 5 slots (dl, dk) = (-1, 0), (0, -1), (0, 0), (0, 1),
    // (1, 0), those outside the axis ranges skipped.
    double sw = 0.0, sqx = 0.0, sqv = 0.0;
    for (int q = 0; q < 5; ++q) {
      int dk, dl;
      bool use;
      if (!three) {
        dk = xlo + (q & 1);
        dl = vlo + (q >> 1);
        use = q < 4;
      } else {
        dk = (q == 1) ? -1 : (q == 3) ? 1 : 0;
        dl = (q == 0) ? -1 : (q == 4) ? 1 : 0;
        use = dk >= xlo && dk <= xhi && dl >= vlo && dl <= vhi;
      }
      if (!use) continue;
      double shift;
      const int k = lattice_col(p, k0 + dk, shift), l = l0 + dl;
      if (k < 0 || l < 0 || l >= p.mv) continue;
      const size_t m = (size_t)(l * p.mx + k);
      double ex, ev;
      element_map<PER>(p, rec + m * RS, xP, vP, ex, ev);
      const double qx = (qm[2 * m] + shift) + ex, qv = qm[2 * m + 1] + ev;
      const double ax = ex * p.rx, av = ev * p.rv;
      const double d = sqrt(fma(ax, ax, av * av));
      const double wt = W_kernel(2.0 * d);
      sw += wt;
      sqx = fma(wt, qx, sqx);
      sqv = fma(wt, qv, sqv);
    }
    double Qx, Qv;
    if (sw > 0.0) {
      Qx = sqx / sw;
      Qv = sqv / sw;
    } else {
      Qx = qm[2 * (size_t)best] + dqx;
      Qv = qm[2 * (size_t)best + 1] + dqv;
    }
    const double sx = (Qx - p.x_min) * p.inv_dx - 0.5;
    const double sv = (Qv - p.v_min) * p.inv_dv - 0.5;
    const FT *C0 = C + (long)PV * p.pitch + PX;
    val = spline_eval<FT, PER>(p, C0, sx, sv);
  }
  if (TO_F == 0)
    Fout[(long)(j + PV) * p.pitch + (i + PX)] = val;
  else
    Fout[(size_t)j * p.nx + i] = val;
}

template <typename FT, int TO_F, int PER>
__global__ __launch_bounds__(512) void k_remap_eval(
    KP p, const double *__restrict__ rec, const double *__restrict__ qm,
    const int *__restrict__ cnt,
    const int *__restrict__ lst, const int *__restrict__ flags,
    const FT *__restrict__ C, FT *__restrict__ Fout,
    unsigned long long *__restrict__ ovf) {
  const int t = xcd_tile(blockIdx.x, p.nbx * p.ngy);
  int bx, gy;
  tile_split(p, t, bx, gy);
  clock_tau(p);
  remap_tile<FT, TO_F, PER>(p, rec, qm, cnt, lst, flags, C, Fout, ovf, bx,
                            gy);
}

// Diagnostics (section 3.2): sums of the per-workgroup partials, potential
// energy from a(i), max |det T - 1|.  out = {mass, e_kin, e_pot, entropy,
// maxdet}.
// E_map alone (the adaptive resampling check): the largest of the
// workgroups' site maxima written by the MODE_EMAP (or MODE_DIAG)
// reconstruction, into out[5] as k_diag does.
__global__ __launch_bounds__(1024) void k_emap_max(
    const double *__restrict__ dpart, long long nwg, double *__restrict__ out) {
  __shared__ double sm[1024];
  const int tid = threadIdx.x;
  double m = 0.0;
  for (long long q = tid; q < nwg; q += blockDim.x)
    m = fmax(m, dpart[DPS * q + DP_EMAP]);
  sm[tid] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s) sm[tid] = fmax(sm[tid], sm[tid + s]);
    __syncthreads();
  }
  if (tid == 0) out[5] = sm[0];
}

__global__ __launch_bounds__(1024) void k_diag(
    KP p, const double *__restrict__ dpart, long long nwg,
    const double *__restrict__ Ml, const double *__restrict__ acc,
    const double *__restrict__ st, double *__restrict__ out) {
  __shared__ double s0[1024], s1[1024], s2[1024], s3[1024], s4[1024],
      s5[1024], s6[1024];
  const int tid = threadIdx.x;
  double kin = 0.0, ent = 0.0, pot = 0.0, mdet = 0.0, emap = 0.0, l1 = 0.0,
         l2 = 0.0;
  for (long long q = tid; q < nwg; q += blockDim.x) {
    kin += dpart[DPS * q + DP_KIN];
    ent += dpart[DPS * q + DP_ENT];
    emap = fmax(emap, dpart[DPS * q + DP_EMAP]);
    l1 += dpart[DPS * q + DP_L1];
    l2 += dpart[DPS * q + DP_L2];
  }
  const double Mtot = Ml[p.nx - 1];
  const int n8 = p.nx + 8;
  if (p.force_mode == 0) {
    // periodic x: the field energy of the zero-mean force alone
    const double GM = p.per ? 0.0 : p.G * Mtot;
    for (int i = tid; i < p.nx; i += blockDim.x) {
      const double a = acc[i + 4];
      pot += a * a - GM * GM;
    }
  } else {
    for (int i = tid; i < p.nx; i += blockDim.x) {
      const double x = site_x(p, i);
      const double phi =
          -(x * (p.a0 + x * (0.5 * p.a1 + x * (p.a2 / 3.0))));
      // rho(i) dx = M(i) = Ml(i) - Ml(i-1)
      const double Mi = Ml[i] - (i > 0 ? Ml[i - 1] : 0.0);
      pot += phi * Mi;
    }
  }
  const size_t E = (size_t)p.E;
  for (int e = tid; e < p.E; e += blockDim.x) {
    const double det = st[S_TXX * E + e] * st[S_TVV * E + e] -
                       st[S_TXV * E + e] * st[S_TVX * E + e];
    mdet = fmax(mdet, fabs(det - 1.0));
  }
  (void)n8;
  s0[tid] = kin;
  s1[tid] = ent;
  s2[tid] = pot;
  s3[tid] = mdet;
  s4[tid] = emap;
  s5[tid] = l1;
  s6[tid] = l2;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s) {
      s0[tid] += s0[tid + s];
      s1[tid] += s1[tid + s];
      s2[tid] += s2[tid + s];
      s3[tid] = fmax(s3[tid], s3[tid + s]);
      s4[tid] = fmax(s4[tid], s4[tid + s]);
      s5[tid] += s5[tid + s];
      s6[tid] += s6[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double cell = p.dx * p.dv;
    out[0] = Mtot;
    out[1] = 0.5 * s0[0] * cell;
    if (p.force_mode == 0)
      out[2] = (p.G != 0.0) ? -s2[0] * p.dx / (4.0 * p.G) : 0.0;
    else
      out[2] = s2[0];
    out[3] = -s1[0] * cell;
    out[4] = s3[0];
    out[5] = s4[0];
    out[6] = s5[0] * cell;
    out[7] = sqrt(s6[0] * cell);
  }
}

// ------------------------------------------------------------- the spline

// Tridiagonal (1, 4, 1) solves with end rows (4, 2) / (2, 4) (Thomas
// elimination; the pivots cp and 1/den depend only on the position and are
// precomputed), along x for every row and then along v for every column.
// The recurrence is strictly sequential along a line, so a workgroup owns
// 64 lines: wavefront 0 runs the 64 recurrences (lane = line) out of LDS,
// while wavefronts 1-4 move tiles of 64 lines x TW positions between HBM
// and a ring of three LDS tiles with coalesced accesses (the next tile is
// loaded while the current one is solved, the previous one is written
// back).  Forward sweep, then back substitution over the tiles in reverse.
//
// Long lines are solved in segments, so that a line's recurrences run in
// parallel instead of one after another: a segment of FIT_SEG_TILES tiles
// is solved over its positions extended by one tile on each side, as the
// system truncated there (its first row without the sub-diagonal, its last
// without the super-diagonal).  The inverse of the (1, 4, 1) matrix decays
// like (2 - sqrt 3)^d = 0.268^d with the distance d from a row, so the
// truncation changes the segment's own values by 0.268^TW of the solution
// (5e-19 for the 32-position double tiles, 3e-37 for the 64-position float
// ones): the same solution to rounding.  The forward sweep keeps the
// segment's eliminated values and sums the back substitution over the last
// tile, c_b = sum_k (-1)^k (prod_{j<k} cp_{b+j}) d_{b+k}, which starts the
// back substitution of the segment at its end b.  A line of at most one
// segment is the plain Thomas elimination.
constexpr int FIT_LINES = 64;
constexpr int FIT_MOVERS = 256;                 // wavefronts 1-4
constexpr int FIT_THREADS = 64 + FIT_MOVERS;
constexpr int FIT_NB = 3;
constexpr int FIT_SEG_TILES = 8;
constexpr int FIT_TW_MAX = 64;  // tile width of the float fit

template <typename FT>
struct FitLds {
  static constexpr int TW = 256 / (int)sizeof(FT);  // positions per tile
  static constexpr int LP = FIT_LINES + 1;           // LDS pitch of a position
  static constexpr int VEC = 16 / (int)sizeof(FT);   // elements per 16-B access
  static constexpr int NV = FIT_LINES * TW / (VEC * FIT_MOVERS);  // per mover
  FT buf[FIT_NB][TW * LP];
  FT coef[FIT_NB][TW];
};
static_assert(FitLds<float>::NV * 4 * FIT_MOVERS == FIT_LINES * 64, "tile");
static_assert(FitLds<double>::NV * 2 * FIT_MOVERS == FIT_LINES * 32, "tile");
static_assert(FitLds<float>::TW == FIT_TW_MAX, "artificial pivot table");

// Segments of a line of n positions (each FIT_SEG_TILES tiles, the last
// one shorter).
template <typename FT>
__host__ __device__ __forceinline__ int fit_segments(int n) {
  constexpr int m = FIT_SEG_TILES * FitLds<FT>::TW;
  return (n + m - 1) / m;
}

// Geometry of one pass: element (line l, position i) lives at
// base[l * ls + i * ps]; LINE_CONTIG says ls == 1 (columns), else ps == 1.
// Rows are 16-byte aligned and the contiguous extent is a multiple of 4, so
// every 16-byte access lies wholly inside or wholly outside the data.
template <typename FT>
struct FitLine {
  const FT *in;
  FT *out;
  long in_ls, in_ps, out_ls, out_ps;
  const FT *coef;  // 1/den (forward) or cp (backward), per position
  const FT *coef_art;  // forward 1/den of a system starting at pb > 0
  int n;           // positions
  int nl;          // lines of this workgroup (<= 64)
  int last2;       // the last row's sub-diagonal is 2 (mirror end), else 1
  int pb, pe;      // forward: the positions [pb, pe) eliminated
  int sa, sb;      // the segment [sa, sb): stored, back-substituted
};

template <typename FT>
struct FitVec {
  static constexpr int VEC = FitLds<FT>::VEC;
  FT v[VEC];
};

// Mover vector w covers VEC consecutive positions of one line (rows) or
// VEC consecutive lines at one position (columns).
template <typename FT, bool LINE_CONTIG>
__device__ __forceinline__ void fit_map(int w, int &l, int &k) {
  constexpr int TW = FitLds<FT>::TW, VEC = FitLds<FT>::VEC;
  if (LINE_CONTIG) {
    k = w / (FIT_LINES / VEC);
    l = (w % (FIT_LINES / VEC)) * VEC;
  } else {
    l = w / (TW / VEC);
    k = (w % (TW / VEC)) * VEC;
  }
}

template <typename FT>
__device__ __forceinline__ void vec_ld(const FT *q, FitVec<FT> &r) {
  if constexpr (sizeof(FT) == 4) {
    const float4 t = *reinterpret_cast<const float4 *>(q);
    r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
  } else {
    const double2 t = *reinterpret_cast<const double2 *>(q);
    r.v[0] = t.x; r.v[1] = t.y;
  }
}

template <typename FT>
__device__ __forceinline__ void vec_st(FT *q, const FitVec<FT> &r) {
  if constexpr (sizeof(FT) == 4)
    *reinterpret_cast<float4 *>(q) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
  else
    *reinterpret_cast<double2 *>(q) = make_double2(r.v[0], r.v[1]);
}

// Registers of one tile in flight: NV vectors + the tile's coefficient.
template <typename FT>
struct FitRegs {
  FitVec<FT> x[FitLds<FT>::NV];
  FT c;
};

template <typename FT, bool LINE_CONTIG>
__device__ __forceinline__ void fit_load(const FitLine<FT> &G, int i0,
                                         FitRegs<FT> &r) {
  constexpr int NV = FitLds<FT>::NV, TW = FitLds<FT>::TW;
  const int mt = (int)threadIdx.x - 64;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    int l, k;
    fit_map<FT, LINE_CONTIG>(mt + q * FIT_MOVERS, l, k);
    if (l < G.nl && i0 + k < G.n)
      vec_ld(G.in + l * G.in_ls + (long)(i0 + k) * G.in_ps, r.x[q]);
    else
#pragma unroll
      for (int u = 0; u < FitLds<FT>::VEC; ++u) r.x[q].v[u] = (FT)0;
  }
  const FT *cf = (i0 == G.pb && G.pb > 0) ? G.coef_art - i0 : G.coef;
  r.c = (mt < TW && i0 + mt < G.n) ? cf[i0 + mt] : (FT)0;
}

template <typename FT, bool LINE_CONTIG>
__device__ __forceinline__ void fit_put(const FitRegs<FT> &r, FT *buf,
                                        FT *coef) {
  constexpr int NV = FitLds<FT>::NV, TW = FitLds<FT>::TW, LP = FitLds<FT>::LP,
                VEC = FitLds<FT>::VEC;
  const int mt = (int)threadIdx.x - 64;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    int l, k;
    fit_map<FT, LINE_CONTIG>(mt + q * FIT_MOVERS, l, k);
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      if (LINE_CONTIG)
        buf[k * LP + l + u] = r.x[q].v[u];
      else
        buf[(k + u) * LP + l] = r.x[q].v[u];
    }
  }
  if (mt < TW) coef[mt] = r.c;
}

template <typename FT, bool LINE_CONTIG>
__device__ __forceinline__ void fit_store(const FitLine<FT> &G, int i0,
                                          const FT *buf) {
  constexpr int NV = FitLds<FT>::NV, LP = FitLds<FT>::LP, VEC = FitLds<FT>::VEC;
  const int mt = (int)threadIdx.x - 64;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    int l, k;
    fit_map<FT, LINE_CONTIG>(mt + q * FIT_MOVERS, l, k);
    if (l < G.nl && i0 + k < G.n) {
      FitVec<FT> t;
#pragma unroll
      for (int u = 0; u < VEC; ++u)
        t.v[u] = LINE_CONTIG ? buf[k * LP + l + u] : buf[(k + u) * LP + l];
      vec_st(G.out + l * G.out_ls + (long)(i0 + k) * G.out_ps, t);
    }
  }
}

// One sweep over the tiles of a segment.  BACK = false: forward
// elimination over [pb, pe), d_i = (6 f_i - s_i d_{i-1}) / den_i with s_i =
// 2 at the line's last position, else 1 (d_{pb-1} = 0 gives the first row
// of the line, or of the truncated system, exactly); the segment's values
// are stored and, over the tile after it, the back substitution's value at
// sb is summed and returned.  BACK = true: back substitution c_i = d_i -
// cp_i c_{i+1} over the segment from c_sb = acc0 (c_n = 0 gives c_{n-1} =
// d_{n-1} exactly).  GHOST: also write the mirror rows c(-1) = c(1) and
// c(n) = c(n - 2) of every line.  Tiles are TW positions from a multiple
// of TW (pb, sa and the segment ends are multiples of TW, or n).
template <typename FT, bool LINE_CONTIG, bool BACK, bool GHOST>
__device__ __forceinline__ FT fit_sweep(const FitLine<FT> &G, FitLds<FT> &S,
                                        FT acc0 = (FT)0) {
  constexpr int TW = FitLds<FT>::TW, LP = FitLds<FT>::LP;
  const int n = G.n;
  const int p0 = BACK ? G.sa : G.pb, p1 = BACK ? G.sb : G.pe;
  const int nt = (p1 - p0 + TW - 1) / TW;
  const int tlast = p0 + (nt - 1) * TW;
  const bool mover = threadIdx.x >= 64;
  const int lane = threadIdx.x & 63;
  // tile t of the sweep order starts at position tile_i0(t)
  auto tile_i0 = [&](int t) { return BACK ? tlast - t * TW : p0 + t * TW; };
  auto stored = [&](int i0) { return i0 >= G.sa && i0 < G.sb; };
  // two register sets: tile u is loaded into set u % 2 three iterations
  // before it is needed and put into LDS one iteration before
  FitRegs<FT> ra, rb;
  if (mover) {
    fit_load<FT, LINE_CONTIG>(G, tile_i0(0), ra);
    fit_put<FT, LINE_CONTIG>(ra, S.buf[0], S.coef[0]);
    if (nt > 1) fit_load<FT, LINE_CONTIG>(G, tile_i0(1), rb);
    if (nt > 2) fit_load<FT, LINE_CONTIG>(G, tile_i0(2), ra);
  }
  __syncthreads();
  auto mover_step = [&](int t, FitRegs<FT> &rs) {
    if (t + 1 < nt) {
      fit_put<FT, LINE_CONTIG>(rs, S.buf[(t + 1) % FIT_NB],
                               S.coef[(t + 1) % FIT_NB]);
      if (t + 3 < nt) fit_load<FT, LINE_CONTIG>(G, tile_i0(t + 3), rs);
    }
  };
  FT acc = acc0, csum = (FT)0, w = (FT)1;
  for (int t = 0; t < nt; ++t) {
    const int b = t % FIT_NB;
    if (!mover) {
      const int i0 = tile_i0(t);
      const int kn = min(TW, n - i0);
      FT *col = S.buf[b] + lane;
      const FT *cf = S.coef[b];
      // positions [0, kb) in unguarded blocks of 16; the tile's remainder
      // (and the last position of the line, whose sub-diagonal is 2) alone
      const int kb = (i0 + kn == n) ? ((kn - 1) & ~15) : kn;
      if (!BACK && i0 >= G.sb) {
        // the tile after the segment: eliminate, and sum the back
        // substitution from its end down to sb
        for (int k = 0; k < kn; ++k) {
          const FT sd = (G.last2 && i0 + k == n - 1) ? (FT)2 * acc : acc;
          acc = ((FT)6 * col[k * LP] - sd) * cf[k];
          csum = fma(w, acc, csum);
          w = -w * cf[k];
        }
      } else if (!BACK) {
        for (int k0 = 0; k0 < kb; k0 += 16) {
          FT v[16], c[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            v[u] = col[(k0 + u) * LP];
            c[u] = cf[k0 + u];
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            acc = ((FT)6 * v[u] - acc) * c[u];
            v[u] = acc;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) col[(k0 + u) * LP] = v[u];
        }
        for (int k = kb; k < kn; ++k) {
          const FT sd = (G.last2 && i0 + k == n - 1) ? (FT)2 * acc : acc;
          acc = ((FT)6 * col[k * LP] - sd) * cf[k];
          col[k * LP] = acc;
        }
      } else {
        auto ghost = [&](int i) {
          if (GHOST && lane < G.nl) {
            if (i == 1) G.out[lane * G.out_ls - G.out_ps] = acc;
            if (i == n - 2) G.out[lane * G.out_ls + (long)n * G.out_ps] = acc;
          }
        };
        for (int k = kn - 1; k >= kb; --k) {
          acc = col[k * LP] - cf[k] * acc;
          col[k * LP] = acc;
          ghost(i0 + k);
        }
        for (int k0 = kb - 16; k0 >= 0; k0 -= 16) {
          FT v[16], c[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            v[u] = col[(k0 + u) * LP];
            c[u] = cf[k0 + u];
          }
#pragma unroll
          for (int u = 15; u >= 0; --u) {
            acc = v[u] - c[u] * acc;
            v[u] = acc;
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) col[(k0 + u) * LP] = v[u];
          if (GHOST && (i0 + k0 <= 1 || i0 + k0 + 15 >= n - 2)) {
            // rare: recover the two mirrored values from the block
#pragma unroll
            for (int u = 0; u < 16; ++u) {
              const int i = i0 + k0 + u;
              if (lane < G.nl && i == 1) G.out[lane * G.out_ls - G.out_ps] = v[u];
              if (lane < G.nl && i == n - 2)
                G.out[lane * G.out_ls + (long)n * G.out_ps] = v[u];
            }
          }
        }
      }
    } else {
      if (t >= 1 && stored(tile_i0(t - 1)))
        fit_store<FT, LINE_CONTIG>(G, tile_i0(t - 1), S.buf[(t - 1) % FIT_NB]);
      if (t & 1)
        mover_step(t, ra);
      else
        mover_step(t, rb);
    }
    __syncthreads();
  }
  if (mover && stored(tile_i0(nt - 1)))
    fit_store<FT, LINE_CONTIG>(G, tile_i0(nt - 1), S.buf[(nt - 1) % FIT_NB]);
  __syncthreads();
  return csum;
}

// Segment seg of a line of n positions: the stored range [sa, sb) and the
// eliminated range [pb, pe), extended by one tile where the segment does not
// reach the line's end.
template <typename FT>
__device__ __forceinline__ void fit_segment(FitLine<FT> &G, int seg) {
  constexpr int TW = FitLds<FT>::TW, m = FIT_SEG_TILES * TW;
  G.sa = seg * m;
  G.sb = min(G.n, G.sa + m);
  G.pb = (G.sa > 0) ? G.sa - TW : 0;
  G.pe = min(G.n, G.sb + TW);
}

// Spline tables (one array, see upload_tables): x pivots cp and 1/den,
// v pivots cp and 1/den, the periodic z and den, and 1/den of a system that
// starts at an artificial first row.
template <typename FT>
struct FitTables {
  const FT *cpx, *rix, *cpv, *riv, *art;
  __device__ __forceinline__ FitTables(const KP &p, const FT *tab)
      : cpx(tab), rix(tab + p.nx), cpv(tab + 2 * p.nx),
        riv(tab + 2 * p.nx + p.nv), art(tab + 3 * p.nx + 2 * p.nv + 1) {}
};

// Solve along x, work item w: rows [64 chunk, 64 chunk + 64) of segment seg
// (w = chunk * segments + seg): F (padded) -> T.
template <typename FT>
__device__ __forceinline__ void fit_x_rows(const KP &p, const FT *__restrict__ F,
                                          FT *__restrict__ T,
                                          const FT *__restrict__ tab,
                                          const int w, FitLds<FT> &S) {
  const FitTables<FT> tb(p, tab);
  const int nseg = fit_segments<FT>(p.nx);
  const int chunk = w / nseg, seg = w - chunk * nseg;
  const int j0 = chunk * FIT_LINES;
  FitLine<FT> G;
  G.n = p.nx;
  G.nl = min(FIT_LINES, p.nv - j0);
  G.in = F + (long)(j0 + PV) * p.pitch + PX;
  G.in_ls = p.pitch;
  G.in_ps = 1;
  G.out = T + (size_t)j0 * p.nx;
  G.out_ls = p.nx;
  G.out_ps = 1;
  G.coef = tb.rix;
  G.coef_art = tb.art;
  G.last2 = !p.per;  // periodic x: the cyclic system's tridiagonal part
  fit_segment<FT>(G, seg);
  const FT cb = fit_sweep<FT, false, false, false>(G, S);
  G.in = G.out;
  G.in_ls = G.out_ls;
  G.coef = tb.cpx;
  fit_sweep<FT, false, true, false>(G, S, cb);
}

// Solve along v, work item w: columns [64 chunk, 64 chunk + 64) of segment
// seg: T -> C (padded, with the mirror ghost rows).
template <typename FT>
__device__ __forceinline__ void fit_v_cols(const KP &p, const FT *__restrict__ T,
                                          FT *__restrict__ C,
                                          const FT *__restrict__ tab,
                                          const int w, FitLds<FT> &S) {
  const FitTables<FT> tb(p, tab);
  const int nseg = fit_segments<FT>(p.nv);
  const int chunk = w / nseg, seg = w - chunk * nseg;
  const int i0 = chunk * FIT_LINES;
  FitLine<FT> G;
  G.n = p.nv;
  G.nl = min(FIT_LINES, p.nx - i0);
  G.in = T + i0;
  G.in_ls = 1;
  G.in_ps = p.nx;
  G.out = C + (long)PV * p.pitch + PX + i0;
  G.out_ls = 1;
  G.out_ps = p.pitch;
  G.coef = tb.riv;
  G.coef_art = tb.art;
  G.last2 = 1;
  fit_segment<FT>(G, seg);
  const FT cb = fit_sweep<FT, true, false, false>(G, S);
  G.in = G.out;
  G.in_ps = G.out_ps;
  G.coef = tb.cpv;
  fit_sweep<FT, true, true, true>(G, S, cb);
}

template <typename FT>
__global__ __launch_bounds__(FIT_THREADS) void k_fit_x(
    KP p, const FT *__restrict__ F, FT *__restrict__ T,
    const FT *__restrict__ tab) {
  __shared__ FitLds<FT> S;
  fit_x_rows<FT>(p, F, T, tab, blockIdx.x, S);
}

template <typename FT>
__global__ __launch_bounds__(FIT_THREADS) void k_fit_v(
    KP p, const FT *__restrict__ T, FT *__restrict__ C,
    const FT *__restrict__ tab) {
  __shared__ FitLds<FT> S;
  fit_v_cols<FT>(p, T, C, tab, blockIdx.x, S);
}

// Mirror ghost columns c(-1, j) = c(1, j), c(nx, j) = c(nx - 2, j) for
// j in [-1, nv] (corners follow from the ghost rows).
template <typename FT>
__device__ __forceinline__ void ghost_x_rows(const KP &p, FT *__restrict__ C,
                                            const int chunk) {
  const int j = chunk * 256 + (int)threadIdx.x - 1;
  if (j > p.nv) return;
  const long pt = p.pitch;
  FT *row = C + (long)(j + PV) * pt + PX;
  row[-1] = row[1];
  row[p.nx] = row[p.nx - 2];
}

template <typename FT>
__global__ __launch_bounds__(256) void k_ghost_x(KP p, FT *__restrict__ C) {
  ghost_x_rows<FT>(p, C, blockIdx.x);
}

// Periodic x, cyclic spline system (Sherman-Morrison): T holds y = B^-1 6F
// per row (B the tridiagonal part, diagonal 8, 4, .., 4, 4.25); with z =
// B^-1 (-4, 0, .., 0, 1) the coefficients are y - [(y_0 - y_{n-1}/4) / den]
// z, den = (1 + z_0) - z_{n-1}/4.  One workgroup per row.
template <typename FT>
__global__ __launch_bounds__(256) void k_fit_x_cyclic(
    KP p, FT *__restrict__ T, const FT *__restrict__ z,
    const FT *__restrict__ den) {
  FT *row = T + (size_t)blockIdx.x * p.nx;
  const FT num = row[0] - (FT)0.25 * row[p.nx - 1];
  const FT fact = num / den[0];
  __syncthreads();  // every thread has read y_0 and y_{n-1}
  for (int i = threadIdx.x; i < p.nx; i += 256) row[i] = row[i] - fact * z[i];
}

// Periodic x: 16 ghost columns on each side of rows [jlo, jhi] hold copies
// of the other end of the row (one thread per row).
template <typename FT>
__global__ __launch_bounds__(256) void k_ghost_periodic(KP p,
                                                        FT *__restrict__ A,
                                                        int jlo, int jhi) {
  const int j = jlo + (int)(blockIdx.x * 256 + threadIdx.x);
  if (j > jhi) return;
  FT *row = A + (long)(j + PV) * p.pitch + PX;
#pragma unroll 4
  for (int k = 1; k <= PX; ++k) {
    row[-k] = row[p.nx - k];
    row[p.nx - 1 + k] = row[k - 1];
  }
}


// Rows [j0, j0 + nrows) of f0 (double, src holds those rows) -> F (padded
// interior), the outermost ring zeroed.
template <typename FT>
__global__ __launch_bounds__(256) void k_load_f0(KP p,
                                                 const double *__restrict__ src,
                                                 int j0, int nrows,
                                                 FT *__restrict__ F) {
  const long long n = (long long)p.nx * nrows;
  const long long gsz = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += gsz) {
    const int jr = (int)(q / p.nx), i = (int)(q - (long long)jr * p.nx);
    const int j = j0 + jr;
    const bool ring = (j == 0 || j == p.nv - 1) ||
                      (!p.per && (i == 0 || i == p.nx - 1));
    F[(long)(j + PV) * p.pitch + (i + PX)] = ring ? (FT)0 : (FT)src[q];
  }
}

// Variable step, first step (section 2.4): column sums of F_ini, one thread
// per column, in the fixed order of the reconstruction's density (8-row
// strips sequential, strips added in order into 64-row groups, groups in
// increasing order; boundaries on rows congruent to ov), into S[nx].
template <typename FT>
__global__ __launch_bounds__(256) void k_colsum_F(KP p,
                                                  const FT *__restrict__ F,
                                                  double *__restrict__ S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.nx) return;
  const FT *col = F + (long)PV * p.pitch + PX + i;
  double tot = 0.0, grp = 0.0, strip = 0.0;
  for (int j = 0; j < p.nv; ++j) {
    strip += (double)col[(long)j * p.pitch];
    const int r = j + 1 - p.ov;
    const bool last = (j == p.nv - 1);
    if ((r & 7) == 0 || last) {
      grp += strip;
      strip = 0.0;
    }
    if ((r & 63) == 0 || last) {
      tot += grp;
      grp = 0.0;
    }
  }
  S[i] = tot;
}

// The clock at t = 0: slot 0 = {dt_0, 0, 0, 0}, dt_0 from the largest
// dv S(i); slot 1 cleared.  One workgroup.
__global__ __launch_bounds__(1024) void k_clock_init(KP p,
                                                     const double *__restrict__ S) {
  __shared__ double red[1024 / 64];
  const int tid = threadIdx.x;
  double m = 0.0;
  for (int i = tid; i < p.nx; i += 1024) m = fmax(m, p.dv * S[i]);
  m = wave_max(m);
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    double r = 0.0;
    for (int w = 0; w < 1024 / 64; ++w) r = fmax(r, red[w]);
    for (int q = 0; q < CK_DOUBLES; ++q) p.clk[q] = 0.0;
    p.clk[CK_DT] = next_dt(p, r);
    p.clk[CK_RHO] = r;
  }
}

}  // namespace vpk
