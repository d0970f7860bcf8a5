// vp4_kernels.hpp -- HIP kernels (gfx950) of the metric semi-Lagrangian
// method in 4D phase space: 2D periodic space (x, y) x 2D velocity (u, w)
// (Colombi & Alard, arXiv:1705.03750: 60 numbers per element, section 2.1;
// 15-point interpolation, section 2.2.1; Fourier solution of Poisson's
// equation for periodic systems, section 2.5).
//
// Arithmetic is written operation by operation (-ffp-contract=off).
//
// Device data (inside the caller's workspace):
//   F, C, f  [nv][nv][ns][ns] (x fastest): F_ini, spline coefficients and a
//            scratch f; no padding -- the interpolations wrap x and y and
//            treat u and w as zero (F) or mirrored (C) outside the grid.
//   state    SoA [60][E]; rec AoS [E][60]: X (4), A = T^-1 (16), H (40).
//   lists    per query block of 4^4 sites: a count and cap element ids;
//            every element whose validity window can reach a site of the
//            block is listed.  Block boundaries sit half an element spacing
//            (mod 4) off the grid origin, on the element lattice, so that an
//            undeformed lattice puts 2 elements per axis in each list; the
//            first and last block of an axis may be partial, and on x and y
//            they are the two halves of the seam block, which share a list.
//   part     density partials [velocity blocks][ns^2] (one row of partial
//            sums per velocity block); rho [ns^2]; spectra and the 12 force
//            fields (a_x, a_y, grad a, Hessian of a) [12][ns^2].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vp4k {

constexpr int NST = 60;
constexpr int S_P = 0, S_T = 4, S_H = 20;  // state rows
constexpr int RS = 60;                     // record doubles
constexpr int BLK = 4;                     // sites per axis of a block
constexpr int SPAN = 4096;                 // max blocks of one element
constexpr int STAGE = 32;                  // records staged per round
enum { FL_NUMERIC = 1, FL_WIDE = 2 };
enum { M_DENSITY = 0, M_F = 1, M_ASSIGN = 2 };

// symmetric pair (b, c), b <= c: 00 01 02 03 11 12 13 22 23 33
__device__ __constant__ const int PB[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
__device__ __constant__ const int PC[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

struct KP {
  int ns, nv, ss, sv, ms, mv, E;
  int o[4];      // block origin offset per axis, (spacing / 2) mod 4
  int ob[4];     // 1 when o > 0 (a partial first block)
  int nb[4];     // blocks per axis
  int nls;       // list columns per space axis (ns / 4)
  int cap;       // list slots per block
  double L, hL, vmax, dx, du, inv_dx, inv_du, G, dt, h, beta;
  double Dm[4], rD[4];
};

__device__ __forceinline__ double coord(const KP &p, int a, int i) {
  return a < 2 ? ((double)i + 0.5) * p.dx : -p.vmax + ((double)i + 0.5) * p.du;
}
__device__ __forceinline__ double lat_q(const KP &p, int a, int k) {
  const int s = a < 2 ? p.ss : p.sv;
  return coord(p, a, s * k + s / 2);
}
__device__ __forceinline__ void lat_index(const KP &p, int e, int k[4]) {
  k[0] = e % p.ms;
  e /= p.ms;
  k[1] = e % p.ms;
  e /= p.ms;
  k[2] = e % p.mv;
  k[3] = e / p.mv;
}
__device__ __forceinline__ double wrapL(const KP &p, double x) {
  if (x < 0.0) {
    x = x + p.L;
    if (x >= p.L) x = 0.0;
  } else if (x >= p.L) {
    x = x - p.L;
    if (x < 0.0) x = 0.0;
  }
  return x;
}
__device__ __forceinline__ double image(const KP &p, double d) {
  if (d > p.hL) return d - p.L;
  if (d < -p.hL) return d + p.L;
  return d;
}

// Query-block geometry: block b of axis a starts at site o_a + 4 (b - ob_a),
// o_a = (element spacing / 2) mod 4, the element lattice's offset.
__device__ __forceinline__ int floordiv4(int i) {
  return (i >= 0) ? i / BLK : -((-i + BLK - 1) / BLK);
}
__device__ __forceinline__ int blk_of(const KP &p, int a, int i) {
  return floordiv4(i - p.o[a]) + p.ob[a];
}
__device__ __forceinline__ int blk_first(const KP &p, int a, int b) {
  return p.o[a] + BLK * (b - p.ob[a]);
}
// List of block (bx, by, bu, bw): x and y wrap onto ns / 4 list columns.
__device__ __forceinline__ long long list_of(const KP &p, int bx, int by, int bu,
                                             int bw) {
  const int lx = ((bx % p.nls) + p.nls) % p.nls;
  const int ly = ((by % p.nls) + p.nls) % p.nls;
  return (((long long)bw * p.nb[2] + bu) * p.nls + ly) * p.nls + lx;
}

// ------------------------------------------------------------- elements

__global__ __launch_bounds__(256) void k4_reset(KP p, double *__restrict__ st) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.E) return;
  const size_t E = (size_t)p.E;
  int k[4];
  lat_index(p, e, k);
  for (int s = 0; s < NST; ++s) st[s * E + e] = 0.0;
  for (int a = 0; a < 4; ++a) {
    st[(S_P + a) * E + e] = lat_q(p, a, k[a]);
    st[(S_T + 5 * a) * E + e] = 1.0;
  }
}

__global__ __launch_bounds__(256) void k4_zero(int *__restrict__ a, long long n) {
  const long long gsz = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += gsz)
    a[i] = 0;
}

// Drift over h of the state held in s[60] (section 2.4 per space axis):
// x_i += h v_i (then the periodic wrap), T_i. += h T_{i+2}., H_i.. += h
// H_{i+2}...
__device__ __forceinline__ void drift4(const KP &p, double *s, double h) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    s[S_P + i] = wrapL(p, fma(h, s[S_P + i + 2], s[S_P + i]));
#pragma unroll
    for (int j = 0; j < 4; ++j)
      s[S_T + 4 * i + j] = fma(h, s[S_T + 4 * (i + 2) + j], s[S_T + 4 * i + j]);
#pragma unroll
    for (int q = 0; q < 10; ++q)
      s[S_H + 10 * i + q] = fma(h, s[S_H + 10 * (i + 2) + q], s[S_H + 10 * i + q]);
  }
}

// A = T^-1 by the adjugate (2 x 2 minors of rows 0-1 and rows 2-3); false
// when det T is not positive and finite.
__device__ __forceinline__ bool inv4(const double *m, double *r, double &det) {
  const double a0 = m[0] * m[5] - m[4] * m[1];
  const double a1 = m[0] * m[6] - m[4] * m[2];
  const double a2 = m[0] * m[7] - m[4] * m[3];
  const double a3 = m[1] * m[6] - m[5] * m[2];
  const double a4 = m[1] * m[7] - m[5] * m[3];
  const double a5 = m[2] * m[7] - m[6] * m[3];
  const double b5 = m[10] * m[15] - m[14] * m[11];
  const double b4 = m[9] * m[15] - m[13] * m[11];
  const double b3 = m[9] * m[14] - m[13] * m[10];
  const double b2 = m[8] * m[15] - m[12] * m[11];
  const double b1 = m[8] * m[14] - m[12] * m[10];
  const double b0 = m[8] * m[13] - m[12] * m[9];
  det = ((((a0 * b5 - a1 * b4) + a2 * b3) + a3 * b2) - a4 * b1) + a5 * b0;
  if (!(det > 0.0) || !isfinite(det)) return false;
  const double q = 1.0 / det;
  r[0] = ((m[5] * b5 - m[6] * b4) + m[7] * b3) * q;
  r[1] = ((-m[1] * b5 + m[2] * b4) - m[3] * b3) * q;
  r[2] = ((m[13] * a5 - m[14] * a4) + m[15] * a3) * q;
  r[3] = ((-m[9] * a5 + m[10] * a4) - m[11] * a3) * q;
  r[4] = ((-m[4] * b5 + m[6] * b2) - m[7] * b1) * q;
  r[5] = ((m[0] * b5 - m[2] * b2) + m[3] * b1) * q;
  r[6] = ((-m[12] * a5 + m[14] * a2) - m[15] * a1) * q;
  r[7] = ((m[8] * a5 - m[10] * a2) + m[11] * a1) * q;
  r[8] = ((m[4] * b4 - m[5] * b2) + m[7] * b0) * q;
  r[9] = ((-m[0] * b4 + m[1] * b2) - m[3] * b0) * q;
  r[10] = ((m[12] * a4 - m[13] * a2) + m[15] * a0) * q;
  r[11] = ((-m[8] * a4 + m[9] * a2) - m[11] * a0) * q;
  r[12] = ((-m[4] * b3 + m[5] * b1) - m[6] * b0) * q;
  r[13] = ((m[0] * b3 - m[1] * b1) + m[2] * b0) * q;
  r[14] = ((-m[12] * a3 + m[13] * a1) - m[14] * a0) * q;
  r[15] = ((m[8] * a3 - m[9] * a1) + m[10] * a0) * q;
  return true;
}

// Can the validity window of the element (record r) hold a site of the
// block whose sites span [g0, g1] per axis (space columns unwrapped)?  l = A dP is
// linear, so over the block's box each l_a ranges over its centre value +-
// sum_b |A_ab| half-width_b; rounding margins as in the 2D engine.
__device__ __forceinline__ bool block_meets(const KP &p, const double *r,
                                            const int g0[4], const int g1[4]) {
  double m[4], h[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double lo = coord(p, a, g0[a]), hi = coord(p, a, g1[a]);
    m[a] = 0.5 * (lo + hi) - r[a];
    h[a] = 0.5 * (hi - lo);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double *A = r + 4 + 4 * a;
    double c = 0.0, rad = 0.0, mag = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      c = fma(A[b], m[b], c);
      rad = fma(fabs(A[b]), h[b], rad);
      mag = fma(fabs(A[b]), fabs(m[b]) + h[b] + 1.0, mag);
    }
    const double tol = 0x1p-36 * (mag + p.Dm[a]);
    if (!(fabs(c) - rad < p.Dm[a] + tol)) return false;
  }
  return true;
}

// Predictor drift (when `drift`), inverse and query record of every
// element, and (when `reg`) its registration in every block its window can
// reach.  Counts must be zero on entry.
__global__ __launch_bounds__(256) void k4_predict(
    KP p, double *__restrict__ st, double *__restrict__ rec,
    int *__restrict__ cnt, int *__restrict__ lst, int *__restrict__ flags,
    int drift, int reg) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.E) return;
  const size_t E = (size_t)p.E;
  double s[NST];
#pragma unroll
  for (int q = 0; q < NST; ++q) s[q] = st[q * E + e];
  if (drift) {
    drift4(p, s, p.h);
#pragma unroll
    for (int q = 0; q < 40; ++q) st[q * E + e] = s[q];
  }
  double A[16], det;
  const bool ok = inv4(s + S_T, A, det);
  double *r = rec + (size_t)e * RS;
#pragma unroll
  for (int a = 0; a < 4; ++a) r[a] = s[S_P + a];
#pragma unroll
  for (int q = 0; q < 16; ++q) r[4 + q] = ok ? A[q] : 0.0;
#pragma unroll
  for (int q = 0; q < 40; ++q) r[20 + q] = s[S_H + q];
  bool bad = !ok;
#pragma unroll
  for (int a = 0; a < 4; ++a) bad = bad || !isfinite(s[S_P + a]);
  if (bad) {
    atomicOr(flags, FL_NUMERIC);
    return;
  }
  if (!reg) return;
  // Eulerian reach per axis: |dP_a| <= sum_b |T_ab| Dm_b, in sites, with
  // a relative margin for the rounding of l = A dP
  int blo[4], bhi[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double reach = 0.0, tsum = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      reach = fma(fabs(s[S_T + 4 * a + b]), p.Dm[b], reach);
      tsum += fabs(s[S_T + 4 * a + b]);
    }
    const double rel = 0x1p-20 + 0x1p-40 * (tsum * tsum) * fabs(1.0 / det);
    const double inv_d = a < 2 ? p.inv_dx : p.inv_du;
    const double rs = reach * inv_d * (1.0 + rel) + 0x1p-20;
    const double c = (a < 2 ? s[S_P + a] : s[S_P + a] + p.vmax) * inv_d - 0.5;
    int lo = (int)ceil(c - rs), hi = (int)floor(c + rs);
    if (a >= 2) {
      lo = max(lo, 0);
      hi = min(hi, p.nv - 1);
      if (lo > hi) return;
    } else if (!(rs < 0.5 * (double)p.ns - 2.0 * BLK) ||
               hi - lo > p.ns - 3 * BLK) {
      atomicOr(flags, FL_WIDE);  // too wide for nearest-image lists
      return;
    }
    blo[a] = blk_of(p, a, lo);  // unwrapped on x and y
    bhi[a] = blk_of(p, a, hi);
  }
  const long long nblk = (long long)(bhi[0] - blo[0] + 1) *
                         (bhi[1] - blo[1] + 1) * (bhi[2] - blo[2] + 1) *
                         (bhi[3] - blo[3] + 1);
  if (nblk > SPAN) {
    atomicOr(flags, FL_WIDE);
    return;
  }
  int b[4], g0[4], g1[4];
  for (b[3] = blo[3]; b[3] <= bhi[3]; ++b[3])
    for (b[2] = blo[2]; b[2] <= bhi[2]; ++b[2])
      for (b[1] = blo[1]; b[1] <= bhi[1]; ++b[1])
        for (b[0] = blo[0]; b[0] <= bhi[0]; ++b[0]) {
          for (int a = 0; a < 4; ++a) {
            g0[a] = blk_first(p, a, b[a]);
            g1[a] = g0[a] + BLK - 1;
            if (a >= 2) {  // the live sites of a partial velocity block
              g0[a] = max(g0[a], 0);
              g1[a] = min(g1[a], p.nv - 1);
            }
          }
          if (!block_meets(p, r, g0, g1)) continue;
          const long long blk = list_of(p, b[0], b[1], b[2], b[3]);
          const int slot = atomicAdd(&cnt[blk], 1);
          if (slot < p.cap) lst[blk * p.cap + slot] = e;
        }
}

// Second-order inverse map of one element (record r) at site P, in two
// parts: l = A dP (nearest image in x, y) with the validity |l_a| < Dm_a,
// then u_a = l^T H_a l over the symmetric pairs and dQ = l - A u / 2.  The
// query evaluates the second part only where the first found the element
// valid, so a wavefront skips it for an element valid at none of its sites.
__device__ __forceinline__ bool map4_l(const KP &p, const double *r,
                                       const double P[4], double l[4]) {
  double d[4];
  d[0] = image(p, P[0] - r[0]);
  d[1] = image(p, P[1] - r[1]);
  d[2] = P[2] - r[2];
  d[3] = P[3] - r[3];
  bool valid = true;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double *A = r + 4 + 4 * a;
    l[a] = fma(A[3], d[3], fma(A[2], d[2], fma(A[1], d[1], A[0] * d[0])));
    valid = valid && (fabs(l[a]) < p.Dm[a]);
  }
  return valid;
}

__device__ __forceinline__ void map4_q(const double *r, const double l[4],
                                       double dq[4]) {
  double u[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double *H = r + 20 + 10 * a;
    double s = H[0] * (l[0] * l[0]);
    s = fma(2.0 * H[1], l[0] * l[1], s);
    s = fma(2.0 * H[2], l[0] * l[2], s);
    s = fma(2.0 * H[3], l[0] * l[3], s);
    s = fma(H[4], l[1] * l[1], s);
    s = fma(2.0 * H[5], l[1] * l[2], s);
    s = fma(2.0 * H[6], l[1] * l[3], s);
    s = fma(H[7], l[2] * l[2], s);
    s = fma(2.0 * H[8], l[2] * l[3], s);
    s = fma(H[9], l[3] * l[3], s);
    u[a] = s;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const double *A = r + 4 + 4 * a;
    double s = l[a];
#pragma unroll
    for (int b = 0; b < 4; ++b) s = fma(-0.5 * A[b], u[b], s);
    dq[a] = s;
  }
}

__device__ __forceinline__ bool map4(const KP &p, const double *r,
                                     const double P[4], double dq[4]) {
  double l[4];
  const bool valid = map4_l(p, r, P, l);
  map4_q(r, l, dq);
  return valid;
}

__device__ __forceinline__ double dist2(const KP &p, const double dq[4]) {
  const double z0 = dq[0] * p.rD[0], z1 = dq[1] * p.rD[1];
  const double z2 = dq[2] * p.rD[2], z3 = dq[3] * p.rD[3];
  return fma(z3, z3, fma(z2, z2, fma(z1, z1, z0 * z0)));
}

// Site of thread t of block blk (blocks numbered x fastest): (i, j, k, l),
// its coordinates, whether it lies on the grid, and the block's list.
__device__ __forceinline__ bool block_site(const KP &p, long long blk, int t,
                                           int g[4], double P[4], int bb[4],
                                           long long &list) {
  long long b = blk;
  bb[0] = (int)(b % p.nb[0]);
  b /= p.nb[0];
  bb[1] = (int)(b % p.nb[1]);
  b /= p.nb[1];
  bb[2] = (int)(b % p.nb[2]);
  bb[3] = (int)(b / p.nb[2]);
  const int loc[4] = {t & 3, (t >> 2) & 3, (t >> 4) & 3, t >> 6};
  bool live = true;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    g[a] = blk_first(p, a, bb[a]) + loc[a];
    P[a] = coord(p, a, g[a]);
    live = live && g[a] >= 0 && g[a] < (a < 2 ? p.ns : p.nv);
  }
  list = list_of(p, bb[0], bb[1], bb[2], bb[3]);
  return live;
}

// Nearest valid element (smallest (d^2, id)) of the workgroup's block: the
// list's records are staged in LDS STAGE at a time; with an overflowed list
// or a too-wide element, every element is scanned.
__device__ __forceinline__ int query4(const KP &p, const double *__restrict__ rec,
                                      const int *__restrict__ L, int n,
                                      bool scan_all, const double P[4],
                                      double bdq[4], double *stage) {
  double bd = __builtin_inf();
  int best = -1;
  for (int a = 0; a < 4; ++a) bdq[a] = 0.0;
  const int tid = threadIdx.x;
  const int total = scan_all ? p.E : n;
  for (int c0 = 0; c0 < total; c0 += STAGE) {
    const int m = min(STAGE, total - c0);
    __syncthreads();
    for (int q = tid; q < m * RS; q += 256) {
      const int k = q / RS, o = q - k * RS;
      const int e = scan_all ? c0 + k : L[c0 + k];
      stage[q] = rec[(size_t)e * RS + o];
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
      const int e = scan_all ? c0 + k : L[c0 + k];
      const double *r = stage + k * RS;
      double l[4];
      if (map4_l(p, r, P, l)) {
        double dq[4];
        map4_q(r, l, dq);
        const double d2 = dist2(p, dq);
        if (d2 < bd || (d2 == bd && e < best)) {
          bd = d2;
          best = e;
          for (int a = 0; a < 4; ++a) bdq[a] = dq[a];
        }
      }
    }
  }
  return best;
}

// ------------------------------------------------------- interpolations

// 15-point second-order interpolation (section 2.2.1 in four dimensions):
// nearest node, its 8 axis neighbours (Lagrange signs), and one cross term
// per axis pair at the floor corner of that plane.  x, y positions clamped
// to [-12, ns + 11] and wrapped; zero outside the u, w grid.  Every stencil
// index along an axis is the nearest node's -1, 0 or +1 (the floor corner
// is the nearest node or the one below), so the wrapped offsets of the
// three are formed once per axis.
template <typename FT>
__device__ __forceinline__ FT int15(const KP &p, const FT *__restrict__ F,
                                    const double sin_[4]) {
  double s[4];
  for (int a = 0; a < 4; ++a) s[a] = sin_[a];
  for (int a = 0; a < 2; ++a) {
    if (s[a] < -12.0) s[a] = -12.0;
    if (s[a] > (double)p.ns + 11.0) s[a] = (double)p.ns + 11.0;
  }
  for (int a = 2; a < 4; ++a)
    if (!(s[a] > -4.0 && s[a] < p.nv + 3.0)) return (FT)0;
  int n[4], cf[4];
  FT dq[4];
  for (int a = 0; a < 4; ++a) {
    const double fn = floor(s[a] + 0.5);
    n[a] = (int)fn;
    cf[a] = (int)floor(s[a]) - n[a] + 1;  // 0 or 1: index of the floor node
    dq[a] = (FT)(s[a] - fn);
  }
  // element offsets of nodes n-1, n, n+1 per axis (-1: off the u, w grid)
  const long long str[4] = {1, p.ns, (long long)p.ns * p.ns,
                            (long long)p.ns * p.ns * p.nv};
  long long off[4][3];
  for (int a = 0; a < 4; ++a) {
    for (int q = 0; q < 3; ++q) {
      int i = n[a] - 1 + q;
      if (a < 2) {
        i = ((i % p.ns) + p.ns) % p.ns;
        off[a][q] = (long long)i * str[a];
      } else {
        off[a][q] = (i >= 0 && i < p.nv) ? (long long)i * str[a] : -1;
      }
    }
  }
  auto at = [&](int q0, int q1, int q2, int q3) -> FT {
    if (off[2][q2] < 0 || off[3][q3] < 0) return (FT)0;
    return F[off[0][q0] + off[1][q1] + off[2][q2] + off[3][q3]];
  };
  FT w0 = (FT)1 - dq[0] * dq[0];
  for (int a = 1; a < 4; ++a) w0 = w0 - dq[a] * dq[a];
  FT f = at(1, 1, 1, 1) * w0;
  for (int a = 0; a < 4; ++a) {
    const FT h = (FT)0.5 * dq[a];
    const FT wp = h * ((FT)1 + dq[a]), wm = h * ((FT)1 - dq[a]);
    int qp[4] = {1, 1, 1, 1}, qm[4] = {1, 1, 1, 1};
    qp[a] = 2;
    qm[a] = 0;
    f = fma(at(qp[0], qp[1], qp[2], qp[3]), wp, f);
    f = fma(-at(qm[0], qm[1], qm[2], qm[3]), wm, f);
  }
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b) {
      int q[4] = {1, 1, 1, 1};
      q[a] = cf[a] + 1;
      q[b] = cf[b] + 1;
      const FT f11 = at(q[0], q[1], q[2], q[3]);
      q[a] = cf[a];
      q[b] = cf[b];
      const FT f00 = at(q[0], q[1], q[2], q[3]);
      q[a] = cf[a] + 1;
      const FT f10 = at(q[0], q[1], q[2], q[3]);
      q[a] = cf[a];
      q[b] = cf[b] + 1;
      const FT f01 = at(q[0], q[1], q[2], q[3]);
      const FT cross = ((f11 + f00) - f10) - f01;
      f = fma(cross, dq[a] * dq[b], f);
    }
  return f;
}

// Cubic B-spline weights.  Double precision: each times the rounded 1/6.
// Single precision: six times the weights, the 1/6^4 of the four axes
// applied once to the sum (two-float constant), because float(1/6) is 3e-8
// too large and that shared rounding would scale every resampled value by
// 1 + 1.2e-7 at each resampling.
template <typename FT>
__device__ __forceinline__ void bspw(double ud, FT b[4]) {
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

constexpr float INV1296_HI = (float)(1.0 / 1296.0);
constexpr float INV1296_LO =
    (float)(1.0 / 1296.0 - (double)(float)(1.0 / 1296.0));

// Tensor cubic B-spline (x, y periodic, clamped to [-12, ns + 11]; u, w on
// [0, nv - 1] with mirror ghosts c(-1) = c(1), c(n) = c(n - 2); 0 outside).
template <typename FT>
__device__ __forceinline__ FT spline4(const KP &p, const FT *__restrict__ C,
                                      const double sin_[4]) {
  double s[4];
  for (int a = 0; a < 4; ++a) s[a] = sin_[a];
  for (int a = 0; a < 2; ++a) {
    if (s[a] < -12.0) s[a] = -12.0;
    if (s[a] > (double)p.ns + 11.0) s[a] = (double)p.ns + 11.0;
  }
  for (int a = 2; a < 4; ++a)
    if (!(s[a] >= 0.0 && s[a] <= (double)(p.nv - 1))) return (FT)0;
  int i0[4];
  FT w[4][4];
  for (int a = 0; a < 4; ++a) {
    int i = (int)floor(s[a]);
    if (a >= 2 && i > p.nv - 2) i = p.nv - 2;
    i0[a] = i;
    bspw<FT>(s[a] - (double)i, w[a]);
  }
  int xi[4], yj[4], uk[4], wl[4];
  for (int q = 0; q < 4; ++q) {
    xi[q] = (((i0[0] - 1 + q) % p.ns) + p.ns) % p.ns;
    yj[q] = (((i0[1] - 1 + q) % p.ns) + p.ns) % p.ns;
    int k = i0[2] - 1 + q, l = i0[3] - 1 + q;
    if (k < 0) k = -k;
    if (k > p.nv - 1) k = 2 * (p.nv - 1) - k;
    if (l < 0) l = -l;
    if (l > p.nv - 1) l = 2 * (p.nv - 1) - l;
    uk[q] = k;
    wl[q] = l;
  }
  FT f = (FT)0;
  for (int l = 0; l < 4; ++l) {
    FT fu = (FT)0;
    for (int k = 0; k < 4; ++k) {
      FT fy = (FT)0;
      for (int j = 0; j < 4; ++j) {
        const FT *row =
            C + (((size_t)wl[l] * p.nv + uk[k]) * p.ns + yj[j]) * p.ns;
        FT r = w[0][0] * row[xi[0]];
        r = fma(w[0][1], row[xi[1]], r);
        r = fma(w[0][2], row[xi[2]], r);
        r = fma(w[0][3], row[xi[3]], r);
        fy = (j == 0) ? w[1][0] * r : fma(w[1][j], r, fy);
      }
      fu = (k == 0) ? w[2][0] * fy : fma(w[2][k], fy, fu);
    }
    f = (l == 0) ? w[3][0] * fu : fma(w[3][l], fu, f);
  }
  if constexpr (sizeof(FT) == 4) f = fmaf(f, INV1296_HI, f * INV1296_LO);
  return f;
}

__device__ __forceinline__ double Wk(double x) {
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

__device__ __forceinline__ void index_pos(const KP &p, const double Q[4],
                                          double s[4]) {
  s[0] = Q[0] * p.inv_dx - 0.5;
  s[1] = Q[1] * p.inv_dx - 0.5;
  s[2] = (Q[2] + p.vmax) * p.inv_du - 0.5;
  s[3] = (Q[3] + p.vmax) * p.inv_du - 0.5;
}

// ------------------------------------------------------- reconstruction

// One workgroup of 256 threads per 4^4-site block, one thread per site.
// M_DENSITY: the block's 16 velocity sites per (x, y) column are summed (w
// outer, u inner) into part[velocity block][y][x]; M_F: f; M_ASSIGN: ids.
template <typename FT, int MODE>
__global__ __launch_bounds__(256) void k4_recon(
    KP p, const double *__restrict__ rec, const int *__restrict__ cnt,
    const int *__restrict__ lst, const int *__restrict__ flags,
    const FT *__restrict__ F, double *__restrict__ part, FT *__restrict__ fout,
    int *__restrict__ aout) {
  __shared__ double stage[STAGE * RS];
  __shared__ double sf[256];
  const long long blk = blockIdx.x;
  const int t = threadIdx.x;
  int g[4], bb[4];
  double P[4];
  long long list;
  const bool live = block_site(p, blk, t, g, P, bb, list);
  const int n = cnt[list];
  const bool scan_all = (n > p.cap) || (flags[0] & FL_WIDE);
  double dq[4];
  const int best = query4(p, rec, lst + list * p.cap, n, scan_all, P, dq, stage);
  const size_t site =
      (((size_t)g[3] * p.nv + g[2]) * p.ns + g[1]) * p.ns + g[0];
  FT fv = (FT)0;
  if (MODE != M_ASSIGN && live && best >= 0) {
    int k[4];
    lat_index(p, best, k);
    double Q[4], s[4];
    for (int a = 0; a < 4; ++a) Q[a] = lat_q(p, a, k[a]) + dq[a];
    index_pos(p, Q, s);
    fv = int15<FT>(p, F, s);
  }
  if (MODE == M_F && live) fout[site] = fv;
  if (MODE == M_ASSIGN && live) aout[site] = best;
  if (MODE == M_DENSITY) {
    sf[t] = (double)fv;  // 0 off the grid
    __syncthreads();
    const int i = blk_first(p, 0, bb[0]) + (t & 3);
    const int j = blk_first(p, 1, bb[1]) + ((t >> 2) & 3);
    if (t < 16 && i >= 0 && i < p.ns && j >= 0 && j < p.ns) {
      double s = 0.0;
      for (int l = 0; l < 4; ++l)
        for (int k = 0; k < 4; ++k) s += sf[l * 64 + k * 16 + t];
      const long long vb = (long long)bb[3] * p.nb[2] + bb[2];
      part[(size_t)vb * p.ns * p.ns + (size_t)j * p.ns + i] = s;
    }
  }
}

// Resampling value of every site (section 2.3.2 axis by axis): nearest
// element, beta-restricted lattice neighbours (no offsets in more than one
// axis when an axis needs three; x, y wrap with a one-period shift), W(2d)
// blend of their Q, tensor spline of F_ini at Q_r; u, w edge rows zero.
// Writes into out (F_ini when resampling).
//
// Four wavefronts per SIMD (at most 128 VGPRs): the per-lane gathers of the
// neighbours' records need the latency hiding.  The slot offsets and the
// lattice wrap are selects, not branches that store into small arrays: the
// branch form, once the register budget made the compiler keep the offsets
// as one 4-lane vector, was miscompiled at this budget (the control-flow
// structurizer rebuilt that vector's phi with an undefined incoming value on
// the path q > 7 of the third axis, so slot 8 re-used slot 7's offsets, the
// diagonal (0, 0, +1, +1) with zero weight, and the +1 neighbour along the
// fourth axis dropped out of the blend).
template <typename FT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k4_remap(
    KP p, const double *__restrict__ rec, const int *__restrict__ cnt,
    const int *__restrict__ lst, const int *__restrict__ flags,
    const FT *__restrict__ C, FT *__restrict__ out) {
  __shared__ double stage[STAGE * RS];
  const long long blk = blockIdx.x;
  const int t = threadIdx.x;
  int g[4], bb[4];
  double P[4];
  long long list;
  const bool live = block_site(p, blk, t, g, P, bb, list);
  const int n = cnt[list];
  const bool scan_all = (n > p.cap) || (flags[0] & FL_WIDE);
  double dq[4];
  const int best = query4(p, rec, lst + list * p.cap, n, scan_all, P, dq, stage);
  if (!live) return;
  const size_t site =
      (((size_t)g[3] * p.nv + g[2]) * p.ns + g[1]) * p.ns + g[0];
  const bool edge = g[2] == 0 || g[2] == p.nv - 1 || g[3] == 0 || g[3] == p.nv - 1;
  if (edge || best < 0) {
    out[site] = (FT)0;
    return;
  }
  int k0[4], lo[4], hi[4];
  bool three = false;
  lat_index(p, best, k0);
  for (int a = 0; a < 4; ++a) {
    const double z = dq[a] * p.rD[a];
    lo[a] = (z < p.beta) ? -1 : 0;
    hi[a] = (z < -p.beta) ? 0 : 1;
    three = three || (hi[a] - lo[a] == 2);
  }
  // The beta-set in the order of the nested loops over the offsets (axis 3
  // slowest, axis 0 fastest), one slot per trip so that a wavefront runs at
  // most 16 neighbour maps whatever its lanes' sets: without a three-valued
  // axis the 16 corners d_a = lo_a + bit a of q; with one, the 9 slots
  // -1 on axes 3, 2, 1, 0, the centre, +1 on axes 0, 1, 2, 3, those outside
  // [lo, hi] skipped.
  double sw = 0.0, sq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int q = 0; q < 16; ++q) {
    int d[4];
    bool use = !three || q == 4;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (!three) {
        d[a] = lo[a] + ((q >> a) & 1);
      } else if (q == 3 - a) {
        d[a] = -1;
        use = lo[a] == -1;
      } else if (q == 5 + a) {
        d[a] = 1;
        use = hi[a] == 1;
      } else {
        d[a] = 0;
      }
    }
    int kk[4];
    double shift[2];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int k = k0[a] + d[a];
      if (a < 2) {  // x, y wrap with a one-period shift
        shift[a] = k < 0 ? -p.L : (k >= p.ms ? p.L : 0.0);
        kk[a] = k < 0 ? k + p.ms : (k >= p.ms ? k - p.ms : k);
      } else {      // u, w: no neighbour beyond the lattice
        use = use && k >= 0 && k < p.mv;
        kk[a] = k;
      }
    }
    if (!use) continue;
    const int m = ((kk[3] * p.mv + kk[2]) * p.ms + kk[1]) * p.ms + kk[0];
    double ex[4];
    map4(p, rec + (size_t)m * RS, P, ex);
    const double wgt = Wk(2.0 * sqrt(dist2(p, ex)));
    sw += wgt;
    for (int a = 0; a < 4; ++a) {
      const double Qa = (lat_q(p, a, kk[a]) + (a < 2 ? shift[a] : 0.0)) + ex[a];
      sq[a] = fma(wgt, Qa, sq[a]);
    }
  }
  double Q[4], s[4];
  for (int a = 0; a < 4; ++a)
    Q[a] = (sw > 0.0) ? sq[a] / sw : lat_q(p, a, k0[a]) + dq[a];
  index_pos(p, Q, s);
  out[site] = spline4<FT>(p, C, s);
}

// ------------------------------------------------------------- the field

// rho(i, j) = du dw sum over velocity blocks (in order) of the partials.
__global__ __launch_bounds__(256) void k4_rho(KP p, const double *__restrict__ part,
                                              double *__restrict__ rho) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int n2 = p.ns * p.ns;
  if (q >= n2) return;
  const int nvb = p.nb[2] * p.nb[3];
  double s = 0.0;
  for (int v = 0; v < nvb; ++v) s += part[(size_t)v * n2 + q];
  rho[q] = (p.du * p.du) * s;
}

// Discrete Fourier transform of Poisson's equation on the periodic square
// (the sums in index order; tw = cos, sin of 2 pi m / ns).  Forward along
// x: R1[j][p] = sum_i rho[j][i] e^{-2 pi i p i / ns}.
__global__ __launch_bounds__(256) void k4_dft_x(KP p, const double *__restrict__ rho,
                                                const double *__restrict__ tw,
                                                double *__restrict__ re,
                                                double *__restrict__ im) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = p.ns;
  if (q >= n * n) return;
  const int j = q / n, pf = q - j * n;
  const double *cs = tw, *sn = tw + n;
  double sr = 0.0, si = 0.0;
  for (int i = 0; i < n; ++i) {
    const int m = (int)(((long long)pf * i) % n);
    const double v = rho[(size_t)j * n + i];
    sr = fma(v, cs[m], sr);
    si = fma(-v, sn[m], si);
  }
  re[q] = sr;
  im[q] = si;
}

// Forward along y: R2[q][p] = sum_j R1[j][p] e^{-2 pi i q j / ns}; then the
// spectra of a_x and a_y: phi^ = -2 G rho^ / |k|^2, a^ = -i k phi^ (k = 0
// and the Nyquist derivative zero).  ar/ai hold [2][ns^2].
__global__ __launch_bounds__(256) void k4_dft_y_spec(
    KP p, const double *__restrict__ re, const double *__restrict__ im,
    const double *__restrict__ tw, double *__restrict__ ar,
    double *__restrict__ ai) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = p.ns;
  if (o >= n * n) return;
  const int qy = o / n, pf = o - qy * n;
  const double *cs = tw, *sn = tw + n;
  double sr = 0.0, si = 0.0;
  for (int j = 0; j < n; ++j) {
    const int m = (int)(((long long)qy * j) % n);
    const double a = re[(size_t)j * n + pf], b = im[(size_t)j * n + pf];
    sr = fma(a, cs[m], fma(b, sn[m], sr));
    si = fma(b, cs[m], fma(-a, sn[m], si));
  }
  const double twopi = 6.283185307179586476925286766559;
  const int half = (n % 2 == 0) ? n / 2 - 1 : n / 2;
  const int pp = (pf <= half) ? pf : pf - n, qq = (qy <= half) ? qy : qy - n;
  const double kx = twopi * (double)pp / p.L, ky = twopi * (double)qq / p.L;
  const double k2 = kx * kx + ky * ky;
  const size_t n2 = (size_t)n * n;
  for (int comp = 0; comp < 2; ++comp) {
    if (pf == 0 && qy == 0) {
      ar[comp * n2 + o] = 0.0;
      ai[comp * n2 + o] = 0.0;
      continue;
    }
    double kd = comp == 0 ? kx : ky;
    if ((comp == 0 ? pf : qy) * 2 == n) kd = 0.0;
    const double gk = (-2.0 * p.G) / k2;
    const double pr = gk * sr, pi = gk * si;
    ar[comp * n2 + o] = kd * pi;
    ai[comp * n2 + o] = -(kd * pr);
  }
}

// Inverse along y for both components: T[c][j][p] = sum_q a^[c][q][p]
// e^{+2 pi i q j / ns}.
__global__ __launch_bounds__(256) void k4_idft_y(KP p, const double *__restrict__ ar,
                                                 const double *__restrict__ ai,
                                                 const double *__restrict__ tw,
                                                 double *__restrict__ tr,
                                                 double *__restrict__ ti) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = p.ns;
  const size_t n2 = (size_t)n * n;
  if (o >= 2 * n * n) return;
  const int comp = o / (n * n), r = o - comp * n * n;
  const int j = r / n, pf = r - j * n;
  const double *cs = tw, *sn = tw + n;
  double sr = 0.0, si = 0.0;
  for (int qy = 0; qy < n; ++qy) {
    const int m = (int)(((long long)qy * j) % n);
    const double a = ar[comp * n2 + (size_t)qy * n + pf];
    const double b = ai[comp * n2 + (size_t)qy * n + pf];
    sr = fma(a, cs[m], fma(-b, sn[m], sr));
    si = fma(b, cs[m], fma(a, sn[m], si));
  }
  tr[comp * n2 + r] = sr;
  ti[comp * n2 + r] = si;
}

// Inverse along x, real part / ns^2: fields 0 (a_x) and 1 (a_y).
__global__ __launch_bounds__(256) void k4_idft_x(KP p, const double *__restrict__ tr,
                                                 const double *__restrict__ ti,
                                                 const double *__restrict__ tw,
                                                 double *__restrict__ fld) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = p.ns;
  const size_t n2 = (size_t)n * n;
  if (o >= 2 * n * n) return;
  const int comp = o / (n * n), r = o - comp * n * n;
  const int j = r / n, i = r - j * n;
  const double *cs = tw, *sn = tw + n;
  double sr = 0.0;
  for (int pf = 0; pf < n; ++pf) {
    const int m = (int)(((long long)pf * i) % n);
    const double a = tr[comp * n2 + (size_t)j * n + pf];
    const double b = ti[comp * n2 + (size_t)j * n + pf];
    sr = fma(a, cs[m], fma(-b, sn[m], sr));
  }
  fld[comp * n2 + r] = sr * (1.0 / ((double)n * (double)n));
}

// Centred differences of a (periodic): fields 2-5 = d a_x/dx, d a_x/dy,
// d a_y/dx, d a_y/dy; 6-8 = a_x,xx a_x,xy a_x,yy; 9-11 the same of a_y.
__global__ __launch_bounds__(256) void k4_fd(KP p, double *__restrict__ fld) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = p.ns;
  const size_t n2 = (size_t)n * n;
  if (o >= n * n) return;
  const int j = o / n, i = o - j * n;
  const int ip = (i + 1) % n, im = (i + n - 1) % n;
  const int jp = (j + 1) % n, jm = (j + n - 1) % n;
  const double dx = p.dx;
  for (int c = 0; c < 2; ++c) {
    const double *A = fld + c * n2;
    auto at = [&](int ii, int jj) { return A[(size_t)jj * n + ii]; };
    fld[(2 + 2 * c) * n2 + o] = (at(ip, j) - at(im, j)) / (2.0 * dx);
    fld[(3 + 2 * c) * n2 + o] = (at(i, jp) - at(i, jm)) / (2.0 * dx);
    fld[(6 + 3 * c) * n2 + o] = ((at(ip, j) + at(im, j)) - 2.0 * at(i, j)) / (dx * dx);
    fld[(7 + 3 * c) * n2 + o] =
        (((at(ip, jp) - at(ip, jm)) - at(im, jp)) + at(im, jm)) / (4.0 * (dx * dx));
    fld[(8 + 3 * c) * n2 + o] = ((at(i, jp) + at(i, jm)) - 2.0 * at(i, j)) / (dx * dx);
  }
}

// 3 x 3 dual TSC of the 12 fields at (x, y).
__device__ __forceinline__ void tsc12(const KP &p, const double *__restrict__ fld,
                                      double x, double y, double v[12]) {
  const int n = p.ns;
  const size_t n2 = (size_t)n * n;
  double u[2] = {x * p.inv_dx - 0.5, y * p.inv_dx - 0.5};
  int i0[2];
  double w[2][3];
  for (int a = 0; a < 2; ++a) {
    if (!(u[a] >= -3.0)) u[a] = -3.0;
    if (u[a] > (double)n + 2.0) u[a] = (double)n + 2.0;
    const double fi = floor(u[a] + 0.5), d = u[a] - fi;
    const double tm = 0.5 - d, tp = 0.5 + d;
    i0[a] = (int)fi;
    w[a][0] = 0.5 * (tm * tm);
    w[a][1] = 0.75 - d * d;
    w[a][2] = 0.5 * (tp * tp);
  }
  int ix[3], jy[3];
  for (int q = 0; q < 3; ++q) {
    ix[q] = (((i0[0] - 1 + q) % n) + n) % n;
    jy[q] = (((i0[1] - 1 + q) % n) + n) % n;
  }
  for (int k = 0; k < 12; ++k) {
    const double *A = fld + k * n2;
    double row[3];
    for (int b = 0; b < 3; ++b) {
      const double *R = A + (size_t)jy[b] * n;
      row[b] = fma(w[0][2], R[ix[2]], fma(w[0][1], R[ix[1]], w[0][0] * R[ix[0]]));
    }
    v[k] = fma(w[1][2], row[2], fma(w[1][1], row[1], w[1][0] * row[0]));
  }
}

// Kick over dt (section 2.4 per space axis, reading R5: the right-hand
// sides use the half-step T and H of the space rows), then the corrector
// drift over dt/2.
__global__ __launch_bounds__(256) void k4_kick(KP p, double *__restrict__ st,
                                               const double *__restrict__ fld) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.E) return;
  const size_t E = (size_t)p.E;
  double s[NST];
#pragma unroll
  for (int q = 0; q < NST; ++q) s[q] = st[q * E + e];
  double fv[12];
  tsc12(p, fld, s[S_P], s[S_P + 1], fv);
  const double dt = p.dt;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double a = fv[i], g0 = fv[2 + 2 * i], g1 = fv[3 + 2 * i];
    const double h00 = fv[6 + 3 * i], h01 = fv[7 + 3 * i], h11 = fv[8 + 3 * i];
    s[S_P + 2 + i] = fma(dt, a, s[S_P + 2 + i]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double v = fma(g1, s[S_T + 4 + j], g0 * s[S_T + j]);
      s[S_T + 4 * (2 + i) + j] = fma(dt, v, s[S_T + 4 * (2 + i) + j]);
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const int jb = PB[q], kc = PC[q];
      const double t0j = s[S_T + jb], t1j = s[S_T + 4 + jb];
      const double t0k = s[S_T + kc], t1k = s[S_T + 4 + kc];
      double v = g0 * s[S_H + q];
      v = fma(g1, s[S_H + 10 + q], v);
      v = fma(h00, t0j * t0k, v);
      v = fma(h01, fma(t0j, t1k, t1j * t0k), v);
      v = fma(h11, t1j * t1k, v);
      s[S_H + 10 * (2 + i) + q] = fma(dt, v, s[S_H + 10 * (2 + i) + q]);
    }
  }
  drift4(p, s, p.h);
#pragma unroll
  for (int q = 0; q < NST; ++q) st[q * E + e] = s[q];
}

// ------------------------------------------------------------- the spline

// One thread per line along axis `ax` (0 x, 1 y, 2 u, 3 w): the tridiagonal
// (1, 4, 1) solve with precomputed pivots -- mirror end rows (4, 2) / (2, 4)
// on u and w, the cyclic system's tridiagonal part plus the Sherman-
// Morrison correction y - [(y_0 - y_{n-1}/4) / den] z on x and y.
// tab: cp[n], ri[n] (and z[n], den on the periodic axes).
template <typename FT>
__global__ __launch_bounds__(256) void k4_fit(KP p, FT *__restrict__ C, int ax,
                                              const FT *__restrict__ tab) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ns = p.ns, nv = p.nv;
  const long long N4 = ns * ns * nv * nv;
  const int n = ax < 2 ? p.ns : p.nv;
  const long long stride = ax == 0 ? 1 : ax == 1 ? ns : ax == 2 ? ns * ns : ns * ns * nv;
  if (q >= N4 / n) return;
  const long long low = q % stride, high = q / stride;
  FT *x = C + high * stride * n + low;
  const FT *cp = tab, *ri = tab + n;
  const bool per = ax < 2;
  FT acc = (FT)0;
  for (int i = 0; i < n; ++i) {
    const FT sub = (!per && i == n - 1) ? (FT)2 : (FT)1;
    acc = ((FT)6 * x[i * stride] - sub * acc) * ri[i];
    x[i * stride] = acc;
  }
  for (int i = n - 2; i >= 0; --i) {
    acc = x[i * stride] - cp[i] * acc;
    x[i * stride] = acc;
  }
  if (per) {
    const FT *z = tab + 2 * n, den = tab[3 * n];
    const FT fact = (x[0] - (FT)0.25 * x[(long long)(n - 1) * stride]) / den;
    for (int i = 0; i < n; ++i) x[i * stride] = x[i * stride] - fact * z[i];
  }
}

// f0 (device doubles) -> F, u and w edge rows zero.
template <typename FT>
__global__ __launch_bounds__(256) void k4_load(KP p, const double *__restrict__ src,
                                               FT *__restrict__ F) {
  const long long N4 = (long long)p.ns * p.ns * p.nv * p.nv;
  const long long gsz = (long long)gridDim.x * blockDim.x;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N4;
       q += gsz) {
    const long long r = q / ((long long)p.ns * p.ns);
    const int k = (int)(r % p.nv), l = (int)(r / p.nv);
    const bool edge = k == 0 || k == p.nv - 1 || l == 0 || l == p.nv - 1;
    F[q] = edge ? (FT)0 : (FT)src[q];
  }
}

// ------------------------------------------------------------ diagnostics

// Per-workgroup partial sums of f, (u^2 + w^2) f and f ln|f| over a range
// of sites (tree order within the workgroup).
template <typename FT>
__global__ __launch_bounds__(256) void k4_diag_part(KP p, const FT *__restrict__ f,
                                                    double *__restrict__ part) {
  __shared__ double s0[256], s1[256], s2[256];
  const long long N4 = (long long)p.ns * p.ns * p.nv * p.nv;
  const long long gsz = (long long)gridDim.x * blockDim.x;
  double m = 0.0, k = 0.0, en = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < N4;
       q += gsz) {
    const long long r = q / ((long long)p.ns * p.ns);
    const double u = coord(p, 2, (int)(r % p.nv)), w = coord(p, 3, (int)(r / p.nv));
    const double v = (double)f[q];
    m += v;
    k += (u * u + w * w) * v;
    if (v != 0.0) en += v * log(fabs(v));
  }
  const int t = threadIdx.x;
  s0[t] = m;
  s1[t] = k;
  s2[t] = en;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      s0[t] += s0[t + s];
      s1[t] += s1[t + s];
      s2[t] += s2[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[3 * blockIdx.x] = s0[0];
    part[3 * blockIdx.x + 1] = s1[0];
    part[3 * blockIdx.x + 2] = s2[0];
  }
}

__global__ __launch_bounds__(256) void k4_diag_final(KP p,
                                                     const double *__restrict__ part,
                                                     int nparts,
                                                     const double *__restrict__ fld,
                                                     double *__restrict__ out) {
  __shared__ double s3[256];
  const int t = threadIdx.x;
  const int n2 = p.ns * p.ns;
  double pot = 0.0;
  for (int q = t; q < n2; q += 256) pot += fld[q] * fld[q] + fld[n2 + q] * fld[n2 + q];
  s3[t] = pot;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) s3[t] += s3[t + s];
    __syncthreads();
  }
  if (t == 0) {
    double m = 0.0, k = 0.0, en = 0.0;
    for (int q = 0; q < nparts; ++q) {
      m += part[3 * q];
      k += part[3 * q + 1];
      en += part[3 * q + 2];
    }
    const double dV = (p.dx * p.dx) * (p.du * p.du);
    out[0] = m * dV;
    out[1] = 0.5 * k * dV;
    out[2] = (p.G != 0.0) ? -s3[0] * (p.dx * p.dx) / (4.0 * p.G) : 0.0;
    out[3] = out[1] + out[2];
    out[4] = -en * dV;
  }
}

}  // namespace vp4k
