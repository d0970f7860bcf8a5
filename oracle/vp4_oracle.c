/*
 * vp4_oracle.c -- plain CPU FP64 oracle of the metric semi-Lagrangian
 * method in 4D phase space (x, y, u, w) with 2D periodic space: the
 * generalisation the paper sketches for higher dimensions (section 2.1: 60
 * numbers per element; section 2.2.1: the 15-point second-order
 * interpolation; section 2.5: FFT Poisson solve for periodic systems).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  Plain loops, one rounding per operation
 * (fma() only where written), every reduction in the order written.  It
 * shares no code with the HIP engine.  Build: gcc -O2 -ffp-contract=off.
 *
 * Readings (listed in the repository's design notes as R24): the force is
 * div a = -2 G (rho - rho_bar) on the periodic square (the 1D convention of
 * eq. acccomp carried to two dimensions), solved by a discrete Fourier
 * transform; its gradient and Hessian by centred finite differences of a;
 * the element force by the 3 x 3 dual TSC; the remap neighbours follow the
 * 2D beta rule axis by axis, dropping every neighbour offset in more than
 * one axis when an axis needs three.
 */
#include "vp4_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NST 60
enum { P0 = 0, T0 = 4, H0 = 20 };

struct or4_ctx {
  or4_params p;
  int ns, nv, ms, mv, E;
  long long N4;
  double dx, du, inv_dx, inv_du;
  double Dm[4], rD[4];          /* element spacing per axis, reciprocal */
  double *F, *C, *f;            /* [N4] */
  double *el;                   /* [60][E] */
  double *A;                    /* [16][E], A = T^-1 */
  double *rho, *fld;            /* [ns^2], [12][ns^2] */
  int *bstart, *bitem;
  int bn[4];
  double bw[4];
  double t;
  int64_t step;
  int ready;
};

#define EL(c, k, e) ((c)->el[(size_t)(k) * (size_t)(c)->E + (size_t)(e)])
#define AM(c, k, e) ((c)->A[(size_t)(k) * (size_t)(c)->E + (size_t)(e)])

/* symmetric pair index of (b, c), b <= c, in the order 00 01 02 03 11 12 13
 * 22 23 33 */
static const int PB[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
static const int PC[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

static double coord(const or4_ctx *c, int a, int i) {
  if (a < 2) return ((double)i + 0.5) * c->dx;
  return -c->p.vmax + ((double)i + 0.5) * c->du;
}
static int spacing(const or4_ctx *c, int a) {
  return a < 2 ? c->p.ss : c->p.sv;
}
static int lat_n(const or4_ctx *c, int a) { return a < 2 ? c->ms : c->mv; }
static void lat_index(const or4_ctx *c, int e, int k[4]) {
  k[0] = e % c->ms;
  e /= c->ms;
  k[1] = e % c->ms;
  e /= c->ms;
  k[2] = e % c->mv;
  k[3] = e / c->mv;
}
static double lat_q(const or4_ctx *c, int a, int k) {
  int s = spacing(c, a);
  return coord(c, a, s * k + s / 2);
}

/* Periodic space: one period at most per drift (as in the 1D variant). */
static double wrap_L(const or4_ctx *c, double x) {
  double L = c->p.L;
  if (x < 0.0) {
    x = x + L;
    if (x >= L) x = 0.0;
  } else if (x >= L) {
    x = x - L;
    if (x < 0.0) x = 0.0;
  }
  return x;
}
static double image(double d, double L) {
  double hL = 0.5 * L;
  if (d > hL) return d - L;
  if (d < -hL) return d + L;
  return d;
}

static void reset_elements(or4_ctx *c) {
  for (int e = 0; e < c->E; ++e) {
    int k[4];
    lat_index(c, e, k);
    for (int s = 0; s < NST; ++s) EL(c, s, e) = 0.0;
    for (int a = 0; a < 4; ++a) {
      EL(c, P0 + a, e) = lat_q(c, a, k[a]);
      EL(c, T0 + 5 * a, e) = 1.0;
    }
  }
}

/* Drift over h (section 2.4 in 2D space): x_i += h v_i, T_i. += h T_{i+2}.,
 * H_i.. += h H_{i+2}.., then the positions re-enter the periodic square. */
static void drift(or4_ctx *c, double h) {
  for (int e = 0; e < c->E; ++e) {
    for (int i = 0; i < 2; ++i) {
      EL(c, P0 + i, e) = wrap_L(c, fma(h, EL(c, P0 + i + 2, e), EL(c, P0 + i, e)));
      for (int j = 0; j < 4; ++j)
        EL(c, T0 + 4 * i + j, e) =
            fma(h, EL(c, T0 + 4 * (i + 2) + j, e), EL(c, T0 + 4 * i + j, e));
      for (int q = 0; q < 10; ++q)
        EL(c, H0 + 10 * i + q, e) =
            fma(h, EL(c, H0 + 10 * (i + 2) + q, e), EL(c, H0 + 10 * i + q, e));
    }
  }
}

/* A = T^-1 by the adjugate (2 x 2 minors of the top and bottom row pairs);
 * det T must stay positive (it is 1 for the exact flow). */
static int inverse4(const double *m, double *inv, double *det_out) {
  double s0 = m[0] * m[5] - m[4] * m[1];
  double s1 = m[0] * m[6] - m[4] * m[2];
  double s2 = m[0] * m[7] - m[4] * m[3];
  double s3 = m[1] * m[6] - m[5] * m[2];
  double s4 = m[1] * m[7] - m[5] * m[3];
  double s5 = m[2] * m[7] - m[6] * m[3];
  double c5 = m[10] * m[15] - m[14] * m[11];
  double c4 = m[9] * m[15] - m[13] * m[11];
  double c3 = m[9] * m[14] - m[13] * m[10];
  double c2 = m[8] * m[15] - m[12] * m[11];
  double c1 = m[8] * m[14] - m[12] * m[10];
  double c0 = m[8] * m[13] - m[12] * m[9];
  double det = ((((s0 * c5 - s1 * c4) + s2 * c3) + s3 * c2) - s4 * c1) + s5 * c0;
  *det_out = det;
  if (!(det > 0.0) || !isfinite(det)) return 0;
  double r = 1.0 / det;
  inv[0] = ((m[5] * c5 - m[6] * c4) + m[7] * c3) * r;
  inv[1] = ((-m[1] * c5 + m[2] * c4) - m[3] * c3) * r;
  inv[2] = ((m[13] * s5 - m[14] * s4) + m[15] * s3) * r;
  inv[3] = ((-m[9] * s5 + m[10] * s4) - m[11] * s3) * r;
  inv[4] = ((-m[4] * c5 + m[6] * c2) - m[7] * c1) * r;
  inv[5] = ((m[0] * c5 - m[2] * c2) + m[3] * c1) * r;
  inv[6] = ((-m[12] * s5 + m[14] * s2) - m[15] * s1) * r;
  inv[7] = ((m[8] * s5 - m[10] * s2) + m[11] * s1) * r;
  inv[8] = ((m[4] * c4 - m[5] * c2) + m[7] * c0) * r;
  inv[9] = ((-m[0] * c4 + m[1] * c2) - m[3] * c0) * r;
  inv[10] = ((m[12] * s4 - m[13] * s2) + m[15] * s0) * r;
  inv[11] = ((-m[8] * s4 + m[9] * s2) - m[11] * s0) * r;
  inv[12] = ((-m[4] * c3 + m[5] * c1) - m[6] * c0) * r;
  inv[13] = ((m[0] * c3 - m[1] * c1) + m[2] * c0) * r;
  inv[14] = ((-m[12] * s3 + m[13] * s1) - m[14] * s0) * r;
  inv[15] = ((m[8] * s3 - m[9] * s1) + m[10] * s0) * r;
  return 1;
}

static int precompute(or4_ctx *c) {
  for (int e = 0; e < c->E; ++e) {
    double m[16], inv[16], det;
    for (int q = 0; q < 16; ++q) m[q] = EL(c, T0 + q, e);
    for (int a = 0; a < 4; ++a)
      if (!isfinite(EL(c, P0 + a, e))) return -5;
    if (!inverse4(m, inv, &det)) return -5;
    for (int q = 0; q < 16; ++q) AM(c, q, e) = inv[q];
  }
  return 0;
}

/* Second-order inverse map (eq. QofP in four dimensions): l = A dP with
 * the nearest periodic image in x and y, u_a = l^T H_a l over the ten
 * symmetric pairs, dQ = l - A u / 2; valid when every |l_a| < Dm_a. */
static int inv_map4(const double *X, const double *A, const double *H,
                    const double *Dm, double L, const double *P, double *dq) {
  double d[4], l[4], u[4];
  d[0] = image(P[0] - X[0], L);
  d[1] = image(P[1] - X[1], L);
  d[2] = P[2] - X[2];
  d[3] = P[3] - X[3];
  int valid = 1;
  for (int a = 0; a < 4; ++a) {
    const double *r = A + 4 * a;
    l[a] = fma(r[3], d[3], fma(r[2], d[2], fma(r[1], d[1], r[0] * d[0])));
    if (!(fabs(l[a]) < Dm[a])) valid = 0;
  }
  for (int a = 0; a < 4; ++a) {
    const double *h = H + 10 * a;
    double s = h[0] * (l[0] * l[0]);
    for (int q = 1; q < 10; ++q) {
      double w = (PB[q] == PC[q]) ? h[q] : 2.0 * h[q];
      s = fma(w, l[PB[q]] * l[PC[q]], s);
    }
    u[a] = s;
  }
  for (int a = 0; a < 4; ++a) {
    const double *r = A + 4 * a;
    double s = l[a];
    for (int b = 0; b < 4; ++b) s = fma(-0.5 * r[b], u[b], s);
    dq[a] = s;
  }
  return valid;
}

static int elem_map(const or4_ctx *c, int e, const double *P, double *dq) {
  double X[4], A[16], H[40];
  for (int a = 0; a < 4; ++a) X[a] = EL(c, P0 + a, e);
  for (int q = 0; q < 16; ++q) A[q] = AM(c, q, e);
  for (int q = 0; q < 40; ++q) H[q] = EL(c, H0 + q, e);
  return inv_map4(X, A, H, c->Dm, c->p.L, P, dq);
}

static double dist2(const or4_ctx *c, const double *dq) {
  double z0 = dq[0] * c->rD[0], z1 = dq[1] * c->rD[1];
  double z2 = dq[2] * c->rD[2], z3 = dq[3] * c->rD[3];
  return fma(z3, z3, fma(z2, z2, fma(z1, z1, z0 * z0)));
}

/* -------------------------------------------------------------- the query */

static int query_brute(const or4_ctx *c, const double *P, double *bdq) {
  int best = -1;
  double bd = INFINITY;
  for (int e = 0; e < c->E; ++e) {
    double dq[4];
    if (!elem_map(c, e, P, dq)) continue;
    double d2 = dist2(c, dq);
    if (d2 < bd) {
      bd = d2;
      best = e;
      memcpy(bdq, dq, sizeof(dq));
    }
  }
  return best;
}

/* Bucket grid: buckets at least as wide as the largest Eulerian reach
 * sum_b |T_ab| Dm_b of any element, equal buckets on the periodic axes;
 * every valid element of a site lies in the 3^4 buckets around it. */
static int build_buckets(or4_ctx *c) {
  double R[4] = {0, 0, 0, 0};
  for (int e = 0; e < c->E; ++e)
    for (int a = 0; a < 4; ++a) {
      double r = 0.0;
      for (int b = 0; b < 4; ++b) r += fabs(EL(c, T0 + 4 * a + b, e)) * c->Dm[b];
      if (r > R[a]) R[a] = r;
    }
  double ext[4] = {c->p.L, c->p.L, 2.0 * c->p.vmax, 2.0 * c->p.vmax};
  long long nb = 1;
  for (int a = 0; a < 4; ++a) {
    double w = R[a] * (1.0 + 0x1p-20) + 0x1p-30 * ext[a];
    if (w < ext[a] / 64.0) w = ext[a] / 64.0;
    int n;
    if (a < 2) {
      n = (int)floor(ext[a] / w);
      if (n < 1) n = 1;
      w = ext[a] / n;
    } else {
      n = (int)ceil(ext[a] / w);
      if (n < 1) n = 1;
    }
    c->bn[a] = n;
    c->bw[a] = w;
    nb *= n;
  }
  free(c->bstart);
  c->bstart = (int *)calloc((size_t)nb + 1, sizeof(int));
  int *bid = (int *)malloc(sizeof(int) * (size_t)c->E);
  int *fill = (int *)malloc(sizeof(int) * (size_t)nb);
  if (!c->bstart || !bid || !fill) {
    free(bid);
    free(fill);
    return -2;
  }
  for (int e = 0; e < c->E; ++e) {
    long long b = 0;
    for (int a = 3; a >= 0; --a) {
      double lo = a < 2 ? 0.0 : -c->p.vmax;
      int k = (int)floor((EL(c, P0 + a, e) - lo) / c->bw[a]);
      if (k < 0) k = 0;
      if (k > c->bn[a] - 1) k = c->bn[a] - 1;
      b = b * c->bn[a] + k;
    }
    bid[e] = (int)b;
    c->bstart[b + 1] += 1;
  }
  for (long long b = 0; b < nb; ++b) c->bstart[b + 1] += c->bstart[b];
  memcpy(fill, c->bstart, sizeof(int) * (size_t)nb);
  for (int e = 0; e < c->E; ++e) c->bitem[fill[bid[e]]++] = e;
  free(fill);
  free(bid);
  return 0;
}

static int query_bucketed(const or4_ctx *c, const double *P, double *bdq) {
  int lo[4], hi[4], k0[4];
  for (int a = 0; a < 4; ++a) {
    double o = a < 2 ? 0.0 : -c->p.vmax;
    int k = (int)floor((P[a] - o) / c->bw[a]);
    if (k < 0) k = 0;
    if (k > c->bn[a] - 1) k = c->bn[a] - 1;
    k0[a] = k;
    lo[a] = k - 1;
    hi[a] = k + 1;
    if (a < 2 && c->bn[a] < 3) {
      lo[a] = 0;
      hi[a] = c->bn[a] - 1;
    }
  }
  (void)k0;
  int best = -1;
  double bd = INFINITY;
  int kk[4];
  for (kk[3] = lo[3]; kk[3] <= hi[3]; ++kk[3])
    for (kk[2] = lo[2]; kk[2] <= hi[2]; ++kk[2])
      for (kk[1] = lo[1]; kk[1] <= hi[1]; ++kk[1])
        for (kk[0] = lo[0]; kk[0] <= hi[0]; ++kk[0]) {
          long long b = 0;
          int skip = 0;
          for (int a = 3; a >= 0; --a) {
            int k = kk[a];
            if (a < 2) k = ((k % c->bn[a]) + c->bn[a]) % c->bn[a];
            if (k < 0 || k >= c->bn[a]) skip = 1;
            b = b * c->bn[a] + k;
          }
          if (skip) continue;
          for (int q = c->bstart[b]; q < c->bstart[b + 1]; ++q) {
            int e = c->bitem[q];
            double dq[4];
            if (!elem_map(c, e, P, dq)) continue;
            double d2 = dist2(c, dq);
            if (d2 < bd || (d2 == bd && e < best)) {
              bd = d2;
              best = e;
              memcpy(bdq, dq, sizeof(dq));
            }
          }
        }
  return best;
}

/* ------------------------------------------------------- interpolations */

static double Fat4(const double *F, int ns, int nv, const int *g) {
  int i = ((g[0] % ns) + ns) % ns, j = ((g[1] % ns) + ns) % ns;
  if (g[2] < 0 || g[2] >= nv || g[3] < 0 || g[3] >= nv) return 0.0;
  return F[(((size_t)g[3] * nv + g[2]) * ns + j) * ns + i];
}

/* 15-point second-order interpolation (section 2.2.1 in four dimensions):
 * the nearest node n, its 8 axis neighbours, and for each of the 6 axis
 * pairs the corner that closes the square around Q's projection, with the
 * Lagrange signs of reading R10.  s4 is the index-space position; x and y
 * are periodic (positions clamped to [-12, ns + 11]), u and w are zero
 * outside the grid. */
double or4_int15(const double *F, int ns, int nv, const double *s4) {
  double s[4];
  for (int a = 0; a < 4; ++a) s[a] = s4[a];
  for (int a = 0; a < 2; ++a) {
    if (s[a] < -12.0) s[a] = -12.0;
    if (s[a] > (double)ns + 11.0) s[a] = (double)ns + 11.0;
  }
  for (int a = 2; a < 4; ++a)
    if (!(s[a] > -4.0 && s[a] < nv + 3.0)) return 0.0;
  int n[4], cf[4];
  double dq[4];
  for (int a = 0; a < 4; ++a) {
    double fn = floor(s[a] + 0.5);
    n[a] = (int)fn;
    cf[a] = (int)floor(s[a]);
    dq[a] = s[a] - fn;
  }
  double w0 = 1.0 - dq[0] * dq[0];
  for (int a = 1; a < 4; ++a) w0 = w0 - dq[a] * dq[a];
  double f = Fat4(F, ns, nv, n) * w0;
  for (int a = 0; a < 4; ++a) {
    double h = 0.5 * dq[a];
    double wp = h * (1.0 + dq[a]), wm = h * (1.0 - dq[a]);
    int g[4];
    memcpy(g, n, sizeof(g));
    g[a] = n[a] + 1;
    f = fma(Fat4(F, ns, nv, g), wp, f);
    g[a] = n[a] - 1;
    f = fma(-Fat4(F, ns, nv, g), wm, f);
  }
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b) {
      int g[4];
      memcpy(g, n, sizeof(g));
      g[a] = cf[a] + 1;
      g[b] = cf[b] + 1;
      double f11 = Fat4(F, ns, nv, g);
      g[a] = cf[a];
      g[b] = cf[b];
      double f00 = Fat4(F, ns, nv, g);
      g[a] = cf[a] + 1;
      double f10 = Fat4(F, ns, nv, g);
      g[a] = cf[a];
      g[b] = cf[b] + 1;
      double f01 = Fat4(F, ns, nv, g);
      double cross = ((f11 + f00) - f10) - f01;
      f = fma(cross, dq[a] * dq[b], f);
    }
  return f;
}

/* Cubic B-spline along one line: cyclic (1, 4, 1) system by Sherman-
 * Morrison (periodic axes, as in the 1D periodic variant) or the mirror
 * end rows (4, 2) / (2, 4) (velocity axes, section 2.2.2). */
static void thomas_rows(int n, const double *b, const double *sub_last,
                        const double *rhs, double *out, double *cp, double *dp,
                        double sup0) {
  double rinv = 1.0 / b[0];
  cp[0] = sup0 * rinv;
  dp[0] = rhs[0] * rinv;
  for (int i = 1; i < n; ++i) {
    double sub = (i == n - 1) ? *sub_last : 1.0;
    double den = b[i] - sub * cp[i - 1];
    rinv = 1.0 / den;
    cp[i] = rinv;
    dp[i] = (rhs[i] - sub * dp[i - 1]) * rinv;
  }
  out[n - 1] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) out[i] = dp[i] - cp[i] * out[i + 1];
}

static void fit_line(int n, int periodic, double *x, double *work) {
  double *b = work, *r = work + n, *y = work + 2 * n, *z = work + 3 * n,
         *u = work + 4 * n, *cp = work + 5 * n, *dp = work + 6 * n;
  for (int i = 0; i < n; ++i) r[i] = 6.0 * x[i];
  if (periodic) {
    double one = 1.0;
    for (int i = 0; i < n; ++i) {
      b[i] = 4.0;
      u[i] = 0.0;
    }
    b[0] = 8.0;
    b[n - 1] = 4.25;
    u[0] = -4.0;
    u[n - 1] = 1.0;
    thomas_rows(n, b, &one, r, y, cp, dp, 1.0);
    thomas_rows(n, b, &one, u, z, cp, dp, 1.0);
    double fact = (y[0] - 0.25 * y[n - 1]) / ((1.0 + z[0]) - 0.25 * z[n - 1]);
    for (int i = 0; i < n; ++i) x[i] = y[i] - fact * z[i];
  } else {
    double two = 2.0;
    for (int i = 0; i < n; ++i) b[i] = 4.0;
    thomas_rows(n, b, &two, r, y, cp, dp, 2.0);
    for (int i = 0; i < n; ++i) x[i] = y[i];
  }
}

int or4_spline_fit(int ns, int nv, const double *F, double *C) {
  if (ns < 3 || nv < 2) return -1;
  size_t N4 = (size_t)ns * ns * nv * nv;
  int nmax = ns > nv ? ns : nv;
  double *line = (double *)malloc(sizeof(double) * nmax);
  double *work = (double *)malloc(sizeof(double) * 7 * nmax);
  if (!line || !work) {
    free(line);
    free(work);
    return -2;
  }
  memcpy(C, F, sizeof(double) * N4);
  size_t stride[4] = {1, (size_t)ns, (size_t)ns * ns, (size_t)ns * ns * nv};
  int len[4] = {ns, ns, nv, nv};
  for (int a = 0; a < 4; ++a) {
    /* every line along axis a, in increasing order of its start offset */
    size_t nlines = N4 / len[a];
    for (size_t q = 0; q < nlines; ++q) {
      size_t lowp = q % stride[a], high = q / stride[a];
      size_t base = high * stride[a] * len[a] + lowp;
      for (int i = 0; i < len[a]; ++i) line[i] = C[base + i * stride[a]];
      fit_line(len[a], a < 2, line, work);
      for (int i = 0; i < len[a]; ++i) C[base + i * stride[a]] = line[i];
    }
  }
  free(line);
  free(work);
  return 0;
}

static void bspline_w(double u, double b[4]) {
  const double sixth = 1.0 / 6.0;
  double t = 1.0 - u;
  double u2 = u * u, u3 = u2 * u;
  b[0] = ((t * t) * t) * sixth;
  b[1] = ((3.0 * u3 - 6.0 * u2) + 4.0) * sixth;
  b[2] = (((-3.0 * u3 + 3.0 * u2) + 3.0 * u) + 1.0) * sixth;
  b[3] = u3 * sixth;
}

static double Cat4(const double *C, int ns, int nv, const int *g) {
  int i = ((g[0] % ns) + ns) % ns, j = ((g[1] % ns) + ns) % ns;
  int k = g[2], l = g[3];
  if (k < 0) k = -k;
  if (k > nv - 1) k = 2 * (nv - 1) - k;
  if (l < 0) l = -l;
  if (l > nv - 1) l = 2 * (nv - 1) - l;
  return C[(((size_t)l * nv + k) * ns + j) * ns + i];
}

/* Tensor cubic B-spline at index-space s4: x, y periodic (clamped to
 * [-12, ns + 11]), u, w on [0, nv - 1] with mirror ghosts, 0 outside. */
double or4_spline_eval(const double *C, int ns, int nv, const double *s4) {
  double s[4];
  int i0[4];
  double bw[4][4];
  for (int a = 0; a < 4; ++a) s[a] = s4[a];
  for (int a = 0; a < 2; ++a) {
    if (s[a] < -12.0) s[a] = -12.0;
    if (s[a] > (double)ns + 11.0) s[a] = (double)ns + 11.0;
  }
  for (int a = 2; a < 4; ++a)
    if (!(s[a] >= 0.0 && s[a] <= (double)(nv - 1))) return 0.0;
  for (int a = 0; a < 4; ++a) {
    int i = (int)floor(s[a]);
    if (a >= 2 && i > nv - 2) i = nv - 2;
    i0[a] = i;
    bspline_w(s[a] - (double)i, bw[a]);
  }
  double f = 0.0;
  int g[4];
  for (int l = 0; l < 4; ++l) {
    double fu = 0.0;
    for (int k = 0; k < 4; ++k) {
      double fy = 0.0;
      for (int j = 0; j < 4; ++j) {
        g[1] = i0[1] - 1 + j;
        g[2] = i0[2] - 1 + k;
        g[3] = i0[3] - 1 + l;
        g[0] = i0[0] - 1;
        double row = bw[0][0] * Cat4(C, ns, nv, g);
        for (int i = 1; i < 4; ++i) {
          g[0] = i0[0] - 1 + i;
          row = fma(bw[0][i], Cat4(C, ns, nv, g), row);
        }
        fy = (j == 0) ? bw[1][0] * row : fma(bw[1][j], row, fy);
      }
      fu = (k == 0) ? bw[2][0] * fy : fma(bw[2][k], fy, fu);
    }
    f = (l == 0) ? bw[3][0] * fu : fma(bw[3][l], fu, f);
  }
  return f;
}

static double W_kernel(double x) {
  if (x <= 1.0) {
    double x2 = x * x;
    return fma(0.75 * x, x2, fma(-1.5, x2, 1.0));
  }
  if (x <= 2.0) {
    double t = 2.0 - x;
    return ((0.25 * t) * t) * t;
  }
  return 0.0;
}

/* -------------------------------------------------------- reconstruction */

static void site_P(const or4_ctx *c, long long q, double *P, int *idx) {
  int ns = c->ns, nv = c->nv;
  idx[0] = (int)(q % ns);
  q /= ns;
  idx[1] = (int)(q % ns);
  q /= ns;
  idx[2] = (int)(q % nv);
  idx[3] = (int)(q / nv);
  for (int a = 0; a < 4; ++a) P[a] = coord(c, a, idx[a]);
}

static void index_pos(const or4_ctx *c, const double *Q, double *s) {
  s[0] = Q[0] * c->inv_dx - 0.5;
  s[1] = Q[1] * c->inv_dx - 0.5;
  s[2] = (Q[2] + c->p.vmax) * c->inv_du - 0.5;
  s[3] = (Q[3] + c->p.vmax) * c->inv_du - 0.5;
}

static double recon_site(const or4_ctx *c, long long q, int brute,
                         int32_t *assign) {
  double P[4], dq[4] = {0, 0, 0, 0};
  int idx[4];
  site_P(c, q, P, idx);
  int e = brute ? query_brute(c, P, dq) : query_bucketed(c, P, dq);
  if (assign) *assign = e;
  if (e < 0) return 0.0;
  int k[4];
  lat_index(c, e, k);
  double Q[4], s[4];
  for (int a = 0; a < 4; ++a) Q[a] = lat_q(c, a, k[a]) + dq[a];
  index_pos(c, Q, s);
  return or4_int15(c->F, c->ns, c->nv, s);
}

static void reconstruct_all(or4_ctx *c, double *f, int brute, int32_t *assign) {
#pragma omp parallel for schedule(dynamic, 64)
  for (long long q = 0; q < c->N4; ++q) {
    int32_t a = -1;
    f[q] = recon_site(c, q, brute, &a);
    if (assign) assign[q] = a;
  }
}

/* Remap value at a site: W(2d)-blend of the beta-restricted lattice
 * neighbours of the nearest element (section 2.3.2, axis by axis; R24),
 * then the tensor cubic spline of F_ini at Q_r; the u and w edge rows are
 * zero. */
static double remap_site(const or4_ctx *c, long long q) {
  double P[4], dq[4] = {0, 0, 0, 0};
  int idx[4];
  site_P(c, q, P, idx);
  if (idx[2] == 0 || idx[2] == c->nv - 1 || idx[3] == 0 || idx[3] == c->nv - 1)
    return 0.0;
  int e = query_bucketed(c, P, dq);
  if (e < 0) return 0.0;
  int k0[4], lo[4], hi[4], three = 0;
  lat_index(c, e, k0);
  for (int a = 0; a < 4; ++a) {
    double z = dq[a] * c->rD[a];
    lo[a] = (z < c->p.beta) ? -1 : 0;
    hi[a] = (z < -c->p.beta) ? 0 : 1;
    if (hi[a] - lo[a] == 2) three = 1;
  }
  double sw = 0.0, sq[4] = {0, 0, 0, 0};
  int d[4];
  for (d[3] = lo[3]; d[3] <= hi[3]; ++d[3])
    for (d[2] = lo[2]; d[2] <= hi[2]; ++d[2])
      for (d[1] = lo[1]; d[1] <= hi[1]; ++d[1])
        for (d[0] = lo[0]; d[0] <= hi[0]; ++d[0]) {
          int nz = (d[0] != 0) + (d[1] != 0) + (d[2] != 0) + (d[3] != 0);
          if (three && nz > 1) continue;
          int kk[4], ok = 1;
          double shift[4] = {0, 0, 0, 0};
          for (int a = 0; a < 4; ++a) {
            int k = k0[a] + d[a], n = lat_n(c, a);
            if (k < 0 || k >= n) {
              if (a >= 2) {
                ok = 0;
                break;
              }
              shift[a] = (k < 0) ? -c->p.L : c->p.L;
              k = (k < 0) ? k + n : k - n;
            }
            kk[a] = k;
          }
          if (!ok) continue;
          int m = ((kk[3] * c->mv + kk[2]) * c->ms + kk[1]) * c->ms + kk[0];
          double ex[4];
          elem_map(c, m, P, ex);
          double dd = sqrt(dist2(c, ex));
          double w = W_kernel(2.0 * dd);
          sw += w;
          for (int a = 0; a < 4; ++a) {
            double Qa = (lat_q(c, a, kk[a]) + shift[a]) + ex[a];
            sq[a] = fma(w, Qa, sq[a]);
          }
        }
  double Q[4], s[4];
  for (int a = 0; a < 4; ++a)
    Q[a] = (sw > 0.0) ? sq[a] / sw : lat_q(c, a, k0[a]) + dq[a];
  index_pos(c, Q, s);
  return or4_spline_eval(c->C, c->ns, c->nv, s);
}

/* ----------------------------------------------------------------- field */

/* rho(i, j) = du dw sum over the velocity sites (u, w): for every spatial
 * site the velocity grid summed sequentially, w outer and u inner, from
 * (0, 0). */
static void density(const or4_ctx *c, const double *f, double *rho) {
  int ns = c->ns, nv = c->nv;
  for (int j = 0; j < ns; ++j)
    for (int i = 0; i < ns; ++i) {
      double s = 0.0;
      for (int l = 0; l < nv; ++l)
        for (int k = 0; k < nv; ++k)
          s += f[(((size_t)l * nv + k) * ns + j) * ns + i];
      rho[(size_t)j * ns + i] = (c->du * c->du) * s;
    }
}

/* div a = -2 G (rho - rho_bar) on the periodic square by the discrete
 * Fourier transform (the plain O(n^3) definition, separable, sums in index
 * order): phi^ = -2 G rho^ / |k|^2 (k != 0), a^ = -i k phi^, with the
 * Nyquist wavenumber's derivative set to zero so that a is real.  Then
 * centred differences for grad a and the Hessian (12 fields, R24). */
static void field(or4_ctx *c, const double *rho) {
  int n = c->ns;
  size_t N2 = (size_t)n * n;
  double *cs = (double *)malloc(sizeof(double) * n);
  double *sn = (double *)malloc(sizeof(double) * n);
  double *re = (double *)calloc(N2, sizeof(double));
  double *im = (double *)calloc(N2, sizeof(double));
  double *r2 = (double *)calloc(N2, sizeof(double));
  double *i2 = (double *)calloc(N2, sizeof(double));
  const double twopi = 6.283185307179586476925286766559;
  for (int m = 0; m < n; ++m) {
    cs[m] = cos(twopi * (double)m / (double)n);
    sn[m] = sin(twopi * (double)m / (double)n);
  }
  /* forward along x: R1(p, j) = sum_i rho(i, j) e^{-2 pi i p i / n} */
  for (int j = 0; j < n; ++j)
    for (int p = 0; p < n; ++p) {
      double sr = 0.0, si = 0.0;
      for (int i = 0; i < n; ++i) {
        int m = (int)(((long long)p * i) % n);
        double v = rho[(size_t)j * n + i];
        sr = fma(v, cs[m], sr);
        si = fma(-v, sn[m], si);
      }
      re[(size_t)j * n + p] = sr;
      im[(size_t)j * n + p] = si;
    }
  /* forward along y */
  for (int p = 0; p < n; ++p)
    for (int qy = 0; qy < n; ++qy) {
      double sr = 0.0, si = 0.0;
      for (int j = 0; j < n; ++j) {
        int m = (int)(((long long)qy * j) % n);
        double a = re[(size_t)j * n + p], b = im[(size_t)j * n + p];
        /* (a + i b) (cos - i sin) */
        sr = fma(a, cs[m], fma(b, sn[m], sr));
        si = fma(b, cs[m], fma(-a, sn[m], si));
      }
      r2[(size_t)qy * n + p] = sr;
      i2[(size_t)qy * n + p] = si;
    }
  for (int comp = 0; comp < 2; ++comp) {
    /* a^_comp = -i k_comp phi^, phi^ = -2G rho^/|k|^2 */
    double *ar = re, *ai = im;  /* reuse as spectrum of a_comp */
    for (int qy = 0; qy < n; ++qy)
      for (int p = 0; p < n; ++p) {
        int pp = (p <= n / 2 - (n % 2 == 0 ? 1 : 0)) ? p : p - n;
        int qq = (qy <= n / 2 - (n % 2 == 0 ? 1 : 0)) ? qy : qy - n;
        double kx = twopi * (double)pp / c->p.L, ky = twopi * (double)qq / c->p.L;
        double k2 = kx * kx + ky * ky;
        size_t o = (size_t)qy * n + p;
        if (p == 0 && qy == 0) {
          ar[o] = 0.0;
          ai[o] = 0.0;
          continue;
        }
        double kd = comp == 0 ? kx : ky;
        int nyq = (comp == 0 ? p : qy) * 2 == n;
        if (nyq) kd = 0.0;
        double g = (-2.0 * c->p.G) / k2;
        double pr = g * r2[o], pi = g * i2[o];
        /* -i kd (pr + i pi) = kd pi - i kd pr */
        ar[o] = kd * pi;
        ai[o] = -(kd * pr);
      }
    /* inverse along y then x, real part, 1/n^2 */
    double *tr = (double *)calloc(N2, sizeof(double));
    double *ti = (double *)calloc(N2, sizeof(double));
    for (int p = 0; p < n; ++p)
      for (int j = 0; j < n; ++j) {
        double sr = 0.0, si = 0.0;
        for (int qy = 0; qy < n; ++qy) {
          int m = (int)(((long long)qy * j) % n);
          double a = ar[(size_t)qy * n + p], b = ai[(size_t)qy * n + p];
          /* (a + i b) (cos + i sin) */
          sr = fma(a, cs[m], fma(-b, sn[m], sr));
          si = fma(b, cs[m], fma(a, sn[m], si));
        }
        tr[(size_t)j * n + p] = sr;
        ti[(size_t)j * n + p] = si;
      }
    double inv_n2 = 1.0 / ((double)n * (double)n);
    double *out = c->fld + (size_t)comp * N2;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double sr = 0.0;
        for (int p = 0; p < n; ++p) {
          int m = (int)(((long long)p * i) % n);
          double a = tr[(size_t)j * n + p], b = ti[(size_t)j * n + p];
          sr = fma(a, cs[m], fma(-b, sn[m], sr));
        }
        out[(size_t)j * n + i] = sr * inv_n2;
      }
    free(tr);
    free(ti);
  }
  /* derivatives: fields 2..5 = d a_x/dx, d a_x/dy, d a_y/dx, d a_y/dy;
   * 6..8 = a_x,xx a_x,xy a_x,yy; 9..11 = a_y,xx a_y,xy a_y,yy */
  double dx = c->dx;
  for (int comp = 0; comp < 2; ++comp) {
    const double *A = c->fld + (size_t)comp * N2;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        int ip = (i + 1) % n, im_ = (i + n - 1) % n;
        int jp = (j + 1) % n, jm = (j + n - 1) % n;
#define AT(ii, jj) A[(size_t)(jj) * n + (ii)]
        size_t o = (size_t)j * n + i;
        c->fld[(size_t)(2 + 2 * comp) * N2 + o] = (AT(ip, j) - AT(im_, j)) / (2.0 * dx);
        c->fld[(size_t)(3 + 2 * comp) * N2 + o] = (AT(i, jp) - AT(i, jm)) / (2.0 * dx);
        c->fld[(size_t)(6 + 3 * comp) * N2 + o] =
            ((AT(ip, j) + AT(im_, j)) - 2.0 * AT(i, j)) / (dx * dx);
        c->fld[(size_t)(7 + 3 * comp) * N2 + o] =
            (((AT(ip, jp) - AT(ip, jm)) - AT(im_, jp)) + AT(im_, jm)) /
            (4.0 * (dx * dx));
        c->fld[(size_t)(8 + 3 * comp) * N2 + o] =
            ((AT(i, jp) + AT(i, jm)) - 2.0 * AT(i, j)) / (dx * dx);
#undef AT
      }
  }
  free(cs);
  free(sn);
  free(re);
  free(im);
  free(r2);
  free(i2);
}

/* 3 x 3 dual TSC of field k at a periodic position (x, y). */
static double tsc2(const or4_ctx *c, int k, double x, double y) {
  int n = c->ns;
  const double *A = c->fld + (size_t)k * n * n;
  double u[2] = {x * c->inv_dx - 0.5, y * c->inv_dx - 0.5};
  int i0[2];
  double w[2][3];
  for (int a = 0; a < 2; ++a) {
    if (u[a] < -3.0) u[a] = -3.0;
    if (u[a] > (double)n + 2.0) u[a] = (double)n + 2.0;
    double fi = floor(u[a] + 0.5), d = u[a] - fi;
    double tm = 0.5 - d, tp = 0.5 + d;
    i0[a] = (int)fi;
    w[a][0] = 0.5 * (tm * tm);
    w[a][1] = 0.75 - d * d;
    w[a][2] = 0.5 * (tp * tp);
  }
  double row[3];
  for (int b = 0; b < 3; ++b) {
    int j = ((i0[1] - 1 + b) % n + n) % n;
    int im_ = ((i0[0] - 1) % n + n) % n, i_ = (i0[0] % n + n) % n,
        ip = ((i0[0] + 1) % n + n) % n;
    row[b] = fma(w[0][2], A[(size_t)j * n + ip],
                 fma(w[0][1], A[(size_t)j * n + i_], w[0][0] * A[(size_t)j * n + im_]));
  }
  return fma(w[1][2], row[2], fma(w[1][1], row[1], w[1][0] * row[0]));
}

/* Kick over dt (section 2.4 in 2D space, R5: the right-hand sides use the
 * half-step T_x and H_x), then the corrector drift over dt/2. */
static void kick_and_correct(or4_ctx *c, double dt) {
  for (int e = 0; e < c->E; ++e) {
    double x = EL(c, P0, e), y = EL(c, P0 + 1, e);
    double fv[12];
    for (int k = 0; k < 12; ++k) fv[k] = tsc2(c, k, x, y);
    for (int i = 0; i < 2; ++i) {
      double a = fv[i], g0 = fv[2 + 2 * i], g1 = fv[3 + 2 * i];
      double h00 = fv[6 + 3 * i], h01 = fv[7 + 3 * i], h11 = fv[8 + 3 * i];
      EL(c, P0 + 2 + i, e) = fma(dt, a, EL(c, P0 + 2 + i, e));
      for (int j = 0; j < 4; ++j) {
        double s = fma(g1, EL(c, T0 + 4 + j, e), g0 * EL(c, T0 + j, e));
        EL(c, T0 + 4 * (2 + i) + j, e) = fma(dt, s, EL(c, T0 + 4 * (2 + i) + j, e));
      }
      for (int q = 0; q < 10; ++q) {
        int jb = PB[q], kc = PC[q];
        double t0j = EL(c, T0 + jb, e), t1j = EL(c, T0 + 4 + jb, e);
        double t0k = EL(c, T0 + kc, e), t1k = EL(c, T0 + 4 + kc, e);
        double s = g0 * EL(c, H0 + q, e);
        s = fma(g1, EL(c, H0 + 10 + q, e), s);
        s = fma(h00, t0j * t0k, s);
        s = fma(h01, fma(t0j, t1k, t1j * t0k), s);
        s = fma(h11, t1j * t1k, s);
        EL(c, H0 + 10 * (2 + i) + q, e) = fma(dt, s, EL(c, H0 + 10 * (2 + i) + q, e));
      }
    }
  }
  drift(c, 0.5 * dt);
}

/* -------------------------------------------------------------- public */

or4_ctx *or4_create(const or4_params *p) {
  if (!p || p->ns < 8 || p->nv < 4 || p->nv % 4 || p->ss < 1 || p->sv < 1 ||
      p->ns % p->ss || p->nv % p->sv || !(p->dt > 0.0) || !(p->L > 0.0) ||
      !(p->vmax > 0.0) || p->n_s < 0 || !(p->beta >= 0.0 && p->beta <= 0.5))
    return NULL;
  or4_ctx *c = (or4_ctx *)calloc(1, sizeof(or4_ctx));
  if (!c) return NULL;
  c->p = *p;
  c->ns = p->ns;
  c->nv = p->nv;
  c->ms = p->ns / p->ss;
  c->mv = p->nv / p->sv;
  c->E = c->ms * c->ms * c->mv * c->mv;
  c->N4 = (long long)p->ns * p->ns * p->nv * p->nv;
  c->dx = p->L / p->ns;
  c->du = 2.0 * p->vmax / p->nv;
  c->inv_dx = 1.0 / c->dx;
  c->inv_du = 1.0 / c->du;
  for (int a = 0; a < 4; ++a) {
    c->Dm[a] = (a < 2 ? p->ss * c->dx : p->sv * c->du);
    c->rD[a] = 1.0 / c->Dm[a];
  }
  size_t N4 = (size_t)c->N4, N2 = (size_t)p->ns * p->ns;
  c->F = (double *)calloc(N4, sizeof(double));
  c->C = (double *)calloc(N4, sizeof(double));
  c->f = (double *)calloc(N4, sizeof(double));
  c->el = (double *)calloc((size_t)NST * c->E, sizeof(double));
  c->A = (double *)calloc((size_t)16 * c->E, sizeof(double));
  c->rho = (double *)calloc(N2, sizeof(double));
  c->fld = (double *)calloc(12 * N2, sizeof(double));
  c->bitem = (int *)calloc(c->E, sizeof(int));
  if (!c->F || !c->C || !c->f || !c->el || !c->A || !c->rho || !c->fld ||
      !c->bitem) {
    or4_destroy(c);
    return NULL;
  }
  reset_elements(c);
  return c;
}

void or4_destroy(or4_ctx *c) {
  if (!c) return;
  free(c->F);
  free(c->C);
  free(c->f);
  free(c->el);
  free(c->A);
  free(c->rho);
  free(c->fld);
  free(c->bitem);
  free(c->bstart);
  free(c);
}

int or4_init_conditions(or4_ctx *c, const double *f0) {
  if (!c || !f0) return -1;
  for (long long q = 0; q < c->N4; ++q) {
    double P[4];
    int idx[4];
    site_P(c, q, P, idx);
    int edge = idx[2] == 0 || idx[2] == c->nv - 1 || idx[3] == 0 ||
               idx[3] == c->nv - 1;
    c->F[q] = edge ? 0.0 : f0[q];
  }
  int rc = or4_spline_fit(c->ns, c->nv, c->F, c->C);
  if (rc) return rc;
  reset_elements(c);
  c->t = 0.0;
  c->step = 0;
  c->ready = 1;
  return 0;
}

static int prepare(or4_ctx *c) {
  int rc = precompute(c);
  if (rc) return rc;
  return build_buckets(c);
}

int or4_remap(or4_ctx *c) {
  if (!c || !c->ready) return -4;
  int rc = prepare(c);
  if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 64)
  for (long long q = 0; q < c->N4; ++q) c->f[q] = remap_site(c, q);
  memcpy(c->F, c->f, sizeof(double) * (size_t)c->N4);
  rc = or4_spline_fit(c->ns, c->nv, c->F, c->C);
  if (rc) return rc;
  reset_elements(c);
  return 0;
}

int or4_step(or4_ctx *c, int nsteps) {
  if (!c || !c->ready) return -4;
  for (int s = 0; s < nsteps; ++s) {
    drift(c, 0.5 * c->p.dt);
    int rc = prepare(c);
    if (rc) return rc;
    reconstruct_all(c, c->f, 0, NULL);
    density(c, c->f, c->rho);
    field(c, c->rho);
    kick_and_correct(c, c->p.dt);
    c->step += 1;
    c->t = (double)c->step * c->p.dt;
    if (c->p.n_s > 0 && c->step % c->p.n_s == 0) {
      rc = or4_remap(c);
      if (rc) return rc;
    }
  }
  return 0;
}

int or4_reconstruct_f(or4_ctx *c, int scheme, double *f_out) {
  if (!c || !c->ready) return -4;
  int rc = prepare(c);
  if (rc) return rc;
  if (scheme == 0) {
    reconstruct_all(c, f_out, 0, NULL);
  } else {
#pragma omp parallel for schedule(dynamic, 64)
    for (long long q = 0; q < c->N4; ++q) f_out[q] = remap_site(c, q);
  }
  return 0;
}

int or4_density(or4_ctx *c, double *rho_out) {
  if (!c || !c->ready) return -4;
  int rc = prepare(c);
  if (rc) return rc;
  reconstruct_all(c, c->f, 0, NULL);
  density(c, c->f, rho_out);
  return 0;
}

int or4_field(or4_ctx *c, const double *rho, double *ax, double *ay) {
  if (!c) return -1;
  field(c, rho);
  size_t N2 = (size_t)c->ns * c->ns;
  memcpy(ax, c->fld, sizeof(double) * N2);
  memcpy(ay, c->fld + N2, sizeof(double) * N2);
  return 0;
}

/* mass, kinetic energy, field energy -(1/4G) sum |a|^2 dx dy, total,
 * entropy -sum f ln|f| dV, t */
int or4_diagnostics(or4_ctx *c, double *out6) {
  if (!c || !c->ready) return -4;
  int rc = prepare(c);
  if (rc) return rc;
  reconstruct_all(c, c->f, 0, NULL);
  density(c, c->f, c->rho);
  field(c, c->rho);
  double dV = (c->dx * c->dx) * (c->du * c->du);
  double mass = 0.0, kin = 0.0, ent = 0.0, pot = 0.0;
  for (long long q = 0; q < c->N4; ++q) {
    double P[4];
    int idx[4];
    site_P(c, q, P, idx);
    double f = c->f[q];
    mass += f;
    kin += (P[2] * P[2] + P[3] * P[3]) * f;
    if (f != 0.0) ent += f * log(fabs(f));
  }
  size_t N2 = (size_t)c->ns * c->ns;
  for (size_t o = 0; o < N2; ++o)
    pot += c->fld[o] * c->fld[o] + c->fld[N2 + o] * c->fld[N2 + o];
  out6[0] = mass * dV;
  out6[1] = 0.5 * kin * dV;
  out6[2] = (c->p.G != 0.0) ? -pot * (c->dx * c->dx) / (4.0 * c->p.G) : 0.0;
  out6[3] = out6[1] + out6[2];
  out6[4] = -ent * dV;
  out6[5] = c->t;
  return 0;
}

int or4_get_elements(or4_ctx *c, double *out) {
  if (!c) return -1;
  memcpy(out, c->el, sizeof(double) * (size_t)NST * c->E);
  return 0;
}

int or4_set_elements(or4_ctx *c, const double *in) {
  if (!c) return -1;
  memcpy(c->el, in, sizeof(double) * (size_t)NST * c->E);
  return 0;
}

int or4_get_assignment(or4_ctx *c, int brute, int32_t *out) {
  if (!c || !c->ready) return -4;
  int rc = prepare(c);
  if (rc) return rc;
  reconstruct_all(c, c->f, brute, out);
  return 0;
}

double or4_time(const or4_ctx *c) { return c ? c->t : 0.0; }

int or4_inverse_map(const double *el60, const double *d4, const double *P4,
                    double L, double *out6) {
  double A[16], det;
  int ok = inverse4(el60 + T0, A, &det);
  double dq[4] = {0, 0, 0, 0};
  int valid = ok ? inv_map4(el60 + P0, A, el60 + H0, d4, L, P4, dq) : 0;
  for (int a = 0; a < 4; ++a) out6[a] = dq[a];
  out6[4] = (double)valid;
  out6[5] = det;
  return 0;
}
