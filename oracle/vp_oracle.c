/*
 * vp_oracle.c -- plain CPU FP64 oracle of the metric semi-Lagrangian
 * Vlasov-Poisson method of Colombi & Alard, "A 'metric' semi-Lagrangian
 * Vlasov-Poisson solver" (arXiv:1705.03750).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg.  It is written to be read against the paper:
 * plain loops, one rounding per operation (fma() only where written), every
 * reduction in the fixed order stated beside it.  It shares no code with the
 * HIP engine.  Build: gcc -O2 -ffp-contract=off (no fast-math), optional
 * OpenMP over independent sites only (results do not depend on the thread
 * count: every sum is taken after the parallel loop, in a fixed order).
 *
 * Readings where the paper is silent, garbled or ambiguous are marked R#
 * and listed in the repository's design notes.
 */
#include "vp_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { SX_ = 0, SV_, TXX, TXV, TVX, TVV, HXXX, HXXV, HXVV, HVXX, HVXV, HVVV,
       NSTATE };

struct or_ctx {
  or_params p;
  int nx, nv, mx, mv, E;
  double dx, dv, inv_dx, inv_dv; /* site spacing and its reciprocal */
  double dxm, dvm, rx, rv;       /* element spacing and its reciprocal */
  double *F;                     /* initial condition F_ini [nv][nx] */
  double *C;                     /* cubic B-spline coefficients [nv][nx] */
  double *el;                    /* element state, SoA [12][E] */
  double *A;                     /* inverse deformation tensor, SoA [4][E] */
  double *f;                     /* scratch: reconstructed f [nv][nx] */
  double *S;                     /* column sums of f [nx] */
  double *Ml;                    /* cumulative mass M_left [nx] */
  double Mtot;
  int per;                       /* periodic in x (reading R23) */
  double Lx;                     /* period x_max - x_min */
  double Bbar;                   /* mean of the periodic field sum B(i) */
  int *bstart, *bitem;           /* bucket grid (counting sort) */
  int bnx, bnv;
  double bex, bev;
  double t;
  double dt_cur;                 /* the step the next or_step takes first */
  int64_t step;
  int ready;
};

/* ------------------------------------------------------------------ grid */

/* Sites are cell centred (reading R1 of the site grid of section 2.2.1). */
static double site_x(const or_ctx *c, int i) {
  return c->p.x_min + ((double)i + 0.5) * c->dx;
}
static double site_v(const or_ctx *c, int j) {
  return c->p.v_min + ((double)j + 0.5) * c->dv;
}
/* Element lattice in Lagrangian space (section 2.3, element grid): element
 * (k, l) sits on site (sx*k + sx/2, sv*l + sv/2) (reading R4). */
static double elem_qx(const or_ctx *c, int k) {
  return site_x(c, c->p.sx * k + c->p.sx / 2);
}
static double elem_qv(const or_ctx *c, int l) {
  return site_v(c, c->p.sv * l + c->p.sv / 2);
}

#define ST(c, k, e) ((c)->el[(size_t)(k) * (size_t)(c)->E + (size_t)(e)])
#define AM(c, k, e) ((c)->A[(size_t)(k) * (size_t)(c)->E + (size_t)(e)])

/* -------------------------------------------------------------- elements */

/* New isotropic elements: P = Q_m, T = I, H = 0 (section 2.1 initial state;
 * the same reset after every resampling, section 1 and 2.3). */
static void reset_elements(or_ctx *c) {
  for (int e = 0; e < c->E; ++e) {
    int k = e % c->mx, l = e / c->mx;
    for (int s = 0; s < NSTATE; ++s) ST(c, s, e) = 0.0;
    ST(c, SX_, e) = elem_qx(c, k);
    ST(c, SV_, e) = elem_qv(c, l);
    ST(c, TXX, e) = 1.0;
    ST(c, TVV, e) = 1.0;
  }
}

/* Periodic x (reading R23): a position that a drift moved out of
 * [x_min, x_max) re-enters from the other side (one period at most; a sum
 * that rounds onto the far edge is put on x_min). */
static double wrap_x(const or_ctx *c, double x) {
  if (x < c->p.x_min) {
    x = x + c->Lx;
    if (x >= c->p.x_max) x = c->p.x_min;
  } else if (x >= c->p.x_max) {
    x = x - c->Lx;
    if (x < c->p.x_min) x = c->p.x_min;
  }
  return x;
}

/* Drift over h (section 2.4, predictor and corrector): positions move with
 * the velocities, T_x. with T_v., H_x with H_v. */
static void drift(or_ctx *c, double h) {
  for (int e = 0; e < c->E; ++e) {
    ST(c, SX_, e) = fma(h, ST(c, SV_, e), ST(c, SX_, e));
    if (c->per) ST(c, SX_, e) = wrap_x(c, ST(c, SX_, e));
    ST(c, TXX, e) = fma(h, ST(c, TVX, e), ST(c, TXX, e));
    ST(c, TXV, e) = fma(h, ST(c, TVV, e), ST(c, TXV, e));
    ST(c, HXXX, e) = fma(h, ST(c, HVXX, e), ST(c, HXXX, e));
    ST(c, HXXV, e) = fma(h, ST(c, HVXV, e), ST(c, HXXV, e));
    ST(c, HXVV, e) = fma(h, ST(c, HVVV, e), ST(c, HXVV, e));
  }
}

/* Per-element inverse A = T^-1, precomputed once per reconstruction as the
 * paper suggests at the end of section 2.1.  det T must stay positive (it is
 * 1 for the exact flow, eq. detJ); anything else is a numerical failure. */
static int precompute(or_ctx *c) {
  for (int e = 0; e < c->E; ++e) {
    double txx = ST(c, TXX, e), txv = ST(c, TXV, e);
    double tvx = ST(c, TVX, e), tvv = ST(c, TVV, e);
    double det = fma(txx, tvv, -(txv * tvx));
    if (!(det > 0.0) || !isfinite(det) || !isfinite(ST(c, SX_, e)) ||
        !isfinite(ST(c, SV_, e)))
      return OR_ENUMERIC;
    double inv = 1.0 / det;
    AM(c, 0, e) = tvv * inv;
    AM(c, 1, e) = -txv * inv;
    AM(c, 2, e) = -tvx * inv;
    AM(c, 3, e) = txx * inv;
  }
  return OR_OK;
}

/* Second-order inverse map of section 2.1, eq. (QofP):
 *   dQ = A dP - 1/2 A (dP^T A^T H A dP),  A = T^-1,
 * written with l = A dP and u_c = l^T H_c l (reading R7: the same quantity as
 * the paper's precomputed A^T H A, one canonical rounding).  Returns whether
 * the element is valid for this site: |l_x| < dx_m and |l_v| < dv_m (reading
 * R8: the first-order Lagrangian offset stays inside one element spacing). */
static int inv_map(double xm, double vm, double axx, double axv, double avx,
                   double avv, const double *h6, double dxm, double dvm,
                   double xP, double vP, double Lx, double *dqx, double *dqv) {
  double dx = xP - xm, dv = vP - vm;
  if (Lx > 0.0) {
    /* periodic x: the nearest image of the element (reading R23) */
    double hL = 0.5 * Lx;
    if (dx > hL)
      dx = dx - Lx;
    else if (dx < -hL)
      dx = dx + Lx;
  }
  double lx = fma(axx, dx, axv * dv);
  double lv = fma(avx, dx, avv * dv);
  int valid = fabs(lx) < dxm && fabs(lv) < dvm;
  double pxx = lx * lx, pxv = lx * lv, pvv = lv * lv;
  double ux = fma(h6[0], pxx, fma(2.0 * h6[1], pxv, h6[2] * pvv));
  double uv = fma(h6[3], pxx, fma(2.0 * h6[4], pxv, h6[5] * pvv));
  *dqx = fma(-0.5 * axx, ux, fma(-0.5 * axv, uv, lx));
  *dqv = fma(-0.5 * avx, ux, fma(-0.5 * avv, uv, lv));
  return valid;
}

static int elem_map(const or_ctx *c, int e, double xP, double vP, double *dqx,
                    double *dqv) {
  double h6[6] = {ST(c, HXXX, e), ST(c, HXXV, e), ST(c, HXVV, e),
                  ST(c, HVXX, e), ST(c, HVXV, e), ST(c, HVVV, e)};
  return inv_map(ST(c, SX_, e), ST(c, SV_, e), AM(c, 0, e), AM(c, 1, e),
                 AM(c, 2, e), AM(c, 3, e), h6, c->dxm, c->dvm, xP, vP,
                 c->per ? c->Lx : 0.0, dqx, dqv);
}

/* Squared Lagrangian distance of eq. (distdef), normalised by the element
 * spacing (reading R9). */
static double dist2(const or_ctx *c, double dqx, double dqv) {
  double zx = dqx * c->rx, zv = dqv * c->rv;
  return fma(zx, zx, zv * zv);
}

/* ------------------------------------------------- nearest-element query */

/* The closest element in Lagrangian space (sections 1 and 2.3): the valid
 * element with the smallest (d^2, id).  Brute force over all elements, in
 * ascending id so that a strict "<" keeps the lowest id on ties. */
static int query_brute(const or_ctx *c, double xP, double vP, double *bdqx,
                       double *bdqv) {
  int best = -1;
  double bd = INFINITY;
  for (int e = 0; e < c->E; ++e) {
    double dqx, dqv;
    if (!elem_map(c, e, xP, vP, &dqx, &dqv)) continue;
    double d2 = dist2(c, dqx, dqv);
    if (d2 < bd) {
      bd = d2;
      best = e;
      *bdqx = dqx;
      *bdqv = dqv;
    }
  }
  return best;
}

/* Bucket grid for the same query.  A valid element satisfies
 * |dP_x| <= |Txx| dx_m + |Txv| dv_m (and likewise for v), so buckets at least
 * as wide as the largest such reach, slightly inflated for rounding, hold
 * every valid element of a site in the 3x3 buckets around it. */
static int build_buckets(or_ctx *c) {
  double Rx = 0.0, Rv = 0.0;
  for (int e = 0; e < c->E; ++e) {
    double rx = fabs(ST(c, TXX, e)) * c->dxm + fabs(ST(c, TXV, e)) * c->dvm;
    double rv = fabs(ST(c, TVX, e)) * c->dxm + fabs(ST(c, TVV, e)) * c->dvm;
    if (rx > Rx) Rx = rx;
    if (rv > Rv) Rv = rv;
  }
  double Lx = c->p.x_max - c->p.x_min, Lv = c->p.v_max - c->p.v_min;
  const int cap = 4096;
  double ex = Rx * (1.0 + 0x1p-20) + 0x1p-30 * Lx;
  double ev = Rv * (1.0 + 0x1p-20) + 0x1p-30 * Lv;
  if (ex < Lx / cap) ex = Lx / cap;
  if (ev < Lv / cap) ev = Lv / cap;
  int bnx = (int)ceil(Lx / ex), bnv = (int)ceil(Lv / ev);
  if (c->per) {
    /* periodic x: equal buckets no narrower than the reach, so that the
     * wrapped neighbouring buckets hold every valid element */
    bnx = (int)floor(Lx / ex);
    if (bnx < 1) bnx = 1;
    ex = Lx / bnx;
  }
  if (bnx < 1) bnx = 1;
  if (bnv < 1) bnv = 1;
  free(c->bstart);
  c->bstart = (int *)calloc((size_t)bnx * bnv + 1, sizeof(int));
  if (!c->bstart) return OR_ENOMEM;
  c->bnx = bnx;
  c->bnv = bnv;
  c->bex = ex;
  c->bev = ev;
  int *bid = (int *)malloc(sizeof(int) * (size_t)c->E);
  if (!bid) return OR_ENOMEM;
  for (int e = 0; e < c->E; ++e) {
    int bx = (int)floor((ST(c, SX_, e) - c->p.x_min) / ex);
    int bv = (int)floor((ST(c, SV_, e) - c->p.v_min) / ev);
    if (bx < 0) bx = 0;
    if (bx > bnx - 1) bx = bnx - 1;
    if (bv < 0) bv = 0;
    if (bv > bnv - 1) bv = bnv - 1;
    bid[e] = bv * bnx + bx;
    c->bstart[bid[e] + 1] += 1;
  }
  for (int b = 0; b < bnx * bnv; ++b) c->bstart[b + 1] += c->bstart[b];
  int *fill = (int *)malloc(sizeof(int) * ((size_t)bnx * bnv));
  if (!fill) {
    free(bid);
    return OR_ENOMEM;
  }
  memcpy(fill, c->bstart, sizeof(int) * ((size_t)bnx * bnv));
  for (int e = 0; e < c->E; ++e) c->bitem[fill[bid[e]]++] = e;
  free(fill);
  free(bid);
  return OR_OK;
}

static int query_bucketed(const or_ctx *c, double xP, double vP, double *bdqx,
                          double *bdqv) {
  int bx = (int)floor((xP - c->p.x_min) / c->bex);
  int bv = (int)floor((vP - c->p.v_min) / c->bev);
  int best = -1;
  double bd = INFINITY;
  if (bx < 0) bx = 0;
  if (bx > c->bnx - 1) bx = c->bnx - 1;
  /* periodic x with fewer than 3 buckets: visit each bucket once */
  int ilo = bx - 1, ihi = bx + 1;
  if (c->per && c->bnx < 3) {
    ilo = 0;
    ihi = c->bnx - 1;
  }
  for (int jb = bv - 1; jb <= bv + 1; ++jb) {
    if (jb < 0 || jb >= c->bnv) continue;
    for (int iu = ilo; iu <= ihi; ++iu) {
      int ib = iu;
      if (c->per) ib = (iu + c->bnx) % c->bnx;
      if (ib < 0 || ib >= c->bnx) continue;
      int b = jb * c->bnx + ib;
      for (int q = c->bstart[b]; q < c->bstart[b + 1]; ++q) {
        int e = c->bitem[q];
        double dqx, dqv;
        if (!elem_map(c, e, xP, vP, &dqx, &dqv)) continue;
        double d2 = dist2(c, dqx, dqv);
        if (d2 < bd || (d2 == bd && e < best)) {
          bd = d2;
          best = e;
          *bdqx = dqx;
          *bdqv = dqv;
        }
      }
    }
  }
  return best;
}

/* ---------------------------------------------------------- interpolation */

static double Fat(const double *F, int nx, int nv, int i, int j, int per) {
  if (per) i = ((i % nx) + nx) % nx;
  if (i < 0 || i >= nx || j < 0 || j >= nv) return 0.0;
  return F[(size_t)j * nx + i];
}

/* Periodic x (reading R23): interpolation positions are clamped to
 * [-12, nx + 11] sites (only elements far outside their validity could
 * reach beyond) and the data repeat with period nx. */
static double clamp_periodic(double sx, int nx) {
  if (sx < -12.0) return -12.0;
  if (sx > (double)nx + 11.0) return (double)nx + 11.0;
  return sx;
}

/* Six-point second-order interpolation of section 2.2.1, eq. (int1), at
 * index-space position (sx, sv) (site (i, j) sits at integer (i, j)).  The
 * F(i_n-1) terms carry a minus sign and the v-row uses F(i_n, j_n-1): the
 * Lagrange form of the quadratic through the cross (reading R10; the printed
 * signs make the weights sum to 1.25).  i_n rounds half up (reading R11). */
static double int1_eval(const double *F, int nx, int nv, double sx,
                        double sv, int per) {
  if (per) {
    sx = clamp_periodic(sx, nx);
    if (!(sv > -4.0 && sv < nv + 3.0)) return 0.0;
  } else if (!(sx > -4.0 && sx < nx + 3.0 && sv > -4.0 && sv < nv + 3.0)) {
    return 0.0;
  }
  double fin = floor(sx + 0.5), fjn = floor(sv + 0.5);
  double fic = floor(sx), fjc = floor(sv);
  int in = (int)fin, jn = (int)fjn, ic = (int)fic, jc = (int)fjc;
  double dqx = sx - fin, dqv = sv - fjn;
  double w0 = (1.0 - dqx * dqx) - dqv * dqv;
  double hx = 0.5 * dqx, hv = 0.5 * dqv;
  double wxp = hx * (1.0 + dqx), wxm = hx * (1.0 - dqx);
  double wvp = hv * (1.0 + dqv), wvm = hv * (1.0 - dqv);
  double wc = dqx * dqv;
  double cross = ((Fat(F, nx, nv, ic + 1, jc + 1, per) +
                   Fat(F, nx, nv, ic, jc, per)) -
                  Fat(F, nx, nv, ic + 1, jc, per)) -
                 Fat(F, nx, nv, ic, jc + 1, per);
  double f = Fat(F, nx, nv, in, jn, per) * w0;
  f = fma(Fat(F, nx, nv, in + 1, jn, per), wxp, f);
  f = fma(-Fat(F, nx, nv, in - 1, jn, per), wxm, f);
  f = fma(Fat(F, nx, nv, in, jn + 1, per), wvp, f);
  f = fma(-Fat(F, nx, nv, in, jn - 1, per), wvm, f);
  f = fma(cross, wc, f);
  return f;
}

double or_int1(const double *F, int nx, int nv, double sx, double sv) {
  return int1_eval(F, nx, nv, sx, sv, 0);
}

double or_int1_periodic(const double *F, int nx, int nv, double sx,
                        double sv) {
  return int1_eval(F, nx, nv, sx, sv, 1);
}

/* Cubic B-spline interpolation with the edge conditions of section 2.2.2:
 * f = 0 and df/dq = 0 on the outermost nodes.  The zero slope is a mirror
 * ghost c(-1) = c(1), c(n) = c(n-2); the zero value is the zeroed edge ring
 * of F (reading R2).  Node values satisfy (c[i-1] + 4 c[i] + c[i+1]) / 6 = F,
 * so each line is the tridiagonal system (1, 4, 1) c = 6 F with end rows
 * (4, 2) and (2, 4), solved by Thomas elimination, along x for every row and
 * then along v for every column (reading R18). */
static void thomas_line(int n, const double *rhs_in, size_t istride,
                        double *out, size_t ostride, double *cp, double *dp) {
  double rinv = 0.25;
  cp[0] = 2.0 * rinv;
  dp[0] = (6.0 * rhs_in[0]) * rinv;
  for (int i = 1; i < n; ++i) {
    double sub = (i == n - 1) ? 2.0 : 1.0;
    double sup = 1.0;
    double den = 4.0 - sub * cp[i - 1];
    rinv = 1.0 / den;
    cp[i] = sup * rinv;
    dp[i] = (6.0 * rhs_in[(size_t)i * istride] - sub * dp[i - 1]) * rinv;
  }
  out[(size_t)(n - 1) * ostride] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i)
    out[(size_t)i * ostride] = dp[i] - cp[i] * out[(size_t)(i + 1) * ostride];
}

/* Periodic line (reading R23): the cyclic system c(i-1) + 4 c(i) + c(i+1)
 * = 6 F(i), indices mod n, by the Sherman-Morrison form of Thomas
 * elimination: with gamma = -4 the corner entries move into the rank-one
 * term u v^T, u = (gamma, 0.., 0, 1), v = (1, 0.., 0, 1/gamma), leaving the
 * tridiagonal B with diagonal (8, 4, .., 4, 4.25) and unit off-diagonals.
 * Solve B y = 6 F and B z = u, then c = y - [(v.y) / (1 + v.z)] z.  n >= 3. */
static void thomas_plain(int n, const double *b, const double *rhs,
                         double *out, double *cp, double *dp) {
  double rinv = 1.0 / b[0];
  cp[0] = rinv;
  dp[0] = rhs[0] * rinv;
  for (int i = 1; i < n; ++i) {
    double den = b[i] - cp[i - 1];
    rinv = 1.0 / den;
    cp[i] = rinv;
    dp[i] = (rhs[i] - dp[i - 1]) * rinv;
  }
  out[n - 1] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) out[i] = dp[i] - cp[i] * out[i + 1];
}

static int cyclic_line(int n, const double *rhs_in, size_t istride,
                       double *out, size_t ostride) {
  double *b = (double *)malloc(sizeof(double) * n);
  double *r = (double *)malloc(sizeof(double) * n);
  double *u = (double *)calloc(n, sizeof(double));
  double *y = (double *)malloc(sizeof(double) * n);
  double *z = (double *)malloc(sizeof(double) * n);
  double *cp = (double *)malloc(sizeof(double) * n);
  double *dp = (double *)malloc(sizeof(double) * n);
  int ok = b && r && u && y && z && cp && dp;
  if (ok) {
    for (int i = 0; i < n; ++i) {
      b[i] = 4.0;
      r[i] = 6.0 * rhs_in[(size_t)i * istride];
    }
    b[0] = 8.0;       /* 4 - gamma */
    b[n - 1] = 4.25;  /* 4 - 1 * 1 / gamma */
    u[0] = -4.0;
    u[n - 1] = 1.0;
    thomas_plain(n, b, r, y, cp, dp);
    thomas_plain(n, b, u, z, cp, dp);
    double num = y[0] - 0.25 * y[n - 1];
    double den = (1.0 + z[0]) - 0.25 * z[n - 1];
    double fact = num / den;
    for (int i = 0; i < n; ++i) out[(size_t)i * ostride] = y[i] - fact * z[i];
  }
  free(b);
  free(r);
  free(u);
  free(y);
  free(z);
  free(cp);
  free(dp);
  return ok ? OR_OK : OR_ENOMEM;
}

/* Periodic in x, edge conditions of section 2.2.2 in v (reading R23). */
int or_spline_fit_periodic(int nx, int nv, const double *F, double *C) {
  if (nx < 3 || nv < 2) return OR_EINVAL;
  double *cp = (double *)malloc(sizeof(double) * nv);
  double *dp = (double *)malloc(sizeof(double) * nv);
  double *T = (double *)malloc(sizeof(double) * (size_t)nx * nv);
  int rc = (cp && dp && T) ? OR_OK : OR_ENOMEM;
  for (int j = 0; j < nv && rc == OR_OK; ++j)
    rc = cyclic_line(nx, F + (size_t)j * nx, 1, T + (size_t)j * nx, 1);
  if (rc == OR_OK)
    for (int i = 0; i < nx; ++i)
      thomas_line(nv, T + i, (size_t)nx, C + i, (size_t)nx, cp, dp);
  free(cp);
  free(dp);
  free(T);
  return rc;
}

int or_spline_fit(int nx, int nv, const double *F, double *C) {
  if (nx < 2 || nv < 2) return OR_EINVAL;
  int nmax = nx > nv ? nx : nv;
  double *cp = (double *)malloc(sizeof(double) * nmax);
  double *dp = (double *)malloc(sizeof(double) * nmax);
  double *T = (double *)malloc(sizeof(double) * (size_t)nx * nv);
  if (!cp || !dp || !T) {
    free(cp);
    free(dp);
    free(T);
    return OR_ENOMEM;
  }
  for (int j = 0; j < nv; ++j)
    thomas_line(nx, F + (size_t)j * nx, 1, T + (size_t)j * nx, 1, cp, dp);
  for (int i = 0; i < nx; ++i)
    thomas_line(nv, T + i, (size_t)nx, C + i, (size_t)nx, cp, dp);
  free(cp);
  free(dp);
  free(T);
  return OR_OK;
}

static double Cat(const double *C, int nx, int nv, int i, int j, int per) {
  if (per) {
    i = ((i % nx) + nx) % nx;          /* periodic x (R23) */
  } else {
    if (i < 0) i = -i;                 /* c(-1) = c(1) */
    if (i > nx - 1) i = 2 * (nx - 1) - i; /* c(n) = c(n-2) */
  }
  if (j < 0) j = -j;
  if (j > nv - 1) j = 2 * (nv - 1) - j;
  return C[(size_t)j * nx + i];
}

static void bspline_weights(double u, double b[4]) {
  const double sixth = 1.0 / 6.0;
  double t = 1.0 - u;
  double u2 = u * u, u3 = u2 * u;
  b[0] = ((t * t) * t) * sixth;
  b[1] = ((3.0 * u3 - 6.0 * u2) + 4.0) * sixth;
  b[2] = (((-3.0 * u3 + 3.0 * u2) + 3.0 * u) + 1.0) * sixth;
  b[3] = u3 * sixth;
}

static double spline_eval_any(const double *C, int nx, int nv, double sx,
                              double sv, int per) {
  if (per) {
    sx = clamp_periodic(sx, nx);
    if (!(sv >= 0.0 && sv <= (double)(nv - 1))) return 0.0;
  } else if (!(sx >= 0.0 && sx <= (double)(nx - 1) && sv >= 0.0 &&
               sv <= (double)(nv - 1))) {
    return 0.0;
  }
  int i = (int)floor(sx), j = (int)floor(sv);
  if (!per && i > nx - 2) i = nx - 2;
  if (j > nv - 2) j = nv - 2;
  double bx[4], bv[4];
  bspline_weights(sx - (double)i, bx);
  bspline_weights(sv - (double)j, bv);
  double f = 0.0;
  for (int b = 0; b < 4; ++b) {
    double row = bx[0] * Cat(C, nx, nv, i - 1, j - 1 + b, per);
    row = fma(bx[1], Cat(C, nx, nv, i, j - 1 + b, per), row);
    row = fma(bx[2], Cat(C, nx, nv, i + 1, j - 1 + b, per), row);
    row = fma(bx[3], Cat(C, nx, nv, i + 2, j - 1 + b, per), row);
    f = (b == 0) ? bv[0] * row : fma(bv[b], row, f);
  }
  return f;
}

double or_spline_eval(const double *C, int nx, int nv, double sx, double sv) {
  return spline_eval_any(C, nx, nv, sx, sv, 0);
}

double or_spline_eval_periodic(const double *C, int nx, int nv, double sx,
                               double sv) {
  return spline_eval_any(C, nx, nv, sx, sv, 1);
}

/* Monaghan cubic-spline kernel of section 2.3.2 (support 2). */
double or_W(double x) {
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

/* ---------------------------------------------------------- reconstruction */

/* Transport-phase value at site (i, j): nearest element, inverse map, then
 * six-point interpolation of F_ini at Q (section 1 summary, sections 2.1 and
 * 2.2.1).  Unmapped sites (no valid element) get 0. */
static double recon_transport_site(const or_ctx *c, int i, int j, int brute,
                                   int *assign) {
  double xP = site_x(c, i), vP = site_v(c, j), dqx = 0.0, dqv = 0.0;
  int e = brute ? query_brute(c, xP, vP, &dqx, &dqv)
                : query_bucketed(c, xP, vP, &dqx, &dqv);
  if (assign) *assign = e;
  if (e < 0) return 0.0;
  double Qx = elem_qx(c, e % c->mx) + dqx;
  double Qv = elem_qv(c, e / c->mx) + dqv;
  double sx = (Qx - c->p.x_min) * c->inv_dx - 0.5;
  double sv = (Qv - c->p.v_min) * c->inv_dv - 0.5;
  return int1_eval(c->F, c->nx, c->nv, sx, sv, c->per);
}

/* Lattice neighbour k of an element column (periodic x, reading R23: the
 * columns wrap and the wrapped neighbour's Lagrangian position moves by one
 * period, *shift = -Lx or +Lx).  Returns -1 when there is no neighbour. */
static int lattice_col(const or_ctx *c, int k, double *shift) {
  *shift = 0.0;
  if (k >= 0 && k < c->mx) return k;
  if (!c->per) return -1;
  if (k < 0) {
    *shift = -c->Lx;
    return k + c->mx;
  }
  *shift = c->Lx;
  return k - c->mx;
}

/* Remap-time value at site (i, j), section 2.3.2: the W-weighted blend
 * Q_r of eq. (interpol) over the beta-restricted neighbours of the nearest
 * element (readings R16, R17), then cubic-spline interpolation of F_ini at
 * Q_r, with the edge ring forced to zero (reading R2). */
static int remap_position(const or_ctx *c, double xP, double vP, double *Qx,
                          double *Qv) {
  double dqx = 0.0, dqv = 0.0;
  int e = query_bucketed(c, xP, vP, &dqx, &dqv);
  if (e < 0) return 0;
  int k0 = e % c->mx, l0 = e / c->mx;
  double zx = dqx * c->rx, zv = dqv * c->rv, beta = c->p.beta;
  int xlo = (zx < beta) ? -1 : 0, xhi = (zx < -beta) ? 0 : 1;
  int vlo = (zv < beta) ? -1 : 0, vhi = (zv < -beta) ? 0 : 1;
  int three = (xhi - xlo == 2) || (vhi - vlo == 2);
  double sw = 0.0, sqx = 0.0, sqv = 0.0;
  for (int dl = vlo; dl <= vhi; ++dl) {
    for (int dk = xlo; dk <= xhi; ++dk) {
      if (three && dk != 0 && dl != 0) continue;
      double shift;
      int k = lattice_col(c, k0 + dk, &shift), l = l0 + dl;
      if (k < 0 || l < 0 || l >= c->mv) continue;
      int m = l * c->mx + k;
      double ex, ev;
      elem_map(c, m, xP, vP, &ex, &ev);
      double qx = (elem_qx(c, k) + shift) + ex, qv = elem_qv(c, l) + ev;
      double d = sqrt(dist2(c, ex, ev));
      double w = or_W(2.0 * d);
      sw += w;
      sqx = fma(w, qx, sqx);
      sqv = fma(w, qv, sqv);
    }
  }
  if (sw > 0.0) {
    *Qx = sqx / sw;
    *Qv = sqv / sw;
  } else {
    *Qx = elem_qx(c, k0) + dqx;
    *Qv = elem_qv(c, l0) + dqv;
  }
  return 1;
}

static double remap_site(const or_ctx *c, int i, int j) {
  if (j == 0 || j == c->nv - 1) return 0.0;
  if (!c->per && (i == 0 || i == c->nx - 1)) return 0.0;
  double Qx, Qv;
  if (!remap_position(c, site_x(c, i), site_v(c, j), &Qx, &Qv)) return 0.0;
  double sx = (Qx - c->p.x_min) * c->inv_dx - 0.5;
  double sv = (Qv - c->p.v_min) * c->inv_dv - 0.5;
  return spline_eval_any(c->C, c->nx, c->nv, sx, sv, c->per);
}

/* Mismatch of the Lagrangian positions predicted at site P by the nearest
 * element and by each of its lattice neighbours (section 2.3.3, end): the
 * Lagrangian distance of eq. (distdef) between the two predictions, in
 * element-spacing units.  Reading R21: the neighbours are the four lattice
 * neighbours (k +- 1, l), (k, l +- 1) of the nearest element that exist and
 * whose validity window holds P (reading R8), and the site value is the
 * largest mismatch over them (0 when none). */
static double emap_site(const or_ctx *c, double xP, double vP) {
  double dqx = 0.0, dqv = 0.0;
  int e = query_bucketed(c, xP, vP, &dqx, &dqv);
  if (e < 0) return 0.0;
  int k0 = e % c->mx, l0 = e / c->mx;
  double qx0 = elem_qx(c, k0) + dqx, qv0 = elem_qv(c, l0) + dqv;
  static const int nk[4] = {-1, 1, 0, 0}, nl[4] = {0, 0, -1, 1};
  double worst = 0.0;
  for (int q = 0; q < 4; ++q) {
    double shift;
    int k = lattice_col(c, k0 + nk[q], &shift), l = l0 + nl[q];
    if (k < 0 || l < 0 || l >= c->mv) continue;
    double ex, ev;
    if (!elem_map(c, l * c->mx + k, xP, vP, &ex, &ev)) continue;
    double mx = ((elem_qx(c, k) + shift) + ex) - qx0;
    double mv = (elem_qv(c, l) + ev) - qv0;
    double d = sqrt(dist2(c, mx, mv));
    if (d > worst) worst = d;
  }
  return worst;
}

/* E_map: the largest neighbour mismatch over all sites, for the current
 * element state (positions at the current time, no drift). */
static double emap_all(const or_ctx *c) {
  int nx = c->nx, nv = c->nv;
  double worst = 0.0;
#pragma omp parallel for schedule(dynamic, 4) reduction(max : worst)
  for (int j = 0; j < nv; ++j)
    for (int i = 0; i < nx; ++i) {
      double d = emap_site(c, site_x(c, i), site_v(c, j));
      if (d > worst) worst = d;
    }
  return worst;
}

static void reconstruct_all(or_ctx *c, double *f, int brute, int32_t *assign) {
  int nx = c->nx, nv = c->nv;
#pragma omp parallel for schedule(dynamic, 4)
  for (int j = 0; j < nv; ++j)
    for (int i = 0; i < nx; ++i) {
      int a = -1;
      f[(size_t)j * nx + i] = recon_transport_site(c, i, j, brute, &a);
      if (assign) assign[(size_t)j * nx + i] = a;
    }
}

/* --------------------------------------------------------------- the field */

/* Column sums S(i) = sum_j f(i, j) of the density projection (section
 * 2.5): every column summed sequentially in increasing j, from row 0. */
static void column_sums(const or_ctx *c, const double *f, double *S) {
  int nx = c->nx, nv = c->nv;
  for (int i = 0; i < nx; ++i) {
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += f[(size_t)j * nx + i];
    S[i] = s;
  }
}

/* Periodic x (reading R23): the force of a mass distribution on a ring
 * with a uniform background of the same total mass (the neutralising ions
 * of a plasma, or the mean density removed from a periodic gravitating
 * system).  B(i) is M_right - M_left of eq. (acccomp) minus the
 * background's own M_right - M_left at site i, M_tot (2 i + 1) / nx; the
 * force is G (B(i) - mean B), the mean making the field periodic.  G < 0
 * repels: a plasma with mean density 1 and G = -1/2 has da/dx = rho - 1,
 * the electron dynamics with a = -E. */
static double periodic_B(const or_ctx *c, long i) {
  double bg = c->Mtot * ((double)(2 * i + 1) / (double)c->nx);
  double Lm = (i >= 1) ? c->Ml[i - 1] : 0.0;
  return (bg - c->Ml[i]) - Lm;
}

/* Cumulative mass M_left(i) = sum_{m <= i} M(m) of section 2.5 as a
 * running sum from site 0.  M_tot is the last cumulative value (R13). */
static void cumulative_mass(or_ctx *c, const double *M) {
  int n = c->nx;
  double run = 0.0;
  for (int i = 0; i < n; ++i) {
    run += M[i];
    c->Ml[i] = run;
  }
  c->Mtot = c->Ml[n - 1];
  if (c->per) {
    /* the mean of B(i) (see acc_at), a running sum from site 0 */
    double tot = 0.0;
    for (int i = 0; i < n; ++i) tot += periodic_B(c, i);
    c->Bbar = tot / (double)n;
  }
}

static double Ml_at(const or_ctx *c, long i) {
  if (i < 0) return 0.0;
  if (i >= c->nx) return c->Mtot;
  return c->Ml[i];
}

/* Force of eq. (acccomp): a(i) = G (M_tot - M_left(i) - M_left(i-1)), the
 * coupling G in the paper's units (reading R14), extended to every integer
 * (a = +G M_tot left of the grid, -G M_tot right of it). */
static double acc_at(const or_ctx *c, long i) {
  if (c->per) {
    long k = ((i % c->nx) + c->nx) % c->nx;
    return c->p.G * (periodic_B(c, k) - c->Bbar);
  }
  return c->p.G * ((c->Mtot - Ml_at(c, i)) - Ml_at(c, i - 1));
}
/* Finite-difference gradient and Hessian of section 2.5, the gradient as a
 * centred difference over 2 dx (reading R12). */
static double dacc_at(const or_ctx *c, long i) {
  return (acc_at(c, i + 1) - acc_at(c, i - 1)) / (2.0 * c->dx);
}
static double d2acc_at(const or_ctx *c, long i) {
  return ((acc_at(c, i + 1) + acc_at(c, i - 1)) - 2.0 * acc_at(c, i)) /
         (c->dx * c->dx);
}

/* Dual TSC interpolation of section 2.5 at index-space position u of a
 * sampled field g(i) (i integer).  Used through tsc_field below. */
static void tsc_weights(double u, long *i0, double w[3]) {
  double fi = floor(u + 0.5);
  double w_ = u - fi;
  double tm = 0.5 - w_, tp = 0.5 + w_;
  *i0 = (long)fi;
  w[0] = 0.5 * (tm * tm);
  w[1] = 0.75 - w_ * w_;
  w[2] = 0.5 * (tp * tp);
}

double or_tsc(const double *g, int n, double u) {
  long i;
  double w[3];
  tsc_weights(u, &i, w);
  double gm = (i - 1 >= 0 && i - 1 < n) ? g[i - 1] : 0.0;
  double g0 = (i >= 0 && i < n) ? g[i] : 0.0;
  double gp = (i + 1 >= 0 && i + 1 < n) ? g[i + 1] : 0.0;
  return fma(w[2], gp, fma(w[1], g0, w[0] * gm));
}

static void force_at_x(const or_ctx *c, double x, double *a, double *da,
                       double *d2a) {
  if (c->p.force_mode == OR_FORCE_EXTERNAL) {
    double a0 = c->p.ext_a0, a1 = c->p.ext_a1, a2 = c->p.ext_a2;
    *a = fma(fma(a2, x, a1), x, a0);
    *da = fma(2.0 * a2, x, a1);
    *d2a = 2.0 * a2;
    return;
  }
  double u = (x - c->p.x_min) * c->inv_dx - 0.5;
  if (u < -3.0) u = -3.0;
  if (u > (double)c->nx + 2.0) u = (double)c->nx + 2.0;
  long i;
  double w[3];
  tsc_weights(u, &i, w);
  *a = fma(w[2], acc_at(c, i + 1), fma(w[1], acc_at(c, i), w[0] * acc_at(c, i - 1)));
  *da = fma(w[2], dacc_at(c, i + 1),
            fma(w[1], dacc_at(c, i), w[0] * dacc_at(c, i - 1)));
  *d2a = fma(w[2], d2acc_at(c, i + 1),
             fma(w[1], d2acc_at(c, i), w[0] * d2acc_at(c, i - 1)));
}

/* f -> S -> rho(i) = dv S(i) -> M(i) = dx rho(i) -> M_left. */
static void field_from_f(or_ctx *c, const double *f, double *rho_out) {
  column_sums(c, f, c->S);
  double *M = (double *)calloc(c->nx, sizeof(double));
  for (int i = 0; i < c->nx; ++i) {
    double rho = c->dv * c->S[i];
    if (rho_out) rho_out[i] = rho;
    M[i] = c->dx * rho;
  }
  cumulative_mass(c, M);
  free(M);
}

/* Kick of section 2.4 over dt (with the right-hand side of the T kick read
 * as T_v.(t), reading R5), then the corrector drift over dt/2. */
static void kick_and_correct(or_ctx *c, double dt) {
  for (int e = 0; e < c->E; ++e) {
    double a, da, d2a;
    force_at_x(c, ST(c, SX_, e), &a, &da, &d2a);
    double txx = ST(c, TXX, e), txv = ST(c, TXV, e);
    double kdt = dt * da;
    ST(c, SV_, e) = fma(dt, a, ST(c, SV_, e));
    ST(c, TVX, e) = fma(kdt, txx, ST(c, TVX, e));
    ST(c, TVV, e) = fma(kdt, txv, ST(c, TVV, e));
    ST(c, HVXX, e) =
        fma(dt, fma(da, ST(c, HXXX, e), d2a * (txx * txx)), ST(c, HVXX, e));
    ST(c, HVXV, e) =
        fma(dt, fma(da, ST(c, HXXV, e), d2a * (txx * txv)), ST(c, HVXV, e));
    ST(c, HVVV, e) =
        fma(dt, fma(da, ST(c, HXVV, e), d2a * (txv * txv)), ST(c, HVVV, e));
  }
  drift(c, 0.5 * dt);
}

/* Variable time step of section 2.4: dt <= C_dyn / sqrt(rho_max), the
 * largest step that satisfies the bound, capped at the nominal dt (reading
 * R22).  rho_max is the largest projected density dv S(i) of the given
 * column sums, taken from 0 so that a distribution without positive
 * density keeps the cap. */
static double rho_max_of(const or_ctx *c, const double *S) {
  double m = 0.0;
  for (int i = 0; i < c->nx; ++i) {
    double rho = c->dv * S[i];
    if (rho > m) m = rho;
  }
  return m;
}
static double next_dt(const or_ctx *c, double rho_max) {
  if (!(rho_max > 0.0)) return c->p.dt;
  double d = c->p.cdyn / sqrt(rho_max);
  return d < c->p.dt ? d : c->p.dt;
}

/* ------------------------------------------------------------------ public */

or_ctx *or_create(const or_params *p) {
  if (!p || p->nx < 8 || p->nv < 8 || p->sx < 1 || p->sv < 1 ||
      p->nx % p->sx || p->nv % p->sv || !(p->dt > 0.0) ||
      !(p->x_max > p->x_min) || !(p->v_max > p->v_min) || p->n_s < 0 ||
      !(p->beta >= 0.0 && p->beta <= 0.5) || !(p->cdyn >= 0.0) ||
      (p->cdyn > 0.0 && p->force_mode != OR_FORCE_SELF) ||
      (p->bc != OR_BC_ISOLATED && p->bc != OR_BC_PERIODIC) ||
      (p->bc == OR_BC_PERIODIC && p->force_mode != OR_FORCE_SELF))
    return NULL;
  or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
  if (!c) return NULL;
  c->p = *p;
  c->nx = p->nx;
  c->nv = p->nv;
  c->mx = p->nx / p->sx;
  c->mv = p->nv / p->sv;
  c->E = c->mx * c->mv;
  c->dx = (p->x_max - p->x_min) / p->nx;
  c->dv = (p->v_max - p->v_min) / p->nv;
  c->inv_dx = 1.0 / c->dx;
  c->inv_dv = 1.0 / c->dv;
  c->dxm = p->sx * c->dx;
  c->dvm = p->sv * c->dv;
  c->rx = 1.0 / c->dxm;
  c->rv = 1.0 / c->dvm;
  c->per = p->bc == OR_BC_PERIODIC;
  c->Lx = p->x_max - p->x_min;
  size_t N2 = (size_t)c->nx * c->nv;
  c->F = (double *)calloc(N2, sizeof(double));
  c->C = (double *)calloc(N2, sizeof(double));
  c->f = (double *)calloc(N2, sizeof(double));
  c->el = (double *)calloc((size_t)NSTATE * c->E, sizeof(double));
  c->A = (double *)calloc((size_t)4 * c->E, sizeof(double));
  c->S = (double *)calloc(c->nx, sizeof(double));
  c->Ml = (double *)calloc(c->nx, sizeof(double));
  c->bitem = (int *)calloc(c->E, sizeof(int));
  if (!c->F || !c->C || !c->f || !c->el || !c->A || !c->S || !c->Ml ||
      !c->bitem) {
    or_destroy(c);
    return NULL;
  }
  reset_elements(c);
  return c;
}

void or_destroy(or_ctx *c) {
  if (!c) return;
  free(c->F);
  free(c->C);
  free(c->f);
  free(c->el);
  free(c->A);
  free(c->S);
  free(c->Ml);
  free(c->bitem);
  free(c->bstart);
  free(c);
}

/* New initial condition (section 1): F_ini = f0 with the edge ring zeroed,
 * spline fitted, isotropic elements, t = 0. */
int or_init_conditions(or_ctx *c, const double *f0) {
  if (!c || !f0) return OR_EINVAL;
  for (int j = 0; j < c->nv; ++j)
    for (int i = 0; i < c->nx; ++i) {
      double v = f0[(size_t)j * c->nx + i];
      if (j == 0 || j == c->nv - 1) v = 0.0;
      if (!c->per && (i == 0 || i == c->nx - 1)) v = 0.0;
      c->F[(size_t)j * c->nx + i] = v;
    }
  int rc = c->per ? or_spline_fit_periodic(c->nx, c->nv, c->F, c->C)
                 : or_spline_fit(c->nx, c->nv, c->F, c->C);
  if (rc) return rc;
  reset_elements(c);
  c->t = 0.0;
  c->step = 0;
  c->dt_cur = c->p.dt;
  if (c->p.cdyn > 0.0) {
    /* the first step obeys the bound for the initial density (R22) */
    column_sums(c, c->F, c->S);
    c->dt_cur = next_dt(c, rho_max_of(c, c->S));
  }
  c->ready = 1;
  return OR_OK;
}

static int prepare_query(or_ctx *c) {
  int rc = precompute(c);
  if (rc) return rc;
  return build_buckets(c);
}

/* Resampling (sections 1 and 2.3.2): f at the resampling time becomes the
 * new initial condition and new isotropic elements are created. */
int or_remap(or_ctx *c) {
  if (!c || !c->ready) return OR_ESTATE;
  int rc = prepare_query(c);
  if (rc) return rc;
  int nx = c->nx, nv = c->nv;
#pragma omp parallel for schedule(dynamic, 4)
  for (int j = 0; j < nv; ++j)
    for (int i = 0; i < nx; ++i) c->f[(size_t)j * nx + i] = remap_site(c, i, j);
  memcpy(c->F, c->f, sizeof(double) * (size_t)nx * nv);
  rc = c->per ? or_spline_fit_periodic(nx, nv, c->F, c->C)
              : or_spline_fit(nx, nv, c->F, c->C);
  if (rc) return rc;
  reset_elements(c);
  return OR_OK;
}

/* One drift-kick-drift step of section 2.4: predictor drift, f at the half
 * step from the drifted elements, force, kick, corrector drift; a resample
 * after every n_s-th step (no remap at t = 0, reading R6).  With C_dyn > 0
 * the step size follows the density bound of section 2.4: the step after
 * this one is sized from the density of this step's half-step
 * reconstruction (R22). */
int or_step(or_ctx *c, int nsteps) {
  if (!c || !c->ready) return OR_ESTATE;
  if (nsteps < 0) return OR_EINVAL;
  for (int s = 0; s < nsteps; ++s) {
    double dt = c->dt_cur;
    drift(c, 0.5 * dt);
    int rc = prepare_query(c);
    if (rc) return rc;
    if (c->p.force_mode == OR_FORCE_SELF) {
      reconstruct_all(c, c->f, 0, NULL);
      field_from_f(c, c->f, NULL);
    }
    kick_and_correct(c, dt);
    c->step += 1;
    if (c->p.cdyn > 0.0) {
      c->t = c->t + dt;
      c->dt_cur = next_dt(c, rho_max_of(c, c->S));
    } else {
      c->t = (double)c->step * c->p.dt;
    }
    int remap = c->p.n_s > 0 && c->step % c->p.n_s == 0;
    if (!remap && c->p.emap_max > 0.0 && c->p.emap_every > 0 &&
        c->step % c->p.emap_every == 0) {
      /* adaptive resampling (section 2.3.3, end): remap when the neighbour
       * mismatch of the current elements exceeds the threshold */
      rc = prepare_query(c);
      if (rc) return rc;
      remap = emap_all(c) > c->p.emap_max;
    }
    if (remap) {
      rc = or_remap(c);
      if (rc) return rc;
    }
  }
  return OR_OK;
}

int or_emap(or_ctx *c, double *emap) {
  if (!c || !c->ready || !emap) return OR_ESTATE;
  int rc = prepare_query(c);
  if (rc) return rc;
  *emap = emap_all(c);
  return OR_OK;
}

int or_reconstruct_f(or_ctx *c, int scheme, double *f_out) {
  if (!c || !c->ready) return OR_ESTATE;
  int rc = prepare_query(c);
  if (rc) return rc;
  if (scheme == OR_SCHEME_TRANSPORT) {
    reconstruct_all(c, f_out, 0, NULL);
  } else if (scheme == OR_SCHEME_REMAP) {
    int nx = c->nx, nv = c->nv;
#pragma omp parallel for schedule(dynamic, 4)
    for (int j = 0; j < nv; ++j)
      for (int i = 0; i < nx; ++i) f_out[(size_t)j * nx + i] = remap_site(c, i, j);
  } else {
    return OR_EINVAL;
  }
  return OR_OK;
}

int or_reconstruct_sites(or_ctx *c, int scheme, int64_t n, const int64_t *site,
                         double *f_out) {
  if (!c || !c->ready) return OR_ESTATE;
  int rc = prepare_query(c);
  if (rc) return rc;
  int64_t N2 = (int64_t)c->nx * c->nv;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < n; ++q) {
    int64_t s = site[q];
    if (s < 0 || s >= N2) {
      f_out[q] = NAN;
      continue;
    }
    int i = (int)(s % c->nx), j = (int)(s / c->nx);
    f_out[q] = scheme == OR_SCHEME_REMAP ? remap_site(c, i, j)
                                         : recon_transport_site(c, i, j, 0, NULL);
  }
  return OR_OK;
}

int or_remap_position(or_ctx *c, int64_t n, const double *P, double *Q) {
  if (!c || !c->ready) return OR_ESTATE;
  int rc = prepare_query(c);
  if (rc) return rc;
  for (int64_t q = 0; q < n; ++q) {
    double Qx = NAN, Qv = NAN;
    remap_position(c, P[2 * q], P[2 * q + 1], &Qx, &Qv);
    Q[2 * q] = Qx;
    Q[2 * q + 1] = Qv;
  }
  return OR_OK;
}

int or_density(or_ctx *c, double *rho_out) {
  if (!c || !c->ready) return OR_ESTATE;
  int rc = prepare_query(c);
  if (rc) return rc;
  reconstruct_all(c, c->f, 0, NULL);
  field_from_f(c, c->f, rho_out);
  return OR_OK;
}

int or_poisson(or_ctx *c, const double *rho, double *a, double *da,
               double *d2a) {
  if (!c) return OR_EINVAL;
  double *M = (double *)calloc(c->nx, sizeof(double));
  if (!M) return OR_ENOMEM;
  for (int i = 0; i < c->nx; ++i) M[i] = c->dx * rho[i];
  cumulative_mass(c, M);
  free(M);
  for (int i = 0; i < c->nx; ++i) {
    a[i] = acc_at(c, i);
    da[i] = dacc_at(c, i);
    d2a[i] = d2acc_at(c, i);
  }
  return OR_OK;
}

/* Neumaier-compensated sum, accurate to a few ulp whatever the order. */
typedef struct {
  double s, c;
} ksum;
static void kadd(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x))
    k->c += (k->s - t) + x;
  else
    k->c += (x - t) + k->s;
  k->s = t;
}
static double kval(const ksum *k) { return k->s + k->c; }

/* Diagnostics of section 3.2 at the current time: mass, kinetic and
 * potential energy E = 1/2 int v^2 f - 1/(4G) int (a^2 - G^2 M_tot^2) dx,
 * the Casimir S = -int f log|f|, max |det T - 1| (eq. detJ), and the L1
 * and L2 norms of f that section 3.2 also monitors, int |f| and
 * (int f^2)^(1/2), every integral a sum over the sites times dx dv.
 * out9 = {mass, E_kin, E_pot, E, S, maxdet, t, L1, L2}. */
int or_diagnostics(or_ctx *c, double *out9) {
  if (!c || !c->ready) return OR_ESTATE;
  int rc = prepare_query(c);
  if (rc) return rc;
  reconstruct_all(c, c->f, 0, NULL);
  field_from_f(c, c->f, NULL);
  int nx = c->nx, nv = c->nv;
  ksum kin = {0, 0}, ent = {0, 0}, pot = {0, 0}, l1 = {0, 0}, l2 = {0, 0};
  for (int j = 0; j < nv; ++j) {
    double v = site_v(c, j);
    for (int i = 0; i < nx; ++i) {
      double f = c->f[(size_t)j * nx + i];
      kadd(&kin, v * v * f);
      if (f != 0.0) kadd(&ent, f * log(fabs(f)));
      kadd(&l1, fabs(f));
      kadd(&l2, f * f);
    }
  }
  double cell = c->dx * c->dv;
  double ekin = 0.5 * kval(&kin) * cell;
  double epot = 0.0;
  if (c->p.force_mode == OR_FORCE_SELF) {
    if (c->p.G != 0.0) {
      /* periodic: the field energy of the zero-mean force (R23) */
      double GM = c->per ? 0.0 : c->p.G * c->Mtot;
      for (int i = 0; i < nx; ++i) {
        double a = acc_at(c, i);
        kadd(&pot, a * a - GM * GM);
      }
      epot = -kval(&pot) * c->dx / (4.0 * c->p.G);
    }
  } else {
    /* external potential phi = -(a0 x + a1 x^2/2 + a2 x^3/3) */
    for (int i = 0; i < nx; ++i) {
      double x = site_x(c, i);
      double phi = -(x * (c->p.ext_a0 + x * (0.5 * c->p.ext_a1 +
                                             x * (c->p.ext_a2 / 3.0))));
      kadd(&pot, phi * c->S[i]);
    }
    epot = kval(&pot) * cell;
  }
  double maxdet = 0.0;
  for (int e = 0; e < c->E; ++e) {
    double det = ST(c, TXX, e) * ST(c, TVV, e) - ST(c, TXV, e) * ST(c, TVX, e);
    double dd = fabs(det - 1.0);
    if (dd > maxdet) maxdet = dd;
  }
  out9[0] = c->Mtot;
  out9[1] = ekin;
  out9[2] = epot;
  out9[3] = ekin + epot;
  out9[4] = -kval(&ent) * cell;
  out9[5] = maxdet;
  out9[6] = c->t;
  out9[7] = kval(&l1) * cell;
  out9[8] = sqrt(kval(&l2) * cell);
  return OR_OK;
}

int or_get_elements(or_ctx *c, double *out) {
  if (!c) return OR_EINVAL;
  memcpy(out, c->el, sizeof(double) * (size_t)NSTATE * c->E);
  return OR_OK;
}

int or_set_elements(or_ctx *c, const double *in) {
  if (!c) return OR_EINVAL;
  memcpy(c->el, in, sizeof(double) * (size_t)NSTATE * c->E);
  return OR_OK;
}

int or_get_assignment(or_ctx *c, int brute, int32_t *out) {
  if (!c) return OR_EINVAL;
  int rc = prepare_query(c);
  if (rc) return rc;
  reconstruct_all(c, c->f, brute, out);
  return OR_OK;
}

int or_get_F(or_ctx *c, double *out) {
  if (!c) return OR_EINVAL;
  memcpy(out, c->F, sizeof(double) * (size_t)c->nx * c->nv);
  return OR_OK;
}

int or_get_coeffs(or_ctx *c, double *out) {
  if (!c) return OR_EINVAL;
  memcpy(out, c->C, sizeof(double) * (size_t)c->nx * c->nv);
  return OR_OK;
}

double or_time(const or_ctx *c) { return c ? c->t : 0.0; }
double or_dt(const or_ctx *c) { return c ? c->dt_cur : 0.0; }
int64_t or_stepcount(const or_ctx *c) { return c ? c->step : 0; }

int or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

int or_inverse_map(const double *el12, double dxm, double dvm, double xP,
                   double vP, double *out4) {
  double txx = el12[TXX], txv = el12[TXV], tvx = el12[TVX], tvv = el12[TVV];
  double det = fma(txx, tvv, -(txv * tvx));
  double inv = 1.0 / det;
  double dqx, dqv;
  int valid = inv_map(el12[SX_], el12[SV_], tvv * inv, -txv * inv, -tvx * inv,
                      txx * inv, el12 + HXXX, dxm, dvm, xP, vP, 0.0, &dqx,
                      &dqv);
  out4[0] = dqx;
  out4[1] = dqv;
  out4[2] = (double)valid;
  out4[3] = det;
  return OR_OK;
}
