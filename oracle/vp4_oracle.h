/*
 * vp4_oracle.h -- plain CPU FP64 oracle of the metric semi-Lagrangian method
 * in 4D phase space (x, y, u, w): 2D periodic space, 2D velocity (Colombi &
 * Alard, arXiv:1705.03750, the generalisation the paper describes in
 * sections 2.1, 2.2.1 and 2.5).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only users.  It shares no code with the HIP
 * engine and must never be reached from the product path.
 *
 * Conventions:
 *   sites    x_i = (i + 1/2) dx, dx = L / ns (same for y), periodic;
 *            u_k = -vmax + (k + 1/2) du, du = 2 vmax / nv (same for w).
 *   arrays   f[((l * nv + k) * ns + j) * ns + i] (x fastest, then y, u, w).
 *   elements (ex, ey, eu, ew), id e = ((ew * mv + eu) * ms + ey) * ms + ex,
 *            created on site (ss ex + ss/2, ss ey + ss/2, sv eu + sv/2,
 *            sv ew + sv/2); ms = ns / ss, mv = nv / sv.
 *   state    SoA [60][E]: P (x, y, u, w), T[a][b] = dP_a/dQ_b (16, row
 *            major), H[a][bc] = d2 P_a / dQ_b dQ_c for b <= c (4 x 10, the
 *            pairs in the order 00 01 02 03 11 12 13 22 23 33).
 */
#ifndef VP4_ORACLE_H
#define VP4_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or4_params {
  int32_t ns, nv;  /* sites per space axis, per velocity axis */
  double L;        /* period of x and y */
  double vmax;     /* velocities in [-vmax, vmax) */
  int32_t ss, sv;  /* element spacing in sites (space, velocity) */
  double G;        /* div a = -2 G (rho - rho_bar) */
  double dt;
  int32_t n_s;     /* steps between resamplings, 0 = never */
  double beta;     /* remap neighbour margin (section 2.3.3) */
} or4_params;

typedef struct or4_ctx or4_ctx;

or4_ctx *or4_create(const or4_params *p);
void or4_destroy(or4_ctx *c);
int or4_init_conditions(or4_ctx *c, const double *f0);
int or4_step(or4_ctx *c, int nsteps);
int or4_remap(or4_ctx *c);
int or4_reconstruct_f(or4_ctx *c, int scheme, double *f_out);
int or4_density(or4_ctx *c, double *rho_out);
int or4_field(or4_ctx *c, const double *rho, double *ax, double *ay);
int or4_diagnostics(or4_ctx *c, double *out6);
int or4_get_elements(or4_ctx *c, double *out);
int or4_set_elements(or4_ctx *c, const double *in);
int or4_get_assignment(or4_ctx *c, int brute, int32_t *out);
double or4_time(const or4_ctx *c);

/* primitives, exposed for the pins */
double or4_int15(const double *F, int ns, int nv, const double *s4);
int or4_spline_fit(int ns, int nv, const double *F, double *C);
double or4_spline_eval(const double *C, int ns, int nv, const double *s4);
int or4_inverse_map(const double *el60, const double *d4, const double *P4,
                    double L, double *out6);

#ifdef __cplusplus
}
#endif
#endif
