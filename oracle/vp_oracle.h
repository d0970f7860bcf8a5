/*
 * vp_oracle.h -- plain CPU FP64 oracle of the metric semi-Lagrangian
 * Vlasov-Poisson method (Colombi & Alard, arXiv:1705.03750).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg are the only users.  It shares no code, header, table or
 * helper with the HIP engine and must never be reached from the product path.
 *
 * Conventions (shared with the engine only through their common definition):
 *   sites   x_i = x_min + (i + 1/2) dx, i = 0..nx-1 (same for v); arrays are
 *           [nv][nx] row-major (v rows, x fastest).
 *   element (k, l), id e = l*mx + k, sits on site (sx*k + sx/2, sv*l + sv/2).
 *   element state, SoA, 12 arrays of E doubles in this order:
 *           x, v, Txx, Txv, Tvx, Tvv, Hx_xx, Hx_xv, Hx_vv, Hv_xx, Hv_xv, Hv_vv
 *           with T_ab = dP_a/dQ_b and H_a[bc] = d2 P_a / dQ_b dQ_c.
 */
#ifndef VP_ORACLE_H
#define VP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_ESTATE (-4)
#define OR_ENUMERIC (-5)

#define OR_FORCE_SELF 0
#define OR_FORCE_EXTERNAL 1

#define OR_BC_ISOLATED 0
#define OR_BC_PERIODIC 1

#define OR_SCHEME_TRANSPORT 0
#define OR_SCHEME_REMAP 1

typedef struct or_params {
  int32_t nx, nv;
  double x_min, x_max, v_min, v_max;
  int32_t sx, sv;
  double G;
  double dt;
  int32_t n_s;
  double beta;
  int32_t force_mode;
  double ext_a0, ext_a1, ext_a2;
  double emap_max;     /* adaptive remap threshold on E_map (<= 0: off) */
  int32_t emap_every;  /* steps between E_map checks (adaptive remap) */
  double cdyn;         /* variable step dt <= cdyn / sqrt(rho_max) (<= 0:
                          fixed dt); self-consistent force only */
  int32_t bc;          /* OR_BC_ISOLATED or OR_BC_PERIODIC (x periodic, force
                          against a uniform background; self force only) */
} or_params;

typedef struct or_ctx or_ctx;

or_ctx *or_create(const or_params *p);
void or_destroy(or_ctx *c);
int or_init_conditions(or_ctx *c, const double *f0);
int or_step(or_ctx *c, int nsteps);
int or_remap(or_ctx *c);
int or_reconstruct_f(or_ctx *c, int scheme, double *f_out);
int or_reconstruct_sites(or_ctx *c, int scheme, int64_t n, const int64_t *site,
                         double *f_out);
int or_remap_position(or_ctx *c, int64_t n, const double *P, double *Q);
int or_density(or_ctx *c, double *rho_out);
int or_poisson(or_ctx *c, const double *rho, double *a, double *da,
               double *d2a);
int or_diagnostics(or_ctx *c, double *out9);
int or_emap(or_ctx *c, double *emap);
int or_get_elements(or_ctx *c, double *out);
int or_set_elements(or_ctx *c, const double *in);
int or_get_assignment(or_ctx *c, int brute, int32_t *out);
int or_get_F(or_ctx *c, double *out);
int or_get_coeffs(or_ctx *c, double *out);
double or_time(const or_ctx *c);
double or_dt(const or_ctx *c);
int64_t or_stepcount(const or_ctx *c);
int or_set_threads(int n);

/* primitives, exposed for the pins */
double or_int1(const double *F, int nx, int nv, double sx, double sv);
double or_int1_periodic(const double *F, int nx, int nv, double sx,
                        double sv);
double or_W(double x);
int or_spline_fit(int nx, int nv, const double *F, double *C);
int or_spline_fit_periodic(int nx, int nv, const double *F, double *C);
double or_spline_eval_periodic(const double *C, int nx, int nv, double sx,
                               double sv);
double or_spline_eval(const double *C, int nx, int nv, double sx, double sv);
int or_inverse_map(const double *el12, double dxm, double dvm, double xP,
                   double vP, double *out4);
double or_tsc(const double *g, int n, double u);

#ifdef __cplusplus
}
#endif
#endif
