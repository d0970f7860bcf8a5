/*
 * vp4.h -- C ABI of the MI355X engine for the metric semi-Lagrangian
 * Vlasov-Poisson method (Colombi & Alard, arXiv:1705.03750) in 4D phase
 * space: 2D periodic space (x, y) x 2D velocity (u, w).
 *
 * The paper develops the method in 2D phase space and describes the
 * generalisation: 4 + 16 + 40 = 60 numbers per element (section 2.1: P, the
 * deformation tensor T = dP/dQ and the 40 independent Hessian terms), the
 * 15-point second-order interpolation (section 2.2.1), and an FFT solution
 * of Poisson's equation for periodic systems (section 2.5).  Here:
 *   force    div a = -2 G (rho - rho_bar) on the periodic square (G < 0: a
 *            plasma, G = -1/2 with mean density 1 gives div a = rho - 1),
 *            rho(x, y) = du dw sum_{u, w} f, solved by the discrete Fourier
 *            transform; gradient and Hessian of a by centred differences;
 *            element force by the 3 x 3 dual TSC;
 *   step     drift dt/2, f at the half step, force, kick, drift dt/2
 *            (section 2.4 per component); resampling every n_s steps with
 *            the W-blended Q_r and the tensor cubic spline (x, y periodic,
 *            u, w with the zero-slope edges of section 2.2.2).
 *
 * Grid and layout:
 *   sites    x_i = (i + 1/2) dx, dx = L / ns (y alike), u_k = -vmax +
 *            (k + 1/2) du, du = 2 vmax / nv (w alike);
 *   f        f[((l * nv + k) * ns + j) * ns + i]: x fastest, then y, u, w;
 *   elements (ex, ey, eu, ew), id ((ew * mv + eu) * ms + ey) * ms + ex,
 *            created on site (ss ex + ss/2, ss ey + ss/2, sv eu + sv/2,
 *            sv ew + sv/2), ms = ns / ss, mv = nv / sv;
 *   state    SoA [60][E] doubles: P (x, y, u, w); T[a][b] row major (16);
 *            H[a][bc] for b <= c in the order 00 01 02 03 11 12 13 22 23 33
 *            (4 x 10).
 *
 * Precision: VP4_FP64 keeps everything in double; VP4_MIXED stores F_ini,
 * the spline coefficients and f in float and interpolates in float
 * (elements, query, Q, density and force in double).
 *
 * Memory, streams, errors: as the 2D engine (vp.h): the caller passes one
 * device workspace of vp4_footprint() bytes and a HIP stream; work is
 * enqueued on the stream; statuses VP4_OK 0, VP4_EINVAL -1, VP4_ENOMEM -2,
 * VP4_EDEVICE -3, VP4_ESTATE -4, VP4_ENUMERIC -5 (a non-finite element or
 * det T <= 0 met on the device, reported by vp4_sync / vp4_diagnostics).
 */
#ifndef VP4_H
#define VP4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VP4_OK 0
#define VP4_EINVAL (-1)
#define VP4_ENOMEM (-2)
#define VP4_EDEVICE (-3)
#define VP4_ESTATE (-4)
#define VP4_ENUMERIC (-5)

#define VP4_FP64 0
#define VP4_MIXED 1

typedef struct vp4_params {
  int32_t ns, nv;   /* sites per space axis, per velocity axis: multiples of
                       4 and of ss / sv; ns >= 8, nv >= 4, ns <= 512 */
  double L;         /* period of x and y, > 0 */
  double vmax;      /* velocities in [-vmax, vmax), > 0 */
  int32_t ss, sv;   /* element spacing in sites */
  double G;         /* div a = -2 G (rho - rho_bar) */
  double dt;        /* time step, > 0 */
  int32_t n_s;      /* steps between resamplings, 0 = never */
  double beta;      /* remap neighbour margin (section 2.3.3), in [0, 1/2] */
  int32_t precision;/* VP4_FP64 or VP4_MIXED */
} vp4_params;

typedef struct vp4_ctx vp4_ctx;

/* Device bytes a run needs.  Pure.  EINVAL on bad parameters. */
int vp4_footprint(const vp4_params *p, size_t *bytes);

/* Bind a run to caller-owned device memory (>= vp4_footprint bytes,
 * 256-byte aligned) and a HIP stream (may be 0). */
int vp4_create(const vp4_params *p, void *dev_workspace, size_t bytes,
               void *hip_stream, vp4_ctx **out);

/* Release the context (not the workspace); synchronises the stream. */
int vp4_destroy(vp4_ctx *ctx);

/* New initial condition (section 1): f0_dev holds ns^2 nv^2 device doubles
 * in the layout above, read before the stream reaches the next call.  The
 * u and w edge rows are zeroed, the spline is fitted, the elements are reset
 * (P = Q_m, T = I, H = 0) and t = 0. */
int vp4_init_conditions(vp4_ctx *ctx, const double *f0_dev);

/* nsteps leapfrog steps with resampling every n_s steps. */
int vp4_step(vp4_ctx *ctx, int nsteps);

/* Resample now. */
int vp4_remap(vp4_ctx *ctx);

/* f at the current time on every site: scheme 0 the transport
 * reconstruction (nearest element, 15-point interpolation), 1 the remap
 * reconstruction (blended Q_r, tensor spline).  f_out_dev: ns^2 nv^2 device
 * values, double (float in VP4_MIXED). */
int vp4_reconstruct_f(vp4_ctx *ctx, int scheme, void *f_out_dev);

/* rho(x, y) of the transport reconstruction at the current time: ns^2
 * device doubles, y rows of x values. */
int vp4_density(vp4_ctx *ctx, double *rho_dev);

/* The force of a density (ns^2 device doubles): a_x, a_y (ns^2 device
 * doubles each).  State unchanged. */
int vp4_field(vp4_ctx *ctx, const double *rho_dev, double *ax_dev,
              double *ay_dev);

/* mass, kinetic energy, field energy -(1/4G) sum |a|^2 dx dy, total energy,
 * entropy -sum f ln|f| dV, t: 6 host doubles.  Synchronises. */
int vp4_diagnostics(vp4_ctx *ctx, double *out6_host);

/* Test hooks: element state (60 E device doubles, SoA) and the nearest
 * element id of every site (ns^2 nv^2 device int32, -1 where none). */
int vp4_get_elements(vp4_ctx *ctx, double *el_dev);
int vp4_set_elements(vp4_ctx *ctx, const double *el_dev);
int vp4_get_assignment(vp4_ctx *ctx, int32_t *assign_dev);

/* Profiling: per kernel kind (0 predict + lists, 1 reconstruction, 2 field,
 * 3 kick, 4 remap evaluation, 5 spline fit, 6 other) summed milliseconds and
 * launch counts between vp4_prof_begin and vp4_prof_end (HIP events on the
 * context's stream). */
#define VP4_PROF_KINDS 7
int vp4_prof_begin(vp4_ctx *ctx, int max_launches);
int vp4_prof_end(vp4_ctx *ctx, double *ms_host, int64_t *n_host);

/* Wait for the stream; report a pending device-side VP4_ENUMERIC. */
int vp4_sync(vp4_ctx *ctx);

/* Text of the last error on this context (NULL: of the last failed
 * create). */
const char *vp4_last_error(vp4_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
