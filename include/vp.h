/*
 * vp.h -- C ABI of the MI355X engine for the metric semi-Lagrangian
 * Vlasov-Poisson method of Colombi & Alard, "A 'metric' semi-Lagrangian
 * Vlasov-Poisson solver" (arXiv:1705.03750), 2D phase space (x, v),
 * self-gravitating 1D systems.
 *
 * Problem statement (section 1 and section 2 of the paper): f(x, v, t) is
 * sampled on a fixed Eulerian grid; a sparse lattice of "metric elements"
 * follows the flow with its position P_m, deformation tensor T_m = dP/dQ and
 * Hessian H_m = d2P/dQ2 (section 2.1).  The value at a site P is the initial
 * condition F_ini interpolated at Q(P), obtained from the closest element by
 * the second-order inverse map (eq. QofP).  Elements advance with a
 * drift-kick-drift leapfrog (section 2.4) under the force of the 1D Poisson
 * equation computed as a cumulative mass sum (section 2.5, eq. acccomp).
 * Every n_s steps f becomes the new initial condition (resampling, with
 * cubic B-splines and a W-weighted blend of neighbour predictions, sections
 * 2.2.2 and 2.3.2).
 *
 * Grid and layout:
 *   sites   x_i = x_min + (i + 1/2) dx, dx = (x_max - x_min)/nx, same for v.
 *   f       nv rows of nx values, row-major: f[j*nx + i] (v rows, x fastest).
 *   elements (k, l), id e = l*mx + k with mx = nx/sx, sit on site
 *           (sx*k + sx/2, sv*l + sv/2) when (re)created.
 *   element state (test hooks): SoA, 12 arrays of E = mx*mv doubles, in the
 *           order x, v, Txx, Txv, Tvx, Tvv, Hx_xx, Hx_xv, Hx_vv, Hv_xx,
 *           Hv_xv, Hv_vv (T_ab = dP_a/dQ_b, H_a[bc] = d2P_a/dQ_b dQ_c).
 *
 * Precision: VP_FP64 keeps everything in double.  VP_MIXED stores F_ini,
 * the spline coefficients and f in float and interpolates in float; element
 * state, the nearest-element query, Q, the mass sums and the force stay in
 * double.
 *
 * Memory and streams: the library allocates no device memory.  The caller
 * passes one device workspace of vp_footprint() bytes (any allocator, e.g. a
 * torch uint8 tensor) and a HIP stream; every call enqueues its work on that
 * stream and returns without waiting unless stated.  One exception: the
 * spline fit that follows a resampling inside vp_step runs on a stream the
 * context creates (default priority), overlapped with the following steps,
 * which read F_ini but not the coefficients; the context's stream waits for
 * it before the coefficients are next read or restaged (the next
 * resampling, vp_reconstruct_f scheme 1, vp_init_conditions) and in
 * vp_sync, vp_prof_end and vp_destroy.  While the context's stream is being
 * captured into a graph the fit stays on it.  Pointers named "dev" are
 * device pointers; "host" ones are host pointers.  The caller keeps the
 * workspace alive until vp_destroy.  One host thread per context at a time.
 *
 * Errors: every call returns a status.  No exception crosses the ABI.
 *   VP_OK 0, VP_EINVAL -1 (bad argument or parameters), VP_ENOMEM -2
 *   (workspace too small), VP_EDEVICE -3 (HIP error; text in
 *   vp_last_error), VP_ESTATE -4
 *   (call before vp_init_conditions), VP_ENUMERIC -5 (a non-finite element
 *   or det T <= 0 met on the device).  Conditions found on the device are
 *   reported by the next synchronising call: vp_sync, vp_diagnostics.
 */
#ifndef VP_H
#define VP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VP_OK 0
#define VP_EINVAL (-1)
#define VP_ENOMEM (-2)
#define VP_EDEVICE (-3)
#define VP_ESTATE (-4)
#define VP_ENUMERIC (-5)

#define VP_FP64 0
#define VP_MIXED 1

#define VP_FORCE_SELF 0     /* a = G (M_right - M_left), eq. acccomp */
#define VP_FORCE_EXTERNAL 1 /* a = a0 + a1 x + a2 x^2 (closed-form tests) */

#define VP_BC_ISOLATED 0 /* isolated system in a fixed box (section 2.5) */
#define VP_BC_PERIODIC 1 /* x periodic: plasma (G < 0) or periodic gravity */

#define VP_SCHEME_TRANSPORT 0 /* nearest element + six-point interpolation */
#define VP_SCHEME_REMAP 1     /* W-blended Q_r + cubic B-spline */

typedef struct vp_params {
  int32_t nx, nv;      /* sites per axis, >= 8, multiples of sx / sv;
                          nx also a multiple of 4 */
  double x_min, x_max; /* phase-space box */
  double v_min, v_max;
  int32_t sx, sv;      /* element spacing in sites (dx_m = sx dx); at most
                          2^30 elements (nx/sx)(nv/sv) */
  double G;            /* coupling: a(i) = G (M_tot - M_left(i) - M_left(i-1)) */
  double dt;           /* time step, > 0 */
  int32_t n_s;         /* steps between resamplings, 0 = never */
  double beta;         /* remap neighbour margin, section 2.3.3; the paper's
                          value is (1 - sqrt(3)/2)/2 */
  int32_t force_mode;  /* VP_FORCE_SELF or VP_FORCE_EXTERNAL */
  double ext_a0, ext_a1, ext_a2; /* external force coefficients */
  int32_t precision;   /* VP_FP64 or VP_MIXED */
  double emap_max;     /* adaptive resampling (end of section 2.3.3): every
                          emap_every steps, resample when E_map (vp_diag)
                          exceeds emap_max; <= 0 disables.  Independent of
                          the fixed cadence n_s.  Not accepted by the
                          serving loop. */
  int32_t emap_every;  /* steps between E_map checks, >= 1 when enabled */
  double c_dyn;        /* variable time step (section 2.4): > 0 makes every
                          step min(dt, c_dyn / sqrt(rho_max)), rho_max the
                          largest projected density -- of F_ini for the
                          first step, of the previous step's half-step
                          reconstruction after that; dt is then the cap.
                          0 = fixed dt.  Self-consistent force only; not
                          accepted by the serving loop.  Step sizes and t
                          stay on the device (vp_time and vp_diagnostics
                          synchronise to read them). */
  int32_t bc;          /* VP_BC_ISOLATED, or VP_BC_PERIODIC: x periodic with
                          period x_max - x_min (the paper notes that its
                          Poisson solve carries over to periodic systems and
                          the method to plasmas, section 2.5 and the
                          conclusions).  The force is that of the ring
                          against a uniform background of the same mass,
                          a(i) = G (B(i) - mean B), B(i) = M_tot (2i+1)/nx -
                          M_left(i) - M_left(i-1): G > 0 gravitating, G < 0
                          repelling (G = -1/2 with mean density 1 is the
                          electron plasma, da/dx = rho - 1).  Elements
                          re-enter the box after each drift and are seen
                          through their nearest image; F_ini and the spline
                          repeat in x; only the v edge rows are zeroed.
                          Requires VP_FORCE_SELF and nx a multiple of 8;
                          element positions passed to vp_set_elements must
                          lie in [x_min, x_max).  Not accepted by the
                          serving loop. */
} vp_params;

typedef struct vp_diag {
  double mass;        /* dx dv sum f (section 3.2) */
  double e_kin;       /* 1/2 sum v^2 f dx dv */
  double e_pot;       /* -1/(4G) sum (a^2 - G^2 M_tot^2) dx (self gravity),
                         -1/(4G) sum a^2 dx (periodic x: the field energy,
                         1/2 sum E^2 dx for the plasma) or sum phi_ext rho
                         dx (external force) */
  double energy;      /* e_kin + e_pot */
  double entropy;     /* Casimir S = -sum f ln|f| dx dv, f != 0 */
  double max_det_dev; /* max over elements of |det T - 1| (eq. detJ) */
  double t;           /* current time */
  int64_t step;       /* steps taken since vp_init_conditions */
  int64_t overflow_blocks; /* query blocks that fell back to a full scan */
  double emap;        /* E_map (end of section 2.3.3): the largest Lagrangian
                         distance, in element spacings, between the position
                         Q predicted at a site by its nearest element and by
                         one of that element's four lattice neighbours whose
                         validity window holds the site */
  double dt;          /* size of the next step (dt unless c_dyn > 0) */
  double l1;          /* L1 norm of f, dx dv sum |f| (section 3.2 also
                         monitors the L1 and L2 norms) */
  double l2;          /* L2 norm of f, (dx dv sum f^2)^(1/2) */
} vp_diag;

typedef struct vp_ctx vp_ctx;

/* Device bytes a run with these parameters needs.  Pure.  EINVAL on bad
 * parameters. */
int vp_footprint(const vp_params *p, size_t *bytes);

/* Bind a run to caller-owned device memory (dev_workspace, `bytes` >=
 * vp_footprint) and a HIP stream (hipStream_t, may be 0).  *out receives an
 * opaque context owned by the library.  Enqueues table set-up on the
 * stream. */
int vp_create(const vp_params *p, void *dev_workspace, size_t bytes,
              void *hip_stream, vp_ctx **out);

/* Release the context (not the workspace).  Synchronises the stream. */
int vp_destroy(vp_ctx *ctx);

/* New initial condition (section 1): f0 is nv*nx doubles, row-major, on the
 * device when f0_on_device != 0 (read before the stream reaches the next
 * call) or on the host (copied before return).  The outermost ring of sites
 * is zeroed (f = 0 and df = 0 on the box edges, section 2.2.2), F_ini is
 * stored (as float in VP_MIXED), the cubic B-spline is fitted, elements are
 * reset to P = Q_m, T = I, H = 0, and t = 0. */
int vp_init_conditions(vp_ctx *ctx, const double *f0, int f0_on_device);

/* nsteps drift-kick-drift steps (section 2.4): predictor drift, f at the
 * half step from the drifted elements, density, force, kick, corrector
 * drift; a resampling after every step whose count is a multiple of n_s. */
int vp_step(vp_ctx *ctx, int nsteps);

/* Resample now (sections 1 and 2.3.2): f from the W-blended Q_r and the
 * cubic spline becomes F_ini; new isotropic elements. */
int vp_remap(vp_ctx *ctx);

/* f at the current time on every site; state unchanged.  Scheme
 * VP_SCHEME_TRANSPORT: the nearest element's second-order inverse map
 * (section 2.1, eq. QofP) and the six-point interpolation of F_ini (section
 * 2.2.1, eq. int1); VP_SCHEME_REMAP: the W-weighted blend Q_r of the
 * neighbours' predictions (section 2.3.2) and the cubic B-spline of F_ini
 * (section 2.2.2), the values a resampling would store.  f_out_dev: nv*nx
 * device values (caller owned), row-major, double (float in VP_MIXED).
 * EINVAL for a bad scheme or null pointer, ESTATE before
 * vp_init_conditions.  Asynchronous. */
int vp_reconstruct_f(vp_ctx *ctx, int scheme, void *f_out_dev);

/* Projected density rho(x_i) = dv sum_j f(i, j) of the transport
 * reconstruction at the current time (section 2.5).  rho_out_dev: nx
 * device doubles. */
int vp_density(vp_ctx *ctx, double *rho_out_dev);

/* 1D Poisson solve of eq. (acccomp) with the finite-difference derivatives
 * of section 2.5, from a density: M(i) = dx rho(i), a(i) = G (M_tot -
 * M_left(i) - M_left(i-1)), a' centred over 2 dx, a'' the three-point second
 * difference.  All pointers: nx device doubles.  Pure (state unchanged). */
int vp_poisson(vp_ctx *ctx, const double *rho_dev, double *a_dev,
               double *da_dev, double *d2a_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the force
 * of vp_poisson for a density without a run context or a workspace.
 * p: the run parameters (only nx, x_min, x_max, G and bc enter; the whole
 * struct must pass the checks of vp_create).  rho_dev: nx device doubles
 * (read); a_dev, da_dev, d2a_dev: nx device doubles each (written, caller
 * owned).  Work is enqueued on hip_stream (NULL: the null stream) and the
 * call returns without waiting.  The intermediate sums live in one
 * library-owned device array of VP_POISSON_STATIC_BYTES per GPU, taken when
 * the library is loaded and held until the process ends; every call on a
 * GPU shares that array and leaves the last call's contents in it, so calls
 * that overlap on one GPU (two streams, two host threads) race.  Results
 * are bit for bit those of vp_poisson.  Errors: VP_EINVAL for invalid
 * parameters, a null pointer or nx > VP_POISSON_STATIC_MAX_NX; VP_EDEVICE
 * on a HIP error; text of either in vp_last_error(NULL). */
#define VP_POISSON_STATIC_MAX_NX 16384
#define VP_POISSON_STATIC_BYTES ((size_t)8 * (5 * 16384 + 24 + 2 * 2048 + 32))
int vp_poisson_static(const vp_params *p, const double *rho_dev,
                      double *a_dev, double *da_dev, double *d2a_dev,
                      void *hip_stream);

/* Diagnostics of section 3.2 at the current time (synchronises). */
int vp_diagnostics(vp_ctx *ctx, vp_diag *out_host);

/* Test hooks: export / inject the element state (12*E device doubles, SoA,
 * order as above) and export the nearest-element id of every site (nv*nx
 * device int32, -1 where no element is valid) for the current state. */
int vp_get_elements(vp_ctx *ctx, double *el_dev);
int vp_set_elements(vp_ctx *ctx, const double *el_dev);
int vp_get_assignment(vp_ctx *ctx, int32_t *assign_dev);

/* Time and step count.  Host values without synchronisation for a fixed
 * step; with c_dyn > 0 the time is read from the device (synchronises). */
int vp_time(vp_ctx *ctx, double *t, int64_t *step);

/* Profiling hooks.  vp_prof_begin makes every later launch of the engine
 * record a pair of HIP events on the stream it runs on (the context's, or
 * for the spline fit after a resampling the context's fit stream; at most
 * max_launches launches per kernel kind); vp_prof_end waits for both and
 * writes,
 * for each kernel kind k in [0, VP_PROF_KINDS), the summed elapsed time in
 * milliseconds (ms_host[k]) and the number of timed launches (n_host[k]),
 * then releases the events.  Kinds: 0 element predictor/record, 1 the
 * transport reconstruction (k_recon; also its E_map-only form in the
 * adaptive resampling check), 2 force, 3 kick, 4 remap evaluation, 5 spline
 * fit, 6 element reset, 7 other.  Returns VP_EDEVICE if events cannot be
 * created. */
#define VP_PROF_KINDS 8
int vp_prof_begin(vp_ctx *ctx, int max_launches);
int vp_prof_end(vp_ctx *ctx, double *ms_host, int64_t *n_host);

/* ---------------------------------------------------------------- serving
 * Continuous batching of independent runs (different grids, element
 * strides, step counts) on one device.  Requests arrive over time; a request
 * is admitted (FIFO) as soon as a run slot is free and its vp_footprint fits
 * in the unused part of the server's device pool; its state (F_ini, spline,
 * elements) stays resident until it completes.  Every tick advances all
 * admitted runs by one step with one fixed sequence of batched launches
 * (captured once as a HIP graph and replayed); a run's arithmetic is the
 * same as a run alone (vp_step, then vp_reconstruct_f with the transport
 * scheme), so its output is bitwise the same alone or in any mix. */
typedef struct vp_server vp_server;

typedef struct vp_request {
  vp_params params;     /* precision must equal the server's */
  const double *f0_dev; /* nv*nx device doubles; read when admitted */
  void *f_out_dev;      /* nv*nx device values (float in VP_MIXED): f after
                           nsteps (transport reconstruction) */
  int32_t nsteps;       /* >= 1 */
  int32_t pad;
  int64_t tag;
  double arrival_s;     /* seconds after vp_server_run starts; ascending */
} vp_request;

typedef struct vp_request_result {
  int64_t tag;
  double arrival_s, admit_s, done_s; /* seconds after the start */
  int32_t status;                    /* VP_OK, or the admission error */
  int32_t pad;
} vp_request_result;

typedef struct vp_server_stats {
  double wall_s;        /* first arrival to last completion */
  double gpu_busy_s;    /* device time of all ticks (HIP events) */
  int64_t ticks, site_updates, admitted, completed;
  int32_t max_active;   /* most runs resident at once */
  int32_t graph_replay; /* 1 when ticks ran as HIP graph replays */
} vp_server_stats;

/* Device bytes the server keeps at the head of its pool for run and work
 * tables (the rest holds the runs' workspaces). */
int vp_server_footprint(int precision, size_t *bytes);

/* Server over caller-owned device memory dev_pool (pool_bytes > the
 * footprint above), at most max_active (1..128) resident runs, all of one
 * precision.  hip_stream: the caller's stream, ordered before and after
 * each vp_server_run (the server runs on a stream of its own). */
int vp_server_create(int precision, int max_active, void *dev_pool,
                     size_t pool_bytes, void *hip_stream, vp_server **out);

/* Serve n requests (ascending arrival_s) to completion, in real time:
 * requests become eligible at their arrival time, are admitted as memory
 * and slots free up, and complete when their last step's results are on
 * the device.  res[i] describes reqs[i].  Returns when all are done. */
int vp_server_run(vp_server *srv, const vp_request *reqs, int n,
                  vp_request_result *res, vp_server_stats *stats);

int vp_server_destroy(vp_server *srv);
const char *vp_server_last_error(vp_server *srv);

/* Wait for the stream; report a pending device-side VP_ENUMERIC. */
int vp_sync(vp_ctx *ctx);

/* Text of the last error on this context (or, when ctx is NULL, of the
 * last failed vp_create or vp_poisson_static on this host thread). */
const char *vp_last_error(vp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
