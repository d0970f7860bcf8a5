// vp_engine.hip -- host side of the MI355X engine: workspace carving, step
// sequencing on the caller's stream, and the C ABI declared in vp.h.
//
// Every step runs k_recon (nearest element, inverse map, six-point
// interpolation, row-group column partials) and then the element pass: on
// grids of at most 2048 columns k_field_chunks (column sums, chunks of the
// cumulative mass) and k_elem_window (carries and force, then TSC, kick,
// corrector drift, the next predictor drift, A = T^-1 and the query-block
// lists), else k_field and k_field_tail (the field) followed by k_elem.  A run's first step, and
// the first after a resampling, starts with k_elem (predictor and lists).
// Every n_s steps the resampling: k_remap_eval, the spline fit (k_fit_x or
// k_fit_x_cyclic, k_fit_v, ghosts) on a second stream beside the following
// steps, k_elem_reset.  Nothing is allocated: all buffers live in the
// caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "vp.h"
#include "vp_batch.hpp"
#include "vp_kernels.hpp"

#include <chrono>
#include <map>
#include <mutex>
#include <thread>

using namespace vpk;

namespace {

thread_local std::string g_create_error;

struct Layout {
  size_t F, C, T, st, rec, qm, cnt, lst, flags, ovf, part, fcnt, Mc, ctot,
      rmx, clk, Ml, acc,
      dpart, dout, tab, total;
  size_t fbytes;  // bytes per f value
  long long nb;
  int nwg_x, nwg_y;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool params_ok(const vp_params *p) {
  return p && p->nx >= 8 && p->nv >= 8 && p->nx % 4 == 0 && p->sx >= 1 &&
         p->sv >= 1 &&
         p->nx % p->sx == 0 && p->nv % p->sv == 0 && p->dt > 0.0 &&
         p->x_max > p->x_min && p->v_max > p->v_min && p->n_s >= 0 &&
         p->beta >= 0.0 && p->beta <= 0.5 &&
         (p->precision == VP_FP64 || p->precision == VP_MIXED) &&
         (p->force_mode == VP_FORCE_SELF ||
          p->force_mode == VP_FORCE_EXTERNAL) &&
         std::isfinite(p->G) && p->nx <= (1 << 17) && p->nv <= (1 << 17) &&
         (int64_t)(p->nx / p->sx) * (p->nv / p->sv) <= (1 << 30) &&
         !(p->emap_max > 0.0 && p->emap_every < 1) && !std::isnan(p->emap_max) &&
         p->c_dyn >= 0.0 && std::isfinite(p->c_dyn) &&
         !(p->c_dyn > 0.0 && p->force_mode != VP_FORCE_SELF) &&
         (p->bc == VP_BC_ISOLATED ||
          (p->bc == VP_BC_PERIODIC && p->force_mode == VP_FORCE_SELF &&
           p->nx % 8 == 0));
}

// list capacity per 8x8 block: about twice the element count whose windows
// reach a block when the lattice is undeformed
int list_cap(int sx, int sv) {
  auto per_axis = [](int s) { return (8 + 2 * s + 2) / s + 2; };
  int c = 2 * per_axis(sx) * per_axis(sv);
  int cap = 16;
  while (cap < c && cap < 256) cap *= 2;
  return cap;
}

KP make_kp(const vp_params *p) {
  KP k{};
  k.nx = p->nx;
  k.nv = p->nv;
  k.sx = p->sx;
  k.sv = p->sv;
  k.mx = p->nx / p->sx;
  k.mv = p->nv / p->sv;
  k.E = k.mx * k.mv;
  k.ox = (p->sx / 2) % 8;
  k.ov = (p->sv / 2) % 8;
  k.obx = 1;  // block columns shift with the element drift (group_ox)
  k.obv = k.ov > 0;
  k.nbx = ((p->nx - 1) >> 3) + 2;  // enough for any offset 0..7
  k.nbv = ((p->nv - 1 - k.ov) >> 3) + k.obv + 1;
  k.ngy = ((p->nv - 1 - k.ov) >> 6) + k.obv + 1;
  k.cap = list_cap(p->sx, p->sv);
  k.pitch = p->nx + 2 * PX;
  k.x_min = p->x_min;
  k.v_min = p->v_min;
  k.dx = (p->x_max - p->x_min) / p->nx;
  k.dv = (p->v_max - p->v_min) / p->nv;
  k.inv_dx = 1.0 / k.dx;
  k.inv_dv = 1.0 / k.dv;
  k.dxm = p->sx * k.dx;
  k.dvm = p->sv * k.dv;
  k.rx = 1.0 / k.dxm;
  k.rv = 1.0 / k.dvm;
  {
    // equal powers of two well inside the normal range: the query may then
    // rank candidates by the unscaled squared offset (the same order)
    int ex = 0;
    const double mant = std::frexp(k.rx, &ex);
    k.r2 = (k.rx == k.rv && mant == 0.5 && ex > -400 && ex < 400) ? 1 : 0;
  }
  // tile index t -> row group t / nbx as (t ceil(2^40 / nbx)) >> 40: exact
  // for every t < nbx ngy when nbx^2 ngy < 2^40 (the rounding excess of the
  // multiplier, below t / 2^40, then stays under 1 / nbx)
  {
    const unsigned long long nbx = (unsigned long long)k.nbx;
    k.tdm = (nbx * nbx * (unsigned long long)k.ngy < (1ull << 40))
                ? ((1ull << 40) + nbx - 1) / nbx
                : 0ull;
  }
  k.G = p->G;
  k.dt = p->dt;
  k.h = 0.5 * p->dt;
  k.beta = p->beta;
  k.force_mode = p->force_mode;
  k.a0 = p->ext_a0;
  k.a1 = p->ext_a1;
  k.a2 = p->ext_a2;
  k.cdyn = p->c_dyn;
  k.clk = nullptr;  // set by vp_create for a variable step
  k.par = 0;
  k.per = p->bc == VP_BC_PERIODIC;
  k.nbl = p->nx / 8;
  k.x_max = p->x_max;
  k.Lx = p->x_max - p->x_min;
  k.hL = 0.5 * k.Lx;
  gox_set(k);
  return k;
}

Layout make_layout(const vp_params *p, const KP &k) {
  Layout L{};
  const size_t fb = (p->precision == VP_MIXED) ? 4 : 8;
  L.fbytes = fb;
  L.nb = (long long)k.nbx * k.nbv;
  L.nwg_x = k.nbx;
  L.nwg_y = k.ngy;
  const size_t padded = (size_t)(k.nv + 2 * PV) * (size_t)k.pitch * fb;
  const size_t N2 = (size_t)k.nx * k.nv;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.F = take(padded);
  L.C = take(padded);
  L.T = take(N2 * fb);
  L.st = take((size_t)NSTATE * k.E * 8);
  L.rec = take((size_t)RS * k.E * 8);
  L.qm = take((size_t)2 * k.E * 8);
  L.cnt = take((size_t)2 * L.nb * 4);  // two count buffers, see vp_ctx::cur
  L.lst = take((size_t)L.nb * k.cap * 4);
  L.flags = take(64);
  L.ovf = take(64);
  L.part = take((size_t)k.ngy * k.nx * 8);
  L.fcnt = take(64);
  L.Mc = take((size_t)k.nx * 8);
  L.ctot = take((size_t)FIELD_CHUNKS * 8);
  L.rmx = take((size_t)FIELD_CHUNKS * 8);  // per-chunk / per-workgroup rho max
  L.clk = take((size_t)CK_DOUBLES * 8);
  L.Ml = take((size_t)k.nx * 8);
  L.acc = take((size_t)3 * (k.nx + 8) * 8);
  L.dpart = take((size_t)DPS * k.nbx * k.ngy * 8);
  L.dout = take(16 * 8);
  // spline tables: x pivots, v pivots, (periodic x) z and den, and the
  // pivots of a system starting at an artificial first row
  L.tab = take((size_t)(3 * k.nx + 2 * k.nv + 1 + FIT_TW_MAX) * fb);
  L.total = o;
  return L;
}

}  // namespace

enum ProfKind {
  PK_PREDICT = 0, PK_RECON, PK_FIELD, PK_KICK, PK_REMAP, PK_FIT, PK_RESET,
  PK_OTHER, PK_N
};

struct vp_ctx {
  vp_params p;
  KP k;
  Layout L;
  hipStream_t stream;
  char *ws;
  double t;
  int64_t step;
  bool ready;
  int cur = 0;  // which of the two block-count buffers holds the live lists
  // The spline fit after a resampling runs on `aux` while the following
  // steps run on `stream` (they read F_ini, not the coefficients); it is
  // joined (`fit_pending`) before anything reads or restages C or T.
  hipStream_t aux = nullptr;
  hipEvent_t ev_eval = nullptr, ev_fit = nullptr;
  bool fit_pending = false;
  int64_t reset_step = 0;  // step of the elements' last reset
  std::string err;
  std::vector<char> host_tab;  // source of the pivot-table upload
  // profiling: event pairs per kernel kind
  bool prof = false;
  int prof_cap = 0;
  std::vector<hipEvent_t> ev[PK_N];
  int ev_used[PK_N] = {};

  template <typename T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(ws + off);
  }
  bool mixed() const { return p.precision == VP_MIXED; }
  int *counts(int which) const { return at<int>(L.cnt) + (size_t)which * L.nb; }
};

namespace {

int dev_fail(vp_ctx *c, hipError_t e, const char *where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return VP_EDEVICE;
}

#define VP_LAUNCH_CHECK(c, where)                       \
  do {                                                  \
    hipError_t _e = hipGetLastError();                  \
    if (_e != hipSuccess) return dev_fail(c, _e, where); \
  } while (0)

// Event pair around one launch when profiling is on.
struct ProfScope {
  vp_ctx *c;
  int kind;
  bool on;
  hipStream_t st;
  ProfScope(vp_ctx *c_, int k, hipStream_t s = nullptr)
      : c(c_), kind(k), on(false), st(s ? s : c_->stream) {
    if (c->prof && c->ev_used[kind] < c->prof_cap) {
      on = true;
      (void)hipEventRecord(c->ev[kind][2 * c->ev_used[kind]], st);
    }
  }
  ~ProfScope() {
    if (on) {
      (void)hipEventRecord(c->ev[kind][2 * c->ev_used[kind] + 1], st);
      c->ev_used[kind] += 1;
    }
  }
};

unsigned grid_for(long long n, int bs) {
  long long g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  if (g > (1ll << 30)) g = 1ll << 30;
  return (unsigned)g;
}

// Element pass (k_elem): optional kick + corrector, optional predictor drift
// and record/registration into count buffer `reg_buf`, optional clearing of
// count buffer `zero_buf` (-1: none).
int launch_elem(vp_ctx *c, int kick, int drift, int predict, int reg,
                int reg_buf, int zero_buf) {
  // a kick completes the step before the current one: it reads that step's
  // clock slot and writes the current one
  KP k = c->k;
  if (kick) k.par ^= 1;
  ProfScope ps(c, kick ? PK_KICK : PK_PREDICT);
  const long long nbz = zero_buf >= 0 ? c->L.nb : 0;
  const long long n =
      std::max<long long>(k.E, std::min<long long>(nbz, 1 << 22));
  // the workgroup table pays where the device atomics queue: many patches
  // of boxes of at most TABLE_RB blocks (strides up to 8).  A launch of a
  // few waves per SIMD waits on their latency instead, and with stride 16
  // (boxes of ~30 blocks) the table was slower too.
  const int np = elem_patches(k.mx, k.mv);
  const bool tab = np >= ELEM_TABLE_MIN_PATCHES && k.sx <= 8 && k.sv <= 8;
  const unsigned grid =
      tab ? std::max<unsigned>(grid_for(n, 256), (unsigned)np)
          : grid_for(n, 256);
  auto kern = tab ? k_elem<true> : k_elem<false>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, c->stream,
                     k, c->at<double>(c->L.st), c->at<double>(c->L.acc),
                     c->at<double>(c->L.rec), c->at<double>(c->L.qm),
                     zero_buf >= 0 ? c->counts(zero_buf) : nullptr, nbz,
                     c->counts(reg_buf), c->at<int>(c->L.lst),
                     c->at<int>(c->L.flags), kick, drift, predict, reg);
  VP_LAUNCH_CHECK(c, "k_elem");
  return VP_OK;
}

// Field from the reconstruction's partials + kick + corrector (+ next
// predictor) for grids of at most FIELD1_MAX columns: the chunks of the
// cumulative mass (k_field_chunks, one wavefront per 64 columns), then the
// element pass that takes its force from them (k_elem_window).
int launch_elem_field(vp_ctx *c, int predict, int reg, int reg_buf,
                      int zero_buf) {
  KP k = c->k;
  k.par ^= 1;  // completes the previous step (see launch_elem)
  ProfScope ps(c, PK_KICK);
  const int nch = (k.nx + MCHUNK - 1) / MCHUNK;
  const double *part = c->at<double>(c->L.part);
  double *Mc = c->at<double>(c->L.Mc), *ctot = c->at<double>(c->L.ctot),
         *cmax = c->at<double>(c->L.rmx);
  hipLaunchKernelGGL(k_field_chunks, dim3(nch), dim3(64), 0, c->stream, k,
                     part, Mc, ctot, cmax);
  VP_LAUNCH_CHECK(c, "k_field_chunks");
  double *st = c->at<double>(c->L.st), *rec = c->at<double>(c->L.rec),
         *qm = c->at<double>(c->L.qm);
  int *cz = c->counts(zero_buf), *cr = c->counts(reg_buf);
  const long long nb = c->L.nb;
  int *lst = c->at<int>(c->L.lst), *flags = c->at<int>(c->L.flags);
  hipLaunchKernelGGL(k_elem_window, dim3(elem_patches(k.mx, k.mv)),
                     dim3(ELEMC_WG), 0, c->stream, k, Mc, ctot, cmax, st, rec,
                     qm, cz, nb, cr, lst, flags, predict, reg);
  VP_LAUNCH_CHECK(c, "k_elem_window");
  return VP_OK;
}

// Time since the elements' last reset at which the block lists are built
// (the positions after the predictor's half drift when `half`); the
// reconstruction that uses the lists reads the same value from c->k.
void set_list_time(vp_ctx *c, bool half) {
  c->k.tau = ((double)(c->step - c->reset_step) + (half ? 0.5 : 0.0)) *
             c->p.dt;
  gox_set(c->k);
}

// Records and block lists for the current element state (no motion).
int launch_predict(vp_ctx *c, int drift, int reg) {
  set_list_time(c, drift != 0);
  return launch_elem(c, 0, drift, 1, reg, c->cur, -1);
}

int launch_zero_counts(vp_ctx *c) {
  ProfScope ps(c, PK_OTHER);
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(c->L.nb, 256)), dim3(256), 0,
                     c->stream, c->counts(c->cur), c->L.nb);
  VP_LAUNCH_CHECK(c, "k_zero_i32");
  return VP_OK;
}

template <typename FT, int MODE>
int launch_recon(vp_ctx *c, void *fout, int *aout, double *rho_out) {
  const KP &k = c->k;
  ProfScope ps(c, PK_RECON);
  auto kern = k.per ? k_recon<FT, MODE, 1> : k_recon<FT, MODE, 0>;
  hipLaunchKernelGGL(kern, dim3(c->L.nwg_x * c->L.nwg_y),
                     dim3(512), 0, c->stream, k, c->at<double>(c->L.rec),
                     c->at<double>(c->L.qm), c->counts(c->cur),
                     c->at<int>(c->L.lst), c->at<int>(c->L.flags),
                     c->at<FT>(c->L.F),
                     c->at<double>(c->L.part), reinterpret_cast<FT *>(fout),
                     aout, c->at<double>(c->L.dpart),
                     c->at<unsigned long long>(c->L.ovf));
  VP_LAUNCH_CHECK(c, "k_recon");
  return VP_OK;
}

// The field launches for a filled FieldArgs: one workgroup up to FIELD1_MAX
// columns, else the column-chunk kernel and, without periodic x, the
// carries, M_left and the force spread over a second launch.  Returns the
// launch status (where names the failing kernel).
hipError_t field_launches(const KP &k, FieldArgs &A, hipStream_t s,
                          const char **where) {
  if (k.nx <= FIELD1_MAX) {
    *where = "k_field1";
    hipLaunchKernelGGL(k_field1, dim3(1), dim3(1024), 0, s, k, A);
    return hipGetLastError();
  }
  const int nch = (k.nx + FIELD_WG - 1) / FIELD_WG;
  A.tail = k.per ? 0 : 1;
  *where = "k_field";
  hipLaunchKernelGGL(k_field, dim3(nch), dim3(FIELD_WG), 0, s, k, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !A.tail) return e;
  *where = "k_field_tail";
  hipLaunchKernelGGL(k_field_tail, dim3(nch), dim3(FIELD_WG), 0, s, k, A);
  return hipGetLastError();
}

int launch_field(vp_ctx *c, const double *in, int from_part, double *rho_out,
                 double *a_out, double *da_out, double *d2a_out) {
  ProfScope ps(c, PK_FIELD);
  FieldArgs A{};
  A.in = in;
  A.ngy = from_part ? c->k.ngy : 0;
  A.in_is_rho = from_part ? 0 : 1;
  A.Mc = c->at<double>(c->L.Mc);
  A.ctot = c->at<double>(c->L.ctot);
  A.fcnt = c->at<int>(c->L.fcnt);
  A.Ml = c->at<double>(c->L.Ml);
  A.acc = c->at<double>(c->L.acc);
  A.rho_out = rho_out;
  A.a_out = a_out;
  A.da_out = da_out;
  A.d2a_out = d2a_out;
  A.rmx = c->at<double>(c->L.rmx);
  const char *where = "field";
  const hipError_t e = field_launches(c->k, A, c->stream, &where);
  if (e != hipSuccess) return dev_fail(c, e, where);
  return VP_OK;
}

// The reconstruction in one of its modes; the density modes are followed
// by the field pass (a, a', a'', optionally rho).
template <int MODE>
int recon(vp_ctx *c, void *fout, int *aout, double *rho_out = nullptr) {
  const int rc = c->mixed() ? launch_recon<float, MODE>(c, fout, aout, rho_out)
                            : launch_recon<double, MODE>(c, fout, aout, rho_out);
  if (rc || (MODE != MODE_DENSITY && MODE != MODE_DIAG)) return rc;
  return launch_field(c, c->at<double>(c->L.part), 1, rho_out, nullptr,
                      nullptr, nullptr);
}

int launch_reset(vp_ctx *c) {
  ProfScope ps(c, PK_RESET);
  const long long n =
      std::max<long long>(c->k.E, std::min<long long>(c->L.nb, 1 << 22));
  hipLaunchKernelGGL(k_elem_reset, dim3(grid_for(n, 256)),
                     dim3(256), 0, c->stream, c->k, c->at<double>(c->L.st),
                     c->counts(c->cur), c->L.nb);
  VP_LAUNCH_CHECK(c, "k_elem_reset");
  return VP_OK;
}

template <typename FT>
int fit_spline_t(vp_ctx *c, hipStream_t st) {
  const KP &k = c->k;
  ProfScope ps(c, PK_FIT, st);
  FT *tab = c->at<FT>(c->L.tab);
  FT *zx = tab + 2 * k.nx + 2 * k.nv, *den = tab + 3 * k.nx + 2 * k.nv;
  hipLaunchKernelGGL((k_fit_x<FT>),
                     dim3(grid_for(k.nv, FIT_LINES) * fit_segments<FT>(k.nx)),
                     dim3(FIT_THREADS), 0,
                     st, k, c->at<FT>(c->L.F), c->at<FT>(c->L.T), tab);
  VP_LAUNCH_CHECK(c, "k_fit_x");
  if (k.per) {
    hipLaunchKernelGGL((k_fit_x_cyclic<FT>), dim3(k.nv), dim3(256), 0,
                       st, k, c->at<FT>(c->L.T), zx, den);
    VP_LAUNCH_CHECK(c, "k_fit_x_cyclic");
  }
  hipLaunchKernelGGL((k_fit_v<FT>),
                     dim3(grid_for(k.nx, FIT_LINES) * fit_segments<FT>(k.nv)),
                     dim3(FIT_THREADS), 0,
                     st, k, c->at<FT>(c->L.T), c->at<FT>(c->L.C), tab);
  VP_LAUNCH_CHECK(c, "k_fit_v");
  if (k.per) {
    hipLaunchKernelGGL((k_ghost_periodic<FT>), dim3(grid_for(k.nv + 2, 256)),
                       dim3(256), 0, st, k, c->at<FT>(c->L.C), -1,
                       k.nv);
    VP_LAUNCH_CHECK(c, "k_ghost_periodic");
    return VP_OK;
  }
  hipLaunchKernelGGL((k_ghost_x<FT>), dim3(grid_for(k.nv + 2, 256)), dim3(256),
                     0, st, k, c->at<FT>(c->L.C));
  VP_LAUNCH_CHECK(c, "k_ghost_x");
  return VP_OK;
}

// Periodic x: the ghost columns of F_ini after its interior was written.
template <typename FT>
int ghost_F_t(vp_ctx *c) {
  hipLaunchKernelGGL((k_ghost_periodic<FT>), dim3(grid_for(c->k.nv, 256)),
                     dim3(256), 0, c->stream, c->k, c->at<FT>(c->L.F), 0,
                     c->k.nv - 1);
  VP_LAUNCH_CHECK(c, "k_ghost_periodic");
  return VP_OK;
}

int ghost_F(vp_ctx *c) {
  if (!c->k.per) return VP_OK;
  return c->mixed() ? ghost_F_t<float>(c) : ghost_F_t<double>(c);
}

int fit_spline(vp_ctx *c, hipStream_t st = nullptr) {
  if (!st) st = c->stream;
  return c->mixed() ? fit_spline_t<float>(c, st) : fit_spline_t<double>(c, st);
}

// Wait (on the context's stream) for a spline fit still running on aux.
int join_fit(vp_ctx *c) {
  if (!c->fit_pending) return VP_OK;
  c->fit_pending = false;
  const hipError_t e = hipStreamWaitEvent(c->stream, c->ev_fit, 0);
  if (e != hipSuccess) return dev_fail(c, e, "join spline fit");
  return VP_OK;
}

// The spline fit of a resampling, overlapped with the steps that follow it
// (they read F_ini only).  Synchronous on the context's stream while that
// stream is being captured into a graph.
int fit_spline_async(vp_ctx *c) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess ||
      cs != hipStreamCaptureStatusNone)
    return fit_spline(c);
  hipError_t e = hipSuccess;
  if (!c->aux) {
    hipStream_t st = nullptr;
    hipEvent_t ea = nullptr, eb = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess)
      e = hipEventCreateWithFlags(&ea, hipEventDisableTiming);
    if (e == hipSuccess)
      e = hipEventCreateWithFlags(&eb, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (eb) (void)hipEventDestroy(eb);
      if (ea) (void)hipEventDestroy(ea);
      if (st) (void)hipStreamDestroy(st);
      return dev_fail(c, e, "fit stream");
    }
    c->aux = st;
    c->ev_eval = ea;
    c->ev_fit = eb;
  }
  e = hipEventRecord(c->ev_eval, c->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->aux, c->ev_eval, 0);
  if (e != hipSuccess) return dev_fail(c, e, "fit stream order");
  const int rc = fit_spline(c, c->aux);
  if (rc) return rc;
  e = hipEventRecord(c->ev_fit, c->aux);
  if (e != hipSuccess) return dev_fail(c, e, "fit stream order");
  c->fit_pending = true;
  return VP_OK;
}

template <typename FT, int TO_F>
int launch_remap_t(vp_ctx *c, void *fout) {
  if (const int rc = join_fit(c)) return rc;
  ProfScope ps(c, PK_REMAP);
  FT *out = TO_F ? reinterpret_cast<FT *>(fout) : c->at<FT>(c->L.F);
  auto kern = c->k.per ? k_remap_eval<FT, TO_F, 1> : k_remap_eval<FT, TO_F, 0>;
  hipLaunchKernelGGL(kern,
                     dim3(c->L.nwg_x * c->L.nwg_y),
                     dim3(512), 0, c->stream, c->k, c->at<double>(c->L.rec),
                     c->at<double>(c->L.qm), c->counts(c->cur),
                     c->at<int>(c->L.lst), c->at<int>(c->L.flags),
                     c->at<FT>(c->L.C), out,
                     c->at<unsigned long long>(c->L.ovf));
  VP_LAUNCH_CHECK(c, "k_remap_eval");
  return VP_OK;
}

int do_remap(vp_ctx *c) {
  int rc;
  if ((rc = launch_predict(c, 0, 1))) return rc;
  rc = c->mixed() ? launch_remap_t<float, 0>(c, nullptr)
                  : launch_remap_t<double, 0>(c, nullptr);
  if (rc) return rc;
  if ((rc = ghost_F(c))) return rc;
  if ((rc = fit_spline_async(c))) return rc;
  c->reset_step = c->step;
  return launch_reset(c);
}

// Diagnostics of the current state (positions at the current time): mass,
// kinetic and potential energy, entropy, max |det T - 1|, E_map, L1, L2
// into h[8], and the count of overflowed query blocks.  Synchronises the
// stream.
int diag_now(vp_ctx *c, double *h, unsigned long long *ovf) {
  int rc;
  if ((rc = launch_predict(c, 0, 1))) return rc;
  if ((rc = recon<MODE_DIAG>(c, nullptr, nullptr))) return rc;
  if ((rc = launch_zero_counts(c))) return rc;
  hipLaunchKernelGGL(k_diag, dim3(1), dim3(1024), 0, c->stream, c->k,
                     c->at<double>(c->L.dpart),
                     (long long)c->L.nwg_x * c->L.nwg_y,
                     c->at<double>(c->L.Ml), c->at<double>(c->L.acc),
                     c->at<double>(c->L.st), c->at<double>(c->L.dout));
  VP_LAUNCH_CHECK(c, "k_diag");
  hipError_t e = hipMemcpyAsync(h, c->at<double>(c->L.dout), 8 * sizeof(double),
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ovf, c->at<unsigned long long>(c->L.ovf), sizeof(*ovf),
                       hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "diagnostics read");
  return VP_OK;
}

// E_map of the current state alone, for the adaptive resampling check: the
// records and lists of the current elements, the reconstruction in its
// E_map-only mode and the maximum over its workgroups (no field, no energy
// or entropy sums).
// Synchronises the stream.
int emap_now(vp_ctx *c, double *emap) {
  int rc;
  if ((rc = launch_predict(c, 0, 1))) return rc;
  rc = c->mixed() ? launch_recon<float, MODE_EMAP>(c, nullptr, nullptr, nullptr)
                  : launch_recon<double, MODE_EMAP>(c, nullptr, nullptr, nullptr);
  if (rc) return rc;
  if ((rc = launch_zero_counts(c))) return rc;
  hipLaunchKernelGGL(k_emap_max, dim3(1), dim3(1024), 0, c->stream,
                     c->at<double>(c->L.dpart),
                     (long long)c->L.nwg_x * c->L.nwg_y,
                     c->at<double>(c->L.dout));
  VP_LAUNCH_CHECK(c, "k_emap_max");
  hipError_t e = hipMemcpyAsync(emap, c->at<double>(c->L.dout) + 5,
                                sizeof(double), hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "E_map read");
  return VP_OK;
}

// n drift-kick-drift steps.  The kick + corrector of a step and the
// predictor of the next one share one element pass (k_elem) unless a
// resampling or the end of the call comes between them, so the elements are
// at integer time whenever control returns to the caller.
int run_steps(vp_ctx *c, int n) {
  int rc;
  const bool self = c->p.force_mode == VP_FORCE_SELF;
  // small grids: the field is rebuilt inside the element pass
  const bool fused = self && c->k.nx <= FIELD1_MAX;
  bool predicted = false;
  for (int s = 0; s < n; ++s) {
    if (!predicted && (rc = launch_predict(c, 1, self ? 1 : 0))) return rc;
    if (self) {
      rc = fused ? (c->mixed() ? launch_recon<float, MODE_DENSITY>(
                                     c, nullptr, nullptr, nullptr)
                               : launch_recon<double, MODE_DENSITY>(
                                     c, nullptr, nullptr, nullptr))
                 : recon<MODE_DENSITY>(c, nullptr, nullptr);
      if (rc) return rc;
    }
    c->step += 1;
    c->k.par = (int)(c->step & 1);
    c->t = (double)c->step * c->p.dt;  // fixed step; the clock holds it else
    const bool remap_due = c->p.n_s > 0 && c->step % c->p.n_s == 0;
    // adaptive resampling: E_map of the post-corrector elements is checked
    // every emap_every steps (end of section 2.3.3)
    const bool check_due = !remap_due && c->p.emap_max > 0.0 &&
                           c->step % c->p.emap_every == 0;
    if (!remap_due && !check_due && s + 1 < n) {
      // kick + corrector of this step, predictor of the next, lists into
      // the other count buffer while this one is cleared
      set_list_time(c, true);
      rc = fused ? launch_elem_field(c, 1, 1, c->cur ^ 1, c->cur)
                 : launch_elem(c, 1, 1, 1, self ? 1 : 0, c->cur ^ 1, c->cur);
      if (rc) return rc;
      c->cur ^= 1;
      predicted = true;
    } else {
      rc = fused ? launch_elem_field(c, 0, 0, c->cur, c->cur)
                 : launch_elem(c, 1, 0, 0, 0, c->cur, c->cur);
      if (rc) return rc;
      predicted = false;
      bool remap = remap_due;
      if (check_due) {
        double emap = 0.0;
        if ((rc = emap_now(c, &emap))) return rc;
        remap = emap > c->p.emap_max;
      }
      if (remap && (rc = do_remap(c))) return rc;
    }
  }
  return VP_OK;
}

template <typename FT>
void host_tables(int n, std::vector<FT> &cp, std::vector<FT> &ri) {
  // Thomas pivots of the (1, 4, 1) system with end rows (4, 2) / (2, 4)
  cp.assign(n, (FT)0);
  ri.assign(n, (FT)0);
  FT rinv = (FT)0.25;
  ri[0] = rinv;
  cp[0] = (FT)2 * rinv;
  for (int i = 1; i < n; ++i) {
    const FT sub = (i == n - 1) ? (FT)2 : (FT)1;
    const FT den = (FT)4 - sub * cp[i - 1];
    rinv = (FT)1 / den;
    ri[i] = rinv;
    cp[i] = (FT)1 * rinv;
  }
}

// Periodic x: Thomas pivots of the tridiagonal part B of the cyclic
// (1, 4, 1) system (diagonal 8, 4, .., 4, 4.25, unit off-diagonals; the
// corners go into the Sherman-Morrison term with gamma = -4), the solution
// z of B z = (-4, 0, .., 0, 1), and den = (1 + z_0) - z_{n-1} / 4.
template <typename FT>
void host_tables_cyclic(int n, std::vector<FT> &cp, std::vector<FT> &ri,
                        std::vector<FT> &z, FT &den) {
  cp.assign(n, (FT)0);
  ri.assign(n, (FT)0);
  z.assign(n, (FT)0);
  auto diag = [n](int i) {
    return i == 0 ? (FT)8 : (i == n - 1 ? (FT)4.25 : (FT)4);
  };
  FT rinv = (FT)1 / diag(0);
  ri[0] = rinv;
  cp[0] = rinv;
  std::vector<FT> d(n);
  d[0] = (FT)-4 * rinv;
  for (int i = 1; i < n; ++i) {
    const FT dn = diag(i) - cp[i - 1];
    rinv = (FT)1 / dn;
    ri[i] = rinv;
    cp[i] = rinv;
    const FT u = (i == n - 1) ? (FT)1 : (FT)0;
    d[i] = (u - d[i - 1]) * rinv;
  }
  z[n - 1] = d[n - 1];
  for (int i = n - 2; i >= 0; --i) z[i] = d[i] - cp[i] * z[i + 1];
  den = ((FT)1 + z[0]) - (FT)0.25 * z[n - 1];
}

template <typename FT>
int upload_tables(vp_ctx *c) {
  std::vector<FT> cpx, rix, cpv, riv, zx;
  FT den = (FT)1;
  if (c->k.per)
    host_tables_cyclic<FT>(c->k.nx, cpx, rix, zx, den);
  else
    host_tables<FT>(c->k.nx, cpx, rix);
  host_tables<FT>(c->k.nv, cpv, riv);
  zx.resize(c->k.nx, (FT)0);
  std::vector<FT> all;
  all.insert(all.end(), cpx.begin(), cpx.end());
  all.insert(all.end(), rix.begin(), rix.end());
  all.insert(all.end(), cpv.begin(), cpv.end());
  all.insert(all.end(), riv.begin(), riv.end());
  all.insert(all.end(), zx.begin(), zx.end());
  all.push_back(den);
  // 1/den of the (1, 4, 1) system from an artificial first row (4, 1): the
  // forward pivots of the first tile of a fit segment that does not start
  // at the line's start
  FT cp = (FT)0;
  for (int q = 0; q < FIT_TW_MAX; ++q) {
    const FT r = (FT)1 / ((FT)4 - cp);
    all.push_back(r);
    cp = r;
  }
  // the host copy lives as long as the context, so no wait is needed
  c->host_tab.assign(reinterpret_cast<const char *>(all.data()),
                     reinterpret_cast<const char *>(all.data() + all.size()));
  hipError_t e = hipMemcpyAsync(c->at<FT>(c->L.tab), c->host_tab.data(),
                                c->host_tab.size(), hipMemcpyHostToDevice,
                                c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "table upload");
  return VP_OK;
}

template <typename T>
int fill(vp_ctx *c, T *ptr, long long n, T val) {
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(std::min<long long>(n, 1 << 22), 256)),
                     dim3(256), 0, c->stream, ptr, n, val);
  VP_LAUNCH_CHECK(c, "k_fill");
  return VP_OK;
}

int load_rows(vp_ctx *c, const double *src, int j0, int nrows) {
  const long long n = (long long)c->k.nx * nrows;
  const unsigned g = grid_for(std::min<long long>(n, 1 << 22), 256);
  if (c->mixed())
    hipLaunchKernelGGL((k_load_f0<float>), dim3(g), dim3(256), 0, c->stream,
                       c->k, src, j0, nrows, c->at<float>(c->L.F));
  else
    hipLaunchKernelGGL((k_load_f0<double>), dim3(g), dim3(256), 0, c->stream,
                       c->k, src, j0, nrows, c->at<double>(c->L.F));
  VP_LAUNCH_CHECK(c, "k_load_f0");
  return VP_OK;
}

// Variable step: the first step from the density of F_ini (column sums in
// the reconstruction's order, then the largest dv S(i)).
template <typename FT>
int clock_init_t(vp_ctx *c) {
  double *S = c->at<double>(c->L.Ml);  // scratch until the first field
  hipLaunchKernelGGL((k_colsum_F<FT>), dim3(grid_for(c->k.nx, 256)), dim3(256),
                     0, c->stream, c->k, c->at<FT>(c->L.F), S);
  VP_LAUNCH_CHECK(c, "k_colsum_F");
  hipLaunchKernelGGL(k_clock_init, dim3(1), dim3(1024), 0, c->stream, c->k, S);
  VP_LAUNCH_CHECK(c, "k_clock_init");
  return VP_OK;
}

int clock_init(vp_ctx *c) {
  return c->mixed() ? clock_init_t<float>(c) : clock_init_t<double>(c);
}

// Current step size and time: host values for a fixed step, the device
// clock's (synchronising) for a variable one.
int read_clock(vp_ctx *c, double *dt, double *t) {
  if (!c->k.clk) {
    *dt = c->p.dt;
    *t = c->t;
    return VP_OK;
  }
  double slot[CK_SLOT];
  hipError_t e = hipMemcpyAsync(slot, c->k.clk + CK_SLOT * c->k.par,
                                sizeof(slot), hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "clock read");
  *dt = slot[CK_DT];
  *t = slot[CK_T];
  return VP_OK;
}

int check_flags(vp_ctx *c) {
  int flags = 0;
  hipError_t e = hipMemcpyAsync(&flags, c->at<int>(c->L.flags), sizeof(int),
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "flag read");
  if (flags & FLAG_NUMERIC) {
    c->err = "non-finite element state or det T <= 0 met on the device";
    return VP_ENUMERIC;
  }
  return VP_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int vp_footprint(const vp_params *p, size_t *bytes) {
  if (!params_ok(p) || !bytes) return VP_EINVAL;
  KP k = make_kp(p);
  *bytes = make_layout(p, k).total;
  return VP_OK;
}

int vp_create(const vp_params *p, void *dev_workspace, size_t bytes,
              void *hip_stream, vp_ctx **out) {
  if (!out) return VP_EINVAL;
  *out = nullptr;
  if (!params_ok(p)) {
    g_create_error = "invalid parameters";
    return VP_EINVAL;
  }
  if (!dev_workspace) {
    g_create_error = "null workspace";
    return VP_EINVAL;
  }
  KP k = make_kp(p);
  Layout L = make_layout(p, k);
  if (bytes < L.total) {
    g_create_error = "workspace smaller than vp_footprint";
    return VP_ENOMEM;
  }
  if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0) {
    g_create_error = "workspace must be 256-byte aligned";
    return VP_EINVAL;
  }
  vp_ctx *c = new (std::nothrow) vp_ctx();
  if (!c) return VP_ENOMEM;
  c->p = *p;
  c->k = k;
  c->L = L;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = reinterpret_cast<char *>(dev_workspace);
  if (p->c_dyn > 0.0) c->k.clk = c->at<double>(L.clk);
  c->t = 0.0;
  c->step = 0;
  c->ready = false;
  // zero the whole workspace once (F padding, counts, flags, counters), then
  // the spline pivot tables and the initial elements
  int rc = fill<int>(c, c->at<int>(0), (long long)(L.total / 4), 0);
  if (!rc)
    rc = c->mixed() ? upload_tables<float>(c) : upload_tables<double>(c);
  if (!rc) rc = launch_reset(c);
  if (rc) {
    g_create_error = c->err;
    delete c;
    return rc;
  }
  *out = c;
  return VP_OK;
}

int vp_destroy(vp_ctx *c) {
  if (!c) return VP_EINVAL;
  const int rc = join_fit(c);
  const hipError_t e = hipStreamSynchronize(c->stream);
  // profiling events of a vp_prof_begin without its vp_prof_end
  for (int k = 0; k < PK_N; ++k)
    for (auto &ev : c->ev[k])
      if (ev) (void)hipEventDestroy(ev);
  if (c->aux) {
    (void)hipEventDestroy(c->ev_eval);
    (void)hipEventDestroy(c->ev_fit);
    (void)hipStreamDestroy(c->aux);
  }
  delete c;
  return (e == hipSuccess && !rc) ? VP_OK : VP_EDEVICE;
}

int vp_init_conditions(vp_ctx *c, const double *f0, int f0_on_device) {
  if (!c || !f0) return VP_EINVAL;
  const int nx = c->k.nx, nv = c->k.nv;
  int rc;
  if ((rc = join_fit(c))) return rc;
  if (f0_on_device) {
    if ((rc = load_rows(c, f0, 0, nv))) return rc;
  } else {
    // host input: stage row blocks through the spline-coefficient buffer,
    // whose contents the fit below rewrites
    const size_t stage_bytes = c->L.T - c->L.C;
    const int rows = (int)std::min<size_t>(nv, stage_bytes / ((size_t)nx * 8));
    double *stage = c->at<double>(c->L.C);
    for (int j0 = 0; j0 < nv; j0 += rows) {
      const int nr = std::min(rows, nv - j0);
      hipError_t e = hipMemcpyAsync(stage, f0 + (size_t)j0 * nx,
                                    (size_t)nr * nx * sizeof(double),
                                    hipMemcpyHostToDevice, c->stream);
      if (e != hipSuccess) return dev_fail(c, e, "f0 upload");
      if ((rc = load_rows(c, stage, j0, nr))) return rc;
      e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return dev_fail(c, e, "f0 upload");
    }
  }
  if ((rc = ghost_F(c))) return rc;
  if ((rc = fit_spline(c))) return rc;
  c->step = 0;
  c->k.par = 0;
  if ((rc = launch_reset(c))) return rc;
  if (c->k.clk && (rc = clock_init(c))) return rc;
  c->t = 0.0;
  c->reset_step = 0;
  c->ready = true;
  return VP_OK;
}

int vp_step(vp_ctx *c, int nsteps) {
  if (!c) return VP_EINVAL;
  if (!c->ready) return VP_ESTATE;
  if (nsteps < 0) return VP_EINVAL;
  return run_steps(c, nsteps);
}

int vp_remap(vp_ctx *c) {
  if (!c) return VP_EINVAL;
  if (!c->ready) return VP_ESTATE;
  return do_remap(c);
}

int vp_reconstruct_f(vp_ctx *c, int scheme, void *f_out_dev) {
  if (!c || !f_out_dev) return VP_EINVAL;
  if (!c->ready) return VP_ESTATE;
  if (scheme != VP_SCHEME_TRANSPORT && scheme != VP_SCHEME_REMAP)
    return VP_EINVAL;
  int rc;
  if ((rc = launch_predict(c, 0, 1))) return rc;
  if (scheme == VP_SCHEME_TRANSPORT) {
    rc = recon<MODE_F>(c, f_out_dev, nullptr);
  } else {
    rc = c->mixed() ? launch_remap_t<float, 1>(c, f_out_dev)
                    : launch_remap_t<double, 1>(c, f_out_dev);
  }
  if (rc) return rc;
  return launch_zero_counts(c);
}

int vp_density(vp_ctx *c, double *rho_out_dev) {
  if (!c || !rho_out_dev) return VP_EINVAL;
  if (!c->ready) return VP_ESTATE;
  int rc;
  if ((rc = launch_predict(c, 0, 1))) return rc;
  if ((rc = recon<MODE_DENSITY>(c, nullptr, nullptr, rho_out_dev))) return rc;
  return launch_zero_counts(c);
}

int vp_poisson(vp_ctx *c, const double *rho, double *a, double *da,
               double *d2a) {
  if (!c || !rho || !a || !da || !d2a) return VP_EINVAL;
  return launch_field(c, rho, 0, nullptr, a, da, d2a);
}

int vp_diagnostics(vp_ctx *c, vp_diag *out) {
  if (!c || !out) return VP_EINVAL;
  if (!c->ready) return VP_ESTATE;
  double h[8];
  unsigned long long ovf = 0;
  int rc = diag_now(c, h, &ovf);
  if (rc) return rc;
  out->mass = h[0];
  out->e_kin = h[1];
  out->e_pot = h[2];
  out->energy = h[1] + h[2];
  out->entropy = h[3];
  out->max_det_dev = h[4];
  out->emap = h[5];
  out->l1 = h[6];
  out->l2 = h[7];
  if ((rc = read_clock(c, &out->dt, &out->t))) return rc;
  out->step = c->step;
  out->overflow_blocks = (int64_t)ovf;
  return check_flags(c);
}

int vp_get_elements(vp_ctx *c, double *el) {
  if (!c || !el) return VP_EINVAL;
  hipError_t e = hipMemcpyAsync(el, c->at<double>(c->L.st),
                                (size_t)NSTATE * c->k.E * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "get_elements");
  return VP_OK;
}

int vp_set_elements(vp_ctx *c, const double *el) {
  if (!c || !el) return VP_EINVAL;
  hipError_t e = hipMemcpyAsync(c->at<double>(c->L.st), el,
                                (size_t)NSTATE * c->k.E * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "set_elements");
  return VP_OK;
}

int vp_get_assignment(vp_ctx *c, int32_t *assign) {
  if (!c || !assign) return VP_EINVAL;
  int rc;
  if ((rc = launch_predict(c, 0, 1))) return rc;
  if ((rc = recon<MODE_ASSIGN>(c, nullptr, assign))) return rc;
  return launch_zero_counts(c);
}

int vp_time(vp_ctx *c, double *t, int64_t *step) {
  if (!c) return VP_EINVAL;
  if (step) *step = c->step;
  if (!t) return VP_OK;
  if (!c->ready) {
    *t = 0.0;
    return VP_OK;
  }
  double dt;
  return read_clock(c, &dt, t);
}

int vp_prof_begin(vp_ctx *c, int max_launches) {
  if (!c || max_launches < 1) return VP_EINVAL;
  if (c->prof) return VP_ESTATE;
  for (int k = 0; k < PK_N; ++k) {
    c->ev[k].assign(2 * (size_t)max_launches, nullptr);
    for (auto &e : c->ev[k]) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return dev_fail(c, r, "hipEventCreate");
    }
    c->ev_used[k] = 0;
  }
  c->prof_cap = max_launches;
  c->prof = true;
  return VP_OK;
}

int vp_prof_end(vp_ctx *c, double *ms, int64_t *n) {
  if (!c || !c->prof) return VP_EINVAL;
  if (const int rc = join_fit(c)) return rc;
  hipError_t r = hipStreamSynchronize(c->stream);
  int rc = VP_OK;
  if (r != hipSuccess) rc = dev_fail(c, r, "prof sync");
  for (int k = 0; k < PK_N; ++k) {
    double tot = 0.0;
    for (int q = 0; q < c->ev_used[k] && rc == VP_OK; ++q) {
      float m = 0.0f;
      r = hipEventElapsedTime(&m, c->ev[k][2 * q], c->ev[k][2 * q + 1]);
      if (r != hipSuccess) rc = dev_fail(c, r, "hipEventElapsedTime");
      tot += m;
    }
    if (ms) ms[k] = tot;
    if (n) n[k] = c->ev_used[k];
    for (auto &e : c->ev[k])
      if (e) (void)hipEventDestroy(e);
    c->ev[k].clear();
    c->ev_used[k] = 0;
  }
  c->prof = false;
  return rc;
}

int vp_sync(vp_ctx *c) {
  if (!c) return VP_EINVAL;
  if (const int rc = join_fit(c)) return rc;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "sync");
  return check_flags(c);
}

const char *vp_last_error(vp_ctx *c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

}  // extern "C"

// ================================ vp_poisson without a context or workspace
//
// The field's intermediate buffers (chunk prefixes, chunk totals and
// maxima, M_left, the force table on [-4, nx + 3], the finished-chunk
// counter) in one file-scope device array.  In host code `scratch` names a
// host-side stand-in, not the device memory: its device address is taken
// with hipGetSymbolAddress once per device (each GPU holds its own copy)
// and only that address is handed to kernels.
namespace {
constexpr size_t SP_NX = VP_POISSON_STATIC_MAX_NX;
constexpr size_t SP_MC = 0;                            // [SP_NX]
constexpr size_t SP_ML = SP_MC + SP_NX;                // [SP_NX]
constexpr size_t SP_ACC = SP_ML + SP_NX;               // [3 (SP_NX + 8)]
constexpr size_t SP_CTOT = SP_ACC + 3 * (SP_NX + 8);   // [FIELD_CHUNKS]
constexpr size_t SP_RMX = SP_CTOT + FIELD_CHUNKS;      // [FIELD_CHUNKS]
constexpr size_t SP_CNT = SP_RMX + FIELD_CHUNKS;       // int counter (256 B)
constexpr size_t SP_DOUBLES = SP_CNT + 32;
static_assert(SP_DOUBLES * sizeof(double) == VP_POISSON_STATIC_BYTES,
              "VP_POISSON_STATIC_BYTES");
static_assert(SP_NX <= (size_t)FIELD_CHUNKS * MCHUNK, "chunk tables");
}  // namespace

static __device__ __align__(256) double scratch[SP_DOUBLES];

namespace {
constexpr int SP_MAX_DEVICES = 64;
std::mutex g_sp_mu;
double *g_sp_ptr[SP_MAX_DEVICES] = {};  // device address of `scratch`

// Device address of the scratch array on the current device, looked up
// on the first call made with that device current.
int static_scratch(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    g_create_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return VP_EDEVICE;
  }
  if (dev < 0 || dev >= SP_MAX_DEVICES) {
    g_create_error = "device index beyond the static scratch table";
    return VP_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_sp_mu);
  if (!g_sp_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      g_create_error = std::string("hipGetSymbolAddress: ") +
                       hipGetErrorString(e);
      return VP_EDEVICE;
    }
    g_sp_ptr[dev] = static_cast<double *>(ptr);
  }
  *out = g_sp_ptr[dev];
  return VP_OK;
}
}  // namespace

extern "C" int vp_poisson_static(const vp_params *p, const double *rho,
                                 double *a, double *da, double *d2a,
                                 void *hip_stream) {
  if (!params_ok(p) || !rho || !a || !da || !d2a) {
    g_create_error = "invalid parameters or null pointer";
    return VP_EINVAL;
  }
  if ((size_t)p->nx > SP_NX) {
    g_create_error = "nx above VP_POISSON_STATIC_MAX_NX";
    return VP_EINVAL;
  }
  double *sp = nullptr;
  if (const int rc = static_scratch(&sp)) return rc;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const KP k = make_kp(p);
  FieldArgs A{};
  A.in = rho;
  A.ngy = 0;
  A.in_is_rho = 1;
  A.Mc = sp + SP_MC;
  A.ctot = sp + SP_CTOT;
  A.fcnt = reinterpret_cast<int *>(sp + SP_CNT);
  A.Ml = sp + SP_ML;
  A.acc = sp + SP_ACC;
  A.rmx = sp + SP_RMX;
  A.a_out = a;
  A.da_out = da;
  A.d2a_out = d2a;
  // the finished-chunk counter starts at zero (a fill kernel, so that the
  // call can be captured into a graph)
  hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, s, A.fcnt, 1LL, 0);
  hipError_t e = hipGetLastError();
  const char *where = "k_fill";
  if (e == hipSuccess) e = field_launches(k, A, s, &where);
  if (e != hipSuccess) {
    g_create_error = std::string(where) + ": " + hipGetErrorString(e);
    return VP_EDEVICE;
  }
  return VP_OK;
}

// ================================================================ serving

namespace {

// First-fit allocator over the server pool (256-byte granules).
class PoolAlloc {
 public:
  void init(size_t base, size_t size) {
    free_.clear();
    if (size) free_[base] = size;
  }
  bool alloc(size_t bytes, size_t &off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Slot {
  bool used = false;
  vp_ctx *c = nullptr;
  int req = -1;
  int nsteps = 0, done = 0;
  bool need_predict = true;
  int list_h = 0;  // half steps since reset at which the live lists were built
  size_t off = 0, bytes = 0;
};

constexpr int RING = 8;          // host work-table buffers in flight
constexpr int MAX_INFLIGHT = 3;  // ticks enqueued ahead of the device
// fixed grids of the batched kernels; the tile grid is larger than the
// device holds at once, so that the dispatcher balances uneven tiles
constexpr int GRID_TILE = 8192;
constexpr int GRID_ELEM = 2048;
constexpr int GRID_FIT = 1024;
constexpr int GRID_FIELD = 256;

size_t header_bytes(int precision) {
  const size_t rd = precision == VP_MIXED ? sizeof(RunDesc<float>)
                                          : sizeof(RunDesc<double>);
  return align_up(MAXR * rd) + align_up(NPH * sizeof(PhaseTable));
}

}  // namespace

struct vp_server {
  int precision = VP_FP64;
  int max_active = 1;
  hipStream_t caller = nullptr, stream = nullptr;
  char *pool = nullptr;
  size_t pool_bytes = 0;
  void *runs_dev = nullptr;
  PhaseTable *tabs_dev = nullptr;
  std::vector<char> runs_host;  // RunDesc mirror, one per slot
  PhaseTable *ring = nullptr;   // pinned host [RING][NPH]
  hipGraph_t graph = nullptr, graph_lean = nullptr;
  hipGraphExec_t exec = nullptr, exec_lean = nullptr;
  bool use_graph = false;
  PoolAlloc alloc;
  Slot slot[MAXR];
  std::string err;

  size_t rd_size() const {
    return precision == VP_MIXED ? sizeof(RunDesc<float>)
                                 : sizeof(RunDesc<double>);
  }
};

namespace {

int srv_fail(vp_server *s, hipError_t e, const char *where) {
  s->err = std::string(where) + ": " + hipGetErrorString(e);
  return VP_EDEVICE;
}

// The launches of one tick.  lean: only the reconstruction, field and kick
// phases -- a tick in which no run starts, resamples or finishes leaves the
// other phases' tables empty, and their launches would find nothing to do.
template <typename FT>
void launch_tick_kernels(vp_server *s, bool lean) {
  const RunDesc<FT> *runs = reinterpret_cast<const RunDesc<FT> *>(s->runs_dev);
  const PhaseTable *t = s->tabs_dev;
  hipStream_t st = s->stream;
  if (!lean)
    hipLaunchKernelGGL(kb_elem<FT>, dim3(GRID_ELEM), dim3(256), 0, st, runs,
                       t + PH_PRED);
  hipLaunchKernelGGL((kb_recon<FT, MODE_DENSITY>), dim3(GRID_TILE), dim3(512),
                     0, st, runs, t + PH_RECON);
  hipLaunchKernelGGL(kb_field<FT>, dim3(GRID_FIELD), dim3(FIELD_WG), 0, st,
                     runs, t + PH_FIELD);
  hipLaunchKernelGGL(kb_elem<FT>, dim3(GRID_ELEM), dim3(256), 0, st, runs,
                     t + PH_KICK);
  if (lean) return;
  hipLaunchKernelGGL(kb_elem<FT>, dim3(GRID_ELEM), dim3(256), 0, st, runs,
                     t + PH_RM_PRED);
  hipLaunchKernelGGL(kb_remap<FT>, dim3(GRID_TILE), dim3(512), 0, st, runs,
                     t + PH_RM_EVAL);
  hipLaunchKernelGGL(kb_fit_x<FT>, dim3(GRID_FIT), dim3(FIT_THREADS), 0, st,
                     runs, t + PH_FIT_X);
  hipLaunchKernelGGL(kb_fit_v<FT>, dim3(GRID_FIT), dim3(FIT_THREADS), 0, st,
                     runs, t + PH_FIT_V);
  hipLaunchKernelGGL(kb_ghost<FT>, dim3(GRID_FIT), dim3(256), 0, st, runs,
                     t + PH_GHOST);
  hipLaunchKernelGGL(kb_elem<FT>, dim3(GRID_ELEM), dim3(256), 0, st, runs,
                     t + PH_RESET);
  hipLaunchKernelGGL(kb_elem<FT>, dim3(GRID_ELEM), dim3(256), 0, st, runs,
                     t + PH_FIN_PRED);
  hipLaunchKernelGGL((kb_recon<FT, MODE_F>), dim3(GRID_TILE), dim3(512), 0, st,
                     runs, t + PH_FIN_RECON);
  hipLaunchKernelGGL(kb_elem<FT>, dim3(GRID_ELEM), dim3(256), 0, st, runs,
                     t + PH_FIN_ZERO);
}

void tick_kernels(vp_server *s, bool lean) {
  if (s->precision == VP_MIXED)
    launch_tick_kernels<float>(s, lean);
  else
    launch_tick_kernels<double>(s, lean);
}

template <typename FT>
void fill_desc(vp_ctx *c, void *fout, void *dst) {
  RunDesc<FT> d{};
  d.k = c->k;
  d.nb = c->L.nb;
  d.st = c->at<double>(c->L.st);
  d.rec = c->at<double>(c->L.rec);
  d.qm = c->at<double>(c->L.qm);
  d.part = c->at<double>(c->L.part);
  d.Mc = c->at<double>(c->L.Mc);
  d.ctot = c->at<double>(c->L.ctot);
  d.Ml = c->at<double>(c->L.Ml);
  d.acc = c->at<double>(c->L.acc);
  d.dpart = c->at<double>(c->L.dpart);
  d.cnt = c->counts(0);
  d.lst = c->at<int>(c->L.lst);
  d.flags = c->at<int>(c->L.flags);
  d.fcnt = c->at<int>(c->L.fcnt);
  d.ovf = c->at<unsigned long long>(c->L.ovf);
  d.F = c->at<FT>(c->L.F);
  d.C = c->at<FT>(c->L.C);
  d.T = c->at<FT>(c->L.T);
  d.tab = c->at<FT>(c->L.tab);
  d.fout = reinterpret_cast<FT *>(fout);
  std::memcpy(dst, &d, sizeof(d));
}

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Work tables of one tick for every resident run, in slot order.  Returns
// the slots that finish with this tick.  Advances the host mirror of each
// run (step count, live count buffer, pending predictor).
void build_tick(vp_server *s, PhaseTable *tab, std::vector<int> &finishing) {
  for (int ph = 0; ph < NPH; ++ph) {
    tab[ph].n = 0;
    tab[ph].total = 0;
  }
  // h: half steps since the run's last element reset at which block lists
  // are built (registration phases) or were built (query phases)
  auto add = [&](int ph, int slot, int items, int arg, int h = 0) {
    PhaseTable &t = tab[ph];
    if (items <= 0) return;
    t.it[t.n].slot = slot;
    t.it[t.n].begin = t.total;
    t.it[t.n].arg = arg;
    t.it[t.n].h = h;
    t.n += 1;
    t.total += items;
  };
  finishing.clear();
  for (int q = 0; q < s->max_active; ++q) {
    Slot &sl = s->slot[q];
    if (!sl.used || sl.done >= sl.nsteps) continue;
    vp_ctx *c = sl.c;
    const KP &k = c->k;
    const int cur = c->cur;
    // predict items of strides up to 8 take one lattice patch each and
    // claim their list slots through the workgroup's table (EA_TAB): a
    // tick's element launch spans every resident run, where the device
    // atomics queue
    const bool tabr = k.sx <= 8 && k.sv <= 8;
    const int tb = tabr ? EA_TAB : 0;
    const long long pe =
        tabr ? std::max<long long>(k.E, 256LL * elem_patches(k.mx, k.mv))
             : k.E;
    const int el_items = ceil_div(pe, 256);
    const int elz_items = ceil_div(std::max<long long>(pe, c->L.nb), 256);
    const int tiles = k.nbx * k.ngy;
    const int regb = cur ? EA_REGBUF1 : 0, zb = cur ? EA_ZEROBUF1 : 0;
    const int since = (int)(sl.done - c->reset_step);
    if (sl.need_predict) {
      sl.list_h = 2 * since + 1;
      add(PH_PRED, q, el_items, EA_PRED | EA_DRIFT | EA_REG | regb | tb,
          sl.list_h);
    }
    add(PH_RECON, q, tiles, cur, sl.list_h);
    add(PH_FIELD, q, (k.nx + FIELD_WG - 1) / FIELD_WG, 0);
    const int step_after = sl.done + 1;
    const bool remap_due = c->p.n_s > 0 && step_after % c->p.n_s == 0;
    const bool finish = step_after == sl.nsteps;
    if (!remap_due && !finish) {
      sl.list_h = 2 * (step_after - (int)c->reset_step) + 1;
      add(PH_KICK, q, elz_items,
          EA_KICK | EA_DRIFT | EA_PRED | EA_REG | (cur ? 0 : EA_REGBUF1) |
              EA_ZERO | zb | tb, sl.list_h);
      c->cur ^= 1;
      sl.need_predict = false;
    } else {
      add(PH_KICK, q, elz_items, EA_KICK | EA_ZERO | zb);
      sl.need_predict = true;
    }
    const int cr = c->cur;
    const int regr = cr ? EA_REGBUF1 : 0, zr = cr ? EA_ZEROBUF1 : 0;
    if (remap_due) {
      const int hr = 2 * (step_after - (int)c->reset_step);
      add(PH_RM_PRED, q, el_items, EA_PRED | EA_REG | regr | tb, hr);
      add(PH_RM_EVAL, q, tiles, cr, hr);
      const int sx = c->mixed() ? fit_segments<float>(k.nx)
                                : fit_segments<double>(k.nx);
      const int sv = c->mixed() ? fit_segments<float>(k.nv)
                                : fit_segments<double>(k.nv);
      add(PH_FIT_X, q, ceil_div(k.nv, 64) * sx, 0);
      add(PH_FIT_V, q, ceil_div(k.nx, 64) * sv, 0);
      add(PH_GHOST, q, ceil_div(k.nv + 2, 256), 0);
      add(PH_RESET, q, elz_items, EA_RESET | EA_ZERO | zr);
      c->reset_step = step_after;
    }
    if (finish) {
      const int hf = 2 * (step_after - (int)c->reset_step);
      add(PH_FIN_PRED, q, el_items, EA_PRED | EA_REG | regr | tb, hf);
      add(PH_FIN_RECON, q, tiles, cr, hf);
      add(PH_FIN_ZERO, q, ceil_div(c->L.nb, 256), EA_ZERO | zr);
      finishing.push_back(q);
    }
    sl.done = step_after;
    c->step = step_after;
    c->t = (double)step_after * c->p.dt;
  }
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

int vp_server_footprint(int precision, size_t *bytes) {
  if (!bytes || (precision != VP_FP64 && precision != VP_MIXED))
    return VP_EINVAL;
  *bytes = header_bytes(precision);
  return VP_OK;
}

int vp_server_create(int precision, int max_active, void *dev_pool,
                     size_t pool_bytes, void *hip_stream, vp_server **out) {
  if (!out) return VP_EINVAL;
  *out = nullptr;
  if ((precision != VP_FP64 && precision != VP_MIXED) || max_active < 1 ||
      max_active > MAXR || !dev_pool ||
      reinterpret_cast<uintptr_t>(dev_pool) % 256 != 0 ||
      pool_bytes <= header_bytes(precision)) {
    g_create_error = "invalid server arguments";
    return VP_EINVAL;
  }
  vp_server *s = new (std::nothrow) vp_server();
  if (!s) return VP_ENOMEM;
  s->precision = precision;
  s->max_active = max_active;
  s->caller = reinterpret_cast<hipStream_t>(hip_stream);
  s->pool = reinterpret_cast<char *>(dev_pool);
  s->pool_bytes = pool_bytes;
  const size_t runs_bytes = align_up(MAXR * s->rd_size());
  s->runs_dev = s->pool;
  s->tabs_dev = reinterpret_cast<PhaseTable *>(s->pool + runs_bytes);
  s->runs_host.assign(MAXR * s->rd_size(), 0);
  s->alloc.init(header_bytes(precision), pool_bytes - header_bytes(precision));
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&s->ring),
                      sizeof(PhaseTable) * NPH * RING, hipHostMallocDefault);
  if (e != hipSuccess) {
    g_create_error = std::string("server set-up: ") + hipGetErrorString(e);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return VP_EDEVICE;
  }
  std::memset(s->ring, 0, sizeof(PhaseTable) * NPH * RING);
  // empty work tables on the device before anything runs
  e = hipMemcpyAsync(s->tabs_dev, s->ring, sizeof(PhaseTable) * NPH,
                     hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  // capture the launch sequence of one tick, full and lean
  for (int lean = 0; lean < 2 && e == hipSuccess; ++lean) {
    if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) !=
        hipSuccess)
      break;
    tick_kernels(s, lean == 1);
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    if (hipStreamEndCapture(s->stream, &g) == hipSuccess && g &&
        hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess) {
      (lean ? s->graph_lean : s->graph) = g;
      (lean ? s->exec_lean : s->exec) = x;
    } else {
      if (g) (void)hipGraphDestroy(g);
      break;
    }
  }
  s->use_graph = s->exec && s->exec_lean;
  (void)hipGetLastError();
  if (e != hipSuccess) {
    g_create_error = std::string("server set-up: ") + hipGetErrorString(e);
    (void)hipStreamDestroy(s->stream);
    (void)hipHostFree(s->ring);
    delete s;
    return VP_EDEVICE;
  }
  *out = s;
  return VP_OK;
}

int vp_server_destroy(vp_server *s) {
  if (!s) return VP_EINVAL;
  (void)hipStreamSynchronize(s->stream);
  for (int q = 0; q < MAXR; ++q) delete s->slot[q].c;
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->exec_lean) (void)hipGraphExecDestroy(s->exec_lean);
  if (s->graph_lean) (void)hipGraphDestroy(s->graph_lean);
  if (s->ring) (void)hipHostFree(s->ring);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return VP_OK;
}

const char *vp_server_last_error(vp_server *s) {
  return s ? s->err.c_str() : g_create_error.c_str();
}

int vp_server_run(vp_server *s, const vp_request *reqs, int n,
                  vp_request_result *res, vp_server_stats *stats) {
  if (!s || (n > 0 && (!reqs || !res))) return VP_EINVAL;
  for (int i = 1; i < n; ++i)
    if (reqs[i].arrival_s < reqs[i - 1].arrival_s) return VP_EINVAL;
  hipError_t e;
  // order after the caller's pending work (inputs)
  hipEvent_t ev_in;
  if ((e = hipEventCreateWithFlags(&ev_in, hipEventDisableTiming)) != hipSuccess)
    return srv_fail(s, e, "event");
  (void)hipEventRecord(ev_in, s->caller);
  (void)hipStreamWaitEvent(s->stream, ev_in, 0);
  // per-tick timing events
  struct Tick {
    hipEvent_t a, b;
    std::vector<int> finishing;
    int ring;
  };
  std::vector<hipEvent_t> evpool;
  auto get_ev = [&]() {
    hipEvent_t ev;
    if (!evpool.empty()) {
      ev = evpool.back();
      evpool.pop_back();
    } else if (hipEventCreate(&ev) != hipSuccess) {
      ev = nullptr;
    }
    return ev;
  };
  std::vector<Tick> inflight;  // FIFO
  std::vector<int> waiting;    // request ids, FIFO
  size_t wait_head = 0;
  int next = 0, completed = 0, active = 0, ring_pos = 0;
  vp_server_stats st{};
  st.graph_replay = s->use_graph ? 1 : 0;
  for (int i = 0; i < n; ++i) {
    res[i].tag = reqs[i].tag;
    res[i].arrival_s = reqs[i].arrival_s;
    res[i].admit_s = res[i].done_s = -1.0;
    res[i].status = VP_OK;
  }
  const double t0 = now_s();
  double busy = 0.0;
  int rc = VP_OK;

  auto retire = [&](Tick &tk, double tnow) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, tk.a, tk.b) == hipSuccess) busy += ms * 1e-3;
    for (int q : tk.finishing) {
      Slot &sl = s->slot[q];
      res[sl.req].done_s = tnow;
      st.site_updates += (int64_t)sl.c->k.nx * sl.c->k.nv * sl.nsteps;
      delete sl.c;  // the device is done with it: its last tick completed
      s->alloc.release(sl.off, sl.bytes);
      sl = Slot();
      active -= 1;
      completed += 1;
    }
    evpool.push_back(tk.a);
    evpool.push_back(tk.b);
  };

  while (completed < n && rc == VP_OK) {
    double tnow = now_s() - t0;
    while (next < n && reqs[next].arrival_s <= tnow) waiting.push_back(next++);
    // completions
    while (!inflight.empty() &&
           hipEventQuery(inflight.front().b) == hipSuccess) {
      retire(inflight.front(), now_s() - t0);
      inflight.erase(inflight.begin());
    }
    // admissions, first come first served
    while (wait_head < waiting.size()) {
      const int r = waiting[wait_head];
      const vp_request &rq = reqs[r];
      size_t need = 0;
      int q = -1;
      if (rq.params.precision != s->precision || rq.nsteps < 1 ||
          !rq.f0_dev || !rq.f_out_dev || rq.params.emap_max > 0.0 ||
          rq.params.c_dyn > 0.0 || rq.params.bc != VP_BC_ISOLATED ||
          vp_footprint(&rq.params, &need) != VP_OK ||
          align_up(need) > s->pool_bytes - header_bytes(s->precision)) {
        res[r].status = VP_EINVAL;
        res[r].admit_s = res[r].done_s = now_s() - t0;
        completed += 1;
        wait_head += 1;
        continue;
      }
      for (int i = 0; i < s->max_active; ++i)
        if (!s->slot[i].used) {
          q = i;
          break;
        }
      size_t off = 0;
      if (q < 0 || !s->alloc.alloc(need, off)) break;
      vp_ctx *c = nullptr;
      int r1 = vp_create(&rq.params, s->pool + off, align_up(need), s->stream,
                         &c);
      if (r1 == VP_OK) r1 = vp_init_conditions(c, rq.f0_dev, 1);
      if (r1 != VP_OK) {
        s->err = c ? c->err : g_create_error;
        delete c;
        s->alloc.release(off, need);
        res[r].status = r1;
        res[r].admit_s = res[r].done_s = now_s() - t0;
        completed += 1;
        wait_head += 1;
        continue;
      }
      Slot &sl = s->slot[q];
      sl.used = true;
      sl.c = c;
      sl.req = r;
      sl.nsteps = rq.nsteps;
      sl.done = 0;
      sl.need_predict = true;
      sl.off = off;
      sl.bytes = need;
      if (s->precision == VP_MIXED)
        fill_desc<float>(c, rq.f_out_dev, s->runs_host.data() + q * s->rd_size());
      else
        fill_desc<double>(c, rq.f_out_dev,
                          s->runs_host.data() + q * s->rd_size());
      e = hipMemcpyAsync(reinterpret_cast<char *>(s->runs_dev) + q * s->rd_size(),
                         s->runs_host.data() + q * s->rd_size(), s->rd_size(),
                         hipMemcpyHostToDevice, s->stream);
      if (e != hipSuccess) {
        rc = srv_fail(s, e, "run table upload");
        break;
      }
      res[r].admit_s = now_s() - t0;
      active += 1;
      st.admitted += 1;
      if (active > st.max_active) st.max_active = active;
      wait_head += 1;
    }
    if (rc) break;
    if (active == 0 || (int)inflight.size() >= MAX_INFLIGHT ||
        // every resident run already has all its ticks enqueued
        [&]() {
          for (int q = 0; q < s->max_active; ++q)
            if (s->slot[q].used && s->slot[q].done < s->slot[q].nsteps)
              return false;
          return true;
        }()) {
      if (!inflight.empty()) {
        e = hipEventSynchronize(inflight.front().b);
        if (e != hipSuccess) {
          rc = srv_fail(s, e, "tick wait");
          break;
        }
        retire(inflight.front(), now_s() - t0);
        inflight.erase(inflight.begin());
      } else if (next < n) {
        const double dt = reqs[next].arrival_s - (now_s() - t0);
        if (dt > 0)
          std::this_thread::sleep_for(std::chrono::duration<double>(
              std::min(dt, 1e-3)));
      }
      continue;
    }
    // one tick for every resident run
    Tick tk;
    tk.ring = ring_pos;
    ring_pos = (ring_pos + 1) % RING;
    PhaseTable *tab = s->ring + (size_t)tk.ring * NPH;
    build_tick(s, tab, tk.finishing);
    tk.a = get_ev();
    tk.b = get_ev();
    if (!tk.a || !tk.b) {
      rc = srv_fail(s, hipErrorOutOfMemory, "event");
      break;
    }
    (void)hipEventRecord(tk.a, s->stream);
    e = hipMemcpyAsync(s->tabs_dev, tab, sizeof(PhaseTable) * NPH,
                       hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) {
      bool lean = true;
      for (int ph = 0; ph < NPH && lean; ++ph)
        if (ph != PH_RECON && ph != PH_FIELD && ph != PH_KICK &&
            tab[ph].total > 0)
          lean = false;
      if (s->use_graph) {
        e = hipGraphLaunch(lean ? s->exec_lean : s->exec, s->stream);
      } else {
        tick_kernels(s, lean);
        e = hipGetLastError();
      }
    }
    if (e != hipSuccess) {
      rc = srv_fail(s, e, "tick launch");
      break;
    }
    (void)hipEventRecord(tk.b, s->stream);
    st.ticks += 1;
    inflight.push_back(tk);
  }
  // drain
  (void)hipStreamSynchronize(s->stream);
  while (!inflight.empty()) {
    retire(inflight.front(), now_s() - t0);
    inflight.erase(inflight.begin());
  }
  for (hipEvent_t ev : evpool) (void)hipEventDestroy(ev);
  (void)hipEventRecord(ev_in, s->stream);
  (void)hipStreamWaitEvent(s->caller, ev_in, 0);
  (void)hipEventDestroy(ev_in);
  double first = n ? reqs[0].arrival_s : 0.0, last = 0.0;
  for (int i = 0; i < n; ++i) last = std::max(last, res[i].done_s);
  st.wall_s = last - first;
  st.gpu_busy_s = busy;
  st.completed = completed;
  if (stats) *stats = st;
  return rc;
}

}  // extern "C"
