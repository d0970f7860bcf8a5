// vp4_engine.hip -- host side of the 4D phase-space engine (C ABI of
// include/vp4.h): workspace carving, launch sequences, pivot and twiddle
// tables, profiling events.
#include "vp4.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "vp4_kernels.hpp"

using namespace vp4k;

namespace {

thread_local std::string g_err4;

struct Layout {
  size_t F, C, fs, st, rec, cnt, lst, flags, part, rho, re, im, ar, ai, tr, ti,
      fld, tw, tabs, tabv, dpart, dout, total;
  long long nb, nl;  // query blocks, lists
};

constexpr int NDIAG = 256;  // workgroups of the diagnostic partial sums

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool params_ok(const vp4_params *p) {
  return p && p->ns >= 8 && p->nv >= 4 && p->ns <= 512 && p->nv <= 512 &&
         p->ss >= 1 && p->sv >= 1 && p->ns % 4 == 0 && p->nv % 4 == 0 &&
         p->ns % p->ss == 0 && p->nv % p->sv == 0 && p->L > 0.0 &&
         std::isfinite(p->L) && p->vmax > 0.0 && std::isfinite(p->vmax) &&
         p->dt > 0.0 && p->n_s >= 0 && p->beta >= 0.0 && p->beta <= 0.5 &&
         std::isfinite(p->G) &&
         (p->precision == VP4_FP64 || p->precision == VP4_MIXED) &&
         (long long)p->ns * p->ns * p->nv * p->nv <= (1ll << 31) &&
         (long long)(p->ns / p->ss) * (p->ns / p->ss) * (p->nv / p->sv) *
                 (p->nv / p->sv) <= (1ll << 24);
}

// list slots per 4^4 block: twice the elements whose undeformed windows
// can reach one block
int list_cap(int ss, int sv) {
  auto per = [](int s) { return (BLK + s - 1) / s + 2; };
  long long c = 2ll * per(ss) * per(ss) * per(sv) * per(sv);
  return (int)std::min<long long>(std::max<long long>(c, 64), 1024);
}

KP make_kp(const vp4_params *p) {
  KP k{};
  k.ns = p->ns;
  k.nv = p->nv;
  k.ss = p->ss;
  k.sv = p->sv;
  k.ms = p->ns / p->ss;
  k.mv = p->nv / p->sv;
  k.E = k.ms * k.ms * k.mv * k.mv;
  for (int a = 0; a < 4; ++a) {
    const int sp = a < 2 ? p->ss : p->sv, n = a < 2 ? p->ns : p->nv;
    k.o[a] = (sp / 2) % BLK;
    k.ob[a] = k.o[a] > 0;
    k.nb[a] = (n - 1 - k.o[a]) / BLK + k.ob[a] + 1;
  }
  k.nls = p->ns / BLK;
  k.cap = list_cap(p->ss, p->sv);
  k.L = p->L;
  k.hL = 0.5 * p->L;
  k.vmax = p->vmax;
  k.dx = p->L / p->ns;
  k.du = 2.0 * p->vmax / p->nv;
  k.inv_dx = 1.0 / k.dx;
  k.inv_du = 1.0 / k.du;
  k.G = p->G;
  k.dt = p->dt;
  k.h = 0.5 * p->dt;
  k.beta = p->beta;
  for (int a = 0; a < 4; ++a) {
    k.Dm[a] = a < 2 ? p->ss * k.dx : p->sv * k.du;
    k.rD[a] = 1.0 / k.Dm[a];
  }
  return k;
}

Layout make_layout(const vp4_params *p, const KP &k) {
  Layout L{};
  const size_t fb = p->precision == VP4_MIXED ? 4 : 8;
  const size_t N4 = (size_t)k.ns * k.ns * k.nv * k.nv, n2 = (size_t)k.ns * k.ns;
  L.nb = (long long)k.nb[0] * k.nb[1] * k.nb[2] * k.nb[3];
  L.nl = (long long)k.nls * k.nls * k.nb[2] * k.nb[3];
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = align_up(o + b);
    return at;
  };
  L.F = take(N4 * fb);
  L.C = take(N4 * fb);
  L.fs = take(N4 * fb);
  L.st = take((size_t)NST * k.E * 8);
  L.rec = take((size_t)RS * k.E * 8);
  L.cnt = take((size_t)L.nl * 4);
  L.lst = take((size_t)L.nl * k.cap * 4);
  L.flags = take(64);
  L.part = take((size_t)k.nb[2] * k.nb[3] * n2 * 8);
  L.rho = take(n2 * 8);
  L.re = take(n2 * 8);
  L.im = take(n2 * 8);
  L.ar = take(2 * n2 * 8);
  L.ai = take(2 * n2 * 8);
  L.tr = take(2 * n2 * 8);
  L.ti = take(2 * n2 * 8);
  L.fld = take(12 * n2 * 8);
  L.tw = take(2 * (size_t)k.ns * 8);
  L.tabs = take((3 * (size_t)k.ns + 1) * fb);
  L.tabv = take(2 * (size_t)k.nv * fb);
  L.dpart = take(3 * NDIAG * 8);
  L.dout = take(8 * 8);
  L.total = o;
  return L;
}

enum { PK_PREDICT = 0, PK_RECON, PK_FIELD, PK_KICK, PK_REMAP, PK_FIT, PK_OTHER,
       PK_N };

}  // namespace

struct vp4_ctx {
  vp4_params p;
  KP k;
  Layout L;
  hipStream_t stream;
  char *ws;
  int64_t step = 0;
  bool ready = false;
  std::string err;
  std::vector<char> host_tab;
  bool prof = false;
  int prof_cap = 0;
  std::vector<hipEvent_t> ev[PK_N];
  int ev_used[PK_N] = {};
  template <typename T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(ws + off);
  }
  bool mixed() const { return p.precision == VP4_MIXED; }
};

namespace {

int dev_fail(vp4_ctx *c, hipError_t e, const char *where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return VP4_EDEVICE;
}

#define VP4_CHECK(c, where)                              \
  do {                                                   \
    hipError_t _e = hipGetLastError();                   \
    if (_e != hipSuccess) return dev_fail(c, _e, where); \
  } while (0)

struct Prof {
  vp4_ctx *c;
  int kind;
  bool on = false;
  Prof(vp4_ctx *c_, int k) : c(c_), kind(k) {
    if (c->prof && c->ev_used[kind] < c->prof_cap) {
      on = true;
      (void)hipEventRecord(c->ev[kind][2 * c->ev_used[kind]], c->stream);
    }
  }
  ~Prof() {
    if (on) {
      (void)hipEventRecord(c->ev[kind][2 * c->ev_used[kind] + 1], c->stream);
      c->ev_used[kind] += 1;
    }
  }
};

unsigned grid_for(long long n, int bs) {
  long long g = (n + bs - 1) / bs;
  return (unsigned)std::max<long long>(1, std::min<long long>(g, 1ll << 30));
}

int zero_counts(vp4_ctx *c) {
  hipLaunchKernelGGL(k4_zero, dim3(grid_for(std::min<long long>(c->L.nl, 1 << 22), 256)),
                     dim3(256), 0, c->stream, c->at<int>(c->L.cnt), c->L.nl);
  VP4_CHECK(c, "k4_zero");
  return VP4_OK;
}

// Records and block lists for the current elements (after the predictor's
// half drift when `drift`).
int predict(vp4_ctx *c, int drift) {
  int rc;
  if ((rc = zero_counts(c))) return rc;
  Prof ps(c, PK_PREDICT);
  hipLaunchKernelGGL(k4_predict, dim3(grid_for(c->k.E, 256)), dim3(256), 0,
                     c->stream, c->k, c->at<double>(c->L.st),
                     c->at<double>(c->L.rec), c->at<int>(c->L.cnt),
                     c->at<int>(c->L.lst), c->at<int>(c->L.flags), drift, 1);
  VP4_CHECK(c, "k4_predict");
  return VP4_OK;
}

template <typename FT, int MODE>
int recon_t(vp4_ctx *c, void *fout, int *aout) {
  Prof ps(c, PK_RECON);
  hipLaunchKernelGGL((k4_recon<FT, MODE>), dim3((unsigned)c->L.nb), dim3(256),
                     0, c->stream, c->k, c->at<double>(c->L.rec),
                     c->at<int>(c->L.cnt), c->at<int>(c->L.lst),
                     c->at<int>(c->L.flags), c->at<FT>(c->L.F),
                     c->at<double>(c->L.part), reinterpret_cast<FT *>(fout),
                     aout);
  VP4_CHECK(c, "k4_recon");
  return VP4_OK;
}

template <int MODE>
int recon(vp4_ctx *c, void *fout, int *aout) {
  return c->mixed() ? recon_t<float, MODE>(c, fout, aout)
                    : recon_t<double, MODE>(c, fout, aout);
}

// Force fields from a density: DFT along x, along y with the spectra of
// a_x and a_y, the inverse transforms, then the finite differences.
int field_from(vp4_ctx *c, const double *rho) {
  Prof ps(c, PK_FIELD);
  const KP &k = c->k;
  const long long n2 = (long long)k.ns * k.ns;
  const double *tw = c->at<double>(c->L.tw);
  double *re = c->at<double>(c->L.re), *im = c->at<double>(c->L.im);
  double *ar = c->at<double>(c->L.ar), *ai = c->at<double>(c->L.ai);
  double *tr = c->at<double>(c->L.tr), *ti = c->at<double>(c->L.ti);
  double *fld = c->at<double>(c->L.fld);
  hipLaunchKernelGGL(k4_dft_x, dim3(grid_for(n2, 256)), dim3(256), 0, c->stream,
                     k, rho, tw, re, im);
  hipLaunchKernelGGL(k4_dft_y_spec, dim3(grid_for(n2, 256)), dim3(256), 0,
                     c->stream, k, re, im, tw, ar, ai);
  hipLaunchKernelGGL(k4_idft_y, dim3(grid_for(2 * n2, 256)), dim3(256), 0,
                     c->stream, k, ar, ai, tw, tr, ti);
  hipLaunchKernelGGL(k4_idft_x, dim3(grid_for(2 * n2, 256)), dim3(256), 0,
                     c->stream, k, tr, ti, tw, fld);
  hipLaunchKernelGGL(k4_fd, dim3(grid_for(n2, 256)), dim3(256), 0, c->stream,
                     k, fld);
  VP4_CHECK(c, "k4 field");
  return VP4_OK;
}

int density_field(vp4_ctx *c, double *rho_out) {
  int rc;
  if ((rc = recon<M_DENSITY>(c, nullptr, nullptr))) return rc;
  double *rho = rho_out ? rho_out : c->at<double>(c->L.rho);
  hipLaunchKernelGGL(k4_rho, dim3(grid_for((long long)c->k.ns * c->k.ns, 256)),
                     dim3(256), 0, c->stream, c->k, c->at<double>(c->L.part),
                     rho);
  VP4_CHECK(c, "k4_rho");
  return field_from(c, rho);
}

template <typename FT>
int fit_t(vp4_ctx *c) {
  Prof ps(c, PK_FIT);
  const KP &k = c->k;
  const size_t N4 = (size_t)k.ns * k.ns * k.nv * k.nv;
  FT *C = c->at<FT>(c->L.C);
  hipError_t e = hipMemcpyAsync(C, c->at<FT>(c->L.F), N4 * sizeof(FT),
                                hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "fit copy");
  for (int ax = 0; ax < 4; ++ax) {
    const int n = ax < 2 ? k.ns : k.nv;
    const FT *tab = ax < 2 ? c->at<FT>(c->L.tabs) : c->at<FT>(c->L.tabv);
    hipLaunchKernelGGL((k4_fit<FT>), dim3(grid_for((long long)(N4 / n), 256)),
                       dim3(256), 0, c->stream, k, C, ax, tab);
  }
  VP4_CHECK(c, "k4_fit");
  return VP4_OK;
}

int fit(vp4_ctx *c) { return c->mixed() ? fit_t<float>(c) : fit_t<double>(c); }

int reset(vp4_ctx *c) {
  hipLaunchKernelGGL(k4_reset, dim3(grid_for(c->k.E, 256)), dim3(256), 0,
                     c->stream, c->k, c->at<double>(c->L.st));
  VP4_CHECK(c, "k4_reset");
  return VP4_OK;
}

template <typename FT>
int remap_eval_t(vp4_ctx *c, void *out) {
  Prof ps(c, PK_REMAP);
  hipLaunchKernelGGL((k4_remap<FT>), dim3((unsigned)c->L.nb), dim3(256), 0,
                     c->stream, c->k, c->at<double>(c->L.rec),
                     c->at<int>(c->L.cnt), c->at<int>(c->L.lst),
                     c->at<int>(c->L.flags), c->at<FT>(c->L.C),
                     reinterpret_cast<FT *>(out));
  VP4_CHECK(c, "k4_remap");
  return VP4_OK;
}

int remap_eval(vp4_ctx *c, void *out) {
  return c->mixed() ? remap_eval_t<float>(c, out) : remap_eval_t<double>(c, out);
}

int do_remap(vp4_ctx *c) {
  int rc;
  if ((rc = predict(c, 0))) return rc;
  if ((rc = remap_eval(c, c->ws + c->L.F))) return rc;
  if ((rc = fit(c))) return rc;
  return reset(c);
}

int run_steps(vp4_ctx *c, int n) {
  int rc;
  for (int s = 0; s < n; ++s) {
    if ((rc = predict(c, 1))) return rc;
    if ((rc = density_field(c, nullptr))) return rc;
    {
      Prof ps(c, PK_KICK);
      hipLaunchKernelGGL(k4_kick, dim3(grid_for(c->k.E, 256)), dim3(256), 0,
                         c->stream, c->k, c->at<double>(c->L.st),
                         c->at<double>(c->L.fld));
      VP4_CHECK(c, "k4_kick");
    }
    c->step += 1;
    if (c->p.n_s > 0 && c->step % c->p.n_s == 0 && (rc = do_remap(c)))
      return rc;
  }
  return VP4_OK;
}

// Pivots of the (1, 4, 1) Thomas solve: mirror end rows (4, 2) / (2, 4), or
// the cyclic system's tridiagonal part (diagonal 8, 4, .., 4, 4.25) with z
// = B^-1 (-4, 0, .., 0, 1) and den = (1 + z_0) - z_{n-1} / 4.
template <typename FT>
void host_pivots(int n, bool cyclic, std::vector<FT> &out) {
  std::vector<FT> cp(n), ri(n);
  auto diag = [&](int i) -> FT {
    if (!cyclic) return (FT)4;
    return i == 0 ? (FT)8 : (i == n - 1 ? (FT)4.25 : (FT)4);
  };
  FT rinv = (FT)1 / diag(0);
  ri[0] = rinv;
  cp[0] = (cyclic ? (FT)1 : (FT)2) * rinv;
  for (int i = 1; i < n; ++i) {
    const FT sub = (!cyclic && i == n - 1) ? (FT)2 : (FT)1;
    const FT den = diag(i) - sub * cp[i - 1];
    rinv = (FT)1 / den;
    ri[i] = rinv;
    cp[i] = rinv;
  }
  out.assign(cp.begin(), cp.end());
  out.insert(out.end(), ri.begin(), ri.end());
  if (cyclic) {
    std::vector<FT> d(n), z(n);
    d[0] = (FT)-4 * ri[0];
    for (int i = 1; i < n; ++i) {
      const FT u = (i == n - 1) ? (FT)1 : (FT)0;
      d[i] = (u - d[i - 1]) * ri[i];
    }
    z[n - 1] = d[n - 1];
    for (int i = n - 2; i >= 0; --i) z[i] = d[i] - cp[i] * z[i + 1];
    out.insert(out.end(), z.begin(), z.end());
    out.push_back(((FT)1 + z[0]) - (FT)0.25 * z[n - 1]);
  }
}

template <typename FT>
int upload_tables(vp4_ctx *c) {
  std::vector<FT> ts, tv;
  host_pivots<FT>(c->k.ns, true, ts);
  host_pivots<FT>(c->k.nv, false, tv);
  std::vector<double> tw(2 * (size_t)c->k.ns);
  const double twopi = 6.283185307179586476925286766559;
  for (int m = 0; m < c->k.ns; ++m) {
    tw[m] = std::cos(twopi * (double)m / (double)c->k.ns);
    tw[c->k.ns + m] = std::sin(twopi * (double)m / (double)c->k.ns);
  }
  const size_t bs = ts.size() * sizeof(FT), bv = tv.size() * sizeof(FT),
               bw = tw.size() * sizeof(double);
  c->host_tab.resize(bs + bv + bw);
  std::copy(reinterpret_cast<const char *>(ts.data()),
            reinterpret_cast<const char *>(ts.data()) + bs, c->host_tab.data());
  std::copy(reinterpret_cast<const char *>(tv.data()),
            reinterpret_cast<const char *>(tv.data()) + bv,
            c->host_tab.data() + bs);
  std::copy(reinterpret_cast<const char *>(tw.data()),
            reinterpret_cast<const char *>(tw.data()) + bw,
            c->host_tab.data() + bs + bv);
  hipError_t e = hipMemcpyAsync(c->ws + c->L.tabs, c->host_tab.data(), bs,
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + c->L.tabv, c->host_tab.data() + bs, bv,
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + c->L.tw, c->host_tab.data() + bs + bv, bw,
                       hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "table upload");
  return VP4_OK;
}

int check_flags(vp4_ctx *c) {
  int fl = 0;
  hipError_t e = hipMemcpyAsync(&fl, c->at<int>(c->L.flags), sizeof(int),
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "flags read");
  if (fl & FL_NUMERIC) {
    c->err = "non-finite element or det T <= 0";
    return VP4_ENUMERIC;
  }
  return VP4_OK;
}

}  // namespace

extern "C" {

int vp4_footprint(const vp4_params *p, size_t *bytes) {
  if (!params_ok(p) || !bytes) return VP4_EINVAL;
  *bytes = make_layout(p, make_kp(p)).total;
  return VP4_OK;
}

int vp4_create(const vp4_params *p, void *ws, size_t bytes, void *stream,
               vp4_ctx **out) {
  if (!out) return VP4_EINVAL;
  *out = nullptr;
  if (!params_ok(p) || !ws) {
    g_err4 = "invalid parameters or null workspace";
    return VP4_EINVAL;
  }
  KP k = make_kp(p);
  Layout L = make_layout(p, k);
  if (bytes < L.total) {
    g_err4 = "workspace smaller than vp4_footprint";
    return VP4_ENOMEM;
  }
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
    g_err4 = "workspace must be 256-byte aligned";
    return VP4_EINVAL;
  }
  vp4_ctx *c = new (std::nothrow) vp4_ctx();
  if (!c) return VP4_ENOMEM;
  c->p = *p;
  c->k = k;
  c->L = L;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = reinterpret_cast<char *>(ws);
  hipLaunchKernelGGL(k4_zero, dim3(grid_for(std::min<long long>(L.total / 4, 1 << 22), 256)),
                     dim3(256), 0, c->stream, c->at<int>(0),
                     (long long)(L.total / 4));
  int rc = hipGetLastError() == hipSuccess ? VP4_OK : VP4_EDEVICE;
  if (!rc) rc = c->mixed() ? upload_tables<float>(c) : upload_tables<double>(c);
  if (!rc) rc = reset(c);
  if (rc) {
    g_err4 = c->err.empty() ? "device error" : c->err;
    delete c;
    return rc;
  }
  *out = c;
  return VP4_OK;
}

int vp4_destroy(vp4_ctx *c) {
  if (!c) return VP4_EINVAL;
  const hipError_t e = hipStreamSynchronize(c->stream);
  for (int k = 0; k < PK_N; ++k)
    for (hipEvent_t ev : c->ev[k])
      if (ev) (void)hipEventDestroy(ev);
  delete c;
  return e == hipSuccess ? VP4_OK : VP4_EDEVICE;
}

int vp4_init_conditions(vp4_ctx *c, const double *f0) {
  if (!c || !f0) return VP4_EINVAL;
  const long long N4 = (long long)c->k.ns * c->k.ns * c->k.nv * c->k.nv;
  if (c->mixed())
    hipLaunchKernelGGL((k4_load<float>), dim3(grid_for(std::min(N4, 1ll << 22), 256)),
                       dim3(256), 0, c->stream, c->k, f0, c->at<float>(c->L.F));
  else
    hipLaunchKernelGGL((k4_load<double>), dim3(grid_for(std::min(N4, 1ll << 22), 256)),
                       dim3(256), 0, c->stream, c->k, f0, c->at<double>(c->L.F));
  VP4_CHECK(c, "k4_load");
  int rc;
  if ((rc = fit(c))) return rc;
  if ((rc = reset(c))) return rc;
  c->step = 0;
  c->ready = true;
  return VP4_OK;
}

int vp4_step(vp4_ctx *c, int n) {
  if (!c || n < 0) return VP4_EINVAL;
  if (!c->ready) return VP4_ESTATE;
  return run_steps(c, n);
}

int vp4_remap(vp4_ctx *c) {
  if (!c) return VP4_EINVAL;
  if (!c->ready) return VP4_ESTATE;
  return do_remap(c);
}

int vp4_reconstruct_f(vp4_ctx *c, int scheme, void *f_out) {
  if (!c || !f_out || (scheme != 0 && scheme != 1)) return VP4_EINVAL;
  if (!c->ready) return VP4_ESTATE;
  int rc;
  if ((rc = predict(c, 0))) return rc;
  return scheme == 0 ? recon<M_F>(c, f_out, nullptr) : remap_eval(c, f_out);
}

int vp4_density(vp4_ctx *c, double *rho) {
  if (!c || !rho) return VP4_EINVAL;
  if (!c->ready) return VP4_ESTATE;
  int rc;
  if ((rc = predict(c, 0))) return rc;
  return density_field(c, rho);
}

int vp4_field(vp4_ctx *c, const double *rho, double *ax, double *ay) {
  if (!c || !rho || !ax || !ay) return VP4_EINVAL;
  int rc;
  if ((rc = field_from(c, rho))) return rc;
  const size_t n2 = (size_t)c->k.ns * c->k.ns * sizeof(double);
  hipError_t e = hipMemcpyAsync(ax, c->at<double>(c->L.fld), n2,
                                hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ay, c->at<double>(c->L.fld) + (size_t)c->k.ns * c->k.ns,
                       n2, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "field copy");
  return VP4_OK;
}

int vp4_diagnostics(vp4_ctx *c, double *out) {
  if (!c || !out) return VP4_EINVAL;
  if (!c->ready) return VP4_ESTATE;
  int rc;
  if ((rc = predict(c, 0))) return rc;
  if ((rc = density_field(c, nullptr))) return rc;
  if ((rc = recon<M_F>(c, c->ws + c->L.fs, nullptr))) return rc;
  if (c->mixed())
    hipLaunchKernelGGL((k4_diag_part<float>), dim3(NDIAG), dim3(256), 0,
                       c->stream, c->k, c->at<float>(c->L.fs),
                       c->at<double>(c->L.dpart));
  else
    hipLaunchKernelGGL((k4_diag_part<double>), dim3(NDIAG), dim3(256), 0,
                       c->stream, c->k, c->at<double>(c->L.fs),
                       c->at<double>(c->L.dpart));
  hipLaunchKernelGGL(k4_diag_final, dim3(1), dim3(256), 0, c->stream, c->k,
                     c->at<double>(c->L.dpart), NDIAG, c->at<double>(c->L.fld),
                     c->at<double>(c->L.dout));
  VP4_CHECK(c, "k4 diagnostics");
  double h[5];
  hipError_t e = hipMemcpyAsync(h, c->at<double>(c->L.dout), sizeof(h),
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "diagnostics read");
  for (int q = 0; q < 5; ++q) out[q] = h[q];
  out[5] = (double)c->step * c->p.dt;
  return check_flags(c);
}

int vp4_get_elements(vp4_ctx *c, double *el) {
  if (!c || !el) return VP4_EINVAL;
  hipError_t e = hipMemcpyAsync(el, c->at<double>(c->L.st),
                                (size_t)NST * c->k.E * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream);
  return e == hipSuccess ? VP4_OK : dev_fail(c, e, "get elements");
}

int vp4_set_elements(vp4_ctx *c, const double *el) {
  if (!c || !el) return VP4_EINVAL;
  hipError_t e = hipMemcpyAsync(c->at<double>(c->L.st), el,
                                (size_t)NST * c->k.E * sizeof(double),
                                hipMemcpyDeviceToDevice, c->stream);
  return e == hipSuccess ? VP4_OK : dev_fail(c, e, "set elements");
}

int vp4_get_assignment(vp4_ctx *c, int32_t *a) {
  if (!c || !a) return VP4_EINVAL;
  if (!c->ready) return VP4_ESTATE;
  int rc;
  if ((rc = predict(c, 0))) return rc;
  return recon<M_ASSIGN>(c, nullptr, a);
}

int vp4_prof_begin(vp4_ctx *c, int max_launches) {
  if (!c || max_launches < 1) return VP4_EINVAL;
  for (int k = 0; k < PK_N; ++k) {
    c->ev[k].assign(2 * (size_t)max_launches, nullptr);
    for (auto &ev : c->ev[k])
      if (hipEventCreate(&ev) != hipSuccess) return VP4_EDEVICE;
    c->ev_used[k] = 0;
  }
  c->prof_cap = max_launches;
  c->prof = true;
  return VP4_OK;
}

int vp4_prof_end(vp4_ctx *c, double *ms, int64_t *n) {
  if (!c || !c->prof) return VP4_ESTATE;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "prof sync");
  for (int k = 0; k < PK_N; ++k) {
    double tot = 0.0;
    for (int i = 0; i < c->ev_used[k]; ++i) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, c->ev[k][2 * i], c->ev[k][2 * i + 1]) ==
          hipSuccess)
        tot += t;
    }
    if (ms) ms[k] = tot;
    if (n) n[k] = c->ev_used[k];
    for (hipEvent_t ev : c->ev[k])
      if (ev) (void)hipEventDestroy(ev);
    c->ev[k].clear();
    c->ev_used[k] = 0;
  }
  c->prof = false;
  return VP4_OK;
}

int vp4_sync(vp4_ctx *c) {
  if (!c) return VP4_EINVAL;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return dev_fail(c, e, "sync");
  return check_flags(c);
}

const char *vp4_last_error(vp4_ctx *c) {
  return c ? c->err.c_str() : g_err4.c_str();
}

}  // extern "C"
