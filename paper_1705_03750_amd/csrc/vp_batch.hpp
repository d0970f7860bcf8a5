// vp_batch.hpp -- batched kernels of the serving loop: one launch advances
// many independent runs (different grids, element strides and step counts).
//
// Every kernel has a fixed grid and walks a per-phase work table: item ids
// [0, total) are split among the runs of the phase (table entry = run slot,
// first item, per-run argument).  A workgroup finds its run by a uniform
// binary search, then calls exactly the same per-tile device routine as the
// single-run kernels, so a run's arithmetic does not depend on its
// batch-mates and its results are bitwise those of a run alone.  Because the
// grids are fixed and all variability lives in device tables, the sequence
// of launches of one tick is captured once in a HIP graph and replayed.
#pragma once

#include "vp_kernels.hpp"

namespace vpk {

constexpr int MAXR = 128;  // run slots of one server

struct PhaseItem {
  int slot, begin, arg;
  int h;  // half steps since the run's last element reset (list geometry)
};
struct PhaseTable {
  int n, total, pad0, pad1;
  PhaseItem it[MAXR];
};

// Phases of one tick, in launch order.
enum {
  PH_PRED = 0,    // predictor drift + records + block lists (first step)
  PH_RECON,       // reconstruction + row-group column partials
  PH_FIELD,       // column sums, cumulative mass, force
  PH_KICK,        // kick + corrector (+ next predictor when continuing)
  PH_RM_PRED,     // remap: records + lists of the post-corrector elements
  PH_RM_EVAL,     // remap evaluation into F_ini
  PH_FIT_X,       // spline fit along x
  PH_FIT_V,       // spline fit along v
  PH_GHOST,       // mirror ghost columns
  PH_RESET,       // new isotropic elements, counts cleared
  PH_FIN_PRED,    // final reconstruction: records + lists
  PH_FIN_RECON,   // final reconstruction into the request's output
  PH_FIN_ZERO,    // counts cleared after the final reconstruction
  NPH
};

// Element-pass argument bits.
enum {
  EA_KICK = 1, EA_DRIFT = 2, EA_PRED = 4, EA_REG = 8, EA_REGBUF1 = 16,
  EA_ZERO = 32, EA_ZEROBUF1 = 64, EA_RESET = 128,
  EA_TAB = 256  // item = lattice patch, slot claims through reg_table
};

template <typename FT>
struct RunDesc {
  KP k;
  long long nb;
  double *st, *rec, *qm, *part, *Mc, *ctot, *Ml, *acc, *dpart;
  int *cnt, *lst, *flags, *fcnt;
  unsigned long long *ovf;
  FT *F, *C, *T;
  const FT *tab;
  FT *fout;
};

__device__ __forceinline__ int find_run(const PhaseTable *__restrict__ t,
                                        int item) {
  int lo = 0, hi = t->n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t->it[mid].begin <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Element passes (predict / kick / remap records / reset / count clearing):
// 256 elements and 256 block counts per item; with EA_TAB the item's
// elements are lattice patch item - begin and their slot claims go through
// the workgroup's table (the flag is uniform over an item, so every thread
// of the workgroup reaches the table's barriers).
template <typename FT>
__global__ __launch_bounds__(256) void kb_elem(
    const RunDesc<FT> *__restrict__ runs, const PhaseTable *__restrict__ tab) {
  __shared__ int rtab[RT * RT];
  const int total = tab->total;
  const int tid = threadIdx.x;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int q = find_run(tab, item);
    const PhaseItem pi = tab->it[q];
    const RunDesc<FT> &R = runs[pi.slot];
    KP p = R.k;
    p.tau = 0.5 * p.dt * pi.h;
    gox_set(p);
    const int arg = pi.arg;
    const bool tabm = arg & EA_TAB;
    if (tabm) {
      // the previous item's table reads are done before it is cleared
      __syncthreads();
      for (int i = tid; i < RT * RT; i += 256) rtab[i] = 0;
    }
    const int local = item - pi.begin;
    const long long idx = (long long)local * 256 + tid;
    if (arg & EA_ZERO) {
      int *cz = R.cnt + ((arg & EA_ZEROBUF1) ? R.nb : 0);
      if (idx < R.nb) cz[idx] = 0;
    }
    const int npx = (p.mx + PATCH - 1) / PATCH;
    const int ek = (local % npx) * PATCH + tid % PATCH;
    const int el = (local / npx) * PATCH + tid / PATCH;
    const bool has = tabm ? local < elem_patches(p.mx, p.mv) && ek < p.mx &&
                                el < p.mv
                          : idx < p.E;
    const int e = !has ? 0 : tabm ? el * p.mx + ek : (int)idx;
    const size_t E = (size_t)p.E;
    if (tabm) {
      const bool kick = arg & EA_KICK, drift = arg & EA_DRIFT;
      ElemState s;
      RegBox B;
      B.n = 0;
      if (has) {
        elem_load(R.st, E, e, s);
        if (kick) elem_kick(p, AccTable{R.acc, p.nx + 8}, s);
        if (drift) elem_drift(p, s);
        if (kick || drift) elem_store(R.st, E, e, s);
        B = elem_record_box(p, s, e, R.rec, R.qm, R.flags,
                            (arg & EA_REG) ? 1 : 0);
      }
      const int tr0 =
          blk(p.sv * ((local / npx) * PATCH + PATCH / 2), p.ov, p.obv) -
          RT / 2;
      const int tc0 =
          blk(p.sx * ((local % npx) * PATCH + PATCH / 2), 0, 1) - RT / 2;
      __syncthreads();  // the cleared table
      reg_table<TABLE_RB>(p, B, e, tr0, tc0, rtab,
                          R.cnt + ((arg & EA_REGBUF1) ? R.nb : 0), R.lst);
      continue;
    }
    if (!has) continue;
    if (arg & EA_RESET) {
      const int k = e % p.mx, l = e / p.mx;
      for (int s = 0; s < NSTATE; ++s) R.st[s * E + e] = 0.0;
      R.st[S_X * E + e] = site_x(p, p.sx * k + p.sx / 2);
      R.st[S_V * E + e] = site_v(p, p.sv * l + p.sv / 2);
      R.st[S_TXX * E + e] = 1.0;
      R.st[S_TVV * E + e] = 1.0;
      continue;
    }
    const bool kick = arg & EA_KICK, drift = arg & EA_DRIFT,
               pred = arg & EA_PRED;
    if (!kick && !pred) continue;
    ElemState s;
    elem_load(R.st, E, e, s);
    if (kick) elem_kick(p, AccTable{R.acc, p.nx + 8}, s);
    if (pred && drift) elem_drift(p, s);
    if (kick || (pred && drift)) elem_store(R.st, E, e, s);
    if (pred)
      elem_record(p, s, e, R.rec, R.qm,
                  R.cnt + ((arg & EA_REGBUF1) ? R.nb : 0), R.lst, R.flags,
                  (arg & EA_REG) ? 1 : 0);
  }
}

// Reconstruction tiles (8 columns x 64 rows per item); arg = live count
// buffer.  MODE_DENSITY also computes the force; MODE_F writes R.fout.
// Eight wavefronts per SIMD, as the single-run kernel (the run lookup
// would otherwise push it over 64 VGPRs).
template <typename FT, int MODE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(8))) void kb_recon(
    const RunDesc<FT> *__restrict__ runs, const PhaseTable *__restrict__ tab) {
  const int total = tab->total;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    __syncthreads();
    const int q = find_run(tab, item);
    const PhaseItem pi = tab->it[q];
    const RunDesc<FT> &R = runs[pi.slot];
    const int local = item - pi.begin;
    const int bx = local % R.k.nbx, gy = local / R.k.nbx;
    KP p = R.k;
    p.tau = 0.5 * p.dt * pi.h;
    gox_set(p);
    recon_tile<FT, MODE, 0>(p, R.rec, R.qm, R.cnt + (pi.arg ? R.nb : 0), R.lst,
                         R.flags, R.F, R.part, R.fout, nullptr, R.dpart, R.ovf,
                         bx, gy);
  }
}

// Field chunks (256 columns per item) from the row-group partials.
template <typename FT>
__global__ __launch_bounds__(FIELD_WG) void kb_field(
    const RunDesc<FT> *__restrict__ runs, const PhaseTable *__restrict__ tab) {
  __shared__ FieldLds L;
  const int total = tab->total;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    __syncthreads();
    const int q = find_run(tab, item);
    const PhaseItem pi = tab->it[q];
    const RunDesc<FT> &R = runs[pi.slot];
    FieldArgs A{};
    A.in = R.part;
    A.ngy = R.k.ngy;
    A.in_is_rho = 0;
    A.Mc = R.Mc;
    A.ctot = R.ctot;
    A.fcnt = R.fcnt;
    A.Ml = R.Ml;
    A.acc = R.acc;
    field_chunk(R.k, A, item - pi.begin, L);
  }
}

template <typename FT>
__global__ __launch_bounds__(512) void kb_remap(
    const RunDesc<FT> *__restrict__ runs, const PhaseTable *__restrict__ tab) {
  const int total = tab->total;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int q = find_run(tab, item);
    const PhaseItem pi = tab->it[q];
    const RunDesc<FT> &R = runs[pi.slot];
    const int local = item - pi.begin;
    const int bx = local % R.k.nbx, gy = local / R.k.nbx;
    KP p = R.k;
    p.tau = 0.5 * p.dt * pi.h;
    gox_set(p);
    remap_tile<FT, 0, 0>(p, R.rec, R.qm, R.cnt + (pi.arg ? R.nb : 0), R.lst,
                      R.flags, R.C, R.F, R.ovf, bx, gy);
  }
}

template <typename FT>
__global__ __launch_bounds__(FIT_THREADS) void kb_fit_x(
    const RunDesc<FT> *__restrict__ runs, const PhaseTable *__restrict__ tab) {
  __shared__ FitLds<FT> S;
  const int total = tab->total;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int q = find_run(tab, item);
    const PhaseItem pi = tab->it[q];
    const RunDesc<FT> &R = runs[pi.slot];
    const KP &p = R.k;
    fit_x_rows<FT>(p, R.F, R.T, R.tab, item - pi.begin, S);
  }
}

template <typename FT>
__global__ __launch_bounds__(FIT_THREADS) void kb_fit_v(
    const RunDesc<FT> *__restrict__ runs, const PhaseTable *__restrict__ tab) {
  __shared__ FitLds<FT> S;
  const int total = tab->total;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int q = find_run(tab, item);
    const PhaseItem pi = tab->it[q];
    const RunDesc<FT> &R = runs[pi.slot];
    const KP &p = R.k;
    fit_v_cols<FT>(p, R.T, R.C, R.tab, item - pi.begin, S);
  }
}

template <typename FT>
__global__ __launch_bounds__(256) void kb_ghost(
    const RunDesc<FT> *__restrict__ runs, const PhaseTable *__restrict__ tab) {
  const int total = tab->total;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int q = find_run(tab, item);
    const PhaseItem pi = tab->it[q];
    const RunDesc<FT> &R = runs[pi.slot];
    ghost_x_rows<FT>(R.k, R.C, item - pi.begin);
  }
}

}  // namespace vpk
