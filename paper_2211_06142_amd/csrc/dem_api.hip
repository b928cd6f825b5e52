// dem_api.hip -- host runtime behind the C ABI of include/dem.h.
//
// Owns the device memory of one context, derives the per-sample constants
// (coarse-graining of section 2.4 applied here), drives the rebuild /
// coupling / force / integration kernels of dem_kernels.hip on the caller's
// stream, and converts between the caller's particle order and the sorted
// device order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <cmath>
#include <string.h>

#include <algorithm>
#include <map>
#include <vector>

#include "dem_internal.h"

using namespace dem;

namespace {

#define HIPCHK(x)                                    \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) return DEM_E_DEVICE;       \
  } while (0)

struct NbrSet {
  int32_t *nrow = nullptr, *nbr = nullptr, *nslot = nullptr, *hrow = nullptr, *sown = nullptr, *spart = nullptr;
  void* hdt[2] = {nullptr, nullptr};
  uint8_t* pfl[2] = {nullptr, nullptr};
  int64_t ent_cap = 0, slot_cap = 0, nent = 0, nslots = 0;
};

struct WallSet {
  int32_t *wrow = nullptr, *wid = nullptr;
  void* wdt = nullptr;
  uint8_t* wfl = nullptr;
  int64_t cap = 0, n = 0;
};

struct ProfRec {
  int cls;
  int64_t step;   // step a launch belongs to (-1: always counted)
  int slot;
};

}  // namespace

struct dem_ctx {
  DevState d;
  hipStream_t stream = nullptr;
  int device = 0;
  int fp64 = 1;
  size_t rsz = 8;  // sizeof(R)
  std::vector<dem_params> params;
  std::vector<SampleConst> sc;
  std::vector<int64_t> offsets;
  int64_t* d_offsets = nullptr;
  NbrSet ns[2];
  WallSet ws[2];
  int live = 0;          // ns[live] / ws[live] is the current list
  int last_overflow_rows = 0;   // rows the last search could not keep in scratch
  DevState* d_dev = nullptr;    // device copy of d
  int use_graphs = 0;           // replay recorded step windows
  hipStream_t cap_stream = nullptr;   // records them
  std::map<int64_t, hipGraphExec_t> graphs;
  // learned closure: factor arrays and their permutation scratch (kept while off)
  double* cl_buf[4] = {nullptr, nullptr, nullptr, nullptr};
  double *cl_feat = nullptr, *cl_feat_tmp = nullptr, *cl_norm = nullptr;
  short* cl_wb = nullptr;
  float* cl_pf = nullptr;
  int hist_old = 0;      // history buffer of the previous list at the next rebuild
  int64_t step = 0;
  int64_t rebuilds = 0;
  int have_fluid = 0;
  int any_fluid = 0;
  int force_rebuild = 0;
  int failed = 0;        // a latched device fault
  int window = 32;       // steps enqueued between host checks
  int* h_flags = nullptr;  // pinned: abort, abort_step, status
  int32_t* h_tot = nullptr;   // pinned: rebuild totals
  double* agg_buf = nullptr;  // aggregate outputs and slice partials
  int64_t fixed_capacity = 0;   // half-pair capacity given without DEM_FLAG_AUTO_REGROW (0: grows)
  int64_t rec_cap = 0;          // slots of the half-pair records d.rec
  int64_t wfrc_cap = 0;         // wall entries of d.wfrc
  int lanes_set = 0;             // lanes chosen by the caller (else the pair mode's default)
  double* stage_aux = nullptr;   // read-back of the held fluid force and wall history
  // fluid solver: cell kinds, fixed pressures, work vectors (the solution kept
  // for warm starts), output staging, pinned scalars
  int8_t* cfd_kind = nullptr;
  double *cfd_pfix = nullptr, *cfd_work = nullptr, *cfd_out = nullptr, *cfd_scal = nullptr;
  int cfd_warm = 0;
  std::vector<void*> allocs;
  // kernel-class timing
  int prof = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfRec> ev_pending;
  size_t ev_used = 0;
  double prof_ms[DEM_PROF_N] = {0, 0, 0, 0};
  int64_t prof_cnt[DEM_PROF_N] = {0, 0, 0, 0};
  // staging for read-back
  double* stage = nullptr;
  uint8_t* stage_alive = nullptr;
};

namespace {

template <typename T> hipError_t dalloc(dem_ctx* c, T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)count);
  if (e == hipSuccess) c->allocs.push_back((void*)*p);
  return e;
}

hipError_t dalloc_bytes(dem_ctx* c, void** p, int64_t bytes) {
  *p = nullptr;
  if (bytes <= 0) bytes = 16;
  hipError_t e = hipMalloc(p, (size_t)bytes);
  if (e == hipSuccess) c->allocs.push_back(*p);
  return e;
}

void dfree(dem_ctx* c, void* p) {
  if (!p) return;
  for (auto& a : c->allocs)
    if (a == p) { (void)hipFree(p); a = nullptr; }
}

bool finite_all(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// copy from host or device memory into a host vector
template <typename T> hipError_t fetch(std::vector<T>& out, const T* src, int64_t count) {
  out.resize((size_t)std::max<int64_t>(count, 0));
  if (count <= 0 || !src) return hipSuccess;
  return hipMemcpy(out.data(), src, sizeof(T) * (size_t)count, hipMemcpyDefault);
}

const double kPi = 3.14159265358979323846;

double beta_of_e(double e) {
  double l = log(e);
  return -l / sqrt(l * l + kPi * kPi);
}

dem_status validate(const dem_params& p) {
  if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return DEM_E_INVAL;
  if (!(p.nu > -1.0 && p.nu < 0.5)) return DEM_E_INVAL;
  if (!(p.e > 0.0 && p.e <= 1.0)) return DEM_E_INVAL;
  if (!(p.k >= 1.0)) return DEM_E_INVAL;
  if (!(p.rho > 0.0) || !(p.E > 0.0) || !(p.mu >= 0.0) || !(p.mu_roll >= 0.0) || !(p.gamma >= 0.0))
    return DEM_E_INVAL;
  if (p.n_walls < 0 || p.n_walls > DEM_MAX_WALLS) return DEM_E_INVAL;
  if (p.normal_model < 0 || p.normal_model > 3) return DEM_E_INVAL;
  if (p.normal_model == DEM_NORMAL_LINEAR && !(p.k_lin > 0.0)) return DEM_E_INVAL;
  if (p.precision != DEM_PREC_FP64 && p.precision != DEM_PREC_MIXED) return DEM_E_INVAL;
  if (p.fluid_on) {
    for (int c = 0; c < 3; ++c)
      if (p.grid.n[c] < 1 || !(p.grid.hi[c] > p.grid.lo[c])) return DEM_E_INVAL;
    // a sample's cells are indexed in 32 bits on the device
    if ((int64_t)p.grid.n[0] * p.grid.n[1] * p.grid.n[2] > (int64_t)1 << 30) return DEM_E_INVAL;
    if (!(p.rho_f > 0.0) || !(p.mu_f > 0.0) || !(p.n_min > 0.0 && p.n_min <= 1.0)) return DEM_E_INVAL;
    if (p.couple_every < 1) return DEM_E_INVAL;
    if (p.voidfrac != DEM_VOID_CIC && p.voidfrac != DEM_VOID_CENTROID) return DEM_E_INVAL;
  }
  for (int w = 0; w < p.n_walls; ++w) {
    const dem_wall& wl = p.walls[w];
    if (wl.kind < 0 || wl.kind > DEM_WALL_PLANE_HOLE) return DEM_E_INVAL;
    if (wl.kind == DEM_WALL_PLANE_HOLE && ((wl.p[3] != 1.0 && wl.p[3] != -1.0) || !(wl.p[4] > 0.0)))
      return DEM_E_INVAL;
  }
  if (p.outlet_kind < DEM_OUTLET_NONE || p.outlet_kind > DEM_OUTLET_ABOVE) return DEM_E_INVAL;
  if (p.outlet_kind == DEM_OUTLET_CAVITY && !(p.outlet[2] > 0.0)) return DEM_E_INVAL;
  if (p.outlet_kind == DEM_OUTLET_ABOVE && !std::isfinite(p.outlet[3])) return DEM_E_INVAL;
  return DEM_OK;
}

// per-sample constants (grain scale) and the binning grid
void derive(const dem_params& p, const double* x, const double* r, const uint8_t* alive, int64_t lo,
            int64_t hi, SampleConst& c) {
  memset(&c, 0, sizeof(c));
  c.Es = p.E / (2.0 * (1.0 - p.nu * p.nu));
  c.Gs = p.E / (4.0 * (2.0 - p.nu) * (1.0 + p.nu));
  c.beta = beta_of_e(p.e);
  c.cdamp = 2.0 * sqrt(5.0 / 6.0) * c.beta;
  c.gamma = p.k * p.gamma;                           // eq 24
  const bool jkr = p.normal_model == DEM_NORMAL_JKR_MOD || p.normal_model == DEM_NORMAL_JKR_ORIG;
  if (!jkr) c.gamma = 0.0;
  c.jkr_break = p.normal_model == DEM_NORMAL_JKR_ORIG ? 27.0 / 16.0 : 3.0 / 16.0;
  c.mu = p.mu;
  c.mu_roll = p.mu_roll;
  c.rho = p.rho;
  c.k_lin = p.k_lin;
  c.f_Es = (float)c.Es;
  c.f_Gs = (float)c.Gs;
  c.f_beta = (float)c.beta;
  c.f_cdamp = (float)c.cdamp;
  c.f_mu = (float)c.mu;
  c.f_mu_roll = (float)c.mu_roll;
  c.f_k_lin = (float)c.k_lin;
  c.kcg = p.k;
  c.k3 = p.k * p.k * p.k;
  c.normal_model = p.normal_model;
  c.fluid_on = p.fluid_on;
  c.voidfrac = p.voidfrac;
  c.u_superficial = p.u_superficial;
  c.rho_f = p.rho_f;
  c.mu_f = p.mu_f;
  c.n_min = p.n_min;
  for (int k = 0; k < 3; ++k) {
    c.g[k] = p.g[k];
    if (p.fluid_on) {
      c.glo[k] = p.grid.lo[k];
      c.gh[k] = (p.grid.hi[k] - p.grid.lo[k]) / p.grid.n[k];
      c.gn[k] = p.grid.n[k];
      c.dn[k] = p.voidfrac == DEM_VOID_CENTROID ? p.grid.n[k] : std::max(p.grid.n[k] - 1, 1);
    } else {
      c.glo[k] = 0.0; c.gh[k] = 1.0; c.gn[k] = 1; c.dn[k] = 1;
    }
  }
  c.vcell = c.gh[0] * c.gh[1] * c.gh[2];
  c.outlet_kind = p.outlet_kind;
  for (int k = 0; k < 4; ++k) c.outlet[k] = p.outlet[k];
  c.n_walls = p.n_walls;
  for (int w = 0; w < p.n_walls; ++w) {
    c.walls[w].kind = p.walls[w].kind;
    for (int k = 0; k < 6; ++k) c.walls[w].p[k] = p.walls[w].p[k];
  }
  double rmin = 1e300, rmax = 0.0, bl[3] = {1e300, 1e300, 1e300}, bh[3] = {-1e300, -1e300, -1e300};
  int64_t nal = 0;
  double mass = 0.0;
  for (int64_t i = lo; i < hi; ++i) {
    rmin = std::min(rmin, r[i]);
    rmax = std::max(rmax, r[i]);
    mass += p.rho * (4.0 / 3.0) * kPi * r[i] * r[i] * r[i];
    if (alive && !alive[i]) continue;
    ++nal;
    for (int k = 0; k < 3; ++k) { bl[k] = std::min(bl[k], x[3 * i + k]); bh[k] = std::max(bh[k], x[3 * i + k]); }
  }
  if (nal == 0) { for (int k = 0; k < 3; ++k) { bl[k] = 0.0; bh[k] = 0.0; } }
  // fixed point of the produced-mass counters: the whole sample stays below
  // 2^61 units, so the rounded masses of up to 2^30 removals cannot overflow
  int ex = 0;
  (void)frexp(mass > 0.0 ? mass : 1.0, &ex);
  c.pm_scale = ldexp(1.0, 61 - ex);
  if (rmax == 0.0) { rmin = rmax = 1e-6; }
  c.skin = p.skin > 0.0 ? p.skin : 0.4 * rmin;   // tuned: fewer rebuilds, rows barely longer
  // largest separation a contact survives, |delta_C| = (3/16)^(1/3) X (Table 1),
  // or |delta_S| = (27/16)^(1/3) X for the original JKR cycle, with the surface
  // energy bounded by twice its value (closure factors are <= 2)
  double gmax = 2.0 * c.gamma;
  double Rsmax = 0.5 * rmax;
  double dC = cbrt(c.jkr_break) * cbrt((kPi * kPi) * gmax * gmax * Rsmax / (c.Es * c.Es));
  c.margin = c.skin + 1.01 * dC;
  double h = 2.0 * rmax + c.margin;
  double ext[3];
  for (int k = 0; k < 3; ++k) {
    c.blo[k] = bl[k] - h;
    ext[k] = (bh[k] - bl[k]) + 2.0 * h;
  }
  int64_t budget = 4 * std::max<int64_t>(hi - lo, 1) + 64;
  for (;;) {
    int64_t tot = 1;
    for (int k = 0; k < 3; ++k) {
      double q = floor(ext[k] / h);
      c.bn[k] = (int)std::max(1.0, std::min(q, (double)(1 << 20)));
      tot *= c.bn[k];
    }
    if (tot <= budget) break;
    h *= 1.25;
  }
  for (int k = 0; k < 3; ++k) c.bh[k] = ext[k] / c.bn[k];
}

void bind_sets(dem_ctx* c) {
  NbrSet& a = c->ns[c->live];
  NbrSet& b = c->ns[1 - c->live];
  DevState& d = c->d;
  d.nrow = a.nrow; d.nbr = a.nbr; d.nslot = a.nslot; d.hrow = a.hrow; d.sown = a.sown; d.spart = a.spart;
  d.hdt[0] = a.hdt[0]; d.hdt[1] = a.hdt[1]; d.pfl[0] = a.pfl[0]; d.pfl[1] = a.pfl[1];
  d.ent_cap = a.ent_cap; d.slot_cap = a.slot_cap; d.nent = a.nent; d.nslots = a.nslots;
  d.nrow_o = b.nrow; d.nbr_o = b.nbr; d.nslot_o = b.nslot; d.sown_o = b.sown; d.spart_o = b.spart;
  d.hdt_o = b.hdt[c->hist_old]; d.pfl_o = b.pfl[c->hist_old]; d.nslots_o = b.nslots;
  WallSet& wa = c->ws[c->live];
  WallSet& wb = c->ws[1 - c->live];
  d.wrow = wa.wrow; d.wid = wa.wid; d.wdt = wa.wdt; d.wfl = wa.wfl; d.wall_cap = wa.cap; d.nwall = wa.n;
  d.wrow_o = wb.wrow; d.wid_o = wb.wid; d.wdt_o = wb.wdt; d.wfl_o = wb.wfl;
}

hipError_t grow_nbr(dem_ctx* c, NbrSet& s, int64_t nent, int64_t nslots) {
  hipError_t e;
  if (nent > s.ent_cap) {
    int64_t cap = std::max<int64_t>(nent + nent / 4 + 1024, s.ent_cap * 2);
    dfree(c, s.nbr); dfree(c, s.nslot);
    if ((e = dalloc(c, &s.nbr, cap)) != hipSuccess) return e;
    if ((e = dalloc(c, &s.nslot, cap)) != hipSuccess) return e;
    s.ent_cap = cap;
  }
  if (nslots > s.slot_cap) {
    int64_t cap = std::max<int64_t>(nslots + nslots / 4 + 1024, s.slot_cap * 2);
    dfree(c, s.sown); dfree(c, s.spart);
    for (int b = 0; b < 2; ++b) { dfree(c, s.hdt[b]); dfree(c, s.pfl[b]); }
    if ((e = dalloc(c, &s.sown, cap)) != hipSuccess) return e;
    if ((e = dalloc(c, &s.spart, cap)) != hipSuccess) return e;
    for (int b = 0; b < 2; ++b) {
      if ((e = dalloc_bytes(c, &s.hdt[b], cap * 4 * (int64_t)c->rsz)) != hipSuccess) return e;
      if ((e = dalloc(c, &s.pfl[b], cap)) != hipSuccess) return e;
    }
    s.slot_cap = cap;
  }
  return hipSuccess;
}

hipError_t grow_walls(dem_ctx* c, WallSet& s, int64_t need) {
  if (need <= s.cap) return hipSuccess;
  int64_t cap = std::max<int64_t>(need + need / 4 + 256, s.cap * 2);
  dfree(c, s.wid); dfree(c, s.wdt); dfree(c, s.wfl);
  hipError_t e;
  if ((e = dalloc(c, &s.wid, cap)) != hipSuccess) return e;
  if ((e = dalloc_bytes(c, &s.wdt, cap * 4 * (int64_t)c->rsz)) != hipSuccess) return e;
  if ((e = dalloc(c, &s.wfl, cap)) != hipSuccess) return e;
  s.cap = cap;
  return hipSuccess;
}

template <typename T> void swp(T& a, T& b) { T t = a; a = b; b = t; }

// event pair around one launch of a kernel class (profiling mode only)
int prof_begin(dem_ctx* c) {
  if (!c->prof) return -1;
  if (c->ev_used + 2 > c->ev_pool.size()) {
    size_t grow = std::max<size_t>(256, c->ev_pool.size());
    for (size_t k = 0; k < grow; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      c->ev_pool.push_back(e);
    }
  }
  int slot = (int)c->ev_used;
  c->ev_used += 2;
  (void)hipEventRecord(c->ev_pool[slot], c->stream);
  return slot;
}

void prof_end(dem_ctx* c, int cls, int slot, int64_t step = -1) {
  if (slot < 0) return;
  (void)hipEventRecord(c->ev_pool[slot + 1], c->stream);
  c->ev_pending.push_back({cls, step, slot});
}

// accumulate completed event pairs (the stream has been synchronised);
// launches of steps >= drop_from did no work (aborted) and are not counted
void prof_collect(dem_ctx* c, int64_t drop_from = INT64_MAX) {
  for (auto& q : c->ev_pending) {
    if (q.step >= 0 && q.step >= drop_from) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[q.slot], c->ev_pool[q.slot + 1]) == hipSuccess) {
      c->prof_ms[q.cls] += ms;
      c->prof_cnt[q.cls] += 1;
    }
  }
  c->ev_pending.clear();
  c->ev_used = 0;
}

dem_status fault(dem_ctx* c, int st);

// full neighbour-list rebuild from the state in buffer d.cur
template <typename R> dem_status rebuild(dem_ctx* c, int first, int mark_bonds) {
  DevState& d = c->d;
  hipStream_t s = c->stream;
  // 1. sort by (sample, cell, id); dead particles to their sample's last bucket
  launch_bin_keys(d, s);
  launch_bucket_sort(d.key, d.n, d.nbins_total, d.orig, d.bucket_cnt, d.cell_start, d.bucket_fill, d.order_tmp,
                     d.order, d.scan_tmp, d.bin_sink, nullptr, s);
  // 2. permute into the other buffer
  launch_permute<R>(d, s);
  c->hist_old = d.cur;
  d.cur = 1 - d.cur;
  swp(d.frc, d.t_r4[0]); swp(d.trq, d.t_r4[1]); swp(d.fdr, d.t_r4[2]);
  swp(d.sample, d.t_i[0]); swp(d.orig, d.t_i[1]);
  if (d.cdrag) { swp(d.cdrag, d.t_d[0]); swp(d.ccoh, d.t_d[1]); }
  if (d.closure_on) swp(d.cfeat, d.t_feat);
  // 3. the live list becomes the previous one
  if (!first) c->live = 1 - c->live;
  bind_sets(c);
  // 4. search into scratch rows, scan the row lengths, fill the CSR rows
  //    (dead particles own no entries: their counts stay zero)
  HIPCHK(hipMemsetAsync(d.ncnt, 0, sizeof(int32_t) * (d.n + 1), s));
  HIPCHK(hipMemsetAsync(d.ocnt, 0, sizeof(int32_t) * (d.n + 1), s));
  HIPCHK(hipMemsetAsync(d.novf, 0, sizeof(int), s));
  launch_nbr_search(d, s);
  scan_exclusive(d.ncnt, d.nrow, d.n + 1, d.scan_tmp, s);
  scan_exclusive(d.ocnt, d.hrow, d.n + 1, d.scan_tmp, s);
  launch_wall_count(d, s);
  HIPCHK(hipMemsetAsync(d.wcnt + d.n, 0, sizeof(int32_t), s));
  scan_exclusive(d.wcnt, d.wrow, d.n + 1, d.scan_tmp, s);
  launch_totals(d, s);   // entries, slots, wall entries, overflow rows: one copy
  HIPCHK(hipMemcpyAsync(c->h_tot, d.totals, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int32_t* tot = c->h_tot;
  NbrSet& ns = c->ns[c->live];
  WallSet& ws = c->ws[c->live];
  if (c->fixed_capacity > 0 &&
      (tot[0] > 2 * c->fixed_capacity || tot[1] > c->fixed_capacity || tot[2] > d.n / 4 + 256))
    return fault(c, kStCapacity);
  if (grow_nbr(c, ns, tot[0], tot[1]) != hipSuccess) return DEM_E_NOMEM;
  if (grow_walls(c, ws, tot[2]) != hipSuccess) return DEM_E_NOMEM;
  if (ws.cap > c->wfrc_cap) {   // wall forces follow the largest wall capacity
    dfree(c, d.wfrc);
    if (dalloc_bytes(c, &d.wfrc, ws.cap * 4 * (int64_t)c->rsz) != hipSuccess) return DEM_E_NOMEM;
    c->wfrc_cap = ws.cap;
  }
  ns.nent = tot[0];
  ns.nslots = tot[1];
  ws.n = tot[2];
  c->last_overflow_rows = tot[3];
  if (ns.slot_cap > c->rec_cap) {   // half-pair records follow the largest slot capacity
    for (int q = 0; q < 2; ++q) {
      dfree(c, d.rec[q]);
      if (dalloc_bytes(c, &d.rec[q], ns.slot_cap * (q == 0 ? 6 : 4) * (int64_t)c->rsz) != hipSuccess)
        return DEM_E_NOMEM;
    }
    c->rec_cap = ns.slot_cap;
  }
  bind_sets(c);
  launch_nbr_fill(d, tot[3], s);
  launch_wall_fill(d, s);
  // 5. carry history
  launch_hist_carry<R>(d, s, first ? 0 : 1);
  if (mark_bonds) launch_mark_bonds<R>(d, s);
  launch_set_xref(d, s);
  c->rebuilds++;
  return DEM_OK;
}

dem_status read_flags(dem_ctx* c) {
  // abort, abort_step and status are adjacent: one copy
  HIPCHK(hipMemcpyAsync(c->h_flags, c->d.abort, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return DEM_OK;
}

dem_status fault(dem_ctx* c, int st) {
  c->failed = st;
  if (st & kStNonFinite) return DEM_E_NONFINITE;
  if (st & kStCapacity) return DEM_E_CAPACITY;
  return DEM_E_STATE;
}

// the step-window kernels read the context's state from its device copy
dem_status upload_state(dem_ctx* c) {
  HIPCHK(hipMemcpyAsync(c->d_dev, &c->d, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  return DEM_OK;
}

void drop_graphs(dem_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

// Enqueue the steps [t, t1) of a window starting from buffer b0.  StepArgs.step
// is relative to the window start (the recorded abort step is too), so a
// window's launches depend only on (b0, t mod couple_every, length): windows
// without the last step of the call replay one recorded graph per such key.
template <typename R> void enqueue_window(dem_ctx* c, int64_t t, int64_t t1, int64_t s_end, int b0, bool eager) {
  DevState& d = c->d;
  const bool fluid = c->any_fluid && c->have_fluid;
  auto body = [&](bool prof, hipStream_t s) {
    int b = b0;
    for (int64_t q = t; q < t1; ++q) {
      if (fluid && (q % d.couple_every) == 0) {
        int pf = prof ? prof_begin(c) : -1;
        launch_fluid<R>(d, b, s);
        if (prof) prof_end(c, DEM_PROF_FLUID, pf, q);
      }
      StepArgs a{q - t, b, 1 - b, q == s_end - 1 ? 1 : 0};
      int pk = prof ? prof_begin(c) : -1;
      launch_step<R>(d, a, s);
      if (prof) prof_end(c, DEM_PROF_STEP, pk, q);
      b = 1 - b;
    }
  };
  if (eager || c->prof || !c->use_graphs) {
    body(c->prof != 0, c->stream);
    return;
  }
  const int64_t key = ((int64_t)b0 << 40) | ((fluid ? t % d.couple_every : 0) << 20) | (t1 - t);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    // recorded on a stream of the library's own (the caller's may be the legacy
    // default stream, which cannot record), replayed on the caller's stream
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    bool ok = true;
    if (!c->cap_stream) ok = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      body(false, c->cap_stream);
      ok = hipStreamEndCapture(c->cap_stream, &g) == hipSuccess && g != nullptr;
    }
    if (ok) ok = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {   // the runtime refused: clear its error, run eagerly, stop recording
      (void)hipGetLastError();
      c->use_graphs = 0;
      body(false, c->stream);
      return;
    }
    it = c->graphs.emplace(key, ge).first;
  }
  (void)hipGraphLaunch(it->second, c->stream);
}

// Steps are enqueued in windows without waiting for the device.  A step that
// finds a particle beyond half the skin raises `abort` and records the next
// step; every later launch of the window exits at entry.  At the end of the
// window the host reads the flags, rebuilds the list from the state the last
// completed step left, and resumes at the recorded step.
template <typename R> dem_status step_impl(dem_ctx* c, int64_t nsteps) {
  DevState& d = c->d;
  hipStream_t s = c->stream;
  if (nsteps <= 0) return DEM_OK;
  const int64_t s_end = c->step + nsteps;
  if (upload_state(c) != DEM_OK) return DEM_E_DEVICE;
  HIPCHK(hipMemsetAsync(d.abort, 0, sizeof(int), s));
  HIPCHK(hipMemsetAsync(d.abort_step, 0x7f, sizeof(int), s));   // none: 0x7f7f7f7f
  // first half kick and drift of the first step
  // (in place: the pair history stays in the buffer of the particle state)
  int ps = prof_begin(c);
  StepArgs pa{0, d.cur, d.cur, 0};
  launch_prologue<R>(d, pa, s);
  prof_end(c, DEM_PROF_PROLOGUE, ps);
  int buf = d.cur;           // buffer holding the drifted state of step c->step
  if (c->force_rebuild) {
    HIPCHK(hipStreamSynchronize(s));
    c->h_flags[3] = 0;
    HIPCHK(hipMemsetAsync(d.abort, 0xff, sizeof(int), s));
    HIPCHK(hipMemcpyAsync(d.abort_step, c->h_flags + 3, sizeof(int), hipMemcpyHostToDevice, s));
    c->force_rebuild = 0;
  }
  int64_t t = c->step;
  while (t < s_end) {
    int64_t t1 = std::min<int64_t>(s_end, t + c->window);
    enqueue_window<R>(c, t, t1, s_end, buf, t1 == s_end);
    dem_status rs = read_flags(c);
    if (rs != DEM_OK) return rs;
    int abort = c->h_flags[0], astep = c->h_flags[1], status = c->h_flags[2];
    if (status) {
      prof_collect(c);
      return fault(c, status);
    }
    if (!abort) {
      prof_collect(c);
      if ((t1 - t) & 1) buf = 1 - buf;
      t = t1;
      continue;
    }
    // resume at the recorded step after a rebuild from the state before it
    if (astep < 0 || astep > t1 - t) return fault(c, kStBadAbort);
    int64_t ta = t + astep;
    prof_collect(c, ta);
    if (astep & 1) buf = 1 - buf;
    d.cur = buf;
    HIPCHK(hipMemsetAsync(d.abort, 0, sizeof(int), s));
    HIPCHK(hipMemsetAsync(d.abort_step, 0x7f, sizeof(int), s));   // none: 0x7f7f7f7f
    int pr = prof_begin(c);
    dem_status st = rebuild<R>(c, 0, 0);
    if (st != DEM_OK) return st;
    prof_end(c, DEM_PROF_REBUILD, pr);
    if (upload_state(c) != DEM_OK) return DEM_E_DEVICE;
    buf = d.cur;
    t = ta;
  }
  d.cur = buf;
  HIPCHK(hipStreamSynchronize(s));
  prof_collect(c);
  c->step = s_end;
  return DEM_OK;
}

}  // namespace

extern "C" {

const char* dem_status_str(dem_status s) {
  switch (s) {
    case DEM_OK: return "ok";
    case DEM_E_INVAL: return "invalid argument";
    case DEM_E_NOMEM: return "device allocation failed";
    case DEM_E_CAPACITY: return "pair capacity exceeded";
    case DEM_E_NONFINITE: return "non-finite force or torque";
    case DEM_E_DEVICE: return "HIP runtime error";
    case DEM_E_STATE:
      return "invalid state (fault latched: a particle moved more than half the skin in one step, a bond "
             "was lost by the neighbour list, or fluid fields are missing)";
  }
  return "unknown status";
}

double dem_rayleigh_dt(double radius, double rho, double E, double nu) {
  double G = E / (2.0 * (1.0 + nu));
  double beta = 0.8766 + 0.163 * nu;
  return kPi * radius / beta * sqrt(rho / G);
}

dem_status dem_cg_material(const dem_params* fine, double* gamma_grain, double* drag_factor) {
  if (!fine || !(fine->k >= 1.0)) return DEM_E_INVAL;
  if (gamma_grain) *gamma_grain = fine->k * fine->gamma;
  if (drag_factor) *drag_factor = fine->k * fine->k * fine->k;
  return DEM_OK;
}

dem_status dem_cg_diameters(int32_t scheme, double k, const double* d_fine, int64_t n_fine, double* d_out,
                            int64_t n_out) {
  if (!(k >= 1.0) || !d_fine || !d_out || n_fine <= 0 || n_out < 0) return DEM_E_INVAL;
  if (scheme == DEM_CG_SSW) {
    if (n_out > n_fine) return DEM_E_INVAL;
    for (int64_t i = 0; i < n_out; ++i) d_out[i] = k * d_fine[i];
    return DEM_OK;
  }
  if (scheme == DEM_CG_SSP) {
    double s = 0.0;
    for (int64_t i = 0; i < n_fine; ++i) s += d_fine[i] * d_fine[i] * d_fine[i];
    double dbar = cbrt(s / (double)n_fine);
    for (int64_t i = 0; i < n_out; ++i) d_out[i] = k * dbar;
    return DEM_OK;
  }
  return DEM_E_INVAL;
}

dem_status dem_init(dem_ctx** out, const dem_params* params, int32_t n_samples, const int64_t* sample_offsets,
                    const dem_state* init, int32_t device, void* hip_stream) {
  if (!out) return DEM_E_INVAL;
  *out = nullptr;
  if (!params || n_samples < 1 || !init || init->n < 0 || !init->x || !init->radius) return DEM_E_INVAL;
  if (n_samples > 1 && !sample_offsets) return DEM_E_INVAL;
  const int64_t n = init->n;
  if (n > (int64_t)1 << 30) return DEM_E_INVAL;
  std::vector<int64_t> offs(n_samples + 1);
  if (sample_offsets) {
    for (int s = 0; s <= n_samples; ++s) offs[s] = sample_offsets[s];
    if (offs[0] != 0 || offs[n_samples] != n) return DEM_E_INVAL;
    for (int s = 0; s < n_samples; ++s)
      if (offs[s + 1] < offs[s]) return DEM_E_INVAL;
  } else {
    offs[0] = 0;
    offs[1] = n;
  }
  for (int s = 0; s < n_samples; ++s) {
    dem_status v = validate(params[s]);
    if (v != DEM_OK) return v;
    if (params[s].dt != params[0].dt || params[s].precision != params[0].precision ||
        params[s].couple_every != params[0].couple_every)
      return DEM_E_INVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DEM_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return DEM_E_DEVICE;
  // host copies of the inputs
  std::vector<double> x, v, w, F, T, r;
  std::vector<uint8_t> alive;
  if (fetch(x, init->x, 3 * n) != hipSuccess || fetch(r, init->radius, n) != hipSuccess) return DEM_E_DEVICE;
  if (init->v && fetch(v, init->v, 3 * n) != hipSuccess) return DEM_E_DEVICE;
  if (init->omega && fetch(w, init->omega, 3 * n) != hipSuccess) return DEM_E_DEVICE;
  if (init->force && fetch(F, init->force, 3 * n) != hipSuccess) return DEM_E_DEVICE;
  if (init->torque && fetch(T, init->torque, 3 * n) != hipSuccess) return DEM_E_DEVICE;
  if (init->alive && fetch(alive, init->alive, n) != hipSuccess) return DEM_E_DEVICE;
  // held state of a resumed run: fluid force and wall history
  std::vector<double> FF, WD;
  if (init->step < 0) return DEM_E_INVAL;
  if (init->fluid_force && fetch(FF, init->fluid_force, 3 * n) != hipSuccess) return DEM_E_DEVICE;
  if (init->wall_dt && fetch(WD, init->wall_dt, 3 * (int64_t)DEM_MAX_WALLS * n) != hipSuccess) return DEM_E_DEVICE;
  if (!finite_all(FF.data(), (int64_t)FF.size()) || !finite_all(WD.data(), (int64_t)WD.size())) return DEM_E_INVAL;
  if (v.empty()) v.assign(3 * n, 0.0);
  if (w.empty()) w.assign(3 * n, 0.0);
  if (F.empty()) F.assign(3 * n, 0.0);
  if (T.empty()) T.assign(3 * n, 0.0);
  if (alive.empty()) alive.assign(n, 1);
  if (!finite_all(x.data(), 3 * n) || !finite_all(v.data(), 3 * n) || !finite_all(w.data(), 3 * n) ||
      !finite_all(F.data(), 3 * n) || !finite_all(T.data(), 3 * n) || !finite_all(r.data(), n))
    return DEM_E_INVAL;
  for (int64_t i = 0; i < n; ++i)
    if (!(r[i] > 0.0)) return DEM_E_INVAL;
  // Rayleigh guard (eq 37-38) for the smallest radius of each sample
  for (int s = 0; s < n_samples; ++s) {
    const dem_params& p = params[s];
    if (p.dt_rayleigh_max_frac > 0.0 && offs[s + 1] > offs[s]) {
      double rmin = 1e300;
      for (int64_t i = offs[s]; i < offs[s + 1]; ++i) rmin = std::min(rmin, r[i]);
      if (p.dt > p.dt_rayleigh_max_frac * dem_rayleigh_dt(rmin, p.rho, p.E, p.nu)) return DEM_E_INVAL;
    }
  }
  // initial pair history (optional)
  std::vector<int64_t> hp;
  std::vector<double> hdt;
  std::vector<uint8_t> hb;
  int64_t np0 = init->n_pairs > 0 ? init->n_pairs : 0;
  if (np0 > 0) {
    if (!init->pair_idx) return DEM_E_INVAL;
    if (fetch(hp, init->pair_idx, 2 * np0) != hipSuccess) return DEM_E_DEVICE;
    if (init->pair_dt && fetch(hdt, init->pair_dt, 3 * np0) != hipSuccess) return DEM_E_DEVICE;
    if (init->pair_bonded && fetch(hb, init->pair_bonded, np0) != hipSuccess) return DEM_E_DEVICE;
    for (int64_t k = 0; k < np0; ++k) {
      int64_t a = hp[2 * k], b = hp[2 * k + 1];
      if (a < 0 || b < 0 || a >= n || b >= n || a == b) return DEM_E_INVAL;
    }
  }

  dem_ctx* c = new dem_ctx();
  c->device = device;
  c->step = init->step;
  c->stream = (hipStream_t)hip_stream;
  c->params.assign(params, params + n_samples);
  c->offsets = offs;
  c->fp64 = params[0].precision == DEM_PREC_FP64;
  c->rsz = c->fp64 ? 8 : 4;
  DevState& d = c->d;
  memset(&d, 0, sizeof(d));
  d.n = n;
  d.nsamples = n_samples;
  d.dt = params[0].dt;
  d.couple_every = params[0].couple_every > 0 ? params[0].couple_every : 1;
  c->sc.resize(n_samples);
  int64_t bin_base = 0, cell_base = 0, dual_base = 0;
  for (int s = 0; s < n_samples; ++s) {
    SampleConst& k = c->sc[s];
    derive(params[s], x.data(), r.data(), alive.data(), offs[s], offs[s + 1], k);
    k.bin_base = bin_base;
    bin_base += (int64_t)k.bn[0] * k.bn[1] * k.bn[2] + 1;
    k.cell_base = cell_base;
    k.dual_base = dual_base;
    if (params[s].fluid_on) {
      cell_base += (int64_t)k.gn[0] * k.gn[1] * k.gn[2];
      c->any_fluid = 1;
    }
    dual_base += (int64_t)k.dn[0] * k.dn[1] * k.dn[2] + 1;
    if (params[s].mu_roll > 0.0) d.rolling = 1;
  }
  d.nbins_total = bin_base;
  d.ncell = cell_base;
  d.ndual = dual_base;
  if (bin_base > ((int64_t)1 << 31) - 2 || dual_base > ((int64_t)1 << 31) - 2) { delete c; return DEM_E_INVAL; }

  auto fail = [&](dem_status st) { dem_destroy(c); return st; };
  const int64_t R4B = 4 * (int64_t)c->rsz;
  bool ok = true;
  for (int b = 0; b < 2; ++b) {
    ok &= dalloc(c, &d.xr[b], n) == hipSuccess && dalloc(c, &d.vel[b], n) == hipSuccess;
    ok &= dalloc_bytes(c, &d.omg[b], n * R4B) == hipSuccess;
    ok &= dalloc(c, &d.alive[b], n) == hipSuccess;
  }
  ok &= dalloc(c, &d.xref, n) == hipSuccess;
  void** r4s[] = {&d.frc, &d.trq, &d.fdr, &d.t_r4[0], &d.t_r4[1], &d.t_r4[2]};
  for (void** q : r4s) ok &= dalloc_bytes(c, q, n * R4B) == hipSuccess;
  ok &= dalloc(c, &d.sample, n) == hipSuccess && dalloc(c, &d.orig, n) == hipSuccess;
  ok &= dalloc(c, &d.t_i[0], n) == hipSuccess && dalloc(c, &d.t_i[1], n) == hipSuccess;
  int64_t nbk = std::max<int64_t>(d.nbins_total, n) + 2;
  ok &= dalloc(c, &d.key, n) == hipSuccess;
  ok &= dalloc(c, &d.bucket_cnt, nbk) == hipSuccess && dalloc(c, &d.bucket_fill, nbk) == hipSuccess;
  ok &= dalloc(c, &d.cell_start, nbk) == hipSuccess && dalloc(c, &d.bin_sample, nbk) == hipSuccess;
  ok &= dalloc(c, &d.bin_sink, nbk) == hipSuccess;
  ok &= dalloc(c, &d.order, n) == hipSuccess && dalloc(c, &d.order_tmp, n) == hipSuccess;
  ok &= dalloc(c, &d.inv_order, n) == hipSuccess;
  ok &= dalloc(c, &d.ncnt, n + 1) == hipSuccess && dalloc(c, &d.ocnt, n + 1) == hipSuccess;
  ok &= dalloc(c, &d.scr, n * kRowMax) == hipSuccess && dalloc(c, &d.ovf, n) == hipSuccess;
  ok &= dalloc(c, &d.novf, 1) == hipSuccess;
  ok &= dalloc(c, &d.wcnt, n + 1) == hipSuccess;
  for (int q = 0; q < 2; ++q) {
    ok &= dalloc(c, &c->ns[q].nrow, n + 1) == hipSuccess;
    ok &= dalloc(c, &c->ns[q].hrow, n + 1) == hipSuccess;
    ok &= dalloc(c, &c->ws[q].wrow, n + 1) == hipSuccess;
  }
  if (!ok) return fail(DEM_E_NOMEM);
  int64_t cap0 = params[0].pair_capacity > 0 ? params[0].pair_capacity : 4 * n + 1024;
  c->fixed_capacity = !(params[0].flags & DEM_FLAG_AUTO_REGROW) ? std::max<int64_t>(params[0].pair_capacity, 0) : 0;
  for (int q = 0; q < 2; ++q) {
    if (grow_nbr(c, c->ns[q], 2 * cap0, cap0) != hipSuccess) return fail(DEM_E_NOMEM);
    if (grow_walls(c, c->ws[q], n / 4 + 256) != hipSuccess) return fail(DEM_E_NOMEM);
  }
  // fluid
  int64_t nc = std::max<int64_t>(d.ncell, 1);
  ok &= dalloc(c, &d.cell_sample, nc) == hipSuccess;
  ok &= dalloc(c, &d.u_in, 3 * nc) == hipSuccess && dalloc(c, &d.gp_in, 3 * nc) == hipSuccess;
  ok &= dalloc(c, &d.cell_n, nc) == hipSuccess && dalloc(c, &d.cell_u, 3 * nc) == hipSuccess;
  ok &= dalloc(c, &d.eps, nc) == hipSuccess && dalloc(c, &d.fdc, 3 * nc) == hipSuccess;
  ok &= dalloc(c, &d.dkey, n) == hipSuccess && dalloc(c, &d.dfr, n) == hipSuccess;
  ok &= dalloc(c, &d.fpart, n) == hipSuccess;
  ok &= dalloc(c, &d.dpart, 32 * (d.ndual + 1)) == hipSuccess;
  ok &= dalloc(c, &d.docc, d.ndual + 1) == hipSuccess && dalloc(c, &d.dual_sample, d.ndual + 1) == hipSuccess;
  ok &= dalloc(c, &d.dlmem, 64 * (d.ndual + 1)) == hipSuccess && dalloc(c, &d.dlcnt, 8 * (d.ndual + 1)) == hipSuccess;
  ok &= dalloc(c, &d.sc, n_samples) == hipSuccess;
  ok &= dalloc(c, &d.broken, n_samples) == hipSuccess;
  ok &= dalloc(c, &d.produced_fx, n_samples) == hipSuccess;
  ok &= dalloc(c, &d.produced_cls, (int64_t)n_samples * DEM_MAX_SIZE_CLASSES) == hipSuccess;
  ok &= dalloc(c, &d.abort, 4) == hipSuccess;   // abort, abort_step, status: adjacent
  d.abort_step = d.abort + 1;
  d.status = d.abort + 2;
  ok &= dalloc(c, &d.totals, 4) == hipSuccess;
  ok &= dalloc_bytes(c, (void**)&c->d_dev, sizeof(DevState)) == hipSuccess;
  d.self = c->d_dev;
  // tuned on the 200 000-sphere cylinder: the gather of the half-pair mode (the
  // default) is fastest with 2 lanes per particle, full rows with 4
  d.group = 2;
  d.pair_mode = DEM_PAIRS_HALF;   // 48.6 against 55.9 us per step at 200 000 spheres
  int64_t scan_n = std::max<int64_t>(nbk, n + 1);
  d.scan_tmp_n = scan_n / 256 + 4096;
  ok &= dalloc(c, &d.scan_tmp, d.scan_tmp_n) == hipSuccess;
  if (!ok) return fail(DEM_E_NOMEM);
  if (hipHostMalloc((void**)&c->h_flags, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) return fail(DEM_E_NOMEM);
  if (hipHostMalloc((void**)&c->h_tot, 4 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) return fail(DEM_E_NOMEM);
  if (dalloc(c, &c->d_offsets, n_samples + 1) != hipSuccess) return fail(DEM_E_NOMEM);

  // upload in the caller's order into buffer 0
  std::vector<double4> hx(n), hv(n);
  std::vector<int32_t> hs(n), ho(n);
  std::vector<char> hw(n * R4B), hF(n * R4B), hT(n * R4B), hFF(n * R4B, 0);
  for (int s = 0; s < n_samples; ++s) {
    const dem_params& p = params[s];
    for (int64_t i = offs[s]; i < offs[s + 1]; ++i) {
      double m = p.rho * (4.0 / 3.0) * kPi * r[i] * r[i] * r[i];
      double I = 0.4 * m * r[i] * r[i];
      hx[i] = make_double4(x[3 * i], x[3 * i + 1], x[3 * i + 2], r[i]);
      hv[i] = make_double4(v[3 * i], v[3 * i + 1], v[3 * i + 2], 1.0 / m);
      hs[i] = s;
      ho[i] = (int32_t)i;
      if (c->fp64) {
        ((double4*)hw.data())[i] = make_double4(w[3 * i], w[3 * i + 1], w[3 * i + 2], 1.0 / I);
        ((double4*)hF.data())[i] = make_double4(F[3 * i], F[3 * i + 1], F[3 * i + 2], 0.0);
        ((double4*)hT.data())[i] = make_double4(T[3 * i], T[3 * i + 1], T[3 * i + 2], 0.0);
        if (!FF.empty()) ((double4*)hFF.data())[i] = make_double4(FF[3 * i], FF[3 * i + 1], FF[3 * i + 2], 0.0);
      } else {
        ((float4*)hw.data())[i] = make_float4((float)w[3 * i], (float)w[3 * i + 1], (float)w[3 * i + 2], (float)(1.0 / I));
        ((float4*)hF.data())[i] = make_float4((float)F[3 * i], (float)F[3 * i + 1], (float)F[3 * i + 2], 0.f);
        ((float4*)hT.data())[i] = make_float4((float)T[3 * i], (float)T[3 * i + 1], (float)T[3 * i + 2], 0.f);
        if (!FF.empty())
          ((float4*)hFF.data())[i] = make_float4((float)FF[3 * i], (float)FF[3 * i + 1], (float)FF[3 * i + 2], 0.f);
      }
    }
  }
  std::vector<int32_t> cs(nc, 0), bs(nbk, 0);
  std::vector<uint8_t> bsink(nbk, 0);
  std::vector<int32_t> dsamp(d.ndual + 1, 0);
  for (int s = 0; s < n_samples; ++s) {
    const SampleConst& k = c->sc[s];
    for (int64_t q = 0; q <= (int64_t)k.dn[0] * k.dn[1] * k.dn[2]; ++q) dsamp[k.dual_base + q] = s;
  }
  for (int s = 0; s < n_samples; ++s) {
    const SampleConst& k = c->sc[s];
    bsink[k.bin_base + (int64_t)k.bn[0] * k.bn[1] * k.bn[2]] = 1;
  }
  for (int s = 0; s < n_samples; ++s) {
    if (params[s].fluid_on)
      for (int64_t q = 0; q < (int64_t)c->sc[s].gn[0] * c->sc[s].gn[1] * c->sc[s].gn[2]; ++q)
        cs[c->sc[s].cell_base + q] = s;
    int64_t nbs = (int64_t)c->sc[s].bn[0] * c->sc[s].bn[1] * c->sc[s].bn[2] + 1;
    for (int64_t q = 0; q < nbs; ++q) bs[c->sc[s].bin_base + q] = s;
  }
  hipStream_t st = c->stream;
  bool up = true;
  d.cur = 0;
  up &= hipMemcpyAsync(d.xr[0], hx.data(), sizeof(double4) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.vel[0], hv.data(), sizeof(double4) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.omg[0], hw.data(), n * R4B, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.alive[0], alive.data(), n, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.frc, hF.data(), n * R4B, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.trq, hT.data(), n * R4B, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.fdr, hFF.data(), n * R4B, hipMemcpyHostToDevice, st) == hipSuccess;
  // the bucket sorts expect their counters at zero (each sort clears them after use)
  up &= hipMemsetAsync(d.bucket_cnt, 0, sizeof(int32_t) * nbk, st) == hipSuccess;
  up &= hipMemsetAsync(d.bucket_fill, 0, sizeof(int32_t) * nbk, st) == hipSuccess;
  up &= hipMemcpyAsync(d.sample, hs.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.orig, ho.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.sc, c->sc.data(), sizeof(SampleConst) * n_samples, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.cell_sample, cs.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.bin_sample, bs.data(), sizeof(int32_t) * nbk, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(d.bin_sink, bsink.data(), nbk, hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemcpyAsync(c->d_offsets, offs.data(), sizeof(int64_t) * (n_samples + 1), hipMemcpyHostToDevice, st) == hipSuccess;
  up &= hipMemsetAsync(d.broken, 0, sizeof(unsigned long long) * n_samples, st) == hipSuccess;
  up &= hipMemsetAsync(d.produced_fx, 0, sizeof(unsigned long long) * n_samples, st) == hipSuccess;
  up &= hipMemsetAsync(d.produced_cls, 0, sizeof(unsigned long long) * n_samples * DEM_MAX_SIZE_CLASSES, st) ==
        hipSuccess;
  up &= hipMemsetAsync(d.status, 0, sizeof(int), st) == hipSuccess;
  up &= hipMemsetAsync(d.abort, 0, sizeof(int), st) == hipSuccess;
  up &= hipMemsetAsync(d.eps, 0, sizeof(double) * nc, st) == hipSuccess;
  up &= hipMemsetAsync(d.docc, 0, d.ndual + 1, st) == hipSuccess;
  up &= hipMemcpyAsync(d.dual_sample, dsamp.data(), sizeof(int32_t) * (d.ndual + 1), hipMemcpyHostToDevice, st) ==
        hipSuccess;
  up &= hipMemsetAsync(d.fdc, 0, sizeof(double) * 3 * nc, st) == hipSuccess;
  up &= hipMemsetAsync(d.u_in, 0, sizeof(double) * 3 * nc, st) == hipSuccess;
  up &= hipMemsetAsync(d.gp_in, 0, sizeof(double) * 3 * nc, st) == hipSuccess;
  // the "previous list" of the first build is the given history: full CSR rows
  // over caller indices (both directions), one slot per pair
  NbrSet& old = c->ns[1];
  WallSet& wold = c->ws[1];
  c->hist_old = 0;
  {
    std::vector<std::pair<std::pair<int64_t, int64_t>, int64_t>> items;
    for (int64_t k = 0; k < np0; ++k) {
      int64_t a = hp[2 * k], b = hp[2 * k + 1];
      items.push_back({{std::min(a, b), std::max(a, b)}, k});
    }
    std::sort(items.begin(), items.end());
    int64_t npair = (int64_t)items.size();
    if (grow_nbr(c, old, 2 * npair, npair) != hipSuccess) return fail(DEM_E_NOMEM);
    std::vector<std::vector<std::pair<int32_t, int32_t>>> rows(n);   // (partner, slot)
    std::vector<int32_t> sown(npair), spart(npair);
    std::vector<uint8_t> pfl(npair);
    std::vector<char> ph(npair * R4B, 0);
    for (int64_t q = 0; q < npair; ++q) {
      int64_t a = items[q].first.first, b = items[q].first.second, k = items[q].second;
      rows[a].push_back({(int32_t)b, (int32_t)q});
      rows[b].push_back({(int32_t)a, (int32_t)q});
      sown[q] = (int32_t)a;
      spart[q] = (int32_t)b;
      double sg = hp[2 * k] < hp[2 * k + 1] ? 1.0 : -1.0;
      pfl[q] = hb.empty() ? 0 : (hb[k] ? 1 : 0);
      if (params[0].normal_model != DEM_NORMAL_JKR_MOD && params[0].normal_model != DEM_NORMAL_JKR_ORIG) pfl[q] = 0;
      double t3[3] = {0, 0, 0};
      if (!hdt.empty()) for (int e = 0; e < 3; ++e) t3[e] = sg * hdt[3 * k + e];
      // a clear flag stands for a zero elongation: a given elongation sets the touching bit
      if (t3[0] != 0.0 || t3[1] != 0.0 || t3[2] != 0.0) pfl[q] |= 2;
      if (c->fp64) ((double4*)ph.data())[q] = make_double4(t3[0], t3[1], t3[2], 0.0);
      else ((float4*)ph.data())[q] = make_float4((float)t3[0], (float)t3[1], (float)t3[2], 0.f);
    }
    std::vector<int32_t> nrow(n + 1, 0), nbr, nslot;
    for (int64_t i = 0; i < n; ++i) {
      std::sort(rows[i].begin(), rows[i].end());
      nrow[i + 1] = nrow[i] + (int32_t)rows[i].size();
      for (auto& e : rows[i]) { nbr.push_back(e.first); nslot.push_back(e.second); }
    }
    up &= hipMemcpyAsync(old.nrow, nrow.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st) == hipSuccess;
    if (npair > 0) {
      up &= hipMemcpyAsync(old.nbr, nbr.data(), sizeof(int32_t) * nbr.size(), hipMemcpyHostToDevice, st) == hipSuccess;
      up &= hipMemcpyAsync(old.nslot, nslot.data(), sizeof(int32_t) * nslot.size(), hipMemcpyHostToDevice, st) == hipSuccess;
      up &= hipMemcpyAsync(old.sown, sown.data(), sizeof(int32_t) * npair, hipMemcpyHostToDevice, st) == hipSuccess;
      up &= hipMemcpyAsync(old.spart, spart.data(), sizeof(int32_t) * npair, hipMemcpyHostToDevice, st) == hipSuccess;
      up &= hipMemcpyAsync(old.pfl[0], pfl.data(), npair, hipMemcpyHostToDevice, st) == hipSuccess;
      up &= hipMemcpyAsync(old.hdt[0], ph.data(), ph.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    }
    old.nent = (int64_t)nbr.size();
    old.nslots = npair;
    // the given wall history as the "previous" wall list: one entry per
    // (particle, wall) with a nonzero elongation, carried by wall id
    std::vector<int32_t> wrow(n + 1, 0), wid;
    std::vector<char> wdt;
    std::vector<uint8_t> wfl;
    for (int s = 0; s < n_samples; ++s)
      for (int64_t i = offs[s]; i < offs[s + 1]; ++i) {
        for (int wl = 0; !WD.empty() && wl < params[s].n_walls; ++wl) {
          const double* h = &WD[3 * (i * DEM_MAX_WALLS + wl)];
          if (h[0] == 0.0 && h[1] == 0.0 && h[2] == 0.0) continue;
          wid.push_back(wl);
          wfl.push_back(2);
          size_t at = wdt.size();
          wdt.resize(at + R4B);
          if (c->fp64) *(double4*)(wdt.data() + at) = make_double4(h[0], h[1], h[2], 0.0);
          else *(float4*)(wdt.data() + at) = make_float4((float)h[0], (float)h[1], (float)h[2], 0.f);
        }
        wrow[i + 1] = (int32_t)wid.size();
      }
    if (grow_walls(c, wold, (int64_t)wid.size()) != hipSuccess) return fail(DEM_E_NOMEM);
    up &= hipMemcpyAsync(wold.wrow, wrow.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st) == hipSuccess;
    if (!wid.empty()) {
      up &= hipMemcpyAsync(wold.wid, wid.data(), sizeof(int32_t) * wid.size(), hipMemcpyHostToDevice, st) == hipSuccess;
      up &= hipMemcpyAsync(wold.wdt, wdt.data(), wdt.size(), hipMemcpyHostToDevice, st) == hipSuccess;
      up &= hipMemcpyAsync(wold.wfl, wfl.data(), wfl.size(), hipMemcpyHostToDevice, st) == hipSuccess;
    }
    wold.n = (int64_t)wid.size();
    up &= hipStreamSynchronize(st) == hipSuccess;
  }
  if (!up) return fail(DEM_E_DEVICE);
  c->live = 0;
  bind_sets(c);
  int mark = (np0 == 0 && params[0].bond_at_init) ? 1 : 0;
  dem_status rs = c->fp64 ? rebuild<double>(c, 1, mark) : rebuild<float>(c, 1, mark);
  if (rs != DEM_OK) return fail(rs);
  if (hipStreamSynchronize(st) != hipSuccess) return fail(DEM_E_DEVICE);
  *out = c;
  return DEM_OK;
}

dem_status dem_step(dem_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 0) return DEM_E_INVAL;
  if (c->failed) return DEM_E_STATE;
  if (c->any_fluid && !c->have_fluid) return DEM_E_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  return c->fp64 ? step_impl<double>(c, nsteps) : step_impl<float>(c, nsteps);
}

dem_status dem_map_fluid(dem_ctx* c, const double* u_cell, const double* gradp_cell, double* eps_out,
                         double* fdrag_out) {
  if (!c) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  int64_t nc = c->d.ncell;
  hipStream_t s = c->stream;
  if (eps_out && nc > 0) HIPCHK(hipMemcpyAsync(eps_out, c->d.eps, sizeof(double) * nc, hipMemcpyDefault, s));
  if (fdrag_out && nc > 0) HIPCHK(hipMemcpyAsync(fdrag_out, c->d.fdc, sizeof(double) * 3 * nc, hipMemcpyDefault, s));
  if (u_cell && gradp_cell && nc > 0) {
    HIPCHK(hipMemcpyAsync(c->d.u_in, u_cell, sizeof(double) * 3 * nc, hipMemcpyDefault, s));
    HIPCHK(hipMemcpyAsync(c->d.gp_in, gradp_cell, sizeof(double) * 3 * nc, hipMemcpyDefault, s));
    if (!c->have_fluid) drop_graphs(c);   // recorded windows hold no coupling yet
    c->have_fluid = 1;
  } else if (u_cell || gradp_cell) {
    return DEM_E_INVAL;
  }
  HIPCHK(hipStreamSynchronize(s));
  return DEM_OK;
}

static dem_status aggregates(dem_ctx* c, std::vector<double>& pm, std::vector<double>& ke,
                             std::vector<long long>& nc, std::vector<long long>& na, std::vector<unsigned long long>& br) {
  int ns = c->d.nsamples;
  if (!c->agg_buf) {   // outputs (4 per sample) and the per-slice partials, kept for later calls
    int64_t bytes = sizeof(double) * (4 * (int64_t)ns + aggregate_scratch_doubles(ns));
    if (dalloc_bytes(c, (void**)&c->agg_buf, bytes) != hipSuccess) return DEM_E_NOMEM;
  }
  double* dpm = c->agg_buf;
  double* dke = dpm + ns;
  long long* dnc = (long long*)(dke + ns);
  long long* dna = dnc + ns;
  double* part = (double*)(dna + ns);
  launch_aggregate_impl(c->d, c->d_offsets, dpm, dke, dnc, dna, part, c->fp64, c->stream);
  pm.resize(ns); ke.resize(ns); nc.resize(ns); na.resize(ns); br.resize(ns);
  bool ok = hipStreamSynchronize(c->stream) == hipSuccess;
  ok &= hipMemcpy(pm.data(), dpm, sizeof(double) * ns, hipMemcpyDeviceToHost) == hipSuccess;
  ok &= hipMemcpy(ke.data(), dke, sizeof(double) * ns, hipMemcpyDeviceToHost) == hipSuccess;
  ok &= hipMemcpy(nc.data(), dnc, sizeof(long long) * ns, hipMemcpyDeviceToHost) == hipSuccess;
  ok &= hipMemcpy(na.data(), dna, sizeof(long long) * ns, hipMemcpyDeviceToHost) == hipSuccess;
  ok &= hipMemcpy(br.data(), c->d.broken, sizeof(unsigned long long) * ns, hipMemcpyDeviceToHost) == hipSuccess;
  return ok ? DEM_OK : DEM_E_DEVICE;
}

dem_status dem_read_state(dem_ctx* c, dem_state* out) {
  if (!c || !out) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  const int64_t n = c->d.n;
  if (!c->stage) {
    if (hipMalloc((void**)&c->stage, sizeof(double) * 15 * std::max<int64_t>(n, 1)) != hipSuccess) return DEM_E_NOMEM;
    if (hipMalloc((void**)&c->stage_alive, std::max<int64_t>(n, 1)) != hipSuccess) return DEM_E_NOMEM;
  }
  double* sx = c->stage;
  double* sv = sx + 3 * n;
  double* sw = sv + 3 * n;
  double* sF = sw + 3 * n;
  double* sT = sF + 3 * n;
  double *sFF = nullptr, *sWD = nullptr;
  if (out->fluid_force || out->wall_dt) {
    if (!c->stage_aux &&
        hipMalloc((void**)&c->stage_aux, sizeof(double) * (3 + 3 * DEM_MAX_WALLS) * std::max<int64_t>(n, 1)) !=
            hipSuccess)
      return DEM_E_NOMEM;
    sFF = c->stage_aux;
    sWD = sFF + 3 * n;
  }
  hipStream_t s = c->stream;
  if (c->fp64) launch_unpermute<double>(c->d, sx, sv, sw, sF, sT, c->stage_alive, sFF, s);
  else launch_unpermute<float>(c->d, sx, sv, sw, sF, sT, c->stage_alive, sFF, s);
  if (out->wall_dt && n > 0) {
    HIPCHK(hipMemsetAsync(sWD, 0, sizeof(double) * 3 * DEM_MAX_WALLS * n, s));
    if (c->fp64) launch_unpermute_walls<double>(c->d, sWD, s);
    else launch_unpermute_walls<float>(c->d, sWD, s);
  }
  if (out->x) HIPCHK(hipMemcpyAsync(out->x, sx, sizeof(double) * 3 * n, hipMemcpyDefault, s));
  if (out->v) HIPCHK(hipMemcpyAsync(out->v, sv, sizeof(double) * 3 * n, hipMemcpyDefault, s));
  if (out->omega) HIPCHK(hipMemcpyAsync(out->omega, sw, sizeof(double) * 3 * n, hipMemcpyDefault, s));
  if (out->force) HIPCHK(hipMemcpyAsync(out->force, sF, sizeof(double) * 3 * n, hipMemcpyDefault, s));
  if (out->torque) HIPCHK(hipMemcpyAsync(out->torque, sT, sizeof(double) * 3 * n, hipMemcpyDefault, s));
  if (out->alive) HIPCHK(hipMemcpyAsync(out->alive, c->stage_alive, n, hipMemcpyDefault, s));
  if (out->fluid_force) HIPCHK(hipMemcpyAsync(out->fluid_force, sFF, sizeof(double) * 3 * n, hipMemcpyDefault, s));
  if (out->wall_dt)
    HIPCHK(hipMemcpyAsync(out->wall_dt, sWD, sizeof(double) * 3 * DEM_MAX_WALLS * n, hipMemcpyDefault, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<double> pm, ke;
  std::vector<long long> nc, na;
  std::vector<unsigned long long> br;
  dem_status st = aggregates(c, pm, ke, nc, na, br);
  if (st != DEM_OK) return st;
  out->n = n;
  out->produced_mass = 0; out->kinetic = 0; out->n_contacts = 0; out->n_alive = 0; out->broken_bonds = 0;
  for (int q = 0; q < c->d.nsamples; ++q) {
    out->produced_mass += pm[q];
    out->kinetic += ke[q];
    out->n_contacts += nc[q];
    out->n_alive += na[q];
    out->broken_bonds += (int64_t)br[q];
  }
  out->coordination = out->n_alive > 0 ? 2.0 * (double)out->n_contacts / (double)out->n_alive : 0.0;
  out->step = c->step;
  out->time = (double)c->step * c->d.dt;
  if (c->failed) return (c->failed & kStNonFinite) ? DEM_E_NONFINITE : DEM_E_STATE;
  return DEM_OK;
}

dem_status dem_read_aggregates(dem_ctx* c, double* produced_mass, double* coordination, int64_t* broken_bonds,
                               int64_t* n_alive) {
  if (!c) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  std::vector<double> pm, ke;
  std::vector<long long> nc, na;
  std::vector<unsigned long long> br;
  dem_status st = aggregates(c, pm, ke, nc, na, br);
  if (st != DEM_OK) return st;
  for (int q = 0; q < c->d.nsamples; ++q) {
    if (produced_mass) produced_mass[q] = pm[q];
    if (coordination) coordination[q] = na[q] > 0 ? 2.0 * (double)nc[q] / (double)na[q] : 0.0;
    if (broken_bonds) broken_bonds[q] = (int64_t)br[q];
    if (n_alive) n_alive[q] = na[q];
  }
  return DEM_OK;
}

dem_status dem_read_wall_forces(dem_ctx* c, double* force) {
  if (!c || !force) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  HIPCHK(hipStreamSynchronize(c->stream));
  const DevState& d = c->d;
  const int ns = d.nsamples;
  std::vector<double> out((size_t)ns * DEM_MAX_WALLS * 3, 0.0);
  const int64_t ne = d.nwall;
  if (ne > 0 && d.wfrc) {
    std::vector<int32_t> wrow(d.n + 1), wid(ne), smp(d.n);
    std::vector<char> fr(ne * 4 * c->rsz);
    HIPCHK(hipMemcpy(wrow.data(), d.wrow, sizeof(int32_t) * (d.n + 1), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(wid.data(), d.wid, sizeof(int32_t) * ne, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(smp.data(), d.sample, sizeof(int32_t) * d.n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(fr.data(), d.wfrc, fr.size(), hipMemcpyDeviceToHost));
    // fixed order: particles in their sorted order, each particle's entries in order
    for (int64_t i = 0; i < d.n; ++i)
      for (int32_t e = wrow[i]; e < wrow[i + 1]; ++e) {
        double f[3];
        if (c->fp64) { double4 q = ((double4*)fr.data())[e]; f[0] = q.x; f[1] = q.y; f[2] = q.z; }
        else { float4 q = ((float4*)fr.data())[e]; f[0] = q.x; f[1] = q.y; f[2] = q.z; }
        double* o = &out[((size_t)smp[i] * DEM_MAX_WALLS + wid[e]) * 3];
        for (int k = 0; k < 3; ++k) o[k] -= f[k];   // the particle's push on the wall
      }
  }
  HIPCHK(hipMemcpy(force, out.data(), sizeof(double) * out.size(), hipMemcpyDefault));
  return DEM_OK;
}

dem_status dem_set_walls(dem_ctx* c, int32_t sample, int32_t n_walls, const dem_wall* walls) {
  if (!c || !walls || sample < 0 || sample >= c->d.nsamples) return DEM_E_INVAL;
  dem_params p = c->params[sample];
  if (n_walls != p.n_walls) return DEM_E_INVAL;
  for (int w = 0; w < n_walls; ++w) p.walls[w] = walls[w];
  if (validate(p) != DEM_OK) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->params[sample] = p;
  SampleConst& k = c->sc[sample];
  for (int w = 0; w < n_walls; ++w) {
    k.walls[w].kind = walls[w].kind;
    for (int q = 0; q < 6; ++q) k.walls[w].p[q] = walls[w].p[q];
  }
  HIPCHK(hipMemcpy(c->d.sc + sample, &k, sizeof(SampleConst), hipMemcpyHostToDevice));
  // the wall lists hold the walls within the skin of each particle: find them again
  c->force_rebuild = 1;
  return DEM_OK;
}

dem_status dem_read_pairs(dem_ctx* c, int32_t which, int64_t cap, int64_t* pair_idx, double* pair_dt,
                          uint8_t* pair_bonded, int64_t* n_out) {
  if (!c || which < 0 || which > 2 || cap < 0) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  HIPCHK(hipStreamSynchronize(c->stream));
  DevState& d = c->d;
  int64_t np = d.nslots;
  std::vector<int32_t> own(np), pj(np), orig(d.n);
  std::vector<uint8_t> fl(np), al(d.n);
  std::vector<char> h(np * 4 * c->rsz);
  std::vector<double4> xr(d.n);
  if (np > 0) {
    HIPCHK(hipMemcpy(own.data(), d.sown, sizeof(int32_t) * np, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(pj.data(), d.spart, sizeof(int32_t) * np, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(fl.data(), d.pfl[d.cur], np, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(h.data(), d.hdt[d.cur], h.size(), hipMemcpyDeviceToHost));
  }
  if (d.n > 0) {
    HIPCHK(hipMemcpy(orig.data(), d.orig, sizeof(int32_t) * d.n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(xr.data(), d.xr[d.cur], sizeof(double4) * d.n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(al.data(), d.alive[d.cur], d.n, hipMemcpyDeviceToHost));
  }
  std::vector<int64_t> oi;
  std::vector<double> odt;
  std::vector<uint8_t> ob;
  for (int64_t p = 0; p < np; ++p) {
    int32_t i = own[p], j = pj[p];
    bool take;
    if (!al[i] || !al[j]) take = false;
    else if (which == 2) take = true;
    else if (which == 0) take = (fl[p] & 3) != 0;
    else {
      double dx = xr[j].x - xr[i].x, dy = xr[j].y - xr[i].y, dz = xr[j].z - xr[i].z;
      double d2 = (dx * dx + dy * dy) + dz * dz;
      double cs = xr[i].w + xr[j].w;
      take = d2 < cs * cs;
    }
    if (!take) continue;
    int64_t a = orig[i], b = orig[j];
    double sg = 1.0;
    if (a > b) { std::swap(a, b); sg = -1.0; }
    oi.push_back(a);
    oi.push_back(b);
    double t3[3] = {0, 0, 0};   // a clear flag stands for a zero elongation
    if (!fl[p]) {
    } else if (c->fp64) { double4 q = ((double4*)h.data())[p]; t3[0] = q.x; t3[1] = q.y; t3[2] = q.z; }
    else { float4 q = ((float4*)h.data())[p]; t3[0] = q.x; t3[1] = q.y; t3[2] = q.z; }
    for (int e = 0; e < 3; ++e) odt.push_back(sg * t3[e]);
    ob.push_back(fl[p] & 1);
  }
  int64_t cnt = (int64_t)ob.size();
  if (n_out) *n_out = cnt;
  int64_t wr = std::min(cnt, cap);
  if (wr > 0) {
    if (pair_idx) HIPCHK(hipMemcpy(pair_idx, oi.data(), sizeof(int64_t) * 2 * wr, hipMemcpyDefault));
    if (pair_dt) HIPCHK(hipMemcpy(pair_dt, odt.data(), sizeof(double) * 3 * wr, hipMemcpyDefault));
    if (pair_bonded) HIPCHK(hipMemcpy(pair_bonded, ob.data(), wr, hipMemcpyDefault));
  }
  return DEM_OK;
}

dem_status dem_fluid_solve(dem_ctx* c, const int8_t* cell_kind, const double* p_fixed, int32_t max_iter,
                           double rel_tol, double* p_out, double* u_out, double* gradp_out, int32_t* iters,
                           double* rel_residual) {
  if (!c || !cell_kind || !p_fixed || max_iter < 0 || !(rel_tol > 0.0)) return DEM_E_INVAL;
  const int64_t nc = c->d.ncell;
  if (nc <= 0) return DEM_E_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  std::vector<int8_t> kd;
  std::vector<double> pf;
  if (fetch(kd, cell_kind, nc) != hipSuccess || fetch(pf, p_fixed, nc) != hipSuccess) return DEM_E_DEVICE;
  for (int64_t k = 0; k < nc; ++k)
    if (kd[k] < 0 || kd[k] > 2 || !std::isfinite(pf[k])) return DEM_E_INVAL;
  const int64_t nw = cfd_work_doubles(nc);
  if (!c->cfd_work) {
    bool ok = dalloc(c, &c->cfd_kind, nc) == hipSuccess && dalloc(c, &c->cfd_pfix, nc) == hipSuccess;
    ok &= dalloc(c, &c->cfd_work, nw) == hipSuccess && dalloc(c, &c->cfd_out, 7 * nc) == hipSuccess;
    if (!ok) return DEM_E_NOMEM;
    if (hipHostMalloc((void**)&c->cfd_scal, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) return DEM_E_NOMEM;
  }
  hipStream_t s = c->stream;
  HIPCHK(hipMemcpyAsync(c->cfd_kind, kd.data(), nc, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->cfd_pfix, pf.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
  double* P = c->cfd_out;
  double* U = P + nc;
  double* GP = U + 3 * nc;
  int it = 0;
  double rel = 0.0;
  dem_status st = cfd_solve(c->d, c->cfd_kind, c->cfd_pfix, c->cfd_work, nw, c->cfd_warm, max_iter, rel_tol, P, U, GP,
                            &it, &rel, c->cfd_scal, s);
  if (st != DEM_OK) return st;
  c->cfd_warm = 1;
  if (p_out) HIPCHK(hipMemcpyAsync(p_out, P, sizeof(double) * nc, hipMemcpyDefault, s));
  if (u_out) HIPCHK(hipMemcpyAsync(u_out, U, sizeof(double) * 3 * nc, hipMemcpyDefault, s));
  if (gradp_out) HIPCHK(hipMemcpyAsync(gradp_out, GP, sizeof(double) * 3 * nc, hipMemcpyDefault, s));
  HIPCHK(hipStreamSynchronize(s));
  if (iters) *iters = it;
  if (rel_residual) *rel_residual = rel;
  return DEM_OK;
}

dem_status dem_set_size_classes(dem_ctx* c, int32_t n_edges, const double* edges) {
  if (!c) return DEM_E_INVAL;
  if (n_edges != 0 && (!edges || n_edges < 2 || n_edges > DEM_MAX_SIZE_CLASSES + 1)) return DEM_E_INVAL;
  for (int k = 0; k < n_edges; ++k)
    if (!std::isfinite(edges[k]) || !(edges[k] >= 0.0) || (k > 0 && !(edges[k] > edges[k - 1]))) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  HIPCHK(hipStreamSynchronize(c->stream));
  DevState& d = c->d;
  HIPCHK(hipMemsetAsync(d.produced_cls, 0, sizeof(unsigned long long) * d.nsamples * DEM_MAX_SIZE_CLASSES,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  d.ncls = edges ? n_edges - 1 : 0;
  for (int k = 0; k <= DEM_MAX_SIZE_CLASSES; ++k) d.cls_edge[k] = k < n_edges && edges ? edges[k] : 0.0;
  return DEM_OK;
}

dem_status dem_read_produced_classes(dem_ctx* c, double* mass) {
  if (!c || !mass) return DEM_E_INVAL;
  DevState& d = c->d;
  if (d.ncls <= 0) return DEM_E_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  HIPCHK(hipStreamSynchronize(c->stream));
  const int ns = d.nsamples;
  std::vector<unsigned long long> q((size_t)ns * DEM_MAX_SIZE_CLASSES);
  HIPCHK(hipMemcpy(q.data(), d.produced_cls, sizeof(unsigned long long) * q.size(), hipMemcpyDeviceToHost));
  std::vector<double> out((size_t)ns * d.ncls);
  for (int s = 0; s < ns; ++s)
    for (int k = 0; k < d.ncls; ++k) out[(size_t)s * d.ncls + k] = (double)q[(size_t)s * DEM_MAX_SIZE_CLASSES + k] / c->sc[s].pm_scale;
  HIPCHK(hipMemcpy(mass, out.data(), sizeof(double) * out.size(), hipMemcpyDefault));
  return DEM_OK;
}

dem_status dem_info(dem_ctx* c, int64_t* ncell, int64_t* n_pairs, int64_t* pair_capacity, int64_t* rebuilds,
                    double* cutoff_margin) {
  if (!c) return DEM_E_INVAL;
  if (ncell) *ncell = c->d.ncell;
  if (n_pairs) *n_pairs = c->d.nslots;
  if (pair_capacity) *pair_capacity = c->d.slot_cap;
  if (rebuilds) *rebuilds = c->rebuilds;
  if (cutoff_margin) *cutoff_margin = c->sc[0].margin;
  return DEM_OK;
}

dem_status dem_profile(dem_ctx* c, int32_t enable) {
  if (!c) return DEM_E_INVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  prof_collect(c);
  if (enable) {
    for (int k = 0; k < DEM_PROF_N; ++k) { c->prof_ms[k] = 0.0; c->prof_cnt[k] = 0; }
  }
  c->prof = enable ? 1 : 0;
  return DEM_OK;
}

dem_status dem_read_profile(dem_ctx* c, double* total_ms, int64_t* launches) {
  if (!c) return DEM_E_INVAL;
  for (int k = 0; k < DEM_PROF_N; ++k) {
    if (total_ms) total_ms[k] = c->prof_ms[k];
    if (launches) launches[k] = c->prof_cnt[k];
  }
  return DEM_OK;
}

dem_status dem_read_fault(dem_ctx* c, int32_t* bits) {
  if (!c || !bits) return DEM_E_INVAL;
  *bits = c->failed;
  return DEM_OK;
}

dem_status dem_set_closure(dem_ctx* c, const dem_mlp* mlp, const double* norm) {
  if (!c) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  drop_graphs(c);
  DevState& d = c->d;
  hipStream_t s = c->stream;
  if (!mlp) {
    if (d.cdrag) {
      c->cl_buf[0] = d.cdrag; c->cl_buf[1] = d.ccoh; c->cl_buf[2] = d.t_d[0]; c->cl_buf[3] = d.t_d[1];
    }
    d.cdrag = d.ccoh = nullptr;
    d.closure_on = 0;
    return DEM_OK;
  }
  if (!norm) return DEM_E_INVAL;
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(norm[k]) || (k >= 6 && !(norm[k] > 0.0))) return DEM_E_INVAL;
  const int64_t n = d.n;
  if (!c->cl_buf[0] && !d.cdrag) {
    bool ok = true;
    for (int q = 0; q < 4; ++q) ok &= dalloc(c, &c->cl_buf[q], n) == hipSuccess;
    ok &= dalloc(c, &c->cl_feat, 6 * n) == hipSuccess && dalloc(c, &c->cl_feat_tmp, 6 * n) == hipSuccess;
    ok &= dalloc(c, &c->cl_norm, 12) == hipSuccess;
    ok &= dalloc(c, &c->cl_wb, DEM_MLP_NPARAMS) == hipSuccess && dalloc(c, &c->cl_pf, DEM_MLP_NPARAMS) == hipSuccess;
    if (!ok) return DEM_E_NOMEM;
    d.cfeat = c->cl_feat;
    d.t_feat = c->cl_feat_tmp;
  }
  if (!d.cdrag) {
    d.cdrag = c->cl_buf[0]; d.ccoh = c->cl_buf[1]; d.t_d[0] = c->cl_buf[2]; d.t_d[1] = c->cl_buf[3];
  }
  // snapshot of the network and the normalisation; factors 1 until the next evaluation
  if (hipStreamSynchronize(mlp_stream(mlp)) != hipSuccess) return DEM_E_DEVICE;
  std::vector<double> ones(n > 0 ? n : 1, 1.0), zf(6 * (n > 0 ? n : 1), 0.0);
  HIPCHK(hipMemcpyAsync(c->cl_wb, mlp_weights_bf16(mlp), sizeof(short) * DEM_MLP_NPARAMS, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->cl_pf, mlp_params_f32(mlp), sizeof(float) * DEM_MLP_NPARAMS, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c->cl_norm, norm, sizeof(double) * 12, hipMemcpyHostToDevice, s));
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(d.cdrag, ones.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.ccoh, ones.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d.cfeat, zf.data(), sizeof(double) * 6 * n, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  d.cl_wb = c->cl_wb;
  d.cl_pf = c->cl_pf;
  d.cl_norm = c->cl_norm;
  d.closure_on = 1;
  return DEM_OK;
}

dem_status dem_read_closure(dem_ctx* c, double* features, double* c_drag, double* c_coh) {
  if (!c) return DEM_E_INVAL;
  if (!c->d.closure_on) return DEM_E_STATE;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  DevState& d = c->d;
  const int64_t n = d.n;
  HIPCHK(hipStreamSynchronize(c->stream));
  std::vector<int32_t> orig(n > 0 ? n : 1);
  std::vector<double> f(6 * (n > 0 ? n : 1)), a(n > 0 ? n : 1), b(n > 0 ? n : 1);
  if (n > 0) {
    HIPCHK(hipMemcpy(orig.data(), d.orig, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(f.data(), d.cfeat, sizeof(double) * 6 * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(a.data(), d.cdrag, sizeof(double) * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(b.data(), d.ccoh, sizeof(double) * n, hipMemcpyDeviceToHost));
  }
  for (int64_t k = 0; k < n; ++k) {
    const int64_t o = orig[k];
    if (features) for (int q = 0; q < 6; ++q) features[6 * o + q] = f[6 * k + q];
    if (c_drag) c_drag[o] = a[k];
    if (c_coh) c_coh[o] = b[k];
  }
  return DEM_OK;
}

dem_status dem_set_lanes(dem_ctx* c, int32_t lanes) {
  if (!c || (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16)) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  c->d.group = lanes;
  c->lanes_set = 1;
  return DEM_OK;
}

dem_status dem_set_pair_mode(dem_ctx* c, int32_t mode) {
  if (!c || (mode != DEM_PAIRS_FULL_ROWS && mode != DEM_PAIRS_HALF)) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  c->d.pair_mode = mode;
  if (!c->lanes_set) c->d.group = mode == DEM_PAIRS_HALF ? 2 : 4;
  return DEM_OK;
}

dem_status dem_set_graphs(dem_ctx* c, int32_t enable) {
  if (!c) return DEM_E_INVAL;
  if (hipSetDevice(c->device) != hipSuccess) return DEM_E_DEVICE;
  HIPCHK(hipStreamSynchronize(c->stream));
  drop_graphs(c);
  c->use_graphs = enable ? 1 : 0;
  return DEM_OK;
}

dem_status dem_request_rebuild(dem_ctx* c) {
  if (!c) return DEM_E_INVAL;
  c->force_rebuild = 1;
  return DEM_OK;
}

void dem_destroy(dem_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void* p : c->allocs)
    if (p) (void)hipFree(p);
  if (c->stage) (void)hipFree(c->stage);
  if (c->stage_alive) (void)hipFree(c->stage_alive);
  if (c->stage_aux) (void)hipFree(c->stage_aux);
  if (c->cfd_scal) (void)hipHostFree(c->cfd_scal);
  if (c->h_flags) (void)hipHostFree(c->h_flags);
  if (c->h_tot) (void)hipHostFree(c->h_tot);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
