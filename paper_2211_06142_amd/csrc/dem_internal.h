// dem_internal.h -- device data layout and launch interfaces of the DEM library.
//
// Layout in HBM.  Particles live in sorted order (sample-major, binning cell,
// particle id; the dead particles of a sample sit in one extra bucket at the
// end of the sample's range):
//   xr[b]    double4  position (x, y, z) and radius           } double-buffered:
//   vel[b]   double4  velocity and 1/m                         } step s reads b,
//   omg[b]   R4       angular velocity and 1/I                 } writes 1-b
//   alive[b] uint8                                             }
//   frc, trq R4       force / torque at the last step boundary
//   fdr      R4       fluid force held since the last coupling evaluation
//   R = double (FP64 mode) or float (mixed mode).
// Neighbour list (rebuilt when a particle has moved more than half the skin):
//   full rows in CSR by particle, partners in increasing order, so the
//   entries with j > i (the half pairs i owns) form the tail of row i;
//   nbr[e]   int32 partner, nslot[e] int32 half-pair slot of the entry
//   half-pair slots: hdt[b][p] R4 tangential elongation (owner -> partner),
//   pfl[b][p] uint8 bit0 bonded, bit1 touching; double-buffered like the
//   particles because both partners read slot p while its owner writes it.
//   A clear flag stands for a zero elongation: hdt[b][p] is read and written
//   only where the flag is set (a pair out of contact costs one byte).
// Wall entries: CSR by particle, private to the particle (single buffer).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dem.h"

namespace dem {

constexpr int kMaxWalls = DEM_MAX_WALLS;
constexpr int kRowMax = 32;      // stride of the scratch rows of the candidate search

enum StatusBits : int {
  kStCapacity = 1,
  kStNonFinite = 2,
  kStTooFast = 4,
  kStLostBond = 8,
  kStBadAbort = 16,
};

struct Wall {
  int kind;
  double p[6];
};

// Per-sample constants, derived on the host from dem_params (grain scale).
struct SampleConst {
  double Es, Gs, beta, cdamp;     // E*, G*, damping ratio, 2 sqrt(5/6) beta
  double gamma, mu, mu_roll, rho, k_lin;
  double kcg, k3;                 // drag rule f = k^3 f(d / k)
  // the contact constants rounded to FP32 (the mixed-precision force path)
  float f_Es, f_Gs, f_beta, f_cdamp, f_mu, f_mu_roll, f_k_lin;
  int normal_model;
  double jkr_break;               // bonded pairs apart hold while (-delta)^3 <= jkr_break pi^2 gamma^2 R*/E*^2:
                                  // 3/16 (point C, modified JKR) or 27/16 (point S, original JKR)
  int fluid_on, voidfrac, u_superficial;
  double rho_f, mu_f, n_min;
  double glo[3], gh[3], vcell;    // fluid grid
  int gn[3];
  int dn[3];                      // bucket grid of the coupling sort
  int64_t cell_base, dual_base;
  double blo[3], bh[3];           // binning grid of the neighbour list
  int bn[3];
  int64_t bin_base;               // first bin; the sample's dead bucket is bin_base + nbins
  double margin;                  // candidate margin: skin + largest pull-off separation
  double skin;
  double pm_scale;                // produced mass counts in units of 1 / pm_scale kg (a power
                                  // of two: the sample's whole mass stays below 2^61 units)
  double g[3];
  int outlet_kind;
  double outlet[4];
  int n_walls;
  Wall walls[kMaxWalls];
};

template <typename R> struct Vec4;
template <> struct Vec4<double> { using type = double4; };
template <> struct Vec4<float> { using type = float4; };
template <typename R> using R4 = typename Vec4<R>::type;

struct DevState {
  const DevState* self;            // device copy of this struct (read by the step-window kernels)
  int64_t n;
  int nsamples;
  double dt;
  int couple_every;
  int rolling;                     // any sample with mu_roll > 0
  int group;                       // lanes per particle of the step kernel (1, 2, 4, 8, 16)
  int pair_mode;                   // DEM_PAIRS_FULL_ROWS or DEM_PAIRS_HALF
  void* rec[2];                    // half-pair mode, per slot (written and read in one step):
                                   // [0] 6 R: force on the owner, n x F_t; [1] R4 rolling torque
                                   // on the owner; written only for slots whose new flag is set
  int cur;                         // buffer holding the current particle state and history
  // double-buffered particle state
  double4 *xr[2], *vel[2];
  void* omg[2];
  uint8_t* alive[2];
  // single-buffered particle arrays (permuted through the tmp buffers)
  void *frc, *trq, *fdr;
  double4* xref;
  int32_t *sample, *orig;
  double *cdrag, *ccoh;            // closure factors (NULL when off)
  int closure_on;                  // learned closure evaluated at every coupling step
  double* cfeat;                   // n x 6 closure features of the latest evaluation
  double* t_feat;                  // permutation scratch of cfeat
  const void* cl_wb;               // closure network: BF16 weights, FP32 parameters,
  const float* cl_pf;              //   feature mean[6] and standard deviation[6]
  const double* cl_norm;
  // permutation scratch
  void *t_r4[3];
  double4* t_d4;
  int32_t *t_i[2];
  double* t_d[2];
  // bucket sort scratch
  uint32_t* key;
  int32_t *bucket_cnt, *bucket_fill, *order, *order_tmp, *inv_order;
  int64_t nbins_total;
  int32_t* cell_start;             // nbins_total + 1
  int32_t* bin_sample;             // nbins_total: sample of each bin
  uint8_t* bin_sink;               // nbins_total: 1 for each sample's dead bucket
  // live neighbour list
  int64_t ent_cap, nent, slot_cap, nslots;
  int32_t *nrow, *nbr, *nslot, *hrow, *sown, *spart;
  void* hdt[2];
  uint8_t* pfl[2];
  int32_t *ncnt, *ocnt;
  int32_t* scr;                    // n * kRowMax: rows found by the search
  int32_t* ovf;                    // rows longer than kRowMax or found outside LDS
  int* novf;
  // previous list (history source at a rebuild)
  int32_t *nrow_o, *nbr_o, *nslot_o;
  void* hdt_o;
  uint8_t* pfl_o;
  int64_t nslots_o;
  int32_t *sown_o, *spart_o;
  // wall entries
  int64_t wall_cap, nwall;
  int32_t *wrow, *wcnt, *wid, *wrow_o, *wid_o;
  void *wdt, *wdt_o;               // R4
  uint8_t *wfl, *wfl_o;
  void* wfrc;                      // R4 per wall entry: the wall's force on the particle at the
                                   // last evaluation (zero out of contact)
  // fluid
  int64_t ncell, ndual;
  int32_t* cell_sample;
  double *u_in, *gp_in;            // 3*ncell
  double *cell_n, *cell_u;         // ncell, 3*ncell
  double *eps, *fdc;               // ncell, 3*ncell (latest evaluation)
  double* dpart;                   // per bucket: 8 solid-volume corner partials, then (from
                                   // 8 * (ndual + 1) on) 24 drag corner partials
  int32_t* dkey;
  uint8_t* docc;                   // ndual: bucket named by some particle's key in this evaluation
  int32_t* dlmem;                  // 64 * ndual: each bucket's members, lane-major in scan order
  uint8_t* dlcnt;                  // 8 * ndual: each lane's count (255: the list overflowed, scan again)
  int32_t* dual_sample;            // ndual: sample of each bucket
  double4* dfr;                    // CIC fractions (fx, fy, fz, volume)
  double4* fpart;                  // particle drag of the latest evaluation
  // per-sample, status
  SampleConst* sc;
  unsigned long long* broken;      // per sample
  // produced sand, exact: each removal adds its mass rounded to 1 / pm_scale
  // (integer sums do not depend on the order of the removals)
  unsigned long long* produced_fx;    // per sample
  unsigned long long* produced_cls;   // per sample x DEM_MAX_SIZE_CLASSES (fine diameter d/k)
  int ncls;                           // size classes (0: off)
  double cls_edge[DEM_MAX_SIZE_CLASSES + 1];
  int* status;
  int* abort;                      // set when a rebuild is due before the next step
  int* abort_step;
  int32_t* totals;                 // rebuild totals gathered for one copy
  int32_t* scan_tmp;
  int64_t scan_tmp_n;
};

struct StepArgs {
  int64_t step;       // absolute step index of this launch
  int in, out;        // buffer indices
  int final_step;     // 1: last step of the call: end at the step boundary
};

// scans and bucket sort
void scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s);
void launch_bucket_sort(const uint32_t* key, int64_t n, int64_t nb, const int32_t* tiebreak, int32_t* cnt,
                        int32_t* off, int32_t* fill, int32_t* order_tmp, int32_t* out_order,
                        int32_t* scan_tmp, const uint8_t* sink, const int* gate, hipStream_t s);

// rebuild
void launch_bin_keys(DevState& d, hipStream_t s);
template <typename R> void launch_permute(DevState& d, hipStream_t s);
void launch_nbr_search(DevState& d, hipStream_t s);
void launch_totals(DevState& d, hipStream_t s);
void launch_nbr_fill(DevState& d, int novf, hipStream_t s);
void launch_wall_count(DevState& d, hipStream_t s);
void launch_wall_fill(DevState& d, hipStream_t s);
template <typename R> void launch_hist_carry(DevState& d, hipStream_t s, int check_lost);
template <typename R> void launch_mark_bonds(DevState& d, hipStream_t s);
void launch_set_xref(DevState& d, hipStream_t s);

// stepping
template <typename R> void launch_prologue(DevState& d, StepArgs a, hipStream_t s);
template <typename R> void launch_step(DevState& d, StepArgs a, hipStream_t s);
template <typename R> void launch_fluid(DevState& d, int buf, hipStream_t s);
void launch_closure_infer(DevState& d, hipStream_t s);
const short* mlp_weights_bf16(const dem_mlp* n);
const float* mlp_params_f32(const dem_mlp* n);
hipStream_t mlp_stream(const dem_mlp* n);

// read-back
template <typename R> void launch_unpermute(DevState& d, double* x, double* v, double* w, double* F,
                                            double* T, uint8_t* alive, double* fluid_force, hipStream_t s);
template <typename R> void launch_unpermute_walls(DevState& d, double* wall_dt, hipStream_t s);
int64_t aggregate_scratch_doubles(int nsamples);
int64_t cfd_work_doubles(int64_t ncell);
dem_status cfd_solve(DevState& d, const int8_t* kind, const double* pfix, double* work, int64_t nwork, int warm,
                     int max_iter, double rel_tol, double* P, double* U, double* GP, int* iters, double* rel_res,
                     double* h_scal, hipStream_t s);
void launch_aggregate_impl(DevState& d, const int64_t* soff, double* produced, double* kinetic,
                           long long* contacts, long long* nalive, double* partial, int fp64, hipStream_t s);

}  // namespace dem
