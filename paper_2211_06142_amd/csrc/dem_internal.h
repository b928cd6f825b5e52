// dem_internal.h -- device data layout and launch interfaces of the DEM library.
//
// Layout in HBM (all per-particle arrays are in the current sorted order:
// sample-major, then binning cell, then particle id; dead particles of a sample
// sit in one extra bucket at the end of that sample's range):
//   xr   double4  position (x, y, z) and radius
//   vel  double4  velocity (x, y, z) and 1/m
//   omg  R4       angular velocity and 1/I
//   frc  R4       force of the last evaluation
//   trq  R4       torque of the last evaluation
//   fdr  R4       fluid force held since the last coupling evaluation (drag + buoyancy)
//   R = double (FP64 mode) or float (mixed mode: forces, torques, spins and
//   tangential history in FP32; positions and velocities FP64).
// Half-pair list (owner = lower sorted index), CSR by owner:
//   pj[p]    int32  partner
//   hdt[p]   R4     tangential elongation, owner -> partner orientation
//   pfl[p]   uint8  bit0 bonded, bit1 touching at the last evaluation
//   recF[p], recC[p], recT[p]  R4  per-step force on the owner, n x F_t, rolling torque
// Wall entries (particle, wall) within the skin, CSR by particle, with history.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dem.h"

namespace dem {

constexpr int kMaxWalls = DEM_MAX_WALLS;

enum StatusBits : int {
  kStCapacity = 1,
  kStNonFinite = 2,
  kStTooFast = 4,
  kStLostBond = 8,
};

struct Wall {
  int kind;
  double p[6];
};

// Per-sample constants, derived on the host from dem_params (grain scale).
struct SampleConst {
  // contact law
  double Es, Gs, beta, cdamp;     // E*, G*, damping ratio, 2 sqrt(5/6) beta
  double gamma, mu, mu_roll, rho, k_lin;
  double jkrK;                    // X^3 / R* = pi^2 gamma^2 / E*^2
  double breakA;                  // ((3/16) pi^2) gamma^2
  double kcg, k3;                 // drag rule f = k^3 f(d / k)
  int normal_model;
  int fluid_on, voidfrac, u_superficial;
  double rho_f, mu_f, n_min;
  // fluid grid
  double glo[3], gh[3], vcell;
  int gn[3];
  int dn[3];                      // bucket grid used by the coupling sort
  int64_t cell_base, dual_base;
  // binning grid for the neighbour list
  double blo[3], bh[3];
  int bn[3];
  int64_t bin_base;               // first bin; the sample's dead bucket is bin_base + nbins
  double margin;                  // candidate margin: skin + largest pull-off separation
  double skin;
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

// ---------------------------------------------------------------------------
// launch interfaces (kernels in dem_kernels.hip)
// ---------------------------------------------------------------------------
struct DevState {
  int64_t n;
  int nsamples;
  double dt;
  int couple_every;
  int rolling;                     // any sample with mu_roll > 0
  // particle arrays (current order) and their permutation buffers
  double4 *xr, *vel, *xr2, *vel2;
  void *omg, *frc, *trq, *fdr, *omg2, *frc2, *trq2, *fdr2;  // R4
  double4* xref;                   // positions at the last rebuild (w unused)
  uint8_t *alive, *alive2;
  int32_t *sample, *sample2;       // sample index per particle
  int32_t *orig, *orig2;           // caller's index
  double *cdrag, *cdrag2, *ccoh, *ccoh2;  // closure factors (NULL when off)
  // sort scratch
  uint32_t* key;
  int32_t *bucket_cnt, *bucket_off, *bucket_fill, *order, *inv_order;
  int64_t nbins_total;             // including one dead bucket per sample
  int32_t* cell_start;             // nbins_total + 1
  // pairs
  int64_t pair_cap, npairs;
  int32_t *prow, *pcnt, *pj, *pown;
  void *hdt, *hdt2;                // R4
  uint8_t *pfl, *pfl2;
  int32_t *prow_old, *pj_old;
  void *recF, *recC, *recT;        // R4
  int32_t *rrow, *rcnt, *ridx;     // reverse CSR
  // wall entries
  int64_t wall_cap, nwall;
  int32_t *wrow, *wcnt, *wid, *wrow_old, *wid_old;
  void *wdt, *wdt2;                // R4
  uint8_t *wfl, *wfl2;
  // fluid
  int64_t ncell, ndual;
  int32_t* cell_sample;
  double *u_in, *gp_in;            // 3*ncell
  double *cell_n, *cell_u;         // ncell, 3*ncell
  double *eps, *fdc;               // ncell, 3*ncell (latest evaluation)
  int32_t* dkey;
  double4* dfr;                    // CIC fractions (fx, fy, fz, volume)
  double4* fpart;                  // particle drag of the latest evaluation
  int32_t *dcnt, *doff, *dfill, *dmem;
  // per-sample
  SampleConst* sc;
  unsigned long long* broken;      // per sample
  int* status;
  int* rebuild_flag;
  int* scratch_i;
  // scan scratch
  int32_t* scan_tmp;
  int64_t scan_tmp_n;
};

// scans and bucket sort
void scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s);

template <typename R> void launch_kick_drift(DevState& d, hipStream_t s);
template <typename R> void launch_gather_kick(DevState& d, hipStream_t s);
template <typename R> void launch_pair_force(DevState& d, hipStream_t s);
template <typename R> void launch_permute(DevState& d, hipStream_t s);
template <typename R> void launch_hist_merge(DevState& d, hipStream_t s, int check_lost);

void launch_bin_keys(DevState& d, hipStream_t s);
void launch_bucket_sort(const uint32_t* key, int64_t n, int64_t nb, const int32_t* tiebreak,
                        int32_t* cnt, int32_t* off, int32_t* fill, int32_t* out_order,
                        int32_t* scan_tmp, hipStream_t s);
void launch_pair_count(DevState& d, hipStream_t s);
void launch_pair_fill(DevState& d, hipStream_t s);
void launch_wall_count(DevState& d, hipStream_t s);
void launch_wall_fill(DevState& d, hipStream_t s);
void launch_reverse(DevState& d, hipStream_t s);
void launch_set_xref(DevState& d, hipStream_t s);
void launch_mark_bonds(DevState& d, hipStream_t s);
template <typename R> void launch_fluid(DevState& d, hipStream_t s);
template <typename R> void launch_unpermute(DevState& d, double* x, double* v, double* w, double* F,
                                            double* T, uint8_t* alive, hipStream_t s);
void launch_aggregate_impl(DevState& d, const int64_t* soff, double* produced, double* kinetic,
                           long long* contacts, long long* nalive, int fp64, hipStream_t s);
void launch_count_old_bonds(DevState& d, int64_t npairs_old, hipStream_t s);
void launch_check_lost(DevState& d, hipStream_t s);

}  // namespace dem
