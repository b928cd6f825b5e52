// dem_kernels.hip -- HIP kernels (gfx950) of the DEM + fluid-coupling step.
//
// One step (arXiv:2211.06142):
//   kick/drift ......... velocity Verlet on eq 1-2, outlet removal
//   [rebuild] .......... bin -> stable bucket sort by (cell, id) -> permute ->
//                        half-pair search (one wavefront per particle, ballot
//                        compaction) -> history merge -> reverse index
//   [coupling] ......... porosity per fluid cell by trilinear deposition, Di Felice
//                        drag (eq 8-11) per particle, drag source per cell (eq 7);
//                        every reduction is a gather over particles bucket-sorted by
//                        cell, in a fixed order (no floating-point atomics)
//   pair force ......... modified JKR / Hertz normal law (eq 12-13, Table 1, Fig. 2),
//                        damping eq 32-33, tangential spring + Coulomb (eq 4, 35),
//                        torque eq 5, rolling resistance
//   gather + kick ...... fixed-order sum of pair records, walls, gravity, fluid force,
//                        second half kick
// Compiled with -ffp-contract=off: the contact and bond predicates use only
// correctly rounded FP64 operations in a fixed order.
#include "dem_internal.h"

#include <math.h>

namespace dem {

constexpr int kBlock = 256;
static inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

template <typename R> __device__ inline R4<R> mk4(R a, R b, R c, R d) { R4<R> v; v.x = a; v.y = b; v.z = c; v.w = d; return v; }

// ---------------------------------------------------------------------------
// scan (exclusive, int32); in and out may alias
// ---------------------------------------------------------------------------
__global__ void k_scan_block(const int32_t* in, int32_t* out, int64_t n, int32_t* bsum) {
  __shared__ int32_t sh[256];
  const int64_t base = (int64_t)blockIdx.x * 1024;
  const int t = threadIdx.x;
  int32_t v[4];
  int32_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int64_t idx = base + t * 4 + k;
    v[k] = idx < n ? in[idx] : 0;
    s += v[k];
  }
  sh[t] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int32_t a = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  int32_t run = sh[t] - s;
  if (t == 255) bsum[blockIdx.x] = sh[255];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int64_t idx = base + t * 4 + k;
    if (idx < n) out[idx] = run;
    run += v[k];
  }
}

__global__ void k_scan_add(int32_t* out, int64_t n, const int32_t* bpre) {
  int64_t idx = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  int32_t add = bpre[blockIdx.x];
  for (int k = 0; k < 4; ++k, idx += 256)
    if (idx < n) out[idx] += add;
}

void scan_exclusive(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + 1023) / 1024;
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(256), 0, s, in, out, n, tmp);
  if (nb > 1) {
    scan_exclusive(tmp, tmp + nb, nb, tmp + 2 * nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, s, out, n, tmp + nb);
  }
}

// ---------------------------------------------------------------------------
// stable bucket sort: members of each bucket ordered by (tiebreak, index)
// ---------------------------------------------------------------------------
__global__ void k_bucket_count(const uint32_t* key, int64_t n, int32_t* cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[key[i]], 1);
}

__global__ void k_bucket_scatter(const uint32_t* key, int64_t n, const int32_t* off, int32_t* fill,
                                 int32_t* order) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t k = key[i];
  int32_t slot = atomicAdd(&fill[k], 1);
  order[off[k] + slot] = (int32_t)i;
}

// the scatter above places members in arbitrary order; restore a fixed one
__global__ void k_bucket_sortseg(const int32_t* off, int64_t nb, int32_t* order, const int32_t* tiebreak) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int32_t lo = off[b], hi = off[b + 1];
  for (int32_t a = lo + 1; a < hi; ++a) {
    int32_t v = order[a];
    int32_t kv = tiebreak ? tiebreak[v] : v;
    int32_t q = a - 1;
    while (q >= lo) {
      int32_t u = order[q];
      int32_t ku = tiebreak ? tiebreak[u] : u;
      if (ku < kv || (ku == kv && u < v)) break;
      order[q + 1] = u;
      --q;
    }
    order[q + 1] = v;
  }
}

void launch_bucket_sort(const uint32_t* key, int64_t n, int64_t nb, const int32_t* tiebreak,
                        int32_t* cnt, int32_t* off, int32_t* fill, int32_t* out_order,
                        int32_t* scan_tmp, hipStream_t s) {
  (void)hipMemsetAsync(cnt, 0, sizeof(int32_t) * (nb + 1), s);
  (void)hipMemsetAsync(fill, 0, sizeof(int32_t) * (nb + 1), s);
  if (n > 0) hipLaunchKernelGGL(k_bucket_count, dim3(nblk(n)), dim3(kBlock), 0, s, key, n, cnt);
  scan_exclusive(cnt, off, nb + 1, scan_tmp, s);
  if (n > 0) hipLaunchKernelGGL(k_bucket_scatter, dim3(nblk(n)), dim3(kBlock), 0, s, key, n, off, fill, out_order);
  hipLaunchKernelGGL(k_bucket_sortseg, dim3(nblk(nb)), dim3(kBlock), 0, s, off, nb, out_order, tiebreak);
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__device__ inline int bin_coord(double x, double lo, double h, int n) {
  double q = floor((x - lo) / h);
  if (q < 0.0) return 0;
  if (q > (double)(n - 1)) return n - 1;
  return (int)q;
}

__global__ void k_bin_keys(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const SampleConst& c = d.sc[d.sample[i]];
  int64_t nb = (int64_t)c.bn[0] * c.bn[1] * c.bn[2];
  if (!d.alive[i]) { d.key[i] = (uint32_t)(c.bin_base + nb); return; }
  double4 p = d.xr[i];
  int cx = bin_coord(p.x, c.blo[0], c.bh[0], c.bn[0]);
  int cy = bin_coord(p.y, c.blo[1], c.bh[1], c.bn[1]);
  int cz = bin_coord(p.z, c.blo[2], c.bh[2], c.bn[2]);
  d.key[i] = (uint32_t)(c.bin_base + ((int64_t)cz * c.bn[1] + cy) * c.bn[0] + cx);
}

void launch_bin_keys(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_keys, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}

// ---------------------------------------------------------------------------
// permutation of the particle arrays: new[k] = old[order[k]]
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_permute(DevState d) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  int32_t o = d.order[k];
  d.xr2[k] = d.xr[o];
  d.vel2[k] = d.vel[o];
  ((R4<R>*)d.omg2)[k] = ((const R4<R>*)d.omg)[o];
  ((R4<R>*)d.frc2)[k] = ((const R4<R>*)d.frc)[o];
  ((R4<R>*)d.trq2)[k] = ((const R4<R>*)d.trq)[o];
  ((R4<R>*)d.fdr2)[k] = ((const R4<R>*)d.fdr)[o];
  d.alive2[k] = d.alive[o];
  d.sample2[k] = d.sample[o];
  d.orig2[k] = d.orig[o];
  if (d.cdrag) { d.cdrag2[k] = d.cdrag[o]; d.ccoh2[k] = d.ccoh[o]; }
  d.inv_order[o] = (int32_t)k;
}

template <typename R> void launch_permute(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_permute<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}
template void launch_permute<double>(DevState&, hipStream_t);
template void launch_permute<float>(DevState&, hipStream_t);

__global__ void k_set_xref(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.n) d.xref[i] = d.xr[i];
}
void launch_set_xref(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_set_xref, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}

// ---------------------------------------------------------------------------
// half-pair search: one wavefront per particle i; candidates j > i in the own
// cell and the 13 forward neighbour cells, tested 64 at a time and compacted
// with a ballot + prefix popcount.  Rows come out sorted by j.
// ---------------------------------------------------------------------------
__constant__ int c_fwd[13][3] = {{1, 0, 0},  {-1, 1, 0}, {0, 1, 0},   {1, 1, 0},  {-1, -1, 1},
                                 {0, -1, 1}, {1, -1, 1}, {-1, 0, 1},  {0, 0, 1},  {1, 0, 1},
                                 {-1, 1, 1}, {0, 1, 1},  {1, 1, 1}};

template <bool kFill>
__global__ __launch_bounds__(256) void k_pair_search(DevState d) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= d.n) return;
  if (!d.alive[i]) {
    if (!kFill && lane == 0) d.pcnt[i] = 0;
    return;
  }
  const SampleConst& c = d.sc[d.sample[i]];
  const double4 pi = d.xr[i];
  const int cx = bin_coord(pi.x, c.blo[0], c.bh[0], c.bn[0]);
  const int cy = bin_coord(pi.y, c.blo[1], c.bh[1], c.bn[1]);
  const int cz = bin_coord(pi.z, c.blo[2], c.bh[2], c.bn[2]);
  const int64_t own = c.bin_base + ((int64_t)cz * c.bn[1] + cy) * c.bn[0] + cx;
  int rs[14], rl[14];
  rs[0] = (int)i + 1;
  rl[0] = d.cell_start[own + 1] - rs[0];
  int total = rl[0];
#pragma unroll
  for (int k = 0; k < 13; ++k) {
    int qx = cx + c_fwd[k][0], qy = cy + c_fwd[k][1], qz = cz + c_fwd[k][2];
    rs[k + 1] = 0;
    rl[k + 1] = 0;
    if (qx >= 0 && qy >= 0 && qz >= 0 && qx < c.bn[0] && qy < c.bn[1] && qz < c.bn[2]) {
      int64_t q = c.bin_base + ((int64_t)qz * c.bn[1] + qy) * c.bn[0] + qx;
      rs[k + 1] = d.cell_start[q];
      rl[k + 1] = d.cell_start[q + 1] - rs[k + 1];
    }
    total += rl[k + 1];
  }
  const int row = kFill ? d.prow[i] : 0;
  int written = 0;
  const double margin = c.margin;
  for (int base = 0; base < total; base += 64) {
    int t = base + lane;
    bool pred = false;
    int j = -1;
    if (t < total) {
      int acc = 0;
#pragma unroll
      for (int k = 0; k < 14; ++k) {
        if (j < 0 && t < acc + rl[k]) j = rs[k] + (t - acc);
        acc += rl[k];
      }
      if (j >= 0 && d.alive[j]) {
        double4 pj = d.xr[j];
        double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
        double d2 = (dx * dx + dy * dy) + dz * dz;
        double cc = (pi.w + pj.w) + margin;
        pred = d2 < cc * cc;
      }
    }
    unsigned long long mask = __ballot(pred);
    if (kFill && pred) {
      int pre = __popcll(mask & ((1ull << lane) - 1ull));
      d.pj[row + written + pre] = j;
      d.pown[row + written + pre] = (int32_t)i;
    }
    written += __popcll(mask);
  }
  if (!kFill && lane == 0) d.pcnt[i] = written;
}

void launch_pair_count(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_search<false>, dim3(nblk(d.n, 4)), dim3(256), 0, s, d);
}
void launch_pair_fill(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_search<true>, dim3(nblk(d.n, 4)), dim3(256), 0, s, d);
}

// ---------------------------------------------------------------------------
// walls
// ---------------------------------------------------------------------------
// signed distance from the wall surface (positive on the particle side) and
// the unit normal pointing into the particle side
__device__ inline bool wall_geom(const Wall& w, double x, double y, double z, double& sd, double nw[3]) {
  if (w.kind == DEM_WALL_PLANE) {
    nw[0] = w.p[0]; nw[1] = w.p[1]; nw[2] = w.p[2];
    sd = ((nw[0] * x + nw[1] * y) + nw[2] * z) - w.p[3];
    return true;
  }
  double ex = x - w.p[0], ey = y - w.p[1];
  double rho = sqrt(ex * ex + ey * ey);
  if (rho == 0.0) return false;
  if (w.kind == DEM_WALL_CYL_IN) {
    sd = w.p[2] - rho;
    nw[0] = -ex / rho; nw[1] = -ey / rho; nw[2] = 0.0;
  } else {
    sd = rho - w.p[2];
    nw[0] = ex / rho; nw[1] = ey / rho; nw[2] = 0.0;
  }
  return true;
}

template <bool kFill>
__global__ void k_wall_search(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  int cnt = 0;
  if (d.alive[i]) {
    const SampleConst& c = d.sc[d.sample[i]];
    double4 p = d.xr[i];
    int row = kFill ? d.wrow[i] : 0;
    for (int w = 0; w < c.n_walls; ++w) {
      double sd, nw[3];
      if (wall_geom(c.walls[w], p.x, p.y, p.z, sd, nw) && sd < p.w + c.skin) {
        if (kFill) d.wid[row + cnt] = w;
        ++cnt;
      }
    }
  }
  if (!kFill) d.wcnt[i] = cnt;
}

void launch_wall_count(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_wall_search<false>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}
void launch_wall_fill(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_wall_search<true>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}

// ---------------------------------------------------------------------------
// history merge: carry (elongation, flags) of every pair and wall entry that
// existed in the previous list (found through the permutation)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_hist_merge(DevState d, int check_lost) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < d.npairs) {
    int32_t i = d.pown[p], j = d.pj[p];
    int32_t oi = d.order[i], oj = d.order[j];
    int32_t o = oi < oj ? oi : oj, q = oi < oj ? oj : oi;
    int32_t lo = d.prow_old[o], hi = d.prow_old[o + 1];
    R4<R> h = mk4<R>(0, 0, 0, 0);
    uint8_t fl = 0;
    while (lo < hi) {                         // rows are sorted by partner
      int32_t mid = (lo + hi) >> 1;
      if (d.pj_old[mid] < q) lo = mid + 1; else hi = mid;
    }
    if (lo < d.prow_old[o + 1] && d.pj_old[lo] == q) {
      h = ((const R4<R>*)d.hdt2)[lo];
      fl = d.pfl2[lo];
      if (oi > oj) { h.x = -h.x; h.y = -h.y; h.z = -h.z; }
      if (check_lost && (fl & 1)) atomicAdd(&d.scratch_i[1], 1);
    }
    ((R4<R>*)d.hdt)[p] = h;
    d.pfl[p] = fl;
  }
  int64_t e = p;
  if (e < d.nwall) {
    int32_t i = 0;
    // owner of wall entry e: binary search in wrow
    int32_t lo = 0, hi = (int32_t)d.n;
    while (lo < hi) {
      int32_t mid = (lo + hi) >> 1;
      if (d.wrow[mid + 1] <= e) lo = mid + 1; else hi = mid;
    }
    i = lo;
    int32_t w = d.wid[e];
    int32_t oi = d.order[i];
    R4<R> h = mk4<R>(0, 0, 0, 0);
    uint8_t fl = 0;
    for (int32_t q = d.wrow_old[oi]; q < d.wrow_old[oi + 1]; ++q)
      if (d.wid_old[q] == w) { h = ((const R4<R>*)d.wdt2)[q]; fl = d.wfl2[q]; }
    ((R4<R>*)d.wdt)[e] = h;
    d.wfl[e] = fl;
  }
}

// bonded pairs of the previous list whose partners are both alive
__global__ void k_count_old_bonds(DevState d, int64_t npairs_old) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs_old) return;
  if (!(d.pfl2[p] & 1)) return;
  // owner of old pair p (old order): binary search in prow_old
  int32_t lo = 0, hi = (int32_t)d.n;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (d.prow_old[mid + 1] <= p) lo = mid + 1; else hi = mid;
  }
  int32_t o = lo, q = d.pj_old[p];
  if (d.alive[d.inv_order[o]] && d.alive[d.inv_order[q]]) atomicAdd(&d.scratch_i[0], 1);
}

__global__ void k_check_lost(DevState d) {
  if (d.scratch_i[0] != d.scratch_i[1]) atomicOr(d.status, (int)kStLostBond);
}

template <typename R> void launch_hist_merge(DevState& d, hipStream_t s, int check_lost) {
  int64_t m = d.npairs > d.nwall ? d.npairs : d.nwall;
  if (m > 0) hipLaunchKernelGGL(k_hist_merge<R>, dim3(nblk(m)), dim3(kBlock), 0, s, d, check_lost);
}
template void launch_hist_merge<double>(DevState&, hipStream_t, int);
template void launch_hist_merge<float>(DevState&, hipStream_t, int);

void launch_count_old_bonds(DevState& d, int64_t npairs_old, hipStream_t s) {
  (void)hipMemsetAsync(d.scratch_i, 0, 2 * sizeof(int), s);
  if (npairs_old > 0)
    hipLaunchKernelGGL(k_count_old_bonds, dim3(nblk(npairs_old)), dim3(kBlock), 0, s, d, npairs_old);
}
void launch_check_lost(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_check_lost, dim3(1), dim3(1), 0, s, d);
}

// bond every touching pair (initial state of the modified JKR model)
__global__ void k_mark_bonds(DevState d) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.npairs) return;
  int32_t i = d.pown[p], j = d.pj[p];
  const SampleConst& c = d.sc[d.sample[i]];
  if (c.normal_model != DEM_NORMAL_JKR_MOD) return;
  double4 a = d.xr[i], b = d.xr[j];
  double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double cs = a.w + b.w;
  if (d2 < cs * cs) d.pfl[p] = 1;
}
void launch_mark_bonds(DevState& d, hipStream_t s) {
  if (d.npairs > 0) hipLaunchKernelGGL(k_mark_bonds, dim3(nblk(d.npairs)), dim3(kBlock), 0, s, d);
}

// ---------------------------------------------------------------------------
// reverse index: for every particle, the half pairs in which it is the partner
// ---------------------------------------------------------------------------
__global__ void k_rev_count(DevState d) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < d.npairs) atomicAdd(&d.rcnt[d.pj[p]], 1);
}
__global__ void k_rev_fill(DevState d, int32_t* fill) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.npairs) return;
  int32_t j = d.pj[p];
  int32_t slot = atomicAdd(&fill[j], 1);
  d.ridx[d.rrow[j] + slot] = (int32_t)p;
}
__global__ void k_rev_sort(DevState d) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  int32_t lo = d.rrow[k], hi = d.rrow[k + 1];
  for (int32_t a = lo + 1; a < hi; ++a) {
    int32_t v = d.ridx[a];
    int32_t q = a - 1;
    while (q >= lo && d.ridx[q] > v) { d.ridx[q + 1] = d.ridx[q]; --q; }
    d.ridx[q + 1] = v;
  }
}

void launch_reverse(DevState& d, hipStream_t s) {
  (void)hipMemsetAsync(d.rcnt, 0, sizeof(int32_t) * (d.n + 1), s);
  if (d.npairs > 0) hipLaunchKernelGGL(k_rev_count, dim3(nblk(d.npairs)), dim3(kBlock), 0, s, d);
  scan_exclusive(d.rcnt, d.rrow, d.n + 1, d.scan_tmp, s);
  (void)hipMemsetAsync(d.bucket_fill, 0, sizeof(int32_t) * (d.n + 1), s);
  if (d.npairs > 0) hipLaunchKernelGGL(k_rev_fill, dim3(nblk(d.npairs)), dim3(kBlock), 0, s, d, d.bucket_fill);
  hipLaunchKernelGGL(k_rev_sort, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}

// ---------------------------------------------------------------------------
// first half kick and drift (eq 1-2), outlet removal, rebuild trigger
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_kick_drift(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  if (!d.alive[i]) return;
  const SampleConst& c = d.sc[d.sample[i]];
  const double dt = d.dt;
  double4 p = d.xr[i];
  double4 v = d.vel[i];
  R4<R> w = ((const R4<R>*)d.omg)[i];
  R4<R> F = ((const R4<R>*)d.frc)[i];
  R4<R> T = ((const R4<R>*)d.trq)[i];
  const double hdt = 0.5 * dt;
  v.x += hdt * (double)F.x * v.w;
  v.y += hdt * (double)F.y * v.w;
  v.z += hdt * (double)F.z * v.w;
  const R hdtR = (R)hdt;
  w.x += hdtR * T.x * w.w;
  w.y += hdtR * T.y * w.w;
  w.z += hdtR * T.z * w.w;
  double sx = dt * v.x, sy = dt * v.y, sz = dt * v.z;
  p.x += sx; p.y += sy; p.z += sz;
  const double hs = 0.5 * c.skin;
  if ((sx * sx + sy * sy) + sz * sz >= hs * hs) atomicOr(d.status, (int)kStTooFast);
  d.xr[i] = p;
  d.vel[i] = v;
  ((R4<R>*)d.omg)[i] = w;
  if (c.outlet_kind == DEM_OUTLET_CAVITY) {
    double ex = p.x - c.outlet[0], ey = p.y - c.outlet[1];
    double rc = c.outlet[2];
    if (ex * ex + ey * ey < rc * rc) {
      d.alive[i] = 0;
      ((R4<R>*)d.frc)[i] = mk4<R>(0, 0, 0, 0);
      ((R4<R>*)d.trq)[i] = mk4<R>(0, 0, 0, 0);
      return;
    }
  }
  double4 q = d.xref[i];
  double ux = p.x - q.x, uy = p.y - q.y, uz = p.z - q.z;
  if ((ux * ux + uy * uy) + uz * uz > hs * hs) atomicOr(d.rebuild_flag, 1);
}

template <typename R> void launch_kick_drift(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}
template void launch_kick_drift<double>(DevState&, hipStream_t);
template void launch_kick_drift<float>(DevState&, hipStream_t);

// ---------------------------------------------------------------------------
// the contact law (shared by particle pairs and walls)
// ---------------------------------------------------------------------------
template <typename R> __device__ inline R rcbrt_(R x);
template <> __device__ inline double rcbrt_<double>(double x) { return cbrt(x); }
template <> __device__ inline float rcbrt_<float>(float x) { return cbrtf(x); }
template <typename R> __device__ inline R rsqrt_(R x);
template <> __device__ inline double rsqrt_<double>(double x) { return sqrt(x); }
template <> __device__ inline float rsqrt_<float>(float x) { return sqrtf(x); }

// Contact radius and elastic force of a bonded JKR contact (eq 12-13).  With
// X^3 = pi^2 gamma^2 R* / E*^2, a0 = sqrt(X R*), delta = X D, a = a0 b^2,
// eq 13 becomes b^4 - 2 b = D and eq 12 F = pi gamma R* (4/3 b^6 - 4 b^3).
// The branch through point C (b_C^3 = 3/2) is taken: two fixed-point steps
// of b = (D + 2b)^(1/4) from b_C, then Newton on the convex, increasing
// quartic.
template <typename R>
__device__ inline void jkr_bonded(R delta, R Rs, R gam, R jkrK, R& a, R& Fel, R& scale) {
  constexpr R kPi = (R)3.14159265358979323846;
  constexpr R kbC = (R)1.1447142425533319;   // (3/2)^(1/3)
  constexpr int kNewton = sizeof(R) == 8 ? 3 : 2;
  R X = rcbrt_<R>(jkrK * Rs);
  R D = delta / X;
  R b = rsqrt_<R>(rsqrt_<R>(D + (R)2 * kbC));
  b = rsqrt_<R>(rsqrt_<R>(D + (R)2 * b));
#pragma unroll
  for (int it = 0; it < kNewton; ++it) {
    R b3 = b * b * b;
    R f = b3 * b - (R)2 * b - D;
    R fp = (R)4 * b3 - (R)2;
    b -= f / fp;
  }
  R b3 = b * b * b;
  R u = kPi * gam * Rs;
  R t1 = u * ((R)4 / (R)3) * b3 * b3;
  R t2 = u * (R)4 * b3;
  Fel = t1 - t2;
  scale = t1 + t2;
  a = rsqrt_<R>(X * Rs) * b * b;
}

template <typename R> struct LawOut {
  R F[3], c[3], Tr[3];
};

// n: unit normal from the body to its partner; vrel: contact-point velocity of
// the body relative to the partner; wrel: relative angular velocity.
template <typename R>
__device__ inline void contact_law(const SampleConst& c, int bonded, R delta, R Rs, R ms, R gam, R jkrK,
                                   const R n[3], const R vrel[3], const R wrel[3], R hdt[3], R dt,
                                   bool rolling, LawOut<R>& o) {
  R a, Fel, kn, kt, etan, etat, L, sc;
  if (c.normal_model == DEM_NORMAL_LINEAR) {
    kn = (R)c.k_lin;
    Fel = kn * delta;
    kt = ((R)2 / (R)7) * kn;
    etan = (R)2 * (R)c.beta * rsqrt_<R>(kn * ms);
    etat = (R)2 * (R)c.beta * rsqrt_<R>(kt * ms);
    L = (R)c.mu * Fel;
  } else {
    if (bonded && gam > (R)0) {
      jkr_bonded<R>(delta, Rs, gam, jkrK, a, Fel, sc);
      L = (R)c.mu * (Fel + (R)2 * ((R)3 * (R)3.14159265358979323846 * gam * Rs));
    } else {
      a = rsqrt_<R>(Rs * (delta > (R)0 ? delta : (R)0));
      Fel = (R)4 * (R)c.Es * a * a * a / ((R)3 * Rs);
      L = (R)c.mu * Fel;
    }
    kn = (R)2 * (R)c.Es * a;
    kt = (R)8 * (R)c.Gs * a;
    etan = (R)c.cdamp * rsqrt_<R>(kn * ms);
    etat = (R)c.cdamp * rsqrt_<R>(kt * ms);
  }
  R vn = (vrel[0] * n[0] + vrel[1] * n[1]) + vrel[2] * n[2];
  R vt[3] = {vrel[0] - vn * n[0], vrel[1] - vn * n[1], vrel[2] - vn * n[2]};
  R Fn = Fel + etan * vn;
  // rotate the stored elongation into the tangent plane, keep its length
  R old = rsqrt_<R>((hdt[0] * hdt[0] + hdt[1] * hdt[1]) + hdt[2] * hdt[2]);
  R dn = (hdt[0] * n[0] + hdt[1] * n[1]) + hdt[2] * n[2];
  R tp[3] = {hdt[0] - dn * n[0], hdt[1] - dn * n[1], hdt[2] - dn * n[2]};
  R tpl = rsqrt_<R>((tp[0] * tp[0] + tp[1] * tp[1]) + tp[2] * tp[2]);
  if (tpl > (R)0) {
    R f = old / tpl;
    hdt[0] = tp[0] * f; hdt[1] = tp[1] * f; hdt[2] = tp[2] * f;
  } else {
    hdt[0] = hdt[1] = hdt[2] = (R)0;
  }
  hdt[0] += vt[0] * dt; hdt[1] += vt[1] * dt; hdt[2] += vt[2] * dt;
  R Ft[3] = {-kt * hdt[0] - etat * vt[0], -kt * hdt[1] - etat * vt[1], -kt * hdt[2] - etat * vt[2]};
  R ftm = rsqrt_<R>((Ft[0] * Ft[0] + Ft[1] * Ft[1]) + Ft[2] * Ft[2]);
  if (ftm > L) {
    R s = L / ftm;
    Ft[0] *= s; Ft[1] *= s; Ft[2] *= s;
    if (kt > (R)0) {
      hdt[0] = -(Ft[0] + etat * vt[0]) / kt;
      hdt[1] = -(Ft[1] + etat * vt[1]) / kt;
      hdt[2] = -(Ft[2] + etat * vt[2]) / kt;
    } else {
      hdt[0] = hdt[1] = hdt[2] = (R)0;
    }
  }
  o.F[0] = -Fn * n[0] + Ft[0];
  o.F[1] = -Fn * n[1] + Ft[1];
  o.F[2] = -Fn * n[2] + Ft[2];
  o.c[0] = n[1] * Ft[2] - n[2] * Ft[1];
  o.c[1] = n[2] * Ft[0] - n[0] * Ft[2];
  o.c[2] = n[0] * Ft[1] - n[1] * Ft[0];
  o.Tr[0] = o.Tr[1] = o.Tr[2] = (R)0;
  if (rolling && c.mu_roll > 0.0) {
    R wn = (wrel[0] * n[0] + wrel[1] * n[1]) + wrel[2] * n[2];
    R wr[3] = {wrel[0] - wn * n[0], wrel[1] - wn * n[1], wrel[2] - wn * n[2]};
    R wm = rsqrt_<R>((wr[0] * wr[0] + wr[1] * wr[1]) + wr[2] * wr[2]);
    if (wm > (R)0) {
      R tm = (R)c.mu_roll * Rs * (Fel < (R)0 ? -Fel : Fel) / wm;
      o.Tr[0] = -tm * wr[0]; o.Tr[1] = -tm * wr[1]; o.Tr[2] = -tm * wr[2];
    }
  }
}

// ---------------------------------------------------------------------------
// pair forces: one thread per half pair
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_pair_force(DevState d) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.npairs) return;
  R4<R>* recF = (R4<R>*)d.recF;
  R4<R>* recC = (R4<R>*)d.recC;
  R4<R>* recT = (R4<R>*)d.recT;
  R4<R>* hdtp = (R4<R>*)d.hdt;
  const R4<R> z4 = mk4<R>(0, 0, 0, 0);
  const int32_t i = d.pown[p], j = d.pj[p];
  uint8_t fl = d.pfl[p];
  auto clear = [&]() {
    recF[p] = z4;
    recC[p] = z4;
    if (d.rolling) recT[p] = z4;
    hdtp[p] = z4;
    d.pfl[p] = 0;
  };
  if (!d.alive[i] || !d.alive[j]) { clear(); return; }
  const int s = d.sample[i];
  const SampleConst& c = d.sc[s];
  const double4 a = d.xr[i], b = d.xr[j];
  const double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double cs = a.w + b.w;
  const double Rsd = a.w * b.w / (a.w + b.w);
  double gam = c.gamma;
  if (d.ccoh) gam = c.gamma * sqrt(d.ccoh[i] * d.ccoh[j]);
  const bool touching = d2 < cs * cs;
  int bonded = fl & 1;
  if (bonded && !touching) {
    // bond persists down to the pull-off overlap of point C (Table 1), tested with cubes
    double sep = sqrt(d2) - cs;
    double lhs = (sep * sep) * sep;
    double rhs = ((3.0 / 16.0) * (M_PI * M_PI)) * (gam * gam) * Rsd / (c.Es * c.Es);
    if (!(lhs <= rhs)) {
      atomicAdd(&d.broken[s], 1ull);
      clear();
      return;
    }
  }
  if (!bonded && !touching) { clear(); return; }
  const double dist = sqrt(d2);
  const R delta = (R)(cs - dist);
  const R n[3] = {(R)(dx / dist), (R)(dy / dist), (R)(dz / dist)};
  const double4 va = d.vel[i], vb = d.vel[j];
  const R4<R> wa = ((const R4<R>*)d.omg)[i], wb = ((const R4<R>*)d.omg)[j];
  const R ra = (R)a.w, rb = (R)b.w;
  const R ws[3] = {ra * wa.x + rb * wb.x, ra * wa.y + rb * wb.y, ra * wa.z + rb * wb.z};
  const R vrel[3] = {(R)(va.x - vb.x) + (ws[1] * n[2] - ws[2] * n[1]),
                     (R)(va.y - vb.y) + (ws[2] * n[0] - ws[0] * n[2]),
                     (R)(va.z - vb.z) + (ws[0] * n[1] - ws[1] * n[0])};
  const R wrel[3] = {wa.x - wb.x, wa.y - wb.y, wa.z - wb.z};
  const R ms = (R)(1.0 / (va.w + vb.w));
  R4<R> h4 = hdtp[p];
  R h[3] = {h4.x, h4.y, h4.z};
  const R gR = (R)gam;
  const R jkrK = (R)((M_PI * M_PI) * (gam * gam) / (c.Es * c.Es));
  LawOut<R> o;
  contact_law<R>(c, bonded, delta, (R)Rsd, ms, gR, jkrK, n, vrel, wrel, h, (R)d.dt, d.rolling != 0, o);
  recF[p] = mk4<R>(o.F[0], o.F[1], o.F[2], (R)0);
  recC[p] = mk4<R>(o.c[0], o.c[1], o.c[2], (R)0);
  if (d.rolling) recT[p] = mk4<R>(o.Tr[0], o.Tr[1], o.Tr[2], (R)0);
  hdtp[p] = mk4<R>(h[0], h[1], h[2], (R)0);
  d.pfl[p] = (uint8_t)(bonded | (touching ? 2 : 0));
}

template <typename R> void launch_pair_force(DevState& d, hipStream_t s) {
  if (d.npairs > 0) hipLaunchKernelGGL(k_pair_force<R>, dim3(nblk(d.npairs)), dim3(kBlock), 0, s, d);
}
template void launch_pair_force<double>(DevState&, hipStream_t);
template void launch_pair_force<float>(DevState&, hipStream_t);

// ---------------------------------------------------------------------------
// gather: fixed-order sum per particle, walls, body forces, second half kick
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_gather_kick(DevState d) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  if (!d.alive[k]) return;
  const SampleConst& c = d.sc[d.sample[k]];
  const R4<R>* recF = (const R4<R>*)d.recF;
  const R4<R>* recC = (const R4<R>*)d.recC;
  const R4<R>* recT = (const R4<R>*)d.recT;
  const double4 p = d.xr[k];
  double4 v = d.vel[k];
  R4<R> w = ((const R4<R>*)d.omg)[k];
  const R r = (R)p.w;
  R F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  for (int32_t q = d.prow[k]; q < d.prow[k + 1]; ++q) {
    R4<R> f = recF[q], cc = recC[q];
    F[0] += f.x; F[1] += f.y; F[2] += f.z;
    T[0] += r * cc.x; T[1] += r * cc.y; T[2] += r * cc.z;
    if (d.rolling) { R4<R> t = recT[q]; T[0] += t.x; T[1] += t.y; T[2] += t.z; }
  }
  for (int32_t q = d.rrow[k]; q < d.rrow[k + 1]; ++q) {
    int32_t e = d.ridx[q];
    R4<R> f = recF[e], cc = recC[e];
    F[0] -= f.x; F[1] -= f.y; F[2] -= f.z;
    T[0] += r * cc.x; T[1] += r * cc.y; T[2] += r * cc.z;
    if (d.rolling) { R4<R> t = recT[e]; T[0] -= t.x; T[1] -= t.y; T[2] -= t.z; }
  }
  // walls: Hertz with R* = r and m* = m (the wall is rigid and static)
  const double m = c.rho * (4.0 / 3.0) * M_PI * p.w * p.w * p.w;
  for (int32_t e = d.wrow[k]; e < d.wrow[k + 1]; ++e) {
    R4<R> h4 = ((const R4<R>*)d.wdt)[e];
    double sd, nw[3];
    const Wall& wl = c.walls[d.wid[e]];
    if (!wall_geom(wl, p.x, p.y, p.z, sd, nw) || !(sd < p.w)) {
      ((R4<R>*)d.wdt)[e] = mk4<R>(0, 0, 0, 0);
      d.wfl[e] = 0;
      continue;
    }
    const R delta = (R)(p.w - sd);
    const R n[3] = {(R)(-nw[0]), (R)(-nw[1]), (R)(-nw[2])};
    const R wr[3] = {r * w.x, r * w.y, r * w.z};
    const R vrel[3] = {(R)v.x + (wr[1] * n[2] - wr[2] * n[1]), (R)v.y + (wr[2] * n[0] - wr[0] * n[2]),
                       (R)v.z + (wr[0] * n[1] - wr[1] * n[0])};
    const R wrel[3] = {w.x, w.y, w.z};
    R h[3] = {h4.x, h4.y, h4.z};
    LawOut<R> o;
    contact_law<R>(c, 0, delta, r, (R)m, (R)0, (R)0, n, vrel, wrel, h, (R)d.dt, true, o);
    F[0] += o.F[0]; F[1] += o.F[1]; F[2] += o.F[2];
    T[0] += r * o.c[0] + o.Tr[0];
    T[1] += r * o.c[1] + o.Tr[1];
    T[2] += r * o.c[2] + o.Tr[2];
    ((R4<R>*)d.wdt)[e] = mk4<R>(h[0], h[1], h[2], (R)0);
    d.wfl[e] = 2;
  }
  F[0] += (R)(m * c.g[0]);
  F[1] += (R)(m * c.g[1]);
  F[2] += (R)(m * c.g[2]);
  if (c.fluid_on) {
    R4<R> fd = ((const R4<R>*)d.fdr)[k];
    F[0] += fd.x; F[1] += fd.y; F[2] += fd.z;
  }
  const double hdt = 0.5 * d.dt;
  v.x += hdt * (double)F[0] * v.w;
  v.y += hdt * (double)F[1] * v.w;
  v.z += hdt * (double)F[2] * v.w;
  const R hdtR = (R)hdt;
  w.x += hdtR * T[0] * w.w;
  w.y += hdtR * T[1] * w.w;
  w.z += hdtR * T[2] * w.w;
  d.vel[k] = v;
  ((R4<R>*)d.omg)[k] = w;
  ((R4<R>*)d.frc)[k] = mk4<R>(F[0], F[1], F[2], (R)0);
  ((R4<R>*)d.trq)[k] = mk4<R>(T[0], T[1], T[2], (R)0);
  if (!isfinite(F[0] + F[1] + F[2] + T[0] + T[1] + T[2])) atomicOr(d.status, (int)kStNonFinite);
}

template <typename R> void launch_gather_kick(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_kick<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}
template void launch_gather_kick<double>(DevState&, hipStream_t);
template void launch_gather_kick<float>(DevState&, hipStream_t);

// ---------------------------------------------------------------------------
// fluid coupling (section 2.2)
// ---------------------------------------------------------------------------
// Bucket of a particle: the cell of the grid of cell centres ("dual cell") that
// holds it after projection onto the hull of the centres (trilinear), or its
// own cell (centroid).  Fractions f are the trilinear weights of the upper
// neighbour in each direction.
__global__ void k_fluid_key(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const SampleConst& c = d.sc[d.sample[i]];
  int64_t nd = (int64_t)c.dn[0] * c.dn[1] * c.dn[2];
  if (!d.alive[i] || !c.fluid_on) { d.dkey[i] = (int32_t)(c.dual_base + nd); return; }
  const double4 p = d.xr[i];
  const double xs[3] = {p.x, p.y, p.z};
  int b[3];
  double f[3];
  for (int k = 0; k < 3; ++k) {
    if (c.voidfrac == DEM_VOID_CENTROID) {
      double q = floor((xs[k] - c.glo[k]) / c.gh[k]);
      if (q < 0.0) q = 0.0;
      if (q > (double)(c.gn[k] - 1)) q = (double)(c.gn[k] - 1);
      b[k] = (int)q;
      f[k] = 0.0;
    } else {
      double t = (xs[k] - c.glo[k]) / c.gh[k] - 0.5;
      double tmax = (double)(c.gn[k] - 1);
      if (t < 0.0) t = 0.0;
      if (t > tmax) t = tmax;
      int bb = (int)floor(t);
      if (c.gn[k] >= 2 && bb > c.gn[k] - 2) bb = c.gn[k] - 2;
      if (c.gn[k] == 1) bb = 0;
      b[k] = bb;
      f[k] = t - (double)bb;
    }
  }
  d.dkey[i] = (int32_t)(c.dual_base + ((int64_t)b[2] * c.dn[1] + b[1]) * c.dn[0] + b[0]);
  const double V = (4.0 / 3.0) * M_PI * p.w * p.w * p.w;
  d.dfr[i] = make_double4(f[0], f[1], f[2], V);
}

// weight of the particle with fractions f in bucket D for cell index cc (one direction)
__device__ inline double cic_w(int cc, int D, double f, int n, int centroid) {
  if (centroid || n == 1) return 1.0;
  return cc == D ? 1.0 - f : f;
}

// porosity of every fluid cell: fixed-order gather over the buckets touching it
__global__ void k_fluid_eps(DevState d) {
  int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= d.ncell) return;
  const SampleConst& c = d.sc[d.cell_sample[C]];
  int64_t l = C - c.cell_base;
  int cx = (int)(l % c.gn[0]), cy = (int)((l / c.gn[0]) % c.gn[1]), cz = (int)(l / ((int64_t)c.gn[0] * c.gn[1]));
  const int cen = c.voidfrac == DEM_VOID_CENTROID;
  int lo[3], hi[3];
  const int cc[3] = {cx, cy, cz};
  for (int k = 0; k < 3; ++k) {
    if (cen) { lo[k] = hi[k] = cc[k]; }
    else if (c.gn[k] == 1) { lo[k] = hi[k] = 0; }
    else { lo[k] = cc[k] - 1 < 0 ? 0 : cc[k] - 1; hi[k] = cc[k] > c.gn[k] - 2 ? c.gn[k] - 2 : cc[k]; }
  }
  double s = 0.0;
  for (int Dz = lo[2]; Dz <= hi[2]; ++Dz)
    for (int Dy = lo[1]; Dy <= hi[1]; ++Dy)
      for (int Dx = lo[0]; Dx <= hi[0]; ++Dx) {
        int64_t key = c.dual_base + ((int64_t)Dz * c.dn[1] + Dy) * c.dn[0] + Dx;
        for (int32_t q = d.doff[key]; q < d.doff[key + 1]; ++q) {
          int32_t i = d.dmem[q];
          double4 fr = d.dfr[i];
          double w = (cic_w(cx, Dx, fr.x, c.gn[0], cen) * cic_w(cy, Dy, fr.y, c.gn[1], cen)) *
                     cic_w(cz, Dz, fr.z, c.gn[2], cen);
          s += w * fr.w;
        }
      }
  double eps = s / c.vcell;
  d.eps[C] = eps;
  double nn = 1.0 - eps;
  if (nn < c.n_min) nn = c.n_min;
  if (nn > 1.0) nn = 1.0;
  d.cell_n[C] = nn;
  for (int k = 0; k < 3; ++k) d.cell_u[3 * C + k] = c.u_superficial ? d.u_in[3 * C + k] / nn : d.u_in[3 * C + k];
}

// Di Felice drag (eq 8-11) with the coarse-grained rule, buoyancy and the
// dynamic pressure gradient; trilinear interpolation of n, u, grad p
template <typename R>
__global__ void k_fluid_drag(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const SampleConst& c = d.sc[d.sample[i]];
  if (!d.alive[i] || !c.fluid_on) {
    ((R4<R>*)d.fdr)[i] = mk4<R>(0, 0, 0, 0);
    d.fpart[i] = make_double4(0, 0, 0, 0);
    return;
  }
  const int cen = c.voidfrac == DEM_VOID_CENTROID;
  int64_t l = d.dkey[i] - c.dual_base;
  int b[3] = {(int)(l % c.dn[0]), (int)((l / c.dn[0]) % c.dn[1]), (int)(l / ((int64_t)c.dn[0] * c.dn[1]))};
  double4 fr = d.dfr[i];
  double f[3] = {fr.x, fr.y, fr.z};
  double np = 0.0, u[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
  int up = cen ? 1 : 2;
  for (int dz = 0; dz < up; ++dz)
    for (int dy = 0; dy < up; ++dy)
      for (int dx = 0; dx < up; ++dx) {
        int kx = b[0] + dx, ky = b[1] + dy, kz = b[2] + dz;
        if (kx >= c.gn[0] || ky >= c.gn[1] || kz >= c.gn[2]) continue;
        double wx = cen ? 1.0 : (dx ? f[0] : 1.0 - f[0]);
        double wy = cen ? 1.0 : (dy ? f[1] : 1.0 - f[1]);
        double wz = cen ? 1.0 : (dz ? f[2] : 1.0 - f[2]);
        double w = (wx * wy) * wz;
        int64_t C = c.cell_base + ((int64_t)kz * c.gn[1] + ky) * c.gn[0] + kx;
        np += w * d.cell_n[C];
        for (int k = 0; k < 3; ++k) {
          u[k] += w * d.cell_u[3 * C + k];
          gp[k] += w * d.gp_in[3 * C + k];
        }
      }
  const double4 v = d.vel[i];
  const double r = d.xr[i].w;
  double s[3] = {u[0] - v.x, u[1] - v.y, u[2] - v.z};
  double sm = sqrt((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
  double fd[3] = {0, 0, 0};
  if (sm > 0.0) {
    double de = 2.0 * r / c.kcg;
    double Re = c.rho_f * de * sm / c.mu_f;
    double cd = 0.63 + 4.8 / sqrt(Re);
    double Cd = cd * cd;
    double lg = 1.5 - log10(Re);
    double chi = 3.7 - 0.65 * exp(-(lg * lg) / 2.0);
    double coef = 0.125 * Cd * c.rho_f * M_PI * de * de * sm * pow(np, -chi);
    double cdr = d.cdrag ? d.cdrag[i] : 1.0;
    for (int k = 0; k < 3; ++k) fd[k] = c.k3 * coef * s[k] * cdr;
  }
  const double V = fr.w;
  double fb[3];
  for (int k = 0; k < 3; ++k) fb[k] = -V * (gp[k] + c.rho_f * c.g[k]);
  d.fpart[i] = make_double4(fd[0], fd[1], fd[2], 0.0);
  ((R4<R>*)d.fdr)[i] = mk4<R>((R)(fd[0] + fb[0]), (R)(fd[1] + fb[1]), (R)(fd[2] + fb[2]), (R)0);
}

// eq 7: drag source of every cell, fixed-order gather
__global__ void k_fluid_fcell(DevState d) {
  int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= d.ncell) return;
  const SampleConst& c = d.sc[d.cell_sample[C]];
  int64_t l = C - c.cell_base;
  int cx = (int)(l % c.gn[0]), cy = (int)((l / c.gn[0]) % c.gn[1]), cz = (int)(l / ((int64_t)c.gn[0] * c.gn[1]));
  const int cen = c.voidfrac == DEM_VOID_CENTROID;
  int lo[3], hi[3];
  const int cc[3] = {cx, cy, cz};
  for (int k = 0; k < 3; ++k) {
    if (cen) { lo[k] = hi[k] = cc[k]; }
    else if (c.gn[k] == 1) { lo[k] = hi[k] = 0; }
    else { lo[k] = cc[k] - 1 < 0 ? 0 : cc[k] - 1; hi[k] = cc[k] > c.gn[k] - 2 ? c.gn[k] - 2 : cc[k]; }
  }
  double s[3] = {0, 0, 0};
  for (int Dz = lo[2]; Dz <= hi[2]; ++Dz)
    for (int Dy = lo[1]; Dy <= hi[1]; ++Dy)
      for (int Dx = lo[0]; Dx <= hi[0]; ++Dx) {
        int64_t key = c.dual_base + ((int64_t)Dz * c.dn[1] + Dy) * c.dn[0] + Dx;
        for (int32_t q = d.doff[key]; q < d.doff[key + 1]; ++q) {
          int32_t i = d.dmem[q];
          double4 fr = d.dfr[i];
          double w = (cic_w(cx, Dx, fr.x, c.gn[0], cen) * cic_w(cy, Dy, fr.y, c.gn[1], cen)) *
                     cic_w(cz, Dz, fr.z, c.gn[2], cen);
          double4 fp = d.fpart[i];
          s[0] += w * fp.x; s[1] += w * fp.y; s[2] += w * fp.z;
        }
      }
  for (int k = 0; k < 3; ++k) d.fdc[3 * C + k] = s[k] / c.vcell;
}

template <typename R> void launch_fluid(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_fluid_key, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
  launch_bucket_sort((const uint32_t*)d.dkey, d.n, d.ndual, nullptr, d.dcnt, d.doff, d.dfill, d.dmem,
                     d.scan_tmp, s);
  if (d.ncell > 0) hipLaunchKernelGGL(k_fluid_eps, dim3(nblk(d.ncell)), dim3(kBlock), 0, s, d);
  hipLaunchKernelGGL(k_fluid_drag<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
  if (d.ncell > 0) hipLaunchKernelGGL(k_fluid_fcell, dim3(nblk(d.ncell)), dim3(kBlock), 0, s, d);
}
template void launch_fluid<double>(DevState&, hipStream_t);
template void launch_fluid<float>(DevState&, hipStream_t);

// ---------------------------------------------------------------------------
// read-back and aggregates
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_unpermute(DevState d, double* x, double* v, double* w, double* F, double* T, uint8_t* alive) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  int64_t o = d.orig[k];
  double4 p = d.xr[k], vv = d.vel[k];
  R4<R> ww = ((const R4<R>*)d.omg)[k], ff = ((const R4<R>*)d.frc)[k], tt = ((const R4<R>*)d.trq)[k];
  if (x) { x[3 * o] = p.x; x[3 * o + 1] = p.y; x[3 * o + 2] = p.z; }
  if (v) { v[3 * o] = vv.x; v[3 * o + 1] = vv.y; v[3 * o + 2] = vv.z; }
  if (w) { w[3 * o] = ww.x; w[3 * o + 1] = ww.y; w[3 * o + 2] = ww.z; }
  if (F) { F[3 * o] = ff.x; F[3 * o + 1] = ff.y; F[3 * o + 2] = ff.z; }
  if (T) { T[3 * o] = tt.x; T[3 * o + 1] = tt.y; T[3 * o + 2] = tt.z; }
  if (alive) alive[o] = d.alive[k];
}

template <typename R>
void launch_unpermute(DevState& d, double* x, double* v, double* w, double* F, double* T, uint8_t* alive,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d, x, v, w, F, T, alive);
}
template void launch_unpermute<double>(DevState&, double*, double*, double*, double*, double*, uint8_t*, hipStream_t);
template void launch_unpermute<float>(DevState&, double*, double*, double*, double*, double*, uint8_t*, hipStream_t);

// one block per sample; fixed-stride partial sums, then a tree in LDS
template <typename R>
__global__ void k_aggregate(DevState d, const int64_t* soff, double* produced, double* kinetic,
                            long long* contacts, long long* nalive) {
  __shared__ double sm[256], sk[256];
  __shared__ long long sc_[256], sa[256];
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  const SampleConst& c = d.sc[s];
  double pm = 0.0, ke = 0.0;
  long long na = 0, nc = 0;
  for (int64_t k = soff[s] + t; k < soff[s + 1]; k += 256) {
    double4 p = d.xr[k], v = d.vel[k];
    double m = c.rho * (4.0 / 3.0) * M_PI * p.w * p.w * p.w;
    if (!d.alive[k]) { pm += m; continue; }
    ++na;
    R4<R> w = ((const R4<R>*)d.omg)[k];
    double I = 0.4 * m * p.w * p.w;
    double wx = w.x, wy = w.y, wz = w.z;
    ke += 0.5 * m * ((v.x * v.x + v.y * v.y) + v.z * v.z) + 0.5 * I * ((wx * wx + wy * wy) + wz * wz);
    for (int32_t q = d.prow[k]; q < d.prow[k + 1]; ++q) nc += (d.pfl[q] & 3) ? 1 : 0;
  }
  sm[t] = pm; sk[t] = ke; sc_[t] = nc; sa[t] = na;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) { sm[t] += sm[t + off]; sk[t] += sk[t + off]; sc_[t] += sc_[t + off]; sa[t] += sa[t + off]; }
    __syncthreads();
  }
  if (t == 0) { produced[s] = sm[0]; kinetic[s] = sk[0]; contacts[s] = sc_[0]; nalive[s] = sa[0]; }
}

void launch_aggregate_impl(DevState& d, const int64_t* soff, double* produced, double* kinetic,
                           long long* contacts, long long* nalive, int fp64, hipStream_t s) {
  if (fp64)
    hipLaunchKernelGGL(k_aggregate<double>, dim3(d.nsamples), dim3(256), 0, s, d, soff, produced, kinetic,
                       contacts, nalive);
  else
    hipLaunchKernelGGL(k_aggregate<float>, dim3(d.nsamples), dim3(256), 0, s, d, soff, produced, kinetic,
                       contacts, nalive);
}

}  // namespace dem
