// dem_rebuild.hip -- neighbour-list rebuild.
//
//   bin keys -> stable bucket sort by (sample, cell, id) -> permute the particle
//   arrays -> candidate search into fixed-stride scratch rows (one workgroup
//   per binning cell) -> scan of the row lengths -> rows and half-pair slots
//   in CSR -> history of every half pair carried over from the previous list.
// Candidate predicate, in FP64 with a fixed operation order:
//   ((dx dx + dy dy) + dz dz) < ((r_i + r_j) + margin)^2.
#include "dem_device.h"

namespace dem {

__global__ void k_bin_keys(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const SampleConst& c = sample_const(d.sc, d.sample[i]);
  int64_t nb = (int64_t)c.bn[0] * c.bn[1] * c.bn[2];
  if (!d.alive[d.cur][i]) { d.key[i] = (uint32_t)(c.bin_base + nb); return; }
  double4 p = d.xr[d.cur][i];
  int cx = bin_coord(p.x, c.blo[0], c.bh[0], c.bn[0]);
  int cy = bin_coord(p.y, c.blo[1], c.bh[1], c.bn[1]);
  int cz = bin_coord(p.z, c.blo[2], c.bh[2], c.bn[2]);
  d.key[i] = (uint32_t)(c.bin_base + ((int64_t)cz * c.bn[1] + cy) * c.bn[0] + cx);
}

void launch_bin_keys(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_keys, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}

// new[k] = old[order[k]]: double-buffered arrays go from buffer cur to 1-cur,
// single arrays to the scratch buffers (the host swaps the pointers)
template <typename R>
__global__ void k_permute(DevState d) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const int a = d.cur, b = 1 - d.cur;
  int32_t o = d.order[k];
  d.xr[b][k] = d.xr[a][o];
  d.vel[b][k] = d.vel[a][o];
  ((R4<R>*)d.omg[b])[k] = ((const R4<R>*)d.omg[a])[o];
  d.alive[b][k] = d.alive[a][o];
  ((R4<R>*)d.t_r4[0])[k] = ((const R4<R>*)d.frc)[o];
  ((R4<R>*)d.t_r4[1])[k] = ((const R4<R>*)d.trq)[o];
  ((R4<R>*)d.t_r4[2])[k] = ((const R4<R>*)d.fdr)[o];
  d.t_i[0][k] = d.sample[o];
  d.t_i[1][k] = d.orig[o];
  if (d.cdrag) {
    d.t_d[0][k] = d.cdrag[o];
    d.t_d[1][k] = d.ccoh[o];
  }
  if (d.closure_on)
    for (int c = 0; c < 6; ++c) d.t_feat[6 * k + c] = d.cfeat[6 * o + c];
  d.inv_order[o] = (int32_t)k;
}

template <typename R> void launch_permute(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_permute<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}
template void launch_permute<double>(DevState&, hipStream_t);
template void launch_permute<float>(DevState&, hipStream_t);

__global__ void k_set_xref(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.n) d.xref[i] = d.xr[d.cur][i];
}
void launch_set_xref(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_set_xref, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}

// ---------------------------------------------------------------------------
// candidate search, one pass.  One workgroup per binning cell: the 27
// neighbour cells are staged in LDS as FP32 positions relative to the home
// cell's corner.  Phase 1: a wavefront per home particle applies a
// conservative FP32 test to 64 candidates at a time (cutoff widened by a
// slack far above the FP32 rounding of the relative coordinates) and compacts
// the survivors in candidate order.  Phase 2: every survivor of the cell takes
// the exact FP64 test, one survivor per lane, all in one round of loads.
// Phase 3: each confirmed row goes to its fixed scratch row (stride kRowMax),
// with its counts.  The exact test alone decides.
// Rows with more FP32 survivors than kRowMax, and every row of a cell whose
// neighbourhood does not fit in LDS, are searched straight from global memory;
// rows longer than kRowMax are listed as overflow rows, which the fill
// searches again and writes directly.
// Candidates come in increasing partner index: the 27 cells in increasing
// binning index, each cell's particles in sorted order.
// ---------------------------------------------------------------------------
constexpr int kLdsCand = 1024;   // staged candidates per home cell
constexpr int kHomeMax = 64;     // home particles of a staged cell

__device__ inline bool is_candidate(const double4& pi, const double4& pj, double margin) {
  double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double cc = (pi.w + pj.w) + margin;
  return d2 < cc * cc;
}

// start and length of neighbour cell t (0..26) of binning cell (cx, cy, cz)
__device__ inline void cell_range(const DevState& d, const SampleConst& c, int cx, int cy, int cz, int t,
                                  int32_t& st, int32_t& len) {
  int qx = cx + t % 3 - 1, qy = cy + (t / 3) % 3 - 1, qz = cz + t / 9 - 1;
  st = 0;
  len = 0;
  if (qx >= 0 && qy >= 0 && qz >= 0 && qx < c.bn[0] && qy < c.bn[1] && qz < c.bn[2]) {
    int64_t q = c.bin_base + ((int64_t)qz * c.bn[1] + qy) * c.bn[0] + qx;
    st = d.cell_start[q];
    len = d.cell_start[q + 1] - st;
  }
}

// particle index of candidate t of the concatenated 27 cells
__device__ inline int32_t cand_index(const int32_t* srs, const int32_t* srl, int t) {
  int acc = 0, j = -1;
#pragma unroll 1
  for (int k = 0; k < 27; ++k) {
    if (j < 0 && t < acc + srl[k]) j = srs[k] + (t - acc);
    acc += srl[k];
  }
  return j;
}

// row i straight from global memory (wavefront-wide), cell by cell in
// candidate order: counts, and the row in its scratch row as far as it fits
__device__ inline void search_row_global(const DevState& d, const double4* X, int32_t i, const int32_t* srs,
                                         const int32_t* srl, double margin, int lane, int& written, int& owned) {
  const double4 pi = X[i];
  for (int k = 0; k < 27; ++k) {
    const int32_t c0 = srs[k], len = srl[k];
    for (int base = 0; base < len; base += 64) {
      const int t = base + lane;
      const int32_t j = c0 + t;
      const bool pred = t < len && j != i && is_candidate(pi, X[j], margin);
      const unsigned long long m = __ballot(pred);
      const int pos = written + __popcll(m & ((1ull << lane) - 1ull));
      if (pred && pos < kRowMax) d.scr[(int64_t)i * kRowMax + pos] = j;
      written += __popcll(m);
      owned += __popcll(__ballot(pred && j > i));
    }
  }
}

__device__ inline void push_overflow(DevState& d, int32_t i) {
  int k = atomicAdd(d.novf, 1);
  d.ovf[k] = i;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_nbr_search(DevState d) {
  __shared__ float4 sx[kLdsCand];
  __shared__ int32_t sj[kLdsCand];
  __shared__ int16_t surv[kHomeMax][kRowMax];   // candidate of each survivor; -1 once rejected
  __shared__ int32_t nsurv[kHomeMax];
  __shared__ int32_t pre[kHomeMax + 1];
  __shared__ int32_t srs[27], srl[27];
  const int64_t cbin = blockIdx.x;
  const int32_t h0 = d.cell_start[cbin], h1 = d.cell_start[cbin + 1];
  if (h1 <= h0) return;
  const SampleConst& c = sample_const(d.sc, d.bin_sample[cbin]);
  const int64_t local = cbin - c.bin_base;
  if (local >= (int64_t)c.bn[0] * c.bn[1] * c.bn[2]) return;   // the dead bucket
  const int cx = (int)(local % c.bn[0]);
  const int cy = (int)((local / c.bn[0]) % c.bn[1]);
  const int cz = (int)(local / ((int64_t)c.bn[0] * c.bn[1]));
  const int t0 = threadIdx.x;
  if (t0 < 27) cell_range(d, c, cx, cy, cz, t0, srs[t0], srl[t0]);
  __syncthreads();
  int total = 0, home_off = 0;
  for (int k = 0; k < 27; ++k) {
    if (k == 13) home_off = total;
    total += srl[k];
  }
  const int nh = h1 - h0;
  const int lane = t0 & 63, wv = t0 >> 6;
  const double margin = c.margin;
  const double4* X = d.xr[d.cur];
  if (total > kLdsCand || nh > kHomeMax) {
    // crowded neighbourhood: count every home row from global memory
    for (int32_t i = h0 + wv; i < h1; i += 4) {
      int written = 0, owned = 0;
      search_row_global(d, X, i, srs, srl, margin, lane, written, owned);
      if (lane == 0) {
        d.ncnt[i] = written;
        d.ocnt[i] = owned;
        if (written > kRowMax) push_overflow(d, i);
      }
    }
    return;
  }
  const double ox = c.blo[0] + cx * c.bh[0], oy = c.blo[1] + cy * c.bh[1], oz = c.blo[2] + cz * c.bh[2];
  for (int t = t0; t < total; t += 256) {
    const int32_t j = cand_index(srs, srl, t);
    const double4 p = X[j];
    sx[t] = make_float4((float)(p.x - ox), (float)(p.y - oy), (float)(p.z - oz), (float)p.w);
    sj[t] = j;
  }
  __syncthreads();
  const float marginf = (float)margin;
  // the relative coordinates span at most two cells, each rounded to FP32
  // (relative error 2^-24); 3e-6 of a cell side covers that many times over
  const float slack = 3e-6f * (float)fmax(c.bh[0], fmax(c.bh[1], c.bh[2]));
  // phase 1: FP32 prefilter
  for (int h = wv; h < nh; h += 4) {
    const int32_t i = h0 + h;
    const float4 q0 = sx[home_off + h];
    int cnt = 0;
    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      bool maybe = false;
      if (t < total && sj[t] != i) {
        const float4 q = sx[t];
        const float ex = q.x - q0.x, ey = q.y - q0.y, ez = q.z - q0.z;
        const float cf = ((q0.w + q.w) + marginf) * 1.0001f + slack;
        maybe = (ex * ex + ey * ey) + ez * ez < cf * cf;
      }
      const unsigned long long m = __ballot(maybe);
      const int pos = cnt + __popcll(m & ((1ull << lane) - 1ull));
      if (maybe && pos < kRowMax) surv[h][pos] = (int16_t)t;
      cnt += __popcll(m);
    }
    if (lane == 0) nsurv[h] = cnt;
  }
  __syncthreads();
  // phase 2: exact FP64 test of every kept survivor (rows with more survivors
  // than kRowMax are counted directly in phase 3)
  if (wv == 0) {
    int v = lane < nh && nsurv[lane] <= kRowMax ? nsurv[lane] : 0;
    for (int off = 1; off < 64; off <<= 1) {
      int u = __shfl_up(v, off, 64);
      if (lane >= off) v += u;
    }
    pre[lane + 1] = v;
    if (lane == 0) pre[0] = 0;
  }
  __syncthreads();
  const int nsv = pre[nh];
  for (int q = t0; q < nsv; q += 256) {
    int lo = 0, hi = nh;
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (pre[mid] <= q) lo = mid; else hi = mid;
    }
    const int k = q - pre[lo];
    if (!is_candidate(X[h0 + lo], X[sj[surv[lo][k]]], margin)) surv[lo][k] = -1;
  }
  __syncthreads();
  // phase 3: rows to scratch in candidate order
  for (int h = wv; h < nh; h += 4) {
    const int32_t i = h0 + h;
    const int ns = nsurv[h];
    int written = 0, owned = 0;
    if (ns <= kRowMax) {
      const int t = lane < ns ? surv[h][lane] : -1;
      const bool pred = t >= 0;
      const int32_t j = pred ? sj[t] : -1;
      const unsigned long long m = __ballot(pred);
      if (pred) d.scr[(int64_t)i * kRowMax + __popcll(m & ((1ull << lane) - 1ull))] = j;
      written = __popcll(m);
      owned = __popcll(__ballot(pred && j > i));
    } else {
      search_row_global(d, X, i, srs, srl, margin, lane, written, owned);
    }
    if (lane == 0) {
      d.ncnt[i] = written;
      d.ocnt[i] = owned;
      if (written > kRowMax) push_overflow(d, i);
    }
  }
}

__global__ void k_totals(DevState d) {
  if (threadIdx.x == 0) {
    d.totals[0] = d.nrow[d.n];
    d.totals[1] = d.hrow[d.n];
    d.totals[2] = d.wrow[d.n];
    d.totals[3] = *d.novf;
  }
}
void launch_totals(DevState& d, hipStream_t s) { hipLaunchKernelGGL(k_totals, dim3(1), dim3(64), 0, s, d); }

void launch_nbr_search(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_nbr_search, dim3((unsigned)d.nbins_total), dim3(256), 0, s, d);
}

// overflow rows: one wavefront per row, candidates straight from global memory,
// written to the final row with the slots of the owner entries
__global__ __launch_bounds__(64) void k_nbr_fill_overflow(DevState d) {
  __shared__ int32_t srs[27], srl[27];
  const int32_t i = d.ovf[blockIdx.x];
  const SampleConst& c = sample_const(d.sc, d.sample[i]);
  const double4* X = d.xr[d.cur];
  const double4 pi = X[i];
  const int cx = bin_coord(pi.x, c.blo[0], c.bh[0], c.bn[0]);
  const int cy = bin_coord(pi.y, c.blo[1], c.bh[1], c.bn[1]);
  const int cz = bin_coord(pi.z, c.blo[2], c.bh[2], c.bn[2]);
  const int lane = threadIdx.x;
  if (lane < 27) cell_range(d, c, cx, cy, cz, lane, srs[lane], srl[lane]);
  __syncthreads();
  const int32_t row = d.nrow[i], hbase = d.hrow[i];
  const int pre_n = d.ncnt[i] - d.ocnt[i];
  int written = 0;
  for (int k = 0; k < 27; ++k) {
    const int32_t c0 = srs[k], len = srl[k];
    for (int base = 0; base < len; base += 64) {
      const int t = base + lane;
      const int32_t j = c0 + t;
      const bool pred = t < len && j != i && is_candidate(pi, X[j], c.margin);
      const unsigned long long m = __ballot(pred);
      if (pred) {
        const int pos = written + __popcll(m & ((1ull << lane) - 1ull));
        d.nbr[row + pos] = j;
        if (j > i) {
          const int slot = hbase + (pos - pre_n);
          d.nslot[row + pos] = slot;
          d.sown[slot] = i;
          d.spart[slot] = j;
        }
      }
      written += __popcll(m);
    }
  }
}

// scratch rows to the final rows: a group of 8 lanes per particle.  Owner
// entries (j > i) get the next half-pair slot of the row; a mirror entry takes
// the slot of the owner entry i in row j, found by binary search in row j
// (its scratch row, or its final row when row j overflowed).
__global__ __launch_bounds__(256) void k_nbr_copy(DevState d) {
  const int sub = threadIdx.x & 7;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  if (i >= d.n) return;
  const int cnt = d.ncnt[i];
  if (cnt > kRowMax) return;
  const int32_t row = d.nrow[i], hbase = d.hrow[i];
  const int pre_n = cnt - d.ocnt[i];
  const int32_t* src = d.scr + i * kRowMax;
  for (int k = sub; k < cnt; k += 8) {
    const int32_t j = src[k];
    d.nbr[row + k] = j;
    int32_t slot;
    if (j > (int32_t)i) {
      slot = hbase + (k - pre_n);
      d.sown[slot] = (int32_t)i;
      d.spart[slot] = j;
    } else {
      const int cj = d.ncnt[j];
      if (cj <= kRowMax) {
        const int32_t* rj = d.scr + (int64_t)j * kRowMax;
        int lo = 0, hi = cj;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (rj[mid] < (int32_t)i) lo = mid + 1; else hi = mid;
        }
        slot = d.hrow[j] + (lo - (cj - d.ocnt[j]));
      } else {
        int32_t lo = d.nrow[j], hi = d.nrow[j + 1];
        while (lo < hi) {
          int32_t mid = (lo + hi) >> 1;
          if (d.nbr[mid] < (int32_t)i) lo = mid + 1; else hi = mid;
        }
        slot = d.nslot[lo];
      }
    }
    d.nslot[row + k] = slot;
  }
}

// mirror entries of the overflow rows (after every owner entry is final):
// one wavefront per row, one binary search per lane
__global__ __launch_bounds__(64) void k_nbr_mirror_overflow(DevState d) {
  const int32_t i = d.ovf[blockIdx.x];
  const int32_t r0 = d.nrow[i];
  const int32_t nmir = d.ncnt[i] - d.ocnt[i];
  for (int32_t e = r0 + (int32_t)threadIdx.x; e < r0 + nmir; e += 64) {
    const int32_t j = d.nbr[e];
    int32_t lo = d.nrow[j], hi = d.nrow[j + 1];
    while (lo < hi) {
      int32_t mid = (lo + hi) >> 1;
      if (d.nbr[mid] < i) lo = mid + 1; else hi = mid;
    }
    d.nslot[e] = d.nslot[lo];
  }
}

void launch_nbr_fill(DevState& d, int novf, hipStream_t s) {
  if (novf > 0) hipLaunchKernelGGL(k_nbr_fill_overflow, dim3(novf), dim3(64), 0, s, d);
  hipLaunchKernelGGL(k_nbr_copy, dim3(nblk(d.n * 8)), dim3(kBlock), 0, s, d);
  if (novf > 0) hipLaunchKernelGGL(k_nbr_mirror_overflow, dim3(novf), dim3(64), 0, s, d);
}

// ---------------------------------------------------------------------------
// walls within the skin
// ---------------------------------------------------------------------------
template <bool kFill>
__global__ void k_wall_search(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  int cnt = 0;
  if (d.alive[d.cur][i]) {
    const SampleConst& c = sample_const(d.sc, d.sample[i]);
    double4 p = d.xr[d.cur][i];
    int row = kFill ? d.wrow[i] : 0;
    for (int w = 0; w < c.n_walls; ++w) {
      double sd, nw[3];
      if (wall_geom(c.walls[w], p.x, p.y, p.z, sd, nw, true) && sd < p.w + c.skin) {
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
// history carry: every half pair and wall entry of the previous list keeps its
// elongation and flags in the new list (found through the permutation)
// ---------------------------------------------------------------------------
// (a clear flag stands for a zero elongation, so the elongations are not cleared)
template <typename R>
__global__ void k_zero_slots(DevState d) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.nslots) return;
  d.pfl[d.cur][p] = 0;
}

// one thread per half pair of the previous list; pairs with no state (not
// touching, not bonded: the flag clear, the elongation zero) have nothing to carry.  A bonded pair
// whose partners are both alive must be in the new list: the candidate margin
// covers the largest pull-off separation, so a miss means the margin failed.
template <typename R>
__global__ void k_carry_pairs(DevState d, int check_lost) {
  int64_t so = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (so >= d.nslots_o) return;
  const uint8_t fl = d.pfl_o[so];
  if (fl == 0) return;
  R4<R> h = ((const R4<R>*)d.hdt_o)[so];
  const int32_t A = d.inv_order[d.sown_o[so]], B = d.inv_order[d.spart_o[so]];
  const uint8_t* al = d.alive[d.cur];
  if (!al[A] || !al[B]) return;
  const int32_t o = A < B ? A : B, q = A < B ? B : A;
  int32_t lo = d.nrow[o], hi = d.nrow[o + 1];
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (d.nbr[mid] < q) lo = mid + 1; else hi = mid;
  }
  if (lo < d.nrow[o + 1] && d.nbr[lo] == q) {
    const int32_t p = d.nslot[lo];
    if (A > B) { h.x = -h.x; h.y = -h.y; h.z = -h.z; }
    ((R4<R>*)d.hdt[d.cur])[p] = h;
    d.pfl[d.cur][p] = fl;
  } else if (check_lost && (fl & 1)) {
    atomicOr(d.status, (int)kStLostBond);
  }
}

// one thread per particle: its wall entries, matched by wall id in its old row
template <typename R>
__global__ void k_carry_walls(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int32_t e0 = d.wrow[i], e1 = d.wrow[i + 1];
  if (e0 == e1) return;
  const int32_t oi = d.order[i];
  const int32_t q0 = d.wrow_o[oi], q1 = d.wrow_o[oi + 1];
  for (int32_t e = e0; e < e1; ++e) {
    const int32_t w = d.wid[e];
    R4<R> h = mk4<R>(0, 0, 0, 0);
    uint8_t fl = 0;
    for (int32_t q = q0; q < q1; ++q)
      if (d.wid_o[q] == w) { h = ((const R4<R>*)d.wdt_o)[q]; fl = d.wfl_o[q]; }
    ((R4<R>*)d.wdt)[e] = h;
    d.wfl[e] = fl;
  }
}

template <typename R> void launch_hist_carry(DevState& d, hipStream_t s, int check_lost) {
  if (d.nslots > 0) hipLaunchKernelGGL(k_zero_slots<R>, dim3(nblk(d.nslots)), dim3(kBlock), 0, s, d);
  if (d.nslots_o > 0) hipLaunchKernelGGL(k_carry_pairs<R>, dim3(nblk(d.nslots_o)), dim3(kBlock), 0, s, d, check_lost);
  if (d.nwall > 0) hipLaunchKernelGGL(k_carry_walls<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
}
template void launch_hist_carry<double>(DevState&, hipStream_t, int);
template void launch_hist_carry<float>(DevState&, hipStream_t, int);

// bond every touching pair (initial state of the JKR models); a pair that had
// no flag gets its zero elongation written (a clear flag stood for it)
template <typename R>
__global__ void k_mark_bonds(DevState d) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.nslots) return;
  int32_t i = d.sown[p], j = d.spart[p];
  const SampleConst& c = sample_const(d.sc, d.sample[i]);
  if (c.normal_model != DEM_NORMAL_JKR_MOD && c.normal_model != DEM_NORMAL_JKR_ORIG) return;
  double4 a = d.xr[d.cur][i], b = d.xr[d.cur][j];
  double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double cs = a.w + b.w;
  if (!(d2 < cs * cs)) return;
  if (d.pfl[d.cur][p] == 0) ((R4<R>*)d.hdt[d.cur])[p] = mk4<R>(0, 0, 0, 0);
  d.pfl[d.cur][p] = 1;
}
template <typename R> void launch_mark_bonds(DevState& d, hipStream_t s) {
  if (d.nslots > 0) hipLaunchKernelGGL(k_mark_bonds<R>, dim3(nblk(d.nslots)), dim3(kBlock), 0, s, d);
}
template void launch_mark_bonds<double>(DevState&, hipStream_t);
template void launch_mark_bonds<float>(DevState&, hipStream_t);

}  // namespace dem
