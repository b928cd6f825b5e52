// dem_rebuild.hip -- neighbour-list rebuild.
//
//   bin keys -> stable bucket sort by (sample, cell, id) -> permute the particle
//   arrays -> candidate search (one workgroup per binning cell: the 27
//   neighbour cells are staged in LDS, one wavefront per home particle tests
//   64 candidates at a time and compacts hits with a ballot and prefix
//   popcount; count pass, scan, fill pass) -> slot of every mirror entry ->
//   history of every half pair carried over from the previous list.
// Candidate predicate, in FP64 with a fixed operation order:
//   ((dx dx + dy dy) + dz dz) < ((r_i + r_j) + margin)^2.
#include "dem_device.h"

namespace dem {

__global__ void k_bin_keys(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const SampleConst& c = d.sc[d.sample[i]];
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
// candidate search.  The 27 neighbour cells of a home cell are staged in LDS as
// FP32 positions relative to the home cell's corner; each lane first applies a
// conservative FP32 test (cutoff widened by a relative slack far above the FP32
// rounding of the relative coordinates), and only the survivors take the exact
// FP64 test on the stored FP64 positions.  The exact test alone decides.
// ---------------------------------------------------------------------------
constexpr int kLdsCand = 2048;

template <bool kFill>
__global__ __launch_bounds__(256) void k_nbr_search(DevState d) {
  __shared__ float4 sx[kLdsCand];
  __shared__ int32_t sj[kLdsCand];
  __shared__ int32_t srs[27], srl[27];
  const int64_t cbin = blockIdx.x;
  const int32_t h0 = d.cell_start[cbin], h1 = d.cell_start[cbin + 1];
  if (h1 <= h0) return;
  const SampleConst& c = d.sc[d.bin_sample[cbin]];
  const int64_t local = cbin - c.bin_base;
  if (local >= (int64_t)c.bn[0] * c.bn[1] * c.bn[2]) return;   // the dead bucket
  const int cx = (int)(local % c.bn[0]);
  const int cy = (int)((local / c.bn[0]) % c.bn[1]);
  const int cz = (int)(local / ((int64_t)c.bn[0] * c.bn[1]));
  const double ox = c.blo[0] + cx * c.bh[0], oy = c.blo[1] + cy * c.bh[1], oz = c.blo[2] + cz * c.bh[2];
  const int t0 = threadIdx.x;
  if (t0 < 27) {
    int dx = t0 % 3 - 1, dy = (t0 / 3) % 3 - 1, dz = t0 / 9 - 1;
    int qx = cx + dx, qy = cy + dy, qz = cz + dz;
    srs[t0] = 0;
    srl[t0] = 0;
    if (qx >= 0 && qy >= 0 && qz >= 0 && qx < c.bn[0] && qy < c.bn[1] && qz < c.bn[2]) {
      int64_t q = c.bin_base + ((int64_t)qz * c.bn[1] + qy) * c.bn[0] + qx;
      srs[t0] = d.cell_start[q];
      srl[t0] = d.cell_start[q + 1] - srs[t0];
    }
  }
  __syncthreads();
  int total = 0;
  for (int k = 0; k < 27; ++k) total += srl[k];
  const bool staged = total <= kLdsCand;
  const double4* X = d.xr[d.cur];
  if (staged) {
    for (int t = t0; t < total; t += 256) {
      int acc = 0, j = -1;
      for (int k = 0; k < 27; ++k) {
        if (j < 0 && t < acc + srl[k]) j = srs[k] + (t - acc);
        acc += srl[k];
      }
      const double4 p = X[j];
      sx[t] = make_float4((float)(p.x - ox), (float)(p.y - oy), (float)(p.z - oz), (float)p.w);
      sj[t] = j;
    }
  }
  __syncthreads();
  const int lane = t0 & 63, wv = t0 >> 6;
  const double margin = c.margin;
  const float marginf = (float)margin;
  // absolute slack: the relative coordinates span at most two cells, each
  // rounded to FP32 (relative error 2^-24); 3e-6 of a cell side covers it many times
  const float slack = 3e-6f * (float)fmax(c.bh[0], fmax(c.bh[1], c.bh[2]));
  for (int32_t i = h0 + wv; i < h1; i += 4) {
    const double4 pi = X[i];
    const float pix = (float)(pi.x - ox), piy = (float)(pi.y - oy), piz = (float)(pi.z - oz), pir = (float)pi.w;
    int written = 0, owned = 0;
    int row = 0, pre_n = 0, hbase = 0;
    if (kFill) {
      row = d.nrow[i];
      pre_n = d.ncnt[i] - d.ocnt[i];
      hbase = d.hrow[i];
    }
    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      bool pred = false;
      int j = -1;
      if (t < total) {
        bool maybe;
        if (staged) {
          const float4 q = sx[t];
          j = sj[t];
          const float ex = q.x - pix, ey = q.y - piy, ez = q.z - piz;
          const float cf = ((pir + q.w) + marginf) * 1.0001f + slack;
          maybe = (ex * ex + ey * ey) + ez * ez < cf * cf;
        } else {
          int acc = 0;
          for (int k = 0; k < 27; ++k) {
            if (j < 0 && t < acc + srl[k]) j = srs[k] + (t - acc);
            acc += srl[k];
          }
          maybe = true;
        }
        if (maybe && j != i) {
          const double4 pj = X[j];
          double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
          double d2 = (dx * dx + dy * dy) + dz * dz;
          double cc = (pi.w + pj.w) + margin;
          pred = d2 < cc * cc;
        }
      }
      const unsigned long long mask = __ballot(pred);
      const unsigned long long omask = __ballot(pred && j > i);
      if (kFill && pred) {
        int pos = written + __popcll(mask & ((1ull << lane) - 1ull));
        d.nbr[row + pos] = j;
        if (j > i) {
          int slot = hbase + (pos - pre_n);
          d.nslot[row + pos] = slot;
          d.sown[slot] = i;
          d.spart[slot] = j;
        }
      }
      written += __popcll(mask);
      owned += __popcll(omask);
    }
    if (!kFill && lane == 0) {
      d.ncnt[i] = written;
      d.ocnt[i] = owned;
    }
  }
}

void launch_nbr_count(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_nbr_search<false>, dim3((unsigned)d.nbins_total), dim3(256), 0, s, d);
}
void launch_nbr_fill(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_nbr_search<true>, dim3((unsigned)d.nbins_total), dim3(256), 0, s, d);
}

// slot of every mirror entry (j < i): the owner entry i in row j, found by
// binary search in that row's sorted partners
__global__ void k_nbr_mirror(DevState d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int32_t r0 = d.nrow[i];
  const int32_t nmir = d.ncnt[i] - d.ocnt[i];
  for (int32_t e = r0; e < r0 + nmir; ++e) {
    int32_t j = d.nbr[e];
    int32_t lo = d.nrow[j], hi = d.nrow[j + 1];
    while (lo < hi) {
      int32_t mid = (lo + hi) >> 1;
      if (d.nbr[mid] < (int32_t)i) lo = mid + 1; else hi = mid;
    }
    d.nslot[e] = d.nslot[lo];
  }
}
void launch_nbr_mirror(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_nbr_mirror, dim3(nblk(d.n)), dim3(kBlock), 0, s, d);
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
    const SampleConst& c = d.sc[d.sample[i]];
    double4 p = d.xr[d.cur][i];
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
// history merge: every half pair and wall entry that existed in the previous
// list keeps its elongation and flags (found through the permutation)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_hist_merge(DevState d, int check_lost) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < d.nslots) {
    int32_t i = d.sown[p], j = d.spart[p];
    int32_t oi = d.order[i], oj = d.order[j];
    int32_t o = oi < oj ? oi : oj, q = oi < oj ? oj : oi;
    int32_t lo = d.nrow_o[o], hi = d.nrow_o[o + 1];
    while (lo < hi) {
      int32_t mid = (lo + hi) >> 1;
      if (d.nbr_o[mid] < q) lo = mid + 1; else hi = mid;
    }
    R4<R> h = mk4<R>(0, 0, 0, 0);
    uint8_t fl = 0;
    if (lo < d.nrow_o[o + 1] && d.nbr_o[lo] == q) {
      int32_t so = d.nslot_o[lo];
      h = ((const R4<R>*)d.hdt_o)[so];
      fl = d.pfl_o[so];
      if (oi > oj) { h.x = -h.x; h.y = -h.y; h.z = -h.z; }
      if (check_lost && (fl & 1)) atomicAdd(&d.scratch_i[1], 1);
    }
    ((R4<R>*)d.hdt[d.cur])[p] = h;
    d.pfl[d.cur][p] = fl;
  }
  int64_t e = p;
  if (e < d.nwall) {
    int32_t lo = 0, hi = (int32_t)d.n;
    while (lo < hi) {
      int32_t mid = (lo + hi) >> 1;
      if (d.wrow[mid + 1] <= e) lo = mid + 1; else hi = mid;
    }
    int32_t i = lo;
    int32_t w = d.wid[e];
    int32_t oi = d.order[i];
    R4<R> h = mk4<R>(0, 0, 0, 0);
    uint8_t fl = 0;
    for (int32_t q = d.wrow_o[oi]; q < d.wrow_o[oi + 1]; ++q)
      if (d.wid_o[q] == w) { h = ((const R4<R>*)d.wdt_o)[q]; fl = d.wfl_o[q]; }
    ((R4<R>*)d.wdt)[e] = h;
    d.wfl[e] = fl;
  }
}

template <typename R> void launch_hist_merge(DevState& d, hipStream_t s, int check_lost) {
  int64_t m = d.nslots > d.nwall ? d.nslots : d.nwall;
  if (m > 0) hipLaunchKernelGGL(k_hist_merge<R>, dim3(nblk(m)), dim3(kBlock), 0, s, d, check_lost);
}
template void launch_hist_merge<double>(DevState&, hipStream_t, int);
template void launch_hist_merge<float>(DevState&, hipStream_t, int);

// bonded half pairs of the previous list whose partners are both alive
__global__ void k_count_old_bonds(DevState d) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.nslots_o) return;
  if (!(d.pfl_o[p] & 1)) return;
  int32_t a = d.inv_order[d.sown_o[p]], b = d.inv_order[d.spart_o[p]];
  if (d.alive[d.cur][a] && d.alive[d.cur][b]) atomicAdd(&d.scratch_i[0], 1);
}
void launch_count_old_bonds(DevState& d, hipStream_t s) {
  (void)hipMemsetAsync(d.scratch_i, 0, 2 * sizeof(int), s);
  if (d.nslots_o > 0) hipLaunchKernelGGL(k_count_old_bonds, dim3(nblk(d.nslots_o)), dim3(kBlock), 0, s, d);
}

__global__ void k_check_lost(DevState d) {
  if (d.scratch_i[0] != d.scratch_i[1]) atomicOr(d.status, (int)kStLostBond);
}
void launch_check_lost(DevState& d, hipStream_t s) {
  hipLaunchKernelGGL(k_check_lost, dim3(1), dim3(1), 0, s, d);
}

// bond every touching pair (initial state of the modified JKR model)
__global__ void k_mark_bonds(DevState d) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.nslots) return;
  int32_t i = d.sown[p], j = d.spart[p];
  const SampleConst& c = d.sc[d.sample[i]];
  if (c.normal_model != DEM_NORMAL_JKR_MOD) return;
  double4 a = d.xr[d.cur][i], b = d.xr[d.cur][j];
  double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double cs = a.w + b.w;
  if (d2 < cs * cs) d.pfl[d.cur][p] = 1;
}
void launch_mark_bonds(DevState& d, hipStream_t s) {
  if (d.nslots > 0) hipLaunchKernelGGL(k_mark_bonds, dim3(nblk(d.nslots)), dim3(kBlock), 0, s, d);
}

}  // namespace dem
