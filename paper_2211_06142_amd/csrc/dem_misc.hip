// dem_misc.hip -- read-back in the caller's order and per-sample aggregates
// (produced mass of eq 40, coordination, kinetic energy).  The aggregate
// sums use a fixed stride and a fixed tree, so they are deterministic; the
// produced mass is an integer (fixed-point) counter added to at each removal.
#include "dem_device.h"

namespace dem {

template <typename R>
__global__ void k_unpermute(DevState d, double* x, double* v, double* w, double* F, double* T, uint8_t* alive,
                            double* FF) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const int b = d.cur;
  int64_t o = d.orig[k];
  double4 p = d.xr[b][k], vv = d.vel[b][k];
  R4<R> ww = ((const R4<R>*)d.omg[b])[k], ff = ((const R4<R>*)d.frc)[k], tt = ((const R4<R>*)d.trq)[k];
  if (x) { x[3 * o] = p.x; x[3 * o + 1] = p.y; x[3 * o + 2] = p.z; }
  if (v) { v[3 * o] = vv.x; v[3 * o + 1] = vv.y; v[3 * o + 2] = vv.z; }
  if (w) { w[3 * o] = ww.x; w[3 * o + 1] = ww.y; w[3 * o + 2] = ww.z; }
  if (F) { F[3 * o] = ff.x; F[3 * o + 1] = ff.y; F[3 * o + 2] = ff.z; }
  if (T) { T[3 * o] = tt.x; T[3 * o + 1] = tt.y; T[3 * o + 2] = tt.z; }
  if (alive) alive[o] = d.alive[b][k];
  if (FF) {
    const R4<R> q = ((const R4<R>*)d.fdr)[k];
    FF[3 * o] = q.x; FF[3 * o + 1] = q.y; FF[3 * o + 2] = q.z;
  }
}

// wall history of each particle to [caller index][wall][xyz] (the output is
// zeroed first: walls out of reach hold no history)
template <typename R>
__global__ void k_unpermute_walls(DevState d, double* wall_dt) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= d.n) return;
  const int64_t o = d.orig[k];
  for (int32_t e = d.wrow[k]; e < d.wrow[k + 1]; ++e) {
    const R4<R> h = ((const R4<R>*)d.wdt)[e];
    double* q = wall_dt + (o * DEM_MAX_WALLS + d.wid[e]) * 3;
    q[0] = h.x; q[1] = h.y; q[2] = h.z;
  }
}

template <typename R> void launch_unpermute_walls(DevState& d, double* wall_dt, hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute_walls<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d, wall_dt);
}
template void launch_unpermute_walls<double>(DevState&, double*, hipStream_t);
template void launch_unpermute_walls<float>(DevState&, double*, hipStream_t);

template <typename R>
void launch_unpermute(DevState& d, double* x, double* v, double* w, double* F, double* T, uint8_t* alive,
                      double* FF, hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d, x, v, w, F, T, alive, FF);
}
template void launch_unpermute<double>(DevState&, double*, double*, double*, double*, double*, uint8_t*, double*,
                                       hipStream_t);
template void launch_unpermute<float>(DevState&, double*, double*, double*, double*, double*, uint8_t*, double*,
                                      hipStream_t);

// Aggregates in two fixed-order passes: kAggChunks blocks per sample each
// reduce one contiguous slice of the sample's particles and half-pair slots
// (tree in LDS), then one thread per sample sums its slices in order.
constexpr int kAggChunks = 256;   // 256 blocks fill the chip for one sample

template <typename R>
__global__ __launch_bounds__(256) void k_aggregate_part(DevState d, const int64_t* soff, double* part) {
  __shared__ double sh[3][256];
  const int s = blockIdx.x / kAggChunks, ch = blockIdx.x % kAggChunks;
  const int t = threadIdx.x;
  const int b = d.cur;
  const SampleConst& c = sample_const(d.sc, s);
  const int64_t a0 = soff[s], a1 = soff[s + 1];
  const int64_t k0 = a0 + (a1 - a0) * ch / kAggChunks, k1 = a0 + (a1 - a0) * (ch + 1) / kAggChunks;
  double ke = 0.0, na = 0.0, nc = 0.0;
  for (int64_t k = k0 + t; k < k1; k += 256) {
    if (!d.alive[b][k]) continue;
    double4 p = d.xr[b][k], v = d.vel[b][k];
    double m = c.rho * (4.0 / 3.0) * M_PI * p.w * p.w * p.w;
    na += 1.0;
    R4<R> w = ((const R4<R>*)d.omg[b])[k];
    double I = 0.4 * m * p.w * p.w;
    double wx = w.x, wy = w.y, wz = w.z;
    ke += 0.5 * m * ((v.x * v.x + v.y * v.y) + v.z * v.z) + 0.5 * I * ((wx * wx + wy * wy) + wz * wz);
  }
  const int64_t p0 = d.hrow[a0], p1 = d.hrow[a1];
  const int64_t q0 = p0 + (p1 - p0) * ch / kAggChunks, q1 = p0 + (p1 - p0) * (ch + 1) / kAggChunks;
  for (int64_t p = q0 + t; p < q1; p += 256)
    if ((d.pfl[b][p] & 3) && d.alive[b][d.sown[p]] && d.alive[b][d.spart[p]]) nc += 1.0;
  sh[0][t] = ke; sh[1][t] = nc; sh[2][t] = na;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off)
      for (int q = 0; q < 3; ++q) sh[q][t] += sh[q][t + off];
    __syncthreads();
  }
  if (t < 3) part[(int64_t)blockIdx.x * 3 + t] = sh[t][0];
}

__global__ void k_aggregate_final(const double* part, int nsamples, const SampleConst* sc,
                                  const unsigned long long* produced_fx, double* produced, double* kinetic,
                                  long long* contacts, long long* nalive) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsamples) return;
  double a[3] = {0, 0, 0};
  for (int ch = 0; ch < kAggChunks; ++ch)
    for (int q = 0; q < 3; ++q) a[q] += part[((int64_t)s * kAggChunks + ch) * 3 + q];
  produced[s] = (double)produced_fx[s] / sc[s].pm_scale;
  kinetic[s] = a[0];
  contacts[s] = (long long)a[1];
  nalive[s] = (long long)a[2];
}

int64_t aggregate_scratch_doubles(int nsamples) { return (int64_t)nsamples * kAggChunks * 3; }

void launch_aggregate_impl(DevState& d, const int64_t* soff, double* produced, double* kinetic, long long* contacts,
                           long long* nalive, double* partial, int fp64, hipStream_t s) {
  const unsigned nb = (unsigned)(d.nsamples * kAggChunks);
  if (fp64)
    hipLaunchKernelGGL(k_aggregate_part<double>, dim3(nb), dim3(256), 0, s, d, soff, partial);
  else
    hipLaunchKernelGGL(k_aggregate_part<float>, dim3(nb), dim3(256), 0, s, d, soff, partial);
  hipLaunchKernelGGL(k_aggregate_final, dim3(nblk(d.nsamples)), dim3(kBlock), 0, s, partial, d.nsamples, d.sc,
                     d.produced_fx, produced, kinetic, contacts, nalive);
}

}  // namespace dem
