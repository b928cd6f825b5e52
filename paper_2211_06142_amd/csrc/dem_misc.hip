// dem_misc.hip -- read-back in the caller's order and per-sample aggregates
// (produced mass of eq 40, coordination, kinetic energy).  The aggregate
// sums use a fixed stride and a fixed tree, so they are deterministic.
#include "dem_device.h"

namespace dem {

template <typename R>
__global__ void k_unpermute(DevState d, double* x, double* v, double* w, double* F, double* T, uint8_t* alive) {
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
}

template <typename R>
void launch_unpermute(DevState& d, double* x, double* v, double* w, double* F, double* T, uint8_t* alive,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_unpermute<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d, x, v, w, F, T, alive);
}
template void launch_unpermute<double>(DevState&, double*, double*, double*, double*, double*, uint8_t*, hipStream_t);
template void launch_unpermute<float>(DevState&, double*, double*, double*, double*, double*, uint8_t*, hipStream_t);

// one 1024-thread block per sample
template <typename R>
__global__ __launch_bounds__(1024) void k_aggregate(DevState d, const int64_t* soff, double* produced,
                                                    double* kinetic, long long* contacts, long long* nalive) {
  __shared__ double sm[1024], sk[1024];
  __shared__ long long sc_[1024], sa[1024];
  const int s = blockIdx.x;
  const int t = threadIdx.x;
  const int b = d.cur;
  const SampleConst& c = d.sc[s];
  double pm = 0.0, ke = 0.0;
  long long na = 0, nc = 0;
  for (int64_t k = soff[s] + t; k < soff[s + 1]; k += 1024) {
    double4 p = d.xr[b][k], v = d.vel[b][k];
    double m = c.rho * (4.0 / 3.0) * M_PI * p.w * p.w * p.w;
    if (!d.alive[b][k]) { pm += m; continue; }
    ++na;
    R4<R> w = ((const R4<R>*)d.omg[b])[k];
    double I = 0.4 * m * p.w * p.w;
    double wx = w.x, wy = w.y, wz = w.z;
    ke += 0.5 * m * ((v.x * v.x + v.y * v.y) + v.z * v.z) + 0.5 * I * ((wx * wx + wy * wy) + wz * wz);
  }
  const int32_t p0 = d.hrow[soff[s]], p1 = d.hrow[soff[s + 1]];
  for (int32_t p = p0 + t; p < p1; p += 1024) {
    if ((d.pfl[b][p] & 3) && d.alive[b][d.sown[p]] && d.alive[b][d.spart[p]]) ++nc;
  }
  sm[t] = pm; sk[t] = ke; sc_[t] = nc; sa[t] = na;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) { sm[t] += sm[t + off]; sk[t] += sk[t + off]; sc_[t] += sc_[t + off]; sa[t] += sa[t + off]; }
    __syncthreads();
  }
  if (t == 0) { produced[s] = sm[0]; kinetic[s] = sk[0]; contacts[s] = sc_[0]; nalive[s] = sa[0]; }
}

void launch_aggregate_impl(DevState& d, const int64_t* soff, double* produced, double* kinetic, long long* contacts,
                           long long* nalive, double* partial, int fp64, hipStream_t s) {
  (void)partial;
  if (fp64)
    hipLaunchKernelGGL(k_aggregate<double>, dim3(d.nsamples), dim3(1024), 0, s, d, soff, produced, kinetic,
                       contacts, nalive);
  else
    hipLaunchKernelGGL(k_aggregate<float>, dim3(d.nsamples), dim3(1024), 0, s, d, soff, produced, kinetic,
                       contacts, nalive);
}

}  // namespace dem
