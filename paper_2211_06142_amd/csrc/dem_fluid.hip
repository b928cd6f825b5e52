// dem_fluid.hip -- fluid-particle coupling (arXiv:2211.06142 section 2.2).
//
// Every reduction is a sorted segmented reduction, no floating-point atomics:
// particles are bucket-sorted by the cell of the grid of fluid-cell centres
// that holds them ("dual cell": its 8 corners are the 8 fluid cells a
// trilinear weight reaches; for centroid deposition the bucket is the fluid
// cell itself); each bucket sums its members in index order into 8 corner
// partials; each fluid cell then sums the corner partials of the (up to 8)
// buckets around it in a fixed order.
//   porosity  n = clamp(1 - sum w V / V_cell, n_min, 1)           (eq 6)
//   drag      Di Felice, coarse-grained k^3 f(d/k), closure factor (eq 8-11)
//   buoyancy  F_b = -V (grad p + rho_f g)                           (eq 1)
//   source    sum w f / V_cell                                      (eq 7)
#include "dem_device.h"

namespace dem {

// Every particle gets a key in range, also when the window was aborted (then
// buffer `buf` may never have been written and every particle goes to its
// sample's skip bucket): the bucket sort that follows is not gated.
__global__ void k_fluid_key(const DevState* __restrict__ dp, int buf) {
  const DevState& d = *dp;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const SampleConst& c = sample_const(d.sc, d.sample[i]);
  int64_t nd = (int64_t)c.dn[0] * c.dn[1] * c.dn[2];
  const int32_t skip = (int32_t)(c.dual_base + nd);
  if (*d.abort || !d.alive[buf][i] || !c.fluid_on) { d.dkey[i] = skip; return; }
  const double4 p = d.xr[buf][i];
  if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) { d.dkey[i] = skip; return; }
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

// trilinear weight of corner (kx, ky, kz) in {0,1}^3 of a bucket
__device__ inline double corner_w(const double4& fr, int kx, int ky, int kz) {
  double wx = kx ? fr.x : 1.0 - fr.x;
  double wy = ky ? fr.y : 1.0 - fr.y;
  double wz = kz ? fr.z : 1.0 - fr.z;
  return (wx * wy) * wz;
}

// corner partials of every bucket: kind 0 volume (8 per bucket), kind 1 drag (24 per bucket)
template <int kKind>
__global__ __launch_bounds__(64) void k_fluid_partials(const DevState* __restrict__ dp) {
  // one thread per bucket, all its outputs (8 corner volumes, or 8 corners x 3
  // drag components): each member is read once, and every output sums the
  // bucket's members in bucket order
  const DevState& d = *dp;
  if (*d.abort) return;
  constexpr int m = kKind == 0 ? 8 : 24;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= d.ndual) return;
  double acc[m];
#pragma unroll
  for (int k = 0; k < m; ++k) acc[k] = 0.0;
  // the skipped particles of a sample sit in its sink bucket, which no cell reads
  // members in groups of four: all loads of a group are issued before any
  // use (a bucket holds a few members, so this is one or two round trips)
  constexpr int kU = 4;
  const auto MEM = G((const int32_t*)d.dmem);
  const auto FR = G((const double4*)d.dfr);
  const auto FP = G((const double4*)d.fpart);
  if (!G((const uint8_t*)d.dual_sink)[b]) {
    const int32_t q1 = G((const int32_t*)d.doff)[b + 1];
    for (int32_t q0 = G((const int32_t*)d.doff)[b]; q0 < q1; q0 += kU) {
      int32_t ii[kU];
      double4 fr[kU], fp[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) ii[u] = q0 + u < q1 ? MEM[q0 + u] : -1;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        fr[u] = ii[u] >= 0 ? gld(FR + ii[u]) : make_double4(0.0, 0.0, 0.0, 0.0);
        fp[u] = kKind == 1 && ii[u] >= 0 ? gld(FP + ii[u]) : make_double4(0.0, 0.0, 0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (ii[u] < 0) break;
#pragma unroll
        for (int corner = 0; corner < 8; ++corner) {
          const double w = corner_w(fr[u], corner & 1, (corner >> 1) & 1, corner >> 2);
          if (kKind == 0) {
            acc[corner] += w * fr[u].w;
          } else {
            acc[3 * corner] += w * fp[u].x;
            acc[3 * corner + 1] += w * fp[u].y;
            acc[3 * corner + 2] += w * fp[u].z;
          }
        }
      }
    }
  }
  const auto PART = G(d.dpart);
#pragma unroll
  for (int k = 0; k < m; ++k) PART[m * b + k] = acc[k];
}

// per fluid cell: fixed-order sum of the corner partials of the adjacent buckets
template <int kKind>
__global__ void k_fluid_cells(const DevState* __restrict__ dp) {
  const DevState& d = *dp;
  if (*d.abort) return;
  int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= d.ncell) return;
  const SampleConst& c = sample_const(d.sc, d.cell_sample[C]);
  int64_t l = C - c.cell_base;
  const int cc[3] = {(int)(l % c.gn[0]), (int)((l / c.gn[0]) % c.gn[1]), (int)(l / ((int64_t)c.gn[0] * c.gn[1]))};
  const int cen = c.voidfrac == DEM_VOID_CENTROID;
  int lo[3], hi[3];
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
        // corner of this cell in the bucket; a direction of one cell folds
        // both trilinear weights onto the only cell
        int kx = (cen || c.gn[0] == 1) ? -1 : cc[0] - Dx;
        int ky = (cen || c.gn[1] == 1) ? -1 : cc[1] - Dy;
        int kz = (cen || c.gn[2] == 1) ? -1 : cc[2] - Dz;
        for (int cz = 0; cz < 2; ++cz) {
          if (kz >= 0 ? cz != kz : (cen && cz != 0)) continue;
          for (int cy = 0; cy < 2; ++cy) {
            if (ky >= 0 ? cy != ky : (cen && cy != 0)) continue;
            for (int cx = 0; cx < 2; ++cx) {
              if (kx >= 0 ? cx != kx : (cen && cx != 0)) continue;
              int corner = (cz << 2) | (cy << 1) | cx;
              if (kKind == 0) {
                s[0] += d.dpart[8 * key + corner];
              } else {
                s[0] += d.dpart[24 * key + 3 * corner];
                s[1] += d.dpart[24 * key + 3 * corner + 1];
                s[2] += d.dpart[24 * key + 3 * corner + 2];
              }
            }
          }
        }
      }
  if (kKind == 0) {
    double eps = s[0] / c.vcell;
    d.eps[C] = eps;
    double nn = 1.0 - eps;
    if (nn < c.n_min) nn = c.n_min;
    if (nn > 1.0) nn = 1.0;
    d.cell_n[C] = nn;
    for (int k = 0; k < 3; ++k) d.cell_u[3 * C + k] = c.u_superficial ? d.u_in[3 * C + k] / nn : d.u_in[3 * C + k];
  } else {
    for (int k = 0; k < 3; ++k) d.fdc[3 * C + k] = s[k] / c.vcell;
  }
}

// Di Felice drag (eq 8-11) with the coarse-grained rule, buoyancy and the
// dynamic pressure gradient; trilinear interpolation of n, u, grad p
// porosity, fluid velocity and dynamic pressure gradient at particle i, with
// the weights of its deposition (trilinear over the 8 surrounding cell centres,
// or its own cell for centroid deposition)
__device__ inline void particle_fluid(const DevState& d, const SampleConst& c, int64_t i, double& np, double u[3],
                                      double gp[3]) {
  const int cen = c.voidfrac == DEM_VOID_CENTROID;
  int64_t l = d.dkey[i] - c.dual_base;
  int b[3] = {(int)(l % c.dn[0]), (int)((l / c.dn[0]) % c.dn[1]), (int)(l / ((int64_t)c.dn[0] * c.dn[1]))};
  double4 fr = d.dfr[i];
  double f[3] = {fr.x, fr.y, fr.z};
  np = 0.0;
  for (int k = 0; k < 3; ++k) { u[k] = 0.0; gp[k] = 0.0; }
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
}

// Learned-closure features of particle i (an extension): porosity at the
// particle, slip speed |u - v|, particle Reynolds number of the drag law
// (eq 11, fine diameter d/k), k, and the mean of delta/R* over the pairs that
// took part in the last force evaluation, with their count.  Dead: zeros.
template <typename R>
__global__ void k_closure_features(const DevState* __restrict__ dp, int buf) {
  const DevState& d = *dp;
  if (*d.abort) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  double* f = d.cfeat + 6 * i;
  const SampleConst& c = sample_const(d.sc, d.sample[i]);
  if (!d.alive[buf][i] || !c.fluid_on) {
    for (int k = 0; k < 6; ++k) f[k] = 0.0;
    return;
  }
  double np, u[3], gp[3];
  particle_fluid(d, c, i, np, u, gp);
  const double4 v = d.vel[buf][i];
  const double4 pi = d.xr[buf][i];
  double s[3] = {u[0] - v.x, u[1] - v.y, u[2] - v.z};
  double sm = sqrt((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
  double sum = 0.0, cnt = 0.0;
  const auto AL = G((const uint8_t*)d.alive[buf]);
  const auto FL = G((const uint8_t*)d.pfl[buf]);
  const auto XR = G((const double4*)d.xr[buf]);
  const auto NBR = G((const int32_t*)d.nbr);
  const auto NSL = G((const int32_t*)d.nslot);
  const int32_t e1 = G((const int32_t*)d.nrow)[i + 1];
  // row entries four at a time: all loads of a group are issued before any
  // use; the sum runs in row order
  constexpr int kU = 4;
  for (int32_t e0 = G((const int32_t*)d.nrow)[i]; e0 < e1; e0 += kU) {
    int32_t jj[kU], ss[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool ok = e0 + u < e1;
      jj[u] = ok ? NBR[e0 + u] : -1;
      ss[u] = ok ? NSL[e0 + u] : 0;
    }
    uint8_t a[kU], fp[kU];
    double4 pj[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool ok = jj[u] >= 0;
      a[u] = ok ? AL[jj[u]] : 0;
      fp[u] = ok ? FL[ss[u]] : 0;
      pj[u] = ok ? gld(XR + jj[u]) : make_double4(0.0, 0.0, 0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (!a[u] || !(fp[u] & 3)) continue;
      double dx = pj[u].x - pi.x, dy = pj[u].y - pi.y, dz = pj[u].z - pi.z;
      double delta = (pi.w + pj[u].w) - sqrt((dx * dx + dy * dy) + dz * dz);
      double Rs = pi.w * pj[u].w / (pi.w + pj[u].w);
      sum += delta / Rs;
      cnt += 1.0;
    }
  }
  f[0] = np;
  f[1] = sm;
  f[2] = c.rho_f * (2.0 * pi.w / c.kcg) * sm / c.mu_f;
  f[3] = c.kcg;
  f[4] = cnt > 0.0 ? sum / cnt : 0.0;
  f[5] = cnt;
}

template <typename R>
__global__ void k_fluid_drag(const DevState* __restrict__ dp, int buf) {
  const DevState& d = *dp;
  if (*d.abort) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const SampleConst& c = sample_const(d.sc, d.sample[i]);
  if (!d.alive[buf][i] || !c.fluid_on) {
    ((R4<R>*)d.fdr)[i] = mk4<R>(0, 0, 0, 0);
    d.fpart[i] = make_double4(0, 0, 0, 0);
    return;
  }
  double np, u[3], gp[3];
  particle_fluid(d, c, i, np, u, gp);
  const double4 fr = d.dfr[i];
  const double4 v = d.vel[buf][i];
  const double r = d.xr[buf][i].w;
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

template <typename R> void launch_fluid(DevState& d, int buf, hipStream_t s) {
  hipLaunchKernelGGL(k_fluid_key, dim3(nblk(d.n)), dim3(kBlock), 0, s, d.self, buf);
  launch_bucket_sort((const uint32_t*)d.dkey, d.n, d.ndual, nullptr, d.dcnt, d.doff, d.dfill, d.dmem_tmp,
                     d.dmem, d.scan_tmp, d.dual_sink, d.abort, s);
  hipLaunchKernelGGL(k_fluid_partials<0>, dim3(nblk(d.ndual, 64)), dim3(64), 0, s, d.self);
  if (d.ncell > 0) hipLaunchKernelGGL(k_fluid_cells<0>, dim3(nblk(d.ncell)), dim3(kBlock), 0, s, d.self);
  if (d.closure_on) {
    hipLaunchKernelGGL(k_closure_features<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d.self, buf);
    launch_closure_infer(d, s);
  }
  hipLaunchKernelGGL(k_fluid_drag<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d.self, buf);
  hipLaunchKernelGGL(k_fluid_partials<1>, dim3(nblk(d.ndual, 64)), dim3(64), 0, s, d.self);
  if (d.ncell > 0) hipLaunchKernelGGL(k_fluid_cells<1>, dim3(nblk(d.ncell)), dim3(kBlock), 0, s, d.self);
}
template void launch_fluid<double>(DevState&, int, hipStream_t);
template void launch_fluid<float>(DevState&, int, hipStream_t);

}  // namespace dem
