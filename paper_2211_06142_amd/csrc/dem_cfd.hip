// dem_cfd.hip -- the fluid side of the coupling: model A (arXiv:2211.06142
// section 2.2, eq 6) in its drag-dominated limit.
//
// In a packed bed the unsteady, advective and viscous terms of eq 6 are small
// against the pressure gradient and the particle-fluid force, the negative of
// the cell drag source of eq 7.  The momentum balance then reads
// n grad(p) = -beta (u - v_s), with beta the cell's drag force per volume and
// unit slip, and for a bed at rest relative to the fluid continuity
// div(n u) = 0 becomes the pressure equation div(K grad p) = 0, K = n^2 / beta,
// for the dynamic pressure.  beta is taken from the latest coupling evaluation
// (|drag source| / |interstitial velocity|: the drag law linearised at the
// current slip) plus 12 mu_f / h_min^2 (viscous flow between plates one cell
// apart), which keeps particle-free cells finite.
//
// Cell-centred finite volumes: the flux from cell a to its neighbour b is
// T (p_a - p_b), T = (face area / centre distance) * 2 K_a K_b / (K_a + K_b),
// none through the grid's outer boundary or into a solid cell.  Cell kinds:
// open (unknown pressure), fixed pressure, solid.  Solved by conjugate
// gradients with the diagonal as preconditioner; every dot product is a
// fixed-order two-pass reduction, so the iterates are reproducible bit for bit.
#include "dem_device.h"

namespace dem {

constexpr int kCfdOpen = DEM_CELL_OPEN, kCfdFixed = DEM_CELL_PRESSURE, kCfdSolid = DEM_CELL_SOLID;

struct CfdBuf {
  const int8_t* kind;     // ncell
  const double* pfix;     // ncell
  double *K, *diag, *x, *r, *z, *p, *q, *b;   // ncell
  double* part;           // block partial sums (3 per block)
  double* scal;           // rz, alpha, beta, rr, bb, pq
  int64_t nblk;
};

__device__ inline void cell_ijk(const SampleConst& c, int64_t l, int& ix, int& iy, int& iz) {
  ix = (int)(l % c.gn[0]);
  iy = (int)((l / c.gn[0]) % c.gn[1]);
  iz = (int)(l / ((int64_t)c.gn[0] * c.gn[1]));
}

// neighbour `f` (0..5: -x, +x, -y, +y, -z, +z) of cell C, or -1 outside the grid
__device__ inline int64_t cell_nb(const SampleConst& c, int64_t C, int ix, int iy, int iz, int f) {
  const int ax = f >> 1, sg = (f & 1) ? 1 : -1;
  const int j[3] = {ix + (ax == 0 ? sg : 0), iy + (ax == 1 ? sg : 0), iz + (ax == 2 ? sg : 0)};
  if (j[0] < 0 || j[1] < 0 || j[2] < 0 || j[0] >= c.gn[0] || j[1] >= c.gn[1] || j[2] >= c.gn[2]) return -1;
  return c.cell_base + ((int64_t)j[2] * c.gn[1] + j[1]) * c.gn[0] + j[0];
}

__device__ inline double face_geo(const SampleConst& c, int ax) {
  return ax == 0 ? c.gh[1] * c.gh[2] / c.gh[0] : ax == 1 ? c.gh[0] * c.gh[2] / c.gh[1] : c.gh[0] * c.gh[1] / c.gh[2];
}

__device__ inline double face_T(const SampleConst& c, int ax, double Ka, double Kb) {
  return face_geo(c, ax) * (2.0 * Ka * Kb / (Ka + Kb));
}

// K, the diagonal, the right-hand side (fixed neighbours), the start x and r = b - A x
// is done in two kernels: coefficients first (K of every cell), then the system rows
__global__ void k_cfd_coeff(DevState d, CfdBuf B) {
  const int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= d.ncell) return;
  const SampleConst& c = sample_const(d.sc, d.cell_sample[C]);
  const double n = d.cell_n[C];
  const double fm = sqrt((d.fdc[3 * C] * d.fdc[3 * C] + d.fdc[3 * C + 1] * d.fdc[3 * C + 1]) + d.fdc[3 * C + 2] * d.fdc[3 * C + 2]);
  const double um = sqrt((d.cell_u[3 * C] * d.cell_u[3 * C] + d.cell_u[3 * C + 1] * d.cell_u[3 * C + 1]) +
                         d.cell_u[3 * C + 2] * d.cell_u[3 * C + 2]);
  const double beta = um > 0.0 ? fm / um : 0.0;
  const double hmin = fmin(c.gh[0], fmin(c.gh[1], c.gh[2]));
  const double beta_open = 12.0 * c.mu_f / (hmin * hmin);
  B.K[C] = n * n / (beta + beta_open);
}

__global__ void k_cfd_rows(DevState d, CfdBuf B, int warm) {
  const int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= d.ncell) return;
  if (B.kind[C] != kCfdOpen) {
    B.diag[C] = 1.0; B.b[C] = 0.0; B.x[C] = 0.0;
    return;
  }
  const SampleConst& c = sample_const(d.sc, d.cell_sample[C]);
  int ix, iy, iz;
  cell_ijk(c, C - c.cell_base, ix, iy, iz);
  double dg = 0.0, rhs = 0.0;
  for (int f = 0; f < 6; ++f) {
    const int64_t j = cell_nb(c, C, ix, iy, iz, f);
    if (j < 0 || B.kind[j] == kCfdSolid) continue;
    const double T = face_T(c, f >> 1, B.K[C], B.K[j]);
    dg += T;
    if (B.kind[j] == kCfdFixed) rhs += T * B.pfix[j];
  }
  B.diag[C] = dg > 0.0 ? dg : 1.0;
  B.b[C] = rhs;
  if (!warm) B.x[C] = 0.0;
}

// y = A v over the open cells (other cells 0); part: block sums of v . y
__global__ __launch_bounds__(256) void k_cfd_apply(DevState d, CfdBuf B, const double* v, double* y, int with_dot) {
  __shared__ double sh[256];
  const int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0, dot = 0.0;
  if (C < d.ncell && B.kind[C] == kCfdOpen) {
    const SampleConst& c = sample_const(d.sc, d.cell_sample[C]);
    int ix, iy, iz;
    cell_ijk(c, C - c.cell_base, ix, iy, iz);
    double dg = 0.0;
    for (int f = 0; f < 6; ++f) {
      const int64_t j = cell_nb(c, C, ix, iy, iz, f);
      if (j < 0 || B.kind[j] == kCfdSolid) continue;
      const double T = face_T(c, f >> 1, B.K[C], B.K[j]);
      dg += T;
      if (B.kind[j] == kCfdOpen) acc -= T * v[j];
    }
    acc += dg * v[C];
    dot = v[C] * acc;
  }
  if (C < d.ncell) y[C] = acc;
  if (!with_dot) return;
  sh[threadIdx.x] = dot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) B.part[blockIdx.x * 3] = sh[0];
}

// block partial sums of up to three products (fixed tree in LDS)
__device__ inline void block_sums3(double a0, double a1, double a2, double* part) {
  __shared__ double sh[3][256];
  sh[0][threadIdx.x] = a0; sh[1][threadIdx.x] = a1; sh[2][threadIdx.x] = a2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

// sums of the block partials in order (one block); mode 0: start (rz, rr, bb);
// 1: alpha = rz / pq; 2: beta = rz_new / rz, rr
__global__ __launch_bounds__(256) void k_cfd_final(CfdBuf B, int mode) {
  __shared__ double sh[3][256];
  double a[3] = {0.0, 0.0, 0.0};
  for (int64_t k = threadIdx.x; k < B.nblk; k += 256)
    for (int q = 0; q < 3; ++q) a[q] += B.part[k * 3 + q];
  for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] = a[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double* S = B.scal;
  if (mode == 0) {
    S[0] = sh[0][0]; S[3] = sh[1][0]; S[4] = sh[2][0];
  } else if (mode == 1) {
    S[5] = sh[0][0];
    S[1] = S[5] != 0.0 ? S[0] / S[5] : 0.0;
  } else {
    const double rz = sh[0][0];
    S[2] = S[0] != 0.0 ? rz / S[0] : 0.0;
    S[0] = rz;
    S[3] = sh[1][0];
  }
}

// r = b - r (r holds A x), z = r / diag, p = z; partials rz, rr, bb
__global__ __launch_bounds__(256) void k_cfd_start(DevState d, CfdBuf B) {
  const int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  if (C < d.ncell) {
    double r = 0.0, z = 0.0;
    if (B.kind[C] == kCfdOpen) {
      r = B.b[C] - B.r[C];
      z = r / B.diag[C];
      bb = B.b[C] * B.b[C];
    }
    B.r[C] = r; B.z[C] = z; B.p[C] = z;
    rz = r * z; rr = r * r;
  }
  block_sums3(rz, rr, bb, B.part);
}

// x += alpha p, r -= alpha q, z = r / diag; partials rz, rr
__global__ __launch_bounds__(256) void k_cfd_update(DevState d, CfdBuf B) {
  const int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (C < d.ncell && B.kind[C] == kCfdOpen) {
    const double al = B.scal[1];
    B.x[C] += al * B.p[C];
    const double r = B.r[C] - al * B.q[C];
    const double z = r / B.diag[C];
    B.r[C] = r; B.z[C] = z;
    rz = r * z; rr = r * r;
  }
  block_sums3(rz, rr, 0.0, B.part);
}

__global__ void k_cfd_dir(DevState d, CfdBuf B) {
  const int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (C < d.ncell && B.kind[C] == kCfdOpen) B.p[C] = B.z[C] + B.scal[2] * B.p[C];
}

// pressure of every cell, cell-centred superficial velocity (mean of the two
// face fluxes of each axis; a missing face carries none) and pressure gradient
// (mean of the available one-sided differences)
__global__ void k_cfd_fields(DevState d, CfdBuf B, double* P, double* U, double* GP) {
  const int64_t C = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= d.ncell) return;
  const int kd = B.kind[C];
  const double pc = kd == kCfdOpen ? B.x[C] : kd == kCfdFixed ? B.pfix[C] : 0.0;
  P[C] = pc;
  if (kd == kCfdSolid) {
    for (int a = 0; a < 3; ++a) { U[3 * C + a] = 0.0; GP[3 * C + a] = 0.0; }
    return;
  }
  const SampleConst& c = sample_const(d.sc, d.cell_sample[C]);
  int ix, iy, iz;
  cell_ijk(c, C - c.cell_base, ix, iy, iz);
  for (int a = 0; a < 3; ++a) {
    double flux[2] = {0.0, 0.0}, gsum = 0.0;
    int ng = 0;
    for (int s = 0; s < 2; ++s) {
      const int64_t j = cell_nb(c, C, ix, iy, iz, 2 * a + s);
      if (j < 0 || B.kind[j] == kCfdSolid) continue;
      const double pj = B.kind[j] == kCfdOpen ? B.x[j] : B.pfix[j];
      const double g = (s ? 1.0 : -1.0) * (pj - pc) / c.gh[a];
      const double Kf = 2.0 * B.K[C] * B.K[j] / (B.K[C] + B.K[j]);
      flux[s] = -Kf * g;
      gsum += g;
      ++ng;
    }
    U[3 * C + a] = 0.5 * (flux[0] + flux[1]);
    GP[3 * C + a] = ng ? gsum / ng : 0.0;
  }
}

dem_status cfd_solve(DevState& d, const int8_t* kind, const double* pfix, double* work, int64_t nwork, int warm,
                     int max_iter, double rel_tol, double* P, double* U, double* GP, int* iters, double* rel_res,
                     double* h_scal, hipStream_t s) {
  const int64_t nc = d.ncell;
  CfdBuf B{};
  B.kind = kind;
  B.pfix = pfix;
  B.nblk = nblk(nc);
  double* w = work;
  B.K = w; w += nc; B.diag = w; w += nc; B.x = w; w += nc; B.r = w; w += nc; B.z = w; w += nc;
  B.p = w; w += nc; B.q = w; w += nc; B.b = w; w += nc;
  B.part = w; w += 3 * B.nblk;
  B.scal = w; w += 8;
  if (w - work > nwork) return DEM_E_NOMEM;
  const dim3 g(nblk(nc)), t(kBlock);
  hipLaunchKernelGGL(k_cfd_coeff, g, t, 0, s, d, B);
  hipLaunchKernelGGL(k_cfd_rows, g, t, 0, s, d, B, warm);
  hipLaunchKernelGGL(k_cfd_apply, g, t, 0, s, d, B, B.x, B.r, 0);
  hipLaunchKernelGGL(k_cfd_start, g, t, 0, s, d, B);
  hipLaunchKernelGGL(k_cfd_final, dim3(1), t, 0, s, B, 0);
  int it = 0;
  double rel = 0.0;
  for (;;) {
    if (hipMemcpyAsync(h_scal, B.scal, 8 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return DEM_E_DEVICE;
    const double bb = h_scal[4], rr = h_scal[3];
    rel = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
    if (!(rel > rel_tol) || it >= max_iter) break;
    // a batch of iterations between host checks
    const int nb = std::min(16, max_iter - it);
    for (int k = 0; k < nb; ++k) {
      hipLaunchKernelGGL(k_cfd_apply, g, t, 0, s, d, B, B.p, B.q, 1);
      hipLaunchKernelGGL(k_cfd_final, dim3(1), t, 0, s, B, 1);
      hipLaunchKernelGGL(k_cfd_update, g, t, 0, s, d, B);
      hipLaunchKernelGGL(k_cfd_final, dim3(1), t, 0, s, B, 2);
      hipLaunchKernelGGL(k_cfd_dir, g, t, 0, s, d, B);
    }
    it += nb;
  }
  hipLaunchKernelGGL(k_cfd_fields, g, t, 0, s, d, B, P, U, GP);
  if (hipGetLastError() != hipSuccess) return DEM_E_DEVICE;
  if (iters) *iters = it;
  if (rel_res) *rel_res = rel;
  return DEM_OK;
}

int64_t cfd_work_doubles(int64_t ncell) { return 8 * ncell + 3 * (int64_t)nblk(ncell) + 8; }

}  // namespace dem
