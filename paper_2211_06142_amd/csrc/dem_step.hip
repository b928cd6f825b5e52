// dem_step.hip -- the fused DEM step.
//
// k_prologue: first half kick and drift of the first step of a call (eq 1-2,
// velocity Verlet), outlet removal, rebuild trigger.
// k_step: a group of lanes per particle.  The particle walks its full neighbour row
// and evaluates every contact in the pair's canonical orientation (owner =
// lower sorted index, n from owner to partner), so both partners compute the
// bit-identical pair force and Newton's third law holds exactly without
// atomics or force records; only the owner writes the pair's new history.
// Then walls, gravity, the held fluid force, the second half kick, and -
// unless the step ends the call - the next step's first half kick, drift,
// outlet removal and rebuild trigger.  State and pair history are read from
// buffer `in` and written to buffer `out`.
#include "dem_device.h"

namespace dem {

// Produced sand (eq 40): the removed mass, rounded once to the sample's fixed
// point, is added to the sample's counter and to the counter of its size class
// (by the fine-scale diameter d/k the grain stands for).
__device__ inline void count_removal(const DevState& d, const SampleConst& c, int s, double r) {
  const double m = c.rho * (4.0 / 3.0) * M_PI * r * r * r;
  const unsigned long long q = __double2ull_rn(m * c.pm_scale);
  atomicAdd(&d.produced_fx[s], q);
  if (d.ncls > 0) {
    const double df = 2.0 * r / c.kcg;
    int k = 0;
    while (k + 1 < d.ncls && df >= d.cls_edge[k + 1]) ++k;
    atomicAdd(&d.produced_cls[(int64_t)s * DEM_MAX_SIZE_CLASSES + k], q);
  }
}

// (xref: the particle's position at the last rebuild)
template <typename R>
__device__ inline void finish_drift(const DevState& d, const SampleConst& c, int s, int64_t i, int out,
                                    int64_t next_step, double4 p, double4 v, R4<R> w, const double4& xref) {
  const double dt = d.dt;
  double sx = dt * v.x, sy = dt * v.y, sz = dt * v.z;
  p.x += sx; p.y += sy; p.z += sz;
  const double hs = 0.5 * c.skin;
  if ((sx * sx + sy * sy) + sz * sz >= hs * hs) {
    atomicOr(d.status, (int)kStTooFast);
    atomicOr(d.abort, 1);
  }
  gst(G(d.xr[out]) + i, p);
  gst(G(d.vel[out]) + i, v);
  gst(G((R4<R>*)d.omg[out]) + i, w);
  uint8_t alive = 1;
  bool leaves = false;
  if (c.outlet_kind == DEM_OUTLET_CAVITY) {
    double ex = p.x - c.outlet[0], ey = p.y - c.outlet[1];
    double rc = c.outlet[2];
    leaves = ex * ex + ey * ey < rc * rc;
  } else if (c.outlet_kind == DEM_OUTLET_ABOVE) {
    leaves = p.z > c.outlet[3];
  }
  if (leaves) {
    alive = 0;
    count_removal(d, c, s, p.w);
    gst(G((R4<R>*)d.frc) + i, mk4<R>(0, 0, 0, 0));
    gst(G((R4<R>*)d.trq) + i, mk4<R>(0, 0, 0, 0));
  }
  G(d.alive[out])[i] = alive;
  if (alive) {
    const double4& q = xref;
    double ux = p.x - q.x, uy = p.y - q.y, uz = p.z - q.z;
    if ((ux * ux + uy * uy) + uz * uz > hs * hs) {
      atomicOr(d.abort, 1);
      atomicMin(d.abort_step, (int)next_step);
    }
  }
}

template <typename R>
__global__ void k_prologue(DevState d, StepArgs a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int in = a.in, out = a.out;
  double4 p = d.xr[in][i];
  double4 v = d.vel[in][i];
  R4<R> w = ((const R4<R>*)d.omg[in])[i];
  if (!d.alive[in][i]) {
    d.xr[out][i] = p;
    d.vel[out][i] = v;
    ((R4<R>*)d.omg[out])[i] = w;
    d.alive[out][i] = 0;
    return;
  }
  const int s = d.sample[i];
  const SampleConst& c = sample_const(d.sc, s);
  const R4<R> F = ((const R4<R>*)d.frc)[i];
  const R4<R> T = ((const R4<R>*)d.trq)[i];
  const double hdt = 0.5 * d.dt;
  v.x += hdt * (double)F.x * v.w;
  v.y += hdt * (double)F.y * v.w;
  v.z += hdt * (double)F.z * v.w;
  const R hdtR = (R)hdt;
  w.x += hdtR * T.x * w.w;
  w.y += hdtR * T.y * w.w;
  w.z += hdtR * T.z * w.w;
  finish_drift<R>(d, c, s, i, out, a.step, p, v, w, d.xref[i]);
}

template <typename R> void launch_prologue(DevState& d, StepArgs a, hipStream_t s) {
  hipLaunchKernelGGL(k_prologue<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d, a);
}
template void launch_prologue<double>(DevState&, StepArgs, hipStream_t);
template void launch_prologue<float>(DevState&, StepArgs, hipStream_t);

// Lanes per particle: a group of G lanes (1, 2, 4, 8 or 16, chosen per context)
// shares one particle's row; lane s evaluates entries s, s + G, ... and the
// group sums its partial forces
// with a fixed xor butterfly (every lane ends with the bit-identical total).
template <typename R, int kGroup>
__device__ inline R group_sum(R v) {
#pragma unroll
  for (int off = kGroup / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kGroup);
  return v;
}

// Per-wave work queue of the step kernel, in LDS.  A round collects the live
// entries (touching or bonded pairs with a live partner) of up to kKCap row
// positions of every lane, at most kQCap of them, in (row position, lane)
// order; the wave then evaluates them densely, each lane taking every
// (number of lanes)-th entry, and finally each lane adds up its own entries in
// row order, so the sum of every particle is formed as with one lane walking
// its row.  An entry's contribution is its force (sign applied) and its
// torque (r (n x F_t) + sign x rolling torque).
// The wave's own particles (position, velocity, angular velocity) are staged
// there too.
constexpr int kQCap = 128;
constexpr int kKCap = 32;
template <typename R, int kGroup> struct WaveQueue {
  static constexpr int kP = 64 / kGroup;   // particles of a wave
  double4 sx[kP], sv[kP];
  R4<R> sw[kP];
  int32_t j[kQCap], p[kQCap];
  uint8_t li[kQCap];
  R f[6][kQCap];
  uint64_t ball[kKCap];   // lanes with a live entry at each row position of the round
  int32_t base[kKCap];    // queue slot of the first of them
};

// What the end of a particle's step reads besides its own state: its wall
// entries and the held fluid force, loaded at the start of the step together
// with the particle's own state (their loads do not wait for the row walk).
template <typename R> struct FinishIn {
  int32_t w0, w1;   // wall entries [w0, w1)
  R4<R> fd;         // held fluid force (zero without fluid)
  double4 xref;     // position at the last rebuild
};
template <typename R>
__device__ __forceinline__ FinishIn<R> finish_in(const DevState& d, const SampleConst& c, int64_t i) {
  FinishIn<R> q;
  q.w0 = G((const int32_t*)d.wrow)[i];
  q.w1 = G((const int32_t*)d.wrow)[i + 1];
  q.fd = c.fluid_on ? gld(G((const R4<R>*)d.fdr) + i) : mk4<R>(0, 0, 0, 0);
  q.xref = gld(G((const double4*)d.xref) + i);
  return q;
}

// Walls, the group's fixed-order sum, gravity, the held fluid force, the
// second half kick and - unless the step ends the call - the next step's
// first half kick, drift and outlet (every lane of the group calls it with its
// partial sums F, T of the pair contributions).
template <typename R, int kGroup>
__device__ __forceinline__ void particle_finish(const DevState& d, const StepArgs& a, const SampleConst& c,
                                                const LawK<R>& lk, int64_t i, int sub, int s, const double4& pi,
                                                double4 v, R4<R> w, R F[3], R T[3], const FinishIn<R>& fin) {
  const int out = a.out;
  const R r = (R)pi.w;
  // walls: Hertz with R* = r and m* = m (rigid, static); entries private to i
  const double m = c.rho * (4.0 / 3.0) * M_PI * pi.w * pi.w * pi.w;
  const auto WDT = G((R4<R>*)d.wdt);
  const auto WFL = G((uint8_t*)d.wfl);
  const auto WFR = G((R4<R>*)d.wfrc);
  const int32_t w1 = fin.w1;
  for (int32_t e = fin.w0 + sub; e < w1; e += kGroup) {
    R4<R> h4 = gld((gptr<const R4<R>>)(WDT + e));
    double sd, nw[3];
    const Wall& wl = c.walls[G((const int32_t*)d.wid)[e]];
    if (!wall_geom(wl, pi.x, pi.y, pi.z, sd, nw) || !(sd < pi.w)) {
      gst(WDT + e, mk4<R>(0, 0, 0, 0));
      WFL[e] = 0;
      gst(WFR + e, mk4<R>(0, 0, 0, 0));
      continue;
    }
    const R delta = (R)(pi.w - sd);
    const R n[3] = {(R)(-nw[0]), (R)(-nw[1]), (R)(-nw[2])};
    const R wr[3] = {r * w.x, r * w.y, r * w.z};
    const R vrel[3] = {(R)v.x + (wr[1] * n[2] - wr[2] * n[1]), (R)v.y + (wr[2] * n[0] - wr[0] * n[2]),
                       (R)v.z + (wr[0] * n[1] - wr[1] * n[0])};
    const R wrel[3] = {w.x, w.y, w.z};
    R h[3] = {h4.x, h4.y, h4.z};
    LawOut<R> o;
    contact_law<R>(lk, 0, delta, r, (R)m, (R)0, (R)0, n, vrel, wrel, h, (R)d.dt, true, o);
    F[0] += o.F[0]; F[1] += o.F[1]; F[2] += o.F[2];
    T[0] += r * o.c[0] + o.Tr[0];
    T[1] += r * o.c[1] + o.Tr[1];
    T[2] += r * o.c[2] + o.Tr[2];
    gst(WDT + e, mk4<R>(h[0], h[1], h[2], (R)0));
    WFL[e] = 2;
    gst(WFR + e, mk4<R>(o.F[0], o.F[1], o.F[2], (R)0));
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    F[k] = group_sum<R, kGroup>(F[k]);
    T[k] = group_sum<R, kGroup>(T[k]);
  }
  if (sub != 0) return;
  F[0] += (R)(m * c.g[0]);
  F[1] += (R)(m * c.g[1]);
  F[2] += (R)(m * c.g[2]);
  if (c.fluid_on) {
    F[0] += fin.fd.x; F[1] += fin.fd.y; F[2] += fin.fd.z;
  }
  if (!isfinite(F[0] + F[1] + F[2] + T[0] + T[1] + T[2])) {
    atomicOr(d.status, (int)kStNonFinite);
    atomicOr(d.abort, 1);
  }
  // second half kick of this step
  const double hdt = 0.5 * d.dt;
  v.x += hdt * (double)F[0] * v.w;
  v.y += hdt * (double)F[1] * v.w;
  v.z += hdt * (double)F[2] * v.w;
  const R hdtR = (R)hdt;
  w.x += hdtR * T[0] * w.w;
  w.y += hdtR * T[1] * w.w;
  w.z += hdtR * T[2] * w.w;
  if (a.final_step) {
    gst(G(d.xr[out]) + i, pi);
    gst(G(d.vel[out]) + i, v);
    gst(G((R4<R>*)d.omg[out]) + i, w);
    G(d.alive[out])[i] = 1;
    gst(G((R4<R>*)d.frc) + i, mk4<R>(F[0], F[1], F[2], (R)0));
    gst(G((R4<R>*)d.trq) + i, mk4<R>(T[0], T[1], T[2], (R)0));
    return;
  }
  // first half kick and drift of the next step
  v.x += hdt * (double)F[0] * v.w;
  v.y += hdt * (double)F[1] * v.w;
  v.z += hdt * (double)F[2] * v.w;
  w.x += hdtR * T[0] * w.w;
  w.y += hdtR * T[1] * w.w;
  w.z += hdtR * T[2] * w.w;
  finish_drift<R>(d, c, s, i, out, a.step + 1, pi, v, w, fin.xref);
}

// Everything of one live particle; `s` is its sample, uniform over the active
// lanes, `lane` the lane in the wave and i0 the wave's first particle.
template <typename R, int kGroup>
__device__ __forceinline__ void particle_step(const DevState& d, const StepArgs& a, int64_t i, int sub, int s,
                                              int lane, int64_t i0, WaveQueue<R, kGroup>& Q) {
  const int in = a.in, out = a.out;
  const SampleConst& c = sample_const(d.sc, s);
  const LawK<R> lk = law_k<R>(c);
  const auto X = G((const double4*)d.xr[in]);
  const auto V = G((const double4*)d.vel[in]);
  const auto W = G((const R4<R>*)d.omg[in]);
  const auto AL = G((const uint8_t*)d.alive[in]);
  const auto Hin = G((const R4<R>*)d.hdt[in]);
  const auto Hout = G((R4<R>*)d.hdt[out]);
  const auto Fin = G((const uint8_t*)d.pfl[in]);
  const auto Fout = G((uint8_t*)d.pfl[out]);
  const auto NBR = G((const int32_t*)d.nbr);
  const auto NSL = G((const int32_t*)d.nslot);
  const auto CC = G((const double*)d.ccoh);
  const bool rolling = d.rolling != 0;
  const uint8_t li = (uint8_t)(lane / kGroup);
  if (sub == 0) {
    Q.sx[li] = gld(X + i);
    Q.sv[li] = gld(V + i);
    Q.sw[li] = gld(W + i);
  }
  wave_lds_sync();
  R F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  const int32_t e0 = G((const int32_t*)d.nrow)[i] + sub;
  const int32_t e1 = G((const int32_t*)d.nrow)[i + 1];
  const int nk = e0 < e1 ? (e1 - e0 + kGroup - 1) / kGroup : 0;   // row positions of this lane
  const uint64_t below = (1ull << lane) - 1;
  const uint64_t live = __ballot(1);
  const bool leader = (live & below) == 0;
  const int nact = __popcll(live), rank = __popcll(live & below);
  for (int k0 = 0; __ballot(k0 < nk);) {
    // collect: a pair that is neither touching nor bonded, or whose partner
    // is gone, gets its history cleared here (by its owner, the lower index)
    // The partner and pair slot of the next row position are fetched one
    // position ahead, and the tests below use every load unconditionally, so
    // a row position costs one memory round trip.
    int total = 0, kk = 0;
    int32_t jn = 0, pn = 0;
    if (k0 < nk) {
      jn = NBR[e0 + k0 * kGroup];
      pn = NSL[e0 + k0 * kGroup];
    }
    for (; kk < kKCap; ++kk) {
      const int k = k0 + kk;
      const bool has = k < nk;
      if (!__ballot(has)) break;
      const int32_t j = jn, p = pn;
      if (k + 1 < nk) {
        jn = NBR[e0 + (k + 1) * kGroup];
        pn = NSL[e0 + (k + 1) * kGroup];
      }
      bool act = false;
      if (has) {
        // read here, not held in registers across the evaluation (the empty
        // statement keeps the compiler from hoisting the read out of the loop)
        asm volatile("" ::: "memory");
        const double4 pi = Q.sx[li];
        const uint8_t alj = AL[j];
        const double4 pj = gld(X + j);
        const uint8_t fp = Fin[p];
        const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        const double cs = pi.w + pj.w;
        act = (alj != 0) & ((d2 < cs * cs) | ((fp & 1) != 0));
        if (!act && j > (int32_t)i) Fout[p] = 0;   // a clear flag: zero history, not written
      }
      const uint64_t b = __ballot(act);
      const int n = __popcll(b);
      if (total + n > kQCap) break;   // this row position opens the next round
      if (act) {
        const int q = total + __popcll(b & below);
        Q.j[q] = j;
        Q.p[q] = p;
        Q.li[q] = li;
      }
      if (leader) {
        Q.ball[kk] = b;
        Q.base[kk] = total;
      }
      total += n;
    }
    wave_lds_sync();
    // evaluate, in the pair's canonical orientation (the owner, the lower
    // index, is body A); only the owner writes the new history
    for (int q = rank; q < total; q += nact) {
      const int32_t j = Q.j[q], p = Q.p[q];
      const int la = Q.li[q];
      const int64_t ia = i0 + la;
      asm volatile("" ::: "memory");
      const double4 pa = Q.sx[la], pj = gld(X + j);
      const double4 va = Q.sv[la], vj = gld(V + j);
      const R4<R> wa = Q.sw[la], wj = gld(W + j);
      // loaded together with the flag (a clear flag's history is stale and unused)
      const R4<R> hraw = gld(Hin + p);
      const uint8_t fp = Fin[p];
      const R4<R> hp = fp ? hraw : mk4<R>(0, 0, 0, 0);
      double gam = c.gamma;
      if (d.ccoh) gam = c.gamma * sqrt(CC[ia] * CC[j]);
      const bool own = j > (int32_t)ia;
      PairOut<R> po;
      const double4 PA = own ? pa : pj, PB = own ? pj : pa;
      const double4 VA = own ? va : vj, VB = own ? vj : va;
      const R4<R> WA = own ? wa : wj, WB = own ? wj : wa;
      pair_eval<R>(lk, c.Es, d.dt, rolling, PA, PB, VA, VB, WA, WB, gam, hp, fp, po);
      if (own) {
        if (po.fl) gst(Hout + p, po.h);
        Fout[p] = po.fl;
        if (po.broke) atomicAdd(&d.broken[s], 1ull);
      }
      // a broken bond contributes +0, which leaves the sums bit for bit as
      // they are (they start at +0 and never become -0)
      R cf[6] = {0, 0, 0, 0, 0, 0};
      if (po.active) {
        const R sg = own ? (R)1 : (R)-1, ra = (R)pa.w;
        cf[0] = sg * po.o.F[0];
        cf[1] = sg * po.o.F[1];
        cf[2] = sg * po.o.F[2];
        cf[3] = ra * po.o.c[0] + sg * po.o.Tr[0];
        cf[4] = ra * po.o.c[1] + sg * po.o.Tr[1];
        cf[5] = ra * po.o.c[2] + sg * po.o.Tr[2];
      }
#pragma unroll
      for (int m = 0; m < 6; ++m) Q.f[m][q] = cf[m];
    }
    wave_lds_sync();
    // add up, each lane its own entries in row order
    for (int t = 0; t < kk; ++t) {
      const uint64_t b = Q.ball[t];
      if ((b >> lane) & 1) {
        const int q = Q.base[t] + __popcll(b & below);
        F[0] += Q.f[0][q]; F[1] += Q.f[1][q]; F[2] += Q.f[2][q];
        T[0] += Q.f[3][q]; T[1] += Q.f[4][q]; T[2] += Q.f[5][q];
      }
    }
    wave_lds_sync();
    k0 += kk;
  }
  const double4 pi = Q.sx[li];
  double4 v = Q.sv[li];
  R4<R> w = Q.sw[li];
  particle_finish<R, kGroup>(d, a, c, lk, i, sub, s, pi, v, w, F, T, finish_in<R>(d, c, i));
}

// A launch exits at entry when a rebuild is due at or before its step: the
// recorded abort step (no rebuild: a large value) is written only by an
// earlier launch or by the launch that finds it due for the NEXT step, so every
// block of one launch takes the same decision.
template <typename R, int kGroup>
// (at most 128 VGPRs, 4 waves per SIMD: 130 registers would leave 3, which
// costs the kernel a sixth of its speed)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_step(
    const DevState* __restrict__ dp, StepArgs a) {
  __shared__ WaveQueue<R, kGroup> wq[kBlock / 64];
  const DevState& d = *dp;
  if (*d.abort_step <= a.step) return;
  const int sub = threadIdx.x & (kGroup - 1);
  const int64_t i = (xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) / kGroup;
  if (i >= d.n) return;   // whole group
  const int in = a.in, out = a.out;
  if (!G((const uint8_t*)d.alive[in])[i]) {   // whole group
    if (sub == 0) {
      gst(G(d.xr[out]) + i, gld(G((const double4*)d.xr[in]) + i));
      gst(G(d.vel[out]) + i, gld(G((const double4*)d.vel[in]) + i));
      gst(G((R4<R>*)d.omg[out]) + i, gld(G((const R4<R>*)d.omg[in]) + i));
      G(d.alive[out])[i] = 0;
    }
    return;
  }
  // The lanes of a wave nearly always belong to one sample (an ensemble changes
  // sample in few waves).  Each distinct sample of the wave is served in turn,
  // so that the sample's constants are wave-uniform scalars.  The loop runs on
  // a wave-uniform mask of the lanes still to serve, so every lane stays in it
  // and runs its work under the branch of the iteration that serves its sample
  // (a lane-wise `break` would let the compiler move the work past the loop,
  // where all lanes have rejoined).  The lowest lane still to serve picks the
  // sample; it is served, so the mask shrinks every iteration.
  const int sl = G((const int32_t*)d.sample)[i];
  const int lane = threadIdx.x & 63;
  uint64_t todo = __ballot(1);
  while (todo) {
    const int first = __builtin_ctzll(todo);
    const bool mine = sl == __builtin_amdgcn_readlane(sl, first);
    if (mine)
      particle_step<R, kGroup>(d, a, i, sub, opaque_readlane(sl, first), lane, i - lane / kGroup,
                               wq[threadIdx.x >> 6]);
    todo &= ~__ballot(mine);
  }
}

// ---------------------------------------------------------------------------
// Half-pair mode: every contact law is evaluated once.  k_pairs takes one lane
// per half-pair slot (owner = lower sorted index, so the pair is in its
// canonical orientation), writes the new flag and, for a pair in contact, the
// new history and the pair's record: the force on the owner and n x F_t (and the
// rolling torque on the owner).  A pair out of contact writes its flag byte
// alone.  k_gather then walks each particle's full row in the lane layout of
// k_step and adds the records of the slots whose new flag is set, with the
// owner's sign (force and rolling torque) and its own radius (n x F_t): the very
// terms k_step adds, in the same order (the pairs out of contact add +0 there,
// which leaves a sum that starts at +0 unchanged), so the two modes agree bit
// for bit; then it finishes the particle (walls, gravity, fluid force, kicks,
// drift).  Measured at 200 000 spheres the records (24 B per slot in contact,
// read back through the row) cost less than the second evaluation.
// ---------------------------------------------------------------------------
// Both kernels are latency-bound (a few loads per lane, each depending on the
// one before), so every load whose address is known is issued in the same
// round trip as the others, ahead of the test that may make it unnecessary: the
// abort step with the slot (or the particle's own state), then everything the
// pair (or the row) needs.  An empty asm that takes the values keeps the
// compiler from sinking the loads below the early exits.
template <typename R> struct PairIn {
  double4 A, B, VA, VB;
  R4<R> WA, WB, h;
  uint8_t fl, alo, alj;
  double gam;
};

template <typename R>
__device__ __forceinline__ void half_pair(const DevState& d, const StepArgs& a, int64_t p, const PairIn<R>& q,
                                          int s) {
  const int out = a.out;
  const SampleConst& c = sample_const(d.sc, s);
  const auto Hout = G((R4<R>*)d.hdt[out]);
  const auto Fout = G((uint8_t*)d.pfl[out]);
  const bool rolling = d.rolling != 0;
  const double dx = q.B.x - q.A.x, dy = q.B.y - q.A.y, dz = q.B.z - q.A.z;
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double cs = q.A.w + q.B.w;
  if (!(q.alo && q.alj && ((d2 < cs * cs) || (q.fl & 1)))) {
    // neither touching nor bonded, or a partner gone: no force, no history
    Fout[p] = 0;
    return;
  }
  const LawK<R> lk = law_k<R>(c);
  const double gam = d.ccoh ? c.gamma * q.gam : c.gamma;
  PairOut<R> po;
  pair_eval<R>(lk, c.Es, d.dt, rolling, q.A, q.B, q.VA, q.VB, q.WA, q.WB, gam, q.h, q.fl, po);
  Fout[p] = po.fl;
  if (po.broke) atomicAdd(&d.broken[s], 1ull);
  // a bond that broke apart leaves the pair out of contact (clear flag, no record)
  if (!po.fl) return;
  gst(Hout + p, po.h);
  rec_put<R>(d.rec[0], p, po.o.F, po.o.c);
  if (rolling) gst(G((R4<R>*)d.rec[1]) + p, mk4<R>(po.o.Tr[0], po.o.Tr[1], po.o.Tr[2], (R)0));
}

template <typename R>
__global__ __launch_bounds__(256) void k_pairs(const DevState* __restrict__ dp, StepArgs a) {
  const DevState& d = *dp;
  const int64_t p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const bool has = p < d.nslots;
  const int64_t ps = has ? p : 0;   // the launch covers at least one slot
  const int in = a.in;
  // round trip 1: the abort step and the slot
  const int32_t abort_at = *G((const int32_t*)d.abort_step);
  const int32_t o = G((const int32_t*)d.sown)[ps], j = G((const int32_t*)d.spart)[ps];
  PairIn<R> q;
  q.fl = G((const uint8_t*)d.pfl[in])[ps];
  asm volatile("" ::"v"(o), "v"(j), "v"((int)q.fl), "s"(abort_at));
  if (abort_at <= a.step || !has) return;
  // round trip 2: both particles, the history, the sample
  const auto X = G((const double4*)d.xr[in]);
  const auto V = G((const double4*)d.vel[in]);
  const auto W = G((const R4<R>*)d.omg[in]);
  const auto AL = G((const uint8_t*)d.alive[in]);
  const int sl = G((const int32_t*)d.sample)[o];
  q.A = gld(X + o);
  q.B = gld(X + j);
  q.VA = gld(V + o);
  q.VB = gld(V + j);
  q.WA = gld(W + o);
  q.WB = gld(W + j);
  q.alo = AL[o];
  q.alj = AL[j];
  q.h = q.fl ? gld(G((const R4<R>*)d.hdt[in]) + p) : mk4<R>(0, 0, 0, 0);
  q.gam = d.ccoh ? sqrt(G((const double*)d.ccoh)[o] * G((const double*)d.ccoh)[j]) : 1.0;
  // serve the wave's samples in turn (constants in scalar registers; see k_step)
  uint64_t todo = __ballot(1);
  while (todo) {
    const int first = __builtin_ctzll(todo);
    const bool mine = sl == __builtin_amdgcn_readlane(sl, first);
    if (mine) half_pair<R>(d, a, p, q, opaque_readlane(sl, first));
    todo &= ~__ballot(mine);
  }
}

// a particle's own inputs of the gather, loaded in one round trip
template <typename R> struct OwnIn {
  double4 x, v;
  R4<R> w;
  int32_t e0, e1, h0, h1;
  FinishIn<R> fin;
};

template <typename R, int kGroup>
__device__ __forceinline__ void particle_gather(const DevState& d, const StepArgs& a, int64_t i, int sub, int s,
                                                const OwnIn<R>& own_in) {
  const SampleConst& c = sample_const(d.sc, s);
  const LawK<R> lk = law_k<R>(c);
  const double4 pi = own_in.x;
  const auto NSL = G((const int32_t*)d.nslot);
  const auto FL = G((const uint8_t*)d.pfl[a.out]);
  const auto RR = G((const R4<R>*)d.rec[1]);
  const bool rolling = d.rolling != 0;
  const R ra = (R)pi.w;
  // the row's owned entries (partners above i) are its tail, their slots consecutive
  const int32_t e1 = own_in.e1, h0 = own_in.h0;
  const int32_t eo = e1 - (own_in.h1 - h0);
  R F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  // four row positions per round: the slots, then the flags and the records
  // together (a record whose flag is clear was not written this step and is not
  // used), then the slots in contact added in row order
  constexpr int kU = 4;
  for (int32_t e0 = own_in.e0 + sub; e0 < e1; e0 += kU * kGroup) {
    int32_t q[kU];
    bool own[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int32_t e = e0 + u * kGroup;
      own[u] = e >= eo;
      q[u] = e < e1 ? (own[u] ? h0 + (e - eo) : NSL[e]) : -1;
    }
    uint8_t fl[kU];
    R f[kU][3], t[kU][3], tr[kU][3];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int32_t qs = q[u] >= 0 ? q[u] : 0;
      fl[u] = q[u] >= 0 ? FL[qs] : 0;
      rec_get<R>(d.rec[0], qs, f[u], t[u]);
      tr[u][0] = tr[u][1] = tr[u][2] = (R)0;
      if (rolling) {
        const R4<R> v = gld(RR + qs);
        tr[u][0] = v.x; tr[u][1] = v.y; tr[u][2] = v.z;
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (!fl[u]) continue;
      const R sg = own[u] ? (R)1 : (R)-1;
      F[0] += sg * f[u][0]; F[1] += sg * f[u][1]; F[2] += sg * f[u][2];
      T[0] += ra * t[u][0] + sg * tr[u][0];
      T[1] += ra * t[u][1] + sg * tr[u][1];
      T[2] += ra * t[u][2] + sg * tr[u][2];
    }
  }
  particle_finish<R, kGroup>(d, a, c, lk, i, sub, s, pi, own_in.v, own_in.w, F, T, own_in.fin);
}

template <typename R, int kGroup>
__global__ __launch_bounds__(256) void k_gather(const DevState* __restrict__ dp, StepArgs a) {
  const DevState& d = *dp;
  const int sub = threadIdx.x & (kGroup - 1);
  const int64_t i = (xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) / kGroup;
  if (i >= d.n) return;   // whole group
  const int in = a.in, out = a.out;
  // round trip 1: the abort step and everything of the particle's own
  const int32_t abort_at = *G((const int32_t*)d.abort_step);
  const uint8_t alive = G((const uint8_t*)d.alive[in])[i];
  const int sl = G((const int32_t*)d.sample)[i];
  OwnIn<R> q;
  q.x = gld(G((const double4*)d.xr[in]) + i);
  q.v = gld(G((const double4*)d.vel[in]) + i);
  q.w = gld(G((const R4<R>*)d.omg[in]) + i);
  q.e0 = G((const int32_t*)d.nrow)[i];
  q.e1 = G((const int32_t*)d.nrow)[i + 1];
  q.h0 = G((const int32_t*)d.hrow)[i];
  q.h1 = G((const int32_t*)d.hrow)[i + 1];
  q.fin.w0 = G((const int32_t*)d.wrow)[i];
  q.fin.w1 = G((const int32_t*)d.wrow)[i + 1];
  q.fin.fd = d.fdr ? gld(G((const R4<R>*)d.fdr) + i) : mk4<R>(0, 0, 0, 0);
  q.fin.xref = gld(G((const double4*)d.xref) + i);
  asm volatile("" ::"v"((int)alive), "v"(sl), "v"(q.e0), "v"(q.e1), "v"(q.h0), "v"(q.h1), "s"(abort_at));
  if (abort_at <= a.step) return;
  if (!alive) {   // whole group
    if (sub == 0) {
      gst(G(d.xr[out]) + i, q.x);
      gst(G(d.vel[out]) + i, q.v);
      gst(G((R4<R>*)d.omg[out]) + i, q.w);
      G(d.alive[out])[i] = 0;
    }
    return;
  }
  uint64_t todo = __ballot(1);
  while (todo) {
    const int first = __builtin_ctzll(todo);
    const bool mine = sl == __builtin_amdgcn_readlane(sl, first);
    if (mine) {
      const int s = opaque_readlane(sl, first);
      // the held fluid force counts only in a sample with fluid
      if (!sample_const(d.sc, s).fluid_on) q.fin.fd = mk4<R>(0, 0, 0, 0);
      particle_gather<R, kGroup>(d, a, i, sub, s, q);
    }
    todo &= ~__ballot(mine);
  }
}

template <typename R, int kGroup> void launch_half(DevState& d, StepArgs a, hipStream_t s) {
  if (d.nslots > 0) hipLaunchKernelGGL(k_pairs<R>, dim3(nblk(d.nslots)), dim3(kBlock), 0, s, d.self, a);
  hipLaunchKernelGGL((k_gather<R, kGroup>), dim3(nblk(d.n * kGroup)), dim3(kBlock), 0, s, d.self, a);
}

template <typename R> void launch_step(DevState& d, StepArgs a, hipStream_t s) {
  if (d.pair_mode == DEM_PAIRS_HALF) {
    switch (d.group) {
      case 1: launch_half<R, 1>(d, a, s); return;
      case 2: launch_half<R, 2>(d, a, s); return;
      case 4: launch_half<R, 4>(d, a, s); return;
      case 16: launch_half<R, 16>(d, a, s); return;
      default: launch_half<R, 8>(d, a, s); return;
    }
  }
  if (d.group == 1)
    hipLaunchKernelGGL((k_step<R, 1>), dim3(nblk(d.n)), dim3(kBlock), 0, s, d.self, a);
  else if (d.group == 2)
    hipLaunchKernelGGL((k_step<R, 2>), dim3(nblk(d.n * 2)), dim3(kBlock), 0, s, d.self, a);
  else if (d.group == 4)
    hipLaunchKernelGGL((k_step<R, 4>), dim3(nblk(d.n * 4)), dim3(kBlock), 0, s, d.self, a);
  else if (d.group == 16)
    hipLaunchKernelGGL((k_step<R, 16>), dim3(nblk(d.n * 16)), dim3(kBlock), 0, s, d.self, a);
  else
    hipLaunchKernelGGL((k_step<R, 8>), dim3(nblk(d.n * 8)), dim3(kBlock), 0, s, d.self, a);
}
template void launch_step<double>(DevState&, StepArgs, hipStream_t);
template void launch_step<float>(DevState&, StepArgs, hipStream_t);

}  // namespace dem
