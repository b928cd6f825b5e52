// dem_device.h -- device functions shared by the kernels: binning, wall
// geometry, and the contact law of one pair (arXiv:2211.06142 sections
// 2.1, 2.3, 2.4).
#pragma once
#include <math.h>

#include "dem_internal.h"

namespace dem {

constexpr int kBlock = 256;
static inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

template <typename R> __device__ inline R4<R> mk4(R a, R b, R c, R d) {
  R4<R> v;
  v.x = a; v.y = b; v.z = c; v.w = d;
  return v;
}

template <typename R> __device__ inline R rcbrt_(R x);
template <> __device__ inline double rcbrt_<double>(double x) { return cbrt(x); }
template <> __device__ inline float rcbrt_<float>(float x) { return cbrtf(x); }
template <typename R> __device__ inline R rsqrt_(R x);
template <> __device__ inline double rsqrt_<double>(double x) { return sqrt(x); }
template <> __device__ inline float rsqrt_<float>(float x) { return sqrtf(x); }

// FP32 path: hardware reciprocal and square root (about 1 ulp); FP64 path:
// correctly rounded operations
template <typename R> __device__ inline R frcp_(R x);
template <> __device__ inline double frcp_<double>(double x) { return 1.0 / x; }
template <> __device__ inline float frcp_<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename R> __device__ inline R fsqrt_(R x);
template <> __device__ inline double fsqrt_<double>(double x) { return sqrt(x); }
template <> __device__ inline float fsqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// Global-address-space views of the state arrays.  The step-window kernels
// read the state struct through a pointer, so the compiler cannot tell where
// the array pointers inside point; without these views every access is a flat
// access with a full 64-bit address per lane.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ inline gptr<T> G(T* p) { return (gptr<T>)p; }
// Loads and stores of the HIP vector types through such views go through the
// compiler's own vector types (whole-vector accesses, no constructors).
typedef double gd4 __attribute__((ext_vector_type(4)));
typedef float gf4 __attribute__((ext_vector_type(4)));
__device__ inline double4 gld(gptr<const double4> p) {
  const gd4 t = *(gptr<const gd4>)p;
  return make_double4(t.x, t.y, t.z, t.w);
}
__device__ inline float4 gld(gptr<const float4> p) {
  const gf4 t = *(gptr<const gf4>)p;
  return make_float4(t.x, t.y, t.z, t.w);
}
__device__ inline void gst(gptr<double4> p, const double4& v) { *(gptr<gd4>)p = gd4{v.x, v.y, v.z, v.w}; }
__device__ inline void gst(gptr<float4> p, const float4& v) { *(gptr<gf4>)p = gf4{v.x, v.y, v.z, v.w}; }

// LDS written by some lanes of a wave and read by others: keep the compiler
// from moving the accesses across this point (the LDS executes the accesses
// of one wave in order).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Pair record of the half-pair mode: the force on the owner and n x F_t, six R
// packed in three 2-vectors (24 B per slot in mixed precision).
template <typename R> struct V2T;
template <> struct V2T<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct V2T<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <typename R> __device__ inline void rec_put(void* base, int64_t p, const R (&f)[3], const R (&t)[3]) {
  using V = typename V2T<R>::type;
  const gptr<V> q = (gptr<V>)base + 3 * p;
  q[0] = V{f[0], f[1]};
  q[1] = V{f[2], t[0]};
  q[2] = V{t[1], t[2]};
}
template <typename R> __device__ inline void rec_get(const void* base, int64_t p, R (&f)[3], R (&t)[3]) {
  using V = typename V2T<R>::type;
  const gptr<const V> q = (gptr<const V>)base + 3 * p;
  const V a = q[0], b = q[1], c = q[2];
  f[0] = a.x; f[1] = a.y; f[2] = b.x;
  t[0] = b.y; t[1] = c.x; t[2] = c.y;
}

// The per-sample constants do not change while a kernel runs.  Reading them
// through the constant address space lets the compiler use scalar loads for a
// wave-uniform sample and hoist the loads out of loops that store.
template <typename T> using cptr = __attribute__((address_space(4))) const T*;
__device__ inline const SampleConst& sample_const(const SampleConst* sc, int s) {
  return *(const SampleConst*)((cptr<SampleConst>)sc + s);
}

// Lane `lane`'s value as a scalar that the optimiser cannot identify with the
// per-lane value it was read from: inside `if (x == readlane(x, l))` it would
// otherwise substitute the per-lane x back and lose the scalar registers.
__device__ inline int opaque_readlane(int v, int lane) {
  int r;
  asm volatile("v_readlane_b32 %0, %1, %2" : "=s"(r) : "v"(v), "s"(lane));
  return r;
}

// Workgroups are dealt to the 8 XCDs of the chip in turn, each with its own L2.
// Remapping gives every XCD one contiguous run of logical blocks, so blocks that
// gather each other's (spatially sorted) particles share an L2.  A bijection on
// [0, nb) for any nb.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  constexpr int kXcd = 8;
  const int64_t q = nb / kXcd, r = nb % kXcd;
  const int64_t x = b % kXcd, k = b / kXcd;
  return x * q + (x < r ? x : r) + k;
}

__device__ inline int bin_coord(double x, double lo, double h, int n) {
  double q = floor((x - lo) / h);
  if (!(q >= 0.0)) return 0;   // also a NaN coordinate
  if (q > (double)(n - 1)) return n - 1;
  return (int)q;
}

// signed distance from the wall surface (positive on the particle side) and
// the unit normal pointing into the particle side
// (search: the candidate search of a rebuild, which ignores a plane's hole,
// since a particle may move out of the hole before the next rebuild)
__device__ inline bool wall_geom(const Wall& w, double x, double y, double z, double& sd, double nw[3],
                                 bool search = false) {
  if (w.kind == DEM_WALL_PLANE) {
    nw[0] = w.p[0]; nw[1] = w.p[1]; nw[2] = w.p[2];
    sd = ((nw[0] * x + nw[1] * y) + nw[2] * z) - w.p[3];
    return true;
  }
  if (w.kind == DEM_WALL_PLANE_HOLE) {
    nw[0] = 0.0; nw[1] = 0.0; nw[2] = w.p[3];
    sd = w.p[3] * (z - w.p[2]);
    const double ex = x - w.p[0], ey = y - w.p[1];
    return search || !(ex * ex + ey * ey < w.p[4] * w.p[4]);
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

// Contact radius and elastic force of a bonded JKR contact (eq 12-13).  With
// X^3 = pi^2 gamma^2 R* / E*^2, a0 = sqrt(X R*), delta = X D and a = a0 b^2,
// eq 13 becomes b^4 - 2 b = D and eq 12 F = pi gamma R* (4/3 b^6 - 4 b^3).
// The branch through point C (b_C^3 = 3/2) is taken: two fixed-point steps of
// b = (D + 2b)^(1/4) from b_C, then Newton on the convex increasing quartic.
// The original JKR cycle reaches below C down to point S (b_S^3 = 1/2, where
// the quartic's slope vanishes): from above the root both iterations decrease
// monotonically towards it, more Newton steps are taken, each kept on the
// branch (b >= b_S).
template <typename R>
__device__ inline void jkr_bonded(R delta, R Rs, R gam, R jkrK, R& a, R& Fel, bool to_S) {
  constexpr R kPi = (R)3.14159265358979323846;
  constexpr R kbC = (R)1.1447142425533319;   // (3/2)^(1/3)
  constexpr R kbS = (R)0.79370052598409974;  // (1/2)^(1/3)
  constexpr int kNewton = sizeof(R) == 8 ? 3 : 2;
  constexpr int kNewtonS = sizeof(R) == 8 ? 12 : 8;
  R X = rcbrt_<R>(jkrK * Rs);
  R D = delta * frcp_<R>(X);
  R b = fsqrt_<R>(fsqrt_<R>(D + (R)2 * kbC));
  b = fsqrt_<R>(fsqrt_<R>(D + (R)2 * b));
  if (!to_S) {
#pragma unroll
    for (int it = 0; it < kNewton; ++it) {
      R b3 = b * b * b;
      R f = b3 * b - (R)2 * b - D;
      R fp = (R)4 * b3 - (R)2;
      b -= f * frcp_<R>(fp);
    }
  } else {
    for (int it = 0; it < kNewtonS; ++it) {
      R b3 = b * b * b;
      R f = b3 * b - (R)2 * b - D;
      R fp = (R)4 * b3 - (R)2;
      if (!(fp > (R)0)) break;
      b -= f * frcp_<R>(fp);
      if (b < kbS) b = kbS;
    }
  }
  R b3 = b * b * b;
  R u = kPi * gam * Rs;
  Fel = u * ((R)4 / (R)3) * b3 * b3 - u * (R)4 * b3;
  a = fsqrt_<R>(X * Rs) * b * b;
}

// Contact-law constants of one sample in the arithmetic type of the forces.
template <typename R> struct LawK {
  R Es, Gs, beta, cdamp, mu, mu_roll, k_lin;
  bool linear;
  bool orig;   // original JKR cycle: contacts form on touch, hold down to point S
};
template <typename R> __device__ inline LawK<R> law_k(const SampleConst& c);
template <> __device__ inline LawK<double> law_k<double>(const SampleConst& c) {
  return {c.Es, c.Gs, c.beta, c.cdamp, c.mu, c.mu_roll, c.k_lin, c.normal_model == DEM_NORMAL_LINEAR,
          c.normal_model == DEM_NORMAL_JKR_ORIG};
}
template <> __device__ inline LawK<float> law_k<float>(const SampleConst& c) {
  return {c.f_Es, c.f_Gs, c.f_beta, c.f_cdamp, c.f_mu, c.f_mu_roll, c.f_k_lin, c.normal_model == DEM_NORMAL_LINEAR,
          c.normal_model == DEM_NORMAL_JKR_ORIG};
}

template <typename R> struct LawOut {
  R F[3], c[3], Tr[3];
};

// One contact (section 2.1 eq 3-5, section 2.3 eq 12-13, section 2.4 eq 32-35).
// n: unit normal from the body to its partner; vrel: contact-point velocity of
// the body relative to the partner; wrel: relative angular velocity; hdt:
// tangential elongation (in/out).  Output: force on the body, n x F_t (the
// torque on each body is its radius times this), rolling torque on the body.
template <typename R>
__device__ inline void contact_law(const LawK<R>& c, int bonded, R delta, R Rs, R ms, R gam, R jkrK,
                                   const R n[3], const R vrel[3], const R wrel[3], R hdt[3], R dt,
                                   bool rolling, LawOut<R>& o) {
  R a, Fel, kn, kt, etan, etat, L;
  if (c.linear) {
    kn = c.k_lin;
    Fel = kn * delta;
    kt = ((R)2 / (R)7) * kn;
    etan = (R)2 * c.beta * fsqrt_<R>(kn * ms);
    etat = (R)2 * c.beta * fsqrt_<R>(kt * ms);
    L = c.mu * Fel;
  } else {
    if (bonded && gam > (R)0) {
      jkr_bonded<R>(delta, Rs, gam, jkrK, a, Fel, c.orig);
      L = c.mu * (Fel + (R)2 * ((R)3 * (R)3.14159265358979323846 * gam * Rs));
    } else {
      a = fsqrt_<R>(Rs * (delta > (R)0 ? delta : (R)0));
      Fel = (R)4 * c.Es * a * a * a * frcp_<R>((R)3 * Rs);
      L = c.mu * Fel;
    }
    kn = (R)2 * c.Es * a;
    kt = (R)8 * c.Gs * a;
    etan = c.cdamp * fsqrt_<R>(kn * ms);
    etat = c.cdamp * fsqrt_<R>(kt * ms);
  }
  R vn = (vrel[0] * n[0] + vrel[1] * n[1]) + vrel[2] * n[2];
  R vt[3] = {vrel[0] - vn * n[0], vrel[1] - vn * n[1], vrel[2] - vn * n[2]};
  R Fn = Fel + etan * vn;
  // rotate the stored elongation into the tangent plane, keep its length
  R old = fsqrt_<R>((hdt[0] * hdt[0] + hdt[1] * hdt[1]) + hdt[2] * hdt[2]);
  R dn = (hdt[0] * n[0] + hdt[1] * n[1]) + hdt[2] * n[2];
  R tp[3] = {hdt[0] - dn * n[0], hdt[1] - dn * n[1], hdt[2] - dn * n[2]};
  R tpl = fsqrt_<R>((tp[0] * tp[0] + tp[1] * tp[1]) + tp[2] * tp[2]);
  if (tpl > (R)0) {
    R f = old * frcp_<R>(tpl);
    hdt[0] = tp[0] * f; hdt[1] = tp[1] * f; hdt[2] = tp[2] * f;
  } else {
    hdt[0] = hdt[1] = hdt[2] = (R)0;
  }
  hdt[0] += vt[0] * dt; hdt[1] += vt[1] * dt; hdt[2] += vt[2] * dt;
  R Ft[3] = {-kt * hdt[0] - etat * vt[0], -kt * hdt[1] - etat * vt[1], -kt * hdt[2] - etat * vt[2]};
  R ftm = fsqrt_<R>((Ft[0] * Ft[0] + Ft[1] * Ft[1]) + Ft[2] * Ft[2]);
  if (ftm > L) {
    R s = L * frcp_<R>(ftm);
    Ft[0] *= s; Ft[1] *= s; Ft[2] *= s;
    if (kt > (R)0) {
      R ik = frcp_<R>(kt);
      hdt[0] = -(Ft[0] + etat * vt[0]) * ik;
      hdt[1] = -(Ft[1] + etat * vt[1]) * ik;
      hdt[2] = -(Ft[2] + etat * vt[2]) * ik;
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
  if (rolling && c.mu_roll > (R)0) {
    R wn = (wrel[0] * n[0] + wrel[1] * n[1]) + wrel[2] * n[2];
    R wr[3] = {wrel[0] - wn * n[0], wrel[1] - wn * n[1], wrel[2] - wn * n[2]};
    R wm = fsqrt_<R>((wr[0] * wr[0] + wr[1] * wr[1]) + wr[2] * wr[2]);
    if (wm > (R)0) {
      R tm = c.mu_roll * Rs * (Fel < (R)0 ? -Fel : Fel) * frcp_<R>(wm);
      o.Tr[0] = -tm * wr[0]; o.Tr[1] = -tm * wr[1]; o.Tr[2] = -tm * wr[2];
    }
  }
}

// Bond persistence down to the pull-off overlap of point C (Table 1, Fig. 2),
// or for the original JKR cycle down to point S, written with cubes so that no
// cube root enters the decision: (-delta)^3 <= brk pi^2 gamma^2 R* / E*^2 with
// brk = 3/16 (C) or 27/16 (S).  Same operation order as the FP64 reference
// definition; called only for bonded pairs that do not touch.
__device__ inline bool bond_holds_apart(double d2, double cs, double Rsd, double gam, double Es, double brk) {
  double sep = sqrt(d2) - cs;
  double lhs = (sep * sep) * sep;
  double rhs = ((brk * (M_PI * M_PI)) * (gam * gam)) * Rsd / (Es * Es);
  return lhs <= rhs;
}

// Result of one half pair in its canonical orientation (a = lower sorted
// index, n from a to b): force on a, n x F_t, rolling torque on a.
template <typename R> struct PairOut {
  LawOut<R> o;
  R4<R> h;
  uint8_t fl;
  bool active;   // contributes a force
  bool broke;    // the bond broke this step
};

template <typename R>
__device__ inline void pair_eval(const LawK<R>& c, double Es, double dt, bool rolling, const double4& A, const double4& B,
                                 const double4& VA, const double4& VB, const R4<R>& WA, const R4<R>& WB,
                                 double gam, R4<R> h4, uint8_t fl, PairOut<R>& out) {
  out.active = false;
  out.broke = false;
  const double dx = B.x - A.x, dy = B.y - A.y, dz = B.z - A.z;
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double cs = A.w + B.w;
  const bool touching = d2 < cs * cs;
  // the original JKR cycle bonds every touching pair (snap-in at point A)
  const int bonded = (fl & 1) | ((c.orig && touching) ? 1 : 0);
  if (bonded && !touching &&
      !bond_holds_apart(d2, cs, A.w * B.w / (A.w + B.w), gam, Es, c.orig ? 27.0 / 16.0 : 3.0 / 16.0)) {
    out.broke = true;
    out.h = mk4<R>(0, 0, 0, 0);
    out.fl = 0;
    return;
  }
  if (!bonded && !touching) {
    out.h = mk4<R>(0, 0, 0, 0);
    out.fl = 0;
    return;
  }
  R delta, n[3];
  if (sizeof(R) == 8) {
    const double dist = sqrt(d2);
    delta = (R)(cs - dist);
    n[0] = (R)(dx / dist); n[1] = (R)(dy / dist); n[2] = (R)(dz / dist);
  } else {
    // overlap from the FP64 difference of squares, normal in FP32
    const R dist = fsqrt_<R>((R)d2);
    delta = (R)(cs * cs - d2) * frcp_<R>((R)cs + dist);
    const R inv = frcp_<R>(dist);
    n[0] = (R)dx * inv; n[1] = (R)dy * inv; n[2] = (R)dz * inv;
  }
  const R ra = (R)A.w, rb = (R)B.w;
  const R ws[3] = {ra * WA.x + rb * WB.x, ra * WA.y + rb * WB.y, ra * WA.z + rb * WB.z};
  const R vrel[3] = {(R)(VA.x - VB.x) + (ws[1] * n[2] - ws[2] * n[1]),
                     (R)(VA.y - VB.y) + (ws[2] * n[0] - ws[0] * n[2]),
                     (R)(VA.z - VB.z) + (ws[0] * n[1] - ws[1] * n[0])};
  const R wrel[3] = {WA.x - WB.x, WA.y - WB.y, WA.z - WB.z};
  R ms, Rs;
  if (sizeof(R) == 8) {
    ms = (R)(1.0 / (VA.w + VB.w));
    Rs = (R)(A.w * B.w / (A.w + B.w));
  } else {
    ms = frcp_<R>((R)VA.w + (R)VB.w);
    Rs = ra * rb * frcp_<R>(ra + rb);
  }
  R h[3] = {h4.x, h4.y, h4.z};
  const R gR = (R)gam;
  const R jkrK = (R)3.14159265358979323846 * (R)3.14159265358979323846 * gR * gR * frcp_<R>(c.Es * c.Es);
  contact_law<R>(c, bonded, delta, Rs, ms, gR, jkrK, n, vrel, wrel, h, (R)dt, rolling, out.o);
  out.h = mk4<R>(h[0], h[1], h[2], (R)0);
  out.fl = (uint8_t)(bonded | (touching ? 2 : 0));
  out.active = true;
}

}  // namespace dem
