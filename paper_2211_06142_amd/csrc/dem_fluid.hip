// dem_fluid.hip -- fluid-particle coupling (arXiv:2211.06142 section 2.2).
//
// Every reduction is a sorted segmented reduction, no floating-point atomics:
// each particle has a bucket, the cell of the grid of fluid-cell centres that
// holds it ("dual cell": its 8 corners are the 8 fluid cells a trilinear weight
// reaches; for centroid deposition the bucket is the fluid cell itself); a
// bucket sums its members' contributions to its 8 corners in a fixed order, and
// a fluid cell sums the partials of the (up to 8) buckets around it in a fixed
// order.  The members are found through the neighbour list's binning (particles
// sorted by binning cell at the last rebuild, none moved more than half the skin
// since), so the coupling needs no sort of its own.
//   porosity  n = clamp(1 - sum w V / V_cell, n_min, 1)           (eq 6)
//   drag      Di Felice, coarse-grained k^3 f(d/k), closure factor (eq 8-11)
//   buoyancy  F_b = -V (grad p + rho_f g)                           (eq 1)
//   source    sum w f / V_cell                                      (eq 7)
#include "dem_device.h"

namespace dem {

// fn(s) for the active lanes of each sample of the wave in turn, with the
// sample index s in a scalar register: the sample's constants are then scalar
// loads through the constant cache.  Lanes of one sample stay together, so the
// groups of 8 lanes of a bucket or a cell (one sample each) stay whole.
template <typename Fn>
__device__ inline void per_sample(int sl, Fn&& fn) {
  uint64_t todo = __ballot(1);
  while (todo) {
    const int first = __builtin_ctzll(todo);
    const bool mine = sl == __builtin_amdgcn_readlane(sl, first);
    if (mine) fn(opaque_readlane(sl, first));
    todo &= ~__ballot(mine);
  }
}

// Key (bucket) and trilinear fractions of every particle; dead particles, and
// every particle of a sample without fluid, get their sample's skip key, which
// no cell reads.
__device__ inline void fluid_key(const DevState& d, const SampleConst& c, int64_t i, uint8_t al, const double4& p) {
  int64_t nd = (int64_t)c.dn[0] * c.dn[1] * c.dn[2];
  const int32_t skip = (int32_t)(c.dual_base + nd);
  if (!al || !c.fluid_on || !isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z)) {
    d.dkey[i] = skip;
    return;
  }
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
  const int64_t key = c.dual_base + ((int64_t)b[2] * c.dn[1] + b[1]) * c.dn[0] + b[0];
  d.dkey[i] = (int32_t)key;
  d.docc[key] = 1;   // the bucket has a member in this evaluation
  const double V = (4.0 / 3.0) * M_PI * p.w * p.w * p.w;
  d.dfr[i] = make_double4(f[0], f[1], f[2], V);
}

__global__ void k_fluid_key(const DevState* __restrict__ dp, int buf) {
  const DevState& d = *dp;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  // one round trip: the abort flag and the particle's own inputs
  const int ab = *G((const int32_t*)d.abort);
  const int32_t sl = G((const int32_t*)d.sample)[i];
  const uint8_t al = G((const uint8_t*)d.alive[buf])[i];
  const double4 p = gld(G((const double4*)d.xr[buf]) + i);
  asm volatile("" ::"s"(ab), "v"(sl), "v"((int)al), "v"(p.x), "v"(p.y), "v"(p.z), "v"(p.w));
  if (ab) return;
  per_sample(sl, [&](int s) { fluid_key(d, sample_const(d.sc, s), i, al, p); });
}

// (x, y, z) of the local index l of a cell or bucket of an nx x ny grid layer
// stack (l < 2^30: a sample's grid is limited to that many cells), in 32-bit
// arithmetic
__device__ inline void unflatten3(int64_t l, int nx, int ny, int (&o)[3]) {
  const int32_t q = (int32_t)l;
  const int32_t t = q / nx;
  o[0] = q - t * nx;
  o[2] = t / ny;
  o[1] = t - o[2] * ny;
}

// trilinear weight of corner (kx, ky, kz) in {0,1}^3 of a bucket
__device__ inline double corner_w(const double4& fr, int kx, int ky, int kz) {
  double wx = kx ? fr.x : 1.0 - fr.x;
  double wy = ky ? fr.y : 1.0 - fr.y;
  double wz = kz ? fr.z : 1.0 - fr.z;
  return (wx * wy) * wz;
}

// Range of binning cells along one axis that can hold a member of bucket b: the
// bucket's extent (open towards the outside at the first and last bucket,
// where the weights fold onto the boundary cells) widened by half the skin,
// the farthest a particle moves between list rebuilds.  Binning cells are those
// of the last rebuild, positions then clamped into the grid as the bucket keys
// clamp them, so bin_coord of the widened ends bounds every member's cell.
__device__ inline void member_bins(const SampleConst& c, int k, int b, int cen, int& q0, int& q1) {
  // (widened a little more than half the skin: the bounds below and the keys
  // are computed with different roundings)
  const double h = c.gh[k], hs = 0.5 * c.skin * (1.0 + 1e-6) + 1e-9 * h;
  const int nb = c.dn[k];
  const double off = cen ? 0.0 : 0.5;
  q0 = b == 0 ? 0 : bin_coord(c.glo[k] + (b + off) * h - hs, c.blo[k], c.bh[k], c.bn[k]);
  q1 = b == nb - 1 ? c.bn[k] - 1 : bin_coord(c.glo[k] + (b + off + 1.0) * h + hs, c.blo[k], c.bh[k], c.bn[k]);
}

// Corner partials of every bucket, a sorted segmented reduction with no sort of
// its own: the members of bucket b are the particles whose key is b, and they
// lie in the binning cells of member_bins, sorted by binning cell since the last
// rebuild; a group of 8 lanes scans those cells' particles in increasing index
// (row by row, lane u taking every 8th of a row, starting at u) and adds each
// member's weighted value to the bucket's 8 corners; the lanes' sums are then
// added in a fixed tree.  The order of every sum is fixed by the binning and the
// keys.  Buckets that no particle's key named in this evaluation (the occupancy
// byte) are skipped.  kind 0: solid volume (8 per bucket); it also records the
// bucket's members in a list of kGroupMem entries (lane 0's in scan order, then
// lane 1's, ...; each lane's count in its byte), so that kind 1, the particle
// drag (24 per bucket), visits the same members in the same order without
// scanning again; a bucket whose members do not fit (more than kGroupMem, or
// more than kLaneMem on one lane) is marked (count 255) and scanned again.
// kind 1 clears the occupancy for the next evaluation.
constexpr int kLaneMem = 16;   // members a lane holds in registers while it scans
constexpr int kGroupMem = 64;  // entries of a bucket's list
// binning-cell rows (runs along x) whose bounds a group stages in LDS; a bucket
// whose widened extent covers more rows scans them one at a time
constexpr int kScanRows = 16;

// member q's weighted value added to the bucket's corners (fr: its fractions and
// volume, fp: its drag)
template <int kKind>
__device__ inline void add_weighted(const double4& fr, const double4& fp, double* acc) {
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    const double w = corner_w(fr, corner & 1, (corner >> 1) & 1, corner >> 2);
    if (kKind == 0) {
      acc[corner] += w * fr.w;
    } else {
      acc[3 * corner] += w * fp.x;
      acc[3 * corner + 1] += w * fp.y;
      acc[3 * corner + 2] += w * fp.z;
    }
  }
}

template <int kKind>
__device__ inline void add_member(const DevState& d, int32_t q, double* acc) {
  const double4 fr = gld(G((const double4*)d.dfr) + q);
  double4 fp = make_double4(0.0, 0.0, 0.0, 0.0);
  if (kKind == 1) fp = gld(G((const double4*)d.fpart) + q);
  add_weighted<kKind>(fr, fp, acc);
}

// Members q[0 .. cnt) in order, four at a time: the inputs of four members
// are fetched before the first of them is added.
constexpr int kChunk = 4;

template <int kKind>
__device__ inline void add_chunk(const DevState& d, const int32_t (&q)[kChunk], int cnt, double* acc) {
  const auto FR = G((const double4*)d.dfr);
  const auto FP = G((const double4*)d.fpart);
  double4 fr[kChunk], fp[kChunk];
#pragma unroll
  for (int v = 0; v < kChunk; ++v) {
    const int32_t qq = v < cnt ? q[v] : 0;   // particle 0 exists: an unused, in-bounds read
    fr[v] = gld(FR + qq);
    fp[v] = kKind == 1 ? gld(FP + qq) : make_double4(0.0, 0.0, 0.0, 0.0);
  }
#pragma unroll
  for (int v = 0; v < kChunk; ++v)
    if (v < cnt) add_weighted<kKind>(fr[v], fp[v], acc);
}

// the members a lane recorded in registers (kind 0)
template <int kKind>
__device__ inline void add_held(const DevState& d, const int32_t (&q)[kLaneMem], int cnt, double* acc) {
#pragma unroll
  for (int c0 = 0; c0 < kLaneMem; c0 += kChunk) {
    if (c0 >= cnt) break;
    const int32_t qc[kChunk] = {q[c0], q[c0 + 1], q[c0 + 2], q[c0 + 3]};
    add_chunk<kKind>(d, qc, cnt - c0, acc);
  }
}

// the members list[0 .. cnt) of a bucket's list (kind 1)
template <int kKind>
__device__ inline void add_list(const DevState& d, gptr<const int32_t> list, int cnt, double* acc) {
  for (int c0 = 0; c0 < cnt; c0 += kChunk) {
    int32_t qc[kChunk];
#pragma unroll
    for (int v = 0; v < kChunk; ++v) qc[v] = c0 + v < cnt ? list[c0 + v] : 0;
    add_chunk<kKind>(d, qc, cnt - c0, acc);
  }
}

// exclusive prefix sum of v over the 8 lanes of a group (lane u of the group)
__device__ inline int group8_excl(int v, int u) {
  int s = v;
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) {
    const int t = __shfl_up(s, off, 8);
    if (u >= off) s += t;
  }
  return s - v;
}

// Sum over the 8 lanes of a group of each of M values (M a multiple of 8) in a
// fixed tree (partners at lane distance 4, then 2, then 1), leaving lane u with
// the totals of values u, u + 8, u + 16, ... in out[0 .. M/8).
template <int M>
__device__ inline void group8_reduce_scatter(const double (&v)[M], int u, double (&out)[M / 8]) {
  const bool h2 = (u >> 2) & 1, h1 = (u >> 1) & 1, h0 = u & 1;
  double w[M / 2], x[M / 4];
#pragma unroll
  for (int j = 0; j < M / 8; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double lo = v[8 * j + r], hi = v[8 * j + r + 4];
      w[4 * j + r] = (h2 ? hi : lo) + __shfl_xor(h2 ? lo : hi, 4, 64);
    }
#pragma unroll
  for (int j = 0; j < M / 8; ++j)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const double lo = w[4 * j + r], hi = w[4 * j + r + 2];
      x[2 * j + r] = (h1 ? hi : lo) + __shfl_xor(h1 ? lo : hi, 2, 64);
    }
#pragma unroll
  for (int j = 0; j < M / 8; ++j) {
    const double lo = x[2 * j], hi = x[2 * j + 1];
    out[j] = (h0 ? hi : lo) + __shfl_xor(h0 ? lo : hi, 1, 64);
  }
}

// The binning cells that can hold a member of bucket b (member_bins along each
// axis): rows (runs along x) in increasing (z, y).
struct ScanBox {
  int q0[3], q1[3];
  int ny, nr;
};

__device__ inline ScanBox scan_box(const SampleConst& c, int64_t b) {
  ScanBox sb;
  const int64_t l = b - c.dual_base;
  int D[3];
  unflatten3(l, c.dn[0], c.dn[1], D);
  const int cen = c.voidfrac == DEM_VOID_CENTROID;
  for (int k = 0; k < 3; ++k) member_bins(c, k, D[k], cen, sb.q0[k], sb.q1[k]);
  sb.ny = sb.q1[1] - sb.q0[1] + 1;
  sb.nr = sb.ny * (sb.q1[2] - sb.q0[2] + 1);
  return sb;
}

__device__ inline int64_t scan_row(const SampleConst& c, const ScanBox& sb, int k) {
  return c.bin_base + ((int64_t)(sb.q0[2] + k / sb.ny) * c.bn[1] + (sb.q0[1] + k % sb.ny)) * c.bn[0];
}

// The group's kLanes lanes load the bounds [first particle, end) of the box's
// rows together into `rows` (the group's kScanRows LDS entries; every lane of
// the group takes part, then the wave syncs before any lane reads them).
template <int kLanes = 8>
__device__ inline void stage_rows(const DevState& d, const SampleConst& c, const ScanBox& sb, int u, int2* rows) {
  const auto CS = G((const int32_t*)d.cell_start);
  if (sb.nr <= kScanRows)
    for (int k = u; k < sb.nr; k += kLanes) {
      const int64_t row = scan_row(c, sb, k);
      rows[k] = make_int2(CS[row + sb.q0[0]], CS[row + sb.q1[0] + 1]);
    }
}

// Lane u of bucket b's group of kLanes lanes: call fn(q) for every member q
// among the candidates it takes (of each row, every kLanes-th, starting at u) in
// scan order.  With the rows staged (at most kScanRows), the lane fetches the
// keys of kU candidates at a time, across row ends, before testing any;
// otherwise it walks the rows one at a time.
template <int kLanes = 8, typename Fn>
__device__ inline void scan_members(const DevState& d, const SampleConst& c, int64_t b, int u, const ScanBox& sb,
                                    const int2* rows, Fn&& fn) {
  const auto KEY = G((const int32_t*)d.dkey);
  const int nr = sb.nr;
  if (nr <= kScanRows) {
    // the lane's next candidate: m in row r (r == nr: none left)
    int r = 0;
    int2 cur = rows[0];
    int32_t m = cur.x + u;
    while (m >= cur.y && ++r < nr) {
      cur = rows[r];
      m = cur.x + u;
    }
    constexpr int kU = 8;
    while (r < nr) {
      int32_t cand[kU], ks[kU];
#pragma unroll
      for (int v = 0; v < kU; ++v) {
        cand[v] = r < nr ? m : -1;
        if (r < nr) {
          m += kLanes;
          while (m >= cur.y && ++r < nr) {
            cur = rows[r];
            m = cur.x + u;
          }
        }
      }
#pragma unroll
      for (int v = 0; v < kU; ++v) ks[v] = cand[v] >= 0 ? KEY[cand[v]] : -1;
#pragma unroll
      for (int v = 0; v < kU; ++v)
        if (ks[v] == (int32_t)b) fn(cand[v]);
    }
    return;
  }
  const auto CS = G((const int32_t*)d.cell_start);
  for (int k = 0; k < nr; ++k) {
    const int64_t row = scan_row(c, sb, k);
    const int32_t m1 = CS[row + sb.q1[0] + 1];
    // four candidates per lane and round: all key loads before any use
    constexpr int kU = 4;
    for (int32_t m0 = CS[row + sb.q0[0]] + u; m0 < m1; m0 += kLanes * kU) {
      int32_t ks[kU];
#pragma unroll
      for (int v = 0; v < kU; ++v) ks[v] = m0 + kLanes * v < m1 ? KEY[m0 + kLanes * v] : -1;
#pragma unroll
      for (int v = 0; v < kU; ++v)
        if (ks[v] == (int32_t)b) fn(m0 + kLanes * v);
    }
  }
}

template <int kKind>
__global__ __launch_bounds__(256) void k_fluid_partials(const DevState* __restrict__ dp) {
  __shared__ int2 rows_lds[256 / 8][kScanRows];
  const DevState& d = *dp;
  constexpr int m = kKind == 0 ? 8 : 24;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = gid >> 3;
  const int u = (int)(gid & 7);
  if (b >= d.ndual) return;   // whole group
  const auto OCC = G((uint8_t*)d.docc);
  const auto PART = G(d.dpart + (kKind == 0 ? 0 : 8 * (d.ndual + 1)));
  const auto LIST = G((int32_t*)d.dlmem) + b * kGroupMem;
  const auto LN = G((uint8_t*)d.dlcnt);
  // one round trip: the abort flag, the occupancy, the bucket's sample and
  // (kind 1) the lane's member count
  const int ab = *G((const int32_t*)d.abort);
  const uint8_t occ = OCC[b];
  const int32_t smp = G((const int32_t*)d.dual_sample)[b];
  const int listed = kKind == 1 ? (int)LN[gid] : 255;
  asm volatile("" ::"s"(ab), "v"((int)occ), "v"(smp), "v"(listed));
  if (ab) return;
  if (!occ) {   // no member: zero partials (lane u writes outputs u, u + 8, ...)
#pragma unroll
    for (int j = 0; j < m / 8; ++j) PART[m * b + 8 * j + u] = 0.0;
    return;
  }
  per_sample(smp, [&](int sc) {
    const SampleConst& c = sample_const(d.sc, sc);
    double acc[m];
#pragma unroll
    for (int k = 0; k < m; ++k) acc[k] = 0.0;
    // the group scans (kind 0 always; kind 1 when its bucket's list overflowed:
    // the count is the same on all the group's lanes then)
    const bool scan = listed == 255;
    int2* rows = rows_lds[threadIdx.x >> 3];
    ScanBox sb;
    if (scan) {
      sb = scan_box(c, b);
      stage_rows(d, c, sb, u, rows);
    }
    wave_lds_sync();
    if (kKind == 1) {
      if (!scan) {
        add_list<kKind>(d, LIST + group8_excl(listed, u), listed, acc);
      } else {
        scan_members(d, c, b, u, sb, rows, [&](int32_t q) { add_member<kKind>(d, q, acc); });
      }
    } else {
      // hold the first kLaneMem members in registers for the bucket's list,
      // add them after the scan (their loads issued together), then (more
      // members) scan again for the rest, in scan order
      int32_t q[kLaneMem];
#pragma unroll
      for (int t = 0; t < kLaneMem; ++t) q[t] = 0;
      int found = 0;
      scan_members(d, c, b, u, sb, rows, [&](int32_t p) {
#pragma unroll
        for (int t = 0; t < kLaneMem; ++t)
          if (found == t) q[t] = p;
        ++found;
      });
      add_held<kKind>(d, q, found < kLaneMem ? found : kLaneMem, acc);
      if (found > kLaneMem) {
        int seen = 0;
        scan_members(d, c, b, u, sb, rows, [&](int32_t p) {
          if (seen >= kLaneMem) add_member<kKind>(d, p, acc);
          ++seen;
        });
      }
      // the bucket's list for kind 1: lane-major, if every lane's members were
      // held and all fit
      const int excl = group8_excl(found, u);
      const int all = __shfl(excl + found, 7, 8);
      int most = found;
#pragma unroll
      for (int off = 4; off > 0; off >>= 1) most = max(most, __shfl_xor(most, off, 8));
      const bool fits = all <= kGroupMem && most <= kLaneMem;
      if (fits) {
#pragma unroll
        for (int t = 0; t < kLaneMem; ++t)
          if (t < found) LIST[excl + t] = q[t];
      }
      LN[gid] = (uint8_t)(fits ? found : 255);
    }
    // the 8 lanes' sums in a fixed tree; lane u writes outputs u, u + 8, ...
    double tot[m / 8];
    group8_reduce_scatter<m>(acc, u, tot);
#pragma unroll
    for (int j = 0; j < m / 8; ++j) PART[m * b + 8 * j + u] = tot[j];
    if (kKind == 1 && u == 0) OCC[b] = 0;
  });
}

// Dense buckets (more than 32 particles per bucket on average: a coarse grid
// over many grains, where the groups of 8 would leave most of the chip idle and
// their lists would overflow): a whole wave per bucket.  Lane u scans every
// 64th candidate of each row and adds its members as it finds them (scan
// order); the lanes' sums are then added in a fixed xor butterfly (partners 32,
// 16, ..., 1), which leaves every lane with the same totals, and lane j writes
// output j.  Both passes scan (no member lists); the drag pass clears the
// occupancy.
template <int kKind>
__global__ __launch_bounds__(256) void k_fluid_partials_wave(const DevState* __restrict__ dp) {
  __shared__ int2 rows_lds[256 / 64][kScanRows];
  const DevState& d = *dp;
  constexpr int m = kKind == 0 ? 8 : 24;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = gid >> 6;
  const int u = (int)(gid & 63);
  if (b >= d.ndual) return;   // whole wave
  const auto OCC = G((uint8_t*)d.docc);
  const auto PART = G(d.dpart + (kKind == 0 ? 0 : 8 * (d.ndual + 1)));
  // one round trip: the abort flag, the occupancy and the bucket's sample
  const int ab = *G((const int32_t*)d.abort);
  const uint8_t occ = OCC[b];
  const int32_t smp = G((const int32_t*)d.dual_sample)[b];
  asm volatile("" ::"s"(ab), "v"((int)occ), "v"(smp));
  if (ab) return;
  if (!occ) {   // no member: zero partials
    if (u < m) PART[m * b + u] = 0.0;
    return;
  }
  const SampleConst& c = sample_const(d.sc, opaque_readlane(smp, 0));   // one bucket per wave
  double acc[m];
#pragma unroll
  for (int k = 0; k < m; ++k) acc[k] = 0.0;
  int2* rows = rows_lds[threadIdx.x >> 6];
  const ScanBox sb = scan_box(c, b);
  stage_rows<64>(d, c, sb, u, rows);
  wave_lds_sync();
  scan_members<64>(d, c, b, u, sb, rows, [&](int32_t q) { add_member<kKind>(d, q, acc); });
  double out = 0.0;
#pragma unroll
  for (int k = 0; k < m; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
    if (u == k) out = acc[k];
  }
  if (u < m) PART[m * b + u] = out;
  if (kKind == 1 && u == 0) OCC[b] = 0;
}

// Per fluid cell: the sum of the corner partials of the (up to 8) adjacent
// buckets.  A group of 8 lanes serves a cell, lane u = (dz dy dx) the bucket at
// offset (dx, dy, dz) from the lowest adjacent one; the lanes' values are added
// in a fixed xor tree (partners 4, 2, 1), which leaves every lane with the same
// total (each stage adds the same two values in either order).  Kind 0: solid
// volume (d.dpart, 8 per bucket) -> porosity and fluid velocity; kind 1: drag
// (d.dpart + 8 (ndual + 1), 24 per bucket) -> the cell's drag source (eq 7).
template <int kKind>
__global__ __launch_bounds__(256) void k_fluid_cells(const DevState* __restrict__ dp) {
  const DevState& d = *dp;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t C = gid >> 3;
  const int u = (int)(gid & 7);
  if (C >= d.ncell) return;   // whole group
  // one round trip: the abort flag, the cell's sample and (kind 0) its inflow
  const int ab = *G((const int32_t*)d.abort);
  const int32_t smp = G((const int32_t*)d.cell_sample)[C];
  double uin[3] = {0.0, 0.0, 0.0};
  if (kKind == 0)
    for (int k = 0; k < 3; ++k) uin[k] = G((const double*)d.u_in)[3 * C + k];
  asm volatile("" ::"s"(ab), "v"(smp), "v"(uin[0]), "v"(uin[1]), "v"(uin[2]));
  if (ab) return;
  per_sample(smp, [&](int sc) {
    const SampleConst& c = sample_const(d.sc, sc);
    const int64_t l = C - c.cell_base;
    int cc[3];
    unflatten3(l, c.gn[0], c.gn[1], cc);
    const int cen = c.voidfrac == DEM_VOID_CENTROID;
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      if (cen) { lo[k] = hi[k] = cc[k]; }
      else if (c.gn[k] == 1) { lo[k] = hi[k] = 0; }
      else { lo[k] = cc[k] - 1 < 0 ? 0 : cc[k] - 1; hi[k] = cc[k] > c.gn[k] - 2 ? c.gn[k] - 2 : cc[k]; }
    }
    constexpr int m = kKind == 0 ? 8 : 24, nv = m / 8;
    const double* part = d.dpart + (kKind == 0 ? 0 : 8 * (d.ndual + 1));
    const int Dx = lo[0] + (u & 1), Dy = lo[1] + ((u >> 1) & 1), Dz = lo[2] + (u >> 2);
    double s[nv];
    for (int v = 0; v < nv; ++v) s[v] = 0.0;
    if (Dx <= hi[0] && Dy <= hi[1] && Dz <= hi[2]) {
      const int64_t key = c.dual_base + ((int64_t)Dz * c.dn[1] + Dy) * c.dn[0] + Dx;
      // corner of this cell in the bucket; a direction of one cell folds both
      // trilinear weights onto the only cell
      const int kx = (cen || c.gn[0] == 1) ? -1 : cc[0] - Dx;
      const int ky = (cen || c.gn[1] == 1) ? -1 : cc[1] - Dy;
      const int kz = (cen || c.gn[2] == 1) ? -1 : cc[2] - Dz;
      for (int cz = 0; cz < 2; ++cz) {
        if (kz >= 0 ? cz != kz : (cen && cz != 0)) continue;
        for (int cy = 0; cy < 2; ++cy) {
          if (ky >= 0 ? cy != ky : (cen && cy != 0)) continue;
          for (int cx = 0; cx < 2; ++cx) {
            if (kx >= 0 ? cx != kx : (cen && cx != 0)) continue;
            const int corner = (cz << 2) | (cy << 1) | cx;
            for (int v = 0; v < nv; ++v) s[v] += part[m * key + nv * corner + v];
          }
        }
      }
    }
#pragma unroll
    for (int v = 0; v < nv; ++v)
#pragma unroll
      for (int off = 4; off > 0; off >>= 1) s[v] += __shfl_xor(s[v], off, 8);
    if (u != 0) return;
    if (kKind == 0) {
      const double eps = s[0] / c.vcell;
      d.eps[C] = eps;
      double nn = 1.0 - eps;
      if (nn < c.n_min) nn = c.n_min;
      if (nn > 1.0) nn = 1.0;
      d.cell_n[C] = nn;
      for (int k = 0; k < 3; ++k) d.cell_u[3 * C + k] = c.u_superficial ? uin[k] / nn : uin[k];
    } else {
      for (int k = 0; k < 3; ++k) d.fdc[3 * C + k] = s[k] / c.vcell;
    }
  });
}

// Porosity, fluid velocity and dynamic pressure gradient at a particle with
// bucket key `key` and fractions fr, with the weights of its deposition
// (trilinear over the 8 surrounding cell centres, or its own cell for centroid
// deposition).  The 8 corners' fields are fetched before the first is added (a
// corner outside the grid reads the sample's first cell and adds nothing); the
// sums run in corner order.
__device__ inline void particle_fluid(const DevState& d, const SampleConst& c, int32_t key, const double4& fr,
                                      double& np, double u[3], double gp[3]) {
  const int cen = c.voidfrac == DEM_VOID_CENTROID;
  int64_t l = key - c.dual_base;
  int b[3];
  unflatten3(l, c.dn[0], c.dn[1], b);
  double f[3] = {fr.x, fr.y, fr.z};
  const int up = cen ? 1 : 2;
  const auto CN = G((const double*)d.cell_n);
  const auto CU = G((const double*)d.cell_u);
  const auto GP = G((const double*)d.gp_in);
  bool ok[8];
  double cn[8], cu[8][3], cg[8][3];
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    const int dx = corner & 1, dy = (corner >> 1) & 1, dz = corner >> 2;
    const int kx = b[0] + dx, ky = b[1] + dy, kz = b[2] + dz;
    ok[corner] = dx < up && dy < up && dz < up && kx < c.gn[0] && ky < c.gn[1] && kz < c.gn[2];
    const int64_t C = ok[corner] ? c.cell_base + ((int64_t)kz * c.gn[1] + ky) * c.gn[0] + kx : c.cell_base;
    cn[corner] = CN[C];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cu[corner][k] = CU[3 * C + k];
      cg[corner][k] = GP[3 * C + k];
    }
  }
  np = 0.0;
  for (int k = 0; k < 3; ++k) { u[k] = 0.0; gp[k] = 0.0; }
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    if (!ok[corner]) continue;
    const int dx = corner & 1, dy = (corner >> 1) & 1, dz = corner >> 2;
    double wx = cen ? 1.0 : (dx ? f[0] : 1.0 - f[0]);
    double wy = cen ? 1.0 : (dy ? f[1] : 1.0 - f[1]);
    double wz = cen ? 1.0 : (dz ? f[2] : 1.0 - f[2]);
    double w = (wx * wy) * wz;
    np += w * cn[corner];
    for (int k = 0; k < 3; ++k) {
      u[k] += w * cu[corner][k];
      gp[k] += w * cg[corner][k];
    }
  }
}

// Learned-closure features of particle i (an extension): porosity at the
// particle, slip speed |u - v|, particle Reynolds number of the drag law
// (eq 11, fine diameter d/k), k, and the mean of delta/R* over the pairs that
// took part in the last force evaluation, with their count.  Dead: zeros.
template <typename R>
__global__ __launch_bounds__(256) void k_closure_features(const DevState* __restrict__ dp, int buf) {
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
  particle_fluid(d, c, d.dkey[i], d.dfr[i], np, u, gp);
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

// Di Felice drag of one particle (eq 8-11, coarse-grained k^3 f(d/k), closure
// factor cdr) and buoyancy with the dynamic pressure gradient (eq 1), from the
// porosity, fluid velocity and pressure gradient at the particle.
__device__ inline void drag_force(const SampleConst& c, double np, const double u[3], const double gp[3],
                                  const double4& v, double r, double V, double cdr, double fd[3], double fb[3]) {
  double s[3] = {u[0] - v.x, u[1] - v.y, u[2] - v.z};
  double sm = sqrt((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
  fd[0] = fd[1] = fd[2] = 0.0;
  if (sm > 0.0) {
    double de = 2.0 * r / c.kcg;
    double Re = c.rho_f * de * sm / c.mu_f;
    double cd = 0.63 + 4.8 / sqrt(Re);
    double Cd = cd * cd;
    double lg = 1.5 - log10(Re);
    double chi = 3.7 - 0.65 * exp(-(lg * lg) / 2.0);
    double coef = 0.125 * Cd * c.rho_f * M_PI * de * de * sm * pow(np, -chi);
    for (int k = 0; k < 3; ++k) fd[k] = c.k3 * coef * s[k] * cdr;
  }
  for (int k = 0; k < 3; ++k) fb[k] = -V * (gp[k] + c.rho_f * c.g[k]);
}

template <typename R>
__global__ __launch_bounds__(256) void k_fluid_drag(const DevState* __restrict__ dp, int buf) {
  const DevState& d = *dp;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  // one round trip: the abort flag and every input of particle i
  const int ab = *G((const int32_t*)d.abort);
  const int32_t sl = G((const int32_t*)d.sample)[i];
  const uint8_t al = G((const uint8_t*)d.alive[buf])[i];
  const int32_t key = G((const int32_t*)d.dkey)[i];
  const double4 fr = gld(G((const double4*)d.dfr) + i);
  const double4 v = gld(G((const double4*)d.vel[buf]) + i);
  const double r = G((const double*)d.xr[buf])[4 * i + 3];
  const double cdr = d.cdrag ? G((const double*)d.cdrag)[i] : 1.0;
  asm volatile("" ::"s"(ab), "v"(sl), "v"((int)al), "v"(key));
  if (ab) return;
  per_sample(sl, [&](int sc) {
    const SampleConst& c = sample_const(d.sc, sc);
    if (!al || !c.fluid_on) {
      ((R4<R>*)d.fdr)[i] = mk4<R>(0, 0, 0, 0);
      d.fpart[i] = make_double4(0, 0, 0, 0);
      return;
    }
    double np, u[3], gp[3];
    particle_fluid(d, c, key, fr, np, u, gp);
    double fd[3], fb[3];
    drag_force(c, np, u, gp, v, r, fr.w, cdr, fd, fb);
    d.fpart[i] = make_double4(fd[0], fd[1], fd[2], 0.0);
    ((R4<R>*)d.fdr)[i] = mk4<R>((R)(fd[0] + fb[0]), (R)(fd[1] + fb[1]), (R)(fd[2] + fb[2]), (R)0);
  });
}

template <typename R> void launch_fluid(DevState& d, int buf, hipStream_t s) {
  hipLaunchKernelGGL(k_fluid_key, dim3(nblk(d.n)), dim3(kBlock), 0, s, d.self, buf);
  // more than 32 particles per bucket on average: a wave per bucket
  const bool dense = d.n > 32 * d.ndual;
  if (dense)
    hipLaunchKernelGGL(k_fluid_partials_wave<0>, dim3(nblk(d.ndual * 64)), dim3(kBlock), 0, s, d.self);
  else
    hipLaunchKernelGGL(k_fluid_partials<0>, dim3(nblk(d.ndual * 8)), dim3(kBlock), 0, s, d.self);
  if (d.ncell > 0) hipLaunchKernelGGL(k_fluid_cells<0>, dim3(nblk(d.ncell * 8)), dim3(kBlock), 0, s, d.self);
  if (d.closure_on) {
    hipLaunchKernelGGL(k_closure_features<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d.self, buf);
    launch_closure_infer(d, s);
  }
  hipLaunchKernelGGL(k_fluid_drag<R>, dim3(nblk(d.n)), dim3(kBlock), 0, s, d.self, buf);
  if (dense)
    hipLaunchKernelGGL(k_fluid_partials_wave<1>, dim3(nblk(d.ndual * 64)), dim3(kBlock), 0, s, d.self);
  else
    hipLaunchKernelGGL(k_fluid_partials<1>, dim3(nblk(d.ndual * 8)), dim3(kBlock), 0, s, d.self);
  if (d.ncell > 0) hipLaunchKernelGGL(k_fluid_cells<1>, dim3(nblk(d.ncell * 8)), dim3(kBlock), 0, s, d.self);
}
template void launch_fluid<double>(DevState&, int, hipStream_t);
template void launch_fluid<float>(DevState&, int, hipStream_t);

}  // namespace dem
