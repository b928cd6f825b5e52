// dem_sort.hip -- exclusive scan and the stable bucket sort used by the
// neighbour-list rebuild (bucket = binning cell) and by the coupling (bucket =
// cell of the grid of fluid-cell centres).  The order produced is a function
// of the keys and tie-break values only, never of scheduling.
#include "dem_device.h"

namespace dem {

// ---------------------------------------------------------------------------
// exclusive scan of int32, three phases; in and out may alias
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
// stable bucket sort: count, scan, scatter to arbitrary slots, then rank every
// bucket's members by (tiebreak, index) -- one wavefront per bucket, members
// staged in LDS when the bucket holds at most 64 of them.  Sink buckets (dead
// particles, particles outside every fluid grid) keep the scatter order,
// written directly to the output: their order reaches no result, and a sink
// can hold a large share of all particles, where the rank (quadratic in the
// bucket size) would not scale.  With a gate flag set, the whole sort does
// nothing.
// ---------------------------------------------------------------------------

// Adds 1 to ctr[k] for every valid lane and returns the lane's slot (the
// counter's value before its own addition).  The first two buckets of the wave
// add per wave (one atomic each, every lane taking its rank among the wave's
// members of that bucket), the remaining lanes one atomic each.  Particles
// arrive in spatial order, so a wave often holds few buckets, and the members
// of a sink bucket (the dead particles) all add to one counter from every XCD
// of the chip: one contended address, whose atomics would serialise across the
// chip as the dead particles accumulate.  More passes would chain their
// atomics where every lane has a bucket of its own (coarse particles).
__device__ inline int32_t bucket_add(int32_t* ctr, uint32_t k, bool valid) {
  const int lane = threadIdx.x & 63;
  int32_t slot = 0;
  bool todo = valid;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const uint64_t pend = __ballot(todo);
    if (!pend) break;                  // wave-uniform
    const int leader = __builtin_ctzll(pend);
    const uint32_t kl = (uint32_t)__shfl((int)k, leader);
    const bool mine = todo && k == kl;
    const uint64_t peers = __ballot(mine);
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(&ctr[kl], __popcll(peers));
    base = __shfl(base, leader);
    if (mine) {
      slot = base + __popcll(peers & ((1ull << lane) - 1ull));
      todo = false;
    }
  }
  if (todo) slot = atomicAdd(&ctr[k], 1);
  return slot;
}

__global__ void k_bucket_count(const uint32_t* key, int64_t n, int32_t* cnt, const int* gate) {
  if (gate && *gate) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const uint32_t k = valid ? key[i] : 0u;
  bucket_add(cnt, k, valid);
}

// Members of a sink bucket go straight to their final array (their order
// reaches no result); the others to the staging array that the rank reorders.
__global__ void k_bucket_scatter(const uint32_t* key, int64_t n, const int32_t* off, int32_t* fill,
                                 int32_t* order, int32_t* final_order, const uint8_t* sink, const int* gate) {
  if (gate && *gate) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const uint32_t k = valid ? key[i] : 0u;
  const bool is_sink = valid && sink && sink[k];
  const int32_t slot = bucket_add(fill, k, valid);
  if (valid) (is_sink ? final_order : order)[off[k] + slot] = (int32_t)i;
}

// The rank also clears the bucket's counter and fill level, which nothing
// reads after the scatter: the next sort finds them at zero (they start at
// zero when allocated), with no clearing launch of its own.
__global__ __launch_bounds__(256) void k_bucket_rank(const int32_t* off, int64_t nb, const int32_t* src,
                                                     const int32_t* tiebreak, int32_t* dst, const uint8_t* sink,
                                                     const int* gate, int32_t* cnt, int32_t* fill) {
  __shared__ int32_t sm[4][64];
  __shared__ int32_t sk[4][64];
  if (gate && *gate) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + w;
  int32_t lo = 0, k = 0;
  if (b < nb) {
    lo = off[b];
    k = off[b + 1] - lo;
    if (lane == 0) {
      cnt[b] = 0;
      fill[b] = 0;
    }
  }
  const bool small = k <= 64;
  if (small && lane < k) {
    int32_t v = src[lo + lane];
    sm[w][lane] = v;
    sk[w][lane] = tiebreak ? tiebreak[v] : v;
  }
  __syncthreads();
  if (b >= nb || k == 0) return;
  if (sink && sink[b]) return;   // written by the scatter
  if (small) {
    if (lane < k) {
      int32_t v = sm[w][lane], kv = sk[w][lane], rank = 0;
      for (int u = 0; u < k; ++u) {
        int32_t ku = sk[w][u];
        rank += (ku < kv || (ku == kv && sm[w][u] < v)) ? 1 : 0;
      }
      dst[lo + rank] = v;
    }
  } else {
    for (int32_t t = lane; t < k; t += 64) {
      int32_t v = src[lo + t];
      int32_t kv = tiebreak ? tiebreak[v] : v;
      int32_t rank = 0;
      for (int32_t u = 0; u < k; ++u) {
        int32_t x = src[lo + u];
        int32_t ku = tiebreak ? tiebreak[x] : x;
        rank += (ku < kv || (ku == kv && x < v)) ? 1 : 0;
      }
      dst[lo + rank] = v;
    }
  }
}

void launch_bucket_sort(const uint32_t* key, int64_t n, int64_t nb, const int32_t* tiebreak, int32_t* cnt,
                        int32_t* off, int32_t* fill, int32_t* order_tmp, int32_t* out_order,
                        int32_t* scan_tmp, const uint8_t* sink, const int* gate, hipStream_t s) {
  // cnt and fill are zero on entry: cleared by the previous sort's rank (see
  // k_bucket_rank) and at allocation
  if (n > 0) hipLaunchKernelGGL(k_bucket_count, dim3(nblk(n)), dim3(kBlock), 0, s, key, n, cnt, gate);
  scan_exclusive(cnt, off, nb + 1, scan_tmp, s);
  if (n > 0)
    hipLaunchKernelGGL(k_bucket_scatter, dim3(nblk(n)), dim3(kBlock), 0, s, key, n, off, fill, order_tmp,
                       out_order, sink, gate);
  hipLaunchKernelGGL(k_bucket_rank, dim3(nblk(nb, 4)), dim3(256), 0, s, off, nb, order_tmp, tiebreak, out_order,
                     sink, gate, cnt, fill);
}

}  // namespace dem
