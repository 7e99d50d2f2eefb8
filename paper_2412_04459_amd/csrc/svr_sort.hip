// Stable LSD radix sort of (u64 key, u32 value) pairs for gfx950, in the
// single-pass-per-digit ("onesweep") form: one kernel reads the keys once and
// builds the digit histograms of every pass; then each 8-bit digit pass is one
// kernel in which a workgroup
//   1. takes a partition of kSortPart pairs in the order given by an atomic ticket
//      (so every partition it waits on is already running),
//   2. ranks its keys stably with wave64 ballots (a match on the 8 digit bits
//      per lane gives each lane its peers) and per-wave digit counters in LDS,
//   3. publishes its per-digit counts and looks back over the preceding
//      partitions' published counts (decoupled look-back) to find where each
//      of its digit runs starts in the output,
//   4. reorders the pairs in LDS by digit and writes each run contiguously.
// This is the sort of Sec. 3.1.2 "Sorting voxels" (Supp. B.1 uses a GPU radix
// sort on the tile / Morton key).  Look-back waits are bounded: a workgroup
// that spins past the limit sets an error bit and finishes, so no launch can
// hang.
#include <type_traits>

#include "svr_internal.h"

namespace svr {

constexpr int kRadix = 256;
constexpr int kPart = kSortPart;
constexpr uint32_t kFlagAgg = 1u << 30;          // partition-local count published
constexpr uint32_t kFlagPre = 2u << 30;          // inclusive prefix published
constexpr uint32_t kValMask = (1u << 30) - 1u;
constexpr int kSpinLimit = 1 << 22;
constexpr int kLookWin = 16;                     // partitions read per look-back round

__device__ __forceinline__ unsigned long long lane_mask_lt() {
  const int lane = threadIdx.x & 63;
  return (1ull << lane) - 1ull;
}

// ---------------------------------------------------------------------------
// digit histograms of key bits [lo, lo + bits), 8 bits per pass
__global__ __launch_bounds__(kBlock) void k_sort_hist(const uint64_t* __restrict__ keys,
                                                      const unsigned long long* __restrict__ n_dev,
                                                      int64_t n_max, int bits, int lo,
                                                      uint32_t* __restrict__ hist) {
  const int passes = (bits + 7) / 8;
  __shared__ uint32_t h[8 * kRadix];
  for (int i = threadIdx.x; i < 8 * kRadix; i += kBlock) h[i] = 0;
  __syncthreads();
  const int64_t n = min((int64_t)*n_dev, n_max);
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const uint64_t k = keys[i];
    for (int p = 0; p < passes; ++p) {
      const uint32_t dmask = (bits - 8 * p >= 8) ? 255u : ((1u << (bits - 8 * p)) - 1u);
      atomicAdd(&h[p * kRadix + (int)((k >> (lo + 8 * p)) & dmask)], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < passes * kRadix; i += kBlock)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// exclusive scan of each pass's 256 digit counts
__global__ __launch_bounds__(kRadix) void k_sort_hist_scan(uint32_t* __restrict__ hist, int passes) {
  __shared__ uint32_t wsum[kRadix / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int p = 0; p < passes; ++p) {
    uint32_t v = hist[p * kRadix + threadIdx.x];
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t t = __shfl_up(inc, d, 64);
      if (lane >= d) inc += t;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int i = 0; i < w; ++i) base += wsum[i];
    hist[p * kRadix + threadIdx.x] = base + inc - v;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_sort_pass(
    int shift, uint32_t dmask, const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
    const unsigned long long* __restrict__ n_dev, int64_t n_max,
    const uint32_t* __restrict__ digit_base, uint32_t* __restrict__ status,
    uint32_t* __restrict__ status_next, uint32_t* __restrict__ ticket, uint32_t* __restrict__ err) {
  __shared__ uint64_t sk[kPart];
  __shared__ uint32_t sv[kPart];
  __shared__ uint32_t wh[4][kRadix];   // per-wave digit counters, then wave offsets
  __shared__ uint32_t dstart[kRadix];  // first local position of each digit
  __shared__ uint32_t gbase[kRadix];   // first global position of each digit
  __shared__ uint32_t wsum[4];
  __shared__ int s_part;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_part = (int)atomicAdd(ticket, 1u);
#pragma unroll
  for (int i = 0; i < 4; ++i) wh[i][tid] = 0;
  __syncthreads();
  const int part = s_part;
  const int64_t n = min((int64_t)*n_dev, n_max);
  const int64_t nparts = (n + kPart - 1) / kPart;
  if (part >= nparts) return;
  const int64_t base = (int64_t)part * kPart;

  uint64_t k[kSortItems];
  uint32_t v[kSortItems];
  uint32_t rank[kSortItems];
  const int64_t wbase = base + (int64_t)w * (kSortItems * 64) + lane;
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const int64_t idx = wbase + it * 64;
    if (idx < n) {
      k[it] = kin[idx];
      v[it] = vin[idx];
    } else {
      k[it] = 0;
      v[it] = 0;
    }
  }
  const unsigned long long lt = lane_mask_lt();
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const bool valid = wbase + it * 64 < n;
    const uint32_t d = (uint32_t)(k[it] >> shift) & dmask;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt);
    uint32_t cbase = 0;
    if (valid) cbase = wh[w][d];
    rank[it] = cbase + below;
    if (valid && below == 0) wh[w][d] = cbase + (uint32_t)__popcll(peers);
  }
  __syncthreads();

  // per-digit totals, wave offsets, local digit starts
  const uint32_t c0 = wh[0][tid], c1 = wh[1][tid], c2 = wh[2][tid], c3 = wh[3][tid];
  const uint32_t tot = c0 + c1 + c2 + c3;
  wh[0][tid] = 0;
  wh[1][tid] = c0;
  wh[2][tid] = c0 + c1;
  wh[3][tid] = c0 + c1 + c2;
  uint32_t inc = tot;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t wb = 0;
  for (int i = 0; i < w; ++i) wb += wsum[i];
  dstart[tid] = wb + inc - tot;

  // decoupled look-back for digit `tid`: each round reads the status words of
  // the next kLookWin preceding partitions at once (independent loads, one
  // round trip) and consumes them nearest first, up to the first one not yet
  // published or the first inclusive prefix.  Only counts travel through the
  // status words, so relaxed device-scope atomics suffice.
  uint32_t* my = status + (int64_t)part * kRadix + tid;
  uint32_t prefix = 0;
  if (part == 0) {
    __hip_atomic_store(my, kFlagPre | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_store(my, kFlagAgg | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int j = part - 1;
    int spins = 0;
    while (true) {
      uint32_t st[kLookWin];
#pragma unroll
      for (int k = 0; k < kLookWin; ++k) {
        const int jj = j - k;
        st[k] = jj >= 0 ? __hip_atomic_load(status + (int64_t)jj * kRadix + tid, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : kFlagPre;
      }
      int used = 0;
      bool stop = false, fin = false;
#pragma unroll
      for (int k = 0; k < kLookWin; ++k) {
        if (stop) continue;
        const uint32_t flag = st[k] & ~kValMask;
        if (flag == 0u) {
          stop = true;
        } else {
          prefix += st[k] & kValMask;
          ++used;
          if (flag == kFlagPre) stop = fin = true;
        }
      }
      if (fin) break;
      j -= used;
      if (used == 0) {
        if (++spins > kSpinLimit) {
          atomicOr(err, 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __hip_atomic_store(my, kFlagPre | ((prefix + tot) & kValMask), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  gbase[tid] = digit_base[tid] + prefix;
  // the next pass uses the other status buffer: clear this partition's row
  status_next[(int64_t)part * kRadix + tid] = 0u;
  __syncthreads();

  // reorder in LDS by digit (stable), then write each digit run out
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    if (wbase + it * 64 < n) {
      const uint32_t d = (uint32_t)(k[it] >> shift) & dmask;
      const uint32_t pos = dstart[d] + wh[w][d] + rank[it];
      sk[pos] = k[it];
      sv[pos] = v[it];
    }
  }
  __syncthreads();
  const int nvalid = (int)min((int64_t)kPart, n - base);
  for (int i = tid; i < nvalid; i += kBlock) {
    const uint64_t kk = sk[i];
    const uint32_t d = (uint32_t)(kk >> shift) & dmask;
    const uint32_t dst = gbase[d] + ((uint32_t)i - dstart[d]);
    if ((int64_t)dst < n) {  // always true unless a look-back gave up (error bit set)
      kout[dst] = kk;
      vout[dst] = sv[i];
    }
  }
}

size_t sort_scratch_bytes(int64_t n, int bits, int64_t* parts_out) {
  const int64_t parts = (n + kPart - 1) / kPart;
  if (parts_out) *parts_out = parts;
  const int passes = (bits + 7) / 8;
  (void)passes;
  // hist [8][256] + two status buffers [parts][256] + tickets/err (64 words)
  return (size_t)(8 * kRadix + 2 * (parts > 0 ? parts : 1) * kRadix + 64) * sizeof(uint32_t);
}

hipError_t launch_radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                             const unsigned long long* n_dev, int64_t n_max, int key_bits, int lo,
                             uint32_t* hist, uint32_t* st0, uint32_t* st1, uint32_t* tickets,
                             uint32_t* err, bool* result_in_1, hipStream_t s) {
  // sort by key bits [lo, key_bits); the order of equal digits is kept
  const int bits = key_bits > lo ? key_bits - lo : 0;
  const int passes = (bits + 7) / 8;
  *result_in_1 = (passes & 1) != 0;
  if (n_max <= 0 || passes == 0) {
    *result_in_1 = false;
    return hipSuccess;
  }
  const int64_t parts = (n_max + kPart - 1) / kPart;
  hipError_t e;
  FillSet z;
  z.add(hist, 8 * kRadix);
  z.add(tickets, 16);
  z.add(st0, parts * kRadix);
  if ((e = launch_zero_u32(z, s)) != hipSuccess) return e;
  // few workgroups: each flushes up to 8 x 256 device-scope atomics into the
  // same histogram, which costs more than streaming more keys per workgroup
  int64_t hb = (n_max + kBlock * 8 - 1) / (kBlock * 8);
  if (hb > 256) hb = 256;
  if (hb < 1) hb = 1;
  SVR_LAUNCH("sort_hist", k_sort_hist, dim3((unsigned)hb), dim3(kBlock), 0, s, k0, n_dev, n_max, bits,
                     lo, hist);
  SVR_LAUNCH("sort_hist_scan", k_sort_hist_scan, dim3(1), dim3(kRadix), 0, s, hist, passes);
  for (int p = 0; p < passes; ++p) {
    const uint64_t* ki = (p & 1) ? k1 : k0;
    const uint32_t* vi = (p & 1) ? v1 : v0;
    uint64_t* ko = (p & 1) ? k0 : k1;
    uint32_t* vo = (p & 1) ? v0 : v1;
    uint32_t* st = (p & 1) ? st1 : st0;
    uint32_t* stn = (p & 1) ? st0 : st1;
    const uint32_t dmask = (bits - 8 * p >= 8) ? 255u : ((1u << (bits - 8 * p)) - 1u);
    SVR_LAUNCH("sort_pass", k_sort_pass, dim3((unsigned)parts), dim3(kBlock), 0, s, lo + 8 * p, dmask, ki,
                       vi, ko, vo, n_dev, n_max, hist + p * kRadix, st, stn, tickets + p, err);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_tile_ranges(const uint64_t* __restrict__ keys,
                                                        const unsigned long long* __restrict__ n_dev,
                                                        int64_t cap, int shift, uint32_t T,
                                                        uint2* __restrict__ range,
                                                        uint32_t* __restrict__ counters) {
  if (blockIdx.x == 0 && threadIdx.x <= (unsigned)kOrderBuckets) counters[threadIdx.x] = 0u;
  const int64_t n = min((int64_t)*n_dev, cap);
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = (uint32_t)(keys[i] >> shift);
  if (t >= T) return;
  if (i == 0 || (uint32_t)(keys[i - 1] >> shift) != t) range[t].x = (uint32_t)i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> shift) != t) range[t].y = (uint32_t)(i + 1);
}

// Render order of the tiles: heaviest first, so that the long tiles start
// early and the short ones fill in behind them.  Bucket b holds the tiles
// whose entry count n has floor(log2(max(n, 1))) = kOrderBuckets - 1 - b
// (capped); within a bucket the order is arbitrary.
__device__ __forceinline__ uint32_t order_bucket(uint2 r) {
  const uint32_t n = r.y - r.x;
  const int lg = 31 - __clz((int)(n | 1u));
  return (uint32_t)(kOrderBuckets - 1 - min(lg, kOrderBuckets - 1));
}

// rank of each tile within its bucket: a workgroup counts its tiles per
// bucket in LDS, then reserves each bucket's run with one global atomic
//
// The same pass lists the backward chunks of heavy tiles: a tile of n >
// kBwdChunk entries reserves ceil(n / kBwdChunk) - 1 items (tile, chunk) for
// all its chunks but the last, and records where they start (split_base).
__global__ __launch_bounds__(kBlock) void k_tile_bucket(const uint2* __restrict__ range, uint32_t T,
                                                        uint32_t* __restrict__ bucket_count,
                                                        uint32_t* __restrict__ rank,
                                                        uint32_t* __restrict__ split_count,
                                                        uint32_t* __restrict__ split_base,
                                                        uint2* __restrict__ split_items,
                                                        uint32_t max_split,
                                                        uint32_t* __restrict__ err,
                                                        uint32_t* __restrict__ tile_count) {
  __shared__ uint32_t cnt[kOrderBuckets], base[kOrderBuckets];
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (threadIdx.x < kOrderBuckets) cnt[threadIdx.x] = 0;
  __syncthreads();
  uint32_t b = 0, local = 0;
  if (t < T) {
    if (tile_count) tile_count[t] = 0u;  // ready for the next counting sort
    const uint2 r = range[t];
    b = order_bucket(r);
    local = atomicAdd(cnt + b, 1u);
    const uint32_t nch = (r.y - r.x + kBwdChunk - 1) / kBwdChunk;
    uint32_t sb = kNoSplit;
    if (nch > 1) {
      const uint32_t at_ = atomicAdd(split_count, nch - 1);
      if (at_ + (nch - 1) <= max_split) {
        sb = at_;
        for (uint32_t m = 0; m + 1 < nch; ++m) split_items[at_ + m] = make_uint2(t, m);
      } else {
        atomicOr(err, 2u);  // cannot happen while the ranges hold <= capacity entries
      }
    }
    split_base[t] = sb;
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && cnt[threadIdx.x] > 0)
    base[threadIdx.x] = atomicAdd(bucket_count + threadIdx.x, cnt[threadIdx.x]);
  __syncthreads();
  if (t < T) rank[t] = base[b] + local;
}

__global__ __launch_bounds__(kBlock) void k_tile_scatter(const uint2* __restrict__ range, uint32_t T,
                                                         const uint32_t* __restrict__ bucket_count,
                                                         const uint32_t* __restrict__ rank,
                                                         uint32_t* __restrict__ order) {
  const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= T) return;
  const uint32_t b = order_bucket(range[t]);
  uint32_t base = 0;
  for (uint32_t i = 0; i < b; ++i) base += bucket_count[i];
  order[base + rank[t]] = t;
}

// ---------------------------------------------------------------------------
// Counting sort by tile (frames of at most kCountTiles tiles whose keys are
// unique within a tile).  Each workgroup owns a chunk of kCountChunk pairs of
// the emitted list:
//   k_tile_count   counts its pairs per tile in an LDS histogram of every
//                  tile and adds the non-zero counts to the global ones
//                  (cleared by the tile-mask kernel of the pre-process, and
//                  again by the tile-order pass after use);
//   k_tile_offsets (one workgroup) turns the counts into the tile ranges
//                  (exclusive scan) and leaves each range's start as the
//                  tile's next free position;
//   k_tile_place   ranks its pairs per tile in LDS, reserves its run of
//                  each tile with one atomic on that position and writes
//                  every pair there.
// Within a tile the pairs land in no fixed order; the tile-range sort that
// follows orders them by their low key bits, which are unique within a tile,
// so the sorted list is the same as after the stable radix passes.  The
// histograms take T words of dynamic LDS.
constexpr int kCountBlock = 1024;
constexpr int kCountPer = 4;  // pairs per thread
constexpr int kCountChunk = kCountBlock * kCountPer;

__global__ __launch_bounds__(kCountBlock) void k_tile_count(const uint64_t* __restrict__ keys,
                                                            const unsigned long long* __restrict__ n_dev,
                                                            int64_t n_max, int shift, uint32_t T,
                                                            uint32_t* __restrict__ count) {
  extern __shared__ uint32_t h[];
  const int64_t n = min((int64_t)*n_dev, n_max);
  const int64_t c0 = (int64_t)blockIdx.x * kCountChunk;
  if (c0 >= n) return;
  uint32_t tt[kCountPer];
#pragma unroll
  for (int k = 0; k < kCountPer; ++k) {
    const int64_t i = c0 + (int64_t)k * kCountBlock + threadIdx.x;
    tt[k] = i < n ? (uint32_t)(keys[i] >> shift) : 0xffffffffu;
  }
  for (uint32_t t = threadIdx.x; t < T; t += kCountBlock) h[t] = 0u;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kCountPer; ++k)
    if (tt[k] < T) atomicAdd(&h[tt[k]], 1u);
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < T; t += kCountBlock) {
    const uint32_t c = h[t];
    if (c) atomicAdd(&count[t], c);
  }
}

// one workgroup: range[t] = [o_t, o_t + count_t) with o the exclusive scan of
// the counts; count[t] becomes o_t.  Also clears the render-order counters
// (as k_tile_ranges does).  A total other than the entry count (counts left
// over from another frame) sets error bit 2 and leaves every range empty, so
// that no later pass reads positions the placement did not write.
__global__ __launch_bounds__(kCountBlock) void k_tile_offsets(uint32_t* __restrict__ count, uint32_t T,
                                                              const unsigned long long* __restrict__ n_dev,
                                                              int64_t n_max, uint2* __restrict__ range,
                                                              uint32_t* __restrict__ counters,
                                                              uint32_t* __restrict__ err) {
  constexpr int kPerThread = kCountTiles / kCountBlock;
  __shared__ uint32_t o[kCountTiles + 1];
  __shared__ uint32_t wsum[kCountBlock / 64];
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid <= kOrderBuckets) counters[tid] = 0u;
  {
    uint32_t c[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const uint32_t t = (uint32_t)(k * kCountBlock + tid);
      c[k] = t < T ? count[t] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) o[k * kCountBlock + tid] = c[k];
  }
  __syncthreads();
  // thread tid scans the run [t0, t1) of consecutive tiles
  const uint32_t per = (T + kCountBlock - 1) / kCountBlock;
  const uint32_t t0 = min((uint32_t)tid * per, T), t1 = min(t0 + per, T);
  uint32_t sum = 0u;
  for (uint32_t t = t0; t < t1; ++t) sum += o[t];
  uint32_t inc = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t v = __shfl_up(inc, d, 64);
    if (lane >= d) inc += v;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = inc - sum;
  for (int i = 0; i < w; ++i) off += wsum[i];
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t c = o[t];
    o[t] = off;
    off += c;
  }
  if (tid == kCountBlock - 1) {
    o[T] = off;
    s_bad = (int64_t)off != min((int64_t)*n_dev, n_max);
    if (s_bad) atomicOr(err, 4u);
  }
  __syncthreads();
  const bool bad = s_bad != 0;
  for (uint32_t t = tid; t < T; t += kCountBlock) {
    const uint32_t a = o[t], b = o[t + 1];
    range[t] = bad ? make_uint2(0u, 0u) : make_uint2(a, b);
    count[t] = a;
  }
}

__global__ __launch_bounds__(kCountBlock) void k_tile_place(const uint64_t* __restrict__ kin,
                                                            const uint32_t* __restrict__ vin,
                                                            uint64_t* __restrict__ kout,
                                                            uint32_t* __restrict__ vout,
                                                            const unsigned long long* __restrict__ n_dev,
                                                            int64_t n_max, int shift, uint32_t T,
                                                            uint32_t* __restrict__ next,
                                                            uint32_t* __restrict__ err) {
  extern __shared__ uint32_t h[];
  const int64_t n = min((int64_t)*n_dev, n_max);
  const int64_t c0 = (int64_t)blockIdx.x * kCountChunk;
  if (c0 >= n) return;
  uint64_t kk[kCountPer];
  uint32_t vv[kCountPer], tt[kCountPer], rk[kCountPer];
#pragma unroll
  for (int k = 0; k < kCountPer; ++k) {
    const int64_t i = c0 + (int64_t)k * kCountBlock + threadIdx.x;
    tt[k] = 0xffffffffu;
    kk[k] = 0ull;
    vv[k] = 0u;
    rk[k] = 0u;
    if (i < n) {
      kk[k] = kin[i];
      vv[k] = vin[i];
    }
  }
  for (uint32_t t = threadIdx.x; t < T; t += kCountBlock) h[t] = 0u;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kCountPer; ++k) {
    const int64_t i = c0 + (int64_t)k * kCountBlock + threadIdx.x;
    if (i < n) tt[k] = (uint32_t)(kk[k] >> shift);
    if (tt[k] < T) rk[k] = atomicAdd(&h[tt[k]], 1u);
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < T; t += kCountBlock) {
    const uint32_t c = h[t];
    if (c) h[t] = atomicAdd(&next[t], c);
  }
  __syncthreads();
  bool bad = false;
#pragma unroll
  for (int k = 0; k < kCountPer; ++k) {
    if (tt[k] < T) {
      const uint32_t pos = h[tt[k]] + rk[k];
      if ((int64_t)pos < n) {
        kout[pos] = kk[k];
        vout[pos] = vv[k];
      } else {
        bad = true;
      }
    }
  }
  if (bad) atomicOr(err, 4u);
}

static hipError_t launch_tile_order(const Layout& L, void* ws, hipStream_t s) {
  uint2* range = at<uint2>(ws, L.tile_range);
  uint32_t* counts = at<uint32_t>(ws, L.tile_range) + 2 * (int64_t)L.T;
  uint32_t* split_count = counts + kOrderBuckets;
  const dim3 tg((unsigned)((L.T + kBlock - 1) / kBlock));
  SVR_LAUNCH("tile_order", k_tile_bucket, tg, dim3(kBlock), 0, s, range, (uint32_t)L.T, counts,
             at<uint32_t>(ws, L.tile_rank), split_count, at<uint32_t>(ws, L.split_base),
             at<uint2>(ws, L.split_items), (uint32_t)L.max_split, &at<WsHeader>(ws, L.hdr)->error,
             L.count_sort ? at<uint32_t>(ws, L.tile_count) : nullptr);
  SVR_LAUNCH("tile_order", k_tile_scatter, tg, dim3(kBlock), 0, s, range, (uint32_t)L.T, counts,
             at<uint32_t>(ws, L.tile_rank), at<uint32_t>(ws, L.tile_order));
  return hipGetLastError();
}

hipError_t launch_tile_ranges(const Layout& L, void* ws, const uint64_t* keys, hipStream_t s) {
  // the ranges start empty (cleared with the tile masks); the bucket and
  // chunk counters behind them are cleared by the first workgroup here
  uint2* range = at<uint2>(ws, L.tile_range);
  uint32_t* counts = at<uint32_t>(ws, L.tile_range) + 2 * (int64_t)L.T;
  // at least one workgroup: the first one clears the counters
  SVR_LAUNCH("tile_ranges", k_tile_ranges,
             dim3((unsigned)max((L.cap + kBlock - 1) / kBlock, (int64_t)1)), dim3(kBlock), 0, s, keys,
             &at<WsHeader>(ws, L.hdr)->n_entries, L.cap, L.key_low, (uint32_t)L.T, range, counts);
  return launch_tile_order(L, ws, s);
}

hipError_t launch_tile_count_sort(const Layout& L, void* ws, int64_t n_max, hipStream_t s) {
  // keys0/vals0 (emission order) -> keys1/vals1 bucketed by tile; the counts
  // start at zero (tile-mask kernel of the pre-process, or the tile-order
  // pass of the previous sort)
  if (L.T <= 0 || L.T > kCountTiles) return hipErrorInvalidValue;
  uint32_t* count = at<uint32_t>(ws, L.tile_count);
  WsHeader* hdr = at<WsHeader>(ws, L.hdr);
  const uint32_t T = (uint32_t)L.T;
  const size_t lds = (size_t)T * 4;
  const dim3 grid((unsigned)max((n_max + kCountChunk - 1) / kCountChunk, (int64_t)1));
  SVR_LAUNCH("tile_count", k_tile_count, grid, dim3(kCountBlock), lds, s, at<uint64_t>(ws, L.keys0),
             &hdr->n_entries, n_max, L.key_low, T, count);
  SVR_LAUNCH("tile_ranges", k_tile_offsets, dim3(1), dim3(kCountBlock), 0, s, count, T, &hdr->n_entries,
             n_max, at<uint2>(ws, L.tile_range), at<uint32_t>(ws, L.tile_range) + 2 * (int64_t)L.T,
             &hdr->error);
  SVR_LAUNCH("tile_place", k_tile_place, grid, dim3(kCountBlock), lds, s, at<uint64_t>(ws, L.keys0),
             at<uint32_t>(ws, L.vals0), at<uint64_t>(ws, L.keys1), at<uint32_t>(ws, L.vals1),
             &hdr->n_entries, n_max, L.key_low, T, count, &hdr->error);
  return launch_tile_order(L, ws, s);
}

// ---------------------------------------------------------------------------
// Order within each tile.  The radix sort orders the entries by tile only
// (the key's high bits) and keeps the emission order within a tile; these
// kernels then sort every tile's range [start, end) in place by the key's low
// bits (the tile bits are equal), which gives exactly the order of a full
// sort of the keys.  Short ranges take a counting rank, one wave per tile;
// long ones LSD radix passes over the low key bits, in LDS up to SEG
// entries, else through the other key/value buffer.  Low key bits are held
// as K (32 bits when they fit).


// tiles of fewer than kSmallSeg entries: one wave each, rank = number of
// smaller keys in the range.  Order ranks are unique within a tile; 64-bit
// low keys (at most 3 * 16 + 3 = 51 bits) carry the entry's index in the
// range below them (kIdxBits), so equal keys keep their order as in a
// stable sort.
constexpr int kSmallSeg = 256;
constexpr int kIdxBits = 13;

template <typename K>
__device__ __forceinline__ K seg_key(uint64_t key, uint64_t lowmask, int i) {
  if (sizeof(K) == 8) return (K)(((key & lowmask) << kIdxBits) | (uint64_t)i);
  return (K)(key & lowmask);
}

template <typename K>
__device__ __forceinline__ uint64_t seg_low(K k) {
  return sizeof(K) == 8 ? (uint64_t)k >> kIdxBits : (uint64_t)k;
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_tile_sort_small(uint64_t* __restrict__ keys,
                                                            uint32_t* __restrict__ vals,
                                                            const uint2* __restrict__ range,
                                                            const uint32_t* __restrict__ order,
                                                            uint32_t T, int lo_bits) {
  constexpr int kWaves = kBlock / 64;
  __shared__ K sk[kWaves][kSmallSeg];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t pos = blockIdx.x * kWaves + w;
  if (pos >= T) return;
  const uint32_t t = order[pos];
  if (t >= T) return;
  const uint2 r = range[t];
  const int n = (int)(r.y - r.x);
  if (n <= 1 || n >= kSmallSeg) return;
  const uint64_t lowmask = lo_bits >= 64 ? ~0ull : ((1ull << lo_bits) - 1ull);
  const uint64_t high = keys[r.x] & ~lowmask;
  if (n <= 64) {
    // one entry per lane; the keys come from the other lanes' registers
    const bool valid = lane < n;
    const K k0 = valid ? seg_key<K>(keys[r.x + lane], lowmask, lane) : (K)~(K)0;
    const uint32_t v0 = valid ? vals[r.x + lane] : 0u;
    int rank0 = 0;
    for (int j = 0; j < n; ++j) {
      K kj;
      if (sizeof(K) == 8) {
        const uint64_t u = (uint64_t)k0;
        kj = (K)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), j) << 32) |
                 (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, j));
      } else {
        kj = (K)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)k0, j);
      }
      rank0 += kj < k0 ? 1 : 0;
    }
    if (valid) {
      keys[r.x + rank0] = high | seg_low<K>(k0);
      vals[r.x + rank0] = v0;
    }
    return;
  }
  // up to P entries per lane (entry lane + 64 e), each compared with every
  // key of the range (LDS broadcast reads)
  auto count_rank = [&](auto per) {
    constexpr int P = decltype(per)::value;
    K k[P];
    uint32_t v[P];
    int rank[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int i = lane + 64 * e;
      k[e] = i < n ? seg_key<K>(keys[r.x + i], lowmask, i) : (K)0;
      v[e] = i < n ? vals[r.x + i] : 0u;
      if (i < n) sk[w][i] = k[e];
      rank[e] = 0;
    }
    wave_sync_lds();
    for (int j = 0; j < n; ++j) {
      const K kj = sk[w][j];
#pragma unroll
      for (int e = 0; e < P; ++e) rank[e] += kj < k[e] ? 1 : 0;
    }
#pragma unroll
    for (int e = 0; e < P; ++e) {
      if (lane + 64 * e < n) {
        keys[r.x + rank[e]] = high | seg_low<K>(k[e]);
        vals[r.x + rank[e]] = v[e];
      }
    }
  };
  if (n <= 128) count_rank(std::integral_constant<int, 2>());
  else count_rank(std::integral_constant<int, kSmallSeg / 64>());
}



// tiles of kSmallSeg or more entries: they open the render order (heaviest
// first, bucketed by floor(log2 n)), so the workgroups walk the order from
// the front, one tile at a time, and stop at the first shorter tile
// one LSD radix pass (digit (key >> shift) & dmask) of n entries from
// (ka, va) to (kb, vb), stable, by a workgroup of kBlock threads; base and wc
// are LDS scratch (base: kRadix words, wc: one kRadix row per wave)
template <typename KA, typename KB>
__device__ __forceinline__ void radix_pass_wg(const KA* ka, const uint32_t* va, KB* kb, uint32_t* vb,
                                              int n, int shift, uint32_t dmask, uint32_t* base,
                                              uint32_t (*wc)[kRadix]) {
  constexpr int kWaves = kBlock / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  // digit counts, then their exclusive scan
  base[tid] = 0u;
  __syncthreads();
  for (int i = tid; i < n; i += kBlock) atomicAdd(&base[(uint32_t)((uint64_t)ka[i] >> shift) & dmask], 1u);
  __syncthreads();
  {
    const uint32_t v = base[tid];
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t u = __shfl_up(inc, d, 64);
      if (lane >= d) inc += u;
    }
    if (lane == 63) wc[w][0] = inc;
    __syncthreads();
    uint32_t wb = 0;
    for (int i = 0; i < w; ++i) wb += wc[i][0];
    __syncthreads();
    base[tid] = wb + inc - v;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) wc[i][tid] = 0u;
    __syncthreads();
  }
  // stable scatter, kBlock entries at a time in index order
  for (int c0 = 0; c0 < n; c0 += kBlock) {
    const int i = c0 + tid;
    const bool valid = i < n;
    const KA kk = valid ? ka[i] : (KA)0;
    const uint32_t v = valid ? va[i] : 0u;
    const uint32_t d = (uint32_t)((uint64_t)kk >> shift) & dmask;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt);
    if (valid && below == 0) wc[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = base[d] + below;
      for (int q = 0; q < w; ++q) off += wc[q][d];
      kb[off] = (KB)kk;
      vb[off] = v;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      add += wc[q][tid];
      wc[q][tid] = 0u;
    }
    base[tid] += add;
    __syncthreads();
  }
}

// tiles of kSmallSeg or more entries: they open the render order (heaviest
// first, bucketed by floor(log2 n)), so the workgroups walk the order from
// the front, one tile at a time, and stop at the first shorter tile.  Up to
// SEG entries: LSD radix passes in LDS (ping-pong); longer: the same passes
// through the other key/value buffer.
template <typename K, int SEG>
__global__ __launch_bounds__(kBlock) void k_tile_sort_big(uint64_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals,
                                                          uint64_t* __restrict__ ktmp,
                                                          uint32_t* __restrict__ vtmp,
                                                          const uint2* __restrict__ range,
                                                          const uint32_t* __restrict__ order,
                                                          uint32_t T, int lo_bits) {
  constexpr int kWaves = kBlock / 64;
  __shared__ K sk[2][SEG];
  __shared__ uint32_t sv[2][SEG];
  __shared__ uint32_t base[kRadix];
  __shared__ uint32_t wc[kWaves][kRadix];
  const int tid = threadIdx.x;
  const uint64_t lowmask = lo_bits >= 64 ? ~0ull : ((1ull << lo_bits) - 1ull);
  const int passes = (lo_bits + 7) / 8;
  for (uint32_t pos = blockIdx.x; pos < T; pos += gridDim.x) {
    const uint32_t t = order[pos];
    if (t >= T) break;
    const uint2 r = range[t];
    const int n = (int)(r.y - r.x);
    if (n < kSmallSeg) break;  // every later tile is shorter too
    if (n <= SEG) {
      const uint64_t high = keys[r.x] & ~lowmask;
      for (int i = tid; i < n; i += kBlock) {
        sk[0][i] = (K)(keys[r.x + i] & lowmask);
        sv[0][i] = vals[r.x + i];
      }
      for (int p = 0; p < passes; ++p) {
        const uint32_t dmask = (lo_bits - 8 * p >= 8) ? 255u : ((1u << (lo_bits - 8 * p)) - 1u);
        radix_pass_wg(sk[p & 1], sv[p & 1], sk[(p + 1) & 1], sv[(p + 1) & 1], n, 8 * p, dmask, base,
                      wc);
      }
      for (int i = tid; i < n; i += kBlock) {
        keys[r.x + i] = high | (uint64_t)sk[passes & 1][i];
        vals[r.x + i] = sv[passes & 1][i];
      }
      __syncthreads();
      continue;
    }
    // long range: the passes through the other key/value buffer
    uint64_t* ks = keys + r.x;
    uint32_t* vs = vals + r.x;
    uint64_t* kd = ktmp + r.x;
    uint32_t* vd = vtmp + r.x;
    for (int p = 0; p < passes; ++p) {
      const uint32_t dmask = (lo_bits - 8 * p >= 8) ? 255u : ((1u << (lo_bits - 8 * p)) - 1u);
      radix_pass_wg(ks, vs, kd, vd, n, 8 * p, dmask, base, wc);
      uint64_t* tk = ks; ks = kd; kd = tk;
      uint32_t* tv = vs; vs = vd; vd = tv;
    }
    if (passes & 1) {
      for (int i = tid; i < n; i += kBlock) {
        keys[r.x + i] = ks[i];
        vals[r.x + i] = vs[i];
      }
    }
    __syncthreads();
  }
}

hipError_t launch_tile_sort(const Layout& L, void* ws, uint64_t* keys, uint32_t* vals, uint64_t* ktmp,
                            uint32_t* vtmp, hipStream_t s) {
  if (L.T == 0) return hipSuccess;
  const uint2* range = at<uint2>(ws, L.tile_range);
  const uint32_t* order = at<uint32_t>(ws, L.tile_order);
  const dim3 small_grid((unsigned)((L.T + kBlock / 64 - 1) / (kBlock / 64)));
  // at most cap / kSmallSeg tiles are long; a few workgroups per CU
  const int64_t nbig = min((int64_t)L.T, min(L.cap / kSmallSeg + 1, (int64_t)2048));
  const dim3 big_grid((unsigned)nbig);
  if (L.key_low <= 32) {
    SVR_LAUNCH("tile_sort_small", k_tile_sort_small<uint32_t>, small_grid, dim3(kBlock), 0, s, keys, vals,
               range, order, (uint32_t)L.T, L.key_low);
    SVR_LAUNCH("tile_sort_big", (k_tile_sort_big<uint32_t, 2048>), big_grid, dim3(kBlock), 0, s, keys,
               vals, ktmp, vtmp, range, order, (uint32_t)L.T, L.key_low);
  } else {
    SVR_LAUNCH("tile_sort_small", k_tile_sort_small<uint64_t>, small_grid, dim3(kBlock), 0, s, keys, vals,
               range, order, (uint32_t)L.T, L.key_low);
    SVR_LAUNCH("tile_sort_big", (k_tile_sort_big<uint64_t, 1024>), big_grid, dim3(kBlock), 0, s, keys,
               vals, ktmp, vtmp, range, order, (uint32_t)L.T, L.key_low);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// corner adjacency of the grid points: sort (grid index, corner slot) pairs by
// grid index (stable, so slots stay increasing), then mark where each grid
// point's run starts
__global__ __launch_bounds__(kBlock) void k_adj_pairs(const int32_t* __restrict__ vox_grid,
                                                      int64_t n8, uint64_t* __restrict__ keys,
                                                      uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n8) return;
  keys[i] = (uint64_t)(uint32_t)vox_grid[i];
  vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_adj_offsets(const uint64_t* __restrict__ keys,
                                                        int64_t n8, int64_t M,
                                                        int32_t* __restrict__ off) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i > n8) return;
  // grid points strictly between the previous key and this one start here
  const int64_t lo = i == 0 ? -1 : (int64_t)keys[i - 1];
  const int64_t hi = i == n8 ? M : min((int64_t)keys[i], M);
  for (int64_t m = lo + 1; m <= hi && m <= M; ++m) off[m] = (int32_t)i;
}

hipError_t launch_grid_adjacency(const int32_t* vox_grid, int64_t N, int64_t M, int32_t* adj_off,
                                 int32_t* adj, void* scratch, hipStream_t s) {
  const int64_t n8 = 8 * N;
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) <= M) ++bits;
  int64_t parts = 0;
  const size_t sb = sort_scratch_bytes(n8, bits, &parts);
  char* p = reinterpret_cast<char*>(scratch);
  auto take = [&](size_t b) { char* q = p; p += (b + 255) / 256 * 256; return q; };
  uint64_t* k0 = reinterpret_cast<uint64_t*>(take((size_t)n8 * 8));
  uint64_t* k1 = reinterpret_cast<uint64_t*>(take((size_t)n8 * 8));
  uint32_t* v1 = reinterpret_cast<uint32_t*>(take((size_t)n8 * 4));
  uint32_t* base = reinterpret_cast<uint32_t*>(take(sb + 256));
  auto* n_dev = reinterpret_cast<unsigned long long*>(base);
  uint32_t* hist = base + 64;
  uint32_t* st0 = hist + 8 * kRadix;
  uint32_t* st1 = st0 + (parts > 0 ? parts : 1) * kRadix;
  uint32_t* v0 = reinterpret_cast<uint32_t*>(adj);
  hipError_t e;
  if ((e = launch_fill_u32(base, 0u, 64, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(base, (uint32_t)(n8 & 0xffffffffu), 1, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(base + 1, (uint32_t)(n8 >> 32), 1, s)) != hipSuccess) return e;
  const unsigned grid = (unsigned)((n8 + kBlock - 1) / kBlock);
  SVR_LAUNCH("adj_pairs", k_adj_pairs, dim3(grid), dim3(kBlock), 0, s, vox_grid, n8, k0, v0);
  bool in1 = false;
  if ((e = launch_radix_sort(k0, v0, k1, v1, n_dev, n8, bits, 0, hist, st0, st1, base + 2, base + 18,
                             &in1, s)) != hipSuccess)
    return e;
  const uint64_t* ks = in1 ? k1 : k0;
  if (in1) {
    if ((e = hipMemcpyAsync(adj, v1, (size_t)n8 * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return e;
  }
  SVR_LAUNCH("adj_offsets", k_adj_offsets, dim3((unsigned)((n8 + kBlock) / kBlock)), dim3(kBlock),
             0, s, ks, n8, M, adj_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-scene order ranks.  Within a tile the sort key orders entries by
// (top 3L path bits XOR s * 0b001..001, s) (Supp. B.1, B.2).  That order over
// all (voxel, sign pattern) pairs is a property of the scene, so it is sorted
// once and each pair gets its rank; the per-frame key tile | rank then has
// ceil(log2(8N)) low bits instead of 3L + 3 and orders the entries exactly as
// before (the pair keys are distinct for L <= 15; at L = 16 equal keys keep
// the pair index order).
__global__ __launch_bounds__(kBlock) void k_rank_keys(const uint64_t* __restrict__ octpath,
                                                      int64_t n8, int L,
                                                      uint64_t* __restrict__ keys,
                                                      uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n8) return;
  const uint64_t top = octpath[i >> 3] >> (3 * (SVR_MAX_LEVELS - L));
  const uint64_t rep = ((1ull << (3 * L)) - 1ull) / 7ull;  // 001 001 ... 001 (L triplets)
  const uint64_t sgn = (uint64_t)(i & 7);
  keys[i] = ((top ^ (sgn * rep)) << 3) | sgn;
  vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_rank_scatter(const uint32_t* __restrict__ vals,
                                                         int64_t n8, uint32_t* __restrict__ rank) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p < n8) rank[vals[p]] = (uint32_t)p;
}

size_t order_rank_scratch_bytes(int64_t N, int L) {
  const int64_t n8 = 8 * N;
  const size_t r = 256;
  auto up = [&](size_t b) { return (b + r - 1) / r * r; };
  return up((size_t)n8 * 8) * 2 + up((size_t)n8 * 4) * 2 +
         up(sort_scratch_bytes(n8, 3 * L + 3, nullptr) + 256);
}

hipError_t launch_order_ranks(const uint64_t* octpath, int64_t N, int L, uint32_t* rank,
                              void* scratch, hipStream_t s) {
  const int64_t n8 = 8 * N;
  const int bits = 3 * L + 3;
  int64_t parts = 0;
  const size_t sb = sort_scratch_bytes(n8, bits, &parts);
  char* p = reinterpret_cast<char*>(scratch);
  auto take = [&](size_t b) { char* q = p; p += (b + 255) / 256 * 256; return q; };
  uint64_t* k0 = reinterpret_cast<uint64_t*>(take((size_t)n8 * 8));
  uint64_t* k1 = reinterpret_cast<uint64_t*>(take((size_t)n8 * 8));
  uint32_t* v0 = reinterpret_cast<uint32_t*>(take((size_t)n8 * 4));
  uint32_t* v1 = reinterpret_cast<uint32_t*>(take((size_t)n8 * 4));
  uint32_t* base = reinterpret_cast<uint32_t*>(take(sb + 256));
  auto* n_dev = reinterpret_cast<unsigned long long*>(base);
  uint32_t* hist = base + 64;
  uint32_t* st0 = hist + 8 * kRadix;
  uint32_t* st1 = st0 + (parts > 0 ? parts : 1) * kRadix;
  hipError_t e;
  if ((e = launch_fill_u32(base, 0u, 64, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(base, (uint32_t)(n8 & 0xffffffffu), 1, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(base + 1, (uint32_t)(n8 >> 32), 1, s)) != hipSuccess) return e;
  const unsigned grid = (unsigned)((n8 + kBlock - 1) / kBlock);
  SVR_LAUNCH("rank_keys", k_rank_keys, dim3(grid), dim3(kBlock), 0, s, octpath, n8, L, k0, v0);
  bool in1 = false;
  if ((e = launch_radix_sort(k0, v0, k1, v1, n_dev, n8, bits, 0, hist, st0, st1, base + 2, base + 18,
                             &in1, s)) != hipSuccess)
    return e;
  SVR_LAUNCH("rank_scatter", k_rank_scatter, dim3(grid), dim3(kBlock), 0, s, in1 ? v1 : v0, n8,
             rank);
  return hipGetLastError();
}

size_t grid_adjacency_scratch_bytes(int64_t N, int64_t M) {
  const int64_t n8 = 8 * N;
  int bits = 1;
  while (bits < 32 && ((int64_t)1 << bits) <= M) ++bits;
  const size_t r = 256;
  auto up = [&](size_t b) { return (b + r - 1) / r * r; };
  return up((size_t)n8 * 8) * 2 + up((size_t)n8 * 4) + up(sort_scratch_bytes(n8, bits, nullptr) + 256);
}

}  // namespace svr
