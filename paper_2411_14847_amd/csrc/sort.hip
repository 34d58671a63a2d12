// Prefix scan and LSD radix sort for wave64 (gfx950).
//
// Radix sort: reduce-then-scan with a fixed grid, so that the element count can stay on the
// device (no host round trip inside a render; the launch sequence is graph-capturable).
// Each pass over a digit of 8 to 11 bits is
//   (1) upsweep: every block histograms its contiguous chunk into LDS (per-wave
//       sub-histograms to spread LDS atomics), written digit-major to global memory;
//   (2) scan: one workgroup per digit turns the [radix][blocks] counts into global offsets;
//   (3) scatter: every block re-reads its chunk in batches of 2048 pairs (4096 for 9- and
//       10-bit digits), ranks them stably
//       with wave ballots (8-11 ballots give each lane the mask of lanes holding the same
//       digit; each wave ranks its own quarter of the batch), orders the batch by digit in
//       LDS and writes each digit's run contiguously.
// A pass never depends on forward progress between workgroups.
#include <algorithm>

#include "dass_internal.h"

namespace dass {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;                      // items per thread per batch
constexpr int kBatch = kSortThreads * kSortItems;  // 2048
constexpr int kMaxRadixBits = 11;  // 32-bit keys; 64-bit keys use at most 10 (LDS per block)
constexpr int kMaxRadix = 1 << kMaxRadixBits;
// at most 512 blocks: the 15.4M 10-bit tile keys of the 20-view, 200k-Gaussian benchmark sort in
// 0.159 ms with 512 (about 30k keys per block), 0.168 with 1024 and 0.194 with 256
constexpr int kMaxSortBlocks = 512;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive scan within a wave of 64 lanes (shuffle-up steps).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan across a 256-thread block; returns the exclusive prefix, *total the sum.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* s_wave, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(x);
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; w++) {
    uint32_t s = s_wave[w];
    if (w < wave) base += s;
    tot += s;
  }
  __syncthreads();
  if (total) *total = tot;
  return base + inc - x;
}

template <int RB, typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
  return (uint32_t)(k >> shift) & ((1u << RB) - 1);
}

__device__ __forceinline__ void chunk_of(uint32_t count, int blocks, uint32_t& lo, uint32_t& hi) {
  const uint32_t chunk = (uint32_t)(((uint64_t)count + blocks - 1) / blocks);
  const uint64_t l = (uint64_t)blockIdx.x * chunk;
  lo = (uint32_t)(l < count ? l : count);
  const uint64_t h = l + chunk;
  hi = (uint32_t)(h < count ? h : count);
}

template <typename K, int RB>
__global__ __launch_bounds__(kSortThreads) void k_upsweep(const K* __restrict__ keys, const uint32_t* __restrict__ d_count,
                                                          int shift, int blocks, uint32_t* __restrict__ hist) {
  constexpr int R = 1 << RB;
  __shared__ uint32_t s_h[4][R];
  const int tid = threadIdx.x, wave = tid >> 6;
  for (int i = tid; i < 4 * R; i += kSortThreads) (&s_h[0][0])[i] = 0;
  __syncthreads();
  uint32_t lo, hi;
  chunk_of(*d_count, blocks, lo, hi);
  uint32_t i = lo + tid;
  // eight independent loads in flight per thread, then their LDS increments
  for (; i + (kSortItems - 1) * kSortThreads < hi; i += kSortItems * kSortThreads) {
    K k[kSortItems];
#pragma unroll
    for (int u = 0; u < kSortItems; u++) k[u] = keys[i + u * kSortThreads];
#pragma unroll
    for (int u = 0; u < kSortItems; u++) atomicAdd(&s_h[wave][digit_of<RB>(k[u], shift)], 1u);
  }
  for (; i < hi; i += kSortThreads) atomicAdd(&s_h[wave][digit_of<RB>(keys[i], shift)], 1u);
  __syncthreads();
  for (int d = tid; d < R; d += kSortThreads)
    hist[(int64_t)d * blocks + blockIdx.x] = s_h[0][d] + s_h[1][d] + s_h[2][d] + s_h[3][d];
}

// Exclusive scan of each digit's row of block counts (one workgroup per digit); the row total
// goes to totals[digit].  The scatter adds the exclusive scan of the totals.
__global__ __launch_bounds__(kSortThreads) void k_scan_rows(uint32_t* __restrict__ hist, int blocks,
                                                            uint32_t* __restrict__ totals) {
  __shared__ uint32_t s_w[4];
  uint32_t* row = hist + (int64_t)blockIdx.x * blocks;
  const int per = (blocks + kSortThreads - 1) / kSortThreads;
  const int b = threadIdx.x * per, e = min(b + per, blocks);
  uint32_t sum = 0;
  for (int i = b; i < e; i++) sum += row[i];
  uint32_t tot;
  uint32_t run = block_excl_scan256(sum, s_w, &tot);
  for (int i = b; i < e; i++) {
    const uint32_t c = row[i];
    row[i] = run;
    run += c;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// Exclusive scan over R digits held D = R/256 per thread (consecutive); returns per-thread
// prefix base (the thread's first digit's offset); *total is the sum of all.
template <int D>
__device__ __forceinline__ uint32_t block_excl_scan_digits(const uint32_t* c, uint32_t* s_tmp, uint32_t* total) {
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < D; i++) sum += c[i];
  return block_excl_scan256(sum, s_tmp, total);
}

// Orders LDS accesses of the lanes of one wave (a wave's LDS instructions complete in order;
// this only keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Each batch of 256 IT pairs is split into four runs of 64 IT consecutive pairs, one per wave; a
// wave ranks its run slot by slot (64 pairs at a time) against its own running digit counts,
// with no workgroup barrier, so the ranks follow the input order.  Waves are then combined by
// an exclusive prefix of their counts per digit, the batch is ordered by digit in LDS, and each
// digit's run is written to its global position.
// IT items per thread per batch: 16 for 10-bit digits, where a 2,048-pair batch would leave
// runs of about two pairs per digit and the stores would barely coalesce (one 10-bit pass over
// the 1.5e7 tile keys of a 20-view call at 64x32 tiles: 0.199 -> 0.167 ms), else 8 (wider
// batches measured slower for 8-bit digits, and for the 11-bit passes over a few 1e5 keys).
template <typename K, int RB, int IT>
__global__ __launch_bounds__(kSortThreads) void k_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                          K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          const uint32_t* __restrict__ d_count, int shift, int blocks,
                                                          const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ totals) {
  constexpr int R = 1 << RB;
  constexpr int D = R / kSortThreads;        // digits owned per thread
  constexpr int kWaveRun = IT * 64;          // consecutive pairs ranked by one wave per batch
  constexpr int kBatchP = kSortThreads * IT;  // pairs per batch
  __shared__ uint32_t s_base[R];             // global write position of the next item of each digit
  __shared__ uint32_t s_boff[R];             // exclusive digit offsets within the batch
  __shared__ uint32_t s_wc[4][R];            // per-wave digit counts, then their prefix over waves
  __shared__ uint32_t s_tmp[4];
  __shared__ K s_k[kBatchP];
  __shared__ uint32_t s_v[kBatchP];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const uint32_t count = *d_count;
  uint32_t lo, hi;
  chunk_of(count, blocks, lo, hi);
  {  // global base of each digit for this block: row prefix + exclusive scan of the digit totals
    uint32_t tv[D];
#pragma unroll
    for (int i = 0; i < D; i++) tv[i] = totals[tid * D + i];
    uint32_t run = block_excl_scan_digits<D>(tv, s_tmp, nullptr);
#pragma unroll
    for (int i = 0; i < D; i++) {
      const int d = tid * D + i;
      s_base[d] = hist[(int64_t)d * blocks + blockIdx.x] + run;
      run += tv[i];
    }
  }
  const uint64_t lt = lanemask_lt();

  for (uint32_t batch = lo; batch < hi; batch += kBatchP) {
    const uint32_t nb = min((uint32_t)kBatchP, hi - batch);
    const uint32_t wbase = batch + (uint32_t)(wave * kWaveRun);
    for (int d = lane; d < R; d += 64) s_wc[wave][d] = 0;
    K key[IT];
    uint32_t val[IT], rank[IT], dig[IT];
#pragma unroll
    for (int s = 0; s < IT; s++) {
      const uint32_t idx = wbase + (uint32_t)(s * 64 + lane);
      if (idx < hi) {
        key[s] = kin[idx];
        val[s] = vin[idx];
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < IT; s++) {
      const bool valid = wbase + (uint32_t)(s * 64 + lane) < hi;
      const uint32_t d = valid ? digit_of<RB>(key[s], shift) : 0u;
      dig[s] = d;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < RB; b++) {
        const uint64_t m = __ballot((d >> b) & 1);
        peers &= ((d >> b) & 1) ? m : ~m;
      }
      const uint32_t rw = __popcll(peers & lt);
      const uint32_t base = s_wc[wave][d];  // every lane of the digit reads before the leader adds
      wave_lds_sync();
      if (valid && rw == 0) s_wc[wave][d] = base + __popcll(peers);
      wave_lds_sync();
      rank[s] = base + rw;
    }
    __syncthreads();
    uint32_t c[D];
#pragma unroll
    for (int i = 0; i < D; i++) {  // thread owns digits tid*D..: prefix over waves, batch count
      const int dd = tid * D + i;
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < 4; w++) {
        const uint32_t x = s_wc[w][dd];
        s_wc[w][dd] = run;
        run += x;
      }
      c[i] = run;
    }
    {
      uint32_t run = block_excl_scan_digits<D>(c, s_tmp, nullptr);
#pragma unroll
      for (int i = 0; i < D; i++) {
        s_boff[tid * D + i] = run;
        run += c[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < IT; s++) {
      if (wbase + (uint32_t)(s * 64 + lane) < hi) {
        const uint32_t pos = s_boff[dig[s]] + s_wc[wave][dig[s]] + rank[s];
        s_k[pos] = key[s];
        s_v[pos] = val[s];
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < IT; s++) {
      const uint32_t j = s * kSortThreads + tid;
      if (j < nb) {
        const K k = s_k[j];
        const uint32_t d = digit_of<RB>(k, shift);
        const uint32_t o = s_base[d] + (j - s_boff[d]);
        if (o < count) {  // always true for a consistent histogram; keeps stores in bounds
          kout[o] = k;
          vout[o] = s_v[j];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < D; i++) s_base[tid * D + i] += c[i];
    __syncthreads();
  }
}

// ---- scan of uint32 -> uint64 (exclusive), 3 phases ----------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                              uint64_t* __restrict__ sums) {
  __shared__ uint64_t s_w[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint64_t acc = 0;
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    const int64_t j = base + i;
    if (j < n) acc += in[j];
  }
  // wave reduce
  for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// exclusive scan of nb block sums in place (single workgroup of 1024), nb <= 1024 * 64
__global__ __launch_bounds__(1024) void k_scan_sums(uint64_t* __restrict__ sums, int nb) {
  __shared__ uint64_t s_w[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (nb + 1023) / 1024;
  const int b = tid * per, e = min(b + per, nb);
  uint64_t sum = 0;
  for (int i = b; i < e; i++) sum += sums[i];
  uint64_t inc = wave_incl_scan64(sum);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint64_t base = 0;
  for (int w = 0; w < wave; w++) base += s_w[w];
  uint64_t run = base + inc - sum;
  for (int i = b; i < e; i++) {
    uint64_t c = sums[i];
    sums[i] = run;
    run += c;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_final(const uint32_t* __restrict__ in, int64_t n,
                                                             const uint64_t* __restrict__ sums,
                                                             uint64_t* __restrict__ out) {
  __shared__ uint64_t s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;  // blocked layout
  uint32_t x[kScanItems];
  uint64_t local = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; i++) {
    const int64_t j = base + i;
    x[i] = j < n ? in[j] : 0u;
    local += x[i];
  }
  uint64_t inc = wave_incl_scan64(local);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint64_t run = sums[blockIdx.x] + inc - local;
  for (int w = 0; w < wave; w++) run += s_w[w];
#pragma unroll
  for (int i = 0; i < kScanItems; i++) {
    const int64_t j = base + i;
    if (j < n) out[j] = run;
    run += x[i];
  }
  if (base <= n - 1 && n - 1 < base + kScanItems) out[n] = run;  // holder of the last element
}

__global__ void k_set_u64(uint64_t* p, uint64_t v) { *p = v; }

template <typename K, int RB>
void radix_pass(K* keys[2], uint32_t* vals[2], int cur, const uint32_t* d_count, int shift, int blocks,
                uint32_t* hist, uint32_t* totals, hipStream_t st) {
  k_upsweep<K, RB><<<blocks, kSortThreads, 0, st>>>(keys[cur], d_count, shift, blocks, hist);
  k_scan_rows<<<1 << RB, kSortThreads, 0, st>>>(hist, blocks, totals);
  k_scatter<K, RB, RB >= 9 ? 16 : 8><<<blocks, kSortThreads, 0, st>>>(keys[cur], vals[cur], keys[cur ^ 1],
                                                                      vals[cur ^ 1], d_count, shift, blocks, hist,
                                                                      totals);
}

template <typename K>
int radix_sort_impl(K* keys[2], uint32_t* vals[2], const uint32_t* d_count, int64_t max_count, int begin_bit,
                    int end_bit, uint32_t* hist, int blocks, hipStream_t st, int digit_cap) {
  int cur = 0;
  if (max_count == 0 || end_bit <= begin_bit) return cur;
  // fewest passes of at most max_bits, with the narrowest digit (>= 8 bits) that keeps that pass
  // count: wider digits cost LDS and ballots per item
  const int max_bits = std::max(8, std::min(digit_cap, sizeof(K) == 4 ? kMaxRadixBits : kMaxRadixBits - 1));
  const int bits = end_bit - begin_bit;
  const int passes = (bits + max_bits - 1) / max_bits;
  const int rb = max(8, (bits + passes - 1) / passes);
  uint32_t* totals = hist + (int64_t)kMaxRadix * kMaxSortBlocks;
  for (int shift = begin_bit; shift < end_bit; shift += rb) {
    switch (rb) {
      case 8: radix_pass<K, 8>(keys, vals, cur, d_count, shift, blocks, hist, totals, st); break;
      case 9: radix_pass<K, 9>(keys, vals, cur, d_count, shift, blocks, hist, totals, st); break;
      case 10: radix_pass<K, 10>(keys, vals, cur, d_count, shift, blocks, hist, totals, st); break;
      default: radix_pass<K, sizeof(K) == 4 ? 11 : 10>(keys, vals, cur, d_count, shift, blocks, hist, totals, st);
    }
    cur ^= 1;
  }
  return cur;
}

}  // namespace

int sort_blocks_for(int64_t max_count) {
  int64_t b = (max_count + 4 * kBatch - 1) / (4 * kBatch);
  const int64_t one = (max_count + kBatch - 1) / kBatch;
  if (b < 256) b = one < 256 ? one : 256;
  if (b < 1) b = 1;
  if (b > kMaxSortBlocks) b = kMaxSortBlocks;
  return (int)b;
}

int radix_sort_u64(uint64_t* keys[2], uint32_t* vals[2], const uint32_t* d_count, int64_t max_count, int begin_bit,
                   int end_bit, uint32_t* hist, int blocks, hipStream_t st) {
  // digits of at most 9 bits: over the 4M 36-bit (view, depth) keys of a 200k-Gaussian, 20-view
  // call four 9-bit passes take 0.219 ms in 2,048-pair batches and 0.205 in 4,096-pair ones, five
  // 8-bit ones 0.233 and four 10-bit ones 0.249 (with 1,024 digits a batch leaves about two pairs
  // per digit run, so the scatter's stores barely coalesce)
  return radix_sort_impl<uint64_t>(keys, vals, d_count, max_count, begin_bit, end_bit, hist, blocks, st, 9);
}

int radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* d_count, int64_t max_count, int begin_bit,
                   int end_bit, uint32_t* hist, int blocks, hipStream_t st, int digit_cap) {
  return radix_sort_impl<uint32_t>(keys, vals, d_count, max_count, begin_bit, end_bit, hist, blocks, st, digit_cap);
}

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

void scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* tmp, hipStream_t st) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (n == 0) {
    k_set_u64<<<1, 1, 0, st>>>(out, 0);
    return;
  }
  k_scan_reduce<<<(unsigned)nb, kScanThreads, 0, st>>>(in, n, tmp);
  k_scan_sums<<<1, 1024, 0, st>>>(tmp, (int)nb);
  k_scan_final<<<(unsigned)nb, kScanThreads, 0, st>>>(in, n, tmp, out);
}

}  // namespace dass
