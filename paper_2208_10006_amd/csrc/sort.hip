// sort.hip -- LSD radix sort (8-bit digits) and exclusive scan, wave64-native.
//
// One pass = histogram -> exclusive scan of the [digit][block] table ->
// stable scatter.  A block owns a tile of 2048 keys (256 threads x 8 rounds,
// striped so every round is a coalesced 256-key load).  Inside a round each
// wave ranks its 64 keys among equal digits with 8 ballots (one per digit
// bit), so the in-tile order is kept without any LDS sort: that rank plus the
// counts of earlier waves and earlier rounds gives the stable local offset.
#include "sbr_device.hpp"
#include "sbr_internal.hpp"
#include "lds_sort.hpp"

namespace sbr {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kTile = kSortThreads * kSortRounds;  // 2048 keys per block
constexpr int kRadix = 256;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                           uint32_t* __restrict__ hist, int nblocks) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xff], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin,
                                                              uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                              int64_t n, int shift,
                                                              const uint32_t* __restrict__ offs, int nblocks) {
  __shared__ uint32_t base_of[kRadix];   // global offset of each digit for this block
  __shared__ uint32_t running[kRadix];   // keys of each digit already placed by earlier rounds
  __shared__ uint32_t wcount[kSortThreads / kWave][kRadix];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  base_of[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
  running[tid] = 0;
  for (int w = 0; w < kSortThreads / kWave; ++w) wcount[w][tid] = 0;
  __syncthreads();
  const int64_t tbase = (int64_t)blockIdx.x * kTile;
  const uint64_t lt = lanemask_lt();
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = tbase + r * kSortThreads + tid;
    const bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    uint32_t val = valid ? vin[i] : 0;
    const uint32_t dig = (uint32_t)(key >> shift) & 0xff;
    // lanes holding the same digit
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1;
      const uint64_t bal = __ballot(bit);
      same &= bit ? bal : ~bal;
    }
    const uint32_t rank = __popcll(same & lt);
    if (valid && rank == 0) wcount[wv][dig] = __popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = base_of[dig] + running[dig] + rank;
      for (int w = 0; w < wv; ++w) pos += wcount[w][dig];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kSortThreads / kWave; ++w) {
      add += wcount[w][tid];
      wcount[w][tid] = 0;
    }
    running[tid] += add;
    __syncthreads();
    (void)lane;
  }
}

// ---------------------------------------------------------------- scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kScanThreads / kWave];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // inclusive wave scan
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint32_t wpre = 0, tot = 0;
  for (int w = 0; w < kScanThreads / kWave; ++w) {
    if (w < wv) wpre += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return wpre + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                            uint32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) s += in[base + j];
  uint32_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of the block sums (serial chunks per thread)
__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t* __restrict__ sums, int64_t nb,
                                                         uint32_t* __restrict__ total_out) {
  const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
  const int64_t lo = (int64_t)threadIdx.x * per;
  uint32_t s = 0;
  for (int64_t i = lo; i < lo + per && i < nb; ++i) s += sums[i];
  uint32_t tot;
  uint32_t pre = block_exclusive_scan(s, &tot);
  for (int64_t i = lo; i < lo + per && i < nb; ++i) {
    uint32_t v = sums[i];
    sums[i] = pre;
    pre += v;
  }
  if (threadIdx.x == 0 && total_out) *total_out = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* in, uint32_t* out, int64_t n,
                                                          const uint32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    s += v[j];
  }
  uint32_t tot;
  uint32_t pre = block_exclusive_scan(s, &tot) + sums[blockIdx.x];
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = pre;
    pre += v[j];
  }
}

// whole scan in one block for short arrays (each thread owns a contiguous run)
__global__ __launch_bounds__(kScanThreads) void k_scan_small(const uint32_t* in, uint32_t* out, int64_t n,
                                                           uint32_t* __restrict__ total_out) {
  const int64_t per = (n + kScanThreads - 1) / kScanThreads;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  uint32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += in[i];
  uint32_t tot;
  uint32_t pre = block_exclusive_scan(s, &tot);
  for (int64_t i = lo; i < hi; ++i) {
    const uint32_t v = in[i];
    out[i] = pre;
    pre += v;
  }
  if (threadIdx.x == 0 && total_out) *total_out = tot;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_iota_u32(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}
__global__ void k_gather_u64(const uint64_t* __restrict__ src, const uint32_t* __restrict__ idx,
                             uint64_t* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t scan_temp_bytes(int64_t n) { return (size_t)(cdiv(n, kScanTile) + 1) * sizeof(uint32_t) + 256; }

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total_dev, void* temp,
                        hipStream_t s) {
  if (n <= 0) {
    if (total_dev) fill_u32(total_dev, 0, 1, s);
    return;
  }
  if (n <= 65536) {
    { ::sbr::TimedLaunch tl_("scan", s); hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kScanThreads), 0, s, in, out, n, total_dev); }
    SBR_LAUNCH_CHECK();
    return;
  }
  const int64_t nb = cdiv(n, kScanTile);
  uint32_t* sums = static_cast<uint32_t*>(temp);
  { ::sbr::TimedLaunch tl_("scan", s); hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums); }
  { ::sbr::TimedLaunch tl_("scan", s); hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, sums, nb, total_dev); }
  { ::sbr::TimedLaunch tl_("scan", s); hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, sums); }
  SBR_LAUNCH_CHECK();
}

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  { ::sbr::TimedLaunch tl_("misc", s); hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, p, v, n); }
  SBR_LAUNCH_CHECK();
}
void iota_u32(uint32_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  { ::sbr::TimedLaunch tl_("misc", s); hipLaunchKernelGGL(k_iota_u32, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, p, n); }
  SBR_LAUNCH_CHECK();
}
void gather_u64(const uint64_t* src, const uint32_t* idx, uint64_t* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  { ::sbr::TimedLaunch tl_("misc", s); hipLaunchKernelGGL(k_gather_u64, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, src, idx, dst, n); }
  SBR_LAUNCH_CHECK();
}

// Small arrays (up to kSmallSort keys): the whole LSD radix sort in one
// workgroup (lds_radix_sort_pairs), keys and values resident in LDS between
// one coalesced load and one coalesced store.
constexpr int kSmallPer = 12, kSmallSort = kSmallThreads * kSmallPer;

__global__ __launch_bounds__(kSmallThreads) void k_radix_sort_small(const uint64_t* __restrict__ kin,
                                                                  const uint32_t* __restrict__ vin,
                                                                  uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                                  int n, int bit_lo, int bit_hi) {
  __shared__ uint64_t lk[kSmallSort];
  __shared__ uint32_t lv[kSmallSort];
  __shared__ uint16_t hist[kSmallWaves][256];
  __shared__ uint32_t dsum[kSmallWaves / 4];
  const int t = threadIdx.x;
  for (int i = t; i < n; i += kSmallThreads) lk[i] = kin[i], lv[i] = vin[i];
  __syncthreads();
  lds_radix_sort_pairs<kSmallPer>(lk, lv, hist, dsum, n, bit_lo, bit_hi);
  for (int i = t; i < n; i += kSmallThreads) {
    kout[i] = lk[i];
    vout[i] = lv[i];
  }
}

size_t radix_sort_temp_bytes(int64_t n) {
  const int64_t nb = cdiv(n > 0 ? n : 1, kTile);
  const int64_t hist = nb * kRadix;
  return (size_t)hist * sizeof(uint32_t) * 2 + scan_temp_bytes(hist) + 512;
}

void radix_sort_pairs(uint64_t* keys_in, uint32_t* vals_in, uint64_t* keys_out, uint32_t* vals_out, int64_t n,
                      int bit_lo, int bit_hi, void* temp, hipStream_t s) {
  SBR_CHECK(n >= 0 && n < (int64_t(1) << 32), SBR_E_UNSUPPORTED, "radix sort of %lld keys", (long long)n);
  const int npass = (bit_hi - bit_lo + 7) / 8;
  if (n == 0) return;
  if (npass <= 0) {
    SBR_HIP(hipMemcpyAsync(keys_out, keys_in, n * 8, hipMemcpyDeviceToDevice, s));
    SBR_HIP(hipMemcpyAsync(vals_out, vals_in, n * 4, hipMemcpyDeviceToDevice, s));
    return;
  }
  if (n <= kSmallSort) {
    { ::sbr::TimedLaunch tl_("sort", s); hipLaunchKernelGGL(k_radix_sort_small, dim3(1), dim3(kSmallThreads), 0, s, keys_in, vals_in, keys_out, vals_out, (int)n, bit_lo, bit_hi); }
    SBR_LAUNCH_CHECK();
    return;
  }
  const int64_t nb = cdiv(n, kTile);
  const int64_t hn = nb * kRadix;
  uint32_t* hist = static_cast<uint32_t*>(temp);
  uint32_t* offs = hist + hn;
  void* stemp = offs + hn;
  uint64_t* ka = keys_in;
  uint32_t* va = vals_in;
  uint64_t* kb = keys_out;
  uint32_t* vb = vals_out;
  for (int p = 0; p < npass; ++p) {
    const int shift = bit_lo + 8 * p;
    { ::sbr::TimedLaunch tl_("sort", s); hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, ka, n, shift, hist, (int)nb); }
    exclusive_scan_u32(hist, offs, hn, nullptr, stemp, s);
    { ::sbr::TimedLaunch tl_("sort", s); hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, ka, va, kb, vb, n, shift,
                       offs, (int)nb); }
    SBR_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  // after an odd number of passes the result sits in *_out already; otherwise copy back
  if (ka != keys_out) {
    SBR_HIP(hipMemcpyAsync(keys_out, ka, n * 8, hipMemcpyDeviceToDevice, s));
    SBR_HIP(hipMemcpyAsync(vals_out, va, n * 4, hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace sbr
