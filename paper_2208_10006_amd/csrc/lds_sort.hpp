// lds_sort.hpp -- stable LSD radix sort of (key, value) pairs resident in
// LDS, run by one workgroup of kSmallThreads threads.
#pragma once
#include <cstdint>

#include "sbr_device.hpp"

namespace sbr {

constexpr int kSmallThreads = 1024, kSmallWaves = kSmallThreads / 64;

// 8-bit digits over key bits [bit_lo, bit_hi).  Wave w owns the contiguous
// block [w * 64 * P, (w + 1) * 64 * P) of the current order, P =
// ceil(n / 1024) <= PER, and walks it in rounds of 64 (element w*64*P +
// u*64 + lane in round u), so the order (wave, round, lane) is the array
// order.  In a round, the lanes holding the same digit are found with eight
// ballots; the lowest of them adds the group's size to the wave's digit
// count in LDS after every lane of the group has read the count, which gives
// each element its place among the wave's equal digits.  A scan of the counts
// in (digit, wave) order turns them into offsets, and every element is
// written to offset + place: a stable counting sort per pass.  Every thread
// of the workgroup must call it (it synchronises); the arrays are sorted in
// place and the call ends with a barrier.
template <int PER>
__device__ inline void lds_radix_sort_pairs(uint64_t* lk, uint32_t* lv, uint16_t (*hist)[256], uint32_t* dsum, int n,
                                            int bit_lo, int bit_hi) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int P = (n + kSmallThreads - 1) / kSmallThreads;  // rounds per wave, <= PER
  const int w0 = wv * 64 * P;
  const int npass = (bit_hi - bit_lo + 7) / 8;
  const uint64_t lt = lanemask_lt();
  for (int p = 0; p < npass; ++p) {
    const int shift = bit_lo + 8 * p;
    for (int d = lane; d < 256; d += 64) hist[wv][d] = 0;
    uint64_t ck[PER];
    uint32_t cv[PER];
    uint32_t place[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      if (u >= P) break;  // wave-uniform
      const int i = w0 + u * 64 + lane;
      const bool ok = i < n;
      uint32_t d = 0;
      if (ok) {
        ck[u] = lk[i], cv[u] = lv[i];
        d = (uint32_t)(ck[u] >> shift) & 255u;
      }
      uint64_t m = __ballot(ok);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot(ok && ((d >> b) & 1u));
        m &= ((d >> b) & 1u) ? bb : ~bb;
      }
      const uint32_t before = ok ? hist[wv][d] : 0u;  // every lane reads before the leader writes
      place[u] = before + (uint32_t)__popcll(m & lt);
      if (ok && (m & lt) == 0) hist[wv][d] = (uint16_t)(before + (uint32_t)__popcll(m));
    }
    __syncthreads();
    // offsets in (digit, wave) order: threads 0..255 own one digit each
    uint32_t excl_digit = 0;
    if (t < 256) {
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < kSmallWaves; ++w) {
        const uint32_t c = hist[w][t];
        hist[w][t] = (uint16_t)run;
        run += c;
      }
      const uint32_t incl = wave_inclusive_scan(run, lane);
      if (lane == 63) dsum[wv] = incl;
      excl_digit = incl - run;  // digits before this one within the scanning wave
    }
    __syncthreads();
    if (t < 256) {
      uint32_t base = excl_digit;
      for (int w = 0; w < wv; ++w) base += dsum[w];
#pragma unroll
      for (int w = 0; w < kSmallWaves; ++w) hist[w][t] = (uint16_t)(hist[w][t] + base);
    }
    __syncthreads();  // offsets complete; every element was read before the first barrier
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      if (u >= P) break;
      const int i = w0 + u * 64 + lane;
      if (i < n) {
        const uint32_t d = (uint32_t)(ck[u] >> shift) & 255u;
        const uint32_t pos = (uint32_t)hist[wv][d] + place[u];
        lk[pos] = ck[u];
        lv[pos] = cv[u];
      }
    }
    __syncthreads();
  }
}

}  // namespace sbr
