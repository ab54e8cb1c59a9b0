// bits.h -- per-row / per-column flag bits in 64-bit words. A flag array of
// the large LP (1.5e7 columns) is 1.9 MB this way: it stays in a chip's L2
// (4 MB per XCD), while a byte or word per column (15-60 MB) does not, so
// the random lookups of the compaction and the hash pass hit in L2.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace psl {

__device__ __forceinline__ bool bit_of(const uint64_t* bits, int64_t j) { return (bits[j >> 6] >> (j & 63)) & 1ull; }

// A word of flags with the number of set flags before it (an exclusive
// scan over the words): one 16-byte lookup gives a flag and its rank.
struct RankWord {
  uint64_t bits;
  int32_t pre;
  int32_t pad;
};

__device__ __forceinline__ bool bit_of(const RankWord* rw, int64_t j) { return (rw[j >> 6].bits >> (j & 63)) & 1ull; }

// j's rank among the set flags (the index of a kept j after compaction)
__device__ __forceinline__ int32_t rank_of(const RankWord* rw, int64_t j) {
  RankWord w = rw[j >> 6];
  return w.pre + (int32_t)__popcll(w.bits & ((1ull << (j & 63)) - 1ull));
}

__device__ __forceinline__ void set_word(uint64_t& w, uint64_t v) { w = v; }
__device__ __forceinline__ void set_word(RankWord& w, uint64_t v) { w.bits = v; }

// Word w of flag f over [0, n): each wavefront takes 64 consecutive indices
// (an aligned word), its ballot is the word. Launched with one thread per
// index (grid-strided in multiples of 64), every lane of a word present.
template <typename W, typename F>
__device__ __forceinline__ void write_bits(W* words, int64_t n, F f) {
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < n; t0 += stride) {
    int64_t t = t0 + threadIdx.x;
    bool v = t < n && f(t);
    unsigned long long w = __ballot(v);
    if ((threadIdx.x & 63) == 0 && t < n) set_word(words[t >> 6], w);
  }
}

}  // namespace psl
