// Device-side building blocks of the propagation kernels (gfx950, wave64).
//
// Every floating point operation that takes a decision (thresholds, sampling
// probabilities, geometric skips, acceptance ratios) is written as separate
// IEEE binary64 operations in a fixed order, and the library is compiled with
// -ffp-contract=off, so no multiply-add is fused and every decision is a
// deterministic function of its inputs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace agp {

constexpr int kWave = 64;
constexpr int kSegLog2 = 6;  // sampled suffixes are cut into 64-position windows
constexpr int kSeg = 1 << kSegLog2;
// Sampling runs (a > 0) end with the degree group floor(log2 d) of their
// first position, except that a run whose rate p* times the positions left in
// its window is at most this many expected candidates takes the rest of the
// window: fewer draws than a run per group, every position still kept with
// probability p_v.
constexpr double kMergeCandidates = 4.0;

// ---------------------------------------------------------------- Philox
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11): ten rounds, each multiplying
// counter words 0 and 2 by the two Philox-4x32 multipliers, exchanging the
// halves and mixing in the key, which advances by the two Weyl increments.
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // one 32 x 32 -> 64-bit product per multiplier (a single v_mad_u64_u32)
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t y0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t y2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c0 = y0;
    c1 = static_cast<uint32_t>(p1);
    c2 = y2;
    c3 = static_cast<uint32_t>(p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// The same generator for a key held in scalar registers (the same key for the
// whole wave).  The key schedule is recomputed round by round with two scalar
// adds; the empty asm statement only hides the key's value from the compiler,
// which would otherwise keep all twenty round keys live for the whole kernel.
__device__ __forceinline__ U4 philox4x32_10_skey(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t y0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t y2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c0 = y0;
    c1 = static_cast<uint32_t>(p1);
    c2 = y2;
    c3 = static_cast<uint32_t>(p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    __asm__ volatile("" : "+s"(k0), "+s"(k1));
  }
  return U4{c0, c1, c2, c3};
}

// 53 random bits (32 from `hi`, the top 21 of `lo`) as a double in [0, 1).
__device__ __forceinline__ double unit_double(uint32_t hi, uint32_t lo) {
  // hi * 2^21 + (lo >> 11) is an integer below 2^53: both terms and the sum
  // are exact in binary64
  const double h = static_cast<double>(hi) * 2097152.0;
  const double l = static_cast<double>(lo >> 11);
  return (h + l) * 0x1p-53;
}

// --------------------------------------------------------- geometric skip
// Complement table of one sampling run: sk[h] = 1 - (1 - p)^(2^h), h = 0..6.
struct SkipTable {
  double sk[7];
};

__device__ __forceinline__ SkipTable make_skip_table(double p) {
  SkipTable t;
  t.sk[0] = p;
#pragma unroll
  for (int h = 1; h < 7; ++h) {
    const double two_minus = 2.0 - t.sk[h - 1];
    t.sk[h] = t.sk[h - 1] * two_minus;
  }
  return t;
}

// Failures before the next success of Bernoulli(p) trials for the uniform u:
// the largest K < 128 with 1 - (1-p)^K <= u, found bit by bit from the top
// using 1-(1-p)^(K + 2^h) = F + s_h - F s_h with F = 1-(1-p)^K.
__device__ __forceinline__ int geometric_skip(const SkipTable& t, double u) {
  double F = 0.0;
  int K = 0;
#pragma unroll
  for (int h = 6; h >= 0; --h) {
    const double plus = F + t.sk[h];
    const double times = F * t.sk[h];
    const double next = plus - times;
    if (next <= u) {
      F = next;
      K |= 1 << h;
    }
  }
  return K;
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t v) {
  uint64_t z = v + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ------------------------------------------------- exact fixed-point sums
// A next-level residue is the exact sum of the contributions a node receives
// in one level, rounded once.  Every contribution of column c is at least
// fl(theta_c) in magnitude, hence an integer multiple of
// unit_c = 2^ue_c = ulp(fl(theta_c)); the sums are kept as integers of that
// unit, so integer atomics add them in any order with the same result.

// Integer count of units in the binary32 value f (exact: |f| >= unit);
// returns false if the count does not fit in 62 bits.
__device__ __forceinline__ bool f32_to_units(float f, double scale, long long* out) {
  const double s = static_cast<double>(f) * scale;  // exact: scale is a power of two
  if (!(s < 0x1p62 && s > -0x1p62)) return false;
  *out = static_cast<long long>(s);
  return true;
}

// Round K * 2^ue to binary32, to nearest even; 0 gives +0.  ue >= -149.
__device__ __forceinline__ float units_to_f32(long long K, int ue) {
  if (K == 0) return 0.0f;
  const bool neg = K < 0;
  unsigned long long m = neg ? (0ull - static_cast<unsigned long long>(K))
                             : static_cast<unsigned long long>(K);
  const int nb = 64 - __clzll(m);
  float r;
  if (nb <= 24) {
    r = ldexpf(static_cast<float>(m), ue);  // exact: at most 24 bits, ue >= -149
  } else {
    int shift = nb - 24;
    unsigned long long q = m >> shift;
    const unsigned long long rem = m & ((1ull << shift) - 1ull);
    const unsigned long long half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1ull))) {
      ++q;
      if (q == (1ull << 24)) {
        q >>= 1;
        ++shift;
      }
    }
    r = ldexpf(static_cast<float>(q), ue + shift);
  }
  return neg ? -r : r;
}

// 128-bit two's complement cells for binary64 working precision.
struct U128 {
  unsigned long long lo;
  long long hi;
};

// floor(log2 |v|) of a finite non-zero double, from its bits.
__device__ __forceinline__ int ilog2_f64(double v) {
  const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(v));
  const int e = static_cast<int>((bits >> 52) & 0x7FFull);
  if (e != 0) return e - 1023;
  const unsigned long long man = bits & 0xFFFFFFFFFFFFFull;
  return -1074 + (63 - __clzll(man));
}

// Units of 2^ue in the binary64 value v (a multiple of 2^ue), as 128 bits.
__device__ __forceinline__ bool f64_to_units(double v, int ue, U128* out) {
  if (v == 0.0) {
    *out = U128{0ull, 0ll};
    return true;
  }
  const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(v));
  const int be = static_cast<int>((bits >> 52) & 0x7FFull);
  unsigned long long man = bits & 0xFFFFFFFFFFFFFull;
  int e2;  // v = man * 2^e2
  if (be != 0) {
    man |= 1ull << 52;
    e2 = be - 1075;
  } else {
    e2 = -1074;
  }
  int sh = e2 - ue;
  while (sh < 0) {  // v has trailing zero bits below the unit
    man >>= 1;
    ++sh;
  }
  if (sh > 73) return false;  // would not fit in 127 bits
  unsigned long long lo, hi;
  if (sh == 0) {
    lo = man;
    hi = 0;
  } else if (sh < 64) {
    lo = man << sh;
    hi = man >> (64 - sh);
  } else {
    lo = 0;
    hi = man << (sh - 64);
  }
  if (v < 0.0) {  // two's complement negate
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  *out = U128{lo, static_cast<long long>(hi)};
  return true;
}

// Round (hi:lo) * 2^ue to binary64, to nearest even; ue >= -1074.
__device__ __forceinline__ double units_to_f64(U128 K, int ue) {
  unsigned long long lo = K.lo;
  unsigned long long hi = static_cast<unsigned long long>(K.hi);
  const bool neg = K.hi < 0;
  if (neg) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  if (hi == 0 && lo == 0) return 0.0;
  const int nb = hi ? 128 - __clzll(hi) : 64 - __clzll(lo);
  double r;
  if (nb <= 53) {
    r = ldexp(static_cast<double>(lo), ue);  // exact
  } else {
    int shift = nb - 53;
    unsigned long long q, rem_hi_bit, sticky;
    // q = (hi:lo) >> shift, 53 bits
    if (shift >= 64) {
      q = hi >> (shift - 64);
    } else {
      q = (lo >> shift) | (shift ? (hi << (64 - shift)) : 0ull);
    }
    // round bit = bit (shift - 1); sticky = any bit below it
    const int rb = shift - 1;
    if (rb >= 64) {
      rem_hi_bit = (hi >> (rb - 64)) & 1ull;
      const unsigned long long below_hi = (rb - 64) ? (hi & ((1ull << (rb - 64)) - 1ull)) : 0ull;
      sticky = (below_hi | lo) ? 1ull : 0ull;
    } else {
      rem_hi_bit = (lo >> rb) & 1ull;
      sticky = rb ? ((lo & ((1ull << rb) - 1ull)) ? 1ull : 0ull) : 0ull;
    }
    if (rem_hi_bit && (sticky || (q & 1ull))) {
      ++q;
      if (q == (1ull << 53)) {
        q >>= 1;
        ++shift;
      }
    }
    r = ldexp(static_cast<double>(q), ue + shift);
  }
  return neg ? -r : r;
}

// ------------------------------------------------------- wave utilities

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Append `item` for every active lane with `pred` to list[], reserving the
// slots with one atomic per wave.  All active lanes must call it together.
__device__ __forceinline__ void wave_append(uint64_t* __restrict__ list,
                                            unsigned long long* __restrict__ count,
                                            uint64_t item, bool pred) {
  const unsigned long long mask = __ballot(pred);
  if (mask == 0ull) return;
  const int leader = __ffsll(static_cast<long long>(mask)) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(count, static_cast<unsigned long long>(__popcll(mask)));
  base = __shfl(base, leader);
  if (pred) {
    const unsigned long long below = mask & ((1ull << lane_id()) - 1ull);
    list[base + static_cast<unsigned long long>(__popcll(below))] = item;
  }
}

// Per-wave LDS staging of list entries: entries are gathered with ballots and
// written out in chunks, one global atomic per chunk.  Every call must be
// made by all lanes of the wave together (wave-uniform control flow).
constexpr int kStage = 512;

__device__ __forceinline__ void stage_flush(uint64_t* stage, int& staged, uint64_t* __restrict__ list,
                                            unsigned long long* __restrict__ count) {
  if (staged == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  unsigned long long base = 0;
  if (lane_id() == 0) base = atomicAdd(count, static_cast<unsigned long long>(staged));
  base = __shfl(base, 0);
  for (int i = lane_id(); i < staged; i += kWave) list[base + i] = stage[i];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  staged = 0;
}

template <int kCap = kStage>
__device__ __forceinline__ void stage_push(uint64_t* stage, int& staged, uint64_t item, bool pred,
                                           uint64_t* __restrict__ list,
                                           unsigned long long* __restrict__ count) {
  const unsigned long long mask = __ballot(pred);
  if (pred) stage[staged + __popcll(mask & ((1ull << lane_id()) - 1ull))] = item;
  staged += __popcll(mask);
  if (staged > kCap - kWave) stage_flush(stage, staged, list, count);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off);
  return v;
}

}  // namespace agp
