// Invariant-divisor unsigned 64-bit division for LIV decoding on the device.
//
// LIV decoding divides by tensor dimensions that are fixed for a whole launch
// (Section 3.1: recomputing LIVs for a new lexicographical order, the "LIV
// shuffle", needs an integer division and modulo per mode; Section 4.1 uses
// division to find regions and shave keys).  A runtime 64-bit division is a
// long instruction sequence on gfx950, so each divisor is turned once on the
// host into a multiply-high plus shifts, following Granlund & Montgomery,
// "Division by invariant integers using multiplication" (PLDI 1994), Figure 4.1:
//   l  = ceil(log2 d),  m' = floor(2^64 * (2^l - d) / d) + 1,
//   t1 = mulhi(m', n),  q = (t1 + ((n - t1) >> 1)) >> (l - 1).
// Powers of two (including d = 1) use a plain shift.
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define LCO_HD __host__ __device__ __forceinline__
#else
#define LCO_HD inline
#endif

namespace lco {

struct FastDiv {
  uint64_t d = 1;      // divisor, >= 1
  uint64_t magic = 0;  // m' (unused for powers of two)
  uint32_t shift = 0;  // log2 d for powers of two; l - 1 otherwise
  uint32_t pow2 = 1;   // 1 if d is a power of two
};

LCO_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

inline FastDiv make_fastdiv(uint64_t d) {
  FastDiv f;
  f.d = d ? d : 1;
  d = f.d;
  if ((d & (d - 1)) == 0) {
    f.pow2 = 1;
    f.shift = (uint32_t)__builtin_ctzll(d);
    f.magic = 0;
  } else {
    const uint32_t l = 64u - (uint32_t)__builtin_clzll(d - 1);  // ceil(log2 d), 2..64
    const uint64_t two_l_minus_d = (l == 64) ? (uint64_t)(0 - d) : ((1ull << l) - d);
    f.magic = (uint64_t)((((unsigned __int128)two_l_minus_d) << 64) / d) + 1;
    f.shift = l - 1;
    f.pow2 = 0;
  }
  return f;
}

LCO_HD uint64_t fd_div(const FastDiv& f, uint64_t n) {
  if (f.pow2) return n >> f.shift;
  const uint64_t t1 = mulhi64(f.magic, n);
  return (t1 + ((n - t1) >> 1)) >> f.shift;
}

// quotient and remainder
LCO_HD uint64_t fd_divmod(const FastDiv& f, uint64_t n, uint64_t& rem) {
  const uint64_t q = fd_div(f, n);
  rem = n - q * f.d;
  return q;
}

}  // namespace lco
