// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) and Box-Muller normals,
// usable from device and host code.
//
// Counter layout: (block, draw, chain << 8 | stream, sub); key = seed split
// into two 32-bit words.  Uniforms are (x + 0.5) 2^-32 in float64 (never 0 or
// 1).  Normals: Box-Muller on word pairs (0, 1) and (2, 3) in float64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmcrng {

enum Stream : uint32_t {
  kMomenta = 3,
  kAccept = 4,
  kChi2 = 5,
  kGig = 6,
  kBias = 7,
  kRjMomenta = 8,
  kRjAccept = 9,
  kTau = 10,
  kWarm = 11,
};

struct U4 {
  uint32_t w[4];
};

__host__ __device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint64_t seed) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c0;
    const uint64_t p1 = (uint64_t)M1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  U4 o;
  o.w[0] = c0;
  o.w[1] = c1;
  o.w[2] = c2;
  o.w[3] = c3;
  return o;
}

__host__ __device__ __forceinline__ U4 block(uint64_t seed, uint32_t chain, uint32_t stream,
                                             uint32_t draw, uint32_t sub, uint32_t blk) {
  return philox(blk, draw, (chain << 8) | stream, sub, seed);
}

__host__ __device__ __forceinline__ double uniform(uint32_t x) {
  return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

// Normal pair from two words: (r cos, r sin), r = sqrt(-2 ln u0), angle 2 pi u1.
__host__ __device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double* z0,
                                                    double* z1) {
  const double u0 = uniform(a), u1 = uniform(b);
  const double r = sqrt(-2.0 * log(u0));
  const double t = 2.0 * 3.14159265358979323846 * u1;
  *z0 = r * cos(t);
  *z1 = r * sin(t);
}

}  // namespace hmcrng
