// Seeded synthetic LPs generated where they are used (host or device), for benchmarks and
// tests: the dense law of the batched configuration, a pure function of (seed, stream,
// index) through one counter-based hash, so any entry can be produced on its own.
//
// Hash: the SplitMix64 finaliser (Steele, Lea & Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014), applied three times:
//   mix(z)   = z += 0x9E3779B97F4A7C15; z = (z ^ z >> 30) * 0xBF58476D1CE4E5B9;
//              z = (z ^ z >> 27) * 0x94D049BB133111EB; z ^ z >> 31          (mod 2^64)
//   h(s,k,i) = mix(mix(mix(s) ^ k) ^ i),   u = (h >> 11) 2^-53,   U(a,b) = a + (b - a) u
// (the multiply and the add rounded separately).  Streams: 1 = A', 2 = b, 3 = c, 6 = the
// batch's sizes, 7 = the batch's per-LP seeds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpgpu {
namespace gen {

constexpr uint64_t kStreamA = 1, kStreamB = 2, kStreamC = 3, kStreamSize = 6, kStreamInst = 7;

__host__ __device__ __forceinline__ uint64_t mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// mix(mix(s) ^ k): the key of one stream, shared by all its indices
__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix(mix(seed) ^ stream);
}
__host__ __device__ __forceinline__ uint64_t hash(uint64_t key, uint64_t idx) { return mix(key ^ idx); }
__host__ __device__ __forceinline__ double uniform(uint64_t key, uint64_t idx, double lo, double hi) {
  const double u = (double)(hash(key, idx) >> 11) * 0x1.0p-53;
  return lo + (hi - lo) * u;
}

}  // namespace gen
}  // namespace lpgpu
