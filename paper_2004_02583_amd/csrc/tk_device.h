// Device-side helpers shared by the gfx950 kernels of libtucker_als.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tk {

// Mode-n view [P, I, Q] of a row-major tensor (Section 2 unfolding without
// materialisation): element (p, i, q) lives at (p*I + i)*Q + q and fibre
// j = p*Q + q is column j of A_(n).
struct View {
  int64_t P, I, Q;
  __host__ __device__ int64_t J() const { return P * Q; }
  __host__ __device__ int64_t fibre_base(int64_t j) const {
    int64_t p, q;
    if (((uint64_t)j | (uint64_t)Q) < (1ull << 32)) {   // 32-bit division when it fits
      const uint32_t pj = (uint32_t)j / (uint32_t)Q;
      p = pj;
      q = (uint32_t)j - pj * (uint32_t)Q;
    } else {
      p = j / Q;
      q = j - p * Q;
    }
    return p * I * Q + q;
  }
};

// bf16 is carried as raw 16-bit patterns.
typedef uint16_t bf16_t;

__host__ __device__ inline float bf16_to_f32(bf16_t h) {
  union { uint32_t u; float f; } v;
  v.u = (uint32_t)h << 16;
  return v.f;
}

// float -> bf16, round to nearest even; NaN stays NaN.
__host__ __device__ inline bf16_t f32_to_bf16(float f) {
  union { uint32_t u; float f; } v;
  v.f = f;
  uint32_t u = v.u;
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
    return (bf16_t)((u >> 16) | 0x40u);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (bf16_t)(u >> 16);
}

template <typename T> struct Elem;
template <> struct Elem<double> {
  typedef double acc;
  __device__ static double load(const double* p) { return *p; }
};
template <> struct Elem<float> {
  typedef float acc;
  __device__ static float load(const float* p) { return *p; }
};
template <> struct Elem<bf16_t> {
  typedef float acc;
  __device__ static float load(const bf16_t* p) { return bf16_to_f32(*p); }
};

// Entry (j, r) of the initial-guess sketch S of mode `mode` (Section 5):
// the counter-th output of a SplitMix64 stream (Steele, Lea & Flood 2014)
// seeded with `seed`, counter = mode*2^48 + j*R + r, mapped to [0,1) by its
// top 24 bits.  State of output c is seed + c*gamma; the output is the
// variant-13 finaliser applied to state + gamma.
__device__ __forceinline__ float sketch_value(uint64_t seed, uint64_t counter) {
  const uint64_t gamma = 0x9E3779B97F4A7C15ull;
  uint64_t z = seed + (counter + 1ull) * gamma;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (float)(uint32_t)(z >> 40) * (1.0f / 16777216.0f);
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) {
  return (a + b - 1) / b;
}

}  // namespace tk
