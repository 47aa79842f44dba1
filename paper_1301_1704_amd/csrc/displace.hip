// One time step of moving particle systems, for the serving form: every
// coordinate moves by sigma * z with z standard normal, then is clamped into
// [0, 1 - 2^-24] so the point stays in the half-open unit cube the build
// requires (Section 1.4). Dynamic problems rebuild the structures after every
// such step (Section 1, Section 2.5); the step itself is not part of the
// paper's build and is here so that a whole serving request runs on the GPU.
//
// Normals are counter based, so any system can be stepped in any batch with
// the same result: coordinate d of point i uses output 3i + d of the
// splitmix64 stream `seed` (Steele, Lea and Flood, OOPSLA 2014: output c is
// mix(seed + (c + 1) * gamma)); its top 24 bits give u1 = (k + 1) * 2^-24 in
// (0, 1] and the next 24 bits u2 = k * 2^-24 in [0, 1); the Box-Muller
// transform z = sqrt(-2 ln u1) cos(2 pi u2) is evaluated in FP32.
#include "internal.h"

namespace fmmds {

__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ float step_coord(float x, uint64_t seed, uint64_t c, float sigma) {
  const uint64_t h = splitmix_mix(seed + (c + 1) * 0x9E3779B97F4A7C15ull);
  const float u1 = (float)((h >> 40) + 1) * 5.9604644775390625e-8f;  // 2^-24
  const float u2 = (float)((h >> 16) & 0xFFFFFFull) * 5.9604644775390625e-8f;
  const float z = sqrtf(-2.0f * logf(u1)) * cosf(6.283185307179586f * u2);
  float v = x + sigma * z;
  // NaN passes through (the build then reports it); finite values are clamped.
  v = v < 0.0f ? 0.0f : v;
  v = v > 0.99999994039535522f ? 0.99999994039535522f : v;
  return v;
}

__global__ __launch_bounds__(256) void k_displace(DisplaceArgs a, float sigma, float* out) {
  const uint64_t total = a.first[a.n];
  for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < total; e += gridDim.x * 256ull) {
    uint32_t k = 0;  // the set holding e: the last k with first[k] <= e
    for (uint32_t step = 16; step > 0; step >>= 1)
      if (k + step < a.n && a.first[k + step] <= e) k += step;
    const uint64_t i = e - a.first[k];
    float* p = a.xyz[k] + 3 * i;
    const float x = step_coord(p[0], a.seed[k], 3 * i, sigma);
    const float y = step_coord(p[1], a.seed[k], 3 * i + 1, sigma);
    const float z = step_coord(p[2], a.seed[k], 3 * i + 2, sigma);
    p[0] = x;
    p[1] = y;
    p[2] = z;
    if (out) {
      float* q = out + 3 * (a.out_first[k] + i);
      q[0] = x;
      q[1] = y;
      q[2] = z;
    }
  }
}

void launch_displace(const DisplaceArgs& a, float sigma, float* out, hipStream_t s) {
  const uint64_t total = a.first[a.n];
  if (total == 0) return;
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(div_up(total, 256), 8192));
  hipLaunchKernelGGL(k_displace, dim3(grid), dim3(256), 0, s, a, sigma, out);
}

}  // namespace fmmds
