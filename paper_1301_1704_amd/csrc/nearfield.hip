// Near-field sum over the E2 lists: the first consumer of the structures.
//
// For every receiver point y in the box b of the finest level, the source
// points of the E2 boxes of b are exactly the points Algorithm 2 gathers:
// the E2 list names nonempty source boxes by rank, and a source box's points
// are consecutive in the sorted order from its bookmark to the next one. The
// sum here is the Laplace potential phi(y) = sum q_i / |x_i - y| over those
// points (the direct part of the FMM, Section 1.2), in FP32, with pairs at
// distance zero left out; the result goes to y's original position through
// the receiver permutation (the paper keeps RecvPermutationIdx for this).
//
// Layout: the sorted source points and their charges are packed once into
// 16-byte records (x, y, z, q), so each source point is one 16-byte load.
// One thread per receiver point in sorted order: the lanes of a wave sit in
// neighboring boxes with overlapping E2 lists, so most source loads are
// shared through the caches.
#include "device.h"
#include "internal.h"

namespace fmmds {

__global__ __launch_bounds__(256) void k_pack_sources(const float* __restrict__ sxyz,
                                                      const uint32_t* __restrict__ sperm,
                                                      const float* __restrict__ charges,
                                                      uint32_t n, float4* __restrict__ out) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += gridDim.x * 256ull) {
    const float q = charges ? charges[sperm[i]] : 1.0f;
    out[i] = make_float4(sxyz[3 * i], sxyz[3 * i + 1], sxyz[3 * i + 2], q);
  }
}

__global__ __launch_bounds__(256) void k_near_field(
    uint32_t n_recv, uint32_t n_rbox, const uint32_t* __restrict__ rbegin,
    const float* __restrict__ rxyz, const uint32_t* __restrict__ rperm,
    const uint32_t* __restrict__ e2_off, const uint32_t* __restrict__ e2_ent,
    const uint32_t* __restrict__ sbegin, const float4* __restrict__ src,
    float* __restrict__ phi, unsigned long long* __restrict__ n_pairs) {
  const uint64_t k = blockIdx.x * 256ull + threadIdx.x;
  uint32_t pairs = 0;
  if (k < n_recv) {
    uint32_t lo = 0, hi = n_rbox;  // the box holding sorted point k: last b with rbegin[b] <= k
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (rbegin[mid] <= k) lo = mid;
      else hi = mid;
    }
    const float yx = rxyz[3 * k], yy = rxyz[3 * k + 1], yz = rxyz[3 * k + 2];
    float acc = 0.0f;
    const uint32_t e1 = e2_off[lo + 1];
    for (uint32_t e = e2_off[lo]; e < e1; ++e) {
      const uint32_t sb = e2_ent[e];
      const uint32_t i1 = sbegin[sb + 1];
      for (uint32_t i = sbegin[sb]; i < i1; ++i) {
        const float4 x = src[i];
        const float dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        acc += r2 > 0.0f ? x.w * rsqrtf(r2) : 0.0f;
      }
      pairs += i1 - sbegin[sb];
    }
    phi[rperm[k]] = acc;
  }
  if (n_pairs) {
    const uint64_t w = wave_sum_u64(pairs);
    if ((threadIdx.x & 63u) == 0 && w) atomicAdd(n_pairs, (unsigned long long)w);
  }
}

void launch_pack_sources(const float* sxyz, const uint32_t* sperm, const float* charges,
                         uint32_t n, float4* out, hipStream_t s) {
  const uint32_t grid = std::min<uint32_t>(div_up(n, 256), 8192);
  hipLaunchKernelGGL(k_pack_sources, dim3(grid), dim3(256), 0, s, sxyz, sperm, charges, n, out);
}

void launch_near_field(uint32_t n_recv, uint32_t n_rbox, const uint32_t* rbegin,
                       const float* rxyz, const uint32_t* rperm, const uint32_t* e2_off,
                       const uint32_t* e2_ent, const uint32_t* sbegin, const float4* src,
                       float* phi, unsigned long long* n_pairs, hipStream_t s) {
  hipLaunchKernelGGL(k_near_field, dim3(div_up(n_recv, 256)), dim3(256), 0, s, n_recv, n_rbox,
                     rbegin, rxyz, rperm, e2_off, e2_ent, sbegin, src, phi, n_pairs);
}

}  // namespace fmmds
