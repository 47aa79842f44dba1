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
// One thread per receiver point in sorted order (its box from a point-to-box
// map): the lanes of a wave sit in neighboring boxes with overlapping E2
// lists, so most source loads are shared through the caches.
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

// The finest receiver box of every sorted receiver point (a thread per box
// writes its points' entries), so that the sum needs no search.
__global__ __launch_bounds__(256) void k_point_box(const uint32_t* __restrict__ rbegin,
                                                   uint32_t n_rbox, uint32_t* __restrict__ box_of) {
  for (uint64_t b = blockIdx.x * 256ull + threadIdx.x; b < n_rbox; b += gridDim.x * 256ull) {
    const uint32_t k1 = rbegin[b + 1];
    for (uint32_t k = rbegin[b]; k < k1; ++k) box_of[k] = (uint32_t)b;
  }
}

// The list is walked eight entries at a time: their source ranks, then their
// bookmarks, then their points (two loads in flight per step), so that the
// dependent loads of eight entries overlap. The terms are added in list
// order, point by point.
constexpr uint32_t kNearBatch = 8;

__global__ __launch_bounds__(256) void k_near_field(
    uint32_t n_recv, const uint32_t* __restrict__ box_of, const float* __restrict__ rxyz,
    const uint32_t* __restrict__ rperm, const uint32_t* __restrict__ e2_off,
    const uint32_t* __restrict__ e2_ent, const uint32_t* __restrict__ sbegin,
    const float4* __restrict__ src, float* __restrict__ phi,
    unsigned long long* __restrict__ n_pairs) {
  const uint64_t k = blockIdx.x * 256ull + threadIdx.x;
  uint32_t pairs = 0;
  if (k < n_recv) {
    const uint32_t b = box_of[k];
    const float yx = rxyz[3 * k], yy = rxyz[3 * k + 1], yz = rxyz[3 * k + 2];
    float acc = 0.0f;
    const uint32_t e0 = e2_off[b], e1 = e2_off[b + 1];
    for (uint32_t e = e0; e < e1; e += kNearBatch) {
      uint32_t sb[kNearBatch], i0[kNearBatch], i1[kNearBatch];
#pragma unroll
      for (uint32_t j = 0; j < kNearBatch; ++j) sb[j] = e + j < e1 ? e2_ent[e + j] : 0u;
#pragma unroll
      for (uint32_t j = 0; j < kNearBatch; ++j) {
        const bool ok = e + j < e1;
        i0[j] = ok ? sbegin[sb[j]] : 0u;
        i1[j] = ok ? sbegin[sb[j] + 1] : 0u;
      }
#pragma unroll
      for (uint32_t j = 0; j < kNearBatch; ++j) {
        uint32_t i = i0[j];
        for (; i + 1 < i1[j]; i += 2) {
          const float4 x = src[i], x2 = src[i + 1];
          const float dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
          const float r2 = dx * dx + dy * dy + dz * dz;
          acc += r2 > 0.0f ? x.w * rsqrtf(r2) : 0.0f;
          const float ex = x2.x - yx, ey = x2.y - yy, ez = x2.z - yz;
          const float s2 = ex * ex + ey * ey + ez * ez;
          acc += s2 > 0.0f ? x2.w * rsqrtf(s2) : 0.0f;
        }
        if (i < i1[j]) {
          const float4 x = src[i];
          const float dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
          const float r2 = dx * dx + dy * dy + dz * dz;
          acc += r2 > 0.0f ? x.w * rsqrtf(r2) : 0.0f;
        }
        pairs += i1[j] - i0[j];
      }
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
                       float* phi, unsigned long long* n_pairs, uint32_t* box_of,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_point_box, dim3(std::min<uint32_t>(div_up(n_rbox, 256), 8192)), dim3(256),
                     0, s, rbegin, n_rbox, box_of);
  hipLaunchKernelGGL(k_near_field, dim3(div_up(n_recv, 256)), dim3(256), 0, s, n_recv, box_of,
                     rxyz, rperm, e2_off, e2_ent, sbegin, src, phi, n_pairs);
}

}  // namespace fmmds
