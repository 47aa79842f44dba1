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
// One thread per receiver box: its points share every source load, and the
// lanes of a wave sit in neighboring boxes with overlapping E2 lists, so most
// of those loads are shared through the caches too.
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

// One thread per receiver box, up to kNearRecv of its points at a time: each
// source point is loaded once for all of them. The list is walked eight
// entries at a time (their source ranks, then their bookmarks, then their
// points), so that the dependent loads of eight entries overlap. Every
// receiver's terms are added in list order, point by point.
constexpr uint32_t kNearBatch = 8;
constexpr uint32_t kNearRecv = 4;

__global__ __launch_bounds__(256) void k_near_field(
    uint32_t n_rbox, const uint32_t* __restrict__ rbegin, const float* __restrict__ rxyz,
    const uint32_t* __restrict__ rperm, const uint32_t* __restrict__ e2_off,
    const uint32_t* __restrict__ e2_ent, const uint32_t* __restrict__ sbegin,
    const float4* __restrict__ src, float* __restrict__ phi,
    unsigned long long* __restrict__ n_pairs) {
  const uint64_t b = blockIdx.x * 256ull + threadIdx.x;
  uint64_t pairs = 0;
  if (b < n_rbox) {
    const uint32_t k0 = rbegin[b], k1 = rbegin[b + 1];
    const uint32_t e0 = e2_off[b], e1 = e2_off[b + 1];
    for (uint32_t kc = k0; kc < k1; kc += kNearRecv) {
      float yx[kNearRecv], yy[kNearRecv], yz[kNearRecv], acc[kNearRecv];
#pragma unroll
      for (uint32_t r = 0; r < kNearRecv; ++r) {
        const uint32_t k = min(kc + r, k1 - 1);  // extra lanes repeat the last point
        yx[r] = rxyz[3 * (uint64_t)k], yy[r] = rxyz[3 * (uint64_t)k + 1],
        yz[r] = rxyz[3 * (uint64_t)k + 2];
        acc[r] = 0.0f;
      }
      uint32_t pts = 0;
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
          for (uint32_t i = i0[j]; i < i1[j]; ++i) {
            const float4 x = src[i];
#pragma unroll
            for (uint32_t r = 0; r < kNearRecv; ++r) {
              const float dx = x.x - yx[r], dy = x.y - yy[r], dz = x.z - yz[r];
              const float r2 = dx * dx + dy * dy + dz * dz;
              acc[r] += r2 > 0.0f ? x.w * rsqrtf(r2) : 0.0f;
            }
          }
          pts += i1[j] - i0[j];
        }
      }
      const uint32_t nr = min(kNearRecv, k1 - kc);
#pragma unroll
      for (uint32_t r = 0; r < kNearRecv; ++r)
        if (r < nr) phi[rperm[kc + r]] = acc[r];
      pairs += (uint64_t)pts * nr;
    }
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

void launch_near_field(uint32_t n_rbox, const uint32_t* rbegin, const float* rxyz,
                       const uint32_t* rperm, const uint32_t* e2_off, const uint32_t* e2_ent,
                       const uint32_t* sbegin, const float4* src, float* phi,
                       unsigned long long* n_pairs, hipStream_t s) {
  if (n_rbox == 0) return;
  hipLaunchKernelGGL(k_near_field, dim3(div_up(n_rbox, 256)), dim3(256), 0, s, n_rbox, rbegin,
                     rxyz, rperm, e2_off, e2_ent, sbegin, src, phi, n_pairs);
}

}  // namespace fmmds
