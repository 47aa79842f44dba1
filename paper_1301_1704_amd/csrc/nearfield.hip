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
//
// Two paths, split by the receiver box's point count:
//   - sparse boxes (at most kNearDenseMin points): one thread per box. Its
//     points share every source load, and the lanes of a wave sit in
//     neighboring boxes with overlapping E2 lists, so most of those loads are
//     shared through the caches too.
//   - dense boxes (clustered input puts hundreds of points in one box): the
//     box is cut into tasks of at most 64 receivers, one wave per task. The
//     wave stages the box's E2 source points in LDS 64 at a time (one
//     coalesced 16-byte load per lane) and every lane sums its receiver
//     against the whole tile. A task of r < 64 receivers splits the tile over
//     64 / R lane groups (R = r rounded up to a power of two) whose partial
//     sums are added by shuffles at the end. After its first task a wave takes
//     the next from an atomic ticket, so boxes of very different sizes balance.
#include <mutex>

#include "device.h"
#include "internal.h"

namespace fmmds {

// Scratch counters of one near-field call (kNearCounters of them): [0]
// tasks written, [1] the dense path's ticket.

__global__ __launch_bounds__(256) void k_pack_sources(const float* __restrict__ sxyz,
                                                      const uint32_t* __restrict__ sperm,
                                                      const float* __restrict__ charges,
                                                      uint32_t n, float4* __restrict__ out,
                                                      uint32_t* __restrict__ counters) {
  if (blockIdx.x == 0 && threadIdx.x < kNearCounters) counters[threadIdx.x] = 0;
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += gridDim.x * 256ull) {
    const float q = charges ? charges[sperm[i]] : 1.0f;
    out[i] = make_float4(sxyz[3 * i], sxyz[3 * i + 1], sxyz[3 * i + 2], q);
  }
}

// One term of the sum: q / |x - y|, zero for coincident points.
__device__ __forceinline__ float pair_term(const float4 x, float yx, float yy, float yz) {
  const float dx = x.x - yx, dy = x.y - yy, dz = x.z - yz;
  const float r2 = dx * dx + dy * dy + dz * dz;
  return r2 > 0.0f ? x.w * rsqrtf(r2) : 0.0f;
}

// Sparse path: one thread per receiver box, up to R of its points at a time:
// each source point is loaded once for all of them. R = 4 suits boxes of one
// or two points (uniform input); with more points per box (sphere, clusters)
// a wave then walks its lists twice whenever one of its boxes has five or
// more, so R = 8 is taken when the receivers average more than two points
// per finest box (measured: 2.24 against 2.86 ms on the uniform benchmark
// build, 4.36 against 3.83 ms on sphere + clusters). The list is
// walked eight entries at a time (their source ranks, then their bookmarks,
// then their points), so that the dependent loads of eight entries overlap.
// Every receiver's terms are added in list order, point by point. A box of
// more than kNearDenseMin points is not summed here: its thread appends the
// box's tasks (box, chunk of 64 receivers) to the dense path's task list.
constexpr uint32_t kNearBatch = 8;

template <uint32_t R>
__global__ __launch_bounds__(256) void k_near_field(
    uint32_t n_rbox, const uint32_t* __restrict__ rbegin, const float* __restrict__ rxyz,
    const uint32_t* __restrict__ rperm, const uint32_t* __restrict__ e2_off,
    const uint32_t* __restrict__ e2_ent, const uint32_t* __restrict__ sbegin,
    const float4* __restrict__ src, float* __restrict__ phi,
    unsigned long long* __restrict__ n_pairs, uint2* __restrict__ tasks,
    uint32_t* __restrict__ counters) {
  const uint64_t b = blockIdx.x * 256ull + threadIdx.x;
  uint64_t pairs = 0;
  uint32_t my_tasks = 0;
  if (b < n_rbox) {
    const uint32_t k0 = rbegin[b], k1 = rbegin[b + 1];
    if (k1 - k0 > kNearDenseMin) {
      my_tasks = (k1 - k0 + 63u) / 64u;
    } else {
      const uint32_t e0 = e2_off[b], e1 = e2_off[b + 1];
      for (uint32_t kc = k0; kc < k1; kc += R) {
        float yx[R], yy[R], yz[R], acc[R];
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
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
              for (uint32_t r = 0; r < R; ++r) acc[r] += pair_term(x, yx[r], yy[r], yz[r]);
            }
            pts += i1[j] - i0[j];
          }
        }
        const uint32_t nr = min(R, k1 - kc);
#pragma unroll
        for (uint32_t r = 0; r < R; ++r)
          if (r < nr) phi[rperm[kc + r]] = acc[r];
        pairs += (uint64_t)pts * nr;
      }
    }
  }
  // Dense boxes: one atomic per wave reserves the wave's tasks.
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t incl = wave_incl_scan(my_tasks);
  const uint32_t total = __shfl(incl, 63, 64);
  if (total) {
    uint32_t base = 0;
    if (lane == 63) base = atomicAdd(&counters[0], total);
    base = __shfl(base, 63, 64);
    for (uint32_t c = 0; c < my_tasks; ++c)
      tasks[base + incl - my_tasks + c] = make_uint2((uint32_t)b, c);
  }
  if (n_pairs) {
    const uint64_t w = wave_sum_u64(pairs);
    if (lane == 0 && w) atomicAdd(n_pairs, (unsigned long long)w);
  }
}

// Dense path: one wave per task, waves taking further tasks from a ticket. Lane l
// first loads E2 entry l of the box (lists hold at most 27 entries) and the
// entries' point counts are scanned across the wave, so that the box's
// source points form one concatenated sequence; each round stages the next
// 64 of them in the wave's LDS tile.
constexpr uint32_t kNearDenseBlock = 256;

__global__ __launch_bounds__(kNearDenseBlock) void k_near_dense(
    const uint32_t* __restrict__ rbegin, const float* __restrict__ rxyz,
    const uint32_t* __restrict__ rperm, const uint32_t* __restrict__ e2_off,
    const uint32_t* __restrict__ e2_ent, const uint32_t* __restrict__ sbegin,
    const float4* __restrict__ src, float* __restrict__ phi,
    unsigned long long* __restrict__ n_pairs, const uint2* __restrict__ tasks,
    uint32_t* __restrict__ counters) {
  constexpr uint32_t kWaves = kNearDenseBlock / 64;
  __shared__ float4 s_tile[kWaves][64];
  __shared__ uint32_t s_pre[kWaves][64];  // inclusive prefix of the entries' point counts
  __shared__ uint32_t s_first[kWaves][64];  // first sorted source point of each entry
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t n_tasks = __hip_atomic_load(&counters[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t n_waves = gridDim.x * kWaves;
  uint64_t pairs = 0;
  // Wave g takes task g first, then tickets past the first n_waves: waves
  // without a task exit without touching the ticket (atomics on one address
  // are serialized, and most waves have nothing to do on sparse input).
  for (uint32_t t = blockIdx.x * kWaves + w; t < n_tasks;) {
    const uint2 task = tasks[t];
    const uint32_t b = task.x;
    const uint32_t k0 = rbegin[b] + 64u * task.y;
    const uint32_t nr = min(64u, rbegin[b + 1] - k0);
    const uint32_t e0 = e2_off[b], ne = e2_off[b + 1] - e0;  // ne <= 27
    uint32_t first = 0, cnt = 0;
    if (lane < ne) {
      const uint32_t sb = e2_ent[e0 + lane];
      first = sbegin[sb];
      cnt = sbegin[sb + 1] - first;
    }
    const uint32_t pre = wave_incl_scan(cnt);
    const uint32_t total = __shfl(pre, 63, 64);
    s_pre[w][lane] = pre;
    s_first[w][lane] = first;
    // lanes: receiver r = lane % R, slice s = lane / R of S = 64 / R slices
    uint32_t R = 1;
    while (R < nr) R <<= 1;
    const uint32_t S = 64u / R, r = lane & (R - 1), s = lane / R;
    const uint32_t k = k0 + min(r, nr - 1);
    const float yx = rxyz[3 * (uint64_t)k], yy = rxyz[3 * (uint64_t)k + 1],
                yz = rxyz[3 * (uint64_t)k + 2];
    float acc = 0.0f;
    for (uint32_t p = 0; p < total; p += 64) {
      // Stage points p .. p + 63 of the concatenation: point q lies in the
      // first entry whose inclusive prefix exceeds q.
      const uint32_t q = p + lane;
      float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
      if (q < total) {
        uint32_t lo = 0, hi = ne - 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_pre[w][mid] > q) hi = mid;
          else lo = mid + 1;
        }
        const uint32_t before = lo ? s_pre[w][lo - 1] : 0u;
        x = src[s_first[w][lo] + (q - before)];
      }
      // every lane's reads of the previous tile were issued before this store
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      s_tile[w][lane] = x;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const uint32_t m = min(64u, total - p);
      uint32_t j = s;
      for (; j + 3 * S < m; j += 4 * S) {
        const float4 a = s_tile[w][j], c = s_tile[w][j + S], d = s_tile[w][j + 2 * S],
                     f = s_tile[w][j + 3 * S];
        acc += pair_term(a, yx, yy, yz);
        acc += pair_term(c, yx, yy, yz);
        acc += pair_term(d, yx, yy, yz);
        acc += pair_term(f, yx, yy, yz);
      }
      for (; j < m; j += S) acc += pair_term(s_tile[w][j], yx, yy, yz);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    for (uint32_t o = R; o < 64u; o <<= 1) acc += __shfl_xor(acc, (int)o, 64);
    if (s == 0 && r < nr) phi[rperm[k]] = acc;
    if (lane == 0) pairs += (uint64_t)total * nr;
    // the next task restages s_pre / s_first: all reads of this one are done
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t next = 0;
    if (lane == 0) next = atomicAdd(&counters[1], 1u);
    t = n_waves + __shfl(next, 0, 64);
  }
  if (n_pairs && lane == 0 && pairs) atomicAdd(n_pairs, (unsigned long long)pairs);
}

uint64_t near_field_max_tasks(uint32_t n_recv) {
  // a dense box of r > kNearDenseMin points has ceil(r / 64) <= r / (kNearDenseMin + 1)
  // tasks (since kNearDenseMin + 1 <= 32)
  static_assert(kNearDenseMin + 1 <= 32, "task bound");
  return (uint64_t)n_recv / (kNearDenseMin + 1) + 1;
}

void launch_pack_sources(const float* sxyz, const uint32_t* sperm, const float* charges,
                         uint32_t n, float4* out, uint32_t* counters, hipStream_t s) {
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(div_up(n, 256), 8192));
  hipLaunchKernelGGL(k_pack_sources, dim3(grid), dim3(256), 0, s, sxyz, sperm, charges, n, out,
                     counters);
}

void launch_near_field(uint32_t n_rbox, uint32_t n_recv, const uint32_t* rbegin,
                       const float* rxyz, const uint32_t* rperm, const uint32_t* e2_off,
                       const uint32_t* e2_ent, const uint32_t* sbegin, const float4* src,
                       float* phi, unsigned long long* n_pairs, uint2* tasks,
                       uint32_t* counters, hipStream_t s) {
  if (n_rbox == 0) return;
  if (n_recv > 2ull * n_rbox)
    hipLaunchKernelGGL(k_near_field<8>, dim3(div_up(n_rbox, 256)), dim3(256), 0, s, n_rbox,
                       rbegin, rxyz, rperm, e2_off, e2_ent, sbegin, src, phi, n_pairs, tasks,
                       counters);
  else
    hipLaunchKernelGGL(k_near_field<4>, dim3(div_up(n_rbox, 256)), dim3(256), 0, s, n_rbox,
                       rbegin, rxyz, rperm, e2_off, e2_ent, sbegin, src, phi, n_pairs, tasks,
                       counters);
  // Persistent waves over the dense tasks: enough for the most tasks the
  // receivers can make, at most eight blocks per compute unit; they exit
  // when the ticket passes the task count.
  const uint32_t waves = kNearDenseBlock / 64;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(
      div_up(near_field_max_tasks(n_recv), waves), 2048);
  hipLaunchKernelGGL(k_near_dense, dim3(grid), dim3(kNearDenseBlock), 0, s, rbegin, rxyz, rperm,
                     e2_off, e2_ent, sbegin, src, phi, n_pairs, tasks, counters);
}

// ---------------------------------------------------------------------------
// Fixed scratch of fmmds_near_field_static, the entry point for callers that
// cannot allocate: packed sources, dense-path tasks and counters live here
// instead of in memory from the cache. Each GPU holds its own copy of the
// array, at its own address, from the library's load on that GPU until the
// process ends. In host code `scratch` names a host-side stand-in, never the
// device memory: the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNearStaticBytes];

fmmds_status near_field_static_scratch(void** out) {
  static std::mutex mu;
  static void* ptr[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return FMMDS_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> g(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return FMMDS_ERR_DEVICE;
    }
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return FMMDS_OK;
}

}  // namespace fmmds
