// Device-side helpers shared by the gfx950 kernels of libfmmds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmmds {

// ---------------------------------------------------------------------------
// Morton index arithmetic (Section 1.4: bit b of the box coordinates x, y, z
// sits at bit 3b, 3b+1, 3b+2 of the index; Section 2.4: interleave and
// deinterleave). Magic-mask bit spreading, 21 bits per axis.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x001f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x001f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x00000000001fffffull;
  return (uint32_t)x;
}

// 10-bit-per-axis variants for keys of at most 30 bits.
__device__ __forceinline__ uint32_t spread3_10(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000ffu;
  x = (x | (x << 8)) & 0x0300f00fu;
  x = (x | (x << 4)) & 0x030c30c3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// Box of a point at level L (1 <= L <= 21): floor(x * 2^L) per axis in FP32
// (the scaling is exact), interleaved. `ok` is false for a coordinate
// outside [0, 1) or NaN; such a point gets box 0.
__device__ __forceinline__ uint64_t point_key(float x, float y, float z, uint32_t L, bool& ok) {
  const float scale = (float)(1u << L);
  const uint32_t qmax = (1u << L) - 1;
  ok = (x >= 0.0f && x < 1.0f) && (y >= 0.0f && y < 1.0f) && (z >= 0.0f && z < 1.0f);
  uint32_t qx = 0, qy = 0, qz = 0;
  if (ok) {
    qx = min((uint32_t)floorf(x * scale), qmax);
    qy = min((uint32_t)floorf(y * scale), qmax);
    qz = min((uint32_t)floorf(z * scale), qmax);
  }
  if (L <= 10) return spread3_10(qx) | (spread3_10(qy) << 1) | (spread3_10(qz) << 2);
  return spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
}

// Blocks are dispatched to the 8 XCDs (each with its own L2) round-robin:
// block b runs on XCD b % 8. Renumbering so that each XCD takes one
// contiguous range of work keeps each XCD's reads and writes in one region
// of memory. A bijection on [0, n).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n) {
  const uint32_t x = b & 7u, q = n >> 3, r = n & 7u;
  return x * q + min(x, r) + (b >> 3);
}

// ---------------------------------------------------------------------------
// Wave64 primitives.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `m` at lanes below this one.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
  return v;
}

// ---------------------------------------------------------------------------
// Decoupled look-back (single-pass chained scan). A status word holds a
// 2-bit state in bits 62..63 and a 62-bit running count: 0 = not ready,
// 1 = this tile's aggregate only, 2 = inclusive prefix up to this tile.
// Tiles take their id from an atomic ticket, so every tile a waiter looks
// back at has already been scheduled and will publish.
// ---------------------------------------------------------------------------
constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStInc = 2ull << 62;
constexpr uint64_t kStVal = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t ld_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A tile whose column holds its aggregate already (published before the
// tile's other work, tile 0 publishing its inclusive value): the walk back to
// the nearest inclusive prefix, W predecessors' status words loaded at once
// per round and summed in order up to the first inclusive prefix; an
// unpublished word ends the round, and the next round starts there. Then the
// tile's inclusive value is published; returns the exclusive prefix.
template <int W>
__device__ __forceinline__ uint64_t lookback_window(uint64_t* col, uint64_t stride, uint32_t tile,
                                                    uint64_t agg) {
  if (tile == 0) return 0;  // tile 0 published its inclusive value already
  uint64_t excl = 0;
  int64_t t = (int64_t)tile - 1;
  while (true) {
    uint64_t s[W];
#pragma unroll
    for (int i = 0; i < W; ++i)  // below tile 0 nothing is read: tile 0 ends every walk
      s[i] = t - i >= 0 ? ld_status(col + (uint64_t)(t - i) * stride) : kStInc;
    bool stop = false, found = false;
    uint32_t used = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      if (!stop) {
        const uint64_t f = s[i] >> 62;
        if (f == 0) {
          stop = true;
        } else {
          excl += s[i] & kStVal;
          ++used;
          if (f == 2) stop = found = true;
        }
      }
    }
    if (found) break;
    t -= used;
    if (used < (uint32_t)W) __builtin_amdgcn_s_sleep(1);
  }
  st_status(col + (uint64_t)tile * stride, kStInc | (excl + agg));
  return excl;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The same chained scan for a single counter, called by all 64 lanes of one
// wave: lane i inspects tile (t - i), so one round covers 64 predecessors.
// The nearest predecessor holding an inclusive prefix ends the walk; every
// tile between it and this one must at least have published its aggregate.
__device__ __forceinline__ uint64_t lookback_wave(uint64_t* status, uint32_t tile, uint64_t agg) {
  const uint32_t lane = lane_id();
  if (tile == 0) {
    if (lane == 0) st_status(status, kStInc | agg);
    return 0;
  }
  if (lane == 0) st_status(status + tile, kStAgg | agg);
  uint64_t excl = 0;
  int64_t hi = (int64_t)tile - 1;
  while (true) {
    const int64_t t = hi - (int64_t)lane;
    const uint64_t s = t >= 0 ? ld_status(status + t) : kStInc;
    const uint64_t f = s >> 62;
    const uint64_t inc = __ballot(f == 2);
    const uint64_t not_ready = __ballot(f == 0);
    const uint32_t first = inc ? (uint32_t)(__ffsll((long long)inc) - 1) : 64u;
    const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1);
    if (not_ready & need) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += wave_sum_u64(lane <= first ? (s & kStVal) : 0);
    if (first < 64) break;
    hi -= 64;
  }
  if (lane == 0) st_status(status + tile, kStInc | (excl + agg));
  return excl;
}

// Chain per-(item, wave) flag counts of a compaction tile across tiles. The
// NSLOT (<= 64) counts sit in s_cnt in element order; on return they hold
// exclusive prefixes within the tile and the result is the tile's exclusive
// prefix over all earlier tiles. Called by every thread of the block.
template <int NSLOT>
__device__ __forceinline__ uint64_t tile_flags_prefix(uint32_t* s_cnt, uint64_t* s_excl,
                                                      uint64_t* status, uint32_t tile) {
  static_assert(NSLOT <= 64, "one wave scans the slots");
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint32_t lane = threadIdx.x;
    const uint32_t c = lane < NSLOT ? s_cnt[lane] : 0;
    const uint32_t inc = wave_incl_scan(c);
    if (lane < NSLOT) s_cnt[lane] = inc - c;
    const uint32_t total = __shfl(inc, 63, 64);
    const uint64_t ex = lookback_wave(status, tile, total);
    if (lane == 0) *s_excl = ex;
  }
  __syncthreads();
  return *s_excl;
}

}  // namespace fmmds
