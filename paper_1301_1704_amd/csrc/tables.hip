// Nonempty-box tables: leaf boundary detection plus stream compaction, and the
// coarser levels, parents, children and child masks.
//
// The paper scans a dense histogram of all 8^lmax boxes (Section 2.3,
// Algorithm 3), which costs memory and time in the number of boxes. Here the
// sorted keys already group the points by box, so a box starts wherever the
// key differs from the previous one (adjacent difference) and the starts are
// compacted with a single-pass scan: the cost follows the nonempty boxes only.
// Coarser levels repeat this on the previous level's keys shifted right by 3
// (the parent of a box is its Morton index shifted by one level, Section 3.2).
#include "device.h"
#include "internal.h"

namespace fmmds {

constexpr int kCompWaves = kCompBlock / 64;

struct P3 {
  float x, y, z;
};

// ---------------------------------------------------------------------------
// K3 + K4: from the sorted (key, index) pairs write the permutation and the
// reordered coordinates (Algorithm 5, steps 3 and 6: SortedSrc / SortedRecv
// and RecvPermutationIdx) and compact the finest level's nonempty boxes: their
// keys and bookmarks (Algorithm 3's NonEmptyIdx and Bookmark).
// ---------------------------------------------------------------------------
// With a batch (set_off != nullptr) the key carries the set id from bit
// `set_shift` up and the permutation is written relative to the set's first
// point.
template <bool PACKED, typename KeyT>
__global__ __launch_bounds__(kCompBlock) void k_leaf(
    const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sv, const P3* __restrict__ xyz,
    uint32_t n, uint32_t* __restrict__ perm, P3* __restrict__ sorted_xyz,
    KeyT* __restrict__ leaf_key, uint32_t* __restrict__ leaf_begin, uint64_t* __restrict__ status,
    uint32_t* __restrict__ tile_counter, uint32_t* __restrict__ n_out,
    const uint64_t* __restrict__ set_off, uint32_t set_shift) {
  __shared__ uint32_t s_cnt[kCompItems * kCompWaves];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, w = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint64_t tbase = (uint64_t)tile * kCompTile;

  uint64_t key[kCompItems];
  uint32_t incl[kCompItems];
  uint32_t flags = 0;
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t e = tbase + (uint64_t)i * kCompBlock + tid;
    const bool valid = e < n;
    uint64_t kk = 0, kp = 0;
    uint32_t idx = 0;
    if (valid) {
      const uint64_t el = sk[e];
      kk = PACKED ? (el >> 32) : el;
      idx = PACKED ? (uint32_t)el : sv[e];
      if (e > 0) kp = PACKED ? (sk[e - 1] >> 32) : sk[e - 1];
      perm[e] = set_off ? idx - (uint32_t)set_off[kk >> set_shift] : idx;
      if (xyz) sorted_xyz[e] = xyz[idx];  // null: the coordinates are already in place
    }
    const bool f = valid && (e == 0 || kk != kp);
    const uint64_t ball = __ballot(f);
    incl[i] = mbcnt(ball) + (f ? 1u : 0u);
    flags |= (f ? 1u : 0u) << i;
    key[i] = kk;
    if ((tid & 63) == 0) s_cnt[i * kCompWaves + w] = (uint32_t)__popcll(ball);
  }
  const uint64_t texcl = tile_flags_prefix<kCompItems * kCompWaves>(s_cnt, &s_excl, status, tile);
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t e = tbase + (uint64_t)i * kCompBlock + tid;
    const uint64_t rank_incl = texcl + s_cnt[i * kCompWaves + w] + incl[i];
    if ((flags >> i) & 1u) {
      leaf_key[rank_incl - 1] = (KeyT)key[i];
      leaf_begin[rank_incl - 1] = (uint32_t)e;
    }
    if (e + 1 == n) {
      leaf_begin[rank_incl] = n;
      *n_out = (uint32_t)rank_incl;
    }
  }
}

void launch_leaf(bool packed, bool key64, const uint64_t* sk, const uint32_t* sv,
                 const float* xyz, uint32_t n, uint32_t* perm, float* sorted_xyz, void* leaf_key,
                 uint32_t* leaf_begin, uint64_t* status, uint32_t* tile_counter, uint32_t* n_out,
                 hipStream_t s, const uint64_t* set_off, uint32_t set_shift) {
  const uint32_t grid = div_up(n, kCompTile);
#define FMMDS_LEAF(P, K)                                                                         \
  hipLaunchKernelGGL((k_leaf<P, K>), dim3(grid), dim3(kCompBlock), 0, s, sk, sv, (const P3*)xyz, \
                     n, perm, (P3*)sorted_xyz, (K*)leaf_key, leaf_begin, status, tile_counter,    \
                     n_out, set_off, set_shift)
  if (packed && key64) FMMDS_LEAF(true, uint64_t);
  else if (packed) FMMDS_LEAF(true, uint32_t);
  else if (key64) FMMDS_LEAF(false, uint64_t);
  else FMMDS_LEAF(false, uint32_t);
#undef FMMDS_LEAF
}

// ---------------------------------------------------------------------------
// K5: level l from level l + 1. Box j of level l+1 starts a new parent when
// its key >> 3 differs from box j-1's. Writes, at level l: keys, bookmarks
// (the first child's bookmark), first-child ranks and the 8-bit mask of
// occupied child octants; at level l+1: the parent rank of every box.
// The number of level-(l+1) boxes is read on the device; the grid covers the
// worst case and surplus tiles exit at once.
// ---------------------------------------------------------------------------
template <typename KeyT>
__global__ __launch_bounds__(kCompBlock) void k_level(
    const KeyT* __restrict__ kin, const uint32_t* __restrict__ bin,
    const uint32_t* __restrict__ n_in_p, uint32_t n_points, KeyT* __restrict__ kout,
    uint32_t* __restrict__ bout, uint32_t* __restrict__ cout, uint8_t* __restrict__ mout,
    uint32_t* __restrict__ pout, uint64_t* __restrict__ status, uint32_t* __restrict__ tile_counter,
    uint32_t* __restrict__ n_out) {
  __shared__ uint32_t s_cnt[kCompItems * kCompWaves];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, w = tid >> 6;
  const uint32_t n_in = *n_in_p;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint64_t tbase = (uint64_t)tile * kCompTile;
  if (tbase >= n_in) return;  // whole block: no valid element in this tile

  // Loads first, from indices clamped into [0, n_in) so that they are
  // unconditional and all in flight at once (results past n_in are
  // discarded); every load precedes every store, since on this GPU a wait
  // for a load also waits for all earlier stores.
  // Lanes 0..7 also load the 8 keys after the wave's last box (a parent's
  // run of children may continue there).
  const uint32_t lane = tid & 63u;
  uint64_t kv[kCompItems], kp[kCompItems], kn[kCompItems];
  uint32_t bfirst[kCompItems];
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t jc = min<uint64_t>(tbase + (uint64_t)i * kCompBlock + tid, n_in - 1);
    kv[i] = (uint64_t)kin[jc];
    kp[i] = (uint64_t)kin[jc > 0 ? jc - 1 : 0];
    bfirst[i] = bin[jc];
    const uint64_t wend = tbase + (uint64_t)i * kCompBlock + (tid & ~63u) + 64;
    const uint64_t jn = min<uint64_t>(wend + lane, n_in - 1);
    kn[i] = lane < 8 ? (uint64_t)kin[jn] : 0;
  }
  uint64_t pkey[kCompItems];
  uint32_t incl[kCompItems];
  uint32_t cmask[kCompItems];  // child octants of the parent a flagged box starts
  uint32_t flags = 0;
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t j = tbase + (uint64_t)i * kCompBlock + tid;
    const bool valid = j < n_in;
    const uint64_t pk = kv[i] >> 3;
    const uint32_t oct = valid ? (uint32_t)(kv[i] & 7u) : 8u;
    const bool f = valid && (j == 0 || pk != (kp[i] >> 3));
    const uint64_t ball = __ballot(f);
    incl[i] = mbcnt(ball) + (f ? 1u : 0u);
    flags |= (f ? 1u : 0u) << i;
    pkey[i] = pk;
    if (lane == 0) s_cnt[i * kCompWaves + w] = (uint32_t)__popcll(ball);
    // Boxes j.. up to the next flag share this parent. Consecutive lanes hold
    // consecutive boxes, so the children inside this wave are the lanes from
    // here to the next flagged lane: one ballot per child octant.
    const uint64_t later = ball & ~((2ull << lane) - 1ull);  // flagged lanes above this one
    const uint32_t end = later ? (uint32_t)(__ffsll((long long)later) - 1) : 64u;
    const uint64_t run = (end == 64 ? ~0ull : ((1ull << end) - 1ull)) & ~((1ull << lane) - 1ull);
    uint32_t m = 0;
#pragma unroll
    for (uint32_t b = 0; b < 8; ++b) m |= ((__ballot(oct == b) & run) ? 1u : 0u) << b;
    // The run may continue past this wave's last lane, over at most the 8
    // boxes loaded above (keys ascend, so the run is a prefix of them).
    const uint64_t wend = j + (64 - lane);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const uint64_t kt = __shfl(kn[i], t, 64);
      if (f && end == 64 && wend + t < n_in && (kt >> 3) == pk) m |= 1u << (kt & 7u);
    }
    cmask[i] = m;
  }
  const uint64_t texcl = tile_flags_prefix<kCompItems * kCompWaves>(s_cnt, &s_excl, status, tile);
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t j = tbase + (uint64_t)i * kCompBlock + tid;
    if (j >= n_in) continue;
    const uint32_t rank = (uint32_t)(texcl + s_cnt[i * kCompWaves + w] + incl[i] - 1);
    pout[j] = rank;
    if ((flags >> i) & 1u) {
      kout[rank] = (KeyT)pkey[i];
      bout[rank] = bfirst[i];
      cout[rank] = (uint32_t)j;
      mout[rank] = (uint8_t)cmask[i];
    }
    if (j + 1 == n_in) {
      bout[rank + 1] = n_points;
      cout[rank + 1] = n_in;
      *n_out = rank + 1;
    }
  }
}

void launch_level(bool key64, const void* kin, const uint32_t* bin, const uint32_t* n_in,
                  uint32_t cap_in, uint32_t n_points, void* kout, uint32_t* bout, uint32_t* cout,
                  uint8_t* mout, uint32_t* pout, uint64_t* status, uint32_t* tile_counter,
                  uint32_t* n_out, hipStream_t s) {
  const uint32_t grid = div_up(cap_in, kCompTile);
  if (key64)
    hipLaunchKernelGGL(k_level<uint64_t>, dim3(grid), dim3(kCompBlock), 0, s, (const uint64_t*)kin,
                       bin, n_in, n_points, (uint64_t*)kout, bout, cout, mout, pout, status,
                       tile_counter, n_out);
  else
    hipLaunchKernelGGL(k_level<uint32_t>, dim3(grid), dim3(kCompBlock), 0, s, (const uint32_t*)kin,
                       bin, n_in, n_points, (uint32_t*)kout, bout, cout, mout, pout, status,
                       tile_counter, n_out);
}

// ---------------------------------------------------------------------------
// K8: largest box occupancy of a level (for the cluster-size depth rule,
// Section 2.1).
// ---------------------------------------------------------------------------
// Each thread takes kOccItems consecutive boxes and loads their
// kOccItems + 1 bookmarks at once (indices clamped to the sentinel at n_in,
// which give 0), so a level is one round of loads rather than a loop of them.
// The block's maximum goes out in one atomic: atomics on one address are
// serialized, and one per wave made the largest levels slower.
constexpr int kOccItems = 16;

__global__ __launch_bounds__(256) void k_max_occupancy(const uint32_t* __restrict__ begin,
                                                       const uint32_t* __restrict__ n_in_p,
                                                       uint32_t* __restrict__ out) {
  const uint32_t n_in = *n_in_p;
  const uint64_t j0 = ((uint64_t)blockIdx.x * 256u + threadIdx.x) * kOccItems;
  uint32_t m = 0;
  if (j0 < n_in) {
    uint32_t b[kOccItems + 1];
#pragma unroll
    for (int i = 0; i <= kOccItems; ++i) {
      const uint64_t j = j0 + (uint64_t)i;
      b[i] = begin[j < n_in ? j : n_in];
    }
#pragma unroll
    for (int i = 0; i < kOccItems; ++i) m = max(m, b[i + 1] - b[i]);
  }
  __shared__ uint32_t s_m[4];
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
    if (m) atomicMax(out, m);
  }
}

void launch_max_occupancy(const uint32_t* begin, const uint32_t* n_in, uint32_t cap,
                          uint32_t* out, hipStream_t s) {
  const uint32_t grid = std::max<uint32_t>(1, div_up(cap, 256u * kOccItems));
  hipLaunchKernelGGL(k_max_occupancy, dim3(grid), dim3(256), 0, s, begin, n_in, out);
}

}  // namespace fmmds
