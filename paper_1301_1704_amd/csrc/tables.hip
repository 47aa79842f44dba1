// Nonempty-box tables: box boundaries of every level, parents, children and
// child masks, from the sorted points.
//
// The paper scans a dense histogram of all 8^lmax boxes (Section 2.3,
// Algorithm 3), which costs memory and time in the number of boxes. Here the
// sorted keys already group the points by box, so a box starts wherever the
// key differs from the previous one (adjacent difference) and the starts are
// compacted by a scan: the cost follows the nonempty boxes only. A box's
// parent is its Morton index shifted by one level (Section 3.2), so the same
// comparison, on the keys shifted, finds the boxes of every coarser level.
#include "device.h"
#include "internal.h"

namespace fmmds {

constexpr int kCompWaves = kCompBlock / 64;

struct P3 {
  float x, y, z;
};

// ---------------------------------------------------------------------------
// The finest level alone, with a chained scan (the dense variant's ordering
// of very full boxes): from the sorted (key, index) pairs write the
// permutation and the reordered coordinates (Algorithm 5, steps 3 and 6:
// SortedSrc / SortedRecv and RecvPermutationIdx) and compact the finest
// level's nonempty boxes: their keys and bookmarks (Algorithm 3's NonEmptyIdx
// and Bookmark).
// ---------------------------------------------------------------------------
template <bool PACKED, typename KeyT>
__global__ __launch_bounds__(kCompBlock) void k_leaf(
    const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sv, const P3* __restrict__ xyz,
    uint32_t n, uint32_t* __restrict__ perm, P3* __restrict__ sorted_xyz,
    KeyT* __restrict__ leaf_key, uint32_t* __restrict__ leaf_begin, uint64_t* __restrict__ status,
    uint32_t* __restrict__ tile_counter, uint32_t* __restrict__ n_out) {
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
      perm[e] = idx;
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
                 hipStream_t s) {
  const uint32_t grid = div_up(n, kCompTile);
#define FMMDS_LEAF(P, K)                                                                         \
  hipLaunchKernelGGL((k_leaf<P, K>), dim3(grid), dim3(kCompBlock), 0, s, sk, sv, (const P3*)xyz, \
                     n, perm, (P3*)sorted_xyz, (K*)leaf_key, leaf_begin, status, tile_counter,    \
                     n_out)
  if (packed && key64) FMMDS_LEAF(true, uint64_t);
  else if (packed) FMMDS_LEAF(true, uint32_t);
  else if (key64) FMMDS_LEAF(false, uint64_t);
  else FMMDS_LEAF(false, uint32_t);
#undef FMMDS_LEAF
}

// ---------------------------------------------------------------------------
// Every level at once from the sorted points (the plain build and the
// rebuild): reduce, scan, write. A point e starts a new box at level l iff
// its key and the previous point's key differ above the lowest 3 (L - l)
// bits, i.e. iff l >= d(e), where d(e) = L - (highest differing bit) / 3 (0
// for the first point; L + 1, no new box, for equal keys). So one pass over
// the points has every level's box starts:
//   k_tab_count  per tile of 2048 points and per level, the number of box
//                starts (one ballot per level and item);
//   k_tab_scan   per level, the exclusive scan of those counts over the
//                tiles, and the level's box count;
//   k_tab_write  per point: the permutation, the coordinates, and for every
//                level l >= d(e) the box's key, bookmark (the point itself),
//                parent (the level l - 1 box holding the point) and first
//                child (the level l + 1 box starting at the point);
//   k_tab_masks  per box of levels 0..L-1, the 8-bit mask of its children's
//                octants, from the children's keys.
// The tile prefixes come from the scan, so no kernel waits on another tile.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t new_box_level(uint64_t k, uint64_t kp, uint32_t L) {
  const uint64_t x = k ^ kp;
  if (x == 0) return L + 1;
  const uint32_t m = (63u - (uint32_t)__clzll((long long)x)) / 3u;  // highest differing digit
  return m >= L ? 0u : L - m;
}

template <bool PACKED>
__device__ __forceinline__ uint64_t elem_key(const uint64_t* __restrict__ sk, uint64_t e) {
  return PACKED ? (sk[e] >> 32) : sk[e];
}

template <bool PACKED>
__global__ __launch_bounds__(kCompBlock) void k_tab_count(const uint64_t* __restrict__ sk,
                                                          uint32_t n, uint32_t L, uint32_t tiles,
                                                          uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_c[kMaxLevel + 1][kCompWaves];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint64_t tbase = (uint64_t)blockIdx.x * kCompTile;
  uint32_t d[kCompItems];
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t e = tbase + (uint64_t)i * kCompBlock + tid;
    d[i] = L + 1;
    if (e < n) d[i] = e == 0 ? 0u : new_box_level(elem_key<PACKED>(sk, e), elem_key<PACKED>(sk, e - 1), L);
  }
  for (uint32_t l = 0; l <= L; ++l) {
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kCompItems; ++i) c += (uint32_t)__popcll(__ballot(d[i] <= l));
    if (lane == 0) s_c[l][w] = c;
  }
  __syncthreads();
  if (tid <= L) {
    uint32_t c = 0;
#pragma unroll
    for (int ww = 0; ww < kCompWaves; ++ww) c += s_c[tid][ww];
    cnt[(uint64_t)tid * tiles + blockIdx.x] = c;
  }
}

// One block per level: exclusive scan of the level's tile counts, in chunks
// of 4096, and the level's box count.
constexpr int kTabScanBlock = 1024;
__global__ __launch_bounds__(kTabScanBlock) void k_tab_scan(const uint32_t* __restrict__ cnt,
                                                            uint32_t tiles,
                                                            uint32_t* __restrict__ pre,
                                                            uint32_t* __restrict__ n_boxes) {
  constexpr int W = kTabScanBlock / 64;
  __shared__ uint32_t s_w[W];
  const uint32_t l = blockIdx.x, tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t* c = cnt + (uint64_t)l * tiles;
  uint32_t* o = pre + (uint64_t)l * tiles;
  uint32_t carry = 0;
  for (uint64_t base = 0; base < tiles; base += 4u * kTabScanBlock) {
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t j = base + 4u * tid + i;
      v[i] = j < tiles ? c[j] : 0u;
      sum += v[i];
    }
    const uint32_t inc = wave_incl_scan(sum);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t run = carry + inc - sum, total = 0;
#pragma unroll
    for (int ww = 0; ww < W; ++ww) {
      run += (uint32_t)ww < w ? s_w[ww] : 0u;
      total += s_w[ww];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t j = base + 4u * tid + i;
      if (j < tiles) o[j] = run;
      run += v[i];
    }
    carry += total;
    __syncthreads();
  }
  if (tid == 0) n_boxes[l] = carry;
}

// With a batch (set_off != nullptr) the key carries the set id from bit
// `set_shift` up and the permutation is written relative to the set's first
// point; a set boundary differs in those bits, so it starts a box at every
// level.
template <bool PACKED, typename KeyT>
__global__ __launch_bounds__(kCompBlock) void k_tab_write(
    const uint64_t* __restrict__ sk, const uint32_t* __restrict__ sv, const P3* __restrict__ xyz,
    uint32_t n, uint32_t L, uint32_t tiles, const uint32_t* __restrict__ pre, TabLevels T,
    uint32_t* __restrict__ perm, P3* __restrict__ sorted_xyz,
    const uint64_t* __restrict__ set_off, uint32_t set_shift) {
  constexpr int NSLOT = kCompItems * kCompWaves;
  __shared__ uint32_t s_c[kMaxLevel + 1][NSLOT];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  // Consecutive tiles on one XCD: with a batch each set's coordinate gather
  // then stays within one XCD's L2 (the batched table pass 1550 -> 1094 us for
  // 512 sets); a single set's gather is random over all of it either way.
  const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
  const uint64_t tbase = (uint64_t)tile * kCompTile;
  uint64_t key[kCompItems];
  uint32_t d[kCompItems];
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t e = tbase + (uint64_t)i * kCompBlock + tid;
    d[i] = L + 1;
    key[i] = 0;
    if (e < n) {
      const uint64_t el = sk[e];
      key[i] = PACKED ? (el >> 32) : el;
      d[i] = e == 0 ? 0u : new_box_level(key[i], elem_key<PACKED>(sk, e - 1), L);
      const uint32_t idx = PACKED ? (uint32_t)el : sv[e];
      perm[e] = set_off ? idx - (uint32_t)set_off[key[i] >> set_shift] : idx;
      if (xyz) sorted_xyz[e] = xyz[idx];  // null: the coordinates are already in place
    }
  }
  // per level and (item, wave) slot: the number of box starts
  for (uint32_t l = 0; l <= L; ++l) {
#pragma unroll
    for (int i = 0; i < kCompItems; ++i) {
      const uint64_t b = __ballot(d[i] <= l);
      if (lane == 0) s_c[l][i * kCompWaves + w] = (uint32_t)__popcll(b);
    }
  }
  __syncthreads();
  // slots in point order (item, then wave): exclusive prefixes plus the tile's
  // prefix from the scan, one level per wave at a time
  for (uint32_t l = w; l <= L; l += kCompWaves) {
    const uint32_t v = lane < NSLOT ? s_c[l][lane] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    if (lane < NSLOT) s_c[l][lane] = pre[(uint64_t)l * tiles + tile] + inc - v;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t e = tbase + (uint64_t)i * kCompBlock + tid;
    const uint32_t slot = i * kCompWaves + w;
    // inclusive count of box starts up to this point: at level l - 1 (prev),
    // l (cur) and l + 1 (next)
    auto incl = [&](uint32_t l) {
      const bool f = d[i] <= l;
      return s_c[l][slot] + mbcnt(__ballot(f)) + (f ? 1u : 0u);
    };
    uint32_t prev = 0, cur = incl(0);
    for (uint32_t l = 0; l <= L; ++l) {
      const uint32_t next = l < L ? incl(l + 1) : 0u;
      if (e < n) {
        if (d[i] <= l) {
          const uint32_t r = cur - 1;
          ((KeyT*)T.key[l])[r] = (KeyT)(key[i] >> (3 * (L - l)));
          T.begin[l][r] = (uint32_t)e;
          if (l >= 1) T.parent[l][r] = prev - 1;
          if (l < L) T.child[l][r] = next - 1;
        }
        if (e + 1 == n) {  // sentinels: cur = boxes of level l, next = of level l + 1
          T.begin[l][cur] = n;
          if (l < L) T.child[l][cur] = next;
        }
      }
      prev = cur;
      cur = next;
    }
  }
}

// Child octant masks of every box of levels 0..L-1 (grid y = level).
template <typename KeyT>
__global__ __launch_bounds__(256) void k_tab_masks(TabLevels T, const uint32_t* __restrict__ n_boxes) {
  const uint32_t l = blockIdx.y;
  const uint32_t nl = n_boxes[l];
  const uint32_t* __restrict__ child = T.child[l];
  const KeyT* __restrict__ ck = (const KeyT*)T.key[l + 1];
  uint8_t* __restrict__ mask = T.mask[l];
  for (uint64_t j = blockIdx.x * 256ull + threadIdx.x; j < nl; j += gridDim.x * 256ull) {
    const uint32_t c0 = child[j], c1 = child[j + 1];
    uint32_t m = 0;
    for (uint32_t c = c0; c < c1; ++c) m |= 1u << ((uint32_t)ck[c] & 7u);
    mask[j] = (uint8_t)m;
  }
}

uint32_t tab_tiles(uint32_t n) { return div_up(n, kCompTile); }

void launch_tables(bool packed, bool key64, const uint64_t* sk, const uint32_t* sv,
                   const float* xyz, uint32_t n, uint32_t L, uint32_t* cnt, uint32_t* pre,
                   const TabLevels& T, uint32_t* perm, float* sorted_xyz, uint32_t* n_boxes,
                   uint32_t mask_cap, hipStream_t s, int phase, const uint64_t* set_off,
                   uint32_t set_shift) {
  const uint32_t tiles = tab_tiles(n);
  if (phase == 0) {
    if (packed)
      hipLaunchKernelGGL(k_tab_count<true>, dim3(tiles), dim3(kCompBlock), 0, s, sk, n, L, tiles, cnt);
    else
      hipLaunchKernelGGL(k_tab_count<false>, dim3(tiles), dim3(kCompBlock), 0, s, sk, n, L, tiles, cnt);
  } else if (phase == 1) {
    hipLaunchKernelGGL(k_tab_scan, dim3(L + 1), dim3(kTabScanBlock), 0, s, cnt, tiles, pre, n_boxes);
  } else if (phase == 2) {
#define FMMDS_TABW(P, K)                                                                         \
  hipLaunchKernelGGL((k_tab_write<P, K>), dim3(tiles), dim3(kCompBlock), 0, s, sk, sv,            \
                     (const P3*)xyz, n, L, tiles, pre, T, perm, (P3*)sorted_xyz, set_off,  \
                     set_shift)
    if (packed && key64) FMMDS_TABW(true, uint64_t);
    else if (packed) FMMDS_TABW(true, uint32_t);
    else if (key64) FMMDS_TABW(false, uint64_t);
    else FMMDS_TABW(false, uint32_t);
#undef FMMDS_TABW
  } else if (L > 0) {
    const dim3 grid(std::max<uint32_t>(1, std::min<uint32_t>(div_up(mask_cap, 256), 2048)), L);
    if (key64) hipLaunchKernelGGL(k_tab_masks<uint64_t>, grid, dim3(256), 0, s, T, n_boxes);
    else hipLaunchKernelGGL(k_tab_masks<uint32_t>, grid, dim3(256), 0, s, T, n_boxes);
  }
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
