// The paper's dense-histogram construction (Sections 2.1-2.3), made
// deterministic: a variant of the build that produces exactly the outputs of
// the sort path, for max levels up to 8 (8^8 boxes per dense array).
//
//   Algorithm 1: every point's finest box, an atomic increment of that box's
//     occupancy counter (Bin) whose old value is the point's provisional rank
//     inside the box.
//   Algorithm 3: per level, one pass over all 8^l boxes scans Bin into the
//     bookmarks (ScannedBin) and the nonempty flags into ScannedRank, and
//     compacts the nonempty boxes (NonEmptyIdx, Bookmark). Coarser levels'
//     counters are sums of eight children.
//   Algorithm 4 and the E4 query: a receiver box's neighbors come from
//     de-interleaved coordinates +-1; a neighbor is looked up directly in the
//     dense source counters, and its list entry is its ScannedRank.
//
// Determinism: the atomic ranks order the points inside a box by timing
// (the paper's pseudo-sort). Each box's points are then put in original
// index order: a thread per box of at most 32 points, a block per box of up
// to 4096 (ranks by counting in LDS). Larger boxes make the runtime sort the
// points instead (the box tables are the same either way).
//
// Lists come out in ascending rank: the receiver's parent's 27 neighbors are
// sorted by Morton index, and walking them in that order, each followed by
// its eight children in octant order, visits the candidate boxes in
// ascending Morton index, hence ascending rank.
#include "device.h"
#include "internal.h"

namespace fmmds {

namespace {

struct P3 {
  float x, y, z;
};

__global__ __launch_bounds__(256) void k_dense_count(const P3* __restrict__ xyz, uint32_t n,
                                                     uint32_t L, uint32_t* __restrict__ bin,
                                                     uint32_t* __restrict__ key_out,
                                                     uint32_t* __restrict__ rank_out,
                                                     uint32_t* __restrict__ err) {
  bool bad = false;
  for (uint64_t j = blockIdx.x * 256ull + threadIdx.x; j < n; j += gridDim.x * 256ull) {
    const P3 p = xyz[j];
    bool ok;
    const uint32_t key = (uint32_t)point_key(p.x, p.y, p.z, L, ok);
    bad |= !ok;
    key_out[j] = key;
    rank_out[j] = atomicAdd(&bin[key], 1u);
  }
  if (bad) atomicOr(err, 1u);
}

__global__ __launch_bounds__(256) void k_dense_reduce(const uint4* __restrict__ fine,
                                                      uint32_t n_coarse,
                                                      uint32_t* __restrict__ coarse) {
  for (uint64_t k = blockIdx.x * 256ull + threadIdx.x; k < n_coarse; k += gridDim.x * 256ull) {
    const uint4 a = fine[2 * k], b = fine[2 * k + 1];
    coarse[k] = a.x + a.y + a.z + a.w + b.x + b.y + b.z + b.w;
  }
}

// Algorithm 3 on one level: tiles of 2048 boxes, 8 consecutive per thread.
// One chained scan carries (points << 25 | nonempty boxes); both fit, with
// at most 2^24 boxes and fewer than 2^32 points.
constexpr uint32_t kDenseItems = 8;
constexpr uint32_t kDenseTile = 256 * kDenseItems;

template <typename KeyT>
__global__ __launch_bounds__(256) void k_dense_scan(
    const uint32_t* __restrict__ bin, uint32_t nbox, uint32_t* __restrict__ sbin,
    uint32_t* __restrict__ srank, KeyT* __restrict__ keys, uint32_t* __restrict__ begin,
    uint32_t* __restrict__ n_out, uint32_t* __restrict__ max_occ, uint64_t* __restrict__ status,
    uint32_t* __restrict__ tile_counter) {
  __shared__ uint64_t s_w[4];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint64_t base = (uint64_t)tile * kDenseTile + (uint64_t)tid * kDenseItems;
  uint32_t c[kDenseItems];
  if (base + kDenseItems <= nbox) {
    const uint4 a = ((const uint4*)(bin + base))[0], b = ((const uint4*)(bin + base))[1];
    c[0] = a.x, c[1] = a.y, c[2] = a.z, c[3] = a.w, c[4] = b.x, c[5] = b.y, c[6] = b.z, c[7] = b.w;
  } else {
#pragma unroll
    for (uint32_t k = 0; k < kDenseItems; ++k) c[k] = base + k < nbox ? bin[base + k] : 0u;
  }
  uint64_t mine = 0;
  uint32_t mx = 0;
#pragma unroll
  for (uint32_t k = 0; k < kDenseItems; ++k) {
    mine += ((uint64_t)c[k] << 25) + (c[k] > 0 ? 1u : 0u);
    mx = max(mx, c[k]);
  }
  // block scan of the packed pairs
  uint64_t inc = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t t = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += t;
  }
  if (lane == 63) s_w[w] = inc;
  mx = wave_max(mx);
  if (lane == 0 && mx) atomicMax(max_occ, mx);
  __syncthreads();
  uint64_t wpre = 0, tot = 0;
#pragma unroll
  for (uint32_t i = 0; i < 4; ++i) {
    if (i < w) wpre += s_w[i];
    tot += s_w[i];
  }
  if (w == 0) {
    const uint64_t ex = lookback_wave(status, tile, tot);
    if (lane == 0) s_excl = ex;
  }
  __syncthreads();
  uint64_t run = s_excl + wpre + inc - mine;  // exclusive, packed
  uint32_t sp[kDenseItems], sr[kDenseItems];
#pragma unroll
  for (uint32_t k = 0; k < kDenseItems; ++k) {
    sp[k] = (uint32_t)(run >> 25);
    sr[k] = (uint32_t)(run & ((1u << 25) - 1));
    run += ((uint64_t)c[k] << 25) + (c[k] > 0 ? 1u : 0u);
  }
  if (base + kDenseItems <= nbox) {
    ((uint4*)(sbin + base))[0] = make_uint4(sp[0], sp[1], sp[2], sp[3]);
    ((uint4*)(sbin + base))[1] = make_uint4(sp[4], sp[5], sp[6], sp[7]);
    ((uint4*)(srank + base))[0] = make_uint4(sr[0], sr[1], sr[2], sr[3]);
    ((uint4*)(srank + base))[1] = make_uint4(sr[4], sr[5], sr[6], sr[7]);
  } else {
#pragma unroll
    for (uint32_t k = 0; k < kDenseItems; ++k)
      if (base + k < nbox) sbin[base + k] = sp[k], srank[base + k] = sr[k];
  }
#pragma unroll
  for (uint32_t k = 0; k < kDenseItems; ++k) {
    if (c[k] > 0) {
      keys[sr[k]] = (KeyT)(base + k);
      begin[sr[k]] = sp[k];
    }
    if (base + k + 1 == nbox) {
      begin[sr[k] + (c[k] > 0 ? 1u : 0u)] = sp[k] + c[k];
      *n_out = sr[k] + (c[k] > 0 ? 1u : 0u);
    }
  }
}

// Children of the nonempty boxes of a level (first child's rank, octant
// mask) from the next level's dense arrays; child[n] = boxes of the next level.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_dense_child(const KeyT* __restrict__ keys,
                                                     const uint32_t* __restrict__ n_p,
                                                     const uint32_t* __restrict__ bin_fine,
                                                     const uint32_t* __restrict__ srank_fine,
                                                     const uint32_t* __restrict__ n_fine_p,
                                                     uint32_t* __restrict__ child,
                                                     uint8_t* __restrict__ mask) {
  const uint32_t n = *n_p;
  for (uint64_t b = blockIdx.x * 256ull + threadIdx.x; b <= n; b += gridDim.x * 256ull) {
    if (b == n) {
      child[n] = *n_fine_p;
      continue;
    }
    const uint64_t k8 = (uint64_t)keys[b] << 3;
    const uint4 a = ((const uint4*)(bin_fine + k8))[0], c = ((const uint4*)(bin_fine + k8))[1];
    const uint32_t m = (a.x > 0) | (a.y > 0) << 1 | (a.z > 0) << 2 | (a.w > 0) << 3 |
                       (c.x > 0) << 4 | (c.y > 0) << 5 | (c.z > 0) << 6 | (c.w > 0) << 7;
    child[b] = srank_fine[k8];
    mask[b] = (uint8_t)m;
  }
}

template <typename KeyT>
__global__ __launch_bounds__(256) void k_dense_parent(const KeyT* __restrict__ keys,
                                                      const uint32_t* __restrict__ n_p,
                                                      const uint32_t* __restrict__ srank_coarse,
                                                      uint32_t* __restrict__ parent) {
  const uint32_t n = *n_p;
  for (uint64_t b = blockIdx.x * 256ull + threadIdx.x; b < n; b += gridDim.x * 256ull)
    parent[b] = srank_coarse[(uint64_t)keys[b] >> 3];
}

__global__ __launch_bounds__(256) void k_dense_scatter(const uint32_t* __restrict__ key,
                                                       const uint32_t* __restrict__ rank,
                                                       uint32_t n, const uint32_t* __restrict__ sbin,
                                                       uint32_t* __restrict__ tmp) {
  for (uint64_t j = blockIdx.x * 256ull + threadIdx.x; j < n; j += gridDim.x * 256ull)
    tmp[sbin[key[j]] + rank[j]] = (uint32_t)j;
}

// Original index order inside each finest box. Boxes of up to 32 points: a
// thread each, every point's rank counted over the box; larger boxes are
// listed for k_dense_canon_block.
constexpr uint32_t kCanonThread = 32;
constexpr uint32_t kCanonBlock = 4096;

__global__ __launch_bounds__(256) void k_dense_canon(const uint32_t* __restrict__ begin,
                                                     const uint32_t* __restrict__ n_p,
                                                     const uint32_t* __restrict__ tmp,
                                                     uint32_t* __restrict__ perm,
                                                     uint32_t* __restrict__ big,
                                                     uint32_t* __restrict__ n_big) {
  const uint32_t n = *n_p;
  for (uint64_t b = blockIdx.x * 256ull + threadIdx.x; b < n; b += gridDim.x * 256ull) {
    const uint32_t b0 = begin[b], c = begin[b + 1] - b0;
    if (c > kCanonThread) {
      big[atomicAdd(n_big, 1u)] = (uint32_t)b;
      continue;
    }
    for (uint32_t i = 0; i < c; ++i) {
      const uint32_t v = tmp[b0 + i];
      uint32_t r = 0;
      for (uint32_t k = 0; k < c; ++k) r += tmp[b0 + k] < v ? 1u : 0u;
      perm[b0 + r] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_dense_canon_block(const uint32_t* __restrict__ begin,
                                                           const uint32_t* __restrict__ big,
                                                           const uint32_t* __restrict__ n_big,
                                                           const uint32_t* __restrict__ tmp,
                                                           uint32_t* __restrict__ perm) {
  __shared__ uint32_t s_v[kCanonBlock];
  const uint32_t nb = *n_big;
  for (uint32_t q = blockIdx.x; q < nb; q += gridDim.x) {
    const uint32_t b = big[q];
    const uint32_t b0 = begin[b], c = begin[b + 1] - b0;  // <= kCanonBlock (checked by the host)
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < c; i += 256) s_v[i] = tmp[b0 + i];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < c; i += 256) {
      const uint32_t v = s_v[i];
      uint32_t r = 0;
      for (uint32_t k = 0; k < c; ++k) r += s_v[k] < v ? 1u : 0u;
      perm[b0 + r] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_dense_gather(const uint32_t* __restrict__ perm,
                                                      uint32_t n, const P3* __restrict__ xyz,
                                                      P3* __restrict__ out) {
  for (uint64_t e = blockIdx.x * 256ull + threadIdx.x; e < n; e += gridDim.x * 256ull)
    out[e] = xyz[perm[e]];
}

// Lists of the receiver boxes of level l (2 <= l <= 8), a thread per box:
// count (FILL false) or write (FILL true) the E2 and E4 entries.
template <typename KeyT, bool FILL>
__global__ __launch_bounds__(256) void k_dense_lists(
    uint32_t l, uint32_t n_recv, const KeyT* __restrict__ rkeys,
    const uint32_t* __restrict__ bin_up, const uint32_t* __restrict__ bin_cur,
    const uint32_t* __restrict__ srank_cur, uint32_t* __restrict__ cnt2,
    uint32_t* __restrict__ cnt4, const uint32_t* __restrict__ off2,
    const uint32_t* __restrict__ off4, uint32_t* __restrict__ ent2, uint32_t* __restrict__ ent4) {
  const uint64_t b = blockIdx.x * 256ull + threadIdx.x;
  if (b >= n_recv) return;
  const uint32_t key = (uint32_t)rkeys[b];
  const int x = (int)compact3(key), y = (int)compact3(key >> 1), z = (int)compact3(key >> 2);
  const int side_up = 1 << (l - 1);
  // The parent's neighbors at level l - 1, sorted by Morton index (absent
  // ones as 0xFFFFFFFF, sorted last).
  uint32_t nk[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    const int px = (x >> 1) + t % 3 - 1, py = (y >> 1) + (t / 3) % 3 - 1, pz = (z >> 1) + t / 9 - 1;
    const bool in = px >= 0 && py >= 0 && pz >= 0 && px < side_up && py < side_up && pz < side_up;
    nk[t] = in ? (spread3_10((uint32_t)px) | spread3_10((uint32_t)py) << 1 |
                  spread3_10((uint32_t)pz) << 2)
               : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int i = 0; i < 26; ++i)
#pragma unroll
    for (int t = 0; t < 26 - i; ++t) {
      const uint32_t a = nk[t], c = nk[t + 1];
      nk[t] = min(a, c);
      nk[t + 1] = max(a, c);
    }
  uint32_t n2 = 0, n4 = 0;
  uint32_t p2 = FILL ? off2[b] : 0, p4 = FILL ? off4[b] : 0;
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    const uint32_t s = nk[t];
    if (s == 0xFFFFFFFFu || bin_up[s] == 0) continue;
    const int sx = (int)compact3(s), sy = (int)compact3(s >> 1), sz = (int)compact3(s >> 2);
    const uint64_t c8 = (uint64_t)s << 3;
    const uint4 lo = ((const uint4*)(bin_cur + c8))[0], hi = ((const uint4*)(bin_cur + c8))[1];
    const uint32_t occ[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      if (occ[o] == 0) continue;
      const int dx = 2 * sx + (o & 1) - x, dy = 2 * sy + ((o >> 1) & 1) - y,
                dz = 2 * sz + ((o >> 2) & 1) - z;
      const bool near = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
      if (FILL) {
        const uint32_t r = srank_cur[c8 + o];
        if (near) ent2[p2++] = r;
        else ent4[p4++] = r;
      } else {
        n2 += near ? 1u : 0u;
        n4 += near ? 0u : 1u;
      }
    }
  }
  if (!FILL) {
    cnt2[b] = n2;
    cnt4[b] = n4;
  }
}

inline uint32_t grid_for(uint64_t n) { return (uint32_t)std::min<uint64_t>(div_up(n, 256), 8192); }

}  // namespace

void launch_dense_count(const float* xyz, uint32_t n, uint32_t L, uint32_t* bin, uint32_t* key,
                        uint32_t* rank, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_count, dim3(grid_for(n)), dim3(256), 0, s, (const P3*)xyz, n, L, bin,
                     key, rank, err);
}

void launch_dense_reduce(const uint32_t* fine, uint32_t n_coarse, uint32_t* coarse,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_dense_reduce, dim3(grid_for(n_coarse)), dim3(256), 0, s,
                     (const uint4*)fine, n_coarse, coarse);
}

uint32_t dense_scan_tiles(uint32_t nbox) { return div_up(nbox, kDenseTile); }

void launch_dense_scan(bool key64, const uint32_t* bin, uint32_t nbox, uint32_t* sbin,
                       uint32_t* srank, void* keys, uint32_t* begin, uint32_t* n_out,
                       uint32_t* max_occ, uint64_t* status, uint32_t* tile_counter,
                       hipStream_t s) {
  const uint32_t grid = dense_scan_tiles(nbox);
  if (key64)
    hipLaunchKernelGGL(k_dense_scan<uint64_t>, dim3(grid), dim3(256), 0, s, bin, nbox, sbin,
                       srank, (uint64_t*)keys, begin, n_out, max_occ, status, tile_counter);
  else
    hipLaunchKernelGGL(k_dense_scan<uint32_t>, dim3(grid), dim3(256), 0, s, bin, nbox, sbin,
                       srank, (uint32_t*)keys, begin, n_out, max_occ, status, tile_counter);
}

void launch_dense_links(bool key64, const void* keys, const uint32_t* n_p, uint32_t cap,
                        const uint32_t* bin_fine, const uint32_t* srank_fine,
                        const uint32_t* n_fine_p, uint32_t* child, uint8_t* mask,
                        const void* keys_fine, uint32_t cap_fine, uint32_t* parent_fine,
                        const uint32_t* srank, hipStream_t s) {
  if (key64) {
    hipLaunchKernelGGL(k_dense_child<uint64_t>, dim3(grid_for((uint64_t)cap + 1)), dim3(256), 0,
                       s, (const uint64_t*)keys, n_p, bin_fine, srank_fine, n_fine_p, child, mask);
    hipLaunchKernelGGL(k_dense_parent<uint64_t>, dim3(grid_for(cap_fine)), dim3(256), 0, s,
                       (const uint64_t*)keys_fine, n_fine_p, srank, parent_fine);
  } else {
    hipLaunchKernelGGL(k_dense_child<uint32_t>, dim3(grid_for((uint64_t)cap + 1)), dim3(256), 0,
                       s, (const uint32_t*)keys, n_p, bin_fine, srank_fine, n_fine_p, child, mask);
    hipLaunchKernelGGL(k_dense_parent<uint32_t>, dim3(grid_for(cap_fine)), dim3(256), 0, s,
                       (const uint32_t*)keys_fine, n_fine_p, srank, parent_fine);
  }
}

void launch_dense_order(const uint32_t* key, const uint32_t* rank, uint32_t n,
                        const uint32_t* sbin, const uint32_t* begin, const uint32_t* n_boxes,
                        uint32_t cap_boxes, uint32_t* tmp, uint32_t* perm, uint32_t* big,
                        uint32_t* n_big, const float* xyz, float* sorted_xyz, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_scatter, dim3(grid_for(n)), dim3(256), 0, s, key, rank, n, sbin, tmp);
  hipLaunchKernelGGL(k_dense_canon, dim3(grid_for(cap_boxes)), dim3(256), 0, s, begin, n_boxes,
                     tmp, perm, big, n_big);
  hipLaunchKernelGGL(k_dense_canon_block, dim3(2048), dim3(256), 0, s, begin, big, n_big, tmp,
                     perm);
  hipLaunchKernelGGL(k_dense_gather, dim3(grid_for(n)), dim3(256), 0, s, perm, n, (const P3*)xyz,
                     (P3*)sorted_xyz);
}

void launch_dense_lists(bool key64, bool fill, uint32_t l, uint32_t n_recv, const void* rkeys,
                        const uint32_t* bin_up, const uint32_t* bin_cur,
                        const uint32_t* srank_cur, uint32_t* cnt2, uint32_t* cnt4,
                        const uint32_t* off2, const uint32_t* off4, uint32_t* ent2,
                        uint32_t* ent4, hipStream_t s) {
  if (n_recv == 0) return;
  const uint32_t grid = div_up(n_recv, 256);
#define FMMDS_DL(K, F)                                                                         \
  hipLaunchKernelGGL((k_dense_lists<K, F>), dim3(grid), dim3(256), 0, s, l, n_recv,            \
                     (const K*)rkeys, bin_up, bin_cur, srank_cur, cnt2, cnt4, off2, off4, ent2,   \
                     ent4)
  if (key64 && fill) FMMDS_DL(uint64_t, true);
  else if (key64) FMMDS_DL(uint64_t, false);
  else if (fill) FMMDS_DL(uint32_t, true);
  else FMMDS_DL(uint32_t, false);
#undef FMMDS_DL
}

}  // namespace fmmds
