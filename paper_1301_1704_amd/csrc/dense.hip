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
// ordered by Morton index, and taking them in that order, each followed by
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
  __shared__ uint32_t s_mx[4];
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
  if (lane == 0) s_mx[w] = mx;
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
  // The level's largest occupancy: one atomic per block, after the look-back.
  // Atomics on one address are serialized, and on this GPU the look-back's
  // waits for its loads would also wait for an atomic issued before them.
  if (tid == 0) {
    const uint32_t m = max(max(s_mx[0], s_mx[1]), max(s_mx[2], s_mx[3]));
    if (m) atomicMax(max_occ, m);
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

// Lists of the receiver boxes of level l (2 <= l <= 8). One half-wave per
// receiver parent p at level l - 1: lane t < 27 takes p's neighbor at offset
// (t % 3 - 1, t / 3 % 3 - 1, t / 9 - 1), keeps it if the dense source counter
// of level l - 1 says it is nonempty, and reads its eight child counters at
// level l (the first child's rank is the dense ScannedRank there). Ordering
// the kept neighbors by Morton index and their children by octant gives the
// union U of the candidates in ascending rank. Counting: for each receiver
// child of p, its E2 count is the number of U entries within one box, and
// E4 the rest. Filling: U goes to LDS with, per entry, the mask of receiver
// octants it is adjacent to, and the whole wave splits U per receiver child
// with one ballot per 64 entries (E2 lanes to the E2 list, the others to
// the E4 list), two parents per wave.
struct DenseListArgs {
  uint32_t l, n_up;          // level; receiver boxes of level l - 1 (the parents)
  const void* rkey_up;       // their keys
  const uint8_t* rmask_up;   // their receiver child masks
  const uint32_t* rchild_up; // their first receiver children
  const uint32_t* bin_up;    // dense source counters, level l - 1
  const uint32_t* bin_cur;   // dense source counters, level l
  const uint32_t* srank_cur; // dense exclusive source ranks, level l
};

// One half-wave: the kept neighbor of lane t (its key, child mask, first
// child rank, axis offsets) and its position and offset in U.
struct Neighbor {
  uint32_t m, cb, upos, total;
  int dx, dy, dz;
};

template <typename KeyT>
__device__ __forceinline__ Neighbor dense_neighbor(const DenseListArgs& a, uint64_t p, bool live,
                                                   uint32_t j) {
  Neighbor nb{};
  uint32_t key = 0xFFFFFFFFu;
  bool keep = false;
  if (live && j < 27) {
    const uint32_t pk = (uint32_t)((const KeyT*)a.rkey_up)[p];
    const int side = 1 << (a.l - 1);
    nb.dx = (int)(j % 3) - 1, nb.dy = (int)(j / 3 % 3) - 1, nb.dz = (int)(j / 9) - 1;
    const int x = (int)compact3(pk) + nb.dx, y = (int)compact3(pk >> 1) + nb.dy,
              z = (int)compact3(pk >> 2) + nb.dz;
    if (x >= 0 && y >= 0 && z >= 0 && x < side && y < side && z < side) {
      key = spread3_10((uint32_t)x) | spread3_10((uint32_t)y) << 1 | spread3_10((uint32_t)z) << 2;
      keep = a.bin_up[key] > 0;
    }
  }
  if (keep) {
    const uint64_t c8 = (uint64_t)key << 3;
    const uint4 lo = ((const uint4*)(a.bin_cur + c8))[0], hi = ((const uint4*)(a.bin_cur + c8))[1];
    nb.m = (lo.x > 0) | (lo.y > 0) << 1 | (lo.z > 0) << 2 | (lo.w > 0) << 3 | (hi.x > 0) << 4 |
           (hi.y > 0) << 5 | (hi.z > 0) << 6 | (hi.w > 0) << 7;
    nb.cb = a.srank_cur[c8];
  }
  if (!keep) key = 0xFFFFFFFFu;
  // position in Morton order among the kept neighbors, and offset in U
  const uint32_t c = (uint32_t)__popc(nb.m);
  uint32_t upos = 0, total = 0;
#pragma unroll 1
  for (uint32_t i = 0; i < 27; ++i) {
    const uint32_t ki = (uint32_t)__shfl(key, (int)i, 32), ci = (uint32_t)__shfl(c, (int)i, 32);
    upos += ki < key ? ci : 0u;
    total += ci;
  }
  nb.upos = upos;
  nb.total = total;
  return nb;
}

template <typename KeyT>
__global__ __launch_bounds__(256) void k_dense_pcount(DenseListArgs a, uint32_t* __restrict__ cnt2,
                                                      uint32_t* __restrict__ cnt4) {
  const uint32_t j = threadIdx.x & 31u, h = threadIdx.x >> 5;
  const uint64_t p = (uint64_t)blockIdx.x * 8 + h;
  if (p >= a.n_up) return;  // whole half-wave
  const Neighbor nb = dense_neighbor<KeyT>(a, p, true, j);
  // Children of the neighbor adjacent to a receiver child whose axis bit is
  // 0 / 1 (offset 0: all; +1: child bit 0 next to receiver bit 1; -1: the
  // mirror); per receiver octant q the number of them, packed 6 bits each.
  const uint32_t ax0 = nb.dx == 0 ? 0xFFu : (nb.dx < 0 ? 0xAAu : 0u);
  const uint32_t ax1 = nb.dx == 0 ? 0xFFu : (nb.dx > 0 ? 0x55u : 0u);
  const uint32_t ay0 = nb.dy == 0 ? 0xFFu : (nb.dy < 0 ? 0xCCu : 0u);
  const uint32_t ay1 = nb.dy == 0 ? 0xFFu : (nb.dy > 0 ? 0x33u : 0u);
  const uint32_t az0 = nb.dz == 0 ? 0xFFu : (nb.dz < 0 ? 0xF0u : 0u);
  const uint32_t az1 = nb.dz == 0 ? 0xFFu : (nb.dz > 0 ? 0x0Fu : 0u);
  uint32_t wa = 0, wb = 0;
#pragma unroll
  for (uint32_t q = 0; q < 8; ++q) {
    const uint32_t adj = ((q & 1u) ? ax1 : ax0) & ((q & 2u) ? ay1 : ay0) & ((q & 4u) ? az1 : az0);
    const uint32_t c2 = (uint32_t)__popc(nb.m & adj);
    if (q < 4) wa |= c2 << (6 * q);
    else wb |= c2 << (6 * (q - 4));
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) {
    wa += (uint32_t)__shfl_xor(wa, o, 32);
    wb += (uint32_t)__shfl_xor(wb, o, 32);
  }
  const uint32_t rmask = a.rmask_up[p], rfirst = a.rchild_up[p];
  if (j < (uint32_t)__popc(rmask)) {
    uint32_t mm = rmask;
    for (uint32_t t = 0; t < j; ++t) mm &= mm - 1;
    const uint32_t q = (uint32_t)__builtin_ctz(mm);
    const uint32_t n2 = q < 4 ? (wa >> (6 * q)) & 63u : (wb >> (6 * (q - 4))) & 63u;
    cnt2[rfirst + j] = n2;
    cnt4[rfirst + j] = nb.total - n2;
  }
}

template <typename KeyT>
__global__ __launch_bounds__(256) void k_dense_pfill(DenseListArgs a,
                                                     const uint32_t* __restrict__ off2,
                                                     const uint32_t* __restrict__ off4,
                                                     uint32_t* __restrict__ ent2,
                                                     uint32_t* __restrict__ ent4) {
  __shared__ uint32_t s_rank[8][256];
  __shared__ uint8_t s_adj[8][256];
  const uint32_t lane = threadIdx.x & 63u, j = lane & 31u, h = threadIdx.x >> 5;
  const uint64_t p = (uint64_t)blockIdx.x * 8 + h;
  if ((uint64_t)blockIdx.x * 8 + (h & ~1u) >= a.n_up) return;  // whole wave
  const bool live = p < a.n_up;
  uint32_t rmask = 0, rfirst = 0;
  if (live) {
    rmask = a.rmask_up[p];
    rfirst = a.rchild_up[p];
  }
  uint32_t my_o2 = 0, my_o4 = 0;  // lane j: list offsets of receiver child j
  if (j < (uint32_t)__popc(rmask)) {
    my_o2 = off2[rfirst + j];
    my_o4 = off4[rfirst + j];
  }
  const Neighbor nb = dense_neighbor<KeyT>(a, p, live, j);
  {
    // receiver octants a child with axis bit 0 / 1 is adjacent to (receivers
    // with the x / y / z bit set: 0xAA / 0xCC / 0xF0)
    const uint32_t xm0 = nb.dx == 0 ? 0xFFu : (nb.dx > 0 ? 0xAAu : 0u);
    const uint32_t xm1 = nb.dx == 0 ? 0xFFu : (nb.dx < 0 ? 0x55u : 0u);
    const uint32_t ym0 = nb.dy == 0 ? 0xFFu : (nb.dy > 0 ? 0xCCu : 0u);
    const uint32_t ym1 = nb.dy == 0 ? 0xFFu : (nb.dy < 0 ? 0x33u : 0u);
    const uint32_t zm0 = nb.dz == 0 ? 0xFFu : (nb.dz > 0 ? 0xF0u : 0u);
    const uint32_t zm1 = nb.dz == 0 ? 0xFFu : (nb.dz < 0 ? 0x0Fu : 0u);
#pragma unroll
    for (uint32_t o = 0; o < 8; ++o) {
      if (nb.m & (1u << o)) {
        const uint32_t r = (uint32_t)__popc(nb.m & ((1u << o) - 1u));
        s_rank[h][nb.upos + r] = nb.cb + r;
        s_adj[h][nb.upos + r] = (uint8_t)(((o & 1u) ? xm1 : xm0) & ((o & 2u) ? ym1 : ym0) &
                                          ((o & 4u) ? zm1 : zm0));
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  uint32_t u[2][4], ad[2], T[2];
#pragma unroll
  for (uint32_t hh = 0; hh < 2; ++hh) {
    T[hh] = (uint32_t)__builtin_amdgcn_readlane(nb.total, 32 * hh);
    ad[hh] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t idx = 64u * k + lane;
      u[hh][k] = idx < T[hh] ? s_rank[(h & ~1u) + hh][idx] : 0u;
      ad[hh] |= (idx < T[hh] ? (uint32_t)s_adj[(h & ~1u) + hh][idx] : 0u) << (8 * k);
    }
  }
#pragma unroll
  for (uint32_t hh = 0; hh < 2; ++hh) {
    const uint32_t n_chunks = (T[hh] + 63u) >> 6;
    uint32_t qm = (uint32_t)__builtin_amdgcn_readlane(rmask, 32 * hh), child = 32 * hh;
#pragma unroll 1
    while (qm) {
      const uint32_t q = __builtin_ctz(qm);
      qm &= qm - 1;
      uint32_t* d2 = ent2 + (uint32_t)__builtin_amdgcn_readlane(my_o2, child);
      uint32_t* d4 = ent4 + (uint32_t)__builtin_amdgcn_readlane(my_o4, child);
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        if (k < n_chunks) {
          const uint32_t rem = T[hh] - 64u * k;
          const bool is2 = (ad[hh] >> (8 * k + q)) & 1u;
          const uint64_t b2 = __ballot(is2);
          const uint32_t i2 = mbcnt(b2);
          uint32_t* dst = is2 ? d2 + i2 : d4 + (lane - i2);
          if (lane < rem) *dst = u[hh][k];
          const uint32_t n2 = (uint32_t)__popcll(b2);
          d2 += n2;
          d4 += min(rem, 64u) - n2;
        }
      }
      ++child;
    }
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

void launch_dense_lists(bool key64, bool fill, uint32_t l, uint32_t n_up, const void* rkey_up,
                        const uint8_t* rmask_up, const uint32_t* rchild_up,
                        const uint32_t* bin_up, const uint32_t* bin_cur,
                        const uint32_t* srank_cur, uint32_t* cnt2, uint32_t* cnt4,
                        const uint32_t* off2, const uint32_t* off4, uint32_t* ent2,
                        uint32_t* ent4, hipStream_t s) {
  if (n_up == 0) return;
  const DenseListArgs a{l, n_up, rkey_up, rmask_up, rchild_up, bin_up, bin_cur, srank_cur};
  const uint32_t grid = div_up(n_up, 8);
  if (fill) {
    if (key64)
      hipLaunchKernelGGL(k_dense_pfill<uint64_t>, dim3(grid), dim3(256), 0, s, a, off2, off4,
                         ent2, ent4);
    else
      hipLaunchKernelGGL(k_dense_pfill<uint32_t>, dim3(grid), dim3(256), 0, s, a, off2, off4,
                         ent2, ent4);
  } else {
    if (key64)
      hipLaunchKernelGGL(k_dense_pcount<uint64_t>, dim3(grid), dim3(256), 0, s, a, cnt2, cnt4);
    else
      hipLaunchKernelGGL(k_dense_pcount<uint32_t>, dim3(grid), dim3(256), 0, s, a, cnt2, cnt4);
  }
}

}  // namespace fmmds
