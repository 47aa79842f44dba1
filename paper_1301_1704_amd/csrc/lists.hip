// E2 neighbor lists and E4 (M2L) interaction lists per level.
//
// Definitions (Section 2.4): for a receiver box r at level l, E2(r) holds the
// nonempty source boxes within one box of r in every coordinate (r included);
// E4(r) holds the nonempty source boxes that are children of boxes in
// E2(parent(r)) at level l - 1 but are not in E2(r). The paper enumerates the
// candidate boxes from de-interleaved coordinates (Section 3.3) and looks them
// up in a dense per-box rank array (Algorithm 4).
//
// Here the candidates come from the parent level's E2 list: the children of
// the nonempty source boxes s in E2(parent(r)) are exactly the nonempty
// source boxes of E2(r) and E4(r) together, they sit at consecutive ranks
// child[s] .. child[s] + popcount(mask[s]) - 1 in octant order, and walking
// E2(parent(r)) in ascending rank then the children in octant order yields
// ascending ranks. No search and no dense array are needed. Whether a child
// in octant o of a neighbor at offset (dx, dy, dz) from the parent is within
// one box of r (octant q) is decided per axis:
//   d = 0: always;  d = +1: child bit 0 and r bit 1;  d = -1: child bit 1 and
//   r bit 0;
// giving an 8-bit mask over the child octants.
#include "device.h"
#include "internal.h"

namespace fmmds {

// Octants with the axis bit clear / set: x is bit 0, y bit 1, z bit 2.
__device__ __forceinline__ uint32_t axis_adjacent(int d, uint32_t rbit, uint32_t clear,
                                                  uint32_t set) {
  return d == 0 ? 0xFFu : (d == 1 ? (rbit ? clear : 0u) : (rbit ? 0u : set));
}

template <typename KeyT, int MODE>  // MODE 0: count, 1: fill
__global__ __launch_bounds__(256) void k_lists(
    ListLevelArgs a, uint32_t* __restrict__ cnt2, uint32_t* __restrict__ cnt4,
    const uint32_t* __restrict__ off2, const uint32_t* __restrict__ off4,
    uint32_t* __restrict__ ent2, uint32_t* __restrict__ ent4) {
  const uint64_t r = blockIdx.x * 256ull + threadIdx.x;
  if (r >= a.n_recv) return;
  const KeyT* __restrict__ rkey = (const KeyT*)a.recv_key;
  const KeyT* __restrict__ skey = (const KeyT*)a.src_key_up;
  const uint64_t rk = (uint64_t)rkey[r];
  const uint32_t q = (uint32_t)(rk & 7u);
  const uint64_t pk = rk >> 3;
  const int px = (int)compact3(pk), py = (int)compact3(pk >> 1), pz = (int)compact3(pk >> 2);
  const uint32_t p = a.recv_parent[r];
  uint32_t j0, j1;
  if (a.up_all) {
    j0 = 0;
    j1 = a.n_src_up;
  } else {
    j0 = a.e2_off_up[p];
    j1 = a.e2_off_up[p + 1];
  }
  uint32_t c2 = 0, c4 = 0;
  uint32_t o2 = 0, o4 = 0;
  if (MODE == 1) {
    o2 = off2[r];
    o4 = off4[r];
  }
  for (uint32_t j = j0; j < j1; ++j) {
    const uint32_t s = a.up_all ? j : a.e2_ent_up[j];
    const uint64_t sk = (uint64_t)skey[s];
    const int dx = (int)compact3(sk) - px;
    const int dy = (int)compact3(sk >> 1) - py;
    const int dz = (int)compact3(sk >> 2) - pz;
    const uint32_t m = a.src_mask_up[s];
    const uint32_t adj = axis_adjacent(dx, q & 1u, 0x55u, 0xAAu) &
                         axis_adjacent(dy, (q >> 1) & 1u, 0x33u, 0xCCu) &
                         axis_adjacent(dz, (q >> 2) & 1u, 0x0Fu, 0xF0u);
    if (MODE == 0) {
      c2 += __popc(m & adj);
      c4 += __popc(m & ~adj);
    } else {
      uint32_t rank = a.src_child_up[s];
      uint32_t mm = m;
      while (mm) {
        const uint32_t bit = mm & (0u - mm);
        if (adj & bit) ent2[o2++] = rank;
        else ent4[o4++] = rank;
        ++rank;
        mm ^= bit;
      }
    }
  }
  if (MODE == 0) {
    cnt2[r] = c2;
    cnt4[r] = c4;
  }
}

void launch_list_count(bool key64, const ListLevelArgs& a, uint32_t* cnt2, uint32_t* cnt4,
                       hipStream_t s) {
  if (a.n_recv == 0) return;
  const uint32_t grid = div_up(a.n_recv, 256);
  if (key64)
    hipLaunchKernelGGL((k_lists<uint64_t, 0>), dim3(grid), dim3(256), 0, s, a, cnt2, cnt4, nullptr,
                       nullptr, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_lists<uint32_t, 0>), dim3(grid), dim3(256), 0, s, a, cnt2, cnt4, nullptr,
                       nullptr, nullptr, nullptr);
}

void launch_list_fill(bool key64, const ListLevelArgs& a, const uint32_t* off2,
                      const uint32_t* off4, uint32_t* ent2, uint32_t* ent4, hipStream_t s) {
  if (a.n_recv == 0) return;
  const uint32_t grid = div_up(a.n_recv, 256);
  if (key64)
    hipLaunchKernelGGL((k_lists<uint64_t, 1>), dim3(grid), dim3(256), 0, s, a, nullptr, nullptr,
                       off2, off4, ent2, ent4);
  else
    hipLaunchKernelGGL((k_lists<uint32_t, 1>), dim3(grid), dim3(256), 0, s, a, nullptr, nullptr,
                       off2, off4, ent2, ent4);
}

// ---------------------------------------------------------------------------
// Exclusive scan of per-box list lengths into CSR offsets (the scan that
// turns NumRecvE2NeiNEBox into NeighborBookmark, Algorithm 4), single pass.
// off[n] = total; the total also goes to *total, and the overflow flag is set
// if it does not fit 32-bit offsets.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCompBlock) void k_scan_counts(
    const uint32_t* __restrict__ cnt, uint32_t n, uint32_t* __restrict__ off,
    uint64_t* __restrict__ total, uint32_t* __restrict__ overflow, uint64_t* __restrict__ status,
    uint32_t* __restrict__ tile_counter) {
  __shared__ uint32_t s_w[kCompBlock / 64];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint64_t base = (uint64_t)tile * kCompTile + (uint64_t)tid * kCompItems;
  uint32_t v[kCompItems];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    v[i] = base + i < n ? cnt[base + i] : 0;
    sum += v[i];
  }
  const uint32_t inc = wave_incl_scan(sum);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t wpre = 0, ttot = 0;
  for (uint32_t i = 0; i < kCompBlock / 64; ++i) {
    if (i < w) wpre += s_w[i];
    ttot += s_w[i];
  }
  if (tid == 0) s_excl = lookback(status, 1, tile, ttot);
  __syncthreads();
  uint64_t pre = s_excl + wpre + inc - sum;
  bool ovf = false;
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    if (base + i < n) {
      off[base + i] = (uint32_t)pre;
      ovf |= pre > 0xFFFFFFFFull;
      pre += v[i];
      if (base + i + 1 == n) {
        off[n] = (uint32_t)pre;
        *total = pre;
        ovf |= pre > 0xFFFFFFFFull;
      }
    }
  }
  if (ovf) atomicOr(overflow, 1u);
}

void launch_scan_counts(const uint32_t* cnt, uint32_t n, uint32_t* off, uint64_t* total,
                        uint32_t* overflow, uint64_t* status, uint32_t* tile_counter,
                        hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_scan_counts, dim3(div_up(n, kCompTile)), dim3(kCompBlock), 0, s, cnt, n,
                     off, total, overflow, status, tile_counter);
}

}  // namespace fmmds
