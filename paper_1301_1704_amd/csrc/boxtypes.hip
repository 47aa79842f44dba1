// Simulated partition and source box types (Section 3).
//
// Partition (Section 3.2): the boxes of the partition level l_par go to the
// ranks in consecutive Morton ranges balanced by receiver points. The
// nonempty receiver box whose first point is the p-th of M (in Morton order;
// p is its bookmark) goes to rank min(R - 1, floor(R p / M)); every other
// Morton index of l_par takes the rank of the nearest nonempty receiver box
// before it (rank 0 if none), so each rank holds one consecutive range.
//
// Box types (Section 3.1, Algorithm 6) for rank J, with l_crit = l_par - 1:
// below l_crit every source box is DOMESTIC. At l_crit a box whose nonempty
// source children (at l_par) are all elsewhere is IMPORT, one with children
// on J and elsewhere is ROOT, and one with all children on J is EXPORT when
// a receiver box with a nonempty receiver child elsewhere has it in its M2L
// list E4, else DOMESTIC. From l_par down a box belongs to the owner of its
// l_par ancestor (its Morton index shifted right, Section 3.2): on J it is
// EXPORT when a receiver box of another rank has it in E4, else DOMESTIC;
// elsewhere it is IMPORT when a receiver box of J has it in E4, else OTHER.
//
// The E4 lists of the build give "r has k in E4(r)" directly, so the marks
// are made by the receivers: a receiver reads its list and marks the source
// boxes it names. A receiver whose whole M2L region lies in l_par boxes of
// its own rank cannot mark anything, nor can a receiver of another rank whose
// region has no box of this rank; only the others are listed and read.
#include "../../include/fmmds.h"
#include "device.h"
#include "internal.h"

namespace fmmds {

constexpr uint32_t kMarkBlocks = 4096;  // step 2: 16384 waves walk the work list

// Coordinate of a Morton index on one axis (bits 3b + axis).
__device__ __forceinline__ uint32_t axis_coord(uint64_t key, int axis) {
  return (uint32_t)compact3(key >> axis);
}

template <typename KeyT>
__global__ __launch_bounds__(256) void k_partition(const KeyT* __restrict__ rkey,
                                                   const uint32_t* __restrict__ rbegin,
                                                   uint32_t n_boxes, uint32_t n_points,
                                                   uint32_t n_ranks, uint64_t n_idx,
                                                   uint32_t* __restrict__ owner) {
  for (uint64_t m = blockIdx.x * 256ull + threadIdx.x; m < n_idx; m += gridDim.x * 256ull) {
    uint32_t lo = 0, hi = n_boxes;  // first box with key > m
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if ((uint64_t)rkey[mid] <= m) lo = mid + 1;
      else hi = mid;
    }
    uint32_t o = 0;
    if (lo > 0) {
      const uint64_t p = rbegin[lo - 1];
      o = (uint32_t)min<uint64_t>(n_ranks - 1, (uint64_t)n_ranks * p / n_points);
    }
    owner[m] = o;
  }
}

__global__ __launch_bounds__(256) void k_fill_u8(uint8_t* __restrict__ p, uint32_t n, uint8_t v) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += gridDim.x * 256ull) p[i] = v;
}

// Marks are bytes in two arrays (needed elsewhere / needed here), set with
// plain stores: every writer stores the same value, so no atomics are needed.
//
// Step 1 (per receiver): does the receiver have to read its E4 list? Those
// that do are appended to a work list (one atomic per wave, at the end).
// Critical level: receivers with a nonempty receiver child on another rank.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_pick_crit(uint32_t n_recv,
                                                   const uint32_t* __restrict__ rchild,
                                                   const KeyT* __restrict__ rkey_par,
                                                   const uint32_t* __restrict__ owner,
                                                   uint32_t rank, uint32_t* __restrict__ work,
                                                   uint32_t* __restrict__ n_work) {
  const uint64_t r = blockIdx.x * 256ull + threadIdx.x;
  bool pick = false;
  if (r < n_recv)
    for (uint32_t c = rchild[r]; c < rchild[r + 1]; ++c)
      pick |= owner[(uint64_t)rkey_par[c]] != rank;
  const uint64_t b = __ballot(pick);
  if (!b) return;
  uint32_t base = 0;
  if ((threadIdx.x & 63u) == 0) base = atomicAdd(n_work, (uint32_t)__popcll(b));
  base = (uint32_t)__builtin_amdgcn_readfirstlane(base);
  if (pick) work[base + mbcnt(b)] = (uint32_t)r;
}

// Levels l >= l_par. The M2L region of r: per axis the level-l coordinates
// 2(p - 1) .. 2(p + 1) + 1 around its parent coordinate p; their l_par
// ancestors are that range shifted right by l - l_par. Marks need a region
// with another rank than r's, and a receiver of another rank marks only boxes
// of `rank`, so its region must also touch `rank`.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_pick_deep(uint32_t n_recv, const KeyT* __restrict__ rkey,
                                                   uint32_t level, uint32_t l_par,
                                                   const uint32_t* __restrict__ owner,
                                                   uint32_t rank, uint32_t* __restrict__ work,
                                                   uint32_t* __restrict__ n_work) {
  const uint64_t r = blockIdx.x * 256ull + threadIdx.x;
  bool pick = false;
  if (r < n_recv) {
    const uint32_t sh = level - l_par;
    const uint64_t kr = (uint64_t)rkey[r];
    const uint32_t o_r = owner[kr >> (3 * sh)];
    const int32_t top = (1 << l_par) - 1;
    int32_t lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      const int32_t p = (int32_t)(axis_coord(kr, d) >> 1);
      lo[d] = max(0, (2 * (p - 1)) >> sh);
      hi[d] = min(top, (2 * (p + 1) + 1) >> sh);
    }
    bool mixed = false, touches = o_r == rank;
    for (int32_t z = lo[2]; z <= hi[2]; ++z)
      for (int32_t y = lo[1]; y <= hi[1]; ++y)
        for (int32_t x = lo[0]; x <= hi[0]; ++x) {
          const uint32_t o = owner[spread3((uint32_t)x) | (spread3((uint32_t)y) << 1) |
                                   (spread3((uint32_t)z) << 2)];
          mixed |= o != o_r;
          touches |= o == rank;
        }
    pick = mixed && touches;
  }
  const uint64_t b = __ballot(pick);
  if (!b) return;
  uint32_t base = 0;
  if ((threadIdx.x & 63u) == 0) base = atomicAdd(n_work, (uint32_t)__popcll(b));
  base = (uint32_t)__builtin_amdgcn_readfirstlane(base);
  if (pick) work[base + mbcnt(b)] = (uint32_t)r;
}

// Step 2: one wave per listed receiver at a time; its E4 entries (at most
// 189) are read three 64-entry chunks at once, every load before any store
// (on this GPU a wait for a load also waits for earlier stores). At the
// critical level (deep == false) every entry is needed elsewhere.
template <typename KeyT, bool DEEP>
__global__ __launch_bounds__(256) void k_mark(const uint32_t* __restrict__ work,
                                              const uint32_t* __restrict__ n_work,
                                              const KeyT* __restrict__ rkey,
                                              const KeyT* __restrict__ skey, uint32_t sh,
                                              const uint32_t* __restrict__ owner, uint32_t rank,
                                              const uint32_t* __restrict__ e4_off,
                                              const uint32_t* __restrict__ e4_ent,
                                              uint8_t* __restrict__ elsewhere,
                                              uint8_t* __restrict__ here) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n = *n_work;
  const uint32_t n_waves = gridDim.x * 4;
  for (uint32_t w = blockIdx.x * 4 + (threadIdx.x >> 6); w < n; w += n_waves) {
    const uint32_t r = work[w];
    const uint32_t lo = e4_off[r], hi = e4_off[r + 1];
    const bool r_here = DEEP ? owner[(uint64_t)rkey[r] >> (3 * sh)] == rank : false;
    uint32_t k[3];
    bool k_here[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint32_t i = lo + 64u * c + lane;
      k[c] = i < hi ? e4_ent[i] : 0xFFFFFFFFu;
    }
    if (DEEP) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        k_here[c] = k[c] != 0xFFFFFFFFu && owner[(uint64_t)skey[k[c]] >> (3 * sh)] == rank;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (k[c] == 0xFFFFFFFFu) continue;
      if (!DEEP) {
        elsewhere[k[c]] = 1;
      } else {
        if (k_here[c] && !r_here) elsewhere[k[c]] = 1;
        if (!k_here[c] && r_here) here[k[c]] = 1;
      }
    }
  }
}

// Critical level, sources: children on this rank and elsewhere.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_types_crit(uint32_t n_src,
                                                    const uint32_t* __restrict__ schild,
                                                    const KeyT* __restrict__ skey_par,
                                                    const uint32_t* __restrict__ owner,
                                                    uint32_t rank,
                                                    const uint8_t* __restrict__ elsewhere,
                                                    uint8_t* __restrict__ types) {
  const uint64_t k = blockIdx.x * 256ull + threadIdx.x;
  if (k >= n_src) return;
  bool on = false, off = false;
  for (uint32_t c = schild[k]; c < schild[k + 1]; ++c) {
    const bool here = owner[(uint64_t)skey_par[c]] == rank;
    on |= here;
    off |= !here;
  }
  uint8_t t;
  if (!on) t = FMMDS_BOX_IMPORT;
  else if (off) t = FMMDS_BOX_ROOT;
  else t = elsewhere[k] ? FMMDS_BOX_EXPORT : FMMDS_BOX_DOMESTIC;
  types[k] = t;
}

template <typename KeyT>
__global__ __launch_bounds__(256) void k_types_deep(uint32_t n_src, const KeyT* __restrict__ skey,
                                                    uint32_t level, uint32_t l_par,
                                                    const uint32_t* __restrict__ owner,
                                                    uint32_t rank,
                                                    const uint8_t* __restrict__ elsewhere,
                                                    const uint8_t* __restrict__ here_mark,
                                                    uint8_t* __restrict__ types) {
  const uint64_t k = blockIdx.x * 256ull + threadIdx.x;
  if (k >= n_src) return;
  const bool here = owner[(uint64_t)skey[k] >> (3 * (level - l_par))] == rank;
  types[k] = here ? (elsewhere[k] ? FMMDS_BOX_EXPORT : FMMDS_BOX_DOMESTIC)
                  : (here_mark[k] ? FMMDS_BOX_IMPORT : FMMDS_BOX_OTHER);
}

static uint32_t grid_for(uint64_t n) {
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 1u << 20));
}

void launch_partition(bool key64, const void* rkey, const uint32_t* rbegin, uint32_t n_boxes,
                      uint32_t n_points, uint32_t n_ranks, uint32_t l_par, uint32_t* owner,
                      hipStream_t s) {
  const uint64_t n_idx = 1ull << (3 * l_par);
  const uint32_t g = (uint32_t)std::min<uint64_t>((n_idx + 255) / 256, 65536);
  if (key64)
    hipLaunchKernelGGL(k_partition<uint64_t>, dim3(g), dim3(256), 0, s, (const uint64_t*)rkey,
                       rbegin, n_boxes, n_points, n_ranks, n_idx, owner);
  else
    hipLaunchKernelGGL(k_partition<uint32_t>, dim3(g), dim3(256), 0, s, (const uint32_t*)rkey,
                       rbegin, n_boxes, n_points, n_ranks, n_idx, owner);
}

void launch_fill_u8(uint8_t* p, uint32_t n, uint8_t v, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_u8, dim3(std::min<uint32_t>(grid_for(n), 4096)), dim3(256), 0, s, p,
                     n, v);
}

template <typename K>
static void types_crit(const BoxTypeLevel& a, hipStream_t s) {
  if (a.n_recv) {
    hipLaunchKernelGGL(k_pick_crit<K>, dim3(grid_for(a.n_recv)), dim3(256), 0, s, a.n_recv,
                       a.rchild, (const K*)a.rkey_par, a.owner, a.rank, a.work, a.n_work);
    hipLaunchKernelGGL((k_mark<K, false>), dim3(kMarkBlocks), dim3(256), 0, s, a.work, a.n_work,
                       (const K*)a.rkey, (const K*)a.skey, 0u, a.owner, a.rank, a.e4_off,
                       a.e4_ent, a.elsewhere, a.here);
  }
  hipLaunchKernelGGL(k_types_crit<K>, dim3(grid_for(a.n_src)), dim3(256), 0, s, a.n_src,
                     a.schild, (const K*)a.skey_par, a.owner, a.rank, a.elsewhere, a.types);
}

template <typename K>
static void types_deep(const BoxTypeLevel& a, hipStream_t s) {
  if (a.n_recv) {
    hipLaunchKernelGGL(k_pick_deep<K>, dim3(grid_for(a.n_recv)), dim3(256), 0, s, a.n_recv,
                       (const K*)a.rkey, a.level, a.l_par, a.owner, a.rank, a.work, a.n_work);
    hipLaunchKernelGGL((k_mark<K, true>), dim3(kMarkBlocks), dim3(256), 0, s, a.work, a.n_work,
                       (const K*)a.rkey, (const K*)a.skey, a.level - a.l_par, a.owner, a.rank,
                       a.e4_off, a.e4_ent, a.elsewhere, a.here);
  }
  hipLaunchKernelGGL(k_types_deep<K>, dim3(grid_for(a.n_src)), dim3(256), 0, s, a.n_src,
                     (const K*)a.skey, a.level, a.l_par, a.owner, a.rank, a.elsewhere, a.here,
                     a.types);
}

void launch_types_crit(bool key64, const BoxTypeLevel& a, hipStream_t s) {
  if (key64) types_crit<uint64_t>(a, s);
  else types_crit<uint32_t>(a, s);
}

void launch_types_deep(bool key64, const BoxTypeLevel& a, hipStream_t s) {
  if (key64) types_deep<uint64_t>(a, s);
  else types_deep<uint32_t>(a, s);
}

}  // namespace fmmds
