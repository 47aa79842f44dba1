// Incremental rebuild for moved points.
//
// The paper motivates the data structures for dynamic problems, where the
// points move between time steps and everything is rebuilt each step
// (Section 1; the pseudo-sort of Section 2.1 reorders all points every time).
// When the points moved only a little, the order of the previous build is
// almost right: most points are still in the same finest-level box.
//
// Reusing the previous permutation: take the points in the previous sorted
// order (slot k holds original point perm_old[k]); a point whose finest box
// did not change is a "stayer". Stayers are still in (key, original index)
// order among themselves, because the old order was sorted by that pair and
// their keys are unchanged. Only the other points ("movers") need sorting;
// then one merge of the two sorted sequences gives the same order a full
// sort gives, and the rest of the build (box tables, hierarchy, lists) runs
// unchanged on it.
//
// The merge works on one 64-bit value per point, (key << ib) | index with ib
// index bits, so that equal keys are ordered by index; a rebuild needs
// 3 L + ib <= 64 (the runtime falls back to the full sort otherwise).
#include "device.h"
#include "internal.h"

namespace fmmds {

namespace {

struct P3 {
  float x, y, z;
};

constexpr int kClsWaves = kCompBlock / 64;

// Classification: tiles of kCompTile slots in slot order (the new positions
// are given in the previous sorted order); a stayer goes to the stayer list
// at its rank among stayers, a mover to the mover list at its rank among
// movers (slot minus stayers before it); both lists keep slot order. One
// chained scan over the tiles counts the stayers. The digit histograms of
// the movers' merge values feed their sort.
__global__ __launch_bounds__(kCompBlock) void k_inc_classify(
    const P3* __restrict__ xyz, const P3* __restrict__ old_xyz, const uint32_t* __restrict__ old_perm,
    uint32_t n, uint32_t L, uint32_t ib, uint32_t n_pass, uint64_t* __restrict__ st_v,
    uint32_t* __restrict__ st_slot, uint64_t* __restrict__ mv_v, uint32_t* __restrict__ mv_slot,
    uint32_t* __restrict__ hist, uint32_t* __restrict__ err, uint64_t* __restrict__ status,
    uint32_t* __restrict__ tile_counter, uint32_t* __restrict__ counts) {
  __shared__ uint32_t s_cnt[kCompItems * kClsWaves];
  __shared__ uint32_t s_hist[kMaxPasses * 256];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, w = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  for (uint32_t i = tid; i < n_pass * 256; i += kCompBlock) s_hist[i] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint64_t tbase = (uint64_t)tile * kCompTile;

  // Loads (indices clamped into range), all before any store.
  uint32_t idx[kCompItems];
  P3 po[kCompItems], pn[kCompItems];
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t ec = min<uint64_t>(tbase + (uint64_t)i * kCompBlock + tid, n - 1);
    idx[i] = old_perm[ec];
    po[i] = old_xyz[ec];
    pn[i] = xyz[ec];
  }
  uint64_t v[kCompItems];
  uint32_t incl[kCompItems];
  uint32_t stay = 0;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t e = tbase + (uint64_t)i * kCompBlock + tid;
    const bool valid = e < n;
    bool ok, ok_old;
    const uint64_t kn = point_key(pn[i].x, pn[i].y, pn[i].z, L, ok);
    const uint64_t ko = point_key(po[i].x, po[i].y, po[i].z, L, ok_old);
    bad |= valid && !ok;
    const bool f = valid && kn == ko;
    v[i] = (kn << ib) | idx[i];
    const uint64_t ball = __ballot(f);
    incl[i] = mbcnt(ball) + (f ? 1u : 0u);
    stay |= (f ? 1u : 0u) << i;
    if ((tid & 63) == 0) s_cnt[i * kClsWaves + w] = (uint32_t)__popcll(ball);
    if (valid && !f)
      for (uint32_t p = 0; p < n_pass; ++p) atomicAdd(&s_hist[p * 256 + ((v[i] >> (8 * p)) & 0xFFu)], 1u);
  }
  if (bad) atomicOr(err, 1u);
  const uint64_t texcl = tile_flags_prefix<kCompItems * kClsWaves>(s_cnt, &s_excl, status, tile);
#pragma unroll
  for (int i = 0; i < kCompItems; ++i) {
    const uint64_t e = tbase + (uint64_t)i * kCompBlock + tid;
    if (e >= n) continue;
    const uint64_t st_incl = texcl + s_cnt[i * kClsWaves + w] + incl[i];  // stayers in [0, e]
    if ((stay >> i) & 1u) {
      st_v[st_incl - 1] = v[i];
      st_slot[st_incl - 1] = (uint32_t)e;
    } else {
      const uint64_t m = e - st_incl;  // movers before e
      mv_v[m] = v[i];
      mv_slot[m] = (uint32_t)e;
    }
    if (e + 1 == n) {
      counts[0] = (uint32_t)st_incl;
      counts[1] = (uint32_t)(n - st_incl);
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < n_pass * 256; i += kCompBlock)
    if (s_hist[i]) atomicAdd(&hist[i], s_hist[i]);
}

// Number of entries of the ascending array a[0..n) below x.
__device__ __forceinline__ uint32_t count_below(const uint64_t* __restrict__ a, uint32_t n,
                                                uint64_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The same count by a whole wave (x the same on every lane): 64 probes per
// round, so about log64(n) rounds of dependent loads instead of log2(n).
__device__ __forceinline__ uint32_t wave_count_below(const uint64_t* __restrict__ a, uint32_t n,
                                                     uint64_t x) {
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t lo = 0, hi = n;  // the count lies in [lo, hi]
  while (hi > lo) {
    const uint32_t step = hi - lo <= 64 ? 1u : (hi - lo + 63) / 64;
    const uint64_t p = lo + (uint64_t)lane * step;
    const bool below = p < hi && a[p] < x;
    const uint32_t c = (uint32_t)__popcll(__ballot(below));  // probes below x: a prefix
    if (step == 1) return lo + c;
    if (c == 0) return lo;
    const uint32_t nlo = lo + (c - 1) * step + 1;
    hi = (uint32_t)min<uint64_t>(hi, lo + (uint64_t)c * step);
    lo = nlo;
  }
  return lo;
}

// Merge: entry i of one sorted list goes to i plus the number of entries of
// the other list below it (all merge values are distinct). Writes the sorted
// pairs in the layout the box-table kernel reads, and the point coordinates
// (xyz here is indexed by slot) in their final order.
template <bool PACKED>
__device__ __forceinline__ void place_one(uint64_t x, uint32_t s, uint64_t pos, uint32_t ib,
                                          const P3* __restrict__ xyz, uint64_t* __restrict__ sk,
                                          uint32_t* __restrict__ sv, P3* __restrict__ sorted_xyz) {
  const uint32_t j = (uint32_t)(x & ((1ull << ib) - 1));
  const P3 p = xyz[s];
  const uint64_t key = x >> ib;
  if (PACKED) {
    sk[pos] = (key << 32) | j;
  } else {
    sk[pos] = key;
    sv[pos] = j;
  }
  sorted_xyz[pos] = p;
}

// Movers against a whole stayer list, a binary search each (the runtime
// uses it when no point stayed: the sorted movers are then the order).
template <bool PACKED>
__global__ __launch_bounds__(256) void k_inc_place_movers(
    const uint64_t* __restrict__ v, const uint32_t* __restrict__ slot, uint32_t cnt,
    const uint64_t* __restrict__ other, uint32_t ocnt, const P3* __restrict__ xyz, uint32_t ib,
    uint64_t* __restrict__ sk, uint32_t* __restrict__ sv, P3* __restrict__ sorted_xyz) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < cnt; i += gridDim.x * 256ull) {
    const uint64_t x = v[i];
    place_one<PACKED>(x, slot[i], i + count_below(other, ocnt, x), ib, xyz, sk, sv,
                                  sorted_xyz);
  }
}

// Both lists at once, kPlaceTile stayers per block. Block b owns the
// movers from its first stayer's value up to the next block's first stayer
// (block 0 also those below every stayer): two searches give that window.
// A stayer x of the block has lo + (window entries below x) movers below it;
// an owned mover has t0 + (block stayers below it) stayers below it, since
// the stayers of earlier blocks are all below it and those of later blocks
// all above. The block's stayers sit in LDS, and so does the window when it
// fits (else the stayers search it in memory).
constexpr uint32_t kPlaceTile = 2048;
constexpr uint32_t kPlaceWindow = 2048;

template <bool PACKED>
__global__ __launch_bounds__(256) void k_inc_merge(
    const uint64_t* __restrict__ st_v, const uint32_t* __restrict__ st_slot, uint32_t ns,
    const uint64_t* __restrict__ mv_v, const uint32_t* __restrict__ mv_slot, uint32_t nm,
    const P3* __restrict__ xyz, uint32_t ib, uint64_t* __restrict__ sk, uint32_t* __restrict__ sv,
    P3* __restrict__ sorted_xyz) {
  __shared__ uint64_t s_st[kPlaceTile];
  __shared__ uint64_t s_win[kPlaceWindow];
  __shared__ uint32_t s_lo, s_hi;
  const uint64_t t0 = (uint64_t)blockIdx.x * kPlaceTile;
  const uint32_t t1 = (uint32_t)min<uint64_t>(t0 + kPlaceTile, ns);
  const bool last = blockIdx.x + 1 == gridDim.x;
  if (threadIdx.x < 64) {
    const uint32_t c = blockIdx.x == 0 ? 0u : wave_count_below(mv_v, nm, st_v[t0]);
    if (threadIdx.x == 0) s_lo = c;
  } else if (threadIdx.x < 128) {
    const uint32_t c = last ? nm : wave_count_below(mv_v, nm, st_v[t1]);
    if (threadIdx.x == 64) s_hi = c;
  }
  // The block's stayers: loads first (clamped into the block), kept in LDS.
  constexpr int kItems = kPlaceTile / 256;
  uint64_t x[kItems];
  uint32_t sl[kItems];
  P3 p[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint64_t i = min<uint64_t>(t0 + (uint64_t)k * 256 + threadIdx.x, t1 - 1);
    x[k] = st_v[i];
    sl[k] = st_slot[i];
  }
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    p[k] = xyz[sl[k]];
    s_st[k * 256 + threadIdx.x] = x[k];  // entries past t1 are never searched
  }
  __syncthreads();
  const uint32_t lo = s_lo, hi = s_hi, w = hi - lo, n_st = t1 - (uint32_t)t0;
  const bool in_lds = w <= kPlaceWindow;
  if (in_lds)
    for (uint32_t k = threadIdx.x; k < w; k += 256) s_win[k] = mv_v[lo + k];
  __syncthreads();
  // Owned movers.
  for (uint32_t m = lo + threadIdx.x; m < hi; m += 256) {
    const uint64_t xm = in_lds ? s_win[m - lo] : mv_v[m];
    const uint32_t slm = mv_slot[m];
    uint32_t a = 0, b = n_st;
    while (a < b) {
      const uint32_t mid = (a + b) >> 1;
      if (s_st[mid] < xm) a = mid + 1;
      else b = mid;
    }
    place_one<PACKED>(xm, slm, (uint64_t)m + t0 + a, ib, xyz, sk, sv, sorted_xyz);
  }
  // Stayers.
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint64_t i = t0 + (uint64_t)k * 256 + threadIdx.x;
    if (i >= t1) continue;
    uint32_t below;
    if (in_lds) {
      uint32_t a = 0, b = w;
      while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if (s_win[mid] < x[k]) a = mid + 1;
        else b = mid;
      }
      below = lo + a;
    } else {
      below = lo + count_below(mv_v + lo, w, x[k]);
    }
    const uint64_t pos = i + below;
    const uint32_t j = (uint32_t)(x[k] & ((1ull << ib) - 1));
    const uint64_t key = x[k] >> ib;
    if (PACKED) {
      sk[pos] = (key << 32) | j;
    } else {
      sk[pos] = key;
      sv[pos] = j;
    }
    sorted_xyz[pos] = p[k];
  }
}

// Positions given in the previous sorted order back to original order.
__global__ __launch_bounds__(256) void k_inc_scatter(const P3* __restrict__ xyz,
                                                     const uint32_t* __restrict__ old_perm,
                                                     uint32_t n, P3* __restrict__ out) {
  for (uint64_t k = blockIdx.x * 256ull + threadIdx.x; k < n; k += gridDim.x * 256ull)
    out[old_perm[k]] = xyz[k];
}

}  // namespace

void launch_inc_scatter(const float* xyz, const uint32_t* old_perm, uint32_t n, float* out,
                        hipStream_t s) {
  const uint32_t grid = std::min<uint32_t>(div_up(n, 256), 8192);
  hipLaunchKernelGGL(k_inc_scatter, dim3(grid), dim3(256), 0, s, (const P3*)xyz, old_perm, n,
                     (P3*)out);
}

void launch_inc_classify(const float* xyz, const float* old_xyz, const uint32_t* old_perm,
                         uint32_t n, uint32_t L, uint32_t ib, uint32_t n_pass, uint64_t* st_v,
                         uint32_t* st_slot, uint64_t* mv_v, uint32_t* mv_slot, uint32_t* hist,
                         uint32_t* err, uint64_t* status, uint32_t* tile_counter,
                         uint32_t* counts, hipStream_t s) {
  const uint32_t grid = div_up(n, kCompTile);
  hipLaunchKernelGGL(k_inc_classify, dim3(grid), dim3(kCompBlock), 0, s, (const P3*)xyz,
                     (const P3*)old_xyz, old_perm, n, L, ib, n_pass, st_v, st_slot, mv_v, mv_slot,
                     hist, err, status, tile_counter, counts);
}

void launch_inc_merge(bool packed, const uint64_t* st_v, const uint32_t* st_slot, uint32_t ns,
                      const uint64_t* mv_v, const uint32_t* mv_slot, uint32_t nm,
                      const float* xyz, uint32_t ib, uint64_t* sk, uint32_t* sv,
                      float* sorted_xyz, hipStream_t s) {
  if (ns > 0) {
    const uint32_t grid = div_up(ns, kPlaceTile);
#define FMMDS_MERGE(P)                                                                         \
  hipLaunchKernelGGL((k_inc_merge<P>), dim3(grid), dim3(256), 0, s, st_v, st_slot, ns, mv_v,    \
                     mv_slot, nm, (const P3*)xyz, ib, sk, sv, (P3*)sorted_xyz)
    if (packed) FMMDS_MERGE(true);
    else FMMDS_MERGE(false);
#undef FMMDS_MERGE
  } else if (nm > 0) {  // every point moved: the sorted movers are the order
    const uint32_t grid = std::min<uint32_t>(div_up(nm, 256), 8192);
#define FMMDS_PLACE(P)                                                                         \
  hipLaunchKernelGGL((k_inc_place_movers<P>), dim3(grid), dim3(256), 0, s, mv_v, mv_slot, nm,  \
                     st_v, 0u, (const P3*)xyz, ib, sk, sv, (P3*)sorted_xyz)
    if (packed) FMMDS_PLACE(true);
    else FMMDS_PLACE(false);
#undef FMMDS_PLACE
  }
}

}  // namespace fmmds
