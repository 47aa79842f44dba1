// Kernels of the batched build: many independent point sets, each with its
// own maximum level, in one launch sequence.
//
// Every point carries a composite key: its set id above 3 * L_all bits, and
// below them the Morton index of its box at the set's own level L_i shifted
// left by 3 * (L_all - L_i), where L_all is the deepest level of the batch.
// The points of a batch arrive grouped by set, in set order, so the sort
// orders each set within its own range on the Morton bits alone (sort tiles
// never straddle two sets, and each set has its own digit offsets); the
// result is the order of the composite keys (set, then box, then index).
// Shifting a composite key right by 3 * (L_all - l) yields, for every set
// with L_i >= l, its level-l Morton index (Section 1.4) with the set id above
// bit 3l. The compaction and hierarchy kernels of the single build then run
// unchanged over the whole batch; the kernels here find where each set starts
// at each level and rewrite the tables in set-local terms.
#include "device.h"
#include "internal.h"

namespace fmmds {

struct P3b {
  float x, y, z;
};

// One block per keygen tile: at most 8192 points, all of one set, so the
// level and scale are the block's. The tile's digit counts go to its set's
// rows of hist with one atomic per nonzero bin.
template <bool PACKED>
__global__ __launch_bounds__(256) void k_batch_keygen(
    const P3b* __restrict__ xyz, const uint32_t* __restrict__ tile_start,
    const uint32_t* __restrict__ tile_set, const uint8_t* __restrict__ set_level, uint32_t L_all,
    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t n_pass,
    uint32_t* __restrict__ hist, uint32_t* __restrict__ err) {
  __shared__ uint32_t s_hist[kMaxPasses * 256];
  for (uint32_t i = threadIdx.x; i < n_pass * 256; i += 256) s_hist[i] = 0;
  const uint32_t t = blockIdx.x;
  const uint32_t begin = tile_start[t], end = tile_start[t + 1];
  const uint32_t set = tile_set[t] & 0x7FFFFFFFu;
  const uint32_t L = set_level[set];
  const float scale = (float)(1u << L);
  const uint32_t qmax = (1u << L) - 1;
  const uint64_t high = (uint64_t)set << (3 * L_all);
  const uint32_t lshift = 3 * (L_all - L);
  __syncthreads();
  bool bad = false;
  for (uint32_t i = begin + threadIdx.x; i < end; i += 256) {
    const P3b p = xyz[i];
    const bool ok = (p.x >= 0.0f && p.x < 1.0f) && (p.y >= 0.0f && p.y < 1.0f) &&
                    (p.z >= 0.0f && p.z < 1.0f);
    bad |= !ok;
    uint32_t qx = 0, qy = 0, qz = 0;
    if (ok) {
      qx = min((uint32_t)floorf(p.x * scale), qmax);
      qy = min((uint32_t)floorf(p.y * scale), qmax);
      qz = min((uint32_t)floorf(p.z * scale), qmax);
    }
    const uint64_t morton = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
    const uint64_t key = high | (morton << lshift);
    if (PACKED) {
      keys[i] = (key << 32) | i;
    } else {
      keys[i] = key;
      vals[i] = i;
    }
    for (uint32_t p8 = 0; p8 < n_pass; ++p8)
      atomicAdd(&s_hist[p8 * 256 + ((key >> (8 * p8)) & 0xFF)], 1u);
  }
  if (bad) atomicOr(err, 1u);
  __syncthreads();
  uint32_t* h = hist + (uint64_t)set * n_pass * 256;
  for (uint32_t i = threadIdx.x; i < n_pass * 256; i += 256)
    if (s_hist[i]) atomicAdd(&h[i], s_hist[i]);
}

void launch_batch_keygen(const float* xyz, const uint32_t* tile_start, const uint32_t* tile_set,
                         uint32_t n_tiles, const uint8_t* set_level, uint32_t L_all, bool packed,
                         uint64_t* keys, uint32_t* vals, uint32_t n_pass, uint32_t* hist,
                         uint32_t* err, hipStream_t s) {
  if (n_tiles == 0) return;
  if (packed)
    hipLaunchKernelGGL(k_batch_keygen<true>, dim3(n_tiles), dim3(256), 0, s, (const P3b*)xyz,
                       tile_start, tile_set, set_level, L_all, keys, vals, n_pass, hist, err);
  else
    hipLaunchKernelGGL(k_batch_keygen<false>, dim3(n_tiles), dim3(256), 0, s, (const P3b*)xyz,
                       tile_start, tile_set, set_level, L_all, keys, vals, n_pass, hist, err);
}

// Block (i, p): exclusive scan of set i's pass-p histogram, offset by the
// set's first element.
__global__ __launch_bounds__(256) void k_batch_digit_offsets(const uint32_t* __restrict__ hist,
                                                             const uint64_t* __restrict__ set_off,
                                                             uint32_t n_pass,
                                                             uint32_t* __restrict__ goff) {
  __shared__ uint32_t s_w[4];
  const uint32_t set = blockIdx.x, p = blockIdx.y, d = threadIdx.x, lane = d & 63, w = d >> 6;
  const uint64_t row = ((uint64_t)set * n_pass + p) * 256;
  const uint32_t c = hist[row + d];
  const uint32_t inc = wave_incl_scan(c);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t base = (uint32_t)set_off[set];
  for (uint32_t i = 0; i < w; ++i) base += s_w[i];
  goff[row + d] = base + inc - c;
}

void launch_batch_digit_offsets(const uint32_t* hist, const uint64_t* set_off, uint32_t n_sets,
                                uint32_t n_pass, uint32_t* goff, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_digit_offsets, dim3(n_sets, n_pass), dim3(256), 0, s, hist, set_off,
                     n_pass, goff);
}

// first[l * (n_sets + 1) + i] = rank of set i's first box at level l: the box
// whose bookmark is the set's first point (a set always starts a new box).
// first[l * (n_sets + 1) + n_sets] = boxes at level l.
__global__ __launch_bounds__(256) void k_batch_first(LevelPtrs lp, uint32_t L_all,
                                                     const uint32_t* __restrict__ n_boxes,
                                                     const uint64_t* __restrict__ set_off,
                                                     uint32_t n_sets,
                                                     uint32_t* __restrict__ first) {
  const uint64_t t = blockIdx.x * 256ull + threadIdx.x;
  const uint64_t per = (uint64_t)n_sets + 1;
  if (t >= per * (L_all + 1)) return;
  const uint32_t l = (uint32_t)(t / per), i = (uint32_t)(t % per);
  const uint32_t nl = n_boxes[l];
  if (i == n_sets) {
    first[t] = nl;
    return;
  }
  const uint32_t* b = lp.begin[l];
  const uint64_t target = set_off[i];
  uint32_t lo = 0, hi = nl;  // first index with b[idx] >= target
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((uint64_t)b[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  first[t] = lo;
}

void launch_batch_first(const LevelPtrs& lp, uint32_t L_all, const uint32_t* n_boxes,
                        const uint64_t* set_off, uint32_t n_sets, uint32_t* first, hipStream_t s) {
  const uint64_t total = ((uint64_t)n_sets + 1) * (L_all + 1);
  hipLaunchKernelGGL(k_batch_first, dim3(div_up(total, 256)), dim3(256), 0, s, lp, L_all, n_boxes,
                     set_off, n_sets, first);
}

// Set-local tables in the per-set layout, every level in one launch
// (blockIdx.y = level): keys, parents and box rows at their batch rank g;
// bookmarks and first children at g + set, which leaves one slot after each
// set for its sentinel.
__global__ __launch_bounds__(256) void k_batch_rebase(RebaseArgs a) {
  const uint32_t l = blockIdx.y;
  const uint32_t n = *a.n_l[l];
  const uint64_t per = (uint64_t)a.n_sets + 1;
  const uint32_t* first_cur = a.first + l * per;
  const uint32_t* first_prev = l >= 1 ? a.first + (l - 1) * per : nullptr;
  const uint32_t* first_next = l < a.L ? a.first + (l + 1) * per : nullptr;
  const uint64_t* gkey = a.gkey[l];
  const uint32_t* gbegin = a.gbegin[l];
  const uint32_t* gparent = a.gparent[l];
  const uint32_t* gchild = a.gchild[l];
  uint64_t* fkey = a.fkey[l];
  uint32_t* fbegin = a.fbegin[l];
  uint32_t* fparent = a.fparent[l];
  uint32_t* fchild = a.fchild[l];
  const uint64_t* set_off = a.set_off;
  for (uint64_t g = blockIdx.x * 256ull + threadIdx.x; g < n; g += gridDim.x * 256ull) {
    const uint64_t key = gkey[g];
    const uint32_t set = (uint32_t)(key >> (3 * l));
    fkey[g] = l == 0 ? 0 : (key & ((1ull << (3 * l)) - 1));
    fbegin[g + set] = (uint32_t)(gbegin[g] - set_off[set]);
    if (gparent) fparent[g] = gparent[g] - first_prev[set];
    if (gchild) fchild[g + set] = gchild[g] - first_next[set];
    if (g + 1 == first_cur[set + 1]) {  // the set's last box: its sentinels
      fbegin[g + 1 + set] = (uint32_t)(set_off[set + 1] - set_off[set]);
      if (gchild) fchild[g + 1 + set] = first_next[set + 1] - first_next[set];
    }
  }
}

void launch_batch_rebase(const RebaseArgs& a, uint32_t max_cap, hipStream_t s) {
  const uint32_t gx = std::max<uint32_t>(1, std::min<uint32_t>(div_up(max_cap, 256), 2048));
  hipLaunchKernelGGL(k_batch_rebase, dim3(gx, a.L + 1), dim3(256), 0, s, a);
}

// List offsets relative to each set's first receiver, in the per-set layout
// (slot g + set, sentinel after each set), and each set's base into the
// batch's entry arrays (base[n_sets] = the level's total); levels 2..L in one
// launch (blockIdx.y = level - 2).
__global__ __launch_bounds__(256) void k_batch_list_rebase(ListRebaseArgs a) {
  const uint32_t l = blockIdx.y + 2;
  const uint32_t n = *a.n_l[l];
  const uint64_t per = (uint64_t)a.n_sets + 1;
  const uint32_t* first_cur = a.first + l * per;
  const uint64_t* gkey = a.gkey[l];
  const uint32_t* goff2 = a.goff2[l];
  const uint32_t* goff4 = a.goff4[l];
  uint32_t* loff2 = a.loff2[l];
  uint32_t* loff4 = a.loff4[l];
  uint32_t* base2 = a.base + (2 * l) * per;
  uint32_t* base4 = a.base + (2 * l + 1) * per;
  for (uint64_t g = blockIdx.x * 256ull + threadIdx.x; g < n; g += gridDim.x * 256ull) {
    const uint32_t set = (uint32_t)(gkey[g] >> (3 * l));
    const uint32_t f = first_cur[set];
    const uint32_t b2 = goff2[f], b4 = goff4[f];
    loff2[g + set] = goff2[g] - b2;
    loff4[g + set] = goff4[g] - b4;
    if (g == f) {
      base2[set] = b2;
      base4[set] = b4;
    }
    if (g + 1 == first_cur[set + 1]) {
      loff2[g + 1 + set] = goff2[g + 1] - b2;
      loff4[g + 1 + set] = goff4[g + 1] - b4;
    }
    if (g + 1 == n) {
      base2[a.n_sets] = goff2[n];
      base4[a.n_sets] = goff4[n];
    }
  }
}

void launch_batch_list_rebase(const ListRebaseArgs& a, uint32_t max_cap, hipStream_t s) {
  if (a.L < 2) return;
  const uint32_t gx = std::max<uint32_t>(1, std::min<uint32_t>(div_up(max_cap, 256), 2048));
  hipLaunchKernelGGL(k_batch_list_rebase, dim3(gx, a.L - 1), dim3(256), 0, s, a);
}

}  // namespace fmmds
