// Key generation and LSD radix sort of (Morton key, point index) pairs.
//
// The paper reorders points by the Morton index of their finest-level box
// with a histogram pseudo-sort whose order inside a box depends on atomic
// timing (Section 2.1, Algorithm 1). This library needs a deterministic order,
// so it sorts (key, original index) pairs stably: an LSD radix sort with 8-bit
// digits, one single-pass "chained scan" kernel per digit.
#include "device.h"
#include "internal.h"

namespace fmmds {

// ---------------------------------------------------------------------------
// Zero fill (a kernel, so that it can sit inside a captured graph).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero(uint4* __restrict__ p, size_t n16) {
  const uint4 z = make_uint4(0, 0, 0, 0);
  for (size_t i = blockIdx.x * 256ull + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256)
    p[i] = z;
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  // Every region handed to this function is 16-byte aligned and sized.
  const size_t n16 = bytes / 16;
  if (n16 == 0) return;
  const uint32_t grid = (uint32_t)std::min<size_t>(div_up(n16, 256), 4096);
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, (uint4*)p, n16);
}

// ---------------------------------------------------------------------------
// K1: Morton key of every point (Section 1.4 box index, Section 2.4
// interleave) plus the digit histograms of every sort pass.
//
// A point (x, y, z) is in the box floor(x * 2^L) per axis; x * 2^L is exact in
// FP32. Coordinates outside [0, 1) (or NaN) raise the range flag; such points
// get box 0 so that later kernels stay in bounds, and the build reports the
// error.
// ---------------------------------------------------------------------------
struct P3 {
  float x, y, z;
};

// Each thread loads kKeyItems points (one 64-point run per wave and item,
// all issued before any is used), so the loads of a block are in flight
// together rather than one per loop trip. Each block writes its digit
// histograms as one row (no atomics: thousands of blocks adding into the same
// 256 bins per pass serialize on those addresses); the digit-offset kernel
// adds the rows.
constexpr int kKeyItems = 8;
constexpr int kKeyChunk = 256 * kKeyItems;
constexpr uint32_t kKeyMaxBlocks = 4096;

template <bool PACKED>
__global__ __launch_bounds__(256) void k_keygen(const P3* __restrict__ xyz, uint32_t n, uint32_t L,
                                                uint64_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals, uint32_t n_pass,
                                                uint32_t* __restrict__ rows,
                                                uint32_t* __restrict__ err) {
  __shared__ uint32_t s_hist[kMaxPasses * 256];
  for (uint32_t i = threadIdx.x; i < n_pass * 256; i += 256) s_hist[i] = 0;
  __syncthreads();
  bool bad = false;
  for (uint64_t base = (uint64_t)blockIdx.x * kKeyChunk; base < n;
       base += (uint64_t)gridDim.x * kKeyChunk) {
    P3 p[kKeyItems];
#pragma unroll
    for (int j = 0; j < kKeyItems; ++j) {
      const uint64_t i = base + (uint64_t)j * 256 + threadIdx.x;
      p[j] = i < n ? xyz[i] : P3{0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int j = 0; j < kKeyItems; ++j) {
      const uint64_t i = base + (uint64_t)j * 256 + threadIdx.x;
      if (i >= n) continue;
      bool ok;
      const uint64_t key = point_key(p[j].x, p[j].y, p[j].z, L, ok);
      bad |= !ok;
      if (PACKED) {
        keys[i] = (key << 32) | (uint32_t)i;
      } else {
        keys[i] = key;
        vals[i] = (uint32_t)i;
      }
      for (uint32_t p8 = 0; p8 < n_pass; ++p8)
        atomicAdd(&s_hist[p8 * 256 + ((key >> (8 * p8)) & 0xFF)], 1u);
    }
  }
  if (bad) atomicOr(err, 1u);
  __syncthreads();
  uint32_t* row = rows + (uint64_t)blockIdx.x * n_pass * 256;
  for (uint32_t i = threadIdx.x; i < n_pass * 256; i += 256) row[i] = s_hist[i];
}

uint32_t keygen_blocks(uint32_t n) {
  return std::max<uint32_t>(1, std::min<uint32_t>(div_up(n, kKeyChunk), kKeyMaxBlocks));
}

void launch_keygen(const float* xyz, uint32_t n, uint32_t L, bool packed, uint64_t* keys,
                   uint32_t* vals, uint32_t n_pass, uint32_t* rows, uint32_t* err,
                   hipStream_t s) {
  const uint32_t grid = keygen_blocks(n);
  if (packed)
    hipLaunchKernelGGL(k_keygen<true>, dim3(grid), dim3(256), 0, s, (const P3*)xyz, n, L, keys,
                       vals, n_pass, rows, err);
  else
    hipLaunchKernelGGL(k_keygen<false>, dim3(grid), dim3(256), 0, s, (const P3*)xyz, n, L, keys,
                       vals, n_pass, rows, err);
}

// Keygen's per-block rows added into the zeroed pass histograms: block
// (b, p) adds rows b, b + gridDim.x, ... of pass p, then one atomic per bin
// (a few dozen per address instead of one per keygen block).
constexpr uint32_t kRowReduceBlocks = 64;
__global__ __launch_bounds__(256) void k_reduce_rows(const uint32_t* __restrict__ rows,
                                                     uint32_t n_rows, uint32_t n_pass,
                                                     uint32_t* __restrict__ hist) {
  const uint32_t p = blockIdx.y, d = threadIdx.x, G = gridDim.x;
  uint32_t c = 0, r = blockIdx.x;
  // eight rows' loads in flight per round
  for (; r + 7 * G < n_rows; r += 8 * G) {
    uint32_t v[8];
#pragma unroll
    for (uint32_t t = 0; t < 8; ++t) v[t] = rows[((uint64_t)(r + t * G) * n_pass + p) * 256 + d];
#pragma unroll
    for (uint32_t t = 0; t < 8; ++t) c += v[t];
  }
  for (; r < n_rows; r += G) c += rows[((uint64_t)r * n_pass + p) * 256 + d];
  if (c) atomicAdd(&hist[p * 256 + d], c);
}

void launch_reduce_rows(const uint32_t* rows, uint32_t n_rows, uint32_t* hist, uint32_t n_pass,
                        hipStream_t s) {
  const dim3 grid(std::min(kRowReduceBlocks, n_rows), n_pass);
  hipLaunchKernelGGL(k_reduce_rows, grid, dim3(256), 0, s, rows, n_rows, n_pass, hist);
}

// Exclusive scan of each pass's 256-bin histogram: where digit d starts.
__global__ __launch_bounds__(256) void k_digit_offsets(const uint32_t* __restrict__ hist,
                                                       uint32_t* __restrict__ goff) {
  __shared__ uint32_t s_w[4];
  const uint32_t p = blockIdx.x, d = threadIdx.x, lane = d & 63, w = d >> 6;
  const uint32_t c = hist[p * 256 + d];
  const uint32_t inc = wave_incl_scan(c);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (uint32_t i = 0; i < w; ++i) base += s_w[i];
  goff[p * 256 + d] = base + inc - c;
}

void launch_digit_offsets(const uint32_t* hist, uint32_t* goff, uint32_t n_pass, hipStream_t s) {
  hipLaunchKernelGGL(k_digit_offsets, dim3(n_pass), dim3(256), 0, s, hist, goff);
}

// ---------------------------------------------------------------------------
// K2: one stable LSD pass on the 8-bit digit at `shift`.
//
// A tile of BLOCK * ITEMS elements is split into contiguous 64 * ITEMS-element
// wave segments, loaded 64 at a time (coalesced). Each wave ranks its
// elements by digit with eight ballots per element (lanes whose digit agrees
// on every bit), keeping running per-digit counts in LDS, so ranks follow
// input order. The tile's 256 digit counts are then chained across tiles by
// decoupled look-back (thread d < 256 owns digit d), the tile is staged in
// LDS in digit order, and written out so that consecutive threads store
// consecutive addresses of one digit's run. The look-back chain is what sets
// the pass's length (without it a 4096-element pass over 2^24 elements takes
// ~75 us instead of ~125 us), so each tile publishes its digit counts (LDS
// atomics) before it ranks, tiles of 8192 packed elements (512 threads)
// halve the chain of 4096-element tiles, and each digit's walk loads four
// predecessors' words at a time.
// ---------------------------------------------------------------------------
// The 8-bit digit at `shift`. A packed element holds the key in its high
// word, and its passes start at shift 32.
template <bool PACKED>
__device__ __forceinline__ uint32_t sort_digit(uint64_t k, uint32_t shift) {
  return PACKED ? __builtin_amdgcn_ubfe((uint32_t)(k >> 32), shift - 32u, 8u)
                : (uint32_t)(k >> shift) & 0xFFu;
}

// With SEG, tiles come from a set-aligned table (SegSort): each tile lies in
// one set, a set's first tile starts its own look-back chain, and the digit
// offsets are that set's, so every set is sorted within its own range.
template <bool PACKED, int BLOCK, int ITEMS, bool SEG>
__global__ __launch_bounds__(BLOCK) void k_sort_pass(
    const uint64_t* __restrict__ kin, uint64_t* __restrict__ kout, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ vout, uint32_t n_host, uint32_t shift, const uint32_t* __restrict__ goff,
    uint64_t* __restrict__ status, uint32_t* __restrict__ tile_counter,
    const uint32_t* __restrict__ n_dev, SegSort sg) {
  static_assert(BLOCK >= 256, "thread d owns digit d");
  constexpr int W = BLOCK / 64;
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int WSEG = 64 * ITEMS;
  __shared__ uint64_t s_key[TILE];
  __shared__ uint32_t s_val[PACKED ? 1 : TILE];
  __shared__ uint32_t s_hist[W][256];
  __shared__ uint32_t s_cnt[256];  // the tile's digit counts, published before the ranking
  __shared__ uint32_t s_lstart[256];
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_scan[4];
  __shared__ uint32_t s_tile;

  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  for (uint32_t i = tid; i < W * 256; i += BLOCK) (&s_hist[0][0])[i] = 0;
  if (tid < 256) s_cnt[tid] = 0;
  __syncthreads();
  const uint32_t tile = __builtin_amdgcn_readfirstlane(s_tile);
  uint64_t tbase, tend;
  bool first;
  const uint32_t* __restrict__ go = goff;
  if (SEG) {
    tbase = sg.start[tile];
    tend = sg.start[tile + 1];
    const uint32_t sw = sg.set[tile];
    first = (sw >> 31) != 0;
    go = sg.goff + ((uint64_t)(sw & 0x7FFFFFFFu) * sg.n_pass + sg.pass) * 256;
  } else {
    const uint32_t n = n_dev ? *n_dev : n_host;
    // With the count on the device the grid covers the capacity; tiles past
    // the count exit (tiles only look back at lower tile ids).
    if ((uint64_t)tile * TILE >= n && tile > 0) return;
    tbase = (uint64_t)tile * TILE;
    tend = min(tbase + TILE, (uint64_t)n);
    first = tile == 0;
  }
  const uint64_t wbase = tbase + (uint64_t)w * WSEG;
  // Item i of this lane is element wbase + 64 i + lane, valid while
  // 64 i + lane < lim (32-bit tests; the wave's base pointer is uniform).
  const uint32_t lim = (uint32_t)min((uint64_t)WSEG, tend > wbase ? tend - wbase : 0ull);
  const uint64_t* __restrict__ kw = kin + wbase;
  const uint32_t* __restrict__ vw = PACKED ? nullptr : vin + wbase;

  uint64_t k[ITEMS];
  uint32_t v[ITEMS];
  uint32_t r[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t j = 64u * i + lane;
    k[i] = j < lim ? kw[j] : 0;
    if (!PACKED) v[i] = j < lim ? vw[j] : 0;
  }
  // The tile's digit counts first (LDS atomics), published at once, so that
  // later tiles' look-backs find them while this tile still ranks.
#pragma unroll
  for (int i = 0; i < ITEMS; ++i)
    if (64u * i + lane < lim) atomicAdd(&s_cnt[sort_digit<PACKED>(k[i], shift)], 1u);
  __syncthreads();
  if (tid < 256) {
    const uint64_t agg = s_cnt[tid];
    st_status(status + (uint64_t)tile * 256 + tid, (first ? kStInc : kStAgg) | agg);
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const bool valid = 64u * i + lane < lim;
    const uint32_t d = sort_digit<PACKED>(k[i], shift);
    // peers: the valid lanes whose digit equals this lane's. Per bit b, m is
    // all ones where this lane's bit is 0, so that (ballot ^ m) keeps the
    // lanes that agree with it on bit b (one three-input bit op per half).
    const uint64_t vb = __ballot(valid);
    uint32_t plo = (uint32_t)vb, phi = (uint32_t)(vb >> 32);
    const uint32_t nd = ~d;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)nd, b, 1);
      const uint64_t bal = __ballot(m == 0u);
      plo &= (uint32_t)bal ^ m;
      phi &= (uint32_t)(bal >> 32) ^ m;
    }
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
    uint32_t prev = 0;
    if (valid) prev = s_hist[w][d];
    r[i] = prev + below;
    if (valid && below == 0) s_hist[w][d] = prev + (uint32_t)(__popc(plo) + __popc(phi));
  }
  __syncthreads();

  // Thread d < 256 owns digit d: wave-exclusive prefixes, tile count, local
  // start, then the tile's global base by look-back.
  uint32_t cnt = 0, inc = 0;
  if (tid < 256) {
    uint32_t run = 0;
#pragma unroll
    for (int ww = 0; ww < W; ++ww) {
      const uint32_t c = s_hist[ww][tid];
      s_hist[ww][tid] = run;
      run += c;
    }
    cnt = run;
    inc = wave_incl_scan(cnt);
    if (lane == 63) s_scan[w] = inc;
  }
  __syncthreads();
  if (tid < 256) {
    const uint32_t d = tid;
    uint32_t wpre = 0;
    for (uint32_t ww = 0; ww < w; ++ww) wpre += s_scan[ww];
    const uint32_t lstart = wpre + inc - cnt;
    s_lstart[d] = lstart;
    const uint64_t excl = first ? 0 : lookback_window<4>(status + d, 256, tile, cnt);
    s_base[d] = go[d] + (uint32_t)excl - lstart;
  }
  __syncthreads();

#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (64u * i + lane < lim) {
      const uint32_t dd = sort_digit<PACKED>(k[i], shift);
      const uint32_t lp = s_lstart[dd] + s_hist[w][dd] + r[i];
      s_key[lp] = k[i];
      if (!PACKED) s_val[lp] = v[i];
    }
  }
  __syncthreads();
  const uint32_t tcount = (uint32_t)(tend - tbase);
  for (uint32_t j = tid; j < tcount; j += BLOCK) {
    const uint64_t kk = s_key[j];
    const uint32_t dd = sort_digit<PACKED>(kk, shift);
    const uint32_t g = s_base[dd] + j;
    kout[g] = kk;
    if (!PACKED) vout[g] = s_val[j];
  }
}

uint32_t sort_tile_elems(int items) { return items == kSortWide ? 8192u : 256u * (uint32_t)items; }

uint32_t sort_tiles(uint32_t n, int items) { return div_up(n, sort_tile_elems(items)); }

template <bool SEG>
void sort_pass_dispatch(bool packed, const uint64_t* kin, uint64_t* kout, const uint32_t* vin,
                        uint32_t* vout, uint32_t n, uint32_t grid, uint32_t shift,
                        const uint32_t* goff, uint64_t* status, uint32_t* tile_counter,
                        hipStream_t s, int items, const uint32_t* n_dev, const SegSort& sg) {
#define FMMDS_SORT(P, B, I)                                                                     \
  hipLaunchKernelGGL((k_sort_pass<P, B, I, SEG>), dim3(grid), dim3(B), 0, s, kin, kout, vin,   \
                     vout, n, shift, goff, status, tile_counter, n_dev, sg)
  if (items == kSortWide && packed) FMMDS_SORT(true, 512, 16);
  else if (items == 8) {
    if (packed) FMMDS_SORT(true, 256, 8);
    else FMMDS_SORT(false, 256, 8);
  } else if (items == 12) {
    if (packed) FMMDS_SORT(true, 256, 12);
    else FMMDS_SORT(false, 256, 12);
  } else {
    if (packed) FMMDS_SORT(true, 256, 16);
    else FMMDS_SORT(false, 256, 16);
  }
#undef FMMDS_SORT
}

void launch_sort_pass(bool packed, const uint64_t* kin, uint64_t* kout, const uint32_t* vin,
                      uint32_t* vout, uint32_t n, uint32_t shift, const uint32_t* goff,
                      uint64_t* status, uint32_t* tile_counter, hipStream_t s, int items,
                      const uint32_t* n_dev) {
  sort_pass_dispatch<false>(packed, kin, kout, vin, vout, n, sort_tiles(n, items), shift, goff,
                            status, tile_counter, s, items, n_dev, SegSort{});
}

void launch_sort_pass_seg(bool packed, const uint64_t* kin, uint64_t* kout, const uint32_t* vin,
                          uint32_t* vout, uint32_t shift, const SegSort& sg, uint64_t* status,
                          uint32_t* tile_counter, hipStream_t s, int items) {
  if (sg.n_tiles == 0) return;
  sort_pass_dispatch<true>(packed, kin, kout, vin, vout, 0, sg.n_tiles, shift, nullptr, status,
                           tile_counter, s, items, nullptr, sg);
}

}  // namespace fmmds
