// E2 neighbor lists and E4 (M2L) interaction lists per level.
//
// Definitions (Section 1.4): for a receiver box r at level l, E2(r) holds the
// nonempty source boxes within one box of r in every coordinate (r included);
// E4(r) holds the nonempty source boxes that are children of boxes in
// E2(parent(r)) at level l - 1 but are not in E2(r). The paper enumerates the
// candidate boxes from de-interleaved coordinates (Section 2.3) and looks them
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

// Work mapping: one half-wave (32 lanes) per receiver box p of level l - 1;
// lane j takes the j-th entry s of E2(p) (at most 27). The lane computes,
// once for all receiver children of p, the offset of s from p, s's child mask
// and first child rank, and for each of the 8 child octants q the number of
// s's children adjacent to a receiver child in octant q. Two packed
// half-wave scans then give every lane its place in the E2 and E4 list of
// every receiver child of p at once (E4 places follow from the scan of all
// children minus the E2 places). For each receiver child r of p, in octant
// order, the lanes put their entries into a per-half-wave LDS buffer and the
// half-wave copies r's two lists out contiguously, 128 bytes per store.
//
// Offsets per axis come from dilated-integer subtraction on the Morton keys:
// with only one axis' bits kept in both operands, borrows run through the
// cleared bits between them, so ((a & M) - (b & M)) & M is the dilated
// difference of the two coordinates on that axis. Here it is 0, +1 or -1,
// i.e. 0, the axis' lowest bit, or all of the axis' bits.
constexpr uint64_t kAxisX = 0x1249249249249249ull;
constexpr int kHalfBuf = 224;  // E4 at [0, 189), E2 at [kE2At, kE2At + 27)
constexpr int kE2At = 192;

template <typename A>
__device__ __forceinline__ int axis_delta(A sk, A pk, A axis_mask, A axis_low) {
  const A d = (A)((sk & axis_mask) - (pk & axis_mask)) & axis_mask;
  return d == 0 ? 0 : (d == axis_low ? 1 : -1);
}

// Inclusive scan within each 32-lane half of the wave.
__device__ __forceinline__ uint32_t half_incl_scan(uint32_t v) {
  const uint32_t j = lane_id() & 31u;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 32);
    if (j >= (uint32_t)o) v += t;
  }
  return v;
}

// E2 count of octant q from the packed words: octants 0..3 sit in bits
// 8 + 6q of word a (bits 0..7 hold the count of all children), 4..7 in bits
// 6(q - 4) of word b.
__device__ __forceinline__ uint32_t octant_field(uint32_t a, uint32_t b, uint32_t q) {
  return q < 4 ? (a >> (8 + 6 * q)) & 63u : (b >> (6 * (q - 4))) & 63u;
}

template <typename KeyT, typename A, int MODE>  // MODE 0: count, 1: fill
__global__ __launch_bounds__(256) void k_lists(
    ListLevelArgs a, uint32_t* __restrict__ cnt2, uint32_t* __restrict__ cnt4,
    const uint32_t* __restrict__ off2, const uint32_t* __restrict__ off4,
    uint32_t* __restrict__ ent2, uint32_t* __restrict__ ent4) {
  __shared__ uint32_t s_buf[MODE == 1 ? 8 : 1][kHalfBuf];
  const KeyT* __restrict__ pkey = (const KeyT*)a.recv_key_up;
  const KeyT* __restrict__ skey = (const KeyT*)a.src_key_up;
  const uint32_t j = threadIdx.x & 31u, h = threadIdx.x >> 5;
  const uint64_t p = (uint64_t)blockIdx.x * 8 + h;
  const uint32_t n_up = a.n_recv_up_dev ? *a.n_recv_up_dev : a.n_recv_up;
  if (p >= n_up) return;  // whole half-wave
  // upbase: batch rank of the set's first box at level - 1 (parent-level E2
  // entries are stored relative to it); base: the same at level l.
  uint32_t j0, cnt, upbase = 0, base = 0;
  if (a.up_all) {
    j0 = 0;
    cnt = a.n_src_up;
  } else {
    j0 = a.e2_off_up[p];
    cnt = a.e2_off_up[p + 1] - j0;
  }
  if (a.first_up) {
    const uint32_t set = (uint32_t)((uint64_t)pkey[p] >> (3 * (a.level - 1)));
    base = a.first_cur[set];
    upbase = a.first_up[set];
    if (a.up_all) cnt = a.first_up[set + 1] - upbase;
    if (a.set_level[set] < a.level) cnt = 0;  // the set's lists stop above this level
  }
  const uint32_t rmask = a.recv_mask_up[p];
  const uint32_t rfirst = a.recv_child_up[p];
  uint32_t m = 0, cb = 0, wa = 0, wb = 0;
  uint32_t ax0 = 0, ax1 = 0, ay0 = 0, ay1 = 0, az0 = 0, az1 = 0;
  if (j < cnt) {
    const uint32_t s = upbase + (a.up_all ? j : a.e2_ent_up[j0 + j]);
    const A sk = (A)skey[s], pk = (A)pkey[p];
    const A X = (A)kAxisX;
    const int dx = axis_delta<A>(sk, pk, X, (A)1);
    const int dy = axis_delta<A>(sk, pk, (A)(X << 1), (A)2);
    const int dz = axis_delta<A>(sk, pk, (A)(X << 2), (A)4);
    m = a.src_mask_up[s];
    if (MODE == 1) cb = a.src_child_up[s] - base;
    // Children of s adjacent to a receiver child whose axis bit is 0 / 1:
    // offset 0: all; +1: child bit 0 and receiver bit 1; -1: child bit 1 and
    // receiver bit 0. Octants with the x / y / z bit clear: 0x55 / 0x33 / 0x0F.
    ax0 = dx == 0 ? 0xFFu : (dx < 0 ? 0xAAu : 0u);
    ax1 = dx == 0 ? 0xFFu : (dx > 0 ? 0x55u : 0u);
    ay0 = dy == 0 ? 0xFFu : (dy < 0 ? 0xCCu : 0u);
    ay1 = dy == 0 ? 0xFFu : (dy > 0 ? 0x33u : 0u);
    az0 = dz == 0 ? 0xFFu : (dz < 0 ? 0xF0u : 0u);
    az1 = dz == 0 ? 0xFFu : (dz > 0 ? 0x0Fu : 0u);
    wa = (uint32_t)__popc(m);
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) {
      const uint32_t adj = ((q & 1u) ? ax1 : ax0) & ((q & 2u) ? ay1 : ay0) & ((q & 4u) ? az1 : az0);
      const uint32_t c2 = __popc(m & adj);
      if (q < 4) wa |= c2 << (8 + 6 * q);
      else wb |= c2 << (6 * (q - 4));
    }
  }
  // Each field's sum over the half-wave stays in range: all children <= 216,
  // E2 of one octant <= 27.
  const uint32_t ia = half_incl_scan(wa), ib = half_incl_scan(wb);
  const uint32_t ea = ia - wa, eb = ib - wb;
  const uint32_t ta = __shfl(ia, 31, 32), tb = __shfl(ib, 31, 32);
  // Offsets of p's receiver children, loaded up front (lane k holds child k)
  // so that no load sits inside the loop below: on this GPU a wait for a load
  // also waits for every store issued before it.
  const uint32_t nchild = __popc(rmask);
  uint32_t my_o2 = 0, my_o4 = 0;
  if (MODE == 1 && j < nchild) {
    my_o2 = off2[rfirst + j];
    my_o4 = off4[rfirst + j];
  }
  uint32_t* buf = s_buf[MODE == 1 ? h : 0];
  uint32_t k = 0;
  uint32_t qm = rmask;
#pragma unroll 1
  while (qm) {
    const uint32_t q = __builtin_ctz(qm);
    qm &= qm - 1;
    const uint32_t n2 = octant_field(ta, tb, q), n4 = (ta & 0xFFu) - n2;
    if (MODE == 0) {
      if (j == 0) {
        cnt2[rfirst + k] = n2;
        cnt4[rfirst + k] = n4;
      }
    } else {
      const uint32_t o2 = __shfl(my_o2, k, 32), o4 = __shfl(my_o4, k, 32);
      const uint32_t adj = ((q & 1u) ? ax1 : ax0) & ((q & 2u) ? ay1 : ay0) & ((q & 4u) ? az1 : az0);
      const uint32_t b2 = kE2At + octant_field(ea, eb, q);
      const uint32_t b4 = (ea & 0xFFu) - octant_field(ea, eb, q);
      const uint32_t e2b = m & adj, e4b = m & ~adj;
      // Child octant o of s: rank cb + (children of s below o); it goes to E2
      // after the E2 children below it, else to E4 after the E4 ones below it.
#pragma unroll
      for (uint32_t o = 0; o < 8; ++o) {
        const uint32_t below = (1u << o) - 1u;
        if (m & (1u << o)) {
          const uint32_t pos = (adj & (1u << o)) ? b2 + __popc(e2b & below)
                                                 : b4 + __popc(e4b & below);
          buf[pos] = cb + __popc(m & below);
        }
      }
      __builtin_amdgcn_wave_barrier();
      uint32_t v4[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const uint32_t idx = j + 32u * i;
        v4[i] = idx < n4 ? buf[idx] : 0u;
      }
      const uint32_t v2 = j < n2 ? buf[kE2At + j] : 0u;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const uint32_t idx = j + 32u * i;
        if (idx < n4) ent4[(uint64_t)o4 + idx] = v4[i];
      }
      if (j < n2) ent2[(uint64_t)o2 + j] = v2;
      __builtin_amdgcn_wave_barrier();
    }
    ++k;
  }
}

template <int MODE>
void launch_lists(bool key64, const ListLevelArgs& a, uint32_t* cnt2, uint32_t* cnt4,
                  const uint32_t* off2, const uint32_t* off4, uint32_t* ent2, uint32_t* ent4,
                  hipStream_t s) {
  if (a.n_recv_up == 0) return;  // with n_recv_up_dev: the capacity
  const uint32_t grid = div_up(a.n_recv_up, 8);
  const bool narrow = a.key_bits_up <= 32;  // parent-level keys fit 32 bits
  if (key64 && narrow)
    hipLaunchKernelGGL((k_lists<uint64_t, uint32_t, MODE>), dim3(grid), dim3(256), 0, s, a, cnt2,
                       cnt4, off2, off4, ent2, ent4);
  else if (key64)
    hipLaunchKernelGGL((k_lists<uint64_t, uint64_t, MODE>), dim3(grid), dim3(256), 0, s, a, cnt2,
                       cnt4, off2, off4, ent2, ent4);
  else
    hipLaunchKernelGGL((k_lists<uint32_t, uint32_t, MODE>), dim3(grid), dim3(256), 0, s, a, cnt2,
                       cnt4, off2, off4, ent2, ent4);
}

void launch_list_count(bool key64, const ListLevelArgs& a, uint32_t* cnt2, uint32_t* cnt4,
                       hipStream_t s) {
  launch_lists<0>(key64, a, cnt2, cnt4, nullptr, nullptr, nullptr, nullptr, s);
}

void launch_list_fill(bool key64, const ListLevelArgs& a, const uint32_t* off2,
                      const uint32_t* off4, uint32_t* ent2, uint32_t* ent4, hipStream_t s) {
  launch_lists<1>(key64, a, nullptr, nullptr, off2, off4, ent2, ent4, s);
}

// ---------------------------------------------------------------------------
// Exclusive scan of per-box list lengths into CSR offsets (the scan that
// turns NumRecvE2NeiNEBox into NeighborBookmark, Algorithm 4), single pass.
// off[n] = total; the total also goes to *total, and the overflow flag is set
// if it does not fit 32-bit offsets.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCompBlock) void k_scan_counts(
    const uint32_t* __restrict__ cnt, uint32_t n_host, const uint32_t* __restrict__ n_dev,
    uint32_t* __restrict__ off, uint64_t* __restrict__ total, uint32_t* __restrict__ overflow,
    uint64_t* __restrict__ status, uint32_t* __restrict__ tile_counter) {
  __shared__ uint32_t s_w[kCompBlock / 64];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t n = n_dev ? *n_dev : n_host;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  if ((uint64_t)tile * kCompTile >= n) return;  // whole block: surplus tile
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
  if (w == 0) {
    const uint64_t ex = lookback_wave(status, tile, ttot);
    if (lane == 0) s_excl = ex;
  }
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
                        hipStream_t s, const uint32_t* n_dev) {
  // n is the exact count, or with n_dev the capacity (the count is read there)
  if (n == 0) return;
  hipLaunchKernelGGL(k_scan_counts, dim3(div_up(n, kCompTile)), dim3(kCompBlock), 0, s, cnt, n,
                     n_dev, off, total, overflow, status, tile_counter);
}

}  // namespace fmmds
