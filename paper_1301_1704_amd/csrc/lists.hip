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

// Counting: one half-wave (32 lanes) per receiver box p of level l - 1; lane
// j takes the j-th entry s of E2(p) (at most 27). The lane computes the
// offset of s from p, s's child mask and, for each of the 8 child octants q,
// the number of s's children adjacent to a receiver child in octant q; two
// packed half-wave scans give the E2 count of every receiver child of p at
// once (E4 = all children minus E2).
//
// Filling: two receiver boxes p per wave, one per half-wave for the setup.
// The children of all s in E2(p), in ascending rank, form one union list U
// (at most 216 boxes), the same for every receiver child of p; the half-wave
// writes U once to LDS together with, per entry, the 8-bit mask of receiver
// octants it is adjacent to. Then the whole wave takes each p in turn: each
// lane keeps its share of U in registers, and for each receiver child the
// wave splits U into the child's E2 and E4 lists with one ballot per 64
// entries: order is kept, so both come out ascending, and each chunk is
// stored to two contiguous ranges.
//
// Offsets per axis come from dilated-integer subtraction on the Morton keys:
// with only one axis' bits kept in both operands, borrows run through the
// cleared bits between them, so ((a & M) - (b & M)) & M is the dilated
// difference of the two coordinates on that axis. Here it is 0, +1 or -1,
// i.e. 0, the axis' lowest bit, or all of the axis' bits.
constexpr uint64_t kAxisX = 0x1249249249249249ull;
constexpr int kUnion = 256;  // >= 27 * 8 children of E2(p)

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

template <typename KeyT, typename A>
__global__ __launch_bounds__(256) void k_list_count(ListLevelArgs a, uint32_t* __restrict__ cnt2,
                                                    uint32_t* __restrict__ cnt4) {
  const KeyT* __restrict__ pkey = (const KeyT*)a.recv_key_up;
  const KeyT* __restrict__ skey = (const KeyT*)a.src_key_up;
  const uint32_t j = threadIdx.x & 31u, h = threadIdx.x >> 5;
  const uint64_t p = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * 8 + h;
  const uint32_t n_up = a.n_recv_up_dev ? *a.n_recv_up_dev : a.n_recv_up;
  if (p >= n_up) return;  // whole half-wave
  // upbase: batch rank of the set's first box at level - 1 (parent-level E2
  // entries are stored relative to it).
  uint32_t j0, cnt, upbase = 0;
  if (a.up_all) {
    j0 = 0;
    cnt = a.n_src_up_dev ? *a.n_src_up_dev : a.n_src_up;
  } else {
    j0 = a.e2_off_up[p];
    cnt = a.e2_off_up[p + 1] - j0;
  }
  if (a.first_up) {
    const uint32_t set = (uint32_t)((uint64_t)pkey[p] >> (3 * (a.level - 1)));
    upbase = a.first_up[set];
    if (a.up_all) cnt = a.first_up[set + 1] - upbase;
    if (a.set_level[set] < a.level) cnt = 0;  // the set's lists stop above this level
  }
  const uint32_t rmask = a.recv_mask_up[p];
  const uint32_t rfirst = a.recv_child_up[p];
  uint32_t wa = 0, wb = 0;
  if (j < cnt) {
    const uint32_t s = upbase + (a.up_all ? j : a.e2_ent_up[j0 + j]);
    const A sk = (A)skey[s], pk = (A)pkey[p];
    const A X = (A)kAxisX;
    const int dx = axis_delta<A>(sk, pk, X, (A)1);
    const int dy = axis_delta<A>(sk, pk, (A)(X << 1), (A)2);
    const int dz = axis_delta<A>(sk, pk, (A)(X << 2), (A)4);
    const uint32_t m = a.src_mask_up[s];
    // Children of s adjacent to a receiver child whose axis bit is 0 / 1:
    // offset 0: all; +1: child bit 0 and receiver bit 1; -1: child bit 1 and
    // receiver bit 0. Octants with the x / y / z bit clear: 0x55 / 0x33 / 0x0F.
    const uint32_t ax0 = dx == 0 ? 0xFFu : (dx < 0 ? 0xAAu : 0u);
    const uint32_t ax1 = dx == 0 ? 0xFFu : (dx > 0 ? 0x55u : 0u);
    const uint32_t ay0 = dy == 0 ? 0xFFu : (dy < 0 ? 0xCCu : 0u);
    const uint32_t ay1 = dy == 0 ? 0xFFu : (dy > 0 ? 0x33u : 0u);
    const uint32_t az0 = dz == 0 ? 0xFFu : (dz < 0 ? 0xF0u : 0u);
    const uint32_t az1 = dz == 0 ? 0xFFu : (dz > 0 ? 0x0Fu : 0u);
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
  const uint32_t ta = __shfl(half_incl_scan(wa), 31, 32);
  const uint32_t tb = __shfl(half_incl_scan(wb), 31, 32);
  // Lane j writes the counts of receiver child j (octant: the j-th set bit
  // of the mask), so the children's counts leave in one store each.
  if (j < (uint32_t)__popc(rmask)) {
    uint32_t mm = rmask;
    for (uint32_t t = 0; t < j; ++t) mm &= mm - 1;
    const uint32_t n2 = octant_field(ta, tb, (uint32_t)__builtin_ctz(mm));
    cnt2[rfirst + j] = n2;
    cnt4[rfirst + j] = (ta & 0xFFu) - n2;
  }
}

// NEXT: also write the counts of level + 1 (see ListLevelArgs). E2(r) for a
// receiver child r of p is the set of U entries marked for r. An entry u
// (child o of the parent neighbor s at offset d' from p) sits at offset
// 2 d' + o - q from r per axis (q: r's octant); the setup stores t - 1 with
// t = 2 d' + o + 2 (2 bits per axis: for entries of some E2(r), t is 1..4).
// During the split the E2 lanes also copy (child mask of u, t - 1) into a
// small per-child LDS list; afterwards the lanes of the wave take one
// (receiver child r, octant q' of r's children) pair each and count, over
// E2(r), the children of u adjacent to r's child q', as the count kernel
// does one level down. The lanes stay busy in that phase, instead of
// counting inside the split where only the E2 lanes are.
constexpr int kE2Max = 27;

template <typename KeyT, typename A, bool NEXT>
__global__ __launch_bounds__(256) void k_list_fill(ListLevelArgs a, const uint32_t* __restrict__ off2,
                                                   const uint32_t* __restrict__ off4,
                                                   uint32_t* __restrict__ ent2,
                                                   uint32_t* __restrict__ ent4) {
  __shared__ uint32_t s_rank[8][kUnion];
  __shared__ uint8_t s_adj[8][kUnion];
  __shared__ uint8_t s_off[NEXT ? 8 : 1][NEXT ? kUnion : 1];
  __shared__ uint32_t s_e2[NEXT ? 4 : 1][NEXT ? 16 : 1][NEXT ? kE2Max : 1];
  const KeyT* __restrict__ pkey = (const KeyT*)a.recv_key_up;
  const KeyT* __restrict__ skey = (const KeyT*)a.src_key_up;
  const uint32_t lane = threadIdx.x & 63u, j = lane & 31u, h = threadIdx.x >> 5;
  const uint64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint64_t p = blk * 8 + h;
  const uint32_t n_up = a.n_recv_up_dev ? *a.n_recv_up_dev : a.n_recv_up;
  if (blk * 8 + (h & ~1u) >= n_up) return;  // whole wave: both parents absent
  const bool live = p < n_up;
  // Setup, one half-wave per parent p (lane j: the j-th entry s of E2(p)).
  // upbase: batch rank of the set's first box at level - 1 (parent-level E2
  // entries are stored relative to it); base: the same at level l.
  uint32_t j0 = 0, cnt = 0, upbase = 0, base = 0, rmask = 0, rfirst = 0;
  bool next_zero = false;  // the set has no lists at level + 1
  if (live) {
    if (a.up_all) {
      cnt = a.n_src_up_dev ? *a.n_src_up_dev : a.n_src_up;
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
      next_zero = a.set_level[set] < a.level + 1;
    }
    rmask = a.recv_mask_up[p];
    rfirst = a.recv_child_up[p];
  }
  // Offsets of p's receiver children (lane j holds child j), and with NEXT
  // their child masks and first children, loaded before any store: on this
  // GPU a wait for a load also waits for earlier stores.
  uint32_t my_o2 = 0, my_o4 = 0, my_rm = 0, my_rc = 0;
  if (j < (uint32_t)__popc(rmask)) {
    my_o2 = off2[rfirst + j];
    my_o4 = off4[rfirst + j];
    if (NEXT) {
      my_rm = a.recv_mask_cur[rfirst + j];
      my_rc = a.recv_child_cur[rfirst + j];
    }
  }
  uint32_t m = 0, cb = 0, xm0 = 0, xm1 = 0, ym0 = 0, ym1 = 0, zm0 = 0, zm1 = 0;
  int dx = 0, dy = 0, dz = 0;
  if (j < cnt) {
    const uint32_t s = upbase + (a.up_all ? j : a.e2_ent_up[j0 + j]);
    const A sk = (A)skey[s], pk = (A)pkey[p];
    const A X = (A)kAxisX;
    dx = axis_delta<A>(sk, pk, X, (A)1);
    dy = axis_delta<A>(sk, pk, (A)(X << 1), (A)2);
    dz = axis_delta<A>(sk, pk, (A)(X << 2), (A)4);
    m = a.src_mask_up[s];
    cb = a.src_child_up[s] - base;
    // Receiver octants a child with axis bit 0 / 1 is adjacent to, per axis:
    // offset 0: all; +1 (s above p on the axis): a child with bit 0 touches
    // the receivers with bit 1; -1: a child with bit 1 touches the receivers
    // with bit 0. Receivers with the x / y / z bit set: 0xAA / 0xCC / 0xF0.
    xm0 = dx == 0 ? 0xFFu : (dx > 0 ? 0xAAu : 0u);
    xm1 = dx == 0 ? 0xFFu : (dx < 0 ? 0x55u : 0u);
    ym0 = dy == 0 ? 0xFFu : (dy > 0 ? 0xCCu : 0u);
    ym1 = dy == 0 ? 0xFFu : (dy < 0 ? 0x33u : 0u);
    zm0 = dz == 0 ? 0xFFu : (dz > 0 ? 0xF0u : 0u);
    zm1 = dz == 0 ? 0xFFu : (dz < 0 ? 0x0Fu : 0u);
  }
  const uint32_t c = (uint32_t)__popc(m);
  const uint32_t incl = half_incl_scan(c);
  const uint32_t total = __shfl(incl, 31, 32);  // |U| of this half's parent, <= 216
  {
    uint32_t* U = s_rank[h];
    uint8_t* ADJ = s_adj[h];
    const uint32_t pos = incl - c;
#pragma unroll
    for (uint32_t o = 0; o < 8; ++o) {
      if (m & (1u << o)) {
        const uint32_t r = (uint32_t)__popc(m & ((1u << o) - 1u));
        U[pos + r] = cb + r;
        ADJ[pos + r] = (uint8_t)(((o & 1u) ? xm1 : xm0) & ((o & 2u) ? ym1 : ym0) &
                                 ((o & 4u) ? zm1 : zm0));
        if (NEXT) {
          const uint32_t tx = (uint32_t)(2 * dx + 1) + (o & 1u);
          const uint32_t ty = (uint32_t)(2 * dy + 1) + ((o >> 1) & 1u);
          const uint32_t tz = (uint32_t)(2 * dz + 1) + ((o >> 2) & 1u);
          s_off[h][pos + r] = (uint8_t)((tx & 3u) | (ty & 3u) << 2 | (tz & 3u) << 4);
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  // Both parents' U into registers; with NEXT also the child masks of the U
  // entries (global loads, issued before any store).
  uint32_t u[2][4], ad[2], uo[2], um[2], T[2];
#pragma unroll
  for (uint32_t hh = 0; hh < 2; ++hh) {
    T[hh] = (uint32_t)__builtin_amdgcn_readlane(total, 32 * hh);
    const uint32_t* U = s_rank[(h & ~1u) + hh];
    const uint8_t* ADJ = s_adj[(h & ~1u) + hh];
    ad[hh] = uo[hh] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t idx = 64u * k + lane;
      u[hh][k] = idx < T[hh] ? U[idx] : 0u;
      ad[hh] |= (idx < T[hh] ? (uint32_t)ADJ[idx] : 0u) << (8 * k);
      if (NEXT) uo[hh] |= (idx < T[hh] ? (uint32_t)s_off[(h & ~1u) + hh][idx] : 0u) << (8 * k);
    }
  }
  if (NEXT) {
#pragma unroll
    for (uint32_t hh = 0; hh < 2; ++hh) {
      const uint32_t gbase = (uint32_t)__builtin_amdgcn_readlane(base, 32 * hh);
      um[hh] = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (64u * k + lane < T[hh])
          um[hh] |= (uint32_t)a.src_mask_cur[gbase + u[hh][k]] << (8 * k);
    }
  }
  // Split, the whole wave on one parent at a time.
  uint32_t my_n2 = 0;  // NEXT: lane 32 hh + i holds |E2| of child i of parent hh
  uint32_t* E2L = NEXT ? &s_e2[threadIdx.x >> 6][0][0] : nullptr;
#pragma unroll
  for (uint32_t hh = 0; hh < 2; ++hh) {
    const uint32_t n_chunks = (T[hh] + 63u) >> 6;
    uint32_t qm = (uint32_t)__builtin_amdgcn_readlane(rmask, 32 * hh), child = 32 * hh;
#pragma unroll 1
    while (qm) {
      const uint32_t q = __builtin_ctz(qm);
      qm &= qm - 1;
      // next free slot of each list (wave-uniform)
      uint32_t* d2 = ent2 + (uint32_t)__builtin_amdgcn_readlane(my_o2, child);
      uint32_t* d4 = ent4 + (uint32_t)__builtin_amdgcn_readlane(my_o4, child);
      uint32_t n2r = 0;
      uint32_t* el = NEXT ? E2L + (8 * hh + (child & 7u)) * kE2Max : nullptr;
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        if (k < n_chunks) {
          const uint32_t rem = T[hh] - 64u * k;  // valid lanes: 0 .. rem - 1
          const bool is2 = (ad[hh] >> (8 * k + q)) & 1u;  // 0 on invalid lanes
          const uint64_t b2 = __ballot(is2);
          const uint32_t i2 = mbcnt(b2);
          // E2 lanes go to d2 in order; the other valid lanes (a prefix of
          // the wave minus the E2 lanes) go to d4 in order.
          uint32_t* dst = is2 ? d2 + i2 : d4 + (lane - i2);
          if (lane < rem) *dst = u[hh][k];
          if (NEXT && is2)
            el[n2r + i2] = ((um[hh] >> (8 * k)) & 0xFFu) | ((uo[hh] >> (8 * k)) & 0xFFu) << 8;
          const uint32_t n2 = (uint32_t)__popcll(b2);
          d2 += n2;
          d4 += min(rem, 64u) - n2;
          n2r += n2;
        }
      }
      if (NEXT && lane == child) my_n2 = n2r;
      ++child;
    }
  }
  if (NEXT) {
    __builtin_amdgcn_wave_barrier();
    // Lane 8 i + q': receiver child i of each parent in turn, octant q' of
    // its children.
    const uint32_t i = lane >> 3, qq = lane & 7u;
    const uint32_t qx = qq & 1u, qy = (qq >> 1) & 1u, qz = (qq >> 2) & 1u;
#pragma unroll
    for (uint32_t hh = 0; hh < 2; ++hh) {
      const uint32_t pm = (uint32_t)__builtin_amdgcn_readlane(rmask, 32 * hh);
      const bool nz = __builtin_amdgcn_readlane(next_zero ? 1 : 0, 32 * hh) != 0;
      const uint32_t rm = (uint32_t)__shfl(my_rm, 32 * hh + i);
      const uint32_t rc = (uint32_t)__shfl(my_rc, 32 * hh + i);
      const uint32_t n2 = (uint32_t)__shfl(my_n2, 32 * hh + i);
      if (i < (uint32_t)__popc(pm) && ((rm >> qq) & 1u)) {
        uint32_t mm = pm;
        for (uint32_t t = 0; t < i; ++t) mm &= mm - 1;
        const uint32_t q = (uint32_t)__builtin_ctz(mm);  // octant of r
        // Per axis, the children of u adjacent to r's child q' for offsets
        // -1, 0, +1 of u from r, in bytes 0, 1, 2 (offset -1: u's children
        // with the bit set, if q' has it clear; +1: those with it clear, if
        // q' has it set), shifted up one byte when r's own axis bit is 1, so
        // that byte t - 1 is the mask.
        const uint32_t Wx = ((qx ? 0u : 0xAAu) | 0xFF00u | (qx ? 0x55u : 0u) << 16) << (8 * (q & 1u));
        const uint32_t Wy = ((qy ? 0u : 0xCCu) | 0xFF00u | (qy ? 0x33u : 0u) << 16)
                            << (8 * ((q >> 1) & 1u));
        const uint32_t Wz = ((qz ? 0u : 0xF0u) | 0xFF00u | (qz ? 0x0Fu : 0u) << 16)
                            << (8 * ((q >> 2) & 1u));
        const uint32_t* el = E2L + (8 * hh + i) * kE2Max;
        uint32_t c_all = 0, c2 = 0;
        for (uint32_t e = 0; e < n2; ++e) {
          const uint32_t v = el[e];
          const uint32_t adj = __builtin_amdgcn_ubfe(Wx, ((v >> 8) & 3u) * 8, 8) &
                               __builtin_amdgcn_ubfe(Wy, ((v >> 10) & 3u) * 8, 8) &
                               __builtin_amdgcn_ubfe(Wz, ((v >> 12) & 3u) * 8, 8);
          c_all += (uint32_t)__popc(v & 0xFFu);
          c2 += (uint32_t)__popc(v & adj);
        }
        const uint32_t slot = rc + (uint32_t)__popc(rm & ((1u << qq) - 1u));
        a.cnt2_next[slot] = nz ? 0u : c2;
        a.cnt4_next[slot] = nz ? 0u : c_all - c2;
      }
    }
  }
}

void launch_list_count(bool key64, const ListLevelArgs& a, uint32_t* cnt2, uint32_t* cnt4,
                       hipStream_t s) {
  if (a.n_recv_up == 0) return;  // with n_recv_up_dev: the capacity
  const uint32_t grid = div_up(a.n_recv_up, 8);
  const bool narrow = a.key_bits_up <= 32;  // parent-level keys fit 32 bits
  if (key64 && narrow)
    hipLaunchKernelGGL((k_list_count<uint64_t, uint32_t>), dim3(grid), dim3(256), 0, s, a, cnt2,
                       cnt4);
  else if (key64)
    hipLaunchKernelGGL((k_list_count<uint64_t, uint64_t>), dim3(grid), dim3(256), 0, s, a, cnt2,
                       cnt4);
  else
    hipLaunchKernelGGL((k_list_count<uint32_t, uint32_t>), dim3(grid), dim3(256), 0, s, a, cnt2,
                       cnt4);
}

template <bool NEXT>
static void list_fill(bool key64, const ListLevelArgs& a, const uint32_t* off2,
                      const uint32_t* off4, uint32_t* ent2, uint32_t* ent4, hipStream_t s) {
  const uint32_t grid = div_up(a.n_recv_up, 8);
  const bool narrow = a.key_bits_up <= 32;
  if (key64 && narrow)
    hipLaunchKernelGGL((k_list_fill<uint64_t, uint32_t, NEXT>), dim3(grid), dim3(256), 0, s, a,
                       off2, off4, ent2, ent4);
  else if (key64)
    hipLaunchKernelGGL((k_list_fill<uint64_t, uint64_t, NEXT>), dim3(grid), dim3(256), 0, s, a,
                       off2, off4, ent2, ent4);
  else
    hipLaunchKernelGGL((k_list_fill<uint32_t, uint32_t, NEXT>), dim3(grid), dim3(256), 0, s, a,
                       off2, off4, ent2, ent4);
}

void launch_list_fill(bool key64, const ListLevelArgs& a, const uint32_t* off2,
                      const uint32_t* off4, uint32_t* ent2, uint32_t* ent4, hipStream_t s) {
  if (a.n_recv_up == 0) return;
  if (a.cnt2_next) list_fill<true>(key64, a, off2, off4, ent2, ent4, s);
  else list_fill<false>(key64, a, off2, off4, ent2, ent4, s);
}

// ---------------------------------------------------------------------------
// Exclusive scans of the per-box E2 and E4 list lengths into CSR offsets (the
// scan that turns NumRecvE2NeiNEBox into NeighborBookmark, Algorithm 4), both
// in one single pass. off[n] = total; the totals also go to total[0..1], and
// the overflow flag is set if a total does not fit 32-bit offsets. Wave 0
// chains the E2 sums across tiles, wave 1 the E4 sums, at the same time.
// Each thread owns 16 consecutive boxes, read and written with 16-byte
// accesses (both count arrays and both offset arrays start 16-byte aligned).
// ---------------------------------------------------------------------------
// 1024 threads x 16 counts per tile: a quarter of the tiles (and of the
// look-back chain) of 256-thread tiles; the largest scan (10.6M boxes) took
// 98 us with 4096-count tiles.
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;  // 16384 boxes

__global__ __launch_bounds__(kScanBlock) void k_scan_counts2(
    const uint32_t* __restrict__ cnt2, const uint32_t* __restrict__ cnt4, uint32_t n_host,
    const uint32_t* __restrict__ n_dev, uint32_t* __restrict__ off2, uint32_t* __restrict__ off4,
    uint64_t* __restrict__ total2, uint64_t* __restrict__ total4, uint32_t* __restrict__ overflow,
    uint64_t* __restrict__ status2, uint64_t* __restrict__ status4,
    uint32_t* __restrict__ tile_counter) {
  __shared__ uint32_t s_w[2][kScanBlock / 64];
  __shared__ uint64_t s_excl[2];
  __shared__ uint32_t s_tile;
  const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint32_t n = n_dev ? *n_dev : n_host;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  if ((uint64_t)tile * kScanTile >= n) return;  // whole block: surplus tile
  const uint64_t base = (uint64_t)tile * kScanTile + (uint64_t)tid * kScanItems;
  uint32_t v2[kScanItems], v4[kScanItems];
  const bool full = base + kScanItems <= n;  // 16-byte loads and stores
  if (full) {
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
      const uint4 a2 = ((const uint4*)(cnt2 + base))[q];
      const uint4 a4 = ((const uint4*)(cnt4 + base))[q];
      v2[4 * q] = a2.x, v2[4 * q + 1] = a2.y, v2[4 * q + 2] = a2.z, v2[4 * q + 3] = a2.w;
      v4[4 * q] = a4.x, v4[4 * q + 1] = a4.y, v4[4 * q + 2] = a4.z, v4[4 * q + 3] = a4.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const bool ok = base + i < n;
      v2[i] = ok ? cnt2[base + i] : 0;
      v4[i] = ok ? cnt4[base + i] : 0;
    }
  }
  uint32_t sum2 = 0, sum4 = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    sum2 += v2[i];
    sum4 += v4[i];
  }
  const uint32_t inc2 = wave_incl_scan(sum2), inc4 = wave_incl_scan(sum4);
  if (lane == 63) {
    s_w[0][w] = inc2;
    s_w[1][w] = inc4;
  }
  __syncthreads();
  uint32_t wpre2 = 0, wpre4 = 0, tot2 = 0, tot4 = 0;
  for (uint32_t i = 0; i < kScanBlock / 64; ++i) {
    if (i < w) {
      wpre2 += s_w[0][i];
      wpre4 += s_w[1][i];
    }
    tot2 += s_w[0][i];
    tot4 += s_w[1][i];
  }
  if (w == 0) {
    const uint64_t ex = lookback_wave(status2, tile, tot2);
    if (lane == 0) s_excl[0] = ex;
  } else if (w == 1) {
    const uint64_t ex = lookback_wave(status4, tile, tot4);
    if (lane == 0) s_excl[1] = ex;
  }
  __syncthreads();
  uint64_t pre2 = s_excl[0] + wpre2 + inc2 - sum2;
  uint64_t pre4 = s_excl[1] + wpre4 + inc4 - sum4;
  bool ovf = false;
  if (full) {
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
      uint4 o2, o4;
      o2.x = (uint32_t)pre2, pre2 += v2[4 * q], o4.x = (uint32_t)pre4, pre4 += v4[4 * q];
      o2.y = (uint32_t)pre2, pre2 += v2[4 * q + 1], o4.y = (uint32_t)pre4, pre4 += v4[4 * q + 1];
      o2.z = (uint32_t)pre2, pre2 += v2[4 * q + 2], o4.z = (uint32_t)pre4, pre4 += v4[4 * q + 2];
      o2.w = (uint32_t)pre2, pre2 += v2[4 * q + 3], o4.w = (uint32_t)pre4, pre4 += v4[4 * q + 3];
      ((uint4*)(off2 + base))[q] = o2;
      ((uint4*)(off4 + base))[q] = o4;
    }
    if (base + kScanItems == n) {
      off2[n] = (uint32_t)pre2;
      off4[n] = (uint32_t)pre4;
      *total2 = pre2;
      *total4 = pre4;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < n) {
        off2[base + i] = (uint32_t)pre2;
        off4[base + i] = (uint32_t)pre4;
        pre2 += v2[i];
        pre4 += v4[i];
        if (base + i + 1 == n) {
          off2[n] = (uint32_t)pre2;
          off4[n] = (uint32_t)pre4;
          *total2 = pre2;
          *total4 = pre4;
        }
      }
    }
  }
  ovf = (pre2 > 0xFFFFFFFFull) || (pre4 > 0xFFFFFFFFull);
  if (ovf) atomicOr(overflow, 1u);
}

uint32_t scan_tiles(uint32_t n) { return div_up(n, kScanTile); }

void launch_scan_counts2(const uint32_t* cnt2, const uint32_t* cnt4, uint32_t n, uint32_t* off2,
                         uint32_t* off4, uint64_t* total2, uint64_t* total4, uint32_t* overflow,
                         uint64_t* status2, uint64_t* status4, uint32_t* tile_counter,
                         hipStream_t s, const uint32_t* n_dev) {
  // n is the exact count, or with n_dev the capacity (the count is read there)
  if (n == 0) return;
  hipLaunchKernelGGL(k_scan_counts2, dim3(scan_tiles(n)), dim3(kScanBlock), 0, s, cnt2, cnt4, n,
                     n_dev, off2, off4, total2, total4, overflow, status2, status4, tile_counter);
}

}  // namespace fmmds
