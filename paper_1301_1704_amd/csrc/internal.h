// Host-side declarations shared by the translation units of libfmmds.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fmmds.h"

namespace fmmds {

constexpr int kMaxLevel = 21;
constexpr int kMaxPasses = 8;  // 63 key bits / 8-bit digits

// Tile shapes of the single-pass kernels.
constexpr int kSortBlock = 256;
// Sort tile sizes, in units of 256 elements: 8, 12 and 16 are tiles of
// 256 threads with that many elements each; kSortWide is a tile of 8192
// elements (512 threads x 16), for packed elements only.
constexpr int kSortItemsDefault = 16;
constexpr int kSortWide = 32;
constexpr int kCompBlock = 256;
constexpr int kCompItems = 8;
constexpr int kCompTile = kCompBlock * kCompItems;  // 2048 elements

inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Small per-build block in device memory, zeroed at the start of a build and
// read back by the host at its synchronization points.
struct DevMeta {
  uint32_t err_range;
  uint32_t overflow;
  uint32_t n_boxes[2][kMaxLevel + 1];
  uint32_t max_occ[2][kMaxLevel + 1];
  uint64_t list_total[2][kMaxLevel + 1];  // [0] = E2, [1] = E4
  uint32_t inc_counts[2][2];              // incremental rebuild: stayers, movers per set
  uint32_t dense_big[2];                  // dense variant: finest boxes ordered by blocks
};

// Sort elements: with `packed`, one uint64 holding (key << 32 | index) for keys
// of at most 32 bits; otherwise a uint64 key array plus a uint32 index array.
struct SortBufs {
  uint64_t* k[2];
  uint32_t* v[2];
};

// ---- sort.hip
void launch_zero(void* p, size_t bytes, hipStream_t s);
// Keys and the sort elements (key, index) of n points, and per block of the
// launch (keygen_blocks(n) of them) one row of n_pass x 256 digit counts.
uint32_t keygen_blocks(uint32_t n);
void launch_keygen(const float* xyz, uint32_t n, uint32_t L, bool packed, uint64_t* keys,
                   uint32_t* vals, uint32_t n_pass, uint32_t* rows, uint32_t* err, hipStream_t s);
// Those rows added into the pass histograms hist (zeroed, n_pass x 256).
void launch_reduce_rows(const uint32_t* rows, uint32_t n_rows, uint32_t* hist, uint32_t n_pass,
                        hipStream_t s);
void launch_digit_offsets(const uint32_t* hist, uint32_t* goff, uint32_t n_pass, hipStream_t s);
uint32_t sort_tile_elems(int items);
uint32_t sort_tiles(uint32_t n, int items);
// Many point sets sorted at once, each within its own range: tile t covers
// elements [start[t], start[t + 1]) of set set[t] & 0x7FFFFFFF, never more
// than one set (the top bit marks a set's first tile); goff holds, per set
// and pass, where each digit's run starts (the set's first element included),
// n_sets x n_pass x 256.
struct SegSort {
  const uint32_t* start;
  const uint32_t* set;
  const uint32_t* goff;
  uint32_t n_tiles, n_pass, pass;
};
void launch_sort_pass(bool packed, const uint64_t* kin, uint64_t* kout, const uint32_t* vin,
                      uint32_t* vout, uint32_t n, uint32_t shift, const uint32_t* goff,
                      uint64_t* status, uint32_t* tile_counter, hipStream_t s, int items,
                      const uint32_t* n_dev = nullptr);  // n_dev: count on the device, n = capacity
void launch_sort_pass_seg(bool packed, const uint64_t* kin, uint64_t* kout, const uint32_t* vin,
                          uint32_t* vout, uint32_t shift, const SegSort& sg, uint64_t* status,
                          uint32_t* tile_counter, hipStream_t s, int items);

// ---- tables.hip
void launch_leaf(bool packed, bool key64, const uint64_t* sk, const uint32_t* sv,
                 const float* xyz, uint32_t n, uint32_t* perm, float* sorted_xyz, void* leaf_key,
                 uint32_t* leaf_begin, uint64_t* status, uint32_t* tile_counter, uint32_t* n_out,
                 hipStream_t s);
// Every level's tables in one pass over the sorted points (plain build and
// rebuild): phase 0 counts box starts per tile and level (cnt: (L + 1) x
// tab_tiles(n)), 1 scans them (pre, same shape; n_boxes[l] = boxes of level
// l), 2 writes permutation, coordinates, keys, bookmarks, parents and first
// children, 3 the child masks (mask_cap: capacity of level L - 1). With
// set_off (a batch), keys carry the set id from bit set_shift up and the
// permutation is written relative to each set's first point.
struct TabLevels {
  void* key[kMaxLevel + 1];
  uint32_t* begin[kMaxLevel + 1];
  uint32_t* parent[kMaxLevel + 1];
  uint32_t* child[kMaxLevel + 1];
  uint8_t* mask[kMaxLevel + 1];
};
uint32_t tab_tiles(uint32_t n);
void launch_tables(bool packed, bool key64, const uint64_t* sk, const uint32_t* sv,
                   const float* xyz, uint32_t n, uint32_t L, uint32_t* cnt, uint32_t* pre,
                   const TabLevels& T, uint32_t* perm, float* sorted_xyz, uint32_t* n_boxes,
                   uint32_t mask_cap, hipStream_t s, int phase,
                   const uint64_t* set_off = nullptr, uint32_t set_shift = 0);
void launch_max_occupancy(const uint32_t* begin, const uint32_t* n_in, uint32_t cap,
                          uint32_t* out, hipStream_t s);

// ---- lists.hip
struct ListLevelArgs {
  uint32_t level;               // lists are built for receiver boxes of this level
  uint32_t n_recv_up;           // receiver boxes at level - 1 (the parents)
  const void* recv_key_up;      // level - 1 receiver keys
  const uint8_t* recv_mask_up;  // level - 1 receiver child masks
  const uint32_t* recv_child_up;// level - 1 receiver first children
  const void* src_key_up;       // level - 1 source keys
  const uint8_t* src_mask_up;   // level - 1 source child masks
  const uint32_t* src_child_up; // level - 1 source first children
  const uint32_t* e2_off_up;    // E2 lists at level - 1 (unused when up_all)
  const uint32_t* e2_ent_up;
  uint32_t up_all;              // level - 1 == 1: E2 there is every source box
  uint32_t n_src_up;            // source boxes at level - 1
  // Batch only (first_up == nullptr otherwise): keys carry the set id from
  // bit 3 * (level - 1) up (at level - 1); a set's boxes at a level occupy
  // ranks [first[set], first[set + 1]); sets shallower than `level` get empty
  // lists; entries are written relative to first_cur[set].
  const uint32_t* first_up;     // level - 1
  const uint32_t* first_cur;    // level
  const uint8_t* set_level;     // per set
  uint32_t key_bits_up;         // bits of the level - 1 keys including the set id
  const uint32_t* n_recv_up_dev;// if set, the parent count is read here and
                                // n_recv_up is only the capacity
  const uint32_t* n_src_up_dev; // if set (up_all), the level - 1 source count
  // Fill only: with cnt2_next set, the fill also writes the E2 / E4 counts of
  // the receiver boxes of level + 1 (what the count kernel would compute
  // there), from the lists it builds for their parents.
  const uint8_t* src_mask_cur;   // level source child masks
  const uint8_t* recv_mask_cur;  // level receiver child masks
  const uint32_t* recv_child_cur;// level receiver first children
  uint32_t* cnt2_next;
  uint32_t* cnt4_next;
};
void launch_list_count(bool key64, const ListLevelArgs& a, uint32_t* cnt2, uint32_t* cnt4,
                       hipStream_t s);
void launch_list_fill(bool key64, const ListLevelArgs& a, const uint32_t* off2,
                      const uint32_t* off4, uint32_t* ent2, uint32_t* ent4, hipStream_t s);
uint32_t scan_tiles(uint32_t n);
void launch_scan_counts2(const uint32_t* cnt2, const uint32_t* cnt4, uint32_t n, uint32_t* off2,
                         uint32_t* off4, uint64_t* total2, uint64_t* total4, uint32_t* overflow,
                         uint64_t* status2, uint64_t* status4, uint32_t* tile_counter,
                         hipStream_t s, const uint32_t* n_dev = nullptr);

// ---- rebuild.hip
void launch_inc_classify(const float* xyz, const float* old_xyz, const uint32_t* old_perm,
                         uint32_t n, uint32_t L, uint32_t ib, uint32_t n_pass, uint64_t* st_v,
                         uint32_t* st_slot, uint64_t* mv_v, uint32_t* mv_slot, uint32_t* hist,
                         uint32_t* err, uint64_t* status, uint32_t* tile_counter,
                         uint32_t* counts, hipStream_t s);  // xyz in the previous sorted order  // staged: 3 n floats, written unless prev_order
void launch_inc_scatter(const float* xyz, const uint32_t* old_perm, uint32_t n, float* out,
                        hipStream_t s);
void launch_inc_merge(bool packed, const uint64_t* st_v, const uint32_t* st_slot, uint32_t ns,
                      const uint64_t* mv_v, const uint32_t* mv_slot, uint32_t nm,
                      const float* xyz, uint32_t ib, uint64_t* sk, uint32_t* sv,
                      float* sorted_xyz, hipStream_t s);  // xyz indexed by slot

// ---- dense.hip (the dense-histogram variant, max level <= 8)
constexpr uint32_t kDenseMaxLevel = 8;
constexpr uint32_t kDenseCanonMax = 4096;  // largest finest box put in order on the device
void launch_dense_count(const float* xyz, uint32_t n, uint32_t L, uint32_t* bin, uint32_t* key,
                        uint32_t* rank, uint32_t* err, hipStream_t s);
void launch_dense_reduce(const uint32_t* fine, uint32_t n_coarse, uint32_t* coarse,
                         hipStream_t s);
uint32_t dense_scan_tiles(uint32_t nbox);
void launch_dense_scan(bool key64, const uint32_t* bin, uint32_t nbox, uint32_t* sbin,
                       uint32_t* srank, void* keys, uint32_t* begin, uint32_t* n_out,
                       uint32_t* max_occ, uint64_t* status, uint32_t* tile_counter,
                       hipStream_t s);
void launch_dense_links(bool key64, const void* keys, const uint32_t* n_p, uint32_t cap,
                        const uint32_t* bin_fine, const uint32_t* srank_fine,
                        const uint32_t* n_fine_p, uint32_t* child, uint8_t* mask,
                        const void* keys_fine, uint32_t cap_fine, uint32_t* parent_fine,
                        const uint32_t* srank, hipStream_t s);
void launch_dense_order(const uint32_t* key, const uint32_t* rank, uint32_t n,
                        const uint32_t* sbin, const uint32_t* begin, const uint32_t* n_boxes,
                        uint32_t cap_boxes, uint32_t* tmp, uint32_t* perm, uint32_t* big,
                        uint32_t* n_big, const float* xyz, float* sorted_xyz, hipStream_t s);
void launch_dense_lists(bool key64, bool fill, uint32_t l, uint32_t n_up, const void* rkey_up,
                        const uint8_t* rmask_up, const uint32_t* rchild_up,
                        const uint32_t* bin_up, const uint32_t* bin_cur,
                        const uint32_t* srank_cur, uint32_t* cnt2, uint32_t* cnt4,
                        const uint32_t* off2, const uint32_t* off4, uint32_t* ent2,
                        uint32_t* ent4, hipStream_t s);  // n_up: receiver boxes of level l - 1

// ---- batch.hip kernels
struct LevelPtrs {
  const uint32_t* begin[kMaxLevel + 1];
};
// Composite keys of a batch, one block per tile of a set-aligned table of
// 8192-element tiles (SegSort's start and set), and each set's digit counts
// of the n_pass sort passes added into hist (zeroed, n_sets x n_pass x 256).
void launch_batch_keygen(const float* xyz, const uint32_t* tile_start, const uint32_t* tile_set,
                         uint32_t n_tiles, const uint8_t* set_level, uint32_t L_all, bool packed,
                         uint64_t* keys, uint32_t* vals, uint32_t n_pass, uint32_t* hist,
                         uint32_t* err, hipStream_t s);
// goff[(i * n_pass + p) * 256 + d] = set_off[i] + the points of set i whose
// pass-p digit is below d.
void launch_batch_digit_offsets(const uint32_t* hist, const uint64_t* set_off, uint32_t n_sets,
                                uint32_t n_pass, uint32_t* goff, hipStream_t s);
void launch_batch_first(const LevelPtrs& lp, uint32_t L_all, const uint32_t* n_boxes,
                        const uint64_t* set_off, uint32_t n_sets, uint32_t* first, hipStream_t s);
struct RebaseArgs {  // every level 0..L of a batch
  const uint32_t* n_l[kMaxLevel + 1];
  const uint64_t* gkey[kMaxLevel + 1];
  const uint32_t* gbegin[kMaxLevel + 1];
  const uint32_t* gparent[kMaxLevel + 1];  // nullptr at level 0
  const uint32_t* gchild[kMaxLevel + 1];   // nullptr at level L
  uint64_t* fkey[kMaxLevel + 1];
  uint32_t* fbegin[kMaxLevel + 1];
  uint32_t* fparent[kMaxLevel + 1];
  uint32_t* fchild[kMaxLevel + 1];
  const uint32_t* first;  // first[l * (n_sets + 1) + i]
  const uint64_t* set_off;
  uint32_t n_sets, L;
};
void launch_batch_rebase(const RebaseArgs& a, uint32_t max_cap, hipStream_t s);
struct ListRebaseArgs {  // levels 2..L of a batch
  const uint32_t* n_l[kMaxLevel + 1];
  const uint64_t* gkey[kMaxLevel + 1];
  const uint32_t* goff2[kMaxLevel + 1];
  const uint32_t* goff4[kMaxLevel + 1];
  uint32_t* loff2[kMaxLevel + 1];
  uint32_t* loff4[kMaxLevel + 1];
  const uint32_t* first;
  uint32_t* base;  // base[(2l + k) * (n_sets + 1) + i], k = 0 (E2) or 1 (E4)
  uint32_t n_sets, L;
};
void launch_batch_list_rebase(const ListRebaseArgs& a, uint32_t max_cap, hipStream_t s);

// ---- displace.hip
constexpr uint32_t kDisplaceSets = 32;  // systems per launch (kernel-argument struct)
struct DisplaceArgs {
  float* xyz[kDisplaceSets];
  uint64_t seed[kDisplaceSets];
  uint64_t first[kDisplaceSets + 1];  // prefix of point counts; first[n] = total
  uint64_t out_first[kDisplaceSets];
  uint32_t n;
};
void launch_displace(const DisplaceArgs& a, float sigma, float* out, hipStream_t s);

// ---- boxtypes.hip
struct BoxTypeLevel {
  uint32_t level, l_par, rank;
  uint32_t n_recv, n_src;       // nonempty boxes of the level
  const void* rkey;             // level keys (uint32 or uint64)
  const void* skey;
  const void* rkey_par;         // critical level: keys of the l_par level
  const void* skey_par;
  const uint32_t* rchild;       // critical level: first children (n + 1)
  const uint32_t* schild;
  const uint32_t* owner;        // rank of every Morton index of l_par
  const uint32_t* e4_off;       // the level's E4 lists
  const uint32_t* e4_ent;
  uint8_t* elsewhere;           // n_src marks "needed by another rank", zeroed
  uint8_t* here;                // n_src marks "needed by this rank", zeroed
  uint32_t* work;               // n_recv slots: receivers that read their lists
  uint32_t* n_work;             // their count, zeroed
  uint8_t* types;               // n_src outputs
};
void launch_partition(bool key64, const void* rkey, const uint32_t* rbegin, uint32_t n_boxes,
                      uint32_t n_points, uint32_t n_ranks, uint32_t l_par, uint32_t* owner,
                      hipStream_t s);
void launch_fill_u8(uint8_t* p, uint32_t n, uint8_t v, hipStream_t s);
void launch_types_crit(bool key64, const BoxTypeLevel& a, hipStream_t s);
void launch_types_deep(bool key64, const BoxTypeLevel& a, hipStream_t s);

// ---- nearfield.hip
// Receiver boxes of more than kNearDenseMin points go to the dense path.
constexpr uint32_t kNearDenseMin = 8;
constexpr uint32_t kNearCounters = 2;
uint64_t near_field_max_tasks(uint32_t n_recv);  // dense-path tasks for n_recv receivers
// Bytes of the fixed scratch array of the near-field entry point that
// allocates nothing, and its device address on the current device (looked up
// once per device). The status is an fmmds_status.
constexpr size_t kNearStaticBytes = FMMDS_NEAR_FIELD_STATIC_BYTES;
fmmds_status near_field_static_scratch(void** out);
void launch_pack_sources(const float* sxyz, const uint32_t* sperm, const float* charges,
                         uint32_t n, float4* out, uint32_t* counters, hipStream_t s);
void launch_near_field(uint32_t n_rbox, uint32_t n_recv, const uint32_t* rbegin,
                       const float* rxyz, const uint32_t* rperm, const uint32_t* e2_off,
                       const uint32_t* e2_ent, const uint32_t* sbegin, const float4* src,
                       float* phi, unsigned long long* n_pairs, uint2* tasks,
                       uint32_t* counters, hipStream_t s);

}  // namespace fmmds
