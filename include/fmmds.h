/*
 * fmmds: FMM data-structure construction on AMD Instinct MI355X (gfx950).
 *
 * Builds, on one GPU, the data structures of a multilevel fast multipole
 * method for N source points and M receiver points in the unit cube, as
 * defined by Hu, Gumerov and Duraiswami, "Parallel Algorithms for
 * Constructing Data Structures for Fast Multipole Methods" (arXiv 1301.1704):
 *
 *   - the Morton index of every point's box at the finest level and the
 *     points reordered by it (Section 2.1, Algorithm 1);
 *   - per level, the Morton indices of the nonempty boxes and their bookmarks,
 *     i.e. the first reordered point of each box (Section 2.2; Algorithm 3 in Section 2.3);
 *   - per level, parent and children links (the parent/children queries of
 *     Section 2.4; the parent index is the child index shifted right by one
 *     level, Section 3.2);
 *   - per level 2..depth, for every nonempty receiver box, the E2 neighbor
 *     list (at most 27 nonempty source boxes, Section 1.4 item 2 and
 *     Algorithm 4) and the E4 interaction (M2L) list (at most 189 nonempty
 *     source boxes, Section 1.4 item 4).
 *
 * Conventions (the paper leaves these open):
 *   - level l has 8^l boxes; a box has integer coordinates (cx, cy, cz) in
 *     [0, 2^l)^3 and Morton index with bit b of cx, cy, cz at bit 3b, 3b+1,
 *     3b+2. A point x is in the box floor(x * 2^l) per axis, computed in FP32
 *     (scaling by 2^l is exact). There is no level marker bit.
 *   - points are ordered by (finest-level Morton index, original index), so
 *     the order is deterministic.
 *   - E2 of a box includes the box itself; the domain is not periodic.
 *   - E4(r) = nonempty source boxes s with max_d |c_s - c_r| >= 2 whose
 *     parent is within max_d |p_s - p_r| <= 1 of r's parent.
 *   - list entries are ranks of nonempty source boxes at the same level (the
 *     index into that level's source tables), in ascending order.
 *   - depth: if cluster_s == 0 the depth is max_level. Otherwise it is the
 *     smallest level l in [2, max_level] at which no source box and no
 *     receiver box holds more than cluster_s points (Section 2.1: the cluster
 *     size fixes the finest level), or max_level if no level qualifies.
 *
 * Memory: every pointer passed in or returned is a DEVICE pointer on the
 * current HIP device unless stated otherwise. The caller owns the inputs; the
 * library owns every output until fmmds_free. Errors never throw; on error
 * *out is set to NULL and nothing leaks.
 *
 * Threading: distinct trees are independent; a tree is read-only after
 * fmmds_build returns, so concurrent reads are safe.
 */
#ifndef FMMDS_H
#define FMMDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMMDS_MAX_LEVEL 21 /* 3 * 21 = 63 key bits */

typedef enum fmmds_status {
  FMMDS_OK = 0,
  FMMDS_ERR_ARG = 1,      /* NULL pointer, n == 0, n >= 2^32 - 1, key_bits not 32/64,
                             max_level outside [2, key_bits / 3] */
  FMMDS_ERR_RANGE = 2,    /* a coordinate is NaN, infinite or outside [0, 1) (-0.0 is accepted) */
  FMMDS_ERR_NOMEM = 3,    /* device (or callback) allocation failed */
  FMMDS_ERR_DEVICE = 4,   /* a HIP runtime call failed */
  FMMDS_ERR_LEVEL = 5,    /* list query outside [2, depth] */
  FMMDS_ERR_OVERFLOW = 6, /* a list at one level would hold 2^32 or more entries */
  FMMDS_ERR_TOO_LARGE = 7 /* the input needs more than an entry point's fixed scratch */
} fmmds_status;

/* Optional allocator: return `bytes` of device memory usable on `stream`
 * (a hipStream_t), aligned to 256 bytes, or NULL on failure. `release` gets back exactly the
 * pointers `alloc` returned, with the same byte counts. */
typedef void* (*fmmds_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*fmmds_release_fn)(void* ctx, void* ptr, size_t bytes, void* stream);

typedef struct fmmds_options {
  uint32_t key_bits;   /* 32 or 64: width of the per-level key arrays */
  uint32_t cluster_s;  /* 0: depth = max_level; else the cluster-size rule above */
  uint32_t max_level;  /* finest level considered, in [2, key_bits / 3] */
  uint32_t reserved;   /* must be 0 */
  void* stream;        /* hipStream_t the build is ordered on; NULL = null stream */
  fmmds_alloc_fn alloc;      /* NULL: the library's caching allocator (see fmmds_trim) */
  fmmds_release_fn release;  /* must be set iff alloc is set */
  void* alloc_ctx;
} fmmds_options;

/* One level of one point set. */
typedef struct fmmds_level {
  uint32_t n;              /* number of nonempty boxes */
  const void* key;         /* n Morton indices, ascending; uint32_t* if key_bits == 32,
                              else uint64_t* */
  const uint32_t* begin;   /* n + 1: first reordered point of each box; begin[n] = points */
  const uint32_t* parent;  /* n: rank of the parent at level - 1; NULL at level 0 */
  const uint32_t* child;   /* n + 1: first child rank at level + 1, child[n] = boxes at
                              level + 1; NULL at level == depth */
} fmmds_level;

typedef struct fmmds_tree {
  uint32_t depth;          /* finest level built (lists exist for 2..depth) */
  uint32_t key_bits;
  uint32_t max_level;
  uint32_t shared;         /* 1: receivers are the sources; recv fields alias src */
  uint32_t n_src, n_recv;
  const uint32_t* src_perm;       /* n_src: original index of each reordered source */
  const uint32_t* recv_perm;      /* n_recv */
  const float* src_sorted_xyz;    /* 3 * n_src: src_xyz[perm[k]], bit copies */
  const float* recv_sorted_xyz;   /* 3 * n_recv */
  fmmds_level src[FMMDS_MAX_LEVEL + 1];   /* levels 0..depth are valid */
  fmmds_level recv[FMMDS_MAX_LEVEL + 1];
  void* impl;                     /* private */
} fmmds_tree;

/*
 * Build all tables and lists (Algorithm 5 of the paper, with the lists of
 * Section 2.2 at every level 2..depth).
 *   src_xyz:  device, 3 * n_src FP32 values, (x, y, z) per point.
 *   recv_xyz: device, 3 * n_recv FP32 values, or NULL: receivers are the
 *             sources and n_recv is ignored.
 *   opt:      host, required.
 *   out:      host; receives a tree owned by the library.
 * Returns once the remaining work is enqueued on opt->stream: every output is
 * complete and visible to work later enqueued there (or once the stream is
 * synchronized), and every read of the inputs has completed, so they may be
 * reused or freed at once. Inputs are not retained. With
 * separate receivers, the receivers' sort and tables run on a library-owned
 * stream of the current device (default priority, created on first use and
 * kept until the process ends) and are joined to opt->stream before the
 * lists. Concurrent calls on one device share that stream: their receiver
 * chains run one after another there, each still ordered after its own
 * caller's stream, so results are unaffected. The call waits on the host for
 * the finest level's list sizes (with cluster_s > 0 also for the box counts
 * and occupancies after the tables, which set the depth), so it cannot be
 * captured into a graph (the batched form can).
 */
fmmds_status fmmds_build(const float* src_xyz, uint32_t n_src, const float* recv_xyz,
                         uint32_t n_recv, const fmmds_options* opt, fmmds_tree** out);

/*
 * The same build through the paper's dense-histogram construction (Algorithm
 * 1's per-box occupancy counters with atomic ranks, Algorithm 3's scans of
 * all 8^l boxes per level, and E2 / E4 entries looked up directly in the
 * dense ScannedRank by neighbor coordinates, Algorithm 4), made
 * deterministic: the result is exactly the tree fmmds_build returns for the
 * same arguments. Arguments, ownership and errors as fmmds_build, plus
 * FMMDS_ERR_ARG when opt->max_level exceeds 8 (three dense arrays of 8^l
 * 32-bit counters per level and point set live during the call). A finest
 * box holding more than 4096 points is put in order by a sort instead.
 */
fmmds_status fmmds_build_dense(const float* src_xyz, uint32_t n_src, const float* recv_xyz,
                               uint32_t n_recv, const fmmds_options* opt, fmmds_tree** out);

/*
 * Rebuild after the points moved (the dynamic problems of Section 1, where
 * the structures are rebuilt every time step), reusing the order of a
 * previous tree: only points whose finest-level box changed are sorted, and
 * merged with the others, which are still in order. The result is exactly
 * the tree fmmds_build would return for the same positions and options.
 *   prev:     host; a tree from fmmds_build, fmmds_rebuild or a batch, with
 *             the point counts of this call; read only, and may be freed
 *             once this call returns.
 *   src_xyz:  device, 3 * prev->n_src FP32 values. With in_prev_order == 0,
 *             row j is original point j (as for fmmds_build); with 1, row k
 *             is the point at prev's sorted position k, i.e. original point
 *             prev->src_perm[k] (e.g. prev->src_sorted_xyz after moving).
 *             Only positions in prev's order are rebuilt incrementally: with
 *             in_prev_order == 0 the call builds from scratch (bringing the
 *             positions into prev's order is a random read per point, which
 *             costs more than the sort it would save), with the same result.
 *   recv_xyz: device, 3 * prev->n_recv values in the same order convention,
 *             or NULL iff prev->shared.
 *   opt:      host; max_level must equal prev->max_level (the sort key);
 *             key_bits, cluster_s, stream and allocator are free.
 *   out:      host; receives a new tree owned by the library. The output
 *             permutations map to original indices in both conventions.
 * FMMDS_ERR_ARG for a NULL argument, in_prev_order > 1, a recv_xyz that does
 * not match prev->shared, or another max_level; otherwise the errors of
 * fmmds_build. When the key and index bits together exceed 64 (deep levels
 * with many points) the points are fully sorted instead, with the same result.
 */
fmmds_status fmmds_rebuild(const fmmds_tree* prev, const float* src_xyz, const float* recv_xyz,
                           uint32_t in_prev_order, const fmmds_options* opt, fmmds_tree** out);

/*
 * E2 neighbor list of every nonempty receiver box at `level` in [2, depth]
 * (Section 2.2, NeighborBookmark / NeighborList), as CSR:
 *   *offsets: device, *n_recv_boxes + 1 entries; box j's list is
 *             entries[offsets[j] .. offsets[j+1]).
 *   *entries: device, *n_entries source ranks at `level`, ascending per box.
 * The arrays belong to the tree. FMMDS_ERR_LEVEL outside [2, depth].
 */
fmmds_status fmmds_neighbors(const fmmds_tree* t, uint32_t level, const uint32_t** offsets,
                             const uint32_t** entries, uint32_t* n_recv_boxes,
                             uint64_t* n_entries);

/*
 * E4 interaction (M2L) list of every nonempty receiver box at `level` in
 * [2, depth] (Section 1.4 item 4), same CSR layout as fmmds_neighbors.
 */
fmmds_status fmmds_interactions(const fmmds_tree* t, uint32_t level, const uint32_t** offsets,
                                const uint32_t** entries, uint32_t* n_recv_boxes,
                                uint64_t* n_entries);

/* Release every output of the tree (ordered on the build's stream). NULL is
 * accepted. Pointers obtained from the tree become invalid. */
void fmmds_free(fmmds_tree* t);

/*
 * Batched form: many independent point sets built by one launch sequence.
 * Each set is built as fmmds_build would build it with its points as both
 * sources and receivers, max_level = levels[i], cluster_s = 0 and 64-bit
 * keys; all of its outputs (ranks, bookmarks, permutation, list offsets and
 * entries) are local to the set. Not from the paper: it serves the dynamic
 * problems the paper motivates (Section 1, Eq. (2)), where every time step
 * rebuilds the structures of many particle systems.
 *
 * fmmds_batch_create plans one batch shape and allocates every buffer for
 * the worst case of that shape (no host synchronization is needed later):
 *   set_offsets: host, n_sets + 1 point offsets, set_offsets[0] = 0, strictly
 *                increasing (no empty set), total < 2^32 - 1; n_sets < 2^31.
 *   levels:      host, n_sets max levels in [2, 21].
 *   opt:         host; key_bits must be 64, cluster_s 0; stream and allocator
 *                as for fmmds_build.
 * fmmds_batch_launch enqueues a build of the concatenated coordinates `xyz`
 * (device, 3 * total FP32, set i at points set_offsets[i] ..) on the batch's
 * stream and returns at once. With capture != 0 the first launch records the
 * kernel sequence into a HIP graph and later launches replay it (the input
 * pointer must then stay the same). Before the first graph capture the sort
 * tile size is chosen by timing the candidates (autotuning) on this input.
 * fmmds_batch_wait waits for the launch, checks its status (FMMDS_ERR_RANGE,
 * FMMDS_ERR_OVERFLOW) and fills the per-set views that fmmds_batch_tree
 * returns; the views stay valid until the next launch or fmmds_batch_free, and
 * fmmds_neighbors / fmmds_interactions accept them. fmmds_free ignores them.
 * A batch is used by one host thread at a time.
 */
typedef struct fmmds_batch fmmds_batch;

fmmds_status fmmds_batch_create(const uint64_t* set_offsets, const uint8_t* levels,
                                uint32_t n_sets, const fmmds_options* opt, fmmds_batch** out);
fmmds_status fmmds_batch_launch(fmmds_batch* b, const float* xyz, int capture);
fmmds_status fmmds_batch_wait(fmmds_batch* b);
const fmmds_tree* fmmds_batch_tree(const fmmds_batch* b, uint32_t set);
/* Device bytes a batch of this shape allocates (host only, no device work):
 * for admission by memory footprint before fmmds_batch_create. */
fmmds_status fmmds_batch_footprint(const uint64_t* set_offsets, const uint8_t* levels,
                                   uint32_t n_sets, uint64_t* bytes);
/* Device bytes the batch holds. */
uint64_t fmmds_batch_bytes(const fmmds_batch* b);
/* Sort tile size the batch uses, in units of 256 elements: 8, 12 or 16
 * (tiles of 256 threads with that many elements each) or 32 (8192 elements,
 * 512 threads). A graph capture times the four and keeps the fastest; the
 * environment variable FMMDS_BATCH_SORT_ITEMS, read by fmmds_batch_create,
 * fixes it instead (8, 12, 16, or 32 when max(1, ceil(log2 n_sets)) plus 3
 * times the deepest level is at most 32; other values are ignored). */
uint32_t fmmds_batch_sort_items(const fmmds_batch* b);
void fmmds_batch_free(fmmds_batch* b);

/*
 * The batched form in one call: plan, allocate, build and wait, i.e.
 * fmmds_batch_create, one fmmds_batch_launch without graph capture and
 * fmmds_batch_wait. Arguments as for those calls; xyz is device memory of
 * set_offsets[n_sets] points. On FMMDS_OK *out holds the finished batch:
 * fmmds_batch_tree gives the per-set views, fmmds_free_batch releases it (it
 * may also be launched again like any batch). On error *out is NULL and
 * nothing leaks.
 */
fmmds_status fmmds_build_batch(const float* xyz, const uint64_t* set_offsets,
                               const uint8_t* levels, uint32_t n_sets, const fmmds_options* opt,
                               fmmds_batch** out);
/* Same as fmmds_batch_free. */
void fmmds_free_batch(fmmds_batch* b);

/*
 * Serving support: one time step of moving particle systems, for the
 * dynamic problems the paper motivates (Section 1, Section 2.5), so that a
 * rebuild request runs on the GPU from the step to the lists. Not a step of
 * the paper's build.
 *
 * Every coordinate of every listed system moves by sigma * z, z ~ N(0, 1),
 * and is clamped into [0, 1 - 2^-24] (NaN is left as it is). z is counter
 * based: coordinate d of point i uses output c = 3i + d of the splitmix64
 * stream `seed` (output c = mix(seed + (c + 1) * 0x9E3779B97F4A7C15) with
 * the published mixing constants); u1 = ((h >> 40) + 1) * 2^-24,
 * u2 = ((h >> 16) & 0xFFFFFF) * 2^-24, z = sqrt(-2 ln u1) cos(2 pi u2) in
 * FP32. A system's result therefore does not depend on which other systems
 * share the call.
 *   sets:   host array of n_sets entries; xyz is device memory of n points
 *           (AoS FP32), updated in place; distinct entries must not overlap.
 *   out:    device or NULL; when set, the displaced points of entry k are
 *           also written at points out_first .. out_first + n - 1 of `out`
 *           (so a batch input can be assembled in the same pass).
 *   stream: hipStream_t the work is ordered on (NULL = null stream).
 * Returns at once (asynchronous); FMMDS_ERR_ARG for NULL pointers or n = 0.
 */
typedef struct fmmds_displace_set {
  float* xyz;
  uint64_t n;
  uint64_t seed;
  uint64_t out_first;
} fmmds_displace_set;
fmmds_status fmmds_displace(const fmmds_displace_set* sets, uint32_t n_sets, float sigma,
                            float* out, void* stream);

/*
 * Simulated partition and source box types (Section 3): what one rank of a
 * multi-node run would compute, here for any rank of a partition simulated
 * on one GPU. Both calls read a finished tree (fmmds_build, or a batch view)
 * and enqueue their work on `stream` (a hipStream_t; NULL = null stream),
 * returning at once; the tree must be complete on that stream.
 *
 * fmmds_partition (Section 3.2: consecutive Morton ranges of the partition
 * level l_par, balanced by receiver points): writes the rank of every Morton
 * index of level l_par to owner[0 .. 8^l_par) (device). The nonempty
 * receiver box whose first point is the p-th of the M receiver points (in
 * Morton order) gets rank min(n_ranks - 1, floor(n_ranks * p / M)); every
 * other index takes the rank of the nearest nonempty receiver box before it
 * (rank 0 if none). Needs 3 <= l_par <= min(depth, 10) (FMMDS_ERR_LEVEL)
 * and n_ranks >= 1 (FMMDS_ERR_ARG).
 *
 * fmmds_box_types (Section 3.1, Algorithm 6): the type of every nonempty
 * source box of levels 2..depth as seen by rank `rank`, for any owner table
 * of level l_par (such as fmmds_partition's). `types` (device) holds
 * sum_{l=2..depth} src[l].n bytes, level l after the levels below it.
 * With l_crit = l_par - 1: below l_crit, DOMESTIC. At l_crit: IMPORT if no
 * nonempty source child (at l_par) is on `rank`; ROOT if some are on `rank`
 * and some elsewhere; otherwise EXPORT if a receiver box with a nonempty
 * receiver child elsewhere has the box in its E4 (M2L) list, else DOMESTIC.
 * From l_par down a box is on the rank of its l_par ancestor: on `rank` it is
 * EXPORT if a receiver box of another rank has it in its E4 list, else
 * DOMESTIC; elsewhere it is IMPORT if a receiver box of `rank` has it in its
 * E4 list, else OTHER. Uses a temporary device buffer from the library's
 * cache: 2 bytes per source box and 4 per receiver box of the largest level.
 */
enum {
  FMMDS_BOX_DOMESTIC = 0,
  FMMDS_BOX_EXPORT = 1,
  FMMDS_BOX_IMPORT = 2,
  FMMDS_BOX_ROOT = 3,
  FMMDS_BOX_OTHER = 4
};
fmmds_status fmmds_partition(const fmmds_tree* t, uint32_t l_par, uint32_t n_ranks,
                             uint32_t* owner, void* stream);
fmmds_status fmmds_box_types(const fmmds_tree* t, uint32_t l_par, const uint32_t* owner,
                             uint32_t rank, uint8_t* types, void* stream);

/*
 * Near-field sum, the first consumer of the lists (Algorithm 2 with a
 * Laplace kernel, the direct part of the FMM sum of Section 1.2): for every
 * receiver point y, phi(y) = sum of q_i / |x_i - y| over the source points
 * x_i of the E2 boxes of y's box at the finest level (exactly the points
 * Algorithm 2 gathers), pairs at distance zero left out. FP32 arithmetic.
 *   charges: device, n_src values in the original source order, or NULL
 *            for unit charges.
 *   phi:     device, n_recv values, written in the original receiver order
 *            (through the receiver permutation).
 *   n_pairs: device uint64 or NULL; if set, the number of (receiver, source)
 *            pairs visited (distance-zero pairs included) is added to it.
 *   stream:  hipStream_t the work is ordered on (NULL = null stream); the
 *            tree must be complete on it. Returns at once.
 * Uses a temporary device buffer of 16 bytes per source point (the library's
 * cache). Works on batch views too (all indices set-local).
 */
fmmds_status fmmds_near_field(const fmmds_tree* t, const float* charges, float* phi,
                              uint64_t* n_pairs, void* stream);

/*
 * fmmds_near_field for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, with the scratch (16
 * bytes per source point for the packed sources, 8 bytes per dense-path task,
 * at most one task per 9 receiver points, and 256 bytes of counters, each
 * part rounded up to 256 bytes) in a fixed device array of
 * FMMDS_NEAR_FIELD_STATIC_BYTES instead of memory from the cache. Each GPU
 * the library runs on holds its own array until the process ends; the call
 * allocates nothing. FMMDS_ERR_TOO_LARGE when the scratch would exceed the
 * array (about 3.9 million source points with as many receivers), otherwise
 * arguments and errors as fmmds_near_field. Every call on one GPU uses that
 * GPU's one array and clears what it needs itself: calls that overlap on one
 * GPU (unordered streams or host threads) race and give wrong results.
 */
#define FMMDS_NEAR_FIELD_STATIC_BYTES (64u << 20)
fmmds_status fmmds_near_field_static(const fmmds_tree* t, const float* charges, float* phi,
                                     uint64_t* n_pairs, void* stream);

/* Memory the library allocates itself (opt->alloc == NULL) is cached after
 * release, per device, and reused by later builds of similar size. This call
 * synchronizes every device the cache holds memory of and returns all cached
 * blocks to HIP. Memory of live trees is not affected. */
void fmmds_trim(void);
/* Counters of that cache (host pointers, each may be NULL): allocations
 * served from it, allocations that went to HIP and their bytes, and the bytes
 * it currently holds unused. */
void fmmds_cache_info(uint64_t* hits, uint64_t* misses, uint64_t* miss_bytes,
                      uint64_t* cached_bytes);

/*
 * Diagnostics: per-kernel timing. While enabled, every kernel a build
 * launches is bracketed by HIP events on the stream it runs on; the
 * durations are added, per kernel, to process-wide totals together with the
 * algorithmic bytes of each launch (the reads and writes the method itself
 * needs, independent of caching). A build does not wait for its timings:
 * they are added once its launches have completed, at the latest when
 * fmmds_profile_read or fmmds_profile_reset is called (both wait for the
 * timed launches still pending). Not thread-safe against concurrent builds.
 */
typedef struct fmmds_kernel_stat {
  char name[32];     /* kernel name, e.g. "sort_pass", "list_fill" */
  uint64_t launches;
  double total_ms;   /* summed event-measured durations */
  double bytes;      /* summed algorithmic bytes */
} fmmds_kernel_stat;

/* on != 0 enables timing; `only` = NULL times every kernel, else only the
 * kernel of that name (so a timed run carries two events per launch of one
 * kernel instead of two per launch of every kernel). on == 2 also runs the
 * receivers' chain of fmmds_build on the build stream instead of the
 * library's second stream, so that no two kernels of a build overlap and
 * each measured duration is that kernel's alone (the results are the same). */
void fmmds_profile_enable(int on, const char* only);
void fmmds_profile_reset(void);
/* Copies up to `cap` entries into `out` (host); returns the number of kernels
 * with statistics. */
uint32_t fmmds_profile_read(fmmds_kernel_stat* out, uint32_t cap);

/* Human-readable name of a status code (static string). */
const char* fmmds_status_string(fmmds_status s);

#ifdef __cplusplus
}
#endif
#endif /* FMMDS_H */
