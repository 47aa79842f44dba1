/*
 * fmmds oracle: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU build of the FMM data structures of
 * Hu, Gumerov and Duraiswami, "Parallel Algorithms for Constructing Data
 * Structures for Fast Multipole Methods" (arXiv 1301.1704). It exists so the
 * GPU library can be checked against it; only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it. It shares no code,
 * header or constant with the GPU library.
 *
 * All pointers are host pointers. Coordinates are FP32 xyz triples (array of
 * structs) in the half-open unit cube [0, 1)^3 (Section 1.4 assumes the
 * points are already scaled into the unit cube).
 *
 * Set index: 0 = sources, 1 = receivers. List kind: 2 = E2 (neighbor list,
 * Section 1.4 item 2 and Section 2.2), 4 = E4 (M2L interaction list,
 * Section 1.4 item 4).
 */
#ifndef FMMDS_ORACLE_H
#define FMMDS_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OREF_OK = 0,
  OREF_ERR_ARG = 1,      /* NULL pointer, n == 0, n >= 2^32-1, bad key_bits or max_level */
  OREF_ERR_RANGE = 2,    /* a coordinate is NaN, infinite or outside [0, 1) */
  OREF_ERR_NOMEM = 3,    /* host allocation failed */
  OREF_ERR_LEVEL = 5,    /* list or table query outside the built levels */
  OREF_ERR_OVERFLOW = 6  /* a list at one level has 2^32 or more entries */
};

typedef struct oref_tree oref_tree;

/* Morton keys of n points at level L (key of box containing each point).
 * Returns OREF_ERR_RANGE if any coordinate is outside [0, 1). */
int oref_point_keys(const float* xyz, uint32_t n, uint32_t level, uint64_t* keys_out);

/* Build the tables (and, if with_lists != 0, E2/E4 lists for levels 2..depth).
 * recv == NULL: receivers are the sources (n_recv ignored). */
int oref_build(const float* src, uint32_t n_src, const float* recv, uint32_t n_recv,
               uint32_t key_bits, uint32_t cluster_s, uint32_t max_level, int with_lists,
               oref_tree** out);
void oref_free(oref_tree* t);

uint32_t oref_depth(const oref_tree* t);
uint32_t oref_n_points(const oref_tree* t, int set);
uint32_t oref_n_boxes(const oref_tree* t, int set, uint32_t level);
/* Max points in one box of the level (used by the depth rule). */
uint32_t oref_max_occupancy(const oref_tree* t, int set, uint32_t level);

int oref_perm(const oref_tree* t, int set, uint32_t* out);                 /* n */
int oref_sorted_xyz(const oref_tree* t, int set, float* out);              /* 3n */
int oref_keys(const oref_tree* t, int set, uint32_t level, uint64_t* out); /* n_l */
int oref_begin(const oref_tree* t, int set, uint32_t level, uint32_t* out);/* n_l + 1 */
int oref_parent(const oref_tree* t, int set, uint32_t level, uint32_t* out);/* n_l, level >= 1 */
int oref_child(const oref_tree* t, int set, uint32_t level, uint32_t* out); /* n_l + 1, level < depth */

/* Whole lists (built with with_lists != 0). */
int oref_list_sizes(const oref_tree* t, int kind, uint32_t level, uint32_t* n_recv_boxes,
                    uint64_t* n_entries);
int oref_list(const oref_tree* t, int kind, uint32_t level, uint32_t* offsets, uint32_t* entries);

/* One receiver box's list, computed on demand from the definition; entries
 * must hold 189. Returns the entry count, or minus a status code. */
int oref_box_list(const oref_tree* t, int kind, uint32_t level, uint32_t recv_box,
                  uint32_t* entries);

/* Lists of the receiver boxes [r0, r1) of one level, from the same
 * definition, without building every list of the tree (complete checks of
 * large builds, a range at a time). A lookup holds the level's source-box
 * membership table; it reads the tree, which must outlive it, and any number
 * of threads may query one lookup at once.
 *   offsets: r1 - r0 + 1 values, relative to box r0 (offsets[0] = 0);
 *   entries: room for 27 (E2) or 189 (E4) entries per box.
 * oref_lookup_open returns NULL for a level outside [2, depth] or when out of
 * memory. */
typedef struct oref_lookup oref_lookup;
oref_lookup* oref_lookup_open(const oref_tree* t, uint32_t level);
void oref_lookup_close(oref_lookup* lk);
int oref_list_range(const oref_lookup* lk, int kind, uint32_t r0, uint32_t r1,
                    uint32_t* offsets, uint32_t* entries);

/* Simulated partition (Section 3.2): the rank owning every Morton index of
 * level l_par (dense, 8^l_par entries), consecutive Morton ranges balanced
 * by receiver points. Needs 3 <= l_par <= depth. */
int oref_partition(const oref_tree* t, uint32_t l_par, uint32_t n_ranks, uint32_t* owner_out);

/* Source box types of rank `rank` (Section 3.1, Algorithm 6) for levels
 * 2..depth, concatenated: DOMESTIC 0, EXPORT 1, IMPORT 2, ROOT 3, OTHER 4.
 * `owner`: 8^l_par ranks as from oref_partition. */
int oref_box_types(const oref_tree* t, uint32_t l_par, const uint32_t* owner, uint32_t rank,
                   uint8_t* types_out);

/* Near-field sum (Algorithm 2 with a Laplace kernel): for every receiver
 * point y, in original order, phi[y] = sum of q_i / |x_i - y| over the source
 * points of the E2 boxes of y's box at the finest level (pairs at distance 0
 * left out) and abs_sum[y] = the same with |q_i|; FP64. charges: n_src, in
 * original source order, or NULL for unit charges. Needs with_lists. */
int oref_near_field(const oref_tree* t, const float* charges, double* phi, double* abs_sum);

/* The same for one receiver point (original index j), from the definition
 * without lists (for sampled checks of large builds). */
int oref_near_field_one(const oref_tree* t, const float* charges, uint32_t j, double* phi,
                        double* abs_sum);

/* The type of one source box, from the definition without lists (for
 * sampled checks of large builds). Returns the type or minus a status. */
int oref_box_type_one(const oref_tree* t, uint32_t l_par, const uint32_t* owner, uint32_t rank,
                      uint32_t level, uint32_t box);

#ifdef __cplusplus
}
#endif
#endif
