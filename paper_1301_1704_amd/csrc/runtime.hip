// Host orchestration of fmmds_build and the rest of the C ABI (include/fmmds.h).
//
// One build enqueues, per point set, on the caller's stream:
//   keygen + digit histograms -> radix passes -> permute + leaf compaction ->
//   levels max_level-1 .. 0 (+ occupancy maxima when the depth rule is on),
// then reads a small metadata block back (box counts, range flag, maxima),
// chooses the depth, and builds the lists level by level: count, scan, read
// the list totals back, allocate exactly, fill. All compute runs in the HIP
// kernels of sort.hip, tables.hip and lists.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <tuple>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "../../include/fmmds.h"
#include "internal.h"

namespace fmmds {
namespace {

struct Fail {
  fmmds_status st;
};

inline void ck(hipError_t e) {
  if (e != hipSuccess) throw Fail{FMMDS_ERR_DEVICE};
}
inline void ck_launch() { ck(hipGetLastError()); }

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Caching device allocator. Builds allocate and release the same sizes over
// and over (rebuilds of moving particles, benchmark loops), and a round trip
// through the HIP allocator costs tens to hundreds of microseconds. Released
// blocks stay cached per device and are handed out again for a request of at
// least half the block's size. A block released on stream S
// may still be used by work queued on S: it is reused at once on S (stream
// order protects it); another stream first waits on an event recorded on S at
// release time. fmmds_trim returns every cached block to HIP.
// ---------------------------------------------------------------------------
// An event shared by the blocks released together; destroyed with the last.
struct SharedEvent {
  hipEvent_t ev = nullptr;
  ~SharedEvent() {
    if (ev) (void)hipEventDestroy(ev);
  }
};
using EventRef = std::shared_ptr<SharedEvent>;

EventRef record_event(hipStream_t stream) {
  EventRef e = std::make_shared<SharedEvent>();
  if (hipEventCreateWithFlags(&e->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(e->ev, stream) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(stream);  // no event: make the block safe now
    if (e->ev) (void)hipEventDestroy(e->ev);
    e->ev = nullptr;
  }
  return e;
}

struct CachedBlock {
  void* p;
  size_t bytes;
  hipStream_t stream;
  EventRef ready;  // completes when the releasing stream is done with the block
};
std::mutex g_cache_mu;
uint64_t g_cache_hits = 0, g_cache_misses = 0, g_cache_miss_bytes = 0;
std::map<int, std::multimap<size_t, CachedBlock>> g_cache;  // device -> size -> block
std::map<void*, size_t> g_live;                              // pointer -> bytes

// Size classes: 4 KiB steps up to 1 MiB, then 8 classes per power of two
// (at most 12.5% over the request), so that blocks released by one build
// fit the next build of a similar but not identical shape.
size_t cache_round(size_t bytes) {
  if (bytes <= (1u << 20)) return round_up(bytes, 4096);
  const int k = 63 - __builtin_clzll((unsigned long long)bytes);
  return round_up(bytes, (size_t)1 << (k - 3));
}

void* cache_alloc(size_t bytes, hipStream_t stream) {
  int dev = 0;
  ck(hipGetDevice(&dev));
  bytes = cache_round(bytes);
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto& m = g_cache[dev];
    auto best = m.end();
    // A cached block of the same class or up to twice the size: first one
    // released on this stream (stream order makes it safe), else one whose
    // last user has finished. A block still in use on another stream is not
    // taken: waiting for it would serialize independent streams.
    int probed = 0;
    for (auto it = m.lower_bound(bytes); it != m.end() && it->first <= 2 * bytes; ++it) {
      if (it->second.stream == stream) {
        best = it;
        break;
      }
      if (best != m.end() || probed >= 8) continue;
      ++probed;
      const CachedBlock& c = it->second;
      if (!c.ready || !c.ready->ev) {
        best = it;
        continue;
      }
      const hipError_t q = hipEventQuery(c.ready->ev);
      if (q == hipSuccess) best = it;
      else (void)hipGetLastError();
    }
    if (best != m.end()) {
      CachedBlock b = best->second;
      m.erase(best);
      g_live[b.p] = b.bytes;
      ++g_cache_hits;
      return b.p;
    }
    ++g_cache_misses;
    g_cache_miss_bytes += bytes;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    // Out of memory: give the cache back to HIP and try once more.
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto& m = g_cache[dev];
    if (!m.empty()) {
      (void)hipDeviceSynchronize();
      for (auto& kv : m) (void)hipFree(kv.second.p);
      m.clear();
      if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
      }
    }
    if (!p) return nullptr;
  }
  std::lock_guard<std::mutex> g(g_cache_mu);
  g_live[p] = bytes;
  return p;
}

// `ready` (optional) completes when all work using the block is done; without
// it an event is recorded on `stream` now.
void cache_release(void* p, hipStream_t stream, EventRef ready = nullptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  if (!ready) ready = record_event(stream);
  std::lock_guard<std::mutex> g(g_cache_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) return;
  g_cache[dev].insert({it->second, CachedBlock{p, it->second, stream, ready}});
  g_live.erase(it);
}

// Pinned host blocks (batch metadata mirrors), cached the same way; a block
// is reused only once the device work that writes it has completed.
struct PinnedBlock {
  void* p;
  EventRef ready;
};
std::multimap<size_t, PinnedBlock> g_pinned_free;

void* pinned_alloc(size_t bytes) {
  bytes = round_up(bytes, 4096);
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    for (auto it = g_pinned_free.lower_bound(bytes);
         it != g_pinned_free.end() && it->first - bytes <= it->first / 8; ++it) {
      if (it->second.ready && it->second.ready->ev &&
          hipEventQuery(it->second.ready->ev) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      void* p = it->second.p;
      g_pinned_free.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void pinned_release(void* p, size_t bytes, EventRef ready) {
  if (!p) return;
  std::lock_guard<std::mutex> g(g_cache_mu);
  g_pinned_free.insert({round_up(bytes, 4096), PinnedBlock{p, ready}});
}

// Device memory through the caller's allocator, or the library's cache.
struct Allocator {
  fmmds_alloc_fn alloc = nullptr;
  fmmds_release_fn release = nullptr;
  void* ctx = nullptr;
  hipStream_t stream = nullptr;

  void* get(size_t bytes) {
    bytes = round_up(std::max<size_t>(bytes, 1), 256);
    void* p = alloc ? alloc(ctx, bytes, (void*)stream) : cache_alloc(bytes, stream);
    if (!p) throw Fail{FMMDS_ERR_NOMEM};
    return p;
  }
  void put(void* p, size_t bytes, const EventRef& ready = nullptr) {
    if (!p) return;
    bytes = round_up(std::max<size_t>(bytes, 1), 256);
    if (release) release(ctx, p, bytes, (void*)stream);
    else cache_release(p, stream, ready);
  }
};

struct Block {
  void* p;
  size_t bytes;
};

// A set of allocations released together.
struct Pool {
  Allocator* A = nullptr;
  std::vector<Block> blocks;
  template <typename T>
  T* get(size_t count) {
    const size_t bytes = count * sizeof(T);
    void* p = A->get(bytes);
    blocks.push_back({p, bytes});
    return (T*)p;
  }
  void release_all(const EventRef& ready = nullptr) {
    EventRef ev = ready;
    if (!ev && !A->release && !blocks.empty()) ev = record_event(A->stream);  // one for all
    for (auto it = blocks.rbegin(); it != blocks.rend(); ++it) A->put(it->p, it->bytes, ev);
    blocks.clear();
  }
};

// Bump allocation of zeroed look-back status words and tile tickets.
struct StatusArena {
  uint64_t* words = nullptr;
  size_t n_words = 0, used_words = 0;
  uint32_t* tickets = nullptr;
  size_t n_tickets = 0, used_tickets = 0;
  uint64_t* take_words(size_t n) {
    if (used_words + n > n_words) throw Fail{FMMDS_ERR_DEVICE};
    uint64_t* p = words + used_words;
    used_words += n;
    return p;
  }
  uint32_t* take_ticket() {
    if (used_tickets >= n_tickets) throw Fail{FMMDS_ERR_DEVICE};
    return tickets + used_tickets++;
  }
};

struct LevelBufs {
  void* key = nullptr;
  uint32_t* begin = nullptr;
  uint32_t* parent = nullptr;
  uint32_t* child = nullptr;
  uint8_t* mask = nullptr;
  uint32_t cap = 0;
};

struct SetBufs {
  const float* xyz = nullptr;
  uint32_t n = 0;
  uint32_t* perm = nullptr;
  float* sorted_xyz = nullptr;
  LevelBufs lv[kMaxLevel + 1];
};

struct ListBufs {
  uint32_t* off[2] = {nullptr, nullptr};
  uint32_t* ent[2] = {nullptr, nullptr};
  uint64_t total[2] = {0, 0};
};

struct TreeImpl {
  bool view = false;  // a set of a batch: owned by the batch, fmmds_free ignores it
  Allocator A;
  Pool outs;
  ListBufs lists[kMaxLevel + 1];
  uint32_t n_recv_boxes[kMaxLevel + 1] = {};
};

uint32_t level_cap(uint32_t n, uint32_t l) {
  const uint64_t boxes = 1ull << (3 * l);
  return (uint32_t)std::min<uint64_t>(n, boxes);
}

// A second stream per device (default priority, created once, kept until
// the process ends) for the receiver chain of a build.
hipStream_t side_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  ck(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Fail{FMMDS_ERR_DEVICE};
  std::lock_guard<std::mutex> g(mu);
  if (!streams[dev]) ck(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  return streams[dev];
}

// Host copy of the metadata block, through a pinned buffer of this thread.
DevMeta* host_meta() {
  thread_local DevMeta* h = nullptr;
  if (!h) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(DevMeta), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{FMMDS_ERR_NOMEM};
    }
    h = (DevMeta*)p;
  }
  return h;
}

void fetch_meta(const DevMeta* d, DevMeta* h, hipStream_t s) {
  ck(hipMemcpyAsync(h, d, sizeof(DevMeta), hipMemcpyDeviceToHost, s));
  ck(hipStreamSynchronize(s));
}


// ---------------------------------------------------------------------------
// Per-kernel event timing (fmmds_profile_*).
// ---------------------------------------------------------------------------
enum KernelClass {
  K_ZERO, K_KEYGEN, K_DIGITS, K_SORT, K_LEAF, K_LEVEL, K_MAXOCC, K_COUNT, K_SCAN, K_FILL,
  K_REBASE, K_CLASSIFY, K_PLACE, K_DCOUNT, K_DSCAN, K_DORDER, K_DLIST, K_TCOUNT, K_TSCAN,
  K_NCLASS
};
const char* const kClassName[K_NCLASS] = {"zero",    "keygen",        "digit_offsets",
                                          "sort_pass", "leaf",        "level",
                                          "max_occupancy", "list_count", "scan_counts",
                                          "list_fill",     "batch_rebase", "inc_classify",
                                          "inc_place",     "dense_count",  "dense_scan",
                                          "dense_order",   "dense_lists",  "tab_count",
                                          "tab_scan"};

struct ClassStat {
  uint64_t launches = 0;
  double ms = 0, bytes = 0;
};
std::atomic<int> g_prof_on{0};
std::atomic<int> g_prof_only{-1};  // -1: every kernel class
std::mutex g_prof_mu;
ClassStat g_prof[K_NCLASS];
std::vector<hipEvent_t> g_events;  // reusable, guarded by g_prof_mu

// Timed launches whose events may still be pending (guarded by g_prof_mu):
// a build hands its records over without waiting for its stream, so that
// profiling does not stall back-to-back builds.
struct PendingRec {
  int cls;
  hipEvent_t a, b;
  double bytes;
};
std::vector<PendingRec> g_pending;

// Adds the launches whose end event has completed (every one, waiting for
// it, with wait = true) to the per-class totals. Call with g_prof_mu held.
void resolve_pending(bool wait) {
  size_t keep = 0;
  for (size_t i = 0; i < g_pending.size(); ++i) {
    const PendingRec r = g_pending[i];
    const hipError_t q = wait ? hipEventSynchronize(r.b) : hipEventQuery(r.b);
    if (q == hipErrorNotReady) {
      (void)hipGetLastError();
      g_pending[keep++] = r;
      continue;
    }
    float ms = 0;
    if (q != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      (void)hipGetLastError();
      ms = 0;
    }
    g_prof[r.cls].launches += 1;
    g_prof[r.cls].ms += ms;
    g_prof[r.cls].bytes += r.bytes;
    g_events.push_back(r.a);
    g_events.push_back(r.b);
  }
  g_pending.resize(keep);
}

constexpr int kListSet = 2;  // Prof record tag: a list kernel (count, scan, fill) of `level`

struct Prof {
  bool on = false;
  hipStream_t s = nullptr;
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double bytes;
    int set, level;  // for launches whose bytes depend on box counts
  };
  std::vector<Rec> recs;

  hipEvent_t ev() {
    {
      std::lock_guard<std::mutex> g(g_prof_mu);
      if (!g_events.empty()) {
        hipEvent_t e = g_events.back();
        g_events.pop_back();
        return e;
      }
    }
    hipEvent_t e;
    ck(hipEventCreate(&e));
    return e;
  }
  int only = -1;
  template <typename F>
  void run(int cls, double bytes, F&& f, int set = -1, int level = -1) {
    if (!on || (only >= 0 && cls != only)) {
      f();
      ck_launch();
      return;
    }
    hipEvent_t a = ev(), b = ev();
    ck(hipEventRecord(a, s));
    f();
    ck_launch();
    ck(hipEventRecord(b, s));
    recs.push_back({cls, a, b, bytes, set, level});
  }
  // `extra(rec)` adds bytes known only after the launch (box counts). The
  // durations are read once the launches have completed (resolve_pending),
  // not by waiting here.
  template <typename X>
  void finish(X&& extra) {
    if (!on) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (Rec& r : recs) g_pending.push_back({r.cls, r.a, r.b, r.bytes + extra(r)});
    recs.clear();
    resolve_pending(false);
  }
  void drop() {
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (Rec& r : recs) {
      g_events.push_back(r.a);
      g_events.push_back(r.b);
    }
    recs.clear();
  }
};

// Index bits of the incremental merge value for n points.
uint32_t index_bits(uint32_t n) { return n <= 2 ? 1u : 32u - (uint32_t)__builtin_clz(n - 1); }

// prev: with a previous tree, the order is rebuilt incrementally from it
// (the coordinates are given in prev's sorted order).
fmmds_status build(const float* src_xyz, uint32_t n_src, const float* recv_xyz, uint32_t n_recv,
                   const fmmds_options* opt, fmmds_tree** out,
                   const fmmds_tree* prev = nullptr, bool dense = false) {
  const bool shared = recv_xyz == nullptr;
  if (shared) n_recv = n_src;
  if (!src_xyz || !opt || n_src == 0 || n_recv == 0 || n_src >= 0xFFFFFFFFu ||
      n_recv >= 0xFFFFFFFFu)
    return FMMDS_ERR_ARG;
  if (opt->key_bits != 32 && opt->key_bits != 64) return FMMDS_ERR_ARG;
  if (opt->max_level < 2 || opt->max_level > opt->key_bits / 3) return FMMDS_ERR_ARG;
  if (opt->reserved != 0 || ((opt->alloc == nullptr) != (opt->release == nullptr)))
    return FMMDS_ERR_ARG;

  if (dense && opt->max_level > kDenseMaxLevel) return FMMDS_ERR_ARG;
  const uint32_t L = opt->max_level;
  const bool key64 = opt->key_bits == 64;
  const bool packed = 3 * L <= 32;
  const uint32_t n_pass = div_up(3 * L, 8);
  const uint32_t ksz = key64 ? 8 : 4;
  const int nsets = shared ? 1 : 2;

  TreeImpl* impl = new (std::nothrow) TreeImpl();
  fmmds_tree* t = new (std::nothrow) fmmds_tree();
  if (!impl || !t) {
    delete impl;
    delete t;
    return FMMDS_ERR_NOMEM;
  }
  std::memset(t, 0, sizeof(*t));
  impl->A.alloc = opt->alloc;
  impl->A.release = opt->release;
  impl->A.ctx = opt->alloc_ctx;
  impl->A.stream = (hipStream_t)opt->stream;
  impl->outs.A = &impl->A;
  Pool temps;
  temps.A = &impl->A;
  const hipStream_t st = impl->A.stream;

  fmmds_status result = FMMDS_OK;
  Prof P;
  P.on = g_prof_on.load() != 0;
  P.only = g_prof_only.load();
  P.s = st;
  hipStream_t side = nullptr;  // the receivers' stream, once this build has used it
  try {
    SetBufs sets[2];
    sets[0].xyz = src_xyz;
    sets[0].n = n_src;
    sets[1].xyz = shared ? src_xyz : recv_xyz;
    sets[1].n = n_recv;

    // Incremental order per set: the merge value (key, index) must fit 64 bits.
    bool inc[2] = {false, false};
    uint32_t ibits[2] = {0, 0}, inc_pass[2] = {0, 0};
    for (int s = 0; s < nsets; ++s) {
      ibits[s] = index_bits(sets[s].n);
      inc[s] = prev != nullptr && 3 * L + ibits[s] <= 64;
      inc_pass[s] = div_up(3 * L + ibits[s], 8);
    }
    if (prev) {
      sets[0].perm = const_cast<uint32_t*>(prev->src_perm);
      sets[0].sorted_xyz = const_cast<float*>(prev->src_sorted_xyz);
      sets[1].perm = const_cast<uint32_t*>(prev->recv_perm);
      sets[1].sorted_xyz = const_cast<float*>(prev->recv_sorted_xyz);
    }

    // ---- workspace: metadata, histograms, digit offsets, status words
    size_t words = 0, tickets = 0;
    for (int s = 0; s < nsets; ++s) {
      const uint32_t n = sets[s].n;
      const uint32_t np = inc[s] ? inc_pass[s] : n_pass;
      // status words of each sort pass, for the tile size that pass runs with
      const int items = (packed && !dense && !inc[s]) ? kSortWide : kSortItemsDefault;
      words += (size_t)np * sort_tiles(n, items) * 256 + 2 * div_up(n, kCompTile);
      tickets += np + 2 + L;
      if (dense) {
        for (uint32_t l = 0; l <= L; ++l) words += dense_scan_tiles(1u << (3 * l));
        tickets += L + 1;
      }
    }
    const size_t meta_b = round_up(sizeof(DevMeta), 256);
    const size_t hist_b = round_up(2 * kMaxPasses * 256 * 4, 256);
    const size_t tick_b = round_up(tickets * 4, 256);
    const size_t ws_b = round_up(meta_b + 2 * hist_b + tick_b + words * 8, 256);
    char* ws = temps.get<char>(ws_b);
    DevMeta* meta = (DevMeta*)ws;
    uint32_t* hist = (uint32_t*)(ws + meta_b);
    uint32_t* goff = (uint32_t*)(ws + meta_b + hist_b);
    StatusArena sa;
    sa.tickets = (uint32_t*)(ws + meta_b + 2 * hist_b);
    sa.n_tickets = tickets;
    sa.words = (uint64_t*)(ws + meta_b + 2 * hist_b + tick_b);
    sa.n_words = words;
    P.run(K_ZERO, (double)ws_b, [&] { launch_zero(ws, ws_b, st); });
    const uint32_t n_max = std::max(sets[0].n, sets[nsets - 1].n);
    SortBufs sb{};
    SortBufs& sb0 = sb;
    sb.k[0] = temps.get<uint64_t>(n_max);
    sb.k[1] = temps.get<uint64_t>(n_max);
    if (!packed || prev) {
      sb.v[0] = temps.get<uint32_t>(n_max);
      sb.v[1] = temps.get<uint32_t>(n_max);
    }
    // incremental: stayer list, and the sorted pairs the merge writes
    uint64_t *inc_sv[2] = {nullptr, nullptr}, *inc_fk = nullptr;
    uint32_t *inc_ss[2] = {nullptr, nullptr}, *inc_fv = nullptr;
    if (prev) {
      inc_sv[0] = inc_sv[1] = temps.get<uint64_t>(n_max);
      inc_ss[0] = inc_ss[1] = temps.get<uint32_t>(n_max);
      inc_fk = temps.get<uint64_t>(n_max);
      inc_fv = temps.get<uint32_t>(n_max);
    }

    // Incremental: classify every set first, then one sync for the counts,
    // so that the movers' sort and the merge launch grids of their size.
    const uint32_t* old_perm[2] = {sets[0].perm, sets[1].perm};  // previous tree
    const float* old_xyz[2] = {sets[0].sorted_xyz, sets[1].sorted_xyz};
    uint64_t* inc_mv[2] = {sb.k[0], sb.k[0]};
    uint32_t* inc_ms[2] = {sb.v[0], sb.v[0]};
    uint32_t n_stay[2] = {0, 0}, n_move[2] = {0, 0};
    if (prev) {
      bool any = false;
      for (int s = 0; s < nsets; ++s) {
        if (!inc[s]) continue;
        any = true;
        const uint32_t n = sets[s].n;
        if (s == 1) {  // set 0's buffers are still in use
          inc_mv[1] = temps.get<uint64_t>(n);
          inc_ms[1] = temps.get<uint32_t>(n);
          inc_sv[1] = temps.get<uint64_t>(n);
          inc_ss[1] = temps.get<uint32_t>(n);
        }
        uint64_t* stw = sa.take_words(div_up(n, kCompTile));
        uint32_t* tk = sa.take_ticket();
        P.run(K_CLASSIFY, (double)n * (4 + 12 + 12 + 12), [&] {
          launch_inc_classify(sets[s].xyz, old_xyz[s], old_perm[s], n, L, ibits[s],
                              inc_pass[s], inc_sv[s], inc_ss[s], inc_mv[s], inc_ms[s],
                              hist + s * kMaxPasses * 256, &meta->err_range, stw, tk,
                              meta->inc_counts[s], st);
        });
      }
      if (any) {
        DevMeta* hm = host_meta();
        fetch_meta(meta, hm, st);
        if (hm->err_range) throw Fail{FMMDS_ERR_RANGE};
        for (int s = 0; s < nsets; ++s) {
          n_stay[s] = hm->inc_counts[s][0];
          n_move[s] = hm->inc_counts[s][1];
        }
      }
    }

    // Dense variant: per set and level the occupancy counters (Bin), their
    // scan (ScannedBin) and the exclusive nonempty rank (ScannedRank), plus
    // every point's finest box and provisional rank.
    struct DenseSet {
      uint32_t* bin[kMaxLevel + 1] = {};
      uint32_t* sbin[kMaxLevel + 1] = {};
      uint32_t* srank[kMaxLevel + 1] = {};
      uint32_t* key = nullptr;
      uint32_t* rank = nullptr;
    } dn[2];

    // Separate source and receiver sets are independent until the lists: the
    // receivers' chain runs on a second stream, so that the latency-bound
    // kernels of the two chains overlap. Every buffer is taken before the
    // chains start (the allocator orders blocks on `st`).
    const bool two = nsets == 2;
    SortBufs sb1 = sb;
    uint64_t* inc_fks[2] = {inc_fk, inc_fk};  // incremental: merged pairs per set
    uint32_t* inc_fvs[2] = {inc_fv, inc_fv};
    float* full_x[2] = {nullptr, nullptr};    // incremental fallback: original order
    if (two) {
      sb1.k[0] = temps.get<uint64_t>(n_max);
      sb1.k[1] = temps.get<uint64_t>(n_max);
      if (!packed || prev) {
        sb1.v[0] = temps.get<uint32_t>(n_max);
        sb1.v[1] = temps.get<uint32_t>(n_max);
      }
      if (prev) {
        inc_fks[1] = temps.get<uint64_t>(n_max);
        inc_fvs[1] = temps.get<uint32_t>(n_max);
      }
    }
    for (int s = 0; s < nsets; ++s)
      if (prev && !inc[s]) full_x[s] = temps.get<float>(3 * (size_t)sets[s].n);
    for (int s = 0; s < nsets; ++s) {
      SetBufs& S = sets[s];
      const uint32_t n = S.n;
      S.perm = impl->outs.get<uint32_t>(n);
      S.sorted_xyz = impl->outs.get<float>(3 * (size_t)n);
      // Tables, sized for the worst case so no host round trip is needed.
      size_t tb = 0;
      for (uint32_t l = 0; l <= L; ++l) {
        const size_t c = level_cap(n, l);
        tb += round_up(c * ksz, 256) + round_up((c + 1) * 4, 256);
        if (l >= 1) tb += round_up(c * 4, 256);
        if (l < L) tb += round_up((c + 1) * 4, 256) + round_up(c, 256);
      }
      char* tp = impl->outs.get<char>(tb);
      for (uint32_t l = 0; l <= L; ++l) {
        LevelBufs& B = S.lv[l];
        const size_t c = level_cap(n, l);
        B.cap = (uint32_t)c;
        B.key = tp;
        tp += round_up(c * ksz, 256);
        B.begin = (uint32_t*)tp;
        tp += round_up((c + 1) * 4, 256);
        if (l >= 1) {
          B.parent = (uint32_t*)tp;
          tp += round_up(c * 4, 256);
        }
        if (l < L) {
          B.child = (uint32_t*)tp;
          tp += round_up((c + 1) * 4, 256);
          B.mask = (uint8_t*)tp;
          tp += round_up(c, 256);
        }
      }
    }
    // keygen's per-block digit-count rows, per set
    uint32_t* krows[2] = {nullptr, nullptr};
    for (int s = 0; s < nsets; ++s)
      krows[s] = temps.get<uint32_t>((size_t)keygen_blocks(sets[s].n) * n_pass * 256);
    // every level's tables in one pass (not the dense variant): per set the
    // per-tile box-start counts of every level and their scan
    uint32_t* tabbuf[2] = {nullptr, nullptr};
    for (int s = 0; !dense && s < nsets; ++s)
      tabbuf[s] = temps.get<uint32_t>((size_t)2 * (L + 1) * tab_tiles(sets[s].n));
    for (int s = 0; dense && s < nsets; ++s) {
      DenseSet& Dn = dn[s];
      for (uint32_t l = 0; l <= L; ++l) {
        const size_t nb = (size_t)1 << (3 * l);
        Dn.bin[l] = temps.get<uint32_t>(std::max<size_t>(nb, 8));
        Dn.sbin[l] = temps.get<uint32_t>(std::max<size_t>(nb, 8));
        Dn.srank[l] = temps.get<uint32_t>(std::max<size_t>(nb, 8));
      }
      Dn.key = temps.get<uint32_t>(sets[s].n);
      Dn.rank = temps.get<uint32_t>(sets[s].n);
    }
    hipStream_t st1 = st;
    // (profiling with on == 2 keeps both chains on the build stream, so that
    // every kernel's event-measured duration is its own)
    if (two && g_prof_on.load() != 2) {
      st1 = side_stream();
      side = st1;
      EventRef e0 = record_event(st);
      if (e0->ev) ck(hipStreamWaitEvent(st1, e0->ev, 0));
    }

    // Plain builds: both chains' key generation is enqueued first, so that
    // the receivers' chain starts while the host enqueues the rest.
    const bool plain = !dense && !prev;
    for (int s = 0; plain && s < nsets; ++s) {
      const hipStream_t st = s == 1 ? st1 : impl->A.stream;
      P.s = st;
      SortBufs& sb = s == 1 ? sb1 : sb0;
      const uint32_t n = sets[s].n;
      uint32_t* h = hist + s * kMaxPasses * 256;
      uint32_t* g = goff + s * kMaxPasses * 256;
      P.run(K_KEYGEN, (double)n * (packed ? 12 + 8 : 12 + 8 + 4), [&] {
        launch_keygen(sets[s].xyz, n, L, packed, sb.k[0], sb.v[0], n_pass, krows[s],
                      &meta->err_range, st);
      });
      P.run(K_DIGITS, (double)keygen_blocks(n) * n_pass * 1024, [&] {
        launch_reduce_rows(krows[s], keygen_blocks(n), h, n_pass, st);
        launch_digit_offsets(h, g, n_pass, st);
      });
    }

    for (int s = 0; s < nsets; ++s) {
      SetBufs& S = sets[s];
      const uint32_t n = S.n;
      // this set's chain: its stream, and the profiler's events on it
      const hipStream_t st = s == 1 ? st1 : impl->A.stream;
      P.s = st;
      SortBufs& sb = s == 1 ? sb1 : sb0;

      if (dense) {
        // Algorithm 1 at level L, the counters of the coarser levels, then
        // Algorithm 3 per level and the parent / child links.
        DenseSet& Dn = dn[s];
        const size_t nbL = (size_t)1 << (3 * L);
        P.run(K_ZERO, (double)nbL * 4, [&] { launch_zero(Dn.bin[L], nbL * 4, st); });
        P.run(K_DCOUNT, (double)n * (12 + 8), [&] {
          launch_dense_count(S.xyz, n, L, Dn.bin[L], Dn.key, Dn.rank, &meta->err_range, st);
        });
        for (int l = (int)L - 1; l >= 0; --l)
          P.run(K_DSCAN, (double)(1u << (3 * l)) * 36, [&] {
            launch_dense_reduce(Dn.bin[l + 1], 1u << (3 * l), Dn.bin[l], st);
          });
        for (uint32_t l = 0; l <= L; ++l) {
          const uint32_t nb = 1u << (3 * l);
          uint64_t* stw = sa.take_words(dense_scan_tiles(nb));
          uint32_t* tk = sa.take_ticket();
          P.run(K_DSCAN, (double)nb * 12, [&] {
            launch_dense_scan(key64, Dn.bin[l], nb, Dn.sbin[l], Dn.srank[l], S.lv[l].key,
                              S.lv[l].begin, &meta->n_boxes[s][l], &meta->max_occ[s][l], stw, tk,
                              st);
          });
        }
        for (uint32_t l = 0; l < L; ++l)
          P.run(K_DSCAN, 0.0, [&] {
            launch_dense_links(key64, S.lv[l].key, &meta->n_boxes[s][l], S.lv[l].cap,
                               Dn.bin[l + 1], Dn.srank[l + 1], &meta->n_boxes[s][l + 1],
                               S.lv[l].child, S.lv[l].mask, S.lv[l + 1].key, S.lv[l + 1].cap,
                               S.lv[l + 1].parent, Dn.srank[l], st);
          });
        continue;  // the point order follows once the largest box is known
      }

      // ---- keys and sort
      uint32_t* h = hist + s * kMaxPasses * 256;
      uint32_t* g = goff + s * kMaxPasses * 256;
      const uint64_t* fin_k = nullptr;
      const uint32_t* fin_v = nullptr;
      const float* leaf_xyz = S.xyz;  // null: the merge already wrote the coordinates
      if (inc[s]) {
        // The movers sorted by (key, index), then merged with the stayers.
        const uint32_t ib = ibits[s], np = inc_pass[s], nm = n_move[s];
        uint64_t* mk[2] = {inc_mv[s], sb.k[1]};
        uint32_t* mv[2] = {inc_ms[s], sb.v[1]};
        uint64_t* inc_fk = inc_fks[s];
        uint32_t* inc_fv = inc_fvs[s];
        P.run(K_DIGITS, (double)np * 2048, [&] { launch_digit_offsets(h, g, np, st); });
        for (uint32_t p = 0; p < np && nm > 0; ++p) {
          const int a = p & 1, b = a ^ 1;
          uint64_t* stw = sa.take_words((size_t)sort_tiles(n, kSortItemsDefault) * 256);
          uint32_t* tk = sa.take_ticket();
          P.run(K_SORT, (double)nm * 24, [&] {
            launch_sort_pass(false, mk[a], mk[b], mv[a], mv[b], nm, 8 * p, g + p * 256, stw, tk,
                             st, kSortItemsDefault);
          });
        }
        const int mf = nm > 0 ? (int)(np & 1) : 0;
        P.run(K_PLACE, (double)n * (8 + 4 + 12 + 8 + (packed ? 0 : 4) + 12), [&] {
          launch_inc_merge(packed, inc_sv[s], inc_ss[s], n_stay[s], mk[mf], mv[mf], nm,
                           S.xyz, ib, inc_fk, inc_fv, S.sorted_xyz,
                           st);
        });
        fin_k = inc_fk;
        fin_v = inc_fv;
        leaf_xyz = nullptr;
      } else {
        if (prev) {
          // the merge value does not fit: full sort, from original order
          float* x = full_x[s];
          P.run(K_PLACE, 0.0, [&] { launch_inc_scatter(S.xyz, old_perm[s], n, x, st); });
          S.xyz = x;
          leaf_xyz = x;
        }
        if (!plain) {  // (plain builds enqueued these above)
          P.run(K_KEYGEN, (double)n * (packed ? 12 + 8 : 12 + 8 + 4), [&] {
            launch_keygen(S.xyz, n, L, packed, sb.k[0], sb.v[0], n_pass, krows[s],
                          &meta->err_range, st);
          });
          P.run(K_DIGITS, (double)keygen_blocks(n) * n_pass * 1024, [&] {
            launch_reduce_rows(krows[s], keygen_blocks(n), h, n_pass, st);
            launch_digit_offsets(h, g, n_pass, st);
          });
        }
        for (uint32_t p = 0; p < n_pass; ++p) {
          const int a = p & 1, b = a ^ 1;
          const uint32_t shift = (packed ? 32 : 0) + 8 * p;
          uint64_t* stw =
              sa.take_words((size_t)sort_tiles(n, packed ? kSortWide : kSortItemsDefault) * 256);
          uint32_t* tk = sa.take_ticket();
          P.run(K_SORT, (double)n * (packed ? 16 : 24), [&] {
            launch_sort_pass(packed, sb.k[a], sb.k[b], sb.v[a], sb.v[b], n, shift, g + p * 256,
                             stw, tk, st, packed ? kSortWide : kSortItemsDefault);
          });
        }
        const int fin = n_pass & 1;
        fin_k = sb.k[fin];
        fin_v = sb.v[fin];
      }

      // ---- every level's tables from the sorted points
      {
        TabLevels T{};
        for (uint32_t l = 0; l <= L; ++l) {
          T.key[l] = S.lv[l].key;
          T.begin[l] = S.lv[l].begin;
          T.parent[l] = S.lv[l].parent;
          T.child[l] = S.lv[l].child;
          T.mask[l] = S.lv[l].mask;
        }
        const uint32_t tiles = tab_tiles(n);
        uint32_t* tcnt = tabbuf[s];
        uint32_t* tpre = tabbuf[s] + (size_t)(L + 1) * tiles;
        const double elem_b = packed ? 8 : 12;
        const double cnt_b = (double)(L + 1) * tiles * 4;
        uint32_t* nbox = &meta->n_boxes[s][0];
        auto tab = [&](int phase) {
          launch_tables(packed, key64, fin_k, fin_v, leaf_xyz, n, L, tcnt, tpre, T, S.perm,
                        S.sorted_xyz, nbox, L > 0 ? S.lv[L - 1].cap : 0, st, phase);
        };
        // sorted elements in, per-tile counts out; the counts scanned; then
        // (box counts known) the tables, and the child masks
        P.run(K_TCOUNT, (double)n * elem_b + cnt_b, [&] { tab(0); });
        P.run(K_TSCAN, 2 * cnt_b, [&] { tab(1); });
        P.run(K_LEAF, (double)n * (elem_b + 4 + (leaf_xyz ? 12 + 12 : 0)) + cnt_b,
              [&] { tab(2); }, s, (int)L);
        P.run(K_LEVEL, 0.0, [&] { tab(3); }, s, -1);
      }
      if (opt->cluster_s > 0) {
        for (uint32_t l = 2; l <= L; ++l) {
          P.run(K_MAXOCC, 0.0, [&] {
            launch_max_occupancy(S.lv[l].begin, &meta->n_boxes[s][l], S.lv[l].cap,
                                 &meta->max_occ[s][l], st);
          }, s, (int)l);
        }
      }
    }

    P.s = st;
    if (two) {
      EventRef e1 = record_event(st1);
      if (e1->ev) ck(hipStreamWaitEvent(st, e1->ev, 0));
    }

    // ---- sync point 1: box counts, range flag, occupancy maxima. A plain
    // build without the depth rule skips it: its list kernels read the box
    // counts on the device over grids sized by capacity, and the range flag
    // and the counts come back at the finest level's sync.
    const bool early = plain && opt->cluster_s == 0 && L >= 2;
    DevMeta* hm = host_meta();
    if (!early) {
      fetch_meta(meta, hm, st);
      if (hm->err_range) throw Fail{FMMDS_ERR_RANGE};
    }
    const int rs = shared ? 0 : 1;
    uint32_t D = L;
    if (opt->cluster_s > 0) {
      for (uint32_t l = 2; l <= L; ++l) {
        if (hm->max_occ[0][l] <= opt->cluster_s && hm->max_occ[rs][l] <= opt->cluster_s) {
          D = l;
          break;
        }
      }
    }
    // nb: box counts (capacities until known, in the early case); lcap: the
    // sizes the lists' buffers and grids are laid out with (fixed from here)
    uint32_t nb[2][kMaxLevel + 1], lcap[2][kMaxLevel + 1];
    auto read_counts = [&]() {
      for (int s = 0; s < 2; ++s)
        for (uint32_t l = 0; l <= L; ++l) nb[s][l] = hm->n_boxes[s < nsets ? s : 0][l];
    };
    if (early) {
      for (int s = 0; s < 2; ++s)
        for (uint32_t l = 0; l <= L; ++l) nb[s][l] = level_cap(sets[s < nsets ? s : 0].n, l);
    } else {
      read_counts();
    }
    for (int s = 0; s < 2; ++s)
      for (uint32_t l = 0; l <= L; ++l) lcap[s][l] = nb[s][l];

    // Dense variant: the point order. Boxes of up to kDenseCanonMax points
    // are put in index order on the device; beyond that the set's points are
    // sorted (its tables stay those of the dense scans: the same values).
    for (int s = 0; dense && s < nsets; ++s) {
      SetBufs& S = sets[s];
      const uint32_t n = S.n;
      if (hm->max_occ[s][L] <= kDenseCanonMax) {
        uint32_t* tmp = temps.get<uint32_t>(n);
        uint32_t* big = temps.get<uint32_t>(std::max<uint32_t>(nb[s][L], 1));
        P.run(K_DORDER, (double)n * (8 + 4 + 4 + 4 + 4 + 4 + 12 + 12), [&] {
          launch_dense_order(dn[s].key, dn[s].rank, n, dn[s].sbin[L], S.lv[L].begin,
                             &meta->n_boxes[s][L], nb[s][L], tmp, S.perm, big,
                             &meta->dense_big[s], S.xyz, S.sorted_xyz, st);
        });
        continue;
      }
      uint32_t* h = hist + s * kMaxPasses * 256;
      uint32_t* g = goff + s * kMaxPasses * 256;
      P.run(K_KEYGEN, 0.0, [&] {
        launch_keygen(S.xyz, n, L, packed, sb.k[0], sb.v[0], n_pass, krows[s], &meta->err_range,
                      st);
      });
      P.run(K_DIGITS, 0.0, [&] {
        launch_reduce_rows(krows[s], keygen_blocks(n), h, n_pass, st);
        launch_digit_offsets(h, g, n_pass, st);
      });
      for (uint32_t p = 0; p < n_pass; ++p) {
        const int a = p & 1, b = a ^ 1;
        uint64_t* stw = sa.take_words((size_t)sort_tiles(n, kSortItemsDefault) * 256);
        uint32_t* tk = sa.take_ticket();
        P.run(K_SORT, 0.0, [&] {
          launch_sort_pass(packed, sb.k[a], sb.k[b], sb.v[a], sb.v[b], n, (packed ? 32 : 0) + 8 * p,
                           g + p * 256, stw, tk, st, kSortItemsDefault);
        });
      }
      uint64_t* stw = sa.take_words(div_up(n, kCompTile));
      uint32_t* tk = sa.take_ticket();
      const int fin = n_pass & 1;
      P.run(K_LEAF, 0.0, [&] {
        launch_leaf(packed, key64, sb.k[fin], sb.v[fin], S.xyz, n, S.perm, S.sorted_xyz,
                    S.lv[L].key, S.lv[L].begin, stw, tk, &meta->n_boxes[s][L], st);
      });
    }

    // ---- lists, levels 2..D
    size_t lwords = 0, lmax = 0;
    for (uint32_t l = 2; l <= D; ++l) {
      lwords += 2 * (size_t)scan_tiles(lcap[rs][l]);
      lmax = std::max<size_t>(lmax, lcap[rs][l]);
    }
    const size_t ltick_b = round_up(2 * (kMaxLevel + 1) * 4, 256);
    const size_t lws_b = round_up(ltick_b + lwords * 8, 256);
    char* lws = temps.get<char>(lws_b);
    StatusArena la;
    la.tickets = (uint32_t*)lws;
    la.n_tickets = 2 * (kMaxLevel + 1);
    la.words = (uint64_t*)(lws + ltick_b);
    la.n_words = lwords;
    P.run(K_ZERO, (double)lws_b, [&] { launch_zero(lws, lws_b, st); });
    // E2 counts, then E4 counts from a 16-byte aligned start (vector loads)
    uint32_t* cnt = temps.get<uint32_t>(2 * round_up(std::max<size_t>(lmax, 1), 4));
    // Levels with at most a quarter of the finest level's receiver boxes get
    // their entries allocated for the worst case (27 E2 and 189 E4 per
    // receiver box) and need no host round trip for their totals, which are
    // read at the next one; the finest level is allocated exactly.
    auto small_level = [&](uint32_t l) {
      return l < D && (uint64_t)lcap[rs][l] * 4 <= (uint64_t)lcap[rs][D];
    };
    auto take_totals = [&](const DevMeta* h, uint32_t upto) {
      for (uint32_t m = 2; m <= upto; ++m)
        for (int k = 0; k < 2; ++k) impl->lists[m].total[k] = h->list_total[k][m];
    };
    // Every level's offsets and the small levels' entries come from one
    // block, taken before the first list kernel, so that the host enqueues
    // the small levels' kernels back to back (they run for microseconds
    // each, less than an allocator call and a launch take on the host).
    size_t lblock_b = 0;
    for (uint32_t l = 2; l <= D; ++l) {
      const size_t nr = lcap[rs][l];
      lblock_b += 2 * round_up((nr + 1) * 4, 256);
      if (small_level(l)) lblock_b += round_up(27 * nr * 4, 256) + round_up(189 * nr * 4, 256);
    }
    char* lblock = impl->outs.get<char>(lblock_b);
    auto carve = [&](size_t count) {
      uint32_t* q = (uint32_t*)lblock;
      lblock += round_up(count * 4, 256);
      return q;
    };
    for (uint32_t l = 2; l <= D; ++l) {
      const uint32_t nr = lcap[rs][l];
      ListLevelArgs a{};
      a.level = l;
      a.n_recv_up = lcap[rs][l - 1];
      if (early) {
        a.n_recv_up_dev = &meta->n_boxes[rs][l - 1];
        a.n_src_up_dev = &meta->n_boxes[0][l - 1];
      }
      a.recv_key_up = sets[rs].lv[l - 1].key;
      a.recv_mask_up = sets[rs].lv[l - 1].mask;
      a.recv_child_up = sets[rs].lv[l - 1].child;
      a.src_key_up = sets[0].lv[l - 1].key;
      a.src_mask_up = sets[0].lv[l - 1].mask;
      a.src_child_up = sets[0].lv[l - 1].child;
      a.up_all = (l - 1 == 1) ? 1u : 0u;
      a.n_src_up = lcap[0][l - 1];
      a.key_bits_up = 3 * (l - 1);
      if (!a.up_all) {
        a.e2_off_up = impl->lists[l - 1].off[0];
        a.e2_ent_up = impl->lists[l - 1].ent[0];
      }
      ListBufs& LB = impl->lists[l];
      // (the bytes of the count, scan and fill launches follow from the box
      // counts and list sizes, added once known: see P.finish below)
      // level 2 only: the fill of each level writes the next level's counts
      if (dense)
        P.run(K_DLIST, 0.0, [&] {
          launch_dense_lists(key64, false, l, nb[rs][l - 1], sets[rs].lv[l - 1].key,
                             sets[rs].lv[l - 1].mask, sets[rs].lv[l - 1].child, dn[0].bin[l - 1],
                             dn[0].bin[l], dn[0].srank[l], cnt, cnt + round_up(nr, 4), nullptr,
                             nullptr, nullptr, nullptr, st);
        });
      else if (l == 2)
        P.run(K_COUNT, 0.0, [&] { launch_list_count(key64, a, cnt, cnt + round_up(nr, 4), st); },
              kListSet, (int)l);
      LB.off[0] = carve((size_t)nr + 1);
      LB.off[1] = carve((size_t)nr + 1);
      {
        uint64_t* st2 = la.take_words(scan_tiles(nr));
        uint64_t* st4 = la.take_words(scan_tiles(nr));
        uint32_t* tk = la.take_ticket();
        P.run(K_SCAN, 0.0, [&] {
          launch_scan_counts2(cnt, cnt + round_up(nr, 4), nr, LB.off[0], LB.off[1], &meta->list_total[0][l],
                              &meta->list_total[1][l], &meta->overflow, st2, st4, tk, st,
                              early ? &meta->n_boxes[rs][l] : nullptr);
        }, kListSet, (int)l);
      }
      if (small_level(l)) {
        for (int k = 0; k < 2; ++k) LB.ent[k] = carve((size_t)nr * (k == 0 ? 27 : 189));
      } else {
        fetch_meta(meta, hm, st);  // sync point: this level's list totals
        if (early) {
          if (hm->err_range) throw Fail{FMMDS_ERR_RANGE};
          read_counts();
        }
        if (hm->overflow) throw Fail{FMMDS_ERR_OVERFLOW};
        take_totals(hm, l);
        for (int k = 0; k < 2; ++k) LB.ent[k] = impl->outs.get<uint32_t>(LB.total[k]);
      }
      if (dense) {
        P.run(K_DLIST, 0.0, [&] {
          launch_dense_lists(key64, true, l, nb[rs][l - 1], sets[rs].lv[l - 1].key,
                             sets[rs].lv[l - 1].mask, sets[rs].lv[l - 1].child, dn[0].bin[l - 1],
                             dn[0].bin[l], dn[0].srank[l], nullptr, nullptr, LB.off[0],
                             LB.off[1], LB.ent[0], LB.ent[1], st);
        });
        continue;
      }
      if (l < D) {  // the next level's counts
        a.src_mask_cur = sets[0].lv[l].mask;
        a.recv_mask_cur = sets[rs].lv[l].mask;
        a.recv_child_cur = sets[rs].lv[l].child;
        a.cnt2_next = cnt;
        a.cnt4_next = cnt + round_up(lcap[rs][l + 1], 4);
      }
      P.run(K_FILL, 0.0,
            [&] { launch_list_fill(key64, a, LB.off[0], LB.off[1], LB.ent[0], LB.ent[1], st); },
            kListSet, (int)l);
    }
    for (uint32_t l = 2; l <= D; ++l) impl->n_recv_boxes[l] = nb[rs][l];

    // Box-count-dependent bytes: leaf keys + bookmarks; a coarser level reads
    // the finer keys and bookmarks and writes keys, bookmarks, first children,
    // masks and the finer level's parents; the occupancy pass reads bookmarks.
    P.finish([&](const Prof::Rec& r) -> double {
      if (r.set == kListSet) {
        const uint32_t l = (uint32_t)r.level;
        const double nr = nb[rs][l];
        if (r.cls == K_SCAN) return nr * 16 + 8;  // two counts in, two offsets out
        // receiver key + parent in, two counts out; the parent lists and the
        // parent-level source keys, masks and first children read once
        const double side = (double)nb[rs][l - 1] * (ksz + 1 + 4 + 8) +
                            (double)nb[0][l - 1] * (ksz + 1 + 4);
        if (r.cls == K_COUNT) return side + nr * 8;
        // a fill: also its entries and the parent level's E2 list read, and
        // below D the next level's counts (masks and first children in, two
        // counts out)
        const ListBufs& LB = impl->lists[l];
        const double e2up = l - 1 >= 2 ? (double)impl->lists[l - 1].total[0] : 0.0;
        const double next_b =
            l < D ? nr * 5 + (double)nb[0][l] + (double)nb[rs][l + 1] * 8 : 0.0;
        return side + nr * 8 + next_b + 4.0 * (double)(LB.total[0] + LB.total[1]) + 4.0 * e2up;
      }
      if (r.set < 0) return 0.0;
      const uint32_t* c = nb[r.set == 0 ? 0 : rs];
      if (r.cls == K_LEAF) {  // every level: key, bookmark, parent, first child
        double b = 0;
        for (uint32_t l = 0; l <= L; ++l)
          b += (double)c[l] * (ksz + 4 + (l >= 1 ? 4 : 0) + (l < L ? 4 : 0)) + 4 + (l < L ? 4 : 0);
        return b;
      }
      if (r.cls == K_LEVEL && r.level < 0) {  // masks: first children in, children's keys in
        double b = 0;
        for (uint32_t l = 0; l < L; ++l) b += (double)c[l] * (4 + 1) + 4 + (double)c[l + 1] * ksz;
        return b;
      }
      if (r.cls == K_LEVEL)
        return (double)c[r.level + 1] * (ksz + 4 + 4) + (double)c[r.level] * (ksz + 4 + 4 + 1);
      if (r.cls == K_MAXOCC) return (double)(c[r.level] + 1) * 4;
      return 0.0;
    });

    // ---- public view
    t->depth = D;
    t->key_bits = opt->key_bits;
    t->max_level = L;
    t->shared = shared ? 1u : 0u;
    t->n_src = n_src;
    t->n_recv = n_recv;
    t->src_perm = sets[0].perm;
    t->src_sorted_xyz = sets[0].sorted_xyz;
    t->recv_perm = sets[rs].perm;
    t->recv_sorted_xyz = sets[rs].sorted_xyz;
    for (int s = 0; s < 2; ++s) {
      const SetBufs& S = sets[s == 0 ? 0 : rs];
      fmmds_level* lv = s == 0 ? t->src : t->recv;
      for (uint32_t l = 0; l <= D; ++l) {
        lv[l].n = nb[s == 0 ? 0 : rs][l];
        lv[l].key = S.lv[l].key;
        lv[l].begin = S.lv[l].begin;
        lv[l].parent = l >= 1 ? S.lv[l].parent : nullptr;
        lv[l].child = l < D ? S.lv[l].child : nullptr;
      }
    }
    t->impl = impl;
    temps.release_all();
  } catch (const Fail& f) {
    result = f.st;
  } catch (const std::bad_alloc&) {
    result = FMMDS_ERR_NOMEM;
  }
  if (result != FMMDS_OK) {
    // Work of this build may still use the buffers: wait for the caller's
    // stream and, when the receivers' chain was enqueued, the side stream
    // (not the whole device).
    (void)hipGetLastError();
    if (side) (void)hipStreamSynchronize(side);
    (void)hipStreamSynchronize(st);
    (void)hipGetLastError();
    P.drop();
    temps.release_all();
    impl->outs.release_all();
    delete impl;
    delete t;
    return result;
  }
  *out = t;
  return FMMDS_OK;
}


// ---------------------------------------------------------------------------
// Batched form (fmmds_batch_*).
// ---------------------------------------------------------------------------
struct TuneKey {
  uint32_t log2n, n_pass, packed;
  bool operator<(const TuneKey& o) const {
    return std::tie(log2n, n_pass, packed) < std::tie(o.log2n, o.n_pass, o.packed);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;  // sort tile size chosen by timing, per shape class

struct BatchImpl {
  uint32_t n_sets = 0, P = 0, L = 0, setbits = 0, keybits = 0, n_pass = 0;
  bool packed = false;
  int items = kSortItemsDefault;
  bool items_fixed = false;  // set from FMMDS_BATCH_SORT_ITEMS: no timing
  std::vector<uint64_t> off;
  std::vector<uint8_t> lev;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Allocator A;
  Pool mem;
  uint64_t* d_off = nullptr;
  uint8_t* d_lev = nullptr;
  // set-aligned sort tiles, one table per tile size (kTileItems), in one block
  uint32_t n_tiles[4] = {};
  uint32_t* d_tiles = nullptr;
  uint32_t* d_tstart[4] = {};
  uint32_t* d_tset[4] = {};
  uint32_t* d_goff = nullptr;  // per set and pass, where each digit's run starts
  SortBufs sb{};
  uint32_t* perm = nullptr;
  float* sxyz = nullptr;
  uint32_t* tabbuf = nullptr;  // per-tile box-start counts of every level, and their scan
  LevelBufs g[kMaxLevel + 1];
  uint64_t* fkey[kMaxLevel + 1] = {};
  uint32_t* fbegin[kMaxLevel + 1] = {};
  uint32_t* fparent[kMaxLevel + 1] = {};
  uint32_t* fchild[kMaxLevel + 1] = {};
  uint32_t cap[kMaxLevel + 1] = {}, rcap[kMaxLevel + 1] = {};
  uint32_t* cnt = nullptr;
  uint32_t* goff[kMaxLevel + 1][2] = {};
  uint32_t* loff[kMaxLevel + 1][2] = {};
  uint32_t* ent[kMaxLevel + 1][2] = {};
  // device block copied back after each launch: DevMeta, first, bases
  char* dblock = nullptr;
  size_t dblock_b = 0, first_at = 0, base_at = 0;
  char* hblock = nullptr;  // pinned mirror, followed by the staged offsets and levels
  size_t hblock_b = 0;
  // zeroed per launch: dblock, the sets' digit histograms, tickets, status words
  char* ws = nullptr;
  size_t ws_b = 0, hist_at = 0, tick_at = 0, words_at = 0;
  size_t n_words = 0, n_tickets = 0, list_words = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const float* graph_xyz = nullptr;
  bool launched = false;
  size_t footprint = 0;  // device bytes of the plan
  EventRef done;         // recorded after the last launch's work
  std::vector<fmmds_tree> trees;
  std::vector<TreeImpl> views;

  DevMeta* meta() const { return (DevMeta*)dblock; }
  uint32_t* first() const { return (uint32_t*)(dblock + first_at); }
  uint32_t* first_l(uint32_t l) const { return first() + (size_t)l * (n_sets + 1); }
  uint32_t* base(uint32_t l, int k) const {
    return (uint32_t*)(dblock + base_at) + ((size_t)(l * 2 + k)) * (n_sets + 1);
  }
};

// The sort tile sizes a batch may use (the autotuned choice indexes them).
constexpr int kTileItems[4] = {8, 12, 16, kSortWide};
int tile_kind(int items) { return items == 8 ? 0 : items == 12 ? 1 : items == 16 ? 2 : 3; }

void batch_sort_passes(BatchImpl& B, StatusArena& sa, Prof& P, int items) {
  const int kd = tile_kind(items);
  for (uint32_t p = 0; p < B.n_pass; ++p) {
    const int a = p & 1, b = a ^ 1;
    const uint32_t shift = (B.packed ? 32 : 0) + 8 * p;
    uint64_t* stw = sa.take_words((size_t)B.n_tiles[kd] * 256);
    uint32_t* tk = sa.take_ticket();
    const SegSort sg{B.d_tstart[kd], B.d_tset[kd], B.d_goff, B.n_tiles[kd], B.n_pass, p};
    P.run(K_SORT, (double)B.P * (B.packed ? 16 : 24), [&] {
      launch_sort_pass_seg(B.packed, B.sb.k[a], B.sb.k[b], B.sb.v[a], B.sb.v[b], shift, sg, stw,
                           tk, B.stream, items);
    });
  }
}

void batch_front(BatchImpl& B, const float* xyz, StatusArena& sa, Prof& P, int items) {
  const hipStream_t st = B.stream;
  sa = StatusArena();
  sa.tickets = (uint32_t*)(B.ws + B.tick_at);
  sa.n_tickets = B.n_tickets;
  sa.words = (uint64_t*)(B.ws + B.words_at);
  sa.n_words = B.n_words;
  // only the status words this launch takes (the sort's depend on its tile
  // size; the workspace is sized for the smallest tiles)
  const size_t used = (size_t)B.n_pass * B.n_tiles[tile_kind(items)] * 256 + B.list_words;
  const size_t zb = std::min(B.ws_b, round_up(B.words_at + used * 8, 256));
  P.run(K_ZERO, (double)zb, [&] { launch_zero(B.ws, zb, st); });
  uint32_t* hist = (uint32_t*)(B.ws + B.hist_at);
  const int kw = tile_kind(kSortWide);  // keygen tiles: 8192 points
  P.run(K_KEYGEN, (double)B.P * (12 + 8 + (B.packed ? 0 : 4)), [&] {
    launch_batch_keygen(xyz, B.d_tstart[kw], B.d_tset[kw], B.n_tiles[kw], B.d_lev, B.L, B.packed,
                        B.sb.k[0], B.sb.v[0], B.n_pass, hist, &B.meta()->err_range, st);
  });
  P.run(K_DIGITS, (double)B.n_sets * B.n_pass * 2048, [&] {
    launch_batch_digit_offsets(hist, B.d_off, B.n_sets, B.n_pass, B.d_goff, st);
  });
}

void batch_enqueue(BatchImpl& B, const float* xyz, Prof& P) {
  const hipStream_t st = B.stream;
  const uint32_t L = B.L;
  StatusArena sa;
  batch_front(B, xyz, sa, P, B.items);
  batch_sort_passes(B, sa, P, B.items);
  const int fin = B.n_pass & 1;
  DevMeta* meta = B.meta();
  {
    // every level's tables in one pass over the sorted points (batch ranks:
    // the composite keys make each set boundary a box boundary at every level)
    TabLevels T{};
    for (uint32_t l = 0; l <= L; ++l) {
      T.key[l] = B.g[l].key;
      T.begin[l] = B.g[l].begin;
      T.parent[l] = B.g[l].parent;
      T.child[l] = B.g[l].child;
      T.mask[l] = B.g[l].mask;
    }
    const uint32_t tiles = tab_tiles(B.P);
    uint32_t* tcnt = B.tabbuf;
    uint32_t* tpre = B.tabbuf + (size_t)(L + 1) * tiles;
    auto tab = [&](int phase) {
      launch_tables(B.packed, true, B.sb.k[fin], B.sb.v[fin], xyz, B.P, L, tcnt, tpre, T, B.perm,
                    B.sxyz, &meta->n_boxes[0][0], L > 0 ? B.cap[L - 1] : 0, st, phase, B.d_off,
                    3 * L);
    };
    P.run(K_TCOUNT, 0.0, [&] { tab(0); });
    P.run(K_TSCAN, 0.0, [&] { tab(1); });
    P.run(K_LEAF, 0.0, [&] { tab(2); });
    P.run(K_LEVEL, 0.0, [&] { tab(3); });
  }
  LevelPtrs lp{};
  for (uint32_t l = 0; l <= L; ++l) lp.begin[l] = B.g[l].begin;
  P.run(K_REBASE, 0.0, [&] {
    launch_batch_first(lp, L, meta->n_boxes[0], B.d_off, B.n_sets, B.first(), st);
  });
  uint32_t max_cap = 1;
  for (uint32_t l = 0; l <= L; ++l) max_cap = std::max(max_cap, B.cap[l]);
  {
    RebaseArgs ra{};
    for (uint32_t l = 0; l <= L; ++l) {
      ra.n_l[l] = &meta->n_boxes[0][l];
      ra.gkey[l] = (const uint64_t*)B.g[l].key;
      ra.gbegin[l] = B.g[l].begin;
      ra.gparent[l] = l >= 1 ? B.g[l].parent : nullptr;
      ra.gchild[l] = l < L ? B.g[l].child : nullptr;
      ra.fkey[l] = B.fkey[l];
      ra.fbegin[l] = B.fbegin[l];
      ra.fparent[l] = B.fparent[l];
      ra.fchild[l] = B.fchild[l];
    }
    ra.first = B.first();
    ra.set_off = B.d_off;
    ra.n_sets = B.n_sets;
    ra.L = L;
    P.run(K_REBASE, 0.0, [&] { launch_batch_rebase(ra, max_cap, st); });
  }
  for (uint32_t l = 2; l <= L; ++l) {
    ListLevelArgs a{};
    a.level = l;
    a.n_recv_up = B.cap[l - 1];
    a.n_recv_up_dev = &meta->n_boxes[0][l - 1];
    a.recv_key_up = B.g[l - 1].key;
    a.recv_mask_up = B.g[l - 1].mask;
    a.recv_child_up = B.g[l - 1].child;
    a.src_key_up = B.g[l - 1].key;
    a.src_mask_up = B.g[l - 1].mask;
    a.src_child_up = B.g[l - 1].child;
    a.up_all = l == 2 ? 1u : 0u;
    if (!a.up_all) {
      a.e2_off_up = B.goff[l - 1][0];
      a.e2_ent_up = B.ent[l - 1][0];
    }
    a.first_up = B.first_l(l - 1);
    a.first_cur = B.first_l(l);
    a.set_level = B.d_lev;
    a.key_bits_up = B.setbits + 3 * (l - 1);
    uint32_t* c2 = B.cnt;
    uint32_t* c4 = B.cnt + round_up(B.cap[l], 4);
    if (l == 2) P.run(K_COUNT, 0.0, [&] { launch_list_count(true, a, c2, c4, st); });
    {
      uint64_t* st2 = sa.take_words(scan_tiles(B.cap[l]));
      uint64_t* st4 = sa.take_words(scan_tiles(B.cap[l]));
      uint32_t* tk = sa.take_ticket();
      P.run(K_SCAN, 0.0, [&] {
        launch_scan_counts2(c2, c4, B.cap[l], B.goff[l][0], B.goff[l][1], &meta->list_total[0][l],
                            &meta->list_total[1][l], &meta->overflow, st2, st4, tk, st,
                            &meta->n_boxes[0][l]);
      });
    }
    if (l < L) {  // the next level's counts (batch ranks; sets ending at l get zeros)
      a.src_mask_cur = B.g[l].mask;
      a.recv_mask_cur = B.g[l].mask;
      a.recv_child_cur = B.g[l].child;
      a.cnt2_next = B.cnt;
      a.cnt4_next = B.cnt + round_up(B.cap[l + 1], 4);
    }
    P.run(K_FILL, 0.0, [&] {
      launch_list_fill(true, a, B.goff[l][0], B.goff[l][1], B.ent[l][0], B.ent[l][1], st);
    });
  }
  {
    ListRebaseArgs la{};
    for (uint32_t l = 2; l <= L; ++l) {
      la.n_l[l] = &meta->n_boxes[0][l];
      la.gkey[l] = (const uint64_t*)B.g[l].key;
      la.goff2[l] = B.goff[l][0];
      la.goff4[l] = B.goff[l][1];
      la.loff2[l] = B.loff[l][0];
      la.loff4[l] = B.loff[l][1];
    }
    la.first = B.first();
    la.base = B.base(0, 0);
    la.n_sets = B.n_sets;
    la.L = L;
    P.run(K_REBASE, 0.0, [&] { launch_batch_list_rebase(la, max_cap, st); });
  }
  ck(hipMemcpyAsync(B.hblock, B.dblock, B.dblock_b, hipMemcpyDeviceToHost, st));
}

// Times each sort tile size on this batch's real keys; keeps the fastest.
int batch_autotune(BatchImpl& B, const float* xyz) {
  const TuneKey key{(uint32_t)(63 - __builtin_clzll((uint64_t)B.P | 1)), B.n_pass,
                    B.packed ? 1u : 0u};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  Prof off;
  hipEvent_t e0, e1;
  ck(hipEventCreate(&e0));
  ck(hipEventCreate(&e1));
  int best = kSortItemsDefault;
  float best_ms = 1e30f;
  for (int items : {8, 12, 16, kSortWide}) {
    if (items == kSortWide && !B.packed) continue;
    float total = 0;
    for (int rep = 0; rep < 2; ++rep) {
      StatusArena sa;
      batch_front(B, xyz, sa, off, items);
      ck(hipEventRecord(e0, B.stream));
      batch_sort_passes(B, sa, off, items);
      ck(hipEventRecord(e1, B.stream));
      ck(hipEventSynchronize(e1));
      float ms = 0;
      ck(hipEventElapsedTime(&ms, e0, e1));
      if (rep == 1) total = ms;  // the first run warms caches and code
    }
    if (total < best_ms) {
      best_ms = total;
      best = items;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = best;
  return best;
}

// Sub-allocation of one block; with base == nullptr it only measures.
struct Carve {
  char* base = nullptr;
  size_t used = 0;
  template <typename T>
  T* get(size_t count) {
    const size_t b = round_up(std::max<size_t>(count * sizeof(T), 1), 256);
    T* p = base ? (T*)(base + used) : nullptr;
    used += b;
    return p;
  }
};

// Validates the shape and fills the scalar plan: levels, key width, passes
// and per-level capacities (boxes of set i at level l are at most
// min(n_i, 8^min(l, L_i))).
fmmds_status batch_plan(const uint64_t* set_offsets, const uint8_t* levels, uint32_t n_sets,
                        BatchImpl& B) {
  // (set ids are 31 bits in the sort's tile tables)
  if (!set_offsets || !levels || n_sets == 0 || n_sets >= 0x80000000u || set_offsets[0] != 0)
    return FMMDS_ERR_ARG;
  uint32_t L = 0;
  for (uint32_t i = 0; i < n_sets; ++i) {
    if (set_offsets[i + 1] <= set_offsets[i]) return FMMDS_ERR_ARG;
    if (levels[i] < 2 || levels[i] > FMMDS_MAX_LEVEL) return FMMDS_ERR_ARG;
    L = std::max<uint32_t>(L, levels[i]);
  }
  if (set_offsets[n_sets] >= 0xFFFFFFFFull) return FMMDS_ERR_ARG;
  uint32_t setbits = 1;
  while ((1ull << setbits) < n_sets) ++setbits;
  if (setbits + 3 * L > 64) return FMMDS_ERR_ARG;
  B.n_sets = n_sets;
  B.P = (uint32_t)set_offsets[n_sets];
  B.L = L;
  B.setbits = setbits;
  B.keybits = setbits + 3 * L;
  B.packed = B.keybits <= 32;
  // each set is sorted within its own range: only the Morton bits are digits
  B.n_pass = div_up(3 * L, 8);
  for (int k = 0; k < 4; ++k) {
    const uint64_t T = sort_tile_elems(kTileItems[k]);
    uint64_t t = 0;
    for (uint32_t i = 0; i < n_sets; ++i) t += (set_offsets[i + 1] - set_offsets[i] + T - 1) / T;
    B.n_tiles[k] = (uint32_t)t;
  }
  for (uint32_t l = 0; l <= L; ++l) {
    uint64_t c = 0, r = 0;
    for (uint32_t i = 0; i < n_sets; ++i) {
      const uint64_t ni = set_offsets[i + 1] - set_offsets[i];
      const uint32_t e = std::min<uint32_t>(l, levels[i]);
      const uint64_t boxes = std::min<uint64_t>(ni, 1ull << (3 * e));
      c += boxes;
      if (levels[i] >= l) r += boxes;
    }
    B.cap[l] = (uint32_t)c;
    B.rcap[l] = (uint32_t)r;
    if (l >= 2 && 189ull * r > 0xFFFFFFFFull) return FMMDS_ERR_OVERFLOW;
  }
  return FMMDS_OK;
}

// Words of the set-aligned tile tables: per tile size, start (n_tiles + 1)
// then set (n_tiles).
size_t tile_table_words(const BatchImpl& B) {
  size_t w = 0;
  for (int k = 0; k < 4; ++k) w += 2 * (size_t)B.n_tiles[k] + 1;
  return w;
}

// Fills the tables tile_table_words describes: tiles of sort_tile_elems
// elements laid over each set in turn (the last one of a set ragged), each
// tile's set with the top bit set on a set's first tile.
void fill_tile_tables(const BatchImpl& B, uint32_t* out) {
  for (int k = 0; k < 4; ++k) {
    const uint64_t T = sort_tile_elems(kTileItems[k]);
    uint32_t* start = out;
    uint32_t* set = out + B.n_tiles[k] + 1;
    uint32_t t = 0;
    for (uint32_t i = 0; i < B.n_sets; ++i)
      for (uint64_t e = B.off[i]; e < B.off[i + 1]; e += T, ++t) {
        start[t] = (uint32_t)e;
        set[t] = i | (e == B.off[i] ? 0x80000000u : 0u);
      }
    start[t] = B.P;
    out += 2 * (size_t)B.n_tiles[k] + 1;
  }
}

// Every device buffer of a planned batch, carved from one block.
void batch_layout(BatchImpl& B, Carve& M) {
  const uint32_t n_sets = B.n_sets, P = B.P, L = B.L;
  B.d_off = M.get<uint64_t>(n_sets + 1);
  B.d_lev = M.get<uint8_t>(n_sets);
  B.d_tiles = M.get<uint32_t>(tile_table_words(B));
  size_t o = 0;
  for (int k = 0; k < 4; ++k) {
    B.d_tstart[k] = B.d_tiles ? B.d_tiles + o : nullptr;
    o += B.n_tiles[k] + 1;
    B.d_tset[k] = B.d_tiles ? B.d_tiles + o : nullptr;
    o += B.n_tiles[k];
  }
  B.d_goff = M.get<uint32_t>((size_t)n_sets * B.n_pass * 256);
  B.sb.k[0] = M.get<uint64_t>(P);
  B.sb.k[1] = M.get<uint64_t>(P);
  B.sb.v[0] = B.sb.v[1] = nullptr;
  if (!B.packed) {
    B.sb.v[0] = M.get<uint32_t>(P);
    B.sb.v[1] = M.get<uint32_t>(P);
  }
  B.perm = M.get<uint32_t>(P);
  B.sxyz = M.get<float>(3 * (size_t)P);
  B.tabbuf = M.get<uint32_t>((size_t)2 * (L + 1) * tab_tiles(P));
  uint32_t cmax = 0;
  for (uint32_t l = 0; l <= L; ++l) {
    const size_t c = B.cap[l];
    cmax = std::max<uint32_t>(cmax, (uint32_t)c);
    LevelBufs& G = B.g[l];
    G = LevelBufs();
    G.cap = (uint32_t)c;
    G.key = M.get<uint64_t>(c);
    G.begin = M.get<uint32_t>(c + 1);
    if (l >= 1) G.parent = M.get<uint32_t>(c);
    if (l < L) {
      G.child = M.get<uint32_t>(c + 1);
      G.mask = M.get<uint8_t>(c);
    }
    B.fkey[l] = M.get<uint64_t>(c);
    B.fbegin[l] = M.get<uint32_t>(c + n_sets);
    B.fparent[l] = l >= 1 ? M.get<uint32_t>(c) : nullptr;
    B.fchild[l] = l < L ? M.get<uint32_t>(c + n_sets) : nullptr;
    if (l >= 2) {
      for (int k = 0; k < 2; ++k) {
        B.goff[l][k] = M.get<uint32_t>(c + 1);
        B.loff[l][k] = M.get<uint32_t>(c + n_sets);
        B.ent[l][k] = M.get<uint32_t>((size_t)(k == 0 ? 27 : 189) * B.rcap[l]);
      }
    }
  }
  B.cnt = M.get<uint32_t>(2 * round_up(std::max<uint32_t>(cmax, 1), 4));
  // metadata block and the zeroed workspace around it
  B.first_at = round_up(sizeof(DevMeta), 256);
  B.base_at = round_up(B.first_at + (size_t)(L + 1) * (n_sets + 1) * 4, 256);
  B.dblock_b = round_up(B.base_at + (size_t)(L + 1) * 2 * (n_sets + 1) * 4, 256);
  B.hist_at = B.dblock_b;
  B.tick_at = B.hist_at + round_up((size_t)n_sets * B.n_pass * 256 * 4, 256);
  B.n_tickets = B.n_pass + 1 + L + 2 * (L + 1);
  B.words_at = B.tick_at + round_up(B.n_tickets * 4, 256);
  B.list_words = 0;
  for (uint32_t l = 2; l <= L; ++l) B.list_words += 2 * (size_t)scan_tiles(B.cap[l]);
  const size_t words =
      (size_t)B.n_pass * *std::max_element(B.n_tiles, B.n_tiles + 4) * 256 + B.list_words;
  B.n_words = words;
  B.ws_b = round_up(B.words_at + words * 8, 256);
  B.ws = M.get<char>(B.ws_b);
  B.dblock = B.ws;
}

fmmds_status batch_create(const uint64_t* set_offsets, const uint8_t* levels, uint32_t n_sets,
                          const fmmds_options* opt, fmmds_batch** out) {
  if (!set_offsets || !levels || !opt || n_sets == 0) return FMMDS_ERR_ARG;
  if (opt->key_bits != 64 || opt->cluster_s != 0 || opt->reserved != 0 ||
      ((opt->alloc == nullptr) != (opt->release == nullptr)))
    return FMMDS_ERR_ARG;
  BatchImpl* B = new (std::nothrow) BatchImpl();
  if (!B) return FMMDS_ERR_NOMEM;
  fmmds_status result = batch_plan(set_offsets, levels, n_sets, *B);
  if (result != FMMDS_OK) {
    delete B;
    return result;
  }
  try {
    B->off.assign(set_offsets, set_offsets + n_sets + 1);
    B->lev.assign(levels, levels + n_sets);
    if (const char* e = std::getenv("FMMDS_BATCH_SORT_ITEMS")) {
      const int v = std::atoi(e);
      if (v == 8 || v == 12 || v == 16 || (v == kSortWide && B->packed)) {
        B->items = v;
        B->items_fixed = true;
      }
    }
    if (opt->stream) {
      B->stream = (hipStream_t)opt->stream;
    } else {
      ck(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking));
      B->own_stream = true;
    }
    B->A.alloc = opt->alloc;
    B->A.release = opt->release;
    B->A.ctx = opt->alloc_ctx;
    B->A.stream = B->stream;
    B->mem.A = &B->A;
    Carve M;
    batch_layout(*B, M);  // measure
    M.base = B->mem.get<char>(M.used);
    M.used = 0;
    batch_layout(*B, M);  // assign
    // Pinned host block: the metadata mirror, then the offsets and levels
    // staged for an asynchronous upload (it lives as long as the batch).
    const size_t stage_off = round_up(B->dblock_b, 256);
    const size_t stage_lev = stage_off + round_up((n_sets + 1) * 8, 256);
    const size_t stage_tiles = stage_lev + round_up(n_sets, 256);
    const size_t tiles_b = tile_table_words(*B) * 4;
    B->hblock_b = stage_tiles + tiles_b;
    B->hblock = (char*)pinned_alloc(B->hblock_b);
    if (!B->hblock) throw Fail{FMMDS_ERR_NOMEM};
    std::memcpy(B->hblock + stage_off, set_offsets, (n_sets + 1) * 8);
    std::memcpy(B->hblock + stage_lev, levels, n_sets);
    fill_tile_tables(*B, (uint32_t*)(B->hblock + stage_tiles));
    ck(hipMemcpyAsync(B->d_off, B->hblock + stage_off, (n_sets + 1) * 8, hipMemcpyHostToDevice,
                      B->stream));
    ck(hipMemcpyAsync(B->d_lev, B->hblock + stage_lev, n_sets, hipMemcpyHostToDevice, B->stream));
    ck(hipMemcpyAsync(B->d_tiles, B->hblock + stage_tiles, tiles_b, hipMemcpyHostToDevice,
                      B->stream));
    B->trees.assign(n_sets, fmmds_tree());
    B->views.resize(n_sets);
    for (uint32_t i = 0; i < n_sets; ++i) B->views[i].view = true;
    B->footprint = cache_round(round_up(M.used, 256));
  } catch (const Fail& f) {
    result = f.st;
  } catch (const std::bad_alloc&) {
    result = FMMDS_ERR_NOMEM;
  }
  if (result != FMMDS_OK) {
    (void)hipGetLastError();
    B->mem.release_all();
    if (B->hblock) {
      (void)hipStreamSynchronize(B->stream);
      pinned_release(B->hblock, B->hblock_b, nullptr);
    }
    if (B->own_stream) (void)hipStreamDestroy(B->stream);
    delete B;
    return result;
  }
  *out = (fmmds_batch*)B;
  return FMMDS_OK;
}

// Device bytes fmmds_batch_create allocates for this shape (host only: the
// same plan and layout, measured, rounded as the allocator rounds).
fmmds_status batch_footprint(const uint64_t* set_offsets, const uint8_t* levels, uint32_t n_sets,
                             uint64_t* bytes) {
  if (!bytes) return FMMDS_ERR_ARG;
  try {
    BatchImpl B;
    const fmmds_status st = batch_plan(set_offsets, levels, n_sets, B);
    if (st != FMMDS_OK) return st;
    Carve M;
    batch_layout(B, M);
    *bytes = cache_round(round_up(M.used, 256));
  } catch (const std::bad_alloc&) {
    return FMMDS_ERR_NOMEM;
  }
  return FMMDS_OK;
}

fmmds_status batch_launch(BatchImpl* B, const float* xyz, int capture) {
  if (!B || !xyz) return FMMDS_ERR_ARG;
  try {
    if (capture) {
      if (B->exec && B->graph_xyz != xyz) return FMMDS_ERR_ARG;
      if (!B->exec) {
        if (!B->items_fixed) B->items = batch_autotune(*B, xyz);
        Prof off;
        ck(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
        try {
          batch_enqueue(*B, xyz, off);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(B->stream, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        ck(hipStreamEndCapture(B->stream, &B->graph));
        ck(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
        B->graph_xyz = xyz;
      }
      ck(hipGraphLaunch(B->exec, B->stream));
    } else if (!B->items_fixed) {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune.find(TuneKey{(uint32_t)(63 - __builtin_clzll((uint64_t)B->P | 1)),
                                    B->n_pass, B->packed ? 1u : 0u});
      if (it != g_tune.end()) B->items = it->second;
    }
    if (!capture) {
      Prof P;
      P.on = g_prof_on.load() != 0;
      P.only = g_prof_only.load();
      P.s = B->stream;
      batch_enqueue(*B, xyz, P);
      P.finish([](const Prof::Rec&) { return 0.0; });
    }
    B->done = record_event(B->stream);
    B->launched = true;
  } catch (const Fail& f) {
    (void)hipGetLastError();
    return f.st;
  }
  return FMMDS_OK;
}

fmmds_status batch_wait(BatchImpl* B) {
  if (!B || !B->launched) return FMMDS_ERR_ARG;
  try {
    ck(hipStreamSynchronize(B->stream));
  } catch (const Fail& f) {
    return f.st;
  }
  const DevMeta* hm = (const DevMeta*)B->hblock;
  if (hm->err_range) return FMMDS_ERR_RANGE;
  if (hm->overflow) return FMMDS_ERR_OVERFLOW;
  const uint32_t* first = (const uint32_t*)(B->hblock + B->first_at);
  const uint32_t* base = (const uint32_t*)(B->hblock + B->base_at);
  const uint32_t ns = B->n_sets;
  for (uint32_t i = 0; i < ns; ++i) {
    fmmds_tree& t = B->trees[i];
    TreeImpl& v = B->views[i];
    const uint32_t Li = B->lev[i];
    const uint64_t o = B->off[i];
    std::memset(&t, 0, sizeof(t));
    t.depth = Li;
    t.key_bits = 64;
    t.max_level = Li;
    t.shared = 1;
    t.n_src = t.n_recv = (uint32_t)(B->off[i + 1] - o);
    t.src_perm = t.recv_perm = B->perm + o;
    t.src_sorted_xyz = t.recv_sorted_xyz = B->sxyz + 3 * o;
    for (uint32_t l = 0; l <= Li; ++l) {
      const uint32_t f = first[(size_t)l * (ns + 1) + i];
      const uint32_t nl = first[(size_t)l * (ns + 1) + i + 1] - f;
      fmmds_level& lv = t.src[l];
      lv.n = nl;
      lv.key = B->fkey[l] + f;
      lv.begin = B->fbegin[l] + f + i;
      lv.parent = l >= 1 ? B->fparent[l] + f : nullptr;
      lv.child = l < Li ? B->fchild[l] + f + i : nullptr;
      t.recv[l] = lv;
      if (l >= 2) {
        for (int k = 0; k < 2; ++k) {
          const uint32_t* bk = base + ((size_t)(l * 2 + k)) * (ns + 1);
          v.lists[l].off[k] = B->loff[l][k] + f + i;
          v.lists[l].ent[k] = B->ent[l][k] + bk[i];
          v.lists[l].total[k] = bk[i + 1] - bk[i];
        }
        v.n_recv_boxes[l] = nl;
      }
    }
    t.impl = &v;
  }
  return FMMDS_OK;
}

// No host wait: the blocks go back to the caches tagged with the event of
// the batch's last launch (or of its creation's uploads).
void batch_free(BatchImpl* B) {
  if (!B) return;
  EventRef ready = B->done ? B->done : record_event(B->stream);
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->mem.release_all(ready);
  pinned_release(B->hblock, B->hblock_b, ready);
  if (B->own_stream) (void)hipStreamDestroy(B->stream);  // returns once its work is queued
  delete B;
}

fmmds_status list_query(const fmmds_tree* t, int kind, uint32_t level, const uint32_t** offsets,
                        const uint32_t** entries, uint32_t* n_recv_boxes, uint64_t* n_entries) {
  if (!t || !t->impl || !offsets || !entries || !n_recv_boxes || !n_entries) return FMMDS_ERR_ARG;
  if (level < 2 || level > t->depth) return FMMDS_ERR_LEVEL;
  const TreeImpl* impl = (const TreeImpl*)t->impl;
  const ListBufs& LB = impl->lists[level];
  *offsets = LB.off[kind];
  *entries = LB.ent[kind];
  *n_recv_boxes = impl->n_recv_boxes[level];
  *n_entries = LB.total[kind];
  return FMMDS_OK;
}

// ---------------------------------------------------------------------------
// Simulated partition and source box types (fmmds_partition, fmmds_box_types).
// ---------------------------------------------------------------------------
bool par_level_ok(const fmmds_tree* t, uint32_t l_par) {
  return l_par >= 3 && l_par <= t->depth && l_par <= 10;
}

fmmds_status partition(const fmmds_tree* t, uint32_t l_par, uint32_t n_ranks, uint32_t* owner,
                       hipStream_t st) {
  if (!t || !t->impl || !owner || n_ranks == 0) return FMMDS_ERR_ARG;
  if (!par_level_ok(t, l_par)) return FMMDS_ERR_LEVEL;
  const fmmds_level& rl = t->recv[l_par];
  launch_partition(t->key_bits == 64, rl.key, rl.begin, rl.n, t->n_recv, n_ranks, l_par, owner,
                   st);
  return hipGetLastError() == hipSuccess ? FMMDS_OK : FMMDS_ERR_DEVICE;
}

fmmds_status box_types(const fmmds_tree* t, uint32_t l_par, const uint32_t* owner, uint32_t rank,
                       uint8_t* types, hipStream_t st) {
  if (!t || !t->impl || !owner || !types) return FMMDS_ERR_ARG;
  if (!par_level_ok(t, l_par)) return FMMDS_ERR_LEVEL;
  const TreeImpl* impl = (const TreeImpl*)t->impl;
  const bool key64 = t->key_bits == 64;
  const uint32_t l_crit = l_par - 1;
  uint32_t n_max = 1, r_max = 1;
  for (uint32_t l = l_crit; l <= t->depth; ++l) {
    n_max = std::max(n_max, t->src[l].n);
    r_max = std::max(r_max, t->recv[l].n);
  }
  // two mark arrays, the work counter and the work list, each 16-byte
  // aligned and zeroed in whole 16-byte words
  const size_t marks_b = round_up((size_t)n_max, 16);
  const size_t clear_b = 2 * marks_b + 16;
  void* flags = cache_alloc(clear_b + round_up((size_t)r_max * 4, 16), st);
  if (!flags) return FMMDS_ERR_NOMEM;
  uint8_t* elsewhere = (uint8_t*)flags;
  uint8_t* here = elsewhere + marks_b;
  uint32_t* n_work = (uint32_t*)(here + marks_b);
  uint32_t* work = n_work + 4;
  size_t at = 0;
  for (uint32_t l = 2; l <= t->depth; ++l) {
    const uint32_t ns = t->src[l].n;
    uint8_t* ty = types + at;
    at += ns;
    if (l < l_crit) {
      launch_fill_u8(ty, ns, FMMDS_BOX_DOMESTIC, st);
      continue;
    }
    launch_zero(flags, clear_b, st);
    BoxTypeLevel a{};
    a.level = l;
    a.l_par = l_par;
    a.rank = rank;
    a.n_recv = t->recv[l].n;
    a.n_src = ns;
    a.rkey = t->recv[l].key;
    a.skey = t->src[l].key;
    a.owner = owner;
    a.e4_off = impl->lists[l].off[1];
    a.e4_ent = impl->lists[l].ent[1];
    a.elsewhere = elsewhere;
    a.here = here;
    a.work = work;
    a.n_work = n_work;
    a.types = ty;
    if (l == l_crit) {
      a.rkey_par = t->recv[l_par].key;
      a.skey_par = t->src[l_par].key;
      a.rchild = t->recv[l].child;
      a.schild = t->src[l].child;
      launch_types_crit(key64, a, st);
    } else {
      launch_types_deep(key64, a, st);
    }
  }
  cache_release(flags, st);
  return hipGetLastError() == hipSuccess ? FMMDS_OK : FMMDS_ERR_DEVICE;
}

// Bytes of the near-field scratch: packed sources, the dense path's tasks,
// its counters.
struct NearScratch {
  size_t src_b, task_b, total;
  explicit NearScratch(const fmmds_tree* t)
      : src_b(round_up((size_t)t->n_src * 16, 256)),
        task_b(round_up(near_field_max_tasks(t->n_recv) * sizeof(uint2), 256)),
        total(src_b + task_b + 256) {}
};

void near_field_launch(const fmmds_tree* t, const NearScratch& ns, char* scratch,
                       const float* charges, float* phi, uint64_t* n_pairs, hipStream_t st) {
  const TreeImpl* impl = (const TreeImpl*)t->impl;
  const uint32_t D = t->depth;
  float4* src4 = (float4*)scratch;
  uint2* tasks = (uint2*)(scratch + ns.src_b);
  uint32_t* counters = (uint32_t*)(scratch + ns.src_b + ns.task_b);
  launch_pack_sources(t->src_sorted_xyz, t->src_perm, charges, t->n_src, src4, counters, st);
  launch_near_field(t->recv[D].n, t->n_recv, t->recv[D].begin, t->recv_sorted_xyz, t->recv_perm,
                    impl->lists[D].off[0], impl->lists[D].ent[0], t->src[D].begin, src4, phi,
                    (unsigned long long*)n_pairs, tasks, counters, st);
}

fmmds_status near_field(const fmmds_tree* t, const float* charges, float* phi,
                        uint64_t* n_pairs, hipStream_t st) {
  if (!t || !t->impl || !phi) return FMMDS_ERR_ARG;
  const NearScratch ns(t);
  char* scratch = (char*)cache_alloc(ns.total, st);
  if (!scratch) return FMMDS_ERR_NOMEM;
  near_field_launch(t, ns, scratch, charges, phi, n_pairs, st);
  cache_release(scratch, st);
  return hipGetLastError() == hipSuccess ? FMMDS_OK : FMMDS_ERR_DEVICE;
}

// The same kernels on the fixed per-device scratch array: no allocation.
fmmds_status near_field_static(const fmmds_tree* t, const float* charges, float* phi,
                               uint64_t* n_pairs, hipStream_t st) {
  if (!t || !t->impl || !phi) return FMMDS_ERR_ARG;
  const NearScratch ns(t);
  if (ns.total > kNearStaticBytes) return FMMDS_ERR_TOO_LARGE;
  void* scratch = nullptr;
  const fmmds_status s = near_field_static_scratch(&scratch);
  if (s != FMMDS_OK) return s;
  near_field_launch(t, ns, (char*)scratch, charges, phi, n_pairs, st);
  return hipGetLastError() == hipSuccess ? FMMDS_OK : FMMDS_ERR_DEVICE;
}

}  // namespace
}  // namespace fmmds

extern "C" {

fmmds_status fmmds_build(const float* src_xyz, uint32_t n_src, const float* recv_xyz,
                         uint32_t n_recv, const fmmds_options* opt, fmmds_tree** out) {
  if (!out) return FMMDS_ERR_ARG;
  *out = nullptr;
  return fmmds::build(src_xyz, n_src, recv_xyz, n_recv, opt, out);
}

fmmds_status fmmds_rebuild(const fmmds_tree* prev, const float* src_xyz, const float* recv_xyz,
                           uint32_t in_prev_order, const fmmds_options* opt, fmmds_tree** out) {
  if (!out) return FMMDS_ERR_ARG;
  *out = nullptr;
  if (!prev || !opt || in_prev_order > 1) return FMMDS_ERR_ARG;
  if ((recv_xyz == nullptr) != (prev->shared != 0)) return FMMDS_ERR_ARG;
  if (opt->max_level != prev->max_level) return FMMDS_ERR_ARG;
  if (!prev->src_perm || !prev->src_sorted_xyz || !prev->recv_perm || !prev->recv_sorted_xyz)
    return FMMDS_ERR_ARG;
  // Positions in the original order: the incremental path would first
  // gather them into the previous order, a random 12-byte read per point,
  // which costs more than the full sort it saves; the fresh build returns the
  // same tree.
  if (in_prev_order == 0)
    return fmmds::build(src_xyz, prev->n_src, recv_xyz, prev->n_recv, opt, out);
  return fmmds::build(src_xyz, prev->n_src, recv_xyz, prev->n_recv, opt, out, prev);
}

fmmds_status fmmds_build_dense(const float* src_xyz, uint32_t n_src, const float* recv_xyz,
                               uint32_t n_recv, const fmmds_options* opt, fmmds_tree** out) {
  if (!out) return FMMDS_ERR_ARG;
  *out = nullptr;
  return fmmds::build(src_xyz, n_src, recv_xyz, n_recv, opt, out, nullptr, true);
}

fmmds_status fmmds_neighbors(const fmmds_tree* t, uint32_t level, const uint32_t** offsets,
                             const uint32_t** entries, uint32_t* n_recv_boxes,
                             uint64_t* n_entries) {
  return fmmds::list_query(t, 0, level, offsets, entries, n_recv_boxes, n_entries);
}

fmmds_status fmmds_interactions(const fmmds_tree* t, uint32_t level, const uint32_t** offsets,
                                const uint32_t** entries, uint32_t* n_recv_boxes,
                                uint64_t* n_entries) {
  return fmmds::list_query(t, 1, level, offsets, entries, n_recv_boxes, n_entries);
}

void fmmds_free(fmmds_tree* t) {
  if (!t) return;
  fmmds::TreeImpl* impl = (fmmds::TreeImpl*)t->impl;
  if (impl && impl->view) return;
  if (impl) {
    impl->outs.release_all();
    delete impl;
  }
  delete t;
}

fmmds_status fmmds_batch_create(const uint64_t* set_offsets, const uint8_t* levels,
                                uint32_t n_sets, const fmmds_options* opt, fmmds_batch** out) {
  if (!out) return FMMDS_ERR_ARG;
  *out = nullptr;
  return fmmds::batch_create(set_offsets, levels, n_sets, opt, out);
}

fmmds_status fmmds_batch_launch(fmmds_batch* b, const float* xyz, int capture) {
  return fmmds::batch_launch((fmmds::BatchImpl*)b, xyz, capture);
}

fmmds_status fmmds_batch_wait(fmmds_batch* b) {
  return fmmds::batch_wait((fmmds::BatchImpl*)b);
}

const fmmds_tree* fmmds_batch_tree(const fmmds_batch* b, uint32_t set) {
  const fmmds::BatchImpl* B = (const fmmds::BatchImpl*)b;
  if (!B || set >= B->n_sets || B->trees[set].impl == nullptr) return nullptr;
  return &B->trees[set];
}

fmmds_status fmmds_batch_footprint(const uint64_t* set_offsets, const uint8_t* levels,
                                   uint32_t n_sets, uint64_t* bytes) {
  return fmmds::batch_footprint(set_offsets, levels, n_sets, bytes);
}

uint64_t fmmds_batch_bytes(const fmmds_batch* b) {
  return b ? ((const fmmds::BatchImpl*)b)->footprint : 0;
}

uint32_t fmmds_batch_sort_items(const fmmds_batch* b) {
  return b ? (uint32_t)((const fmmds::BatchImpl*)b)->items : 0;
}

void fmmds_batch_free(fmmds_batch* b) { fmmds::batch_free((fmmds::BatchImpl*)b); }

fmmds_status fmmds_build_batch(const float* xyz, const uint64_t* set_offsets,
                               const uint8_t* levels, uint32_t n_sets, const fmmds_options* opt,
                               fmmds_batch** out) {
  if (!out) return FMMDS_ERR_ARG;
  *out = nullptr;
  if (!xyz) return FMMDS_ERR_ARG;
  fmmds_batch* b = nullptr;
  fmmds_status st = fmmds::batch_create(set_offsets, levels, n_sets, opt, &b);
  if (st != FMMDS_OK) return st;
  st = fmmds::batch_launch((fmmds::BatchImpl*)b, xyz, 0);
  if (st == FMMDS_OK) st = fmmds::batch_wait((fmmds::BatchImpl*)b);
  if (st != FMMDS_OK) {
    fmmds::batch_free((fmmds::BatchImpl*)b);
    return st;
  }
  *out = b;
  return FMMDS_OK;
}

void fmmds_free_batch(fmmds_batch* b) { fmmds::batch_free((fmmds::BatchImpl*)b); }

fmmds_status fmmds_displace(const fmmds_displace_set* sets, uint32_t n_sets, float sigma,
                            float* out, void* stream) {
  if (!sets || n_sets == 0) return FMMDS_ERR_ARG;
  for (uint32_t i = 0; i < n_sets; ++i)
    if (!sets[i].xyz || sets[i].n == 0) return FMMDS_ERR_ARG;
  fmmds::DisplaceArgs a;
  for (uint32_t b = 0; b < n_sets; b += fmmds::kDisplaceSets) {
    a.n = std::min<uint32_t>(n_sets - b, fmmds::kDisplaceSets);
    a.first[0] = 0;
    for (uint32_t k = 0; k < a.n; ++k) {
      const fmmds_displace_set& d = sets[b + k];
      a.xyz[k] = d.xyz;
      a.seed[k] = d.seed;
      a.out_first[k] = d.out_first;
      a.first[k + 1] = a.first[k] + d.n;
    }
    fmmds::launch_displace(a, sigma, out, (hipStream_t)stream);
  }
  if (hipGetLastError() != hipSuccess) return FMMDS_ERR_DEVICE;
  return FMMDS_OK;
}

fmmds_status fmmds_partition(const fmmds_tree* t, uint32_t l_par, uint32_t n_ranks,
                             uint32_t* owner, void* stream) {
  return fmmds::partition(t, l_par, n_ranks, owner, (hipStream_t)stream);
}

fmmds_status fmmds_box_types(const fmmds_tree* t, uint32_t l_par, const uint32_t* owner,
                             uint32_t rank, uint8_t* types, void* stream) {
  return fmmds::box_types(t, l_par, owner, rank, types, (hipStream_t)stream);
}

fmmds_status fmmds_near_field(const fmmds_tree* t, const float* charges, float* phi,
                              uint64_t* n_pairs, void* stream) {
  return fmmds::near_field(t, charges, phi, n_pairs, (hipStream_t)stream);
}

fmmds_status fmmds_near_field_static(const fmmds_tree* t, const float* charges, float* phi,
                                     uint64_t* n_pairs, void* stream) {
  return fmmds::near_field_static(t, charges, phi, n_pairs, (hipStream_t)stream);
}

void fmmds_cache_info(uint64_t* hits, uint64_t* misses, uint64_t* miss_bytes,
                      uint64_t* cached_bytes) {
  std::lock_guard<std::mutex> g(fmmds::g_cache_mu);
  uint64_t c = 0;
  for (auto& d : fmmds::g_cache)
    for (auto& kv : d.second) c += kv.first;
  if (hits) *hits = fmmds::g_cache_hits;
  if (misses) *misses = fmmds::g_cache_misses;
  if (miss_bytes) *miss_bytes = fmmds::g_cache_miss_bytes;
  if (cached_bytes) *cached_bytes = c;
}

void fmmds_trim(void) {
  std::lock_guard<std::mutex> g(fmmds::g_cache_mu);
  int dev = 0;
  (void)hipGetDevice(&dev);
  bool any = false;
  for (auto& d : fmmds::g_cache) any |= !d.second.empty();
  if (!any) return;
  (void)hipDeviceSynchronize();
  for (auto& d : fmmds::g_cache) {
    (void)hipSetDevice(d.first);
    for (auto& kv : d.second) (void)hipFree(kv.second.p);
    d.second.clear();
  }
  (void)hipSetDevice(dev);
}

void fmmds_profile_enable(int on, const char* only) {
  int cls = -1;
  if (only) {
    for (int k = 0; k < fmmds::K_NCLASS; ++k)
      if (std::strcmp(only, fmmds::kClassName[k]) == 0) cls = k;
  }
  fmmds::g_prof_only.store(cls);
  fmmds::g_prof_on.store(on == 2 ? 2 : on ? 1 : 0);
}

void fmmds_profile_reset(void) {
  std::lock_guard<std::mutex> g(fmmds::g_prof_mu);
  fmmds::resolve_pending(true);
  for (auto& c : fmmds::g_prof) c = fmmds::ClassStat();
}

uint32_t fmmds_profile_read(fmmds_kernel_stat* out, uint32_t cap) {
  std::lock_guard<std::mutex> g(fmmds::g_prof_mu);
  fmmds::resolve_pending(true);
  uint32_t n = 0;
  for (int k = 0; k < fmmds::K_NCLASS; ++k) {
    if (fmmds::g_prof[k].launches == 0) continue;
    if (out && n < cap) {
      std::memset(out[n].name, 0, sizeof(out[n].name));
      std::strncpy(out[n].name, fmmds::kClassName[k], sizeof(out[n].name) - 1);
      out[n].launches = fmmds::g_prof[k].launches;
      out[n].total_ms = fmmds::g_prof[k].ms;
      out[n].bytes = fmmds::g_prof[k].bytes;
    }
    ++n;
  }
  return n;
}

const char* fmmds_status_string(fmmds_status s) {
  switch (s) {
    case FMMDS_OK: return "ok";
    case FMMDS_ERR_ARG: return "invalid argument";
    case FMMDS_ERR_RANGE: return "coordinate outside [0, 1)";
    case FMMDS_ERR_NOMEM: return "out of device memory";
    case FMMDS_ERR_DEVICE: return "HIP runtime error";
    case FMMDS_ERR_LEVEL: return "level outside [2, depth]";
    case FMMDS_ERR_OVERFLOW: return "list too long for 32-bit offsets";
    case FMMDS_ERR_TOO_LARGE: return "input larger than the fixed scratch of the entry point";
  }
  return "unknown status";
}

}  // extern "C"
