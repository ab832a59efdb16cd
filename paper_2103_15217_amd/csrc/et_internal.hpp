// Internal declarations of the Euler-tour library: context, scratch pool,
// device status bits, wave64 helpers and the launchers each .hip unit
// exports to the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>
#include <map>
#include <string>
#include <vector>

#include "../../include/et.h"

struct et_tree;

namespace et {

// ---------------------------------------------------------------- status bits
// Kernels OR these into the context's device status word.
enum : uint32_t {
  ST_BAD_PARENT = 1u << 0,   // parent id out of range or self parent
  ST_ROOTS = 1u << 1,        // zero or several roots
  ST_UNREACHED = 1u << 2,    // an element / node is not reachable from a head (cycle)
  ST_BAD_SUCC = 1u << 3,     // successor out of range
  ST_BAD_HEAD = 1u << 4,     // list head out of range or unused
  ST_OVERFLOW = 1u << 5,     // walk bound or continuation space exhausted
  ST_BAD_QUERY = 1u << 6,    // query id out of range
  ST_BAD_CSR = 1u << 7,      // CSR not symmetric / column out of range / rows unsorted
  ST_BAD_INDEX = 1u << 8,    // a gathered table index failed its bounds check
  ST_OUT_SIZE = 1u << 9,     // a caller's output buffer is smaller than the result
};

// ---------------------------------------------------------------- context
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};

// Launch shape of the sublist list ranking (tunable per context).
struct LrShape {
  int k1_log2 = 4;       // level 1: one splitter per 2^k1 consecutive ids
  int per_wave1 = 256;   // level 1: sublists owned by one wavefront
  int kn_log2 = 3;       // upper levels: one splitter per 2^kn elements
  int per_waven = 128;   // upper levels: sublists per wavefront
};

// Range-minimum block size and query workgroup size (tunable per context).
struct QueryShape {
  int rmq_log = 5;   // range-minimum blocks of 2^rmq_log positions (5 or 6)
  int block = 256;   // threads per workgroup of the LCA query kernels
};
constexpr int kQueryBlockMax = 1024;

struct Ctx {
  int device = 0;
  LrShape lr;
  QueryShape qs;
  // kernel timing: when enabled, every instrumented launch is bracketed by
  // a pair of events on its stream
  bool profiling = false;
  std::string prof_only;  // time only this kernel when non-empty
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> spare_events;
  std::vector<hipEvent_t> spare_sync;  // timing-free events for cross-stream pool reuse
  uint32_t* d_status = nullptr;      // accumulated status bits
  int32_t* d_scalars = nullptr;      // small per-call device scalars (root, head, counters)
  int64_t* d_bcount = nullptr;       // bridge count of the last et_bridges
  void* d_fixed = nullptr;           // this device's fixed scratch (et_list_rank_noalloc)
  uint32_t* d_fused = nullptr;       // work counter pair of the one-launch small-tree batch
  // caching pool: free blocks by size, each with the stream that released it
  struct FreeBlock {
    void* p;
    hipStream_t s;
  };
  std::multimap<size_t, FreeBlock> free_blocks;
  std::map<void*, size_t> live_blocks;
  size_t pool_bytes = 0;       // device bytes the pool holds (live + cached)
  size_t pool_live = 0;        // of which handed out
  size_t pool_peak_live = 0;   // largest pool_live since the last reset
};

// Scratch allocation from the context pool. Reuse is stream-ordered: a
// block released on stream A and taken for work on stream B makes B wait
// for an event recorded on A at that moment (which follows every use of the
// block enqueued on A); on the same stream no wait is needed. During stream
// capture the wait is skipped (capture starts from a synchronised device).
void* pool_get(Ctx* c, size_t bytes, hipStream_t s);
void pool_put(Ctx* c, void* p, hipStream_t s);

hipEvent_t prof_event(Ctx* c);
hipEvent_t sync_event(Ctx* c);

// Brackets the launches issued during its lifetime with events (if enabled).
struct ProfScope {
  Ctx* c;
  hipStream_t s;
  const char* name;
  hipEvent_t a = nullptr;
  ProfScope(Ctx* ctx, hipStream_t st, const char* nm) : c(ctx), s(st), name(nm) {
    if (c->profiling && (c->prof_only.empty() || c->prof_only == nm)) {
      a = prof_event(c);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = prof_event(c);
      if (b) {
        (void)hipEventRecord(b, s);
        c->prof.push_back({name, a, b});
      }
    }
  }
};
#define ET_CAT2(a, b) a##b
#define ET_CAT(a, b) ET_CAT2(a, b)
#define ET_PROF(ctx, stream, name) ::et::ProfScope ET_CAT(et_prof_, __LINE__)(ctx, stream, name)

// Scratch of one call. Pool mode (the default): blocks come from the
// context's pool and go back to it, on the call's stream, at scope exit.
// Arena mode: blocks are carved in order from a caller-provided region
// (nothing is allocated; running past its end sets `failed`). Counting mode
// (arena with a null base): nothing is handed out that may be used, only
// `used` is summed, to size an arena before any launch.
struct Scratch {
  Ctx* c;
  hipStream_t s;
  std::vector<void*> blocks;
  bool failed = false;
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  bool arena_mode = false, counting = false;
  Scratch(Ctx* ctx, hipStream_t st) : c(ctx), s(st) {}
  Scratch(Ctx* ctx, hipStream_t st, void* base, size_t bytes)
      : c(ctx), s(st), arena(static_cast<char*>(base)), cap(bytes), arena_mode(true), counting(base == nullptr) {}
  template <typename T>
  T* get(size_t count) {
    const size_t bytes = count * sizeof(T) + 16;
    if (arena_mode) {
      const size_t at = (used + 255) & ~(size_t)255;
      used = at + bytes;
      if (counting) return reinterpret_cast<T*>((uintptr_t)(at + 256));  // an address never dereferenced
      if (used > cap) {
        failed = true;
        return nullptr;
      }
      return reinterpret_cast<T*>(arena + at);
    }
    void* p = pool_get(c, bytes, s);
    if (!p) failed = true;
    else blocks.push_back(p);
    return static_cast<T*>(p);
  }
  ~Scratch() {
    for (void* p : blocks) pool_put(c, p, s);
  }
};

// Bytes one Scratch::get(count) of T takes from the pool (pool blocks are
// whole multiples of 256 bytes), for the footprint functions below.
template <typename T>
constexpr size_t scratch_block(size_t count) {
  return (count * sizeof(T) + 16 + 255) & ~(size_t)255;
}

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ uint64_t lanemask_lt() {
  const unsigned lane = __lane_id();
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ void flag(uint32_t* status, uint32_t bits) {
  atomicOr(status, bits);
}

// 32-bit integer mixer (lowbias32 of C. Wellons); used to place splitters
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ int msb32(uint32_t x) { return 31 - __clz((int)x); }
__device__ __forceinline__ int ctz32(uint32_t x) { return __ffs((int)x) - 1; }
__device__ __forceinline__ int ctz64(uint64_t x) { return __ffsll((unsigned long long)x) - 1; }

// (used by the one-launch small-instance kernels)
// Exclusive scan in place by a workgroup of kFT lanes of the m values
// a[at(0)], a[at(1)], ..., a[at(m - 1)] (at maps scan order to storage);
// wsum: kFT / 64 + 1 slots.
template <int kFT, typename At>
__device__ inline void wg_scan_excl_at(uint32_t* a, int m, int32_t* wsum, At at) {
  constexpr int kFW = kFT / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int per = (m + kFT - 1) / kFT;
  const int lo = min(tid * per, m), hi = min(lo + per, m);
  uint32_t sum = 0;
  for (int i = lo; i < hi; ++i) sum += a[at(i)];
  uint32_t incl = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t v = __shfl_up(incl, d);
    if (lane >= d) incl += v;
  }
  if (lane == 63) wsum[w] = (int32_t)incl;
  __syncthreads();
  if (tid < 64) {
    const uint32_t v = tid < kFW ? (uint32_t)wsum[tid] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kFW; d <<= 1) {
      const uint32_t y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (tid < kFW) wsum[tid] = (int32_t)(x - v);
  }
  __syncthreads();
  uint32_t run = (uint32_t)wsum[w] + incl - sum;
  for (int i = lo; i < hi; ++i) {
    const uint32_t x = a[at(i)];
    a[at(i)] = run;
    run += x;
  }
  __syncthreads();
}

// Exclusive scan of a[0..m) in place by a workgroup of kFT lanes.
template <int kFT>
__device__ inline void wg_scan_excl(uint32_t* a, int m, int32_t* wsum) {
  wg_scan_excl_at<kFT>(a, m, wsum, [](int i) { return i; });
}

// In-block range-minimum masks: one bit per position of a block of 2^LOG
// positions (LOG 5: 32-bit words, LOG 6: 64-bit words, one wavefront).
template <int LOG>
struct RmqMask;
template <>
struct RmqMask<5> {
  using type = uint32_t;
  static __device__ __forceinline__ int ctz(uint32_t x) { return ctz32(x); }
};
template <>
struct RmqMask<6> {
  using type = uint64_t;
  static __device__ __forceinline__ int ctz(uint64_t x) { return ctz64(x); }
};

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }
inline int floor_log2(long long x) {  // -1 for x < 1
  int r = -1;
  while (x > 0) {
    x >>= 1;
    ++r;
  }
  return r;
}

// queries per dispatch: a dispatch holds fewer than 2^32 work-items
constexpr int64_t kQueryChunk = (int64_t)1 << 31;

// Schieber-Vishkin inlabel (Section 3.1): the member of [pre+1, pre+size]
// with the most trailing zeros, in closed form (j >> k) << k with j =
// pre + size and k the highest bit in which pre and j differ.
__device__ __forceinline__ uint32_t inlabel_of(int32_t pre, int32_t size) {
  const uint32_t j = (uint32_t)pre + (uint32_t)size;          // pre+1 .. pre+size, 1-based
  const int k = msb32((uint32_t)pre ^ j);                      // (p-1) xor j with p = pre+1
  return (j >> k) << k;
}

// ---------------------------------------------------------------- launchers
// scan.hip: inclusive scan of u32 over [0, n) with + or xor
enum class ScanOp { Add, Xor };
int scan_u32(Ctx* c, const uint32_t* in, uint32_t* out, int64_t n, ScanOp op, bool exclusive,
             hipStream_t s);

// radix.hip: stable grouping of child ids by parent id (LSD radix sort of
// (parent, child) pairs). keys_out / vals_out receive the sorted parents and
// children; scalars[0] = root id, scalars[1] = number of roots; succ[2c] of
// every non-root c is set to 2c+1 and succ[2c+1] to -2 (the successor step
// writes it), both root ids to -2.
int group_by_parent_impl(Ctx* c, const int32_t* parent, int32_t n, uint32_t* keys_out,
                         int32_t* vals_out, int32_t* succ, int32_t* scalars, hipStream_t s);

// listrank.hip
struct LRResult {
  // level-1 sublist decomposition, valid after list_rank_core
  uint64_t* packed = nullptr;  // per element: sublist id | local rank << 32 | inclusive local down << 48
  int2* off = nullptr;         // per level-1 sublist: {rank of its first element, down-count before it}
  int32_t nsub = 0;            // number of level-1 sublist slots
};
// tree_weights: element e counts as "down" iff e is even (tree half-edges).
// expected_reach: number of elements the heads must reach (device scalar or null)
// weighted 1 or 2: succ holds {successor, weight} int32 pairs and the
// weights are summed instead (sublist sums in the second channel of
// out->off); packed then holds {sublist, inclusive local sum} per element
// (1), or two words {sublist | local rank << 32, inclusive local sum} (2)
int list_rank_core(Ctx* c, Scratch& sc, const int32_t* succ, int32_t len, const int32_t* heads,
                   int32_t nheads, bool tree_weights, const int32_t* expected_reach,
                   LRResult* out, hipStream_t s, bool empty_head_ok = false, int weighted = 0);
// radix.hip: stable sort of (key, value) pairs by the low `bits` key bits
int sort_pairs_u32(Ctx* c, const uint32_t* keys, const int32_t* vals, int32_t n, int bits, uint32_t* keys_out,
                   int32_t* vals_out, hipStream_t s);
// tree.hip: head table, path labels and ascendants of a tree whose node
// records {inlabel, -, depth, pre} and compact inlabels are written;
// t->d_root[0] must hold the root id; plab needs n+1 slots of scratch
int inlabel_phase(Ctx* c, et_tree* t, const int32_t* parent, const uint32_t* inl, uint32_t* plab, hipStream_t s);
// edges.hip: tree tables from an unordered edge list (the DCEL construction)
int tree_build_edges(Ctx* c, et_tree* t, const int32_t* eu, const int32_t* ev, int32_t root, int32_t* parent_out,
                     hipStream_t s);
// bridges.hip / ck.hip: bridge finding. kAlgoTV = Tarjan-Vishkin (low /
// high), kAlgoCK = Chaitanya-Kothapalli marking on a BFS forest, kAlgoHybrid
// = marking on the connectivity forest rooted by the Euler tour.
enum { kAlgoTV = 0, kAlgoCK = 1, kAlgoHybrid = 2 };
int bridges_run(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, uint32_t* mask,
                hipStream_t s, int algo);
int spanning_forest(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, int32_t* cc,
                    uint32_t* tbits, int32_t* big, hipStream_t s);
int ck_bfs_forest(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, const int32_t* cc,
                  int32_t* par, int32_t* lvl, int32_t* pslot, int32_t* uslot, uint32_t* tbits, hipStream_t s);
int ck_mark(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, const uint32_t* tbits,
            const int32_t* par, const int32_t* lvl, const int32_t* pslot, const int32_t* uslot, uint32_t* mask,
            hipStream_t s);
int bridges_ck_bfs(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, uint32_t* mask,
                   hipStream_t s);
// bridges_batch.hip: a batch of graphs as one disjoint union
int bridges_batch_run(Ctx* c, const int32_t* rows, const int32_t* col, const int64_t* voff, const int64_t* soff,
                      int32_t T, int32_t V, int32_t nnz, uint32_t* mask, int64_t mask_words, int64_t* counts,
                      hipStream_t s);
// rmq.hip: LCA by range minima over the Euler tour
int tree_rmq_build(Ctx* c, et_tree* t, const int32_t* parent, hipStream_t s);
int tree_lca_rmq(Ctx* c, const et_tree* t, const int32_t* qx, const int32_t* qy, int64_t q, int32_t* out,
                 hipStream_t s);
// naive.hip: node levels by pointer jumping and climbing LCA queries
int levels_run(Ctx* c, const int32_t* parent, int32_t n, int32_t* level, hipStream_t s);
int lca_naive_run(Ctx* c, const int32_t* parent, const int32_t* level, int32_t n, const int32_t* qx,
                  const int32_t* qy, int64_t q, int32_t* out, hipStream_t s);
int list_rank_generic(Ctx* c, const int32_t* succ, int32_t len, const int32_t* heads,
                      int32_t nheads, int32_t* rank, hipStream_t s);
// Footprints: an upper bound on the scratch each call takes from a context's
// pool, from the same sizes its allocations use: the sum of all of them, so
// a pool with nothing cached grows by at most this much. (A pool that
// already caches blocks grows by less, but may hand out a block up to twice
// the size asked for.)
size_t scan_scratch_bytes(int64_t n);
size_t group_by_parent_scratch_bytes(int32_t n);
size_t list_rank_plan_bytes(const Ctx* c, int32_t len, int32_t nheads, int weighted);
size_t tree_build_scratch_bytes(const Ctx* c, int32_t n, int32_t batch);
size_t bridges_scratch_bytes(const Ctx* c, int32_t n, int32_t nnz);
size_t bridges_batch_scratch_bytes(const Ctx* c, int32_t n_graphs, int32_t n_total, int32_t nnz_total);
// the device bytes a built tree's own tables take (et_tree_build / _batch)
size_t tree_table_bytes(int32_t n, int32_t batch);
// the same ranking with its scratch carved from a caller-provided device
// region (nothing allocated); list_rank_scratch_bytes gives the bytes it needs
size_t list_rank_scratch_bytes(Ctx* c, int32_t len, int32_t nheads);
int list_rank_arena(Ctx* c, void* arena, size_t bytes, const int32_t* succ, int32_t len, const int32_t* heads,
                    int32_t nheads, int32_t* rank, hipStream_t s);
int list_scan_generic(Ctx* c, const int32_t* succ, const int32_t* weights, int32_t len, const int32_t* heads,
                      int32_t nheads, int32_t* rank, int32_t* sum, hipStream_t s);
// Grid of a persistent kernel (one launch, workgroups taking work items
// from a counter): as many workgroups as stay resident on the current device
// with `lds` bytes of dynamic LDS each, at most `items`. Device limits, the
// kernel's LDS attribute and its occupancy are looked up once and cached.
// ET_ESIZE if one workgroup cannot take `lds` bytes.
int persistent_grid(const void* kern, int threads, uint32_t lds, int64_t items, int* grid);
// small_bridges.hip: bridges of many graphs of at most 1024 vertices and 8192
// CSR slots in one launch; moff[t] is graph t's first mask word
int small_bridges_run(Ctx* c, const int32_t* row_ptr, const int32_t* col, const int64_t* voff, const int64_t* soff,
                      const int64_t* moff, int32_t T, int32_t n_total, int32_t nnz_total, int32_t max_vertices,
                      int32_t max_slots, uint32_t* mask, int64_t mask_words, int64_t* counts, const int32_t* order,
                      hipStream_t s);
// small.hip: build and query many trees of at most 4096 nodes in one launch
size_t small_batch_lds_bytes(int32_t max_nodes);
int small_batch_run(Ctx* c, const int32_t* parent, const int64_t* off, int32_t T, int64_t n_total,
                    int32_t max_nodes, const int64_t* qoff, const int32_t* qx, const int32_t* qy, int64_t q_total,
                    int32_t* out, int32_t* depth, int32_t* pre, int32_t* size, const int32_t* order,
                    hipStream_t s);

}  // namespace et

// the public opaque types
struct et_ctx {
  et::Ctx impl;
};

struct et_tree {
  et_ctx* ctx;
  int32_t n;           // nodes in the tables (a batch adds one virtual root)
  int32_t batch;       // 0 for one tree, else the number of trees of a batch
  int64_t* d_off;      // batch: node offsets of the trees [batch+1]
  int32_t* d_root_of;  // batch: root id of every tree [batch]
  int32_t* d_succ;     // [2n]
  int32_t* d_rank;     // [2n]
  int32_t* d_pre;      // [n]
  int32_t* d_size;     // [n]
  int4* d_rec;         // [n] {inlabel, asc, depth, pre}
  int2* d_head;        // [n+2] by inlabel: {parent of path top, its depth}
  int32_t* d_root;     // device scalar
  int32_t from_edges;  // built by et_tree_build_edges (half-edge ids follow the edge list)
  // optional RMQ query engine (et_tree_rmq_build)
  uint64_t* d_rmq_e;     // [2(n-1)] {depth, node} after every tour half-edge
  void* d_rmq_mask;      // [2(n-1)] in-block suffix-minimum masks (32- or 64-bit words)
  uint64_t* d_rmq_st;    // sparse table over the block minima, level-major
  int32_t rmq_nb;        // number of blocks
  int32_t rmq_log;       // blocks of 2^rmq_log positions
};
