// C-ABI entry points of the Euler-tour library (declared in include/et.h),
// the per-context scratch pool and the device status word.
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <utility>

#include "et_internal.hpp"

namespace et {

int tree_build(Ctx* c, et_tree* t, const int32_t* parent, hipStream_t s);
int tree_export(const et_tree* t, int32_t* succ, int32_t* rank, int32_t* depth, int32_t* pre, int32_t* size,
                uint32_t* inl, uint32_t* asc, hipStream_t s);
int tree_export_tour(Ctx* c, const et_tree* t, int32_t* tour, hipStream_t s);
int tree_lca(Ctx* c, const et_tree* t, const int32_t* qx, const int32_t* qy, int64_t q, int32_t* out,
             hipStream_t s);
int tree_build_batch(Ctx* c, et_tree* t, const int32_t* parent, hipStream_t s);
int tree_lca_batch(Ctx* c, const et_tree* t, const int32_t* qt, const int32_t* qx, const int32_t* qy, int64_t q,
                   int32_t* out, hipStream_t s);

namespace {
constexpr size_t kAlign = 256;
}

void* pool_get(Ctx* c, size_t bytes, hipStream_t s) {
  bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
  // smallest cached block that fits without wasting more than half of it
  auto it = c->free_blocks.lower_bound(bytes);
  if (it != c->free_blocks.end() && it->first <= 2 * bytes + (1u << 20)) {
    void* p = it->second.p;
    const hipStream_t from = it->second.s;
    if (from != s) {
      hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(s, &cap) != hipSuccess) {
        (void)hipGetLastError();
        cap = hipStreamCaptureStatusNone;
      }
      if (cap == hipStreamCaptureStatusNone) {
        // every use of the block was enqueued on `from` before it came back
        hipEvent_t e = sync_event(c);
        if (!e || hipEventRecord(e, from) != hipSuccess || hipStreamWaitEvent(s, e, 0) != hipSuccess) {
          (void)hipGetLastError();
          if (hipStreamSynchronize(from) != hipSuccess) return nullptr;
        }
        if (e) c->spare_sync.push_back(e);
      }
    }
    c->live_blocks[p] = it->first;
    c->pool_live += it->first;
    c->pool_peak_live = std::max(c->pool_peak_live, c->pool_live);
    c->free_blocks.erase(it);
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    // release cached blocks and retry once (hipFree waits for the device)
    for (auto& kv : c->free_blocks) {
      (void)hipFree(kv.second.p);
      c->pool_bytes -= kv.first;
    }
    c->free_blocks.clear();
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  c->pool_bytes += bytes;
  c->live_blocks[p] = bytes;
  c->pool_live += bytes;
  c->pool_peak_live = std::max(c->pool_peak_live, c->pool_live);
  return p;
}

hipEvent_t sync_event(Ctx* c) {
  if (!c->spare_sync.empty()) {
    hipEvent_t e = c->spare_sync.back();
    c->spare_sync.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

hipEvent_t prof_event(Ctx* c) {
  if (!c->spare_events.empty()) {
    hipEvent_t e = c->spare_events.back();
    c->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void pool_put(Ctx* c, void* p, hipStream_t s) {
  auto it = c->live_blocks.find(p);
  if (it == c->live_blocks.end()) return;
  c->free_blocks.emplace(it->second, Ctx::FreeBlock{p, s});
  c->pool_live -= it->second;
  c->live_blocks.erase(it);
}

// The tables of a tree with n node slots (a batch: its nodes + the virtual
// root), in allocation order: succ, rank, pre, size, node records, head
// table, the root scalar, and for a batch the offsets and per-tree roots.
int tree_table_sizes(int32_t n, int32_t batch, size_t sz[9]) {
  const size_t N = (size_t)n;
  sz[0] = 2 * N * sizeof(int32_t);
  sz[1] = 2 * N * sizeof(int32_t);
  sz[2] = N * sizeof(int32_t);
  sz[3] = N * sizeof(int32_t);
  sz[4] = N * sizeof(int4);
  sz[5] = (N + 2) * sizeof(int2);
  sz[6] = 64;
  if (!batch) return 7;
  sz[7] = ((size_t)batch + 1) * sizeof(int64_t);
  sz[8] = (size_t)batch * sizeof(int32_t);
  return 9;
}

size_t tree_table_bytes(int32_t n, int32_t batch) {
  size_t sz[9], b = 0;
  const int k = tree_table_sizes(n, batch, sz);
  for (int i = 0; i < k; ++i) b += (sz[i] + kAlign - 1) & ~(kAlign - 1);  // pool blocks are multiples of 256 B
  return b;
}

}  // namespace et

using et::Ctx;

// Fixed scratch of et_list_rank_noalloc. Each GPU that loads the library's
// code holds its own copy of this array (until the process ends), at its own
// address. On the host the name is only a stand-in for the symbol, never a
// device address: kernels and copies get the address resolved per device by
// hipGetSymbolAddress below.
static __device__ __align__(256) char scratch[ET_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void* g_fixed[kMaxDevices] = {};

// Device address of `scratch` on device dev (which must be current),
// resolved once per device. nullptr if it cannot be resolved.
void* fixed_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_fixed_mu);
  if (!g_fixed[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_fixed[dev] = p;
  }
  return g_fixed[dev];
}
}  // namespace

namespace et {

int persistent_grid(const void* kern, int threads, uint32_t lds, int64_t items, int* grid) {
  struct DevInfo {
    int max_lds = 0, cus = 0;
  };
  static std::mutex mu;
  static std::map<int, DevInfo> devs;
  static std::map<std::pair<int, const void*>, bool> attr_set;
  static std::map<std::tuple<int, const void*, int, uint32_t>, int> occ;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ET_EHIP;
  std::lock_guard<std::mutex> lock(mu);
  auto d = devs.find(dev);
  if (d == devs.end()) {
    DevInfo info;
    if (hipDeviceGetAttribute(&info.max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&info.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return ET_EHIP;
    d = devs.emplace(dev, info).first;
  }
  if ((int)lds > d->second.max_lds) return ET_ESIZE;
  if (!attr_set[{dev, kern}]) {
    // allow every dynamic LDS size this device offers, once per kernel
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, d->second.max_lds) != hipSuccess)
      return ET_EHIP;
    attr_set[{dev, kern}] = true;
  }
  const auto key = std::make_tuple(dev, kern, threads, lds);
  auto o = occ.find(key);
  if (o == occ.end()) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess) return ET_EHIP;
    o = occ.emplace(key, std::max(per_cu, 1)).first;
  }
  *grid = (int)std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)o->second * d->second.cus));
  return ET_OK;
}

}  // namespace et

extern "C" {

int et_version(void) { return 100; }

const char* et_strerror(int code) {
  switch (code) {
    case ET_OK: return "ok";
    case ET_EINVAL: return "invalid argument";
    case ET_ENOMEM: return "out of device memory";
    case ET_EHIP: return "HIP runtime error";
    case ET_EINPUT: return "malformed input detected on the device";
    case ET_ESIZE: return "input beyond a fixed-size limit of this call";
    default: return "unknown error";
  }
}

int et_ctx_create(et_ctx** out) {
  if (!out) return ET_EINVAL;
  *out = nullptr;
  et_ctx* ctx = new (std::nothrow) et_ctx();
  if (!ctx) return ET_ENOMEM;
  Ctx* c = &ctx->impl;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete ctx;
    return ET_EHIP;
  }
  void* p = nullptr;
  if (hipMalloc(&p, 256) != hipSuccess) {
    delete ctx;
    return ET_ENOMEM;
  }
  if (hipMemset(p, 0, 256) != hipSuccess) {
    (void)hipFree(p);
    delete ctx;
    return ET_EHIP;
  }
  c->d_status = static_cast<uint32_t*>(p);
  c->d_scalars = reinterpret_cast<int32_t*>(static_cast<char*>(p) + 64);
  c->d_bcount = reinterpret_cast<int64_t*>(static_cast<char*>(p) + 128);
  c->d_fused = reinterpret_cast<uint32_t*>(static_cast<char*>(p) + 192);  // zero; kept zero between launches
  // the fixed scratch of et_list_rank_noalloc on this device (resolved here,
  // so that the non-allocating call itself makes no runtime set-up call)
  c->d_fixed = fixed_scratch(c->device);
  *out = ctx;
  return ET_OK;
}

void et_ctx_destroy(et_ctx* ctx) {
  if (!ctx) return;
  Ctx* c = &ctx->impl;
  (void)hipDeviceSynchronize();
  for (auto& kv : c->free_blocks) (void)hipFree(kv.second.p);
  for (auto& kv : c->live_blocks) (void)hipFree(kv.first);
  for (auto e : c->spare_sync) (void)hipEventDestroy(e);
  (void)hipFree(c->d_status);
  for (auto& r : c->prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->spare_events) (void)hipEventDestroy(e);
  delete ctx;
}

int et_ctx_set_param(et_ctx* ctx, const char* name, int64_t value) {
  if (!ctx || !name) return ET_EINVAL;
  et::LrShape& lr = ctx->impl.lr;
  const std::string k(name);
  if (k == "lr_k1_log2" && value >= 1 && value <= 10) lr.k1_log2 = (int)value;
  else if (k == "lr_per_wave1" && value >= 64 && value <= 65536) lr.per_wave1 = (int)value;
  else if (k == "lr_kn_log2" && value >= 1 && value <= 10) lr.kn_log2 = (int)value;
  else if (k == "lr_per_waven" && value >= 64 && value <= 65536) lr.per_waven = (int)value;
  else if (k == "rmq_block_log2" && (value == 5 || value == 6)) ctx->impl.qs.rmq_log = (int)value;
  else if (k == "query_block" && value >= 64 && value <= et::kQueryBlockMax && (value & (value - 1)) == 0)
    ctx->impl.qs.block = (int)value;
  else return ET_EINVAL;
  return ET_OK;
}

int et_ctx_profile(et_ctx* ctx, int enable) {
  if (!ctx) return ET_EINVAL;
  ctx->impl.profiling = enable != 0;
  return ET_OK;
}

int et_ctx_profile_only(et_ctx* ctx, const char* kernel_name) {
  if (!ctx) return ET_EINVAL;
  ctx->impl.prof_only = kernel_name ? kernel_name : "";
  return ET_OK;
}

int et_ctx_profile_read(et_ctx* ctx, hipStream_t s, char* h_buf, int32_t buflen) {
  if (!ctx || !h_buf || buflen < 3) return ET_EINVAL;
  Ctx* c = &ctx->impl;
  if (hipStreamSynchronize(s) != hipSuccess) return ET_EHIP;
  struct Agg {
    long n = 0;
    double total = 0, mx = 0;
  };
  std::map<std::string, Agg> agg;
  for (auto& r : c->prof) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    Agg& g = agg[r.name];
    g.n++;
    g.total += ms;
    if (ms > g.mx) g.mx = ms;
  }
  std::string out = "{";
  char tmp[256];
  for (auto& kv : agg) {
    snprintf(tmp, sizeof(tmp), "%s\"%s\": [%ld, %.6f, %.6f]", out.size() > 1 ? ", " : "", kv.first.c_str(),
             kv.second.n, kv.second.total, kv.second.mx);
    out += tmp;
  }
  out += "}";
  if ((int64_t)out.size() + 1 > buflen) return ET_EINVAL;
  std::memcpy(h_buf, out.c_str(), out.size() + 1);
  for (auto& r : c->prof) {
    c->spare_events.push_back(r.a);
    c->spare_events.push_back(r.b);
  }
  c->prof.clear();
  return ET_OK;
}

// clears the status word with a kernel rather than a memset node, so the
// stream's work stays free of memset operations
__global__ void k_clear_status(uint32_t* status) { *status = 0u; }

int et_ctx_status_bits(et_ctx* ctx, hipStream_t s, uint32_t* h_bits) {
  if (!ctx || !h_bits) return ET_EINVAL;
  Ctx* c = &ctx->impl;
  uint32_t bits = 0;
  if (hipMemcpyAsync(&bits, c->d_status, sizeof(bits), hipMemcpyDeviceToHost, s) != hipSuccess) return ET_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return ET_EHIP;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, c->d_status);
  if (hipGetLastError() != hipSuccess) return ET_EHIP;
  *h_bits = bits;
  return ET_OK;
}

int et_ctx_status(et_ctx* ctx, hipStream_t s) {
  uint32_t bits = 0;
  int rc = et_ctx_status_bits(ctx, s, &bits);
  if (rc) return rc;
  return bits ? ET_EINPUT : ET_OK;
}

int et_list_rank(et_ctx* ctx, const int32_t* d_succ, int32_t len, const int32_t* d_heads, int32_t n_heads,
                 int32_t* d_rank, hipStream_t s) {
  if (!ctx || len < 0 || n_heads < 0 || len > 0x7fffffff - (1 << 20)) return ET_EINVAL;
  if (len > 0 && (!d_succ || !d_rank)) return ET_EINVAL;
  if (n_heads > 0 && !d_heads) return ET_EINVAL;
  if (len > 0 && n_heads == 0) return ET_EINVAL;
  return et::list_rank_generic(&ctx->impl, d_succ, len, d_heads, n_heads, d_rank, s);
}

int et_list_rank_noalloc(et_ctx* ctx, const int32_t* d_succ, int32_t len, const int32_t* d_heads,
                         int32_t n_heads, int32_t* d_rank, hipStream_t s) {
  if (!ctx || len < 0 || n_heads < 0) return ET_EINVAL;
  if (len > 0 && (!d_succ || !d_rank)) return ET_EINVAL;
  if (n_heads > 0 && !d_heads) return ET_EINVAL;
  if (len > 0 && n_heads == 0) return ET_EINVAL;
  if (len > ET_NOALLOC_MAX_LEN || n_heads > ET_NOALLOC_MAX_HEADS) return ET_ESIZE;
  Ctx* c = &ctx->impl;
  if (!c->d_fixed) return ET_EHIP;
  if (et::list_rank_scratch_bytes(c, len, n_heads) > ET_NOALLOC_SCRATCH_BYTES) return ET_ESIZE;
  return et::list_rank_arena(c, c->d_fixed, ET_NOALLOC_SCRATCH_BYTES, d_succ, len, d_heads, n_heads, d_rank, s);
}

int et_list_scan(et_ctx* ctx, const int32_t* d_succ, const int32_t* d_weight, int32_t len, const int32_t* d_heads,
                 int32_t n_heads, int32_t* d_rank, int32_t* d_sum, hipStream_t s) {
  if (!ctx || len < 0 || n_heads < 0 || len > 0x7fffffff - (1 << 20)) return ET_EINVAL;
  if (len > 0 && (!d_succ || !d_weight || !d_sum)) return ET_EINVAL;
  if (n_heads > 0 && !d_heads) return ET_EINVAL;
  if (len > 0 && n_heads == 0) return ET_EINVAL;
  return et::list_scan_generic(&ctx->impl, d_succ, d_weight, len, d_heads, n_heads, d_rank, d_sum, s);
}

static et_tree* tree_alloc(et_ctx* ctx, int32_t n, int32_t batch, hipStream_t s) {
  Ctx* c = &ctx->impl;
  et_tree* t = new (std::nothrow) et_tree();
  if (!t) return nullptr;
  t->ctx = ctx;
  t->n = n;
  t->batch = batch;
  size_t sz[9];
  const int k = et::tree_table_sizes(n, batch, sz);
  void* p[9] = {};
  bool ok = true;
  for (int i = 0; i < k; ++i) ok = ((p[i] = et::pool_get(c, sz[i], s)) != nullptr) && ok;
  t->d_succ = static_cast<int32_t*>(p[0]);
  t->d_rank = static_cast<int32_t*>(p[1]);
  t->d_pre = static_cast<int32_t*>(p[2]);
  t->d_size = static_cast<int32_t*>(p[3]);
  t->d_rec = static_cast<int4*>(p[4]);
  t->d_head = static_cast<int2*>(p[5]);
  t->d_root = static_cast<int32_t*>(p[6]);
  if (batch) {
    t->d_off = static_cast<int64_t*>(p[7]);
    t->d_root_of = static_cast<int32_t*>(p[8]);
  }
  if (!ok) {
    et_tree_free(t, s);
    return nullptr;
  }
  return t;
}

int et_tree_footprint(const et_ctx* ctx, int64_t n_total, int32_t n_trees, int64_t* h_table_bytes,
                      int64_t* h_scratch_bytes) {
  if (n_trees < 0 || n_total < 1 || (n_trees == 0 && n_total >= (1 << 30)) ||
      (n_trees > 0 && (n_total < n_trees || n_total + 1 >= (1 << 30))))
    return ET_EINVAL;
  const int32_t n = (int32_t)(n_trees ? n_total + 1 : n_total);  // a batch adds its virtual root
  const Ctx* c = ctx ? &ctx->impl : nullptr;
  if (h_table_bytes) *h_table_bytes = (int64_t)et::tree_table_bytes(n, n_trees);
  if (h_scratch_bytes) *h_scratch_bytes = (int64_t)et::tree_build_scratch_bytes(c, n, n_trees);
  return ET_OK;
}

int et_bridges_footprint(const et_ctx* ctx, int32_t n_total, int32_t nnz_total, int32_t n_graphs,
                         int64_t* h_scratch_bytes) {
  if (n_graphs < 0 || n_total < 0 || n_total >= (1 << 30) || nnz_total < 0 || !h_scratch_bytes) return ET_EINVAL;
  const Ctx* c = ctx ? &ctx->impl : nullptr;
  *h_scratch_bytes = (int64_t)(n_graphs ? et::bridges_batch_scratch_bytes(c, n_graphs, n_total, nnz_total)
                                        : et::bridges_scratch_bytes(c, n_total, nnz_total));
  return ET_OK;
}

int et_tree_bytes(const et_tree* tree, int64_t* h_bytes) {
  if (!tree || !h_bytes) return ET_EINVAL;
  const Ctx* c = &tree->ctx->impl;
  const void* blocks[] = {tree->d_succ, tree->d_rank, tree->d_pre,   tree->d_size,  tree->d_rec,     tree->d_head,
                          tree->d_root, tree->d_off,  tree->d_root_of, tree->d_rmq_e, tree->d_rmq_mask, tree->d_rmq_st};
  int64_t b = 0;
  for (const void* p : blocks) {
    if (!p) continue;
    auto it = c->live_blocks.find(const_cast<void*>(p));
    if (it != c->live_blocks.end()) b += (int64_t)it->second;
  }
  *h_bytes = b;
  return ET_OK;
}

int et_ctx_pool_stats(et_ctx* ctx, int64_t* h_held, int64_t* h_live, int64_t* h_peak_live, int reset_peak) {
  if (!ctx) return ET_EINVAL;
  Ctx* c = &ctx->impl;
  if (h_held) *h_held = (int64_t)c->pool_bytes;
  if (h_live) *h_live = (int64_t)c->pool_live;
  if (h_peak_live) *h_peak_live = (int64_t)c->pool_peak_live;
  if (reset_peak) c->pool_peak_live = c->pool_live;
  return ET_OK;
}

int et_tree_build(et_ctx* ctx, const int32_t* d_parent, int32_t n, hipStream_t s, et_tree** out) {
  if (!out) return ET_EINVAL;
  *out = nullptr;
  if (!ctx || !d_parent || n < 1 || n >= (1 << 30)) return ET_EINVAL;
  et_tree* t = tree_alloc(ctx, n, 0, s);
  if (!t) return ET_ENOMEM;
  int rc = et::tree_build(&ctx->impl, t, d_parent, s);
  if (rc) {
    et_tree_free(t, s);
    return rc;
  }
  *out = t;
  return ET_OK;
}

int et_tree_build_edges(et_ctx* ctx, const int32_t* d_u, const int32_t* d_v, int32_t n, int32_t root,
                        int32_t* d_parent_out, hipStream_t s, et_tree** out) {
  if (!out) return ET_EINVAL;
  *out = nullptr;
  if (!ctx || n < 1 || n >= (1 << 30) || root < 0 || root >= n) return ET_EINVAL;
  if (n > 1 && (!d_u || !d_v)) return ET_EINVAL;
  et_tree* t = tree_alloc(ctx, n, 0, s);
  if (!t) return ET_ENOMEM;
  t->from_edges = 1;
  int rc = et::tree_build_edges(&ctx->impl, t, d_u, d_v, root, d_parent_out, s);
  if (rc) {
    et_tree_free(t, s);
    return rc;
  }
  *out = t;
  return ET_OK;
}

int et_tree_rmq_build(et_tree* tree, const int32_t* d_parent, hipStream_t s) {
  if (!tree || tree->batch || tree->from_edges || (tree->n > 1 && !d_parent)) return ET_EINVAL;
  Ctx* c = &tree->ctx->impl;
  for (void** p : {reinterpret_cast<void**>(&tree->d_rmq_e), reinterpret_cast<void**>(&tree->d_rmq_mask),
                   reinterpret_cast<void**>(&tree->d_rmq_st)})
    if (*p) {
      et::pool_put(c, *p, s);
      *p = nullptr;
    }
  return et::tree_rmq_build(c, tree, d_parent, s);
}

int et_lca_rmq(const et_tree* tree, const int32_t* d_qx, const int32_t* d_qy, int64_t q, int32_t* d_out,
               hipStream_t s) {
  if (!tree || tree->batch || q < 0 || q > (int64_t)0x7fffffff * 64) return ET_EINVAL;
  if (tree->n > 1 && !tree->d_rmq_e) return ET_EINVAL;  // et_tree_rmq_build first
  if (q > 0 && (!d_qx || !d_qy || !d_out)) return ET_EINVAL;
  return et::tree_lca_rmq(&tree->ctx->impl, tree, d_qx, d_qy, q, d_out, s);
}

int et_tree_build_batch(et_ctx* ctx, const int32_t* d_parent, const int64_t* d_offsets, int32_t n_trees,
                        int64_t n_total, hipStream_t s, et_tree** out) {
  if (!out) return ET_EINVAL;
  *out = nullptr;
  if (!ctx || !d_parent || !d_offsets || n_trees < 1 || n_total < n_trees || n_total + 1 >= (1 << 30))
    return ET_EINVAL;
  et_tree* t = tree_alloc(ctx, (int32_t)(n_total + 1), n_trees, s);
  if (!t) return ET_ENOMEM;
  if (hipMemcpyAsync(t->d_off, d_offsets, ((size_t)n_trees + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s) !=
      hipSuccess) {
    et_tree_free(t, s);
    return ET_EHIP;
  }
  int rc = et::tree_build_batch(&ctx->impl, t, d_parent, s);
  if (rc) {
    et_tree_free(t, s);
    return rc;
  }
  *out = t;
  return ET_OK;
}

int et_lca_batch(const et_tree* tree, const int32_t* d_qtree, const int32_t* d_qx, const int32_t* d_qy, int64_t q,
                 int32_t* d_out, hipStream_t s) {
  if (!tree || !tree->batch || q < 0 || q > (int64_t)0x7fffffff * 64) return ET_EINVAL;
  if (q > 0 && (!d_qtree || !d_qx || !d_qy || !d_out)) return ET_EINVAL;
  return et::tree_lca_batch(&tree->ctx->impl, tree, d_qtree, d_qx, d_qy, q, d_out, s);
}

int et_lca_batch_fused(et_ctx* ctx, const int32_t* d_parent, const int64_t* d_offsets, int32_t n_trees,
                       int64_t n_total, int32_t max_tree_nodes, const int64_t* d_qoffsets, const int32_t* d_qx,
                       const int32_t* d_qy, int64_t q_total, int32_t* d_out, int32_t* d_depth, int32_t* d_pre,
                       int32_t* d_size, const int32_t* d_order, hipStream_t s) {
  if (!ctx || n_trees < 0 || n_total < n_trees || q_total < 0) return ET_EINVAL;
  if (n_trees == 0) return n_total == 0 && q_total == 0 ? ET_OK : ET_EINVAL;
  if (!d_parent || !d_offsets || !d_qoffsets || max_tree_nodes < 1) return ET_EINVAL;
  if (q_total > 0 && (!d_qx || !d_qy || !d_out)) return ET_EINVAL;
  if (n_total > (int64_t)n_trees * max_tree_nodes) return ET_EINVAL;  // some tree would exceed the bound
  if (max_tree_nodes > ET_FUSED_MAX_NODES) return ET_ESIZE;
  return et::small_batch_run(&ctx->impl, d_parent, d_offsets, n_trees, n_total, max_tree_nodes, d_qoffsets, d_qx,
                             d_qy, q_total, d_out, d_depth, d_pre, d_size, d_order, s);
}

int et_bridges_batch_fused(et_ctx* ctx, const int32_t* d_row_ptr, const int32_t* d_col, const int64_t* d_voff,
                           const int64_t* d_soff, const int64_t* d_moff, int32_t n_graphs, int32_t n_total,
                           int32_t nnz_total, int32_t max_graph_vertices, int32_t max_graph_slots,
                           uint32_t* d_mask, int64_t mask_words, int64_t* d_counts, const int32_t* d_order,
                           hipStream_t s) {
  if (!ctx || n_graphs < 0 || n_total < 0 || nnz_total < 0 || mask_words < 0) return ET_EINVAL;
  if (max_graph_vertices < 0 || max_graph_slots < 0) return ET_EINVAL;
  if (n_graphs == 0) return n_total == 0 && nnz_total == 0 ? ET_OK : ET_EINVAL;
  if (!d_row_ptr || !d_voff || !d_soff || !d_moff || (nnz_total > 0 && (!d_col || !d_mask))) return ET_EINVAL;
  if ((int64_t)n_total > (int64_t)n_graphs * max_graph_vertices ||
      (int64_t)nnz_total > (int64_t)n_graphs * max_graph_slots)
    return ET_EINVAL;  // some graph would exceed the bounds
  if (max_graph_vertices > ET_FUSED_MAX_VERTICES || max_graph_slots > ET_FUSED_MAX_SLOTS) return ET_ESIZE;
  return et::small_bridges_run(&ctx->impl, d_row_ptr, d_col, d_voff, d_soff, d_moff, n_graphs, n_total, nnz_total,
                               max_graph_vertices, max_graph_slots, d_mask, mask_words, d_counts, d_order, s);
}

int32_t et_tree_batch_size(const et_tree* tree) { return tree ? tree->batch : -1; }

int et_tree_export_tour(const et_tree* tree, int32_t* d_tour, hipStream_t s) {
  if (!tree || (tree->n > 1 && !d_tour)) return ET_EINVAL;
  return et::tree_export_tour(&tree->ctx->impl, tree, d_tour, s);
}

int32_t et_tree_size(const et_tree* tree) {
  if (!tree) return -1;
  return tree->batch ? tree->n - 1 : tree->n;
}

int et_tree_export(const et_tree* tree, int32_t* d_succ, int32_t* d_rank, int32_t* d_depth, int32_t* d_pre,
                   int32_t* d_size, uint32_t* d_inlabel, uint32_t* d_asc, hipStream_t s) {
  if (!tree) return ET_EINVAL;
  return et::tree_export(tree, d_succ, d_rank, d_depth, d_pre, d_size, d_inlabel, d_asc, s);
}

void et_tree_free(et_tree* tree, hipStream_t s) {
  if (!tree) return;
  Ctx* c = &tree->ctx->impl;
  void* blocks[] = {tree->d_succ, tree->d_rank, tree->d_pre,   tree->d_size,    tree->d_rec,     tree->d_head,
                    tree->d_root, tree->d_off,  tree->d_root_of, tree->d_rmq_e, tree->d_rmq_mask, tree->d_rmq_st};
  for (void* p : blocks)
    if (p) et::pool_put(c, p, s);
  delete tree;
}

int et_lca(const et_tree* tree, const int32_t* d_qx, const int32_t* d_qy, int64_t q, int32_t* d_out,
           hipStream_t s) {
  if (!tree || tree->batch || q < 0 || q > (int64_t)0x7fffffff * 64) return ET_EINVAL;
  if (q > 0 && (!d_qx || !d_qy || !d_out)) return ET_EINVAL;
  return et::tree_lca(&tree->ctx->impl, tree, d_qx, d_qy, q, d_out, s);
}

int et_bridges(et_ctx* ctx, const int32_t* d_row_ptr, const int32_t* d_col, int32_t n, int32_t nnz,
               uint32_t* d_mask, int64_t* h_count, hipStream_t s) {
  if (!ctx || n < 0 || n >= (1 << 30) || nnz < 0 || !d_row_ptr) return ET_EINVAL;  // 2(n-1) forest half-edges fit int32
  if (nnz > 0 && (!d_col || !d_mask)) return ET_EINVAL;
  Ctx* c = &ctx->impl;
  int rc = et::bridges_run(c, d_row_ptr, d_col, n, nnz, d_mask, s, et::kAlgoTV);
  if (rc) return rc;
  if (h_count) {
    if (hipMemcpyAsync(h_count, c->d_bcount, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
      return ET_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return ET_EHIP;
  }
  return ET_OK;
}

int et_bridges_batch(et_ctx* ctx, const int32_t* d_row_ptr, const int32_t* d_col, const int64_t* d_voff,
                     const int64_t* d_soff, int32_t n_graphs, int32_t n_total, int32_t nnz_total, uint32_t* d_mask,
                     int64_t mask_words, int64_t* d_counts, hipStream_t s) {
  if (!ctx || n_graphs < 1 || n_total < 0 || n_total >= (1 << 30) || nnz_total < 0 || mask_words < 0) return ET_EINVAL;
  if (!d_row_ptr || !d_voff || !d_soff || (mask_words > 0 && !d_mask)) return ET_EINVAL;
  if (nnz_total > 0 && (!d_col || n_total == 0 || mask_words == 0)) return ET_EINVAL;
  return et::bridges_batch_run(&ctx->impl, d_row_ptr, d_col, d_voff, d_soff, n_graphs, n_total, nnz_total, d_mask,
                               mask_words, d_counts, s);
}

int et_levels(et_ctx* ctx, const int32_t* d_parent, int32_t n, int32_t* d_level, hipStream_t s) {
  if (!ctx || n < 1 || n >= (1 << 30) || !d_parent || !d_level) return ET_EINVAL;
  return et::levels_run(&ctx->impl, d_parent, n, d_level, s);
}

int et_lca_naive(et_ctx* ctx, const int32_t* d_parent, const int32_t* d_level, int32_t n, const int32_t* d_qx,
                 const int32_t* d_qy, int64_t q, int32_t* d_out, hipStream_t s) {
  if (!ctx || n < 1 || n >= (1 << 30) || !d_parent || !d_level || q < 0) return ET_EINVAL;
  if (q > 0 && (!d_qx || !d_qy || !d_out)) return ET_EINVAL;
  return et::lca_naive_run(&ctx->impl, d_parent, d_level, n, d_qx, d_qy, q, d_out, s);
}

int et_bridges_ck(et_ctx* ctx, const int32_t* d_row_ptr, const int32_t* d_col, int32_t n, int32_t nnz,
                  int32_t spanning, uint32_t* d_mask, int64_t* h_count, hipStream_t s) {
  if (!ctx || n < 0 || n >= (1 << 30) || nnz < 0 || !d_row_ptr || (spanning != 0 && spanning != 1)) return ET_EINVAL;
  if (nnz > 0 && (!d_col || !d_mask)) return ET_EINVAL;
  Ctx* c = &ctx->impl;
  int rc = et::bridges_run(c, d_row_ptr, d_col, n, nnz, d_mask, s, spanning == 0 ? et::kAlgoCK : et::kAlgoHybrid);
  if (rc) return rc;
  if (h_count) {
    if (hipMemcpyAsync(h_count, c->d_bcount, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
      return ET_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return ET_EHIP;
  }
  return ET_OK;
}

int et_bridges_count(et_ctx* ctx, int64_t* d_count, hipStream_t s) {
  if (!ctx || !d_count) return ET_EINVAL;
  return hipMemcpyAsync(d_count, ctx->impl.d_bcount, sizeof(int64_t), hipMemcpyDeviceToDevice, s) == hipSuccess
             ? ET_OK
             : ET_EHIP;
}

}  // extern "C"
