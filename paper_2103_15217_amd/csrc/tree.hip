// Euler tour of a rooted tree, node statistics and the Inlabel tables
// (Sections 2.1, 2.2 and 3.1), and the LCA query kernel (Section 3.1).
//
// Build, for a parent array of n nodes:
//   1. group_by_parent: children of every node, ascending (radix.hip).
//   2. k_succ: over the grouped order, succ(2c+1) = 2 * next sibling of c,
//      or 2 * parent(c) + 1 after the last sibling (-1 below the root), and
//      succ(2p) = 2 * first child of p; leaves keep succ(2c) = 2c+1. This is
//      next(twin(e)) of the paper's DCEL with the children of a node in
//      ascending order and the tour split before the root's first child.
//   3. one list ranking of the 2n half-edges, carrying the number of down
//      half-edges (Section 2: weights on the tour give preorder and level).
//   4. k_node: rank(2c) = R0, number of down half-edges up to it = D; then
//      pre(c) = D, depth(c) = 2D - R0 - 1, size(c) = (rank(2c+1) - R0 + 1)/2,
//      and inlabel(c) = the member of [pre+1, pre+size] with the most
//      trailing zeros, in closed form (j >> k) << k with j = pre + size and
//      k the highest bit in which pre and j differ.
//   5. k_head: a node is the top of its inlabel path iff it is the root or
//      its parent's inlabel differs; head[inlabel] = {parent, depth - 1},
//      and the label of the parent's path is recorded per label.
//   6. ascendant(v) (the OR of 2^h over the labels of v's ancestors) only
//      depends on v's path: it is the ascendant of the path above plus the
//      path's own level bit. Labels on a root path have strictly decreasing
//      levels, so one pass per level, from the highest down, fills a table
//      by label; k_asc copies it into the node records.
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kB = 256;

enum { SC_ROOT = 0, SC_NROOTS = 1, SC_HEAD = 2, SC_EXPECT = 3 };

__global__ void k_succ(const uint32_t* __restrict__ keys, const int32_t* __restrict__ vals, int32_t n,
                       int32_t* __restrict__ sc, int32_t* __restrict__ succ, uint32_t* __restrict__ status) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t root = sc[SC_ROOT];
  if (k == 0) {
    if (sc[SC_NROOTS] != 1) flag(status, ST_ROOTS);
    sc[SC_EXPECT] = 2 * (n - 1);
  }
  const int32_t c = vals[k];
  if (c == root) return;
  const uint32_t p = keys[k];
  if (p >= (uint32_t)n) return;  // invalid parent, already flagged
  int64_t k2 = k + 1;
  if (k2 < n && vals[k2] == root) ++k2;
  int32_t nxt;
  if (k2 < n && keys[k2] == p) nxt = 2 * vals[k2];
  else nxt = ((int32_t)p == root) ? -1 : (int32_t)(2 * p + 1);
  succ[2 * c + 1] = nxt;
  int64_t k0 = k - 1;
  if (k0 >= 0 && vals[k0] == root) --k0;
  if (k0 < 0 || keys[k0] != p) {
    if ((int32_t)p == root) sc[SC_HEAD] = 2 * c;
    else succ[2 * p] = 2 * c;
  }
}

__global__ void k_node(const uint64_t* __restrict__ packed, const int2* __restrict__ off, int32_t nsub,
                       int32_t n, const int32_t* __restrict__ sc, int32_t* __restrict__ rank,
                       int32_t* __restrict__ pre_out, int32_t* __restrict__ size_out, int4* __restrict__ rec,
                       uint32_t* __restrict__ inl_out, uint32_t* __restrict__ status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int32_t root = sc[SC_ROOT];
  int32_t depth, pre, size, r0, r1;
  if (c == root) {
    depth = 0; pre = 0; size = n; r0 = -1; r1 = -1;
  } else {
    const ulonglong2 pk = reinterpret_cast<const ulonglong2*>(packed)[c];
    uint32_t s0 = (uint32_t)pk.x, s1 = (uint32_t)pk.y;
    if (s0 >= (uint32_t)nsub || s1 >= (uint32_t)nsub) {
      flag(status, ST_BAD_INDEX);
      s0 = 0; s1 = 0;
    }
    const int2 o0 = off[s0];
    const int2 o1 = off[s1];
    r0 = o0.x + (int32_t)((pk.x >> 32) & 0xffffu);
    const int32_t dn = o0.y + (int32_t)(pk.x >> 48);
    r1 = o1.x + (int32_t)((pk.y >> 32) & 0xffffu);
    pre = dn;
    depth = 2 * dn - r0 - 1;
    size = (r1 - r0 + 1) >> 1;
  }
  reinterpret_cast<int2*>(rank)[c] = make_int2(r0, r1);
  pre_out[c] = pre;
  size_out[c] = size;
  const uint32_t inl = inlabel_of(pre, size);
  rec[c] = make_int4((int32_t)inl, 0, depth, pre);
  inl_out[c] = inl;
}

// Path tops: a node is the top of its inlabel path iff it is the root or its
// parent's inlabel differs. head[I] = {parent of the top, its depth}, and
// plab[I] = the inlabel of that parent (0 for the root's path).
__global__ void k_head(const int32_t* __restrict__ parent, const int4* __restrict__ rec,
                       const uint32_t* __restrict__ inl_of, int32_t n, const int32_t* __restrict__ sc,
                       int2* __restrict__ head, uint32_t* __restrict__ plab, uint32_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t root = sc[SC_ROOT];
  const int4 rv = rec[v];
  const uint32_t inl = (uint32_t)rv.x;
  const int32_t p = parent[v];
  bool top;
  uint32_t pinl = 0;
  if (v == root) {
    top = true;
  } else if ((uint32_t)p < (uint32_t)n) {
    pinl = inl_of[p];
    top = pinl != inl;
  } else {
    top = true;
    flag(status, ST_BAD_INDEX);
  }
  if (top) {
    if (inl >= 1u && inl <= (uint32_t)n) {
      head[inl] = make_int2(v == root ? -1 : p, rv.z - 1);
      plab[inl] = (v == root) ? 0u : pinl;
    } else {
      flag(status, ST_BAD_INDEX);
    }
  }
}

// Ascendant of a path label I at level t = h(I): the ascendant of the path
// it hangs from (a label of a strictly higher level, already done) plus bit
// t. plab[] holds the parent path's label on entry and the ascendant on
// exit; unused labels keep kUnused.
constexpr uint32_t kUnused = 0xffffffffu;

__global__ void k_asc_level(uint32_t* __restrict__ plab, int32_t n, int t, uint32_t* __restrict__ status) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t I = ((2 * k + 1) << t);
  if (I > n) return;
  const uint32_t pl = plab[I];
  if (pl == kUnused) return;
  uint32_t up = 0;
  if (pl != 0) {
    if (pl <= (uint32_t)n && ctz32(pl) > t) up = plab[pl];
    else flag(status, ST_BAD_INDEX);
  }
  plab[I] = up | (1u << t);
}

// The levels hi .. lo, each holding at most blockDim.x labels, in one
// workgroup: one label per lane per level, a barrier between levels (the
// labels of a level are read by the next one down).
constexpr int kAscTop = 1024;

__global__ __launch_bounds__(kAscTop) void k_asc_top(uint32_t* __restrict__ plab, int32_t n, int hi, int lo,
                                                    uint32_t* __restrict__ status) {
  for (int t = hi; t >= lo; --t) {
    const int64_t I = ((2 * (int64_t)threadIdx.x + 1) << t);
    if (I <= n) {
      const uint32_t pl = plab[I];
      if (pl != kUnused) {
        uint32_t up = 0;
        if (pl != 0) {
          if (pl <= (uint32_t)n && ctz32(pl) > t) up = plab[pl];
          else flag(status, ST_BAD_INDEX);
        }
        plab[I] = up | (1u << t);
      }
    }
    __syncthreads();
  }
}

__global__ void k_asc(int4* __restrict__ rec, const uint32_t* __restrict__ inl_of,
                      const uint32_t* __restrict__ asc_of_label, int32_t n, uint32_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint32_t inl = inl_of[v];  // the compact copy: a quarter of the record's lines
  uint32_t a = 0;
  if (inl >= 1u && inl <= (uint32_t)n) a = asc_of_label[inl];
  else flag(status, ST_BAD_INDEX);
  reinterpret_cast<int32_t*>(rec)[4 * v + 1] = (int32_t)a;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// n == 1: the root is the only node
__global__ void k_single(const int32_t* __restrict__ parent, int32_t* __restrict__ sc, int32_t* __restrict__ succ,
                         int32_t* __restrict__ rank, int32_t* __restrict__ pre, int32_t* __restrict__ size,
                         int4* __restrict__ rec, int2* __restrict__ head, uint32_t* __restrict__ status) {
  if (parent[0] != -1) flag(status, ST_ROOTS);
  sc[SC_ROOT] = 0;
  succ[0] = succ[1] = -2;
  rank[0] = rank[1] = -1;
  pre[0] = 0;
  size[0] = 1;
  rec[0] = make_int4(1, 1, 0, 0);
  head[1] = make_int2(-1, -1);
}

__global__ void k_fill_zero(int32_t* __restrict__ p, int32_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_export_rec(const int4* __restrict__ rec, int32_t n, int32_t* __restrict__ depth,
                             uint32_t* __restrict__ inl, uint32_t* __restrict__ asc) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int4 r = rec[v];
  if (depth) depth[v] = r.z;
  if (inl) inl[v] = (uint32_t)r.x;
  if (asc) asc[v] = (uint32_t)r.y;
}

// Schieber-Vishkin query, one lane per query. a = inlabel(x), b = inlabel(y).
//  - a == b: x and y lie on one path; the shallower one is the LCA.
//  - otherwise the LCA of a and b in the binary tree has height
//    i = max(h(a), h(b), msb(a xor b)); the LCA's inlabel has height
//    j = the lowest common ascendant bit at or above i; on each side the
//    node closest to it on the LCA's path is the side itself (if its own
//    label has height j) or the parent of the top of the path entered
//    below it, whose label keeps the bits above the highest ascendant bit
//    k < j and sets bit k; the shallower of the two is the LCA.
__device__ __forceinline__ int32_t sv_query(const int4* __restrict__ rec, const int2* __restrict__ head,
                                            uint32_t n, int32_t x, int32_t y, bool* bad) {
  const int4 rx = rec[x];
  const int4 ry = rec[y];
  const uint32_t a = (uint32_t)rx.x, b = (uint32_t)ry.x;
  if (a == b) return (rx.z <= ry.z) ? x : y;
  const int ha = ctz32(a), hb = ctz32(b);
  const int i0 = max(max(ha, hb), msb32(a ^ b));
  const uint32_t ax = (uint32_t)rx.y, ay = (uint32_t)ry.y;
  const uint32_t common = ax & ay & (~0u << i0);
  if (common == 0u) {
    *bad = true;
    return -1;
  }
  const int j = ctz32(common);
  const uint32_t low = (1u << j) - 1u;
  int32_t xv = x, xd = rx.z, yv = y, yd = ry.z;
  if (ha != j) {
    const int k = msb32(ax & low);
    const uint32_t w = ((a >> (k + 1)) << (k + 1)) | (1u << k);
    const int2 h = head[min(w, n)];
    xv = h.x;
    xd = h.y;
  }
  if (hb != j) {
    const int k = msb32(ay & low);
    const uint32_t w = ((b >> (k + 1)) << (k + 1)) | (1u << k);
    const int2 h = head[min(w, n)];
    yv = h.x;
    yd = h.y;
  }
  return (xd <= yd) ? xv : yv;
}

__global__ __launch_bounds__(kQueryBlockMax) void k_lca(const int4* __restrict__ rec, const int2* __restrict__ head, int32_t n,
                                           const int32_t* __restrict__ qx, const int32_t* __restrict__ qy,
                                           int64_t q, int32_t* __restrict__ out, uint32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  const int32_t x = qx[i], y = qy[i];
  if ((uint32_t)x >= (uint32_t)n || (uint32_t)y >= (uint32_t)n) {
    flag(status, ST_BAD_QUERY);
    out[i] = -1;
    return;
  }
  bool bad = false;
  const int32_t r = sv_query(rec, head, (uint32_t)n, x, y, &bad);
  if (bad) flag(status, ST_BAD_INDEX);
  out[i] = r;
}

// Batched trees: tree t's nodes are the global ids [off[t], off[t+1]); all
// trees hang below a virtual root (global id N), so the LCA of two nodes of
// one tree is the LCA in the combined tree.
__device__ __forceinline__ int32_t tree_of(const int64_t* __restrict__ off, int32_t T, int64_t v) {
  int32_t lo = 0, hi = T;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Per-node passes over a batch: each lane takes kPerLane nodes a block
// width apart, so its tree id only moves forward; it searches once at its
// first node and again only when a node lies past its current tree.
constexpr int kPerLane = 16;

__device__ __forceinline__ int32_t tree_from(const int64_t* __restrict__ off, int32_t t, int32_t T, int64_t v) {
  if (off[t + 1] > v) return t;
  int32_t lo = t, hi = T;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kQueryBlockMax) void k_lca_batch(const int4* __restrict__ rec, const int2* __restrict__ head,
                                                 int32_t n, const int64_t* __restrict__ off, int32_t T,
                                                 const int32_t* __restrict__ qt, const int32_t* __restrict__ qx,
                                                 const int32_t* __restrict__ qy, int64_t q, int32_t* __restrict__ out,
                                                 uint32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  const int32_t t = qt[i];
  if ((uint32_t)t >= (uint32_t)T) {
    flag(status, ST_BAD_QUERY);
    out[i] = -1;
    return;
  }
  const int64_t base = off[t];
  const int64_t nt = off[t + 1] - base;
  const int32_t x = qx[i], y = qy[i];
  if ((int64_t)(uint32_t)x >= nt || (int64_t)(uint32_t)y >= nt || base + nt > n) {
    flag(status, ST_BAD_QUERY);
    out[i] = -1;
    return;
  }
  bool bad = false;
  const int32_t r = sv_query(rec, head, (uint32_t)n, (int32_t)(base + x), (int32_t)(base + y), &bad);
  if (bad || r < base || r >= base + nt) {
    flag(status, ST_BAD_INDEX);
    out[i] = -1;
    return;
  }
  out[i] = (int32_t)(r - base);
}

// combined parent array: roots of the trees hang below the virtual root N
__global__ void k_batch_parent(const int32_t* __restrict__ parent, const int64_t* __restrict__ off, int32_t T,
                               int32_t N, int32_t* __restrict__ gp, int32_t* __restrict__ nroots,
                               int32_t* __restrict__ root_of, uint32_t* __restrict__ status) {
  const int64_t first = (int64_t)blockIdx.x * blockDim.x * kPerLane + threadIdx.x;
  if (first > N) return;
  int32_t t = tree_of(off, T, min(first, (int64_t)N - 1));
  for (int i = 0; i < kPerLane; ++i) {
    const int64_t v = first + (int64_t)i * blockDim.x;
    if (v > N) break;
    if (v == N) {
      gp[N] = -1;
      if (off[0] != 0 || off[T] != N) flag(status, ST_BAD_PARENT);
      break;
    }
    t = tree_from(off, t, T, v);
    const int64_t base = off[t], nt = off[t + 1] - base;
    const int32_t p = parent[v];
    if (p == -1) {
      gp[v] = N;
      atomicAdd(nroots + t, 1);
      root_of[t] = (int32_t)v;
    } else if (p >= 0 && p < nt && base + p != v) {
      gp[v] = (int32_t)(base + p);
    } else {
      flag(status, ST_BAD_PARENT);
      gp[v] = N;
    }
  }
}

__global__ void k_batch_check(const int64_t* __restrict__ off, int32_t T, const int32_t* __restrict__ nroots,
                              uint32_t* __restrict__ status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  if (nroots[t] != 1 || off[t + 1] <= off[t]) flag(status, ST_ROOTS);
}

// per-tree statistics of a batch: preorder and depth relative to the tree's root
__global__ void k_export_batch(const int4* __restrict__ rec, const int32_t* __restrict__ size_in,
                               const int64_t* __restrict__ off, int32_t T, int32_t N,
                               const int32_t* __restrict__ root_of, int32_t* __restrict__ depth,
                               int32_t* __restrict__ pre, int32_t* __restrict__ size) {
  const int64_t first = (int64_t)blockIdx.x * blockDim.x * kPerLane + threadIdx.x;
  if (first >= N) return;
  int32_t t = tree_of(off, T, first);
  for (int i = 0; i < kPerLane; ++i) {
    const int64_t v = first + (int64_t)i * blockDim.x;
    if (v >= N) break;
    t = tree_from(off, t, T, v);
    const int32_t r = root_of[t];
    const int4 rv = rec[v];
    const int32_t rp = ((uint32_t)r < (uint32_t)N) ? rec[r].w : 0;
    if (depth) depth[v] = rv.z - 1;
    if (pre) pre[v] = rv.w - rp;
    if (size) size[v] = size_in[v];
  }
}

}  // namespace

// Scratch of tree_build: the grouping buffer and the compact inlabels, the
// grouping's own scratch (released before the ranking starts, but counted
// as if held: the pool may hand a released block to a smaller request) and
// the ranking's buffers; a batch adds its combined parent array and root
// counts.
size_t tree_build_scratch_bytes(const Ctx* c, int32_t n, int32_t batch) {
  size_t b = 0;
  if (batch) {
    b += scratch_block<int32_t>((size_t)n) + scratch_block<int32_t>((size_t)batch);  // n counts the virtual root
  }
  if (n <= 1) return b;
  b += scratch_block<uint32_t>(2 * (size_t)n) + scratch_block<uint32_t>((size_t)n);
  return b + group_by_parent_scratch_bytes(n) + list_rank_plan_bytes(c, 2 * n, 1, 0);
}

int tree_build(Ctx* c, et_tree* t, const int32_t* parent, hipStream_t s) {
  const int32_t n = t->n;
  int32_t* sc = t->d_root;
  if (n == 1) {
    hipLaunchKernelGGL(k_single, dim3(1), dim3(1), 0, s, parent, sc, t->d_succ, t->d_rank, t->d_pre, t->d_size,
                       t->d_rec, t->d_head, c->d_status);
    return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
  }
  const int32_t L2 = 2 * n;          // half-edge id space (the tour uses 2(n-1) of them)
  Scratch scr(c, s);
  uint32_t* kv = scr.get<uint32_t>((size_t)L2);  // sorted parents | children, later the path-label table
  if (scr.failed) return ET_ENOMEM;
  uint32_t* keys = kv;
  int32_t* vals = reinterpret_cast<int32_t*>(kv + n);
  const int gn = ceil_div(n, kB);
  LRResult lr;
  uint32_t* inl = scr.get<uint32_t>((size_t)n);  // inlabel of every node, compact for gathers
  if (scr.failed) return ET_ENOMEM;
  int rc;
  {
    ET_PROF(c, s, "phase:tour");
    rc = group_by_parent_impl(c, parent, n, keys, vals, t->d_succ, sc, s);
    if (rc) return rc;
    {
      ET_PROF(c, s, "k_succ");
      hipLaunchKernelGGL(k_succ, dim3(gn), dim3(kB), 0, s, keys, vals, n, sc, t->d_succ, c->d_status);
    }
    rc = list_rank_core(c, scr, t->d_succ, L2, sc + SC_HEAD, 1, true, sc + SC_EXPECT, &lr, s);
    if (rc) return rc;
    {
      ET_PROF(c, s, "k_node");
      hipLaunchKernelGGL(k_node, dim3(gn), dim3(kB), 0, s, lr.packed, lr.off, lr.nsub, n, sc, t->d_rank, t->d_pre,
                         t->d_size, t->d_rec, inl, c->d_status);
    }
  }
  return inlabel_phase(c, t, parent, inl, kv, s);  // n+1 label slots: the grouping keys are dead by now
}

int inlabel_phase(Ctx* c, et_tree* t, const int32_t* parent, const uint32_t* inl, uint32_t* plab, hipStream_t s) {
  const int32_t n = t->n;
  int32_t* sc = t->d_root;
  const int gn = ceil_div(n, kB);
  ET_PROF(c, s, "phase:inlabel");
  hipLaunchKernelGGL(k_fill_u32, dim3(std::min(ceil_div((int64_t)n + 1, kB), 8192)), dim3(kB), 0, s, plab,
                     (int64_t)n + 1, kUnused);
  {
    ET_PROF(c, s, "k_head");
    hipLaunchKernelGGL(k_head, dim3(gn), dim3(kB), 0, s, parent, t->d_rec, inl, n, sc, t->d_head, plab,
                       c->d_status);
  }
  {
    ET_PROF(c, s, "k_asc_level");
    int top = 0;
    while ((2ll << top) <= n) ++top;  // highest level a label <= n can have
    // labels (2k+1) 2^lv <= n of level lv: (n >> lv) / 2 + 1 candidates
    int lo = top;
    while (lo > 0 && (((int64_t)n >> (lo - 1)) / 2 + 1) <= kAscTop) --lo;
    hipLaunchKernelGGL(k_asc_top, dim3(1), dim3(kAscTop), 0, s, plab, n, top, lo, c->d_status);
    for (int lv = lo - 1; lv >= 0; --lv) {
      const int64_t cand = ((int64_t)n >> lv) / 2 + 1;
      hipLaunchKernelGGL(k_asc_level, dim3(ceil_div(cand, kB)), dim3(kB), 0, s, plab, n, lv, c->d_status);
    }
  }
  {
    ET_PROF(c, s, "k_asc");
    hipLaunchKernelGGL(k_asc, dim3(gn), dim3(kB), 0, s, t->d_rec, inl, plab, n, c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int tree_export(const et_tree* t, int32_t* succ, int32_t* rank, int32_t* depth, int32_t* pre, int32_t* size,
                uint32_t* inl, uint32_t* asc, hipStream_t s) {
  if (t->batch) {
    if (succ || rank || inl || asc) return ET_EINVAL;  // global tables of a batch are internal
    const int32_t N = t->n - 1;
    if (depth || pre || size)
      hipLaunchKernelGGL(k_export_batch, dim3(ceil_div(N, (int64_t)kB * kPerLane)), dim3(kB), 0, s, t->d_rec,
                         t->d_size, t->d_off,
                         t->batch, N, t->d_root_of, depth, pre, size);
    return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
  }
  const int32_t n = t->n;
  const size_t b = (size_t)n * sizeof(int32_t);
  if (succ && hipMemcpyAsync(succ, t->d_succ, 2 * b, hipMemcpyDeviceToDevice, s) != hipSuccess) return ET_EHIP;
  if (rank && hipMemcpyAsync(rank, t->d_rank, 2 * b, hipMemcpyDeviceToDevice, s) != hipSuccess) return ET_EHIP;
  if (pre && hipMemcpyAsync(pre, t->d_pre, b, hipMemcpyDeviceToDevice, s) != hipSuccess) return ET_EHIP;
  if (size && hipMemcpyAsync(size, t->d_size, b, hipMemcpyDeviceToDevice, s) != hipSuccess) return ET_EHIP;
  if (depth || inl || asc)
    hipLaunchKernelGGL(k_export_rec, dim3(ceil_div(n, kB)), dim3(kB), 0, s, t->d_rec, n, depth, inl, asc);
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

namespace {
// tour[rank(e)] = e for every half-edge on the tour
__global__ void k_tour(const int32_t* __restrict__ rank, int64_t E, int32_t L, int32_t* __restrict__ tour,
                       uint32_t* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int32_t r = rank[e];
  if (r < 0) return;  // the root's two unused ids
  if (r >= L) {
    flag(status, ST_BAD_INDEX);
    return;
  }
  tour[r] = (int32_t)e;
}
}  // namespace

int tree_export_tour(Ctx* c, const et_tree* t, int32_t* tour, hipStream_t s) {
  if (t->batch) return ET_EINVAL;  // the combined tour of a batch is internal
  const int32_t L = 2 * (t->n - 1);
  if (L == 0) return ET_OK;
  // a parent-array tree numbers its half-edges 2c / 2c+1 over all n nodes,
  // an edge-list tree 2i / 2i+1 over its n-1 edges
  const int64_t E = t->from_edges ? (int64_t)L : 2 * (int64_t)t->n;
  hipLaunchKernelGGL(k_tour, dim3(ceil_div(E, kB)), dim3(kB), 0, s, t->d_rank, E, L, tour, c->d_status);
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int tree_lca_batch(Ctx* c, const et_tree* t, const int32_t* qt, const int32_t* qx, const int32_t* qy, int64_t q,
                   int32_t* out, hipStream_t s) {
  if (q == 0) return ET_OK;
  const int bs = c->qs.block;
  ET_PROF(c, s, "k_lca_batch");
  for (int64_t q0 = 0; q0 < q; q0 += kQueryChunk) {  // one dispatch holds < 2^32 work-items
    const int64_t m = std::min(q - q0, kQueryChunk);
    hipLaunchKernelGGL(k_lca_batch, dim3((unsigned)((m + bs - 1) / bs)), dim3(bs), 0, s, t->d_rec, t->d_head, t->n,
                       t->d_off, t->batch, qt + q0, qx + q0, qy + q0, m, out + q0, c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int tree_build_batch(Ctx* c, et_tree* t, const int32_t* parent, hipStream_t s) {
  const int32_t N = t->n - 1, T = t->batch;
  Scratch scr(c, s);
  int32_t* gp = scr.get<int32_t>((size_t)N + 1);
  int32_t* nroots = scr.get<int32_t>((size_t)T);
  if (scr.failed) return ET_ENOMEM;
  hipLaunchKernelGGL(k_fill_zero, dim3(ceil_div(T, kB)), dim3(kB), 0, s, nroots, T);
  {
    ET_PROF(c, s, "k_batch_parent");
    hipLaunchKernelGGL(k_batch_parent, dim3(ceil_div((int64_t)N + 1, (int64_t)kB * kPerLane)), dim3(kB), 0, s, parent,
                       t->d_off, T, N,
                       gp, nroots, t->d_root_of, c->d_status);
  }
  hipLaunchKernelGGL(k_batch_check, dim3(ceil_div(T, kB)), dim3(kB), 0, s, t->d_off, T, nroots, c->d_status);
  return tree_build(c, t, gp, s);
}

int tree_lca(Ctx* c, const et_tree* t, const int32_t* qx, const int32_t* qy, int64_t q, int32_t* out,
             hipStream_t s) {
  if (q == 0) return ET_OK;
  const int bs = c->qs.block;
  ET_PROF(c, s, "k_lca");
  for (int64_t q0 = 0; q0 < q; q0 += kQueryChunk) {  // one dispatch holds < 2^32 work-items
    const int64_t m = std::min(q - q0, kQueryChunk);
    hipLaunchKernelGGL(k_lca, dim3((unsigned)((m + bs - 1) / bs)), dim3(bs), 0, s, t->d_rec, t->d_head, t->n, qx + q0,
                       qy + q0, m, out + q0, c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
