// Euler tour and tree tables from an unordered edge list: the DCEL
// construction of Section 2.1 as the paper states it, for inputs that are
// not already a parent array.
//
//  1. Half-edges: edge i gives 2i = (u_i -> v_i) and its twin 2i+1.
//  2. B = the half-edges in lexicographic (source, target) order: a stable
//     radix sort by target, then one by source (the paper's sort, which it
//     notes dominates this construction).
//  3. first[x] = start of x's run in B; next(e) = the half-edge after e in
//     its run, wrapping to the run's start; succ(e) = next(twin(e)), written
//     from the sorted side: the thread at B-position k holding h sets
//     succ(h xor 1) = next(h). The cycle is cut before the root's first
//     half-edge. At a node entered from p the children follow in cyclic id
//     order after p.
//  4. One list ranking. A half-edge goes down iff it precedes its twin
//     (Section 2), which gives every node its parent, subtree size (from the
//     two ranks) and the rank of its entering half-edge; a scan of the down
//     flags in tour order gives preorder, and depth = 2 * preorder - rank - 1.
//  5. The Inlabel tables as for a parent array (tree.hip).
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kB = 256;
enum { SC_ROOT = 0, SC_HEAD = 2, SC_EXPECT = 3 };

__global__ void k_fill(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// both ends of every half-edge; ids out of range or a self-loop are flagged
// and replaced by 0 so that every later index stays in bounds
__global__ void k_expand(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev, int32_t m, int32_t n,
                         int32_t* __restrict__ srcA, uint32_t* __restrict__ dst_key, int32_t* __restrict__ ids,
                         uint32_t* __restrict__ status) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= 2 * (int64_t)m) return;
  int32_t a = eu[h >> 1], b = ev[h >> 1];
  if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n || a == b) {
    flag(status, ST_BAD_PARENT);
    a = 0;
    b = 0;
  }
  srcA[h] = (h & 1) ? b : a;
  dst_key[h] = (uint32_t)((h & 1) ? a : b);
  ids[h] = (int32_t)h;
}

__global__ void k_src_key(const int32_t* __restrict__ order, const int32_t* __restrict__ srcA, int32_t L,
                          uint32_t* __restrict__ key) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < L) key[k] = (uint32_t)srcA[order[k]];
}

__global__ void k_run_first(const uint32_t* __restrict__ srcB, int32_t L, int32_t* __restrict__ first) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const uint32_t x = srcB[k];
  if (k == 0 || srcB[k - 1] != x) first[x] = (int32_t)k;
}

__global__ void k_set_head(const int32_t* __restrict__ first, const int32_t* __restrict__ B, int32_t root,
                           int32_t L, int32_t* __restrict__ sc, int32_t* __restrict__ succ,
                           int32_t* __restrict__ rank, uint32_t* __restrict__ status) {
  const int32_t f = first[root];
  sc[SC_ROOT] = root;
  sc[SC_EXPECT] = L;
  if (f < 0 || f >= L) {
    flag(status, ST_ROOTS);  // the root has no edge: not one tree
    sc[SC_HEAD] = -1;
  } else {
    sc[SC_HEAD] = B[f];
  }
  succ[L] = succ[L + 1] = -2;  // the two ids past 2(n-1) are unused
  rank[L] = rank[L + 1] = -1;
}

__global__ void k_dcel_succ(const int32_t* __restrict__ B, const uint32_t* __restrict__ srcB,
                            const int32_t* __restrict__ first, int32_t L, const int32_t* __restrict__ sc,
                            int32_t* __restrict__ succ) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const int32_t h = B[k];
  const uint32_t x = srcB[k];
  const int32_t nxt = (k + 1 < L && srcB[k + 1] == x) ? B[k + 1] : B[first[x]];
  succ[h ^ 1] = (nxt == sc[SC_HEAD]) ? -1 : nxt;
}

__global__ void k_ranks(const uint64_t* __restrict__ packed, const int2* __restrict__ off, int32_t nsub, int32_t L,
                        int32_t* __restrict__ rank, uint32_t* __restrict__ status) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= L) return;
  const uint64_t p = packed[h];
  uint32_t sub = (uint32_t)p;
  if (sub >= (uint32_t)nsub) {
    flag(status, ST_BAD_INDEX);
    sub = 0;
  }
  rank[h] = off[sub].x + (int32_t)((p >> 32) & 0xffffu);
}

// per edge: the half-edge that goes down, its child's record
// {parent, subtree size, rank of the entering half-edge}, and the down flag
// at that rank
__global__ void k_edge_dir(const int32_t* __restrict__ rank, const int32_t* __restrict__ srcA, int32_t m,
                           int32_t n, int32_t L, uint32_t* __restrict__ dw, int4* __restrict__ vrec,
                           uint32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t r0 = rank[2 * i], r1 = rank[2 * i + 1];
  if ((uint32_t)r0 >= (uint32_t)L || (uint32_t)r1 >= (uint32_t)L) {
    flag(status, ST_BAD_INDEX);
    return;
  }
  const int64_t down = (r0 < r1) ? 2 * i : 2 * i + 1;
  const int32_t rd = min(r0, r1), ru = max(r0, r1);
  const int32_t child = srcA[down ^ 1], par = srcA[down];
  if ((uint32_t)child >= (uint32_t)n) {
    flag(status, ST_BAD_INDEX);
    return;
  }
  vrec[child] = make_int4(par, (ru - rd + 1) >> 1, rd, 0);
  dw[rd] = 1u;
}

__global__ void k_edge_node(const int4* __restrict__ vrec, const uint32_t* __restrict__ I, int32_t n, int32_t L,
                            int32_t root, int32_t* __restrict__ parent, int32_t* __restrict__ pre_out,
                            int32_t* __restrict__ size_out, int4* __restrict__ rec, uint32_t* __restrict__ inl_out,
                            uint32_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t par = -1, pre = 0, size = n, depth = 0;
  if (v != root) {
    const int4 r = vrec[v];
    par = r.x;
    size = r.y;
    if ((uint32_t)par >= (uint32_t)n || (uint32_t)r.z >= (uint32_t)L || size < 1) {
      flag(status, ST_UNREACHED);  // no edge brought the tour into v
      par = root;
      pre = 0;
      size = 1;
    } else {
      pre = (int32_t)I[r.z];                 // down half-edges up to and including v's entering one
      depth = 2 * pre - r.z - 1;
    }
  }
  parent[v] = par;
  pre_out[v] = pre;
  size_out[v] = size;
  const uint32_t inl = inlabel_of(pre, size);
  rec[v] = make_int4((int32_t)inl, 0, depth, pre);
  inl_out[v] = inl;
}

__global__ void k_single_edges(int32_t* __restrict__ sc, int32_t* __restrict__ succ, int32_t* __restrict__ rank,
                               int32_t* __restrict__ pre, int32_t* __restrict__ size, int4* __restrict__ rec,
                               int2* __restrict__ head, int32_t* __restrict__ parent) {
  sc[SC_ROOT] = 0;
  succ[0] = succ[1] = -2;
  rank[0] = rank[1] = -1;
  pre[0] = 0;
  size[0] = 1;
  rec[0] = make_int4(1, 1, 0, 0);
  head[1] = make_int2(-1, -1);
  if (parent) parent[0] = -1;
}

}  // namespace

int tree_build_edges(Ctx* c, et_tree* t, const int32_t* eu, const int32_t* ev, int32_t root, int32_t* parent_out,
                     hipStream_t s) {
  const int32_t n = t->n;
  int32_t* sc = t->d_root;
  if (n == 1) {
    hipLaunchKernelGGL(k_single_edges, dim3(1), dim3(1), 0, s, sc, t->d_succ, t->d_rank, t->d_pre, t->d_size,
                       t->d_rec, t->d_head, parent_out);
    return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
  }
  const int32_t m = n - 1;
  const int32_t L = 2 * m;
  int bits = 1;
  while (bits < 31 && (1ll << bits) < n) ++bits;
  Scratch scr(c, s);
  int32_t* srcA = scr.get<int32_t>((size_t)L);
  uint32_t* key = scr.get<uint32_t>((size_t)L);
  int32_t* ids = scr.get<int32_t>((size_t)L);
  uint32_t* key2 = scr.get<uint32_t>((size_t)L);
  int32_t* ord = scr.get<int32_t>((size_t)L);
  int32_t* first = scr.get<int32_t>((size_t)n);
  int32_t* parent = parent_out ? parent_out : scr.get<int32_t>((size_t)n);
  uint32_t* inl = scr.get<uint32_t>((size_t)n);
  int4* vrec = scr.get<int4>((size_t)n);
  uint32_t* plab = scr.get<uint32_t>((size_t)n + 1);
  if (scr.failed) return ET_ENOMEM;
  const int gl = ceil_div(L, kB), gn = ceil_div(n, kB), gm = ceil_div(m, kB);
  int rc;
  {
    ET_PROF(c, s, "phase:dcel");
    {
      ET_PROF(c, s, "k_expand");
      hipLaunchKernelGGL(k_expand, dim3(gl), dim3(kB), 0, s, eu, ev, m, n, srcA, key, ids, c->d_status);
    }
    rc = sort_pairs_u32(c, key, ids, L, bits, key2, ord, s);  // by target
    if (rc) return rc;
    {
      ET_PROF(c, s, "k_src_key");
      hipLaunchKernelGGL(k_src_key, dim3(gl), dim3(kB), 0, s, ord, srcA, L, key);
    }
    rc = sort_pairs_u32(c, key, ord, L, bits, key2, ids, s);  // then stably by source: B = ids, sources = key2
    if (rc) return rc;
    hipLaunchKernelGGL(k_fill, dim3(std::min(gn, 4096)), dim3(kB), 0, s, first, (int64_t)n, -1);
    hipLaunchKernelGGL(k_run_first, dim3(gl), dim3(kB), 0, s, key2, L, first);
    hipLaunchKernelGGL(k_set_head, dim3(1), dim3(1), 0, s, first, ids, root, L, sc, t->d_succ, t->d_rank,
                       c->d_status);
    {
      ET_PROF(c, s, "k_dcel_succ");
      hipLaunchKernelGGL(k_dcel_succ, dim3(gl), dim3(kB), 0, s, ids, key2, first, L, sc, t->d_succ);
    }
  }
  LRResult lr;
  rc = list_rank_core(c, scr, t->d_succ, L, sc + SC_HEAD, 1, false, sc + SC_EXPECT, &lr, s);
  if (rc) return rc;
  uint32_t* dw = key;  // the sort keys are dead: down flags in tour order, then their scan
  {
    ET_PROF(c, s, "phase:nodes");
    hipLaunchKernelGGL(k_ranks, dim3(gl), dim3(kB), 0, s, lr.packed, lr.off, lr.nsub, L, t->d_rank, c->d_status);
    hipLaunchKernelGGL(k_fill, dim3(std::min(gl, 8192)), dim3(kB), 0, s, reinterpret_cast<int32_t*>(dw),
                       (int64_t)L, 0);
    hipLaunchKernelGGL(k_fill, dim3(std::min(4 * (int64_t)gn, (int64_t)8192)), dim3(kB), 0, s,
                       reinterpret_cast<int32_t*>(vrec), 4 * (int64_t)n, -1);
    {
      ET_PROF(c, s, "k_edge_dir");
      hipLaunchKernelGGL(k_edge_dir, dim3(gm), dim3(kB), 0, s, t->d_rank, srcA, m, n, L, dw, vrec, c->d_status);
    }
    rc = scan_u32(c, dw, dw, L, ScanOp::Add, false, s);
    if (rc) return rc;
    {
      ET_PROF(c, s, "k_edge_node");
      hipLaunchKernelGGL(k_edge_node, dim3(gn), dim3(kB), 0, s, vrec, dw, n, L, root, parent, t->d_pre, t->d_size,
                         t->d_rec, inl, c->d_status);
    }
  }
  return inlabel_phase(c, t, parent, inl, plab, s);
}

}  // namespace et
