// Bridges by the Tarjan-Vishkin method (Section 4.1) on a symmetric CSR.
//
//  1. Spanning forest (the paper uses the connectivity code of Jaiganesh and
//     Burtscher, which yields a spanning tree as a by-product): union-find
//     hooking where a successful compare-and-swap of a root joins two
//     different trees, so its edge is a forest edge; both of its slots are
//     marked in a bitmask. Parallel copies of an edge are never forest edges
//     and self-loops are skipped. Every vertex first hooks its first two
//     distinct neighbours; then the most frequent root of a sample names the
//     big component, and only rows of vertices outside it hook all their
//     edges (an edge inside the big component joins nothing new).
//  2. Euler tour of the forest as the paper's DCEL (Section 2.1) read from
//     the CSR: the forest slots of a row, in row order, are the sorted run
//     of B for that vertex, next() wraps inside the run, twin() is found by
//     a search in the neighbour's run, succ = next(twin). The tours of all
//     components are chained into one list (component roots in id order).
//  3. One list ranking; a half-edge goes down iff it precedes its twin
//     (Section 2), which gives every vertex its parent edge and subtree
//     size. The preorder comes from an array scan over tour order of
//     (down + starts-a-component) weights (Section 2.2).
//  4. For every vertex the minimum and maximum preorder over itself and its
//     non-forest neighbours (the paper's segreduce); stored by preorder.
//  5. low(v) / high(v) = range minimum / maximum of those over v's subtree
//     interval, with a sparse table over 32-element blocks and per-position
//     suffix-extreme bitmasks inside a block (the paper uses a segment tree).
//  6. The forest edge above v is a bridge iff low(v) and high(v) both lie
//     inside [pre(v), pre(v) + size(v)) (Tarjan 1974; including pre(v)
//     itself makes the test two equalities). Both slots get their bit.
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kB = 256;
constexpr int kRowsPerBlock = 256;
constexpr int kMaxGrid = 1 << 20;  // workgroups of a grid-stride launch (a dispatch holds < 2^32 work-items)

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_iota(int32_t* __restrict__ p, int32_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

__device__ __forceinline__ int32_t ld(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Union-find over cc[]: roots satisfy cc[r] == r. A link always hangs the
// root with the larger key under the node with the smaller key, where the
// key is the vertex id except that the designated big component's root (if
// any) counts as smallest; keys therefore strictly decrease towards the
// root, so the forest stays acyclic under concurrent links, and every
// successful compare-and-swap joins two different trees: its edge is a
// spanning-forest edge.
//
// Loads are ordinary cached loads, which may return an out-of-date parent
// (each XCD has its own L2); an out-of-date parent is still an ancestor.
// Only the device-scope compare-and-swap decides a link, and when it fails
// it returns the node's current parent, from which the link continues.
__device__ __forceinline__ int32_t ldc(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void stc(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// an ancestor-or-self of x that looked like a root; halves the path on the way
__device__ int32_t cc_find(int32_t* cc, int32_t x) {
  int32_t cur = x;
  for (;;) {
    const int32_t p = ldc(cc + cur);
    if (p == cur) return cur;
    const int32_t gp = ldc(cc + p);
    if (gp != p) stc(cc + cur, gp);
    cur = gp;
  }
}

__device__ __forceinline__ int64_t cc_key(int32_t v, int32_t big) { return v == big ? -1 : (int64_t)v; }

// Climbing link of the trees of u and w: keep one ancestor of each, and at
// every step try to hang the one with the larger key (if it is a root)
// under the other, else move it up to its grandparent and the other one up
// to its parent. A node of one tree is never hung under a node of the same
// tree: the larger key of two such nodes is never that tree's root. Every
// step moves the larger-key side strictly up, so the loop ends.
// Returns true iff this call linked two trees (edge {u, w} joins the forest).
__device__ bool cc_hook(int32_t* cc, int32_t u, int32_t w, int32_t big, bool* over) {
  int32_t p1 = ldc(cc + u), p2 = ldc(cc + w);
  for (int it = 0; it < (1 << 22); ++it) {
    if (p1 == p2) return false;
    const bool up1 = cc_key(p1, big) > cc_key(p2, big);
    const int32_t hi = up1 ? p1 : p2, lo = up1 ? p2 : p1;
    int32_t ph = ldc(cc + hi);
    if (ph == lo) return false;
    if (ph == hi) {
      const int32_t old = atomicCAS(cc + hi, hi, lo);
      if (old == hi) return true;
      ph = old;  // linked meanwhile: continue from its current parent
    }
    p1 = ldc(cc + ph);
    p2 = ldc(cc + lo);
  }
  *over = true;
  return false;
}

// mark slot k = (u, w) and its twin, the first (w, u) slot of row w
__device__ void mark_forest(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int32_t nnz,
                            uint32_t* __restrict__ tbits, int32_t k, int32_t u, int32_t w, bool* bad) {
  atomicOr(tbits + (k >> 5), 1u << (k & 31));
  const int32_t wbeg = min(max(row_ptr[w], 0), nnz);
  const int32_t wend = min(max(row_ptr[w + 1], wbeg), nnz);
  int32_t lo = wbeg, hi = wend;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (col[mid] < u) lo = mid + 1;
    else hi = mid;
  }
  if (lo < wend && col[lo] == u) atomicOr(tbits + (lo >> 5), 1u << (lo & 31));
  else *bad = true;
}

__device__ __forceinline__ int32_t clampi(int32_t x, int32_t lo, int32_t hi) { return min(max(x, lo), hi); }

// row_ptr must be monotone from 0 to nnz; anything else is flagged
__global__ void k_check_csr(const int32_t* __restrict__ row_ptr, int32_t n, int32_t nnz,
                            uint32_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t a = row_ptr[v], b = row_ptr[v + 1];
  bool bad = a > b || a < 0 || b > nnz;
  if (v == 0 && a != 0) bad = true;
  if (v == n - 1 && b != nnz) bad = true;
  if (bad) flag(status, ST_BAD_CSR);
}

// rows [b*256, b*256+256) of the CSR; lane-strided over their slots
__device__ __forceinline__ int row_of(const int32_t* rp_lds, int cnt, int32_t k) {
  int lo = 0, hi = cnt;  // largest i in [0, cnt) with rp[i] <= k
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rp_lds[mid] <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Sampling phase: in round j every vertex hooks its j-th distinct neighbour
// (rounds 0 .. kSample-1, each followed by a full path compression).
constexpr int kSample = 2;

__global__ void k_hook_sample(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int32_t n,
                              int32_t nnz, int32_t* cc, uint32_t* __restrict__ tbits, uint32_t* __restrict__ status,
                              int jsel) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int32_t a = clampi(row_ptr[u], 0, nnz), b = clampi(row_ptr[u + 1], a, nnz);
  bool bad = false, over = false;
  int taken = 0;
  for (int32_t k = a; k < b && taken <= jsel; ++k) {
    const int32_t w = col[k];
    if ((uint32_t)w >= (uint32_t)n) {
      bad = true;
      continue;
    }
    if (w == u || (k > a && col[k - 1] == w)) continue;  // self-loop or a parallel copy
    if (taken++ != jsel) continue;
    if (cc_hook(cc, (int32_t)u, w, -1, &over)) mark_forest(row_ptr, col, nnz, tbits, k, (int32_t)u, w, &bad);
  }
  if (bad) flag(status, ST_BAD_CSR);
  if (over) flag(status, ST_OVERFLOW);
}

__global__ void k_cc_compress(int32_t* cc, int32_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) st(cc + v, cc_find(cc, (int32_t)v));
}

// The most frequent root among 1024 sampled vertices: the big component.
constexpr int kBigSample = 1024;

__global__ __launch_bounds__(kBigSample) void k_big_component(const int32_t* cc, int32_t n, int32_t* __restrict__ big) {
  __shared__ int32_t r[kBigSample];
  __shared__ int32_t best, best_count;
  const int t = threadIdx.x;
  const uint32_t v = mix32(0x2545f491u + (uint32_t)t) % (uint32_t)n;
  r[t] = ld(cc + v);
  if (t == 0) {
    best = INT32_MAX;
    best_count = 0;
  }
  __syncthreads();
  for (int k = 2; k <= kBigSample; k <<= 1) {  // bitonic sort
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int o = t ^ j;
      if (o > t) {
        const bool up = (t & k) == 0;
        const int32_t x = r[t], y = r[o];
        if ((x > y) == up) {
          r[t] = y;
          r[o] = x;
        }
      }
      __syncthreads();
    }
  }
  // the longest run of equal roots wins (smallest root on a tie)
  int len = 0;
  if (t == 0 || r[t - 1] != r[t]) {
    // the run's end by a binary search in the sorted samples (walking it
    // took one LDS read per member: ~1000 in a row when one component
    // holds nearly every sample)
    const int32_t x = r[t];
    int lo = t + 1, hi = kBigSample;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (r[mid] == x) lo = mid + 1;
      else hi = mid;
    }
    len = lo - t;
    atomicMax(&best_count, len);
  }
  __syncthreads();
  if (len > 0 && len == best_count) atomicMin(&best, r[t]);
  __syncthreads();
  if (t == 0) *big = best;
}

// Remaining phase: rows of vertices outside the big component hook every
// distinct neighbour. An edge between two vertices of the big component is
// already inside one tree; any other edge is seen from an endpoint outside.
__global__ __launch_bounds__(kB) void k_hook_rest(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                 int32_t n, int32_t nnz, int32_t* cc, const int32_t* __restrict__ bigp,
                                                 uint32_t* __restrict__ tbits, uint32_t* __restrict__ status) {
  __shared__ int32_t rp[kRowsPerBlock + 1];
  __shared__ uint8_t skip[kRowsPerBlock];
  const int32_t r0 = blockIdx.x * kRowsPerBlock;
  const int cnt = min(kRowsPerBlock, n - r0);
  const int32_t big = *bigp;
  for (int i = threadIdx.x; i <= cnt; i += kB) rp[i] = clampi(row_ptr[r0 + i], 0, nnz);
  for (int i = threadIdx.x; i < cnt; i += kB) skip[i] = (cc_find(cc, r0 + i) == big);
  __syncthreads();
  const int32_t kbeg = rp[0], kend = rp[cnt];
  bool bad = false, over = false;
  // 64-bit counter: kend may lie within one stride of 2^31
  for (int64_t kk = (int64_t)kbeg + threadIdx.x; kk < kend; kk += kB) {
    const int32_t k = (int32_t)kk;
    const int ri = row_of(rp, cnt, k);
    if (skip[ri]) continue;
    const int32_t u = r0 + ri;
    const int32_t w = col[k];
    if ((uint32_t)w >= (uint32_t)n) {
      bad = true;
      continue;
    }
    if (w == u || (k > rp[ri] && col[k - 1] == w)) continue;
    if (cc_hook(cc, u, w, big, &over)) mark_forest(row_ptr, col, nnz, tbits, k, u, w, &bad);
  }
  if (bad) flag(status, ST_BAD_CSR);
  if (over) flag(status, ST_OVERFLOW);
}

__device__ __forceinline__ uint32_t bits_in(const uint32_t* tbits, int32_t a, int32_t b, int32_t wd) {
  // forest bits of slots [a, b) that fall into word wd
  uint32_t x = tbits[wd];
  const int64_t base = (int64_t)wd << 5;  // 64-bit: base + 32 reaches 2^31 in the last word
  if (a > base) x &= ~0u << (int)(a - base);
  if (b < base + 32) x &= (b - base <= 0) ? 0u : (~0u >> (int)(32 - (b - base)));
  return x;
}

__global__ void k_tree_deg(const int32_t* __restrict__ row_ptr, const uint32_t* __restrict__ tbits, int32_t n,
                           int32_t nnz, uint32_t* __restrict__ tdeg) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int32_t a = clampi(row_ptr[u], 0, nnz), b = clampi(row_ptr[u + 1], a, nnz);
  uint32_t d = 0;
  if (a < b)
    for (int32_t wd = a >> 5; wd <= (b - 1) >> 5; ++wd) d += __popc(bits_in(tbits, a, b, wd));
  tdeg[u] = d;
}

// Forest entries of every vertex u at tptr[u]..: its forest slots in slot
// order, the neighbour at each, and u. The vertices of a workgroup own one
// contiguous output range; when it holds at most kFillStage entries it is
// built in LDS and stored with consecutive lanes on consecutive addresses
// (a lane per vertex storing its own entries leaves every line partly
// written, four times the bytes); a longer range (a hub) is stored directly.
constexpr int kFillStage = 2048;

__global__ __launch_bounds__(kB) void k_tree_fill(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                            const uint32_t* __restrict__ tbits, const uint32_t* __restrict__ tptr, int32_t n,
                            int32_t nnz, int32_t Lcap, int32_t* __restrict__ tslot, int32_t* __restrict__ tnbr,
                            int32_t* __restrict__ tsrc) {
  __shared__ int32_t st_slot[kFillStage], st_nbr[kFillStage], st_src[kFillStage];
  const int64_t u0 = (int64_t)blockIdx.x * kB;
  const int64_t u = u0 + threadIdx.x;
  // tptr is an exclusive scan of the forest degrees (n + 1 entries), so the
  // workgroup's entries are [J0, J1), cut at Lcap
  const uint32_t J0 = tptr[u0];
  const int64_t ue = (u0 + kB < (int64_t)n) ? u0 + kB : (int64_t)n;
  const uint32_t J1 = min(tptr[ue], (uint32_t)Lcap);
  const bool staged = J1 <= J0 || J1 - J0 <= (uint32_t)kFillStage;  // the same for every lane
  if (u < n) {
    const int32_t a = clampi(row_ptr[u], 0, nnz), b = clampi(row_ptr[u + 1], a, nnz);
    uint32_t j = tptr[u];
    for (int32_t wd = a >> 5; a < b && wd <= (b - 1) >> 5; ++wd) {
      uint32_t x = bits_in(tbits, a, b, wd);
      while (x) {
        const int bit = __ffs((int)x) - 1;
        x &= x - 1;
        const int32_t k = (wd << 5) + bit;
        if (j >= (uint32_t)Lcap) {  // only with a malformed CSR (flagged)
          x = 0;
          wd = b;
          break;
        }
        if (staged) {
          st_slot[j - J0] = k;
          st_nbr[j - J0] = col[k];
          st_src[j - J0] = (int32_t)u;
        } else {
          tslot[j] = k;
          tnbr[j] = col[k];
          tsrc[j] = (int32_t)u;
        }
        ++j;
      }
    }
  }
  if (!staged) return;
  __syncthreads();
  if (J1 <= J0) return;
  for (uint32_t i = threadIdx.x; i < J1 - J0; i += kB) {
    tslot[J0 + i] = st_slot[i];
    tnbr[J0 + i] = st_nbr[i];
    tsrc[J0 + i] = st_src[i];
  }
}

// scalars: [0] = L (forest half-edges), [1] = global head, [2] = reach
// twin and cyclic-next successor of every forest half-edge; ids >= L unused
__global__ void k_succ_csr(const int32_t* __restrict__ tnbr, const int32_t* __restrict__ tsrc,
                           const uint32_t* __restrict__ tptr, int32_t n, int32_t Lcap,
                           const int32_t* __restrict__ sc, int32_t* __restrict__ ttwin, int32_t* __restrict__ succ,
                           uint32_t* __restrict__ status) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= Lcap) return;
  const int32_t L = sc[0];
  if (h >= L) {
    succ[h] = -2;
    return;
  }
  const int32_t u = tsrc[h], w = tnbr[h];
  if ((uint32_t)u >= (uint32_t)n || (uint32_t)w >= (uint32_t)n) {  // malformed CSR only
    flag(status, ST_BAD_CSR);
    ttwin[h] = (int32_t)h;
    succ[h] = -1;
    return;
  }
  const int32_t beg = min((int32_t)tptr[w], L);
  const int32_t end = clampi((int32_t)tptr[w + 1], beg, L);
  int32_t lo = beg, hi = end;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (tnbr[mid] < u) lo = mid + 1;
    else hi = mid;
  }
  int32_t t = lo;
  if (t >= end || tnbr[t] != u) {
    flag(status, ST_BAD_CSR);
    t = (int32_t)h;
  }
  ttwin[h] = t;
  succ[h] = (t + 1 < end) ? t + 1 : beg;  // next() wraps to the run start
}

// component roots in id order: root u has cc[u] == u and forest degree > 0.
// rflag[u] = 1 for roots (scanned afterwards into rpos).
__global__ void k_root_flags(const int32_t* __restrict__ cc, const uint32_t* __restrict__ tdeg, int32_t n,
                             uint32_t* __restrict__ rflag) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  rflag[u] = (ld(cc + u) == (int32_t)u && tdeg[u] > 0) ? 1u : 0u;
}

__global__ void k_root_list(const uint32_t* __restrict__ rflag, const uint32_t* __restrict__ rpos, int32_t n,
                            int32_t* __restrict__ roots) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  if (rflag[u]) roots[rpos[u]] = (int32_t)u;
}

__global__ void k_set_len(const uint32_t* __restrict__ tptr, int32_t n, int32_t* __restrict__ sc) {
  const int32_t L = (int32_t)min(tptr[n], (uint32_t)(2 * (n - 1)));
  sc[0] = L;    // forest half-edges
  sc[1] = -1;   // head, set by k_link_roots
  sc[2] = L;    // elements the head must reach
}

// tail of component i (the half-edge into its root from the root's last
// forest neighbour) links to the head of component i+1
__global__ void k_link_roots(const int32_t* __restrict__ roots, const uint32_t* __restrict__ rpos,
                             const uint32_t* __restrict__ rflag, const uint32_t* __restrict__ tptr,
                             const int32_t* __restrict__ ttwin, int32_t n, int32_t* __restrict__ succ,
                             int32_t* __restrict__ sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t nroots = (int32_t)(rpos[n - 1] + rflag[n - 1]);
  const int32_t L = sc[0];
  if (i == 0) sc[1] = (nroots > 0 && (int32_t)tptr[roots[0]] < L) ? (int32_t)tptr[roots[0]] : -1;
  if (i >= nroots) return;
  const int32_t r = roots[i];
  const int32_t last = (int32_t)tptr[r + 1] - 1;
  if (last < 0 || last >= L) return;  // only with a malformed CSR (flagged)
  const int32_t tail = ttwin[last];
  int32_t nxt = -1;
  if (i + 1 < nroots) nxt = min((int32_t)tptr[roots[i + 1]], L - 1);
  succ[tail] = nxt;
}

__global__ void k_rank_of(const uint64_t* __restrict__ packed, const int2* __restrict__ off, int32_t nsub,
                          int32_t Lcap, const int32_t* __restrict__ sc, int32_t* __restrict__ rank,
                          uint32_t* __restrict__ status) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= Lcap) return;
  if (h >= sc[0]) return;
  const uint64_t p = packed[h];
  uint32_t s = (uint32_t)p;
  if (s >= (uint32_t)nsub) {
    flag(status, ST_BAD_INDEX);
    s = 0;
  }
  rank[h] = off[s].x + (int32_t)((p >> 32) & 0xffffu);
}

// per forest half-edge: direction, parent edge and subtree size of the
// child, and the scan weight in tour order. Each vertex gets one record
// vrec = {rank of its entering half-edge (or of its component's first
// half-edge), subtree size, CSR slot of its parent edge at the parent,
// slot of the same edge in its own row}; the two slots are -1 at a root.
__global__ void k_direction(const int32_t* __restrict__ rank, const int32_t* __restrict__ ttwin,
                            const int32_t* __restrict__ tsrc, const int32_t* __restrict__ tnbr,
                            const int32_t* __restrict__ tslot, const uint32_t* __restrict__ tptr,
                            const int32_t* cc, int32_t n, int32_t Lcap, const int32_t* __restrict__ sc,
                            uint32_t* __restrict__ dw, int4* __restrict__ vrec, uint32_t* __restrict__ dd,
                            uint32_t* __restrict__ status) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t L = sc[0];
  if (h >= L) {
    if (h < Lcap) {
      dw[h] = 0u;
      if (dd) dd[h] = 0u;
    }
    return;
  }
  const int32_t r = rank[h];
  const int32_t t = ttwin[h];
  const int32_t u = tsrc[h], w = tnbr[h];
  if ((uint32_t)t >= (uint32_t)L || (uint32_t)u >= (uint32_t)n || (uint32_t)w >= (uint32_t)n) {
    flag(status, ST_BAD_INDEX);
    return;
  }
  const int32_t rt = rank[t];
  const bool down = r < rt;
  const bool head = (h == (int64_t)tptr[u]) && (ld(cc + u) == u);
  if ((uint32_t)r >= (uint32_t)L) {
    flag(status, ST_BAD_INDEX);
    return;
  }
  dw[r] = (uint32_t)down + (uint32_t)head;
  if (dd) dd[r] = down ? 1u : 0xffffffffu;  // +1 / -1: a prefix sum gives the depth (component tours are balanced)
  if (down) vrec[w] = make_int4(r, (rt - r + 1) >> 1, tslot[h], tslot[t]);
  if (head) {
    const int32_t tail = ttwin[clampi((int32_t)tptr[u + 1] - 1, 0, L - 1)];
    vrec[u] = make_int4(r, ((rank[tail] - r + 1) >> 1) + 1, -1, -1);
  }
}

// preorder of every vertex (-1 if isolated), and the vertex's subtree size
// and forest-edge slots stored by preorder for the bridge test
__global__ void k_preorder(const int4* __restrict__ vrec, const uint32_t* __restrict__ I, int32_t n, int32_t Lcap,
                           int32_t* __restrict__ pre, int4* __restrict__ byp) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int4 vr = vrec[v];
  const int32_t r = vr.x;
  if (r < 0 || r >= Lcap) {
    pre[v] = -1;
    return;
  }
  const int32_t ps = vr.z;
  const int32_t p = (int32_t)I[r] - (ps < 0 ? 2 : 1);
  pre[v] = p;
  if ((uint32_t)p < (uint32_t)n) byp[p] = make_int4(vr.y, ps, vr.w, 0);
}

// per vertex: min / max preorder over itself and its non-forest neighbours,
// stored at its own preorder position (the paper's segreduce). 16 lanes
// share a row: they read its slots side by side and combine with shuffles.
constexpr int kRowLanes = 16;

__global__ __launch_bounds__(kB) void k_minmax(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                              const uint32_t* __restrict__ tbits, const int32_t* __restrict__ pre,
                                              int32_t n, int32_t nnz, int32_t* __restrict__ amin,
                                              int32_t* __restrict__ amax) {
  const int sub = threadIdx.x & (kRowLanes - 1);
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kRowLanes);
  // rows stride over the grid: 16 lanes per row would exceed the 2^32
  // work-items of one dispatch beyond 2^28 rows
  for (int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes; u < n; u += groups) {
    const int32_t p = pre[u];
    if (p < 0 || p >= n) continue;    // isolated vertex (the whole row group skips together)
    const int32_t a = clampi(row_ptr[u], 0, nnz), b = clampi(row_ptr[u + 1], a, nnz);
    int32_t mn = p, mx = p;
    for (int64_t kk = (int64_t)a + sub; kk < b; kk += kRowLanes) {  // b may lie within one stride of 2^31
      const int32_t k = (int32_t)kk;
      if ((tbits[k >> 5] >> (k & 31)) & 1u) continue;
      const int32_t w = col[k];
      if ((uint32_t)w >= (uint32_t)n) continue;
      const int32_t pw = pre[w];
      mn = min(mn, pw);
      mx = max(mx, pw);
    }
#pragma unroll
    for (int o = kRowLanes / 2; o > 0; o >>= 1) {
      mn = min(mn, __shfl_xor(mn, o, kRowLanes));
      mx = max(mx, __shfl_xor(mx, o, kRowLanes));
    }
    if (sub == 0) {
      amin[p] = mn;
      amax[p] = mx;
    }
  }
}

// In-block RMQ by suffix-extreme bitmasks: for position o of a block of
// B = 2^LOG elements, bit j <= o of mmin[o] is set iff element j is smaller
// than every element after it up to o. The minimum of [l, o] is then the
// element at the lowest set bit at or above l: that element is a suffix
// minimum and no suffix minimum between l and it can be smaller. Likewise
// for maxima. Lane o of each B-lane group builds its two masks; lane B-1
// also yields the block's extremes (level 0 of the sparse table).
template <int LOG>
__global__ __launch_bounds__(kB) void k_rmq_blocks(const int32_t* __restrict__ amin, const int32_t* __restrict__ amax,
                                                  int32_t n, typename RmqMask<LOG>::type* __restrict__ mmin,
                                                  typename RmqMask<LOG>::type* __restrict__ mmax,
                                                  int32_t* __restrict__ bmin, int32_t* __restrict__ bmax) {
  using M = typename RmqMask<LOG>::type;
  constexpr int B = 1 << LOG;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < n;
  const int32_t vmin = ok ? amin[i] : INT32_MAX;
  const int32_t vmax = ok ? amax[i] : INT32_MIN;
  const int o = __lane_id() & (B - 1);
  M fmin = 0, fmax = 0;
  int32_t rmin = INT32_MAX, rmax = INT32_MIN;
#pragma unroll
  for (int j = B - 1; j >= 0; --j) {
    const int32_t x = __shfl(vmin, j, B);
    const int32_t y = __shfl(vmax, j, B);
    if (j <= o) {
      if (x < rmin) {
        fmin |= (M)1 << j;
        rmin = x;
      }
      if (y > rmax) {
        fmax |= (M)1 << j;
        rmax = y;
      }
    }
  }
  if (ok) {
    mmin[i] = fmin;
    mmax[i] = fmax;
  }
  if (o == B - 1 && (i >> LOG) < (((int64_t)n + B - 1) >> LOG)) {
    bmin[i >> LOG] = rmin;
    bmax[i >> LOG] = rmax;
  }
}

__global__ void k_sparse_level(const int32_t* __restrict__ pmn, const int32_t* __restrict__ pmx, int32_t nb,
                               int32_t half, int32_t* __restrict__ qmn, int32_t* __restrict__ qmx) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t o = b + half;
  qmn[b] = (o < nb) ? min(pmn[b], pmn[o]) : pmn[b];
  qmx[b] = (o < nb) ? max(pmx[b], pmx[o]) : pmx[b];
}

template <int LOG>
struct Rmq {
  const int32_t *amin, *amax;
  const typename RmqMask<LOG>::type *mmin, *mmax;
  const int32_t* stmin;  // sparse table levels concatenated: level k at k * nb
  const int32_t* stmax;
  int32_t nb;
};

// extremes of [l, r] inside one block, r's block
template <int LOG>
__device__ __forceinline__ void rmq_in_block(const Rmq<LOG>& q, int32_t l, int32_t r, int32_t* mn, int32_t* mx) {
  using M = typename RmqMask<LOG>::type;
  const int32_t base = r & ~((1 << LOG) - 1);
  const M keep = ~(M)0 << (l - base);
  *mn = q.amin[base + RmqMask<LOG>::ctz(q.mmin[r] & keep)];
  *mx = q.amax[base + RmqMask<LOG>::ctz(q.mmax[r] & keep)];
}

template <int LOG>
__device__ __forceinline__ void rmq(const Rmq<LOG>& q, int32_t l, int32_t r, int32_t* lo, int32_t* hi) {
  const int32_t bl = l >> LOG, br = r >> LOG;
  int32_t mn, mx;
  if (bl == br) {
    rmq_in_block(q, l, r, &mn, &mx);
  } else {
    int32_t a0, a1, b0, b1;
    rmq_in_block(q, l, (bl << LOG) + (1 << LOG) - 1, &a0, &a1);
    rmq_in_block(q, br << LOG, r, &b0, &b1);
    mn = min(a0, b0);
    mx = max(a1, b1);
    if (bl + 1 <= br - 1) {
      const int32_t a = bl + 1, b = br - 1;
      const int k = msb32((uint32_t)(b - a + 1));
      const int64_t base = (int64_t)k * q.nb;
      mn = min(mn, min(q.stmin[base + a], q.stmin[base + b - (1 << k) + 1]));
      mx = max(mx, max(q.stmax[base + a], q.stmax[base + b - (1 << k) + 1]));
    }
  }
  *lo = mn;
  *hi = mx;
}

// workgroups of the bridge test at most
constexpr int kTestBlocks = 2048;

// one lane per preorder position i < (number of non-isolated vertices, the
// last value of the preorder scan), in a grid-stride loop: the subtree
// interval starts at i, so neighbouring lanes read neighbouring RMQ entries
template <int LOG>
__global__ __launch_bounds__(kB) void k_bridge_test(const int4* __restrict__ byp, const uint32_t* __restrict__ I,
                                                   int32_t Lcap, int32_t n, Rmq<LOG> q, uint32_t* __restrict__ mask,
                                                   int64_t* __restrict__ count) {
  const int32_t npre = min((int32_t)I[Lcap - 1], n);
  uint32_t found = 0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < npre; i += (int64_t)gridDim.x * kB) {
    const int4 b = byp[i];
    const int32_t l = (int32_t)i, r = l + b.x - 1;
    if (b.y >= 0 && r >= l && r < npre) {
      int32_t lo, hi;
      rmq(q, l, r, &lo, &hi);
      if (lo == l && hi == r) {
        ++found;
        atomicOr(mask + (b.y >> 5), 1u << (b.y & 31));
        if (b.z >= 0) atomicOr(mask + (b.z >> 5), 1u << (b.z & 31));
      }
    }
  }
  // one count update per workgroup: every wavefront adding its own to the
  // one counter serialised some 65K same-address atomics at 2^22 vertices
  __shared__ uint32_t wsum[kB / 64];
  uint32_t t = found;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
  if (__lane_id() == 0) wsum[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kB / 64; ++w) tot += wsum[w];
    if (tot) atomicAdd((unsigned long long*)count, (unsigned long long)tot);
  }
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

// hybrid: parent, level and the two slots of the parent edge of every vertex
// from the direction records and the depth prefix sums
__global__ void k_hybrid_nodes(const int4* __restrict__ vrec, const uint32_t* __restrict__ depth_at,
                               const int32_t* __restrict__ col, int32_t n, int32_t nnz, int32_t Lcap,
                               int32_t* __restrict__ par, int32_t* __restrict__ lvl, int32_t* __restrict__ pslot,
                               int32_t* __restrict__ uslot, uint32_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int4 r = vrec[v];
  int32_t p = -1, l = -1, ps = -1, us = -1;
  if (r.x >= 0 && r.x < Lcap) {
    if (r.z < 0) {
      p = -2;  // a component root
      l = 0;
    } else if ((uint32_t)r.w < (uint32_t)nnz && (uint32_t)r.z < (uint32_t)nnz) {
      p = col[r.w];
      l = (int32_t)depth_at[r.x];
      ps = r.z;
      us = r.w;
    } else {
      flag(status, ST_BAD_INDEX);
    }
  }
  par[v] = p;
  lvl[v] = l;
  pslot[v] = ps;
  uslot[v] = us;
}

}  // namespace

// Connectivity labels and a spanning forest (both slots of every forest
// edge set in tbits): sampled hooking rounds, then the rows outside the
// largest sampled component. cc[v] == v marks one root per component.
int spanning_forest(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, int32_t* cc,
                    uint32_t* tbits, int32_t* big, hipStream_t s) {
  const int32_t words = (int32_t)(((int64_t)nnz + 31) >> 5);
  const int gn = ceil_div(n, kB);
  const int grows = ceil_div(n, kRowsPerBlock);
  {
    ET_PROF(c, s, "k_check_csr");
    hipLaunchKernelGGL(k_check_csr, dim3(gn), dim3(kB), 0, s, row_ptr, n, nnz, c->d_status);
  }
  hipLaunchKernelGGL(k_iota, dim3(gn), dim3(kB), 0, s, cc, n);
  hipLaunchKernelGGL(k_fill_i32, dim3(std::min(ceil_div(words, kB), 4096)), dim3(kB), 0, s,
                     reinterpret_cast<int32_t*>(tbits), (int64_t)words, 0);
  for (int j = 0; j < kSample; ++j) {
    {
      ET_PROF(c, s, "k_hook_sample");
      hipLaunchKernelGGL(k_hook_sample, dim3(gn), dim3(kB), 0, s, row_ptr, col, n, nnz, cc, tbits, c->d_status, j);
    }
    {
      ET_PROF(c, s, "k_cc_compress");
      hipLaunchKernelGGL(k_cc_compress, dim3(gn), dim3(kB), 0, s, cc, n);
    }
  }
  {
    ET_PROF(c, s, "k_big_component");
    hipLaunchKernelGGL(k_big_component, dim3(1), dim3(kBigSample), 0, s, cc, n, big);
  }
  {
    ET_PROF(c, s, "k_hook_rest");
    hipLaunchKernelGGL(k_hook_rest, dim3(grows), dim3(kB), 0, s, row_ptr, col, n, nnz, cc, big, tbits,
                       c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

// Scratch of the Tarjan-Vishkin path of bridges_run: every array below, the
// ranking's buffers (same scope) and the partials of its three scans.
size_t bridges_scratch_bytes(const Ctx* c, int32_t n, int32_t nnz) {
  if (n <= 1 || nnz == 0) return 0;
  const size_t N = (size_t)n, L = 2 * (size_t)(n - 1), words = ((size_t)nnz + 31) >> 5;
  const int rlog = c ? c->qs.rmq_log : QueryShape{}.rmq_log;
  const size_t nb = (N + (1u << rlog) - 1) >> rlog;
  size_t levels = 1;
  while (((size_t)1 << levels) <= nb) ++levels;
  size_t b = scratch_block<int32_t>(N) + scratch_block<uint32_t>(words) + 2 * scratch_block<uint32_t>(N + 1) +
             7 * scratch_block<int32_t>(L) + 3 * scratch_block<uint32_t>(N) + 2 * scratch_block<int4>(N) +
             3 * scratch_block<int32_t>(N) + 2 * scratch_block<uint32_t>(N << (rlog - 5)) +
             2 * scratch_block<int32_t>(levels * nb) + scratch_block<int32_t>(8);
  b += list_rank_plan_bytes(c, (int32_t)L, 1, 0);
  return b + scan_scratch_bytes((int64_t)N + 1) + scan_scratch_bytes((int64_t)N) + scan_scratch_bytes((int64_t)L);
}

int bridges_run(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, uint32_t* mask,
                hipStream_t s, int algo) {
  if (algo == kAlgoCK) return bridges_ck_bfs(c, row_ptr, col, n, nnz, mask, s);
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, c->d_bcount);
  const int32_t words = (int32_t)(((int64_t)nnz + 31) >> 5);
  if (words > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3(std::min(ceil_div(words, kB), 4096)), dim3(kB), 0, s,
                       reinterpret_cast<int32_t*>(mask), (int64_t)words, 0);
  if (n <= 1 || nnz == 0) return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;

  const int32_t Lcap = 2 * (n - 1);  // forest half-edges are at most 2(n-1)
  Scratch sc(c, s);
  int32_t* cc = sc.get<int32_t>(n);
  uint32_t* tbits = sc.get<uint32_t>(words);
  uint32_t* tdeg = sc.get<uint32_t>((size_t)n + 1);
  uint32_t* tptr = sc.get<uint32_t>((size_t)n + 1);
  int32_t* tslot = sc.get<int32_t>(Lcap);
  int32_t* tnbr = sc.get<int32_t>(Lcap);
  int32_t* tsrc = sc.get<int32_t>(Lcap);
  int32_t* ttwin = sc.get<int32_t>(Lcap);
  int32_t* succ = sc.get<int32_t>(Lcap);
  int32_t* rank = sc.get<int32_t>(Lcap);
  uint32_t* dw = sc.get<uint32_t>(Lcap);
  uint32_t* rflag = sc.get<uint32_t>(n);
  uint32_t* rpos = sc.get<uint32_t>(n);
  int32_t* roots = sc.get<int32_t>(n);
  int4* vrec = sc.get<int4>(n);
  int32_t* pre = sc.get<int32_t>(n);
  int4* byp = sc.get<int4>(n);
  int32_t* amin = sc.get<int32_t>(n);
  int32_t* amax = sc.get<int32_t>(n);
  const int rlog = c->qs.rmq_log;                        // range-minimum blocks of 2^rlog vertices
  uint32_t* mmin = sc.get<uint32_t>((size_t)n << (rlog - 5));
  uint32_t* mmax = sc.get<uint32_t>((size_t)n << (rlog - 5));
  const int32_t nb = (int32_t)(((int64_t)n + (1 << rlog) - 1) >> rlog);
  int levels = 1;
  while ((1 << levels) <= nb) ++levels;
  int32_t* stmin = sc.get<int32_t>((size_t)levels * nb);
  int32_t* stmax = sc.get<int32_t>((size_t)levels * nb);
  int32_t* scal = sc.get<int32_t>(8);
  if (sc.failed) return ET_ENOMEM;

  const int gn = ceil_div(n, kB);
  const int gl = ceil_div(Lcap, kB);
  // 1. spanning forest
  ET_PROF(c, s, "phase:bridges");
  int rc = spanning_forest(c, row_ptr, col, n, nnz, cc, tbits, scal + 4, s);
  if (rc) return rc;
  // 2. forest CSR, twins, successors, component chaining
  {
    ET_PROF(c, s, "k_tree_deg");
    hipLaunchKernelGGL(k_tree_deg, dim3(gn), dim3(kB), 0, s, row_ptr, tbits, n, nnz, tdeg);
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, s, reinterpret_cast<int32_t*>(tdeg + n), (int64_t)1, 0);
  rc = scan_u32(c, tdeg, tptr, (int64_t)n + 1, ScanOp::Add, true, s);
  if (rc) return rc;
  {
    ET_PROF(c, s, "k_tree_fill");
    hipLaunchKernelGGL(k_tree_fill, dim3(gn), dim3(kB), 0, s, row_ptr, col, tbits, tptr, n, nnz, Lcap, tslot, tnbr,
                       tsrc);
  }
  {
    ET_PROF(c, s, "k_root_flags");
    hipLaunchKernelGGL(k_root_flags, dim3(gn), dim3(kB), 0, s, cc, tdeg, n, rflag);
  }
  rc = scan_u32(c, rflag, rpos, n, ScanOp::Add, true, s);
  if (rc) return rc;
  {
    ET_PROF(c, s, "k_root_list");
    hipLaunchKernelGGL(k_root_list, dim3(gn), dim3(kB), 0, s, rflag, rpos, n, roots);
  }
  hipLaunchKernelGGL(k_set_len, dim3(1), dim3(1), 0, s, tptr, n, scal);
  {
    ET_PROF(c, s, "k_succ_csr");
    hipLaunchKernelGGL(k_succ_csr, dim3(gl), dim3(kB), 0, s, tnbr, tsrc, tptr, n, Lcap, scal, ttwin, succ,
                       c->d_status);
  }
  {
    ET_PROF(c, s, "k_link_roots");
    hipLaunchKernelGGL(k_link_roots, dim3(gn), dim3(kB), 0, s, roots, rpos, rflag, tptr, ttwin, n, succ, scal);
  }
  // 3. one list ranking, directions, preorder
  LRResult lr;
  rc = list_rank_core(c, sc, succ, Lcap, scal + 1, 1, false, scal + 2, &lr, s, true);
  if (rc) return rc;
  {
    ET_PROF(c, s, "k_rank_of");
    hipLaunchKernelGGL(k_rank_of, dim3(gl), dim3(kB), 0, s, lr.packed, lr.off, lr.nsub, Lcap, scal, rank,
                       c->d_status);
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(std::min(4 * (int64_t)gn, (int64_t)8192)), dim3(kB), 0, s,
                     reinterpret_cast<int32_t*>(vrec), 4 * (int64_t)n, -1);
  {
    ET_PROF(c, s, "k_direction");
    hipLaunchKernelGGL(k_direction, dim3(gl), dim3(kB), 0, s, rank, ttwin, tsrc, tnbr, tslot, tptr, cc, n, Lcap, scal,
                       dw, vrec, algo == kAlgoHybrid ? reinterpret_cast<uint32_t*>(succ) : nullptr, c->d_status);
  }
  if (algo == kAlgoHybrid) {
    // the hybrid of Section 4.1: this rooted forest, levels from the tour,
    // then Chaitanya-Kothapalli marking instead of low / high
    uint32_t* depth_at = reinterpret_cast<uint32_t*>(succ);  // the successors are dead after the ranking
    rc = scan_u32(c, depth_at, depth_at, Lcap, ScanOp::Add, false, s);
    if (rc) return rc;
    int32_t* par = pre;                                   // per-vertex arrays of the test phase are unused
    int32_t* lvl = amin;
    int32_t* pslot = amax;
    int32_t* uslot = reinterpret_cast<int32_t*>(mmin);
    {
      ET_PROF(c, s, "k_hybrid_nodes");
      hipLaunchKernelGGL(k_hybrid_nodes, dim3(gn), dim3(kB), 0, s, vrec, depth_at, col, n, nnz, Lcap, par, lvl,
                         pslot, uslot, c->d_status);
    }
    return ck_mark(c, row_ptr, col, n, nnz, tbits, par, lvl, pslot, uslot, mask, s);
  }
  rc = scan_u32(c, dw, dw, Lcap, ScanOp::Add, false, s);
  if (rc) return rc;
  {
    ET_PROF(c, s, "k_preorder");
    hipLaunchKernelGGL(k_preorder, dim3(gn), dim3(kB), 0, s, vrec, dw, n, Lcap, pre, byp);
  }
  // 4. non-forest extremes by preorder
  {
    ET_PROF(c, s, "k_minmax");
    hipLaunchKernelGGL(k_minmax, dim3(std::min(ceil_div((int64_t)n * kRowLanes, kB), kMaxGrid)), dim3(kB), 0, s,
                       row_ptr, col, tbits, pre, n, nnz, amin, amax);
  }
  // 5. range extremes
  {
    ET_PROF(c, s, "k_rmq_blocks");
    if (rlog == 6)
      hipLaunchKernelGGL(k_rmq_blocks<6>, dim3(gn), dim3(kB), 0, s, amin, amax, n, reinterpret_cast<uint64_t*>(mmin),
                         reinterpret_cast<uint64_t*>(mmax), stmin, stmax);
    else
      hipLaunchKernelGGL(k_rmq_blocks<5>, dim3(gn), dim3(kB), 0, s, amin, amax, n, mmin, mmax, stmin, stmax);
  }
  for (int k = 1; k < levels; ++k) {
    ET_PROF(c, s, "k_sparse_level");
    hipLaunchKernelGGL(k_sparse_level, dim3(ceil_div(nb, kB)), dim3(kB), 0, s, stmin + (size_t)(k - 1) * nb,
                       stmax + (size_t)(k - 1) * nb, nb, 1 << (k - 1), stmin + (size_t)k * nb,
                       stmax + (size_t)k * nb);
  }
  // 6. test
  {
    ET_PROF(c, s, "k_bridge_test");
    if (rlog == 6) {
      Rmq<6> q{amin, amax, reinterpret_cast<const uint64_t*>(mmin), reinterpret_cast<const uint64_t*>(mmax), stmin,
               stmax, nb};
      hipLaunchKernelGGL(k_bridge_test<6>, dim3(std::min(gn, kTestBlocks)), dim3(kB), 0, s, byp, dw, Lcap, n, q, mask,
                         c->d_bcount);
    } else {
      Rmq<5> q{amin, amax, mmin, mmax, stmin, stmax, nb};
      hipLaunchKernelGGL(k_bridge_test<5>, dim3(std::min(gn, kTestBlocks)), dim3(kB), 0, s, byp, dw, Lcap, n, q, mask,
                         c->d_bcount);
    }
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
