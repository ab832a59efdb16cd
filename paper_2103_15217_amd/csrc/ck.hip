// Bridges by Chaitanya-Kothapalli marking (Section 4.1, "Chaitanya-Kothapalli
// (CK) Algorithm" and "The Hybrid Algorithm"), the paper's comparison
// method for Tarjan-Vishkin.
//
// Phase 1 roots a spanning forest: here a breadth-first search (CK), or in
// bridges.hip the connectivity forest rooted by the Euler tour (hybrid).
// Phase 2 (shared): for every non-tree edge {u, w}, one lane walks from u
// and w up to their lowest common ancestor, the deeper end first, marking
// the tree edge above every node it leaves. A tree edge that no walk marks
// is a bridge. Work is the total length of those paths, so it grows with
// the tree's depth, which is why a BFS tree is the usual choice.
//
// BFS: level-synchronous and top-down from one root per component (the
// roots of the connectivity labels), 16 lanes per frontier vertex; a
// neighbour is claimed by compare-and-swap on its parent entry, which also
// records the claiming CSR slot as its tree edge. A large frontier gets one
// grid launch per level (issued 16 at a time between reads of the frontier
// size); while the frontier is small (long chains, the tail of a search) a
// single workgroup runs level after level in one launch, synchronising at a
// workgroup barrier instead of a kernel boundary, so sparse high-diameter
// stretches do not cost a launch per level.
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kB = 256;
constexpr int kLanes = 16;          // lanes per frontier vertex / per row
constexpr int kLevelsPerCheck = 16;
constexpr int kSmallFrontier = 128;  // frontier size handled by the one-workgroup kernel
constexpr int kSmallThreads = 1024;

__global__ void k_fill32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// the roots of the connectivity labels start the search at level 0
__global__ void k_bfs_seed(const int32_t* __restrict__ cc, int32_t n, int32_t* __restrict__ par,
                           int32_t* __restrict__ lvl, int32_t* __restrict__ queue, int32_t* __restrict__ cnt) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (cc[v] == (int32_t)v) {
    par[v] = -2;
    lvl[v] = 0;
    queue[atomicAdd(cnt, 1)] = (int32_t)v;
  }
}

// cnt[0] = current frontier size, cnt[1] = next frontier size, cnt[2] = the
// current level; the frontier of level l is in q0 for even l, q1 for odd l.
__device__ __forceinline__ int32_t ldcnt(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// one frontier vertex per kLanes lanes: claim its unvisited neighbours
__device__ __forceinline__ void bfs_expand(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                           int32_t n, int32_t nnz, int32_t u, int sub, int32_t level, int32_t* next,
                                           int32_t* cnt, int32_t* par, int32_t* lvl, int32_t* pslot) {
  const int32_t a = min(max(row_ptr[u], 0), nnz), b = min(max(row_ptr[u + 1], a), nnz);
  for (int64_t kk = (int64_t)a + sub; kk < b; kk += kLanes) {
    const int32_t k = (int32_t)kk;
    const int32_t w = col[k];
    if ((uint32_t)w >= (uint32_t)n || w == u) continue;
    if (ldcnt(par + w) != -1) continue;
    if (atomicCAS(par + w, -1, u) == -1) {
      lvl[w] = level + 1;
      pslot[w] = k;
      next[atomicAdd(cnt + 1, 1)] = w;
    }
  }
}

__global__ __launch_bounds__(kB) void k_bfs_level(const int32_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col, int32_t n, int32_t nnz, int32_t* q0,
                                                 int32_t* q1, int32_t* cnt, int32_t* par, int32_t* __restrict__ lvl,
                                                 int32_t* __restrict__ pslot) {
  const int32_t fsize = min(cnt[0], n);
  const int32_t level = cnt[2];
  const int32_t* frontier = (level & 1) ? q1 : q0;
  int32_t* next = (level & 1) ? q0 : q1;
  const int sub = threadIdx.x & (kLanes - 1);
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kLanes);
  for (int64_t f = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes; f < fsize; f += groups)
    bfs_expand(row_ptr, col, n, nnz, frontier[f], sub, level, next, cnt, par, lvl, pslot);
}

__global__ void k_bfs_advance(int32_t* __restrict__ cnt) {
  cnt[0] = cnt[1];
  cnt[1] = 0;
  cnt[2] += 1;
}

// one workgroup, many levels: runs while the frontier is non-empty and at
// most kSmallFrontier vertices; every level ends at a workgroup barrier.
// Thread 0 reads the frontier size and level and broadcasts them through
// LDS, so every thread takes the same exit at the same barrier. Stores are
// fenced at device scope before each barrier and read back with device-scope
// loads. Each pass advances the level and claims every vertex at most once,
// so the loop ends after at most n passes.
__global__ __launch_bounds__(kSmallThreads) void k_bfs_small(const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col, int32_t n, int32_t nnz,
                                                            int32_t* q0, int32_t* q1, int32_t* cnt, int32_t* par,
                                                            int32_t* __restrict__ lvl, int32_t* __restrict__ pslot) {
  __shared__ int32_t s_fsize, s_level;
  const int sub = threadIdx.x & (kLanes - 1);
  const int group = threadIdx.x / kLanes;
  constexpr int kGroups = kSmallThreads / kLanes;
  for (int32_t pass = 0; pass <= n; ++pass) {
    if (threadIdx.x == 0) {
      s_fsize = ldcnt(cnt);
      s_level = ldcnt(cnt + 2);
    }
    __syncthreads();
    const int32_t fsize = s_fsize, level = s_level;
    if (fsize == 0 || fsize > kSmallFrontier) break;  // the same value in every thread
    const int32_t* frontier = (level & 1) ? q1 : q0;
    int32_t* next = (level & 1) ? q0 : q1;
    for (int32_t f = group; f < fsize; f += kGroups)
      bfs_expand(row_ptr, col, n, nnz, __hip_atomic_load(frontier + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                 sub, level, next, cnt, par, lvl, pslot);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_store(cnt, ldcnt(cnt + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(cnt + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(cnt + 2, level + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
    }
    __syncthreads();
  }
}

// both slots of every tree edge in the bitmask: the claiming slot in the
// parent's row, and the first (v, parent) slot of v's own row
__global__ void k_bfs_slots(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int32_t n,
                            int32_t nnz, const int32_t* __restrict__ par, const int32_t* __restrict__ pslot,
                            int32_t* __restrict__ uslot, uint32_t* __restrict__ tbits, uint32_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t p = par[v];
  if (p < 0) {
    uslot[v] = -1;
    if (p == -1) flag(status, ST_UNREACHED);  // no search reached v: the labels were not components
    return;
  }
  const int32_t k = pslot[v];
  atomicOr(tbits + (k >> 5), 1u << (k & 31));
  const int32_t a = min(max(row_ptr[v], 0), nnz), b = min(max(row_ptr[v + 1], a), nnz);
  int32_t lo = a, hi = b;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (col[mid] < p) lo = mid + 1;
    else hi = mid;
  }
  if (lo < b && col[lo] == p) {
    uslot[v] = lo;
    atomicOr(tbits + (lo >> 5), 1u << (lo & 31));
  } else {
    uslot[v] = -1;
    flag(status, ST_BAD_CSR);
  }
}

// one lane per non-tree slot (u, w) with u < w: walk both ends up to their
// LCA, marking the tree edge above every node left behind
__global__ __launch_bounds__(kB) void k_ck_mark(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                               int32_t n, int32_t nnz, const uint32_t* __restrict__ tbits,
                                               const int32_t* __restrict__ par, const int32_t* __restrict__ lvl,
                                               uint8_t* __restrict__ mark, uint32_t* __restrict__ status) {
  const int sub = threadIdx.x & (kLanes - 1);
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kLanes);
  bool bad = false;
  for (int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kLanes; u < n; u += groups) {
  const int32_t a = min(max(row_ptr[u], 0), nnz), b = min(max(row_ptr[u + 1], a), nnz);
  for (int64_t kk = (int64_t)a + sub; kk < b; kk += kLanes) {
    const int32_t k = (int32_t)kk;
    const int32_t w = col[k];
    if ((uint32_t)w >= (uint32_t)n || w <= u) continue;            // each undirected edge once; no self-loops
    if ((tbits[k >> 5] >> (k & 31)) & 1u) continue;                 // a tree edge
    int32_t x = (int32_t)u, y = w;
    int32_t lx = lvl[x], ly = lvl[y];
    if (lx < 0 || ly < 0) {
      bad = true;
      continue;
    }
    for (; lx > ly; --lx) {
      mark[x] = 1;
      x = par[x];
      if (x < 0) break;
    }
    for (; ly > lx && x >= 0; --ly) {
      mark[y] = 1;
      y = par[y];
      if (y < 0) break;
    }
    for (; x >= 0 && y >= 0 && x != y; --lx) {
      if (lx <= 0) {  // two roots: the ends lie in different trees
        x = -1;
        break;
      }
      mark[x] = 1;
      mark[y] = 1;
      x = par[x];
      y = par[y];
    }
    if (x < 0 || y < 0) bad = true;
  }
  }
  if (bad) flag(status, ST_BAD_INDEX);
}

// a tree edge nobody marked is a bridge: both of its slots get their bit
__global__ __launch_bounds__(kB) void k_ck_out(const int32_t* __restrict__ par, const int32_t* __restrict__ pslot,
                         const int32_t* __restrict__ uslot, const uint8_t* __restrict__ mark, int32_t n,
                         uint32_t* __restrict__ mask, int64_t* __restrict__ count) {
  uint32_t found = 0;
  for (int64_t v = (int64_t)blockIdx.x * kB + threadIdx.x; v < n; v += (int64_t)gridDim.x * kB) {
    if (par[v] >= 0 && !mark[v]) {
      ++found;
      const int32_t k = pslot[v], t = uslot[v];
      if (k >= 0) atomicOr(mask + (k >> 5), 1u << (k & 31));
      if (t >= 0) atomicOr(mask + (t >> 5), 1u << (t & 31));
    }
  }
  // one count update per workgroup (not one per wavefront on the one counter)
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

}  // namespace

int ck_mark(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, const uint32_t* tbits,
            const int32_t* par, const int32_t* lvl, const int32_t* pslot, const int32_t* uslot, uint32_t* mask,
            hipStream_t s) {
  Scratch sc(c, s);
  uint8_t* mark = sc.get<uint8_t>((size_t)n);
  if (sc.failed) return ET_ENOMEM;
  hipLaunchKernelGGL(k_fill32, dim3(std::min(ceil_div(n, 4 * kB), 4096)), dim3(kB), 0, s,
                     reinterpret_cast<int32_t*>(mark), ((int64_t)n + 3) / 4, 0);
  {
    ET_PROF(c, s, "k_ck_mark");
    hipLaunchKernelGGL(k_ck_mark, dim3(std::min(ceil_div((int64_t)n * kLanes, kB), 1 << 20)), dim3(kB), 0, s, row_ptr,
                       col, n, nnz, tbits, par, lvl, mark, c->d_status);
  }
  {
    ET_PROF(c, s, "k_ck_out");
    hipLaunchKernelGGL(k_ck_out, dim3(std::min(ceil_div(n, kB), 2048)), dim3(kB), 0, s, par, pslot, uslot, mark, n, mask,
                       c->d_bcount);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int ck_bfs_forest(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, const int32_t* cc,
                  int32_t* par, int32_t* lvl, int32_t* pslot, int32_t* uslot, uint32_t* tbits, hipStream_t s) {
  Scratch sc(c, s);
  int32_t* q0 = sc.get<int32_t>((size_t)n);
  int32_t* q1 = sc.get<int32_t>((size_t)n);
  int32_t* cnt = sc.get<int32_t>(4);
  int32_t* h_cnt = nullptr;
  if (sc.failed) return ET_ENOMEM;
  if (hipHostMalloc(reinterpret_cast<void**>(&h_cnt), sizeof(int32_t)) != hipSuccess) return ET_ENOMEM;
  const int gn = ceil_div(n, kB);
  hipLaunchKernelGGL(k_fill32, dim3(std::min(gn, 4096)), dim3(kB), 0, s, par, (int64_t)n, -1);
  hipLaunchKernelGGL(k_fill32, dim3(std::min(gn, 4096)), dim3(kB), 0, s, lvl, (int64_t)n, -1);
  hipLaunchKernelGGL(k_fill32, dim3(1), dim3(kB), 0, s, cnt, (int64_t)4, 0);  // sizes and level 0
  hipLaunchKernelGGL(k_bfs_seed, dim3(gn), dim3(kB), 0, s, cc, n, par, lvl, q0, cnt);
  // a frontier of f vertices needs f * kLanes lanes; the grid strides over larger ones
  const int grid = std::max(1, std::min(ceil_div((int64_t)n * kLanes, kB), 8192));
  int rc = ET_OK;
  {
    ET_PROF(c, s, "k_bfs_level");
    // every round either ends the search, runs small levels until the frontier
    // grows or empties, or runs kLevelsPerCheck grid levels: at most n rounds
    for (int32_t round = 0; round <= n; ++round) {
      if (hipMemcpyAsync(h_cnt, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        rc = ET_EHIP;
        break;
      }
      const int32_t f = *h_cnt;
      if (f == 0) break;
      if (f <= kSmallFrontier) {
        hipLaunchKernelGGL(k_bfs_small, dim3(1), dim3(kSmallThreads), 0, s, row_ptr, col, n, nnz, q0, q1, cnt, par,
                           lvl, pslot);
      } else {
        // size the grid for a frontier up to 8x the one just read (larger ones stride)
        const int g = std::max(64, std::min(ceil_div((int64_t)f * 8 * kLanes, kB), grid));
        for (int j = 0; j < kLevelsPerCheck; ++j) {
          hipLaunchKernelGGL(k_bfs_level, dim3(g), dim3(kB), 0, s, row_ptr, col, n, nnz, q0, q1, cnt, par, lvl,
                             pslot);
          hipLaunchKernelGGL(k_bfs_advance, dim3(1), dim3(1), 0, s, cnt);
        }
      }
    }
  }
  (void)hipHostFree(h_cnt);
  if (rc) return rc;
  {
    ET_PROF(c, s, "k_bfs_slots");
    hipLaunchKernelGGL(k_bfs_slots, dim3(gn), dim3(kB), 0, s, row_ptr, col, n, nnz, par, pslot, uslot, tbits,
                       c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int bridges_ck_bfs(Ctx* c, const int32_t* row_ptr, const int32_t* col, int32_t n, int32_t nnz, uint32_t* mask,
                   hipStream_t s) {
  const int32_t words = (int32_t)(((int64_t)nnz + 31) >> 5);
  hipLaunchKernelGGL(k_fill32, dim3(1), dim3(1), 0, s, reinterpret_cast<int32_t*>(c->d_bcount), (int64_t)2, 0);
  if (words > 0)
    hipLaunchKernelGGL(k_fill32, dim3(std::min(ceil_div(words, kB), 4096)), dim3(kB), 0, s,
                       reinterpret_cast<int32_t*>(mask), (int64_t)words, 0);
  if (n <= 1 || nnz == 0) return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
  Scratch sc(c, s);
  int32_t* cc = sc.get<int32_t>((size_t)n);
  uint32_t* tbits = sc.get<uint32_t>((size_t)words);
  int32_t* big = sc.get<int32_t>(4);
  int32_t* par = sc.get<int32_t>((size_t)n);
  int32_t* lvl = sc.get<int32_t>((size_t)n);
  int32_t* pslot = sc.get<int32_t>((size_t)n);
  int32_t* uslot = sc.get<int32_t>((size_t)n);
  if (sc.failed) return ET_ENOMEM;
  ET_PROF(c, s, "phase:bridges_ck");
  // connectivity labels only choose one search root per component
  int rc = spanning_forest(c, row_ptr, col, n, nnz, cc, tbits, big, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_fill32, dim3(std::min(ceil_div(words, kB), 4096)), dim3(kB), 0, s,
                     reinterpret_cast<int32_t*>(tbits), (int64_t)words, 0);
  rc = ck_bfs_forest(c, row_ptr, col, n, nnz, cc, par, lvl, pslot, uslot, tbits, s);
  if (rc) return rc;
  return ck_mark(c, row_ptr, col, n, nnz, tbits, par, lvl, pslot, uslot, mask, s);
}

}  // namespace et
