// LCA by range-minimum queries over the Euler tour: the alternative query
// engine to Inlabel that the paper's LCA section measures against (the
// RMQ approach of Bender and Farach-Colton, Section 3).
//
// The tour, read as the sequence of nodes it visits, is root, then after
// every half-edge the node it leads to: for the down half-edge 2c that is c
// at depth(c), for the up half-edge 2c+1 it is parent(c) at depth(c) - 1.
// E[r] holds (depth << 32 | node) for the node after the half-edge of rank
// r. A non-root node x is first visited at E[rank(2x)], so for two distinct
// non-root nodes the LCA is the node of the smallest key in E between their
// first visits; the root is the LCA of any pair that contains it.
//
// The minimum uses blocks of 2^LOG positions (32 or 64, a tunable of the
// context): per position a mask of the block positions that are smaller
// than everything after them up to this one (the minimum of [l, o] inside a
// block is then at the lowest set bit at or above l), and a sparse table
// over the block minima. A query reads two ranks, up to four keys, two
// masks and two table entries.
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kB = 256;

__device__ __forceinline__ uint64_t ekey(int32_t depth, int32_t node) {
  return ((uint64_t)(uint32_t)depth << 32) | (uint32_t)node;
}

__global__ void k_rmq_euler(const int32_t* __restrict__ rank, const int4* __restrict__ rec,
                            const int32_t* __restrict__ parent, int32_t n, const int32_t* __restrict__ sc,
                            int32_t L, uint64_t* __restrict__ E, uint32_t* __restrict__ status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || c == sc[0]) return;
  const int2 r = reinterpret_cast<const int2*>(rank)[c];
  const int32_t d = rec[c].z;
  const int32_t p = parent[c];
  if ((uint32_t)r.x >= (uint32_t)L || (uint32_t)r.y >= (uint32_t)L || (uint32_t)p >= (uint32_t)n) {
    flag(status, ST_BAD_INDEX);  // the parent array is not the one the tree was built from
    return;
  }
  E[r.x] = ekey(d, (int32_t)c);
  E[r.y] = ekey(d - 1, p);
}

template <int LOG>
__global__ __launch_bounds__(kB) void k_rmq_masks(const uint64_t* __restrict__ E, int32_t L,
                                                 typename RmqMask<LOG>::type* __restrict__ mask,
                                                 uint64_t* __restrict__ bmin) {
  using M = typename RmqMask<LOG>::type;
  constexpr int B = 1 << LOG;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = i < L;
  const uint64_t v = ok ? E[i] : ~0ull;
  const int o = __lane_id() & (B - 1);
  M f = 0;
  uint64_t run = ~0ull;
#pragma unroll
  for (int j = B - 1; j >= 0; --j) {
    const uint64_t x = __shfl(v, j, B);
    if (j <= o && x < run) {
      f |= (M)1 << j;
      run = x;
    }
  }
  if (ok) mask[i] = f;
  if (o == B - 1 && (i >> LOG) < (((int64_t)L + B - 1) >> LOG)) bmin[i >> LOG] = run;
}

__global__ void k_rmq_level(const uint64_t* __restrict__ prev, int32_t nb, int32_t half,
                            uint64_t* __restrict__ next) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t o = b + half;
  next[b] = (o < nb) ? min(prev[b], prev[o]) : prev[b];
}

template <int LOG>
struct RmqTables {
  const uint64_t* E;
  const typename RmqMask<LOG>::type* mask;
  const uint64_t* st;  // level k at k * nb
  int32_t nb;
};

template <int LOG>
__device__ __forceinline__ uint64_t in_block(const RmqTables<LOG>& t, int32_t l, int32_t r) {
  using M = typename RmqMask<LOG>::type;
  const int32_t base = r & ~((1 << LOG) - 1);
  return t.E[base + RmqMask<LOG>::ctz(t.mask[r] & (~(M)0 << (l - base)))];
}

template <int LOG>
__device__ __forceinline__ uint64_t range_min(const RmqTables<LOG>& t, int32_t l, int32_t r) {
  const int32_t bl = l >> LOG, br = r >> LOG;
  if (bl == br) return in_block(t, l, r);
  uint64_t m = min(in_block(t, l, (bl << LOG) + (1 << LOG) - 1), in_block(t, br << LOG, r));
  if (bl + 1 <= br - 1) {
    const int32_t a = bl + 1, b = br - 1;
    const int k = msb32((uint32_t)(b - a + 1));
    const int64_t base = (int64_t)k * t.nb;
    m = min(m, min(t.st[base + a], t.st[base + b - (1 << k) + 1]));
  }
  return m;
}

template <int LOG>
__global__ __launch_bounds__(kQueryBlockMax) void k_lca_rmq(RmqTables<LOG> t, const int32_t* __restrict__ rank,
                                                           int32_t n, const int32_t* __restrict__ sc, int32_t L,
                                                           const int32_t* __restrict__ qx,
                                                           const int32_t* __restrict__ qy, int64_t q,
                                                           int32_t* __restrict__ out, uint32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  const int32_t x = qx[i], y = qy[i];
  if ((uint32_t)x >= (uint32_t)n || (uint32_t)y >= (uint32_t)n) {
    flag(status, ST_BAD_QUERY);
    out[i] = -1;
    return;
  }
  const int32_t root = sc[0];
  if (x == y || x == root || y == root) {
    out[i] = (x == y) ? x : root;
    return;
  }
  int32_t a = rank[2 * (int64_t)x], b = rank[2 * (int64_t)y];
  if ((uint32_t)a >= (uint32_t)L || (uint32_t)b >= (uint32_t)L) {
    flag(status, ST_BAD_INDEX);
    out[i] = -1;
    return;
  }
  if (a > b) {
    const int32_t tmp = a;
    a = b;
    b = tmp;
  }
  out[i] = (int32_t)(uint32_t)range_min(t, a, b);
}

}  // namespace

int tree_rmq_build(Ctx* c, et_tree* t, const int32_t* parent, hipStream_t s) {
  const int32_t n = t->n;
  const int32_t L = 2 * (n - 1);
  if (L == 0) return ET_OK;
  const int lg = c->qs.rmq_log;
  const int32_t nb = (int32_t)(((int64_t)L + (1 << lg) - 1) >> lg);
  int levels = 1;
  while ((1 << levels) <= nb) ++levels;
  t->d_rmq_e = static_cast<uint64_t*>(pool_get(c, (size_t)L * sizeof(uint64_t), s));
  t->d_rmq_mask = pool_get(c, ((size_t)L << (lg - 5)) * sizeof(uint32_t), s);
  t->d_rmq_st = static_cast<uint64_t*>(pool_get(c, (size_t)levels * nb * sizeof(uint64_t), s));
  if (!t->d_rmq_e || !t->d_rmq_mask || !t->d_rmq_st) return ET_ENOMEM;
  t->rmq_nb = nb;
  t->rmq_log = lg;
  ET_PROF(c, s, "phase:rmq_build");
  {
    ET_PROF(c, s, "k_rmq_euler");
    hipLaunchKernelGGL(k_rmq_euler, dim3(ceil_div(n, kB)), dim3(kB), 0, s, t->d_rank, t->d_rec, parent, n, t->d_root,
                       L, t->d_rmq_e, c->d_status);
  }
  {
    ET_PROF(c, s, "k_rmq_masks");
    const dim3 grid(ceil_div((int64_t)nb << lg, kB));
    if (lg == 6)
      hipLaunchKernelGGL(k_rmq_masks<6>, grid, dim3(kB), 0, s, t->d_rmq_e, L, static_cast<uint64_t*>(t->d_rmq_mask),
                         t->d_rmq_st);
    else
      hipLaunchKernelGGL(k_rmq_masks<5>, grid, dim3(kB), 0, s, t->d_rmq_e, L, static_cast<uint32_t*>(t->d_rmq_mask),
                         t->d_rmq_st);
  }
  for (int k = 1; k < levels; ++k)
    hipLaunchKernelGGL(k_rmq_level, dim3(ceil_div(nb, kB)), dim3(kB), 0, s, t->d_rmq_st + (size_t)(k - 1) * nb, nb,
                       1 << (k - 1), t->d_rmq_st + (size_t)k * nb);
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int tree_lca_rmq(Ctx* c, const et_tree* t, const int32_t* qx, const int32_t* qy, int64_t q, int32_t* out,
                 hipStream_t s) {
  if (q == 0) return ET_OK;
  const int32_t L = 2 * (t->n - 1);
  const int bs = c->qs.block;
  ET_PROF(c, s, "k_lca_rmq");
  for (int64_t q0 = 0; q0 < q; q0 += kQueryChunk) {  // one dispatch holds < 2^32 work-items
    const int64_t m = std::min(q - q0, kQueryChunk);
    const dim3 grid((unsigned)((m + bs - 1) / bs));
    if (t->rmq_log == 6) {
      RmqTables<6> tab{t->d_rmq_e, static_cast<const uint64_t*>(t->d_rmq_mask), t->d_rmq_st, t->rmq_nb};
      hipLaunchKernelGGL(k_lca_rmq<6>, grid, dim3(bs), 0, s, tab, t->d_rank, t->n, t->d_root, L, qx + q0, qy + q0, m,
                         out + q0, c->d_status);
    } else {
      RmqTables<5> tab{t->d_rmq_e, static_cast<const uint32_t*>(t->d_rmq_mask), t->d_rmq_st, t->rmq_nb};
      hipLaunchKernelGGL(k_lca_rmq<5>, grid, dim3(bs), 0, s, tab, t->d_rank, t->n, t->d_root, L, qx + q0, qy + q0, m,
                         out + q0, c->d_status);
    }
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
