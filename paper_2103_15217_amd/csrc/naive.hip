// The naive LCA algorithm that the paper compares against (Section 3.1,
// "The Naive Algorithm", after Martins et al.): node levels by pointer
// jumping, then one lane per query climbing parent pointers.
//
// Levels. Every node keeps a jump record {ancestor, distance to it},
// initially {parent, 1}; the root's level is 0. A node whose ancestor has a
// known level takes that level plus the distance; otherwise its ancestor is
// replaced by the ancestor's ancestor (distances add). As in the paper, a
// lane makes five jumps between global synchronisations (kernel
// boundaries). Records are updated in place: a jump may read a record that
// another lane has already advanced in the same launch, which only moves
// further up. At a launch's start every unresolved record spans at least D
// edges and every jump adds at least D more, so after a launch it spans at
// least 6D; ceil(log6 n) + 2 launches therefore resolve every node of a
// tree with no host round trip. A node still unresolved after them lies on
// a cycle or hangs from a bad parent and is flagged.
//
// Queries. The deeper pointer climbs to the other's level, then both climb
// together until they meet; time is proportional to the x-y distance.
// Every climb is bounded by the levels, so an inconsistent level array
// ends in a flag, never in a hang.
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kB = 256;
constexpr int kJumps = 5;

__device__ __forceinline__ uint64_t jrec(int32_t anc, int32_t dist) {
  return (uint64_t)(uint32_t)anc | ((uint64_t)(uint32_t)dist << 32);
}
__device__ __forceinline__ uint64_t ld64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st32(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_zero1(int32_t* p) { *p = 0; }

// scalars[0] = number of roots
__global__ void k_lvl_init(const int32_t* __restrict__ parent, int32_t n, uint64_t* __restrict__ jump,
                           int32_t* __restrict__ level, int32_t* __restrict__ scalars,
                           uint32_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t p = parent[v];
  if (p == -1) {
    atomicAdd(scalars, 1);
    level[v] = 0;
    jump[v] = jrec((int32_t)v, 0);
  } else if (p >= 0 && p < n && p != v) {
    level[v] = -1;
    jump[v] = jrec(p, 1);
  } else {
    flag(status, ST_BAD_PARENT);
    level[v] = -1;
    jump[v] = jrec((int32_t)v, 0);  // never resolves: reported by the check
  }
}

__global__ void k_lvl_jump(uint64_t* jump, int32_t* level, int32_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || ld32(level + v) >= 0) return;
  const uint64_t r = ld64(jump + v);
  int32_t a = (int32_t)(uint32_t)r;
  int32_t d = (int32_t)(r >> 32);
  for (int k = 0; k < kJumps; ++k) {
    const int32_t la = ld32(level + a);
    if (la >= 0) {
      st32(level + v, la + d);
      return;
    }
    const uint64_t ra = ld64(jump + a);
    a = (int32_t)(uint32_t)ra;
    d = min(d + (int32_t)(ra >> 32), n);  // saturates only on a cycle
  }
  st64(jump + v, jrec(a, d));
}

__global__ void k_lvl_check(const int32_t* __restrict__ level, int32_t n, const int32_t* __restrict__ scalars,
                            uint32_t* __restrict__ status) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0 && scalars[0] != 1) flag(status, ST_ROOTS);
  if (v < n && level[v] < 0) flag(status, ST_UNREACHED);
}

__global__ __launch_bounds__(kB) void k_lca_naive(const int32_t* __restrict__ parent,
                                                 const int32_t* __restrict__ level, int32_t n,
                                                 const int32_t* __restrict__ qx, const int32_t* __restrict__ qy,
                                                 int64_t q, int32_t* __restrict__ out,
                                                 uint32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  int32_t x = qx[i], y = qy[i];
  if ((uint32_t)x >= (uint32_t)n || (uint32_t)y >= (uint32_t)n) {
    flag(status, ST_BAD_QUERY);
    out[i] = -1;
    return;
  }
  int32_t lx = level[x], ly = level[y];
  bool ok = lx >= 0 && ly >= 0;
  // climb the deeper side to the other's level, then both together
  for (; ok && lx > ly; --lx) {
    x = parent[x];
    ok = (uint32_t)x < (uint32_t)n;
  }
  for (; ok && ly > lx; --ly) {
    y = parent[y];
    ok = (uint32_t)y < (uint32_t)n;
  }
  for (; ok && x != y; --lx) {
    if (lx == 0) {  // both at level 0 and still apart: not one tree
      ok = false;
      break;
    }
    x = parent[x];
    y = parent[y];
    ok = (uint32_t)x < (uint32_t)n && (uint32_t)y < (uint32_t)n;
  }
  if (!ok) {
    flag(status, ST_BAD_INDEX);
    out[i] = -1;
    return;
  }
  out[i] = x;
}

}  // namespace

int levels_run(Ctx* c, const int32_t* parent, int32_t n, int32_t* level, hipStream_t s) {
  if (n == 0) return ET_OK;
  Scratch sc(c, s);
  uint64_t* jump = sc.get<uint64_t>((size_t)n);
  int32_t* roots = sc.get<int32_t>(1);
  if (sc.failed) return ET_ENOMEM;
  const int g = ceil_div(n, kB);
  hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, s, roots);
  {
    ET_PROF(c, s, "k_lvl_init");
    hipLaunchKernelGGL(k_lvl_init, dim3(g), dim3(kB), 0, s, parent, n, jump, level, roots, c->d_status);
  }
  int launches = 2;
  for (double span = 1.0; span < (double)n; span *= 1.0 + kJumps) ++launches;
  {
    ET_PROF(c, s, "k_lvl_jump");
    for (int t = 0; t < launches; ++t)
      hipLaunchKernelGGL(k_lvl_jump, dim3(g), dim3(kB), 0, s, jump, level, n);
  }
  hipLaunchKernelGGL(k_lvl_check, dim3(g), dim3(kB), 0, s, level, n, roots, c->d_status);
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int lca_naive_run(Ctx* c, const int32_t* parent, const int32_t* level, int32_t n, const int32_t* qx,
                  const int32_t* qy, int64_t q, int32_t* out, hipStream_t s) {
  if (q == 0) return ET_OK;
  ET_PROF(c, s, "k_lca_naive");
  for (int64_t q0 = 0; q0 < q; q0 += kQueryChunk) {  // one dispatch holds < 2^32 work-items
    const int64_t m = std::min(q - q0, kQueryChunk);
    hipLaunchKernelGGL(k_lca_naive, dim3((unsigned)((m + kB - 1) / kB)), dim3(kB), 0, s, parent, level, n, qx + q0,
                       qy + q0, m, out + q0, c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
