// Bridges of a batch of independent graphs in one pass (Section 4, applied
// to many instances at once as the tree batch of Section 3.3 is).
//
// Bridges are a property of each connected component, so the batch is run
// as the disjoint union of its graphs: instance t's local vertex ids are
// shifted by voff[t] and its slots keep their place in the concatenated
// column array (the union's CSR row pointers are the local ones shifted by
// soff[t]). The union has one spanning forest, one chained Euler tour and
// one set of range tables, so the number of launches does not depend on
// the number of graphs. The union's mask is then cut into one word-aligned
// mask per graph (graph t's slot k at bit k of its own words, as et_bridges
// gives it alone), and per-graph counts are half the set bits of each
// graph's words (both slots of a bridge are set).
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kB = 256;

// largest t in [0, T) with off[t] <= k: the instance holding vertex, slot
// or output word k (empty instances share their offset with the next one
// and are skipped)
template <typename O>
__device__ __forceinline__ int32_t owner(const O* __restrict__ off, int32_t T, int64_t k) {
  int32_t lo = 0, hi = T;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if ((int64_t)off[mid] <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

// the owner of k given the owner t of an earlier element: forward search,
// binary only when k lies past instance t
template <typename O>
__device__ __forceinline__ int32_t owner_from(const O* __restrict__ off, int32_t t, int32_t T, int64_t k) {
  if ((int64_t)off[t + 1] > k) return t;
  int32_t lo = t, hi = T;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if ((int64_t)off[mid] <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

// element passes: each lane takes kPerLane elements a block width apart, so
// its owner only moves forward (one binary search per lane, not per element)
constexpr int kPerLane = 16;

// per instance: offsets non-decreasing and the local row pointers run from
// 0 to the instance's slot count; wc[t] = mask words of instance t
// (wc[T] = 0, so an exclusive scan gives the word offsets and the total)
__global__ void k_gb_check(const int32_t* __restrict__ rows, const int64_t* __restrict__ voff,
                           const int64_t* __restrict__ soff, int32_t T, int32_t V, int32_t nnz,
                           uint32_t* __restrict__ wc, uint32_t* __restrict__ status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > T) return;
  if (t == T) {
    wc[T] = 0;
    return;
  }
  const int64_t v0 = voff[t], v1 = voff[t + 1], s0 = soff[t], s1 = soff[t + 1];
  bool bad = v0 > v1 || s0 > s1 || v0 < 0 || v1 > V || s0 < 0 || s1 > nnz;
  if (t == 0 && (v0 != 0 || s0 != 0)) bad = true;
  if (t == T - 1 && (v1 != V || s1 != nnz)) bad = true;
  if (!bad) {
    // rows[] holds V + T entries: instance t's V_t + 1 start at v0 + t
    if (rows[v0 + t] != 0 || (int64_t)rows[v1 + t] != s1 - s0) bad = true;
    if (s1 > s0 && v1 == v0) bad = true;  // slots without a vertex
  }
  if (bad) flag(status, ST_BAD_CSR);
  wc[t] = bad ? 0u : (uint32_t)((s1 - s0 + 31) >> 5);
}

// union row pointers: row_g[v] = soff[t] + the local row pointer of v
__global__ void k_gb_rows(const int32_t* __restrict__ rows, const int64_t* __restrict__ voff,
                          const int64_t* __restrict__ soff, int32_t T, int32_t V, int32_t nnz,
                          int32_t* __restrict__ row_g, uint32_t* __restrict__ status) {
  const int64_t first = (int64_t)blockIdx.x * blockDim.x * kPerLane + threadIdx.x;
  if (first > V) return;
  int32_t t = owner(voff, T, min(first, (int64_t)V - 1));
  for (int i = 0; i < kPerLane; ++i) {
    const int64_t v = first + (int64_t)i * blockDim.x;
    if (v > V) break;
    if (v == V) {
      row_g[V] = nnz;
      break;
    }
    t = owner_from(voff, t, T, v);
    const int32_t r = rows[v + t];
    const int64_t g = soff[t] + (int64_t)r;
    if (r < 0 || g > soff[t + 1] || g > nnz) {
      flag(status, ST_BAD_CSR);
      row_g[v] = 0;  // keeps the union's row pointers in range
    } else {
      row_g[v] = (int32_t)g;
    }
  }
}

// union columns: col_g[k] = voff[t] + the local column of slot k
__global__ void k_gb_cols(const int32_t* __restrict__ col, const int64_t* __restrict__ voff,
                          const int64_t* __restrict__ soff, int32_t T, int32_t V, int32_t nnz,
                          int32_t* __restrict__ col_g, uint32_t* __restrict__ status) {
  const int64_t first = (int64_t)blockIdx.x * blockDim.x * kPerLane + threadIdx.x;
  if (first >= nnz) return;
  int32_t t = owner(soff, T, first);
  for (int i = 0; i < kPerLane; ++i) {
    const int64_t k = first + (int64_t)i * blockDim.x;
    if (k >= nnz) break;
    t = owner_from(soff, t, T, k);
    const int32_t w = col[k];
    const int64_t g = voff[t] + (int64_t)w;
    if (w < 0 || g >= voff[t + 1] || g >= V) {
      flag(status, ST_BAD_CSR);  // a column outside its own graph
      col_g[k] = 0;
    } else {
      col_g[k] = (int32_t)g;
    }
  }
}

__global__ void k_gb_zero(int64_t* __restrict__ counts, int32_t T) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < T) counts[t] = 0;
}

// graph t's output word j - wo[t] = the 32 union bits from slot
// soff[t] + 32 (j - wo[t]) on, cut at the graph's last slot
__global__ void k_gb_split(const uint32_t* __restrict__ umask, int32_t uwords, const int64_t* __restrict__ soff,
                           const uint32_t* __restrict__ wo, int32_t T, int32_t nnz, uint32_t* __restrict__ mask,
                           int64_t mask_words, int64_t* __restrict__ counts, uint32_t* __restrict__ status) {
  const int64_t used = wo[T];
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (first == 0 && used > mask_words) flag(status, ST_OUT_SIZE);
  for (int64_t j = first; j < mask_words; j += (int64_t)gridDim.x * blockDim.x) {
    uint32_t val = 0;
    if (j < used) {
      const int32_t t = owner(wo, T, j);
      const int64_t b = soff[t] + 32 * (j - (int64_t)wo[t]);
      const int64_t nb = min((int64_t)32, soff[t + 1] - b);
      if (b >= 0 && b < nnz && nb > 0) {
        const int64_t lo = b >> 5;
        const int sh = (int)(b & 31);
        val = umask[lo] >> sh;
        if (sh != 0 && lo + 1 < uwords) val |= umask[lo + 1] << (32 - sh);
        if (nb < 32) val &= (1u << nb) - 1u;
        if (counts && val) atomicAdd(reinterpret_cast<unsigned long long*>(counts + t), (unsigned long long)__popc(val));
      }
    }
    mask[j] = val;
  }
}

__global__ void k_gb_halve(int64_t* __restrict__ counts, int32_t T) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < T) counts[t] >>= 1;
}

}  // namespace

size_t bridges_batch_scratch_bytes(const Ctx* c, int32_t T, int32_t V, int32_t nnz) {
  const size_t uwords = ((size_t)nnz + 31) >> 5;
  const size_t b = scratch_block<int32_t>((size_t)V + 1) + scratch_block<int32_t>((size_t)std::max(nnz, 1)) +
                   scratch_block<uint32_t>(std::max<size_t>(uwords, 1)) + 2 * scratch_block<uint32_t>((size_t)T + 1);
  return b + scan_scratch_bytes((int64_t)T + 1) + bridges_scratch_bytes(c, V, nnz);
}

int bridges_batch_run(Ctx* c, const int32_t* rows, const int32_t* col, const int64_t* voff, const int64_t* soff,
                      int32_t T, int32_t V, int32_t nnz, uint32_t* mask, int64_t mask_words, int64_t* counts,
                      hipStream_t s) {
  const int32_t uwords = (int32_t)(((int64_t)nnz + 31) >> 5);
  Scratch sc(c, s);
  int32_t* row_g = sc.get<int32_t>((size_t)V + 1);
  int32_t* col_g = sc.get<int32_t>((size_t)std::max(nnz, 1));
  uint32_t* umask = sc.get<uint32_t>((size_t)std::max(uwords, 1));
  uint32_t* wc = sc.get<uint32_t>((size_t)T + 1);
  uint32_t* wo = sc.get<uint32_t>((size_t)T + 1);
  if (sc.failed) return ET_ENOMEM;
  {
    ET_PROF(c, s, "k_gb_check");
    hipLaunchKernelGGL(k_gb_check, dim3(ceil_div((int64_t)T + 1, kB)), dim3(kB), 0, s, rows, voff, soff, T, V, nnz,
                       wc, c->d_status);
  }
  int rc = scan_u32(c, wc, wo, (int64_t)T + 1, ScanOp::Add, true, s);
  if (rc) return rc;
  {
    ET_PROF(c, s, "k_gb_rows");
    hipLaunchKernelGGL(k_gb_rows, dim3(ceil_div((int64_t)V + 1, (int64_t)kB * kPerLane)), dim3(kB), 0, s, rows, voff,
                       soff, T, V, nnz, row_g, c->d_status);
  }
  if (nnz > 0) {
    ET_PROF(c, s, "k_gb_cols");
    hipLaunchKernelGGL(k_gb_cols, dim3(ceil_div(nnz, (int64_t)kB * kPerLane)), dim3(kB), 0, s, col, voff, soff, T, V,
                       nnz, col_g, c->d_status);
  }
  rc = bridges_run(c, row_g, col_g, V, nnz, umask, s, kAlgoTV);
  if (rc) return rc;
  if (counts) hipLaunchKernelGGL(k_gb_zero, dim3(ceil_div(T, kB)), dim3(kB), 0, s, counts, T);
  if (mask_words > 0) {
    ET_PROF(c, s, "k_gb_split");
    hipLaunchKernelGGL(k_gb_split, dim3((unsigned)std::min<int64_t>((mask_words + kB - 1) / kB, 1 << 16)), dim3(kB),
                       0, s, umask, uwords, soff, wo, T, nnz, mask, mask_words, counts, c->d_status);
  }
  if (counts) hipLaunchKernelGGL(k_gb_halve, dim3(ceil_div(T, kB)), dim3(kB), 0, s, counts, T);
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
