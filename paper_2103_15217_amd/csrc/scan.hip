// Array scans (prefix sums) over u32 with + or xor.
//
// The paper turns every prefix sum on the Euler tour, after a single list
// ranking, into an array scan (Section 2.2). This is a three-kernel
// reduce-then-scan: each workgroup owns a contiguous range of 4096-element
// chunks, reduces it, one workgroup scans the per-range totals, and each
// range is scanned again with its carry (with at most 512 ranges each range
// adds up the totals before it and the middle launch is skipped). Arrays of
// at most four chunks are scanned by one workgroup in one launch. Inside a chunk every lane holds 16
// consecutive items (four 16-byte loads), scans them serially, and the lane
// totals are combined across the wavefront with shuffles and across the
// four wavefronts through LDS.
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kChunk = kThreads * kItems;
constexpr int kMaxRanges = 4096;
constexpr int kSmallChunks = 4;  // arrays of at most 16K items take the one-launch path
constexpr int kRawRanges = 512;  // up to this many ranges sum their carries themselves

template <ScanOp OP>
__device__ __forceinline__ uint32_t combine(uint32_t a, uint32_t b) {
  return OP == ScanOp::Add ? a + b : a ^ b;
}

template <ScanOp OP>
__device__ __forceinline__ uint32_t wave_inclusive(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v = combine<OP>(v, o);
  }
  return v;
}

// Block-wide exclusive prefix of one value per thread; returns the prefix
// and writes the block total to *total.
template <ScanOp OP>
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kThreads / 64];
  const int lane = __lane_id();
  const int wave = threadIdx.x >> 6;
  uint32_t inc = wave_inclusive<OP>(v);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wave) before = combine<OP>(before, wsum[w]);
    all = combine<OP>(all, wsum[w]);
  }
  __syncthreads();
  *total = all;
  uint32_t excl = (OP == ScanOp::Add) ? inc - v : inc ^ v;
  return combine<OP>(before, excl);
}

__device__ __forceinline__ void load16(const uint32_t* in, int64_t base, int64_t n, uint32_t* x) {
  if (base + kItems <= n && ((base & 3) == 0)) {
    const uint4* p = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
    for (int k = 0; k < kItems / 4; ++k) {
      uint4 v = p[k];
      x[4 * k] = v.x; x[4 * k + 1] = v.y; x[4 * k + 2] = v.z; x[4 * k + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kItems; ++k) x[k] = (base + k < n) ? in[base + k] : 0u;
  }
}

__device__ __forceinline__ void store16(uint32_t* out, int64_t base, int64_t n, const uint32_t* x) {
  if (base + kItems <= n && ((base & 3) == 0)) {
    uint4* p = reinterpret_cast<uint4*>(out + base);
#pragma unroll
    for (int k = 0; k < kItems / 4; ++k) p[k] = make_uint4(x[4 * k], x[4 * k + 1], x[4 * k + 2], x[4 * k + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < kItems; ++k)
      if (base + k < n) out[base + k] = x[k];
  }
}

template <ScanOp OP>
__global__ __launch_bounds__(kThreads) void k_range_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                           int64_t chunks_per_range,
                                                           uint32_t* __restrict__ partial) {
  const int64_t c0 = (int64_t)blockIdx.x * chunks_per_range;
  uint32_t acc = 0;
  for (int64_t c = c0; c < c0 + chunks_per_range; ++c) {
    int64_t base = c * kChunk + (int64_t)threadIdx.x * kItems;
    if (base >= n) break;
    uint32_t x[kItems];
    load16(in, base, n, x);
#pragma unroll
    for (int k = 0; k < kItems; ++k) acc = combine<OP>(acc, x[k]);
  }
  uint32_t total;
  (void)block_exclusive<OP>(acc, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// one workgroup of 1024 lanes: exclusive scan of up to kMaxRanges totals
template <ScanOp OP>
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* __restrict__ partial, int nranges) {
  __shared__ uint32_t wsum[16];
  const int per = (nranges + 1023) / 1024;  // <= 4
  const int t = threadIdx.x;
  uint32_t x[4] = {0, 0, 0, 0};
  uint32_t acc = 0;
  for (int k = 0; k < per; ++k) {
    int i = t * per + k;
    x[k] = (i < nranges) ? partial[i] : 0u;
    acc = combine<OP>(acc, x[k]);
  }
  const int lane = __lane_id(), wave = t >> 6;
  uint32_t inc = wave_inclusive<OP>(acc);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before = combine<OP>(before, wsum[w]);
  uint32_t run = combine<OP>(before, (OP == ScanOp::Add) ? inc - acc : inc ^ acc);
  for (int k = 0; k < per; ++k) {
    int i = t * per + k;
    if (i < nranges) partial[i] = run;
    run = combine<OP>(run, x[k]);
  }
}

template <ScanOp OP, bool EXCL>
__global__ __launch_bounds__(kThreads) void k_range_scan(const uint32_t* __restrict__ in,
                                                         uint32_t* __restrict__ out, int64_t n,
                                                         int64_t chunks_per_range,
                                                         const uint32_t* __restrict__ partial, bool raw) {
  // carry into this range: none for a single range, the scanned partial, or
  // (raw partials of a few ranges) their combination over the ranges before
  uint32_t carry = 0u;
  if (partial && !raw) {
    carry = partial[blockIdx.x];
  } else if (partial) {
    uint32_t acc = 0u;
    for (int r = threadIdx.x; r < (int)blockIdx.x; r += kThreads) acc = combine<OP>(acc, partial[r]);
    (void)block_exclusive<OP>(acc, &carry);
  }
  const int64_t c0 = (int64_t)blockIdx.x * chunks_per_range;
  for (int64_t c = c0; c < c0 + chunks_per_range; ++c) {
    if (c * kChunk >= n) break;
    int64_t base = c * kChunk + (int64_t)threadIdx.x * kItems;
    uint32_t x[kItems];
    load16(in, base, n, x);
    uint32_t local = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) local = combine<OP>(local, x[k]);
    uint32_t total;
    uint32_t run = combine<OP>(carry, block_exclusive<OP>(local, &total));
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      uint32_t v = x[k];
      if (EXCL) {
        x[k] = run;
        run = combine<OP>(run, v);
      } else {
        run = combine<OP>(run, v);
        x[k] = run;
      }
    }
    store16(out, base, n, x);
    carry = combine<OP>(carry, total);
  }
}

template <ScanOp OP>
int scan_impl(Ctx* c, const uint32_t* in, uint32_t* out, int64_t n, bool exclusive, hipStream_t s) {
  if (n <= 0) return ET_OK;
  int64_t chunks = (n + kChunk - 1) / kChunk;
  if (chunks <= kSmallChunks) {
    // short arrays: one workgroup scans the few chunks in order, so the
    // reduce and carry launches are skipped
    ET_PROF(c, s, OP == ScanOp::Add ? "k_range_scan<add>" : "k_range_scan<xor>");
    if (exclusive)
      hipLaunchKernelGGL((k_range_scan<OP, true>), dim3(1), dim3(kThreads), 0, s, in, out, n, chunks, nullptr,
                         false);
    else
      hipLaunchKernelGGL((k_range_scan<OP, false>), dim3(1), dim3(kThreads), 0, s, in, out, n, chunks, nullptr,
                         false);
    return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
  }
  int64_t per = (chunks + kMaxRanges - 1) / kMaxRanges;
  int nranges = (int)((chunks + per - 1) / per);
  Scratch sc(c, s);
  uint32_t* partial = sc.get<uint32_t>(nranges);
  if (sc.failed) return ET_ENOMEM;
  {
    ET_PROF(c, s, OP == ScanOp::Add ? "k_range_reduce<add>" : "k_range_reduce<xor>");
    hipLaunchKernelGGL(k_range_reduce<OP>, dim3(nranges), dim3(kThreads), 0, s, in, n, per, partial);
  }
  // a few ranges: each adds up the raw totals before it, one launch fewer
  const bool raw = nranges <= kRawRanges;
  if (!raw) {
    ET_PROF(c, s, OP == ScanOp::Add ? "k_scan_partials<add>" : "k_scan_partials<xor>");
    hipLaunchKernelGGL(k_scan_partials<OP>, dim3(1), dim3(1024), 0, s, partial, nranges);
  }
  if (exclusive) {
    ET_PROF(c, s, OP == ScanOp::Add ? "k_range_scan<add,excl>" : "k_range_scan<xor,excl>");
    hipLaunchKernelGGL((k_range_scan<OP, true>), dim3(nranges), dim3(kThreads), 0, s, in, out, n, per,
                       partial, raw);
  } else {
    ET_PROF(c, s, OP == ScanOp::Add ? "k_range_scan<add,incl>" : "k_range_scan<xor,incl>");
    hipLaunchKernelGGL((k_range_scan<OP, false>), dim3(nranges), dim3(kThreads), 0, s, in, out, n, per,
                       partial, raw);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  if (chunks <= kSmallChunks) return 0;
  const int64_t per = (chunks + kMaxRanges - 1) / kMaxRanges;
  return scratch_block<uint32_t>((size_t)((chunks + per - 1) / per));
}

int scan_u32(Ctx* c, const uint32_t* in, uint32_t* out, int64_t n, ScanOp op, bool exclusive,
             hipStream_t s) {
  return op == ScanOp::Add ? scan_impl<ScanOp::Add>(c, in, out, n, exclusive, s)
                           : scan_impl<ScanOp::Xor>(c, in, out, n, exclusive, s);
}

}  // namespace et
