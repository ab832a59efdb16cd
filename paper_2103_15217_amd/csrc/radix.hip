// Stable grouping of the children of every node by parent id.
//
// The paper builds the DCEL by lexicographically sorting half-edges
// (Section 2.1) and remarks that this sort dominates construction. With a
// parent array as input the half-edges of node x are its children, and a
// stable sort of the child ids by parent id puts every node's children next
// to each other in ascending id order, which is all the successor step
// needs. This is an LSD radix sort over the ceil(log2 n) key bits with 8-bit
// digits (3 passes at n = 2^24, 4 at 2^27), or 9-bit digits for short
// arrays where that saves a pass (2 passes of 9 and 8 bits at 2^17):
//
//   upsweep    per 4096-element tile, a digit histogram (one LDS histogram
//              per wavefront), stored digit-major so that one exclusive scan
//              gives every (digit, tile) its output offset;
//   scan       the array scan of scan.hip;
//   downsweep  512 lanes per tile; each wavefront ranks its 8 rounds of 64
//              keys stably: 8 ballots find the lanes that share a digit, the
//              lowest such lane bumps the wavefront's LDS counter for that
//              digit, and the eight wavefront counters are chained per
//              digit. The tile is then sorted by digit in LDS and written
//              out run by run, so consecutive lanes store to consecutive
//              addresses.
//
// Both kernels take their tile from xcd_tile(): workgroups are handed to the
// eight XCDs in turn, and each XCD is given a contiguous range of tiles, so
// the runs of one digit that adjacent tiles write (neighbours in the output)
// and the histogram entries they write meet in the same L2, which merges
// their partial lines before they go to memory. With the 512-lane shape
// this takes a downsweep pass over 2^24 uniform keys from 126 to 83 us, and
// one of a 2^24-node tree build from 116 to 91 us.
//
// The first pass reads the parent array directly (the root's -1 becomes the
// all-ones key and sorts last), validates it, finds the root, and writes
// the successor of every down half-edge of a leaf (2c -> 2c+1).
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kThreads = 256;  // histogram pass
constexpr int kWaves = kThreads / 64;
constexpr int kRounds = 16;
constexpr int kTile = kThreads * kRounds;  // 4096 keys per tile
constexpr int kDownThreads = 512;          // downsweep: 8 wavefronts of 8 rounds per tile
constexpr int kDownWaves = kDownThreads / 64;
constexpr int kDownRounds = kTile / kDownThreads;
constexpr int kXcds = 8;
constexpr int kMaxBits = 9;                // widest digit
constexpr int kMaxDigits = 1 << kMaxBits;  // kernels are built for 256 or 512 digits

// tile of this workgroup: XCD x = blockIdx % 8 takes the x-th contiguous
// range of tiles (a bijection of [0, ntiles) for any ntiles)
__device__ __forceinline__ int32_t xcd_tile(int32_t ntiles) {
  const int32_t b = (int32_t)blockIdx.x;
  const int32_t q = ntiles / kXcds, r = ntiles % kXcds, x = b % kXcds;
  return x * q + min(x, r) + b / kXcds;
}

__device__ __forceinline__ uint32_t parent_key(int32_t p, int32_t n) {
  return (p >= 0 && p < n) ? (uint32_t)p : 0xffffffffu;
}

// scalars[0] = root id, scalars[1] = number of roots
template <bool FIRST, int DIG>
__global__ __launch_bounds__(kThreads) void k_upsweep(const void* __restrict__ keys_in, int32_t n, int shift,
                                                      int nbits, int32_t ntiles, uint32_t* __restrict__ hist,
                                                      int32_t* __restrict__ succ, int32_t* __restrict__ scalars,
                                                      uint32_t* __restrict__ status) {
  __shared__ uint32_t h[kWaves][DIG];
  const int wave = threadIdx.x >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  for (int i = threadIdx.x; i < kWaves * DIG; i += kThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  const int32_t tile = xcd_tile(ntiles);
  const int64_t base = (int64_t)tile * kTile;
  bool bad = false;
  // all of a lane's loads first (guarded, not cut short), then the counts
  uint32_t raw[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t idx = base + r * kThreads + threadIdx.x;
    raw[r] = idx < n ? static_cast<const uint32_t*>(keys_in)[idx] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t idx = base + r * kThreads + threadIdx.x;
    if (idx >= n) break;
    uint32_t key;
    if (FIRST) {
      const int32_t p = (int32_t)raw[r];
      key = parent_key(p, n);
      if (p == -1) {
        atomicAdd(&scalars[1], 1);
        scalars[0] = (int32_t)idx;
        succ[2 * idx] = -2;
        succ[2 * idx + 1] = -2;
      } else {
        if (p < 0 || p >= n || p == idx) bad = true;
        // succ(2c) = 2c+1 (a leaf unless the successor step writes the first
        // child); succ(2c+1) is always written by that step, so the pair is
        // stored whole: one full 8-byte store instead of a strided 4-byte one
        reinterpret_cast<int2*>(succ)[idx] = make_int2((int32_t)(2 * idx + 1), -2);
      }
    } else {
      key = raw[r];
    }
    atomicAdd(&h[wave][(key >> shift) & mask], 1u);
  }
  if (bad) flag(status, ST_BAD_PARENT);
  __syncthreads();
  for (int d = threadIdx.x; d <= (int)mask; d += kThreads)
    hist[(int64_t)d * ntiles + tile] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

template <bool FIRST, int DIG>
__global__ __launch_bounds__(kDownThreads, 2) void k_downsweep(const void* __restrict__ keys_in,
                                                        const int32_t* __restrict__ vals_in, int32_t n, int shift,
                                                        int nbits, int32_t ntiles,
                                                        const uint32_t* __restrict__ offsets,
                                                        uint32_t* __restrict__ keys_out,
                                                        int32_t* __restrict__ vals_out) {
  constexpr int kPer = (DIG + kDownThreads - 1) / kDownThreads;  // digits owned by one thread in the tile scan
  __shared__ uint32_t cnt[kDownWaves][DIG];
  __shared__ uint32_t lstart[DIG];   // tile-local start of each digit's run
  __shared__ uint32_t gstart[DIG];   // global start of this tile's run of each digit
  __shared__ uint32_t skey[kTile];
  __shared__ int32_t sval[kTile];
  const int wave = threadIdx.x >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  for (int i = threadIdx.x; i < kDownWaves * DIG; i += kDownThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const int32_t tile = xcd_tile(ntiles);
  const int64_t tbase = (int64_t)tile * kTile;
  const int64_t wbase = tbase + (int64_t)wave * (64 * kDownRounds) + __lane_id();
  const uint64_t below = lanemask_lt();
  uint32_t key[kDownRounds];
  int32_t val[kDownRounds];
  uint32_t rnk[kDownRounds];
#pragma unroll
  for (int r = 0; r < kDownRounds; ++r) {
    const int64_t idx = wbase + r * 64;
    const bool valid = idx < n;
    if (FIRST) {
      key[r] = valid ? parent_key(static_cast<const int32_t*>(keys_in)[idx], n) : 0u;
      val[r] = (int32_t)idx;
    } else {
      key[r] = valid ? static_cast<const uint32_t*>(keys_in)[idx] : 0u;
      val[r] = valid ? vals_in[idx] : 0;
    }
    const uint32_t dg = (key[r] >> shift) & mask;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < (DIG > 256 ? 9 : 8); ++b) {
      if (b >= nbits) break;
      const bool bit = (dg >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t lower = (uint32_t)__popcll(peers & below);
    const uint32_t c0 = cnt[wave][dg];
    rnk[r] = c0 + lower;
    if (valid && lower == 0) cnt[wave][dg] = c0 + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: chain the wave counters, then an exclusive scan over digits
  // gives each digit's run inside the tile; thread t owns digits kPer*t ..
  // kPer*t + kPer - 1
  {
    uint32_t tots[kPer];
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int d = kPer * threadIdx.x + q;
      uint32_t td = 0;
      if (d < DIG && d <= (int)mask) {
#pragma unroll
        for (int w = 0; w < kDownWaves; ++w) {
          const uint32_t c = cnt[w][d];
          cnt[w][d] = td;  // exclusive prefix over the waves
          td += c;
        }
        gstart[d] = offsets[(int64_t)d * ntiles + tile];
      }
      tots[q] = td;
      tot += td;
    }
    // block exclusive scan of the per-thread totals over the 512 threads (8 waves)
    uint32_t inc = tot;
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(inc, o, 64);
      if (lane >= o) inc += u;
    }
    __shared__ uint32_t wsum[kDownWaves];
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t run = inc - tot;
    for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int d = kPer * threadIdx.x + q;
      if (d < DIG) lstart[d] = run;
      run += tots[q];
    }
  }
  __syncthreads();
  // place every key at its tile-local sorted position
#pragma unroll
  for (int r = 0; r < kDownRounds; ++r) {
    const int64_t idx = wbase + r * 64;
    if (idx < n) {
      const uint32_t dg = (key[r] >> shift) & mask;
      const uint32_t lp = lstart[dg] + cnt[wave][dg] + rnk[r];
      skey[lp] = key[r];
      sval[lp] = val[r];
    }
  }
  __syncthreads();
  // write the tile out digit run by digit run: consecutive lanes, consecutive addresses
  const int valid_in_tile = (int)min<int64_t>((int64_t)kTile, n - tbase);
#pragma unroll
  for (int r = 0; r < kDownRounds; ++r) {
    const int i = r * kDownThreads + threadIdx.x;
    if (i < valid_in_tile) {
      const uint32_t k = skey[i];
      const uint32_t dg = (k >> shift) & mask;
      const uint32_t pos = gstart[dg] + (uint32_t)i - lstart[dg];
      keys_out[pos] = k;
      vals_out[pos] = sval[i];
    }
  }
}

__global__ void k_reset_root(int32_t* __restrict__ scalars) {
  scalars[0] = -1;
  scalars[1] = 0;
}

// Digit widths of the passes over `bits` key bits of n keys, balanced. A
// 9-bit pass costs more than an 8-bit one (runs per tile half as long, a
// larger LDS footprint per workgroup), so 9-bit digits are used
// only for sorts of at most 2^21 keys, where the number of passes (each a
// few launches) matters more than their bandwidth.
int plan_passes(int bits, int64_t n, int* width) {
  const int p8 = (bits + 7) / 8, p9 = (bits + kMaxBits - 1) / kMaxBits;
  const int passes = (n <= (1 << 21)) ? std::min(p8, p9) : p8;
  for (int p = 0; p < passes; ++p) width[p] = bits / passes + (p < bits % passes ? 1 : 0);
  return passes;
}

}  // namespace

// histograms of every tile and the ping-pong keys and values, plus the
// largest histogram scan's partials
size_t group_by_parent_scratch_bytes(int32_t n) {
  const int32_t ntiles = ceil_div(n, kTile);
  return scratch_block<uint32_t>((size_t)kMaxDigits * ntiles) + scratch_block<uint32_t>((size_t)n) +
         scratch_block<int32_t>((size_t)n) + scan_scratch_bytes((int64_t)kMaxDigits * ntiles);
}

// keys_out / vals_out receive the stable order; scalars[0] = root, scalars[1]
// = number of roots; succ[2c] of every non-root c is set to 2c+1 and
// succ[2c+1] to -2 (the successor step writes it), both root ids to -2.
int group_by_parent_impl(Ctx* c, const int32_t* parent, int32_t n, uint32_t* keys_out, int32_t* vals_out,
                         int32_t* succ, int32_t* scalars, hipStream_t s) {
  int bits = 1;
  while (bits < 31 && (1ll << bits) < n) ++bits;
  int width[8];
  const int passes = plan_passes(bits, n, width);
  const int32_t ntiles = ceil_div(n, kTile);
  Scratch sc(c, s);
  uint32_t* hist = sc.get<uint32_t>((size_t)kMaxDigits * ntiles);
  uint32_t* tk = sc.get<uint32_t>((size_t)n);
  int32_t* tv = sc.get<int32_t>((size_t)n);
  if (sc.failed) return ET_ENOMEM;
  hipLaunchKernelGGL(k_reset_root, dim3(1), dim3(1), 0, s, scalars);
  const void* kin = parent;
  const int32_t* vin = nullptr;
  for (int p = 0, shift = 0; p < passes; shift += width[p], ++p) {
    const int nbits = width[p];
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    uint32_t* kout = to_out ? keys_out : tk;
    int32_t* vout = to_out ? vals_out : tv;
    if (p == 0) {
      ET_PROF(c, s, "k_upsweep<true>");
      const auto kern = (nbits > 8) ? k_upsweep<true, 512> : k_upsweep<true, 256>;
      hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kThreads), 0, s, kin, n, shift, nbits, ntiles, hist, succ, scalars,
                         c->d_status);
    } else {
      ET_PROF(c, s, "k_upsweep<false>");
      const auto kern = (nbits > 8) ? k_upsweep<false, 512> : k_upsweep<false, 256>;
      hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kThreads), 0, s, kin, n, shift, nbits, ntiles, hist, succ, scalars,
                         c->d_status);
    }
    int rc = scan_u32(c, hist, hist, (int64_t)(1 << nbits) * ntiles, ScanOp::Add, true, s);
    if (rc) return rc;
    if (p == 0) {
      ET_PROF(c, s, "k_downsweep<true>");
      const auto kern = (nbits > 8) ? k_downsweep<true, 512> : k_downsweep<true, 256>;
      hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kDownThreads), 0, s, kin, vin, n, shift, nbits, ntiles, hist, kout,
                         vout);
    } else {
      ET_PROF(c, s, "k_downsweep<false>");
      const auto kern = (nbits > 8) ? k_downsweep<false, 512> : k_downsweep<false, 256>;
      hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kDownThreads), 0, s, kin, vin, n, shift, nbits, ntiles, hist, kout,
                         vout);
    }
    kin = kout;
    vin = vout;
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

// Stable sort of (key, value) pairs by the low `bits` bits of the key, with
// the same kernels: keys_out / vals_out receive the sorted pairs; the inputs
// are left as they are.
int sort_pairs_u32(Ctx* c, const uint32_t* keys, const int32_t* vals, int32_t n, int bits, uint32_t* keys_out,
                   int32_t* vals_out, hipStream_t s) {
  if (n <= 0) return ET_OK;
  bits = std::max(1, std::min(bits, 32));
  int width[8];
  const int passes = plan_passes(bits, n, width);
  const int32_t ntiles = ceil_div(n, kTile);
  Scratch sc(c, s);
  uint32_t* hist = sc.get<uint32_t>((size_t)kMaxDigits * ntiles);
  uint32_t* tk = sc.get<uint32_t>((size_t)n);
  int32_t* tv = sc.get<int32_t>((size_t)n);
  if (sc.failed) return ET_ENOMEM;
  const void* kin = keys;
  const int32_t* vin = vals;
  for (int p = 0, shift = 0; p < passes; shift += width[p], ++p) {
    const int nbits = width[p];
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    uint32_t* kout = to_out ? keys_out : tk;
    int32_t* vout = to_out ? vals_out : tv;
    {
      ET_PROF(c, s, "k_upsweep<false>");
      const auto kern = (nbits > 8) ? k_upsweep<false, 512> : k_upsweep<false, 256>;
      hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kThreads), 0, s, kin, n, shift, nbits, ntiles, hist, nullptr,
                         nullptr, c->d_status);
    }
    int rc = scan_u32(c, hist, hist, (int64_t)(1 << nbits) * ntiles, ScanOp::Add, true, s);
    if (rc) return rc;
    {
      ET_PROF(c, s, "k_downsweep<false>");
      const auto kern = (nbits > 8) ? k_downsweep<false, 512> : k_downsweep<false, 256>;
      hipLaunchKernelGGL(kern, dim3(ntiles), dim3(kDownThreads), 0, s, kin, vin, n, shift, nbits, ntiles, hist, kout,
                         vout);
    }
    kin = kout;
    vin = vout;
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
