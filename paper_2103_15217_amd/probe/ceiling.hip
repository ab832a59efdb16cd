// Random-access ceilings of the GPU, the bound that the tree walk, the
// gathers of the node and query kernels and the bridge passes run against:
// they move a few bytes per random address, so their speed is set by how
// many random requests per second the memory system serves, not by the
// streaming bandwidth.
//
//   ceiling [log2n]      (default 25: the 2^25 half-edges of a 2^24-node tree)
//
// Over an int32 array of 2^log2n elements it times, best of 5 launches:
//   copy        streaming copy of 8 B per element (reference bandwidth)
//   read        streaming read of the same 8 B per element: the read-only
//               bandwidth
//   gather      out[i] = a[idx[i]], idx a random permutation (independent random reads)
//   gather8     the same with 8-byte elements (an array of 8 B x 2^log2n)
//   gather16    the same with 16-byte elements (the query kernel's record loads)
//   scatter4    out[idx[i]] = i, 4-byte stores (the successor kernel's stores)
//   scatter8    rec[idx[i]] = i, 8-byte records (independent random writes)
//   chase       2^19 lanes each follow a[] through a disjoint piece of one random
//               cycle (dependent random reads, one chain per lane)
//   chase+w8    chase that also stores an 8-byte record at every visited index
//               (the access pattern of the level-1 list-ranking walk)
// and prints one JSON object per measurement: elements per second and
// bytes moved per second counting only the bytes the kernel asks for.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#define CHECK(x)                                                                        \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                     \
    }                                                                                   \
  } while (0)

namespace {

constexpr int kB = 256;

__global__ void k_copy(const int4* __restrict__ a, int4* __restrict__ b, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) b[i] = a[i];
}

__global__ void k_read(const int4* __restrict__ a, int32_t* __restrict__ out, int64_t n4) {
  // one 16-byte load per lane; the store is taken only for a value the
  // array never holds, so the kernel reads and (in effect) writes nothing
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n4) return;
  const int4 v = a[i];
  if ((v.x ^ v.y ^ v.z ^ v.w) == 0x7fffffff) out[i >> 6] = 1;
}

__global__ void k_gather(const int32_t* __restrict__ a, const int32_t* __restrict__ idx, int32_t* __restrict__ out,
                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[idx[i]];
}

template <typename T>
__global__ void k_gather_w(const T* __restrict__ a, const int32_t* __restrict__ idx, int32_t* __restrict__ out,
                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const T v = a[idx[i]];
    out[i] = (int32_t)(reinterpret_cast<const uint32_t*>(&v)[0] ^ reinterpret_cast<const uint32_t*>(&v)[sizeof(T) / 4 - 1]);
  }
}

__global__ void k_scatter4(const int32_t* __restrict__ idx, int32_t* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[idx[i]] = (int32_t)i;
}

__global__ void k_scatter8(const int32_t* __restrict__ idx, uint64_t* __restrict__ rec, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rec[idx[i]] = (uint64_t)i;
}

template <bool STORE>
__global__ void k_chase(const int32_t* __restrict__ a, const int32_t* __restrict__ start, int32_t lanes,
                        int32_t steps, uint64_t* __restrict__ rec, int32_t* __restrict__ out) {
  const int32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= lanes) return;
  int32_t p = start[l], acc = 0;
  for (int32_t k = 0; k < steps; ++k) {
    const int32_t q = a[p];
    if (STORE) rec[p] = ((uint64_t)(uint32_t)l << 32) | (uint32_t)k;
    acc += q;
    p = q;
  }
  out[l] = acc;
}

}  // namespace

int main(int argc, char** argv) {
  const int log2n = argc > 1 ? std::atoi(argv[1]) : 25;
  if (log2n < 20 || log2n > 28) {
    std::fprintf(stderr, "log2n must be in [20, 28]\n");
    return 2;
  }
  const int64_t n = int64_t(1) << log2n;
  const int lanes_log = 19;
  const int32_t lanes = 1 << lanes_log;
  const int32_t steps = (int32_t)(n >> lanes_log);

  // a random permutation and the single cycle a[perm[i]] = perm[i + 1]
  std::mt19937_64 rng(12345);
  std::vector<int32_t> perm(n), cyc(n), start(lanes);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  std::shuffle(perm.begin(), perm.end(), rng);
  for (int64_t i = 0; i < n; ++i) cyc[perm[i]] = perm[(i + 1) % n];
  for (int32_t l = 0; l < lanes; ++l) start[l] = perm[(int64_t)l * steps];

  int32_t *d_a, *d_idx, *d_out, *d_start, *d_lane;
  uint64_t* d_rec;
  int4 *d_c0, *d_c1, *d_g16;
  CHECK(hipMalloc(&d_a, n * 4));
  CHECK(hipMalloc(&d_idx, n * 4));
  CHECK(hipMalloc(&d_out, n * 4));
  CHECK(hipMalloc(&d_rec, n * 8));
  CHECK(hipMalloc(&d_c0, n * 8));
  CHECK(hipMalloc(&d_c1, n * 8));
  CHECK(hipMalloc(&d_g16, n * 16));
  CHECK(hipMalloc(&d_start, lanes * 4));
  CHECK(hipMalloc(&d_lane, lanes * 4));
  CHECK(hipMemcpy(d_idx, perm.data(), n * 4, hipMemcpyHostToDevice));
  CHECK(hipMemcpy(d_a, cyc.data(), n * 4, hipMemcpyHostToDevice));
  CHECK(hipMemcpy(d_start, start.data(), lanes * 4, hipMemcpyHostToDevice));
  CHECK(hipMemset(d_c0, 1, n * 8));
  CHECK(hipMemset(d_g16, 3, n * 16));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));

  auto measure = [&](const char* name, double bytes_per_elem, auto launch) {
    launch();
    CHECK(hipDeviceSynchronize());
    float best = 1e30f;
    for (int r = 0; r < 5; ++r) {
      CHECK(hipEventRecord(e0));
      launch();
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      best = std::min(best, ms);
    }
    std::printf("{\"probe\": \"%s\", \"log2n\": %d, \"ms\": %.4f, \"elements_per_s\": %.4e, \"GB_per_s\": %.1f}\n", name,
                log2n, best, (double)n / (best * 1e-3), bytes_per_elem * (double)n / (best * 1e-3) / 1e9);
    std::fflush(stdout);
  };
  const unsigned g = (unsigned)((n + kB - 1) / kB);
  const unsigned gl = (unsigned)((lanes + kB - 1) / kB);
  measure("copy", 16.0, [&] { hipLaunchKernelGGL(k_copy, dim3((unsigned)((n / 2 + kB - 1) / kB)), dim3(kB), 0, 0, d_c0, d_c1, n / 2); });
  // the copy's source, read only (a store would go to d_out[i / 64] < n)
  measure("read", 8.0, [&] { hipLaunchKernelGGL(k_read, dim3((unsigned)((n / 2 + kB - 1) / kB)), dim3(kB), 0, 0, d_c0, d_out, n / 2); });
  measure("gather", 12.0, [&] { hipLaunchKernelGGL(k_gather, dim3(g), dim3(kB), 0, 0, d_a, d_idx, d_out, n); });
  measure("gather8", 16.0, [&] {
    hipLaunchKernelGGL(k_gather_w<uint64_t>, dim3(g), dim3(kB), 0, 0, reinterpret_cast<const uint64_t*>(d_c0), d_idx,
                       d_out, n);
  });
  measure("gather16", 24.0, [&] {
    hipLaunchKernelGGL(k_gather_w<int4>, dim3(g), dim3(kB), 0, 0, d_g16, d_idx, d_out, n);
  });
  measure("scatter4", 8.0, [&] { hipLaunchKernelGGL(k_scatter4, dim3(g), dim3(kB), 0, 0, d_idx, d_out, n); });
  measure("scatter8", 12.0, [&] { hipLaunchKernelGGL(k_scatter8, dim3(g), dim3(kB), 0, 0, d_idx, d_rec, n); });
  measure("chase", 4.0, [&] {
    hipLaunchKernelGGL(k_chase<false>, dim3(gl), dim3(kB), 0, 0, d_a, d_start, lanes, steps, d_rec, d_lane);
  });
  measure("chase+w8", 12.0, [&] {
    hipLaunchKernelGGL(k_chase<true>, dim3(gl), dim3(kB), 0, 0, d_a, d_start, lanes, steps, d_rec, d_lane);
  });
  CHECK(hipGetLastError());
  for (void* p : {(void*)d_a, (void*)d_idx, (void*)d_out, (void*)d_rec, (void*)d_c0, (void*)d_c1, (void*)d_g16, (void*)d_start,
                  (void*)d_lane})
    CHECK(hipFree(p));
  return 0;
}
