// List ranking and list prefix sums (Section 2.2).
//
// The paper ranks the tour with the GPU sublist algorithm of Wei and JaJa
// rather than pointer jumping. This is an MI355X design of the same idea:
//
//  level 1  Splitters: one pseudo-randomly placed element in every chunk of
//           K consecutive ids (plus every list head) starts a sublist. A
//           wavefront owns a contiguous range of sublist ids; its 64 lanes
//           each walk one sublist, and a lane whose sublist ends takes the
//           next id of the wave's range (ballot + popcount, no atomics), so
//           lanes stay busy even though sublist lengths are geometric. Each
//           visited element gets one 8-byte record {sublist, local rank,
//           local down-count}; each sublist gets {next sublist, length,
//           down-count}. Sublists longer than 65535 elements are split into
//           continuation sublists so the local fields fit 16 bits.
//  level k  The list of sublists is ranked the same way with the sublist
//           lengths as weights, until it has at most kLdsMax elements.
//  final    One workgroup ranks the last list in LDS by jumping predecessor
//           pointers (Wyllie) and checks that every used element is reached
//           from a head; offsets are then pushed back down the levels.
//
// Every walk is bounded and every gathered index is range checked, so a
// malformed list (a cycle, a shared successor, an id out of range) sets a
// status bit instead of faulting or hanging.
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kCap = 65535;        // level-1 sublist length cap (16-bit local fields)
constexpr int kLdsMax = 4096;      // elements the final LDS kernel ranks
constexpr int kWalkThreads = 256;
constexpr uint32_t kSalt = 0x9e3779b9u;

__device__ __forceinline__ bool is_splitter(int32_t e, int ks, uint32_t salt) {
  const uint32_t m = (1u << ks) - 1u;
  return ((uint32_t)e & m) == (mix32(((uint32_t)e >> ks) ^ salt) & m);
}

__device__ __forceinline__ int32_t splitter_of_chunk(int32_t i, int ks, uint32_t salt) {
  const uint32_t m = (1u << ks) - 1u;
  return (int32_t)(((uint32_t)i << ks) + (mix32((uint32_t)i ^ salt) & m));
}

__global__ void k_set_scalar(int32_t* __restrict__ p, int32_t v) { *p = v; }

// The second channel (down counts of a tour, or element weights) adds in
// 32-bit two's complement: weight sums wrap instead of overflowing.
__device__ __forceinline__ int32_t wadd(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
__device__ __forceinline__ int32_t wsub(int32_t a, int32_t b) { return (int32_t)((uint32_t)a - (uint32_t)b); }

// start of a ranking: the continuation counter and the reached-element
// count at zero, the continuation records [begin, end) marked unused
__global__ void k_lr_init(int32_t* __restrict__ ctr, int4* __restrict__ rec, int32_t begin, int32_t end) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctr[0] = 0;
    ctr[1] = 0;
  }
  if (begin + i < end) rec[begin + i] = make_int4(-3, 0, 0, 0);
}

// ------------------------------------------------------------------ level 1
// TREE: even ids count as "down" (tree half-edges) and a leaf's two
// half-edges share one load and one store. W > 0: succ holds {successor,
// weight} pairs (one 8-byte load per step) and the weights are summed
// instead (wrapping in 32 bits); the inclusive local sum does not fit the
// 16-bit field, so the record is {sublist, local sum} (W = 1, 8 bytes) or,
// when ranks are wanted too, {sublist | local rank << 32, local sum}
// (W = 2, 16 bytes).
template <bool TREE, int W>
__device__ __forceinline__ void walk1_body(
    const int32_t* __restrict__ succ, int32_t L, const int32_t* __restrict__ heads, int32_t H, int ks,
    uint32_t salt, int32_t S, int32_t per_wave, uint64_t* __restrict__ packed, int4* __restrict__ srec,
    int32_t* __restrict__ cont_ctr, int32_t cont_base, int32_t cont_max, bool empty_ok,
    uint32_t* __restrict__ status) {
  constexpr int kStride = W > 0 ? 2 : 1;  // int32 words per element in succ
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int32_t total = S + H;
  int32_t next_id = (int32_t)min<int64_t>(wave * per_wave, total);
  const int32_t end_id = (int32_t)min<int64_t>((int64_t)next_id + per_wave, total);
  int32_t cur = -1, sub = 0, j = 0, d = 0;
  int64_t steps = 0;
  for (;;) {
    const bool idle = cur < 0;
    const uint64_t idle_mask = __ballot(idle);
    if (idle_mask != 0ull && next_id < end_id) {
      if (idle) {
        const int32_t id = next_id + __popcll(idle_mask & lanemask_lt());
        if (id < end_id) {
          if (id < S) {
            const int32_t e = splitter_of_chunk(id, ks, salt);
            if (e >= L || succ[kStride * (int64_t)e] == -2) {
              srec[id] = make_int4(-3, 0, 0, 0);  // no element here
            } else {
              cur = e; sub = id; j = 0; d = 0;
            }
          } else {
            const int32_t e = heads[id - S];
            if (e == -1 && empty_ok) {
              srec[id] = make_int4(-1, 0, 0, 0);  // an empty list
            } else if (e < 0 || e >= L || succ[kStride * (int64_t)e] == -2) {
              flag(status, ST_BAD_HEAD);
              srec[id] = make_int4(-1, 0, 0, 0);
            } else if (is_splitter(e, ks, salt)) {
              srec[id] = make_int4(e >> ks, 0, 0, 0);  // the head's own chunk splitter walks it
            } else {
              cur = e; sub = id; j = 0; d = 0;
            }
          }
        }
      }
      next_id = min(end_id, next_id + (int32_t)__popcll(idle_mask));
    }
    if (__ballot(cur >= 0) == 0ull) {
      if (next_id >= end_id) break;
      continue;
    }
    if (cur >= 0) {
      int32_t nx;
      bool pair = false;
      if (TREE && (cur & 1) == 0) {
        // A leaf's down half-edge 2c is followed by its own up half-edge
        // 2c+1; both successors share one aligned 8-byte load and both
        // records one 16-byte store, unless 2c+1 starts a sublist or the
        // pair would reach the length cap.
        const int2 sp = *reinterpret_cast<const int2*>(succ + cur);
        nx = sp.x;
        if (nx == cur + 1 && j + 2 < kCap && !is_splitter(cur + 1, ks, salt)) {
          ++d;
          const uint64_t lo = (uint64_t)(uint32_t)sub | ((uint64_t)(uint32_t)d << 48);
          *reinterpret_cast<ulonglong2*>(packed + cur) =
              make_ulonglong2(lo | ((uint64_t)(uint32_t)j << 32), lo | ((uint64_t)(uint32_t)(j + 1) << 32));
          j += 2;
          steps += 2;
          nx = sp.y;
          pair = true;
        }
      } else if (W > 0) {
        const int2 sw = *reinterpret_cast<const int2*>(succ + 2 * (int64_t)cur);
        nx = sw.x;
        d = wadd(d, sw.y);
        if (W == 1)
          packed[cur] = (uint64_t)(uint32_t)sub | ((uint64_t)(uint32_t)d << 32);
        else
          *reinterpret_cast<ulonglong2*>(packed + 2 * (int64_t)cur) =
              make_ulonglong2((uint64_t)(uint32_t)sub | ((uint64_t)(uint32_t)j << 32), (uint64_t)(uint32_t)d);
        ++j;
        ++steps;
      } else {
        nx = succ[cur];
      }
      if (!pair && W == 0) {
        if (TREE) d += ((cur & 1) == 0);
        packed[cur] = (uint64_t)(uint32_t)sub | ((uint64_t)(uint32_t)j << 32) | ((uint64_t)(uint32_t)d << 48);
        ++j;
        ++steps;
      }
      bool stop = true;
      int32_t link = -1;
      if (nx == -1) {
        link = -1;
      } else if (nx < 0 || nx >= L) {
        flag(status, ST_BAD_SUCC);
      } else if (is_splitter(nx, ks, salt)) {
        link = nx >> ks;
      } else if (steps > L) {
        flag(status, ST_OVERFLOW);
      } else if (j == kCap) {
        const int32_t nid = atomicAdd(cont_ctr, 1);
        if (nid >= cont_max) {
          flag(status, ST_OVERFLOW);
        } else {
          srec[sub] = make_int4(cont_base + nid, j, d, 0);
          sub = cont_base + nid;
          j = 0;
          d = 0;
          stop = false;
        }
      } else {
        stop = false;
      }
      if (stop) {
        srec[sub] = make_int4(link, j, d, 0);
        cur = -1;
      } else {
        cur = nx;
      }
    }
  }
}

template <bool TREE>
__global__ __launch_bounds__(kWalkThreads) void k_walk1(
    const int32_t* __restrict__ succ, int32_t L, const int32_t* __restrict__ heads, int32_t H, int ks,
    uint32_t salt, int32_t S, int32_t per_wave, uint64_t* __restrict__ packed, int4* __restrict__ srec,
    int32_t* __restrict__ cont_ctr, int32_t cont_base, int32_t cont_max, bool empty_ok,
    uint32_t* __restrict__ status) {
  walk1_body<TREE, 0>(succ, L, heads, H, ks, salt, S, per_wave, packed, srec, cont_ctr, cont_base, cont_max,
                      empty_ok, status);
}

// the same walk over {successor, weight} pairs, summing the weights; RANK:
// the records keep the local ranks too
template <bool RANK>
__global__ __launch_bounds__(kWalkThreads) void k_walk1w(
    const int32_t* __restrict__ sw, int32_t L, const int32_t* __restrict__ heads, int32_t H, int ks,
    uint32_t salt, int32_t S, int32_t per_wave, uint64_t* __restrict__ packed, int4* __restrict__ srec,
    int32_t* __restrict__ cont_ctr, int32_t cont_base, int32_t cont_max, bool empty_ok,
    uint32_t* __restrict__ status) {
  walk1_body<false, RANK ? 2 : 1>(sw, L, heads, H, ks, salt, S, per_wave, packed, srec, cont_ctr, cont_base,
                                  cont_max, empty_ok, status);
}

// ------------------------------------------------------------------ level k >= 2
// Input records rec[e] = {next, len, down}; next == -3 marks an unused element.
// Output per element: el[e] = {sublist, exclusive local len, exclusive local down}.
__global__ __launch_bounds__(kWalkThreads) void k_walkN(
    const int4* __restrict__ rec, int32_t T, int32_t hb, int32_t H, int ks, uint32_t salt, int32_t S,
    int32_t per_wave, int4* __restrict__ el, int4* __restrict__ srec, uint32_t* __restrict__ status) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int32_t total = S + H;
  int32_t next_id = (int32_t)min<int64_t>(wave * per_wave, total);
  const int32_t end_id = (int32_t)min<int64_t>((int64_t)next_id + per_wave, total);
  int32_t cur = -1, sub = 0, al = 0, ad = 0;
  int64_t steps = 0;
  for (;;) {
    const bool idle = cur < 0;
    const uint64_t idle_mask = __ballot(idle);
    if (idle_mask != 0ull && next_id < end_id) {
      if (idle) {
        const int32_t id = next_id + __popcll(idle_mask & lanemask_lt());
        if (id < end_id) {
          if (id < S) {
            const int32_t e = splitter_of_chunk(id, ks, salt);
            if (e >= T || rec[e].x == -3) {
              srec[id] = make_int4(-3, 0, 0, 0);
            } else {
              cur = e; sub = id; al = 0; ad = 0;
            }
          } else {
            const int32_t e = hb + (id - S);
            if (e < 0 || e >= T) {
              flag(status, ST_BAD_HEAD);
              srec[id] = make_int4(-1, 0, 0, 0);
            } else if (is_splitter(e, ks, salt)) {
              srec[id] = make_int4(e >> ks, 0, 0, 0);
            } else {
              cur = e; sub = id; al = 0; ad = 0;
            }
          }
        }
      }
      next_id = min(end_id, next_id + (int32_t)__popcll(idle_mask));
    }
    if (__ballot(cur >= 0) == 0ull) {
      if (next_id >= end_id) break;
      continue;
    }
    if (cur >= 0) {
      const int4 r = rec[cur];
      el[cur] = make_int4(sub, al, ad, 0);
      al += r.y;
      ad = wadd(ad, r.z);
      ++steps;
      const int32_t nx = r.x;
      bool stop = true;
      int32_t link = -1;
      if (nx == -1) {
        link = -1;
      } else if (nx < 0 || nx >= T) {
        flag(status, ST_BAD_SUCC);
      } else if (is_splitter(nx, ks, salt)) {
        link = nx >> ks;
      } else if (steps > T) {
        flag(status, ST_OVERFLOW);
      } else {
        stop = false;
      }
      if (stop) {
        srec[sub] = make_int4(link, al, ad, 0);
        cur = -1;
      } else {
        cur = nx;
      }
    }
  }
}

// ------------------------------------------------------------------ final level (LDS)
// Exclusive prefix (len, down) from each element's list head, by jumping
// predecessor pointers in LDS. T <= kLdsMax. Elements whose predecessor
// chain does not start at a head are unreachable (malformed input).
constexpr int kFinalThreads = 1024;
constexpr int kFinalPer = kLdsMax / kFinalThreads;

__global__ __launch_bounds__(kFinalThreads) void k_final_lds(const int4* __restrict__ rec, int32_t T,
                                                             int32_t hb, int32_t H, int2* __restrict__ off,
                                                             int32_t* __restrict__ reached,
                                                             const int32_t* __restrict__ expected,
                                                             uint32_t* __restrict__ status) {
  __shared__ int32_t pred[kLdsMax];
  __shared__ int32_t acl[kLdsMax];
  __shared__ int32_t acd[kLdsMax];
  __shared__ int32_t top[kLdsMax];
  const int t = threadIdx.x;
  int32_t wl[kFinalPer], wd[kFinalPer];
  bool used[kFinalPer];
  for (int k = 0; k < kFinalPer; ++k) pred[t + k * kFinalThreads] = -1;
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < kFinalPer; ++k) {
    const int e = t + k * kFinalThreads;
    int4 r = (e < T) ? rec[e] : make_int4(-3, 0, 0, 0);
    used[k] = (r.x != -3);
    wl[k] = used[k] ? r.y : 0;
    wd[k] = used[k] ? r.z : 0;
    acl[e] = wl[k];
    acd[e] = wd[k];
    top[e] = e;
    if (used[k] && r.x >= 0) {
      if (r.x < T) pred[r.x] = e;
      else bad = true;
    }
  }
  if (bad) flag(status, ST_BAD_SUCC);
  __syncthreads();
  int rounds = 1;
  while ((1 << (rounds - 1)) < T) ++rounds;
  for (int it = 0; it < rounds; ++it) {
    int32_t np[kFinalPer], nl[kFinalPer], nd[kFinalPer], nt[kFinalPer];
    for (int k = 0; k < kFinalPer; ++k) {
      const int e = t + k * kFinalThreads;
      const int32_t p = pred[e];
      if (p >= 0) {
        np[k] = pred[p];
        nl[k] = acl[e] + acl[p];
        nd[k] = wadd(acd[e], acd[p]);
        nt[k] = top[p];
      } else {
        np[k] = p; nl[k] = acl[e]; nd[k] = acd[e]; nt[k] = top[e];
      }
    }
    __syncthreads();
    for (int k = 0; k < kFinalPer; ++k) {
      const int e = t + k * kFinalThreads;
      pred[e] = np[k]; acl[e] = nl[k]; acd[e] = nd[k]; top[e] = nt[k];
    }
    __syncthreads();
  }
  int32_t mine = 0;
  bool unreached = false;
  for (int k = 0; k < kFinalPer; ++k) {
    const int e = t + k * kFinalThreads;
    if (e >= T) continue;
    const bool from_head = (top[e] >= hb && top[e] < hb + H && pred[e] < 0);
    if (used[k] && !from_head) unreached = true;
    if (from_head) mine += wl[k];
    off[e] = make_int2(acl[e] - wl[k], wsub(acd[e], wd[k]));
  }
  if (unreached) flag(status, ST_UNREACHED);
  for (int dd = 32; dd >= 1; dd >>= 1) mine += __shfl_xor(mine, dd, 64);
  if (__lane_id() == 0) atomicAdd(reached, mine);
  // every element must be reached from a head: the whole count is in once
  // all wavefronts have added theirs
  __syncthreads();
  if (threadIdx.x == 0 && expected && atomicAdd(reached, 0) != *expected) flag(status, ST_UNREACHED);
}

// Final level when many heads keep the list above kLdsMax: one lane per
// head walks its (short) list.
__global__ void k_final_walk(const int4* __restrict__ rec, int32_t T, int32_t hb, int32_t H,
                             int2* __restrict__ off, int32_t* __restrict__ reached,
                             uint32_t* __restrict__ status) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t al = 0, ad = 0;
  if (h < H) {
    int32_t e = hb + (int32_t)h;
    int64_t steps = 0;
    while (e != -1) {
      if (e < 0 || e >= T || ++steps > T) {
        flag(status, ST_BAD_SUCC);
        break;
      }
      const int4 r = rec[e];
      off[e] = make_int2(al, ad);
      al += r.y;
      ad = wadd(ad, r.z);
      e = r.x;
    }
  }
  // one add per wavefront to the shared count, not one per head
  for (int dd = 32; dd >= 1; dd >>= 1) al += __shfl_xor(al, dd, 64);
  if (__lane_id() == 0 && al) atomicAdd(reached, al);
}

__global__ void k_check_reached(const int32_t* __restrict__ reached, const int32_t* __restrict__ expected,
                                uint32_t* __restrict__ status) {
  if (expected && *reached != *expected) flag(status, ST_UNREACHED);
}

// off_k[e] = off_{k+1}[el[e].sub] + (el[e].len, el[e].down) for used elements
__global__ void k_push_down(const int4* __restrict__ rec, const int4* __restrict__ el, int32_t T,
                            const int2* __restrict__ off_up, int32_t T_up, int2* __restrict__ off,
                            uint32_t* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T) return;
  if (rec[e].x == -3) return;
  const int4 x = el[e];
  if ((uint32_t)x.x >= (uint32_t)T_up) {
    flag(status, ST_BAD_INDEX);
    off[e] = make_int2(0, 0);
    return;
  }
  const int2 o = off_up[x.x];
  off[e] = make_int2(o.x + x.y, wadd(o.y, x.z));
}

// weighted list prefix sums: sum[e] = the weight sum before e's sublist +
// the inclusive local sum; RANK: also rank as in k_rank_fix (16-byte
// records). Unused slots get rank -1 and sum 0.
template <bool RANK>
__global__ void k_scan_fix(const int2* __restrict__ sw, const uint64_t* __restrict__ packed, int32_t L,
                           const int2* __restrict__ off, int32_t T1, int32_t* __restrict__ rank,
                           int32_t* __restrict__ sum, uint32_t* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L) return;
  if (sw[e].x == -2) {
    if (RANK) rank[e] = -1;
    sum[e] = 0;
    return;
  }
  uint32_t sub, lsum, lrank = 0;
  if (RANK) {
    const ulonglong2 pk = reinterpret_cast<const ulonglong2*>(packed)[e];
    sub = (uint32_t)pk.x;
    lrank = (uint32_t)(pk.x >> 32) & 0xffffu;
    lsum = (uint32_t)pk.y;
  } else {
    const uint64_t p = packed[e];
    sub = (uint32_t)p;
    lsum = (uint32_t)(p >> 32);
  }
  if (sub >= (uint32_t)T1) {
    flag(status, ST_BAD_INDEX);
    if (RANK) rank[e] = -1;
    sum[e] = 0;
    return;
  }
  const int2 o = off[sub];
  if (RANK) rank[e] = o.x + (int32_t)lrank;
  sum[e] = wadd(o.y, (int32_t)lsum);
}

// generic rank: rank[e] = off[sub] + local rank, -1 for unused slots
__global__ void k_rank_fix(const int32_t* __restrict__ succ, const uint64_t* __restrict__ packed, int32_t L,
                           const int2* __restrict__ off, int32_t T1, int32_t* __restrict__ rank,
                           uint32_t* __restrict__ status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= L) return;
  if (succ[e] == -2) {
    rank[e] = -1;
    return;
  }
  const uint64_t p = packed[e];
  const uint32_t sub = (uint32_t)p;
  if (sub >= (uint32_t)T1) {
    flag(status, ST_BAD_INDEX);
    rank[e] = -1;
    return;
  }
  rank[e] = off[sub].x + (int32_t)((p >> 32) & 0xffffu);
}

__global__ void k_count_used(const int32_t* __restrict__ succ, int32_t L, int32_t* __restrict__ count) {
  __shared__ int32_t part[4];
  int32_t c = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L; e += (int64_t)gridDim.x * blockDim.x)
    c += (succ[e] != -2);
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if (__lane_id() == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(count, part[0] + part[1] + part[2] + part[3]);
}

// {successor, weight} pairs for the weighted walk, and the number of used
// elements (successor other than -2) as in k_count_used
__global__ void k_pair_count(const int32_t* __restrict__ succ, const int32_t* __restrict__ w, int32_t L,
                             int2* __restrict__ sw, int32_t* __restrict__ count) {
  __shared__ int32_t part[4];
  int32_t c = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = succ[e];
    sw[e] = make_int2(x, w[e]);
    c += (x != -2);
  }
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if (__lane_id() == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(count, part[0] + part[1] + part[2] + part[3]);
}

int walk_grid(int32_t total, int32_t per_wave) {
  const int64_t waves = (total + (int64_t)per_wave - 1) / per_wave;
  return (int)((waves * 64 + kWalkThreads - 1) / kWalkThreads);
}

}  // namespace

// Every buffer of a ranking is taken from the scratch before the first
// launch (the level sizes follow from the list length, the number of heads
// and the launch shape alone), so a fixed-size arena can be checked, or a
// pool request fail, before anything is enqueued.
struct LrLevel {
  int4* rec;        // this level's records (level 1: the sublist records)
  int32_t T, hb;    // records and the index of the first head record
  int4* el;         // per record: {sublist, exclusive local len, down} of the level above
  int2* off;        // per record: exclusive prefix {len, down} from its head
  int ks;           // splitter spacing of the level above (2^ks)
  int32_t S_up;     // chunk splitters of the level above
  int32_t per_wave; // sublists per wavefront of the level above's walk
};

struct LrPlan {
  int ks1 = 0;
  int32_t S1 = 0, cont_max = 0, T1 = 0, per_wave1 = 0;
  uint64_t* packed = nullptr;
  int4* rec1 = nullptr;
  int32_t* ctr = nullptr;
  std::vector<LrLevel> lv;
};

static void list_rank_plan(Ctx* c, Scratch& sc, int32_t L, int32_t H, int weighted, LrPlan* pl) {
  // Level-1 splitter spacing K = 2^ks1 (a sublist averages K elements).
  // Shorter lists keep more, shorter sublists: below about 2^25 elements the
  // walk is bound by its dependent steps rather than by line fetches, so the
  // spacing drops by half per factor 4 of length (2^24 -> 16, 2^22 -> 8,
  // 2^20 -> 4), down to 4; the context's value is the largest spacing used.
  pl->ks1 = std::min(c->lr.k1_log2, std::max(2, (floor_log2(L) - 15) / 2));
  pl->S1 = (int32_t)(((int64_t)L + (1 << pl->ks1) - 1) >> pl->ks1);
  pl->cont_max = L / kCap + H + 64;
  pl->T1 = pl->S1 + H + pl->cont_max;
  pl->packed = sc.get<uint64_t>((size_t)L * (weighted == 2 ? 2 : 1));
  pl->rec1 = sc.get<int4>((size_t)pl->T1);
  pl->ctr = sc.get<int32_t>(4);
  // sublists per wavefront: the context's value, fewer when that would leave
  // under 4096 wavefronts (at least 64, one per lane)
  pl->per_wave1 = std::min(c->lr.per_wave1, std::max(64, (pl->S1 + H) >> 12));
  pl->lv.clear();
  pl->lv.push_back({pl->rec1, pl->T1, pl->S1, nullptr, nullptr, 0, 0, 0});
  for (;;) {
    LrLevel& cur = pl->lv.back();
    if (cur.T <= kLdsMax) break;
    const int ks = c->lr.kn_log2;
    const int32_t S = (int32_t)(((int64_t)cur.T + (1 << ks) - 1) >> ks);
    const int32_t Tn = S + H;
    if ((int64_t)Tn * 2 > cur.T) break;  // many heads: shrinking stalls
    cur.el = sc.get<int4>((size_t)cur.T);
    int4* rec = sc.get<int4>((size_t)Tn);
    cur.ks = ks;
    cur.S_up = S;
    cur.per_wave = std::min(c->lr.per_waven, std::max(64, Tn >> 12));
    pl->lv.push_back({rec, Tn, S, nullptr, nullptr, 0, 0, 0});
  }
  for (auto& l : pl->lv) l.off = sc.get<int2>((size_t)l.T);
}

static int list_rank_launch(Ctx* c, const LrPlan& pl, const int32_t* succ, int32_t L, const int32_t* heads,
                            int32_t H, bool tree_weights, const int32_t* expected_reach, hipStream_t s,
                            bool empty_head_ok, int weighted) {
  const int32_t S1 = pl.S1, T1 = pl.T1, cont_max = pl.cont_max;
  hipLaunchKernelGGL(k_lr_init, dim3(ceil_div(cont_max, 256)), dim3(256), 0, s, pl.ctr, pl.rec1, S1 + H, T1);
  const dim3 g1(walk_grid(S1 + H, pl.per_wave1));
  if (tree_weights) {
    ET_PROF(c, s, "k_walk1<true>");
    hipLaunchKernelGGL(k_walk1<true>, g1, dim3(kWalkThreads), 0, s, succ, L, heads, H, pl.ks1, kSalt, S1,
                       pl.per_wave1, pl.packed, pl.rec1, pl.ctr, S1 + H, cont_max, empty_head_ok, c->d_status);
  } else if (weighted) {
    ET_PROF(c, s, weighted == 2 ? "k_walk1w<true>" : "k_walk1w<false>");
    const auto kern = weighted == 2 ? k_walk1w<true> : k_walk1w<false>;
    hipLaunchKernelGGL(kern, g1, dim3(kWalkThreads), 0, s, succ, L, heads, H, pl.ks1, kSalt, S1, pl.per_wave1,
                       pl.packed, pl.rec1, pl.ctr, S1 + H, cont_max, empty_head_ok, c->d_status);
  } else {
    ET_PROF(c, s, "k_walk1<false>");
    hipLaunchKernelGGL(k_walk1<false>, g1, dim3(kWalkThreads), 0, s, succ, L, heads, H, pl.ks1, kSalt, S1,
                       pl.per_wave1, pl.packed, pl.rec1, pl.ctr, S1 + H, cont_max, empty_head_ok, c->d_status);
  }
  // upper levels: level k's records are walked into level k+1's
  const auto& lv = pl.lv;
  for (size_t k = 0; k + 1 < lv.size(); ++k) {
    const LrLevel& cur = lv[k];
    const int32_t Tn = lv[k + 1].T;
    ET_PROF(c, s, "k_walkN");
    hipLaunchKernelGGL(k_walkN, dim3(walk_grid(Tn, cur.per_wave)), dim3(kWalkThreads), 0, s, cur.rec, cur.T,
                       cur.hb, H, cur.ks, kSalt ^ (uint32_t)(k + 1), cur.S_up, cur.per_wave, cur.el, lv[k + 1].rec,
                       c->d_status);
  }
  const LrLevel& top = lv.back();
  if (top.T <= kLdsMax) {
    ET_PROF(c, s, "k_final_lds");
    hipLaunchKernelGGL(k_final_lds, dim3(1), dim3(kFinalThreads), 0, s, top.rec, top.T, top.hb, H, top.off,
                       pl.ctr + 1, expected_reach, c->d_status);
  } else {
    {
      ET_PROF(c, s, "k_final_walk");
      hipLaunchKernelGGL(k_final_walk, dim3(ceil_div(H, 256)), dim3(256), 0, s, top.rec, top.T, top.hb, H,
                         top.off, pl.ctr + 1, c->d_status);
    }
    hipLaunchKernelGGL(k_check_reached, dim3(1), dim3(1), 0, s, pl.ctr + 1, expected_reach, c->d_status);
  }
  for (int k = (int)lv.size() - 2; k >= 0; --k) {
    ET_PROF(c, s, "k_push_down");
    hipLaunchKernelGGL(k_push_down, dim3(ceil_div(lv[k].T, 256)), dim3(256), 0, s, lv[k].rec, lv[k].el, lv[k].T,
                       lv[k + 1].off, lv[k + 1].T, lv[k].off, c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int list_rank_core(Ctx* c, Scratch& sc, const int32_t* succ, int32_t len, const int32_t* heads,
                   int32_t nheads, bool tree_weights, const int32_t* expected_reach, LRResult* out,
                   hipStream_t s, bool empty_head_ok, int weighted) {
  LrPlan pl;
  list_rank_plan(c, sc, len, nheads, weighted, &pl);
  if (sc.failed) return ET_ENOMEM;
  const int rc = list_rank_launch(c, pl, succ, len, heads, nheads, tree_weights, expected_reach, s, empty_head_ok,
                                  weighted);
  out->packed = pl.packed;
  out->off = pl.lv[0].off;
  out->nsub = pl.T1;
  return rc;
}

// Plain ranking with the scratch taken from `sc` (the pool, or an arena):
// every buffer is reserved before the first launch.
static int list_rank_with(Ctx* c, Scratch& sc, const int32_t* succ, int32_t len, const int32_t* heads,
                          int32_t nheads, int32_t* rank, hipStream_t s) {
  int32_t* expected = sc.get<int32_t>(1);
  LrPlan pl;
  list_rank_plan(c, sc, len, nheads, 0, &pl);
  if (sc.failed || sc.counting) return sc.failed ? ET_ENOMEM : ET_OK;
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, expected, 0);
  {
    ET_PROF(c, s, "k_count_used");
    hipLaunchKernelGGL(k_count_used, dim3(std::min(ceil_div(len, 256), 2048)), dim3(256), 0, s, succ, len,
                       expected);
  }
  int rc = list_rank_launch(c, pl, succ, len, heads, nheads, false, expected, s, false, 0);
  if (rc) return rc;
  {
    ET_PROF(c, s, "k_rank_fix");
    hipLaunchKernelGGL(k_rank_fix, dim3(ceil_div(len, 256)), dim3(256), 0, s, succ, pl.packed, len, pl.lv[0].off,
                       pl.T1, rank, c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

int list_rank_generic(Ctx* c, const int32_t* succ, int32_t len, const int32_t* heads, int32_t nheads,
                      int32_t* rank, hipStream_t s) {
  if (len == 0) return ET_OK;
  Scratch sc(c, s);
  return list_rank_with(c, sc, succ, len, heads, nheads, rank, s);
}

size_t list_rank_plan_bytes(const Ctx* c, int32_t len, int32_t nheads, int weighted) {
  if (len == 0) return 0;
  Ctx shape;  // the plan reads only the launch shape
  shape.lr = c ? c->lr : LrShape{};
  Scratch count(&shape, nullptr, nullptr, 0);
  LrPlan pl;
  list_rank_plan(&shape, count, len, nheads, weighted, &pl);
  // as pool blocks: every block, the last one too, takes whole 256-byte units
  return (count.used + 255) & ~(size_t)255;
}

size_t list_rank_scratch_bytes(Ctx* c, int32_t len, int32_t nheads) {
  if (len == 0) return 0;
  Scratch count(c, nullptr, nullptr, 0);
  (void)list_rank_with(c, count, nullptr, len, nullptr, nheads, nullptr, nullptr);
  return count.used;
}

int list_rank_arena(Ctx* c, void* arena, size_t bytes, const int32_t* succ, int32_t len, const int32_t* heads,
                    int32_t nheads, int32_t* rank, hipStream_t s) {
  if (len == 0) return ET_OK;
  Scratch sc(c, s, arena, bytes);
  return list_rank_with(c, sc, succ, len, heads, nheads, rank, s);
}

int list_scan_generic(Ctx* c, const int32_t* succ, const int32_t* weights, int32_t len, const int32_t* heads,
                      int32_t nheads, int32_t* rank, int32_t* sum, hipStream_t s) {
  if (len == 0) return ET_OK;
  Scratch sc(c, s);
  int32_t* expected = sc.get<int32_t>(1);
  int2* sw = sc.get<int2>((size_t)len);
  if (sc.failed) return ET_ENOMEM;
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, s, expected, 0);
  {
    ET_PROF(c, s, "k_pair_count");
    hipLaunchKernelGGL(k_pair_count, dim3(std::min(ceil_div(len, 256), 2048)), dim3(256), 0, s, succ, weights,
                       len, sw, expected);
  }
  LRResult r;
  int rc = list_rank_core(c, sc, reinterpret_cast<const int32_t*>(sw), len, heads, nheads, false, expected, &r, s,
                          false, rank ? 2 : 1);
  if (rc) return rc;
  {
    ET_PROF(c, s, rank ? "k_scan_fix<true>" : "k_scan_fix<false>");
    const auto kern = rank ? k_scan_fix<true> : k_scan_fix<false>;
    hipLaunchKernelGGL(kern, dim3(ceil_div(len, 256)), dim3(256), 0, s, sw, r.packed, len, r.off, r.nsub, rank, sum,
                       c->d_status);
  }
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
