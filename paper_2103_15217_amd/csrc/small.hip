// Many small trees built and queried in one launch (Section 3.3: a batch of
// LCA queries answered on trees that are preprocessed once; Section 2 and
// 3.1 for what each tree goes through).
//
// A workgroup of 1024 lanes (256 when no tree has more than 1024 nodes and
// the trees outnumber the compute units) takes one tree at a time from an
// atomic counter, in the caller's order when one is given
// (the grid is sized to what stays resident, so the launch is persistent)
// and runs the tree's whole path in LDS, reading only its parent array and
// its queries from HBM and writing only the answers (and, on request, the
// node statistics):
//   1. parents into LDS, checked (one root, ids in range, no self parent);
//   2. children grouped by parent in ascending id order: a stable LSD radix
//      sort of the child ids by parent id (7-bit digits, the root's key n
//      sorts last), ranks within a wavefront by ballots and per-wavefront
//      digit counters scanned digit-major;
//   3. successors over the grouped order (next sibling, else back up to the
//      parent; the first child under its parent's down half-edge), the same
//      rule as the multi-kernel build;
//   4. list ranking of the tour: both half-edges of every 2^k-th node (and
//      the head) start a sublist that one lane walks, recording its length
//      and down count, and per half-edge its rank and inclusive down count
//      within the sublist and (in place of its successor, which no other
//      lane reads) the sublist's index; pointer jumping over the sublists
//      gives suffix sums, hence each sublist's offset, which one pass over
//      the nodes adds to the half-edges' local values. The tour must reach
//      all 2(n-1) half-edges;
//   5. depth, preorder, size and inlabel per node from the two ranks of its
//      half-edges, the head table and parent path labels per inlabel path,
//      each node's ascendant from its chain of parent path labels;
//   6. the tree's queries by the Schieber-Vishkin rule on the LDS tables.
// Ids are below 2^16 here (a tree has at most 4096 nodes, 8192 half-edges),
// so the LDS tables hold 16-bit entries.
#include "et_internal.hpp"

namespace et {
namespace {

// Two shapes: 1024 lanes for trees of up to 4096 nodes, 256 lanes (four
// workgroups in the place of one) when no tree exceeds 1024 nodes. Either
// way a lane holds at most kRoundsMax nodes of its tree.
constexpr int kFMax = 4096;         // nodes per tree at most
constexpr int kFSmall = 1024;       // nodes per tree at most for the 256-lane shape
constexpr int kRoundsMax = 4;
constexpr int kWavesMax = 16;       // wavefronts per workgroup at most
constexpr uint16_t kEnd = 0xffff;   // list end, no node, unused label
constexpr uint16_t kNoSucc = 0xfffe;  // a half-edge id of the root (not on the tour)
constexpr int kDigitBits = 7;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kCP = kDigits + 1;    // a wavefront's digit counters: one row, padded so rows start in other banks
constexpr int kSubMax = 1025;       // sublists: at most 1024 regular ones and the head's
constexpr int kQPer = 4;            // queries a lane loads before answering them

__host__ __device__ inline uint32_t al64(uint32_t x) { return (x + 63u) & ~63u; }

// Byte offsets of the LDS regions for trees of at most N nodes (N a
// multiple of 64). Regions are reused as the phases go:
//   p   parent u16[N]                                  (whole tree)
//   rb  successor u16[2N] (an entry becomes its half-edge's sublist index
//       once walked), later head u32[N+1]
//   rc  radix counters u32[waves][kDigits + 1], later per node the rank of its
//       two half-edges and the down count at the first (u16[N] each),
//       later parent path labels u16[N+1]
//   rd  sort buffers u16[2][N], then the sublists (next u16[2][kSubMax],
//       length and down count packed u32[2][kSubMax]), later inlabel,
//       ascendant, depth u16[N] each
//   sc  scalars and wavefront sums
// (at N = 4096 about 73 KB: two 1024-lane workgroups share a compute unit)
struct SmallLayout {
  uint32_t p, rb, rc, rd, rf, sc, total;
};

__host__ __device__ inline SmallLayout small_layout(uint32_t N) {
  SmallLayout L;
  uint32_t at = 0;
  L.p = at;
  at += al64(2 * N);
  L.rb = at;
  at += al64(4 * N + 4);
  L.rc = at;
  at += al64(max(6 * N + 2, (uint32_t)(kCP * kWavesMax * 4)));
  L.rd = at;
  L.rf = at;  // the sublists live between the sort and the node statistics
  at += al64(max(6 * N, (uint32_t)(12 * kSubMax)));
  L.sc = at;
  at += 256;
  L.total = at;
  return L;
}

enum { S_ROOT = 0, S_NROOTS, S_BAD, S_HEAD, S_TREE, S_FAIL, S_WSUM = 16 };  // int32 scalar slots

__device__ __forceinline__ int clog2(uint32_t x) { return x <= 1 ? 0 : 32 - __clz((int)(x - 1)); }

// lanes of the wavefront whose digit equals this lane's (among valid lanes)
__device__ __forceinline__ uint64_t match_digit(bool valid, uint32_t d) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kDigitBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__device__ __forceinline__ uint16_t root_key(uint16_t p, uint32_t n) { return p == kEnd ? (uint16_t)n : p; }

template <int kFT>
__global__ __launch_bounds__(kFT, kFT == 1024 ? 8 : 1) void k_small_batch(
    const int32_t* __restrict__ parent, const int64_t* __restrict__ off, int32_t T, int64_t n_total, uint32_t N,
    int32_t nmax, const int64_t* __restrict__ qoff, int64_t q_total, const int32_t* __restrict__ qx,
    const int32_t* __restrict__ qy, int32_t* __restrict__ out, int32_t* __restrict__ depth_out,
    int32_t* __restrict__ pre_out, int32_t* __restrict__ size_out, const int32_t* __restrict__ order,
    uint32_t* __restrict__ counters, uint32_t* __restrict__ status) {
  constexpr int kFW = kFT / 64;  // wavefronts per workgroup
  static_assert(kFT * kRoundsMax >= kFSmall && kFW <= kWavesMax, "a lane holds at most kRoundsMax nodes");
  extern __shared__ __align__(16) unsigned char lds[];
  const SmallLayout L = small_layout(N);
  uint16_t* P = reinterpret_cast<uint16_t*>(lds + L.p);
  uint16_t* SUCC = reinterpret_cast<uint16_t*>(lds + L.rb);
  uint32_t* HEAD = reinterpret_cast<uint32_t*>(lds + L.rb);
  uint32_t* CNT = reinterpret_cast<uint32_t*>(lds + L.rc);
  uint16_t* R0 = reinterpret_cast<uint16_t*>(lds + L.rc);  // rank of 2c
  uint16_t* R1 = R0 + N;                                     // rank of 2c + 1
  uint16_t* D0 = R0 + 2 * N;                                 // down count through 2c
  uint16_t* PLAB = reinterpret_cast<uint16_t*>(lds + L.rc);
  uint16_t* ORD0 = reinterpret_cast<uint16_t*>(lds + L.rd);
  uint16_t* ORD1 = ORD0 + N;
  uint16_t* INL = reinterpret_cast<uint16_t*>(lds + L.rd);
  uint16_t* ASC = INL + N;
  uint16_t* DEP = ASC + N;
  // sublist next, and length << 16 | down count (both below 2^16, so one
  // 32-bit add sums both), two buffers each (pointer jumping)
  uint16_t* SUB = reinterpret_cast<uint16_t*>(lds + L.rf);
  uint32_t* LDa = reinterpret_cast<uint32_t*>(lds + L.rf + 4 * kSubMax);
#define NX(b) (SUB + (b) * kSubMax)
#define LD(b) (LDa + (b) * kSubMax)
  int32_t* SC = reinterpret_cast<int32_t*>(lds + L.sc);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  if (blockIdx.x == 0 && tid == 0) {
    if (off[0] != 0 || off[T] != n_total) flag(status, ST_BAD_PARENT);
    if (qoff[0] != 0 || qoff[T] != q_total) flag(status, ST_BAD_QUERY);
  }
  for (;;) {
    if (tid == 0) SC[S_TREE] = (int32_t)atomicAdd(&counters[0], 1u);
    __syncthreads();
    const int32_t k = SC[S_TREE];
    if (k >= T) break;
    const int32_t t = order ? order[k] : k;  // the k-th tree taken
    const bool t_ok = (uint32_t)t < (uint32_t)T;
    if (!t_ok && tid == 0) flag(status, ST_BAD_PARENT);
    const int64_t base = t_ok ? off[t] : 0, nt = t_ok ? off[t + 1] - base : 0;
    const int64_t qb = t_ok ? qoff[t] : 0, nq = t_ok ? qoff[t + 1] - qb : 0;
    const bool q_ok = t_ok && qb >= 0 && nq >= 0 && qb + nq <= q_total;
    if (t_ok && !q_ok && tid == 0) flag(status, ST_BAD_QUERY);
    const bool tree_ok = t_ok && base >= 0 && nt >= 1 && nt <= (int64_t)nmax && base + nt <= n_total;
    if (!tree_ok && tid == 0) flag(status, ST_BAD_PARENT);
    const uint32_t n = tree_ok ? (uint32_t)nt : 0u;

    // 1. parents
    if (tid == 0) {
      SC[S_NROOTS] = 0;
      SC[S_BAD] = 0;
      SC[S_FAIL] = tree_ok ? 0 : 1;
      SC[S_HEAD] = -1;
    }
    __syncthreads();
    int32_t praw[kRoundsMax];  // all of a lane's parent loads first
#pragma unroll
    for (int r = 0; r < kRoundsMax; ++r) {
      const uint32_t c = tid + r * kFT;
      praw[r] = c < n ? parent[base + c] : 0;
    }
#pragma unroll
    for (int r = 0; r < kRoundsMax; ++r) {
      const uint32_t c = tid + r * kFT;
      if (c >= n) break;
      const int32_t p = praw[r];
      if (p == -1) {
        P[c] = kEnd;
        atomicAdd(&SC[S_NROOTS], 1);
        SC[S_ROOT] = (int32_t)c;
      } else if (p >= 0 && (uint32_t)p < n && (uint32_t)p != c) {
        P[c] = (uint16_t)p;
      } else {
        P[c] = 0;
        SC[S_BAD] = 1;
      }
    }
    __syncthreads();
    if (tree_ok && (SC[S_NROOTS] != 1 || SC[S_BAD])) {
      if (tid == 0) {
        flag(status, SC[S_BAD] ? ST_BAD_PARENT : ST_ROOTS);
        SC[S_FAIL] = 1;
      }
    }
    __syncthreads();
    const uint32_t root = (uint32_t)SC[S_ROOT];
    const uint32_t E = 2 * n;

    if (!SC[S_FAIL] && n > 1) {
      // 2. stable radix sort of child ids by parent id
      for (uint32_t i = tid; i < n; i += kFT) ORD0[i] = (uint16_t)i;
      uint16_t* src = ORD0;
      uint16_t* dst = ORD1;
      const int kbits = 32 - __clz((int)n);   // bits of the largest key (n, the root's)
      const uint32_t seg = ((n + kFT - 1) / kFT) * 64;  // elements per wavefront, whole rounds
      const int rounds = (int)(seg / 64);
      const uint64_t below = lanemask_lt();
      for (int sh = 0; sh < kbits; sh += kDigitBits) {
        for (int i = tid; i < kCP * kFW; i += kFT) CNT[i] = 0;
        __syncthreads();
        uint32_t lr[kRoundsMax], dg[kRoundsMax];
        uint16_t vv[kRoundsMax];
#pragma unroll
        for (int r = 0; r < kRoundsMax; ++r) {
          if (r >= rounds) break;
          const uint32_t idx = w * seg + r * 64 + lane;
          const bool valid = idx < n;
          const uint16_t v = valid ? src[idx] : (uint16_t)0;
          const uint32_t d = valid ? ((uint32_t)root_key(P[v], n) >> sh) & (kDigits - 1) : 0u;
          const uint64_t peers = match_digit(valid, d);
          uint32_t old = 0;
          if (valid) old = CNT[w * kCP + d];
          if (valid && lane == __ffsll((unsigned long long)peers) - 1)
            CNT[w * kCP + d] = old + (uint32_t)__popcll(peers);
          lr[r] = old + (uint32_t)__popcll(peers & below);
          dg[r] = d;
          vv[r] = v;
        }
        __syncthreads();
        // digit-major: digit d of wavefront w is number d * kFW + w in the scan
        wg_scan_excl_at<kFT>(CNT, kDigits * kFW, SC + S_WSUM, [](int i) { return (i % kFW) * kCP + i / kFW; });
#pragma unroll
        for (int r = 0; r < kRoundsMax; ++r) {
          if (r >= rounds) break;
          const uint32_t idx = w * seg + r * 64 + lane;
          if (idx < n) dst[CNT[w * kCP + dg[r]] + lr[r]] = vv[r];
        }
        __syncthreads();
        uint16_t* tmp = src;
        src = dst;
        dst = tmp;
      }
      const uint16_t* ord = src;

      // 3. successors; the root sorts last (position n-1)
      for (uint32_t e = tid; e < E; e += kFT)
        SUCC[e] = ((e >> 1) == root) ? kNoSucc : ((e & 1u) ? kEnd : (uint16_t)(e + 1));
      __syncthreads();
      for (uint32_t k = tid; k + 1 < n; k += kFT) {
        const uint32_t c = ord[k];
        const uint16_t p = P[c];
        uint16_t nxt;
        if (k + 2 < n && P[ord[k + 1]] == p) nxt = (uint16_t)(2 * ord[k + 1]);
        else nxt = (p == root) ? kEnd : (uint16_t)(2 * p + 1);
        SUCC[2 * c + 1] = nxt;
        if (k == 0 || P[ord[k - 1]] != p) {
          if (p == root) SC[S_HEAD] = (int32_t)(2 * c);
          else SUCC[2 * p] = (uint16_t)(2 * c);
        }
      }
      __syncthreads();
      if (SC[S_HEAD] < 0) {  // the root has no child: the other nodes form cycles
        if (tid == 0) {
          flag(status, ST_UNREACHED);
          SC[S_FAIL] = 1;
        }
      }
      __syncthreads();
    }
    if (!SC[S_FAIL] && n > 1) {
      // 4. sublists: both half-edges of every 2^m-th node id start one (so
      // the runs down into and up out of a subtree both meet splitters),
      // and so does the head; at most 1024 regular ones
      const int m = max(0, clog2(n) - 9);
      const uint32_t M = (1u << m) - 1u;
      const uint32_t Sreg = 2 * ((n + M) >> m);
      const uint32_t S = Sreg + 1;
      const uint32_t head = (uint32_t)SC[S_HEAD];
      const uint32_t hsub = ((head >> 1) & M) ? Sreg : (((head >> 1) >> m) << 1);
      for (uint32_t s = tid; s < S; s += kFT) {
        const uint32_t e0 = (s == Sreg) ? head : ((((s >> 1) << m) << 1) | (s & 1u));
        const bool valid = (s == Sreg) ? ((head >> 1) & M) != 0 : (e0 < E && SUCC[e0] != kNoSucc);
        uint32_t len = 0, dn = 0, nxs = kEnd;
        if (valid) {
          uint32_t e = e0;
          for (;;) {
            const uint32_t nx = SUCC[e];
            SUCC[e] = (uint16_t)s;  // only this lane reads e's successor
            if (e & 1u) {
              R1[e >> 1] = (uint16_t)len;
            } else {
              R0[e >> 1] = (uint16_t)len;
              D0[e >> 1] = (uint16_t)(dn + 1);
            }
            ++len;
            dn += !(e & 1u);
            if (nx == kEnd) break;
            if (nx >= E || len >= E) {
              SC[S_BAD] = 1;
              break;
            }
            if (!((nx >> 1) & M)) {
              nxs = (((nx >> 1) >> m) << 1) | (nx & 1u);
              break;
            }
            e = nx;
          }
        }
        NX(0)[s] = (uint16_t)nxs;
        LD(0)[s] = (len << 16) | dn;
      }
      __syncthreads();
      // suffix sums along the sublist list by pointer jumping
      int cur = 0;
      const int jumps = clog2(S) + 1;
      for (int it = 0; it < jumps; ++it) {
        for (uint32_t s = tid; s < S; s += kFT) {
          const uint16_t nx = NX(cur)[s];
          if (nx != kEnd && nx < S) {
            NX(cur ^ 1)[s] = NX(cur)[nx];
            LD(cur ^ 1)[s] = LD(cur)[s] + LD(cur)[nx];
          } else {
            NX(cur ^ 1)[s] = kEnd;
            LD(cur ^ 1)[s] = LD(cur)[s];
          }
        }
        __syncthreads();
        cur ^= 1;
      }
      const uint32_t total = LD(cur)[hsub] >> 16, total_dn = LD(cur)[hsub] & 0xffffu;
      if (tid == 0 && (SC[S_BAD] || total != E - 2)) {
        flag(status, ST_UNREACHED);
        SC[S_FAIL] = 1;
      }
      __syncthreads();
      if (!SC[S_FAIL]) {
        // each half-edge's rank and inclusive down count: its sublist's
        // offset plus its value within the sublist
        for (uint32_t c = tid; c < n; c += kFT) {
          if (c == root) continue;
          const uint32_t s0 = SUCC[2 * c], s1 = SUCC[2 * c + 1];
          if (s0 >= S || s1 >= S) {  // not walked: cannot happen once the tour covers every half-edge
            SC[S_BAD] = 1;
            continue;
          }
          const uint32_t l0 = LD(cur)[s0];
          R0[c] = (uint16_t)(R0[c] + total - (l0 >> 16));
          D0[c] = (uint16_t)(D0[c] + total_dn - (l0 & 0xffffu));
          R1[c] = (uint16_t)(R1[c] + total - (LD(cur)[s1] >> 16));
        }
      }
      __syncthreads();
      if (tid == 0 && SC[S_BAD] && !SC[S_FAIL]) {
        flag(status, ST_UNREACHED);
        SC[S_FAIL] = 1;
      }
      __syncthreads();
    }

    if (!SC[S_FAIL]) {
      // 5. node statistics and inlabels (RD's sort buffers are dead)
      for (uint32_t c = tid; c < n; c += kFT) {
        int32_t dep, pre, size;
        if (c == root) {
          dep = 0;
          pre = 0;
          size = (int32_t)n;
        } else {
          const int32_t r0 = R0[c], d0 = D0[c], r1 = R1[c];
          pre = d0;
          dep = 2 * d0 - r0 - 1;
          size = (r1 - r0 + 1) >> 1;
        }
        INL[c] = (uint16_t)inlabel_of(pre, size);
        DEP[c] = (uint16_t)dep;
        if (depth_out) depth_out[base + c] = dep;
        if (pre_out) pre_out[base + c] = pre;
        if (size_out) size_out[base + c] = size;
      }
      __syncthreads();  // the ranks are dead from here: PLAB takes RC
      for (uint32_t I = tid; I <= n; I += kFT) PLAB[I] = kEnd;
      __syncthreads();
      // path tops: head[label] = {parent of the top, its depth}, plab = the parent's label
      for (uint32_t v = tid; v < n; v += kFT) {
        const uint16_t inl = INL[v];
        const uint16_t p = P[v];
        const bool is_root = v == root;
        const uint16_t pinl = is_root ? (uint16_t)0 : INL[p];
        if (is_root || pinl != inl) {
          if (inl >= 1 && inl <= n) {
            HEAD[inl] = (uint32_t)(is_root ? kEnd : p) | ((uint32_t)(uint16_t)(DEP[v] - 1) << 16);
            PLAB[inl] = pinl;
          } else {
            SC[S_BAD] = 1;
          }
        }
      }
      __syncthreads();
      // ascendant of each node: the level bits of the labels on its chain of
      // parent path labels (levels strictly rise along it: at most 16 links)
      for (uint32_t v = tid; v < n; v += kFT) {
        uint32_t I = INL[v], acc = 0;
        for (int k = 0; k < 16; ++k) {
          if (I < 1 || I > n) {  // flagged where the labels were made
            SC[S_BAD] = 1;
            break;
          }
          const int lv = __ffs((int)I) - 1;
          acc |= 1u << lv;
          const uint32_t pl = PLAB[I];
          if (pl == 0) break;  // the root's path
          if (pl > n || (__ffs((int)pl) - 1) <= lv) {
            SC[S_BAD] = 1;
            break;
          }
          I = pl;
        }
        ASC[v] = (uint16_t)acc;
      }
      __syncthreads();
      if (tid == 0 && SC[S_BAD]) flag(status, ST_BAD_INDEX);
    }

    // 6. queries
    if (q_ok) {
      const bool fail = SC[S_FAIL] != 0;
      for (int64_t i0 = qb; i0 < qb + nq; i0 += (int64_t)kQPer * kFT) {
        int32_t xs[kQPer], ys[kQPer];  // a lane's query loads first, then the lookups
#pragma unroll
        for (int j = 0; j < kQPer; ++j) {
          const int64_t i = i0 + (int64_t)j * kFT + tid;
          xs[j] = i < qb + nq ? qx[i] : 0;
          ys[j] = i < qb + nq ? qy[i] : 0;
        }
#pragma unroll
        for (int j = 0; j < kQPer; ++j) {
          const int64_t i = i0 + (int64_t)j * kFT + tid;
          if (i >= qb + nq) break;
          const int32_t x = xs[j], y = ys[j];
          int32_t r = -1;
          if ((uint32_t)x >= n || (uint32_t)y >= n) {
            if (!fail) flag(status, ST_BAD_QUERY);
          } else if (!fail) {
            const uint32_t a = INL[x], b = INL[y];
            const int32_t dx = DEP[x], dy = DEP[y];
            if (a == b) {
              r = dx <= dy ? x : y;
            } else {
              const int ha = __ffs((int)a) - 1, hb = __ffs((int)b) - 1;
              const int lb = max(max(ha, hb), 31 - __clz((int)(a ^ b)));  // b-level of the labels' LCA
              const uint32_t ax = ASC[x], ay = ASC[y];
              const uint32_t common = ax & ay & (~0u << lb);
              if (common == 0u) {
                flag(status, ST_BAD_INDEX);
              } else {
                const int jl = __ffs((int)common) - 1;
                const uint32_t low = (1u << jl) - 1u;
                int32_t xv = x, xd = dx, yv = y, yd = dy;
                if (ha != jl) {
                  const int k = 31 - __clz((int)(ax & low));
                  const uint32_t wl = ((a >> (k + 1)) << (k + 1)) | (1u << k);
                  const uint32_t h = HEAD[min(wl, n)];
                  xv = (h & 0xffffu) == kEnd ? -1 : (int32_t)(h & 0xffffu);
                  xd = (int32_t)(int16_t)(h >> 16);
                }
                if (hb != jl) {
                  const int k = 31 - __clz((int)(ay & low));
                  const uint32_t wl = ((b >> (k + 1)) << (k + 1)) | (1u << k);
                  const uint32_t h = HEAD[min(wl, n)];
                  yv = (h & 0xffffu) == kEnd ? -1 : (int32_t)(h & 0xffffu);
                  yd = (int32_t)(int16_t)(h >> 16);
                }
                r = xd <= yd ? xv : yv;
              }
            }
          }
          out[i] = r;
        }
      }
    }
    __syncthreads();  // the tables and SC[S_TREE] are rewritten by the next tree
  }
  // the last workgroup out resets the counters for the next launch
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(&counters[1], 1u) == gridDim.x - 1) {
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
#undef NX
#undef LD
}

}  // namespace

size_t small_batch_lds_bytes(int32_t max_nodes) {
  const uint32_t N = al64((uint32_t)std::max(max_nodes, 1));
  return small_layout(N).total;
}

int small_batch_run(Ctx* c, const int32_t* parent, const int64_t* off, int32_t T, int64_t n_total,
                    int32_t max_nodes, const int64_t* qoff, const int32_t* qx, const int32_t* qy, int64_t q_total,
                    int32_t* out, int32_t* depth, int32_t* pre, int32_t* size, const int32_t* order,
                    hipStream_t s) {
  if (T == 0) return ET_OK;
  if (max_nodes < 1 || max_nodes > kFMax) return ET_ESIZE;
  const uint32_t N = al64((uint32_t)max_nodes);
  const uint32_t lds = small_layout(N).total;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) return ET_EHIP;
  // 256 lanes hold four trees where 1024 lanes hold one; worth it once there
  // are more trees than compute units (one 1024-lane workgroup fits a unit)
  const bool narrow = max_nodes <= kFSmall && T > cus;
  const int threads = narrow ? 256 : 1024;
  const void* kern = narrow ? reinterpret_cast<const void*>(k_small_batch<256>)
                            : reinterpret_cast<const void*>(k_small_batch<1024>);
  int grid = 0;
  const int rc = persistent_grid(kern, threads, lds, T, &grid);
  if (rc) return rc;
  ET_PROF(c, s, "k_small_batch");
  if (narrow)
    hipLaunchKernelGGL(k_small_batch<256>, dim3(grid), dim3(256), lds, s, parent, off, T, n_total, N, max_nodes,
                       qoff, q_total, qx, qy, out, depth, pre, size, order, c->d_fused, c->d_status);
  else
    hipLaunchKernelGGL(k_small_batch<1024>, dim3(grid), dim3(1024), lds, s, parent, off, T, n_total, N, max_nodes,
                       qoff, q_total, qx, qy, out, depth, pre, size, order, c->d_fused, c->d_status);
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
