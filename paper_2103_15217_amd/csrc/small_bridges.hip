// Bridges of many small graphs in one launch (Section 4.1, Tarjan-Vishkin,
// for a batch of instances as the tree batch of Section 3.3 does for LCA).
//
// A workgroup of 1024 lanes takes one graph at a time from an atomic counter
// (in the caller's order when one is given)
// (a persistent grid sized to what stays resident) and runs the whole method
// on it in LDS, reading only its CSR from HBM and writing only its mask words
// and its bridge count:
//   1. row pointers and columns into LDS, checked (monotone rows from 0 to
//      the slot count, sorted rows, every slot's twin present);
//   2. spanning forest: union-find over the first slot of every run of equal
//      columns (u < w), the larger root linked under the smaller by an LDS
//      compare-and-swap; a successful link marks the slot and its twin as a
//      forest edge;
//   3. the forest's half-edges per vertex in row order, twins by binary
//      search, succ = next(twin) cyclically per vertex (Section 2.1), the
//      component tours cut before each root's first half-edge and chained in
//      root order;
//   4. ranks along the chained tour by pointer jumping, a half-edge going
//      down iff it comes before its twin, preorder from a scan of the down
//      flags in tour order, subtree sizes from the two ranks of each edge;
//   5. per vertex the min / max preorder over its non-forest slots (itself
//      included), low / high as range min / max over the subtree interval
//      (in-block prefix and suffix extremes plus a sparse table over
//      32-position blocks), and the bridge test: low == pre and high ==
//      pre + size - 1, for an edge of multiplicity one.
// Ids, slots, ranks and preorder numbers are below 2^16 here (a graph has at
// most 1024 vertices and 8192 CSR slots), so the LDS tables hold 16-bit
// entries.
#include "et_internal.hpp"

namespace et {
namespace {

constexpr int kBT = 1024;            // lanes per workgroup
constexpr int kBW = kBT / 64;
constexpr int kGMaxV = 1024;         // vertices of a graph at most
constexpr int kGMaxS = 8192;         // CSR slots of a graph at most
constexpr uint16_t kNil = 0xffff;    // list end, no slot
constexpr int kRB = 32;              // range-minimum block (positions)
constexpr int kRLev = 6;             // sparse-table levels over at most 32 blocks

__host__ __device__ inline uint32_t a64(uint32_t x) { return (x + 63u) & ~63u; }

// LDS regions for graphs of at most N vertices and M slots (multiples of 64):
//   rp u16[N+1], col u16[M]                   the CSR
//   uf u32[N]                                 union-find parents, then roots
//   tf, mb u32[M/32]                          forest-slot bits, bridge bits
//   tptr u16[N+1], hs/tsl/tnb/ttw u16[2N]     forest half-edges per vertex
//                                             (tour order later takes hs,
//                                             then each vertex's parent and
//                                             the slot of its edge's twin)
//   row u16[M]                                the row of every slot while
//                                             the CSR is checked and the
//                                             forest made; then
//   nx, dd: u32[2N] each                      the successors (u16, in dd),
//                                             then pointer jumping over
//                                             next << 16 | distance; later the
//                                             extremes per preorder position:
//                                             amn/amx u32[N], pmn/smn/pmx/smx u16[N]
//   dc u32[2N]                                scans (degrees, roots, down flags)
//   pre/size/pslot/ridx/rl u16[N]             per vertex; root list
//   st u16[2][kRLev][N/32]                    sparse tables over 32-position blocks
// (about 77 KB at 1024 vertices and 8192 slots: two workgroups per compute unit)
struct BLayout {
  uint32_t rp, col, uf, tf, mb, tptr, hs, tsl, tnb, ttw, nx, dd, tour, dc, pre, size, pslot, ridx, rl, amn, amx,
      pmn, smn, pmx, smx, row, st, sc, total;
};

__host__ __device__ inline BLayout blayout(uint32_t N, uint32_t M) {
  BLayout L;
  uint32_t at = 0;
  auto take = [&](uint32_t bytes) {
    const uint32_t r = at;
    at += a64(bytes);
    return r;
  };
  L.rp = take(2 * (N + 1));
  L.col = take(2 * M);
  L.uf = take(4 * N);
  L.tf = take(M / 8 + 4);
  L.mb = take(M / 8 + 4);
  L.tptr = take(2 * (N + 1));
  L.hs = take(4 * N);
  L.tour = L.hs;  // the half-edges' rows are dead once successors and twins are known
  L.tsl = take(4 * N);
  L.tnb = take(4 * N);
  L.ttw = take(4 * N);
  // pointer jumping, then (once preorder and sizes are known) the extremes
  L.nx = at;
  L.dd = at + 8 * N;
  L.amn = at;
  L.amx = at + 4 * N;
  L.pmn = at + 8 * N;
  L.smn = at + 10 * N;
  L.pmx = at + 12 * N;
  L.smx = at + 14 * N;
  L.row = at;  // before any of these: the row of every slot, u16[M]
  at += a64(max(16 * N, 2 * M));
  L.dc = take(8 * N);
  L.pre = take(2 * N);
  L.size = take(2 * N);
  L.pslot = take(2 * N);
  L.ridx = take(2 * N);
  L.rl = take(2 * N);
  L.st = take(2 * 2 * kRLev * (N / kRB + 1));
  L.sc = take(256);
  L.total = at;
  return L;
}

enum { B_GRAPH = 0, B_FAIL, B_BAD, B_ET, B_NR, B_HEAD, B_CNT, B_TOT, B_WSUM = 16 };

// first index in [lo, hi) of the sorted u16 array a with a[i] >= x
__device__ __forceinline__ uint32_t lower16(const uint16_t* a, uint32_t lo, uint32_t hi, uint32_t x) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// row of slot k: the last v < n with rp[v] <= k (rows may be empty)
__device__ __forceinline__ uint32_t row_of_slot(const uint16_t* rp, uint32_t n, uint32_t k) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (rp[mid] <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Inclusive prefix maximum of the u16 values a[0..m) in place by the
// workgroup; wsum: kBW slots.
__device__ inline void wg_prefix_max_u16(uint16_t* a, int m, int32_t* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int per = (m + kBT - 1) / kBT;
  const int lo = min(tid * per, m), hi = min(lo + per, m);
  uint32_t mx = 0;
  for (int i = lo; i < hi; ++i) mx = max(mx, (uint32_t)a[i]);
  uint32_t incl = mx;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t v = __shfl_up(incl, d);
    if (lane >= d) incl = max(incl, v);
  }
  if (lane == 63) wsum[w] = (int32_t)incl;
  __syncthreads();
  if (tid < 64) {
    uint32_t x = tid < kBW ? (uint32_t)wsum[tid] : 0u;
#pragma unroll
    for (int d = 1; d < kBW; d <<= 1) {
      const uint32_t y = __shfl_up(x, d);
      if (lane >= d) x = max(x, y);
    }
    const uint32_t before = __shfl_up(x, 1);  // the waves before this one
    if (tid < kBW) wsum[tid] = (int32_t)(tid == 0 ? 0u : before);
  }
  __syncthreads();
  const uint32_t lanes_before = __shfl_up(incl, 1);
  uint32_t run = max((uint32_t)wsum[w], lane == 0 ? 0u : lanes_before);
  for (int i = lo; i < hi; ++i) {
    run = max(run, (uint32_t)a[i]);
    a[i] = (uint16_t)run;
  }
  __syncthreads();
}

__device__ __forceinline__ uint32_t uf_find(uint32_t* uf, uint32_t x) {
  for (;;) {
    const uint32_t p = uf[x];
    if (p == x) return x;
    const uint32_t g = uf[p];
    if (g != p) uf[x] = g;  // path halving; only a non-root is ever rewritten
    x = g;
  }
}

__global__ __launch_bounds__(kBT, 8) void k_small_bridges(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const int64_t* __restrict__ voff,
    const int64_t* __restrict__ soff, const int64_t* __restrict__ moff, int32_t T, int64_t n_total,
    int64_t nnz_total, int64_t mask_words, uint32_t N, uint32_t M, int32_t vmax, int32_t smax,
    uint32_t* __restrict__ mask, int64_t* __restrict__ counts, const int32_t* __restrict__ order,
    uint32_t* __restrict__ counters, uint32_t* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char lds[];
  const BLayout L = blayout(N, M);
  uint16_t* RP = reinterpret_cast<uint16_t*>(lds + L.rp);
  uint16_t* COL = reinterpret_cast<uint16_t*>(lds + L.col);
  uint32_t* UF = reinterpret_cast<uint32_t*>(lds + L.uf);
  uint32_t* TF = reinterpret_cast<uint32_t*>(lds + L.tf);
  uint32_t* MB = reinterpret_cast<uint32_t*>(lds + L.mb);
  uint16_t* TPTR = reinterpret_cast<uint16_t*>(lds + L.tptr);
  uint16_t* HS = reinterpret_cast<uint16_t*>(lds + L.hs);
  uint16_t* TSL = reinterpret_cast<uint16_t*>(lds + L.tsl);
  uint16_t* TNB = reinterpret_cast<uint16_t*>(lds + L.tnb);
  uint16_t* TTW = reinterpret_cast<uint16_t*>(lds + L.ttw);
  uint16_t* NXa = reinterpret_cast<uint16_t*>(lds + L.nx);
  uint16_t* ROW = reinterpret_cast<uint16_t*>(lds + L.row);
  uint16_t* DDa = reinterpret_cast<uint16_t*>(lds + L.dd);
  uint16_t* TOUR = reinterpret_cast<uint16_t*>(lds + L.tour);
  uint32_t* DC = reinterpret_cast<uint32_t*>(lds + L.dc);
  uint16_t* PRE = reinterpret_cast<uint16_t*>(lds + L.pre);
  uint16_t* SIZE = reinterpret_cast<uint16_t*>(lds + L.size);
  uint16_t* PSLOT = reinterpret_cast<uint16_t*>(lds + L.pslot);
  uint16_t* RIDX = reinterpret_cast<uint16_t*>(lds + L.ridx);
  uint16_t* RL = reinterpret_cast<uint16_t*>(lds + L.rl);
  uint32_t* AMN = reinterpret_cast<uint32_t*>(lds + L.amn);
  uint32_t* AMX = reinterpret_cast<uint32_t*>(lds + L.amx);
  uint16_t* PMN = reinterpret_cast<uint16_t*>(lds + L.pmn);
  uint16_t* SMN = reinterpret_cast<uint16_t*>(lds + L.smn);
  uint16_t* PMX = reinterpret_cast<uint16_t*>(lds + L.pmx);
  uint16_t* SMX = reinterpret_cast<uint16_t*>(lds + L.smx);
  uint16_t* ST = reinterpret_cast<uint16_t*>(lds + L.st);
  int32_t* SC = reinterpret_cast<int32_t*>(lds + L.sc);
  const uint32_t tid = threadIdx.x;
  const uint32_t nbk = N / kRB + 1;  // sparse-table row length
#define STMN(l) (ST + (l) * nbk)
#define STMX(l) (ST + (kRLev + (l)) * nbk)

  if (blockIdx.x == 0 && tid == 0) {
    if (voff[0] != 0 || voff[T] != n_total || soff[0] != 0 || soff[T] != nnz_total || moff[0] != 0 ||
        moff[T] > mask_words)
      flag(status, ST_BAD_CSR);
  }
  for (;;) {
    if (tid == 0) SC[B_GRAPH] = (int32_t)atomicAdd(&counters[0], 1u);
    __syncthreads();
    const int32_t k = SC[B_GRAPH];
    if (k >= T) break;
    const int32_t t = order ? order[k] : k;  // the k-th graph taken
    const bool t_ok = (uint32_t)t < (uint32_t)T;
    const int64_t vb = t_ok ? voff[t] : 0, nv = t_ok ? voff[t + 1] - vb : 0;
    const int64_t sb = t_ok ? soff[t] : 0, ns = t_ok ? soff[t + 1] - sb : 0;
    const int64_t mw = t_ok ? moff[t] : 0, nw = t_ok ? moff[t + 1] - mw : 0;
    const bool out_ok = t_ok && mw >= 0 && nw == (ns + 31) / 32 && mw + nw <= mask_words && ns >= 0;
    const bool g_ok = out_ok && vb >= 0 && nv >= 0 && nv <= vmax && sb >= 0 && ns <= smax &&
                      vb + nv <= n_total && sb + ns <= nnz_total;
    if (!g_ok && tid == 0) flag(status, ST_BAD_CSR);
    const uint32_t n = g_ok ? (uint32_t)nv : 0u, m = g_ok ? (uint32_t)ns : 0u;
    const int32_t* rpg = row_ptr + vb + t;  // graph t's n + 1 row pointers
    if (tid == 0) {
      SC[B_FAIL] = g_ok ? 0 : 1;
      SC[B_BAD] = 0;
      SC[B_CNT] = 0;
      SC[B_NR] = 0;
    }
    for (uint32_t i = tid; i < (m + 31) / 32 + 1; i += kBT) {
      TF[i] = 0;
      MB[i] = 0;
    }
    __syncthreads();

    // 1. the CSR (nothing is read for a graph whose offsets are out of range)
    for (uint32_t v = tid; g_ok && v <= n; v += kBT) {
      const int32_t r = rpg[v];
      if (r < 0 || (uint32_t)r > m || (v == 0 && r != 0) || (v == n && (uint32_t)r != m)) {
        SC[B_BAD] = 1;
        RP[v] = 0;
      } else {
        RP[v] = (uint16_t)r;
      }
    }
    for (uint32_t k = tid; k < m; k += kBT) {
      const int32_t w = col[sb + k];
      if (w < 0 || (uint32_t)w >= n) {
        SC[B_BAD] = 1;
        COL[k] = 0;
      } else {
        COL[k] = (uint16_t)w;
      }
    }
    __syncthreads();
    for (uint32_t v = tid; v < n; v += kBT)
      if (RP[v] > RP[v + 1]) SC[B_BAD] = 1;
    __syncthreads();
    if (!SC[B_BAD] && n > 0) {
      // the row of every slot: each non-empty row's first slot marked with
      // the row, then a prefix maximum (rows are stored in vertex order)
      for (uint32_t k = tid; k < m; k += kBT) ROW[k] = 0;
      __syncthreads();
      for (uint32_t v = tid; v < n; v += kBT)
        if (RP[v] < RP[v + 1]) ROW[RP[v]] = (uint16_t)v;
      __syncthreads();
      wg_prefix_max_u16(ROW, (int)m, SC + B_WSUM);
      for (uint32_t k = tid; k < m; k += kBT) {
        const uint32_t lo = ROW[k];
        const uint32_t w = COL[k];
        if (k > RP[lo] && COL[k - 1] > w) SC[B_BAD] = 1;  // rows sorted
        const uint32_t tw = lower16(COL, RP[w], RP[w + 1], lo);
        if (tw >= RP[w + 1] || COL[tw] != lo) SC[B_BAD] = 1;  // the twin slot
      }
    }
    __syncthreads();
    if (tid == 0 && SC[B_BAD] && !SC[B_FAIL]) {
      flag(status, ST_BAD_CSR);
      SC[B_FAIL] = 1;
    }
    __syncthreads();

    if (!SC[B_FAIL] && m > 0) {
      // 2. spanning forest
      for (uint32_t v = tid; v < n; v += kBT) UF[v] = v;
      __syncthreads();
      for (uint32_t k = tid; k < m; k += kBT) {
        const uint32_t u = ROW[k], w = COL[k];
        if (u >= w || (k > RP[u] && COL[k - 1] == w)) continue;  // one slot per u-w run, u < w
        uint32_t ru = uf_find(UF, u), rw = uf_find(UF, w);
        while (ru != rw) {
          const uint32_t lo = min(ru, rw), hi = max(ru, rw);
          if (atomicCAS(&UF[hi], hi, lo) == hi) {
            const uint32_t tw = lower16(COL, RP[w], RP[w + 1], u);
            atomicOr(&TF[k >> 5], 1u << (k & 31));
            atomicOr(&TF[tw >> 5], 1u << (tw & 31));
            break;
          }
          ru = uf_find(UF, ru);
          rw = uf_find(UF, rw);
        }
      }
      __syncthreads();
      for (uint32_t v = tid; v < n; v += kBT) UF[v] = uf_find(UF, v);  // roots (the least id of each component)
      __syncthreads();

      // 3. forest half-edges per vertex, in row order: rows are stored in
      // slot order, so a forest slot's half-edge is its rank among the
      // forest slots (forest bits before its word, then within the word)
      const uint32_t nwd = (m + 31) / 32;
      for (uint32_t i = tid; i < nwd; i += kBT) DC[i] = __popc(TF[i]);
      __syncthreads();
      const uint32_t wlast = DC[nwd - 1];
      wg_scan_excl<kBT>(DC, (int)nwd, SC + B_WSUM);
      const uint32_t Et = DC[nwd - 1] + wlast;
      for (uint32_t v = tid; v <= n; v += kBT) {
        const uint32_t k = RP[v];
        TPTR[v] = (uint16_t)(k >= m ? Et : DC[k >> 5] + __popc(TF[k >> 5] & ((1u << (k & 31)) - 1u)));
      }
      for (uint32_t k = tid; k < m; k += kBT) {
        const uint32_t bits = TF[k >> 5];
        if (!((bits >> (k & 31)) & 1u)) continue;
        const uint32_t h = DC[k >> 5] + __popc(bits & ((1u << (k & 31)) - 1u));
        TSL[h] = (uint16_t)k;
        TNB[h] = COL[k];
      }
      __syncthreads();
      for (uint32_t v = tid; v < n; v += kBT)
        for (uint32_t h = TPTR[v]; h < TPTR[v + 1]; ++h) HS[h] = (uint16_t)v;
      __syncthreads();
      uint16_t* SUCC = DDa;  // the successors, in the upper half of the pointer-jumping region
      for (uint32_t h = tid; h < Et; h += kBT) {
        const uint32_t u = HS[h], w = TNB[h];
        const uint32_t tw = lower16(TNB, TPTR[w], TPTR[w + 1], u);
        TTW[h] = (uint16_t)tw;
        // succ(h) = next(twin(h)) in w's cyclic list
        SUCC[h] = (uint16_t)((tw + 1 == TPTR[w + 1]) ? TPTR[w] : tw + 1);
      }
      // component roots that own forest edges, in id order
      for (uint32_t v = tid; v < n; v += kBT) DC[v] = (UF[v] == v && TPTR[v + 1] > TPTR[v]) ? 1u : 0u;
      __syncthreads();
      const uint32_t rlast = n ? DC[n - 1] : 0;
      wg_scan_excl<kBT>(DC, (int)n, SC + B_WSUM);
      for (uint32_t v = tid; v < n; v += kBT)
        if (UF[v] == v && TPTR[v + 1] > TPTR[v]) {
          RIDX[v] = (uint16_t)DC[v];
          RL[DC[v]] = (uint16_t)v;
        }
      if (tid == 0) {
        SC[B_NR] = (int32_t)(n ? DC[n - 1] + rlast : 0);
        SC[B_ET] = (int32_t)Et;
      }
      __syncthreads();
      const uint32_t R = (uint32_t)SC[B_NR];
      // cut each component's cycle before its root's first half-edge and chain them
      for (uint32_t i = tid; i < R; i += kBT) {
        const uint32_t r = RL[i];
        const uint32_t last = TTW[TPTR[r + 1] - 1];  // its successor is r's first half-edge
        SUCC[last] = (i + 1 < R) ? TPTR[RL[i + 1]] : kNil;
      }
      __syncthreads();

      if (R > 0) {
        // 4. ranks: distance to the end by pointer jumping
        // (next << 16 | distance) per half-edge, two buffers: one 32-bit add
        // sums the distances
        uint32_t* PJ0 = reinterpret_cast<uint32_t*>(NXa);
        uint32_t* PJ1 = reinterpret_cast<uint32_t*>(DDa);
        for (uint32_t h = tid; h < Et; h += kBT) {
          const uint32_t x = SUCC[h];
          PJ0[h] = (x << 16) | (x == kNil ? 0u : 1u);
        }
        __syncthreads();
        const int jumps = (32 - __clz((int)Et)) + 1;
        for (int it = 0; it < jumps; ++it) {
          for (uint32_t h = tid; h < Et; h += kBT) {
            const uint32_t p = PJ0[h], x = p >> 16;
            if (x != kNil && x < Et) {
              const uint32_t q = PJ0[x];
              PJ1[h] = (q & 0xffff0000u) | ((p + q) & 0xffffu);
            } else {
              PJ1[h] = ((uint32_t)kNil << 16) | (p & 0xffffu);
            }
          }
          __syncthreads();
          uint32_t* tp = PJ0;
          PJ0 = PJ1;
          PJ1 = tp;
        }
        const uint32_t head = TPTR[RL[0]];
        if (tid == 0 && (PJ0[head] & 0xffffu) + 1 != Et) {
          flag(status, ST_UNREACHED);
          SC[B_FAIL] = 1;
        }
        __syncthreads();
        if (!SC[B_FAIL]) {
          uint16_t* RK = reinterpret_cast<uint16_t*>(PJ1);  // rank = Et - 1 - distance to the end
          for (uint32_t h = tid; h < Et; h += kBT) {
            const uint32_t r = Et - 1 - (PJ0[h] & 0xffffu);
            RK[h] = (uint16_t)r;
            TOUR[r] = (uint16_t)h;
          }
          __syncthreads();
          for (uint32_t r = tid; r < Et; r += kBT) {
            const uint32_t h = TOUR[r];
            DC[r] = RK[h] < RK[TTW[h]] ? 1u : 0u;
          }
          __syncthreads();
          wg_scan_excl<kBT>(DC, (int)Et, SC + B_WSUM);  // down half-edges before each tour position
          // preorder and subtree size: a down half-edge (u -> w) enters w;
          // the bridge test also takes u and the slot of (w -> u), kept in
          // the tour order's place (dead now)
          uint16_t* PU = TOUR;
          uint16_t* PTW = TOUR + N;
          for (uint32_t h = tid; h < Et; h += kBT) {
            const uint32_t t = TTW[h];
            const uint32_t r = RK[h], rt = RK[t];
            if (r < rt) {
              const uint32_t w = TNB[h];
              PRE[w] = (uint16_t)(RIDX[UF[w]] + DC[r] + 1);
              SIZE[w] = (uint16_t)((rt - r + 1) >> 1);
              PSLOT[w] = TSL[h];
              PU[w] = TNB[t];
              PTW[w] = TSL[t];
            }
          }
          for (uint32_t i = tid; i < R; i += kBT) {
            const uint32_t r = RL[i];
            const uint32_t start = RK[TPTR[r]];
            const uint32_t end = (i + 1 < R) ? RK[TPTR[RL[i + 1]]] : Et;  // one past its last half-edge
            PRE[r] = (uint16_t)(i + DC[start]);
            SIZE[r] = (uint16_t)((end - start) / 2 + 1);
            PSLOT[r] = kNil;
          }
          __syncthreads();

          // 5. non-forest extremes per preorder position
          const uint32_t P = Et / 2 + R;  // vertices in components with forest edges
          for (uint32_t v = tid; v < n; v += kBT)
            if (TPTR[v + 1] > TPTR[v]) {
              AMN[PRE[v]] = PRE[v];
              AMX[PRE[v]] = PRE[v];
            }
          __syncthreads();
          for (uint32_t k = tid; k < m; k += kBT) {
            if ((TF[k >> 5] >> (k & 31)) & 1u) continue;
            const uint32_t u = row_of_slot(RP, n, k), w = COL[k];
            if (TPTR[u + 1] == TPTR[u]) continue;  // a loop on a vertex without forest edges
            atomicMin(&AMN[PRE[u]], (uint32_t)PRE[w]);
            atomicMax(&AMX[PRE[u]], (uint32_t)PRE[w]);
          }
          __syncthreads();
          // in-block prefix / suffix extremes by shuffles within 32-lane
          // segments (one lane per position, a segment per block), then the
          // sparse table over the at most 32 blocks by one wavefront
          const uint32_t nb = (P + kRB - 1) / kRB;
          for (uint32_t i = tid; i < nb * kRB; i += kBT) {
            const uint32_t j = i & (kRB - 1);
            const uint32_t a = i < P ? AMN[i] : 0xffffu, x = i < P ? AMX[i] : 0u;
            uint32_t pmn = a, pmx = x, smn = a, smx = x;
#pragma unroll
            for (int d = 1; d < kRB; d <<= 1) {
              const uint32_t p0 = __shfl_up(pmn, d, kRB), p1 = __shfl_up(pmx, d, kRB);
              const uint32_t s0 = __shfl_down(smn, d, kRB), s1 = __shfl_down(smx, d, kRB);
              if (j >= (uint32_t)d) {
                pmn = min(pmn, p0);
                pmx = max(pmx, p1);
              }
              if (j + d < (uint32_t)kRB) {
                smn = min(smn, s0);
                smx = max(smx, s1);
              }
            }
            if (i < P) {
              PMN[i] = (uint16_t)pmn;
              PMX[i] = (uint16_t)pmx;
              SMN[i] = (uint16_t)smn;
              SMX[i] = (uint16_t)smx;
            }
            if (j == kRB - 1) {
              STMN(0)[i / kRB] = (uint16_t)pmn;
              STMX(0)[i / kRB] = (uint16_t)pmx;
            }
          }
          __syncthreads();
          if (tid < 64) {  // nb <= 32: one wavefront, one block per lane
            uint32_t vmn = tid < nb ? STMN(0)[tid] : 0xffffu, vmx = tid < nb ? STMX(0)[tid] : 0u;
            for (int l = 1; l < kRLev; ++l) {
              const uint32_t h = 1u << (l - 1);
              const uint32_t omn = __shfl_down(vmn, h), omx = __shfl_down(vmx, h);
              vmn = min(vmn, omn);
              vmx = max(vmx, omx);
              if (tid + (1u << l) <= nb) {
                STMN(l)[tid] = (uint16_t)vmn;
                STMX(l)[tid] = (uint16_t)vmx;
              }
            }
          }
          __syncthreads();
          // the bridge test for the forest edge above every non-root vertex
          for (uint32_t w = tid; w < n; w += kBT) {
            const uint32_t k = PSLOT[w];
            if (TPTR[w + 1] == TPTR[w] || k == kNil) continue;
            const uint32_t l = PRE[w], r = l + SIZE[w] - 1;
            uint32_t mn, mx;
            const uint32_t bl = l / kRB, br = r / kRB;
            if (bl == br) {
              mn = 0xffffu;
              mx = 0;
              for (uint32_t i = l; i <= r; ++i) {
                mn = min(mn, AMN[i]);
                mx = max(mx, AMX[i]);
              }
            } else {
              mn = min((uint32_t)SMN[l], (uint32_t)PMN[r]);
              mx = max((uint32_t)SMX[l], (uint32_t)PMX[r]);
              if (br > bl + 1) {
                const uint32_t a = bl + 1, cnt = br - bl - 1;
                const int lev = 31 - __clz((int)cnt);
                const uint32_t b2 = a + cnt - (1u << lev);
                mn = min(mn, (uint32_t)min(STMN(lev)[a], STMN(lev)[b2]));
                mx = max(mx, (uint32_t)max(STMX(lev)[a], STMX(lev)[b2]));
              }
            }
            if (mn != l || mx != r) continue;
            const uint32_t u = PU[w];
            if (k + 1 < RP[u + 1] && COL[k + 1] == w) continue;  // a parallel edge is never a bridge
            const uint32_t tw = PTW[w];
            atomicOr(&MB[k >> 5], 1u << (k & 31));
            atomicOr(&MB[tw >> 5], 1u << (tw & 31));
            atomicAdd(&SC[B_CNT], 1);
          }
          __syncthreads();
        }
      }
    }
    // 6. the graph's mask words and count
    if (out_ok) {
      const bool fail = SC[B_FAIL] != 0;
      for (int64_t i = tid; i < nw; i += kBT) mask[mw + i] = fail ? 0u : MB[i];
      if (tid == 0 && counts) counts[t] = fail ? 0 : SC[B_CNT];
    }
    __syncthreads();  // the tables and SC[B_GRAPH] are rewritten by the next graph
  }
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(&counters[1], 1u) == gridDim.x - 1) {
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
#undef STMN
#undef STMX
}

}  // namespace

int small_bridges_run(Ctx* c, const int32_t* row_ptr, const int32_t* col, const int64_t* voff, const int64_t* soff,
                      const int64_t* moff, int32_t T, int32_t n_total, int32_t nnz_total, int32_t max_vertices,
                      int32_t max_slots, uint32_t* mask, int64_t mask_words, int64_t* counts, const int32_t* order,
                      hipStream_t s) {
  if (T == 0) return ET_OK;
  if (max_vertices < 0 || max_slots < 0) return ET_EINVAL;
  if (max_vertices > kGMaxV || max_slots > kGMaxS) return ET_ESIZE;
  const uint32_t N = a64((uint32_t)std::max(max_vertices, 1)), M = a64((uint32_t)std::max(max_slots, 1));
  const uint32_t lds = blayout(N, M).total;
  int grid = 0;
  const int rc = persistent_grid(reinterpret_cast<const void*>(k_small_bridges), kBT, lds, T, &grid);
  if (rc) return rc;
  ET_PROF(c, s, "k_small_bridges");
  hipLaunchKernelGGL(k_small_bridges, dim3(grid), dim3(kBT), lds, s, row_ptr, col, voff, soff, moff, T,
                     (int64_t)n_total, (int64_t)nnz_total, mask_words, N, M, max_vertices, max_slots, mask, counts,
                     order, c->d_fused, c->d_status);
  return hipGetLastError() == hipSuccess ? ET_OK : ET_EHIP;
}

}  // namespace et
