// Plans of a persistent neighborhood all-to-all-v, built on the GPU for every
// rank of a decomposition (all setup at initialisation, MPI Advance Sec. 2.2).
//
// Data structures (no sorting anywhere; order comes from bit positions and
// prefix sums):
//   B[r]      bitmap over global columns of rank r's off-rank references
//             (halo discovery; compacting it with a block-wide prefix scan of
//             popcounts yields the halo N_r sorted and duplicate-free)
//   M[r][q]   |N_r ∩ owned(q)|: dense rank-pair message sizes.  Its rows are
//             the receive lists; its transpose gives the send lists; row
//             prefix sums give every displacement
//   NB[m]     node bitmap: OR of B[s] over the ranks s of node m.  A set bit c
//             owned by a remote rank q is one entry of the deduplicated
//             aggregated message D(q -> m) (a value crosses a node pair once,
//             Sec. 2.2, last paragraph); its position inside D(q -> m) is a
//             bitmap rank (popcount prefix)
// Every list entry is then written by a scatter whose destination is a closed
// form of these prefix sums, so the result is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <memory>
#include <numeric>
#include <vector>

#include "common.h"
#include "internal.h"

namespace hx {
namespace {

constexpr int TB = 256;

unsigned blocks_for(int64_t n, int per = TB) {
  int64_t b = (n + per - 1) / per;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16));
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// Largest p in [0, R) with starts[p] <= v.
__device__ __forceinline__ int upper_rank(const int64_t* __restrict__ starts, int R, int64_t v) {
  int lo = 0, hi = R - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Placement of R ranks on NN = ceil(R / ppn) nodes (Sec. 2.2 groups ranks by
// node without fixing which ranks share one).  Block: node p / ppn, local rank
// p % ppn, the last node may hold fewer ranks.  Cyclic (round robin): node
// p % NN, local rank p / NN.
struct Place {
  int R, ppn, NN, cyc;
  __device__ int node(int p) const { return cyc ? p % NN : p / ppn; }
  __device__ int lrank(int p) const { return cyc ? p / NN : p % ppn; }
  __device__ int cnt(int m) const { return cyc ? (R - 1 - m) / NN + 1 : min(ppn, R - m * ppn); }
  __device__ int rank_at(int m, int l) const { return cyc ? l * NN + m : m * ppn + l; }
  // The rank of node m that receives rank q's deduplicated message: the one
  // whose local rank is q's modulo the size of node m.
  __device__ int partner(int q, int m) const { return rank_at(m, lrank(q) % cnt(m)); }
};

// 3-step (one message per node pair, block placement only): the rank of node
// n that sends node n's data for node m, and the rank of node m that receives it.
__device__ __forceinline__ int aggr_of(const Place& P, int n, int m) { return P.rank_at(n, m % P.cnt(n)); }
__device__ __forceinline__ int recv_of(const Place& P, int n, int m) { return P.rank_at(m, n % P.cnt(m)); }
// The forwarder on node m of the entries owned by rank q (the rank their
// aggregated stage-1 message lands on), the sender of that message, and the
// first row of the column range the message deduplicates over.
__device__ __forceinline__ int fwd_of(const Place& P, int q, int m, int v3) {
  return v3 ? recv_of(P, P.node(q), m) : P.partner(q, m);
}
__device__ __forceinline__ int agg_sender(const Place& P, int q, int m, int v3) {
  return v3 ? aggr_of(P, P.node(q), m) : q;
}
__device__ __forceinline__ int64_t agg_base(const Place& P, int q, const int64_t* __restrict__ rs, int v3) {
  return v3 ? rs[P.rank_at(P.node(q), 0)] : rs[q];
}

template <class T>
__device__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum (every thread gets it).  blockDim.x is a multiple of 64, <= 1024.
template <class T>
__device__ T block_sum(T v) {
  __shared__ T sh[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T t = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

// Block-wide exclusive scan; *total = block sum.
template <class T>
__device__ T block_exscan(T v, T* total) {
  __shared__ T sh[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  T base = 0, tot = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
    if (i < wid) base += sh[i];
    tot += sh[i];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// Rank of bit c in bitmap row (words NB, exclusive word prefix NBP): number of
// set bits below c.  Rows carry one extra zero word so c may equal n.
__device__ __forceinline__ int32_t bit_rank(const uint32_t* __restrict__ NB, const int32_t* __restrict__ NBP,
                                            int64_t c) {
  const int64_t w = c >> 5;
  const uint32_t below = (uint32_t)((1ull << (c & 31)) - 1ull);
  return NBP[w] + __popc(NB[w] & below);
}

// ---------------------------------------------------------------------------
// Generic device utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  GRID_STRIDE(i, n) p[i] = v;
}

constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_BLOCK = TB * SCAN_ITEMS;

__global__ void k_scan_partials(const int32_t* __restrict__ in, int64_t n, int64_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK;
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + (int64_t)k * TB + threadIdx.x;
    if (i < n) s += in[i];
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_scan_part_scan(int64_t* part, int64_t nparts) {
  int64_t base = 0;
  for (int64_t c0 = 0; c0 < nparts; c0 += blockDim.x) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < nparts ? part[i] : 0;
    int64_t tot;
    const int64_t pre = block_exscan(v, &tot);
    if (i < nparts) part[i] = base + pre;
    base += tot;
  }
  if (threadIdx.x == 0) part[nparts] = base;
}

__global__ void k_scan_final(const int32_t* __restrict__ in, int64_t n, const int64_t* __restrict__ part,
                             int32_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK;
  // each thread takes SCAN_ITEMS consecutive items
  const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t v[SCAN_ITEMS];
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = (i0 + k < n) ? in[i0 + k] : 0;
    s += v[k];
  }
  int64_t tot;
  int64_t run = part[blockIdx.x] + block_exscan(s, &tot);
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (i0 + k < n) out[i0 + k] = (int32_t)run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (int32_t)part[gridDim.x];
}

__global__ void k_count_keys(const int32_t* __restrict__ keys, int64_t n, int64_t nkeys, int32_t* cnt, int* err) {
  GRID_STRIDE(i, n) {
    const int32_t key = keys[i];
    if (key < 0 || key >= nkeys) atomicOr(err, 16);
    else atomicAdd(cnt + key, 1);
  }
}

// err |= 16 if some idx[i] is outside [0, hi).
__global__ void k_check_range(const int32_t* __restrict__ idx, int64_t n, int64_t hi, int* err) {
  GRID_STRIDE(i, n) {
    const int32_t v = idx[i];
    if (v < 0 || v >= hi) atomicOr(err, 16);
  }
}

__global__ void k_place_keys(const int32_t* __restrict__ keys, int64_t n, int64_t nkeys, int32_t* cursor,
                             int32_t* perm, int* err) {
  GRID_STRIDE(i, n) {
    const int32_t key = keys[i];
    if (key < 0 || key >= nkeys) {
      atomicOr(err, 16);
      continue;
    }
    const int32_t pos = atomicAdd(cursor + key, 1);
    if (pos < 0 || pos >= n) {
      atomicOr(err, 16);
      continue;
    }
    perm[pos] = (int32_t)i;
  }
}

// Sort each group ascending (groups are short: the fan-out of a row).
__global__ void k_sort_groups(const int32_t* __restrict__ ptr, int64_t nkeys, int32_t* perm) {
  GRID_STRIDE(g, nkeys) {
    const int32_t a = ptr[g], b = ptr[g + 1];
    for (int32_t i = a + 1; i < b; ++i) {
      const int32_t v = perm[i];
      int32_t j = i - 1;
      while (j >= a && perm[j] > v) {
        perm[j + 1] = perm[j];
        --j;
      }
      perm[j + 1] = v;
    }
  }
}

__global__ void k_flag(const int32_t* __restrict__ idx, int64_t n, int64_t domain, int32_t* flags) {
  GRID_STRIDE(i, n) {
    const int32_t v = idx[i];
    if (v >= 0 && v < domain) flags[v] = 1;
  }
}

__global__ void k_sum_i32(const int32_t* __restrict__ a, int64_t n, unsigned long long* out) {
  int64_t s = 0;
  GRID_STRIDE(i, n) s += a[i];
  s = block_sum(s);
  if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)s);
}

// ---------------------------------------------------------------------------
// Halo discovery
// ---------------------------------------------------------------------------
// Marks every off-rank column of each row in its rank's bitmap.
// Rows [i0, i0 + rows) belong to ranks r0, r0 + 1, ...; their bitmaps are the
// rows of B counted from r0.
__global__ void k_mark_csr(const int64_t* __restrict__ rs, int R, int64_t n, int64_t i0, int64_t rows, int r0,
                           const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ cols, uint32_t* B,
                           int64_t W, int* err) {
  GRID_STRIDE(k, rows) {
    const int64_t i = i0 + k;
    const int r = upper_rank(rs, R, i);
    const int64_t lo = rs[r], hi = rs[r + 1];
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    if (e1 < e0) {
      atomicOr(err, 8);
      continue;
    }
    uint32_t* Br = B + (size_t)(r - r0) * W;
    for (int64_t e = e0; e < e1; ++e) {
      const int64_t c = cols[e];
      if (c < 0 || c >= n) {
        atomicOr(err, 1);
        continue;
      }
      if (c >= lo && c < hi) continue;
      atomicOr(Br + (c >> 5), 1u << (c & 31));
    }
  }
}

// Number of set bits of each rank's bitmap (one block per rank).
__global__ void k_popc_rows(const uint32_t* __restrict__ B, int64_t W, int64_t* cnt) {
  const uint32_t* Br = B + (size_t)blockIdx.x * W;
  int64_t s = 0;
  for (int64_t w = threadIdx.x; w < W; w += blockDim.x) s += __popc(Br[w]);
  s = block_sum(s);
  if (threadIdx.x == 0) cnt[blockIdx.x] = s;
}

// Writes the set bits of each rank's bitmap as ascending column ids.
__global__ void k_compact_bits(const uint32_t* __restrict__ B, int64_t W, const int64_t* __restrict__ off,
                               int32_t* __restrict__ out) {
  const uint32_t* Br = B + (size_t)blockIdx.x * W;
  const int64_t end = off[blockIdx.x + 1];
  int64_t base = off[blockIdx.x];
  for (int64_t w0 = 0; w0 < W; w0 += blockDim.x) {
    const int64_t w = w0 + threadIdx.x;
    uint32_t bits = w < W ? Br[w] : 0u;
    int64_t tot;
    int64_t o = base + block_exscan((int64_t)__popc(bits), &tot);
    while (bits) {
      const int b = __ffs(bits) - 1;
      if (o < end) out[o] = (int32_t)(w * 32 + b);
      ++o;
      bits &= bits - 1u;
    }
    base += tot;
  }
}

// Per halo entry: its rank, its owner, and the rank-pair count M[r][q].
__global__ void k_entry_info(const int32_t* __restrict__ hcol, int64_t nH, const int64_t* __restrict__ hoff,
                             const int64_t* __restrict__ rs, int R, int64_t n, int check, int32_t* hrank,
                             int32_t* own, int32_t* M, int* err) {
  GRID_STRIDE(e, nH) {
    const int r = upper_rank(hoff, R, e);
    const int64_t c = hcol[e];
    if (check) {
      if (c < 0 || c >= n) {
        atomicOr(err, 1);
        continue;
      }
      if (e > hoff[r] && hcol[e - 1] >= c) atomicOr(err, 2);
      if (c >= rs[r] && c < rs[r + 1]) {
        atomicOr(err, 4);
        continue;
      }
    }
    const int q = upper_rank(rs, R, c);
    hrank[e] = r;
    own[e] = q;
    atomicAdd(M + (size_t)r * R + q, 1);
  }
}

// ---------------------------------------------------------------------------
// Dense rank-pair tables
// ---------------------------------------------------------------------------
__global__ void k_transpose(const int32_t* __restrict__ A, int32_t* __restrict__ AT, int R) {
  __shared__ int32_t t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int y = threadIdx.y; y < 32; y += blockDim.y) {
    const int r = by + y, c = bx + threadIdx.x;
    if (r < R && c < R) t[y][threadIdx.x] = A[(size_t)r * R + c];
  }
  __syncthreads();
  for (int y = threadIdx.y; y < 32; y += blockDim.y) {
    const int r = bx + y, c = by + threadIdx.x;
    if (r < R && c < R) AT[(size_t)r * R + c] = t[threadIdx.x][y];
  }
}

// Row-wise exclusive prefix P, row sums and row nonzero counts (block per row).
__global__ void k_row_exscan(const int32_t* __restrict__ A, int32_t* __restrict__ P, int R, int64_t* rowsum,
                             int64_t* rownnz) {
  const size_t r = blockIdx.x;
  int64_t base = 0, nnz = 0;
  for (int c0 = 0; c0 < R; c0 += blockDim.x) {
    const int c = c0 + threadIdx.x;
    const int32_t v = c < R ? A[r * R + c] : 0;
    int64_t tot;
    const int64_t pre = block_exscan((int64_t)v, &tot);
    if (c < R) P[r * R + c] = (int32_t)(base + pre);
    base += tot;
    nnz += block_sum((int64_t)(v != 0));
  }
  if (threadIdx.x == 0) {
    rowsum[r] = base;
    rownnz[r] = nnz;
  }
}

// Nonzeros of each row as (column, value, prefix) lists (block per row).
__global__ void k_row_compact(const int32_t* __restrict__ A, const int32_t* __restrict__ P, int R,
                              const int64_t* __restrict__ list_off, int32_t* procs, int32_t* counts,
                              int32_t* displs) {
  const size_t r = blockIdx.x;
  const int64_t end = list_off[r + 1];
  int64_t base = list_off[r];
  for (int c0 = 0; c0 < R; c0 += blockDim.x) {
    const int c = c0 + threadIdx.x;
    const int32_t v = c < R ? A[r * R + c] : 0;
    int64_t tot;
    const int64_t pre = block_exscan((int64_t)(v != 0), &tot);
    if (v != 0 && base + pre < end) {
      const int64_t o = base + pre;
      procs[o] = c;
      counts[o] = v;
      displs[o] = P[r * R + c];
    }
    base += tot;
  }
}

// ---------------------------------------------------------------------------
// Locality-aware (2-step) tables
// ---------------------------------------------------------------------------
__global__ void k_node_mark(const int32_t* __restrict__ hcol, const int32_t* __restrict__ hrank, int64_t nH,
                            Place P, uint32_t* NB, int64_t W1) {
  GRID_STRIDE(e, nH) {
    const int64_t c = hcol[e];
    const int m = P.node(hrank[e]);
    atomicOr(NB + (size_t)m * W1 + (c >> 5), 1u << (c & 31));
  }
}

// Exclusive word prefix of popcounts per node row (block per row).
__global__ void k_word_exscan(const uint32_t* __restrict__ NB, int64_t W1, int32_t* NBP) {
  const size_t m = blockIdx.x;
  int64_t base = 0;
  for (int64_t w0 = 0; w0 < W1; w0 += blockDim.x) {
    const int64_t w = w0 + threadIdx.x;
    const int64_t v = w < W1 ? __popc(NB[m * W1 + w]) : 0;
    int64_t tot;
    const int64_t pre = block_exscan(v, &tot);
    if (w < W1) NBP[m * W1 + w] = (int32_t)(base + pre);
    base += tot;
  }
}

// MD[m][q] = |D(q -> m)| for q off node m (else 0).  3-step: |D(n -> m)| of
// q's node n at q = the pair's aggregator (else 0).
__global__ void k_dedup_counts(const uint32_t* __restrict__ NB, const int32_t* __restrict__ NBP, int64_t W1,
                               const int64_t* __restrict__ rs, Place P, int v3, int32_t* MD) {
  const int R = P.R;
  GRID_STRIDE(i, (int64_t)P.NN * R) {
    const int m = (int)(i / R), q = (int)(i % R);
    int32_t v = 0;
    if (P.node(q) != m) {
      const uint32_t* nb = NB + (size_t)m * W1;
      const int32_t* np = NBP + (size_t)m * W1;
      if (!v3) {
        v = bit_rank(nb, np, rs[q + 1]) - bit_rank(nb, np, rs[q]);
      } else {
        const int n = P.node(q);
        const int first = P.rank_at(n, 0);  // block: node n's rows are contiguous
        if (q == aggr_of(P, n, m))
          v = bit_rank(nb, np, rs[first + P.cnt(n)]) - bit_rank(nb, np, rs[first]);
      }
    }
    MD[i] = v;
  }
}

// Stage-1 message sizes S1[q][d]: direct to on-node d, deduplicated to partners.
__global__ void k_stage1_sizes(const int32_t* __restrict__ MT, const int32_t* __restrict__ MD, Place P, int v3,
                               int32_t* S1) {
  const int R = P.R;
  GRID_STRIDE(i, (int64_t)R * R) {
    const int q = (int)(i / R), d = (int)(i % R);
    int32_t v = 0;
    if (d != q) {
      const int nq = P.node(q), nd = P.node(d);
      if (nq == nd) v = MT[i];
      else if (v3 ? (q == aggr_of(P, nq, nd) && d == recv_of(P, nq, nd)) : d == P.partner(q, nd))
        v = MD[(size_t)nd * R + q];
    }
    S1[i] = v;
  }
}

// Stage-2 message sizes S2[t][s] (t forwards to s on its node): the entries of
// N_s owned by remote ranks whose aggregated message lands on t.
__global__ void k_stage2_sizes(const int32_t* __restrict__ M, Place P, int v3, int32_t* S2) {
  const int R = P.R;
  GRID_STRIDE(i, (int64_t)R * R) {
    const int t = (int)(i / R), s = (int)(i % R);
    int64_t v = 0;
    const int n = P.node(t);
    if (s != t && P.node(s) == n) {
      const int cn = P.cnt(n);
      const int lt = P.lrank(t);
      const int32_t* Ms = M + (size_t)s * R;
      for (int m = 0; m < P.NN; ++m) {
        if (m == n) continue;
        const int cm = P.cnt(m);
        if (v3) {  // every rank of the nodes whose pair message lands on t
          if (m % cn == lt)
            for (int l = 0; l < cm; ++l) v += Ms[P.rank_at(m, l)];
        } else {
          for (int l = lt; l < cm; l += cn) v += Ms[P.rank_at(m, l)];
        }
      }
    }
    S2[i] = (int32_t)v;
  }
}

// QP[s][q]: for q off s's node, the number of entries of N_s owned by the
// ranks before q (ascending) that share q's partner on s's node.  Class l0 of
// node n: the remote ranks whose local rank is l0 modulo the size of node n
// (3-step: every rank of the nodes m with m mod cn == l0).
__global__ void k_class_prefix(const int32_t* __restrict__ M, Place P, int v3, int32_t* QP) {
  const int R = P.R;
  GRID_STRIDE(i, (int64_t)R * P.ppn) {
    const int s = (int)(i / P.ppn), l0 = (int)(i % P.ppn);
    const int n = P.node(s);
    const int cn = P.cnt(n);
    if (l0 >= cn) continue;
    const int32_t* Ms = M + (size_t)s * R;
    int32_t* Qs = QP + (size_t)s * R;
    int32_t run = 0;
    if (P.cyc) {  // rank l*NN + m ascends with the local rank first, then the node
      for (int l = l0; l < P.ppn; l += cn)
        for (int m = 0; m < P.NN; ++m) {
          if (m == n || l >= P.cnt(m)) continue;
          const int q = P.rank_at(m, l);
          Qs[q] = run;
          run += Ms[q];
        }
      continue;
    }
    for (int m = 0; m < P.NN; ++m) {  // block: rank m*ppn + l ascends with the node first
      if (m == n) continue;
      const int cm = P.cnt(m);
      if (v3) {
        if (m % cn != l0) continue;
        for (int l = 0; l < cm; ++l) {
          const int q = P.rank_at(m, l);
          Qs[q] = run;
          run += Ms[q];
        }
      } else {
        for (int l = l0; l < cm; l += cn) {
          const int q = P.rank_at(m, l);
          Qs[q] = run;
          run += Ms[q];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// List entries (scatters with closed-form destinations)
// ---------------------------------------------------------------------------
// Stage-1 send entries carrying one halo entry each: every entry (plain) or
// the on-node ones (locality).
__global__ void k_s1_direct(const int32_t* __restrict__ hcol, const int32_t* __restrict__ hrank,
                            const int32_t* __restrict__ own, int64_t nH, const int64_t* __restrict__ hoff,
                            const int64_t* __restrict__ rs, Place P, int onnode_only, int v3,
                            const int32_t* __restrict__ PS1, const int32_t* __restrict__ PM,
                            const int64_t* __restrict__ s1_off, int32_t* s1_idx, int* err) {
  const int R = P.R;
  GRID_STRIDE(e, nH) {
    const int s = hrank[e], q = own[e];
    if (onnode_only && P.node(q) != P.node(s)) continue;
    const int64_t j = e - hoff[s];
    const int64_t pos = s1_off[q] + PS1[(size_t)q * R + s] + (j - PM[(size_t)s * R + q]);
    if (pos < s1_off[q] || pos >= s1_off[q + 1]) {
      atomicOr(err, 32);
      continue;
    }
    s1_idx[pos] = (int32_t)(hcol[e] - agg_base(P, q, rs, v3));  // 3-step: rows of the node
  }
}

// Stage-1 aggregated entries: one per set bit of a node bitmap owned off-node.
__global__ void k_s1_agg(const uint32_t* __restrict__ NB, const int32_t* __restrict__ NBP, int64_t W1,
                         int64_t W, const int64_t* __restrict__ rs, Place P, int v3,
                         const int32_t* __restrict__ PS1, const int64_t* __restrict__ s1_off, int32_t* s1_idx,
                         int* err) {
  const int R = P.R;
  GRID_STRIDE(i, (int64_t)P.NN * W) {
    const int m = (int)(i / W);
    const int64_t w = i % W;
    const uint32_t* nb = NB + (size_t)m * W1;
    const int32_t* np = NBP + (size_t)m * W1;
    uint32_t bits = nb[w];
    while (bits) {
      const int b = __ffs(bits) - 1;
      bits &= bits - 1u;
      const int64_t c = w * 32 + b;
      const int q = upper_rank(rs, R, c);
      if (P.node(q) == m) continue;
      const int t = fwd_of(P, q, m, v3);
      const int a = agg_sender(P, q, m, v3);
      const int64_t base = agg_base(P, q, rs, v3);
      const int64_t pos = s1_off[a] + PS1[(size_t)a * R + t] + (bit_rank(nb, np, c) - bit_rank(nb, np, base));
      if (pos < s1_off[a] || pos >= s1_off[a + 1]) {
        atomicOr(err, 32);
        continue;
      }
      s1_idx[pos] = (int32_t)(c - base);
    }
  }
}

// Stage-2 (redistribution) entries: halo entries of s owned off-node whose
// aggregated message landed on another rank t of s's node.
__global__ void k_s2_src(const int32_t* __restrict__ hcol, const int32_t* __restrict__ hrank,
                         const int32_t* __restrict__ own, int64_t nH, const int64_t* __restrict__ hoff,
                         const int64_t* __restrict__ rs, Place P, const int32_t* __restrict__ PS2,
                         const int32_t* __restrict__ QP, const int32_t* __restrict__ PM,
                         const int32_t* __restrict__ PR1, const uint32_t* __restrict__ NB,
                         const int32_t* __restrict__ NBP, int64_t W1, const int64_t* __restrict__ s2_off,
                         int v3, int32_t* s2_src, int* err) {
  const int R = P.R;
  GRID_STRIDE(e, nH) {
    const int s = hrank[e], q = own[e];
    const int n = P.node(s);
    if (P.node(q) == n) continue;
    const int t = fwd_of(P, q, n, v3);
    if (t == s) continue;
    const int64_t j = e - hoff[s];
    const int64_t c = hcol[e];
    const uint32_t* nb = NB + (size_t)n * W1;
    const int32_t* np = NBP + (size_t)n * W1;
    const int64_t pos = s2_off[t] + PS2[(size_t)t * R + s] + QP[(size_t)s * R + q] + (j - PM[(size_t)s * R + q]);
    if (pos < s2_off[t] || pos >= s2_off[t + 1]) {
      atomicOr(err, 32);
      continue;
    }
    s2_src[pos] = PR1[(size_t)t * R + agg_sender(P, q, n, v3)] +
                  (bit_rank(nb, np, c) - bit_rank(nb, np, agg_base(P, q, rs, v3)));
  }
}

// Unpack map: slot of each halo entry in [stage-1 recv | stage-2 recv].
__global__ void k_unpack_map(const int32_t* __restrict__ hcol, const int32_t* __restrict__ hrank,
                             const int32_t* __restrict__ own, int64_t nH, const int64_t* __restrict__ hoff,
                             const int64_t* __restrict__ rs, Place P, int locality, int v3,
                             const int32_t* __restrict__ PM, const int32_t* __restrict__ PR1,
                             const int32_t* __restrict__ PR2, const int32_t* __restrict__ QP,
                             const uint32_t* __restrict__ NB, const int32_t* __restrict__ NBP, int64_t W1,
                             const int64_t* __restrict__ r1_tot, int32_t* unpack) {
  const int R = P.R;
  GRID_STRIDE(e, nH) {
    const int r = hrank[e];
    const int64_t j = e - hoff[r];
    if (!locality) {
      unpack[e] = (int32_t)j;
      continue;
    }
    const int q = own[e];
    const int n = P.node(r);
    const int64_t c = hcol[e];
    int64_t v;
    if (P.node(q) == n) {
      v = PR1[(size_t)r * R + q] + (j - PM[(size_t)r * R + q]);
    } else {
      const int t = fwd_of(P, q, n, v3);
      const uint32_t* nb = NB + (size_t)n * W1;
      const int32_t* np = NBP + (size_t)n * W1;
      if (t == r)
        v = PR1[(size_t)r * R + agg_sender(P, q, n, v3)] +
            (bit_rank(nb, np, c) - bit_rank(nb, np, agg_base(P, q, rs, v3)));
      else
        v = r1_tot[r] + PR2[(size_t)r * R + t] + QP[(size_t)r * R + q] + (j - PM[(size_t)r * R + q]);
    }
    unpack[e] = (int32_t)v;
  }
}

// ---------------------------------------------------------------------------
// Transpose of the pack map
// ---------------------------------------------------------------------------
// Keys of the per-rank pack transposes: rank q's pack rows occupy
// [koff[q], koff[q+1]) of one key space (its own rows; its node's rows for
// the 3-step plan), so one stable grouping yields every rank's transpose.
__global__ void k_pack_keys(const int32_t* __restrict__ s1_idx, int64_t E, const int64_t* __restrict__ s1_off,
                            const int64_t* __restrict__ koff, int R, int32_t* keys) {
  GRID_STRIDE(k, E) {
    const int q = upper_rank(s1_off, R, k);
    keys[k] = (int32_t)(koff[q] + s1_idx[k]);
  }
}

// Per-rank transpose arrays from that grouping (pack rows of rank q occupy
// [koff[q], koff[q+1]) and its slots [s1_off[q], s1_off[q+1])).
__global__ void k_local_bt_ptr(const int32_t* __restrict__ gptr, const int64_t* __restrict__ bt_off,
                               const int64_t* __restrict__ koff, const int64_t* __restrict__ s1_off, int R,
                               int64_t total, int32_t* bt_ptr) {
  GRID_STRIDE(i, total) {
    const int q = upper_rank(bt_off, R, i);
    const int64_t li = i - bt_off[q];
    bt_ptr[i] = (int32_t)(gptr[koff[q] + li] - s1_off[q]);
  }
}

__global__ void k_local_bt_perm(const int32_t* __restrict__ gperm, int64_t E, const int64_t* __restrict__ s1_off,
                                int R, int32_t* bt_perm) {
  GRID_STRIDE(k, E) {
    const int q = upper_rank(s1_off, R, k);
    bt_perm[k] = (int32_t)(gperm[k] - s1_off[q]);
  }
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
int check_err(const DevMem& err, const char* what) {
  int h = 0;
  HX_HIP(hipMemcpy(&h, err.p, sizeof h, hipMemcpyDeviceToHost));
  if (h & 1) return fail(HX_ERR_RANGE, "%s: a column index is outside [0, n)", what);
  if (h & 8) return fail(HX_ERR_ARG, "%s: row_ptr is not non-decreasing", what);
  if (h & 2) return fail(HX_ERR_RANGE, "%s: a rank's halo is not strictly increasing", what);
  if (h & 4) return fail(HX_ERR_RANGE, "%s: a halo column is owned by its own rank", what);
  if (h & 16) return fail(HX_ERR_RANGE, "%s: an index is outside its range", what);
  if (h & 32) return fail(HX_ERR_HIP, "%s: internal error: a list entry fell outside its list", what);
  return HX_SUCCESS;
}

int to_host64(const DevMem& d, int64_t n, std::vector<int64_t>* out) {
  out->resize((size_t)n);
  if (n) HX_HIP(hipMemcpy(out->data(), d.p, (size_t)n * 8, hipMemcpyDeviceToHost));
  return HX_SUCCESS;
}

std::vector<int64_t> prefix(const std::vector<int64_t>& v) {
  std::vector<int64_t> o(v.size() + 1, 0);
  for (size_t i = 0; i < v.size(); ++i) o[i + 1] = o[i] + v[i];
  return o;
}

struct Dense {
  DevMem A, P;
  std::vector<int64_t> sum, nnz;  // host per-row sums and nonzero counts
};

// Prefix sums, row sums and nonzero counts of a dense R x R table.
int dense_stats(Dense* t, int R, hipStream_t s) {
  HX_TRY(t->P.alloc((size_t)R * R * 4));
  DevMem sum, nnz;
  HX_TRY(sum.alloc((size_t)R * 8));
  HX_TRY(nnz.alloc((size_t)R * 8));
  hipLaunchKernelGGL(k_row_exscan, dim3(R), dim3(TB), 0, s, t->A.as<int32_t>(), t->P.as<int32_t>(), R,
                     sum.as<int64_t>(), nnz.as<int64_t>());
  HX_HIP(hipGetLastError());
  HX_HIP(hipStreamSynchronize(s));
  HX_TRY(to_host64(sum, R, &t->sum));
  HX_TRY(to_host64(nnz, R, &t->nnz));
  for (int64_t v : t->sum)
    if (v >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "a rank's list exceeds 2^31 entries");
  return HX_SUCCESS;
}

// Emits the (procs, counts, displs) lists of the rows of a dense table.
int dense_lists(const Dense& t, int R, hipStream_t s, hx_plan* p, int f_procs) {
  std::vector<int64_t> off = prefix(t.nnz);
  DevMem off_d;
  HX_TRY(upload_vec(off_d, off));
  const int64_t tot = off.back();
  for (int k = 0; k < 3; ++k) {
    p->off[f_procs + k] = off;
    HX_TRY(p->d[f_procs + k].alloc((size_t)tot * 4));
  }
  if (tot > 0) {
    hipLaunchKernelGGL(k_row_compact, dim3(R), dim3(TB), 0, s, t.A.as<int32_t>(), t.P.as<int32_t>(), R,
                       off_d.as<int64_t>(), p->d[f_procs].as<int32_t>(), p->d[f_procs + 1].as<int32_t>(),
                       p->d[f_procs + 2].as<int32_t>());
    HX_HIP(hipGetLastError());
  }
  HX_HIP(hipStreamSynchronize(s));
  return HX_SUCCESS;
}

int dense_transpose(const DevMem& A, DevMem* AT, int R, hipStream_t s) {
  HX_TRY(AT->alloc((size_t)R * R * 4));
  dim3 g((R + 31) / 32, (R + 31) / 32), b(32, 8);
  hipLaunchKernelGGL(k_transpose, g, b, 0, s, A.as<int32_t>(), AT->as<int32_t>(), R);
  HX_HIP(hipGetLastError());
  return HX_SUCCESS;
}

int zeros(DevMem* d, size_t bytes, hipStream_t s) {
  HX_TRY(d->alloc(bytes));
  if (bytes) HX_HIP(hipMemsetAsync(d->p, 0, bytes, s));
  return HX_SUCCESS;
}

// Builds every plan array from the halos of all ranks (device hcol, host offsets).
int build_from_halos(hx_plan* p, DevMem& hcol, const std::vector<int64_t>& hoff, int check, hipStream_t s) {
  const int R = p->R;
  const int ppn = p->ppn;
  const int64_t n = p->n;
  const int64_t nH = hoff.back();
  const bool loc = p->variant != HX_PLAIN;
  const int v3 = p->variant == HX_LOCALITY_3STEP ? 1 : 0;
  const int NN = (R + ppn - 1) / ppn;
  const Place PL{R, ppn, NN, p->node_map == HX_NODES_CYCLIC ? 1 : 0};
  const int64_t W = (n + 31) / 32;
  const int64_t W1 = W + 1;

  DevMem hoff_d, hrank, own, err;
  HX_TRY(upload_vec(hoff_d, hoff));
  HX_TRY(hrank.alloc((size_t)nH * 4));
  HX_TRY(own.alloc((size_t)nH * 4));
  HX_TRY(zeros(&err, 4, s));
  Dense M;
  HX_TRY(zeros(&M.A, (size_t)R * R * 4, s));
  if (nH > 0) {
    hipLaunchKernelGGL(k_entry_info, dim3(blocks_for(nH)), dim3(TB), 0, s, hcol.as<int32_t>(), nH,
                       hoff_d.as<int64_t>(), p->row_starts_d.as<int64_t>(), R, n, check, hrank.as<int32_t>(),
                       own.as<int32_t>(), M.A.as<int32_t>(), err.as<int>());
    HX_HIP(hipGetLastError());
  }
  HX_HIP(hipStreamSynchronize(s));
  HX_TRY(check_err(err, "halo"));
  HX_TRY(dense_stats(&M, R, s));
  DevMem MT;
  HX_TRY(dense_transpose(M.A, &MT, R, s));

  // halo field
  p->off[HX_F_HALO] = hoff;
  p->off[HX_F_UNPACK_SRC] = hoff;
  p->d[HX_F_HALO] = std::move(hcol);

  // node bitmaps (locality)
  DevMem NB, NBP, MD;
  Dense S1, R1, S2, R2;
  DevMem QP;
  if (loc) {
    HX_TRY(zeros(&NB, (size_t)NN * W1 * 4, s));
    HX_TRY(NBP.alloc((size_t)NN * W1 * 4));
    if (nH > 0) {
      hipLaunchKernelGGL(k_node_mark, dim3(blocks_for(nH)), dim3(TB), 0, s, p->d[HX_F_HALO].as<int32_t>(),
                         hrank.as<int32_t>(), nH, PL, NB.as<uint32_t>(), W1);
      HX_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_word_exscan, dim3(NN), dim3(TB), 0, s, NB.as<uint32_t>(), W1, NBP.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_TRY(MD.alloc((size_t)NN * R * 4));
    hipLaunchKernelGGL(k_dedup_counts, dim3(blocks_for((int64_t)NN * R)), dim3(TB), 0, s, NB.as<uint32_t>(),
                       NBP.as<int32_t>(), W1, p->row_starts_d.as<int64_t>(), PL, v3, MD.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_TRY(S1.A.alloc((size_t)R * R * 4));
    hipLaunchKernelGGL(k_stage1_sizes, dim3(blocks_for((int64_t)R * R)), dim3(TB), 0, s, MT.as<int32_t>(),
                       MD.as<int32_t>(), PL, v3, S1.A.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_TRY(S2.A.alloc((size_t)R * R * 4));
    hipLaunchKernelGGL(k_stage2_sizes, dim3(blocks_for((int64_t)R * R)), dim3(TB), 0, s, M.A.as<int32_t>(), PL,
                       v3, S2.A.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_TRY(zeros(&QP, (size_t)R * R * 4, s));
    hipLaunchKernelGGL(k_class_prefix, dim3(blocks_for((int64_t)R * ppn)), dim3(TB), 0, s, M.A.as<int32_t>(), PL,
                       v3, QP.as<int32_t>());
    HX_HIP(hipGetLastError());
    HX_TRY(dense_transpose(S1.A, &R1.A, R, s));
    HX_TRY(dense_transpose(S2.A, &R2.A, R, s));
    HX_TRY(dense_stats(&S1, R, s));
    HX_TRY(dense_stats(&R1, R, s));
    HX_TRY(dense_stats(&S2, R, s));
    HX_TRY(dense_stats(&R2, R, s));
  } else {
    S1.A = std::move(MT);
    HX_TRY(dense_stats(&S1, R, s));
    // stage-1 receive = M (its prefix sums are the receive displacements)
    R1.A = std::move(M.A);
    R1.P = std::move(M.P);
    R1.sum = M.sum;
    R1.nnz = M.nnz;
  }

  // lists
  HX_TRY(dense_lists(S1, R, s, p, HX_F_S1_PROCS));
  HX_TRY(dense_lists(R1, R, s, p, HX_F_R1_PROCS));
  std::vector<int64_t> s1_off = prefix(S1.sum);
  std::vector<int64_t> s2_off, r1_tot = R1.sum;
  p->off[HX_F_S1_IDX] = s1_off;
  p->off[HX_F_BT_PERM] = s1_off;
  if (loc) {
    HX_TRY(dense_lists(S2, R, s, p, HX_F_S2_PROCS));
    HX_TRY(dense_lists(R2, R, s, p, HX_F_R2_PROCS));
    s2_off = prefix(S2.sum);
  } else {
    std::vector<int64_t> z((size_t)R + 1, 0);
    for (int f : {HX_F_S2_PROCS, HX_F_S2_COUNTS, HX_F_S2_DISPLS, HX_F_R2_PROCS, HX_F_R2_COUNTS, HX_F_R2_DISPLS})
      p->off[f] = z;
    s2_off = z;
  }
  p->off[HX_F_S2_SRC] = s2_off;
  p->r1_off = prefix(R1.sum);
  p->r2_off = loc ? prefix(R2.sum) : std::vector<int64_t>((size_t)R + 1, 0);

  const int64_t E1 = s1_off.back(), E2 = s2_off.back();
  if (E1 >= INT32_MAX || E2 >= INT32_MAX || nH >= INT32_MAX)
    return fail(HX_ERR_UNSUPPORTED, "plan lists beyond 2^31 entries");
  DevMem s1o_d, s2o_d, r1t_d;
  HX_TRY(upload_vec(s1o_d, s1_off));
  HX_TRY(upload_vec(s2o_d, s2_off));
  HX_TRY(upload_vec(r1t_d, r1_tot));
  HX_TRY(p->d[HX_F_S1_IDX].alloc((size_t)E1 * 4));
  HX_TRY(p->d[HX_F_S2_SRC].alloc((size_t)E2 * 4));
  HX_TRY(p->d[HX_F_UNPACK_SRC].alloc((size_t)nH * 4));
  const int32_t* PM = loc ? M.P.as<int32_t>() : R1.P.as<int32_t>();
  if (nH > 0) {
    hipLaunchKernelGGL(k_s1_direct, dim3(blocks_for(nH)), dim3(TB), 0, s, p->d[HX_F_HALO].as<int32_t>(),
                       hrank.as<int32_t>(), own.as<int32_t>(), nH, hoff_d.as<int64_t>(),
                       p->row_starts_d.as<int64_t>(), PL, loc ? 1 : 0, v3, S1.P.as<int32_t>(), PM,
                       s1o_d.as<int64_t>(), p->d[HX_F_S1_IDX].as<int32_t>(), err.as<int>());
    HX_HIP(hipGetLastError());
  }
  if (loc) {
    if (NN * W > 0) {
      hipLaunchKernelGGL(k_s1_agg, dim3(blocks_for((int64_t)NN * W)), dim3(TB), 0, s, NB.as<uint32_t>(),
                         NBP.as<int32_t>(), W1, W, p->row_starts_d.as<int64_t>(), PL, v3,
                         S1.P.as<int32_t>(), s1o_d.as<int64_t>(), p->d[HX_F_S1_IDX].as<int32_t>(), err.as<int>());
      HX_HIP(hipGetLastError());
    }
    if (nH > 0) {
      hipLaunchKernelGGL(k_s2_src, dim3(blocks_for(nH)), dim3(TB), 0, s, p->d[HX_F_HALO].as<int32_t>(),
                         hrank.as<int32_t>(), own.as<int32_t>(), nH, hoff_d.as<int64_t>(),
                         p->row_starts_d.as<int64_t>(), PL, S2.P.as<int32_t>(), QP.as<int32_t>(), PM,
                         R1.P.as<int32_t>(), NB.as<uint32_t>(), NBP.as<int32_t>(), W1, s2o_d.as<int64_t>(), v3,
                         p->d[HX_F_S2_SRC].as<int32_t>(), err.as<int>());
      HX_HIP(hipGetLastError());
    }
  }
  if (nH > 0) {
    hipLaunchKernelGGL(k_unpack_map, dim3(blocks_for(nH)), dim3(TB), 0, s, p->d[HX_F_HALO].as<int32_t>(),
                       hrank.as<int32_t>(), own.as<int32_t>(), nH, hoff_d.as<int64_t>(),
                       p->row_starts_d.as<int64_t>(), PL, loc ? 1 : 0, v3, PM, R1.P.as<int32_t>(),
                       loc ? R2.P.as<int32_t>() : nullptr, loc ? QP.as<int32_t>() : nullptr,
                       loc ? NB.as<uint32_t>() : nullptr, loc ? NBP.as<int32_t>() : nullptr, W1,
                       r1t_d.as<int64_t>(), p->d[HX_F_UNPACK_SRC].as<int32_t>());
    HX_HIP(hipGetLastError());
  }

  HX_HIP(hipStreamSynchronize(s));
  HX_TRY(check_err(err, "plan lists"));

  // transpose of the pack map, per rank over its pack rows (its own rows;
  // its node's rows for the 3-step plan)
  std::vector<int64_t> pack_rows((size_t)R);
  for (int q = 0; q < R; ++q) {
    const int nq = q / ppn;
    pack_rows[q] = v3 ? p->row_starts[std::min(R, (nq + 1) * ppn)] - p->row_starts[nq * ppn]
                      : p->row_starts[q + 1] - p->row_starts[q];
  }
  const std::vector<int64_t> koff = prefix(pack_rows);
  if (koff.back() >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "pack-transpose key space beyond 2^31");
  std::vector<int64_t> bt_off((size_t)R + 1, 0);
  for (int q = 0; q < R; ++q) bt_off[q + 1] = bt_off[q] + pack_rows[q] + 1;
  p->off[HX_F_BT_PTR] = bt_off;
  HX_TRY(p->d[HX_F_BT_PTR].alloc((size_t)bt_off.back() * 4));
  HX_TRY(p->d[HX_F_BT_PERM].alloc((size_t)E1 * 4));
  {
    DevMem keys, gptr, gperm, bto_d, koff_d;
    HX_TRY(keys.alloc((size_t)E1 * 4));
    HX_TRY(gptr.alloc((size_t)(koff.back() + 1) * 4));
    HX_TRY(gperm.alloc((size_t)E1 * 4));
    HX_TRY(upload_vec(bto_d, bt_off));
    HX_TRY(upload_vec(koff_d, koff));
    if (E1 > 0) {
      hipLaunchKernelGGL(k_pack_keys, dim3(blocks_for(E1)), dim3(TB), 0, s, p->d[HX_F_S1_IDX].as<int32_t>(), E1,
                         s1o_d.as<int64_t>(), koff_d.as<int64_t>(), R, keys.as<int32_t>());
      HX_HIP(hipGetLastError());
    }
    HX_TRY(dev_check_range(keys.as<int32_t>(), E1, koff.back(), "pack rows", s));
    HX_TRY(dev_group_by_key(keys.as<int32_t>(), E1, koff.back(), gptr.as<int32_t>(), gperm.as<int32_t>(), s));
    hipLaunchKernelGGL(k_local_bt_ptr, dim3(blocks_for(bt_off.back())), dim3(TB), 0, s, gptr.as<int32_t>(),
                       bto_d.as<int64_t>(), koff_d.as<int64_t>(), s1o_d.as<int64_t>(), R, bt_off.back(),
                       p->d[HX_F_BT_PTR].as<int32_t>());
    HX_HIP(hipGetLastError());
    if (E1 > 0) {
      hipLaunchKernelGGL(k_local_bt_perm, dim3(blocks_for(E1)), dim3(TB), 0, s, gperm.as<int32_t>(), E1,
                         s1o_d.as<int64_t>(), R, p->d[HX_F_BT_PERM].as<int32_t>());
      HX_HIP(hipGetLastError());
    }
    HX_HIP(hipStreamSynchronize(s));
  }
  return HX_SUCCESS;
}

int plan_common_checks(int nranks, const int64_t* row_starts, const hx_info* info, hx_plan** out) {
  if (!out) return fail(HX_ERR_ARG, "null out");
  *out = nullptr;
  if (!info) return fail(HX_ERR_ARG, "null info");
  if (nranks <= 0 || !row_starts) return fail(HX_ERR_ARG, "bad nranks / row_starts");
  if (nranks > HX_PLAN_MAX_RANKS) return fail(HX_ERR_UNSUPPORTED, "more than %d ranks", HX_PLAN_MAX_RANKS);
  const int variant = info->variant;
  if (variant != HX_PLAIN && variant != HX_LOCALITY_2STEP && variant != HX_LOCALITY_3STEP)
    return fail(HX_ERR_ARG, "bad variant");
  if (info->ppn < 1) return fail(HX_ERR_ARG, "ppn must be >= 1");
  if (info->node_map != HX_NODES_BLOCK && info->node_map != HX_NODES_CYCLIC)
    return fail(HX_ERR_ARG, "bad node map");
  if (variant == HX_LOCALITY_3STEP && info->node_map != HX_NODES_BLOCK)
    return fail(HX_ERR_UNSUPPORTED, "the 3-step variant needs block placement (a node's rows contiguous)");
  if (row_starts[0] != 0) return fail(HX_ERR_ARG, "row_starts[0] must be 0");
  for (int r = 0; r < nranks; ++r)
    if (row_starts[r + 1] < row_starts[r]) return fail(HX_ERR_ARG, "row_starts must be non-decreasing");
  if (row_starts[nranks] >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "more than 2^31 rows");
  return HX_SUCCESS;
}

int plan_alloc(int nranks, const int64_t* row_starts, const hx_info* info, std::unique_ptr<hx_plan>* p) {
  p->reset(new (std::nothrow) hx_plan);
  if (!*p) return fail(HX_ERR_NOMEM, "out of host memory");
  (*p)->R = nranks;
  // more ranks per node than ranks is one node of every rank (under either
  // map); clamping keeps every node-index product inside int
  (*p)->ppn = std::min(info->ppn, nranks);
  (*p)->node_map = info->node_map;
  (*p)->variant = info->variant;
  (*p)->n = row_starts[nranks];
  (*p)->row_starts.assign(row_starts, row_starts + nranks + 1);
  HX_TRY(upload_vec((*p)->row_starts_d, (*p)->row_starts));
  return HX_SUCCESS;
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported device utilities
// ---------------------------------------------------------------------------
int dev_exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, (n + SCAN_BLOCK - 1) / SCAN_BLOCK);
  DevMem part;
  HX_TRY(part.alloc((size_t)(nb + 1) * 8));
  hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)nb), dim3(TB), 0, s, in, n, part.as<int64_t>());
  HX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_part_scan, dim3(1), dim3(1024), 0, s, part.as<int64_t>(), nb);
  HX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(TB), 0, s, in, n, part.as<int64_t>(), out);
  HX_HIP(hipGetLastError());
  HX_HIP(hipStreamSynchronize(s));
  return HX_SUCCESS;
}

int dev_group_by_key(const int32_t* keys, int64_t n, int64_t nkeys, int32_t* ptr, int32_t* perm, hipStream_t s) {
  DevMem cnt, cursor, err;
  HX_TRY(zeros(&cnt, (size_t)std::max<int64_t>(nkeys, 1) * 4, s));
  HX_TRY(zeros(&err, 4, s));
  if (n > 0) {
    hipLaunchKernelGGL(k_count_keys, dim3(blocks_for(n)), dim3(TB), 0, s, keys, n, nkeys, cnt.as<int32_t>(),
                       err.as<int>());
    HX_HIP(hipGetLastError());
    HX_HIP(hipStreamSynchronize(s));
    HX_TRY(check_err(err, "grouping"));
  }
  HX_TRY(dev_exclusive_scan_i32(cnt.as<int32_t>(), ptr, nkeys, s));
  if (n > 0) {
    HX_TRY(cursor.alloc((size_t)nkeys * 4));
    HX_HIP(hipMemcpyAsync(cursor.p, ptr, (size_t)nkeys * 4, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_place_keys, dim3(blocks_for(n)), dim3(TB), 0, s, keys, n, nkeys, cursor.as<int32_t>(),
                       perm, err.as<int>());
    HX_HIP(hipGetLastError());
    HX_HIP(hipStreamSynchronize(s));
    HX_TRY(check_err(err, "grouping"));
    hipLaunchKernelGGL(k_sort_groups, dim3(blocks_for(nkeys)), dim3(TB), 0, s, ptr, nkeys, perm);
    HX_HIP(hipGetLastError());
  }
  HX_HIP(hipStreamSynchronize(s));
  return HX_SUCCESS;
}

int dev_check_range(const int32_t* idx, int64_t n, int64_t hi, const char* what, hipStream_t s) {
  if (n <= 0) return HX_SUCCESS;
  DevMem err;
  HX_TRY(zeros(&err, 4, s));
  hipLaunchKernelGGL(k_check_range, dim3(blocks_for(n)), dim3(TB), 0, s, idx, n, hi, err.as<int>());
  HX_HIP(hipGetLastError());
  HX_HIP(hipStreamSynchronize(s));
  return check_err(err, what);
}

int dev_count_nonzero_flags(const int32_t* idx, int64_t n, int64_t domain, int64_t* distinct, hipStream_t s) {
  *distinct = 0;
  if (n <= 0 || domain <= 0) return HX_SUCCESS;
  DevMem flags, acc;
  HX_TRY(zeros(&flags, (size_t)domain * 4, s));
  HX_TRY(zeros(&acc, 8, s));
  hipLaunchKernelGGL(k_flag, dim3(blocks_for(n)), dim3(TB), 0, s, idx, n, domain, flags.as<int32_t>());
  HX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_i32, dim3(blocks_for(domain)), dim3(TB), 0, s, flags.as<int32_t>(), domain,
                     acc.as<unsigned long long>());
  HX_HIP(hipGetLastError());
  unsigned long long h = 0;
  HX_HIP(hipMemcpyAsync(&h, acc.p, 8, hipMemcpyDeviceToHost, s));
  HX_HIP(hipStreamSynchronize(s));
  *distinct = (int64_t)h;
  return HX_SUCCESS;
}

}  // namespace hx

using namespace hx;

// ===========================================================================
// Public plan API
// ===========================================================================
extern "C" int hx_plan_from_csr(int nranks, const int64_t* row_starts, const hx_info* info,
                                const int64_t* row_ptr, const int32_t* cols, void* stream, hx_plan** out) {
  HX_TRY(plan_common_checks(nranks, row_starts, info, out));
  const int64_t n = row_starts[nranks];
  if (n > 0 && !row_ptr) return fail(HX_ERR_ARG, "null row_ptr");
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<hx_plan> p;
  HX_TRY(plan_alloc(nranks, row_starts, info, &p));
  const int64_t W = (n + 31) / 32;
  // Halo discovery marks one bit per (rank, column).  The bitmaps of a group
  // of ranks are built, counted and compacted before the next group, so the
  // bitmap memory stays within a budget whatever the rank count.
  int64_t budget = (int64_t)1 << 30;
  if (const char* e = std::getenv("HX_PLAN_BITMAP_BYTES")) budget = std::max<int64_t>(1, std::atoll(e));
  const int64_t group = std::max<int64_t>(1, std::min<int64_t>(nranks, budget / std::max<int64_t>(W * 4, 1)));
  DevMem B, err, cnt;
  HX_TRY(B.alloc((size_t)std::max<int64_t>(group * W * 4, 4)));
  HX_TRY(zeros(&err, 4, s));
  HX_TRY(cnt.alloc((size_t)group * 8));
  std::vector<int64_t> hoff(1, 0);
  std::vector<DevMem> parts;
  for (int r0 = 0; r0 < nranks; r0 += (int)group) {
    const int g = (int)std::min<int64_t>(group, nranks - r0);
    const int64_t i0 = row_starts[r0], rows = row_starts[r0 + g] - i0;
    if (W > 0) HX_HIP(hipMemsetAsync(B.p, 0, (size_t)g * W * 4, s));
    if (rows > 0) {
      hipLaunchKernelGGL(k_mark_csr, dim3(blocks_for(rows)), dim3(TB), 0, s, p->row_starts_d.as<int64_t>(), nranks,
                         n, i0, rows, r0, row_ptr, cols, B.as<uint32_t>(), W, err.as<int>());
      HX_HIP(hipGetLastError());
    }
    HX_HIP(hipStreamSynchronize(s));
    HX_TRY(check_err(err, "csr"));
    hipLaunchKernelGGL(k_popc_rows, dim3(g), dim3(TB), 0, s, B.as<uint32_t>(), W, cnt.as<int64_t>());
    HX_HIP(hipGetLastError());
    HX_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> hc;
    HX_TRY(to_host64(cnt, g, &hc));
    std::vector<int64_t> off = prefix(hc);
    if (hoff.back() + off.back() >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "total halo beyond 2^31 entries");
    for (int k = 0; k < g; ++k) hoff.push_back(hoff.back() + hc[k]);
    parts.emplace_back();
    if (off.back() > 0) {
      DevMem off_d;
      HX_TRY(upload_vec(off_d, off));
      HX_TRY(parts.back().alloc((size_t)off.back() * 4));
      hipLaunchKernelGGL(k_compact_bits, dim3(g), dim3(TB), 0, s, B.as<uint32_t>(), W, off_d.as<int64_t>(),
                         parts.back().as<int32_t>());
      HX_HIP(hipGetLastError());
      HX_HIP(hipStreamSynchronize(s));
    }
  }
  B.release();
  DevMem hcol;
  if (parts.size() == 1) {
    hcol = std::move(parts[0]);
  } else {
    HX_TRY(hcol.alloc((size_t)hoff.back() * 4));
    int64_t at = 0;
    for (DevMem& d : parts) {
      const int64_t len = (int64_t)(d.bytes / 4);
      if (len > 0)
        HX_HIP(hipMemcpyAsync(hcol.as<int32_t>() + at, d.p, (size_t)len * 4, hipMemcpyDeviceToDevice, s));
      at += len;
    }
    HX_HIP(hipStreamSynchronize(s));
    parts.clear();
  }
  HX_TRY(build_from_halos(p.get(), hcol, hoff, 0, s));
  *out = p.release();
  return HX_SUCCESS;
}

extern "C" int hx_plan_from_halos(int nranks, const int64_t* row_starts, const hx_info* info,
                                  const int64_t* halo_ptr, const int32_t* halo_cols, void* stream,
                                  hx_plan** out) {
  HX_TRY(plan_common_checks(nranks, row_starts, info, out));
  if (!halo_ptr) return fail(HX_ERR_ARG, "null halo_ptr");
  if (halo_ptr[0] != 0) return fail(HX_ERR_ARG, "halo_ptr[0] must be 0");
  for (int r = 0; r < nranks; ++r)
    if (halo_ptr[r + 1] < halo_ptr[r]) return fail(HX_ERR_ARG, "halo_ptr must be non-decreasing");
  const int64_t nH = halo_ptr[nranks];
  if (nH >= INT32_MAX) return fail(HX_ERR_UNSUPPORTED, "total halo beyond 2^31 entries");
  if (nH > 0 && !halo_cols) return fail(HX_ERR_ARG, "null halo_cols");
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<hx_plan> p;
  HX_TRY(plan_alloc(nranks, row_starts, info, &p));
  DevMem hcol;
  HX_TRY(hcol.alloc((size_t)nH * 4));
  if (nH) HX_HIP(hipMemcpyAsync(hcol.p, halo_cols, (size_t)nH * 4, hipMemcpyDeviceToDevice, s));
  std::vector<int64_t> hoff(halo_ptr, halo_ptr + nranks + 1);
  HX_TRY(build_from_halos(p.get(), hcol, hoff, 1, s));
  *out = p.release();
  return HX_SUCCESS;
}

extern "C" int hx_plan_free(hx_plan** p) {
  if (!p) return HX_SUCCESS;
  delete *p;
  *p = nullptr;
  return HX_SUCCESS;
}

extern "C" int hx_plan_field_size(const hx_plan* p, int rank, hx_field f, int64_t* count) {
  if (!p || !count) return fail(HX_ERR_ARG, "null argument");
  if (rank < 0 || rank >= p->R || (int)f < 0 || f >= HX_F_COUNT) return fail(HX_ERR_RANGE, "bad rank or field");
  *count = p->size(f, rank);
  return HX_SUCCESS;
}

extern "C" int hx_plan_describe(const hx_plan* p, int* nranks, int64_t* n, hx_info* info, int64_t* row_starts) {
  if (!p) return fail(HX_ERR_ARG, "null plan");
  if (nranks) *nranks = p->R;
  if (n) *n = p->n;
  if (info) {
    info->variant = p->variant;
    info->ppn = p->ppn;
    info->node_map = p->node_map;
  }
  if (row_starts) std::copy(p->row_starts.begin(), p->row_starts.end(), row_starts);
  return HX_SUCCESS;
}

extern "C" int hx_plan_field_all(const hx_plan* p, hx_field f, int64_t* offsets, int32_t* dst) {
  if (!p) return fail(HX_ERR_ARG, "null plan");
  if ((int)f < 0 || f >= HX_F_COUNT) return fail(HX_ERR_RANGE, "bad field");
  if (offsets) std::copy(p->off[f].begin(), p->off[f].end(), offsets);
  const int64_t c = p->tot(f);
  if (dst && c > 0) HX_HIP(hipMemcpy(dst, p->d[f].p, (size_t)c * 4, hipMemcpyDeviceToHost));
  return HX_SUCCESS;
}

extern "C" int hx_plan_field_copy(const hx_plan* p, int rank, hx_field f, int32_t* dst) {
  int64_t c = 0;
  HX_TRY(hx_plan_field_size(p, rank, f, &c));
  if (c == 0) return HX_SUCCESS;
  if (!dst) return fail(HX_ERR_ARG, "null destination");
  HX_HIP(hipMemcpy(dst, p->d[f].as<int32_t>() + p->off[f][rank], (size_t)c * 4, hipMemcpyDeviceToHost));
  return HX_SUCCESS;
}
