// SILK seeding (paper Section 3.2, Algorithm 4) on gfx950.  Every
// intermediate size stays on the device: kernels read their counts from
// device words and launches are sized by host upper bounds, so the call
// never waits for the GPU and can be captured in a HIP graph.
//
// Once per call:
//   k_silk_setup      global bucket ids (tables one after another), sizes of
//                     the open-addressing table, zeroed counters
//   k_extent          start and size of every bucket in the member array
//   k_mark_starts, scan, k_bucket_of   the global bucket of every (table, object)
// For each SILK table:
//   k_sig / k_sig_big G(B) = (min_{x in B} pi_k(x))_k for every bucket, with the
//                     hash evaluations counted as they are made
//   k_ht_*            bins = buckets with identical G: an open-addressing table
//                     on the exact G; a bin is named by its smallest bucket id
//   k_vote            per object, over its T buckets: the bins of two or more
//                     buckets in which it lies in more than half of the buckets.
//                     The buckets of one table are disjoint, so an object lies
//                     in exactly one bucket per table and its count in a bin is
//                     the number of those T buckets that the bin holds.
//   k_emit_flags, scans, k_commit   C_shared sizes, delta, room left in C
//   k_count_kept, scan, k_kept_pairs, radix sort by bin, k_c_write
//                     the new sets of C, ids ascending
// De-duplication (one more table over the sets of C): sets sorted by their
// K-tuple (radix sort) so that runs of equal tuples are the bins, in
// ascending lexicographic order; a bin of one set passes it through, a bin of
// several sets is majority-voted ((bin, id) pairs sorted and counted) and
// delta-filtered; the seeds are written in bin order.
#include <vector>

#include "common.hpp"
#include "radix.hpp"

namespace geek {

constexpr int SK_BIG = 64;       // buckets larger than this are hashed by a wavefront
constexpr int SG_GRID = 2048;    // blocks of the grid-stride kernels
constexpr int SV_LDS = 8192;     // LDS entries (two words each) of a vote block
constexpr int SILK_MAX_T = 128;  // transform tables the vote kernel holds in LDS

// Device-side sizes and counters of one call.
struct SilkState {
  unsigned long long hash_evals, pairs, multi, need_s, need_m;
  uint32_t nb;       // buckets of all tables
  uint32_t ht_mask;  // open-addressing table: mask + 1 slots in use
  uint32_t big;      // buckets queued for k_sig_big
  uint32_t es, em;   // this table's emitted sets / members
  uint32_t kp;       // this table's kept (bin, id) pairs of emitted bins
  uint32_t cs, cm;   // sets / members of C committed so far
  uint32_t over;     // C ran out of room
  uint32_t fit;      // this table's sets are written to C
  uint32_t base_s, base_m;
  // de-duplication
  uint32_t nb2, P2, R2, kept2, k, tot_m, fit_out;
};

GEEK_D uint32_t gtid() { return blockIdx.x * blockDim.x + threadIdx.x; }
GEEK_D uint32_t gstride() { return gridDim.x * blockDim.x; }

// Block sum of one 64-bit value per thread, added to *dst by one thread.
GEEK_D void block_add(unsigned long long v, unsigned long long* dst) {
  __shared__ unsigned long long red[16];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) t += red[w];
    if (t) atomicAdd(dst, t);
  }
}

__global__ void k_silk_setup(const uint32_t* __restrict__ nbuckets, int T, int64_t n, uint32_t* __restrict__ base,
                             SilkState* S) {
  if (blockIdx.x || threadIdx.x) return;
  uint32_t r = 0;
  for (int t = 0; t < T; ++t) {
    base[t] = r;
    const uint32_t v = nbuckets[t];
    r += v < (uint32_t)n ? v : (uint32_t)n;
  }
  base[T] = r;
  uint32_t slots = 1024;
  while (slots < 2u * r && slots < 0x80000000u) slots <<= 1;
  *S = SilkState{};
  S->nb = r;
  S->ht_mask = slots - 1;
}

// Start (in the flattened [T][n] member array) and size of every bucket.
__global__ void k_extent(const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ base, int T, int64_t n,
                         const SilkState* S, uint32_t* __restrict__ gstart, uint32_t* __restrict__ gsize) {
  const uint32_t NB = S->nb;
  for (uint32_t g = gtid(); g < NB; g += gstride()) {
    int lo = 0, hi = T;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (base[mid] <= g) lo = mid; else hi = mid;
    }
    const uint32_t j = g - base[lo];
    const uint32_t o = offsets[(int64_t)lo * (n + 1) + j], e = offsets[(int64_t)lo * (n + 1) + j + 1];
    gstart[g] = (uint32_t)((int64_t)lo * n + o);
    gsize[g] = e - o;
  }
}

__global__ void k_sk_fill(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

__global__ void k_mark_starts(const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ count,
                              uint32_t* __restrict__ flag) {
  const uint32_t ns = *count;
  for (uint32_t g = gtid(); g < ns; g += gstride()) flag[gstart[g]] = 1u;
}

// Position q of the flattened member array lies in bucket fscan[q] + flag[q]
// - 1 (buckets are numbered in member-array order); its object's entry of
// table q / n gets that bucket.
__global__ void k_bucket_of(const uint32_t* __restrict__ members, int64_t Tn, int64_t n,
                            const uint32_t* __restrict__ flag, const uint32_t* __restrict__ fscan,
                            uint32_t* __restrict__ bof) {
  for (int64_t q = gtid(); q < Tn; q += gstride()) {
    const int64_t t = q / n;
    const uint32_t m = members[q];
    if (m < (uint32_t)n) bof[t * n + m] = fscan[q] + flag[q] - 1u;
  }
}

// Signature of every set (one thread per set of at most SK_BIG members;
// larger sets are queued for k_sig_big).  *count sets, the K key pairs of
// this table at keys.  Adds the pi evaluations made to *evals.
__global__ __launch_bounds__(256) void k_sig(const uint32_t* __restrict__ mem, const uint32_t* __restrict__ gstart,
                                             const uint32_t* __restrict__ gsize, const uint32_t* __restrict__ count,
                                             const uint32_t* __restrict__ keys, int K, uint32_t* __restrict__ G,
                                             uint32_t* __restrict__ big_list, uint32_t* big_count,
                                             unsigned long long* evals) {
  const uint32_t ns = *count;
  uint32_t a[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = k < K ? (keys[2 * k] | 1u) : 1u;
    b[k] = k < K ? keys[2 * k + 1] : 0u;
  }
  unsigned long long done = 0;
  for (uint32_t g = gtid(); g < ns; g += gstride()) {
    const uint32_t sz = gsize[g];
    if (sz > SK_BIG) {
      big_list[atomicAdd(big_count, 1u)] = g;
      continue;
    }
    uint32_t mn[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    const uint32_t* p = mem + gstart[g];
    for (uint32_t q = 0; q < sz; ++q) {
      const uint32_t y = fmix32(p[q]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t v = perm_premixed(a[k], b[k], y);
        mn[k] = v < mn[k] ? v : mn[k];
      }
    }
    done += (unsigned long long)sz * K;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < K) G[(int64_t)g * K + k] = mn[k];
  }
  if (evals) block_add(done, evals);
}

// Signatures of the queued large sets: one wavefront per set, the lanes
// striding over its members, then a shuffle reduction of the K minima.
__global__ __launch_bounds__(256) void k_sig_big(const uint32_t* __restrict__ mem,
                                                 const uint32_t* __restrict__ gstart,
                                                 const uint32_t* __restrict__ gsize,
                                                 const uint32_t* __restrict__ keys, int K,
                                                 uint32_t* __restrict__ G, const uint32_t* big_list,
                                                 const uint32_t* big_count, unsigned long long* evals) {
  const uint32_t nbig = *big_count;
  const int lane = threadIdx.x & 63;
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
  uint32_t a[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = k < K ? (keys[2 * k] | 1u) : 1u;
    b[k] = k < K ? keys[2 * k + 1] : 0u;
  }
  unsigned long long done = 0;
  for (uint32_t bi = wave; bi < nbig; bi += nwave) {
    const uint32_t g = big_list[bi];
    uint32_t mn[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    const uint32_t* p = mem + gstart[g];
    const uint32_t sz = gsize[g];
    // four members per lane and step, their loads issued together
    for (uint32_t q0 = 0; q0 < sz; q0 += 256) {
      uint32_t x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t q = q0 + u * 64 + lane;
        x[u] = q < sz ? p[q] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (q0 + u * 64 + lane >= sz) continue;
        const uint32_t y = fmix32(x[u]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t v = perm_premixed(a[k], b[k], y);
          mn[k] = v < mn[k] ? v : mn[k];
        }
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t v = (uint32_t)__shfl_xor((int)mn[k], o);
        mn[k] = v < mn[k] ? v : mn[k];
      }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (lane == k && k < K) G[(int64_t)g * K + k] = mn[k];
    done += (unsigned long long)sz * K;
  }
  if (evals && lane == 0 && done) atomicAdd(evals, done);
}

// ---- bins of identical G (SILK tables) ---------------------------------------
GEEK_D uint32_t g_hash(const uint32_t* __restrict__ G, uint32_t g, int K) {
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  for (int k = 0; k < K; ++k) w[k] = G[(int64_t)g * K + k];
  return key_hash(w, 4);
}
GEEK_D bool g_eq(const uint32_t* __restrict__ G, uint32_t a, uint32_t b, int K) {
  for (int k = 0; k < K; ++k)
    if (G[(int64_t)a * K + k] != G[(int64_t)b * K + k]) return false;
  return true;
}

__global__ void k_ht_clear(const SilkState* S, uint32_t* __restrict__ ht, uint32_t* __restrict__ binmin,
                           uint32_t* __restrict__ bcount, uint32_t* __restrict__ ksize) {
  const uint32_t NB = S->nb, slots = S->ht_mask + 1u;
  const uint32_t top = slots > NB ? slots : NB;
  for (uint32_t i = gtid(); i < top; i += gstride()) {
    if (i < slots) ht[i] = 0u;
    if (i < NB) {
      binmin[i] = 0xFFFFFFFFu;
      bcount[i] = 0u;
      ksize[i] = 0u;
    }
  }
}

// Open addressing with linear probing: a slot holds 1 + the bucket that
// claimed it; a probe that meets another bucket compares the exact G (the
// claimant's G is complete before this kernel starts), so no slot is ever
// read before its key exists.  rep[g] = the claimant of g's G.
__global__ void k_ht_insert(const uint32_t* __restrict__ G, int K, const SilkState* S, uint32_t* __restrict__ ht,
                            uint32_t* __restrict__ rep) {
  const uint32_t NB = S->nb, mask = S->ht_mask;
  for (uint32_t g = gtid(); g < NB; g += gstride()) {
    uint32_t h = g_hash(G, g, K) & mask;
    uint32_t r = g;
    for (;;) {  // at most mask + 1 > NB probes: the table is never full
      const uint32_t prev = atomicCAS(&ht[h], 0u, g + 1u);
      if (prev == 0u) break;
      if (g_eq(G, prev - 1u, g, K)) {
        r = prev - 1u;
        break;
      }
      h = (h + 1u) & mask;
    }
    rep[g] = r;
  }
}

__global__ void k_ht_min(const uint32_t* __restrict__ rep, const SilkState* S, uint32_t* __restrict__ binmin,
                         uint32_t* __restrict__ bcount) {
  const uint32_t NB = S->nb;
  for (uint32_t g = gtid(); g < NB; g += gstride()) {
    const uint32_t r = rep[g];
    atomicMin(&binmin[r], g);
    atomicAdd(&bcount[r], 1u);
  }
}

// info[g] = (bin id = smallest bucket of the bin, number of buckets in it);
// counts the bins of two or more buckets.
__global__ __launch_bounds__(256) void k_bin_info(const uint32_t* __restrict__ rep,
                                                  const uint32_t* __restrict__ binmin,
                                                  const uint32_t* __restrict__ bcount, SilkState* S,
                                                  uint2* __restrict__ info) {
  const uint32_t NB = S->nb;
  unsigned long long multi = 0;
  for (uint32_t g = gtid(); g < NB; g += gstride()) {
    const uint32_t r = rep[g];
    const uint32_t b = binmin[r], c = bcount[r];
    info[g] = make_uint2(b, c);
    multi += (b == g && c >= 2u) ? 1ull : 0ull;
  }
  block_add(multi, &S->multi);
}

// Majority vote per object.  Object i lies in bucket bof[t][i] of table t;
// the entries whose bin holds two or more buckets go to this thread's LDS
// column, then each distinct bin is counted.  The object joins C_shared of a
// bin when 2 * count > |Bin| (count >= 2, so at most T / 2 bins per object);
// those bins are listed in kbin[j][i], their number in kc[i], and ksize[bin]
// counts the bin's voted ids.  Adds the (bin, id) pairs voted to S->pairs.
__global__ __launch_bounds__(256) void k_vote(const uint32_t* __restrict__ bof, const uint2* __restrict__ info,
                                              int64_t n, int T, uint32_t* __restrict__ kbin,
                                              uint32_t* __restrict__ kc, uint32_t* __restrict__ ksize,
                                              SilkState* S) {
  extern __shared__ uint32_t vl[];  // [2][T][blockDim.x]: bin id, bin size
  const int VT = blockDim.x;
  uint32_t* lb = vl;
  uint32_t* ls = vl + (size_t)T * VT;
  unsigned long long pairs = 0;
  const int x = threadIdx.x;
  const uint32_t NB = S->nb;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    int c = 0;
    for (int t = 0; t < T; ++t) {
      const uint32_t g = bof[(int64_t)t * n + i];
      const uint2 e = g < NB ? info[g] : make_uint2(0u, 0u);  // bounded even for a malformed CSR
      if (e.y >= 2u) {
        lb[c * VT + x] = e.x;
        ls[c * VT + x] = e.y;
        ++c;
      }
    }
    pairs += (unsigned long long)c;
    uint32_t kept = 0;
    for (int a = 0; a < c; ++a) {
      const uint32_t b = lb[a * VT + x];
      bool first = true;
      for (int q = 0; q < a && first; ++q) first = lb[q * VT + x] != b;
      if (!first) continue;
      uint32_t cnt = 1;
      for (int q = a + 1; q < c; ++q) cnt += lb[q * VT + x] == b ? 1u : 0u;
      if (2u * cnt > ls[a * VT + x]) {
        kbin[(int64_t)kept * n + i] = b;
        ++kept;
        atomicAdd(&ksize[b], 1u);
      }
    }
    kc[i] = kept;
  }
  block_add(pairs, &S->pairs);
}

// The same vote with the object's T <= TT bin ids in registers
// (compile-time indices, no LDS round trips): entries of bins with fewer than
// two buckets, and entries past T, hold no bin.  A bin's size is read back
// from its smallest bucket's entry (info[bin] = (bin, size)) once per
// distinct bin.  The per-table loads go in batches of VB tables (their
// buckets, then those buckets' bin entries), each batch issued whole before
// its values are used.
constexpr int VB = 8;
template <int TT>
__global__ __launch_bounds__(256) void k_vote_reg(const uint32_t* __restrict__ bof, const uint2* __restrict__ info,
                                                  int64_t n, int T, uint32_t* __restrict__ kbin,
                                                  uint32_t* __restrict__ kc, uint32_t* __restrict__ ksize,
                                                  SilkState* S) {
  constexpr uint32_t NONE = 0xFFFFFFFFu;
  const uint32_t NB = S->nb;
  unsigned long long pairs = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    uint32_t lb[TT];
#pragma unroll
    for (int t0 = 0; t0 < TT; t0 += VB) {
      uint32_t g[VB];
#pragma unroll
      for (int u = 0; u < VB; ++u) g[u] = t0 + u < T ? bof[(int64_t)(t0 + u) * n + i] : NONE;
      uint2 e[VB];
#pragma unroll
      for (int u = 0; u < VB; ++u) {
        e[u] = make_uint2(0u, 0u);
        if (g[u] < NB) e[u] = info[g[u]];  // bounded even for a malformed CSR
      }
#pragma unroll
      for (int u = 0; u < VB; ++u) {
        lb[t0 + u] = e[u].y >= 2u ? e[u].x : NONE;
        pairs += e[u].y >= 2u ? 1u : 0u;
      }
    }
    // entry a is taken at lb[0]; the array turns left by one per step, so
    // the entries before a sit at positions TT - a .. TT - 1 (each step's
    // comparisons are used at once instead of kept for later steps)
    uint32_t kept = 0;
#pragma unroll 1
    for (int a = 0; a < T; ++a) {
      const uint32_t h = lb[0];
      uint32_t cnt = 0;
      bool first = true;
#pragma unroll
      for (int q = 0; q < TT; ++q) {
        const bool eq = lb[q] == h;
        cnt += eq ? 1u : 0u;
        if (q >= TT - a) first = first && !eq;
      }
      // a majority needs cnt >= 2 (2 * cnt > size >= 2)
      if (h != NONE && first && cnt >= 2u && 2u * cnt > info[h].y) {
        kbin[(int64_t)kept * n + i] = h;
        ++kept;
        atomicAdd(&ksize[h], 1u);
      }
#pragma unroll
      for (int q = 0; q < TT - 1; ++q) lb[q] = lb[q + 1];
      lb[TT - 1] = h;
    }
    kc[i] = kept;
  }
  block_add(pairs, &S->pairs);
}

// Bins that join C: named by their smallest bucket, two or more buckets,
// C_shared non-empty and of at least delta ids.
__global__ void k_emit_flags(const uint2* __restrict__ info, const uint32_t* __restrict__ ksize, int delta,
                             const SilkState* S, uint32_t* __restrict__ eone, uint32_t* __restrict__ esz) {
  const uint32_t NB = S->nb;
  const uint32_t dmin = delta > 1 ? (uint32_t)delta : 1u;
  for (uint32_t g = gtid(); g < NB; g += gstride()) {
    const uint2 e = info[g];
    const uint32_t ks = ksize[g];
    const bool on = e.x == g && e.y >= 2u && ks >= dmin;
    eone[g] = on ? 1u : 0u;
    esz[g] = on ? ks : 0u;
  }
}

// Room in C for this table's sets (C holds scap sets and mcap members); once
// C has run out of room no later table writes to it, but the sizes needed are
// still counted.
__global__ void k_commit(SilkState* S, uint32_t scap, uint32_t mcap) {
  if (blockIdx.x || threadIdx.x) return;
  const uint32_t es = S->es, em = S->em;
  S->need_s += es;
  S->need_m += em;
  if (!S->over && (uint64_t)S->cs + es <= scap && (uint64_t)S->cm + em <= mcap) {
    S->fit = 1u;
    S->base_s = S->cs;
    S->base_m = S->cm;
    S->cs += es;
    S->cm += em;
  } else {
    S->fit = 0u;
    S->over = 1u;
  }
}

// Emitted bins per object (zero for every object when the table does not
// fit in C, so the sort that follows has nothing to do).
__global__ void k_count_kept(const uint32_t* __restrict__ kbin, const uint32_t* __restrict__ kc, int64_t n,
                             const uint32_t* __restrict__ eone, const SilkState* S, uint32_t* __restrict__ kc2) {
  const bool fit = S->fit != 0u;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    uint32_t m = 0;
    if (fit) {
      const uint32_t c = kc[i];
      for (uint32_t j = 0; j < c; ++j) m += eone[kbin[(int64_t)j * n + i]];
    }
    kc2[i] = m;
  }
}

// (emitted bin index, id) pairs in id order: a stable sort by the bin index
// then lists every C_shared with its ids ascending.
__global__ void k_kept_pairs(const uint32_t* __restrict__ kbin, const uint32_t* __restrict__ kc, int64_t n,
                             const uint32_t* __restrict__ eone, const uint32_t* __restrict__ eidx,
                             const uint32_t* __restrict__ kpos, const SilkState* S, uint32_t* __restrict__ phi,
                             uint32_t* __restrict__ plo) {
  if (!S->fit) return;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint32_t c = kc[i];
    uint32_t p = kpos[i];
    for (uint32_t j = 0; j < c; ++j) {
      const uint32_t b = kbin[(int64_t)j * n + i];
      if (eone[b]) {
        phi[p] = eidx[b];
        plo[p] = (uint32_t)i;
        ++p;
      }
    }
  }
}

__global__ void k_c_write(const uint32_t* __restrict__ sorted_ids, const uint32_t* __restrict__ eone,
                          const uint32_t* __restrict__ eidx, const uint32_t* __restrict__ eoff, const SilkState* S,
                          uint32_t* __restrict__ cmem, uint32_t* __restrict__ coff) {
  if (!S->fit) return;
  const uint32_t em = S->em, NB = S->nb, bs = S->base_s, bm = S->base_m;
  for (uint32_t q = gtid(); q < em; q += gstride()) cmem[bm + q] = sorted_ids[q];
  for (uint32_t g = gtid(); g < NB; g += gstride())
    if (eone[g]) coff[bs + eidx[g]] = bm + eoff[g];
}

// ---- de-duplication ------------------------------------------------------------
__global__ void k_dd_setup(SilkState* S, uint32_t* __restrict__ coff) {
  if (blockIdx.x || threadIdx.x) return;
  coff[S->cs] = S->cm;
}

__global__ void k_set_extent(const uint32_t* __restrict__ coff, const SilkState* S, uint32_t* __restrict__ gstart,
                             uint32_t* __restrict__ gsize) {
  const uint32_t cs = S->cs;
  for (uint32_t s = gtid(); s < cs; s += gstride()) {
    gstart[s] = coff[s];
    gsize[s] = coff[s + 1] - coff[s];
  }
}

// The K-tuples of C's sets as separate key words (word 0 most significant)
// with the set index as payload.
__global__ void k_dd_tuples(const uint32_t* __restrict__ G, int K, const SilkState* S, uint32_t* __restrict__ w0,
                            uint32_t* __restrict__ w1, uint32_t* __restrict__ w2, uint32_t* __restrict__ w3,
                            uint32_t* __restrict__ val) {
  const uint32_t cs = S->cs;
  for (uint32_t s = gtid(); s < cs; s += gstride()) {
    w0[s] = G[(int64_t)s * K];
    w1[s] = K > 1 ? G[(int64_t)s * K + 1] : 0u;
    w2[s] = K > 2 ? G[(int64_t)s * K + 2] : 0u;
    w3[s] = K > 3 ? G[(int64_t)s * K + 3] : 0u;
    val[s] = s;
  }
}

// Heads of runs of equal tuples in sorted order.
__global__ void k_dd_heads(const uint32_t* __restrict__ w0, const uint32_t* __restrict__ w1,
                           const uint32_t* __restrict__ w2, const uint32_t* __restrict__ w3, const SilkState* S,
                           uint32_t* __restrict__ h) {
  const uint32_t cs = S->cs;
  for (uint32_t r = gtid(); r < cs; r += gstride())
    h[r] = (r == 0 || w0[r] != w0[r - 1] || w1[r] != w1[r - 1] || w2[r] != w2[r - 1] || w3[r] != w3[r - 1]) ? 1u
                                                                                                               : 0u;
}

// Bin of every sorted position, each bin's first position (bstart[nb2] =
// cs), the voting pairs of every set in a bin of two or more sets, and the
// sorted position of every set.
__global__ void k_dd_bins(const uint32_t* __restrict__ h, const uint32_t* __restrict__ hs,
                          const uint32_t* __restrict__ ord, const SilkState* S, uint32_t* __restrict__ binofr,
                          uint32_t* __restrict__ bstart, uint32_t* __restrict__ inv) {
  const uint32_t cs = S->cs;
  for (uint32_t r = gtid(); r < cs; r += gstride()) {
    const uint32_t b = hs[r] + h[r] - 1u;
    binofr[r] = b;
    if (h[r]) bstart[b] = r;
    if (r == cs - 1u) bstart[b + 1u] = cs;
    inv[ord[r]] = r;
  }
}

__global__ void k_dd_cnt(const uint32_t* __restrict__ ord, const uint32_t* __restrict__ binofr,
                         const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ gsize, const SilkState* S,
                         uint32_t* __restrict__ cnt) {
  const uint32_t cs = S->cs;
  for (uint32_t r = gtid(); r < cs; r += gstride()) {
    const uint32_t b = binofr[r];
    cnt[r] = (bstart[b + 1] - bstart[b] >= 2u) ? gsize[ord[r]] : 0u;
  }
}

// One thread per member position of C: (bin, id) of members of sets in bins
// of two or more sets.
__global__ void k_dd_pairs(const uint32_t* __restrict__ cmem, const uint32_t* __restrict__ flag,
                           const uint32_t* __restrict__ fscan, const uint32_t* __restrict__ coff,
                           const uint32_t* __restrict__ inv, const uint32_t* __restrict__ cnt,
                           const uint32_t* __restrict__ poff, const uint32_t* __restrict__ binofr, const SilkState* S,
                           uint32_t* __restrict__ hi, uint32_t* __restrict__ lo) {
  const uint32_t cm = S->cm;
  for (uint32_t q = gtid(); q < cm; q += gstride()) {
    const uint32_t s = fscan[q] + flag[q] - 1u;
    const uint32_t r = inv[s];
    if (cnt[r] == 0u) continue;
    const uint32_t p = poff[r] + (q - coff[s]);
    hi[p] = binofr[r];
    lo[p] = cmem[q];
  }
}

__global__ void k_run_heads(const uint32_t* __restrict__ hi, const uint32_t* __restrict__ lo,
                            const uint32_t* __restrict__ count, uint32_t* __restrict__ h) {
  const uint32_t P = *count;
  for (uint32_t q = gtid(); q < P; q += gstride())
    h[q] = (q == 0 || hi[q] != hi[q - 1] || lo[q] != lo[q - 1]) ? 1u : 0u;
}

__global__ void k_starts(const uint32_t* __restrict__ h, const uint32_t* __restrict__ hs,
                         const uint32_t* __restrict__ count, const uint32_t* __restrict__ total,
                         uint32_t* __restrict__ start) {
  const uint32_t P = *count;
  for (uint32_t q = gtid(); q <= P; q += gstride()) {
    if (q == P) start[*total] = P;
    else if (h[q]) start[hs[q]] = q;
  }
}

// Majority of every (bin, id) run of the de-duplication pairs.
__global__ void k_dd_keep(const uint32_t* __restrict__ rstart, const uint32_t* __restrict__ hi,
                          const uint32_t* __restrict__ bstart, const SilkState* S, uint32_t* __restrict__ kept) {
  const uint32_t R = S->R2;
  for (uint32_t r = gtid(); r < R; r += gstride()) {
    const uint32_t len = rstart[r + 1] - rstart[r];
    const uint32_t b = hi[rstart[r]];
    kept[r] = (2u * len > bstart[b + 1] - bstart[b]) ? 1u : 0u;
  }
}

__global__ void k_dd_compact(const uint32_t* __restrict__ rstart, const uint32_t* __restrict__ kept,
                             const uint32_t* __restrict__ kidx, const uint32_t* __restrict__ hi,
                             const uint32_t* __restrict__ lo, const SilkState* S, uint32_t* __restrict__ klo,
                             uint32_t* __restrict__ khi) {
  const uint32_t R = S->R2;
  for (uint32_t r = gtid(); r < R; r += gstride()) {
    if (!kept[r]) continue;
    khi[kidx[r]] = hi[rstart[r]];
    klo[kidx[r]] = lo[rstart[r]];
  }
}

// The kept ids are sorted by bin: each bin's run [kstart, kend) from the run
// boundaries (bins with no kept id keep 0, 0).
__global__ void k_dd_kruns(const uint32_t* __restrict__ khi, const SilkState* S, uint32_t* __restrict__ kstart,
                           uint32_t* __restrict__ kend) {
  const uint32_t K2 = S->kept2;
  for (uint32_t q = gtid(); q < K2; q += gstride()) {
    const uint32_t b = khi[q];
    if (q == 0 || khi[q - 1] != b) kstart[b] = q;
    if (q + 1 == K2 || khi[q + 1] != b) kend[b] = q + 1;
  }
}

// Seed size of every de-duplication bin (bins in ascending tuple order): a
// single set passes through; several sets keep their voted ids when at least
// delta (and at least one) of them remain.
__global__ void k_dd_size(const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ ord,
                          const uint32_t* __restrict__ gsize, const uint32_t* __restrict__ kstart,
                          const uint32_t* __restrict__ kend, int delta, const SilkState* S,
                          uint32_t* __restrict__ ssz, uint32_t* __restrict__ one) {
  const uint32_t nb2 = S->nb2;
  const uint32_t dmin = delta > 1 ? (uint32_t)delta : 1u;
  for (uint32_t b = gtid(); b < nb2; b += gstride()) {
    const uint32_t bs = bstart[b + 1] - bstart[b];
    const uint32_t kz = kend[b] - kstart[b];
    uint32_t v;
    if (bs == 1u) v = gsize[ord[bstart[b]]];
    else v = kz >= dmin ? kz : 0u;
    ssz[b] = v;
    one[b] = v ? 1u : 0u;
  }
}

__global__ void k_silk_finish(SilkState* S, uint64_t cap_k, uint64_t cap_m, uint32_t* __restrict__ seed_off,
                              uint32_t* k_out, unsigned long long* needed, unsigned long long* counters,
                              int32_t* st) {
  if (blockIdx.x || threadIdx.x) return;
  S->fit_out = 0u;
  if (counters) {
    counters[0] = S->hash_evals;
    counters[1] = S->pairs;
    counters[2] = S->need_s;
    counters[3] = S->multi;
  }
  if (S->over) {
    // C did not fit: report the room for its members that makes it fit (the
    // seeds are not known yet)
    needed[0] = 0;
    needed[1] = 0;
    needed[2] = S->need_m;
    *k_out = 0;
    set_status(st, GEEK_ERR_CAPACITY);
    return;
  }
  const uint32_t k = S->cs ? S->k : 0u, m = S->cs ? S->tot_m : 0u;
  needed[0] = k;
  needed[1] = m;
  needed[2] = S->cm;
  if (k > cap_k || m > cap_m) {
    *k_out = 0;
    set_status(st, GEEK_ERR_CAPACITY);
    return;
  }
  seed_off[k] = m;
  *k_out = k;
  S->fit_out = 1u;
  if (k == 0) set_status(st, GEEK_ERR_NO_SEEDS);
}

__global__ void k_emit_seeds(const uint32_t* __restrict__ ssz, const uint32_t* __restrict__ soff,
                             const uint32_t* __restrict__ sidx, const SilkState* S, uint32_t* __restrict__ seed_off) {
  if (!S->fit_out || !S->cs) return;
  const uint32_t nb2 = S->nb2;
  for (uint32_t b = gtid(); b < nb2; b += gstride())
    if (ssz[b]) seed_off[sidx[b]] = soff[b];
}

// The last index r in [0, cnt) with off[r] <= e (off non-decreasing): the
// non-empty entry whose output range holds position e.
GEEK_D uint32_t range_of(const uint32_t* __restrict__ off, uint32_t cnt, uint32_t e) {
  uint32_t lo = 0, hi = cnt - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One thread per seed member: from the set that passes through or from the
// bin's voted ids.
__global__ void k_seed_copy(const uint32_t* __restrict__ soff, const uint32_t* __restrict__ bstart,
                            const uint32_t* __restrict__ ord, const uint32_t* __restrict__ cmem,
                            const uint32_t* __restrict__ coff, const uint32_t* __restrict__ klo,
                            const uint32_t* __restrict__ kstart, const SilkState* S,
                            uint32_t* __restrict__ seed_mem) {
  if (!S->fit_out || !S->cs) return;
  const uint32_t tot = S->tot_m, nb2 = S->nb2;
  for (uint32_t e = gtid(); e < tot; e += gstride()) {
    const uint32_t b = range_of(soff, nb2, e);
    const uint32_t q = e - soff[b];
    const uint32_t bs = bstart[b + 1] - bstart[b];
    seed_mem[e] = bs == 1u ? cmem[coff[ord[bstart[b]]] + q] : klo[kstart[b] + q];
  }
}

// ---------------------------------------------------------------- host side
struct SilkWs {
  int64_t Tn, Ccap, Cs, KPmax, NS, NM;  // C's members / sets; NS, NM: sets, positions of either phase
  uint32_t ht_slots;
  SilkState* S;
  uint32_t *base, *gstart, *gsize, *G, *bof, *flag, *fscan, *ht, *rep, *binmin, *bcount, *ksize;
  uint2* info;
  uint32_t *eone, *esz, *eidx, *eoff, *kbin, *kc, *kc2, *kpos;
  uint32_t *phi, *plo, *phi2, *plo2;
  uint32_t *cmem, *coff;
  uint32_t *tw[4], *tv, *tw2[4], *tv2;
  uint32_t *h, *hs, *binofr, *bstart, *inv, *cnt, *poff, *rstart, *kept, *kidx, *klo, *khi, *kend, *kstart;
  uint32_t *ssz, *sone, *soff, *sidx;
  uint32_t *big_list, *radix_tmp, *scan_tmp;
};

// Room of the multiset C: cap_c members (4 * cap_members when cap_c is 0);
// every set of C holds at least max(delta, 1) members, which bounds its sets.
static int64_t c_members(const geek_silk_job& J) {
  return J.cap_c > 0 ? J.cap_c : 4 * (J.cap_members > 0 ? J.cap_members : 1);
}

static size_t carve_silk(const geek_silk_job& J, void* ws, SilkWs& W) {
  Carver c(ws);
  W.Tn = (int64_t)J.T * J.n;
  W.Ccap = c_members(J);
  W.Cs = W.Ccap / (J.delta > 1 ? J.delta : 1) + 1;
  W.KPmax = (int64_t)((J.T + 1) / 2) * J.n;
  W.NS = W.Tn > W.Cs ? W.Tn : W.Cs;
  W.NM = W.Tn > W.Ccap ? W.Tn : W.Ccap;
  uint64_t slots = 1024;
  while (slots < 2u * (uint64_t)W.Tn && slots < 0x80000000ull) slots <<= 1;
  W.ht_slots = (uint32_t)slots;
  const int64_t NS = W.NS, Tn = W.Tn, Cc = W.Ccap, Cs = W.Cs;
  const int64_t npairs = W.KPmax > Cc ? W.KPmax : Cc;
  W.S = c.take<SilkState>(1);
  W.base = c.take<uint32_t>(J.T + 1);
  W.gstart = c.take<uint32_t>(NS + 1);
  W.gsize = c.take<uint32_t>(NS + 1);
  W.G = c.take<uint32_t>(NS * J.K);
  W.bof = c.take<uint32_t>(Tn);
  W.flag = c.take<uint32_t>(W.NM + 1);
  W.fscan = c.take<uint32_t>(W.NM + 1);
  W.ht = c.take<uint32_t>(slots);
  W.rep = c.take<uint32_t>(Tn);
  W.binmin = c.take<uint32_t>(Tn);
  W.bcount = c.take<uint32_t>(Tn);
  W.ksize = c.take<uint32_t>(Tn);
  W.info = c.take<uint2>(Tn);
  W.eone = c.take<uint32_t>(Tn + 1);
  W.esz = c.take<uint32_t>(Tn + 1);
  W.eidx = c.take<uint32_t>(Tn + 1);
  W.eoff = c.take<uint32_t>(Tn + 1);
  W.kbin = c.take<uint32_t>(W.KPmax);
  W.kc = c.take<uint32_t>(J.n + 1);
  W.kc2 = c.take<uint32_t>(J.n + 1);
  W.kpos = c.take<uint32_t>(J.n + 1);
  W.phi = c.take<uint32_t>(npairs);
  W.plo = c.take<uint32_t>(npairs);
  W.phi2 = c.take<uint32_t>(npairs);
  W.plo2 = c.take<uint32_t>(npairs);
  // C and the de-duplication table: member-indexed, then set-indexed
  W.cmem = c.take<uint32_t>(Cc);
  W.rstart = c.take<uint32_t>(Cc + 1);
  W.kept = c.take<uint32_t>(Cc + 1);
  W.kidx = c.take<uint32_t>(Cc + 1);
  W.klo = c.take<uint32_t>(Cc);
  W.khi = c.take<uint32_t>(Cc);
  W.coff = c.take<uint32_t>(Cs + 1);
  for (int w = 0; w < 4; ++w) W.tw[w] = c.take<uint32_t>(Cs);
  W.tv = c.take<uint32_t>(Cs);
  for (int w = 0; w < 4; ++w) W.tw2[w] = c.take<uint32_t>(Cs);
  W.tv2 = c.take<uint32_t>(Cs);
  W.h = c.take<uint32_t>(Cs + 1);
  W.hs = c.take<uint32_t>(Cs + 1);
  W.binofr = c.take<uint32_t>(Cs + 1);
  W.bstart = c.take<uint32_t>(Cs + 2);
  W.inv = c.take<uint32_t>(Cs + 1);
  W.cnt = c.take<uint32_t>(Cs + 1);
  W.poff = c.take<uint32_t>(Cs + 1);
  W.kend = c.take<uint32_t>(Cs);
  W.kstart = c.take<uint32_t>(Cs);
  W.ssz = c.take<uint32_t>(Cs + 1);
  W.sone = c.take<uint32_t>(Cs + 1);
  W.soff = c.take<uint32_t>(Cs + 1);
  W.sidx = c.take<uint32_t>(Cs + 1);
  W.big_list = c.take<uint32_t>(NS + 1);
  const int64_t nsort = npairs > NS ? npairs : NS;
  W.radix_tmp = c.take<uint32_t>(radix_tmp_words(nsort));
  W.scan_tmp = c.take<uint32_t>(exscan_tmp_words((W.NM > NS ? W.NM : NS) + 1) + 16);
  return c.used + 256;
}

int32_t silk_check(const geek_silk_job& J) {
  if (J.n < 1 || J.n >= (1ll << 31) || J.T < 1 || J.K < 1 || J.K > 4 || J.L < 0 || !J.members || !J.offsets ||
      !J.nbuckets || !J.silk_keys || !J.seed_offsets || !J.seed_members || !J.k_out || !J.needed ||
      J.cap_k < 0 || J.cap_members < 0)
    return GEEK_ERR_ARG;
  if (J.T > SILK_MAX_T) return GEEK_ERR_UNSUPPORTED;
  if ((int64_t)J.T * J.n >= (1ll << 31) || J.cap_c < 0 || c_members(J) >= (1ll << 31) ||
      J.cap_k >= (1ll << 32) - 1)
    return GEEK_ERR_UNSUPPORTED;
  return GEEK_OK;
}

size_t silk_ws(const geek_silk_job& J) {
  SilkWs W;
  return carve_silk(J, nullptr, W);
}

static inline int ggrid(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return b < 1 ? 1 : b > SG_GRID ? SG_GRID : (int)b;
}

static int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 32 && (maxval >> b) != 0) ++b;
  return b;
}

int32_t silk_run(const geek_silk_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s) {
  if (int32_t rc = silk_check(J)) return rc;
  SilkWs W;
  if (!ws || ws_bytes < carve_silk(J, ws, W)) return GEEK_ERR_WORKSPACE;
  prof_begin(GEEK_PROF_SILK, s);
  const int K = J.K, T = J.T;
  const int64_t n = J.n, Tn = W.Tn, Cc = W.Ccap;
  SilkState* S = W.S;
  // ---- setup: global buckets and the bucket of every (table, object)
  hipLaunchKernelGGL(k_silk_setup, dim3(1), dim3(1), 0, s, J.nbuckets, T, n, W.base, S);
  hipLaunchKernelGGL(k_extent, dim3(ggrid(Tn)), dim3(256), 0, s, J.offsets, W.base, T, n, S, W.gstart, W.gsize);
  hipLaunchKernelGGL(k_sk_fill, dim3(ggrid(Tn)), dim3(256), 0, s, W.flag, Tn, 0u);
  hipLaunchKernelGGL(k_mark_starts, dim3(ggrid(Tn)), dim3(256), 0, s, W.gstart, &S->nb, W.flag);
  exscan_u32(W.flag, W.fscan, Tn, W.scan_tmp, nullptr, s);
  hipLaunchKernelGGL(k_bucket_of, dim3(ggrid(Tn)), dim3(256), 0, s, J.members, Tn, n, W.flag, W.fscan, W.bof);
  // vote blocks: T LDS entries per thread
  int VT = 256;
  while (VT > 64 && VT * T > SV_LDS) VT >>= 1;
  const size_t vlds = sizeof(uint32_t) * 2 * (size_t)T * VT;
  const int vgrid = (int)std::min<int64_t>((n + VT - 1) / VT, 4096);
  // kept pairs sorted by the emitted bin index (< number of buckets)
  int kw[4], ksh[4], knp = 0;
  for (int sh = 0; sh < bits_for((uint64_t)(Tn - 1)); sh += 8) {
    kw[knp] = 0;
    ksh[knp++] = sh;
  }
  for (int t = 0; t < J.L; ++t) {
    const uint32_t* keys = J.silk_keys + 2 * (int64_t)t * K;
    hipLaunchKernelGGL(k_sk_fill, dim3(1), dim3(64), 0, s, &S->big, (int64_t)1, 0u);
    hipLaunchKernelGGL(k_sig, dim3(ggrid(Tn)), dim3(256), 0, s, J.members, W.gstart, W.gsize, &S->nb, keys, K, W.G,
                       W.big_list, &S->big, &S->hash_evals);
    hipLaunchKernelGGL(k_sig_big, dim3(SG_GRID), dim3(256), 0, s, J.members, W.gstart, W.gsize, keys, K, W.G,
                       W.big_list, &S->big, &S->hash_evals);
    // bins of identical G
    hipLaunchKernelGGL(k_ht_clear, dim3(SG_GRID), dim3(256), 0, s, S, W.ht, W.binmin, W.bcount, W.ksize);
    hipLaunchKernelGGL(k_ht_insert, dim3(ggrid(Tn)), dim3(256), 0, s, W.G, K, S, W.ht, W.rep);
    hipLaunchKernelGGL(k_ht_min, dim3(ggrid(Tn)), dim3(256), 0, s, W.rep, S, W.binmin, W.bcount);
    hipLaunchKernelGGL(k_bin_info, dim3(ggrid(Tn)), dim3(256), 0, s, W.rep, W.binmin, W.bcount, S, W.info);
    // majority votes and the bins that join C
    if (T <= 16)
      hipLaunchKernelGGL(k_vote_reg<16>, dim3(ggrid(n)), dim3(256), 0, s, W.bof, W.info, n, T, W.kbin, W.kc,
                         W.ksize, S);
    else if (T <= 32)
      hipLaunchKernelGGL(k_vote_reg<32>, dim3(ggrid(n)), dim3(256), 0, s, W.bof, W.info, n, T, W.kbin, W.kc,
                         W.ksize, S);
    else
      hipLaunchKernelGGL(k_vote, dim3(vgrid), dim3(VT), vlds, s, W.bof, W.info, n, T, W.kbin, W.kc, W.ksize, S);
    hipLaunchKernelGGL(k_emit_flags, dim3(ggrid(Tn)), dim3(256), 0, s, W.info, W.ksize, J.delta, S, W.eone, W.esz);
    exscan_u32_dn(W.eone, W.eidx, Tn, &S->nb, W.scan_tmp, &S->es, s);
    exscan_u32_dn(W.esz, W.eoff, Tn, &S->nb, W.scan_tmp, &S->em, s);
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(1), 0, s, S, (uint32_t)W.Cs, (uint32_t)Cc);
    // this table's sets of C, ids ascending
    hipLaunchKernelGGL(k_count_kept, dim3(ggrid(n)), dim3(256), 0, s, W.kbin, W.kc, n, W.eone, S, W.kc2);
    exscan_u32(W.kc2, W.kpos, n, W.scan_tmp, &S->kp, s);
    hipLaunchKernelGGL(k_kept_pairs, dim3(ggrid(n)), dim3(256), 0, s, W.kbin, W.kc, n, W.eone, W.eidx, W.kpos, S,
                       W.phi, W.plo);
    RsView A{{W.phi, nullptr, nullptr, nullptr}, W.plo}, B{{W.phi2, nullptr, nullptr, nullptr}, W.plo2};
    const int alt = radix_sort_dn(A, B, 1, W.KPmax, &S->kp, kw, ksh, knp, W.radix_tmp, s);
    hipLaunchKernelGGL(k_c_write, dim3(ggrid(Tn)), dim3(256), 0, s, alt ? W.plo2 : W.plo, W.eone, W.eidx, W.eoff, S,
                       W.cmem, W.coff);
  }
  // ---- de-duplication: one more table over the sets of C (Cs bounds its
  // sets and bins, Cc its members and voting pairs)
  const int64_t Cs = W.Cs;
  const uint32_t* dkeys = J.silk_keys + 2 * (int64_t)J.L * K;
  hipLaunchKernelGGL(k_dd_setup, dim3(1), dim3(1), 0, s, S, W.coff);
  hipLaunchKernelGGL(k_set_extent, dim3(ggrid(Cs)), dim3(256), 0, s, W.coff, S, W.gstart, W.gsize);
  hipLaunchKernelGGL(k_sk_fill, dim3(1), dim3(64), 0, s, &S->big, (int64_t)1, 0u);
  hipLaunchKernelGGL(k_sig, dim3(ggrid(Cs)), dim3(256), 0, s, W.cmem, W.gstart, W.gsize, &S->cs, dkeys, K, W.G,
                     W.big_list, &S->big, (unsigned long long*)nullptr);
  hipLaunchKernelGGL(k_sig_big, dim3(SG_GRID), dim3(256), 0, s, W.cmem, W.gstart, W.gsize, dkeys, K, W.G, W.big_list,
                     &S->big, (unsigned long long*)nullptr);
  hipLaunchKernelGGL(k_dd_tuples, dim3(ggrid(Cs)), dim3(256), 0, s, W.G, K, S, W.tw[0], W.tw[1], W.tw[2], W.tw[3],
                     W.tv);
  int tw[16], tsh[16], tnp = 0;
  for (int k = K - 1; k >= 0; --k)
    for (int sh = 0; sh < 32; sh += 8) {
      tw[tnp] = k;
      tsh[tnp++] = sh;
    }
  RsView TA{{W.tw[0], W.tw[1], W.tw[2], W.tw[3]}, W.tv}, TB{{W.tw2[0], W.tw2[1], W.tw2[2], W.tw2[3]}, W.tv2};
  const int talt = radix_sort_dn(TA, TB, 4, Cs, &S->cs, tw, tsh, tnp, W.radix_tmp, s);
  const RsView& TS = talt ? TB : TA;
  const uint32_t* ord = TS.v;
  hipLaunchKernelGGL(k_dd_heads, dim3(ggrid(Cs)), dim3(256), 0, s, TS.k[0], TS.k[1], TS.k[2], TS.k[3], S, W.h);
  exscan_u32_dn(W.h, W.hs, Cs, &S->cs, W.scan_tmp, &S->nb2, s);
  hipLaunchKernelGGL(k_dd_bins, dim3(ggrid(Cs)), dim3(256), 0, s, W.h, W.hs, ord, S, W.binofr, W.bstart, W.inv);
  hipLaunchKernelGGL(k_dd_cnt, dim3(ggrid(Cs)), dim3(256), 0, s, ord, W.binofr, W.bstart, W.gsize, S, W.cnt);
  exscan_u32_dn(W.cnt, W.poff, Cs, &S->cs, W.scan_tmp, &S->P2, s);
  hipLaunchKernelGGL(k_sk_fill, dim3(ggrid(Cc)), dim3(256), 0, s, W.flag, Cc + 1, 0u);
  hipLaunchKernelGGL(k_mark_starts, dim3(ggrid(Cs)), dim3(256), 0, s, W.gstart, &S->cs, W.flag);
  exscan_u32_dn(W.flag, W.fscan, Cc, &S->cm, W.scan_tmp, nullptr, s);
  hipLaunchKernelGGL(k_dd_pairs, dim3(ggrid(Cc)), dim3(256), 0, s, W.cmem, W.flag, W.fscan, W.coff, W.inv, W.cnt,
                     W.poff, W.binofr, S, W.phi, W.plo);
  int pw[12], psh[12], pnp = 0;
  for (int sh = 0; sh < bits_for((uint64_t)(n - 1)); sh += 8) {
    pw[pnp] = 0;
    psh[pnp++] = sh;
  }
  for (int sh = 0; sh < bits_for((uint64_t)(Cs - 1)); sh += 8) {
    pw[pnp] = 1;
    psh[pnp++] = sh;
  }
  RsView PA{{W.plo, W.phi, nullptr, nullptr}, nullptr}, PB{{W.plo2, W.phi2, nullptr, nullptr}, nullptr};
  const int palt = radix_sort_dn(PA, PB, 2, Cc, &S->P2, pw, psh, pnp, W.radix_tmp, s);
  const uint32_t* phi = palt ? W.phi2 : W.phi;
  const uint32_t* plo = palt ? W.plo2 : W.plo;
  hipLaunchKernelGGL(k_run_heads, dim3(ggrid(Cc)), dim3(256), 0, s, phi, plo, &S->P2, W.kept);
  exscan_u32_dn(W.kept, W.kidx, Cc, &S->P2, W.scan_tmp, &S->R2, s);
  hipLaunchKernelGGL(k_starts, dim3(ggrid(Cc + 1)), dim3(256), 0, s, W.kept, W.kidx, &S->P2, &S->R2, W.rstart);
  hipLaunchKernelGGL(k_dd_keep, dim3(ggrid(Cc)), dim3(256), 0, s, W.rstart, phi, W.bstart, S, W.kept);
  exscan_u32_dn(W.kept, W.kidx, Cc, &S->R2, W.scan_tmp, &S->kept2, s);
  hipLaunchKernelGGL(k_dd_compact, dim3(ggrid(Cc)), dim3(256), 0, s, W.rstart, W.kept, W.kidx, phi, plo, S, W.klo,
                     W.khi);
  hipLaunchKernelGGL(k_sk_fill, dim3(ggrid(Cs)), dim3(256), 0, s, W.kstart, Cs, 0u);
  hipLaunchKernelGGL(k_sk_fill, dim3(ggrid(Cs)), dim3(256), 0, s, W.kend, Cs, 0u);
  hipLaunchKernelGGL(k_dd_kruns, dim3(ggrid(Cc)), dim3(256), 0, s, W.khi, S, W.kstart, W.kend);
  hipLaunchKernelGGL(k_dd_size, dim3(ggrid(Cs)), dim3(256), 0, s, W.bstart, ord, W.gsize, W.kstart, W.kend, J.delta,
                     S, W.ssz, W.sone);
  exscan_u32_dn(W.ssz, W.soff, Cs, &S->nb2, W.scan_tmp, &S->tot_m, s);
  exscan_u32_dn(W.sone, W.sidx, Cs, &S->nb2, W.scan_tmp, &S->k, s);
  hipLaunchKernelGGL(k_silk_finish, dim3(1), dim3(1), 0, s, S, (uint64_t)J.cap_k, (uint64_t)J.cap_members,
                     J.seed_offsets, J.k_out, J.needed, J.counters, st);
  hipLaunchKernelGGL(k_emit_seeds, dim3(ggrid(Cs)), dim3(256), 0, s, W.ssz, W.soff, W.sidx, S, J.seed_offsets);
  hipLaunchKernelGGL(k_seed_copy, dim3(ggrid(Cc)), dim3(256), 0, s, W.soff, W.bstart, ord, W.cmem, W.coff, W.klo,
                     W.kstart, S, J.seed_members);
  prof_end(GEEK_PROF_SILK, s);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
