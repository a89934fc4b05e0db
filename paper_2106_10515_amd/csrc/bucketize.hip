// Buckets of every table (paper Algorithms 2 and 3: T[G(x_j)].push(j)) on
// gfx950: group the objects whose table keys are identical.
//
//  1. A partition of (key, id) records into 2^nb bins per table, the bin
//     being the top bits of a 32-bit mix of the exact key (equal keys always
//     share a bin).  Up to 2^PT_B1 bins it is one pass (k_bin_count, the
//     scans, k_p1_scatter); beyond, a second pass splits every first-pass bin
//     by the next bits (k_p2_*).  Each scatter sorts rounds of PT_ROUND
//     records by bin in LDS before writing, so the stores are runs of
//     consecutive records instead of single scattered records.
//  2. k_bin_group: one workgroup per bin groups its records with an LDS hash
//     table on the exact key; objects sharing a key get (head = smallest id,
//     rank among the bucket's ids, bucket size at the head) in id-indexed
//     arrays plus a flag bit.  Bins too large for LDS are sorted by
//     k_big_sort (workgroup LSD radix sort in global memory) and their runs
//     recorded by k_big_runs.
//  3. k_bz_reduce / k_scan_chunks / k_bz_apply: a scan over ids in id order
//     gives every bucket its rank in smallest-member order and its CSR
//     offset; every head (including objects alone in their bucket) is
//     written to its slot at once.
//  4. k_bz_members: the remaining members of buckets of two or more go to
//     head offset + rank.
#include "common.hpp"

namespace geek {

constexpr int BZ_THREADS = 256;
constexpr int BZ_CAP = 2048;      // largest bin grouped in LDS
constexpr int BZ_HT = 4096;       // LDS hash slots per bin
constexpr int BZ_SMALL = 32;      // largest group ranked by walking its member list
constexpr int BZ_MAXBITS = 14;    // at most 16384 bins per table
constexpr int SC_CHUNK = 4096;    // elements per block in the scans
constexpr int BIG_THREADS = 1024;

struct BzArgs {
  const uint32_t* keys;
  int64_t n;
  int T;
  int kw;
  int64_t tstride, rstride;
  int nb;  // bin bits
};

GEEK_D uint4 load_key(const BzArgs& a, int t, int64_t i) {
  const uint32_t* k = a.keys + (int64_t)t * a.tstride + i * a.rstride;
  uint4 r;
  r.x = k[0];
  r.y = a.kw > 1 ? k[1] : 0u;
  r.z = a.kw > 2 ? k[2] : 0u;
  r.w = a.kw > 3 ? k[3] : 0u;
  return r;
}
GEEK_D uint32_t bin_of(const uint4& k, int nb) {
  const uint32_t w[4] = {k.x, k.y, k.z, k.w};
  return nb ? key_hash(w, 4) >> (32 - nb) : 0u;
}
GEEK_D bool key_eq(const uint4& a, const uint4& b) {
  return a.x == b.x && a.y == b.y && a.z == b.z && a.w == b.w;
}
GEEK_D bool rec_less(const uint4& a, uint32_t ia, const uint4& b, uint32_t ib) {
  if (a.x != b.x) return a.x < b.x;
  if (a.y != b.y) return a.y < b.y;
  if (a.z != b.z) return a.z < b.z;
  if (a.w != b.w) return a.w < b.w;
  return ia < ib;
}

// ---------------------------------------------------------------- partition
__global__ __launch_bounds__(BZ_THREADS) void k_bin_count(BzArgs a, int nblk, int chunk, uint32_t* counts) {
  extern __shared__ uint32_t hist[];
  const int t = blockIdx.y, blk = blockIdx.x;
  const int nbins = 1 << a.nb;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS) hist[b] = 0;
  __syncthreads();
  const int64_t s = (int64_t)blk * chunk;
  const int64_t e = s + chunk < a.n ? s + chunk : a.n;
  for (int64_t i = s + threadIdx.x; i < e; i += BZ_THREADS)
    atomicAdd(&hist[bin_of(load_key(a, t, i), a.nb)], 1u);
  __syncthreads();
  uint32_t* out = counts + ((int64_t)t * nblk + blk) * nbins;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS) out[b] = hist[b];
}

// Per (table, bin): exclusive scan over blocks; bin totals.
__global__ void k_bin_colscan(int T, int nblk, int nbins, uint32_t* counts, uint32_t* bintot) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)T * nbins) return;
  const int t = (int)(g / nbins), b = (int)(g % nbins);
  uint32_t run = 0;
  uint32_t* c = counts + (int64_t)t * nblk * nbins + b;
  int k = 0;
  for (; k + 8 <= nblk; k += 8) {  // eight loads in flight
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = c[(int64_t)(k + u) * nbins];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[(int64_t)(k + u) * nbins] = run;
      run += v[u];
    }
  }
  for (; k < nblk; ++k) {
    const uint32_t v = c[(int64_t)k * nbins];
    c[(int64_t)k * nbins] = run;
    run += v;
  }
  bintot[g] = run;
}

// Block-wide exclusive scan of one value per thread (blockDim.x <= 1024).
__device__ uint32_t block_exscan(uint32_t v, uint32_t* total, uint32_t* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t r = 0;
    for (int k = 0; k < nw; ++k) {
      const uint32_t c = sh[k];
      sh[k] = r;
      r += c;
    }
    sh[16] = r;
  }
  __syncthreads();
  const uint32_t res = x - v + sh[wv];
  if (total) *total = sh[16];
  __syncthreads();
  return res;
}

// Per table: exclusive scan of bin totals -> bin starts (one block per table).
__global__ __launch_bounds__(1024) void k_bin_rowscan(int nbins, const uint32_t* bintot, uint32_t* binstart) {
  __shared__ uint32_t sh[17];
  const int t = blockIdx.x;
  const uint32_t* in = bintot + (int64_t)t * nbins;
  uint32_t* out = binstart + (int64_t)t * nbins;
  const int per = (nbins + 1023) / 1024;
  uint32_t loc = 0;
  for (int q = 0; q < per; ++q) {
    const int b = threadIdx.x * per + q;
    loc += b < nbins ? in[b] : 0u;
  }
  uint32_t base = block_exscan(loc, nullptr, sh);
  for (int q = 0; q < per; ++q) {
    const int b = threadIdx.x * per + q;
    if (b < nbins) {
      out[b] = base;
      base += in[b];
    }
  }
}

constexpr int PT_B1 = 6;          // bits of the first partition pass (64 bins)
constexpr int PT_ROUND = 2048;    // records sorted by bin in LDS per round
constexpr int PT_SUPER = 16384;   // records per workgroup of a partition pass
constexpr int PT_RPT = PT_ROUND / BZ_THREADS;

// One round of a partition scatter: the block's `cnt` records (key, id,
// bin) are counted per bin, placed in LDS in bin order, and written out so
// that consecutive threads store consecutive records of a bin.  cur[b] is
// the global position of bin b's next record and advances by the round's
// count.  Records of a bin keep no particular order (the grouping that
// follows does not depend on it).
struct PartLds {
  uint4 key[PT_ROUND];
  uint32_t id[PT_ROUND];
  uint16_t bin[PT_ROUND];
  uint32_t hist[256], lst[256], cur[256], sh[17];
};

template <class Load>
__device__ void part_round(PartLds& L, int nbins, int cnt, const Load& load, uint4* out_keys,
                           uint32_t* out_ids) {
  const int tid = threadIdx.x;
  for (int b = tid; b < nbins; b += BZ_THREADS) L.hist[b] = 0u;
  __syncthreads();
  uint4 k[PT_RPT];
  uint32_t id[PT_RPT], rk[PT_RPT];
  int bn[PT_RPT];
#pragma unroll
  for (int u = 0; u < PT_RPT; ++u) {
    const int q = tid + u * BZ_THREADS;
    if (q < cnt) {
      load(q, k[u], id[u], bn[u]);
      rk[u] = atomicAdd(&L.hist[bn[u]], 1u);
    }
  }
  __syncthreads();
  // exclusive scan of the round's bin counts (nbins <= 256 = one per thread)
  const uint32_t hv = tid < nbins ? L.hist[tid] : 0u;
  const uint32_t ex = block_exscan(hv, nullptr, L.sh);
  if (tid < nbins) L.lst[tid] = ex;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PT_RPT; ++u) {
    const int q = tid + u * BZ_THREADS;
    if (q < cnt) {
      const uint32_t p = L.lst[bn[u]] + rk[u];
      L.key[p] = k[u];
      L.id[p] = id[u];
      L.bin[p] = (uint16_t)bn[u];
    }
  }
  __syncthreads();
  for (int p = tid; p < cnt; p += BZ_THREADS) {
    const int b = L.bin[p];
    const uint32_t gp = L.cur[b] + (uint32_t)p - L.lst[b];
    out_keys[gp] = L.key[p];
    out_ids[gp] = L.id[p];
  }
  __syncthreads();
  for (int b = tid; b < nbins; b += BZ_THREADS) L.cur[b] += L.hist[b];
}

// First pass: block (chunk of PT_SUPER ids, table) -> 2^a.nb bins (a.nb <= PT_B1).
__global__ __launch_bounds__(BZ_THREADS) void k_p1_scatter(BzArgs a, int nblk, const uint32_t* counts,
                                                           const uint32_t* binstart, uint4* out_keys,
                                                           uint32_t* out_ids) {
  __shared__ PartLds L;
  const int t = blockIdx.y, blk = blockIdx.x;
  const int nbins = 1 << a.nb;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS)
    L.cur[b] = binstart[(int64_t)t * nbins + b] + counts[((int64_t)t * nblk + blk) * nbins + b];
  const int64_t s = (int64_t)blk * PT_SUPER;
  const int64_t e = s + PT_SUPER < a.n ? s + PT_SUPER : a.n;
  for (int64_t r0 = s; r0 < e; r0 += PT_ROUND) {
    const int cnt = (int)(e - r0 < PT_ROUND ? e - r0 : PT_ROUND);
    part_round(L, nbins, cnt,
               [&](int q, uint4& k, uint32_t& id, int& bn) {
                 k = load_key(a, t, r0 + q);
                 id = (uint32_t)(r0 + q);
                 bn = (int)bin_of(k, a.nb);
               },
               out_keys + (int64_t)t * a.n, out_ids + (int64_t)t * a.n);
  }
}

// Second pass.  The records of first-pass bin (t, B) are cut into chunks of
// PT_SUPER; cbase[t * 2^PT_B1 + B] is the first global chunk of that bin.
__global__ __launch_bounds__(1024) void k_p2_chunks(int nb1bins, const uint32_t* bintot1, uint32_t* cbase) {
  __shared__ uint32_t sh[17];
  const int per = (nb1bins + 1023) / 1024;
  uint32_t loc = 0;
  for (int q = 0; q < per; ++q) {
    const int i = threadIdx.x * per + q;
    loc += i < nb1bins ? (bintot1[i] + PT_SUPER - 1) / PT_SUPER : 0u;
  }
  uint32_t total;
  uint32_t base = block_exscan(loc, &total, sh);
  for (int q = 0; q < per; ++q) {
    const int i = threadIdx.x * per + q;
    if (i < nb1bins) {
      cbase[i] = base;
      base += (bintot1[i] + PT_SUPER - 1) / PT_SUPER;
    }
  }
  if (threadIdx.x == 0) cbase[nb1bins] = total;
}

// The first-pass bin of global chunk g (the last i with cbase[i] <= g).
GEEK_D int p2_bin_of_chunk(const uint32_t* cbase, int nb1bins, uint32_t g) {
  int lo = 0, hi = nb1bins - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cbase[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Per chunk: counts of the second-pass bins (the next nb - PT_B1 bits).
__global__ __launch_bounds__(BZ_THREADS) void k_p2_count(int64_t n, int nb, const uint32_t* cbase, int nb1bins,
                                                         const uint32_t* bintot1, const uint32_t* binstart1,
                                                         const uint4* keys1, uint32_t* counts2) {
  __shared__ uint32_t hist[256];
  const uint32_t g = blockIdx.x;
  if (g >= cbase[nb1bins]) return;
  const int F = 1 << (nb - PT_B1);
  const int tb = p2_bin_of_chunk(cbase, nb1bins, g);
  const int t = tb >> PT_B1;
  const uint32_t off = (g - cbase[tb]) * (uint32_t)PT_SUPER;
  const uint32_t cnt = min((uint32_t)PT_SUPER, bintot1[tb] - off);
  const uint4* src = keys1 + (int64_t)t * n + binstart1[tb] + off;
  for (int b = threadIdx.x; b < F; b += BZ_THREADS) hist[b] = 0u;
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < cnt; q += BZ_THREADS) {
    const uint4 k = src[q];
    atomicAdd(&hist[bin_of(k, nb) & (uint32_t)(F - 1)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < F; b += BZ_THREADS) counts2[(int64_t)g * F + b] = hist[b];
}

// Per (first-pass bin, second-pass bin): exclusive scan over the bin's
// chunks; totals in bintot [t][B * F + f] (the final 2^nb bins per table).
__global__ void k_p2_colscan(int nb1bins, int F, const uint32_t* cbase, uint32_t* counts2, uint32_t* bintot) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)nb1bins * F) return;
  const int tb = (int)(i / F), f = (int)(i % F);
  uint32_t run = 0;
  for (uint32_t g = cbase[tb]; g < cbase[tb + 1]; ++g) {
    const uint32_t v = counts2[(int64_t)g * F + f];
    counts2[(int64_t)g * F + f] = run;
    run += v;
  }
  bintot[(int64_t)tb * F + f] = run;
}

__global__ __launch_bounds__(BZ_THREADS) void k_p2_scatter(int64_t n, int nb, const uint32_t* cbase, int nb1bins,
                                                           const uint32_t* bintot1, const uint32_t* binstart1,
                                                           const uint4* keys1, const uint32_t* ids1,
                                                           const uint32_t* counts2, const uint32_t* binstart,
                                                           uint4* out_keys, uint32_t* out_ids) {
  __shared__ PartLds L;
  const uint32_t g = blockIdx.x;
  if (g >= cbase[nb1bins]) return;
  const int F = 1 << (nb - PT_B1);
  const int tb = p2_bin_of_chunk(cbase, nb1bins, g);
  const int t = tb >> PT_B1;
  const uint32_t off = (g - cbase[tb]) * (uint32_t)PT_SUPER;
  const uint32_t cnt_all = min((uint32_t)PT_SUPER, bintot1[tb] - off);
  const int64_t s = (int64_t)t * n + binstart1[tb] + off;
  for (int b = threadIdx.x; b < F; b += BZ_THREADS)
    L.cur[b] = binstart[(int64_t)tb * F + b] + counts2[(int64_t)g * F + b];
  for (uint32_t r0 = 0; r0 < cnt_all; r0 += PT_ROUND) {
    const int cnt = (int)min((uint32_t)PT_ROUND, cnt_all - r0);
    part_round(L, F, cnt,
               [&](int q, uint4& k, uint32_t& id, int& bn) {
                 k = keys1[s + r0 + q];
                 id = ids1[s + r0 + q];
                 bn = (int)(bin_of(k, nb) & (uint32_t)(F - 1));
               },
               out_keys + (int64_t)t * n, out_ids + (int64_t)t * n);
  }
}

// ---------------------------------------------------------------- per-bin grouping
// Id-indexed results of the grouping, per table (only objects that share
// their key with another object are recorded; every other object is a
// bucket of its own):
//   flags  bit i set iff object i is in a bucket of two or more
//   info   for flagged i: x = head (smallest id of the bucket),
//          y = bucket size if i is the head, else the rank of i in its bucket
//          (number of smaller ids)
struct GroupOut {
  uint32_t* flags;  // [T][flag_words]
  uint2* info;      // [T][n]
  int64_t flag_words;
};

GEEK_D void group_record(const GroupOut& go, int t, int64_t n, uint32_t id, uint32_t head, uint32_t y) {
  go.info[(int64_t)t * n + id] = make_uint2(head, y);
  atomicOr(&go.flags[(int64_t)t * go.flag_words + (id >> 5)], 1u << (id & 31));
}

// One workgroup per (bin, table).  Each thread keeps its records (key, id,
// slot) in registers; an LDS hash table keyed by the exact key gives each
// record its group (slot) and the group sizes; keys of slot owners are
// re-read from the bin's staging copy (cache-resident) for comparisons.
// Ranks inside groups of at most BZ_SMALL come from a walk of the group's
// member list; bins with a larger group sort (slot, id) pairs in LDS
// (bitonic) and rank by position.  A slot word holds the group size in its
// high 16 bits and, in its low 16 bits, first the owning record + 1
// (0: empty), then the member-list head + 1, then the first sorted position
// + 1.  LDS stays small enough for four workgroups per CU.
constexpr int BZ_RPT = BZ_CAP / BZ_THREADS;  // records per thread
__global__ __launch_bounds__(BZ_THREADS) void k_bin_group(int64_t n, int nb, const uint32_t* bintot,
                                                          const uint32_t* binstart, const uint4* st_keys,
                                                          const uint32_t* st_ids, GroupOut go,
                                                          uint32_t* big_list, uint32_t* big_count) {
  __shared__ uint32_t hw[BZ_HT];
  __shared__ int16_t nxt[BZ_CAP];
  __shared__ unsigned long long sc[BZ_CAP];  // (slot, id) sort array
  __shared__ uint32_t smax;
  const int t = blockIdx.y, bin = blockIdx.x;
  const int nbins = 1 << nb;
  const uint32_t size = bintot[(int64_t)t * nbins + bin];
  if (size <= 1) return;  // empty, or one record: a bucket of its own
  if (size > BZ_CAP) {
    if (threadIdx.x == 0) big_list[atomicAdd(big_count, 1u)] = (uint32_t)(t * nbins + bin);
    return;
  }
  const uint32_t s0 = binstart[(int64_t)t * nbins + bin];
  const uint4* gk = st_keys + (int64_t)t * n + s0;
  const uint32_t* gi = st_ids + (int64_t)t * n + s0;
  uint4 kr[BZ_RPT];
  uint32_t idr[BZ_RPT];
  int slot[BZ_RPT];
#pragma unroll
  for (int u = 0; u < BZ_RPT; ++u) {
    const int q = threadIdx.x + u * BZ_THREADS;
    if (q < (int)size) {
      kr[u] = gk[q];
      idr[u] = gi[q];
    }
  }
  for (int q = threadIdx.x; q < BZ_HT; q += BZ_THREADS) hw[q] = 0u;
  if (threadIdx.x == 0) smax = 0;
  __syncthreads();
  // insert with linear probing; an owned slot's key is already in memory
#pragma unroll
  for (int u = 0; u < BZ_RPT; ++u) {
    const int q = threadIdx.x + u * BZ_THREADS;
    slot[u] = 0;
    if (q >= (int)size) continue;
    const uint4 k = kr[u];
    const uint32_t w[4] = {k.x, k.y, k.z, k.w};
    int h = (int)(key_hash(w, 4) & (BZ_HT - 1));
    for (;;) {
      uint32_t cur = hw[h] & 0xFFFFu;
      if (cur == 0u) {
        const uint32_t prev = atomicCAS(&hw[h], 0u, (uint32_t)(q + 1));
        if (prev == 0u) break;
        cur = prev & 0xFFFFu;
      }
      if (key_eq(gk[cur - 1], k)) break;
      h = (h + 1) & (BZ_HT - 1);
    }
    slot[u] = h;
    atomicAdd(&hw[h], 0x10000u);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < BZ_HT; q += BZ_THREADS) hw[q] &= 0xFFFF0000u;
  __syncthreads();
  // member lists (order arbitrary)
#pragma unroll
  for (int u = 0; u < BZ_RPT; ++u) {
    const int q = threadIdx.x + u * BZ_THREADS;
    if (q >= (int)size) continue;
    const int g = slot[u];
    uint32_t old = hw[g];
    for (;;) {
      const uint32_t prev = atomicCAS(&hw[g], old, (old & 0xFFFF0000u) | (uint32_t)(q + 1));
      if (prev == old) break;
      old = prev;
    }
    nxt[q] = (int16_t)((int)(old & 0xFFFFu) - 1);
    if ((old >> 16) > 1u) atomicMax(&smax, old >> 16);
  }
  __syncthreads();
  const uint32_t big = smax;
  if (big <= 1) return;  // all keys distinct
  if (big <= BZ_SMALL) {
#pragma unroll
    for (int u = 0; u < BZ_RPT; ++u) {
      const int q = threadIdx.x + u * BZ_THREADS;
      if (q >= (int)size) continue;
      const uint32_t v = hw[slot[u]];
      const uint32_t c = v >> 16;
      if (c == 1) continue;
      const uint32_t me = idr[u];
      uint32_t r = 0, head = me;
      for (int e = (int)(v & 0xFFFFu) - 1; e >= 0; e = nxt[e]) {
        const uint32_t o = gi[e];
        r += o < me;
        head = min(head, o);
      }
      group_record(go, t, n, me, head, r == 0 ? c : r);
    }
    return;
  }
  // a larger group: sort (slot, id) pairs, rank by position
  int P2 = 1;
  while (P2 < (int)size) P2 <<= 1;
#pragma unroll
  for (int u = 0; u < BZ_RPT; ++u) {
    const int q = threadIdx.x + u * BZ_THREADS;
    if (q < P2) sc[q] = q < (int)size ? ((unsigned long long)slot[u] << 32) | idr[u] : ~0ull;
  }
  for (int q = threadIdx.x; q < BZ_HT; q += BZ_THREADS) hw[q] |= 0xFFFFu;
  __syncthreads();
  for (int kk = 2; kk <= P2; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int q = threadIdx.x; q < P2; q += BZ_THREADS) {
        const int o = q ^ jj;
        if (o > q) {
          const unsigned long long a = sc[q], b = sc[o];
          const bool up = (q & kk) == 0;
          if (up ? (b < a) : (a < b)) {
            sc[q] = b;
            sc[o] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < (int)size; q += BZ_THREADS) {
    const int g = (int)(sc[q] >> 32);
    atomicMin(&hw[g], (hw[g] & 0xFFFF0000u) | (uint32_t)(q + 1));
  }
  __syncthreads();
  for (int q = threadIdx.x; q < (int)size; q += BZ_THREADS) {
    const uint32_t v = hw[(int)(sc[q] >> 32)];
    const uint32_t c = v >> 16;
    if (c == 1) continue;
    const int f = (int)(v & 0xFFFFu) - 1;
    const uint32_t me = (uint32_t)sc[q], head = (uint32_t)sc[f];
    group_record(go, t, n, me, head, q == f ? c : (uint32_t)(q - f));
  }
}

// Oversize bins: LSD radix sort (8-bit digits, stable) of the bin's records
// by (key, id) in global memory, one workgroup per bin; passes whose digit is
// constant over the bin are skipped.
__global__ __launch_bounds__(BIG_THREADS) void k_big_sort(int64_t n, int nb, int kw, const uint32_t* bintot,
                                                          const uint32_t* binstart, uint4* st_keys,
                                                          uint32_t* st_ids, uint4* alt_keys,
                                                          uint32_t* alt_ids, const uint32_t* big_list,
                                                          const uint32_t* big_count) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[16][256];
  __shared__ int skip;
  const int nbins = 1 << nb;
  const uint32_t nbig = *big_count;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const uint32_t tb = big_list[bi];
    const int t = (int)(tb / nbins);
    const uint32_t size = bintot[tb], s0 = binstart[tb];
    uint4* k0 = st_keys + (int64_t)t * n + s0;
    uint32_t* i0 = st_ids + (int64_t)t * n + s0;
    uint4* k1 = alt_keys + (int64_t)t * n + s0;
    uint32_t* i1 = alt_ids + (int64_t)t * n + s0;
    const int npass = 4 + 4 * kw;  // id bytes first (least significant), then key words
    for (int pass = 0; pass < npass; ++pass) {
      // digit extractor: passes 0..3 id bytes; then word (kw-1 .. 0) bytes
      auto digit = [&](const uint4& k, uint32_t id) -> uint32_t {
        if (pass < 4) return (id >> (8 * pass)) & 255u;
        const int wp = (pass - 4) >> 2, by = (pass - 4) & 3;
        const int word = kw - 1 - wp;
        const uint32_t w = word == 0 ? k.x : word == 1 ? k.y : word == 2 ? k.z : k.w;
        return (w >> (8 * by)) & 255u;
      };
      for (int q = threadIdx.x; q < 256; q += BIG_THREADS) hist[q] = 0;
      __syncthreads();
      for (uint32_t q = threadIdx.x; q < size; q += BIG_THREADS) atomicAdd(&hist[digit(k0[q], i0[q])], 1u);
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t r = 0;
        int sk = 0;
        for (int b = 0; b < 256; ++b) {
          base[b] = r;
          r += hist[b];
          sk |= (hist[b] == size);
        }
        skip = sk;
      }
      __syncthreads();
      if (skip) continue;
      // stable scatter, BIG_THREADS records per round in thread order
      for (uint32_t r0 = 0; r0 < size; r0 += BIG_THREADS) {
        const uint32_t q = r0 + threadIdx.x;
        const bool has = q < size;
        uint4 kk = make_uint4(0, 0, 0, 0);
        uint32_t id = 0, dg = 0;
        if (has) {
          kk = k0[q];
          id = i0[q];
          dg = digit(kk, id);
        }
        // lanes of this wave with the same digit
        uint64_t mask = __ballot(has);
        for (int b = 0; b < 8; ++b) {
          const uint64_t bb = __ballot(has && ((dg >> b) & 1u));
          mask &= ((dg >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        for (int b = threadIdx.x; b < 16 * 256; b += BIG_THREADS) (&wcnt[0][0])[b] = 0;
        __syncthreads();
        if (has && below == 0) wcnt[wv][dg] = (uint32_t)__popcll(mask);
        __syncthreads();
        if (has) {
          uint32_t before = 0;
          for (int w2 = 0; w2 < wv; ++w2) before += wcnt[w2][dg];
          const uint32_t pos = base[dg] + before + below;
          k1[pos] = kk;
          i1[pos] = id;
        }
        __syncthreads();
        if (threadIdx.x < 256) {
          uint32_t tot = 0;
          for (int w2 = 0; w2 < 16; ++w2) tot += wcnt[w2][threadIdx.x];
          base[threadIdx.x] += tot;
        }
        __syncthreads();
      }
      // copy back so the sorted data is always in (k0, i0)
      for (uint32_t q = threadIdx.x; q < size; q += BIG_THREADS) {
        k0[q] = k1[q];
        i0[q] = i1[q];
      }
      __syncthreads();
    }
  }
}

// Run detection of a sorted oversize bin (one workgroup per bin); records
// the runs of two or more in the grouping output.
__global__ __launch_bounds__(BIG_THREADS) void k_big_runs(int64_t n, int nb, const uint32_t* bintot,
                                                          const uint32_t* binstart, const uint4* st_keys,
                                                          const uint32_t* st_ids, GroupOut go,
                                                          const uint32_t* big_list, const uint32_t* big_count) {
  __shared__ int ss[BIG_THREADS];
  __shared__ int carry;
  const int nbins = 1 << nb;
  const uint32_t nbig = *big_count;
  for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const uint32_t tb = big_list[bi];
    const int t = (int)(tb / nbins);
    const uint32_t size = bintot[tb], s0 = binstart[tb];
    const uint4* k = st_keys + (int64_t)t * n + s0;
    const uint32_t* ids = st_ids + (int64_t)t * n + s0;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t r0 = 0; r0 < size; r0 += BIG_THREADS) {
      const uint32_t q = r0 + threadIdx.x;
      int v = -1;
      if (q < size) v = (q == 0 || !key_eq(k[q], k[q - 1])) ? (int)q : -1;
      ss[threadIdx.x] = v;
      __syncthreads();
      for (int o = 1; o < BIG_THREADS; o <<= 1) {
        const int y = threadIdx.x >= (unsigned)o ? ss[threadIdx.x - o] : -1;
        __syncthreads();
        ss[threadIdx.x] = max(ss[threadIdx.x], y);
        __syncthreads();
      }
      const int rs = max(ss[threadIdx.x], carry);
      if (q < size) {
        const uint32_t f = ids[rs];
        const bool last = (q == size - 1) || !key_eq(k[q + 1], k[q]);
        if ((int)q != rs) {
          group_record(go, t, n, ids[q], f, q - (uint32_t)rs);
          if (last) group_record(go, t, n, f, f, q - (uint32_t)rs + 1u);
        }
      }
      __syncthreads();
      if (threadIdx.x == BIG_THREADS - 1) carry = rs;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- scans and emission
// Each thread owns BZ_PER consecutive ids of a SC_CHUNK-id chunk; their flag
// bits sit in one flag word.
constexpr int BZ_PER = SC_CHUNK / BZ_THREADS;
static_assert(BZ_PER == 16, "16 ids per thread: one half flag word");

// Bucket head / bucket length of id i (0 length for non-head members).
GEEK_D void id_bucket(const GroupOut& go, int t, int64_t n, int64_t i, bool flagged, uint32_t& is_head,
                      uint32_t& len, uint2& inf) {
  if (!flagged) {
    is_head = 1;
    len = 1;
    return;
  }
  inf = go.info[(int64_t)t * n + i];
  is_head = inf.x == (uint32_t)i;
  len = is_head ? inf.y : 0u;
}

GEEK_D uint32_t flag_bits16(const GroupOut& go, int t, int64_t i0) {
  return (go.flags[(int64_t)t * go.flag_words + (i0 >> 5)] >> (i0 & 31)) & 0xFFFFu;
}

__global__ __launch_bounds__(BZ_THREADS) void k_bz_reduce(int64_t n, int nch, GroupOut go, uint2* ctot) {
  __shared__ uint32_t sh[17];
  const int t = blockIdx.y, c = blockIdx.x;
  const int64_t i0 = (int64_t)c * SC_CHUNK + (int64_t)threadIdx.x * BZ_PER;
  uint32_t h = 0, l = 0;
  if (i0 < n) {
    const uint32_t fb = flag_bits16(go, t, i0);
#pragma unroll
    for (int u = 0; u < BZ_PER; ++u) {
      const int64_t i = i0 + u;
      if (i >= n) break;
      uint32_t ih, len;
      uint2 inf;
      id_bucket(go, t, n, i, (fb >> u) & 1u, ih, len, inf);
      h += ih;
      l += len;
    }
  }
  uint32_t th, tl;
  block_exscan(h, &th, sh);
  block_exscan(l, &tl, sh);
  if (threadIdx.x == 0) ctot[(int64_t)t * nch + c] = make_uint2(th, tl);
}

__global__ __launch_bounds__(1024) void k_scan_chunks(int nch, uint2* ctot, uint32_t* nbuckets) {
  __shared__ uint32_t sh[17];
  const int t = blockIdx.x;
  uint2* ct = ctot + (int64_t)t * nch;
  const int per = (nch + 1023) / 1024;
  uint32_t lh = 0, ll = 0;
  for (int q = 0; q < per; ++q) {
    const int c = threadIdx.x * per + q;
    if (c < nch) {
      lh += ct[c].x;
      ll += ct[c].y;
    }
  }
  uint32_t tot;
  uint32_t bh = block_exscan(lh, &tot, sh);
  uint32_t bl = block_exscan(ll, nullptr, sh);
  for (int q = 0; q < per; ++q) {
    const int c = threadIdx.x * per + q;
    if (c < nch) {
      const uint2 v = ct[c];
      ct[c] = make_uint2(bh, bl);
      bh += v.x;
      bl += v.y;
    }
  }
  if (threadIdx.x == 0) nbuckets[t] = tot;
}

// Bucket ranks and CSR offsets in smallest-member order; heads (and every
// object alone in its bucket) are written to their slot; heads of larger
// buckets leave (start, rank) for their members.  Each thread scans 16
// consecutive ids; the chunk's heads (consecutive ranks) are staged in LDS
// and written by consecutive threads, so the offsets and the member slots of
// buckets of one are stored as contiguous runs.
__global__ __launch_bounds__(BZ_THREADS) void k_bz_apply(int64_t n, int nch, GroupOut go, const uint2* ctot,
                                                         uint2* hs, uint32_t* members, uint32_t* offsets,
                                                         uint32_t* bucket_of, const uint32_t* nbuckets) {
  __shared__ uint32_t sh[17];
  __shared__ uint32_t s_slot[SC_CHUNK];  // member slot of the chunk's q-th head
  __shared__ uint32_t s_id[SC_CHUNK];    // its id
  __shared__ uint32_t s_bof[SC_CHUNK];   // bucket rank of each head id of the chunk, else ~0
  const int t = blockIdx.y, c = blockIdx.x;
  const int64_t c0 = (int64_t)c * SC_CHUNK;
  const int64_t i0 = c0 + (int64_t)threadIdx.x * BZ_PER;
  const int64_t tn = (int64_t)t * n;
  uint32_t fb = 0, lh = 0, ll = 0;
  uint32_t ihv[BZ_PER], lenv[BZ_PER];
  if (i0 < n) fb = flag_bits16(go, t, i0);
#pragma unroll
  for (int u = 0; u < BZ_PER; ++u) {
    const int64_t i = i0 + u;
    ihv[u] = 0;
    lenv[u] = 0;
    if (i < n) {
      uint2 inf;
      id_bucket(go, t, n, i, (fb >> u) & 1u, ihv[u], lenv[u], inf);
    }
    lh += ihv[u];
    ll += lenv[u];
  }
  const uint2 base = ctot[(int64_t)t * nch + c];
  uint32_t nh;
  const uint32_t q0 = block_exscan(lh, &nh, sh);
  uint32_t bl = block_exscan(ll, nullptr, sh) + base.y;
  uint32_t q = q0;
#pragma unroll
  for (int u = 0; u < BZ_PER; ++u) {
    const int l = threadIdx.x * BZ_PER + u;
    if (bucket_of) s_bof[l] = ihv[u] ? base.x + q : 0xFFFFFFFFu;
    if (!ihv[u]) continue;
    const uint32_t i = (uint32_t)(i0 + u);
    s_slot[q] = bl;
    s_id[q] = i;
    if ((fb >> u) & 1u) hs[tn + i] = make_uint2(bl, base.x + q);
    ++q;
    bl += lenv[u];
  }
  __syncthreads();
  uint32_t* off = offsets + (int64_t)t * (n + 1);
  for (uint32_t k = threadIdx.x; k < nh; k += BZ_THREADS) {
    const uint32_t sl = s_slot[k];
    off[base.x + k] = sl;
    members[tn + sl] = s_id[k];
  }
  if (bucket_of) {
    const int64_t cl = n - c0 < SC_CHUNK ? n - c0 : SC_CHUNK;
    for (int l = threadIdx.x; l < cl; l += BZ_THREADS)
      if (s_bof[l] != 0xFFFFFFFFu) bucket_of[tn + c0 + l] = s_bof[l];
  }
  if (c == 0 && threadIdx.x == 0) off[nbuckets[t]] = (uint32_t)n;
}

// Members of buckets of two or more, other than the head.
__global__ __launch_bounds__(BZ_THREADS) void k_bz_members(int64_t n, GroupOut go, const uint2* hs,
                                                           uint32_t* members, uint32_t* bucket_of) {
  const int t = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * SC_CHUNK + (int64_t)threadIdx.x * BZ_PER;
  if (i0 >= n) return;
  const uint32_t fb = flag_bits16(go, t, i0);
  if (!fb) return;
  const int64_t tn = (int64_t)t * n;
#pragma unroll
  for (int u = 0; u < BZ_PER; ++u) {
    const int64_t i = i0 + u;
    if (i >= n || !((fb >> u) & 1u)) continue;
    const uint2 inf = go.info[tn + i];
    if (inf.x == (uint32_t)i) continue;  // head: already written
    const uint2 h = hs[tn + inf.x];
    members[tn + h.x + inf.y] = (uint32_t)i;
    if (bucket_of) bucket_of[tn + i] = h.y;
  }
}

// ---------------------------------------------------------------- host side
// Chunks of the second partition pass: at most one partial chunk per
// first-pass bin beyond the full ones.
static size_t p2_max_chunks(int64_t n, int T) {
  return (size_t)T * ((size_t)1 << PT_B1) + (size_t)ceil_div((int64_t)T * n, PT_SUPER);
}

static int bin_bits(int64_t n) {
  int nb = 0;
  while (nb < BZ_MAXBITS && (n >> nb) > 1536) ++nb;
  return nb;
}

struct BzWs {
  uint32_t *counts, *bintot, *binstart, *st_ids, *alt_ids, *flags;
  uint32_t *counts2, *bintot1, *binstart1, *cbase;  // second partition pass
  uint4 *st_keys, *alt_keys;
  uint2 *info, *hs, *ctot;
  uint32_t *big_list, *big_count;
};

static size_t carve_bz(const geek_bucketize_job& J, void* ws, BzWs& W) {
  Carver c(ws);
  const int nb = bin_bits(J.n);
  const int nbins = 1 << nb;
  const int nblk = ceil_div(J.n, PT_SUPER);
  const int nch = ceil_div(J.n, SC_CHUNK);
  const size_t Tn = (size_t)J.T * J.n;
  const int64_t fw = ceil_div(J.n, 32);
  const bool two = nb > PT_B1;
  const int nb1bins = 1 << (two ? PT_B1 : nb);
  W.counts = c.take<uint32_t>((size_t)J.T * nblk * nb1bins);
  const size_t maxchunks = two ? p2_max_chunks(J.n, J.T) : 0;
  W.counts2 = c.take<uint32_t>(two ? maxchunks * ((size_t)1 << (nb - PT_B1)) : 4);
  W.bintot1 = c.take<uint32_t>((size_t)J.T * nb1bins);
  W.binstart1 = c.take<uint32_t>((size_t)J.T * nb1bins);
  W.cbase = c.take<uint32_t>((size_t)J.T * nb1bins + 1);
  W.bintot = c.take<uint32_t>((size_t)J.T * nbins);
  W.binstart = c.take<uint32_t>((size_t)J.T * nbins);
  W.st_keys = c.take<uint4>(Tn);
  W.alt_keys = c.take<uint4>(Tn);
  W.hs = reinterpret_cast<uint2*>(W.alt_keys);  // used after the oversize-bin sorts
  W.st_ids = c.take<uint32_t>(Tn);
  W.alt_ids = c.take<uint32_t>(Tn);
  W.flags = c.take<uint32_t>((size_t)J.T * fw);
  W.info = c.take<uint2>(Tn);
  W.ctot = c.take<uint2>((size_t)J.T * nch);
  W.big_list = c.take<uint32_t>((size_t)J.T * nbins);
  W.big_count = c.take<uint32_t>(4);
  return c.used + 256;
}

size_t bucketize_ws(const geek_bucketize_job& J) {
  BzWs W;
  return carve_bz(J, nullptr, W);
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

int32_t bucketize_run(const geek_bucketize_job& J, void* ws, size_t ws_bytes, int32_t* st,
                      hipStream_t s) {
  (void)st;
  BzWs W;
  if (ws_bytes < carve_bz(J, ws, W)) return GEEK_ERR_WORKSPACE;
  const int nb = bin_bits(J.n);
  const int nbins = 1 << nb;
  const int nblk = ceil_div(J.n, PT_SUPER);
  const int nch = ceil_div(J.n, SC_CHUNK);
  const int64_t fw = ceil_div(J.n, 32);
  BzArgs a{J.keys, J.n, J.T, J.key_words, J.table_stride, J.row_stride, nb};
  GroupOut go{W.flags, W.info, fw};
  const size_t hbytes = (size_t)nbins * 4;
  prof_begin(GEEK_PROF_BUCKETIZE, s);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, W.big_count, (int64_t)4);
  hipLaunchKernelGGL(k_zero_u32, dim3(ceil_div((int64_t)J.T * fw, 256)), dim3(256), 0, s, W.flags,
                     (int64_t)J.T * fw);
  if (nb <= PT_B1) {
    hipLaunchKernelGGL(k_bin_count, dim3(nblk, J.T), dim3(BZ_THREADS), hbytes, s, a, nblk, PT_SUPER, W.counts);
    hipLaunchKernelGGL(k_bin_colscan, dim3(ceil_div((int64_t)J.T * nbins, 256)), dim3(256), 0, s, J.T,
                       nblk, nbins, W.counts, W.bintot);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, nbins, W.bintot, W.binstart);
    hipLaunchKernelGGL(k_p1_scatter, dim3(nblk, J.T), dim3(BZ_THREADS), 0, s, a, nblk, W.counts, W.binstart,
                       W.st_keys, W.st_ids);
  } else {
    // first pass into the alternate buffers by the top PT_B1 bits, second
    // pass by the next nb - PT_B1 bits into the staging buffers
    BzArgs a1 = a;
    a1.nb = PT_B1;
    const int nb1bins = J.T << PT_B1;
    const int F = 1 << (nb - PT_B1);
    const int maxchunks = (int)p2_max_chunks(J.n, J.T);
    hipLaunchKernelGGL(k_bin_count, dim3(nblk, J.T), dim3(BZ_THREADS), (size_t)4 << PT_B1, s, a1, nblk, PT_SUPER,
                       W.counts);
    hipLaunchKernelGGL(k_bin_colscan, dim3(ceil_div(nb1bins, 256)), dim3(256), 0, s, J.T, nblk, 1 << PT_B1,
                       W.counts, W.bintot1);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, 1 << PT_B1, W.bintot1, W.binstart1);
    hipLaunchKernelGGL(k_p1_scatter, dim3(nblk, J.T), dim3(BZ_THREADS), 0, s, a1, nblk, W.counts, W.binstart1,
                       W.alt_keys, W.alt_ids);
    hipLaunchKernelGGL(k_p2_chunks, dim3(1), dim3(1024), 0, s, nb1bins, W.bintot1, W.cbase);
    hipLaunchKernelGGL(k_p2_count, dim3(maxchunks), dim3(BZ_THREADS), 0, s, J.n, nb, W.cbase, nb1bins, W.bintot1,
                       W.binstart1, W.alt_keys, W.counts2);
    hipLaunchKernelGGL(k_p2_colscan, dim3(ceil_div((int64_t)nb1bins * F, 256)), dim3(256), 0, s, nb1bins, F,
                       W.cbase, W.counts2, W.bintot);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, nbins, W.bintot, W.binstart);
    hipLaunchKernelGGL(k_p2_scatter, dim3(maxchunks), dim3(BZ_THREADS), 0, s, J.n, nb, W.cbase, nb1bins,
                       W.bintot1, W.binstart1, W.alt_keys, W.alt_ids, W.counts2, W.binstart, W.st_keys, W.st_ids);
  }
  prof_begin(GEEK_PROF_BZ_SORT, s);
  hipLaunchKernelGGL(k_bin_group, dim3(nbins, J.T), dim3(BZ_THREADS), 0, s, J.n, nb, W.bintot, W.binstart,
                     W.st_keys, W.st_ids, go, W.big_list, W.big_count);
  prof_end(GEEK_PROF_BZ_SORT, s);
  hipLaunchKernelGGL(k_big_sort, dim3(256), dim3(BIG_THREADS), 0, s, J.n, nb, J.key_words, W.bintot,
                     W.binstart, W.st_keys, W.st_ids, W.alt_keys, W.alt_ids, W.big_list, W.big_count);
  hipLaunchKernelGGL(k_big_runs, dim3(256), dim3(BIG_THREADS), 0, s, J.n, nb, W.bintot, W.binstart,
                     W.st_keys, W.st_ids, go, W.big_list, W.big_count);
  hipLaunchKernelGGL(k_bz_reduce, dim3(nch, J.T), dim3(BZ_THREADS), 0, s, J.n, nch, go, W.ctot);
  hipLaunchKernelGGL(k_scan_chunks, dim3(J.T), dim3(1024), 0, s, nch, W.ctot, J.nbuckets);
  hipLaunchKernelGGL(k_bz_apply, dim3(nch, J.T), dim3(BZ_THREADS), 0, s, J.n, nch, go, W.ctot, W.hs,
                     J.members, J.offsets, J.bucket_of, J.nbuckets);
  hipLaunchKernelGGL(k_bz_members, dim3(nch, J.T), dim3(BZ_THREADS), 0, s, J.n, go, W.hs, J.members,
                     J.bucket_of);
  prof_end(GEEK_PROF_BUCKETIZE, s);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
