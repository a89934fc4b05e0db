// Buckets of every table (paper Algorithms 2 and 3: T[G(x_j)].push(j)) on
// gfx950: group the objects whose table keys are identical.
//
//  1. k_fp_count: a 32-bit fingerprint f of every exact key (written once)
//     and the histogram of its top bits per chunk of ids.
//  2. A stable partition of (f, id) records into 2^nb bins per table by the
//     top nb bits of f (equal keys always share a bin): up to 2^PT_B1 bins in
//     one pass, else a second pass splits every first-pass bin by the next
//     bits.  Each scatter ranks the records of a round in index order
//     (wavefront ballots on the bin) and writes every bin's run contiguously,
//     so each bin keeps its ids ascending.
//  3. k_group: one workgroup per (bin, table) streams the bin's records in
//     order through an LDS table keyed by the exact key (fingerprint first,
//     the exact keys compared only when fingerprints match).  With the ids in
//     order, a record's rank in its bucket is the number of earlier records of
//     that bucket: per step, wavefront ballots on the slot give the ranks
//     within the step and a per-slot counter carries them across steps; the
//     rank-0 record is the bucket's head (smallest id).  Objects that share
//     their key record (head, rank) -- or (head, size) at the head -- in
//     id-indexed arrays plus a flag bit; objects alone in their bucket write
//     nothing.  A bin with more distinct keys than the table holds is
//     processed in sub-ranges of a second hash of the exact key.
//  4. k_bz_reduce / k_scan_chunks / k_bz_apply: a scan over ids in id order
//     gives every bucket its rank in smallest-member order and its CSR
//     offset; every head (including objects alone in their bucket) is
//     written to its slot at once.
//  5. k_bz_members: the remaining members of buckets of two or more go to
//     head offset + rank.
#include "common.hpp"

namespace geek {

constexpr int BZ_THREADS = 256;
constexpr int BZ_MAXBITS = 14;    // at most 16384 bins per table
constexpr int SC_CHUNK = 4096;    // elements per block in the scans

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
GEEK_D uint32_t fp_of(const uint4& k) {
  const uint32_t w[4] = {k.x, k.y, k.z, k.w};
  return key_hash(w, 4);
}
// A second hash of the exact key (independent of the fingerprint): splits a
// bin whose distinct keys overflow the grouping table.
GEEK_D uint32_t fp2_of(const uint4& k) {
  const uint32_t w[4] = {k.x ^ 0x3C6EF372u, k.y ^ 0xA54FF53Au, k.z ^ 0x510E527Fu, k.w ^ 0x9B05688Cu};
  return fmix32(key_hash(w, 4) + 0x1F83D9ABu);
}
GEEK_D uint32_t bin_bits_of(uint32_t f, int nb) { return nb ? f >> (32 - nb) : 0u; }
GEEK_D bool key_eq(const uint4& a, const uint4& b) {
  return a.x == b.x && a.y == b.y && a.z == b.z && a.w == b.w;
}

// ---------------------------------------------------------------- partition
// Fingerprint of every (table, id) and the per-chunk histogram of its top nb
// bits.
__global__ __launch_bounds__(BZ_THREADS) void k_fp_count(BzArgs a, int nblk, int chunk, uint32_t* counts,
                                                         uint32_t* fp) {
  extern __shared__ uint32_t hist[];
  const int t = blockIdx.y, blk = blockIdx.x;
  const int nbins = 1 << a.nb;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS) hist[b] = 0;
  __syncthreads();
  const int64_t s = (int64_t)blk * chunk;
  const int64_t e = s + chunk < a.n ? s + chunk : a.n;
  for (int64_t i = s + threadIdx.x; i < e; i += BZ_THREADS) {
    const uint32_t f = fp_of(load_key(a, t, i));
    fp[(int64_t)t * a.n + i] = f;
    atomicAdd(&hist[bin_bits_of(f, a.nb)], 1u);
  }
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
constexpr int PT_ROUND = 2048;    // records placed in LDS per round
constexpr int PT_SUPER = 16384;   // records per workgroup of a partition pass
constexpr int PT_RPT = PT_ROUND / BZ_THREADS;

// One round of a stable partition scatter: the round's `cnt` records
// (fingerprint, id, bin), taken in index order, get their place among the
// round's records of the same bin (sub-rounds of BZ_THREADS records in order;
// within a sub-round wavefront ballots match the bin bits, earlier waves'
// counts come from LDS), are staged in LDS in bin order and written out so
// that consecutive threads store consecutive records of a bin.  cur[b] is
// the global position of bin b's next record and advances by the round's
// count; every bin receives its records in index order.
struct PartLds {
  uint32_t f[PT_ROUND];
  uint32_t id[PT_ROUND];
  uint16_t bin[PT_ROUND];
  uint32_t hist[256], lst[256], lrun[256], cur[256], sh[17];
  uint32_t wcnt[BZ_THREADS / 64][256];
};

template <class Load>
__device__ void part_round(PartLds& L, int nbins, int nbits, int cnt, const Load& load, uint32_t* out_f,
                           uint32_t* out_id) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int b = tid; b < nbins; b += BZ_THREADS) L.hist[b] = 0u;
  for (int w = 0; w < BZ_THREADS / 64; ++w)
    for (int b = tid; b < nbins; b += BZ_THREADS) L.wcnt[w][b] = 0u;
  __syncthreads();
  uint32_t f[PT_RPT], id[PT_RPT];
  int bn[PT_RPT];
#pragma unroll
  for (int u = 0; u < PT_RPT; ++u) {
    const int q = u * BZ_THREADS + tid;
    bn[u] = 0;
    if (q < cnt) {
      load(q, f[u], id[u], bn[u]);
      atomicAdd(&L.hist[bn[u]], 1u);
    }
  }
  __syncthreads();
  // exclusive scan of the round's bin counts (nbins <= 256 = one per thread)
  const uint32_t hv = tid < nbins ? L.hist[tid] : 0u;
  const uint32_t ex = block_exscan(hv, nullptr, L.sh);
  if (tid < nbins) {
    L.lst[tid] = ex;
    L.lrun[tid] = ex;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PT_RPT; ++u) {
    const int q = u * BZ_THREADS + tid;
    const bool has = q < cnt;
    const uint32_t dg = has ? (uint32_t)bn[u] : 0u;
    uint64_t mask = __ballot(has);
    for (int b = 0; b < nbits; ++b) {
      const uint64_t bb = __ballot(has && ((dg >> b) & 1u));
      mask &= ((dg >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    const bool leader = has && below == 0;
    if (leader) L.wcnt[wv][dg] = (uint32_t)__popcll(mask);
    __syncthreads();
    if (has) {
      uint32_t before = 0;
      for (int w2 = 0; w2 < wv; ++w2) before += L.wcnt[w2][dg];
      const uint32_t p = L.lrun[dg] + before + below;
      L.f[p] = f[u];
      L.id[p] = id[u];
      L.bin[p] = (uint16_t)dg;
    }
    __syncthreads();
    if (tid < nbins) {
      uint32_t tot = 0;
      for (int w2 = 0; w2 < BZ_THREADS / 64; ++w2) tot += L.wcnt[w2][tid];
      L.lrun[tid] += tot;
    }
    __syncthreads();
    if (leader) L.wcnt[wv][dg] = 0u;
    __syncthreads();
  }
  for (int p = tid; p < cnt; p += BZ_THREADS) {
    const int b = L.bin[p];
    const uint32_t gp = L.cur[b] + (uint32_t)p - L.lst[b];
    out_f[gp] = L.f[p];
    out_id[gp] = L.id[p];
  }
  __syncthreads();
  for (int b = tid; b < nbins; b += BZ_THREADS) L.cur[b] += L.hist[b];
}

// First pass: block (chunk of PT_SUPER ids, table) -> 2^nb1 bins by the top
// nb1 bits of the fingerprint (nb1 <= PT_B1).
__global__ __launch_bounds__(BZ_THREADS) void k_p1_scatter(BzArgs a, int nb1, int nblk, const uint32_t* counts,
                                                           const uint32_t* binstart, const uint32_t* fp,
                                                           uint32_t* out_f, uint32_t* out_id) {
  __shared__ PartLds L;
  const int t = blockIdx.y, blk = blockIdx.x;
  const int nbins = 1 << nb1;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS)
    L.cur[b] = binstart[(int64_t)t * nbins + b] + counts[((int64_t)t * nblk + blk) * nbins + b];
  const int64_t s = (int64_t)blk * PT_SUPER;
  const int64_t e = s + PT_SUPER < a.n ? s + PT_SUPER : a.n;
  const uint32_t* fpt = fp + (int64_t)t * a.n;
  for (int64_t r0 = s; r0 < e; r0 += PT_ROUND) {
    const int cnt = (int)(e - r0 < PT_ROUND ? e - r0 : PT_ROUND);
    part_round(L, nbins, nb1, cnt,
               [&](int q, uint32_t& f, uint32_t& id, int& bn) {
                 f = fpt[r0 + q];
                 id = (uint32_t)(r0 + q);
                 bn = (int)bin_bits_of(f, nb1);
               },
               out_f + (int64_t)t * a.n, out_id + (int64_t)t * a.n);
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
                                                         const uint32_t* f1, uint32_t* counts2) {
  __shared__ uint32_t hist[256];
  const uint32_t g = blockIdx.x;
  if (g >= cbase[nb1bins]) return;
  const int F = 1 << (nb - PT_B1);
  const int tb = p2_bin_of_chunk(cbase, nb1bins, g);
  const int t = tb >> PT_B1;
  const uint32_t off = (g - cbase[tb]) * (uint32_t)PT_SUPER;
  const uint32_t cnt = min((uint32_t)PT_SUPER, bintot1[tb] - off);
  const uint32_t* src = f1 + (int64_t)t * n + binstart1[tb] + off;
  for (int b = threadIdx.x; b < F; b += BZ_THREADS) hist[b] = 0u;
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < cnt; q += BZ_THREADS)
    atomicAdd(&hist[bin_bits_of(src[q], nb) & (uint32_t)(F - 1)], 1u);
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
                                                           const uint32_t* f1, const uint32_t* ids1,
                                                           const uint32_t* counts2, const uint32_t* binstart,
                                                           uint32_t* out_f, uint32_t* out_id) {
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
    part_round(L, F, nb - PT_B1, cnt,
               [&](int q, uint32_t& f, uint32_t& id, int& bn) {
                 f = f1[s + r0 + q];
                 id = ids1[s + r0 + q];
                 bn = (int)(bin_bits_of(f, nb) & (uint32_t)(F - 1));
               },
               out_f + (int64_t)t * n, out_id + (int64_t)t * n);
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

// One workgroup per (bin, table).  The bin's records (fingerprint, id) are in
// ascending id order.  An LDS table maps each distinct exact key to a slot:
// a slot word holds the fingerprint and 1 + the bin position of the record
// that claimed it; a record whose fingerprint matches a slot compares its
// exact key with the claimant's (both read from the keys array), so only
// records that share a fingerprint touch the keys.  Records go through in
// steps of BZ_THREADS in order; ranks come from ballots on the slot within
// each wavefront, the per-wavefront counts of earlier wavefronts (cleared at
// the end of each step) and the slot's count of earlier steps.  Bins of at most GB_FILL records fit the
// table whatever their keys (one pass); larger bins build the table first and
// are processed in sub-ranges of a second key hash (1, 64, 4096, ... of them)
// if their distinct keys do not fit.
constexpr int GB_HT = 2048;             // slots of the table
constexpr int GB_FILL = 1792;           // distinct keys per (sub-)range
constexpr int GB_SBITS = 11;            // bits of a slot index
constexpr int GB_LEVELS = 5;            // sub-range splits: 1, 2^6, 2^12, 2^18, 2^24
struct GroupLds {
  unsigned long long slot[GB_HT];
  uint32_t cnt[GB_HT];
  uint32_t head[GB_HT];
  uint16_t wc[BZ_THREADS / 64][GB_HT];  // records of each wavefront in the slot, this step
  uint32_t nslot, over;
};

// Slot of a record's exact key; inserts it when `ins`.  -1: the table has no
// room (or, without insertion, the key is absent).
GEEK_D int gb_slot(GroupLds& G, const BzArgs& a, int t, uint32_t f, uint32_t pos, uint32_t id,
                   const uint32_t* __restrict__ bin_ids, bool ins) {
  uint32_t h = f & (GB_HT - 1);
  uint4 mine = make_uint4(0u, 0u, 0u, 0u);
  bool have = false;
  for (int probe = 0; probe < GB_HT; ++probe) {
    unsigned long long s = G.slot[h];
    if (s == 0ull) {
      if (!ins) return -1;
      const unsigned long long v = ((unsigned long long)f << 32) | (unsigned long long)(pos + 1u);
      const unsigned long long prev = atomicCAS(&G.slot[h], 0ull, v);
      if (prev == 0ull) {
        atomicAdd(&G.nslot, 1u);
        return (int)h;
      }
      s = prev;
    }
    if ((uint32_t)(s >> 32) == f) {
      const uint32_t opos = (uint32_t)s - 1u;
      if (opos == pos) return (int)h;
      if (!have) {
        mine = load_key(a, t, id);
        have = true;
      }
      if (key_eq(load_key(a, t, bin_ids[opos]), mine)) return (int)h;
    }
    h = (h + 1u) & (GB_HT - 1);
  }
  return -1;
}

__global__ __launch_bounds__(BZ_THREADS) void k_group(BzArgs a, const uint32_t* bintot, const uint32_t* binstart,
                                                      const uint32_t* st_f, const uint32_t* st_id, GroupOut go,
                                                      int32_t* st) {
  __shared__ GroupLds G;
  const int t = blockIdx.y, bin = blockIdx.x;
  const int nbins = 1 << a.nb;
  const uint32_t size = bintot[(int64_t)t * nbins + bin];
  if (size <= 1) return;  // empty, or one record: a bucket of its own
  const int64_t n = a.n;
  const uint32_t s0 = binstart[(int64_t)t * nbins + bin];
  const uint32_t* fptr = st_f + (int64_t)t * n + s0;
  const uint32_t* iptr = st_id + (int64_t)t * n + s0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int level = 0; level < GB_LEVELS; ++level) {
    const int sbits = 6 * level;
    const uint32_t nsub = 1u << sbits;
    bool done = true;
    for (uint32_t r = 0; r < nsub; ++r) {
      // the records of this sub-range: all records at level 0, else those
      // whose second key hash has r in its low sbits bits
      auto in_range = [&](uint32_t q) -> bool {
        if (level == 0) return true;
        return (fp2_of(load_key(a, t, iptr[q])) & (nsub - 1u)) == r;
      };
      for (int h = tid; h < GB_HT; h += BZ_THREADS) {
        G.slot[h] = 0ull;
        G.cnt[h] = 0u;
#pragma unroll
        for (int w = 0; w < BZ_THREADS / 64; ++w) G.wc[w][h] = 0;
      }
      if (tid == 0) {
        G.nslot = 0u;
        G.over = 0u;
      }
      __syncthreads();
      // a range that could hold more distinct keys than fit: build the table first
      const bool build = level > 0 || size > (uint32_t)GB_FILL;
      if (build) {
        for (uint32_t q0 = 0; q0 < size; q0 += BZ_THREADS) {
          const uint32_t q = q0 + tid;
          if (q < size && in_range(q)) {
            const int g = gb_slot(G, a, t, fptr[q], q, iptr[q], iptr, true);
            if (g < 0) G.over = 1u;
          }
          __syncthreads();
          if (G.over || G.nslot > (uint32_t)GB_FILL) break;  // uniform: read after the barrier
          __syncthreads();
        }
        __syncthreads();
        if (G.over || G.nslot > (uint32_t)GB_FILL) {
          done = false;
          __syncthreads();
          break;  // split this bin more finely
        }
      }
      for (uint32_t q0 = 0; q0 < size; q0 += BZ_THREADS) {
        const uint32_t q = q0 + tid;
        bool valid = q < size && in_range(q);
        uint32_t id = 0u;
        int g = -1;
        if (valid) {
          id = iptr[q];
          g = gb_slot(G, a, t, fptr[q], q, id, iptr, !build);
          valid = g >= 0;
        }
        __syncthreads();  // every insertion of the step is done
        uint64_t mask = __ballot(valid);
        for (int b = 0; b < GB_SBITS; ++b) {
          const uint64_t bb = __ballot(valid && ((g >> b) & 1));
          mask &= ((g >> b) & 1) ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        const uint32_t wcount = (uint32_t)__popcll(mask);
        const bool leader = valid && below == 0;
        if (leader) G.wc[wv][g] = (uint16_t)wcount;
        __syncthreads();
        uint32_t rank = 0u;
        if (valid) {
          uint32_t before = 0u;
          for (int w2 = 0; w2 < wv; ++w2) before += G.wc[w2][g];
          rank = G.cnt[g] + before + below;
          if (rank == 0u) G.head[g] = id;
        }
        __syncthreads();
        if (valid && rank > 0u) group_record(go, t, n, id, G.head[g], rank);
        if (leader) {
          atomicAdd(&G.cnt[g], wcount);
          G.wc[wv][g] = 0;
        }
        __syncthreads();
      }
      // heads of buckets of two or more: (head, size)
      for (int h = tid; h < GB_HT; h += BZ_THREADS)
        if (G.slot[h] != 0ull && G.cnt[h] >= 2u) group_record(go, t, n, G.head[h], G.head[h], G.cnt[h]);
      __syncthreads();
    }
    if (done) return;
  }
  // more than GB_FILL distinct keys share 24 bits of the second hash in one
  // bin: not handled
  if (tid == 0) set_status(st, GEEK_ERR_KEYS);
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
  uint32_t *counts, *bintot, *binstart, *fp, *st_f, *st_id, *alt_f, *alt_id, *flags;
  uint32_t *counts2, *bintot1, *binstart1, *cbase;  // second partition pass
  uint2 *info, *hs, *ctot;
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
  W.fp = c.take<uint32_t>(Tn);
  W.st_f = c.take<uint32_t>(Tn);
  W.st_id = c.take<uint32_t>(Tn);
  W.alt_f = two ? c.take<uint32_t>(Tn) : nullptr;
  W.alt_id = two ? c.take<uint32_t>(Tn) : nullptr;
  W.flags = c.take<uint32_t>((size_t)J.T * fw);
  W.info = c.take<uint2>(Tn);
  W.hs = c.take<uint2>(Tn);
  W.ctot = c.take<uint2>((size_t)J.T * nch);
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
  BzWs W;
  if (ws_bytes < carve_bz(J, ws, W)) return GEEK_ERR_WORKSPACE;
  const int nb = bin_bits(J.n);
  const int nbins = 1 << nb;
  const int nblk = ceil_div(J.n, PT_SUPER);
  const int nch = ceil_div(J.n, SC_CHUNK);
  const int64_t fw = ceil_div(J.n, 32);
  BzArgs a{J.keys, J.n, J.T, J.key_words, J.table_stride, J.row_stride, nb};
  GroupOut go{W.flags, W.info, fw};
  prof_begin(GEEK_PROF_BUCKETIZE, s);
  hipLaunchKernelGGL(k_zero_u32, dim3(ceil_div((int64_t)J.T * fw, 256)), dim3(256), 0, s, W.flags,
                     (int64_t)J.T * fw);
  if (nb <= PT_B1) {
    hipLaunchKernelGGL(k_fp_count, dim3(nblk, J.T), dim3(BZ_THREADS), (size_t)nbins * 4, s, a, nblk, PT_SUPER,
                       W.counts, W.fp);
    hipLaunchKernelGGL(k_bin_colscan, dim3(ceil_div((int64_t)J.T * nbins, 256)), dim3(256), 0, s, J.T,
                       nblk, nbins, W.counts, W.bintot);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, nbins, W.bintot, W.binstart);
    hipLaunchKernelGGL(k_p1_scatter, dim3(nblk, J.T), dim3(BZ_THREADS), 0, s, a, nb, nblk, W.counts, W.binstart,
                       W.fp, W.st_f, W.st_id);
  } else {
    // first pass into the alternate buffers by the top PT_B1 bits, second
    // pass by the next nb - PT_B1 bits into the staging buffers
    BzArgs a1 = a;
    a1.nb = PT_B1;
    const int nb1bins = J.T << PT_B1;
    const int F = 1 << (nb - PT_B1);
    const int maxchunks = (int)p2_max_chunks(J.n, J.T);
    hipLaunchKernelGGL(k_fp_count, dim3(nblk, J.T), dim3(BZ_THREADS), (size_t)4 << PT_B1, s, a1, nblk, PT_SUPER,
                       W.counts, W.fp);
    hipLaunchKernelGGL(k_bin_colscan, dim3(ceil_div(nb1bins, 256)), dim3(256), 0, s, J.T, nblk, 1 << PT_B1,
                       W.counts, W.bintot1);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, 1 << PT_B1, W.bintot1, W.binstart1);
    hipLaunchKernelGGL(k_p1_scatter, dim3(nblk, J.T), dim3(BZ_THREADS), 0, s, a1, PT_B1, nblk, W.counts,
                       W.binstart1, W.fp, W.alt_f, W.alt_id);
    hipLaunchKernelGGL(k_p2_chunks, dim3(1), dim3(1024), 0, s, nb1bins, W.bintot1, W.cbase);
    hipLaunchKernelGGL(k_p2_count, dim3(maxchunks), dim3(BZ_THREADS), 0, s, J.n, nb, W.cbase, nb1bins, W.bintot1,
                       W.binstart1, W.alt_f, W.counts2);
    hipLaunchKernelGGL(k_p2_colscan, dim3(ceil_div((int64_t)nb1bins * F, 256)), dim3(256), 0, s, nb1bins, F,
                       W.cbase, W.counts2, W.bintot);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, nbins, W.bintot, W.binstart);
    hipLaunchKernelGGL(k_p2_scatter, dim3(maxchunks), dim3(BZ_THREADS), 0, s, J.n, nb, W.cbase, nb1bins,
                       W.bintot1, W.binstart1, W.alt_f, W.alt_id, W.counts2, W.binstart, W.st_f, W.st_id);
  }
  prof_begin(GEEK_PROF_BZ_SORT, s);
  hipLaunchKernelGGL(k_group, dim3(nbins, J.T), dim3(BZ_THREADS), 0, s, a, W.bintot, W.binstart, W.st_f,
                     W.st_id, go, st);
  prof_end(GEEK_PROF_BZ_SORT, s);
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
