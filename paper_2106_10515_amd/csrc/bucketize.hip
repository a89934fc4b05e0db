// Buckets of every table (paper Algorithms 2 and 3: T[G(x_j)].push(j)) on
// gfx950: group the objects whose table keys are identical.
//
//  1. k_fp_count: a 32-bit fingerprint f of every exact key (written once,
//     or the caller's: geek_hash can write them beside the keys) and the
//     histogram of its top bits per chunk of ids.
//  2. A stable partition of (f, id) records into 2^nb bins per table by the
//     top nb bits of f (equal keys always share a bin): up to 2^PT_B1 bins in
//     one pass, else a second pass splits every first-pass bin by the next
//     bits.  Each scatter ranks a round's records in index order (per
//     wavefront: ballots on the bin and a running count; one scan over
//     (bin, wavefront) joins the wavefronts) and writes every bin's run
//     contiguously, so each bin keeps its ids ascending.
//  3. k_group: one workgroup per (bin, table) takes the bin's records in
//     order through an LDS table keyed by the exact key (fingerprint first,
//     the exact keys compared only when fingerprints match).  With the ids in
//     order, a record's rank in its bucket is the number of earlier records of
//     that bucket, counted per wavefront and joined per chunk; the rank-0
//     record is the bucket's head (smallest id).  Objects that share their key
//     record (head, rank) -- or (head, size) at the head -- in id-indexed
//     arrays plus a flag byte; objects alone in their bucket write nothing.
//     A bin with more distinct keys than the table holds is processed in
//     sub-ranges of further fingerprint bits.
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
// A partitioned record: fingerprint in the low word, id in the high word.
typedef unsigned long long BzRec;
GEEK_D BzRec rec_make(uint32_t f, uint32_t id) { return ((BzRec)id << 32) | (BzRec)f; }
GEEK_D uint32_t rec_f(BzRec r) { return (uint32_t)r; }
GEEK_D uint32_t rec_id(BzRec r) { return (uint32_t)(r >> 32); }
GEEK_D bool key_eq(const uint4& a, const uint4& b) {
  return a.x == b.x && a.y == b.y && a.z == b.z && a.w == b.w;
}

// ---------------------------------------------------------------- partition
// Fingerprint of every (table, id) and the per-chunk histogram of its top nb
// bits.  With `given` (the caller's fingerprints of these keys) the keys are
// not read and nothing is written but the histogram.
__global__ __launch_bounds__(BZ_THREADS) void k_fp_count(BzArgs a, int nblk, int chunk, uint32_t* counts,
                                                         uint32_t* fp, const uint32_t* given) {
  extern __shared__ uint32_t hist[];
  const int t = blockIdx.y, blk = blockIdx.x;
  const int nbins = 1 << a.nb;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS) hist[b] = 0;
  __syncthreads();
  const int64_t s = (int64_t)blk * chunk;
  const int64_t e = s + chunk < a.n ? s + chunk : a.n;
  for (int64_t i = s + threadIdx.x; i < e; i += BZ_THREADS) {
    uint32_t f;
    if (given) {
      f = given[(int64_t)t * a.n + i];
    } else {
      f = fp_of(load_key(a, t, i));
      fp[(int64_t)t * a.n + i] = f;
    }
    atomicAdd(&hist[bin_bits_of(f, a.nb)], 1u);
  }
  __syncthreads();
  uint32_t* out = counts + ((int64_t)t * nblk + blk) * nbins;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS) out[b] = hist[b];
}

// Fingerprints of every (table, id) when each object's T keys lie within its
// row (the bands of a signature row): FR_LANES lanes share an object and lane
// q takes tables q, q + FR_LANES, ..., so consecutive lanes read consecutive
// keys of one row, where the pass per table reads one key out of every row.
constexpr int FR_LANES = 16;
__global__ __launch_bounds__(BZ_THREADS) void k_fp_rows(BzArgs a, uint32_t* fp) {
  const int64_t i = ((int64_t)blockIdx.x * BZ_THREADS + threadIdx.x) / FR_LANES;
  const int q = (int)(threadIdx.x % FR_LANES);
  if (i >= a.n) return;
  for (int t = q; t < a.T; t += FR_LANES) fp[(int64_t)t * a.n + i] = fp_of(load_key(a, t, i));
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
constexpr int PT_ROUND = 4096;    // records placed in LDS per round (longer runs per bin)
constexpr int PT_SUPER = 16384;   // records per workgroup of a partition pass
constexpr int PT_RPT = PT_ROUND / BZ_THREADS;
constexpr int PT_SEG = PT_ROUND / (BZ_THREADS / 64);  // records of one wavefront per round

// One round of a stable partition scatter.  The round's `cnt` records
// (fingerprint, id, bin) are in index order; wavefront w holds the
// contiguous segment [w * PT_SEG, (w + 1) * PT_SEG), 64 records per step.
// Each wavefront ranks its records among its own records of the same bin
// (ballots on the bin bits, a per-wavefront running count in LDS, no
// barrier); one exclusive scan over (bin, wavefront) then gives every record
// its place among the round's records of its bin.  The records are staged in
// LDS in bin order and written out so that consecutive threads store
// consecutive records of a bin.  cur[b] is the global position of bin b's
// next record and advances by the round's count, so every bin receives its
// records in index order.
struct PartLds {
  BzRec rec[PT_ROUND];
  uint32_t wc[BZ_THREADS / 64][256];  // records of each bin in the wavefront, then its first place
  uint32_t hist[256], lst[256], cur[256], sh[17];
};

struct PartRecs {
  uint32_t f[PT_RPT], id[PT_RPT];
};

// Records of one round: record q = wave * PT_SEG + step * 64 + lane.  The
// loads are unconditional (lanes past the end read record cnt - 1 and are
// ignored), so all of a round's loads are in flight at once.
template <class Load>
GEEK_D void part_load(int cnt, const Load& load, PartRecs& R) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < PT_RPT; ++u) {
    const int q = wv * PT_SEG + u * 64 + lane;
    load(q < cnt ? q : cnt - 1, R.f[u], R.id[u]);
  }
}

// A record's bin is (f >> shift) & (nbins - 1).
__device__ void part_round(PartLds& L, int nbins, int nbits, int shift, int cnt, const PartRecs& R, BzRec* out) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = BZ_THREADS / 64;
  for (int b = lane; b < nbins; b += 64) L.wc[wv][b] = 0u;  // this wavefront's row only
  uint32_t lr[PT_RPT], bn[PT_RPT];
#pragma unroll
  for (int u = 0; u < PT_RPT; ++u) bn[u] = nbins > 1 ? (R.f[u] >> shift) & (uint32_t)(nbins - 1) : 0u;
#pragma unroll
  for (int u = 0; u < PT_RPT; ++u) {
    const int q = wv * PT_SEG + u * 64 + lane;
    const bool has = q < cnt;
    const uint32_t dg = has ? bn[u] : 0u;
    uint64_t mask = __ballot(has);
    for (int b = 0; b < nbits; ++b) {
      const uint64_t bb = __ballot(has && ((dg >> b) & 1u));
      mask &= ((dg >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    lr[u] = L.wc[wv][dg] + below;
    __builtin_amdgcn_wave_barrier();
    if (has && below == 0) L.wc[wv][dg] += (uint32_t)__popcll(mask);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per bin: the round's count, its start among the round's records, and
  // the first place of each wavefront's records of the bin
  uint32_t c[NW], tot = 0u;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    c[w] = tid < nbins ? L.wc[w][tid] : 0u;
    tot += c[w];
  }
  const uint32_t ex = block_exscan(tot, nullptr, L.sh);
  if (tid < nbins) {
    L.hist[tid] = tot;
    L.lst[tid] = ex;
    uint32_t run = ex;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      L.wc[w][tid] = run;
      run += c[w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PT_RPT; ++u) {
    const int q = wv * PT_SEG + u * 64 + lane;
    if (q < cnt) L.rec[L.wc[wv][bn[u]] + lr[u]] = rec_make(R.f[u], R.id[u]);
  }
  __syncthreads();
  for (int p = tid; p < cnt; p += BZ_THREADS) {
    const BzRec r = L.rec[p];
    const int b = nbins > 1 ? (int)((rec_f(r) >> shift) & (uint32_t)(nbins - 1)) : 0;
    out[L.cur[b] + (uint32_t)p - L.lst[b]] = r;
  }
  __syncthreads();
  if (tid < nbins) L.cur[tid] += L.hist[tid];
}

// Rounds of one workgroup.
template <class Load>
__device__ void part_rounds(PartLds& L, int nbins, int nbits, int shift, int64_t total, const Load& load,
                            BzRec* out) {
  for (int64_t r0 = 0; r0 < total; r0 += PT_ROUND) {
    const int cnt = (int)(total - r0 < PT_ROUND ? total - r0 : PT_ROUND);
    PartRecs cur;
    part_load(cnt, [&](int q, uint32_t& f, uint32_t& id) { load(r0 + q, f, id); }, cur);
    part_round(L, nbins, nbits, shift, cnt, cur, out);
  }
}

// First pass: block (chunk of PT_SUPER ids, table) -> 2^nb1 bins by the top
// nb1 bits of the fingerprint (nb1 <= PT_B1).
__global__ __launch_bounds__(BZ_THREADS) void k_p1_scatter(BzArgs a, int nb1, int nblk, const uint32_t* counts,
                                                           const uint32_t* binstart, const uint32_t* fp,
                                                           BzRec* out) {
  __shared__ PartLds L;
  const int t = blockIdx.y, blk = blockIdx.x;
  const int nbins = 1 << nb1;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS)
    L.cur[b] = binstart[(int64_t)t * nbins + b] + counts[((int64_t)t * nblk + blk) * nbins + b];
  const int64_t s = (int64_t)blk * PT_SUPER;
  const int64_t e = s + PT_SUPER < a.n ? s + PT_SUPER : a.n;
  const uint32_t* fpt = fp + (int64_t)t * a.n;
  part_rounds(L, nbins, nb1, 32 - nb1, e - s,
              [&](int64_t q, uint32_t& f, uint32_t& id) {
                f = fpt[s + q];
                id = (uint32_t)(s + q);
              },
              out + (int64_t)t * a.n);
}

// Second pass.  The records of first-pass bin (t, B) are cut into chunks of
// PT_SUPER; cbase[t * 2^PT_B1 + B] is the first global chunk of that bin and
// cbin[g] the first-pass bin of global chunk g.
__global__ __launch_bounds__(1024) void k_p2_chunks(int nb1bins, const uint32_t* bintot1, uint32_t* cbase,
                                                    uint32_t* cbin) {
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
      const uint32_t nc = (bintot1[i] + PT_SUPER - 1) / PT_SUPER;
      for (uint32_t j = 0; j < nc; ++j) cbin[base + j] = (uint32_t)i;
      base += nc;
    }
  }
  if (threadIdx.x == 0) cbase[nb1bins] = total;
}

// Per chunk: counts of the second-pass bins (the next nb - PT_B1 bits).
__global__ __launch_bounds__(BZ_THREADS) void k_p2_count(int64_t n, int nb, const uint32_t* cbase,
                                                         const uint32_t* cbin, int nb1bins,
                                                         const uint32_t* bintot1, const uint32_t* binstart1,
                                                         const BzRec* r1, uint32_t* counts2) {
  __shared__ uint32_t hist[256];
  const uint32_t g = blockIdx.x;
  if (g >= cbase[nb1bins]) return;
  const int F = 1 << (nb - PT_B1);
  const int tb = (int)cbin[g];
  const int t = tb >> PT_B1;
  const uint32_t off = (g - cbase[tb]) * (uint32_t)PT_SUPER;
  const uint32_t cnt = min((uint32_t)PT_SUPER, bintot1[tb] - off);
  const BzRec* src = r1 + (int64_t)t * n + binstart1[tb] + off;
  for (int b = threadIdx.x; b < F; b += BZ_THREADS) hist[b] = 0u;
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < cnt; q += BZ_THREADS)
    atomicAdd(&hist[bin_bits_of(rec_f(src[q]), nb) & (uint32_t)(F - 1)], 1u);
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

__global__ __launch_bounds__(BZ_THREADS) void k_p2_scatter(int64_t n, int nb, const uint32_t* cbase,
                                                           const uint32_t* cbin, int nb1bins,
                                                           const uint32_t* bintot1, const uint32_t* binstart1,
                                                           const BzRec* r1, const uint32_t* counts2,
                                                           const uint32_t* binstart, BzRec* out) {
  __shared__ PartLds L;
  const uint32_t g = blockIdx.x;
  if (g >= cbase[nb1bins]) return;
  const int F = 1 << (nb - PT_B1);
  const int tb = (int)cbin[g];
  const int t = tb >> PT_B1;
  const uint32_t off = (g - cbase[tb]) * (uint32_t)PT_SUPER;
  const uint32_t cnt_all = min((uint32_t)PT_SUPER, bintot1[tb] - off);
  const int64_t s = (int64_t)t * n + binstart1[tb] + off;
  for (int b = threadIdx.x; b < F; b += BZ_THREADS)
    L.cur[b] = binstart[(int64_t)tb * F + b] + counts2[(int64_t)g * F + b];
  part_rounds(L, F, nb - PT_B1, 32 - nb, (int64_t)cnt_all,
              [&](int64_t q, uint32_t& f, uint32_t& id) {
                const BzRec r = r1[s + q];
                f = rec_f(r);
                id = rec_id(r);
              },
              out + (int64_t)t * n);
}

// ---------------------------------------------------------------- per-bin grouping
// Id-indexed results of the grouping, per table (only objects that share
// their key with another object are recorded; every other object is a
// bucket of its own):
//   flag8  byte i is 1 iff object i is in a bucket of two or more (plain byte
//          stores: no atomics)
//   info   for flagged i: x = head (smallest id of the bucket),
//          y = bucket size if i is the head, else the rank of i in its bucket
//          (number of smaller ids)
struct GroupOut {
  uint8_t* flag8;   // [T][fstride]
  uint2* info;      // [T][n]
  int64_t fstride;  // n rounded up to 16
};

GEEK_D void group_record(const GroupOut& go, int t, int64_t n, uint32_t id, uint32_t head, uint32_t y) {
  go.info[(int64_t)t * n + id] = make_uint2(head, y);
  go.flag8[(int64_t)t * go.fstride + id] = 1;
}

// General-path grouping of one bin's records (fingerprint, id), taken in
// ascending id order -- the bins the fast path below leaves (more than
// GF_MAXREC records, or many records sharing keys).  An LDS table maps each
// distinct exact key to a slot: a slot word holds the fingerprint and 1 +
// the id of the record that claimed it; a record whose fingerprint matches a
// slot claimed by another id compares its exact key with the claimant's (the
// key loads of a chunk are issued together).  Records are taken in chunks of
// GB_CAP, lane-private in LDS while they probe; wavefront w holds the
// contiguous segment [w * GB_SEG, (w + 1) * GB_SEG) of a chunk, 64 records
// per step.  Every record is inserted first (its slot kept in a bin-ordered
// scratch array); then every wavefront counts its records per slot in order
// (ballots on the slot bits and a running count), one pass over the slots
// turns the counts into the first rank of each wavefront's records (plus the
// slot's count of earlier chunks), and the rank-0 record is the head.  A bin
// whose distinct keys do not fit the table is done in sub-ranges of further
// fingerprint bits (equal keys have equal fingerprints, so a key never spans
// two sub-ranges).
constexpr int GB_HT = 2048;                 // slots of the table
constexpr int GB_FILL = 1792;               // distinct keys per (sub-)range
constexpr int GB_SBITS = 11;                // bits of a slot index
constexpr int GB_CAP = 1024;                // records per chunk
constexpr int GB_RPL = GB_CAP / BZ_THREADS; // records per lane and chunk
constexpr int GB_SEG = GB_CAP / (BZ_THREADS / 64);
constexpr int GB_LIST = BZ_THREADS;         // listed records of the fast path
constexpr int GB_SUBBITS = 5;               // sub-range bits added per level
constexpr int GB_LEVELS = 4;                // 1, 2^5, 2^10, 2^15 sub-ranges
constexpr uint16_t GB_NONE = 0xFFFFu;
// Probe results of a record (16 bits): a slot (bits 0-10) with GB_CLAIM set
// when this record inserted it; GB_PEND | slot: the slot's claimant has the
// same fingerprint, keys not compared yet; GB_CONT | slot: it holds another
// key, probe on after it; GB_FULL: no room; GB_NONE: no record.
constexpr uint16_t GB_CLAIM = 0x1000u, GB_PEND = 0x8000u, GB_CONT = 0x4000u, GB_FULL = 0xFFFEu;
constexpr uint32_t GB_SLOTMASK = GB_HT - 1;
struct GroupLds {
  unsigned long long slot[GB_HT];
  union {
    struct {             // probing: the lane's records, thread-private
      uint32_t f[GB_CAP];
      uint32_t id[GB_CAP];
      uint16_t res[GB_CAP];
    } rec;
    struct {             // general-path ranks
      uint16_t wc[BZ_THREADS / 64][GB_HT];  // per wavefront: records this chunk, then first rank in it
      uint32_t cnt[GB_HT];                  // records of the slot's key in earlier chunks
      uint32_t head[GB_HT];                 // the key's smallest id
    } rk;
  };
  uint32_t nslot, over;
};

// A slot word: (fingerprint << 32) | (claimant id + 1); 0 = free.
// Probe for the slot of (f, id) from slot h on, visiting at most `budget`
// slots.  Returns the slot (*claimed: this call inserted it); -1: no room
// within the budget; -2: slot *ph holds the same fingerprint for another id,
// the exact keys decide.  A record's probes, continued past fingerprints of
// other keys, share one budget of GB_HT slots: the walk from its home slot
// covers the table at most once, so it ends even when the table is full.
GEEK_D int gb_probe(GroupLds& G, uint32_t f, uint32_t id, uint32_t h, int budget, uint32_t* ph, bool* claimed) {
  const unsigned long long v = ((unsigned long long)f << 32) | (unsigned long long)(id + 1u);
#pragma unroll 1
  for (int probe = 0; probe < budget; ++probe) {
    unsigned long long s = G.slot[h];
    if (s == 0ull) {
      s = atomicCAS(&G.slot[h], 0ull, v);
      if (s == 0ull) {
        *claimed = true;
        return (int)h;
      }
    }
    if ((uint32_t)(s >> 32) == f) {
      if ((uint32_t)s == id + 1u) return (int)h;
      *ph = h;
      return -2;
    }
    h = (h + 1u) & GB_SLOTMASK;
  }
  return -1;
}

GEEK_D uint16_t gb_code(int r, bool claimed, uint32_t ph) {
  if (r >= 0) return (uint16_t)((uint32_t)r | (claimed ? GB_CLAIM : 0u));
  return r == -1 ? GB_FULL : (uint16_t)(GB_PEND | ph);
}
GEEK_D uint32_t gb_claimant(const GroupLds& G, uint32_t h) { return (uint32_t)G.slot[h] - 1u; }

// Slots of the lane's records of one chunk, left in G.rec.res: probes first
// (one loop over the lane's records), then the exact-key comparisons of all
// pending records with their loads issued together, then the rare records
// whose fingerprint met another key, probing on one by one.
GEEK_D void gb_slots(GroupLds& G, const BzArgs& a, int t) {
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int u = 0; u < GB_RPL; ++u) {
    const int i = u * BZ_THREADS + tid;
    if (G.rec.res[i] == GB_NONE) continue;
    uint32_t ph = 0u;
    bool cl = false;
    const uint32_t f = G.rec.f[i];
    const int r = gb_probe(G, f, G.rec.id[i], f & GB_SLOTMASK, GB_HT, &ph, &cl);
    G.rec.res[i] = gb_code(r, cl, ph);
  }
  uint4 mk[GB_RPL], ck[GB_RPL];
#pragma unroll
  for (int u = 0; u < GB_RPL; ++u) {
    const int i = u * BZ_THREADS + tid;
    const uint16_t c = G.rec.res[i];
    if ((c & 0xC000u) == GB_PEND) {
      mk[u] = load_key(a, t, G.rec.id[i]);
      ck[u] = load_key(a, t, gb_claimant(G, c & GB_SLOTMASK));
    }
  }
#pragma unroll
  for (int u = 0; u < GB_RPL; ++u) {
    const int i = u * BZ_THREADS + tid;
    const uint16_t c = G.rec.res[i];
    if ((c & 0xC000u) == GB_PEND)
      G.rec.res[i] = key_eq(mk[u], ck[u]) ? (uint16_t)(c & GB_SLOTMASK) : (uint16_t)(GB_CONT | (c & GB_SLOTMASK));
  }
#pragma unroll 1
  for (int u = 0; u < GB_RPL; ++u) {
    const int i = u * BZ_THREADS + tid;
    uint16_t c = G.rec.res[i];
    if ((c & 0xC000u) != GB_CONT) continue;
    const uint32_t f = G.rec.f[i], id = G.rec.id[i];
    const uint4 mine = load_key(a, t, id);
    while ((c & 0xC000u) == GB_CONT) {
      uint32_t ph = 0u;
      bool cl = false;
      // slots left of the record's walk from its home slot f & GB_SLOTMASK
      const int left = GB_HT - 1 - (int)(((c & GB_SLOTMASK) - f) & GB_SLOTMASK);
      const int r = gb_probe(G, f, id, ((c & GB_SLOTMASK) + 1u) & GB_SLOTMASK, left, &ph, &cl);
      c = gb_code(r, cl, ph);
      if ((c & 0xC000u) == GB_PEND)
        c = key_eq(mine, load_key(a, t, gb_claimant(G, ph))) ? (uint16_t)ph : (uint16_t)(GB_CONT | ph);
    }
    G.rec.res[i] = c;
  }
}

// The lane's records of one chunk into G.rec (res = 0: to probe, GB_NONE: none).
GEEK_D void gb_stage(GroupLds& G, const uint32_t* f, const uint32_t* id, const bool* in) {
#pragma unroll
  for (int u = 0; u < GB_RPL; ++u) {
    const int i = u * BZ_THREADS + threadIdx.x;
    G.rec.f[i] = f[u];
    G.rec.id[i] = id[u];
    G.rec.res[i] = in[u] ? (uint16_t)0u : GB_NONE;
  }
}

// General-path ranks of one chunk (g < 0: no record) and their records;
// G.rk.cnt / G.rk.head carry across chunks, G.rk.wc is zero on entry and
// on exit (a wavefront's count of one slot in one chunk is at most GB_SEG,
// so 16 bits hold it).
GEEK_D void gb_rank_chunk(GroupLds& G, const GroupOut& go, int t, int64_t n, const int* g, const uint32_t* id) {
  constexpr int NW = BZ_THREADS / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  uint32_t lr[GB_RPL];
#pragma unroll
  for (int u = 0; u < GB_RPL; ++u) {
    const bool v = g[u] >= 0;
    const uint32_t gg = v ? (uint32_t)g[u] : 0u;
    uint64_t mask = __ballot(v);
    for (int b = 0; b < GB_SBITS; ++b) {
      const uint64_t bb = __ballot(v && ((gg >> b) & 1u));
      mask &= ((gg >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    lr[u] = (uint32_t)G.rk.wc[wv][gg] + below;
    __builtin_amdgcn_wave_barrier();
    if (v && below == 0) G.rk.wc[wv][gg] = (uint16_t)(G.rk.wc[wv][gg] + __popcll(mask));
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // the chunk's count of each slot stays with the thread that owns the slot
  // until the ranks have read the earlier chunks' counts
  constexpr int SPT = GB_HT / BZ_THREADS;
  uint32_t tot[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int h = j * BZ_THREADS + tid;
    uint32_t run = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t cw = G.rk.wc[w][h];
      G.rk.wc[w][h] = (uint16_t)run;
      run += cw;
    }
    tot[j] = run;
  }
  __syncthreads();
  uint32_t rank[GB_RPL];
#pragma unroll
  for (int u = 0; u < GB_RPL; ++u) {
    rank[u] = 0u;
    if (g[u] >= 0) {
      rank[u] = G.rk.cnt[g[u]] + G.rk.wc[wv][g[u]] + lr[u];
      if (rank[u] == 0u) G.rk.head[g[u]] = id[u];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < GB_RPL; ++u)
    if (g[u] >= 0 && rank[u] > 0u) group_record(go, t, n, id[u], G.rk.head[g[u]], rank[u]);
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int h = j * BZ_THREADS + tid;
    G.rk.cnt[h] += tot[j];
#pragma unroll
    for (int w = 0; w < NW; ++w) G.rk.wc[w][h] = 0u;
  }
  __syncthreads();
}

GEEK_D void gb_rank_clear(GroupLds& G) {
  constexpr int NW = BZ_THREADS / 64;
  for (int h = threadIdx.x; h < GB_HT; h += BZ_THREADS) {
    G.rk.cnt[h] = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) G.rk.wc[w][h] = 0u;
  }
}

// Heads of buckets of two or more: (head, size).
GEEK_D void gb_heads(GroupLds& G, const GroupOut& go, int t, int64_t n) {
  for (int h = threadIdx.x; h < GB_HT; h += BZ_THREADS)
    if (G.slot[h] != 0ull && G.rk.cnt[h] >= 2u) group_record(go, t, n, G.rk.head[h], G.rk.head[h], G.rk.cnt[h]);
}

// One bin by the general path: inserts first (slots kept in sptr), in
// sub-ranges of further fingerprint bits if its distinct keys do not fit,
// then ranks chunk by chunk.
__device__ void gb_large_bin(GroupLds& G, const BzArgs& a, int t, uint32_t size, const BzRec* rptr,
                             uint16_t* sptr, const GroupOut& go, int32_t* st) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t n = a.n;
  for (int level = 0; level < GB_LEVELS; ++level) {
    const int sbits = GB_SUBBITS * level;
    const uint32_t nsub = 1u << sbits;
    bool done = true;
    for (uint32_t r = 0; r < nsub; ++r) {
      for (int h = tid; h < GB_HT; h += BZ_THREADS) G.slot[h] = 0ull;
      if (tid == 0) {
        G.nslot = 0u;
        G.over = 0u;
      }
      __syncthreads();
      bool anydup = false, full = false;
      for (uint32_t c0 = 0; c0 < size; c0 += GB_CAP) {
        uint32_t f[GB_RPL], id[GB_RPL];
        bool in[GB_RPL];
#pragma unroll
        for (int u = 0; u < GB_RPL; ++u) {
          const uint32_t q = c0 + wv * GB_SEG + u * 64 + lane;
          in[u] = q < size;
          const BzRec rr = in[u] ? rptr[q] : 0ull;
          f[u] = rec_f(rr);
          id[u] = rec_id(rr);
          in[u] = in[u] && (level == 0 || ((f[u] << a.nb) >> (32 - sbits)) == r);
        }
        gb_stage(G, f, id, in);
        gb_slots(G, a, t);
        uint32_t nc = 0u;
#pragma unroll
        for (int u = 0; u < GB_RPL; ++u) {
          const uint32_t q = c0 + wv * GB_SEG + u * 64 + lane;
          const uint16_t c = G.rec.res[u * BZ_THREADS + tid];
          const bool ok = c < GB_CONT;
          anydup |= ok && !(c & GB_CLAIM);
          nc += (uint32_t)__popcll(__ballot(ok && (c & GB_CLAIM)));
          if (c == GB_FULL) G.over = 1u;
          if (q < size) sptr[q] = ok ? (uint16_t)(c & GB_SLOTMASK) : GB_NONE;
        }
        if (lane == 0) atomicAdd(&G.nslot, nc);
        __syncthreads();
        full = G.over || G.nslot > (uint32_t)GB_FILL;  // uniform: read between two barriers
        __syncthreads();
        if (full) break;
      }
      if (full) {
        done = false;
        break;  // split this bin more finely
      }
      // every key of the (sub-)range alone: nothing to record
      if (!__syncthreads_or(anydup)) continue;
      gb_rank_clear(G);
      __syncthreads();
      for (uint32_t c0 = 0; c0 < size; c0 += GB_CAP) {
        int g[GB_RPL];
        uint32_t id[GB_RPL];
#pragma unroll
        for (int u = 0; u < GB_RPL; ++u) {
          const uint32_t q = c0 + wv * GB_SEG + u * 64 + lane;
          const uint16_t sl = q < size ? sptr[q] : GB_NONE;
          id[u] = sl != GB_NONE ? rec_id(rptr[q]) : 0u;
          g[u] = sl != GB_NONE ? (int)sl : -1;
        }
        gb_rank_chunk(G, go, t, n, g, id);
      }
      gb_heads(G, go, t, n);
      __syncthreads();
    }
    if (done) return;
  }
  // more than GB_FILL distinct keys share every fingerprint bit the
  // sub-ranges can split on: not handled
  if (tid == 0) set_status(st, GEEK_ERR_KEYS);
}

// Fast grouping of the bins that hold few shared keys (the common case), a
// persistent kernel: workgroup b takes the (table, bin) items b, b + grid,
// ...; the next item's records and the one after's extent are loaded while
// the current one is grouped.  A record sets bit (f mod 2^16) of a "seen"
// bitmap; a bit that was already set also goes into "seen twice".  Records
// whose bit is in "seen twice" -- every record of a key shared in the bin,
// plus a few whose 16 bits merely coincide -- are listed; listed records
// that share their full fingerprint with another listed one get their exact
// keys, and their rank (number of smaller listed ids with the same key),
// bucket size and head come from one pass over the list.  Every other
// record is alone in its bucket.  Bins larger than GF_MAXREC or
// with more than GB_LIST listed records go to a list of hard items for
// k_group_hard.
constexpr int GF_BITS = 1 << 16;
constexpr int GF_MAXREC = 2048;                   // records of a fast-path bin
constexpr int GF_RPL = GF_MAXREC / BZ_THREADS;    // per lane
constexpr int GF_SEG = GF_MAXREC / (BZ_THREADS / 64);
struct FastLds {
  uint32_t seen[GF_BITS / 32];
  uint32_t twice[GF_BITS / 32];
  uint32_t lid[GB_LIST], lf[GB_LIST];
  uint4 lkey[GB_LIST];
  uint32_t nlist[2];  // list lengths, used by alternate bins
};
static_assert(GB_LIST % 8 == 0, "the list is read eight fingerprints at a time");

__global__ __launch_bounds__(BZ_THREADS) void k_group(BzArgs a, const uint32_t* bintot, const uint32_t* binstart,
                                                      const BzRec* recs, GroupOut go, uint32_t* hard,
                                                      uint32_t* nhard) {
  __shared__ FastLds S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nbins = 1 << a.nb;
  const int64_t nwork = (int64_t)a.T * nbins;
  const int64_t n = a.n;
  const int64_t step = gridDim.x;
  auto extent = [&](int64_t w, uint32_t& size, uint32_t& s0) {
    size = 0u;
    s0 = 0u;
    if (w < nwork) {
      size = bintot[w];
      s0 = binstart[w];
    }
  };
  auto records = [&](int64_t w, uint32_t size, uint32_t s0, uint32_t* f, uint32_t* id) {
    const int64_t base = (w / nbins) * n + s0;
#pragma unroll
    for (int u = 0; u < GF_RPL; ++u) {
      const uint32_t q = wv * GF_SEG + u * 64 + lane;
      const bool in = size > 1u && size <= (uint32_t)GF_MAXREC && q < size;
      const BzRec r = in ? recs[base + q] : 0ull;
      f[u] = rec_f(r);
      id[u] = rec_id(r);
    }
  };
  int64_t w = blockIdx.x;
  uint32_t sz0, b0, sz1, b1;
  extent(w, sz0, b0);
  extent(w + step, sz1, b1);
  uint32_t f0[GF_RPL], i0[GF_RPL];
  records(w, sz0, b0, f0, i0);
  // bins that reach the bitmaps alternate between the two list counters: a
  // bin's counter was last read by the bin before the previous one, so it is
  // reset after the first barrier of the previous bin without a barrier of
  // its own
  uint32_t par = 0u;
  if (tid == 0) S.nlist[0] = S.nlist[1] = 0u;
  for (; w < nwork; w += step) {
    const uint32_t size = sz0;
    uint32_t f[GF_RPL], id[GF_RPL];
#pragma unroll
    for (int u = 0; u < GF_RPL; ++u) {
      f[u] = f0[u];
      id[u] = i0[u];
    }
    uint32_t sz2, b2;
    extent(w + 2 * step, sz2, b2);
    records(w + step, sz1, b1, f0, i0);
    sz0 = sz1;
    b0 = b1;
    sz1 = sz2;
    b1 = b2;
    if (size <= 1u) continue;  // empty, or one record: a bucket of its own
    if (size > (uint32_t)GF_MAXREC) {
      if (tid == 0) hard[atomicAdd(nhard, 1u)] = (uint32_t)w;
      continue;
    }
    const int t = (int)(w / nbins);
    bool in[GF_RPL];
#pragma unroll
    for (int u = 0; u < GF_RPL; ++u) in[u] = (uint32_t)(wv * GF_SEG + u * 64 + lane) < size;
    {
      uint4* s4 = reinterpret_cast<uint4*>(S.seen);  // seen and twice are adjacent
      for (int i = tid; i < GF_BITS / 64; i += BZ_THREADS) s4[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    if (tid == 0) S.nlist[par ^ 1u] = 0u;  // the next bin's counter
#pragma unroll
    for (int u = 0; u < GF_RPL; ++u) {
      if (!in[u]) continue;
      const uint32_t b = f[u] & (GF_BITS - 1), m = 1u << (b & 31);
      if (atomicOr(&S.seen[b >> 5], m) & m) atomicOr(&S.twice[b >> 5], m);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GF_RPL; ++u) {
      const uint32_t b = f[u] & (GF_BITS - 1);
      if (in[u] && ((S.twice[b >> 5] >> (b & 31)) & 1u)) {
        const uint32_t p = atomicAdd(&S.nlist[par], 1u);
        if (p < (uint32_t)GB_LIST) {
          S.lid[p] = id[u];
          S.lf[p] = f[u];
        }
      }
    }
    __syncthreads();
    const uint32_t k = S.nlist[par];
    par ^= 1u;
    if (k == 0u) continue;  // every key alone
    if (k > (uint32_t)GB_LIST) {
      if (tid == 0) hard[atomicAdd(nhard, 1u)] = (uint32_t)w;
      continue;
    }
    // a listed record whose full fingerprint no other listed record shares is
    // alone (equal keys have equal fingerprints): only the others need their
    // exact keys.  Eight fingerprints per two broadcast reads (entries past k
    // are stale and skipped; the list holds GB_LIST, a multiple of eight).
    bool twin = false;
    if ((uint32_t)tid < k) {
      const uint32_t mf = S.lf[tid];
      uint32_t nf = 0u;
      for (uint32_t j0 = 0; j0 < k; j0 += 8) {
        const uint4 fa = *reinterpret_cast<const uint4*>(S.lf + j0);
        const uint4 fb = *reinterpret_cast<const uint4*>(S.lf + j0 + 4);
        const uint32_t fv[8] = {fa.x, fa.y, fa.z, fa.w, fb.x, fb.y, fb.z, fb.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) nf += (j0 + (uint32_t)e < k && fv[e] == mf) ? 1u : 0u;
      }
      twin = nf >= 2u;
      if (twin) S.lkey[tid] = load_key(a, t, S.lid[tid]);
    }
    __syncthreads();
    // (no barrier after this pass: the next bin writes the list only after
    // two barriers that every thread reaches once done here)
    if (twin) {
      const uint32_t me = S.lid[tid], mf = S.lf[tid];
      const uint4 mk = S.lkey[tid];
      uint32_t rank = 0u, cnt = 0u, head = me;
      // an exact key is read only on a fingerprint match (whose key is loaded)
      for (uint32_t j0 = 0; j0 < k; j0 += 8) {
        const uint4 fa = *reinterpret_cast<const uint4*>(S.lf + j0);
        const uint4 fb = *reinterpret_cast<const uint4*>(S.lf + j0 + 4);
        const uint32_t fv[8] = {fa.x, fa.y, fa.z, fa.w, fb.x, fb.y, fb.z, fb.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t j = j0 + (uint32_t)e;
          if (j < k && fv[e] == mf && key_eq(S.lkey[j], mk)) {
            const uint32_t ij = S.lid[j];
            ++cnt;
            rank += ij < me;
            head = min(head, ij);
          }
        }
      }
      if (cnt >= 2u) group_record(go, t, n, me, head, rank ? rank : cnt);
    }
  }
}

// The hard items: the general path (insertion into the slot table, ranks by
// ballots), persistent over the list k_group left.
__global__ __launch_bounds__(BZ_THREADS) void k_group_hard(BzArgs a, const uint32_t* bintot,
                                                           const uint32_t* binstart, const BzRec* recs,
                                                           uint16_t* sc_slot, GroupOut go,
                                                           const uint32_t* hard, const uint32_t* nhard,
                                                           int32_t* st) {
  __shared__ GroupLds G;
  const int nbins = 1 << a.nb;
  const int64_t n = a.n;
  const uint32_t cnt = *nhard;
  for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const uint32_t w = hard[i];
    const int t = (int)(w / (uint32_t)nbins);
    const uint32_t size = bintot[w], s0 = binstart[w];
    gb_large_bin(G, a, t, size, recs + (int64_t)t * n + s0, sc_slot + (int64_t)t * n + s0, go, st);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- scans and emission
// Each thread owns BZ_PER consecutive ids of a SC_CHUNK-id chunk; their flag
// bits sit in one flag word.
constexpr int BZ_PER = SC_CHUNK / BZ_THREADS;
static_assert(BZ_PER == 16, "16 ids per thread: one half flag word");

// The grouping records of ids i0 .. i0 + 15 that have one (flag bit set).
// All loads are issued before any is used.
GEEK_D void load_infos(const GroupOut& go, int t, int64_t n, int64_t i0, uint32_t fb, uint2* inf) {
#pragma unroll
  for (int u = 0; u < BZ_PER; ++u) {
    inf[u] = make_uint2(0u, 0u);
    if ((fb >> u) & 1u) inf[u] = go.info[(int64_t)t * n + i0 + u];
  }
}
// Bucket head / bucket length of id i (0 length for non-head members); ids
// past n (never flagged) count as nothing.
GEEK_D void id_bucket(int64_t n, int64_t i, bool flagged, const uint2& inf, uint32_t& is_head, uint32_t& len) {
  if (!flagged) {
    is_head = i < n ? 1u : 0u;
    len = is_head;
    return;
  }
  is_head = inf.x == (uint32_t)i;
  len = is_head ? inf.y : 0u;
}

// Flags of ids i0 .. i0 + 15 (i0 a multiple of 16) as bits.
GEEK_D uint32_t flag_bits16(const GroupOut& go, int t, int64_t i0) {
  const uint4 v = *reinterpret_cast<const uint4*>(go.flag8 + (int64_t)t * go.fstride + i0);
  auto nib = [](uint32_t w) { return (w & 1u) | ((w >> 7) & 2u) | ((w >> 14) & 4u) | ((w >> 21) & 8u); };
  return nib(v.x) | (nib(v.y) << 4) | (nib(v.z) << 8) | (nib(v.w) << 12);
}

__global__ __launch_bounds__(BZ_THREADS) void k_bz_reduce(int64_t n, int nch, GroupOut go, uint2* ctot) {
  __shared__ uint32_t sh[17];
  const int t = blockIdx.y, c = blockIdx.x;
  const int64_t i0 = (int64_t)c * SC_CHUNK + (int64_t)threadIdx.x * BZ_PER;
  uint32_t h = 0, l = 0;
  if (i0 < n) {
    const uint32_t fb = flag_bits16(go, t, i0);
    uint2 inf[BZ_PER];
    load_infos(go, t, n, i0, fb, inf);
#pragma unroll
    for (int u = 0; u < BZ_PER; ++u) {
      uint32_t ih, len;
      id_bucket(n, i0 + u, (fb >> u) & 1u, inf[u], ih, len);
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
// buckets of one are stored as contiguous runs.  The staging arrays skip one
// word in 17 (bz_pad), so the 16-word strides of the scan do not fall into
// one LDS bank.
GEEK_D int bz_pad(int x) { return x + (x >> 4); }
constexpr int SC_PADDED = SC_CHUNK + SC_CHUNK / 16;
__global__ __launch_bounds__(BZ_THREADS) void k_bz_apply(int64_t n, int nch, GroupOut go, const uint2* ctot,
                                                         uint2* hs, uint32_t* members, uint32_t* offsets,
                                                         uint32_t* bucket_of, const uint32_t* nbuckets) {
  __shared__ uint32_t sh[17];
  __shared__ uint32_t s_slot[SC_PADDED];  // member slot of the chunk's q-th head
  __shared__ uint32_t s_id[SC_PADDED];    // its id
  __shared__ uint32_t s_bof[SC_PADDED];   // bucket rank of each head id of the chunk, else ~0
  const int t = blockIdx.y, c = blockIdx.x;
  const int64_t c0 = (int64_t)c * SC_CHUNK;
  const int64_t i0 = c0 + (int64_t)threadIdx.x * BZ_PER;
  const int64_t tn = (int64_t)t * n;
  uint32_t fb = 0, lh = 0, ll = 0;
  uint32_t ihv[BZ_PER], lenv[BZ_PER];
  if (i0 < n) fb = flag_bits16(go, t, i0);
  {
    uint2 inf[BZ_PER];
    load_infos(go, t, n, i0, fb, inf);
#pragma unroll
    for (int u = 0; u < BZ_PER; ++u) {
      id_bucket(n, i0 + u, (fb >> u) & 1u, inf[u], ihv[u], lenv[u]);
      lh += ihv[u];
      ll += lenv[u];
    }
  }
  const uint2 base = ctot[(int64_t)t * nch + c];
  uint32_t nh;
  const uint32_t q0 = block_exscan(lh, &nh, sh);
  uint32_t bl = block_exscan(ll, nullptr, sh) + base.y;
  uint32_t q = q0;
#pragma unroll
  for (int u = 0; u < BZ_PER; ++u) {
    const int l = threadIdx.x * BZ_PER + u;
    if (bucket_of) s_bof[bz_pad(l)] = ihv[u] ? base.x + q : 0xFFFFFFFFu;
    if (!ihv[u]) continue;
    const uint32_t i = (uint32_t)(i0 + u);
    s_slot[bz_pad((int)q)] = bl;
    s_id[bz_pad((int)q)] = i;
    if ((fb >> u) & 1u) hs[tn + i] = make_uint2(bl, base.x + q);
    ++q;
    bl += lenv[u];
  }
  __syncthreads();
  uint32_t* off = offsets + (int64_t)t * (n + 1);
  for (uint32_t k = threadIdx.x; k < nh; k += BZ_THREADS) {
    const uint32_t sl = s_slot[bz_pad((int)k)];
    off[base.x + k] = sl;
    members[tn + sl] = s_id[bz_pad((int)k)];
  }
  if (bucket_of) {
    const int64_t cl = n - c0 < SC_CHUNK ? n - c0 : SC_CHUNK;
    for (int l = threadIdx.x; l < cl; l += BZ_THREADS)
      if (s_bof[bz_pad(l)] != 0xFFFFFFFFu) bucket_of[tn + c0 + l] = s_bof[bz_pad(l)];
  }
  if (c == 0 && threadIdx.x == 0) off[nbuckets[t]] = (uint32_t)n;
}

// The members of ids i0 .. i0 + 15 other than heads (fb: their flags).
GEEK_D void bz_members16(int64_t n, const GroupOut& go, const uint2* hs, uint32_t* members, uint32_t* bucket_of,
                         int t, int64_t i0, uint32_t fb) {
  const int64_t tn = (int64_t)t * n;
  uint2 inf[BZ_PER], h[BZ_PER];
  load_infos(go, t, n, i0, fb, inf);
  uint32_t mem = 0u;  // members other than the head
#pragma unroll
  for (int u = 0; u < BZ_PER; ++u) {
    h[u] = make_uint2(0u, 0u);
    if (((fb >> u) & 1u) && inf[u].x != (uint32_t)(i0 + u)) {
      mem |= 1u << u;
      h[u] = hs[tn + inf[u].x];
    }
  }
#pragma unroll
  for (int u = 0; u < BZ_PER; ++u) {
    if (!((mem >> u) & 1u)) continue;
    members[tn + h[u].x + inf[u].y] = (uint32_t)(i0 + u);
    if (bucket_of) bucket_of[tn + i0 + u] = h[u].y;
  }
}


// Members of buckets of two or more, other than the head; BZ_MEMCH chunks
// of ids per workgroup.
constexpr int BZ_MEMCH = 4;
__global__ __launch_bounds__(BZ_THREADS) void k_bz_members(int64_t n, GroupOut go, const uint2* hs,
                                                           uint32_t* members, uint32_t* bucket_of) {
  const int t = blockIdx.y;
  for (int j = 0; j < BZ_MEMCH; ++j) {
    const int64_t i0 = ((int64_t)blockIdx.x * BZ_MEMCH + j) * SC_CHUNK + (int64_t)threadIdx.x * BZ_PER;
    if (i0 >= n) return;
    const uint32_t fb = flag_bits16(go, t, i0);
    if (fb) bz_members16(n, go, hs, members, bucket_of, t, i0, fb);
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
  uint32_t *counts, *bintot, *binstart, *fp;
  BzRec *st, *alt;  // partitioned records: final bins, first-pass bins
  uint8_t* flag8;
  uint32_t* hard;
  uint32_t *counts2, *bintot1, *binstart1, *cbase, *cbin;  // second partition pass
  uint2 *info, *hs, *ctot;
};

static size_t carve_bz(const geek_bucketize_job& J, void* ws, BzWs& W) {
  Carver c(ws);
  const int nb = bin_bits(J.n);
  const int nbins = 1 << nb;
  const int nblk = ceil_div(J.n, PT_SUPER);
  const int nch = ceil_div(J.n, SC_CHUNK);
  const size_t Tn = (size_t)J.T * J.n;
  const int64_t fw = ceil_div(J.n, 16) * 16;
  const bool two = nb > PT_B1;
  const int nb1bins = 1 << (two ? PT_B1 : nb);
  W.counts = c.take<uint32_t>((size_t)J.T * nblk * nb1bins);
  const size_t maxchunks = two ? p2_max_chunks(J.n, J.T) : 0;
  W.counts2 = c.take<uint32_t>(two ? maxchunks * ((size_t)1 << (nb - PT_B1)) : 4);
  W.bintot1 = c.take<uint32_t>((size_t)J.T * nb1bins);
  W.binstart1 = c.take<uint32_t>((size_t)J.T * nb1bins);
  W.cbase = c.take<uint32_t>((size_t)J.T * nb1bins + 1);
  W.cbin = c.take<uint32_t>(two ? maxchunks : 1);
  W.bintot = c.take<uint32_t>((size_t)J.T * nbins);
  W.binstart = c.take<uint32_t>((size_t)J.T * nbins);
  W.fp = c.take<uint32_t>(Tn);
  W.st = c.take<BzRec>(Tn);
  W.alt = two ? c.take<BzRec>(Tn) : nullptr;
  W.flag8 = c.take<uint8_t>((size_t)J.T * fw + 16);  // + the hard-item counter, cleared with the flags
  W.hard = c.take<uint32_t>((size_t)J.T * nbins);
  W.info = c.take<uint2>(Tn);
  W.hs = c.take<uint2>(Tn);
  W.ctot = c.take<uint2>((size_t)J.T * nch);
  return c.used + 256;
}

size_t bucketize_ws(const geek_bucketize_job& J) {
  BzWs W;
  return carve_bz(J, nullptr, W);
}

__global__ void k_zero_u4(uint4* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

int32_t bucketize_run(const geek_bucketize_job& J, void* ws, size_t ws_bytes, int32_t* st,
                      hipStream_t s) {
  BzWs W;
  if (ws_bytes < carve_bz(J, ws, W)) return GEEK_ERR_WORKSPACE;
  const int nb = bin_bits(J.n);
  const int nbins = 1 << nb;
  const int nblk = ceil_div(J.n, PT_SUPER);
  const int nch = ceil_div(J.n, SC_CHUNK);
  const int64_t fw = ceil_div(J.n, 16) * 16;
  BzArgs a{J.keys, J.n, J.T, J.key_words, J.table_stride, J.row_stride, nb};
  GroupOut go{W.flag8, W.info, fw};
  prof_begin(GEEK_PROF_BUCKETIZE, s);
  // the fingerprints: the caller's (geek_hash wrote them with the keys) or
  // computed here into the workspace -- row by row first when every table's
  // key of an object lies in the object's row, else by the count pass
  const uint32_t* fps = J.key_fp ? J.key_fp : W.fp;
  const uint32_t* given = J.key_fp;
  if (!J.key_fp && J.T > 1 && J.table_stride * J.T <= J.row_stride) {
    hipLaunchKernelGGL(k_fp_rows, dim3(ceil_div(J.n * FR_LANES, BZ_THREADS)), dim3(BZ_THREADS), 0, s, a, W.fp);
    given = W.fp;
  }
  hipLaunchKernelGGL(k_zero_u4, dim3(ceil_div((int64_t)J.T * fw / 16 + 1, 256)), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(W.flag8), (int64_t)J.T * fw / 16 + 1);
  uint32_t* nhard = reinterpret_cast<uint32_t*>(W.flag8 + (size_t)J.T * fw);
  if (nb <= PT_B1) {
    hipLaunchKernelGGL(k_fp_count, dim3(nblk, J.T), dim3(BZ_THREADS), (size_t)nbins * 4, s, a, nblk, PT_SUPER,
                       W.counts, W.fp, given);
    hipLaunchKernelGGL(k_bin_colscan, dim3(ceil_div((int64_t)J.T * nbins, 256)), dim3(256), 0, s, J.T,
                       nblk, nbins, W.counts, W.bintot);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, nbins, W.bintot, W.binstart);
    hipLaunchKernelGGL(k_p1_scatter, dim3(nblk, J.T), dim3(BZ_THREADS), 0, s, a, nb, nblk, W.counts, W.binstart,
                       fps, W.st);
  } else {
    // first pass into the alternate buffers by the top PT_B1 bits, second
    // pass by the next nb - PT_B1 bits into the staging buffers
    BzArgs a1 = a;
    a1.nb = PT_B1;
    const int nb1bins = J.T << PT_B1;
    const int F = 1 << (nb - PT_B1);
    const int maxchunks = (int)p2_max_chunks(J.n, J.T);
    hipLaunchKernelGGL(k_fp_count, dim3(nblk, J.T), dim3(BZ_THREADS), (size_t)4 << PT_B1, s, a1, nblk, PT_SUPER,
                       W.counts, W.fp, given);
    hipLaunchKernelGGL(k_bin_colscan, dim3(ceil_div(nb1bins, 256)), dim3(256), 0, s, J.T, nblk, 1 << PT_B1,
                       W.counts, W.bintot1);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, 1 << PT_B1, W.bintot1, W.binstart1);
    hipLaunchKernelGGL(k_p1_scatter, dim3(nblk, J.T), dim3(BZ_THREADS), 0, s, a1, PT_B1, nblk, W.counts,
                       W.binstart1, fps, W.alt);
    hipLaunchKernelGGL(k_p2_chunks, dim3(1), dim3(1024), 0, s, nb1bins, W.bintot1, W.cbase, W.cbin);
    hipLaunchKernelGGL(k_p2_count, dim3(maxchunks), dim3(BZ_THREADS), 0, s, J.n, nb, W.cbase, W.cbin, nb1bins,
                       W.bintot1,
                       W.binstart1, W.alt, W.counts2);
    hipLaunchKernelGGL(k_p2_colscan, dim3(ceil_div((int64_t)nb1bins * F, 256)), dim3(256), 0, s, nb1bins, F,
                       W.cbase, W.counts2, W.bintot);
    hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, nbins, W.bintot, W.binstart);
    hipLaunchKernelGGL(k_p2_scatter, dim3(maxchunks), dim3(BZ_THREADS), 0, s, J.n, nb, W.cbase, W.cbin, nb1bins,
                       W.bintot1, W.binstart1, W.alt, W.counts2, W.binstart, W.st);
  }
  prof_begin(GEEK_PROF_BZ_SORT, s);
  {
    const int64_t items = (int64_t)J.T * nbins;
    const int grid = (int)(items < 1792 ? items : 1792);  // persistent: 7 per CU are resident
    hipLaunchKernelGGL(k_group, dim3(grid), dim3(BZ_THREADS), 0, s, a, W.bintot, W.binstart, W.st, go,
                       W.hard, nhard);
    // the fingerprints are dead after the first scatter: their space keeps
    // the general path's slots
    hipLaunchKernelGGL(k_group_hard, dim3(grid < 768 ? grid : 768), dim3(BZ_THREADS), 0, s, a, W.bintot,
                       W.binstart, W.st, reinterpret_cast<uint16_t*>(W.fp), go, W.hard, nhard, st);
  }
  prof_end(GEEK_PROF_BZ_SORT, s);
  hipLaunchKernelGGL(k_bz_reduce, dim3(nch, J.T), dim3(BZ_THREADS), 0, s, J.n, nch, go, W.ctot);
  hipLaunchKernelGGL(k_scan_chunks, dim3(J.T), dim3(1024), 0, s, nch, W.ctot, J.nbuckets);
  hipLaunchKernelGGL(k_bz_apply, dim3(nch, J.T), dim3(BZ_THREADS), 0, s, J.n, nch, go, W.ctot, W.hs,
                     J.members, J.offsets, J.bucket_of, J.nbuckets);
  hipLaunchKernelGGL(k_bz_members, dim3(ceil_div(nch, BZ_MEMCH), J.T), dim3(BZ_THREADS), 0, s, J.n, go, W.hs,
                     J.members,
                     J.bucket_of);
  prof_end(GEEK_PROF_BUCKETIZE, s);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
