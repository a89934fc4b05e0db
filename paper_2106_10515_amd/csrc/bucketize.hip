// Buckets of every table (paper Algorithms 2 and 3: T[G(x_j)].push(j)) on
// gfx950: group the objects whose table keys are identical.
//
//  1. k_bin_count / k_bin_scan / k_bin_scatter: a one-pass MSD partition of
//     (key, id) records into 2^nb bins per table, the bin being the top bits
//     of a 32-bit mix of the exact key (equal keys always share a bin).
//  2. k_bin_sort: one workgroup per bin sorts its records by (key, id) in
//     LDS (bitonic), finds runs of equal keys and records, for every run, its
//     smallest id (the run head: ids ascend within a run), length and start.
//     Bins too large for LDS are sorted by k_big_sort (workgroup LSD radix
//     sort in global memory) and scanned by k_big_runs.
//  3. k_scan_*: a segmented scan over ids of (is-head, run length) gives each
//     bucket its rank in "smallest member" order and its CSR offset.
//  4. k_emit: every record is copied to its canonical CSR slot and bucket_of.
#include "common.hpp"

namespace geek {

constexpr int BZ_THREADS = 256;
constexpr int BZ_CHUNK = 32768;   // records per block in count / scatter
constexpr int BZ_CAP = 2048;      // largest bin sorted in LDS
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
__global__ __launch_bounds__(BZ_THREADS) void k_bin_count(BzArgs a, int nblk, uint32_t* counts) {
  extern __shared__ uint32_t hist[];
  const int t = blockIdx.y, blk = blockIdx.x;
  const int nbins = 1 << a.nb;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS) hist[b] = 0;
  __syncthreads();
  const int64_t s = (int64_t)blk * BZ_CHUNK;
  const int64_t e = s + BZ_CHUNK < a.n ? s + BZ_CHUNK : a.n;
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
  for (int k = 0; k < nblk; ++k) {
    uint32_t* c = counts + ((int64_t)t * nblk + k) * nbins + b;
    const uint32_t v = *c;
    *c = run;
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

__global__ __launch_bounds__(BZ_THREADS) void k_bin_scatter(BzArgs a, int nblk, const uint32_t* counts,
                                                            const uint32_t* binstart, uint4* st_keys,
                                                            uint32_t* st_ids) {
  extern __shared__ uint32_t cur[];
  const int t = blockIdx.y, blk = blockIdx.x;
  const int nbins = 1 << a.nb;
  const uint32_t* c = counts + ((int64_t)t * nblk + blk) * nbins;
  const uint32_t* bs = binstart + (int64_t)t * nbins;
  for (int b = threadIdx.x; b < nbins; b += BZ_THREADS) cur[b] = bs[b] + c[b];
  __syncthreads();
  const int64_t s = (int64_t)blk * BZ_CHUNK;
  const int64_t e = s + BZ_CHUNK < a.n ? s + BZ_CHUNK : a.n;
  uint4* sk = st_keys + (int64_t)t * a.n;
  uint32_t* si = st_ids + (int64_t)t * a.n;
  for (int64_t i = s + threadIdx.x; i < e; i += BZ_THREADS) {
    const uint4 k = load_key(a, t, i);
    const uint32_t pos = atomicAdd(&cur[bin_of(k, a.nb)], 1u);
    sk[pos] = k;
    si[pos] = (uint32_t)i;
  }
}

// ---------------------------------------------------------------- per-bin sort
struct RunOut {
  uint32_t* st_ids;    // [T][n] sorted ids (written back)
  uint32_t* rec_head;  // [T][n] per record: first id of its run
  uint32_t* run_len;   // [T][n] per id: run length if the id heads a run, else 0
  uint32_t* run_pos;   // [T][n] per head id: start of its run in the staging order
};

__global__ __launch_bounds__(BZ_THREADS) void k_bin_sort(int64_t n, int nb, const uint32_t* bintot,
                                                         const uint32_t* binstart, const uint4* st_keys,
                                                         RunOut ro, uint32_t* big_list,
                                                         uint32_t* big_count) {
  __shared__ uint4 sk[BZ_CAP];
  __shared__ uint32_t sid[BZ_CAP];
  __shared__ int sst[BZ_CAP];
  const int t = blockIdx.y, bin = blockIdx.x;
  const int nbins = 1 << nb;
  const uint32_t size = bintot[(int64_t)t * nbins + bin];
  if (size == 0) return;
  const uint32_t s0 = binstart[(int64_t)t * nbins + bin];
  if (size > BZ_CAP) {
    if (threadIdx.x == 0) big_list[atomicAdd(big_count, 1u)] = (uint32_t)(t * nbins + bin);
    return;
  }
  int P2 = 1;
  while (P2 < (int)size) P2 <<= 1;
  const uint4* gk = st_keys + (int64_t)t * n + s0;
  const uint32_t* gi = ro.st_ids + (int64_t)t * n + s0;
  for (int q = threadIdx.x; q < P2; q += BZ_THREADS) {
    if (q < (int)size) {
      sk[q] = gk[q];
      sid[q] = gi[q];
    } else {
      sk[q] = make_uint4(~0u, ~0u, ~0u, ~0u);
      sid[q] = ~0u;
    }
  }
  __syncthreads();
  // bitonic sort by (key, id)
  for (int kk = 2; kk <= P2; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int q = threadIdx.x; q < P2; q += BZ_THREADS) {
        const int o = q ^ jj;
        if (o > q) {
          const bool up = (q & kk) == 0;
          const uint4 ka = sk[q], kb = sk[o];
          const uint32_t ia = sid[q], ib = sid[o];
          const bool sw = up ? rec_less(kb, ib, ka, ia) : rec_less(ka, ia, kb, ib);
          if (sw) {
            sk[q] = kb;
            sk[o] = ka;
            sid[q] = ib;
            sid[o] = ia;
          }
        }
      }
      __syncthreads();
    }
  }
  // run starts: inclusive max-scan of (head ? q : -1)
  for (int q = threadIdx.x; q < (int)size; q += BZ_THREADS)
    sst[q] = (q == 0 || !key_eq(sk[q], sk[q - 1])) ? q : -1;
  __syncthreads();
  for (int o = 1; o < (int)size; o <<= 1) {
    int tmp[BZ_CAP / BZ_THREADS];
#pragma unroll
    for (int u = 0; u < BZ_CAP / BZ_THREADS; ++u) {
      const int q = threadIdx.x + u * BZ_THREADS;
      tmp[u] = (q < (int)size && q >= o) ? max(sst[q], sst[q - o]) : (q < (int)size ? sst[q] : 0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BZ_CAP / BZ_THREADS; ++u) {
      const int q = threadIdx.x + u * BZ_THREADS;
      if (q < (int)size) sst[q] = tmp[u];
    }
    __syncthreads();
  }
  uint32_t* oi = ro.st_ids + (int64_t)t * n + s0;
  uint32_t* oh = ro.rec_head + (int64_t)t * n + s0;
  uint32_t* rl = ro.run_len + (int64_t)t * n;
  uint32_t* rp = ro.run_pos + (int64_t)t * n;
  for (int q = threadIdx.x; q < (int)size; q += BZ_THREADS) {
    const int rs = sst[q];
    const uint32_t f = sid[rs];
    const uint32_t id = sid[q];
    oi[q] = id;
    oh[q] = f;
    const bool last = (q == (int)size - 1) || (sst[q + 1] == q + 1);
    if (last) {
      rl[f] = (uint32_t)(q - rs + 1);
      rp[f] = s0 + (uint32_t)rs;
    }
    if (q != rs) rl[id] = 0u;
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

// Run detection of a sorted oversize bin (one workgroup per bin).
__global__ __launch_bounds__(BIG_THREADS) void k_big_runs(int64_t n, int nb, const uint32_t* bintot,
                                                          const uint32_t* binstart, const uint4* st_keys,
                                                          RunOut ro, const uint32_t* big_list,
                                                          const uint32_t* big_count) {
  __shared__ int ss[BIG_THREADS];
  __shared__ int carry;
  const int nbins = 1 << nb;
  const uint32_t nbig = *big_count;
  for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const uint32_t tb = big_list[bi];
    const int t = (int)(tb / nbins);
    const uint32_t size = bintot[tb], s0 = binstart[tb];
    const uint4* k = st_keys + (int64_t)t * n + s0;
    const uint32_t* ids = ro.st_ids + (int64_t)t * n + s0;
    uint32_t* oh = ro.rec_head + (int64_t)t * n + s0;
    uint32_t* rl = ro.run_len + (int64_t)t * n;
    uint32_t* rp = ro.run_pos + (int64_t)t * n;
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
        const uint32_t id = ids[q];
        oh[q] = f;
        const bool last = (q == size - 1) || !key_eq(k[q + 1], k[q]);
        if (last) {
          rl[f] = q - (uint32_t)rs + 1u;
          rp[f] = s0 + (uint32_t)rs;
        }
        if ((int)q != rs) rl[id] = 0u;
      }
      __syncthreads();
      if (threadIdx.x == BIG_THREADS - 1) carry = rs;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- scans
// Segmented (per table) scan over ids of (heads, run lengths).
__global__ __launch_bounds__(BZ_THREADS) void k_scan_reduce(int64_t n, int nch, const uint32_t* run_len,
                                                            uint2* ctot) {
  __shared__ uint32_t sh[17];
  const int t = blockIdx.y, c = blockIdx.x;
  const int64_t s = (int64_t)c * SC_CHUNK;
  const uint32_t* rl = run_len + (int64_t)t * n;
  uint32_t h = 0, l = 0;
  for (int64_t i = s + threadIdx.x; i < s + SC_CHUNK && i < n; i += BZ_THREADS) {
    const uint32_t v = rl[i];
    h += v != 0;
    l += v;
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

__global__ __launch_bounds__(BZ_THREADS) void k_scan_apply(int64_t n, int nch, const uint2* ctot,
                                                           uint32_t* run_len /* -> rank */,
                                                           uint32_t* hoff, uint32_t* offsets,
                                                           const uint32_t* nbuckets) {
  __shared__ uint32_t sh[17];
  const int t = blockIdx.y, c = blockIdx.x;
  const int64_t s = (int64_t)c * SC_CHUNK;
  constexpr int PER = SC_CHUNK / BZ_THREADS;
  uint32_t* rl = run_len + (int64_t)t * n;
  uint32_t* ho = hoff + (int64_t)t * n;
  uint32_t* off = offsets + (int64_t)t * (n + 1);
  uint32_t v[PER];
  uint32_t lh = 0, ll = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t i = s + threadIdx.x * PER + u;
    v[u] = i < n ? rl[i] : 0u;
    lh += v[u] != 0;
    ll += v[u];
  }
  uint32_t bh = block_exscan(lh, nullptr, sh) + ctot[(int64_t)t * nch + c].x;
  uint32_t bl = block_exscan(ll, nullptr, sh) + ctot[(int64_t)t * nch + c].y;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t i = s + threadIdx.x * PER + u;
    if (i < n && v[u]) {
      rl[i] = bh;   // bucket rank of head i
      ho[i] = bl;   // CSR offset of that bucket
      off[bh] = bl;
      ++bh;
      bl += v[u];
    }
  }
  if (c == 0 && threadIdx.x == 0) off[nbuckets[t]] = (uint32_t)n;
}

__global__ void k_emit(int64_t n, int T, const uint32_t* st_ids, const uint32_t* rec_head,
                       const uint32_t* rank, const uint32_t* hoff, const uint32_t* run_pos,
                       uint32_t* members, uint32_t* bucket_of) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)T * n) return;
  const int t = (int)(g / n);
  const int64_t s = g - (int64_t)t * n;
  const int64_t tb = (int64_t)t * n;
  const uint32_t id = st_ids[g];
  const uint32_t f = rec_head[g];
  const uint32_t pos0 = run_pos[tb + f];
  members[tb + hoff[tb + f] + (uint32_t)(s - pos0)] = id;
  if (bucket_of) bucket_of[tb + id] = rank[tb + f];
}

// ---------------------------------------------------------------- host side
static int bin_bits(int64_t n) {
  int nb = 0;
  while (nb < BZ_MAXBITS && (n >> nb) > 1536) ++nb;
  return nb;
}

struct BzWs {
  uint32_t *counts, *bintot, *binstart, *st_ids, *rec_head, *run_len, *run_pos, *hoff, *alt_ids;
  uint4 *st_keys, *alt_keys;
  uint2* ctot;
  uint32_t *big_list, *big_count;
};

static size_t carve_bz(const geek_bucketize_job& J, void* ws, BzWs& W) {
  Carver c(ws);
  const int nb = bin_bits(J.n);
  const int nbins = 1 << nb;
  const int nblk = ceil_div(J.n, BZ_CHUNK);
  const int nch = ceil_div(J.n, SC_CHUNK);
  const size_t Tn = (size_t)J.T * J.n;
  W.counts = c.take<uint32_t>((size_t)J.T * nblk * nbins);
  W.bintot = c.take<uint32_t>((size_t)J.T * nbins);
  W.binstart = c.take<uint32_t>((size_t)J.T * nbins);
  W.st_keys = c.take<uint4>(Tn);
  W.alt_keys = c.take<uint4>(Tn);
  W.st_ids = c.take<uint32_t>(Tn);
  W.alt_ids = c.take<uint32_t>(Tn);
  W.rec_head = c.take<uint32_t>(Tn);
  W.run_len = c.take<uint32_t>(Tn);
  W.run_pos = c.take<uint32_t>(Tn);
  W.hoff = c.take<uint32_t>(Tn);
  W.ctot = c.take<uint2>((size_t)J.T * nch);
  W.big_list = c.take<uint32_t>((size_t)J.T * nbins);
  W.big_count = c.take<uint32_t>(4);
  return c.used + 256;
}

size_t bucketize_ws(const geek_bucketize_job& J) {
  BzWs W;
  return carve_bz(J, nullptr, W);
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

int32_t bucketize_run(const geek_bucketize_job& J, void* ws, size_t ws_bytes, int32_t* st,
                      hipStream_t s) {
  (void)st;
  BzWs W;
  if (ws_bytes < carve_bz(J, ws, W)) return GEEK_ERR_WORKSPACE;
  const int nb = bin_bits(J.n);
  const int nbins = 1 << nb;
  const int nblk = ceil_div(J.n, BZ_CHUNK);
  const int nch = ceil_div(J.n, SC_CHUNK);
  BzArgs a{J.keys, J.n, J.T, J.key_words, J.table_stride, J.row_stride, nb};
  const size_t hbytes = (size_t)nbins * 4;
  prof_begin(GEEK_PROF_BUCKETIZE, s);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, W.big_count, 4);
  hipLaunchKernelGGL(k_bin_count, dim3(nblk, J.T), dim3(BZ_THREADS), hbytes, s, a, nblk, W.counts);
  hipLaunchKernelGGL(k_bin_colscan, dim3(ceil_div((int64_t)J.T * nbins, 256)), dim3(256), 0, s, J.T,
                     nblk, nbins, W.counts, W.bintot);
  hipLaunchKernelGGL(k_bin_rowscan, dim3(J.T), dim3(1024), 0, s, nbins, W.bintot, W.binstart);
  hipLaunchKernelGGL(k_bin_scatter, dim3(nblk, J.T), dim3(BZ_THREADS), hbytes, s, a, nblk, W.counts,
                     W.binstart, W.st_keys, W.st_ids);
  RunOut ro{W.st_ids, W.rec_head, W.run_len, W.run_pos};
  prof_begin(GEEK_PROF_BZ_SORT, s);
  hipLaunchKernelGGL(k_bin_sort, dim3(nbins, J.T), dim3(BZ_THREADS), 0, s, J.n, nb, W.bintot,
                     W.binstart, W.st_keys, ro, W.big_list, W.big_count);
  prof_end(GEEK_PROF_BZ_SORT, s);
  hipLaunchKernelGGL(k_big_sort, dim3(256), dim3(BIG_THREADS), 0, s, J.n, nb, J.key_words, W.bintot,
                     W.binstart, W.st_keys, W.st_ids, W.alt_keys, W.alt_ids, W.big_list, W.big_count);
  hipLaunchKernelGGL(k_big_runs, dim3(256), dim3(BIG_THREADS), 0, s, J.n, nb, W.bintot, W.binstart,
                     W.st_keys, ro, W.big_list, W.big_count);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nch, J.T), dim3(BZ_THREADS), 0, s, J.n, nch, W.run_len, W.ctot);
  hipLaunchKernelGGL(k_scan_chunks, dim3(J.T), dim3(1024), 0, s, nch, W.ctot, J.nbuckets);
  hipLaunchKernelGGL(k_scan_apply, dim3(nch, J.T), dim3(BZ_THREADS), 0, s, J.n, nch, W.ctot, W.run_len,
                     W.hoff, J.offsets, J.nbuckets);
  hipLaunchKernelGGL(k_emit, dim3(ceil_div((int64_t)J.T * J.n, 256)), dim3(256), 0, s, J.n, J.T,
                     W.st_ids, W.rec_head, W.run_len, W.hoff, W.run_pos, J.members, J.bucket_of);
  prof_end(GEEK_PROF_BUCKETIZE, s);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
