// SILK seeding (paper Section 3.2, Algorithm 4) on gfx950.
//
// For each SILK table s:
//   k_sig / k_sig_big   G(B) = (min_{x in B} pi_k(x))_k for every bucket
//   bucketize_run       bins = buckets with identical G
//   k_pair_count        pairs (bin, id) of the buckets of bins with >= 2 buckets
//   radix_sort          sort the pairs by (bin, id)
//   k_runs / k_keep     count each (bin, id); keep it when 2*count > |Bin|
//   k_seg_*             C_shared per bin; append it to C when |C_shared| >= delta
// De-duplication: the same steps once more over the sets of C (one table,
// key rows L*K..), a bin holding a single set passes it through; bins are
// then ordered by their K-tuple (radix sort) and emitted as the seeds.
//
// The sizes of the intermediate collections are only known on the device,
// so the host reads them back between steps (the call synchronizes).
#include <vector>

#include "common.hpp"
#include "radix.hpp"

namespace geek {

size_t bucketize_ws(const geek_bucketize_job& J);
int32_t bucketize_run(const geek_bucketize_job& J, void* ws, size_t ws_bytes, int32_t* st,
                      hipStream_t s);

constexpr int SK_BIG = 64;  // buckets larger than this are hashed by a block

__global__ void k_tab_base(const uint32_t* nb, int T, uint32_t* base) {
  if (blockIdx.x || threadIdx.x) return;
  uint32_t r = 0;
  for (int t = 0; t < T; ++t) {
    base[t] = r;
    r += nb[t];
  }
  base[T] = r;
}

// Global extent of every bucket of every table: start position in the
// flattened member array and size.
__global__ void k_extent(const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ base, int T,
                         int64_t n, int64_t NB, uint32_t* __restrict__ gstart,
                         uint32_t* __restrict__ gsize) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= NB) return;
  int lo = 0, hi = T;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= (uint32_t)g) lo = mid; else hi = mid;
  }
  const uint32_t j = (uint32_t)g - base[lo];
  const uint32_t o = offsets[(int64_t)lo * (n + 1) + j], e = offsets[(int64_t)lo * (n + 1) + j + 1];
  gstart[g] = (uint32_t)((int64_t)lo * n + o);
  gsize[g] = e - o;
}

__global__ void k_set_extent(const uint32_t* __restrict__ off, int64_t ns, uint32_t* __restrict__ gstart,
                             uint32_t* __restrict__ gsize) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= ns) return;
  gstart[g] = off[g];
  gsize[g] = off[g + 1] - off[g];
}

// Signature of every set (thread per set); large sets go to k_sig_big.
__global__ void k_sig(const uint32_t* __restrict__ mem, const uint32_t* __restrict__ gstart,
                      const uint32_t* __restrict__ gsize, int64_t ns, const uint32_t* __restrict__ keys,
                      int K, uint32_t* __restrict__ G, uint32_t* big_list, uint32_t* big_count) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= ns) return;
  const uint32_t sz = gsize[g];
  if (sz > SK_BIG) {
    big_list[atomicAdd(big_count, 1u)] = (uint32_t)g;
    return;
  }
  uint32_t a[4], b[4], mn[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = k < K ? (keys[2 * k] | 1u) : 1u;
    b[k] = k < K ? keys[2 * k + 1] : 0u;
    mn[k] = 0xFFFFFFFFu;
  }
  const uint32_t* p = mem + gstart[g];
  for (uint32_t q = 0; q < sz; ++q) {
    const uint32_t y = fmix32(p[q]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t v = perm_premixed(a[k], b[k], y);
      mn[k] = v < mn[k] ? v : mn[k];
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < K) G[g * K + k] = mn[k];
}

__global__ __launch_bounds__(256) void k_sig_big(const uint32_t* __restrict__ mem,
                                                 const uint32_t* __restrict__ gstart,
                                                 const uint32_t* __restrict__ gsize,
                                                 const uint32_t* __restrict__ keys, int K,
                                                 uint32_t* __restrict__ G, const uint32_t* big_list,
                                                 const uint32_t* big_count) {
  __shared__ uint32_t red[4][256];
  const uint32_t nbig = *big_count;
  for (uint32_t bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const uint32_t g = big_list[bi];
    uint32_t a[4], b[4], mn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = k < K ? (keys[2 * k] | 1u) : 1u;
      b[k] = k < K ? keys[2 * k + 1] : 0u;
      mn[k] = 0xFFFFFFFFu;
    }
    const uint32_t* p = mem + gstart[g];
    const uint32_t sz = gsize[g];
    for (uint32_t q = threadIdx.x; q < sz; q += blockDim.x) {
      const uint32_t y = fmix32(p[q]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t v = perm_premixed(a[k], b[k], y);
        mn[k] = v < mn[k] ? v : mn[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = mn[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const uint32_t v = red[k][threadIdx.x + o];
          if (v < red[k][threadIdx.x]) red[k][threadIdx.x] = v;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x < (unsigned)K) G[(int64_t)g * K + threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
  }
}

// For each set: members to vote with when its bin holds >= 2 sets.
__global__ void k_pair_count(const uint32_t* __restrict__ bin_of, const uint32_t* __restrict__ binoff,
                             const uint32_t* __restrict__ binmem, const uint32_t* __restrict__ gsize, int64_t ns,
                             uint32_t* __restrict__ cnt, uint32_t* multi_bins) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= ns) return;
  const uint32_t b = bin_of[g];
  const uint32_t bs = binoff[b + 1] - binoff[b];
  cnt[g] = bs >= 2 ? gsize[g] : 0u;
  if (bs >= 2 && binmem[binoff[b]] == (uint32_t)g) atomicAdd(multi_bins, 1u);
}

__global__ void k_fill0(uint32_t* p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ void k_mark_starts(const uint32_t* __restrict__ gstart, int64_t ns, uint32_t base0,
                              uint32_t* __restrict__ flag) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= ns) return;
  flag[gstart[g] - base0] = 1u;
}

// One thread per member position q of the flattened sets: set index of q is
// (exclusive count of set starts) + flag - 1.
__global__ void k_pairs(const uint32_t* __restrict__ mem, int64_t npos, uint32_t base0,
                        const uint32_t* __restrict__ flag, const uint32_t* __restrict__ fscan,
                        const uint32_t* __restrict__ gstart, const uint32_t* __restrict__ cnt,
                        const uint32_t* __restrict__ poff, const uint32_t* __restrict__ bin_of,
                        uint32_t* __restrict__ hi, uint32_t* __restrict__ lo) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= npos) return;
  const uint32_t g = fscan[q] + flag[q] - 1u;
  if (cnt[g] == 0u) return;
  const uint32_t p = poff[g] + ((uint32_t)q + base0 - gstart[g]);
  hi[p] = bin_of[g];
  lo[p] = mem[q];
}

__global__ void k_run_heads(const uint32_t* __restrict__ hi, const uint32_t* __restrict__ lo, int64_t P,
                            uint32_t* __restrict__ h) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= P) return;
  h[q] = (q == 0 || hi[q] != hi[q - 1] || lo[q] != lo[q - 1]) ? 1u : 0u;
}

__global__ void k_seg_heads(const uint32_t* __restrict__ hi, int64_t P, uint32_t* __restrict__ h) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= P) return;
  h[q] = (q == 0 || hi[q] != hi[q - 1]) ? 1u : 0u;
}

__global__ void k_starts(const uint32_t* __restrict__ h, const uint32_t* __restrict__ hs, int64_t P,
                         uint32_t* __restrict__ start) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q > P) return;
  if (q == P) {
    start[hs[P]] = (uint32_t)P;  // hs[P] = total heads
    return;
  }
  if (h[q]) start[hs[q]] = (uint32_t)q;
}

// Majority vote of every (bin, id) run: keep iff 2 * count > |Bin|.
__global__ void k_keep(const uint32_t* __restrict__ rstart, int64_t R, const uint32_t* __restrict__ hi,
                       const uint32_t* __restrict__ binoff, uint32_t* __restrict__ kept) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= R) return;
  const uint32_t len = rstart[r + 1] - rstart[r];
  const uint32_t b = hi[rstart[r]];
  const uint32_t bs = binoff[b + 1] - binoff[b];
  kept[r] = (2u * len > bs) ? 1u : 0u;
}

__global__ void k_compact_runs(const uint32_t* __restrict__ rstart, int64_t R, const uint32_t* __restrict__ kept,
                               const uint32_t* __restrict__ kidx, const uint32_t* __restrict__ hi,
                               const uint32_t* __restrict__ lo, uint32_t* __restrict__ khi,
                               uint32_t* __restrict__ klo) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= R || !kept[r]) return;
  khi[kidx[r]] = hi[rstart[r]];
  klo[kidx[r]] = lo[rstart[r]];
}

// Segment (one bin's kept ids) sizes passing the threshold.
__global__ void k_seg_emit_size(const uint32_t* __restrict__ sstart, int64_t S, int delta,
                                uint32_t* __restrict__ esize, uint32_t* __restrict__ eone) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t len = sstart[s + 1] - sstart[s];
  const bool ok = (int64_t)len >= (int64_t)delta;
  esize[s] = ok ? len : 0u;
  eone[s] = ok ? 1u : 0u;
}

__global__ void k_seg_emit(const uint32_t* __restrict__ sstart, int64_t S, const uint32_t* __restrict__ esize,
                           const uint32_t* __restrict__ eoff, const uint32_t* __restrict__ eidx,
                           const uint32_t* __restrict__ klo, uint32_t m0, uint32_t s0,
                           uint32_t* __restrict__ cmem, uint32_t* __restrict__ coff) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= S || esize[s] == 0u) return;
  coff[s0 + eidx[s]] = m0 + eoff[s];  // the members are copied by k_seg_copy
}

// The last index r in [0, cnt) with off[r] <= e (off non-decreasing): the
// non-empty entry whose output range holds position e.
GEEK_D int64_t range_of(const uint32_t* __restrict__ off, int64_t cnt, uint32_t e) {
  int64_t lo = 0, hi = cnt - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One thread per emitted member: C's members of this table, segment by
// segment (a segment can hold a large share of the table, so the copy is
// spread over threads rather than done by one thread per segment).
__global__ void k_seg_copy(const uint32_t* __restrict__ sstart, int64_t S, const uint32_t* __restrict__ eoff,
                           const uint32_t* __restrict__ klo, uint32_t m0, uint32_t em, uint32_t* __restrict__ cmem) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= em) return;
  const int64_t s = range_of(eoff, S, (uint32_t)e);
  cmem[m0 + e] = klo[sstart[s] + ((uint32_t)e - eoff[s])];
}

__global__ void k_put(uint32_t* p, int64_t i, uint32_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) p[i] = v;
}

// ---- de-duplication output --------------------------------------------------
// Seed size of every de-duplication bin: a single set passes through; a bin of
// several sets keeps its voted C_shared when it meets the threshold.
__global__ void k_dedup_size(const uint32_t* __restrict__ binoff, const uint32_t* __restrict__ binmem,
                             int64_t nbins, const uint32_t* __restrict__ gsize,
                             uint32_t* __restrict__ ssize, uint32_t* __restrict__ src_kind) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const uint32_t bs = binoff[b + 1] - binoff[b];
  if (bs == 1) {
    ssize[b] = gsize[binmem[binoff[b]]];
    src_kind[b] = 1u;
  } else {
    ssize[b] = 0u;
    src_kind[b] = 0u;
  }
}

__global__ void k_dedup_multi(const uint32_t* __restrict__ sstart, int64_t S, const uint32_t* __restrict__ khi,
                              int delta, uint32_t* __restrict__ ssize, uint32_t* __restrict__ segof) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t len = sstart[s + 1] - sstart[s];
  const uint32_t b = khi[sstart[s]];
  if ((int64_t)len >= (int64_t)delta) ssize[b] = len;
  segof[b] = (uint32_t)s;
}

// Tuple key words of every bin (the G of its first set), value = bin id.
__global__ void k_bin_tuples(const uint32_t* __restrict__ binoff, const uint32_t* __restrict__ binmem,
                             int64_t nbins, const uint32_t* __restrict__ G, int K,
                             uint32_t* __restrict__ w0, uint32_t* __restrict__ w1, uint32_t* __restrict__ w2,
                             uint32_t* __restrict__ w3, uint32_t* __restrict__ val) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const uint32_t g = binmem[binoff[b]];
  w0[b] = G[(int64_t)g * K];
  w1[b] = K > 1 ? G[(int64_t)g * K + 1] : 0u;
  w2[b] = K > 2 ? G[(int64_t)g * K + 2] : 0u;
  w3[b] = K > 3 ? G[(int64_t)g * K + 3] : 0u;
  val[b] = (uint32_t)b;
}

__global__ void k_order_sizes(const uint32_t* __restrict__ ord, int64_t nbins, const uint32_t* __restrict__ ssize,
                              uint32_t* __restrict__ osz, uint32_t* __restrict__ oone) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= nbins) return;
  const uint32_t v = ssize[ord[r]];
  osz[r] = v;
  oone[r] = v ? 1u : 0u;
}

__global__ void k_emit_seeds(const uint32_t* __restrict__ ord, int64_t nbins, const uint32_t* __restrict__ osz,
                             const uint32_t* __restrict__ ooff, const uint32_t* __restrict__ oidx,
                             const uint32_t* __restrict__ src_kind, const uint32_t* __restrict__ binoff,
                             const uint32_t* __restrict__ binmem, const uint32_t* __restrict__ cmem,
                             const uint32_t* __restrict__ coff, const uint32_t* __restrict__ segof,
                             const uint32_t* __restrict__ sstart, const uint32_t* __restrict__ klo,
                             uint32_t* __restrict__ seed_off, uint32_t* __restrict__ seed_mem) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= nbins || osz[r] == 0u) return;
  seed_off[oidx[r]] = ooff[r];  // the members are copied by k_seed_copy
}

// One thread per seed member: from the set that passes through (C) or from
// the voted ids of the bin.
__global__ void k_seed_copy(const uint32_t* __restrict__ ord, int64_t nbins, const uint32_t* __restrict__ ooff,
                            const uint32_t* __restrict__ src_kind, const uint32_t* __restrict__ binoff,
                            const uint32_t* __restrict__ binmem, const uint32_t* __restrict__ cmem,
                            const uint32_t* __restrict__ coff, const uint32_t* __restrict__ segof,
                            const uint32_t* __restrict__ sstart, const uint32_t* __restrict__ klo, uint32_t tot,
                            uint32_t* __restrict__ seed_mem) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= tot) return;
  const int64_t r = range_of(ooff, nbins, (uint32_t)e);
  const uint32_t b = ord[r];
  const uint32_t q = (uint32_t)e - ooff[r];
  seed_mem[e] = src_kind[b] ? cmem[coff[binmem[binoff[b]]] + q] : klo[sstart[segof[b]] + q];
}

__global__ void k_silk_capacity(unsigned long long ns, unsigned long long nm, uint32_t* k_out,
                                unsigned long long* needed, unsigned long long* counters,
                                unsigned long long c0, unsigned long long c1, unsigned long long c2,
                                unsigned long long c3, int32_t* st) {
  if (blockIdx.x || threadIdx.x) return;
  needed[0] = ns;
  needed[1] = nm;
  *k_out = 0;
  set_status(st, GEEK_ERR_CAPACITY);
  if (counters) {
    counters[0] = c0;
    counters[1] = c1;
    counters[2] = c2;
    counters[3] = c3;
  }
}

__global__ void k_silk_finish(uint32_t k, uint32_t members, uint64_t cap_k, uint64_t cap_m,
                              uint32_t* seed_off, uint32_t* k_out, unsigned long long* needed,
                              unsigned long long* counters, unsigned long long c0, unsigned long long c1,
                              unsigned long long c2, unsigned long long c3, int32_t* st) {
  if (blockIdx.x || threadIdx.x) return;
  needed[0] = k;
  needed[1] = members;
  if (k > cap_k || members > cap_m) {
    set_status(st, GEEK_ERR_CAPACITY);
    *k_out = 0;
  } else {
    seed_off[k] = members;
    *k_out = k;
    if (k == 0) set_status(st, GEEK_ERR_NO_SEEDS);
  }
  if (counters) {
    counters[0] = c0;
    counters[1] = c1;
    counters[2] = c2;
    counters[3] = c3;
  }
}

// ---------------------------------------------------------------- host side
struct SilkWs {
  int64_t N1, Ccap;
  uint32_t *base, *gstart, *gsize, *G, *binmem, *binoff, *nbins, *bin_of, *flag, *fscan, *cnt, *poff;
  uint32_t *hi, *lo, *hi2, *lo2, *h, *hs, *rstart, *kept, *kidx, *khi, *klo;
  uint32_t *sflag, *sscan, *sstart, *esize, *eoff, *eone, *eidx;
  uint32_t *cmem, *coff, *ssize, *src_kind, *segof;
  uint32_t *tw[4], *tv, *tw2[4], *tv2;
  uint32_t *radix_tmp, *scan_tmp, *big_list, *small;
  void* bz_ws;
  size_t bz_bytes;
};

static geek_bucketize_job bz_job_for(int64_t n, int K) {
  geek_bucketize_job b{};
  b.n = n < 1 ? 1 : n;
  b.T = 1;
  b.key_words = K;
  b.table_stride = 0;
  b.row_stride = K;
  return b;
}

static size_t carve_silk(const geek_silk_job& J, void* ws, SilkWs& W) {
  Carver c(ws);
  const int64_t Tn = (int64_t)J.T * J.n;
  W.Ccap = 4 * (J.cap_members > 0 ? J.cap_members : 1);
  W.N1 = Tn > W.Ccap ? Tn : W.Ccap;
  const int64_t N1 = W.N1;
  W.base = c.take<uint32_t>(J.T + 1);
  W.gstart = c.take<uint32_t>(N1 + 1);
  W.gsize = c.take<uint32_t>(N1 + 1);
  W.G = c.take<uint32_t>(N1 * 4);
  W.binmem = c.take<uint32_t>(N1);
  W.binoff = c.take<uint32_t>(N1 + 1);
  W.nbins = c.take<uint32_t>(4);
  W.bin_of = c.take<uint32_t>(N1);
  W.flag = c.take<uint32_t>(N1 + 1);
  W.fscan = c.take<uint32_t>(N1 + 1);
  W.cnt = c.take<uint32_t>(N1 + 1);
  W.poff = c.take<uint32_t>(N1 + 1);
  W.hi = c.take<uint32_t>(N1);
  W.lo = c.take<uint32_t>(N1);
  W.hi2 = c.take<uint32_t>(N1);
  W.lo2 = c.take<uint32_t>(N1);
  W.h = c.take<uint32_t>(N1 + 1);
  W.hs = c.take<uint32_t>(N1 + 1);
  W.rstart = c.take<uint32_t>(N1 + 1);
  W.kept = c.take<uint32_t>(N1 + 1);
  W.kidx = c.take<uint32_t>(N1 + 1);
  W.khi = c.take<uint32_t>(N1);
  W.klo = c.take<uint32_t>(N1);
  W.sflag = c.take<uint32_t>(N1 + 1);
  W.sscan = c.take<uint32_t>(N1 + 1);
  W.sstart = c.take<uint32_t>(N1 + 1);
  W.esize = c.take<uint32_t>(N1 + 1);
  W.eoff = c.take<uint32_t>(N1 + 1);
  W.eone = c.take<uint32_t>(N1 + 1);
  W.eidx = c.take<uint32_t>(N1 + 1);
  W.cmem = c.take<uint32_t>(W.Ccap);
  W.coff = c.take<uint32_t>(W.Ccap + 1);
  W.ssize = c.take<uint32_t>(N1 + 1);
  W.src_kind = c.take<uint32_t>(N1 + 1);
  W.segof = c.take<uint32_t>(N1 + 1);
  for (int w = 0; w < 4; ++w) W.tw[w] = c.take<uint32_t>(N1);
  W.tv = c.take<uint32_t>(N1);
  for (int w = 0; w < 4; ++w) W.tw2[w] = c.take<uint32_t>(N1);
  W.tv2 = c.take<uint32_t>(N1);
  W.radix_tmp = c.take<uint32_t>(radix_tmp_words(N1));
  W.scan_tmp = c.take<uint32_t>(exscan_tmp_words(N1 + 1) + 16);
  W.big_list = c.take<uint32_t>(N1 + 1);
  W.small = c.take<uint32_t>(64);
  W.bz_bytes = bucketize_ws(bz_job_for(N1, 4));
  W.bz_ws = c.take<char>(W.bz_bytes);
  return c.used + 256;
}

size_t silk_ws(const geek_silk_job& J) {
  SilkWs W;
  return carve_silk(J, nullptr, W);
}

static inline int nblk(int64_t n) { return (int)((n + 255) / 256) > 0 ? (int)((n + 255) / 256) : 1; }

struct Host {
  hipStream_t s;
  uint32_t read(const uint32_t* p) {
    uint32_t v = 0;
    hipMemcpyAsync(&v, p, 4, hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    return v;
  }
};

static int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 32 && (maxval >> b) != 0) ++b;
  return b;
}

// One voting round over `ns` sets (start/size in gstart/gsize, members in
// mem starting at position base0 covering npos positions) whose signatures are
// in W.G: bins, pairs, majority.  Leaves the kept (bin, id) pairs in khi/klo
// (sorted) and their bin segments in sstart; returns the segment count.
struct VoteOut {
  uint32_t nbins, P, R, Kept, S, multi;
};



static int32_t vote_round(SilkWs& W, const uint32_t* mem, int64_t ns, uint32_t base0, int64_t npos, int K,
                          int id_bits, Host& H, int32_t* st, VoteOut& o) {
  hipStream_t s = H.s;
  // bins of identical signatures
  geek_bucketize_job bj = bz_job_for(ns, K);
  bj.keys = W.G;
  bj.members = W.binmem;
  bj.offsets = W.binoff;
  bj.nbuckets = W.nbins;
  bj.bucket_of = W.bin_of;
  if (int32_t rc = bucketize_run(bj, W.bz_ws, W.bz_bytes, st, s)) return rc;
  o.nbins = H.read(W.nbins);
  // pairs of multi-set bins
  hipLaunchKernelGGL(k_put, dim3(1), dim3(1), 0, s, W.small, 9, 0u);
  hipLaunchKernelGGL(k_pair_count, dim3(nblk(ns)), dim3(256), 0, s, W.bin_of, W.binoff, W.binmem, W.gsize, ns,
                     W.cnt, W.small + 9);
  o.multi = H.read(W.small + 9);
  exscan_u32(W.cnt, W.poff, ns, W.scan_tmp, W.small + 0, s);
  o.P = H.read(W.small + 0);
  o.R = o.Kept = o.S = 0;
  if (o.P == 0) return GEEK_OK;
  hipLaunchKernelGGL(k_fill0, dim3(nblk(npos)), dim3(256), 0, s, W.flag, npos);
  hipLaunchKernelGGL(k_mark_starts, dim3(nblk(ns)), dim3(256), 0, s, W.gstart, ns, base0, W.flag);
  exscan_u32(W.flag, W.fscan, npos, W.scan_tmp, nullptr, s);
  hipLaunchKernelGGL(k_pairs, dim3(nblk(npos)), dim3(256), 0, s, mem, npos, base0, W.flag, W.fscan, W.gstart,
                     W.cnt, W.poff, W.bin_of, W.hi, W.lo);
  // sort by (bin, id): lo is word 0, hi is word 1
  int words[12], shifts[12], np = 0;
  for (int sh = 0; sh < id_bits; sh += 8) {
    words[np] = 0;
    shifts[np++] = sh;
  }
  const int bb = bits_for(o.nbins ? o.nbins - 1 : 0);
  for (int sh = 0; sh < bb; sh += 8) {
    words[np] = 1;
    shifts[np++] = sh;
  }
  RsView A{{W.lo, W.hi, nullptr, nullptr}, nullptr}, B{{W.lo2, W.hi2, nullptr, nullptr}, nullptr};
  const int in_alt = radix_sort(A, B, 2, o.P, words, shifts, np, W.radix_tmp, s);
  uint32_t* hi = in_alt ? W.hi2 : W.hi;
  uint32_t* lo = in_alt ? W.lo2 : W.lo;
  // runs of equal (bin, id) and the majority vote
  hipLaunchKernelGGL(k_run_heads, dim3(nblk(o.P)), dim3(256), 0, s, hi, lo, (int64_t)o.P, W.h);
  exscan_u32(W.h, W.hs, o.P, W.scan_tmp, W.hs + o.P, s);
  hipLaunchKernelGGL(k_starts, dim3(nblk(o.P + 1)), dim3(256), 0, s, W.h, W.hs, (int64_t)o.P, W.rstart);
  o.R = H.read(W.hs + o.P);
  hipLaunchKernelGGL(k_keep, dim3(nblk(o.R)), dim3(256), 0, s, W.rstart, (int64_t)o.R, hi, W.binoff, W.kept);
  exscan_u32(W.kept, W.kidx, o.R, W.scan_tmp, W.kidx + o.R, s);
  hipLaunchKernelGGL(k_compact_runs, dim3(nblk(o.R)), dim3(256), 0, s, W.rstart, (int64_t)o.R, W.kept, W.kidx,
                     hi, lo, W.khi, W.klo);
  o.Kept = H.read(W.kidx + o.R);
  if (o.Kept == 0) return GEEK_OK;
  hipLaunchKernelGGL(k_seg_heads, dim3(nblk(o.Kept)), dim3(256), 0, s, W.khi, (int64_t)o.Kept, W.sflag);
  exscan_u32(W.sflag, W.sscan, o.Kept, W.scan_tmp, W.sscan + o.Kept, s);
  hipLaunchKernelGGL(k_starts, dim3(nblk(o.Kept + 1)), dim3(256), 0, s, W.sflag, W.sscan, (int64_t)o.Kept,
                     W.sstart);
  o.S = H.read(W.sscan + o.Kept);
  return GEEK_OK;
}

int32_t silk_run(const geek_silk_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s) {
  if (J.n < 1 || J.T < 1 || J.K < 1 || J.K > 4 || J.L < 0 || !J.members || !J.offsets || !J.nbuckets ||
      !J.silk_keys || !J.seed_offsets || !J.seed_members || !J.k_out || !J.needed || J.cap_k < 0 ||
      J.cap_members < 0)
    return GEEK_ERR_ARG;
  if ((int64_t)J.T * J.n >= (1ll << 32) - 2) return GEEK_ERR_UNSUPPORTED;
  SilkWs W;
  if (!ws || ws_bytes < carve_silk(J, ws, W)) return GEEK_ERR_WORKSPACE;
  Host H{s};
  prof_begin(GEEK_PROF_SILK, s);
  const int K = J.K;
  const int64_t Tn = (int64_t)J.T * J.n;
  hipLaunchKernelGGL(k_tab_base, dim3(1), dim3(1), 0, s, J.nbuckets, J.T, W.base);
  const uint32_t NB = H.read(W.base + J.T);
  unsigned long long pairs = 0, multi = 0;
  uint32_t cm = 0, cs = 0;  // members / sets of C so far
  bool overflow = false;
  uint64_t need_m = 0, need_s = 0;
  const int id_bits = bits_for((uint64_t)(J.n - 1));
  hipLaunchKernelGGL(k_extent, dim3(nblk(NB)), dim3(256), 0, s, J.offsets, W.base, J.T, J.n, (int64_t)NB,
                     W.gstart, W.gsize);
  for (int t = 0; t < J.L; ++t) {
    hipLaunchKernelGGL(k_put, dim3(1), dim3(1), 0, s, W.small + 8, 0, 0u);
    hipLaunchKernelGGL(k_sig, dim3(nblk(NB)), dim3(256), 0, s, J.members, W.gstart, W.gsize, (int64_t)NB,
                       J.silk_keys + 2 * t * K, K, W.G, W.big_list, W.small + 8);
    hipLaunchKernelGGL(k_sig_big, dim3(512), dim3(256), 0, s, J.members, W.gstart, W.gsize,
                       J.silk_keys + 2 * t * K, K, W.G, W.big_list, W.small + 8);
    VoteOut o;
    if (int32_t rc = vote_round(W, J.members, NB, 0u, Tn, K, id_bits, H, st, o)) return rc;
    pairs += o.P;
    multi += o.multi;
    if (o.S == 0) continue;
    hipLaunchKernelGGL(k_seg_emit_size, dim3(nblk(o.S)), dim3(256), 0, s, W.sstart, (int64_t)o.S, J.delta,
                       W.esize, W.eone);
    exscan_u32(W.esize, W.eoff, o.S, W.scan_tmp, W.eoff + o.S, s);
    exscan_u32(W.eone, W.eidx, o.S, W.scan_tmp, W.eidx + o.S, s);
    const uint32_t em = H.read(W.eoff + o.S), es = H.read(W.eidx + o.S);
    need_m += em;
    need_s += es;
    if ((int64_t)cm + em > W.Ccap || (int64_t)cs + es > W.Ccap) {
      overflow = true;
      continue;
    }
    hipLaunchKernelGGL(k_seg_emit, dim3(nblk(o.S)), dim3(256), 0, s, W.sstart, (int64_t)o.S, W.esize, W.eoff,
                       W.eidx, W.klo, cm, cs, W.cmem, W.coff);
    if (em)
      hipLaunchKernelGGL(k_seg_copy, dim3(nblk(em)), dim3(256), 0, s, W.sstart, (int64_t)o.S, W.eoff, W.klo, cm, em,
                         W.cmem);
    cm += em;
    cs += es;
  }
  const unsigned long long hash_evals = (unsigned long long)K * J.L * Tn;
  if (overflow) {
    // C did not fit: report the capacities that make it fit (C holds up to
    // 4 * cap_members members and sets)
    hipLaunchKernelGGL(k_silk_capacity, dim3(1), dim3(1), 0, s, (unsigned long long)((need_s + 3) / 4),
                       (unsigned long long)((need_m + 3) / 4), J.k_out, J.needed, J.counters, hash_evals,
                       pairs, (unsigned long long)need_s, multi, st);
    hipStreamSynchronize(s);
    prof_end(GEEK_PROF_SILK, s);
    return GEEK_OK;
  }
  if (cs == 0) {
    hipLaunchKernelGGL(k_silk_finish, dim3(1), dim3(1), 0, s, 0u, 0u, (unsigned long long)J.cap_k,
                       (unsigned long long)J.cap_members, J.seed_offsets, J.k_out, J.needed, J.counters,
                       hash_evals, pairs, 0ull, multi, st);
    hipLaunchKernelGGL(k_put, dim3(1), dim3(1), 0, s, J.seed_offsets, 0, 0u);
    hipStreamSynchronize(s);
    prof_end(GEEK_PROF_SILK, s);
    return GEEK_OK;
  }
  // ---- de-duplication: one more table over the sets of C
  hipLaunchKernelGGL(k_put, dim3(1), dim3(1), 0, s, W.coff, (int64_t)cs, cm);
  hipLaunchKernelGGL(k_set_extent, dim3(nblk(cs)), dim3(256), 0, s, W.coff, (int64_t)cs, W.gstart, W.gsize);
  hipLaunchKernelGGL(k_put, dim3(1), dim3(1), 0, s, W.small + 8, 0, 0u);
  hipLaunchKernelGGL(k_sig, dim3(nblk(cs)), dim3(256), 0, s, W.cmem, W.gstart, W.gsize, (int64_t)cs,
                     J.silk_keys + 2 * J.L * K, K, W.G, W.big_list, W.small + 8);
  hipLaunchKernelGGL(k_sig_big, dim3(512), dim3(256), 0, s, W.cmem, W.gstart, W.gsize, J.silk_keys + 2 * J.L * K,
                     K, W.G, W.big_list, W.small + 8);
  VoteOut o;
  if (int32_t rc = vote_round(W, W.cmem, cs, 0u, cm, K, id_bits, H, st, o)) return rc;
  const int64_t nb2 = o.nbins;
  hipLaunchKernelGGL(k_dedup_size, dim3(nblk(nb2)), dim3(256), 0, s, W.binoff, W.binmem, nb2, W.gsize, W.ssize,
                     W.src_kind);
  if (o.S)
    hipLaunchKernelGGL(k_dedup_multi, dim3(nblk(o.S)), dim3(256), 0, s, W.sstart, (int64_t)o.S, W.khi, J.delta,
                       W.ssize, W.segof);
  // order bins by their K-tuple (word 0 most significant)
  hipLaunchKernelGGL(k_bin_tuples, dim3(nblk(nb2)), dim3(256), 0, s, W.binoff, W.binmem, nb2, W.G, K, W.tw[0],
                     W.tw[1], W.tw[2], W.tw[3], W.tv);
  int words[16], shifts[16], np = 0;
  for (int k = K - 1; k >= 0; --k)
    for (int sh = 0; sh < 32; sh += 8) {
      words[np] = k;
      shifts[np++] = sh;
    }
  RsView A{{W.tw[0], W.tw[1], W.tw[2], W.tw[3]}, W.tv}, B{{W.tw2[0], W.tw2[1], W.tw2[2], W.tw2[3]}, W.tv2};
  const int in_alt = radix_sort(A, B, 4, nb2, words, shifts, np, W.radix_tmp, s);
  const uint32_t* ord = in_alt ? W.tv2 : W.tv;
  hipLaunchKernelGGL(k_order_sizes, dim3(nblk(nb2)), dim3(256), 0, s, ord, nb2, W.ssize, W.esize, W.eone);
  exscan_u32(W.esize, W.eoff, nb2, W.scan_tmp, W.eoff + nb2, s);
  exscan_u32(W.eone, W.eidx, nb2, W.scan_tmp, W.eidx + nb2, s);
  const uint32_t tot_m = H.read(W.eoff + nb2), k = H.read(W.eidx + nb2);
  if ((int64_t)k <= J.cap_k && (int64_t)tot_m <= J.cap_members) {
    hipLaunchKernelGGL(k_emit_seeds, dim3(nblk(nb2)), dim3(256), 0, s, ord, nb2, W.esize, W.eoff, W.eidx,
                       W.src_kind, W.binoff, W.binmem, W.cmem, W.coff, W.segof, W.sstart, W.klo, J.seed_offsets,
                       J.seed_members);
    if (tot_m)
      hipLaunchKernelGGL(k_seed_copy, dim3(nblk(tot_m)), dim3(256), 0, s, ord, nb2, W.eoff, W.src_kind, W.binoff,
                         W.binmem, W.cmem, W.coff, W.segof, W.sstart, W.klo, tot_m, J.seed_members);
  }
  hipLaunchKernelGGL(k_silk_finish, dim3(1), dim3(1), 0, s, k, tot_m, (unsigned long long)J.cap_k,
                     (unsigned long long)J.cap_members, J.seed_offsets, J.k_out, J.needed, J.counters, hash_evals,
                     pairs, (unsigned long long)cs, multi, st);
  prof_end(GEEK_PROF_SILK, s);
  hipStreamSynchronize(s);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
