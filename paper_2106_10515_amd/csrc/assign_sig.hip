// Assignment of MinHash signatures to the modes of the seeds (paper Section
// 3.3: the central vector of sets is the mode; Section 2.1: Dist = 1 - Sim)
// on gfx950.
//
//   modes       items (seed j, position f, value) sorted by (j*F + f, value);
//               each (j, f) occupies a fixed, known segment of the sorted
//               array, scanned by one thread for its longest run (smallest
//               value on ties).
//   index       an exact inverted index: (f, mode value) -> ascending list of
//               seeds j, as a hash table of run extents over the sorted
//               (f, value, j) triples.
//   assign      one wavefront per row probes its F (f, sig[f]) pairs, gathers
//               the matching seeds in LDS, sorts them and takes the longest
//               run (lowest j on ties); a row whose matches overflow the LDS
//               list is compared against every mode instead.  Rows with no
//               match at all take seed 0 (every count is 0).
#include <algorithm>

#include "common.hpp"
#include "radix.hpp"

namespace geek {

void sse_and_radius(const double* dist, const int32_t* assign, int64_t n, int k, double* sse, double* radius,
                    int take_sqrt, double* sse_blk, hipStream_t s);
size_t sse_blk_words(int64_t n);

constexpr int SG_CAP = 2048;  // matched seeds held in LDS per row
// k * F up to which every row is compared against every mode directly
constexpr int64_t SIG_DENSE_MAX = 1 << 20;

__device__ __forceinline__ int seed_of(const uint32_t* __restrict__ so, int k, uint32_t pos) {
  int lo = 0, hi = k;  // so[lo] <= pos < so[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (so[mid] <= pos) lo = mid; else hi = mid;
  }
  return lo;
}

// items of seed j, member q, position f at j's segment: so[j]*F + f*s_j + q
__global__ void k_mode_items(const uint32_t* __restrict__ V, int64_t ldv, int F, int64_t n,
                             const uint32_t* __restrict__ so, const uint32_t* __restrict__ sm, int k,
                             int64_t NC, uint32_t* __restrict__ val, uint32_t* __restrict__ seg,
                             int32_t* st) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= NC * F) return;
  const uint32_t mpos = (uint32_t)(g / F);
  const int f = (int)(g % F);
  const int j = seed_of(so, k, mpos);
  const uint32_t sj = so[j + 1] - so[j];
  const uint32_t q = mpos - so[j];
  const uint32_t id = sm[mpos];
  if ((int64_t)id >= n) {
    set_status(st, GEEK_ERR_ARG);
    return;
  }
  const int64_t at = (int64_t)so[j] * F + (int64_t)f * sj + q;
  val[at] = V[(int64_t)id * ldv + f];
  seg[at] = (uint32_t)j * (uint32_t)F + (uint32_t)f;
}

__global__ void k_mode_pick(const uint32_t* __restrict__ val, const uint32_t* __restrict__ so, int k, int F,
                            uint32_t* __restrict__ modes, int32_t* st) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)k * F) return;
  const int j = (int)(g / F), f = (int)(g % F);
  const uint32_t sj = so[j + 1] - so[j];
  if (sj == 0) {
    set_status(st, GEEK_ERR_EMPTY_SET);
    modes[g] = 0u;
    return;
  }
  const uint32_t* p = val + (int64_t)so[j] * F + (int64_t)f * sj;
  uint32_t best = p[0], bcnt = 0, cur = p[0], ccnt = 0;
  for (uint32_t q = 0; q < sj; ++q) {
    if (p[q] == cur) {
      ++ccnt;
    } else {
      if (ccnt > bcnt) {
        bcnt = ccnt;
        best = cur;
      }
      cur = p[q];
      ccnt = 1;
    }
  }
  if (ccnt > bcnt) best = cur;
  modes[g] = best;
}

// (f, value, j) triples of the modes for the inverted index
__global__ void k_index_items(const uint32_t* __restrict__ modes, int k, int F, uint32_t* __restrict__ wj,
                              uint32_t* __restrict__ wv, uint32_t* __restrict__ wf) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)k * F) return;
  wj[g] = (uint32_t)(g / F);
  wf[g] = (uint32_t)(g % F);
  wv[g] = modes[g];
}

__device__ __forceinline__ uint64_t pack_fv(uint32_t f, uint32_t v) { return ((uint64_t)f << 32) | v; }
__device__ __forceinline__ uint32_t slot_of(uint64_t key, uint32_t mask) {
  return fmix32((uint32_t)key ^ fmix32((uint32_t)(key >> 32) + 0x9E3779B9u)) & mask;
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Insert every run head of the sorted (f, v) keys: value = start << 32 | len.
__global__ void k_index_insert(const uint32_t* __restrict__ sv, const uint32_t* __restrict__ sf, int64_t NI,
                               unsigned long long* __restrict__ hkey, unsigned long long* __restrict__ hval,
                               uint32_t mask) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= NI) return;
  if (q > 0 && sv[q] == sv[q - 1] && sf[q] == sf[q - 1]) return;
  int64_t e = q + 1;
  while (e < NI && sv[e] == sv[q] && sf[e] == sf[q]) ++e;
  const uint64_t key = pack_fv(sf[q], sv[q]);
  uint32_t h = slot_of(key, mask);
  while (true) {
    const unsigned long long old = atomicCAS(&hkey[h], ~0ull, (unsigned long long)key);
    if (old == ~0ull || old == key) break;
    h = (h + 1) & mask;
  }
  hval[h] = ((unsigned long long)q << 32) | (unsigned long long)(e - q);
}

__device__ __forceinline__ bool index_find(const unsigned long long* __restrict__ hkey,
                                           const unsigned long long* __restrict__ hval, uint32_t mask,
                                           uint32_t f, uint32_t v, uint32_t& start, uint32_t& len) {
  const uint64_t key = pack_fv(f, v);
  uint32_t h = slot_of(key, mask);
  while (true) {
    const unsigned long long kk = hkey[h];
    if (kk == key) {
      const unsigned long long vv = hval[h];
      start = (uint32_t)(vv >> 32);
      len = (uint32_t)vv;
      return true;
    }
    if (kk == ~0ull) return false;
    h = (h + 1) & mask;
  }
}

// One wavefront (block of 64) per row.
__global__ __launch_bounds__(64) void k_sig_assign(const uint32_t* __restrict__ S, int64_t lds, int F, int64_t n,
                                                   const unsigned long long* __restrict__ hkey,
                                                   const unsigned long long* __restrict__ hval, uint32_t mask,
                                                   const uint32_t* __restrict__ jlist, int32_t* __restrict__ assign,
                                                   double* __restrict__ dist, uint32_t* __restrict__ dense,
                                                   uint32_t* __restrict__ dense_count,
                                                   unsigned long long* __restrict__ ctr) {
  __shared__ uint32_t lst[SG_CAP];
  __shared__ uint32_t cnt;
  unsigned long long my_rows = 0, my_matches = 0;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const uint32_t* row = S + i * lds;
    for (int f = threadIdx.x; f < F; f += 64) {
      uint32_t st, ln;
      if (index_find(hkey, hval, mask, (uint32_t)f, row[f], st, ln)) {
        const uint32_t at = atomicAdd(&cnt, ln);
        for (uint32_t e = 0; e < ln; ++e)
          if (at + e < SG_CAP) lst[at + e] = jlist[st + e];
      }
    }
    __syncthreads();
    const uint32_t c = cnt;
    if (c > SG_CAP) {
      if (threadIdx.x == 0) dense[atomicAdd(dense_count, 1u)] = (uint32_t)i;
      __syncthreads();
      continue;
    }
    int P2 = 1;
    while (P2 < (int)c) P2 <<= 1;
    for (int q = (int)c + threadIdx.x; q < P2; q += 64) lst[q] = 0xFFFFFFFFu;
    __syncthreads();
    for (int kk = 2; kk <= P2; kk <<= 1) {
      for (int jj = kk >> 1; jj > 0; jj >>= 1) {
        for (int q = threadIdx.x; q < P2; q += 64) {
          const int o = q ^ jj;
          if (o > q) {
            const uint32_t a = lst[q], b = lst[o];
            const bool up = (q & kk) == 0;
            if (up ? (b < a) : (a < b)) {
              lst[q] = b;
              lst[o] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    if (threadIdx.x == 0) {
      uint32_t best = 0, bcnt = 0, cur = 0, ccnt = 0;
      for (uint32_t q = 0; q < c; ++q) {
        if (q > 0 && lst[q] == cur) {
          ++ccnt;
        } else {
          if (q > 0 && ccnt > bcnt) {
            bcnt = ccnt;
            best = cur;
          }
          cur = lst[q];
          ccnt = 1;
        }
      }
      if (c > 0 && ccnt > bcnt) {
        bcnt = ccnt;
        best = cur;
      }
      assign[i] = (int32_t)best;  // no match: every count is 0, seed 0 wins
      dist[i] = 1.0 - (double)bcnt / (double)F;
      ++my_rows;
      my_matches += c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && ctr) {
    atomicAdd(ctr + 0, my_rows);
    atomicAdd(ctr + 3, my_matches);
  }
}

// Rows whose match lists overflowed: count against every mode, lowest j on
// ties.  One lane per row, 256 rows per workgroup; blocks of 32 seeds x 256
// signature positions are staged in LDS and read by every lane at the same
// address (broadcast); each lane keeps 16 of its row's words and 32 match
// counters in registers (a compare and an add-with-carry per comparison).
constexpr int SD_SEEDS = 32;   // seeds per register block
constexpr int SD_F = 16;       // signature words per register chunk
constexpr int SD_SEG = 256;    // signature positions per LDS segment
__global__ __launch_bounds__(256) void k_sig_dense(const uint32_t* __restrict__ S, int64_t lds, int F,
                                                   const uint32_t* __restrict__ modes, int k,
                                                   const uint32_t* __restrict__ rows,
                                                   const uint32_t* __restrict__ count, int64_t n_rows,
                                                   int32_t* __restrict__ assign, double* __restrict__ dist,
                                                   unsigned long long* __restrict__ ctr) {
  __shared__ __attribute__((aligned(16))) uint32_t lm[SD_SEEDS * SD_SEG];
  const int64_t nr = rows ? (int64_t)*count : n_rows;  // rows == nullptr: every row
  const int lane = threadIdx.x & 63;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < nr; base += (int64_t)gridDim.x * 256) {
    const int64_t pos = base + threadIdx.x;
    const bool live = pos < nr;
    const int64_t i = !live ? 0 : rows ? (int64_t)rows[pos] : pos;
    const uint32_t* srow = S + i * lds;
    const bool row_vec = (lds & 3) == 0;
    uint32_t best = 0, bj = 0x7fffffffu;
    for (int jb = 0; jb < k; jb += SD_SEEDS) {
      uint32_t cnt[SD_SEEDS];
#pragma unroll
      for (int q = 0; q < SD_SEEDS; ++q) cnt[q] = 0u;
      for (int fs = 0; fs < F; fs += SD_SEG) {
        const int seg = F - fs < SD_SEG ? F - fs : SD_SEG;
        __syncthreads();  // previous segment consumed
        for (int t = threadIdx.x; t < SD_SEEDS * SD_SEG; t += 256) {
          const int q = t / SD_SEG, f = t % SD_SEG;
          lm[t] = (jb + q < k && f < seg) ? modes[(int64_t)(jb + q) * F + fs + f] : 0u;
        }
        __syncthreads();
        for (int f0 = 0; f0 < seg; f0 += SD_F) {
          if (row_vec && f0 + SD_F <= seg) {
            uint32_t x[SD_F];
#pragma unroll
            for (int e = 0; e < SD_F; e += 4) {
              const uint4 v = *reinterpret_cast<const uint4*>(srow + fs + f0 + e);
              x[e] = v.x;
              x[e + 1] = v.y;
              x[e + 2] = v.z;
              x[e + 3] = v.w;
            }
#pragma unroll
            for (int q = 0; q < SD_SEEDS; ++q) {
#pragma unroll
              for (int e = 0; e < SD_F; e += 4) {
                const uint4 m = *reinterpret_cast<const uint4*>(lm + q * SD_SEG + f0 + e);
                cnt[q] += (x[e] == m.x) ? 1u : 0u;
                cnt[q] += (x[e + 1] == m.y) ? 1u : 0u;
                cnt[q] += (x[e + 2] == m.z) ? 1u : 0u;
                cnt[q] += (x[e + 3] == m.w) ? 1u : 0u;
              }
            }
          } else {
            for (int f = f0; f < seg && f < f0 + SD_F; ++f) {
              const uint32_t xv = srow[fs + f];
#pragma unroll
              for (int q = 0; q < SD_SEEDS; ++q) cnt[q] += (xv == lm[q * SD_SEG + f]) ? 1u : 0u;
            }
          }
        }
      }
      // strict > with ascending j keeps the lowest index on ties
#pragma unroll
      for (int q = 0; q < SD_SEEDS; ++q) {
        const int j = jb + q;
        if (j < k && (cnt[q] > best || bj == 0x7fffffffu)) {
          best = cnt[q];
          bj = (uint32_t)j;
        }
      }
    }
    if (live) {
      assign[i] = (int32_t)bj;
      dist[i] = 1.0 - (double)best / (double)F;
    }
    if (ctr) {
      const unsigned long long nlive = __popcll(__ballot(live));
      if (lane == 0 && nlive) atomicAdd(ctr + 2, nlive);
    }
  }
}

__global__ void k_zero_words(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}
__global__ void k_copy_ctr(const unsigned long long* a, unsigned long long* b) {
  if (threadIdx.x < 4) b[threadIdx.x] = a[threadIdx.x];
}

// ---------------------------------------------------------------- host side
struct SigWs {
  int64_t NI;  // mode items: members * F
  uint32_t *val, *seg, *val2, *seg2;
  uint32_t *wj, *wv, *wf, *wj2, *wv2, *wf2;
  unsigned long long *hkey, *hval, *ctr;
  uint32_t *dense, *small, *rtmp;
  double *dist, *sse_blk;
  uint32_t hmask;
};

static uint32_t pow2_at_least(uint64_t v) {
  uint32_t p = 1;
  while (p < v && p < (1u << 31)) p <<= 1;
  return p;
}

static size_t carve_sig(const geek_assign_job& J, void* ws, SigWs& W) {
  Carver c(ws);
  const int64_t F = J.F;
  const int64_t NI = J.n_members * F;
  const int64_t KI = (int64_t)J.k * F;
  const int64_t NR = NI > KI ? NI : KI;
  W.NI = NI;
  W.val = c.take<uint32_t>(NR + 1);
  W.seg = c.take<uint32_t>(NR + 1);
  W.val2 = c.take<uint32_t>(NR + 1);
  W.seg2 = c.take<uint32_t>(NR + 1);
  W.wj = c.take<uint32_t>(KI + 1);
  W.wv = c.take<uint32_t>(KI + 1);
  W.wf = c.take<uint32_t>(KI + 1);
  W.wj2 = c.take<uint32_t>(KI + 1);
  W.wv2 = c.take<uint32_t>(KI + 1);
  W.wf2 = c.take<uint32_t>(KI + 1);
  const uint32_t HS = pow2_at_least(2 * (uint64_t)KI + 2);
  W.hmask = HS - 1;
  W.hkey = c.take<unsigned long long>(HS);
  W.hval = c.take<unsigned long long>(HS);
  W.ctr = c.take<unsigned long long>(4);
  W.dense = c.take<uint32_t>(J.n + 1);
  W.small = c.take<uint32_t>(16);
  W.rtmp = c.take<uint32_t>(radix_tmp_words(NR));
  W.dist = c.take<double>(J.dist ? 1 : J.n);
  W.sse_blk = c.take<double>(sse_blk_words(J.n));
  return c.used + 256;
}

size_t assign_sig_ws(const geek_assign_job& J) {
  SigWs W;
  return carve_sig(J, nullptr, W);
}

static int bits_of(uint64_t v) {
  int b = 0;
  while (b < 32 && (v >> b)) ++b;
  return b;
}

int32_t modes_run(const uint32_t* V, int64_t ldv, int F, int64_t n, const uint32_t* so, const uint32_t* sm, int k,
                  int64_t NC, uint32_t* modes, SigWs& W, int32_t* st, hipStream_t s) {
  const int64_t NI = NC * F;
  if (NI > 0) {
    hipLaunchKernelGGL(k_mode_items, dim3(ceil_div(NI, 256)), dim3(256), 0, s, V, ldv, F, n, so, sm, k, NC,
                       W.val, W.seg, st);
    int words[8], shifts[8], np = 0;
    for (int sh = 0; sh < 32; sh += 8) {
      words[np] = 0;
      shifts[np++] = sh;
    }
    const int sb = bits_of((uint64_t)k * F - 1);
    for (int sh = 0; sh < sb; sh += 8) {
      words[np] = 1;
      shifts[np++] = sh;
    }
    RsView A{{W.val, W.seg, nullptr, nullptr}, nullptr}, B{{W.val2, W.seg2, nullptr, nullptr}, nullptr};
    const int alt = radix_sort(A, B, 2, NI, words, shifts, np, W.rtmp, s);
    hipLaunchKernelGGL(k_mode_pick, dim3(ceil_div((int64_t)k * F, 256)), dim3(256), 0, s, alt ? W.val2 : W.val,
                       so, k, F, modes, st);
  }
  return GEEK_OK;
}

// Standalone modes of an integer matrix (the categorical attributes of
// heterogeneous rows), with its own workspace.
size_t modes_ws(int64_t n_members, int F, int k) {
  Carver c(nullptr);
  const int64_t NI = n_members * F, KI = (int64_t)k * F;
  const int64_t NR = NI > KI ? NI : KI;
  for (int q = 0; q < 4; ++q) c.take<uint32_t>(NR + 1);
  c.take<uint32_t>(radix_tmp_words(NR));
  return c.used + 256;
}

int32_t modes_compute(const uint32_t* V, int64_t ldv, int F, int64_t n, const uint32_t* so, const uint32_t* sm,
                      int k, int64_t NC, uint32_t* modes, void* ws, int32_t* st, hipStream_t s) {
  Carver c(ws);
  const int64_t NI = NC * F, KI = (int64_t)k * F;
  const int64_t NR = NI > KI ? NI : KI;
  SigWs W{};
  W.val = c.take<uint32_t>(NR + 1);
  W.seg = c.take<uint32_t>(NR + 1);
  W.val2 = c.take<uint32_t>(NR + 1);
  W.seg2 = c.take<uint32_t>(NR + 1);
  W.rtmp = c.take<uint32_t>(radix_tmp_words(NR));
  return modes_run(V, ldv, F, n, so, sm, k, NC, modes, W, st, s);
}

int32_t assign_sig(const geek_assign_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s) {
  SigWs W;
  if (ws_bytes < carve_sig(J, ws, W)) return GEEK_ERR_WORKSPACE;
  const int64_t NC = J.n_members;
  prof_begin(GEEK_PROF_ASSIGN, s);
  const int F = J.F, k = J.k;
  double* dist = J.dist ? J.dist : W.dist;
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, W.small, 16);
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(W.ctr), 8);
  modes_run(J.sig, F, F, J.n, J.seed_offsets, J.seed_members, k, NC, J.modes, W, st, s);
  // inverted index over (f, mode value) -> seeds
  const int64_t KI = (int64_t)k * F;
  hipLaunchKernelGGL(k_index_items, dim3(ceil_div(KI, 256)), dim3(256), 0, s, J.modes, k, F, W.wj, W.wv, W.wf);
  int words[12], shifts[12], np = 0;
  for (int sh = 0; sh < bits_of((uint64_t)k - 1); sh += 8) {
    words[np] = 0;
    shifts[np++] = sh;
  }
  for (int sh = 0; sh < 32; sh += 8) {
    words[np] = 1;
    shifts[np++] = sh;
  }
  for (int sh = 0; sh < bits_of((uint64_t)F - 1); sh += 8) {
    words[np] = 2;
    shifts[np++] = sh;
  }
  RsView A{{W.wj, W.wv, W.wf, nullptr}, nullptr}, B{{W.wj2, W.wv2, W.wf2, nullptr}, nullptr};
  const int alt = radix_sort(A, B, 3, KI, words, shifts, np, W.rtmp, s);
  const uint32_t* sj = alt ? W.wj2 : W.wj;
  const uint32_t* sv = alt ? W.wv2 : W.wv;
  const uint32_t* sf = alt ? W.wf2 : W.wf;
  hipLaunchKernelGGL(k_fill_u64, dim3(ceil_div((int64_t)W.hmask + 1, 256)), dim3(256), 0, s, W.hkey,
                     (int64_t)W.hmask + 1, ~0ull);
  hipLaunchKernelGGL(k_index_insert, dim3(ceil_div(KI, 256)), dim3(256), 0, s, sv, sf, KI, W.hkey, W.hval,
                     W.hmask);
  prof_begin(GEEK_PROF_ASSIGN_SCAN, s);
  const int dgrid = (int)std::max<int64_t>(1, std::min<int64_t>(2048, ceil_div(J.n, 256)));
  if ((int64_t)k * F <= SIG_DENSE_MAX) {
    // few seeds: comparing against every mode costs less than building and
    // sorting per-row match lists
    hipLaunchKernelGGL(k_sig_dense, dim3(dgrid), dim3(256), 0, s, J.sig, (int64_t)F, F, J.modes, k, nullptr,
                       nullptr, J.n, J.assign, dist, W.ctr);
  } else {
    const int grid = J.n < 65536 ? (int)J.n : 65536;
    hipLaunchKernelGGL(k_sig_assign, dim3(grid), dim3(64), 0, s, J.sig, (int64_t)F, F, J.n, W.hkey, W.hval,
                       W.hmask, sj, J.assign, dist, W.dense, W.small, W.ctr);
    hipLaunchKernelGGL(k_sig_dense, dim3(dgrid), dim3(256), 0, s, J.sig, (int64_t)F, F, J.modes, k, W.dense,
                       W.small, (int64_t)0, J.assign, dist, W.ctr);
  }
  prof_end(GEEK_PROF_ASSIGN_SCAN, s);
  sse_and_radius(dist, J.assign, J.n, k, J.sse, J.radius, 0, W.sse_blk, s);
  if (J.counters) hipLaunchKernelGGL(k_copy_ctr, dim3(1), dim3(64), 0, s, W.ctr, J.counters);
  prof_end(GEEK_PROF_ASSIGN, s);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
