// Device-wide primitives used by SILK and the signature assignment:
// an exclusive scan of uint32 arrays and a stable LSD radix sort of
// multi-word uint32 keys (structure of arrays) with an optional payload.
#include "common.hpp"
#include "radix.hpp"

namespace geek {

constexpr int GS_THREADS = 256;
constexpr int GS_PER = 16;
constexpr int GS_CHUNK = GS_THREADS * GS_PER;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive block scan of one value per thread; *total = block sum.
__device__ uint32_t blk_exscan(uint32_t v, uint32_t* total, uint32_t* sh) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  const uint32_t x = wave_incl_scan(v);
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

// Element count of a device-count call: *n_dev (when given) bounded by the
// host bound n that sized the grid.
GEEK_D int64_t dev_count(int64_t n, const uint32_t* n_dev) {
  if (!n_dev) return n;
  const int64_t v = (int64_t)*n_dev;
  return v < n ? v : n;
}

__global__ __launch_bounds__(GS_THREADS) void k_gs_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                          const uint32_t* __restrict__ n_dev,
                                                          uint32_t* __restrict__ ctot) {
  __shared__ uint32_t sh[17];
  n = dev_count(n, n_dev);
  const int64_t s = (int64_t)blockIdx.x * GS_CHUNK + threadIdx.x * GS_PER;
  uint32_t a = 0;
#pragma unroll
  for (int u = 0; u < GS_PER; ++u) a += (s + u < n) ? in[s + u] : 0u;
  uint32_t tot;
  blk_exscan(a, &tot, sh);
  if (threadIdx.x == 0) ctot[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_gs_scan_tot(uint32_t* ctot, int nch, uint32_t* total_out) {
  __shared__ uint32_t sh[17];
  const int per = (nch + 1023) / 1024;
  uint32_t loc = 0;
  for (int q = 0; q < per; ++q) {
    const int c = threadIdx.x * per + q;
    if (c < nch) loc += ctot[c];
  }
  uint32_t tot;
  uint32_t base = blk_exscan(loc, &tot, sh);
  for (int q = 0; q < per; ++q) {
    const int c = threadIdx.x * per + q;
    if (c < nch) {
      const uint32_t v = ctot[c];
      ctot[c] = base;
      base += v;
    }
  }
  if (threadIdx.x == 0 && total_out) *total_out = tot;
}

__global__ __launch_bounds__(GS_THREADS) void k_gs_apply(const uint32_t* __restrict__ in, int64_t n,
                                                         const uint32_t* __restrict__ n_dev,
                                                         const uint32_t* __restrict__ ctot,
                                                         uint32_t* __restrict__ out) {
  __shared__ uint32_t sh[17];
  n = dev_count(n, n_dev);
  if ((int64_t)blockIdx.x * GS_CHUNK >= n) return;  // uniform: the chunk lies past the count
  const int64_t s = (int64_t)blockIdx.x * GS_CHUNK + threadIdx.x * GS_PER;
  uint32_t v[GS_PER];
  uint32_t a = 0;
#pragma unroll
  for (int u = 0; u < GS_PER; ++u) {
    v[u] = (s + u < n) ? in[s + u] : 0u;
    a += v[u];
  }
  uint32_t base = blk_exscan(a, nullptr, sh) + ctot[blockIdx.x];
#pragma unroll
  for (int u = 0; u < GS_PER; ++u) {
    if (s + u < n) out[s + u] = base;
    base += v[u];
  }
}

size_t exscan_tmp_words(int64_t n) { return (size_t)((n + GS_CHUNK - 1) / GS_CHUNK) + 1; }

void exscan_u32_dn(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* n_dev, uint32_t* tmp,
                   uint32_t* total, hipStream_t s) {
  const int nch = (int)((n + GS_CHUNK - 1) / GS_CHUNK);
  if (nch == 0) {
    hipLaunchKernelGGL(k_gs_scan_tot, dim3(1), dim3(1024), 0, s, tmp, 0, total);
    return;
  }
  hipLaunchKernelGGL(k_gs_reduce, dim3(nch), dim3(GS_THREADS), 0, s, in, n, n_dev, tmp);
  hipLaunchKernelGGL(k_gs_scan_tot, dim3(1), dim3(1024), 0, s, tmp, nch, total);
  hipLaunchKernelGGL(k_gs_apply, dim3(nch), dim3(GS_THREADS), 0, s, in, n, n_dev, tmp, out);
}

void exscan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, uint32_t* total,
                hipStream_t s) {
  exscan_u32_dn(in, out, n, nullptr, tmp, total, s);
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint32_t* __restrict__ kw, int64_t n,
                                                        const uint32_t* __restrict__ n_dev, int shift,
                                                        uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t h[256];
  n = dev_count(n, n_dev);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t i = s + r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(kw[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items of a tile are ranked in index order (rounds of 256
// in thread order; within a wave by ballot matching of the 8 digit bits),
// placed in LDS in digit order, then written out by consecutive threads, so
// every digit's items of the tile leave as one contiguous run.  The tile's
// digit counts come from the scanned histogram (the next entry of the
// flattened [digit][tile] scan, or n for the last).
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(RsView in, RsView out, int W, int64_t n,
                                                           const uint32_t* __restrict__ n_dev, int word,
                                                           int shift, const uint32_t* __restrict__ hist,
                                                           int nblk) {
  n = dev_count(n, n_dev);
  if ((int64_t)blockIdx.x * RS_TILE >= n) return;  // uniform: the tile lies past the count
  extern __shared__ uint32_t rs_stage[];  // [W (+1 with a payload)][RS_TILE]
  __shared__ uint32_t gstart[256], lstart[256], lrun[256];
  __shared__ uint32_t wcnt[RS_THREADS / 64][256];
  __shared__ uint32_t sh[17];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t flat = (int64_t)threadIdx.x * nblk + blockIdx.x;
  const uint32_t g0 = hist[flat];
  const uint32_t g1 = flat + 1 < (int64_t)256 * nblk ? hist[flat + 1] : (uint32_t)n;
  gstart[threadIdx.x] = g0;
  const uint32_t l0 = blk_exscan(g1 - g0, nullptr, sh);
  lstart[threadIdx.x] = l0;
  lrun[threadIdx.x] = l0;
  for (int w2 = 0; w2 < RS_THREADS / 64; ++w2) wcnt[w2][threadIdx.x] = 0;
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * RS_TILE;
  const int len = n - s < RS_TILE ? (int)(n - s) : RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t i = s + r * RS_THREADS + threadIdx.x;
    const bool has = i < n;
    uint32_t key[4] = {0u, 0u, 0u, 0u};
    uint32_t val = 0u;
    if (has) {
#pragma unroll
      for (int w = 0; w < 4; ++w)
        if (w < W) key[w] = in.k[w][i];
      if (in.v) val = in.v[i];
    }
    const uint32_t kv = word == 0 ? key[0] : word == 1 ? key[1] : word == 2 ? key[2] : key[3];
    const uint32_t dg = has ? (kv >> shift) & 255u : 0u;
    uint64_t mask = __ballot(has);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot(has && ((dg >> b) & 1u));
      mask &= ((dg >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    const bool leader = has && below == 0;
    if (leader) wcnt[wv][dg] = (uint32_t)__popcll(mask);
    __syncthreads();
    if (has) {
      uint32_t before = 0;
      for (int w2 = 0; w2 < wv; ++w2) before += wcnt[w2][dg];
      const uint32_t lp = lrun[dg] + before + below;
#pragma unroll
      for (int w = 0; w < 4; ++w)
        if (w < W) rs_stage[w * RS_TILE + lp] = key[w];
      if (in.v) rs_stage[W * RS_TILE + lp] = val;
    }
    __syncthreads();
    {
      uint32_t tot = 0;
      for (int w2 = 0; w2 < RS_THREADS / 64; ++w2) tot += wcnt[w2][threadIdx.x];
      lrun[threadIdx.x] += tot;
    }
    __syncthreads();
    if (leader) wcnt[wv][dg] = 0u;
    __syncthreads();
  }
  // the tile in digit order: position q of digit d goes to gstart[d] + q - lstart[d]
  for (int q = threadIdx.x; q < len; q += RS_THREADS) {
    const uint32_t d = (rs_stage[word * RS_TILE + q] >> shift) & 255u;
    const uint32_t pos = gstart[d] + (uint32_t)q - lstart[d];
#pragma unroll
    for (int w = 0; w < 4; ++w)
      if (w < W) out.k[w][pos] = rs_stage[w * RS_TILE + q];
    if (out.v) out.v[pos] = in.v ? rs_stage[W * RS_TILE + q] : 0u;
  }
}

size_t radix_tmp_words(int64_t n) {
  const int64_t nblk = (n + RS_TILE - 1) / RS_TILE;
  return (size_t)(256 * nblk) + exscan_tmp_words(256 * nblk) + 16;
}

// Sorts by the listed (word, shift) digits, least significant first.
// Returns 1 if the sorted data ended in `alt`, 0 if in `buf`.
int radix_sort(RsView buf, RsView alt, int W, int64_t n, const int* words, const int* shifts, int npass,
               uint32_t* tmp, hipStream_t s) {
  return radix_sort_dn(buf, alt, W, n, nullptr, words, shifts, npass, tmp, s);
}

int radix_sort_dn(RsView buf, RsView alt, int W, int64_t n, const uint32_t* n_dev, const int* words,
                  const int* shifts, int npass, uint32_t* tmp, hipStream_t s) {
  if (n <= 0 || npass == 0) return 0;
  const int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
  uint32_t* hist = tmp;
  uint32_t* stmp = tmp + (size_t)256 * nblk;
  RsView a = buf, b = alt;
  for (int p = 0; p < npass; ++p) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(RS_THREADS), 0, s, a.k[words[p]], n, n_dev, shifts[p],
                       hist, nblk);
    exscan_u32(hist, hist, (int64_t)256 * nblk, stmp, nullptr, s);
    const size_t stage = sizeof(uint32_t) * RS_TILE * (size_t)(W + (a.v ? 1 : 0));
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(RS_THREADS), stage, s, a, b, W, n, n_dev, words[p],
                       shifts[p], hist, nblk);
    RsView t = a;
    a = b;
    b = t;
  }
  return npass & 1;
}

}  // namespace geek
