// Quantile bucketing of dense data (paper Algorithm 1): for each projection
// a_p, the objects are ranked by the QALSH value a_p . x_i (ties by id) and
// the ranks split evenly into t buckets, rank r going to bucket
// floor(r t / n).  Exact float64 values of all tables first (the attributes
// summed in order, one rounding per addition, products exact; X read once
// per group of projections); then per table a stable LSD radix sort
// of the values' order-preserving 64-bit patterns carrying the ids (so equal
// values keep id order); then every bucket's ids in ascending order: sorted
// in LDS per bucket when buckets hold at most QS_MAX objects, else by a
// second stable sort of the ids keyed by bucket (rank-derived).  Bucket b
// starts at rank ceil(b n / t).
#include <math.h>

#include "common.hpp"
#include "radix.hpp"

namespace geek {

constexpr int QV_ROWS = 64;     // rows of X staged in LDS per block
constexpr int QV_THREADS = 256;
constexpr int QV_AFLOATS = 4096;  // projection values staged per launch (pm * d <= this)
constexpr int QV_ILP = 8;         // float64 chains per thread

// values of projections p0 .. p0 + pm - 1 for QV_ROWS rows: the rows and the
// projections are staged in LDS (X is read once per launch, not once per
// table; rows padded to a multiple of four attributes plus four), then each
// thread takes one row and the projections w, w + 4, w + 8, ... (w = its
// wave): up to QV_ILP independent float64 chains advance together, each in
// attribute order, four attributes per 16-byte LDS read (the projection
// reads are wave-uniform).  The value is written as an order-preserving
// pattern (negative values complemented, positive ones with the sign bit
// set; -0 becomes +0 so that equal values compare equal) into the table's
// key words.
__global__ __launch_bounds__(QV_THREADS) void k_qv(const float* __restrict__ X, int64_t ldx, int64_t n, int d,
                                                   const float* __restrict__ A, int p0, int pm,
                                                   uint32_t* __restrict__ klo, uint32_t* __restrict__ khi,
                                                   int32_t* st) {
  extern __shared__ __attribute__((aligned(16))) float qv_smem[];
  const int d4 = (d + 3) & ~3, xstr = d4 + 4;
  float* xs = qv_smem;                   // [QV_ROWS][xstr]
  float* as = qv_smem + QV_ROWS * xstr;  // [pm][d4]
  const int64_t i0 = (int64_t)blockIdx.x * QV_ROWS;
  for (int q = threadIdx.x; q < QV_ROWS * d4; q += QV_THREADS) {
    const int r = q / d4, c = q % d4;
    xs[r * xstr + c] = (i0 + r < n && c < d) ? X[(i0 + r) * ldx + c] : 0.f;
  }
  for (int q = threadIdx.x; q < pm * d4; q += QV_THREADS) {
    const int pp = q / d4, c = q % d4;
    as[q] = c < d ? A[(int64_t)(p0 + pp) * d + c] : 0.f;
  }
  __syncthreads();
  const int r = threadIdx.x % QV_ROWS, w = threadIdx.x / QV_ROWS;
  constexpr int NW = QV_THREADS / QV_ROWS;
  if (i0 + r >= n) return;
  const float* xr = xs + r * xstr;
  for (int pb = w; pb < pm; pb += NW * QV_ILP) {
    double acc[QV_ILP];
    bool finite = true;
#pragma unroll
    for (int u = 0; u < QV_ILP; ++u) acc[u] = 0.0;
    for (int c = 0; c < d4; c += 4) {
      const float4 xv = *reinterpret_cast<const float4*>(xr + c);
      finite = finite && isfinite(xv.x) && isfinite(xv.y) && isfinite(xv.z) && isfinite(xv.w);
#pragma unroll
      for (int u = 0; u < QV_ILP; ++u) {
        const int pp = pb + u * NW < pm ? pb + u * NW : pm - 1;  // repeats are not written
        const float4 av = *reinterpret_cast<const float4*>(as + pp * d4 + c);
        finite = finite && isfinite(av.x) && isfinite(av.y) && isfinite(av.z) && isfinite(av.w);
        // attributes past d are zero on both sides: exact zero products
        acc[u] = __fma_rn((double)av.x, (double)xv.x, acc[u]);
        acc[u] = __fma_rn((double)av.y, (double)xv.y, acc[u]);
        acc[u] = __fma_rn((double)av.z, (double)xv.z, acc[u]);
        acc[u] = __fma_rn((double)av.w, (double)xv.w, acc[u]);
      }
    }
    if (!finite) set_status(st, GEEK_ERR_NONFINITE);
#pragma unroll
    for (int u = 0; u < QV_ILP; ++u) {
      const int pp = pb + u * NW;
      if (pp >= pm) break;
      const double sv = acc[u] + 0.0;  // -0 -> +0
      uint64_t uv = (uint64_t)__double_as_longlong(sv);
      uv = (uv >> 63) ? ~uv : (uv | 0x8000000000000000ull);
      const int64_t o = (int64_t)(p0 + pp) * n + i0 + r;
      klo[o] = (uint32_t)uv;
      khi[o] = (uint32_t)(uv >> 32);
    }
  }
}

__global__ void k_q_iota(int64_t n, uint32_t* __restrict__ ids) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) ids[q] = (uint32_t)q;
}

// bucket of every object from its rank; the id-ordered bucket keys and ids
// feed the second sort
__global__ void k_q_rank(const uint32_t* __restrict__ sorted_ids, int64_t n, int t, uint32_t* __restrict__ bkey,
                         uint32_t* __restrict__ ids, uint32_t* __restrict__ bucket_of) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint32_t i = sorted_ids[r];
  const uint32_t b = (uint32_t)((uint64_t)r * (uint64_t)t / (uint64_t)n);
  bkey[i] = b;
  ids[r] = (uint32_t)r;  // id order for the second sort (position r holds id r)
  if (bucket_of) bucket_of[i] = b;
}

__global__ void k_q_copy(const uint32_t* __restrict__ src, int64_t n, uint32_t* __restrict__ dst) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) dst[q] = src[q];
}

// Buckets of at most QS_MAX objects: bucket b's ids (ranks ceil(b n / t) ..
// ceil((b + 1) n / t) - 1 of the value order) are sorted ascending in LDS
// (bitonic, padded with ~0) and written as its members; bucket_of is
// scattered from the same LDS copy.  One workgroup per bucket.
constexpr int QS_MAX = 4096;
__global__ __launch_bounds__(256) void k_q_segsort(const uint32_t* __restrict__ sorted_ids, int64_t n, int t,
                                                   uint32_t* __restrict__ members, uint32_t* __restrict__ bucket_of) {
  __shared__ uint32_t v[QS_MAX];
  const int b = blockIdx.x;
  const int64_t s0 = ((uint64_t)b * (uint64_t)n + (uint64_t)t - 1) / (uint64_t)t;
  const int64_t s1 = ((uint64_t)(b + 1) * (uint64_t)n + (uint64_t)t - 1) / (uint64_t)t;
  const int len = (int)(s1 - s0);
  int P = 1;
  while (P < len) P <<= 1;
  for (int q = threadIdx.x; q < P; q += blockDim.x) v[q] = q < len ? sorted_ids[s0 + q] : 0xFFFFFFFFu;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = threadIdx.x; q < P; q += blockDim.x) {
        const int o = q ^ j;
        if (o > q) {
          const uint32_t a = v[q], c = v[o];
          const bool up = (q & k) == 0;
          if ((a > c) == up) {
            v[q] = c;
            v[o] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int q = threadIdx.x; q < len; q += blockDim.x) {
    members[s0 + q] = v[q];
    if (bucket_of) bucket_of[v[q]] = (uint32_t)b;
  }
}

// bucket b starts at rank ceil(b n / t)
__global__ void k_q_offsets(int64_t n, int t, uint32_t* __restrict__ off) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b > t) return;
  off[b] = (uint32_t)(((uint64_t)b * (uint64_t)n + (uint64_t)t - 1) / (uint64_t)t);
}

struct QWs {
  uint32_t *klo, *khi;                  // [m][n] value patterns of every table
  uint32_t *ids, *klo2, *khi2, *ids2;   // [n] sort buffers of one table
  uint32_t* rtmp;
};

static size_t carve_q(const geek_quantile_job& J, void* base, QWs& W) {
  Carver c(base);
  W.klo = c.take<uint32_t>((size_t)J.m * J.n);
  W.khi = c.take<uint32_t>((size_t)J.m * J.n);
  W.ids = c.take<uint32_t>(J.n);
  W.klo2 = c.take<uint32_t>(J.n);
  W.khi2 = c.take<uint32_t>(J.n);
  W.ids2 = c.take<uint32_t>(J.n);
  W.rtmp = c.take<uint32_t>(radix_tmp_words(J.n));
  return c.used + 256;
}

size_t quantile_ws(const geek_quantile_job& J) {
  QWs W;
  return carve_q(J, nullptr, W);
}

int32_t quantile_run(const geek_quantile_job& J, void* ws, int32_t* st, hipStream_t s) {
  QWs W;
  carve_q(J, ws, W);
  const int grid = ceil_div(J.n, 256);
  // values of all tables, as many projections per pass over X as the
  // staging area holds
  const int d4 = (J.d + 3) & ~3;
  const int per = QV_AFLOATS / d4;
  for (int p0 = 0; p0 < J.m; p0 += per) {
    const int pm = J.m - p0 < per ? J.m - p0 : per;
    const size_t lds = sizeof(float) * ((size_t)QV_ROWS * (d4 + 4) + (size_t)pm * d4);
    hipLaunchKernelGGL(k_qv, dim3(ceil_div(J.n, QV_ROWS)), dim3(QV_THREADS), lds, s, J.X, J.ldx, J.n, J.d, J.A,
                       p0, pm, W.klo, W.khi, st);
  }
  for (int p = 0; p < J.m; ++p) {
    uint32_t* members = J.members + (int64_t)p * J.n;
    uint32_t* bof = J.bucket_of ? J.bucket_of + (int64_t)p * J.n : nullptr;
    uint32_t* klo = W.klo + (int64_t)p * J.n;
    uint32_t* khi = W.khi + (int64_t)p * J.n;
    hipLaunchKernelGGL(k_q_iota, dim3(grid), dim3(256), 0, s, J.n, W.ids);
    // 64-bit value patterns, least significant byte first; ties keep id order
    const int words[8] = {0, 0, 0, 0, 1, 1, 1, 1}, shifts[8] = {0, 8, 16, 24, 0, 8, 16, 24};
    RsView A{{klo, khi, nullptr, nullptr}, W.ids}, B{{W.klo2, W.khi2, nullptr, nullptr}, W.ids2};
    const int alt = radix_sort(A, B, 2, J.n, words, shifts, 8, W.rtmp, s);
    const uint32_t* sorted_ids = alt ? W.ids2 : W.ids;
    if ((J.n + J.t - 1) / J.t <= QS_MAX) {  // every bucket fits one workgroup's LDS
      hipLaunchKernelGGL(k_q_segsort, dim3(J.t), dim3(256), 0, s, sorted_ids, J.n, J.t, members, bof);
      hipLaunchKernelGGL(k_q_offsets, dim3(ceil_div((int64_t)J.t + 1, 256)), dim3(256), 0, s, J.n, J.t,
                         J.offsets + (int64_t)p * (J.t + 1));
      continue;
    }
    // second sort: ids in id order keyed by bucket, in the buffers the first
    // sort's result does not occupy (the table's own key words are free now)
    uint32_t* bkey = alt ? klo : W.klo2;
    uint32_t* bid = alt ? W.ids : W.ids2;
    hipLaunchKernelGGL(k_q_rank, dim3(grid), dim3(256), 0, s, sorted_ids, J.n, J.t, bkey, bid, bof);
    int w2[4], s2[4], np = 0;
    for (int sh = 0; sh < 32 && ((uint32_t)(J.t - 1) >> sh) != 0u; sh += 8) {
      w2[np] = 0;
      s2[np++] = sh;
    }
    uint32_t* bkey2 = alt ? khi : W.khi2;
    uint32_t* bid2 = alt ? W.ids2 : W.ids;
    RsView C{{bkey, nullptr, nullptr, nullptr}, bid}, D{{bkey2, nullptr, nullptr, nullptr}, bid2};
    const int alt2 = radix_sort(C, D, 1, J.n, w2, s2, np, W.rtmp, s);
    hipLaunchKernelGGL(k_q_copy, dim3(grid), dim3(256), 0, s, alt2 ? bid2 : bid, J.n, members);
    hipLaunchKernelGGL(k_q_offsets, dim3(ceil_div((int64_t)J.t + 1, 256)), dim3(256), 0, s, J.n, J.t,
                       J.offsets + (int64_t)p * (J.t + 1));
  }
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
