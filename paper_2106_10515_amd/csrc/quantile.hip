// Quantile bucketing of dense data (paper Algorithm 1): for each projection
// a_p, the objects are ranked by the QALSH value a_p . x_i (ties by id) and
// the ranks split evenly into t buckets, rank r going to bucket
// floor(r t / n).  Per table: exact float64 values (the attributes summed in
// order, one rounding per addition, products exact), a stable LSD radix sort
// of the values' order-preserving 64-bit patterns carrying the ids (so equal
// values keep id order), each object's bucket from its rank, and a second
// stable sort of the ids by bucket, which lists every bucket's members in
// ascending id.  Bucket b starts at rank ceil(b n / t).
#include <math.h>

#include "common.hpp"
#include "radix.hpp"

namespace geek {

constexpr int QV_ROWS = 64;     // rows of X staged in LDS per block
constexpr int QV_THREADS = 256;
constexpr int QV_MAXD = 256;

// values of one projection for QV_ROWS rows: the rows are staged in LDS
// (coalesced), then each of the first QV_ROWS threads sums one row's products
// in attribute order; the value is written as an order-preserving pattern
// (negative values complemented, positive ones with the sign bit set; -0
// becomes +0 so that equal values compare equal)
__global__ __launch_bounds__(QV_THREADS) void k_qv(const float* __restrict__ X, int64_t ldx, int64_t n, int d,
                                                   const float* __restrict__ a, uint32_t* __restrict__ klo,
                                                   uint32_t* __restrict__ khi, uint32_t* __restrict__ ids,
                                                   int32_t* st) {
  __shared__ float xs[QV_ROWS][QV_MAXD + 1];
  __shared__ float as[QV_MAXD];
  const int64_t i0 = (int64_t)blockIdx.x * QV_ROWS;
  for (int q = threadIdx.x; q < QV_ROWS * d; q += QV_THREADS) {
    const int r = q / d, c = q % d;
    xs[r][c] = i0 + r < n ? X[(i0 + r) * ldx + c] : 0.f;
  }
  for (int c = threadIdx.x; c < d; c += QV_THREADS) as[c] = a[c];
  __syncthreads();
  const int r = threadIdx.x;
  if (r >= QV_ROWS || i0 + r >= n) return;
  double s = 0.0;
  bool finite = true;
  for (int c = 0; c < d; ++c) {
    const float xv = xs[r][c];
    finite = finite && isfinite(xv) && isfinite(as[c]);
    s = __fma_rn((double)as[c], (double)xv, s);
  }
  if (!finite) set_status(st, GEEK_ERR_NONFINITE);
  s = s + 0.0;  // -0 -> +0
  uint64_t u = (uint64_t)__double_as_longlong(s);
  u = (u >> 63) ? ~u : (u | 0x8000000000000000ull);
  klo[i0 + r] = (uint32_t)u;
  khi[i0 + r] = (uint32_t)(u >> 32);
  ids[i0 + r] = (uint32_t)(i0 + r);
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

// bucket b starts at rank ceil(b n / t)
__global__ void k_q_offsets(int64_t n, int t, uint32_t* __restrict__ off) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b > t) return;
  off[b] = (uint32_t)(((uint64_t)b * (uint64_t)n + (uint64_t)t - 1) / (uint64_t)t);
}

struct QWs {
  uint32_t *klo, *khi, *ids, *klo2, *khi2, *ids2, *rtmp;
};

static size_t carve_q(int64_t n, void* base, QWs& W) {
  Carver c(base);
  W.klo = c.take<uint32_t>(n);
  W.khi = c.take<uint32_t>(n);
  W.ids = c.take<uint32_t>(n);
  W.klo2 = c.take<uint32_t>(n);
  W.khi2 = c.take<uint32_t>(n);
  W.ids2 = c.take<uint32_t>(n);
  W.rtmp = c.take<uint32_t>(radix_tmp_words(n));
  return c.used + 256;
}

size_t quantile_ws(const geek_quantile_job& J) {
  QWs W;
  return carve_q(J.n, nullptr, W);
}

int32_t quantile_run(const geek_quantile_job& J, void* ws, int32_t* st, hipStream_t s) {
  QWs W;
  carve_q(J.n, ws, W);
  const int grid = ceil_div(J.n, 256);
  for (int p = 0; p < J.m; ++p) {
    uint32_t* members = J.members + (int64_t)p * J.n;
    uint32_t* bof = J.bucket_of ? J.bucket_of + (int64_t)p * J.n : nullptr;
    hipLaunchKernelGGL(k_qv, dim3(ceil_div(J.n, QV_ROWS)), dim3(QV_THREADS), 0, s, J.X, J.ldx, J.n, J.d,
                       J.A + (int64_t)p * J.d, W.klo, W.khi, W.ids, st);
    // 64-bit value patterns, least significant byte first; ties keep id order
    const int words[8] = {0, 0, 0, 0, 1, 1, 1, 1}, shifts[8] = {0, 8, 16, 24, 0, 8, 16, 24};
    RsView A{{W.klo, W.khi, nullptr, nullptr}, W.ids}, B{{W.klo2, W.khi2, nullptr, nullptr}, W.ids2};
    const int alt = radix_sort(A, B, 2, J.n, words, shifts, 8, W.rtmp, s);
    const uint32_t* sorted_ids = alt ? W.ids2 : W.ids;
    // second sort: ids in id order keyed by bucket (klo2 / ids2 free again
    // when the sorted ids are in ids, and vice versa)
    uint32_t* bkey = alt ? W.klo : W.klo2;
    uint32_t* bid = alt ? W.ids : W.ids2;
    hipLaunchKernelGGL(k_q_rank, dim3(grid), dim3(256), 0, s, sorted_ids, J.n, J.t, bkey, bid, bof);
    int w2[4], s2[4], np = 0;
    for (int sh = 0; sh < 32 && ((uint32_t)(J.t - 1) >> sh) != 0u; sh += 8) {
      w2[np] = 0;
      s2[np++] = sh;
    }
    uint32_t* bkey2 = alt ? W.khi : W.khi2;
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
