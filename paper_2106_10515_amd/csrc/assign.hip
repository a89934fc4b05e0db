// One-pass data assignment (paper Section 3.3, Eq. (1)) on gfx950.
//
// Pipeline for Euclidean data (all stream-ordered, no host synchronization):
//   k_centroids   float64 centroids, one thread per (seed, dim), members summed
//                 in ascending order one rounding at a time (exact parity),
//                 their values loaded 32 at a time.
//   k_cprep       centroid copies in the matrix-core input type (fp32 / bf16),
//                 |c|^2 and max |c| for the error bound.
//   k_scan<M,DP>  matrix-core tile |x|^2 - 2 x.c + |c|^2 over all centroids for
//                 a block of rows.  Float32: per row it keeps every centroid
//                 whose approximate distance lies within 2*eps_i of the
//                 running minimum (eps_i a rigorous bound of the approximation
//                 error), up to TCAND candidates (TCAND32 in the rescan of
//                 ambiguous rows).  The BF16 first pass keeps only the best
//                 and second-best values (branch-free); a row is settled when
//                 the runner-up lies beyond 2*eps_i, else it is rescanned in
//                 float32.  FP8 keeps a TCAND window like float32.
//   k_finalize    float64 distance (the reference formula, same operation
//                 order) for each candidate; lowest index wins exact ties.
//                 Rows whose candidate window overflowed are escalated.
//   k_fallback64  float64 distance to every centroid for the rows left
//                 (64 x 64 row-seed tiles, split over workgroups for few rows).
//   k_sse_*       SSE in fixed 4096-row blocks; radius per cluster.
//
// Heterogeneous rows (numeric attributes + categorical attributes) use the
// same pipeline with D = D_num + gamma * #mismatching attributes: the
// mismatch count is exact and added in the scan epilogue; the categorical
// central vector is the per-attribute mode (assign_sig.hip computes modes).
#include <math.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "scan.hpp"

namespace geek {

constexpr int SSE_BLOCK = 4096;

// ---------------------------------------------------------------- centroids
// The sum over a seed's members is one chain of float64 additions (the
// reference order), so a seed with many members is bound by memory latency:
// members are taken CB at a time, their values loaded together (the next
// batch's ids already in flight), then added in order.
constexpr int CB = 32;
__global__ void k_centroids(const float* __restrict__ X, int64_t ldx, int64_t n, int d,
                            const uint32_t* __restrict__ offs, const uint32_t* __restrict__ mem,
                            int k, const uint32_t* __restrict__ kdev, double* __restrict__ C, int32_t* st) {
  int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)k * d) return;
  int j = (int)(gid / d), t = (int)(gid % d);
  // seeds counted on the device: those past the count take no part
  const int kv = kdev ? (int)min(*kdev, (uint32_t)k) : k;
  if (j >= kv) {
    if (kv == 0 && gid == 0) set_status(st, GEEK_ERR_NO_SEEDS);
    C[gid] = 0.0;
    return;
  }
  uint32_t s = offs[j], e = offs[j + 1];
  if (e <= s) {
    set_status(st, GEEK_ERR_EMPTY_SET);
    C[gid] = 0.0;
    return;
  }
  double acc = 0.0;
  bool bad = false;
  // ids of member q (clamped into the seed's range: reads past the end are
  // repeated ids whose values are not added)
  auto id_at = [&](uint32_t q) { return mem[q < e ? q : e - 1]; };
  uint32_t ids[CB];
#pragma unroll
  for (int u = 0; u < CB; ++u) ids[u] = id_at(s + u);
  for (uint32_t q = s; q < e; q += CB) {
    float v[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      const bool ok = (int64_t)ids[u] < n;
      bad |= !ok;
      v[u] = X[(int64_t)(ok ? ids[u] : 0u) * ldx + t];
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) ids[u] = id_at(q + CB + u);
    const uint32_t cnt = e - q < (uint32_t)CB ? e - q : (uint32_t)CB;
#pragma unroll
    for (int u = 0; u < CB; ++u)
      if ((uint32_t)u < cnt) acc = __dadd_rn(acc, (double)v[u]);
  }
  if (bad) set_status(st, GEEK_ERR_ARG);
  C[gid] = acc / (double)(e - s);
}

// Seeds with many members (a further assignment pass takes whole clusters
// as seeds): the members' values are first gathered into groups of four
// member positions, Xt[q / 4][t][q % 4] = X[mem[q]][t] (a 64 x 64 tile
// transposed through LDS), so that the (seed, dim) chains of one wave read
// four values each per 16-byte load, the wave's loads one contiguous run:
// streaming, where loads of whole rows of scattered members (or of
// dimension-major rows far apart) were bound by address translation.
constexpr int GT_TILE = 64;
__global__ __launch_bounds__(256) void k_gather_t(const float* __restrict__ X, int64_t ldx, int64_t n, int d,
                                                  const uint32_t* __restrict__ offs, int k,
                                                  const uint32_t* __restrict__ mem, int64_t nm_cap, int64_t nm_pad,
                                                  float* __restrict__ Xt, int32_t* st) {
  __shared__ float tile[GT_TILE][GT_TILE + 1];
  // members actually used (seed_offsets[k]); positions past them are zeros
  const int64_t nm = offs[k] < nm_cap ? (int64_t)offs[k] : nm_cap;
  const int64_t q0 = (int64_t)blockIdx.x * GT_TILE;
  const int t0 = blockIdx.y * GT_TILE;
  const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
#pragma unroll 4
  for (int r = r0; r < GT_TILE; r += 4) {
    const int64_t q = q0 + r;
    float v = 0.f;
    if (q < nm && t0 + c < d) {
      const uint32_t i = mem[q];
      if ((int64_t)i < n) v = X[(int64_t)i * ldx + t0 + c];
      else set_status(st, GEEK_ERR_ARG);
    }
    tile[r][c] = v;
  }
  __syncthreads();
  // group g of the tile (members q0 + 4g .. + 3) covers the contiguous run
  // Xt[(q0 / 4 + g) * 4 d + 4 t0 ..] of 4 x 64 values: thread i writes its
  // element i of the run
#pragma unroll 4
  for (int i = threadIdx.x; i < GT_TILE * GT_TILE; i += 256) {
    const int g = i >> 8, rem = i & 255, tl = rem >> 2, r = rem & 3;
    const int64_t q = q0 + g * 4 + r;
    if (q < nm_pad && t0 + tl < d) Xt[(q >> 2) * 4 * (int64_t)d + (int64_t)(t0 + tl) * 4 + r] = tile[g * 4 + r][tl];
  }
}

// Centroids from the grouped copy: the same ascending chain of float64
// additions as k_centroids.
constexpr int CT_B = 16;  // 16-byte loads in flight per batch (64 members)
__global__ void k_centroids_t(const float* __restrict__ Xt, int64_t nm, int d,
                              const uint32_t* __restrict__ offs, int k, double* __restrict__ C, int32_t* st) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)k * d) return;
  const int j = (int)(gid / d), t = (int)(gid % d);
  const int64_t s = offs[j], e = offs[j + 1];
  if (e <= s) {
    set_status(st, GEEK_ERR_EMPTY_SET);
    C[gid] = 0.0;
    return;
  }
  if (e > nm) {  // seed_offsets disagree with the member count of the job
    set_status(st, GEEK_ERR_ARG);
    C[gid] = 0.0;
    return;
  }
  const int64_t gs = 4 * (int64_t)d;  // floats per group of four members
  const float* p = Xt + (int64_t)t * 4;
  auto at = [&](int64_t q) { return p[(q >> 2) * gs + (q & 3)]; };
  double acc = 0.0;
  int64_t q = s;
  for (; q < e && (q & 3); ++q) acc = __dadd_rn(acc, (double)at(q));
  for (; q + 4 * CT_B <= e; q += 4 * CT_B) {
    float4 v[CT_B];
#pragma unroll
    for (int u = 0; u < CT_B; ++u) v[u] = *reinterpret_cast<const float4*>(p + ((q >> 2) + u) * gs);
#pragma unroll
    for (int u = 0; u < CT_B; ++u) {
      acc = __dadd_rn(acc, (double)v[u].x);
      acc = __dadd_rn(acc, (double)v[u].y);
      acc = __dadd_rn(acc, (double)v[u].z);
      acc = __dadd_rn(acc, (double)v[u].w);
    }
  }
  for (; q < e; ++q) acc = __dadd_rn(acc, (double)at(q));
  C[gid] = acc / (double)(e - s);
}

// Whether the centroids go through the dimension-major copy: seeds of 64
// members or more on average, with the member count known.
static bool centroids_transposed(const geek_assign_job& J) {
  return !J.k_dev && J.n_members > 0 && J.n_members >= 64 * (int64_t)J.k;
}
static int64_t members_pad(const geek_assign_job& J) { return (J.n_members + 3) / 4 * 4; }

// Largest |value| of a float32 matrix / float64 centroids (FP8 scaling).
__global__ void k_absmax_x(const float* __restrict__ X, int64_t ldx, int64_t n, int d, float* __restrict__ out) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  float m = 0.f;
  for (int64_t e = g; e < n * d; e += (int64_t)gridDim.x * blockDim.x) {
    const float v = fabsf(X[(e / d) * ldx + (e % d)]);
    if (v > m) m = v;  // NaN compares false and is ignored here
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(out, m);
}

__global__ void k_absmax_c(const double* __restrict__ C, int64_t kd, float* __restrict__ out) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  float m = 0.f;
  for (int64_t e = g; e < kd; e += (int64_t)gridDim.x * blockDim.x) m = fmaxf(m, (float)fabs(C[e]) * 1.0001f);
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomic_max_nonneg(out, m);
}

// scale = 2^floor(log2(224 / max)), so scaled values stay inside every
// e4m3 variant's normal range; 1 when everything is zero.
__global__ void k_fp8_scale(const float* __restrict__ mx, const float* __restrict__ mc, float* __restrict__ scale) {
  if (blockIdx.x || threadIdx.x) return;
  const float m = fmaxf(*mx, *mc);
  // 2^e with max |value| * 2^e in [112, 224]; e is clamped at 60 for tiny
  // data (the absolute error term covers it); data too large for a safe
  // 2^e gets scale 0, which makes every row's bound infinite (escalation)
  if (!(m > 0.f)) {
    *scale = 1.0f;
    return;
  }
  const float e = floorf(log2f(224.0f / m));
  *scale = e < -60.f ? 0.0f : exp2f(fminf(e, 60.f));
}

// Matrix-core input copies of the centroids, zero-padded to [k_pad][DP];
// padded rows get |c|^2 = +inf so they never enter a window.
template <class M>
__global__ void k_cprep(const double* __restrict__ C, int k, int d, int k_pad, int DP,
                        typename M::ce* __restrict__ cl, float* __restrict__ nc, float* __restrict__ cmax,
                        const float* __restrict__ scale_p, const uint32_t* __restrict__ kdev) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k_pad) return;
  const float sc = M::SCALED ? *scale_p : 1.0f;
  // seeds past a device-side count are padding too
  if (j >= (kdev ? (int)min(*kdev, (uint32_t)k) : k)) {
    for (int t = 0; t < DP; t += M::KPER) M::store_zero(cl + (int64_t)j * DP + t);
    if (nc) nc[j] = INFINITY;
    return;
  }
  double sq = 0.0;
  float v[M::KPER];
  for (int t = 0; t < DP; t += M::KPER) {
#pragma unroll
    for (int e = 0; e < M::KPER; ++e) {
      const double c = t + e < d ? C[(int64_t)j * d + t + e] : 0.0;
      sq = __dadd_rn(sq, __dmul_rn(c, c));
      v[e] = (float)c;
    }
    M::store(cl + (int64_t)j * DP + t, v, sc);
  }
  if (nc) {
    nc[j] = (float)sq;
    atomic_max_nonneg(cmax, (float)(sqrt(sq) * (1.0 + 0x1p-20)));
  }
}

// Two workgroups per CU (at most 256 registers a wavefront) for the BF16
// first pass of point rows up to 128 attributes, whose stage pipeline keeps
// two blocks' accumulators live; the compiler would otherwise go just past
// 256 and halve the occupancy.
template <class M, int DP, bool HET, int NCB>
constexpr int scan_min_blocks() {
  return (std::is_same<M, ModeBF16>::value && !HET && NCB == 2 && DP <= 128) ? 2 : 1;
}

template <class M, int DP, bool HET, int NCB, int NBUF, bool T2, bool WIDE>
__global__ __launch_bounds__(SCAN_THREADS, (scan_min_blocks<M, DP, HET, NCB>())) void k_scan(
    const float* __restrict__ X, int64_t ldx, int d, int64_t n_rows,
    const uint32_t* __restrict__ rows, const uint32_t* __restrict__ rows_count,
    const typename M::ce* __restrict__ cl, const float* __restrict__ nc, int k_pad,
    const float* __restrict__ cmax_p, const float* __restrict__ scale_p, Het het, int k,
    int32_t* __restrict__ rec, int32_t* st) {
  scan_tiles<M, DP, HET, NCB, NBUF, T2, WIDE>(X, ldx, d, n_rows, rows, rows_count, cl, nc, k_pad, cmax_p, scale_p, het,
                                        k, rec, st, blockIdx.x, INT64_MAX, gridDim.x);
}

constexpr int SCANJOB_CHUNK = 32;  // table entries written per launch
struct ScanJobChunk {
  int count;
  ScanJob jobs[SCANJOB_CHUNK];
};
__global__ void k_put_jobs(ScanJobChunk c, ScanJob* dst) {
  const int i = threadIdx.x;
  if (i < c.count) dst[i] = c.jobs[i];
}

__global__ void k_clock_since(const unsigned long long* t0, unsigned long long* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = wall_clock64() - *t0;
}
__global__ void k_clock_now(unsigned long long* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = wall_clock64();
}

// ---------------------------------------------------------------- float64 checks
// Categorical attributes of row i that differ from seed j's modes.
GEEK_D int mismatches(const Het& het, int64_t i, int j) {
  int mm = 0;
  for (int a = 0; a < het.n_cat; ++a)
    mm += ((uint32_t)het.cat[i * het.n_cat + a] != het.mode[(int64_t)j * het.n_cat + a]) ? 1 : 0;
  return mm;
}

GEEK_D double d64(const float* __restrict__ xr, const double* __restrict__ cr, int d) {
  double acc = 0.0;
  int t = 0;
  // 16-byte loads when both rows are aligned; the summation order is
  // unchanged.  32 attributes at a time: the 24 loads of one x cache line
  // and two centroid lines are issued before the first use, one memory round
  // trip per 32 attributes
  if (((reinterpret_cast<uintptr_t>(xr) | reinterpret_cast<uintptr_t>(cr)) & 15) == 0) {
    for (; t + 32 <= d; t += 32) {
      float4 xv[8];
      double2 cv[16];
#pragma unroll
      for (int u = 0; u < 8; ++u) xv[u] = *reinterpret_cast<const float4*>(xr + t + 4 * u);
#pragma unroll
      for (int u = 0; u < 16; ++u) cv[u] = *reinterpret_cast<const double2*>(cr + t + 2 * u);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float xs[4] = {xv[u].x, xv[u].y, xv[u].z, xv[u].w};
        const double cs[4] = {cv[2 * u].x, cv[2 * u].y, cv[2 * u + 1].x, cv[2 * u + 1].y};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double delta = __dadd_rn((double)xs[e], -cs[e]);
          acc = __dadd_rn(acc, __dmul_rn(delta, delta));
        }
      }
    }
    for (; t + 4 <= d; t += 4) {
      const float4 xv = *reinterpret_cast<const float4*>(xr + t);
      const double2 c0 = *reinterpret_cast<const double2*>(cr + t);
      const double2 c1 = *reinterpret_cast<const double2*>(cr + t + 2);
      double delta = __dadd_rn((double)xv.x, -c0.x);
      acc = __dadd_rn(acc, __dmul_rn(delta, delta));
      delta = __dadd_rn((double)xv.y, -c0.y);
      acc = __dadd_rn(acc, __dmul_rn(delta, delta));
      delta = __dadd_rn((double)xv.z, -c1.x);
      acc = __dadd_rn(acc, __dmul_rn(delta, delta));
      delta = __dadd_rn((double)xv.w, -c1.y);
      acc = __dadd_rn(acc, __dmul_rn(delta, delta));
    }
  }
  for (; t < d; ++t) {
    const double delta = __dadd_rn((double)xr[t], -cr[t]);
    acc = __dadd_rn(acc, __dmul_rn(delta, delta));
  }
  return acc;
}

// D_num + gamma * mismatches, in that float64 order (reference formula).
GEEK_D double d64h(const float* __restrict__ xr, const double* __restrict__ cr, int d, const Het& het,
                   int64_t i, int j) {
  const double dn = d64(xr, cr, d);
  if (!het.cat) return dn;
  return __dadd_rn(dn, __dmul_rn(het.gamma, (double)mismatches(het, i, j)));
}

__device__ void block_add_u64(unsigned long long* dst, unsigned long long v) {
  // one atomic per wave
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

// Candidate windows (RECW records: the FP8 and float32 first passes, the
// rescans): a lane per row, each lane walking its own row's candidates.
__global__ void k_finalize_win(const float* __restrict__ X, int64_t ldx, int d,
                           const double* __restrict__ C, int k, Het het, int64_t n_rows,
                           const uint32_t* __restrict__ rows, const uint32_t* __restrict__ rows_count,
                           const int32_t* __restrict__ rec, int rstride, int32_t* __restrict__ assign,
                           double* __restrict__ dist, uint32_t* __restrict__ esc,
                           uint32_t* __restrict__ esc_count, unsigned long long* __restrict__ ctr,
                           int ctr_rows) {
  const int64_t count = rows ? (int64_t)*rows_count : n_rows;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t iters = (count + stride - 1) / stride;
  unsigned long long nrow = 0, ncand = 0;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t pos = start + it * stride;
    if (pos >= count) continue;
    const int64_t i = rows ? (int64_t)rows[pos] : pos;
    const int32_t* rr = rec + pos * rstride;
    const int c = rr[0];
    if (c <= 0) {  // window overflow (or no finite candidate): escalate
      const uint32_t q = atomicAdd(esc_count, 1u);
      esc[q] = (uint32_t)i;
      continue;
    }
    double best = INFINITY;
    int bj = 0x7fffffff;
    const float* xr = X + i * ldx;
    for (int q = 0; q < c; ++q) {
      const int j = rr[1 + q];
      if ((unsigned)j >= (unsigned)k) continue;
      const double D = d64h(xr, C + (int64_t)j * d, d, het, i, j);
      if (D < best || (D == best && j < bj)) {
        best = D;
        bj = j;
      }
    }
    if (bj == 0x7fffffff) bj = 0;
    assign[i] = bj;
    dist[i] = best;
    nrow += 1;
    ncand += (unsigned long long)c;
  }
  if (ctr) {
    block_add_u64(ctr + ctr_rows, nrow);
    block_add_u64(ctr + 3, ncand);
  }
}

// The BF16 first pass's records (RECW_T2: at most one candidate).  Eight
// lanes per row:
// lane e loads attributes t0 + 4e .. t0 + 4e + 3 of the row and of the
// candidate centroid for t0 = 0, 32, ... (one x cache line and two centroid
// lines per step, coalesced over the eight lanes), forms the rounded
// squared differences, and lane 0 of the eight adds the 32 squares of a step
// in attribute order from LDS: D = sum over t = 0..d-1 in order of
// (x_t - c_t)^2, each difference, square and sum rounded to float64 (plus
// gamma * mismatches for heterogeneous rows).  With a lane per row, every
// load touched 64 cache lines and the lines were evicted between the row's
// steps.
constexpr int FZ_ROWS = 8;   // rows per wavefront and step
constexpr int FZ_STEP = 32;  // attributes per step
__global__ __launch_bounds__(256) void k_finalize(const float* __restrict__ X, int64_t ldx, int d,
                                                  const double* __restrict__ C, int k, Het het, int64_t n_rows,
                                                  const uint32_t* __restrict__ rows,
                                                  const uint32_t* __restrict__ rows_count,
                                                  const int32_t* __restrict__ rec, int rstride,
                                                  int32_t* __restrict__ assign, double* __restrict__ dist,
                                                  uint32_t* __restrict__ esc, uint32_t* __restrict__ esc_count,
                                                  unsigned long long* __restrict__ ctr, int ctr_rows) {
  __shared__ double sq[4][FZ_ROWS][FZ_STEP + 2];  // + 2: the eight row leaders read distinct banks
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 3, e = lane & 7;  // row slot, lane within the row
  const int64_t count = rows ? (int64_t)*rows_count : n_rows;
  const int64_t stride = (int64_t)gridDim.x * 4 * FZ_ROWS;
  const bool xal = ((reinterpret_cast<uintptr_t>(X) | (uintptr_t)(ldx * 4)) & 15) == 0;
  const bool cal = ((reinterpret_cast<uintptr_t>(C) | (uintptr_t)(d * 8)) & 15) == 0;
  unsigned long long nrow = 0, ncand = 0;
  for (int64_t base = ((int64_t)blockIdx.x * 4 + wv) * FZ_ROWS; base < count; base += stride) {
    const int64_t pos = base + g;
    const bool live = pos < count;
    const int64_t i = live ? (rows ? (int64_t)rows[pos] : pos) : 0;
    const int32_t* rr = rec + (live ? pos : 0) * rstride;
    int c = live ? rr[0] : 0;
    if (live && c <= 0) {  // window overflow (or no finite candidate): escalate
      if (e == 0) esc[atomicAdd(esc_count, 1u)] = (uint32_t)i;
      c = 0;
    }
    int maxc = c;  // the wavefront walks the largest candidate count of its rows
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) maxc = max(maxc, __shfl_xor(maxc, o));
    double best = INFINITY;
    int bj = 0x7fffffff;
    const float* xr = X + i * ldx;
    for (int q = 0; q < maxc; ++q) {
      const int j = q < c ? rr[1 + q] : -1;
      const bool act = j >= 0 && j < k;
      const double* cr = C + (int64_t)(act ? j : 0) * d;
      double acc = 0.0;
      for (int t0 = 0; t0 < d; t0 += FZ_STEP) {
        const int t = t0 + 4 * e;
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        if (act && t < d) {
          float xs[4];
          double cs[4];
          if (xal && cal && t + 4 <= d) {
            const float4 xv = *reinterpret_cast<const float4*>(xr + t);
            const double2 c0 = *reinterpret_cast<const double2*>(cr + t);
            const double2 c1 = *reinterpret_cast<const double2*>(cr + t + 2);
            xs[0] = xv.x, xs[1] = xv.y, xs[2] = xv.z, xs[3] = xv.w;
            cs[0] = c0.x, cs[1] = c0.y, cs[2] = c1.x, cs[3] = c1.y;
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              xs[u] = t + u < d ? xr[t + u] : 0.f;
              cs[u] = t + u < d ? cr[t + u] : 0.0;
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double delta = __dadd_rn((double)xs[u], -cs[u]);
            s4[u] = __dmul_rn(delta, delta);
          }
        }
        *reinterpret_cast<double2*>(&sq[wv][g][4 * e]) = make_double2(s4[0], s4[1]);
        *reinterpret_cast<double2*>(&sq[wv][g][4 * e + 2]) = make_double2(s4[2], s4[3]);
        // the row's squares in attribute order (a wavefront's LDS accesses
        // complete in order, so the eight lanes' stores are visible here)
        if (e == 0 && act) {
          const int lim = d - t0 < FZ_STEP ? d - t0 : FZ_STEP;
          for (int u = 0; u < lim; ++u) acc = __dadd_rn(acc, sq[wv][g][u]);
        }
      }
      if (e == 0 && act) {
        const double D = het.cat ? __dadd_rn(acc, __dmul_rn(het.gamma, (double)mismatches(het, i, j))) : acc;
        if (D < best || (D == best && j < bj)) {
          best = D;
          bj = j;
        }
      }
    }
    if (e == 0 && live && c > 0) {
      if (bj == 0x7fffffff) bj = 0;
      assign[i] = bj;
      dist[i] = best;
      nrow += 1;
      ncand += (unsigned long long)c;
    }
  }
  if (ctr) {
    block_add_u64(ctr + ctr_rows, nrow);
    block_add_u64(ctr + 3, ncand);
  }
}

// Rows left after the rescans: float64 distance to every seed, lowest index on
// ties.  A workgroup takes FB_R rows and a range of FB_C-seed tiles; each
// thread holds a 4 x 4 block of (row, seed) sums with both operands staged in
// LDS, so one read of a seed row from L2 serves FB_R rows.  Every sum runs
// over t = 0..d-1 in order with the operations of d64 (the zero padding of
// t >= d adds +0.0, which leaves a sum of squares unchanged), so the values
// are those of the reference formula.  With fewer row groups than workgroups
// the seed tiles of a group are split over up to FB_SPLIT workgroups, whose
// per-row (D, j) minima k_fb_merge combines.
constexpr int FB_R = 64, FB_C = 64, FB_TK = 16, FB_GRID = 1024, FB_SPLIT = 16;
constexpr int FB_XS = FB_R + 4;  // LDS row stride (floats) of the staged rows
constexpr int FB_CS = FB_C + 2;  // LDS row stride (doubles) of a seed chunk

// Row groups and seed-tile splits for `count` rows against k seeds.
GEEK_HD void fb_shape(uint32_t count, int k, int64_t* R, int* S) {
  *R = ((int64_t)count + FB_R - 1) / FB_R;
  const int T = (k + FB_C - 1) / FB_C;
  int sp = 1;
  if (*R > 0 && *R < FB_GRID) {
    const int want = (int)((FB_GRID + *R - 1) / *R);
    sp = want < T ? want : T;
    if (sp > FB_SPLIT) sp = FB_SPLIT;
    if (sp < 1) sp = 1;
  }
  *S = sp;
}

// Capacity (entries) of the partial minima buffer for n rows.
inline int64_t fb_part_cap(int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>(n * FB_SPLIT, (int64_t)2 * FB_GRID * FB_R));
}

template <int DP>
__global__ __launch_bounds__(256) void k_fallback64(
    const float* __restrict__ X, int64_t ldx, int d, const double* __restrict__ C, int k,
    const uint32_t* __restrict__ kdev, Het het,
    const uint32_t* __restrict__ rows, const uint32_t* __restrict__ rows_count, int32_t* __restrict__ assign,
    double* __restrict__ dist, double* __restrict__ part_d, int32_t* __restrict__ part_j,
    unsigned long long* __restrict__ ctr) {
  constexpr int XS_WORDS = DP * FB_XS > FB_R * 16 * 3 ? DP * FB_XS : FB_R * 16 * 3;
  __shared__ __attribute__((aligned(16))) float xs[XS_WORDS];  // [t][row]; later the reduction
  __shared__ __attribute__((aligned(16))) double cs[FB_TK * FB_CS];  // [t][seed]
  __shared__ int64_t rid[FB_R];
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;  // rows 4tr..4tr+3, seeds 4tc..4tc+3 of a tile
  const uint32_t count = *rows_count;
  int64_t R;
  int S;
  fb_shape(count, k, &R, &S);
  const int T = (k + FB_C - 1) / FB_C;
  const int kv = kdev ? (int)min(*kdev, (uint32_t)k) : k;  // seeds that take part
  const int dp16 = (d + FB_TK - 1) / FB_TK * FB_TK;
  const int nch = dp16 / FB_TK;
  for (int64_t q = blockIdx.x; q < R * S; q += gridDim.x) {
    const int64_t g = q / S;
    const int sp = (int)(q % S);
    const int tile0 = (int)((int64_t)sp * T / S), tile1 = (int)((int64_t)(sp + 1) * T / S);
    __syncthreads();  // the previous item's reduction has read xs and rid
    if (tid < FB_R) {
      const int64_t pos = g * FB_R + tid;
      rid[tid] = pos < count ? (int64_t)rows[pos] : -1;
    }
    __syncthreads();
    for (int idx = tid; idx < FB_R * dp16; idx += 256) {
      const int r = idx / dp16, t = idx - r * dp16;
      const int64_t i = rid[r];
      xs[t * FB_XS + r] = (i >= 0 && t < d) ? X[i * ldx + t] : 0.f;
    }
    double best[4];
    int bj[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      best[a] = INFINITY;
      bj[a] = 0x7fffffff;
    }
    // register prefetch of the next (tile, chunk) of seeds
    double pre[4];
    auto fetch = [&](int tile, int ch) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int idx = tid + u * 256;
        const int jj = idx >> 4, tt = idx & 15;
        const int j = tile * FB_C + jj, t = ch * FB_TK + tt;
        pre[u] = (j < kv && t < d) ? C[(int64_t)j * d + t] : 0.0;
      }
    };
    if (tile0 < tile1) fetch(tile0, 0);
    for (int tile = tile0; tile < tile1; ++tile) {
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int ch = 0; ch < nch; ++ch) {
        __syncthreads();  // readers of the previous chunk are done (and xs is staged)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int idx = tid + u * 256;
          cs[(idx & 15) * FB_CS + (idx >> 4)] = pre[u];
        }
        __syncthreads();
        if (ch + 1 < nch) fetch(tile, ch + 1);
        else if (tile + 1 < tile1) fetch(tile + 1, 0);
        const float* xp = xs + ch * FB_TK * FB_XS + tr * 4;
        const double* cp = cs + tc * 4;
#pragma unroll 4
        for (int tt = 0; tt < FB_TK; ++tt) {
          const float4 xv = *reinterpret_cast<const float4*>(xp + tt * FB_XS);
          const double2 c01 = *reinterpret_cast<const double2*>(cp + tt * FB_CS);
          const double2 c23 = *reinterpret_cast<const double2*>(cp + tt * FB_CS + 2);
          const double xd[4] = {(double)xv.x, (double)xv.y, (double)xv.z, (double)xv.w};
          const double cd[4] = {c01.x, c01.y, c23.x, c23.y};
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const double delta = __dadd_rn(xd[a], -cd[b]);
              acc[a][b] = __dadd_rn(acc[a][b], __dmul_rn(delta, delta));
            }
        }
      }
      // j increases along this thread's sequence: strict < keeps the lowest
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int64_t i = rid[tr * 4 + a];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int j = tile * FB_C + tc * 4 + b;
          if (j >= kv) continue;
          double D = acc[a][b];
          if (het.cat && i >= 0) D = __dadd_rn(D, __dmul_rn(het.gamma, (double)mismatches(het, i, j)));
          if (D < best[a]) {
            best[a] = D;
            bj[a] = j;
          }
        }
      }
    }
    // combine the 16 column threads of each row, in seed order
    __syncthreads();
    double* red_d = reinterpret_cast<double*>(xs);
    int* red_j = reinterpret_cast<int*>(xs + FB_R * 16 * 2);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      red_d[(tr * 4 + a) * 16 + tc] = best[a];
      red_j[(tr * 4 + a) * 16 + tc] = bj[a];
    }
    __syncthreads();
    unsigned long long done = 0;
    if (tid < FB_R && rid[tid] >= 0) {
      double bd = INFINITY;
      int bb = 0x7fffffff;
      for (int c = 0; c < 16; ++c) {
        const double od = red_d[tid * 16 + c];
        const int oj = red_j[tid * 16 + c];
        if (od < bd || (od == bd && oj < bb)) {
          bd = od;
          bb = oj;
        }
      }
      const int64_t i = rid[tid];
      if (S == 1) {
        // no finite distance (non-finite input, already flagged): seed 0
        assign[i] = bb == 0x7fffffff ? 0 : bb;
        dist[i] = bd;
        done = 1;
      } else {
        const int64_t e = (g * FB_R + tid) * S + sp;
        part_d[e] = bd;
        part_j[e] = bb;
      }
    }
    if (ctr && tid < 64) block_add_u64(ctr + 2, done);
  }
}

// Per-row minimum over the seed-tile splits of k_fallback64 (split order is
// seed order, so (D, j) comparison keeps the lowest index on ties).
__global__ void k_fb_merge(const uint32_t* __restrict__ rows, const uint32_t* __restrict__ rows_count, int k,
                           const double* __restrict__ part_d, const int32_t* __restrict__ part_j,
                           int32_t* __restrict__ assign, double* __restrict__ dist,
                           unsigned long long* __restrict__ ctr) {
  const uint32_t count = *rows_count;
  int64_t R;
  int S;
  fb_shape(count, k, &R, &S);
  if (S == 1) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t iters = ((int64_t)count + stride - 1) / stride;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t pos = it * stride + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned long long done = 0;
    if (pos < count) {
      double bd = INFINITY;
      int bb = 0x7fffffff;
      for (int sp = 0; sp < S; ++sp) {
        const double od = part_d[pos * S + sp];
        const int oj = part_j[pos * S + sp];
        if (od < bd || (od == bd && oj < bb)) {
          bd = od;
          bb = oj;
        }
      }
      const int64_t i = rows[pos];
      assign[i] = bb == 0x7fffffff ? 0 : bb;
      dist[i] = bd;
      done = 1;
    }
    if (ctr) block_add_u64(ctr + 2, done);
  }
}

// ---------------------------------------------------------------- SSE, radius
// One wavefront per 4096-row block: a coalesced copy into LDS, then one lane
// adds the block's values in row order (the reference summation order).
__global__ __launch_bounds__(64) void k_sse_blocks(const double* __restrict__ dist, int64_t n,
                                                   double* __restrict__ blk) {
  __shared__ double v[SSE_BLOCK];
  const int64_t b = blockIdx.x;
  const int64_t s = b * SSE_BLOCK;
  const int cnt = (int)(n - s < SSE_BLOCK ? n - s : SSE_BLOCK);
  for (int i = threadIdx.x; i < cnt; i += 64) v[i] = dist[s + i];
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int i = 0; i < cnt; ++i) acc = __dadd_rn(acc, v[i]);
    blk[b] = acc;
  }
}

__global__ void k_sse_total(const double* __restrict__ blk, int64_t nb, double* __restrict__ out) {
  if (blockIdx.x || threadIdx.x) return;
  double acc = 0.0;
  for (int64_t b = 0; b < nb; ++b) acc = __dadd_rn(acc, blk[b]);
  *out = acc;
}

__global__ void k_radius(const int32_t* __restrict__ assign, const double* __restrict__ dist,
                         int64_t n, int k, double* __restrict__ rad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n || (unsigned)assign[i] >= (unsigned)k) return;
  const double v = dist[i];
  double* slot = rad + assign[i];
  if (v > __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomic_max_nonneg(slot, v);
}

// Up to CAP clusters: per-workgroup maxima in LDS (bit patterns of
// non-negative doubles order like the values), then one global atomic per
// touched slot.
constexpr int RAD_LDS = 4096, RAD_LDS_BIG = 16384;
template <int CAP>
__global__ __launch_bounds__(256) void k_radius_lds(const int32_t* __restrict__ assign,
                                                    const double* __restrict__ dist, int64_t n, int k,
                                                    double* __restrict__ rad) {
  __shared__ unsigned long long m[CAP];
  for (int j = threadIdx.x; j < k; j += 256) m[j] = 0ull;
  __syncthreads();
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int a = assign[i];
    if ((unsigned)a < (unsigned)k) atomicMax(&m[a], (unsigned long long)__double_as_longlong(dist[i]));
  }
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += 256)
    if (m[j]) atomic_max_nonneg(rad + j, __longlong_as_double((long long)m[j]));
}

__global__ void k_sqrt_inplace(double* __restrict__ v, int k, int do_sqrt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k && do_sqrt) v[j] = sqrt(v[j]);
}

__global__ void k_pad_modes(const uint32_t* __restrict__ mode, int k, int n_cat, int k_pad,
                            uint32_t* __restrict__ out) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)k_pad * MAX_CAT) return;
  const int j = (int)(g / MAX_CAT), a = (int)(g % MAX_CAT);
  out[g] = (j < k && a < n_cat) ? mode[(int64_t)j * n_cat + a] : 0u;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_copy_u64(const unsigned long long* a, unsigned long long* b, int n) {
  const int i = threadIdx.x;
  if (i < n) b[i] = a[i];
}

// ---------------------------------------------------------------- host side
// SSE over 4096-row blocks and the per-cluster radius (sqrt of the largest
// member distance when `take_sqrt`), shared by every metric.
void sse_and_radius(const double* dist, const int32_t* assign, int64_t n, int k, double* sse, double* radius,
                    int take_sqrt, double* sse_blk, hipStream_t s) {
  const int64_t nblk = (n + SSE_BLOCK - 1) / SSE_BLOCK;
  hipLaunchKernelGGL(k_sse_blocks, dim3(nblk), dim3(64), 0, s, dist, n, sse_blk);
  hipLaunchKernelGGL(k_sse_total, dim3(1), dim3(1), 0, s, sse_blk, nblk, sse);
  if (radius) {
    hipLaunchKernelGGL(k_fill_f64, dim3(ceil_div(k, 256)), dim3(256), 0, s, radius, k, 0.0);
    if (k <= RAD_LDS)
      hipLaunchKernelGGL(k_radius_lds<RAD_LDS>, dim3((int)std::min<int64_t>(ceil_div(n, 4096), 512)), dim3(256), 0,
                         s, assign, dist, n, k, radius);
    else if (k <= RAD_LDS_BIG)  // 128 KB of LDS: one workgroup per CU, fewer of them
      hipLaunchKernelGGL(k_radius_lds<RAD_LDS_BIG>, dim3((int)std::min<int64_t>(ceil_div(n, 16384), 128)), dim3(256),
                         0, s, assign, dist, n, k, radius);
    else
      hipLaunchKernelGGL(k_radius, dim3(ceil_div(n, 256)), dim3(256), 0, s, assign, dist, n, k, radius);
    hipLaunchKernelGGL(k_sqrt_inplace, dim3(ceil_div(k, 256)), dim3(256), 0, s, radius, k, take_sqrt);
  }
}

size_t sse_blk_words(int64_t n) { return (size_t)((n + SSE_BLOCK - 1) / SSE_BLOCK + 1); }

static int pick_dp(int d) { return d <= 32 ? 32 : d <= 64 ? 64 : d <= 128 ? 128 : d <= 256 ? 256 : 0; }

size_t modes_ws(int64_t n_members, int F, int k);
int32_t modes_compute(const uint32_t* V, int64_t ldv, int F, int64_t n, const uint32_t* so, const uint32_t* sm,
                      int k, int64_t NC, uint32_t* modes, void* ws, int32_t* st, hipStream_t s);

struct AssignWs {
  float* cl32;
  void* cllow;  // bf16 / fp8 copy for the first pass
  float* nc;
  float* cmax;   // [0] max |c|, [1] max |x_t|, [2] max |c_t|, [3] fp8 scale
  int32_t* rec;
  uint32_t* esc;
  uint32_t* fb;
  uint32_t* counts;  // [0] esc count, [1] fb count
  double* part_d;    // per-split minima of the float64 full scans
  int32_t* part_j;
  unsigned long long* ctr;
  double* dist;
  double* sse_blk;
  void* modes_ws;
  size_t modes_bytes;
  uint32_t* mode16;
  float* xt;  // dimension-major member values (centroids_transposed)
};

static size_t carve_assign(const geek_assign_job& J, void* ws, AssignWs* out) {
  Carver c(ws);
  const int DP = pick_dp(J.d);
  const int64_t k_pad = ((int64_t)J.k + SCAN_BC - 1) / SCAN_BC * SCAN_BC;
  out->cl32 = c.take<float>(k_pad * DP);
  const size_t low = J.precision == GEEK_PREC_BF16 ? 2 : J.precision == GEEK_PREC_FP8 ? 1 : 0;
  out->cllow = c.take<char>(low ? k_pad * DP * low : 16);
  out->nc = c.take<float>(k_pad);
  out->cmax = c.take<float>(4);
  out->rec = c.take<int32_t>(J.n * RECW);
  out->esc = c.take<uint32_t>(J.n);
  out->fb = c.take<uint32_t>(J.n);
  out->counts = c.take<uint32_t>(4);
  out->part_d = c.take<double>(fb_part_cap(J.n));
  out->part_j = c.take<int32_t>(fb_part_cap(J.n));
  out->ctr = c.take<unsigned long long>(4);
  out->dist = c.take<double>(J.dist ? 1 : J.n);
  out->sse_blk = c.take<double>((J.n + SSE_BLOCK - 1) / SSE_BLOCK + 1);
  out->modes_bytes = J.metric == GEEK_METRIC_HETERO ? modes_ws(J.n_members, J.n_cat, J.k) : 0;
  out->modes_ws = c.take<char>(out->modes_bytes + 16);
  out->mode16 = c.take<uint32_t>(J.metric == GEEK_METRIC_HETERO ? k_pad * MAX_CAT : 4);
  out->xt = c.take<float>(centroids_transposed(J) ? (size_t)members_pad(J) * J.d : 4);
  return c.used + 256;
}

size_t assign_euclid_ws(const geek_assign_job& J) {
  AssignWs W;
  return carve_assign(J, nullptr, &W);
}

// Column blocks per wave and LDS buffering per mode: the low-precision modes
// reuse every LDS fragment for two column blocks and double-buffer; float32
// (16x fewer flops per cycle) keeps one block and one buffer.
// The BF16 first pass keeps the best two values per row (T2); FP8 and the
// float32 pass, which also rescans rows with several candidates, keep the
// full candidate window.
// Heterogeneous rows carry their categorical values in registers: one
// column block.
template <class M, bool HET> struct ScanShape {
  // FP8's candidate window with two column blocks per wave runs 2-3x slower
  // than with one (measured across depths); BF16 keeps two off HET
  static constexpr int NCB = (HET || std::is_same<M, ModeFP8>::value) ? 1 : 2, NBUF = 2;
  // e4m3's coarse rounding leaves most rows with a few candidates: FP8 keeps
  // the full candidate window (float64 recheck of up to TCAND) instead
  static constexpr bool T2 = std::is_same<M, ModeBF16>::value;
};
template <bool HET> struct ScanShape<ModeF32, HET> {
  static constexpr int NCB = 1, NBUF = 1;
  static constexpr bool T2 = false;
};

template <class M>
int scan_rows_per_tile(bool het_on) {
  return 128 * (het_on ? ScanShape<M, true>::NCB : ScanShape<M, false>::NCB);
}

template <class M, bool HET, bool WIDE>
static void launch_scan(int DP, int grid, hipStream_t s, const geek_assign_job& J, int64_t n_rows,
                        const uint32_t* rows, const uint32_t* rows_count, const void* cl, const AssignWs& W,
                        int k_pad, const Het& het, int32_t* st) {
  using CE = typename M::ce;
  constexpr int NCB = ScanShape<M, HET>::NCB, NBUF = ScanShape<M, HET>::NBUF;
  constexpr bool T2 = ScanShape<M, HET>::T2;
  switch (DP) {
#define GEEK_SCAN_CASE(DPV)                                                                            \
  case DPV:                                                                                            \
    hipLaunchKernelGGL((k_scan<M, DPV, HET, NCB, NBUF, T2, WIDE>), dim3(grid), dim3(SCAN_THREADS), 0, s, J.X,\
                       J.ldx, J.d, n_rows, rows, rows_count, static_cast<const CE*>(cl), W.nc, k_pad,  \
                       W.cmax, W.cmax + 3, het, J.k, W.rec, st);                                       \
    break;
    GEEK_SCAN_CASE(32)
    GEEK_SCAN_CASE(64)
    GEEK_SCAN_CASE(128)
    GEEK_SCAN_CASE(256)
#undef GEEK_SCAN_CASE
  }
}

template <class M, bool WIDE = false>
static void scan_any(bool het_on, int DP, int grid, hipStream_t s, const geek_assign_job& J, int64_t n_rows,
                     const uint32_t* rows, const uint32_t* rows_count, const void* cl, const AssignWs& W,
                     int k_pad, const Het& het, int32_t* st) {
  if (het_on)
    launch_scan<M, true, WIDE>(DP, grid, s, J, n_rows, rows, rows_count, cl, W, k_pad, het, st);
  else
    launch_scan<M, false, WIDE>(DP, grid, s, J, n_rows, rows, rows_count, cl, W, k_pad, het, st);
}

// Per-job state between the three phases of an assignment.
struct AssignCtx {
  AssignWs W;
  int DP = 0;
  int k_pad = 0;
  double* dist = nullptr;
  bool het_on = false;
  Het het{nullptr, nullptr, nullptr, 0, 0.f, 0.0};
};

// Centroids (and modes), matrix-core copies, |c|^2, bounds and scale.
static int32_t assign_prep(const geek_assign_job& J, void* ws, AssignCtx& C, int32_t* st, hipStream_t s) {
  carve_assign(J, ws, &C.W);
  AssignWs& W = C.W;
  C.DP = pick_dp(J.d);
  C.k_pad = (J.k + SCAN_BC - 1) / SCAN_BC * SCAN_BC;
  C.dist = J.dist ? J.dist : W.dist;
  C.het_on = J.metric == GEEK_METRIC_HETERO;
  if (C.het_on) C.het = Het{J.cat, J.modes, W.mode16, J.n_cat, (float)J.gamma, J.gamma};
  const int DP = C.DP, k_pad = C.k_pad;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, W.counts, 4, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(W.ctr), 8, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(W.cmax), 4, 0u);
  if (centroids_transposed(J)) {
    const int64_t nmp = members_pad(J);
    hipLaunchKernelGGL(k_gather_t, dim3(ceil_div(nmp, GT_TILE), ceil_div(J.d, GT_TILE)), dim3(256), 0, s, J.X,
                       J.ldx, J.n, J.d, J.seed_offsets, J.k, J.seed_members, J.n_members, nmp, W.xt, st);
    hipLaunchKernelGGL(k_centroids_t, dim3(ceil_div((int64_t)J.k * J.d, 256)), dim3(256), 0, s, W.xt,
                       J.n_members, J.d, J.seed_offsets, J.k, J.centroids, st);
  } else {
    hipLaunchKernelGGL(k_centroids, dim3(ceil_div((int64_t)J.k * J.d, 256)), dim3(256), 0, s, J.X,
                       J.ldx, J.n, J.d, J.seed_offsets, J.seed_members, J.k, J.k_dev, J.centroids, st);
  }
  if (C.het_on) {
    if (int32_t rc = modes_compute(reinterpret_cast<const uint32_t*>(J.cat), J.n_cat, J.n_cat, J.n,
                                   J.seed_offsets, J.seed_members, J.k, J.n_members, J.modes, W.modes_ws, st, s))
      return rc;
    hipLaunchKernelGGL(k_pad_modes, dim3(ceil_div((int64_t)k_pad * MAX_CAT, 256)), dim3(256), 0, s, J.modes, J.k,
                       J.n_cat, k_pad, W.mode16);
  }
  hipLaunchKernelGGL(k_cprep<ModeF32>, dim3(ceil_div(k_pad, 128)), dim3(128), 0, s, J.centroids, J.k, J.d, k_pad,
                     DP, W.cl32, W.nc, W.cmax, W.cmax + 3, J.k_dev);
  if (J.precision == GEEK_PREC_BF16) {
    hipLaunchKernelGGL(k_cprep<ModeBF16>, dim3(ceil_div(k_pad, 128)), dim3(128), 0, s, J.centroids, J.k, J.d,
                       k_pad, DP, static_cast<__bf16*>(W.cllow), nullptr, nullptr, W.cmax + 3, J.k_dev);
  } else if (J.precision == GEEK_PREC_FP8) {
    hipLaunchKernelGGL(k_absmax_x, dim3(1024), dim3(256), 0, s, J.X, J.ldx, J.n, J.d, W.cmax + 1);
    hipLaunchKernelGGL(k_absmax_c, dim3(256), dim3(256), 0, s, J.centroids, (int64_t)J.k * J.d, W.cmax + 2);
    hipLaunchKernelGGL(k_fp8_scale, dim3(1), dim3(1), 0, s, W.cmax + 1, W.cmax + 2, W.cmax + 3);
    hipLaunchKernelGGL(k_cprep<ModeFP8>, dim3(ceil_div(k_pad, 128)), dim3(128), 0, s, J.centroids, J.k, J.d,
                       k_pad, DP, static_cast<uint8_t*>(W.cllow), nullptr, nullptr, W.cmax + 3, J.k_dev);
  }
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

// Workgroups of a persistent pass over a device-counted subset of n rows.
static int esc_grid(int64_t n, int rows_per_group) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(n, rows_per_group)));
}

static bool low_precision(const geek_assign_job& J) {
  return J.precision == GEEK_PREC_BF16 || J.precision == GEEK_PREC_FP8;
}

// The first pass of one job: every row gets a candidate record.
static void assign_first_pass(const geek_assign_job& J, AssignCtx& C, int32_t* st, hipStream_t s) {
  if (J.precision == GEEK_PREC_BF16) {
    const int grid_all = ceil_div(J.n, scan_rows_per_tile<ModeBF16>(C.het_on));
    scan_any<ModeBF16>(C.het_on, C.DP, grid_all, s, J, J.n, nullptr, nullptr, C.W.cllow, C.W, C.k_pad, C.het, st);
  } else if (J.precision == GEEK_PREC_FP8) {
    const int grid_all = ceil_div(J.n, scan_rows_per_tile<ModeFP8>(C.het_on));
    scan_any<ModeFP8>(C.het_on, C.DP, grid_all, s, J, J.n, nullptr, nullptr, C.W.cllow, C.W, C.k_pad, C.het, st);
  } else {
    const int grid_all = ceil_div(J.n, scan_rows_per_tile<ModeF32>(C.het_on));
    scan_any<ModeF32>(C.het_on, C.DP, grid_all, s, J, J.n, nullptr, nullptr, C.W.cl32, C.W, C.k_pad, C.het, st);
  }
}

// Float64 checks, rescans and fallbacks, SSE, radius, counters.
static void assign_finish(const geek_assign_job& J, AssignCtx& C, int32_t* st, hipStream_t s,
                          const unsigned long long* t0) {
  AssignWs& W = C.W;
  unsigned long long* ctr = W.ctr;
  const int fz_grid = (int)std::min<int64_t>(ceil_div(J.n, 4 * FZ_ROWS), 8192);
  const int rstride = J.precision == GEEK_PREC_BF16 ? RECW_T2 : RECW;
  // eight lanes per row for the BF16 records of large jobs (10^7 rows at
  // d = 128: 3.3 against 4.0 ms); the batched workload's jobs (10^3 .. 10^6
  // rows on four streams) ran 36 ms slower in all with it than with a lane
  // per row, for reasons not yet found, so smaller jobs keep a lane per row
  if (rstride == RECW_T2 && J.n >= ((int64_t)1 << 20))
    hipLaunchKernelGGL(k_finalize, dim3(fz_grid), dim3(256), 0, s, J.X, J.ldx, J.d, J.centroids, J.k, C.het, J.n,
                       nullptr, nullptr, W.rec, rstride, J.assign, C.dist, W.esc, W.counts + 0, ctr, 0);
  else
    hipLaunchKernelGGL(k_finalize_win, dim3(ceil_div(J.n, 256)), dim3(256), 0, s, J.X, J.ldx, J.d, J.centroids, J.k,
                       C.het, J.n, nullptr, nullptr, W.rec, rstride, J.assign, C.dist, W.esc, W.counts + 0, ctr, 0);
  // rows with several first-pass candidates: float32 rescan of those rows with
  // a wider window (persistent grids, at most one row tile / block per group)
  scan_any<ModeF32, true>(C.het_on, C.DP, esc_grid(J.n, 128), s, J, 0, W.esc, W.counts + 0, W.cl32, W, C.k_pad,
                          C.het, st);
  hipLaunchKernelGGL(k_finalize_win, dim3(esc_grid(J.n, 256)), dim3(256), 0, s, J.X, J.ldx, J.d, J.centroids,
                     J.k, C.het, (int64_t)0, W.esc, W.counts + 0, W.rec, RECW, J.assign, C.dist, W.fb, W.counts + 1,
                     ctr, 1);
  const int fb_grid = (int)std::min<int64_t>(FB_GRID, ceil_div(J.n, FB_R) * FB_SPLIT);
  switch (C.DP) {
#define GEEK_FB_CASE(DPV)                                                                                  \
  case DPV:                                                                                                \
    hipLaunchKernelGGL(k_fallback64<DPV>, dim3(fb_grid), dim3(256), 0, s, J.X, J.ldx, J.d, J.centroids, J.k, \
                       J.k_dev, C.het, W.fb, W.counts + 1, J.assign, C.dist, W.part_d, W.part_j, ctr);               \
    break;
    GEEK_FB_CASE(32)
    GEEK_FB_CASE(64)
    GEEK_FB_CASE(128)
    GEEK_FB_CASE(256)
#undef GEEK_FB_CASE
  }
  hipLaunchKernelGGL(k_fb_merge, dim3(esc_grid(J.n, 256)), dim3(256), 0, s, W.fb, W.counts + 1, J.k, W.part_d,
                     W.part_j, J.assign, C.dist, ctr);
  sse_and_radius(C.dist, J.assign, J.n, J.k, J.sse, J.radius, C.het_on ? 0 : 1, W.sse_blk, s);
  if (J.counters) hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, s, ctr, J.counters, 4);
  if (J.t_done) {
    if (t0) hipLaunchKernelGGL(k_clock_since, dim3(1), dim3(64), 0, s, t0, J.t_done);
    else hipLaunchKernelGGL(k_clock_now, dim3(1), dim3(64), 0, s, J.t_done);
  }
}

int32_t assign_euclid(const geek_assign_job& J, void* ws, size_t ws_bytes, int32_t* st,
                      hipStream_t s) {
  AssignCtx C;
  if (ws_bytes < carve_assign(J, ws, &C.W)) return GEEK_ERR_WORKSPACE;
  prof_begin(GEEK_PROF_ASSIGN, s);
  if (int32_t rc = assign_prep(J, ws, C, st, s)) return rc;
  prof_begin(GEEK_PROF_ASSIGN_SCAN, s);
  assign_first_pass(J, C, st, s);
  prof_end(GEEK_PROF_ASSIGN_SCAN, s);
  assign_finish(J, C, st, s, nullptr);
  prof_end(GEEK_PROF_ASSIGN, s);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

// ---------------------------------------------------------------- batches
// Jobs of one call that can share persistent first-pass launches: Euclidean,
// all in the same precision.  Each job gets its own workspace slice.
bool assign_batchable(const geek_assign_job* jobs, int njobs) {
  if (njobs < 2) return false;
  for (int j = 0; j < njobs; ++j)
    if (jobs[j].metric != GEEK_METRIC_EUCLID || jobs[j].precision != jobs[0].precision || jobs[j].k_dev)
      return false;
  return true;
}

static size_t slice_bytes(const geek_assign_job& J) {
  AssignWs W;
  return (carve_assign(J, nullptr, &W) + 255) / 256 * 256;
}

size_t assign_batch_ws(const geek_assign_job* jobs, int njobs) {
  size_t b = 0;
  for (int j = 0; j < njobs; ++j) b += slice_bytes(jobs[j]);
  return b + (size_t)njobs * sizeof(ScanJob) + 512;
}

int32_t assign_euclid_batch(const geek_assign_job* jobs, int njobs, void* ws, size_t ws_bytes, int32_t* st,
                            hipStream_t s) {
  if (ws_bytes < assign_batch_ws(jobs, njobs)) return GEEK_ERR_WORKSPACE;
  std::vector<AssignCtx> C(njobs);
  std::vector<char*> slice(njobs);
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  for (int j = 0; j < njobs; ++j) {
    slice[j] = base + off;
    off += slice_bytes(jobs[j]);
  }
  ScanJob* table = reinterpret_cast<ScanJob*>(base + (off + 255) / 256 * 256);
  unsigned long long* t0 = reinterpret_cast<unsigned long long*>(table + njobs);
  const geek_assign_job& J0 = jobs[0];
  prof_begin(GEEK_PROF_ASSIGN, s);
  hipLaunchKernelGGL(k_clock_now, dim3(1), dim3(64), 0, s, t0);
  {  // jobs prepared concurrently on the fan-out lanes (independent slices)
    Fan fan(s, njobs);
    for (int j = 0; j < njobs; ++j)
      if (int32_t rc = assign_prep(jobs[j], slice[j], C[j], st, fan.lane(j))) return rc;
  }
  // one persistent launch per padded depth, jobs in call order, with the
  // tile shape set for that (precision, depth)
  const bool low = low_precision(J0);
  prof_begin(GEEK_PROF_ASSIGN_SCAN, s);
  int tslot = 0;
  for (const int DP : {32, 64, 128, 256}) {
    const int rows_per_tile = 128 * scan_tiles_get(J0.precision, DP).ncb;
    std::vector<ScanJob> tab;
    int64_t total = 0;
    for (int j = 0; j < njobs; ++j) {
      if (C[j].DP != DP) continue;
      const geek_assign_job& J = jobs[j];
      const AssignWs& W = C[j].W;
      ScanJob e{};
      e.X = J.X;
      e.ldx = J.ldx;
      e.n = J.n;
      e.cl = low ? W.cllow : static_cast<const void*>(W.cl32);
      e.nc = W.nc;
      e.cmax = W.cmax;
      e.scale = W.cmax + 3;
      e.rec = W.rec;
      e.tile_begin = total;
      e.d = J.d;
      e.k = J.k;
      e.k_pad = C[j].k_pad;
      tab.push_back(e);
      total += ceil_div(J.n, rows_per_tile);
    }
    if (tab.empty()) continue;
    ScanJob* dst = table + tslot;
    for (size_t c0 = 0; c0 < tab.size(); c0 += SCANJOB_CHUNK) {
      ScanJobChunk ch{};
      ch.count = (int)std::min<size_t>(SCANJOB_CHUNK, tab.size() - c0);
      for (int i = 0; i < ch.count; ++i) ch.jobs[i] = tab[c0 + i];
      hipLaunchKernelGGL(k_put_jobs, dim3(1), dim3(SCANJOB_CHUNK), 0, s, ch, dst + c0);
    }
    launch_scan_batch(J0.precision, DP, dst, (int)tab.size(), total, st, s);
    tslot += (int)tab.size();
  }
  prof_end(GEEK_PROF_ASSIGN_SCAN, s);
  {
    Fan fan(s, njobs);
    for (int j = 0; j < njobs; ++j) assign_finish(jobs[j], C[j], st, fan.lane(j), t0);
  }
  prof_end(GEEK_PROF_ASSIGN, s);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
