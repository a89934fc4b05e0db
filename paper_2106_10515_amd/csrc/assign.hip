// One-pass data assignment (paper Section 3.3, Eq. (1)) on gfx950.
//
// Pipeline for Euclidean data (all stream-ordered, no host synchronization):
//   k_centroids   float64 centroids, one thread per (seed, dim), members summed
//                 in ascending order one rounding at a time (exact parity).
//   k_cprep       centroid copies in the matrix-core input type (fp32 / bf16),
//                 |c|^2 and max |c| for the error bound.
//   k_scan<M,DP>  matrix-core tile |x|^2 - 2 x.c + |c|^2 over all centroids for
//                 a block of rows; per row it keeps every centroid whose
//                 approximate distance lies within 2*eps_i of the running
//                 minimum (eps_i a rigorous bound of the approximation error),
//                 up to TCAND candidates.
//   k_finalize    float64 distance (the reference formula, same operation
//                 order) for each candidate; lowest index wins exact ties.
//                 Rows whose candidate window overflowed are escalated.
//   k_fallback64  float64 distance to every centroid for the rows left.
//   k_sse_*       SSE in fixed 4096-row blocks; radius per cluster.
#include <math.h>

#include "common.hpp"

namespace geek {

constexpr int TCAND = 8;
constexpr int SSE_BLOCK = 4096;
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_BN = 128;  // rows per block (4 waves x 32 rows)
constexpr int SCAN_BC = 64;   // centroids per LDS stage

// ---------------------------------------------------------------- centroids
__global__ void k_centroids(const float* __restrict__ X, int64_t ldx, int64_t n, int d,
                            const uint32_t* __restrict__ offs, const uint32_t* __restrict__ mem,
                            int k, double* __restrict__ C, int32_t* st) {
  int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)k * d) return;
  int j = (int)(gid / d), t = (int)(gid % d);
  uint32_t s = offs[j], e = offs[j + 1];
  if (e <= s) {
    set_status(st, GEEK_ERR_EMPTY_SET);
    C[gid] = 0.0;
    return;
  }
  double acc = 0.0;
  for (uint32_t q = s; q < e; ++q) {
    uint32_t i = mem[q];
    if ((int64_t)i >= n) {
      set_status(st, GEEK_ERR_ARG);
      break;
    }
    acc = __dadd_rn(acc, (double)X[(int64_t)i * ldx + t]);
  }
  C[gid] = acc / (double)(e - s);
}

// Matrix-core input copies of the centroids, zero-padded to [k_pad][DP];
// padded rows get |c|^2 = +inf so they never enter a window.
template <class CE>
__global__ void k_cprep(const double* __restrict__ C, int k, int d, int k_pad, int DP,
                        CE* __restrict__ cl, float* __restrict__ nc, float* __restrict__ cmax) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k_pad) return;
  if (j >= k) {
    for (int t = 0; t < DP; ++t) cl[(int64_t)j * DP + t] = (CE)0.0f;
    nc[j] = INFINITY;
    return;
  }
  double s = 0.0;
  for (int t = 0; t < DP; ++t) {
    double c = t < d ? C[(int64_t)j * d + t] : 0.0;
    s = __dadd_rn(s, __dmul_rn(c, c));
    cl[(int64_t)j * DP + t] = (CE)(float)c;
  }
  nc[j] = (float)s;
  atomic_max_nonneg(cmax, (float)(sqrt(s) * (1.0 + 0x1p-20)));
}

// ---------------------------------------------------------------- modes
struct ModeF32 {
  static constexpr int KPER = 1;  // K elements per lane per instruction
  using ce = float;
  using frag = float;
  static constexpr double UX = 0.0;        // x is already float32
  static constexpr double UC = 0x1p-24;    // float64 -> float32 rounding
  GEEK_D static f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  GEEK_D static frag load_lds(const ce* p) { return *p; }
  GEEK_D static frag from_f32(const float* v) { return v[0]; }
};

struct ModeBF16 {
  static constexpr int KPER = 8;
  using ce = __bf16;
  using frag = bf16x8;
  static constexpr double UX = 0x1p-8;  // conservative for any rounding to bf16
  static constexpr double UC = 0x1p-8;
  GEEK_D static f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  GEEK_D static frag load_lds(const ce* p) { return *reinterpret_cast<const bf16x8*>(p); }
  GEEK_D static frag from_f32(const float* v) {
    frag f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = (__bf16)v[e];
    return f;
  }
};

GEEK_D double gamma_n(double nn, double u) { return nn * u / (1.0 - nn * u); }

// Rigorous bound on |(|x|^2 + v_j) - D64(i, j)| for every j, where v_j is the
// float32 epilogue value fma(-2, acc, |c_j|^2) and D64 the float64 reference.
template <class M, int DP>
GEEK_D float two_eps(double xn, double cm) {
  const double u32 = 0x1p-24;
  const double ux = M::UX, uc = M::UC;
  const double g_acc = gamma_n(DP + 1, 2.0 * u32);
  const double g64 = gamma_n(DP + 2, 0x1p-53);
  const double xc = xn * cm;
  const double s2 = (xn + cm) * (xn + cm);
  double eps = 2.0 * ((ux + uc + ux * uc) + g_acc * (1.0 + ux) * (1.0 + uc)) * xc  // 2 x.c
               + (u32 + g64) * cm * cm                    // |c|^2 stored as float32
               + u32 * (cm * cm + 2.01 * xc)              // epilogue rounding
               + g64 * s2                                 // float64 reference rounding
               + 4.0 * u32 * s2                           // threshold arithmetic
               + DP * 0x1p-120;                           // flushed subnormal products
  eps *= 1.01;
  return (float)(2.0 * eps * (1.0 + 0x1p-20));
}

// ---------------------------------------------------------------- scan
// Block = 4 waves; wave w owns rows [w*32, w*32+32) of the block's tile.
// MFMA 32x32: A = 32 centroids (rows), B = 32 points (columns).  Lane l
// supplies point p = l%32 and K half h = l/32; the K index of step s,
// element e is h*DP/2 + s*KPER + e (any bijection works for a dot product
// as long as A and B agree).  Accumulator register r of lane l holds
// centroid row (r/4)*8 + h*4 + r%4 of point p.
template <class M, int DP>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan(
    const float* __restrict__ X, int64_t ldx, int d, int64_t n_rows,
    const uint32_t* __restrict__ rows, const uint32_t* __restrict__ rows_count,
    const typename M::ce* __restrict__ cl, const float* __restrict__ nc, int k_pad,
    const float* __restrict__ cmax_p, int32_t* __restrict__ rec, int32_t* st) {
  using CE = typename M::ce;
  constexpr int S = DP / 2 / M::KPER;       // MFMA steps over K
  constexpr int STR = DP + 16 / (int)sizeof(CE);  // padded LDS row (elements)
  __shared__ __attribute__((aligned(16))) CE lds_c[SCAN_BC * STR];
  __shared__ float lds_nc[SCAN_BC];
  __shared__ float lds_lv[SCAN_THREADS * TCAND];
  __shared__ int lds_lj[SCAN_THREADS * TCAND];

  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int p = lane & 31, h = lane >> 5;
  float* lv = lds_lv + tid * TCAND;
  int* lj = lds_lj + tid * TCAND;

  const int64_t count = rows ? (int64_t)*rows_count : n_rows;
  const double cm = (double)*cmax_p;
  const bool vec4 = ((d & 3) == 0) && ((ldx & 3) == 0);

  for (int64_t tile = blockIdx.x; tile * SCAN_BN < count; tile += gridDim.x) {
    const int64_t pos = tile * SCAN_BN + w * 32 + p;
    const bool valid = pos < count;
    const int64_t i = valid ? (rows ? (int64_t)rows[pos] : pos) : 0;
    const float* xr = X + i * ldx;

    // ---- this lane's half row of x as MFMA B fragments; exact |x|^2
    float xv[DP / 2];
#pragma unroll
    for (int q = 0; q < DP / 2; q += 4) {
      const int t0 = h * (DP / 2) + q;
      float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
      if (valid) {
        if (vec4 && t0 + 3 < d) {
          val = *reinterpret_cast<const float4*>(xr + t0);
        } else {
          val.x = t0 < d ? xr[t0] : 0.f;
          val.y = t0 + 1 < d ? xr[t0 + 1] : 0.f;
          val.z = t0 + 2 < d ? xr[t0 + 2] : 0.f;
          val.w = t0 + 3 < d ? xr[t0 + 3] : 0.f;
        }
      }
      xv[q] = val.x;
      xv[q + 1] = val.y;
      xv[q + 2] = val.z;
      xv[q + 3] = val.w;
    }
    double nrm = 0.0;
    bool finite = true;
#pragma unroll
    for (int q = 0; q < DP / 2; ++q) {
      finite = finite && isfinite(xv[q]);
      nrm += (double)xv[q] * (double)xv[q];
    }
    typename M::frag xb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) xb[s] = M::from_f32(xv + s * M::KPER);
    if (!finite) set_status(st, GEEK_ERR_NONFINITE);
    nrm += __shfl_xor(nrm, 32);
    const float twoeps = two_eps<M, DP>(sqrt(nrm) * (1.0 + 1e-12), cm);

    // thr starts at the largest finite float: padded centroids (|c|^2 = +inf)
    // and non-finite values never enter the window
    float b0 = INFINITY, thr = 3.402823466e38f;
    int cnt = 0;
    bool ovf = false;

    for (int c0 = 0; c0 < k_pad; c0 += SCAN_BC) {
      __syncthreads();
      // cooperative load of SCAN_BC centroid rows (16-byte chunks)
      constexpr int CH = DP * (int)sizeof(CE) / 16;  // chunks per row
      for (int q = tid; q < SCAN_BC * CH; q += SCAN_THREADS) {
        const int r = q / CH, c = q % CH;
        const uint4 val = *reinterpret_cast<const uint4*>(
            reinterpret_cast<const char*>(cl + (int64_t)(c0 + r) * DP) + c * 16);
        *reinterpret_cast<uint4*>(reinterpret_cast<char*>(lds_c + r * STR) + c * 16) = val;
      }
      if (tid < SCAN_BC) lds_nc[tid] = nc[c0 + tid];
      __syncthreads();

#pragma unroll
      for (int rb = 0; rb < SCAN_BC / 32; rb += 2) {
        f32x16 acc0 = {}, acc1 = {};
        const CE* a0p = lds_c + (rb * 32 + p) * STR + h * (DP / 2);
        const CE* a1p = a0p + 32 * STR;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          acc0 = M::mma(M::load_lds(a0p + s * M::KPER), xb[s], acc0);
          acc1 = M::mma(M::load_lds(a1p + s * M::KPER), xb[s], acc1);
        }
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const f32x16& acc = half ? acc1 : acc0;
          const int jb = (rb + half) * 32;
          float v[16];
          float vmin = INFINITY;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = (r >> 2) * 8 + h * 4 + (r & 3);
            v[r] = __builtin_fmaf(-2.0f, acc[r], lds_nc[jb + row]);
            vmin = fminf(vmin, v[r]);
          }
          if (vmin <= thr) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              if (v[r] <= thr) {
                const int j = c0 + jb + (r >> 2) * 8 + h * 4 + (r & 3);
                if (v[r] < b0) {
                  b0 = v[r];
                  thr = b0 + twoeps;
                }
                if (!ovf) {
                  if (cnt == TCAND) {
                    int kept = 0;
#pragma unroll 1
                    for (int q = 0; q < TCAND; ++q) {
                      const float ev = lv[q];
                      const int ej = lj[q];
                      if (ev <= thr) {
                        lv[kept] = ev;
                        lj[kept] = ej;
                        ++kept;
                      }
                    }
                    cnt = kept;
                    ovf = (cnt == TCAND);
                  }
                  if (!ovf) {
                    lv[cnt] = v[r];
                    lj[cnt] = j;
                    ++cnt;
                  }
                }
              }
            }
          }
        }
      }
    }

    // ---- merge the two lanes that share a point, write the candidate record
    const float bo = __shfl_xor(b0, 32);
    const float bfin = fminf(b0, bo);
    const float tfin = bfin < INFINITY ? bfin + twoeps : 3.402823466e38f;
    int kept = 0;
    for (int q = 0; q < cnt; ++q) {
      const float ev = lv[q];
      const int ej = lj[q];
      if (ev <= tfin) {
        lv[kept] = ev;
        lj[kept] = ej;
        ++kept;
      }
    }
    const int kept_o = __shfl_xor(kept, 32);
    const int ovf_o = __shfl_xor((int)ovf, 32);
    const bool over = ovf || ovf_o || (kept + kept_o > TCAND);
    if (valid) {
      int32_t* rr = rec + pos * (TCAND + 1);
      if (over) {
        if (h == 0) rr[0] = -1;
      } else {
        if (h == 0) rr[0] = kept + kept_o;
        const int off = h ? kept_o : 0;
        for (int q = 0; q < kept; ++q) rr[1 + off + q] = lj[q];
      }
    }
  }
}

// ---------------------------------------------------------------- float64 checks
GEEK_D double d64(const float* __restrict__ xr, const double* __restrict__ cr, int d) {
  double acc = 0.0;
  for (int t = 0; t < d; ++t) {
    const double delta = __dadd_rn((double)xr[t], -cr[t]);
    acc = __dadd_rn(acc, __dmul_rn(delta, delta));
  }
  return acc;
}

__device__ void block_add_u64(unsigned long long* dst, unsigned long long v) {
  // one atomic per wave
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

__global__ void k_finalize(const float* __restrict__ X, int64_t ldx, int d,
                           const double* __restrict__ C, int k, int64_t n_rows,
                           const uint32_t* __restrict__ rows, const uint32_t* __restrict__ rows_count,
                           const int32_t* __restrict__ rec, int32_t* __restrict__ assign,
                           double* __restrict__ dist, uint32_t* __restrict__ esc,
                           uint32_t* __restrict__ esc_count, unsigned long long* __restrict__ ctr,
                           int ctr_rows) {
  const int64_t count = rows ? (int64_t)*rows_count : n_rows;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t iters = (count + stride - 1) / stride;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t pos = start + it * stride;
    unsigned long long nrow = 0, ncand = 0;
    if (pos < count) {
      const int64_t i = rows ? (int64_t)rows[pos] : pos;
      const int32_t* rr = rec + pos * (TCAND + 1);
      const int c = rr[0];
      if (c <= 0) {  // window overflow (or no finite candidate): escalate
        const uint32_t q = atomicAdd(esc_count, 1u);
        esc[q] = (uint32_t)i;
      } else {
        double best = INFINITY;
        int bj = 0x7fffffff;
        const float* xr = X + i * ldx;
        for (int q = 0; q < c; ++q) {
          const int j = rr[1 + q];
          if ((unsigned)j >= (unsigned)k) continue;
          const double D = d64(xr, C + (int64_t)j * d, d);
          if (D < best || (D == best && j < bj)) {
            best = D;
            bj = j;
          }
        }
        if (bj == 0x7fffffff) bj = 0;
        assign[i] = bj;
        dist[i] = best;
        nrow = 1;
        ncand = (unsigned long long)c;
      }
    }
    if (ctr) {
      block_add_u64(ctr + ctr_rows, nrow);
      block_add_u64(ctr + 3, ncand);
    }
  }
}

// One block per row: float64 distance to every centroid, lowest index on ties.
__global__ __launch_bounds__(256) void k_fallback64(
    const float* __restrict__ X, int64_t ldx, int d, const double* __restrict__ C, int k,
    const uint32_t* __restrict__ rows, const uint32_t* __restrict__ rows_count,
    int32_t* __restrict__ assign, double* __restrict__ dist, unsigned long long* __restrict__ ctr) {
  __shared__ float xs[1024];
  __shared__ double bd[256];
  __shared__ int bjs[256];
  const uint32_t count = *rows_count;
  for (uint32_t pos = blockIdx.x; pos < count; pos += gridDim.x) {
    const int64_t i = rows[pos];
    __syncthreads();
    for (int t = threadIdx.x; t < d; t += blockDim.x) xs[t] = X[i * ldx + t];
    __syncthreads();
    double best = INFINITY;
    int bj = 0x7fffffff;
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      const double D = d64(xs, C + (int64_t)j * d, d);
      if (D < best) {  // j increases along this thread: strict keeps the lowest
        best = D;
        bj = j;
      }
    }
    bd[threadIdx.x] = best;
    bjs[threadIdx.x] = bj;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        const double od = bd[threadIdx.x + o];
        const int oj = bjs[threadIdx.x + o];
        if (od < bd[threadIdx.x] || (od == bd[threadIdx.x] && oj < bjs[threadIdx.x])) {
          bd[threadIdx.x] = od;
          bjs[threadIdx.x] = oj;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      // no finite distance (non-finite input, already flagged): centroid 0
      assign[i] = bjs[0] == 0x7fffffff ? 0 : bjs[0];
      dist[i] = bd[0];
      if (ctr) atomicAdd(ctr + 2, 1ull);
    }
  }
}

// ---------------------------------------------------------------- SSE, radius
__global__ void k_sse_blocks(const double* __restrict__ dist, int64_t n, double* __restrict__ blk) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t s = b * SSE_BLOCK;
  if (s >= n) return;
  const int64_t e = s + SSE_BLOCK < n ? s + SSE_BLOCK : n;
  double acc = 0.0;
  for (int64_t i = s; i < e; ++i) acc = __dadd_rn(acc, dist[i]);
  blk[b] = acc;
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

__global__ void k_sqrt_inplace(double* __restrict__ v, int k, int do_sqrt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k && do_sqrt) v[j] = sqrt(v[j]);
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
static int pick_dp(int d) { return d <= 32 ? 32 : d <= 64 ? 64 : d <= 128 ? 128 : d <= 256 ? 256 : 0; }

struct AssignWs {
  float* cl32;
  __bf16* cl16;
  float* nc;
  float* cmax;
  int32_t* rec;
  uint32_t* esc;
  uint32_t* fb;
  uint32_t* counts;  // [0] esc count, [1] fb count
  unsigned long long* ctr;
  double* dist;
  double* sse_blk;
};

static size_t carve_assign(const geek_assign_job& J, void* ws, AssignWs* out) {
  Carver c(ws);
  const int DP = pick_dp(J.d);
  const int64_t k_pad = ((int64_t)J.k + SCAN_BC - 1) / SCAN_BC * SCAN_BC;
  out->cl32 = c.take<float>(k_pad * DP);
  out->cl16 = c.take<__bf16>(J.precision == GEEK_PREC_BF16 ? k_pad * DP : 1);
  out->nc = c.take<float>(k_pad);
  out->cmax = c.take<float>(1);
  out->rec = c.take<int32_t>(J.n * (TCAND + 1));
  out->esc = c.take<uint32_t>(J.n);
  out->fb = c.take<uint32_t>(J.n);
  out->counts = c.take<uint32_t>(4);
  out->ctr = c.take<unsigned long long>(4);
  out->dist = c.take<double>(J.dist ? 1 : J.n);
  out->sse_blk = c.take<double>((J.n + SSE_BLOCK - 1) / SSE_BLOCK + 1);
  return c.used + 256;
}

size_t assign_euclid_ws(const geek_assign_job& J) {
  AssignWs W;
  return carve_assign(J, nullptr, &W);
}

template <class M>
static void launch_scan(int DP, int grid, hipStream_t s, const geek_assign_job& J, int64_t n_rows,
                        const uint32_t* rows, const uint32_t* rows_count,
                        const typename M::ce* cl, const AssignWs& W, int k_pad, int32_t* st) {
  switch (DP) {
#define GEEK_SCAN_CASE(DPV)                                                                 \
  case DPV:                                                                                 \
    hipLaunchKernelGGL((k_scan<M, DPV>), dim3(grid), dim3(SCAN_THREADS), 0, s, J.X, J.ldx, \
                       J.d, n_rows, rows, rows_count, cl, W.nc, k_pad, W.cmax, W.rec, st); \
    break;
    GEEK_SCAN_CASE(32)
    GEEK_SCAN_CASE(64)
    GEEK_SCAN_CASE(128)
    GEEK_SCAN_CASE(256)
#undef GEEK_SCAN_CASE
  }
}

int32_t assign_euclid(const geek_assign_job& J, void* ws, size_t ws_bytes, int32_t* st,
                      hipStream_t s) {
  AssignWs W;
  const size_t need = carve_assign(J, ws, &W);
  if (ws_bytes < need) return GEEK_ERR_WORKSPACE;
  const int DP = pick_dp(J.d);
  const int k_pad = (J.k + SCAN_BC - 1) / SCAN_BC * SCAN_BC;
  double* dist = J.dist ? J.dist : W.dist;
  const int nb_rows = ceil_div(J.n, 256);

  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, W.counts, 4, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(W.ctr), 8, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(W.cmax), 1, 0u);
  hipLaunchKernelGGL(k_centroids, dim3(ceil_div((int64_t)J.k * J.d, 256)), dim3(256), 0, s, J.X,
                     J.ldx, J.n, J.d, J.seed_offsets, J.seed_members, J.k, J.centroids, st);
  hipLaunchKernelGGL(k_cprep<float>, dim3(ceil_div(k_pad, 128)), dim3(128), 0, s, J.centroids, J.k,
                     J.d, k_pad, DP, W.cl32, W.nc, W.cmax);
  if (J.precision == GEEK_PREC_BF16)
    hipLaunchKernelGGL(k_cprep<__bf16>, dim3(ceil_div(k_pad, 128)), dim3(128), 0, s, J.centroids,
                       J.k, J.d, k_pad, DP, W.cl16, W.nc, W.cmax);
  GEEK_LAUNCH_CHECK();

  const int grid_all = ceil_div(J.n, SCAN_BN);
  unsigned long long* ctr = W.ctr;
  if (J.precision == GEEK_PREC_BF16) {
    launch_scan<ModeBF16>(DP, grid_all, s, J, J.n, nullptr, nullptr, W.cl16, W, k_pad, st);
    hipLaunchKernelGGL(k_finalize, dim3(nb_rows), dim3(256), 0, s, J.X, J.ldx, J.d, J.centroids,
                       J.k, J.n, nullptr, nullptr, W.rec, J.assign, dist, W.esc, W.counts + 0, ctr, 0);
    // rows whose bf16 window overflowed: float32 rescan of those rows
    launch_scan<ModeF32>(DP, 1024, s, J, 0, W.esc, W.counts + 0, W.cl32, W, k_pad, st);
    hipLaunchKernelGGL(k_finalize, dim3(1024), dim3(256), 0, s, J.X, J.ldx, J.d, J.centroids,
                       J.k, (int64_t)0, W.esc, W.counts + 0, W.rec, J.assign, dist, W.fb,
                       W.counts + 1, ctr, 1);
  } else {
    launch_scan<ModeF32>(DP, grid_all, s, J, J.n, nullptr, nullptr, W.cl32, W, k_pad, st);
    hipLaunchKernelGGL(k_finalize, dim3(nb_rows), dim3(256), 0, s, J.X, J.ldx, J.d, J.centroids,
                       J.k, J.n, nullptr, nullptr, W.rec, J.assign, dist, W.fb, W.counts + 1, ctr, 0);
  }
  hipLaunchKernelGGL(k_fallback64, dim3(1024), dim3(256), 0, s, J.X, J.ldx, J.d, J.centroids, J.k,
                     W.fb, W.counts + 1, J.assign, dist, ctr);
  const int64_t nblk = (J.n + SSE_BLOCK - 1) / SSE_BLOCK;
  hipLaunchKernelGGL(k_sse_blocks, dim3(ceil_div(nblk, 64)), dim3(64), 0, s, dist, J.n, W.sse_blk);
  hipLaunchKernelGGL(k_sse_total, dim3(1), dim3(1), 0, s, W.sse_blk, nblk, J.sse);
  if (J.radius) {
    hipLaunchKernelGGL(k_fill_f64, dim3(ceil_div(J.k, 256)), dim3(256), 0, s, J.radius, J.k, 0.0);
    hipLaunchKernelGGL(k_radius, dim3(nb_rows), dim3(256), 0, s, J.assign, dist, J.n, J.k, J.radius);
    hipLaunchKernelGGL(k_sqrt_inplace, dim3(ceil_div(J.k, 256)), dim3(256), 0, s, J.radius, J.k, 1);
  }
  if (J.counters) hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, s, ctr, J.counters, 4);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
