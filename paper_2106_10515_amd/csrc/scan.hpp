// Matrix-core assignment scan shared by the single-job and batched passes
// (paper Section 3.3, Eq. (1)): input modes, the rigorous error bound of the
// expanded form, the tile loop with its candidate epilogues, and the
// persistent multi-job kernel.
#pragma once
#include <math.h>

#include <type_traits>

#include "common.hpp"

namespace geek {

template <int V>
using IC = std::integral_constant<int, V>;

constexpr int TCAND = 8;       // candidates per lane window, BF16/FP8 passes
constexpr int TCAND32 = 32;    // float32 pass (also the rescan of ambiguous rows)
constexpr int RECW = TCAND32 + 1;  // candidate record per row: count, then ids
constexpr int RECW_T2 = 2;         // the BF16 pass's record: 1 and the index, or -1
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_BC = 64;   // centroids per LDS stage

// ---------------------------------------------------------------- modes
struct ModeF32 {
  static constexpr int KPER = 1;  // K elements per lane per instruction
  static constexpr int KB = 16;   // products per fresh-accumulator block (0 = one chain)
  static constexpr bool SCALED = false;
  using ce = float;
  using frag = float;
  static constexpr double UX = 0.0;        // x is already float32
  static constexpr double UC = 0x1p-24;    // float64 -> float32 rounding
  static constexpr double A0 = 0.0;        // absolute error per element (scaled units)
  GEEK_D static f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  GEEK_D static frag load_lds(const ce* p) { return *p; }
  GEEK_D static frag from_f32(const float* v, float) { return v[0]; }
  GEEK_D static void store(ce* p, const float* v, float) { p[0] = v[0]; }
  GEEK_D static void store_zero(ce* p) { p[0] = 0.f; }
};

struct ModeBF16 {
  static constexpr int KPER = 8;
  static constexpr int KB = 0;  // input rounding (2^-8) dominates the accumulation
  static constexpr bool SCALED = false;
  using ce = __bf16;
  using frag = bf16x8;
  static constexpr double UX = 0x1p-8;  // conservative for any rounding to bf16
  static constexpr double UC = 0x1p-8;
  static constexpr double A0 = 0.0;
  GEEK_D static f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  GEEK_D static frag load_lds(const ce* p) { return *reinterpret_cast<const bf16x8*>(p); }
  GEEK_D static frag from_f32(const float* v, float) {
    frag f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = (__bf16)v[e];
    return f;
  }
  GEEK_D static void store(ce* p, const float* v, float) {
#pragma unroll
    for (int e = 0; e < 8; ++e) p[e] = (__bf16)v[e];
  }
  GEEK_D static void store_zero(ce* p) {
#pragma unroll
    for (int e = 0; e < 8; ++e) p[e] = (__bf16)0.0f;
  }
};

// e4m3 inputs, scaled by a power of two into the normal range; products are
// exact in float32.  Relative rounding 2^-3 (conservative), absolute error
// 2^-10 per element in scaled units (half the smallest subnormal spacing of
// either e4m3 variant).
struct ModeFP8 {
  static constexpr int KPER = 8;
  static constexpr int KB = 0;
  static constexpr bool SCALED = true;
  using ce = uint8_t;
  using frag = long;
  static constexpr double UX = 0x1p-3;
  static constexpr double UC = 0x1p-3;
  static constexpr double A0 = 0x1p-10;
  GEEK_D static f32x16 mma(frag a, frag b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b, c, 0, 0, 0);
  }
  GEEK_D static frag load_lds(const ce* p) { return *reinterpret_cast<const long*>(p); }
  GEEK_D static frag from_f32(const float* v, float sc) {
    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0] * sc, v[1] * sc, 0, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[2] * sc, v[3] * sc, lo, true);
    int hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[4] * sc, v[5] * sc, 0, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[6] * sc, v[7] * sc, hi, true);
    return (long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo);
  }
  GEEK_D static void store(ce* p, const float* v, float sc) {
    *reinterpret_cast<long*>(p) = from_f32(v, sc);
  }
  GEEK_D static void store_zero(ce* p) { *reinterpret_cast<long*>(p) = 0; }
};

// Categorical part of heterogeneous rows (cat == nullptr: Euclidean only).
struct Het {
  const int32_t* cat;     // [n][n_cat]
  const uint32_t* mode;   // [k][n_cat] per-attribute modes of the seeds
  const uint32_t* mode16; // [k_pad][MAX_CAT] zero-padded copy streamed by the scan
  int n_cat;
  float gamma_f;          // gamma, exactly representable in float32
  double gamma;
};
constexpr int MAX_CAT = 16;

GEEK_D double gamma_n(double nn, double u) { return nn * u / (1.0 - nn * u); }

// Rigorous bound on |(|x|^2 + v_j) - D64(i, j)| for every j, where v_j is the
// float32 epilogue value fma(-2/s^2, acc, |c_j|^2) (+ gamma * mismatches)
// and D64 the float64 reference.  X = |x|, cm = max |c|; the inputs are
// rounded with relative error UX/UC and absolute error A0/s per element, so
// |x^ - x| <= ex = UX X + A0 sqrt(DP) / s (likewise ec) and, by Cauchy-
// Schwarz, |x^.c^ - x.c| <= ex cm + X ec + ex ec; the float32 accumulation of
// the (exact) products adds gamma_n(2u) |x^| |c^| with n = DP + 1 roundings
// per product for one accumulator chain, or n = KB + DP/KB + 1 when blocks of
// KB products start from zero and their sums are added to the running value.
template <class M, int DP, bool T2, bool BLK>
GEEK_D float two_eps(double xn, double cm, double inv_scale, double het_max) {
  const double u32 = 0x1p-24;
  constexpr int NACC = BLK ? M::KB + DP / M::KB + 1 : DP + 1;
  const double g_acc = gamma_n(NACC, 2.0 * u32);
  const double g64 = gamma_n(DP + 2, 0x1p-53);
  const double ab = M::A0 * inv_scale * sqrt((double)DP);
  const double ex = M::UX * xn + ab, ec = M::UC * cm + ab;
  const double dot = ex * cm + xn * ec + ex * ec + g_acc * (xn + ex) * (cm + ec);
  const double vmax = cm * cm + 2.0 * (xn + ex) * (cm + ec) + het_max;
  const double s2 = (xn + cm) * (xn + cm) + het_max;
  // accumulations that could overflow float32 give no bound: rows escalate
  if (!(4.0 * vmax < 0x1p120)) return INFINITY;
  double eps = 2.0 * dot                       // 2 x.c
               + g_acc * cm * cm                // |c|^2 / 2 as the accumulator's start
               + 0x1p-124 * inv_scale * inv_scale  // its float32 subnormal rounding
               + (u32 + g64) * cm * cm          // |c|^2 stored as float32
               + 2.0 * u32 * vmax               // epilogue roundings
               + g64 * s2 + 0x1p-52 * het_max   // float64 reference rounding
               + 4.0 * u32 * s2                 // threshold arithmetic
               + DP * 0x1p-120                  // flushed subnormal products
               + (T2 ? 0x1p-18 * vmax : 0.0);   // index bits in the low mantissa
  eps *= 1.01;
  return (float)(2.0 * eps * (1.0 + 0x1p-20));
}

// ---------------------------------------------------------------- scan
// Block = 4 waves; wave w owns NCB column blocks of 32 rows (points) each.
// MFMA 32x32: A = 32 centroids (rows), B = 32 points (columns).  Lane l
// supplies point p = l%32 of every column block and K half h = l/32; the K
// index of step s, element e is h*DP/2 + s*KPER + e (any bijection works for
// a dot product as long as A and B agree).  Accumulator register r of lane l
// holds centroid row (r/4)*8 + h*4 + r%4 of point p.  Each A fragment read
// from LDS feeds NCB MFMAs.  With NBUF = 2 the next stage of centroids is
// in flight while the current one is consumed (LDS DMA where rows are at
// least 64 bytes, else through registers).
template <class M, int DP, bool HET, int NCB, int NBUF, bool T2, bool WIDE>
__device__ __forceinline__ void scan_tiles(
    const float* __restrict__ X, int64_t ldx, int d, int64_t n_rows,
    const uint32_t* __restrict__ rows, const uint32_t* __restrict__ rows_count,
    const typename M::ce* __restrict__ cl, const float* __restrict__ nc, int k_pad,
    const float* __restrict__ cmax_p, const float* __restrict__ scale_p, Het het, int k,
    int32_t* __restrict__ rec, int32_t* st, int64_t tile0, int64_t tile_end, int64_t tstep) {
  using CE = typename M::ce;
  constexpr int S = DP / 2 / M::KPER;             // MFMA steps over K
  constexpr int CH = DP * (int)sizeof(CE) / 16;   // 16-byte chunks per centroid row
  // DMA: stages stream global -> LDS directly (global_load_lds_dwordx4, one
  // 16-byte chunk per lane, lane-contiguous in LDS), rows unpadded with the
  // chunk index XOR-swizzled by the row; otherwise registers stage the copy
  // into rows padded by 16 bytes.
  constexpr bool DMA = NBUF == 2 && CH >= 4;
  constexpr int STR = DMA ? DP : DP + 16 / (int)sizeof(CE);  // LDS row (elements)
  constexpr int BN = 128 * NCB;                   // rows per tile
  constexpr int CPT = DMA ? 1 : (SCAN_BC * CH + SCAN_THREADS - 1) / SCAN_THREADS;
  // one LDS object per stage buffer: with the buffer known at compile time
  // the compiler can tell that reads of the current stage do not alias the
  // LDS DMA filling the next one, and does not wait for that DMA
  __shared__ __attribute__((aligned(16))) CE lds_c0[SCAN_BC * STR];
  __shared__ __attribute__((aligned(16))) CE lds_c1[NBUF == 2 ? SCAN_BC * STR : 1];
  __shared__ float lds_nc[NBUF][SCAN_BC];
  __shared__ __attribute__((aligned(16))) uint32_t lds_mode0[HET ? SCAN_BC * MAX_CAT : 1];
  __shared__ __attribute__((aligned(16))) uint32_t lds_mode1[HET && NBUF == 2 ? SCAN_BC * MAX_CAT : 1];
  auto cbuf = [&](auto bc) -> CE* {
    if constexpr (decltype(bc)::value == 0) return lds_c0;
    else return lds_c1;
  };
  auto mbuf = [&](auto bc) -> uint32_t* {
    if constexpr (decltype(bc)::value == 0) return lds_mode0;
    else return lds_mode1;
  };
  // window capacity per lane: the rescan of rows whose first-pass window was
  // ambiguous keeps more candidates
  constexpr int TC = WIDE ? TCAND32 : TCAND;
  // blocked accumulation: float32 rescans of ambiguous rows, where the
  // tighter bound keeps candidate windows from overflowing (the categorical
  // epilogue leaves no registers for the block sums; a first pass, whose rows
  // are mostly clear-cut, keeps the single chain)
  constexpr bool BLK = M::KB > 0 && !HET && WIDE;
  __shared__ float lds_lv[T2 ? 1 : SCAN_THREADS * NCB * TC];
  __shared__ int lds_lj[T2 ? 1 : SCAN_THREADS * NCB * TC];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (scalar) for LDS DMA bases
  const int p = lane & 31, h = lane >> 5;

  const int64_t count = rows ? (int64_t)*rows_count : n_rows;
  const double cm = (double)*cmax_p;
  const float sc = M::SCALED ? *scale_p : 1.0f;
  const float m2s = -2.0f / (sc * sc);  // power of two: exact rescaling
  // T2 starts every accumulator at -s^2 |c_j|^2 / 2 (exact power-of-two
  // scalings), so acc = s^2 (x.c - |c_j|^2 / 2) and v_j = m2s * acc
  const float nc_mul = T2 ? -0.5f * sc * sc : 1.0f;
  // padded centroids (|c|^2 = +inf) start T2 accumulators at -FLT_MAX / 4:
  // far below any real value, and finite even after the heterogeneous
  // epilogue doubles it (an infinity would turn into a NaN once the index
  // bits are inserted)
  auto nc_stage = [nc_mul](float v) { return T2 ? fmaxf(v * nc_mul, -0x1p126f) : v; };
  const bool vec4 = ((d & 3) == 0) && ((ldx & 3) == 0);
  const double het_max = HET ? het.gamma * het.n_cat : 0.0;

  // stage loading: registers <- global, LDS <- registers
  constexpr int MPT = HET ? (SCAN_BC * MAX_CAT + SCAN_THREADS - 1) / SCAN_THREADS : 1;
  uint4 stg[CPT];
  float stg_nc = 0.f;
  uint32_t stg_mode[MPT];
#define GEEK_LOAD_REGS(C0)                                                                                 \
  do {                                                                                                     \
    _Pragma("unroll") for (int u = 0; u < CPT; ++u) {                                                     \
      const int q = min(tid + u * SCAN_THREADS, SCAN_BC * CH - 1); /* clamped: always in bounds */        \
      const int r = q / CH, c = q % CH;                                                                    \
      stg[u] = *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(cl + (int64_t)((C0) + r) * DP) + \
                                               c * 16);                                                    \
    }                                                                                                      \
    stg_nc = nc[(C0) + (tid & (SCAN_BC - 1))];                                                             \
    if constexpr (HET) {                                                                                   \
      _Pragma("unroll") for (int u = 0; u < MPT; ++u) {                                                   \
        const int q = min(tid + u * SCAN_THREADS, SCAN_BC * MAX_CAT - 1);                                  \
        const int r = q / MAX_CAT, a = q % MAX_CAT;                                                        \
        const bool ok = a < het.n_cat && (C0) + r < k;                                                     \
        const uint32_t mv = het.mode[ok ? (int64_t)((C0) + r) * het.n_cat + a : 0];                        \
        stg_mode[u] = ok ? mv : 0u;                                                                        \
      }                                                                                                    \
    }                                                                                                      \
  } while (0)
#define GEEK_STORE_LDS(B)                                                                                  \
  do {                                                                                                     \
    _Pragma("unroll") for (int u = 0; u < CPT; ++u) {                                                     \
      const int q = tid + u * SCAN_THREADS;                                                                \
      if (q < SCAN_BC * CH) {                                                                              \
        const int r = q / CH, c = q % CH;                                                                  \
        *reinterpret_cast<uint4*>(reinterpret_cast<char*>(cbuf(IC<(B)>{}) + r * STR) + c * 16) = stg[u];   \
      }                                                                                                    \
    }                                                                                                      \
    if (tid < SCAN_BC) lds_nc[B][tid] = nc_stage(stg_nc);                                                  \
    if constexpr (HET) {                                                                                   \
      _Pragma("unroll") for (int u = 0; u < MPT; ++u) {                                                   \
        const int q = tid + u * SCAN_THREADS;                                                              \
        if (q < SCAN_BC * MAX_CAT) mbuf(IC<(B)>{})[q] = stg_mode[u];                                       \
      }                                                                                                    \
    }                                                                                                      \
  } while (0)
#define GEEK_DMA_STAGE(C0, B)                                                                              \
  do {                                                                                                     \
    _Pragma("unroll") for (int u = 0; u < CH / 4; ++u) {                                                  \
      const int slot0 = w * (SCAN_BC * CH / 4) + u * 64; /* wave-uniform LDS chunk */                     \
      const int slot = slot0 + lane;                                                                       \
      const int r = slot / CH, c = (slot % CH) ^ (r & (CH - 1));                                           \
      __builtin_amdgcn_global_load_lds(                                                                    \
          reinterpret_cast<const char*>(cl + (int64_t)((C0) + r) * DP) + c * 16,                           \
          reinterpret_cast<char*>(cbuf(IC<(B)>{})) + slot0 * 16, 16, 0, 0);                               \
    }                                                                                                      \
    /* raw |c|^2 in a register, converted when lds_nc[B] is stored: a use here \
       would make the wave wait for the whole stage at once */                 \
    stg_nc = nc[(C0) + (tid & (SCAN_BC - 1))];                                                             \
    if constexpr (HET)                                                                                     \
      __builtin_amdgcn_global_load_lds(                                                                    \
          reinterpret_cast<const char*>(het.mode16 + (int64_t)(C0) * MAX_CAT) + (w * 64 + lane) * 16,     \
          reinterpret_cast<char*>(mbuf(IC<(B)>{})) + w * 64 * 16, 16, 0, 0);                              \
  } while (0)

  for (int64_t tile = tile0; tile < tile_end && tile * BN < count; tile += tstep) {
    typename M::frag xb[NCB][S];
    float twoeps[NCB];
    int32_t crow[NCB][HET ? MAX_CAT : 1];
    bool valid[NCB];
    int64_t posv[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int64_t pos = tile * BN + (int64_t)w * (32 * NCB) + cb * 32 + p;
      valid[cb] = pos < count;
      posv[cb] = pos;
      const int64_t i = valid[cb] ? (rows ? (int64_t)rows[pos] : pos) : 0;
      const float* xr = X + i * ldx;
      // this lane's half row of x as MFMA B fragments; exact |x|^2
      float xv[DP / 2];
#pragma unroll
      for (int q = 0; q < DP / 2; q += 4) {
        const int t0 = h * (DP / 2) + q;
        float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
        if (valid[cb]) {
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
#pragma unroll
      for (int s = 0; s < S; ++s) xb[cb][s] = M::from_f32(xv + s * M::KPER, sc);
      if (!finite) set_status(st, GEEK_ERR_NONFINITE);
      nrm += __shfl_xor(nrm, 32);
      twoeps[cb] = two_eps<M, DP, T2, BLK>(sqrt(nrm) * (1.0 + 1e-12), cm, 1.0 / sc, het_max);
      if constexpr (HET) {
#pragma unroll
        for (int a = 0; a < MAX_CAT; ++a)
          crow[cb][a] = (valid[cb] && a < het.n_cat) ? het.cat[i * het.n_cat + a] : 0;
      }
    }

    // Window: thr starts at the largest finite float, so padded centroids
    // (|c|^2 = +inf) and non-finite values never enter it; lost is the
    // smallest value dropped from a full window.
    // T2: best (a1) and second best (a2) of the values seen, in accumulator
    // units where larger is nearer.  Each value carries its position within
    // the lane's 16 values of a 32-centroid block in its low 4 mantissa bits;
    // blk is the block where a1 last changed.
    float b0[NCB], thr[NCB], lost[NCB];
    // thr at the window's last compaction: while thr has not dropped below
    // it, every stored value is still within thr and a compaction of a full
    // window would keep all of them, so it is skipped
    float cthr[NCB];
    int cnt[NCB];
    float a1[NCB], a2[NCB];
    int blk[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      b0[cb] = INFINITY;
      thr[cb] = 3.402823466e38f;
      lost[cb] = INFINITY;
      cthr[cb] = INFINITY;
      cnt[cb] = 0;
      a1[cb] = -3.402823466e38f;
      a2[cb] = -3.402823466e38f;
      blk[cb] = 0;
    }

    __syncthreads();  // previous tile done with the LDS buffers
    if constexpr (DMA) {
      GEEK_DMA_STAGE(0, 0);
      if (tid < SCAN_BC) lds_nc[0][tid] = nc_stage(stg_nc);
      __builtin_amdgcn_s_waitcnt(0);
    } else {
      GEEK_LOAD_REGS(0);
      GEEK_STORE_LDS(0);
    }
    __syncthreads();
    // T2: values of 32 centroids enter the running best two with one bit
    // insert and two med3 each; blk records the block where a1 changed
    auto t2_update = [&](int cb, const f32x16& t, int gb) {
      const float a1_prev = a1[cb];
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        const float u = __uint_as_float((__float_as_uint(t[r]) & ~15u) | (uint32_t)r);
        const float v = __uint_as_float((__float_as_uint(t[r + 1]) & ~15u) | (uint32_t)(r + 1));
        // with a1 >= a2: the second best of {a1, a2, u, v} is
        // max(a2, median(a1, u, v)); the best is max(a1, u, v)
        const float mid = __builtin_amdgcn_fmed3f(a1[cb], u, v);
        a1[cb] = fmaxf(fmaxf(a1[cb], u), v);
        a2[cb] = fmaxf(a2[cb], mid);
      }
      blk[cb] = a1[cb] != a1_prev ? gb : blk[cb];
    };
    // T2 fast path: the second block's accumulators of a stage are carried
    // into the next stage, whose first block's products run while their
    // values enter the running best two (the same order of updates)
    f32x16 pendB[T2 ? NCB : 1];
    int pend_g = -1;
    // one stage of SCAN_BC centroids from buffer `cur` (a compile-time
    // constant), with the next stage loading into the other buffer
    auto stage = [&](auto curc, const int c0, const int it) {
      constexpr int cur = NBUF == 2 ? decltype(curc)::value : 0;
      constexpr int nxt = NBUF == 2 ? 1 - cur : 0;
      const bool more = c0 + SCAN_BC < k_pad;
      if constexpr (DMA) {
        if (more) GEEK_DMA_STAGE(c0 + SCAN_BC, nxt);
      } else {
        if (NBUF == 2 && more) GEEK_LOAD_REGS(c0 + SCAN_BC);
      }

      // A fragments of a 32-row block: all S of them in registers, the next
      // block's loaded while this block's epilogue runs (modes with at most
      // eight K steps per block; float32's 64 steps read them one by one)
      constexpr bool PF = !BLK && S <= 8;
      auto afrag_rb = [&](int rb, int s) {
        const int R = rb * 32 + p;
        if constexpr (DMA) {
          const char* rowp = reinterpret_cast<const char*>(cbuf(IC<cur>{})) + R * CH * 16;
          const int off = (h * (DP / 2) + s * M::KPER) * (int)sizeof(CE);
          return M::load_lds(reinterpret_cast<const CE*>(rowp + (((off >> 4) ^ (R & (CH - 1))) << 4) + (off & 15)));
        } else {
          return M::load_lds(cbuf(IC<cur>{}) + R * STR + h * (DP / 2) + s * M::KPER);
        }
      };
      typename M::frag af[PF ? S : 1];
      if constexpr (PF) {
#pragma unroll
        for (int s = 0; s < S; ++s) af[s] = afrag_rb(0, s);
      }
      // first pass of point rows (top two, no categorical part): both 32-row
      // blocks of the stage go to the matrix cores back to back, into two
      // accumulator sets, so the first block's epilogue runs while the
      // second block's products are still in the matrix pipe
      if constexpr (T2 && PF && !HET && SCAN_BC == 64) {
        f32x16 accA[NCB], accB[NCB];
        {
          f32x16 initA;
#pragma unroll
          for (int r = 0; r < 16; ++r) initA[r] = lds_nc[cur][(r >> 2) * 8 + h * 4 + (r & 3)];
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) accA[cb] = initA;
        }
        if (pend_g >= 0) {
          // block A's products step by step, each followed by its share of
          // the previous stage's block B values
          float a1q[NCB];
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) a1q[cb] = a1[cb];
#pragma unroll
          for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) accA[cb] = M::mma(af[s], xb[cb][s], accA[cb]);
#pragma unroll
            for (int q = 8 * s / S; q < 8 * (s + 1) / S; ++q) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) {
                const int r = 2 * q;
                const float u = __uint_as_float((__float_as_uint(pendB[cb][r]) & ~15u) | (uint32_t)r);
                const float v = __uint_as_float((__float_as_uint(pendB[cb][r + 1]) & ~15u) | (uint32_t)(r + 1));
                const float mid = __builtin_amdgcn_fmed3f(a1[cb], u, v);
                a1[cb] = fmaxf(fmaxf(a1[cb], u), v);
                a2[cb] = fmaxf(a2[cb], mid);
              }
            }
            if (s + 1 < S) {
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) asm volatile("" : "+v"(af[s + 1]) : "v"(a1[cb]), "v"(a2[cb]));
            }
          }
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) blk[cb] = a1[cb] != a1q[cb] ? pend_g : blk[cb];
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) accA[cb] = M::mma(af[s], xb[cb][s], accA[cb]);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) af[s] = afrag_rb(1, s);
        {
          f32x16 initB;
#pragma unroll
          for (int r = 0; r < 16; ++r) initB[r] = lds_nc[cur][32 + (r >> 2) * 8 + h * 4 + (r & 3)];
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) accB[cb] = initB;
        }
        const int g0 = it * (SCAN_BC / 32);
        // block B's products step by step, each step followed by its share
        // of block A's eight value pairs per column block: the vector
        // instructions issue while the matrix pipe works on B
        float a1p[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) a1p[cb] = a1[cb];
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) accB[cb] = M::mma(af[s], xb[cb][s], accB[cb]);
#pragma unroll
          for (int q = 8 * s / S; q < 8 * (s + 1) / S; ++q) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
              const int r = 2 * q;
              const float u = __uint_as_float((__float_as_uint(accA[cb][r]) & ~15u) | (uint32_t)r);
              const float v = __uint_as_float((__float_as_uint(accA[cb][r + 1]) & ~15u) | (uint32_t)(r + 1));
              const float mid = __builtin_amdgcn_fmed3f(a1[cb], u, v);
              a1[cb] = fmaxf(fmaxf(a1[cb], u), v);
              a2[cb] = fmaxf(a2[cb], mid);
            }
          }
          // the next step's fragment "depends" on this step's updates (an
          // empty asm, no instruction): its products issue after them
          if (s + 1 < S) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) asm volatile("" : "+v"(af[s + 1]) : "v"(a1[cb]), "v"(a2[cb]));
          }
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) blk[cb] = a1[cb] != a1p[cb] ? g0 : blk[cb];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) pendB[cb] = accB[cb];
        pend_g = g0 + 1;
      } else
#pragma unroll 1
      for (int rb = 0; rb < SCAN_BC / 32; ++rb) {
        const int jb = rb * 32;
        f32x16 acc[NCB];
        f32x16 init = f32x16{};
        if constexpr (T2) {
#pragma unroll
          for (int r = 0; r < 16; ++r) init[r] = lds_nc[cur][jb + (r >> 2) * 8 + h * 4 + (r & 3)];
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = init;
        const CE* ap = cbuf(IC<cur>{}) + (rb * 32 + p) * STR + h * (DP / 2);
        const int R = rb * 32 + p;
        const char* rowp = reinterpret_cast<const char*>(cbuf(IC<cur>{})) + R * CH * 16;
        auto afrag = [&](int s) {
          if constexpr (DMA) {
            const int off = (h * (DP / 2) + s * M::KPER) * (int)sizeof(CE);
            return M::load_lds(reinterpret_cast<const CE*>(rowp + (((off >> 4) ^ (R & (CH - 1))) << 4) + (off & 15)));
          } else {
            return M::load_lds(ap + s * M::KPER);
          }
        };
        if constexpr (BLK) {
          // blocks of KB products (KB / (2 KPER) steps) in fresh accumulators,
          // then added to the running sums (see two_eps)
          constexpr int SB = M::KB / (2 * M::KPER);
#pragma unroll
          for (int s0 = 0; s0 < S; s0 += SB) {
            f32x16 blk[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) blk[cb] = f32x16{};
#pragma unroll
            for (int s = s0; s < s0 + SB; ++s) {
              const typename M::frag a = afrag(s);
#pragma unroll
              for (int cb = 0; cb < NCB; ++cb) blk[cb] = M::mma(a, xb[cb][s], blk[cb]);
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
              for (int r = 0; r < 16; ++r) acc[cb][r] += blk[cb][r];
          }
        } else if constexpr (PF) {
#pragma unroll
          for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[cb] = M::mma(af[s], xb[cb][s], acc[cb]);
          }
          if (rb + 1 < SCAN_BC / 32) {
#pragma unroll
            for (int s = 0; s < S; ++s) af[s] = afrag_rb(rb + 1, s);
          }
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const typename M::frag a = afrag(s);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[cb] = M::mma(a, xb[cb][s], acc[cb]);
          }
        }
        if constexpr (T2) {
          // branch-free: per value one bit insert and two med3
          const int gblk = it * (SCAN_BC / 32) + rb;
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) {
            float t[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              t[r] = acc[cb][r];
              if constexpr (HET) {
                // -(v_num + gamma * mismatches), one rounding
                const uint32_t* md = mbuf(IC<cur>{}) + (jb + (r >> 2) * 8 + h * 4 + (r & 3)) * MAX_CAT;
                int mm = 0;
#pragma unroll
                for (int q = 0; q < MAX_CAT; ++q) mm += (q < het.n_cat && (uint32_t)crow[cb][q] != md[q]) ? 1 : 0;
                t[r] = __builtin_fmaf(-m2s, t[r], -het.gamma_f * (float)mm);
              }
            }
            f32x16 tv;
#pragma unroll
            for (int r = 0; r < 16; ++r) tv[r] = t[r];
            t2_update(cb, tv, gblk);
          }
        } else {
        float ncv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) ncv[r] = lds_nc[cur][jb + (r >> 2) * 8 + h * 4 + (r & 3)];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          float v[16];
          float vmin = INFINITY;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            v[r] = __builtin_fmaf(m2s, acc[cb][r], ncv[r]);
            if constexpr (HET) {
              const uint32_t* md = mbuf(IC<cur>{}) + (jb + (r >> 2) * 8 + h * 4 + (r & 3)) * MAX_CAT;
              int mm = 0;
#pragma unroll
              for (int a = 0; a < MAX_CAT; ++a) mm += (a < het.n_cat && (uint32_t)crow[cb][a] != md[a]) ? 1 : 0;
              v[r] = v[r] + het.gamma_f * (float)mm;
            }
            vmin = fminf(vmin, v[r]);
          }
          if (vmin <= thr[cb]) {
            float* lv = lds_lv + (tid * NCB + cb) * TC;
            int* lj = lds_lj + (tid * NCB + cb) * TC;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              if (v[r] <= thr[cb]) {
                const int j = c0 + jb + (r >> 2) * 8 + h * 4 + (r & 3);
                if (v[r] < b0[cb]) {
                  b0[cb] = v[r];
                  thr[cb] = b0[cb] + twoeps[cb];
                }
                if (cnt[cb] == TC && thr[cb] < cthr[cb]) {
                  cthr[cb] = thr[cb];
                  int kept = 0;
#pragma unroll 1
                  for (int q = 0; q < TC; ++q) {
                    const float ev = lv[q];
                    const int ej = lj[q];
                    if (ev <= thr[cb]) {
                      lv[kept] = ev;
                      lj[kept] = ej;
                      ++kept;
                    }
                  }
                  cnt[cb] = kept;
                }
                if (cnt[cb] < TC) {
                  lv[cnt[cb]] = v[r];
                  lj[cnt[cb]] = j;
                  ++cnt[cb];
                } else {
                  lost[cb] = fminf(lost[cb], v[r]);
                }
              }
            }
          }
        }
        }
      }
      if (more) {
        if constexpr (DMA) {
          if (tid < SCAN_BC) lds_nc[nxt][tid] = nc_stage(stg_nc);
          __builtin_amdgcn_s_waitcnt(0);  // this wave's chunks of the next stage landed
        } else if (NBUF == 2) {
          GEEK_STORE_LDS(nxt);
        } else {
          __syncthreads();
          GEEK_LOAD_REGS(c0 + SCAN_BC);
          GEEK_STORE_LDS(0);
        }
      }
      __syncthreads();
    };
    for (int c0 = 0, it = 0; c0 < k_pad;) {
      stage(IC<0>{}, c0, it);
      c0 += SCAN_BC;
      ++it;
      if constexpr (NBUF == 2) {
        if (c0 < k_pad) {
          stage(IC<1>{}, c0, it);
          c0 += SCAN_BC;
          ++it;
        }
      }
    }

    if constexpr (T2) {  // the last stage's second block
      if (pend_g >= 0) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) t2_update(cb, pendB[cb], pend_g);
      }
    }

    // ---- merge the two lanes that share a point, write the candidate record
    if constexpr (T2) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float a1o = __shfl_xor(a1[cb], 32), a2o = __shfl_xor(a2[cb], 32);
        const int blko = __shfl_xor(blk[cb], 32);
        const bool mine = a1[cb] > a1o;  // equal values: a tie, never unique
        const float best = mine ? a1[cb] : a1o;
        const float second = fmaxf(fminf(a1[cb], a1o), fmaxf(a2[cb], a2o));
        const int rbits = (int)(__float_as_uint(best) & 15u);
        const int jbest = (mine ? blk[cb] : blko) * 32 + (rbits >> 2) * 8 + (mine ? h : 1 - h) * 4 + (rbits & 3);
        // back to distance units (exact): v = m2s * acc, or -t for HET
        const float vs = HET ? -1.0f : m2s;
        const float v1 = vs * best, v2 = vs * second;
        // one candidate iff the runner-up lies beyond the 2 eps window; the
        // best must be a normal float (its index bits intact)
        const bool unique = best > -1e37f && best < 1e37f && fabsf(best) >= 0x1p-126f && isfinite(v1) &&
                            v2 > v1 + twoeps[cb] && jbest < k;
        if (valid[cb] && h == 0) {
          int32_t* rr = rec + posv[cb] * RECW_T2;
          rr[0] = unique ? 1 : -1;
          if (unique) rr[1] = jbest;
        }
      }
    } else {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      float* lv = lds_lv + (tid * NCB + cb) * TC;
      int* lj = lds_lj + (tid * NCB + cb) * TC;
      const float bo = __shfl_xor(b0[cb], 32);
      const float bfin = fminf(b0[cb], bo);
      const float tfin = bfin < INFINITY ? bfin + twoeps[cb] : 3.402823466e38f;
      int kept = 0;
      for (int q = 0; q < cnt[cb]; ++q) {
        const float ev = lv[q];
        const int ej = lj[q];
        if (ev <= tfin) {
          lv[kept] = ev;
          lj[kept] = ej;
          ++kept;
        }
      }
      const int kept_o = __shfl_xor(kept, 32);
      const float lost_all = fminf(lost[cb], __shfl_xor(lost[cb], 32));
      // complete unless a dropped value could still be a candidate
      const bool over = lost_all <= tfin || (kept + kept_o > TC);
      if (valid[cb]) {
        int32_t* rr = rec + posv[cb] * RECW;
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
  }
}

#undef GEEK_LOAD_REGS
#undef GEEK_STORE_LDS
#undef GEEK_DMA_STAGE

// One job of a batched first pass (Euclidean rows, one precision, one DP).
struct ScanJob {
  const float* X;
  int64_t ldx;
  int64_t n;
  const void* cl;
  const float* nc;
  const float* cmax;
  const float* scale;
  int32_t* rec;
  int64_t tile_begin;  // first global tile of this job
  int d, k, k_pad, pad0;
};
// Tile shape of the batched first pass for one (precision, padded depth):
// column blocks per wave (rows per tile = 128 * ncb), LDS stages, and
// persistent workgroups per compute unit.
struct ScanTiles {
  int ncb, nbuf, blocks_per_cu;
};
ScanTiles scan_tiles_get(int precision, int dp);
int32_t scan_tiles_set(int precision, int dp, ScanTiles t);
// Launches the batched first pass of one padded depth with the current tile
// shape; `table` holds nj jobs whose tile_begin were laid out with
// 128 * ncb rows per tile.
void launch_scan_batch(int precision, int dp, const ScanJob* table, int nj, int64_t total_tiles, int32_t* st,
                       hipStream_t s);

// Persistent first pass over the tiles of many jobs: global tile gt belongs
// to the last job whose tile_begin <= gt; every tile runs exactly the
// single-job code, so each job's records equal those of its own launch.
template <class M, int DP, int NCB, int NBUF, bool T2>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_batch(const ScanJob* __restrict__ jobs, int njobs,
                                                             int64_t total_tiles, int32_t* st) {
  const Het none{nullptr, nullptr, nullptr, 0, 0.f, 0.0};
  for (int64_t gt = blockIdx.x; gt < total_tiles; gt += gridDim.x) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].tile_begin <= gt) lo = mid;
      else hi = mid - 1;
    }
    const ScanJob J = jobs[lo];
    const int64_t tile = gt - J.tile_begin;
    scan_tiles<M, DP, false, NCB, NBUF, T2, false>(J.X, J.ldx, J.d, J.n, nullptr, nullptr,
                                            static_cast<const typename M::ce*>(J.cl), J.nc, J.k_pad, J.cmax,
                                            J.scale, none, J.k, J.rec, st, tile, tile + 1, 1);
  }
}


}  // namespace geek
