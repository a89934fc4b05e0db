// LSH values of the data transformation (paper Section 3.1) on gfx950.
//
// Dense E2LSH: code[i][p] = floor((a_p . x_i + b_p) / w).  The projection is
// a GEMM X[n x d] . A^T[d x P] on the matrix cores (for d <= 128 from exact
// three-piece bf16 splits of a and x, else in float32); the epilogue adds
// b, scales by 1/w, floors and certifies the result: the float32 quotient q
// differs from the float64 reference quotient (sum over t in order, + b, / w)
// by at most tau = c * (|a_p| |x_i| + |b_p|) / w, so when [q - tau, q + tau]
// holds no integer the float32 floor equals the reference floor.  Otherwise
// the pair gets a float64 dot product (FMA, by the two lanes that hold x), certified the same way
// with a radius of a few float64 ulps, and only the pairs that this leaves
// open are summed in exactly the reference order.  The m codes of each table
// are then packed into a 128-bit exact key.
//
// MinHash of sets / heterogeneous rows: one wavefront per object; lane f
// handles functions f, f+64, ...; the tokens of the object are loaded once
// and broadcast, so each lane runs a plain min over the set with no
// cross-lane reduction.
#include <math.h>

#include <type_traits>

#include <mutex>

#include "common.hpp"

namespace geek {

constexpr int H_THREADS = 256;
constexpr int H_BN = 128;   // points per block
constexpr int H_BC = 64;    // projection rows per chunk (two 32-row MFMA blocks)
constexpr int H_CS = H_BC + 1;  // LDS stride of a point's codes (odd: conflict-free stores)
constexpr int H_KB = 16;        // products per accumulation block of the GEMM

// Certification constant of the projection: |q_fast - q64| <= coef *
// (|a||x| + |b|) / w.  Float32 products (B3 false): the GEMM sums blocks of
// H_KB products in fresh accumulators and then adds the block sums to
// accumulators that start at b, so a term passes through at most H_KB +
// DP/H_KB + 1 roundings (2u each); then * (1/w) with 1/w rounded, and the
// float64 reference's own rounding.  Bfloat16 pieces (B3 true): a and x are
// each the exact sum of three bf16 pieces (hi, mid, lo; round-to-nearest
// splits, so |mid| <= 2^-8 |v| and |lo| <= 2^-16 |v|); a K step of 16 sums
// mid*mid, hi*lo, lo*hi, hi*mid, mid*hi and last hi*hi in one fresh
// accumulator (every bf16 product is exact in float32), which is then added
// to the running sums: the hi*hi terms (at most (1 + 2^-8)^2 |a_t x_t|)
// see the same 16 + DP/16 + 1 roundings, the smaller terms (at most
// (2^-7 + 3 * 2^-16)(1 + 2^-8)^2 |a_t x_t| together) up to 6 * 16 + DP/16
// + 1, and the dropped mid*lo, lo*mid, lo*lo are at most 2^-23 |a_t x_t| +
// 2^-32 |a_t x_t|.
template <int DP, bool B3>
GEEK_HD double e2lsh_coef() {
  const double u32 = 0x1p-24;
  constexpr int NR = H_KB + DP / H_KB + 1;
  const double main = NR * 2.0 * u32 / (1.0 - NR * 2.0 * u32) * (B3 ? 1.0079 : 1.0);
  constexpr int NRS = 6 * H_KB + DP / H_KB + 1;
  const double small =
      B3 ? (NRS * 2.0 * u32 / (1.0 - NRS * 2.0 * u32)) * 0x1.06p-7 + 0x1p-23 + 0x1p-32 : 0.0;
  return (main + small + 6.0 * u32 + (DP + 3) * 0x1p-53) * 1.01;
}

// One chunk of projection rows (whole tables, at most H_BC rows) in the
// hash kernel's LDS: H_BC rows of a in float32, zero-padded to DP
// attributes and to H_BC rows, at a stride of DP + 4 floats; with B3 the
// three bf16 pieces of the same rows (hi, mid, lo; a = hi + mid + lo
// exactly), each at a stride of DP + 8 bf16; then per row b, t1 and t0 (the
// radius tau = t1 * |x| + t0) and |a| rounded up, H_BC each; then the
// chunk's largest |a| and |b| and two unused words.  `k_e2lsh_prep` writes
// the same image to global memory without the 16-byte pad of each row, and
// the hash kernel copies it to LDS with LDS DMA, one 16-byte piece per lane,
// filling each row's pad with a duplicate piece.
template <int DP, bool B3>
struct E2Chunk {
  static constexpr int CH = DP / 4;                // 16-byte pieces of a float32 row
  static constexpr int STR = DP + 4;               // LDS float32 row stride (floats)
  static constexpr int NPC = B3 ? 3 : 0;           // bf16 pieces per row
  static constexpr int PCH = DP / 8;               // 16-byte pieces of a bf16 row
  static constexpr int PSTR = DP / 2 + 4;          // LDS bf16 row stride (floats)
  static constexpr int INFO = 4 * H_BC + 4;        // b, t1, t0, |a|, maxima
  static constexpr int G_A = H_BC * DP;            // global: float32 rows (floats)
  static constexpr int G_P = H_BC * DP / 2;        // global: one bf16 piece of the rows (floats)
  static constexpr int G_FLOATS = G_A + NPC * G_P + INFO;  // per chunk in global memory
  static constexpr int L_A = H_BC * STR;
  static constexpr int L_P = H_BC * PSTR;
  static constexpr int L_INFO = L_A + NPC * L_P;   // LDS offset of the per-row data (floats)
  static constexpr int L_FLOATS = L_INFO + INFO;
  static constexpr int PIECES = L_FLOATS / 4;
  static constexpr int A_PIECES = H_BC * (CH + 1);
  static constexpr int P_PIECES = H_BC * (PCH + 1);
};

// Chunk c = blockIdx.x holds tables c*tpc .. c*tpc + tpc - 1 (rows
// c*tpc*m ..).  |a| is the float64 norm in attribute order, rounded up.
template <int DP, bool B3>
__global__ __launch_bounds__(H_THREADS) void k_e2lsh_prep(const float* __restrict__ A, const float* __restrict__ bvec,
                                                          int d, int m, int L, float w, int tpc,
                                                          float* __restrict__ out) {
  using C = E2Chunk<DP, B3>;
  const int c = blockIdx.x, tid = threadIdx.x;
  const int tb = c * tpc;
  const int ntab = (L - tb) < tpc ? (L - tb) : tpc;
  const int rows_used = ntab * m, p0 = tb * m;
  float* o = out + (int64_t)c * C::G_FLOATS;
  __bf16* pc = reinterpret_cast<__bf16*>(o + C::G_A);
  for (int q = tid; q < H_BC * DP; q += H_THREADS) {
    const int r = q / DP, k = q % DP;
    const float v = (r < rows_used && k < d) ? A[(int64_t)(p0 + r) * d + k] : 0.f;
    o[q] = v;
    if constexpr (B3) {
      const __bf16 hi = (__bf16)v;
      const float r1 = v - (float)hi;
      const __bf16 mid = (__bf16)r1;
      pc[q] = hi;
      pc[2 * C::G_P + q] = mid;
      pc[4 * C::G_P + q] = (__bf16)(r1 - (float)mid);
    }
  }
  if (tid < H_BC) {  // wavefront 0: one row per lane
    const bool live = tid < rows_used;
    double ss = 0.0;
    if (live)
      for (int k = 0; k < d; ++k) {
        const double v = (double)A[(int64_t)(p0 + tid) * d + k];
        ss += v * v;
      }
    const float an = live ? (float)(sqrt(ss) * (1.0 + 0x1p-20)) : 0.f;
    const float bv = live ? bvec[p0 + tid] : 0.f;
    const float inv_w = 1.0f / w;
    const float tscale = (float)e2lsh_coef<DP, B3>() * inv_w;
    float* info = o + C::G_A + C::NPC * C::G_P;
    info[tid] = bv;
    info[H_BC + tid] = tscale * an;
    info[2 * H_BC + tid] = live ? __builtin_fmaf(tscale, fabsf(bv), 0x1p-22f) : 0.f;
    info[3 * H_BC + tid] = an;
    float am = an, bm = fabsf(bv);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      am = fmaxf(am, __shfl_xor(am, off));
      bm = fmaxf(bm, __shfl_xor(bm, off));
    }
    if (tid < 4) info[4 * H_BC + tid] = tid == 0 ? am : tid == 1 ? bm : 0.f;
  }
}

// The keys of point pk of a block for tables t0, t0 + step, ... < ntab
// (table tb + t): code j + 2^(B-1) at bits j*B .. j*B+B-1 of four words,
// little-endian.  M > 0 fixes m at compile time (shifts and words become
// constants); M == 0 takes m at run time.  Returns the OR of the offset
// codes (a code is in range when that OR has no bit at or above B).
template <int M>
__device__ __forceinline__ uint32_t pack_keys(const int* __restrict__ lds_code, int pk, int t0, int step,
                                              int ntab, int tb, int m_rt, int B_rt, uint32_t code_off,
                                              int64_t n, int64_t ii, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ key_fp) {
  const int m = M > 0 ? M : m_rt;
  const int B = M > 0 ? (128 / M < 32 ? 128 / M : 32) : B_rt;
  uint32_t orr = 0u;
  for (int t = t0; t < ntab; t += step) {
    const int* cp = lds_code + pk * H_CS + t * m;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if constexpr (M > 0) {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const uint32_t u = (uint32_t)cp[j] + code_off;
        orr |= u;
        const int bit = j * B, sh = bit & 31;
        w[bit >> 5] |= u << sh;
        if (sh + B > 32) w[(bit >> 5) + 1] |= u >> (32 - sh);
      }
    } else {
      for (int j = 0; j < m; ++j) {
        const uint32_t u = (uint32_t)cp[j] + code_off;
        orr |= u;
        const int bit = j * B, sh = bit & 31;
        const bool spill = sh + B > 32;  // the code continues in the next word
        switch (bit >> 5) {
          case 0:
            w[0] |= u << sh;
            if (spill) w[1] |= u >> (32 - sh);
            break;
          case 1:
            w[1] |= u << sh;
            if (spill) w[2] |= u >> (32 - sh);
            break;
          case 2:
            w[2] |= u << sh;
            if (spill) w[3] |= u >> (32 - sh);
            break;
          default:
            w[3] |= u << sh;
        }
      }
    }
    const int64_t at = (int64_t)(tb + t) * n + ii;
    *reinterpret_cast<uint4*>(keys + at * 4) = make_uint4(w[0], w[1], w[2], w[3]);
    // the key's fingerprint as bucketize takes it (all four words)
    if (key_fp) key_fp[at] = key_hash(w, 4);
  }
  return orr;
}

// Two floats to packed bf16 (round to nearest even -- the instruction the
// compiler itself emits for a float-to-bf16 conversion; the first in the
// low half).  An opaque instruction: the split of x is loop-invariant, and
// hoisted out of the chunk loop it would hold 96 more VGPRs.
GEEK_D uint32_t cvt_pk_bf16(float a, float b) {
  uint32_t r;
  asm volatile("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

// The three bf16 pieces of eight floats: v = hi + mid + lo exactly (each
// remainder is exact in float32).
GEEK_D void split3_bf16(const float* v, bf16x8& hi, bf16x8& mid, bf16x8& lo) {
  u32x4v H, M, O;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float v0 = v[2 * q], v1 = v[2 * q + 1];
    const uint32_t h = cvt_pk_bf16(v0, v1);
    const float r0 = v0 - __uint_as_float(h << 16), r1 = v1 - __uint_as_float(h & 0xFFFF0000u);
    const uint32_t mm = cvt_pk_bf16(r0, r1);
    const float s0 = r0 - __uint_as_float(mm << 16), s1 = r1 - __uint_as_float(mm & 0xFFFF0000u);
    H[q] = h;
    M[q] = mm;
    O[q] = cvt_pk_bf16(s0, s1);
  }
  hi = __builtin_bit_cast(bf16x8, H);
  mid = __builtin_bit_cast(bf16x8, M);
  lo = __builtin_bit_cast(bf16x8, O);
}

// Wavefront wv owns 32 points; lane (p, h) holds point p's x at the K
// indices kidx(h, s), s < DP/2: the K half h (float32 products, 32x32x2
// fragments) or, with B3, the 8-wide half h of every 16-wide K step
// (32x32x16 bf16 fragments).  B3 blocks have eight wavefronts (the chunk
// image with its bf16 pieces leaves LDS for one block per CU).
template <int DP, bool B3>
GEEK_D constexpr int e2lsh_kidx(int h, int s) {
  return B3 ? (s / 8) * 16 + h * 8 + (s % 8) : h * (DP / 2) + s;
}

template <int DP, bool B3>
__global__ __launch_bounds__(B3 ? 2 * H_THREADS : H_THREADS, B3 ? 1 : 2) void k_e2lsh(
    const float* __restrict__ X, int64_t ldx, int d, int64_t n, const float* __restrict__ chunks, int m,
    int L, float w, int tpc, uint32_t* __restrict__ keys, uint32_t* __restrict__ key_fp,
    int32_t* __restrict__ codes_out, unsigned long long* __restrict__ n_fixup, int32_t* st) {
  using C = E2Chunk<DP, B3>;
  constexpr int S = DP / 2;
  constexpr int STR = C::STR;
  constexpr int NT = B3 ? 2 * H_THREADS : H_THREADS;  // threads per block
  constexpr int BPTS = NT / 2;                        // points per block
  constexpr int DMA_ROUNDS = (C::PIECES + NT - 1) / NT;
  // the chunk's rows of a (and their bf16 pieces), then per row b, the two
  // factors of the certification radius tau = t1 * |x| + t0, |a_p| rounded
  // up, and the chunk's largest |a_p| and |b_p| (layout of E2Chunk)
  __shared__ __attribute__((aligned(16))) float lds_chunk[C::L_FLOATS];
  float* const lds_a = lds_chunk;
  float* const lds_b = lds_chunk + C::L_INFO;
  float* const lds_t1 = lds_b + H_BC;
  float* const lds_t0 = lds_t1 + H_BC;
  float* const lds_an = lds_t0 + H_BC;
  float* const lds_qb = lds_an + H_BC;
  // codes of a point are H_CS ints apart: the epilogue's stores (one row,
  // 32 points per instruction) then fall into distinct banks
  __shared__ int lds_code[BPTS * H_CS];

  const int P = m * L;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int p = lane & 31, h = lane >> 5;
  const int64_t i0 = (int64_t)blockIdx.x * BPTS;
  const int64_t i = i0 + wv * 32 + p;
  const bool valid = i < n;
  const float* xr = X + (valid ? i : 0) * ldx;
  const bool vec4 = ((d & 3) == 0) && ((ldx & 3) == 0);
  const float inv_w = 1.0f / w;
  const int B = 128 / m < 32 ? 128 / m : 32;
  const uint32_t code_off = B == 32 ? 0x80000000u : (1u << (B - 1));
  const int wu = __builtin_amdgcn_readfirstlane(wv);  // wave-uniform, for the LDS DMA bases

  // Copy of chunk c into LDS: 16-byte piece q of the LDS image from its
  // place in the global image (a row's pad piece takes the row's first
  // piece).  Lane-contiguous pieces, one DMA instruction per wave and round.
  auto issue_chunk = [&](int c) {
    const float* g = chunks + (int64_t)c * C::G_FLOATS;
#pragma unroll
    for (int u = 0; u < DMA_ROUNDS; ++u) {
      const int q0 = u * NT + wu * 64;  // wave-uniform first piece
      const int q = q0 + lane;
      if (q0 < C::PIECES && q < C::PIECES) {
        int src;
        if (q < C::A_PIECES) {
          const int r = q / (C::CH + 1), pc = q % (C::CH + 1);
          src = r * DP + (pc < C::CH ? pc * 4 : 0);
        } else if (q < C::A_PIECES + C::NPC * C::P_PIECES) {
          const int qq = q - C::A_PIECES, seg = qq / C::P_PIECES, rr = qq % C::P_PIECES;
          const int r = rr / (C::PCH + 1), pc = rr % (C::PCH + 1);
          src = C::G_A + seg * C::G_P + r * (DP / 2) + (pc < C::PCH ? pc * 4 : 0);
        } else {
          src = C::G_A + C::NPC * C::G_P + (q - C::A_PIECES - C::NPC * C::P_PIECES) * 4;
        }
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(g + src),
                                         reinterpret_cast<void*>(lds_chunk + q0 * 4), 16, 0, 0);
      }
    }
  };
  issue_chunk(0);

  // ---- x fragments (K index of step s for half h: h*DP/2 + s), exact |x|^2
  float xb[S];
#pragma unroll
  for (int q = 0; q < S; q += 4) {
    const int t0 = e2lsh_kidx<DP, B3>(h, q);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
      if (vec4 && t0 + 3 < d) {
        v = *reinterpret_cast<const float4*>(xr + t0);
      } else {
        v.x = t0 < d ? xr[t0] : 0.f;
        v.y = t0 + 1 < d ? xr[t0 + 1] : 0.f;
        v.z = t0 + 2 < d ? xr[t0 + 2] : 0.f;
        v.w = t0 + 3 < d ? xr[t0 + 3] : 0.f;
      }
    }
    xb[q] = v.x;
    xb[q + 1] = v.y;
    xb[q + 2] = v.z;
    xb[q + 3] = v.w;
  }
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < S; ++q) nrm += (double)xb[q] * (double)xb[q];
  nrm += __shfl_xor(nrm, 32);
  // a NaN or infinite attribute makes the float64 sum of squares NaN or
  // infinite; finite float32 values cannot overflow it (d * FLT_MAX^2 is far
  // below DBL_MAX)
  if (!isfinite(nrm)) set_status(st, GEEK_ERR_NONFINITE);
  const float xn = (float)(sqrt(nrm) * (1.0 + 0x1p-20));
  // second stage (float64 dot: four FMA chains per K half, summed pairwise,
  // then across the halves; + b; * (1/w) with 1/w rounded): |q_fast - q64|
  // <= coef64 * (|a||x| + |b|) / w, covering both float64 evaluations
  const double coef64 = ((DP / 8 + 8) + (DP + 3)) * 0x1p-53 * 1.02;
  const double inv_wd = 1.0 / (double)w;


  unsigned long long nfix = 0;  // uncertified pairs owned by this lane
  for (int tb = 0; tb < L; tb += tpc) {
    const int ntab = (L - tb) < tpc ? (L - tb) : tpc;
    const int rows_used = ntab * m;
    const int p0 = tb * m;
    const int c = tb / tpc;
    // this wave's pieces of the chunk have landed; then everyone's
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // the accumulators start at b (b is one more term of the sum)
    f32x16 acc0, acc1;
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
      const float4 b0 = *reinterpret_cast<const float4*>(lds_b + g4 * 8 + h * 4);
      const float4 b1 = *reinterpret_cast<const float4*>(lds_b + 32 + g4 * 8 + h * 4);
      acc0[g4 * 4] = b0.x, acc0[g4 * 4 + 1] = b0.y, acc0[g4 * 4 + 2] = b0.z, acc0[g4 * 4 + 3] = b0.w;
      acc1[g4 * 4] = b1.x, acc1[g4 * 4 + 1] = b1.y, acc1[g4 * 4 + 2] = b1.z, acc1[g4 * 4 + 3] = b1.w;
    }
    if constexpr (B3) {
      // K step ks: x's three bf16 pieces for this lane's 8 K indices, split
      // here from the float32 copy (kept for the float64 checks), and a's
      // pieces from LDS; the small products first, hi*hi last, in a fresh
      // accumulator that is then added to the running sums
      const __bf16* pa = reinterpret_cast<const __bf16*>(lds_chunk + C::L_A);
      auto afrag = [&](int seg, int row, int ks) -> bf16x8 {
        return *reinterpret_cast<const bf16x8*>(pa + (seg * C::L_P + row * C::PSTR) * 2 + ks * 16 + h * 8);
      };
      const f32x16 zero = {};
      if (rows_used > 32) {
#pragma unroll
        for (int ks = 0; ks < DP / 16; ++ks) {
          bf16x8 xh, xm, xl;
          split3_bf16(xb + ks * 8, xh, xm, xl);
          // one row block's chain after the other: a dependent MFMA takes its
          // accumulator from the previous one without a stall, and only one
          // block's pieces are live at a time
          f32x16 b0, b1;
          {
            const bf16x8 ah = afrag(0, p, ks), am = afrag(1, p, ks), al = afrag(2, p, ks);
            b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, xm, zero, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl, b0, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh, b0, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xm, b0, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, xh, b0, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh, b0, 0, 0, 0);
          }
          {
            const bf16x8 ah = afrag(0, p + 32, ks), am = afrag(1, p + 32, ks), al = afrag(2, p + 32, ks);
            b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, xm, zero, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xl, b1, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, xh, b1, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xm, b1, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, xh, b1, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, xh, b1, 0, 0, 0);
          }
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            acc0[r] += b0[r];
            acc1[r] += b1[r];
          }
        }
      } else {  // the second 32-row block holds no projection of this chunk
#pragma unroll
        for (int ks = 0; ks < DP / 16; ++ks) {
          bf16x8 xh, xm, xl;
          split3_bf16(xb + ks * 8, xh, xm, xl);
          const bf16x8 ah0 = afrag(0, p, ks), am0 = afrag(1, p, ks), al0 = afrag(2, p, ks);
          f32x16 b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am0, xm, zero, 0, 0, 0);
          b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, xl, b0, 0, 0, 0);
          b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al0, xh, b0, 0, 0, 0);
          b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, xm, b0, 0, 0, 0);
          b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am0, xh, b0, 0, 0, 0);
          b0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah0, xh, b0, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 16; ++r) acc0[r] += b0[r];
        }
      }
    } else {
      const float* a0p = lds_a + p * STR + h * S;
      const float* a1p = a0p + 32 * STR;
      // A fragments: four K steps per 16-byte LDS read (rows STR = DP + 4
      // floats apart, so eight consecutive lanes cover all banks)
      // blocks of H_KB / 2 steps (H_KB products per output) accumulate from
      // zero and are then added to the running sums
      if (rows_used > 32) {
  #pragma unroll
        for (int s0 = 0; s0 < S; s0 += H_KB / 2) {
          f32x16 b0 = {}, b1 = {};
  #pragma unroll
          for (int s = s0; s < s0 + H_KB / 2; s += 4) {
            const float4 a0 = *reinterpret_cast<const float4*>(a0p + s);
            const float4 a1 = *reinterpret_cast<const float4*>(a1p + s);
            b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.x, xb[s], b0, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.x, xb[s], b1, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.y, xb[s + 1], b0, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.y, xb[s + 1], b1, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.z, xb[s + 2], b0, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.z, xb[s + 2], b1, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.w, xb[s + 3], b0, 0, 0, 0);
            b1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1.w, xb[s + 3], b1, 0, 0, 0);
          }
  #pragma unroll
          for (int r = 0; r < 16; ++r) {
            acc0[r] += b0[r];
            acc1[r] += b1[r];
          }
        }
      } else {  // the second 32-row block holds no projection of this chunk
  #pragma unroll
        for (int s0 = 0; s0 < S; s0 += H_KB / 2) {
          f32x16 b0 = {};
  #pragma unroll
          for (int s = s0; s < s0 + H_KB / 2; s += 4) {
            const float4 a0 = *reinterpret_cast<const float4*>(a0p + s);
            b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.x, xb[s], b0, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.y, xb[s + 1], b0, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.z, xb[s + 2], b0, 0, 0, 0);
            b0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0.w, xb[s + 3], b0, 0, 0, 0);
          }
  #pragma unroll
          for (int r = 0; r < 16; ++r) acc0[r] += b0[r];
        }
      }
    }
    const int pl = wv * 32 + p;  // point within block
    // Register r of half hf holds row hf*32 + (r/4)*8 + h*4 + r%4.  The
    // lane's uncertified rows collect in `own`, bit hf*16 + r for that row;
    // rows past rows_used (zero A rows) are stored but never flagged or read.
    // |q| < 2^22 for every row of the chunk when (max|a| |x| + max|b|) / w
    // < 2^21: floor, the fraction and the int conversion are then exact.
    // Otherwise (huge x) every row of the point goes to the float64 check.
    const bool qsafe = __builtin_fmaf(lds_qb[0], xn, lds_qb[1]) * inv_w < 0x1p21f;
    uint32_t own = 0u;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half == 1 && rows_used <= 32) break;
      const f32x16& acc = half ? acc1 : acc0;
      uint32_t bad = 0u;
      // registers from the last to the first: each value's sign bit enters
      // at bit 0 as the earlier ones move up (one funnel shift per value)
#pragma unroll
      for (int g4 = 3; g4 >= 0; --g4) {
        const int rbase = half * 32 + g4 * 8 + h * 4;
        const float4 t1 = *reinterpret_cast<const float4*>(lds_t1 + rbase);
        const float4 t0 = *reinterpret_cast<const float4*>(lds_t0 + rbase);
        const float t1v[4] = {t1.x, t1.y, t1.z, t1.w};
        const float t0v[4] = {t0.x, t0.y, t0.z, t0.w};
#pragma unroll
        for (int e = 3; e >= 0; --e) {
          const int r = g4 * 4 + e;
          const float q = acc[r] * inv_w;
          const float fq = floorf(q);
          const float frac = q - fq;  // exact
          const float tau = __builtin_fmaf(t1v[e], xn, t0v[e]);
          // distance to the nearest integer (exact: 1 - frac is exact when
          // it is the smaller) less the radius; negative = not certified
          const float marg = fminf(frac, 1.0f - frac) - tau;
          lds_code[pl * H_CS + rbase + e] = (int)fq;
          bad = __builtin_amdgcn_alignbit(bad, __float_as_uint(marg), 31);
        }
      }
      uint32_t live = 0xFFFFu;
      const int rem = rows_used - half * 32;  // rows of this half in use
      if (rem < 32) {  // the chunk's last rows are padding
        live = 0u;
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
          const int k = rem - g4 * 8 - h * 4;
          live |= ((1u << (k < 0 ? 0 : k > 4 ? 4 : k)) - 1u) << (g4 * 4);
        }
      }
      bad = (qsafe ? bad : 0xFFFFu) & live;
      own |= (valid ? bad : 0u) << (half * 16);
    }
    // ---- float64 check of the uncertified pairs, by the two lanes that hold
    // the point's x (each its half of the K range, in registers).  Both lanes
    // walk the union of their flagged rows in the same order: FMA partial
    // sums over their halves, added across the pair, give q_fast; when no
    // integer lies within coef64 * (|a||x| + |b|) / w of it, its floor is the
    // reference floor, else the lane that owns the row evaluates the
    // reference sum itself.  The owner writes the code it stored before.
    {
      nfix += __popc(own);
      // the pair's union, bit hk*32 + hf*16 + r: lane hk's register r of half hf
      const uint32_t oth = __shfl_xor(own, 32);
      unsigned long long fl = h ? (((unsigned long long)own << 32) | oth) : (((unsigned long long)oth << 32) | own);
      while (__any(fl != 0ull)) {
        const int kb = fl ? __ffsll((long long)fl) - 1 : 0;
        const int hk = kb >> 5;
        const int row = ((kb >> 4) & 1) * 32 + ((kb >> 2) & 3) * 8 + hk * 4 + (kb & 3);
        double part = 0.0;
        if (fl) {
          // four independent FMA chains (k mod 4), then summed pairwise
          const float* ap = lds_a + row * STR;
          double p4[4] = {0.0, 0.0, 0.0, 0.0};
          // the row is read sixteen attributes at a time: four LDS reads in
          // flight per wait
#pragma unroll
          for (int k0 = 0; k0 < S; k0 += 16) {
            float4 av[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              av[u] = *reinterpret_cast<const float4*>(ap + e2lsh_kidx<DP, B3>(h, k0 + 4 * u));
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int k = k0 + 4 * u;
              // x converted to float64 here, by an opaque instruction:
              // converting all of x once, outside the loop over flagged
              // rows, would need 2*S more registers
              double xd[4];
#pragma unroll
              for (int c = 0; c < 4; ++c) asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(xd[c]) : "v"(xb[k + c]));
              p4[0] = __fma_rn((double)av[u].x, xd[0], p4[0]);
              p4[1] = __fma_rn((double)av[u].y, xd[1], p4[1]);
              p4[2] = __fma_rn((double)av[u].z, xd[2], p4[2]);
              p4[3] = __fma_rn((double)av[u].w, xd[3], p4[3]);
            }
          }
          part = (p4[0] + p4[1]) + (p4[2] + p4[3]);
        }
        part += __shfl_xor(part, 32);
        if (fl && hk == h) {
          const double bv = (double)lds_b[row];
          const double qf = (part + bv) * inv_wd;
          const double rad = coef64 * ((double)lds_an[row] * (double)xn + fabs(bv)) / (double)w;
          double flo = floor(qf);
          if (!(qf - flo > rad && flo + 1.0 - qf > rad)) {
            const float* ar = lds_a + row * STR;
            double sacc = 0.0;
            for (int t = 0; t < d; ++t) sacc = __dadd_rn(sacc, __dmul_rn((double)ar[t], (double)xr[t]));
            flo = floor(__dadd_rn(sacc, bv) / (double)w);
          }
          const bool fits = flo >= -2147483648.0 && flo <= 2147483647.0;
          if (!fits) set_status(st, GEEK_ERR_RANGE);
          lds_code[pl * H_CS + row] = fits ? (int)flo : 0;
        }
        fl &= fl - 1ull;
      }
    }
    __syncthreads();
    // every wave is done with this chunk's LDS rows: the next chunk's copy
    // runs during the packing
    if (tb + tpc < L) issue_chunk(c + 1);
    // ---- pack the m codes of every (table, point) into a 128-bit key (m = 10
    // at compile time; more compile-time cases push the kernel past its
    // register budget)
    const int64_t np = (n - i0) < BPTS ? (n - i0) : BPTS;
    const int pk = tid % BPTS;  // this thread's point; tables tid / BPTS, + 2, ...
    if (keys && pk < np) {
      const int64_t ii = i0 + pk;
      const int t0 = tid / BPTS, step = NT / BPTS;
      uint32_t orr;
#define GEEK_PACK(MM) pack_keys<MM>(lds_code, pk, t0, step, ntab, tb, m, B, code_off, n, ii, keys, key_fp)
      if (m == 10)
        orr = GEEK_PACK(10);
      else
        orr = GEEK_PACK(0);
#undef GEEK_PACK
      if (B < 32 && (orr >> B) != 0u) set_status(st, GEEK_ERR_RANGE);
    }
    if (codes_out) {
      for (int q = tid; q < BPTS * rows_used; q += NT) {
        const int pp = q / rows_used, row = q % rows_used;
        if (pp < np) codes_out[(i0 + pp) * P + p0 + row] = lds_code[pp * H_CS + row];
      }
    }
  }
  if (n_fixup) {
    for (int o = 32; o > 0; o >>= 1) nfix += __shfl_xor(nfix, o);
    if (lane == 0 && nfix) atomicAdd(n_fixup, nfix);
  }
}

__global__ void k_check_finite(const float* __restrict__ v, int64_t n, int32_t* st) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && !isfinite(v[i])) set_status(st, GEEK_ERR_NONFINITE);
}

// ---------------------------------------------------------------- MinHash
// One wavefront per object.  Lane f keeps the running minimum of pi_g for
// g = f, f + 64, ... (up to FPL functions per lane, F <= 64 * FPL).
// `get_token` supplies token q of object i; tokens are read once per
// wavefront (uniform address) and mixed once, then every lane applies its
// affine maps.
template <int FPL, class TokenFn>
__device__ void minhash_row(int64_t i, int ntok, const TokenFn& get_token,
                            const uint32_t* __restrict__ mh_keys, int F, uint32_t* __restrict__ sig) {
  const int lane = threadIdx.x & 63;
  uint32_t a[FPL], b[FPL], mn[FPL];
#pragma unroll
  for (int u = 0; u < FPL; ++u) {
    const int f = lane + 64 * u;
    a[u] = f < F ? (mh_keys[2 * f] | 1u) : 1u;
    b[u] = f < F ? mh_keys[2 * f + 1] : 0u;
    mn[u] = 0xFFFFFFFFu;
  }
  for (int q0 = 0; q0 < ntok; q0 += 64) {
    // each lane loads and premixes one token, then they are broadcast
    const uint32_t mine = (q0 + lane < ntok) ? fmix32(get_token(q0 + lane)) : 0u;
    const int lim = (ntok - q0) < 64 ? (ntok - q0) : 64;
    for (int q = 0; q < lim; ++q) {
      const uint32_t y = __shfl(mine, q);
#pragma unroll
      for (int u = 0; u < FPL; ++u) {
        const uint32_t v = perm_premixed(a[u], b[u], y);
        mn[u] = v < mn[u] ? v : mn[u];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < FPL; ++u) {
    const int f = lane + 64 * u;
    if (f < F) sig[i * F + f] = mn[u];
  }
}

template <int FPL>
__global__ __launch_bounds__(256) void k_minhash_sets(const int64_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ tokens,
                                                       int64_t n, const uint32_t* __restrict__ mh_keys,
                                                       int F, uint32_t* __restrict__ sig, int32_t* st) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t s = offsets[i], e = offsets[i + 1];
  if (e <= s) {
    set_status(st, GEEK_ERR_EMPTY_SET);
    return;
  }
  const uint32_t* tk = tokens + s;
  minhash_row<FPL>(i, (int)(e - s), [&](int q) { return tk[q]; }, mh_keys, F, sig);
}

// Heterogeneous rows: categorical tokens (a << 16) | v and numeric tokens
// 0x80000000 | (p << 16) | (code + 32768), then MinHash of the token set.
template <int FPL>
__global__ __launch_bounds__(256) void k_minhash_hetero(const int32_t* __restrict__ cat, int n_cat,
                                                         const int32_t* __restrict__ codes, int P,
                                                         int64_t n, const uint32_t* __restrict__ mh_keys,
                                                         int F, uint32_t* __restrict__ sig, int32_t* st) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int32_t* cr = cat + i * n_cat;
  const int32_t* co = codes + i * P;
  auto tok = [&](int q) -> uint32_t {
    if (q < n_cat) {
      const int32_t v = cr[q];
      if (v < 0 || v > 0xFFFF) set_status(st, GEEK_ERR_RANGE);
      return ((uint32_t)q << 16) | ((uint32_t)v & 0xFFFFu);
    }
    const int pp = q - n_cat;
    const int32_t c = co[pp];
    if (c < -32768 || c > 32767) set_status(st, GEEK_ERR_RANGE);
    return 0x80000000u | ((uint32_t)pp << 16) | ((uint32_t)(c + 32768) & 0xFFFFu);
  };
  minhash_row<FPL>(i, n_cat + P, tok, mh_keys, F, sig);
}

// ---------------------------------------------------------------- DOPH
// Densified one-permutation hashing (Algorithm 3's first step, after
// Shrivastava and Li, ICML 2014): one keyed permutation pi of the 32-bit
// token universe, D equal ranges of [0, 2^32) (value v lies in bin
// floor(v * D / 2^32)), the smallest permuted value of the set in every bin,
// and rotation densification: an empty bin takes the value of the first
// non-empty bin to its right, cyclically.  A value names its own bin, so the
// borrowed values of different distances never coincide.
//
// One wavefront per set: the lanes hash the set's tokens (one permutation
// each) into a private LDS row of D minima plus an occupancy bit per bin
// (LDS min / or atomics), then lane-strided over the bins each lane finds the
// source bin from the occupancy words and writes the row (consecutive lanes,
// consecutive words).

__global__ __launch_bounds__(256) void k_doph(const int64_t* __restrict__ offsets,
                                              const uint32_t* __restrict__ tokens, int64_t n,
                                              const uint32_t* __restrict__ key, int D,
                                              uint32_t* __restrict__ sig, int32_t* st) {
  extern __shared__ uint32_t doph_lds[];
  const int nw = (D + 31) >> 5;
  const int stride = D + nw;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* mins = doph_lds + wv * stride;
  uint32_t* occ = mins + D;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= n) return;  // the wave's LDS row is its own: no block barrier below
  const int64_t s = offsets[i], e = offsets[i + 1];
  if (e <= s) {
    set_status(st, GEEK_ERR_EMPTY_SET);
    return;
  }
  for (int j = lane; j < D; j += 64) mins[j] = 0xFFFFFFFFu;
  for (int j = lane; j < nw; j += 64) occ[j] = 0u;
  // lanes of one wave share the row: order the LDS accesses of the phases
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  const uint32_t a = key[0] | 1u, b = key[1];
  const uint64_t Du = (uint64_t)D;
  for (int64_t q = s + lane; q < e; q += 64) {
    const uint32_t v = perm_premixed(a, b, fmix32(tokens[q]));
    const uint32_t bin = (uint32_t)(((uint64_t)v * Du) >> 32);
    atomicMin(&mins[bin], v);
    atomicOr(&occ[bin >> 5], 1u << (bin & 31u));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  uint32_t* out = sig + i * (int64_t)D;
  for (int j = lane; j < D; j += 64) {
    int w = j >> 5;
    uint32_t m = occ[w] & (0xFFFFFFFFu << (j & 31));
    // the set is non-empty, so some word has a bit: at most nw + 1 steps
    while (m == 0u) {
      w = (w + 1 == nw) ? 0 : w + 1;
      m = occ[w];
    }
    out[j] = mins[(w << 5) + __builtin_ctz(m)];
  }
}

// ---------------------------------------------------------------- host side
static int pick_dp_h(int d) { return d <= 32 ? 32 : d <= 64 ? 64 : d <= 128 ? 128 : d <= 256 ? 256 : 0; }

// Floats of the projection-row chunks that k_e2lsh_prep writes.
static size_t e2lsh_chunk_floats(const geek_hash_job& J) {
  if (J.kind != GEEK_HASH_DENSE && J.kind != GEEK_HASH_HETERO) return 0;
  if (J.m < 1 || J.m > H_BC) return 0;
  const int nchunks = ceil_div(J.L, H_BC / J.m);
  switch (pick_dp_h(J.d)) {
    case 32: return (size_t)nchunks * E2Chunk<32, true>::G_FLOATS;
    case 64: return (size_t)nchunks * E2Chunk<64, true>::G_FLOATS;
    case 128: return (size_t)nchunks * E2Chunk<128, true>::G_FLOATS;
    default: return (size_t)nchunks * E2Chunk<256, false>::G_FLOATS;
  }
}

size_t hash_ws(const geek_hash_job& J) {
  Carver c(nullptr);
  c.take<float>(e2lsh_chunk_floats(J) + 64);
  if (J.kind == GEEK_HASH_HETERO) c.take<int32_t>((size_t)J.n * J.m * J.L);
  c.take<unsigned long long>(1);
  return c.used + 256;
}

static int32_t launch_e2lsh(const geek_hash_job& J, float* chunks, uint32_t* keys, uint32_t* key_fp,
                            int32_t* codes, unsigned long long* nfix, int32_t* st, hipStream_t s) {
  const int tpc = H_BC / J.m;  // whole tables per 64-row chunk
  const int nchunks = ceil_div(J.L, tpc);
  switch (pick_dp_h(J.d)) {
#define GEEK_H_CASE(DPV, B3V)                                                                              \
  case DPV: {                                                                                              \
    constexpr int nt = B3V ? 2 * H_THREADS : H_THREADS;                                                    \
    hipLaunchKernelGGL((k_e2lsh_prep<DPV, B3V>), dim3(nchunks), dim3(H_THREADS), 0, s, J.A, J.b, J.d, J.m, \
                       J.L, J.w, tpc, chunks);                                                             \
    const int64_t grid = ceil_div(J.n, (int64_t)nt / 2);                                                   \
    if (grid == 0) return GEEK_OK;                                                                         \
    prof_begin(GEEK_PROF_E2LSH, s);                                                                        \
    hipLaunchKernelGGL((k_e2lsh<DPV, B3V>), dim3(grid), dim3(nt), 0, s, J.X, J.ldx, J.d, J.n, chunks, J.m, \
                       J.L, J.w, tpc, keys, key_fp, codes, nfix, st);                                      \
    prof_end(GEEK_PROF_E2LSH, s);                                                                          \
    break;                                                                                                 \
  }
    // d <= 128: products from bf16 pieces; d = 256: float32 products (the
    // chunk image with bf16 pieces would not fit in LDS)
    GEEK_H_CASE(32, true)
    GEEK_H_CASE(64, true)
    GEEK_H_CASE(128, true)
    GEEK_H_CASE(256, false)
#undef GEEK_H_CASE
    default:
      return GEEK_ERR_UNSUPPORTED;
  }
  return GEEK_OK;
}

template <class Fn>
static int32_t dispatch_fpl(int F, Fn&& fn) {
  if (F <= 64) return fn(std::integral_constant<int, 1>{});
  if (F <= 128) return fn(std::integral_constant<int, 2>{});
  if (F <= 256) return fn(std::integral_constant<int, 4>{});
  if (F <= 512) return fn(std::integral_constant<int, 8>{});
  return GEEK_ERR_UNSUPPORTED;
}

int32_t hash_run(const geek_hash_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s) {
  Carver c(ws);
  float* chunks = c.take<float>(e2lsh_chunk_floats(J) + 64);
  int32_t* hcodes = (J.kind == GEEK_HASH_HETERO) ? c.take<int32_t>((size_t)J.n * J.m * J.L) : nullptr;
  unsigned long long* dummy = c.take<unsigned long long>(1);
  (void)dummy;
  if (ws_bytes < c.used + 256) return GEEK_ERR_WORKSPACE;
  int32_t rc = GEEK_OK;
  if (J.kind == GEEK_HASH_DENSE) {
    rc = launch_e2lsh(J, chunks, J.keys, J.key_fp, J.codes, J.n_fixup, st, s);
  } else if (J.kind == GEEK_HASH_DOPH) {
    if (J.n == 0) return GEEK_OK;
    const size_t lds = sizeof(uint32_t) * 4 * (size_t)(J.F + (J.F + 31) / 32);
    prof_begin(GEEK_PROF_MINHASH, s);
    hipLaunchKernelGGL(k_doph, dim3(ceil_div(J.n, 4)), dim3(256), lds, s, J.offsets, J.tokens, J.n, J.mh_keys,
                       J.F, J.sig, st);
    prof_end(GEEK_PROF_MINHASH, s);
  } else if (J.kind == GEEK_HASH_SETS) {
    if (J.n == 0) return GEEK_OK;
    prof_begin(GEEK_PROF_MINHASH, s);
    rc = dispatch_fpl(J.F, [&](auto fpl) {
      hipLaunchKernelGGL((k_minhash_sets<decltype(fpl)::value>), dim3(ceil_div(J.n, 4)), dim3(256),
                         0, s, J.offsets, J.tokens, J.n, J.mh_keys, J.F, J.sig, st);
      return GEEK_OK;
    });
    prof_end(GEEK_PROF_MINHASH, s);
  } else {
    // numeric codes without keys, then the token sets
    uint32_t* no_keys = nullptr;
    geek_hash_job D = J;
    D.kind = GEEK_HASH_DENSE;
    rc = launch_e2lsh(D, chunks, no_keys, nullptr, hcodes, J.n_fixup, st, s);
    if (rc != GEEK_OK) return rc;
    if (J.n == 0) return GEEK_OK;
    const int P = J.m * J.L;
    rc = dispatch_fpl(J.F, [&](auto fpl) {
      hipLaunchKernelGGL((k_minhash_hetero<decltype(fpl)::value>), dim3(ceil_div(J.n, 4)), dim3(256),
                         0, s, J.cat, J.n_cat, hcodes, P, J.n, J.mh_keys, J.F, J.sig, st);
      return GEEK_OK;
    });
  }
  if (rc != GEEK_OK) return rc;
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

// ---------------------------------------------------------------- no allocation
// geek_hash_noalloc keeps its scratch (the projections' norms, the codes of
// heterogeneous rows) in this file-scope device array instead of a caller
// workspace.  Each GPU holds its own copy; host code takes the copy's device
// address from hipGetSymbolAddress once per device and never passes the
// array's name itself to a kernel.
__device__ __align__(256) unsigned char scratch[GEEK_NOALLOC_SCRATCH_BYTES];

int32_t hash_check(const geek_hash_job& J);

namespace {
constexpr int NA_DEVS = 64;
std::mutex g_na_mu;
void* g_na_ptr[NA_DEVS];  // scratch's device address per device, null until looked up

int32_t scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= NA_DEVS) return GEEK_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> g(g_na_mu);
  if (!g_na_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
    g_na_ptr[dev] = p;
  }
  *out = g_na_ptr[dev];
  return GEEK_OK;
}
}  // namespace

}  // namespace geek

extern "C" int32_t geek_hash_noalloc(const geek_hash_job* jobs, int32_t njobs, int32_t* d_status, void* stream) {
  using namespace geek;
  if (!jobs || njobs < 1) return GEEK_ERR_ARG;
  for (int j = 0; j < njobs; ++j) {
    if (int32_t rc = hash_check(jobs[j])) return rc;
    if (ws_slice(hash_ws(jobs[j])) > (size_t)GEEK_NOALLOC_SCRATCH_BYTES) return GEEK_ERR_WORKSPACE;
  }
  void* ws = nullptr;
  if (int32_t rc = scratch_ptr(&ws)) return rc;
  // the jobs share the scratch, so they run one after another on `stream`;
  // every kernel writes the scratch words it reads, nothing needs clearing
  for (int j = 0; j < njobs; ++j) {
    int32_t rc = hash_run(jobs[j], ws, GEEK_NOALLOC_SCRATCH_BYTES, d_status, (hipStream_t)stream);
    if (rc) return rc;
  }
  return GEEK_OK;
}
