// Batched first pass of the assignment (many Euclidean jobs in one
// persistent launch per padded depth): the tile shapes it is compiled for,
// the table that picks one per (precision, padded depth), and the launch.
// The table is filled by measurement (the package's autotuner) through
// geek_set_scan_tiles; every shape yields the same records, so the choice
// affects speed only.
#include <algorithm>
#include <atomic>

#include "scan.hpp"

namespace geek {

namespace {

int prec_index(int precision) { return precision >= 0 && precision <= 2 ? precision : -1; }
int dp_index(int dp) { return dp == 32 ? 0 : dp == 64 ? 1 : dp == 128 ? 2 : dp == 256 ? 3 : -1; }

// float32 fragments of two column blocks fit the registers only up to a
// padded depth of 64, and then without the second LDS stage
constexpr bool shape_ok(int precision, int dp, int ncb, int nbuf) {
  return ncb >= 1 && ncb <= 2 && nbuf >= 1 && nbuf <= 2 &&
         !(precision == GEEK_PREC_FP32 && ncb == 2 && (dp > 64 || nbuf == 2));
}

ScanTiles default_tiles(int precision) {
  return precision == GEEK_PREC_FP32 ? ScanTiles{1, 1, 8} : ScanTiles{2, 2, 8};
}

// packed ncb | nbuf << 4 | blocks_per_cu << 8; 0 = the default shape
std::atomic<uint32_t> g_tiles[3][4];

int cu_count() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cached[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
  cached[dev].store(v, std::memory_order_relaxed);
  return v;
}

template <class M, int DP, int NCB, int NBUF>
void launch_one(dim3 grid, const ScanJob* table, int nj, int64_t total, int32_t* st, hipStream_t s) {
  constexpr bool T2 = std::is_same<M, ModeBF16>::value;
  hipLaunchKernelGGL((k_scan_batch<M, DP, NCB, NBUF, T2>), grid, dim3(SCAN_THREADS), 0, s, table, nj, total, st);
}

template <class M, int PREC, int DP>
void launch_dp(const ScanTiles& t, dim3 grid, const ScanJob* table, int nj, int64_t total, int32_t* st,
               hipStream_t s) {
  if (t.ncb == 1 && t.nbuf == 1) launch_one<M, DP, 1, 1>(grid, table, nj, total, st, s);
  else if (t.ncb == 1) launch_one<M, DP, 1, 2>(grid, table, nj, total, st, s);
  else if constexpr (shape_ok(PREC, DP, 2, 2)) {
    if (t.nbuf == 2) launch_one<M, DP, 2, 2>(grid, table, nj, total, st, s);
    else launch_one<M, DP, 2, 1>(grid, table, nj, total, st, s);
  } else if constexpr (shape_ok(PREC, DP, 2, 1)) {
    launch_one<M, DP, 2, 1>(grid, table, nj, total, st, s);
  }
}

template <class M, int PREC>
void launch_prec(int dp, const ScanTiles& t, dim3 grid, const ScanJob* table, int nj, int64_t total, int32_t* st,
                 hipStream_t s) {
  switch (dp) {
    case 32: launch_dp<M, PREC, 32>(t, grid, table, nj, total, st, s); break;
    case 64: launch_dp<M, PREC, 64>(t, grid, table, nj, total, st, s); break;
    case 128: launch_dp<M, PREC, 128>(t, grid, table, nj, total, st, s); break;
    case 256: launch_dp<M, PREC, 256>(t, grid, table, nj, total, st, s); break;
  }
}

}  // namespace

ScanTiles scan_tiles_get(int precision, int dp) {
  const int a = prec_index(precision), b = dp_index(dp);
  if (a < 0 || b < 0) return default_tiles(GEEK_PREC_FP32);
  const uint32_t v = g_tiles[a][b].load(std::memory_order_relaxed);
  if (!v) return default_tiles(precision);
  return ScanTiles{(int)(v & 15u), (int)((v >> 4) & 15u), (int)(v >> 8)};
}

int32_t scan_tiles_set(int precision, int dp, ScanTiles t) {
  const int a = prec_index(precision), b = dp_index(dp);
  if (a < 0 || b < 0) return GEEK_ERR_ARG;
  if (t.ncb == 0 && t.nbuf == 0 && t.blocks_per_cu == 0) {  // back to the default
    g_tiles[a][b].store(0u, std::memory_order_relaxed);
    return GEEK_OK;
  }
  if (t.blocks_per_cu < 1 || t.blocks_per_cu > 64) return GEEK_ERR_ARG;
  if (!shape_ok(precision, dp, t.ncb, t.nbuf)) return GEEK_ERR_UNSUPPORTED;
  g_tiles[a][b].store((uint32_t)t.ncb | ((uint32_t)t.nbuf << 4) | ((uint32_t)t.blocks_per_cu << 8),
                      std::memory_order_relaxed);
  return GEEK_OK;
}

void launch_scan_batch(int precision, int dp, const ScanJob* table, int nj, int64_t total_tiles, int32_t* st,
                       hipStream_t s) {
  const ScanTiles t = scan_tiles_get(precision, dp);
  const int64_t want = (int64_t)t.blocks_per_cu * cu_count();
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(total_tiles, want)));
  if (precision == GEEK_PREC_BF16)
    launch_prec<ModeBF16, GEEK_PREC_BF16>(dp, t, grid, table, nj, total_tiles, st, s);
  else if (precision == GEEK_PREC_FP8)
    launch_prec<ModeFP8, GEEK_PREC_FP8>(dp, t, grid, table, nj, total_tiles, st, s);
  else
    launch_prec<ModeF32, GEEK_PREC_FP32>(dp, t, grid, table, nj, total_tiles, st, s);
}

}  // namespace geek
