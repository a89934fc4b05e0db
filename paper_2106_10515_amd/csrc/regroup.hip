// Clusters of an assignment as the seeds of a further assignment pass
// (paper Section 4.3, Clustering Performance): cluster j = {i : assign[i] ==
// j} with ascending members, empty clusters dropped, the others in the order
// of j.  The objects are sorted by label with the stable LSD radix sort
// (ids ride along as the payload, so members stay ascending within a label);
// a label's first position in the sorted order starts a cluster, and an
// exclusive scan of those starts numbers the clusters.
#include "common.hpp"
#include "radix.hpp"

namespace geek {

constexpr int RG_THREADS = 256;

// label and id of every object; labels outside [0, k) are reported and
// replaced by 0 so that the sort stays within its digits
__global__ void k_rg_init(const int32_t* __restrict__ assign, int64_t n, int k, uint32_t* __restrict__ lab,
                          uint32_t* __restrict__ idx, int32_t* st) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t a = assign[i];
  const bool ok = a >= 0 && a < k;
  if (!ok) set_status(st, GEEK_ERR_RANGE);
  lab[i] = ok ? (uint32_t)a : 0u;
  idx[i] = (uint32_t)i;
}

// 1 where a sorted position starts a new label
__global__ void k_rg_starts(const uint32_t* __restrict__ lab, int64_t n, uint32_t* __restrict__ flag) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  flag[p] = (p == 0 || lab[p] != lab[p - 1]) ? 1u : 0u;
}

// members in sorted order; at every start, the cluster's offset and label;
// the last position closes the CSR with n
__global__ void k_rg_emit(const uint32_t* __restrict__ lab, const uint32_t* __restrict__ idx,
                          const uint32_t* __restrict__ rank, int64_t n, uint32_t* __restrict__ offsets,
                          uint32_t* __restrict__ members, int32_t* __restrict__ label_of) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  members[p] = idx[p];
  const bool start = p == 0 || lab[p] != lab[p - 1];
  if (start) {
    offsets[rank[p]] = (uint32_t)p;
    if (label_of) label_of[rank[p]] = (int32_t)lab[p];
  }
  if (p == n - 1) offsets[rank[p] + (start ? 1u : 0u)] = (uint32_t)n;
}

// no objects: no clusters
__global__ void k_rg_empty(uint32_t* offsets, uint32_t* k_out) {
  if (threadIdx.x == 0) {
    offsets[0] = 0u;
    *k_out = 0u;
  }
}

struct RgWs {
  uint32_t *lab, *idx, *lab2, *idx2, *rank, *stmp, *rtmp;
};

static size_t carve_rg(int64_t n, void* base, RgWs& W) {
  Carver c(base);
  const int64_t m = n > 0 ? n : 1;
  W.lab = c.take<uint32_t>(m);
  W.idx = c.take<uint32_t>(m);
  W.lab2 = c.take<uint32_t>(m);
  W.idx2 = c.take<uint32_t>(m);
  W.rank = c.take<uint32_t>(m);
  W.stmp = c.take<uint32_t>(exscan_tmp_words(m));
  W.rtmp = c.take<uint32_t>(radix_tmp_words(m));
  return c.used + 256;
}

size_t regroup_ws(const geek_regroup_job& J) {
  RgWs W;
  return carve_rg(J.n, nullptr, W);
}

int32_t regroup_run(const geek_regroup_job& J, void* ws, int32_t* st, hipStream_t s) {
  if (J.n == 0) {
    hipLaunchKernelGGL(k_rg_empty, dim3(1), dim3(64), 0, s, J.seed_offsets, J.k_out);
    GEEK_LAUNCH_CHECK();
    return GEEK_OK;
  }
  RgWs W;
  carve_rg(J.n, ws, W);
  const int grid = ceil_div(J.n, RG_THREADS);
  hipLaunchKernelGGL(k_rg_init, dim3(grid), dim3(RG_THREADS), 0, s, J.assign, J.n, J.k, W.lab, W.idx, st);
  // 8-bit digits of the label, least significant first, as many as k - 1 needs
  int words[4], shifts[4], np = 0;
  for (int sh = 0; sh < 32 && ((uint32_t)(J.k - 1) >> sh) != 0u; sh += 8) {
    words[np] = 0;
    shifts[np++] = sh;
  }
  RsView A{{W.lab, nullptr, nullptr, nullptr}, W.idx}, B{{W.lab2, nullptr, nullptr, nullptr}, W.idx2};
  const int alt = radix_sort(A, B, 1, J.n, words, shifts, np, W.rtmp, s);
  const uint32_t* slab = alt ? W.lab2 : W.lab;
  const uint32_t* sidx = alt ? W.idx2 : W.idx;
  hipLaunchKernelGGL(k_rg_starts, dim3(grid), dim3(RG_THREADS), 0, s, slab, J.n, W.rank);
  exscan_u32(W.rank, W.rank, J.n, W.stmp, J.k_out, s);
  hipLaunchKernelGGL(k_rg_emit, dim3(grid), dim3(RG_THREADS), 0, s, slab, sidx, W.rank, J.n, J.seed_offsets,
                     J.seed_members, J.label_of);
  GEEK_LAUNCH_CHECK();
  return GEEK_OK;
}

}  // namespace geek
