// Assignment of MinHash signatures to the modes of the seeds (paper Section
// 3.3, central vector = mode; Dist = 1 - Sim, Section 2.1) on gfx950.
#include "common.hpp"

namespace geek {

size_t assign_sig_ws(const geek_assign_job& J) {
  (void)J;
  return 256;
}

int32_t assign_sig(const geek_assign_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s) {
  (void)J; (void)ws; (void)ws_bytes; (void)st; (void)s;
  return GEEK_ERR_UNSUPPORTED;
}

}  // namespace geek
