// SILK seeding (paper Section 3.2, Algorithm 4) on gfx950.
#include "common.hpp"

namespace geek {

size_t silk_ws(const geek_silk_job& J) {
  (void)J;
  return 256;
}

int32_t silk_run(const geek_silk_job& J, void* ws, size_t ws_bytes, int32_t* st, hipStream_t s) {
  (void)J; (void)ws; (void)ws_bytes; (void)st; (void)s;
  return GEEK_ERR_UNSUPPORTED;
}

}  // namespace geek
