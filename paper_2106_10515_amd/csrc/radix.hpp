// Device-wide exclusive scan and stable LSD radix sort (see radix.hip).
#pragma once

#include "common.hpp"

namespace geek {

// Up to four uint32 key words (structure of arrays) and an optional payload.
struct RsView {
  uint32_t* k[4];
  uint32_t* v;
};

// Exclusive scan of n words (in may equal out); *total (device, optional)
// receives the sum.  tmp: exscan_tmp_words(n) words.
size_t exscan_tmp_words(int64_t n);
void exscan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, uint32_t* total,
                hipStream_t s);
// The same with the element count read on the device: min(*n_dev, n) elements
// (n, the host bound, sizes the launch; n_dev null = n).  No host read-back.
void exscan_u32_dn(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* n_dev, uint32_t* tmp,
                   uint32_t* total, hipStream_t s);

// Stable sort of n items by 8-bit digits (word words[p], bits shifts[p] ..
// shifts[p]+7), least significant pass first.  tmp: radix_tmp_words(n).
// Returns 1 when the result is in `alt`, 0 when in `buf`.
size_t radix_tmp_words(int64_t n);
int radix_sort(RsView buf, RsView alt, int W, int64_t n, const int* words, const int* shifts, int npass,
               uint32_t* tmp, hipStream_t s);
// The same over min(*n_dev, n) items (n sizes the launches and tmp).
int radix_sort_dn(RsView buf, RsView alt, int W, int64_t n, const uint32_t* n_dev, const int* words,
                  const int* shifts, int npass, uint32_t* tmp, hipStream_t s);

}  // namespace geek
