// Shared device/host helpers of libgeek (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "geek.h"

#define GEEK_HD __host__ __device__ __forceinline__
#define GEEK_D __device__ __forceinline__

namespace geek {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---- device status word (first error wins) --------------------------------
GEEK_D void set_status(int32_t* st, int32_t code) {
  if (st) atomicCAS(st, 0, code);
}
GEEK_D bool status_bad(const int32_t* st) {
  return st && __hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// ---- MinHash permutation of 32-bit words -----------------------------------
// fmix32 is MurmurHash3's 32-bit finalizer (Appleby, public domain): two
// multiply rounds by odd constants separated by xor-shifts; each step is
// invertible, so the map is a bijection.  pi(x) = a*fmix32(x) + b mod 2^32
// with a odd is then a keyed bijection (Eq. (2) needs a random permutation).
GEEK_HD uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}
GEEK_HD uint32_t perm_premixed(uint32_t a_odd, uint32_t b, uint32_t mixed) {
  return a_odd * mixed + b;
}

// 32-bit mixing hash of a key of up to four words (bin selection only; any
// function of the exact key works because equal keys land in one bin).
GEEK_HD uint32_t key_hash(const uint32_t* k, int words) {
  uint32_t h = 0x9E3779B9u;
  for (int i = 0; i < words; ++i) h = fmix32(h ^ k[i]) + 0x7F4A7C15u * (uint32_t)(i + 1);
  return fmix32(h);
}

// ---- float atomics on non-negative values via their bit patterns ----------
GEEK_D void atomic_max_nonneg(float* p, float v) {
  atomicMax(reinterpret_cast<unsigned int*>(p), __float_as_uint(v));
}
GEEK_D void atomic_max_nonneg(double* p, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(p),
            (unsigned long long)__double_as_longlong(v));
}

// ---- host-side workspace carving -------------------------------------------
struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    used = (used + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Opt-in event timing of the main kernels (see geek_profile in geek.h).
void prof_begin(int id, hipStream_t s);
void prof_end(int id, hipStream_t s);

// Independent per-job work of a multi-job call fanned out over up to
// FAN_LANES streams and joined back into the caller's stream: an event
// recorded on the caller's stream is waited on by every lane, and the caller's
// stream waits on an event recorded on every lane at the end (HIP graph
// capture records this as parallel branches).  The lane streams (default
// priority, one set per device) and events are created on the first call that
// fans out and kept until the process ends; a mutex keeps the enqueue of one
// fanned-out call from interleaving with another's.  With one lane, or if the
// streams cannot be created, everything stays on the caller's stream.
constexpr int FAN_LANES = 4;
class Fan {
 public:
  Fan(hipStream_t main, int jobs);
  ~Fan();
  int lanes() const { return n_; }
  hipStream_t lane(int j) const { return n_ > 1 ? side_[j % n_] : main_; }

 private:
  hipStream_t main_;
  int n_ = 1, dev_ = 0;
  hipStream_t side_[FAN_LANES] = {};
};

// Workspace bytes rounded up to a 256-byte slice.
size_t ws_slice(size_t bytes);

// Records the HIP error string for geek_last_hip_error and maps to a status.
int32_t hip_fail(hipError_t e);
#define GEEK_LAUNCH_CHECK()                                   \
  do {                                                        \
    hipError_t _e = hipGetLastError();                        \
    if (_e != hipSuccess) return ::geek::hip_fail(_e);        \
  } while (0)

}  // namespace geek
