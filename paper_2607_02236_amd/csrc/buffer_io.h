// Raw buffer loads and stores (MUBUF) with the base and range in a scalar
// buffer descriptor and a 32-bit per-lane byte offset: accesses at or beyond the
// range read 0 / are dropped by the hardware.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tacaw {

// Raw buffer load of one element at base + off (off < range, else 0): the base
// and the range live in scalar registers, the offset in one VGPR.
template <typename T>
__device__ __forceinline__ T buffer_load(const char* base, uint32_t range, uint32_t off) {
  __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)range, 0x00020000);
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
  }
}

// The same with a scalar offset: element at base + soffset + off, range counted
// from base (one descriptor serves several row groups).
template <typename T>
__device__ __forceinline__ T buffer_load_so(const char* base, uint32_t range, uint32_t off,
                                            uint32_t soff) {
  __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)range, 0x00020000);
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, (int)soff, 0));
  }
}

// Store of one element at base + off (off < range, else dropped).
template <typename T>
__device__ __forceinline__ void buffer_store(const T& v, char* base, uint32_t range, uint32_t off) {
  __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)range, 0x00020000);
  if constexpr (sizeof(T) == 8) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
  } else {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)off, 0, 0);
  }
}

}  // namespace tacaw
