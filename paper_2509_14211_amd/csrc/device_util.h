// Device helpers shared by the gfx950 kernels: cross-workgroup hand-off,
// wave-uniform values, buffer-resource memory access and the counter-based
// random stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbgrb {

// ------------------------------------------------------- hand-off between
// workgroups: values are published with device-scope atomic stores, the
// wave waits for them to complete, then bumps a counter; readers use
// device-scope atomic loads.  No L2 write-back / invalidate is needed.

// s_waitcnt vmcnt(0): every vector memory operation of this wave is done.
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <typename V>
__device__ __forceinline__ void publish(V* p, V v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename V>
__device__ __forceinline__ V consume(const V* p) {
  return __hip_atomic_load(const_cast<V*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned ticket_add(unsigned* p) {
  return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int counter_add(int* p) {
  return __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------- wave-uniform values
// Values that are the same in every lane of the wavefront, moved to scalar
// registers so that branches on them are uniform.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int4 wave_uniform(int4 v) {
  return make_int4(wave_uniform(v.x), wave_uniform(v.y), wave_uniform(v.z), wave_uniform(v.w));
}
__device__ __forceinline__ float wave_uniform(float v) {
  return __builtin_bit_cast(float, wave_uniform(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double wave_uniform(double v) {
  const int2 h = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(wave_uniform(h.x), wave_uniform(h.y)));
}

// Lane `k`'s value of v (k a constant or wave-uniform), in scalar registers.
__device__ __forceinline__ int lane_value(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ float lane_value(float v, int k) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), k));
}

// Descriptor t (t wave-uniform) of a read-only table through the scalar
// cache: a scalar load does not wait behind the wavefront's outstanding
// vector loads.
__device__ __forceinline__ int4 tile_desc(const int4* tiles, int t) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const __attribute__((address_space(4))) int4* const_int4_ptr;
  return ((const_int4_ptr)tiles)[wave_uniform(t)];
#else
  return tiles[t];
#endif
}

// ------------------------------------------------------- buffer resources
// A load at a byte offset at or past the resource's size returns zero
// without touching memory, which keeps per-lane bounds out of the control
// flow.  The address is base + voff (per lane) + soff (scalar).
constexpr unsigned BUF_SKIP = 0xFFFFFFF0u;  // offset of a lane that must not load
constexpr int CP_NT = 2;                    // nontemporal cache policy

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename V, int AUX = 0>
__device__ __forceinline__ V buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff = 0) {
  if constexpr (sizeof(V) == 2)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, AUX));
  else if constexpr (sizeof(V) == 4)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX));
  else if constexpr (sizeof(V) == 8)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX));
  else
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, AUX));
}

template <typename V, int AUX = 0>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, V v, unsigned voff, unsigned soff = 0) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  if constexpr (sizeof(V) == 2)
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)voff, (int)soff, AUX);
  else if constexpr (sizeof(V) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, AUX);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, AUX);
}

// ------------------------------------------------------- random stream
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) as a counter-based
// generator: draw k of the stream seeded with `seed` is the output after
// k+1 increments of the state.
__device__ __forceinline__ uint64_t splitmix_draw(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// u in [0, 1) from the top 53 bits of a draw.
__device__ __forceinline__ double draw_unit(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

}  // namespace nbgrb
