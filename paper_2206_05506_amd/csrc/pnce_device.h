// pnce_device.h -- device helpers shared by the kernel files: vector types,
// the frame-bounded buffer resource, windows of the sequence bit stream and
// the placement of column runs in Eq. 8 segments.
#pragma once

#include "pnce_internal.h"

namespace pnce {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f4a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef float f2a8 __attribute__((ext_vector_type(2), aligned(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Complex64 rows come through a raw buffer resource bounded by the frame:
// reads at or past its end (antennas at or beyond R, the tail of the last
// row) return zeros, so every load is unconditional and the compiler can
// count them exactly (a load in a divergent branch forces it to wait for all
// outstanding loads). The whole byte offset goes in the per-lane offset,
// which the hardware checks against the frame size (the scalar offset is not
// checked), so no load ever touches memory past the frame.
constexpr int kRsrcFlags = 0x00020000;  // raw buffer, 32-bit dwords

__device__ __forceinline__ __amdgpu_buffer_rsrc_t frame_rsrc(const void *base, long long bytes) {
  // The descriptor lives in scalar registers: make its parts provably uniform.
  const uint64_t b = (uint64_t)base;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  const int n = __builtin_amdgcn_readfirstlane((int)bytes);
  return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), (short)0, n,
                                           kRsrcFlags);
}

// 8 bits of the periodic stream starting at bit p (p + 63 < 32 * nbw).
__device__ __forceinline__ uint32_t window8(const uint32_t *sbits, int p) {
  const uint32_t w0 = sbits[p >> 5];
  const uint32_t w1 = sbits[(p >> 5) + 1];
  return __builtin_amdgcn_alignbit(w1, w0, (uint32_t)(p & 31)) & 0xFFu;
}

// 32 bits of the periodic stream starting at bit p.
__device__ __forceinline__ uint32_t window32(const uint32_t *sbits, int p) {
  const uint32_t w0 = sbits[p >> 5];
  const uint32_t w1 = sbits[(p >> 5) + 1];
  return __builtin_amdgcn_alignbit(w1, w0, (uint32_t)(p & 31));
}

__device__ __forceinline__ int pos_mod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// Where a run of columns starting at dealt-out column v0 sits: its first lag,
// its first stored column, and how many of its columns are stored (<= 0:
// none). The run must not cross a segment (see seg_pad).
struct SegPos {
  int lag0, ocol0, n_out;
};
__device__ __forceinline__ SegPos seg_pos(int v0, int pad, int seg_len, int seg_lag, int c_len) {
  if (!seg_lag) return {v0, v0, c_len - v0};
  const int j = v0 / pad;
  const int l0 = v0 - j * pad;
  return {j * seg_lag + l0, j * seg_len + l0, min(seg_len, c_len - j * seg_len) - l0};
}

}  // namespace pnce
