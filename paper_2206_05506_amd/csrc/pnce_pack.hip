// pnce_pack.hip -- the quantiser of libpnce.so: complex64 frames to planar
// bf16 / f16 / e4m3 codes with a per-frame power-of-two scale (the conversion
// to half precision ahead of the correlation, Section III-B).
//
// Code layout per frame and antenna: the real plane then the imaginary plane,
// N + 1 codes each (one zero pad sample, so a row is a power of two long).
// The scale of frame b is the smallest 2^e with maxabs_b <= target * 2^e
// (target 1 for bf16 / f16, 448 for e4m3; at least 2^-126; 1 for frames of
// zeros or with a non-finite maxabs), and every code is the value times
// 1/scale_b rounded to nearest even. Three launch plans give the same codes:
//  - one workgroup per frame (batches of 256+ frames of at most 1 MiB): the
//    frame is read, reduced in LDS, and read again for the conversion, the
//    second read served by the Infinity Cache;
//  - slices of a frame at consecutive workgroups (every other batch, when the
//    caller gives a workspace and a frame's slices fit half of what the chip
//    holds at once): one HBM read, the slice held in registers until the
//    frame's maximum is known (pack_slices_kernel);
//  - a per-frame max pass then a conversion pass (no workspace, or frames too
//    large for the slices).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "pnce_internal.h"

namespace pnce {

typedef float f2a8 __attribute__((ext_vector_type(2), aligned(8)));

__device__ __forceinline__ uint32_t bf16_bits(float x) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x);
}

// Smallest power of two 2^e with m <= target * 2^e (m finite, > 0).
__device__ float pow2_scale(float m, float target) {
  int e;
  (void)frexpf(m / target, &e);
  while ((double)m > (double)target * ldexp(1.0, e)) ++e;
  while ((double)m <= (double)target * ldexp(1.0, e - 1)) --e;
  // at least the smallest normal float, so that the reciprocal is finite
  // for frames of subnormal samples
  return ldexpf(1.0f, e < -126 ? -126 : e);
}

// The frame maximum travels as the bit pattern of |v|: for non-negative
// floats the unsigned order is the numeric order, and every NaN pattern sits
// above +inf, so one unsigned max also flags non-finite frames.
__device__ __forceinline__ float scale_from_maxbits(uint32_t mb, float target) {
  if (mb == 0u || mb >= 0x7F800000u) return 1.0f;  // zeros, inf or NaN
  return pow2_scale(__builtin_bit_cast(float, mb), target);
}

__global__ __launch_bounds__(256) void zero_u32_kernel(uint32_t *p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Grid (slices, frames): each workgroup reduces one slice of a frame's R*N
// complex samples and folds it into the frame's word with one atomic max.
constexpr int kMaxUnroll = 8;
__global__ __launch_bounds__(256) void frame_max_kernel(const f2a8 *y, uint32_t *maxbits,
                                                        long per_frame) {
  const f2a8 *f = y + (size_t)blockIdx.y * per_frame;
  const long step = (long)gridDim.x * 256;
  uint32_t m = 0u;
  for (long i0 = (long)blockIdx.x * 256 + threadIdx.x; i0 < per_frame; i0 += step * kMaxUnroll) {
    f2a8 v[kMaxUnroll];
#pragma unroll
    for (int u = 0; u < kMaxUnroll; ++u) {
      const long i = i0 + u * step;
      v[u] = i < per_frame ? f[i] : f2a8{0.0f, 0.0f};
    }
#pragma unroll
    for (int u = 0; u < kMaxUnroll; ++u) {
      // by-value floats: a bit cast of a vector element lvalue is not safe here
      const float re = v[u].x, im = v[u].y;
      m = max(m, __builtin_bit_cast(uint32_t, re) & 0x7FFFFFFFu);
      m = max(m, __builtin_bit_cast(uint32_t, im) & 0x7FFFFFFFu);
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
  __shared__ uint32_t sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = max(max(sm[0], sm[1]), max(sm[2], sm[3]));
    if (m) atomicMax(maxbits + blockIdx.y, m);
  }
}

// Rows with a stride (raw blocks whose cyclic prefix is skipped): grid
// (row slices, frames); a workgroup reduces whole rows r = x, x + slices, ...
__global__ __launch_bounds__(256) void frame_max_rows_kernel(const f2a8 *y, uint32_t *maxbits,
                                                             int R, int N, int ld) {
  uint32_t m = 0u;
  for (int r = blockIdx.x; r < R; r += gridDim.x) {
    const f2a8 *row = y + ((size_t)blockIdx.y * R + r) * ld;
    for (int n = threadIdx.x; n < N; n += 256) {
      const f2a8 v = row[n];
      const float re = v.x, im = v.y;
      m = max(m, __builtin_bit_cast(uint32_t, re) & 0x7FFFFFFFu);
      m = max(m, __builtin_bit_cast(uint32_t, im) & 0x7FFFFFFFu);
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
  __shared__ uint32_t sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = max(max(sm[0], sm[1]), max(sm[2], sm[3]));
    if (m) atomicMax(maxbits + blockIdx.y, m);
  }
}

// Max bits -> power-of-two scale, in place, once every pack block has read them.
__global__ __launch_bounds__(256) void finalize_scale_kernel(float *scales, int batch,
                                                             float target, uint32_t *flag) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b < batch)
    scales[b] = scale_from_maxbits(__builtin_bit_cast(uint32_t, scales[b]), target);
  if (flag && b == 0) *flag = 0u;  // nothing waited (see pack_slices_kernel)
}

// Two values to OCP e4m3fn codes (a in bits 0-7, b in bits 8-15), round to
// nearest even, saturating at +-448, NaN to 0x7F with its sign. The
// hardware conversion (v_cvt_pk_fp8_f32) rounds every finite value of
// magnitude up to 448 exactly so (subnormals included; checked against the
// e4m3fn grid on the whole bf16 range and at every rounding midpoint) but
// does not saturate, so values beyond +-448 (and infinities) are clamped
// first and NaN lanes are patched after.
__device__ __forceinline__ uint32_t e4m3_pair(float a, float b) {
  const float ca = __builtin_fminf(__builtin_fmaxf(a, -448.0f), 448.0f);
  const float cb = __builtin_fminf(__builtin_fmaxf(b, -448.0f), 448.0f);
  uint32_t r = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(ca, cb, 0, false) & 0xFFFFu;
  if (a != a) r = (r & 0xFF00u) | 0x7Fu | ((__builtin_bit_cast(uint32_t, a) >> 24) & 0x80u);
  if (b != b)
    r = (r & 0x00FFu) | ((0x7Fu | ((__builtin_bit_cast(uint32_t, b) >> 24) & 0x80u)) << 8);
  return r;
}

// Four consecutive samples n0 .. n0+3 of one padded output row (those at
// or past N are zero) to codes n0 .. n0+3 of the row's two planes (real at
// q_row, imaginary at q_row + Np), each value times inv, rounded to nearest
// even (e4m3: saturating). The padded row length N + 1 is a power of two, so
// each quad is one aligned 8-byte (16-bit codes) or 4-byte (e4m3) store per
// plane.
template <int FMT>
__device__ __forceinline__ void store_quad(const f2a8 (&v)[4], void *yq, size_t o, int valid,
                                           int Np, float inv) {
  if constexpr (FMT == 3) {
    // samples at or past `valid` are zero and encode as 0
    (void)valid;
    const uint32_t cr = e4m3_pair(v[0].x * inv, v[1].x * inv) |
                        (e4m3_pair(v[2].x * inv, v[3].x * inv) << 16);
    const uint32_t ci = e4m3_pair(v[0].y * inv, v[1].y * inv) |
                        (e4m3_pair(v[2].y * inv, v[3].y * inv) << 16);
    uint8_t *q = (uint8_t *)yq;
    *(uint32_t *)(q + o) = cr;
    *(uint32_t *)(q + o + Np) = ci;
  } else {
    uint64_t cr = 0u, ci = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < valid) {
        uint32_t r, m;
        if constexpr (FMT == 1) {
          r = bf16_bits(v[u].x * inv);
          m = bf16_bits(v[u].y * inv);
        } else {
          r = __builtin_bit_cast(uint16_t, (_Float16)(v[u].x * inv));
          m = __builtin_bit_cast(uint16_t, (_Float16)(v[u].y * inv));
        }
        cr |= (uint64_t)r << (16 * u);
        ci |= (uint64_t)m << (16 * u);
      }
    }
    uint16_t *q = (uint16_t *)yq;
    *(uint64_t *)(q + o) = cr;
    *(uint64_t *)(q + o + Np) = ci;
  }
}

// Samples n0 .. n0+3 of a row (those at or past N read as zero).
__device__ __forceinline__ void load_quad(const f2a8 *y_row, int n0, int N, f2a8 (&v)[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = n0 + u < N ? y_row[n0 + u] : f2a8{0.0f, 0.0f};
}

template <int FMT>
__device__ __forceinline__ void pack_quad(const f2a8 *y_row, void *yq, size_t q_row, int n0,
                                          int N, int Np, float inv) {
  f2a8 v[4];
  load_quad(y_row, n0, N, v);
  store_quad<FMT>(v, yq, q_row + n0, N - n0, Np, inv);
}

template <int FMT>
__global__ __launch_bounds__(256) void pack_kernel(const f2a8 *y, void *yq, const uint32_t *maxbits,
                                                   int R, int N, int ld, float target,
                                                   long total) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;  // (row, quad)
  if (i >= total) return;
  const int Np = N + 1, nq = Np >> 2;
  const long row = i / nq;  // frame * R + antenna
  const int n0 = (int)(i - row * nq) * 4;
  const int b = (int)(row / R);
  const float inv = 1.0f / scale_from_maxbits(maxbits[b], target);
  pack_quad<FMT>(y + row * ld, yq, (size_t)row * 2 * Np, n0, N, Np, inv);
}

// The whole quantiser in one launch when the batch has at least one frame
// per CU: workgroup b reduces frame b's max-abs word in LDS, then converts
// the frame (its second read mostly served by the caches) and writes the
// frame's scale. No atomics and no counters to clear; the codes equal those
// of the four-launch path (same maximum, same conversions).
constexpr int kPackFrameThreads = 1024;
template <int FMT>
__global__ __launch_bounds__(kPackFrameThreads) void pack_frame_kernel(
    const f2a8 *y, void *yq, float *scales, int R, int N, int ld, float target, uint32_t *flag) {
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const f2a8 *f = y + (size_t)b * R * ld;
  uint32_t m = 0u;
  auto fold = [&](f2a8 v) {
    const float re = v.x, im = v.y;
    m = max(m, __builtin_bit_cast(uint32_t, re) & 0x7FFFFFFFu);
    m = max(m, __builtin_bit_cast(uint32_t, im) & 0x7FFFFFFFu);
  };
  constexpr int U = 4;
  if (ld == N) {  // one contiguous run of R*N samples
    const long per = (long)R * N;
    for (long i0 = tid; i0 < per; i0 += (long)kPackFrameThreads * U) {
      f2a8 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long i = i0 + (long)u * kPackFrameThreads;
        v[u] = i < per ? f[i] : f2a8{0.0f, 0.0f};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) fold(v[u]);
    }
  } else {  // rows of N samples at a stride of ld
    for (int r = 0; r < R; ++r)
      for (int n = tid; n < N; n += kPackFrameThreads) fold(f[(size_t)r * ld + n]);
  }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
  __shared__ uint32_t wmax[kPackFrameThreads / 64];
  if ((tid & 63) == 0) wmax[tid >> 6] = m;
  __syncthreads();
  m = 0u;
#pragma unroll
  for (int w = 0; w < kPackFrameThreads / 64; ++w) m = max(m, wmax[w]);
  const float scale = scale_from_maxbits(m, target);
  const float inv = 1.0f / scale;
  const int Np = N + 1, nq = Np >> 2;
  const long total = (long)R * nq;
  for (long i = tid; i < total; i += kPackFrameThreads) {
    const int r = (int)(i / nq);
    const int n0 = (int)(i - (long)r * nq) * 4;
    const long row = (long)b * R + r;
    pack_quad<FMT>(f + (size_t)r * ld, yq, (size_t)row * 2 * Np, n0, N, Np, inv);
  }
  if (tid == 0) scales[b] = scale;
  if (flag && b == 0 && tid == 0) *flag = 0u;  // nothing waited (see pack_slices_kernel)
}

// scales doubles as the per-frame max word until the last launch turns it
// into the scale, so the four launches must stay in this order on one stream.
hipError_t launch_pack(const float *y, void *yq, float *scales, int batch, int R, int N,
                       int ld, int fmt, hipStream_t s, uint32_t *flag) {
  if (fmt < 1 || fmt > 3) return hipErrorInvalidValue;
  const float target = (fmt == 3) ? 448.0f : 1.0f;
  if (batch >= kPackFrameBatch && (long long)R * ld * 8 <= kPackFrameMaxBytes) {
    const dim3 grid((unsigned)batch), block(kPackFrameThreads);
    const f2a8 *yc = (const f2a8 *)y;
    if (fmt == 1)
      hipLaunchKernelGGL((pack_frame_kernel<1>), grid, block, 0, s, yc, yq, scales, R, N, ld,
                         target, flag);
    else if (fmt == 2)
      hipLaunchKernelGGL((pack_frame_kernel<2>), grid, block, 0, s, yc, yq, scales, R, N, ld,
                         target, flag);
    else
      hipLaunchKernelGGL((pack_frame_kernel<3>), grid, block, 0, s, yc, yq, scales, R, N, ld,
                         target, flag);
    return hipGetLastError();
  }
  uint32_t *mb = (uint32_t *)scales;
  const f2a8 *yc = (const f2a8 *)y;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, mb, batch);
  if (ld == N) {
    const long per_frame = (long)R * N;
    const long slices = std::max(1L, std::min(64L, per_frame / (256L * kMaxUnroll)));
    hipLaunchKernelGGL(frame_max_kernel, dim3((unsigned)slices, (unsigned)batch), dim3(256), 0,
                       s, yc, mb, per_frame);
  } else {
    hipLaunchKernelGGL(frame_max_rows_kernel, dim3((unsigned)std::min(R, 64), (unsigned)batch),
                       dim3(256), 0, s, yc, mb, R, N, ld);
  }
  const long total = (long)batch * R * ((N + 1) >> 2);
  const dim3 grid((unsigned)((total + 255) / 256));
  if (fmt == 1)
    hipLaunchKernelGGL((pack_kernel<1>), grid, dim3(256), 0, s, yc, yq, mb, R, N, ld, target,
                       total);
  else if (fmt == 2)
    hipLaunchKernelGGL((pack_kernel<2>), grid, dim3(256), 0, s, yc, yq, mb, R, N, ld, target,
                       total);
  else
    hipLaunchKernelGGL((pack_kernel<3>), grid, dim3(256), 0, s, yc, yq, mb, R, N, ld, target,
                       total);
  hipLaunchKernelGGL(finalize_scale_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, scales,
                     batch, target, flag);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// One HBM read of large frames. A frame's padded sample space (R rows of
// N + 1 samples, the pad reading as zero) is cut into slices of TH * Q
// quads, one workgroup per slice, the slices of frame b at workgroups
// b * slices .. b * slices + slices - 1. A workgroup loads its slice into
// registers, writes the slice's max-abs word into its own slot of the
// frame's line in the workspace (the top bit set: the max-abs bits of a
// float never use it), then one wave polls the frame's slots until every
// one is written, takes their maximum, and the workgroup converts its
// registers and stores the codes.
//
// Every slot is a single word written once by one workgroup and read by
// the others with device-scope atomic loads: each word is coherent on its
// own, and the flag and the value arrive in the same word, so no ordering
// between locations and no cache write-back or invalidation is needed, and
// no read-modify-write serialises the slices of a frame at one address.
//
// The wait needs the frame's workgroups to run at the same time. Workgroups
// are dispatched in index order, so the lowest frame not yet done always has
// all its workgroups dispatched once the frames before it have finished,
// provided the chip holds `slices` workgroups at once (also with a second
// such launch running beside it); the launch therefore takes this path only
// when slices <= half of what the chip holds. The wait is still bounded
// (spin_limit polls, one to two seconds): a workgroup that reaches the bound
// sets *err and goes on with the slots it has seen, and every other waiting
// workgroup sees *err within 64 polls and goes on too, so a broken residency
// assumption shows as a flag and a delay of one bound, not as a hang.
// work: per frame a line of kPackSyncWords words whose first `slices` are
// the slots (a line per frame also spreads the polls of the frames in
// flight over memory channels), zeroed before the launch; err: one word,
// zeroed before the launch.
// ---------------------------------------------------------------------------
constexpr int kSliceThreads = 256;
constexpr int kSliceQuads = 16;  // quads per thread: 64 complex samples in registers
constexpr uint32_t kSpinLimit = 1u << 20;  // polls of one to two microseconds each
constexpr uint32_t kSlotWritten = 0x80000000u;

template <int FMT, int Q, int TH>
__global__ __launch_bounds__(TH) void pack_slices_kernel(const f2a8 *y, void *yq, float *scales,
                                                         uint32_t *work, uint32_t *err, int R,
                                                         int N, int ld, float target, int slices,
                                                         uint32_t spin_limit) {
  const int tid = threadIdx.x;
  const int b = (int)(blockIdx.x / (unsigned)slices);
  const int sl = (int)(blockIdx.x - (unsigned)b * (unsigned)slices);
  // N + 1 is a power of two, so is the number of quads per padded row; the
  // R * (N + 1) / 4 quads of a frame stay below 2^30
  const int Np = N + 1;
  const int sh = __builtin_ctz((unsigned)Np) - 2;
  const int quads = R << sh;
  const f2a8 *f = y + (size_t)b * R * ld;
  f2a8 v[Q][4];
#pragma unroll
  for (int u = 0; u < Q; ++u) {
    const int q = (sl * Q + u) * TH + tid;
    if (q < quads) {
      const int r = q >> sh;
      load_quad(f + (size_t)r * ld, (q - (r << sh)) * 4, N, v[u]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[u][j] = f2a8{0.0f, 0.0f};
    }
  }
  uint32_t m = 0u;
#pragma unroll
  for (int u = 0; u < Q; ++u)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float re = v[u][j].x, im = v[u][j].y;
      m = max(m, __builtin_bit_cast(uint32_t, re) & 0x7FFFFFFFu);
      m = max(m, __builtin_bit_cast(uint32_t, im) & 0x7FFFFFFFu);
    }
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
  __shared__ uint32_t s_wave[TH / 64];
  __shared__ uint32_t s_frame;
  if ((tid & 63) == 0) s_wave[tid >> 6] = m;
  __syncthreads();
  uint32_t *line = work + (size_t)kPackSyncWords * b;
  if (tid < 64) {
    if (tid == 0) {
      m = 0u;
#pragma unroll
      for (int w = 0; w < TH / 64; ++w) m = max(m, s_wave[w]);
      __hip_atomic_store(line + sl, m | kSlotWritten, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t polls = 0u, fm;
    while (true) {
      uint32_t lane_max = 0u;
      bool lane_all = true;
      for (int i = tid; i < slices; i += 64) {
        const uint32_t w = __hip_atomic_load(line + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        lane_all = lane_all && (w & kSlotWritten);
        lane_max = max(lane_max, w & ~kSlotWritten);
      }
      for (int o = 32; o > 0; o >>= 1) lane_max = max(lane_max, (uint32_t)__shfl_xor((int)lane_max, o));
      fm = lane_max;
      if (__all(lane_all)) break;
      if (++polls >= spin_limit) {
        if (tid == 0) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      // once any workgroup of the launch has given up, stop waiting too, so
      // a launch is delayed by one bound at most, not one per frame
      if ((polls & 63u) == 0u &&
          __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
        break;
      __builtin_amdgcn_s_sleep(16);
    }
    if (tid == 0) s_frame = fm;
  }
  __syncthreads();
  const float scale = scale_from_maxbits(s_frame, target);
  const float inv = 1.0f / scale;
#pragma unroll
  for (int u = 0; u < Q; ++u) {
    const int q = (sl * Q + u) * TH + tid;
    if (q < quads) {
      const int r = q >> sh;
      const int n0 = (q - (r << sh)) * 4;
      store_quad<FMT>(v[u], yq, ((size_t)b * R + r) * 2 * Np + n0, N - n0, Np, inv);
    }
  }
  if (sl == 0 && tid == 0) scales[b] = scale;
}

// Clears the first `slices` words of every frame's line and the flag after
// the lines.
__global__ __launch_bounds__(256) void zero_sync_kernel(uint32_t *work, int batch, int slices) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const long n = (long)batch * slices;
  if (i < n) {
    const long b = i / slices;
    work[(size_t)kPackSyncWords * b + (size_t)(i - b * slices)] = 0u;
  } else if (i == n) {
    work[(size_t)kPackSyncWords * batch] = 0u;
  }
}

// Workgroups of pack_slices_kernel<FMT> the current device holds at once.
static int slice_capacity(int fmt) {
  static std::mutex mu;
  static std::vector<int> cache;  // [device * 3 + fmt - 1], 0 = not yet known
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  const size_t at = (size_t)dev * 3 + (size_t)(fmt - 1);
  if (cache.size() <= at) cache.resize(at + 1, 0);
  if (!cache[at]) {
    int per_cu = 0, cus = 0;
    const void *k =
        fmt == 1   ? (const void *)pack_slices_kernel<1, kSliceQuads, kSliceThreads>
        : fmt == 2 ? (const void *)pack_slices_kernel<2, kSliceQuads, kSliceThreads>
                   : (const void *)pack_slices_kernel<3, kSliceQuads, kSliceThreads>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kSliceThreads, 0) != hipSuccess)
      return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    cache[at] = per_cu * cus;
  }
  return cache[at];
}

int pack_slices_per_frame(int R, int N) {
  const long quads = (long)R * ((N + 1) >> 2);  // N + 1 = 2^d, d >= 2
  const long per = (long)kSliceThreads * kSliceQuads;
  return (int)std::min<long>((quads + per - 1) / per, 1L << 30);
}

hipError_t launch_pack_ws(const float *y, void *yq, float *scales, uint32_t *work, int batch,
                          int R, int N, int ld, int fmt, hipStream_t s) {
  if (fmt < 1 || fmt > 3) return hipErrorInvalidValue;
  const bool small_frames = (long long)R * ld * 8 <= kPackFrameMaxBytes;
  uint32_t *err = work + (size_t)kPackSyncWords * batch;
  if (batch >= kPackFrameBatch && small_frames)
    return launch_pack(y, yq, scales, batch, R, N, ld, fmt, s, err);
  const int slices = pack_slices_per_frame(R, N);
  const int cap = slice_capacity(fmt);
  if (cap <= 0 || slices > cap / 2 || slices > kPackSyncWords ||
      (long long)slices * batch > 0x7FFFFFFFLL)
    return launch_pack(y, yq, scales, batch, R, N, ld, fmt, s, err);
  const float target = (fmt == 3) ? 448.0f : 1.0f;
  const long zero_n = (long)batch * slices + 1;
  hipLaunchKernelGGL(zero_sync_kernel, dim3((unsigned)((zero_n + 255) / 256)), dim3(256), 0, s,
                     work, batch, slices);
  const dim3 grid((unsigned)(slices * batch)), block(kSliceThreads);
  const f2a8 *yc = (const f2a8 *)y;
  if (fmt == 1)
    hipLaunchKernelGGL((pack_slices_kernel<1, kSliceQuads, kSliceThreads>), grid, block, 0, s,
                       yc, yq, scales, work, err, R, N, ld, target, slices, kSpinLimit);
  else if (fmt == 2)
    hipLaunchKernelGGL((pack_slices_kernel<2, kSliceQuads, kSliceThreads>), grid, block, 0, s,
                       yc, yq, scales, work, err, R, N, ld, target, slices, kSpinLimit);
  else
    hipLaunchKernelGGL((pack_slices_kernel<3, kSliceQuads, kSliceThreads>), grid, block, 0, s,
                       yc, yq, scales, work, err, R, N, ld, target, slices, kSpinLimit);
  return hipGetLastError();
}

}  // namespace pnce
