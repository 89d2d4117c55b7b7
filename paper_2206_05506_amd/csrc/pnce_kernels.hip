// pnce_kernels.hip -- gfx950 kernels of the PN-sequence correlation channel
// estimator (arXiv 2206.05506, Eq. 3 and Eq. 10) and of its adjoint.
//
// Both operations are Toeplitz +-1 contractions of complex rows:
//   out[r][c] = alpha * sum_t in[r][t] * s'[(t - c) mod N] + beta * cin[r][c]
// with s' the sequence (correlator: t = sample n, c = lag k) or the sequence
// read backwards (adjoint: t = lag k, c = sample n). The +-1 operand is never
// read from memory: every lane expands it from a bit stream held in LDS.
//
// Tiling (one workgroup = 4 wave64s):
//  - tile = 32 antennas x (4 waves * 32*NC output columns);
//  - input chunks of the tile (32 rows x 32..128 samples) arrive in register
//    sets by unconditional buffer loads bounded by the frame, are converted
//    to the operand format of the matrix core while stored into LDS, and are
//    double-buffered with one barrier per chunk; all 4 waves read a chunk
//    (each owns 32*NC columns);
//  - matrix-core A operand = input rows (real and imaginary planes), B operand
//    = the +-1 Toeplitz tile, C = FP32 accumulators (2*NC 32x32 blocks);
//  - Toeplitz reuse: the B fragment of column block c at k-step i equals the
//    fragment of block 0 at k-step i - 2c, so a wave expands ONE new fragment
//    per k-step and rotates 2*NC of them through registers.
#include <algorithm>
#include <type_traits>

#include "pnce_device.h"

namespace pnce {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kRows = 32;      // antennas per tile
constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

// ---------------------------------------------------------------------------
// Samples per LDS stage (one barrier each) and operand formats of a stage.
// Between barriers a wave runs KS = ch/16 k-steps of matrix-core work, so a
// stage is as long as the register sets that feed it allow: complex64 input
// needs twice the registers of packed codes per sample, and the FP32-accurate
// and FP32 modes do 3x / 4x more matrix work per k-step already.
// Rows are padded by 4 dwords so that the 16-byte fragment reads of 8
// consecutive rows fall in distinct LDS banks.
//   MODE_F32            : 2 fp32 planes (re, im), 32 samples + pad   -> 36 dwords
//   MODE_F32S           : 6 bf16 planes (re hi/mid/lo, im hi/mid/lo) -> 20 dwords
//   MODE_BF16, complex64: 2 bf16 planes, 64 samples + pad            -> 36 dwords
//   MODE_BF16, codes    : 2 bf16/f16 planes, 128 samples + pad       -> 68 dwords
// ---------------------------------------------------------------------------
template <int MODE, int IN = IN_C64> struct StageGeom;
template <int IN> struct StageGeom<MODE_F32, IN> { static constexpr int ch = 32, planes = 2, rs = 36; };
template <int IN> struct StageGeom<MODE_F32S, IN> { static constexpr int ch = 32, planes = 6, rs = 20; };
template <int IN> struct StageGeom<MODE_BF16, IN> { static constexpr int ch = 128, planes = 2, rs = 68; };
template <> struct StageGeom<MODE_BF16, IN_C64> { static constexpr int ch = 64, planes = 2, rs = 36; };
template <> struct StageGeom<MODE_BF16, IN_C64_LAGS> : StageGeom<MODE_BF16, IN_C64> {};

// e4m3 codes (tg_fp8_kernel): 256 codes per stage (four k-steps of 64), rows
// padded by 4 dwords like the 16-bit code stages.
constexpr int kFp8Chunk = 256;
constexpr int kFp8RowDw = kFp8Chunk / 4 + 4;  // padded plane row in dwords

template <int MODE, int IN = IN_C64> constexpr int stage_dwords() {
  return StageGeom<MODE, IN>::planes * kRows * StageGeom<MODE, IN>::rs;
}

__device__ __forceinline__ uint32_t bf16_bits(float x) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float bf16_value(uint32_t b) {
  return __builtin_bit_cast(float, b << 16);
}
__device__ __forceinline__ uint32_t pack2(uint32_t lo, uint32_t hi) {
  return lo | (hi << 16);
}
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// Two FP32 values rounded to bf16 (nearest even) in one packed conversion:
// lo in bits 0-15, hi in bits 16-31.
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

// Exact three-way bf16 split of an FP32 value: x = hi + mid + lo up to
// 2^-24 relative (each part rounds the remainder to nearest even; the
// remainders are exact in FP32). Non-finite x keeps hi = x, mid = lo = 0.
__device__ __forceinline__ void split3(float x, uint32_t &hi, uint32_t &mid,
                                       uint32_t &lo) {
  hi = bf16_bits(x);
  float r1 = x - bf16_value(hi);
  r1 = __builtin_isfinite(x) ? r1 : 0.0f;
  mid = bf16_bits(r1);
  float r2 = r1 - bf16_value(mid);
  lo = bf16_bits(r2);
}

// ---------------------------------------------------------------------------
// Global -> register loads of one stage: 32 rows x 32 samples.
// c64 input: 512 sample pairs, thread t takes pairs t and t+256
//   (row = pair >> 4, samples 2*(pair & 15) and +1): each wave instruction
//   reads 4 rows x 256 contiguous bytes.
// packed input: 32 rows x 2 planes x 64 bytes, thread t takes 16 bytes
//   (row = t >> 3, plane = (t >> 2) & 1, 8 codes at 8*(t & 3)).
// Samples at or beyond t_len and antennas at or beyond R read as zero.
// ---------------------------------------------------------------------------
// One thread's share of a CH-sample stage held in registers (plain loads,
// waited for by the compiler): complex64 input, CH/16 sample pairs; packed
// input, CH/32 pieces of 8 codes.
template <int CH> struct RawC64 {
  f32x4 v[CH / 16];
};
template <int CH> struct RawPacked {
  u32x4 v[CH / 32];
};

// Complex64 stages come through the frame-bounded buffer resource
// (frame_rsrc): thread t reads sample pairs q = t + 256 i of a stage (row
// q / (CH/2), samples 2 (q % (CH/2)) and +1); a wave instruction reads 64
// consecutive pairs.
// Byte offset of this thread's pair i of a stage at sample 0.
template <int CH>
__device__ __forceinline__ uint32_t pair_voff(int i, int a0, int ld_in, int tid) {
  const int q = tid + kThreads * i;
  return ((uint32_t)(a0 + q / (CH / 2)) * (uint32_t)ld_in + 2u * (q % (CH / 2))) * 8u;
}

// A pair cut by the end of its row (n + 1 == t_len, t_len >= 2) is read one
// sample early, so the 16 bytes end at the row's end; mask_stage shifts it.
template <int CH>
__device__ __forceinline__ void load_stage(RawC64<CH> &raw, __amdgpu_buffer_rsrc_t rsrc,
                                           const uint32_t (&voff)[CH / 16], int n0, int t_len,
                                           int tid) {
  const int n = n0 + 2 * (tid % (CH / 2));
  const uint32_t off = 8u * n0 - (n + 1 == t_len ? 8u : 0u);
#pragma unroll
  for (int i = 0; i < CH / 16; ++i)
    raw.v[i] = __builtin_bit_cast(
        f32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[i] + off, 0, 0));
}

// Pairs cut by the end of the row keep only their valid sample (read one
// sample early: it arrives in the upper half); pairs past it (the next row's
// samples, or zeros past the frame) become zero. Only the last stage needs it.
template <int CH>
__device__ __forceinline__ void mask_stage(RawC64<CH> &raw, int n0, int t_len, int tid) {
  const int n = n0 + 2 * (tid % (CH / 2));
#pragma unroll
  for (int i = 0; i < CH / 16; ++i) {
    if (n >= t_len) {
      raw.v[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    } else if (n + 1 == t_len) {
      raw.v[i] = f32x4{raw.v[i].z, raw.v[i].w, 0.f, 0.f};
    }
  }
}

// Rows of lag blocks (IN_C64_LAGS): reduction position u holds term
// j * len + l of the row when u = j * step + l, l < len, j < n, and zero
// otherwise (the guard lags between blocks). Each sample is one 8-byte load;
// a position without a term is read at an offset past any frame (zero).
// rowoff[i]: byte offset of the row of this thread's pair i.
struct LagBlocks {
  int len, step, n;
};
template <int CH>
__device__ __forceinline__ void load_stage_lags(RawC64<CH> &raw, __amdgpu_buffer_rsrc_t rsrc,
                                                const uint32_t (&rowoff)[CH / 16], int n0,
                                                LagBlocks g, int tid) {
  const int u = n0 + 2 * (tid % (CH / 2));
  uint32_t src[2], off_frame[2];  // byte offset in the row; bit 31 if no term
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int j = (u + e) / g.step;
    const int l = u + e - j * g.step;
    src[e] = 8u * (uint32_t)(j * g.len + l);
    off_frame[e] = (j < g.n && l < g.len) ? 0u : 0x80000000u;
  }
#pragma unroll
  for (int i = 0; i < CH / 16; ++i) {
    const f32x2 lo = __builtin_bit_cast(
        f32x2,
        __builtin_amdgcn_raw_buffer_load_b64(rsrc, (rowoff[i] + src[0]) | off_frame[0], 0, 0));
    const f32x2 hi = __builtin_bit_cast(
        f32x2,
        __builtin_amdgcn_raw_buffer_load_b64(rsrc, (rowoff[i] + src[1]) | off_frame[1], 0, 0));
    raw.v[i] = f32x4{lo.x, lo.y, hi.x, hi.y};
  }
}

// Packed rows: 32 rows x 2 planes x CH codes in 16-byte pieces; piece
// q = t + 256 i covers row q / (CH/4), plane (q / (CH/8)) & 1, codes
// 8 (q % (CH/8)) .. +7. Rows that are not 8-code aligned, or a t_len that is
// not a multiple of 8 (N + 1 = 4, d = 2), take this code-by-code loader.
template <int CH>
__device__ __forceinline__ void load_stage_codes(RawPacked<CH> &raw, const uint16_t *in_frame,
                                                 int R, int a0, int ld_in, int t_len, int n0,
                                                 int tid) {
#pragma unroll
  for (int i = 0; i < CH / 32; ++i) {
    const int q = tid + kThreads * i;
    const int row = q / (CH / 4);
    const int plane = (q / (CH / 8)) & 1;
    const int n = n0 + 8 * (q % (CH / 8));
    const int a = a0 + row;
    u32x4 x = {0u, 0u, 0u, 0u};
    if (a < R) {
      const uint16_t *p = in_frame + ((size_t)a * 2 + plane) * ld_in + n;
      uint32_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) e[j] = (n + j < t_len) ? p[j] : 0u;
      x = u32x4{pack2(e[0], e[1]), pack2(e[2], e[3]), pack2(e[4], e[5]), pack2(e[6], e[7])};
    }
    raw.v[i] = x;
  }
}

// Aligned packed rows (8-code aligned, t_len a multiple of 8) through the
// frame-bounded buffer resource: piece q = t + 256 i at byte offset
// ((a0 + row) * 2 + plane) * ld_in * 2 + 16 * (q % (CH/8)) + 2 * n0.
template <int CH>
__device__ __forceinline__ uint32_t piece_voff(int i, int a0, int ld_in, int tid) {
  const int q = tid + kThreads * i;
  const int row = q / (CH / 4);
  const int plane = (q / (CH / 8)) & 1;
  return ((uint32_t)((a0 + row) * 2 + plane) * (uint32_t)ld_in) * 2u + 16u * (q % (CH / 8));
}

template <int CH>
__device__ __forceinline__ void load_stage(RawPacked<CH> &raw, __amdgpu_buffer_rsrc_t rsrc,
                                           const uint32_t (&voff)[CH / 16], int n0) {
#pragma unroll
  for (int i = 0; i < CH / 32; ++i)
    raw.v[i] = __builtin_bit_cast(
        u32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[i] + 2u * n0, 0, 0));
}

// Pieces at or past t_len (they read the next plane) become zero.
template <int CH>
__device__ __forceinline__ void mask_stage(RawPacked<CH> &raw, int n0, int t_len, int tid) {
#pragma unroll
  for (int i = 0; i < CH / 32; ++i) {
    const int q = tid + kThreads * i;
    if (n0 + 8 * (q % (CH / 8)) >= t_len) raw.v[i] = u32x4{0u, 0u, 0u, 0u};
  }
}

// Register -> LDS: one sample pair (re0, im0, re1, im1) of stage row `row`,
// pair `pr`, converted to the operand format while stored.
template <int MODE>
__device__ __forceinline__ void store_pair(uint32_t *st, int row, int pr, f32x4 x) {
  constexpr int RS = StageGeom<MODE>::rs;
  constexpr int PS = kRows * RS;  // plane stride in dwords
  if constexpr (MODE == MODE_F32) {
    *(f2a8 *)(st + row * RS + 2 * pr) = f2a8{x.x, x.z};
    *(f2a8 *)(st + PS + row * RS + 2 * pr) = f2a8{x.y, x.w};
  } else if constexpr (MODE == MODE_BF16) {
    st[row * RS + pr] = bf16_pair(x.x, x.z);
    st[PS + row * RS + pr] = bf16_pair(x.y, x.w);
  } else {  // MODE_F32S
    uint32_t h0, m0, l0, h1, m1, l1;
    split3(x.x, h0, m0, l0);
    split3(x.z, h1, m1, l1);
    st[0 * PS + row * RS + pr] = pack2(h0, h1);
    st[1 * PS + row * RS + pr] = pack2(m0, m1);
    st[2 * PS + row * RS + pr] = pack2(l0, l1);
    split3(x.y, h0, m0, l0);
    split3(x.w, h1, m1, l1);
    st[3 * PS + row * RS + pr] = pack2(h0, h1);
    st[4 * PS + row * RS + pr] = pack2(m0, m1);
    st[5 * PS + row * RS + pr] = pack2(l0, l1);
  }
}

template <int MODE, int CH>
__device__ __forceinline__ void store_stage(uint32_t *st, const RawC64<CH> &raw, int tid) {
#pragma unroll
  for (int i = 0; i < CH / 16; ++i) {
    const int q = tid + kThreads * i;
    store_pair<MODE>(st, q / (CH / 2), q % (CH / 2), raw.v[i]);
  }
}

template <int MODE, int CH>
__device__ __forceinline__ void store_stage(uint32_t *st, const RawPacked<CH> &raw, int tid) {
  constexpr int RS = StageGeom<MODE, IN_BF16>::rs;
  constexpr int PS = kRows * RS;
#pragma unroll
  for (int i = 0; i < CH / 32; ++i) {
    const int q = tid + kThreads * i;
    const int row = q / (CH / 4);
    const int plane = (q / (CH / 8)) & 1;
    *(u32x4 *)(st + plane * PS + row * RS + 4 * (q % (CH / 8))) = raw.v[i];
  }
}

// Expand 8 bits into 8 16-bit +-1 values (bit 1 -> sign set). ONE is the
// 16-bit pattern of +1 in both halves: 0x3F803F80 (bf16), 0x3C003C00 (f16).
template <uint32_t ONE>
__device__ __forceinline__ u32x4 expand16(uint32_t x) {
  u32x4 r;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    r[e] = ONE | ((x << (15 - 2 * e)) & 0x8000u) | ((x << (30 - 2 * e)) & 0x80000000u);
  return r;
}

// Window slot register file: 16-bit modes keep the expanded fragment, the
// FP32 mode keeps the raw 8 bits and expands one bit per MFMA.
template <int MODE> struct Win { u32x4 f; };
template <> struct Win<MODE_F32> { uint32_t f; };

// 16-bit modes read the expanded fragment of an 8-bit window from a 256-entry
// LDS table (4 KiB, filled once per workgroup by fill_lut).
template <int MODE, int IN>
__device__ __forceinline__ void make_window(Win<MODE> &w, uint32_t bits8, const uint32_t *lut) {
  if constexpr (MODE == MODE_F32) {
    w.f = bits8;
  } else {
    w.f = *(const u32x4 *)(lut + 4 * bits8);
  }
}

constexpr int kLutDw = 256 * 4;

template <int IN>
__device__ __forceinline__ void fill_lut(uint32_t *lut) {
  const int e = threadIdx.x;  // kThreads == 256 entries
  const u32x4 v = (IN == IN_F16) ? expand16<0x3C003C00u>((uint32_t)e)
                                 : expand16<0x3F803F80u>((uint32_t)e);
  *(u32x4 *)(lut + 4 * e) = v;
}

// ---------------------------------------------------------------------------
// The tiled kernel.
// ---------------------------------------------------------------------------
// Stages in flight (register sets): 32 KiB of complex64, or 32 KiB of
// codes, per workgroup.
template <int MODE, int IN> struct RegDepth {
  static constexpr int value = StageGeom<MODE, IN>::ch >= 64 ? 2 : 4;
};

// LDS dwords of one workgroup tile: bit stream + window table + two stages.
template <int MODE, int IN>
constexpr int tile_lds_dwords(int nbw_pad) {
  return nbw_pad + kLutDw + 2 * stage_dwords<MODE, IN>();
}

// LDS of the largest kernel for a bit stream of nbw words: the tiled kernel
// on packed 16-bit codes (the widest stages) holds the most besides the
// stream; the FP64 and e4m3 kernels hold less.
size_t max_lds_bytes(int nbw) {
  const int nbw_pad = (nbw + 3) & ~3;
  int d = tile_lds_dwords<MODE_BF16, IN_BF16>(nbw_pad);
  d = std::max(d, tile_lds_dwords<MODE_F32S, IN_C64>(nbw_pad));
  d = std::max(d, tile_lds_dwords<MODE_F32, IN_C64>(nbw_pad));
  d = std::max(d, tile_lds_dwords<MODE_BF16, IN_C64>(nbw_pad));
  d = std::max(d, nbw_pad + 2 * stage_dwords<MODE_F32>());
  d = std::max(d, nbw_pad + 2 * 2 * kRows * kFp8RowDw);
  return (size_t)d * 4;
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Sum over the 32 lanes of each half-wave, result in every lane: lane moves
// within 16-lane rows (quad permutes for xor 1 and xor 2, then the half-row
// and row mirrors, which pair each 4- and 8-lane group with the other one),
// then one shuffle across the two rows.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float half_wave_sum(float x) {
  x += dpp_move<0xB1>(x);   // quad_perm [1,0,3,2]: lane ^ 1
  x += dpp_move<0x4E>(x);   // quad_perm [2,3,0,1]: lane ^ 2
  x += dpp_move<0x141>(x);  // row_half_mirror: the other quad of each 8 lanes
  x += dpp_move<0x140>(x);  // row_mirror: the other 8 lanes of each row
  return x + __shfl_xor(x, 16);
}

// One workgroup tile of the contraction: 32 antennas from a0, 4 waves x
// 32*NC output columns from colg, of one frame whose rows start at `in`
// (input) and `out` / `cin` (output). The sequence bits must already be in
// LDS (sbits); the first barrier below publishes them.
struct Tile {
  const void *in;
  float *out;
  const float *cin;
  int R, t_len, ld_in, c_len, ld_out, N;
  int a0, colg;
  float alpha, beta;
  bool ls;  // least-squares rows (the tile holds every lag of its rows)
  int seg_len, seg_lag, poff;  // column segments and sequence shift (TgArgs)
  int rseg_len, rseg_lag, rseg_n;  // reduction blocks of IN_C64_LAGS rows
};

// SB: column segments (Eq. 8 lags) with every 32-column block in its own
// segment: each block has its own first lag and builds its own B fragment per
// k-step (no reuse across blocks), so a wave's blocks may sit in different
// transmitters' segments and segments are padded to 32 columns only.
struct NoPre {
  __device__ void operator()() const {}
};

// pre(): the caller's set-up of the LDS tables (sequence bits, window
// table), run after the first stages' loads are issued so that their
// latency overlaps it; the barrier below publishes both.
template <int MODE, int IN, int NC, bool AL, bool SB = false, typename Pre = NoPre>
__device__ __forceinline__ void run_tile(const Tile &tl, const uint32_t *sbits,
                                         const uint32_t *lut, uint32_t *stage,
                                         const Pre &pre = Pre{}) {
  constexpr int NWIN = 2 * NC;
  constexpr int RS = StageGeom<MODE, IN>::rs;
  constexpr int PS = kRows * RS;
  constexpr int SDW = stage_dwords<MODE, IN>();
  constexpr int CH = StageGeom<MODE, IN>::ch;  // samples per stage
  constexpr int KS = CH / 16;                // k-steps per stage
  constexpr bool LAGS = IN == IN_C64_LAGS;   // gathered by lag blocks
  constexpr bool C64 = IN == IN_C64 || LAGS;
  constexpr int PF = RegDepth<MODE, IN>::value;  // stages in flight
  // Chunks per unrolled body: the window rotation (NWIN k-steps) and the
  // register-set rotation (PF) both repeat after CPB chunks.
  constexpr int CPW = (NWIN > KS) ? NWIN / KS : 1;
  constexpr int CPB = (CPW > PF) ? CPW : PF;
  static_assert((CPB * KS) % NWIN == 0 && CPB % PF == 0, "body must cover rotations");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m = lane & 31;
  const int h = lane >> 5;
  const int a0 = tl.a0;
  // this wave's 32*NC columns: lags sp.lag0 + j, stored at sp.ocol0 + j for
  // j < sp.n_out (SB: block c's 32 columns from sb[c] likewise)
  const int v0 = tl.colg + wave * 32 * NC;
  const SegPos sp = seg_pos(v0, seg_pad(tl.seg_len, tl.seg_lag, SB ? 32 : 32 * NC), tl.seg_len,
                            tl.seg_lag, tl.c_len);
  [[maybe_unused]] SegPos sb[SB ? NC : 1];
  if constexpr (SB) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
      sb[c] = seg_pos(v0 + 32 * c, seg_pad(tl.seg_len, tl.seg_lag, 32), tl.seg_len, tl.seg_lag,
                      tl.c_len);
  }
  // block c: first stored column, and how many of its 32 columns are stored
  auto ocol = [&](int c) { return SB ? sb[c].ocol0 : sp.ocol0 + 32 * c; };
  auto nout = [&](int c) { return SB ? sb[c].n_out : sp.n_out - 32 * c; };

  const int nchunks = (tl.t_len + CH - 1) / CH;
  const int last = nchunks - 1;
  // global -> registers (PF chunks ahead) -> LDS stage in operand format.
  using Raw = std::conditional_t<C64, RawC64<CH>, RawPacked<CH>>;
  Raw raw[PF];
  // complex64 and aligned packed rows: unconditional loads through the
  // frame-bounded buffer resource, masked once in the last chunk.
  constexpr bool BUF = C64 || AL;
  // the frame ends with its last row's last term (rows may be strided past it)
  const int row_terms = LAGS ? tl.rseg_n * tl.rseg_len : tl.t_len;
  const __amdgpu_buffer_rsrc_t rsrc = frame_rsrc(
      tl.in, C64 ? ((long long)(tl.R - 1) * tl.ld_in + row_terms) * 8
                 : ((long long)(2 * tl.R - 1) * tl.ld_in + tl.t_len) * 2);
  uint32_t voff[CH / 16] = {};
#pragma unroll
  for (int i = 0; i < CH / 16; ++i)
    voff[i] = LAGS  ? pair_voff<CH>(i, a0, tl.ld_in, tid) - 16u * (uint32_t)(tid % (CH / 2))
              : C64 ? pair_voff<CH>(i, a0, tl.ld_in, tid)
                    : piece_voff<CH>(i, a0, tl.ld_in, tid);
  // chunk -> register set ISET; past the end: re-read the last chunk
  auto fetch = [&](int chunk, auto iset) {
    constexpr int S = decltype(iset)::value;
    const int c = chunk < last ? chunk : last;
    if constexpr (LAGS)
      load_stage_lags<CH>(raw[S], rsrc, voff, c * CH, LagBlocks{tl.rseg_len, tl.rseg_lag, tl.rseg_n},
                          tid);
    else if constexpr (C64)
      load_stage<CH>(raw[S], rsrc, voff, c * CH, tl.t_len, tid);
    else if constexpr (BUF)
      load_stage<CH>(raw[S], rsrc, voff, c * CH);
    else
      load_stage_codes<CH>(raw[S], (const uint16_t *)tl.in, tl.R, a0, tl.ld_in, tl.t_len,
                           c * CH, tid);
  };
  // register set ISET (holding `chunk`) -> LDS stage st
  auto land = [&](int chunk, auto iset, uint32_t *st) {
    constexpr int S = decltype(iset)::value;
    if constexpr (BUF && !LAGS) {
      if (chunk == last) mask_stage<CH>(raw[S], chunk * CH, tl.t_len, tid);
    }
    store_stage<MODE>(st, raw[S], tid);
  };
  using I0 = std::integral_constant<int, 0>;

  static_for<0, PF>([&](auto ij) { fetch(decltype(ij)::value, ij); });
  pre();
  land(0, I0{}, stage);
  fetch(PF, I0{});
  __syncthreads();

  // Bit position of this lane's B fragment for block 0 at k-step 0:
  // reduction index t0 = 8h (+ e), lag sp.lag0 + m.
  const int p_base = pos_mod(8 * h - m - sp.lag0 + tl.poff, tl.N);

  Win<MODE> win[SB ? 1 : NWIN];
  // SB: block c's fragments of k-steps i (slot i & 1) and i + 1
  [[maybe_unused]] Win<MODE> wb[SB ? NC : 1][2];
  [[maybe_unused]] int pb[SB ? NC : 1];
  if constexpr (SB) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      pb[c] = pos_mod(8 * h - m - sb[c].lag0 + tl.poff, tl.N);
      make_window<MODE, IN>(wb[c][0], window8(sbits, pb[c]), lut);
    }
  } else {
    // Prologue: fragments of k-steps -(NWIN-2) .. -1 (used by blocks c >= 1
    // during the first 2c k-steps).
#pragma unroll
    for (int j = 1; j <= NWIN - 2; ++j) {
      const int p = pos_mod(p_base - 16 * j, tl.N);
      make_window<MODE, IN>(win[NWIN - j], window8(sbits, p), lut);
    }
    make_window<MODE, IN>(win[0], window8(sbits, p_base), lut);  // k-step 0
  }
  // B fragment of block c at k-step i (slot q of the rotation)
  auto bfrag = [&](int c, int q, int i) -> const Win<MODE> & {
    if constexpr (SB)
      return wb[c][i & 1];
    else
      return win[(q - 2 * c + NWIN) % NWIN];
  };

  f32x16 acc_re[NC], acc_im[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      acc_re[c][v] = 0.f;
      acc_im[c][v] = 0.f;
    }
  }

  // One chunk of matrix-core work from LDS stage (chunk & 1); cc is the
  // chunk's position in the unrolled body, which fixes the window slots.
  // Software pipelined: during k-step i the window of step i + 1 is built
  // (its slot held step i + 1 - NWIN, an odd offset no block reads at step i)
  // and, in the one-plane 16-bit mode, the A operands of step i + 1 are read,
  // so no LDS round trip sits between two bursts of matrix-core ops.
  constexpr int NP = (MODE == MODE_F32S) ? 3 : 1;
  constexpr int AB = (MODE == MODE_BF16) ? 2 : 1;  // A operand buffers
  auto read_a = [&](const uint32_t *st, int u, u32x4 (&are)[NP], u32x4 (&aim)[NP]) {
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      are[s] = *(const u32x4 *)(st + s * PS + m * RS + 8 * u + 4 * h);
      aim[s] = *(const u32x4 *)(st + (NP + s) * PS + m * RS + 8 * u + 4 * h);
    }
  };
  auto do_chunk = [&](auto icc, int chunk) {
    constexpr int cc = decltype(icc)::value;
    const uint32_t *st = stage + (chunk & 1) * SDW;
    [[maybe_unused]] u32x4 are[AB][NP], aim[AB][NP];
    if constexpr (AB == 2) read_a(st, 0, are[0], aim[0]);
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int q = (KS * cc + u) % NWIN;  // slot of k-step i = KS*chunk + u
      const int i = KS * chunk + u;
      // (KS is even, so i & 1 == u & 1 is known at compile time)
      if constexpr (SB) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
          make_window<MODE, IN>(wb[c][(u + 1) & 1], window8(sbits, pb[c] + 16 * (i + 1)), lut);
      } else {
        make_window<MODE, IN>(win[(q + 1) % NWIN], window8(sbits, p_base + 16 * (i + 1)), lut);
      }
      if constexpr (MODE == MODE_F32) {
        const float *pre = (const float *)st + m * RS + 16 * u + 8 * h;
        const float *pim = pre + PS;
        f32x4 r0 = *(const f32x4 *)pre, r1 = *(const f32x4 *)(pre + 4);
        f32x4 i0 = *(const f32x4 *)pim, i1 = *(const f32x4 *)(pim + 4);
        float fre[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
        float fim[8] = {i0.x, i0.y, i0.z, i0.w, i1.x, i1.y, i1.z, i1.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const uint32_t x = bfrag(c, q, u).f;
            const float bv =
                __builtin_bit_cast(float, 0x3F800000u | ((x << (31 - j)) & 0x80000000u));
            acc_re[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(fre[j], bv, acc_re[c], 0, 0, 0);
            acc_im[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(fim[j], bv, acc_im[c], 0, 0, 0);
          }
        }
      } else {
        const int cur = (AB == 2) ? (u & 1) : 0;
        if constexpr (AB == 2) {
          if (u + 1 < KS) read_a(st, u + 1, are[(u + 1) & 1], aim[(u + 1) & 1]);
        } else {
          read_a(st, u, are[0], aim[0]);
        }
        // split part outer, lag block inner: the dependent updates of one
        // accumulator are 2*NC matrix-core ops apart
#pragma unroll
        for (int s = 0; s < NP; ++s) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const u32x4 bw = bfrag(c, q, u).f;
            if constexpr (IN == IN_F16) {
              acc_re[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                  __builtin_bit_cast(f16x8, are[cur][s]), __builtin_bit_cast(f16x8, bw),
                  acc_re[c], 0, 0, 0);
              acc_im[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                  __builtin_bit_cast(f16x8, aim[cur][s]), __builtin_bit_cast(f16x8, bw),
                  acc_im[c], 0, 0, 0);
            } else {
              acc_re[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  __builtin_bit_cast(bf16x8, are[cur][s]), __builtin_bit_cast(bf16x8, bw),
                  acc_re[c], 0, 0, 0);
              acc_im[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  __builtin_bit_cast(bf16x8, aim[cur][s]), __builtin_bit_cast(bf16x8, bw),
                  acc_im[c], 0, 0, 0);
            }
          }
        }
      }
    }
  };

  // Chunk c: matrix-core work on stage (c & 1); then chunk c + 1, fetched PF
  // chunks ago into set (c + 1), is staged, set (c + 1) is refilled with
  // chunk c + 1 + PF, and one barrier publishes the stage.
  // Steady state: bodies whose chunks stage only chunks before the last run
  // without a branch, so the compiler waits for exactly one register set per
  // chunk; the remaining 2 .. CPB + 1 chunks run with their checks.
  const int nmain = last >= 1 ? (last - 1) / CPB : 0;
  for (int body = 0; body < nmain; ++body) {
    static_for<0, CPB>([&](auto icc) {
      constexpr int cc = decltype(icc)::value;
      const int chunk = body * CPB + cc;
      do_chunk(icc, chunk);
      using IS = std::integral_constant<int, (cc + 1) % PF>;  // set of chunk + 1
      store_stage<MODE>(stage + ((chunk + 1) & 1) * SDW, raw[IS::value], tid);
      fetch(chunk + 1 + PF, IS{});
      __syncthreads();
      // Do not let the next chunk's conversion move up: it would wait for
      // every set in flight instead of one.
      __builtin_amdgcn_sched_barrier(0);
    });
  }
  static_for<0, CPB + 1>([&](auto icc) {
    constexpr int cc = decltype(icc)::value;
    const int chunk = nmain * CPB + cc;
    if (chunk < nchunks) {
      do_chunk(std::integral_constant<int, cc % CPB>{}, chunk);
      using IS = std::integral_constant<int, (cc + 1) % PF>;
      if (chunk + 1 < nchunks) land(chunk + 1, IS{}, stage + ((chunk + 1) & 1) * SDW);
      if (chunk + 1 + PF < nchunks) fetch(chunk + 1 + PF, IS{});
      __syncthreads();
    }
  });

  // Epilogue: lane (m, h) holds, for block c, output column ocol(c) + m
  // (stored when m < nout(c)) and rows 8*(v/4) + 4*h + (v%4) of the 32x32
  // accumulator.
  float alpha = tl.alpha;
  f32x16 tot_re = {}, tot_im = {};  // least squares: alpha * row sums
  if (tl.ls) {
    // Row sums over this wave's stored columns, then over the 32
    // lanes of each half-wave, then over the 4 waves through LDS (the stage
    // is no longer read); every lane then holds the sums of its 16 rows.
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const bool in = m < nout(c);
        sr += in ? acc_re[c][v] : 0.f;
        si += in ? acc_im[c][v] : 0.f;
      }
      tot_re[v] = half_wave_sum(sr);
      tot_im[v] = half_wave_sum(si);
    }
    float *red = (float *)stage;  // [wave][row][re, im]
    __syncthreads();
    if (m == 0) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int r = 8 * (v >> 2) + 4 * h + (v & 3);
        red[(wave * kRows + r) * 2] = tot_re[v];
        red[(wave * kRows + r) * 2 + 1] = tot_im[v];
      }
    }
    __syncthreads();
    const float c1 = (float)tl.N / (float)(tl.N + 1);
    const float c2 = 1.0f / (float)(tl.N + 1 - tl.c_len);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 8 * (v >> 2) + 4 * h + (v & 3);
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        sr += red[(w * kRows + r) * 2];
        si += red[(w * kRows + r) * 2 + 1];
      }
      tot_re[v] = c1 * alpha * c2 * sr;
      tot_im[v] = c1 * alpha * c2 * si;
    }
    alpha *= c1;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = ocol(c) + m;
    if (m < nout(c)) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int ant = a0 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (ant < tl.R) {
          const size_t o = ((size_t)ant * tl.ld_out + col) * 2;
          float re = alpha * acc_re[c][v] + tot_re[v];
          float im = alpha * acc_im[c][v] + tot_im[v];
          if (tl.beta != 0.0f) {
            const f2a8 old = *(const f2a8 *)(tl.cin + o);
            re += tl.beta * old.x;
            im += tl.beta * old.y;
          }
          // streaming store: the CIRs are not read again by this launch
          __builtin_nontemporal_store(f2a8{re, im}, (f2a8 *)(tl.out + o));
        }
      }
    }
  }
}


// One tile per workgroup over a uniform batch.
template <int MODE, int IN, int NC, bool AL, bool SB>
__global__ __launch_bounds__(kThreads, 2) void tg_kernel(TgArgs a, int tiles_r, int tiles_c,
                                                         int nbw_pad) {
  extern __shared__ __attribute__((aligned(16))) uint32_t smem[];
  // Tile order: column groups of one (frame, antenna block) are consecutive,
  // and consecutive tiles go to the same XCD (workgroups are dealt to the 8
  // XCDs round robin), so a row block's input is fetched into one L2.
  const int nt = a.batch * tiles_r * tiles_c;
  const int bid = blockIdx.x;
  const int t = (nt % 8 == 0) ? (bid % 8) * (nt / 8) + bid / 8 : bid;
  const int cg = t % tiles_c;
  const int rest = t / tiles_c;
  const int rb = rest % tiles_r;
  const int b = rest / tiles_r;

  // One word of the bit stream per thread is loaded before the first
  // stages' loads are issued and stored after them (see run_tile's pre);
  // longer streams are copied there in a loop.
  const bool one = a.nbw <= kThreads;
  const uint32_t bw = (one && (int)threadIdx.x < a.nbw) ? a.bits[threadIdx.x] : 0u;
  auto pre = [&]() {
    if (one) {
      if ((int)threadIdx.x < a.nbw) smem[threadIdx.x] = bw;
    } else {
      for (int i = threadIdx.x; i < a.nbw; i += kThreads) smem[i] = a.bits[i];
    }
    fill_lut<IN>(smem + nbw_pad);
  };
  Tile tl;
  if constexpr (IN == IN_C64 || IN == IN_C64_LAGS)
    tl.in = (const float *)a.in + (size_t)b * a.R * a.ld_in * 2;
  else
    tl.in = (const uint16_t *)a.in + (size_t)b * a.R * 2 * a.ld_in;
  tl.out = a.out + (size_t)b * a.R * a.ld_out * 2;
  tl.cin = a.cin ? a.cin + (size_t)b * a.R * a.ld_out * 2 : nullptr;
  tl.R = a.R;
  tl.t_len = a.t_len;
  tl.ld_in = a.ld_in;
  tl.c_len = a.c_len;
  tl.ld_out = a.ld_out;
  tl.N = a.N;
  tl.a0 = rb * kRows;
  tl.colg = cg * (kWaves * 32 * NC);
  tl.alpha = a.alpha * (a.scales ? a.scales[b] : 1.0f);
  tl.beta = a.beta;
  tl.ls = a.ls != 0;
  tl.seg_len = a.seg_len;
  tl.seg_lag = a.seg_lag;
  tl.poff = a.poff;
  tl.rseg_len = a.rseg_len;
  tl.rseg_lag = a.rseg_lag;
  tl.rseg_n = a.rseg_n;
  run_tile<MODE, IN, NC, AL, SB>(tl, smem, smem + nbw_pad, smem + nbw_pad + kLutDw, pre);
}

// Persistent kernel over an uneven batch: workgroup w walks its slice of a
// host-built work list; each tile names its frame (shape, sequence length,
// offsets) and its column width (32*nc lags per wave), so frames of any
// (R, N, T*L) share one launch. The bit stream is reloaded only when the
// sequence length changes between consecutive tiles.
template <int MODE, int IN>
__global__ __launch_bounds__(kThreads, 2) void varlen_kernel(VArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint32_t smem[];
  const int nbw_pad = (a.nbw_max + 3) & ~3;
  const uint32_t *lut = smem + nbw_pad;
  uint32_t *stage = smem + nbw_pad + kLutDw;
  fill_lut<IN>(smem + nbw_pad);
  int cur_bits = -1;
  const int end = a.wg_start[blockIdx.x + 1];
  for (int i = a.wg_start[blockIdx.x]; i < end; ++i) {
    const VTile vt = a.tiles[i];
    const VFrame f = a.frames[vt.frame];
    if (f.bits_off != cur_bits) {
      for (int j = threadIdx.x; j < f.nbw; j += kThreads) smem[j] = a.bits[f.bits_off + j];
      cur_bits = f.bits_off;
    }
    Tile tl;
    tl.in = (const uint16_t *)a.in + f.y_off;
    tl.out = a.out + f.h_off * 2;
    tl.cin = nullptr;
    tl.R = f.R;
    tl.t_len = f.N + 1;
    tl.ld_in = f.N + 1;
    tl.c_len = f.K;
    tl.ld_out = f.K;
    tl.N = f.N;
    tl.a0 = vt.a0;
    tl.colg = vt.colg;
    tl.alpha = (a.scales ? a.scales[vt.frame] : 1.0f) / (float)f.N;
    tl.beta = 0.0f;
    tl.ls = false;
    tl.seg_len = 0;
    tl.seg_lag = 0;
    tl.poff = 0;
    tl.rseg_len = tl.rseg_lag = tl.rseg_n = 0;
    if (f.N >= 7) {  // N + 1 = 2^d, d >= 3: rows 8-code aligned
      if (vt.nc == 4)
        run_tile<MODE, IN, 4, true>(tl, smem, lut, stage);
      else if (vt.nc == 2)
        run_tile<MODE, IN, 2, true>(tl, smem, lut, stage);
      else
        run_tile<MODE, IN, 1, true>(tl, smem, lut, stage);
    } else {
      run_tile<MODE, IN, 1, false>(tl, smem, lut, stage);
    }
  }
}

hipError_t launch_varlen(int in_fmt, const VArgs &a, int n_wg, hipStream_t s) {
  if (n_wg <= 0) return hipErrorInvalidValue;
  const int nbw_pad = (a.nbw_max + 3) & ~3;
  const size_t lds = (size_t)tile_lds_dwords<MODE_BF16, IN_BF16>(nbw_pad) * 4;
  if (in_fmt == IN_BF16) {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void *)varlen_kernel<MODE_BF16, IN_BF16>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((varlen_kernel<MODE_BF16, IN_BF16>), dim3(n_wg), dim3(kThreads), lds, s,
                       a);
  } else if (in_fmt == IN_F16) {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void *)varlen_kernel<MODE_BF16, IN_F16>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((varlen_kernel<MODE_BF16, IN_F16>), dim3(n_wg), dim3(kThreads), lds, s,
                       a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64-accumulating contraction on FP64 matrix cores (v_mfma_f64_16x16x4_f64)
// for complex64 rows: the last residual of least-squares refinement. Inputs
// are FP32, products with +-1 are exact in FP64 and every sum is FP64; the
// result is rounded to FP32 once.
// Tile: 32 antennas (two 16-row blocks) x 4 waves x 16*NB columns; the
// input is staged through LDS in 32-term chunks as FP32 planes (the MODE_F32
// stage layout). Lane (j, g) = (lane % 16, lane / 16) supplies reduction
// index t0 + g for row j (A) and column j (B); the B bit of column block c
// at k-step i (4 terms) sits at p_base + 4i - 16c.
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

// GA: rows of lag blocks (IN_C64_LAGS), gathered sample by sample.
template <int NB, bool GA>
__global__ __launch_bounds__(kThreads, 2) void tg_f64mm_kernel(TgArgs a, int tiles_r,
                                                               int tiles_c, int nbw_pad) {
  extern __shared__ __attribute__((aligned(16))) uint32_t smem[];
  constexpr int RS = StageGeom<MODE_F32>::rs;
  constexpr int PS = kRows * RS;
  constexpr int SDW = stage_dwords<MODE_F32>();
  constexpr int PF = 2;
  uint32_t *sbits = smem;
  uint32_t *stage = smem + nbw_pad;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int j16 = lane & 15;
  const int g = lane >> 4;

  const int nt = a.batch * tiles_r * tiles_c;
  const int bid = blockIdx.x;
  const int t = (nt % 8 == 0) ? (bid % 8) * (nt / 8) + bid / 8 : bid;
  const int cg = t % tiles_c;
  const int rest = t / tiles_c;
  const int rb = rest % tiles_r;
  const int b = rest / tiles_r;
  const int a0 = rb * kRows;
  const int col0 = cg * (kWaves * 16 * NB) + wave * 16 * NB;
  // column block c: lags sp[c].lag0 + j, stored at sp[c].ocol0 + j, j < n_out
  SegPos sp[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    sp[c] = seg_pos(col0 + 16 * c, seg_pad(a.seg_len, a.seg_lag, 16), a.seg_len, a.seg_lag,
                    a.c_len);

  const float *fin = (const float *)a.in + (size_t)b * a.R * a.ld_in * 2;
  constexpr int CH = 32;  // 8 k-steps of 4 terms per stage
  const int nchunks = (a.t_len + CH - 1) / CH;
  const int last = nchunks - 1;
  const int row_terms = GA ? a.rseg_n * a.rseg_len : a.t_len;
  const __amdgpu_buffer_rsrc_t rsrc =
      frame_rsrc(fin, ((long long)(a.R - 1) * a.ld_in + row_terms) * 8);
  uint32_t voff[CH / 16];
#pragma unroll
  for (int i = 0; i < CH / 16; ++i)
    voff[i] = pair_voff<CH>(i, a0, a.ld_in, tid) - (GA ? 16u * (uint32_t)(tid % (CH / 2)) : 0u);
  // chunk -> set (past the end: the last chunk again); set -> stage, masked
  // when it holds the last chunk
  auto fetch = [&](RawC64<CH> &r, int chunk) {
    const int n0 = (chunk < last ? chunk : last) * CH;
    if constexpr (GA)
      load_stage_lags<CH>(r, rsrc, voff, n0, LagBlocks{a.rseg_len, a.rseg_lag, a.rseg_n}, tid);
    else
      load_stage<CH>(r, rsrc, voff, n0, a.t_len, tid);
  };
  auto land = [&](uint32_t *st, RawC64<CH> &r, int chunk) {
    if (!GA && chunk == last) mask_stage<CH>(r, chunk * CH, a.t_len, tid);
    store_stage<MODE_F32>(st, r, tid);
  };
  RawC64<CH> raw[PF];
#pragma unroll
  for (int c = 0; c < PF; ++c) fetch(raw[c], c);
  for (int i = tid; i < a.nbw; i += kThreads) sbits[i] = a.bits[i];
  land(stage, raw[0], 0);
  fetch(raw[0], PF);
  __syncthreads();

  int p_base[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) p_base[c] = pos_mod(g - j16 - sp[c].lag0 + a.poff, a.N);
  f64x4 acc[2][2][NB];  // [row block][re, im][column block]
#pragma unroll
  for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
    for (int ri = 0; ri < 2; ++ri)
#pragma unroll
      for (int c = 0; c < NB; ++c) acc[r2][ri][c] = f64x4{0.0, 0.0, 0.0, 0.0};

  for (int chunk0 = 0; chunk0 < nchunks; chunk0 += PF) {
#pragma unroll
    for (int cc = 0; cc < PF; ++cc) {
      const int chunk = chunk0 + cc;
      if (chunk < nchunks) {
        const float *st = (const float *)(stage + (chunk & 1) * SDW);
        // 32-bit windows: bits p_base[c] + 32*chunk + 4j, j = 0..7
        uint32_t w[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c)
          w[c] = window32(sbits, pos_mod(p_base[c] + 32 * chunk, a.N));
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          double av[2][2];
#pragma unroll
          for (int r2 = 0; r2 < 2; ++r2) {
            av[r2][0] = (double)st[(16 * r2 + j16) * RS + 4 * j + g];
            av[r2][1] = (double)st[PS + (16 * r2 + j16) * RS + 4 * j + g];
          }
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            const uint64_t bb =
                (uint64_t)(0x3FF00000u | (((w[c] >> (4 * j)) & 1u) << 31)) << 32;
            const double bv = __builtin_bit_cast(double, bb);
#pragma unroll
            for (int r2 = 0; r2 < 2; ++r2)
#pragma unroll
              for (int ri = 0; ri < 2; ++ri)
                acc[r2][ri][c] =
                    __builtin_amdgcn_mfma_f64_16x16x4f64(av[r2][ri], bv, acc[r2][ri][c], 0, 0, 0);
          }
        }
        if (chunk + 1 < nchunks) land(stage + ((chunk + 1) & 1) * SDW, raw[(cc + 1) % PF], chunk + 1);
        fetch(raw[(cc + 1) % PF], chunk + 1 + PF);
        __syncthreads();
      }
    }
  }

  // Lane (j, g) holds, per block, column sp[c].ocol0 + j and rows g + 4v (the
  // FP64 16x16 result interleaves rows across the four lane groups).
  const double alpha = (double)a.alpha * (a.scales ? (double)a.scales[b] : 1.0);
  const double beta = (double)a.beta;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int col = sp[c].ocol0 + j16;
    if (j16 < sp[c].n_out) {
#pragma unroll
      for (int r2 = 0; r2 < 2; ++r2) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ant = a0 + 16 * r2 + g + 4 * v;
          if (ant < a.R) {
            const size_t o = ((size_t)(b * a.R + ant) * a.ld_out + col) * 2;
            double re = alpha * acc[r2][0][c][v];
            double im = alpha * acc[r2][1][c][v];
            if (beta != 0.0) {
              const f2a8 old = *(const f2a8 *)(a.cin + o);
              re += beta * (double)old.x;
              im += beta * (double)old.y;
            }
            __builtin_nontemporal_store(f2a8{(float)re, (float)im}, (f2a8 *)(a.out + o));
          }
        }
      }
    }
  }
}

hipError_t launch_f64mm(const TgArgs &a, hipStream_t s) {
  constexpr int NB = 4;
  const int tiles_r = (a.R + kRows - 1) / kRows;
  const int cols_per_tile = kWaves * 16 * NB;
  const int tiles_c =
      (virtual_cols(a.c_len, a.seg_len, a.seg_lag, 16) + cols_per_tile - 1) / cols_per_tile;
  const long nt = (long)a.batch * tiles_r * tiles_c;
  if (nt <= 0 || nt > 0x7FFFFFFFL) return hipErrorInvalidValue;
  const int nbw_pad = (a.nbw + 3) & ~3;
  const size_t lds = (size_t)(nbw_pad + 2 * stage_dwords<MODE_F32>()) * 4;
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void *)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)nt), dim3(kThreads), lds, s, a, tiles_r, tiles_c,
                       nbw_pad);
    return hipGetLastError();
  };
  return a.rseg_lag ? go(tg_f64mm_kernel<NB, true>) : go(tg_f64mm_kernel<NB, false>);
}

// ---------------------------------------------------------------------------
// FP8 (OCP e4m3fn) correlator on quantised planes, v_mfma_f32_32x32x64_f8f6f4.
// Same tiling as tg_kernel; four 64-code k-steps per LDS stage (32 rows x
// 2 planes x 256 codes), two stages in flight in registers. Lane (m, h) supplies codes n0 + 32h .. +31 of row m
// and the matching 32 sequence bits; +-1 in e4m3 is 0x38 / 0xB8. The B
// fragment of lag block c at k-step i is the 32-bit window at bit
// p_base + 32(2i - c), so two new windows per k-step serve all blocks.
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8;

// 32 bits -> 32 e4m3 codes of +-1 (bit i -> byte i; 1 -> sign set).
__device__ __forceinline__ i32x8 expand_e4m3(uint32_t x) {
  i32x8 r;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t n4 = (x >> (4 * j)) & 0xFu;
    // copies of the nibble at bits 7, 14, 21, 28 put nibble bit j at 8j + 7
    r[j] = (int)(0x38383838u | ((n4 * 0x10204080u) & 0x80808080u));
  }
  return r;
}

// AL: rows are 16-code aligned and t_len is a multiple of 16, so every
// 16-code piece is read by one unconditional buffer load (zeros past the
// frame) and only the last chunk is masked; otherwise codes are read one by
// one.

template <int NC, bool AL>
__global__ __launch_bounds__(kThreads, 2) void tg_fp8_kernel(TgArgs a, int tiles_r, int tiles_c,
                                                             int nbw_pad) {
  extern __shared__ __attribute__((aligned(16))) uint32_t smem[];
  constexpr int NW = 2 * NC;       // window slots (32-sample granularity)
  constexpr int CH = kFp8Chunk;    // codes per stage
  constexpr int KS = CH / 64;      // k-steps of 64 codes per stage
  constexpr int RS = kFp8RowDw;    // dwords per plane row: CH codes + pad
  constexpr int PS = kRows * RS;
  constexpr int SDW = 2 * PS;
  constexpr int NPC = CH / 64;     // 16-code pieces per thread and stage
  constexpr int PF = 2;            // stages in flight (register sets)
  // chunks per unrolled body: covers the register-set rotation (PF) and the
  // window rotation (NW slots, 2 per k-step)
  constexpr int CPB = (NW > 2 * KS * PF) ? NW / (2 * KS) : PF;
  static_assert(CPB % PF == 0 && (2 * KS * CPB) % NW == 0, "body must cover both rotations");

  uint32_t *sbits = smem;
  uint32_t *stage = smem + nbw_pad;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m = lane & 31;
  const int h = lane >> 5;

  const int nt = a.batch * tiles_r * tiles_c;
  const int bid = blockIdx.x;
  const int t = (nt % 8 == 0) ? (bid % 8) * (nt / 8) + bid / 8 : bid;
  const int cg = t % tiles_c;
  const int rest = t / tiles_c;
  const int rb = rest % tiles_r;
  const int b = rest / tiles_r;
  const int a0 = rb * kRows;
  // this wave's columns (see run_tile)
  const SegPos sp = seg_pos(cg * (kWaves * 32 * NC) + wave * 32 * NC,
                            seg_pad(a.seg_len, a.seg_lag, 32 * NC), a.seg_len, a.seg_lag,
                            a.c_len);

  const int nchunks = (a.t_len + CH - 1) / CH;
  const int last = nchunks - 1;
  const uint8_t *fin = (const uint8_t *)a.in + (size_t)b * a.R * 2 * a.ld_in;
  // piece q = t + 256 i of a stage: 16 codes of row q / (CH/8), plane
  // (q / (CH/16)) & 1, codes 16 (q % (CH/16)) .. +15
  int prow[NPC], pplane[NPC], ppart[NPC];
  uint32_t voff[NPC];
#pragma unroll
  for (int i = 0; i < NPC; ++i) {
    const int q = tid + kThreads * i;
    prow[i] = q / (CH / 8);
    pplane[i] = (q / (CH / 16)) & 1;
    ppart[i] = q % (CH / 16);
    voff[i] = (uint32_t)((a0 + prow[i]) * 2 + pplane[i]) * (uint32_t)a.ld_in + 16u * ppart[i];
  }
  const __amdgpu_buffer_rsrc_t rsrc =
      frame_rsrc(fin, (long long)(2 * a.R - 1) * a.ld_in + a.t_len);
  using Raw = u32x4[NPC];
  // codes one by one (rows not 16-code aligned or t_len not a multiple of 16)
  auto load_codes = [&](Raw &r, int chunk) {
#pragma unroll
    for (int i = 0; i < NPC; ++i) {
      const int n = chunk * CH + 16 * ppart[i];
      const int arow = a0 + prow[i];
      u32x4 x = {0u, 0u, 0u, 0u};
      if (arow < a.R) {
        const uint8_t *p = fin + ((size_t)arow * 2 + pplane[i]) * a.ld_in + n;
        uint32_t e[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) e[j] = (n + j < a.t_len) ? p[j] : 0u;
#pragma unroll
        for (int w = 0; w < 4; ++w)
          x[w] = e[4 * w] | (e[4 * w + 1] << 8) | (e[4 * w + 2] << 16) | (e[4 * w + 3] << 24);
      }
      r[i] = x;
    }
  };
  auto store_chunk = [&](uint32_t *st, const Raw &r) {
#pragma unroll
    for (int i = 0; i < NPC; ++i)
      *(u32x4 *)(st + pplane[i] * PS + prow[i] * RS + 4 * ppart[i]) = r[i];
  };
  // chunk -> registers (past the end: the last chunk again)
  auto fetch = [&](Raw &r, int chunk) {
    const int c = chunk < last ? chunk : last;
    if constexpr (AL) {
#pragma unroll
      for (int i = 0; i < NPC; ++i)
        r[i] = __builtin_bit_cast(
            u32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[i] + (uint32_t)(c * CH), 0, 0));
    } else {
      load_codes(r, c);
    }
  };
  // registers holding `chunk` -> stage; pieces past t_len (the next plane's
  // codes) are zeroed in the last chunk
  auto land = [&](uint32_t *st, Raw &r, int chunk) {
    if constexpr (AL) {
      if (chunk == last) {
#pragma unroll
        for (int i = 0; i < NPC; ++i)
          if (chunk * CH + 16 * ppart[i] >= a.t_len) r[i] = u32x4{0u, 0u, 0u, 0u};
      }
    }
    store_chunk(st, r);
  };

  Raw raw[PF];
#pragma unroll
  for (int j = 0; j < PF; ++j) fetch(raw[j], j);
  for (int i = tid; i < a.nbw; i += kThreads) sbits[i] = a.bits[i];
  land(stage, raw[0], 0);
  fetch(raw[0], PF);
  __syncthreads();

  const int p_base = pos_mod(32 * h - m - sp.lag0 + a.poff, a.N);
  i32x8 win[NW];
  // windows W(j), j = -(NC-1) .. -1, for blocks c >= 1 of the first k-steps
#pragma unroll
  for (int j = 1; j <= NC - 1; ++j)
    win[NW - j] = expand_e4m3(window32(sbits, pos_mod(p_base - 32 * j, a.N)));

  f32x16 acc_re[NC], acc_im[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      acc_re[c][v] = 0.f;
      acc_im[c][v] = 0.f;
    }
  }

  // matrix-core work of chunk `chunk` (k-steps KS*chunk .. +KS-1) from stage
  // (chunk & 1); cc = chunk mod CPB fixes the window slots
  auto compute = [&](auto icc, int chunk) {
    constexpr int cc = decltype(icc)::value;
    const uint32_t *st = stage + (chunk & 1) * SDW;
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int i = KS * chunk + u;         // k-step
      const int q = (2 * (KS * cc + u)) % NW;  // slot of W(2i)
      win[q] = expand_e4m3(window32(sbits, p_base + 64 * i));
      win[(q + 1) % NW] = expand_e4m3(window32(sbits, p_base + 64 * i + 32));
      const u32x4 r0 = *(const u32x4 *)(st + m * RS + 16 * u + 8 * h);
      const u32x4 r1 = *(const u32x4 *)(st + m * RS + 16 * u + 8 * h + 4);
      const u32x4 i0 = *(const u32x4 *)(st + PS + m * RS + 16 * u + 8 * h);
      const u32x4 i1 = *(const u32x4 *)(st + PS + m * RS + 16 * u + 8 * h + 4);
      const i32x8 are = {(int)r0.x, (int)r0.y, (int)r0.z, (int)r0.w,
                         (int)r1.x, (int)r1.y, (int)r1.z, (int)r1.w};
      const i32x8 aim = {(int)i0.x, (int)i0.y, (int)i0.z, (int)i0.w,
                         (int)i1.x, (int)i1.y, (int)i1.z, (int)i1.w};
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const i32x8 bw = win[(q - c + NW) % NW];
        acc_re[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(are, bw, acc_re[c], 0, 0,
                                                                    0, 0, 0, 0);
        acc_im[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(aim, bw, acc_im[c], 0, 0,
                                                                    0, 0, 0, 0);
      }
    }
  };
  // Steady state without branches (exact waits), then 2 .. CPB + 1 chunks
  // with their checks; same scheme as the 16-bit kernel.
  const int nmain = last >= 1 ? (last - 1) / CPB : 0;
  for (int body = 0; body < nmain; ++body) {
    static_for<0, CPB>([&](auto icc) {
      constexpr int cc = decltype(icc)::value;
      const int i = body * CPB + cc;
      compute(icc, i);
      store_chunk(stage + ((i + 1) & 1) * SDW, raw[(cc + 1) % PF]);
      fetch(raw[(cc + 1) % PF], i + 1 + PF);
      __syncthreads();
      __builtin_amdgcn_sched_barrier(0);
    });
  }
  static_for<0, CPB + 1>([&](auto icc) {
    constexpr int cc = decltype(icc)::value;
    const int i = nmain * CPB + cc;
    if (i < nchunks) {
      compute(std::integral_constant<int, cc % CPB>{}, i);
      if (i + 1 < nchunks) land(stage + ((i + 1) & 1) * SDW, raw[(cc + 1) % PF], i + 1);
      if (i + 1 + PF < nchunks) fetch(raw[(cc + 1) % PF], i + 1 + PF);
      __syncthreads();
    }
  });

  const float alpha = a.alpha * (a.scales ? a.scales[b] : 1.0f);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = sp.ocol0 + 32 * c + m;
    if (32 * c + m < sp.n_out) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int ant = a0 + 8 * (v >> 2) + 4 * h + (v & 3);
        if (ant < a.R) {
          const size_t o = ((size_t)(b * a.R + ant) * a.ld_out + col) * 2;
          float re = alpha * acc_re[c][v];
          float im = alpha * acc_im[c][v];
          if (a.beta != 0.0f) {
            const f2a8 old = *(const f2a8 *)(a.cin + o);
            re += a.beta * old.x;
            im += a.beta * old.y;
          }
          __builtin_nontemporal_store(f2a8{re, im}, (f2a8 *)(a.out + o));
        }
      }
    }
  }
}

template <int NC, bool AL>
static hipError_t launch_fp8_nc_al(const TgArgs &a, hipStream_t s) {
  const int tiles_r = (a.R + kRows - 1) / kRows;
  const int cols_per_tile = kWaves * 32 * NC;
  const int tiles_c =
      (virtual_cols(a.c_len, a.seg_len, a.seg_lag, 32 * NC) + cols_per_tile - 1) / cols_per_tile;
  const long nt = (long)a.batch * tiles_r * tiles_c;
  if (nt <= 0 || nt > 0x7FFFFFFFL) return hipErrorInvalidValue;
  const int nbw_pad = (a.nbw + 3) & ~3;
  const size_t lds = (size_t)(nbw_pad + 2 * 2 * kRows * kFp8RowDw) * 4;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)tg_fp8_kernel<NC, AL>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((tg_fp8_kernel<NC, AL>), dim3((unsigned)nt), dim3(kThreads), lds, s, a,
                     tiles_r, tiles_c, nbw_pad);
  return hipGetLastError();
}

template <int NC>
static hipError_t launch_fp8_nc(const TgArgs &a, hipStream_t s) {
  if ((a.ld_in & 15) == 0 && (a.t_len & 15) == 0) return launch_fp8_nc_al<NC, true>(a, s);
  return launch_fp8_nc_al<NC, false>(a, s);
}

template <int MODE, int IN, int NC, bool AL, bool SB>
static hipError_t launch_tg_nc_al_sb(const TgArgs &a, hipStream_t s) {
  const int tiles_r = (a.R + kRows - 1) / kRows;
  const int cols_per_tile = kWaves * 32 * NC;
  const int tiles_c =
      (virtual_cols(a.c_len, a.seg_len, a.seg_lag, SB ? 32 : 32 * NC) + cols_per_tile - 1) /
      cols_per_tile;
  const long nt = (long)a.batch * tiles_r * tiles_c;
  if (nt <= 0 || nt > 0x7FFFFFFFL) return hipErrorInvalidValue;
  const int nbw_pad = (a.nbw + 3) & ~3;
  const size_t lds = (size_t)tile_lds_dwords<MODE, IN>(nbw_pad) * 4;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)tg_kernel<MODE, IN, NC, AL, SB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (a.ls && tiles_c > 1) {
    // the rows' lags span several workgroups: plain correlation, then the
    // least-squares correction as a second launch
    TgArgs b = a;
    b.ls = 0;
    hipLaunchKernelGGL((tg_kernel<MODE, IN, NC, AL, SB>), dim3((unsigned)nt), dim3(kThreads), lds,
                       s, b, tiles_r, tiles_c, nbw_pad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_debias(a.out, (long)a.batch * a.R, a.c_len, a.N, s);
  }
  hipLaunchKernelGGL((tg_kernel<MODE, IN, NC, AL, SB>), dim3((unsigned)nt), dim3(kThreads), lds, s,
                     a, tiles_r, tiles_c, nbw_pad);
  return hipGetLastError();
}

// Column segments (Eq. 8 lags) take the per-block variant; rows of lag
// blocks (the adjoint's input) never have column segments.
template <int MODE, int IN, int NC, bool AL>
static hipError_t launch_tg_nc_al(const TgArgs &a, hipStream_t s) {
  if constexpr (IN == IN_C64_LAGS) {
    if (a.seg_lag) return hipErrorInvalidValue;
    return launch_tg_nc_al_sb<MODE, IN, NC, AL, false>(a, s);
  } else {
    if (a.seg_lag) return launch_tg_nc_al_sb<MODE, IN, NC, AL, true>(a, s);
    return launch_tg_nc_al_sb<MODE, IN, NC, AL, false>(a, s);
  }
}

// Packed rows take the branch-free loader when rows are 8-code aligned and
// the reduction length is a multiple of 8; complex64 rows always do.
template <int MODE, int IN, int NC>
static hipError_t launch_tg_nc(const TgArgs &a, hipStream_t s) {
  if constexpr (IN == IN_C64 || IN == IN_C64_LAGS) {
    return launch_tg_nc_al<MODE, IN, NC, true>(a, s);
  } else {
    if ((a.ld_in & 7) == 0 && (a.t_len & 7) == 0) return launch_tg_nc_al<MODE, IN, NC, true>(a, s);
    return launch_tg_nc_al<MODE, IN, NC, false>(a, s);
  }
}

// Column width per wave: the widest that the output needs (fewest re-reads
// of the input), narrowed while the launch has fewer tiles than the chip has
// compute units, so small batches (one frame) spread over more of them.
// Column segments are padded to `gran(nc)` columns: 32 for the tiled kernel
// (a segment per 32-column block), 32*nc for the e4m3 kernel (a segment per
// wave), which is then kept no wider than a segment (rounded up to 32) needs.
static int pick_nc(const TgArgs &a, bool per_block) {
  auto gran = [&](int n) { return per_block ? 32 : 32 * n; };
  const int width = virtual_cols(a.c_len, a.seg_len, a.seg_lag, 32);
  int nc = width > 256 ? 4 : (width > 128 ? 2 : 1);
  if (a.seg_lag && !per_block)
    while (nc > 1 && seg_pad(a.seg_len, 1, 32 * nc) != seg_pad(a.seg_len, 1, 32)) nc /= 2;
  const long rows = (long)a.batch * ((a.R + kRows - 1) / kRows);
  auto tiles = [&](int n) {
    const int w = kWaves * 32 * n;
    return rows * ((virtual_cols(a.c_len, a.seg_len, a.seg_lag, gran(n)) + w - 1) / w);
  };
  while (nc > 1 && tiles(nc) < 256) nc /= 2;
  return nc;
}

template <int MODE, int IN>
static hipError_t launch_tg_mode(const TgArgs &a, hipStream_t s) {
  const int nc = pick_nc(a, true);
  if (nc == 4) return launch_tg_nc<MODE, IN, 4>(a, s);
  if (nc == 2) return launch_tg_nc<MODE, IN, 2>(a, s);
  return launch_tg_nc<MODE, IN, 1>(a, s);
}

hipError_t launch_tg_frame(int in_fmt, int nc, const TgArgs &a, hipStream_t s) {
  if (in_fmt == IN_BF16) {
    if (nc == 4) return launch_tg_nc<MODE_BF16, IN_BF16, 4>(a, s);
    if (nc == 2) return launch_tg_nc<MODE_BF16, IN_BF16, 2>(a, s);
    return launch_tg_nc<MODE_BF16, IN_BF16, 1>(a, s);
  }
  if (in_fmt == IN_F16) {
    if (nc == 4) return launch_tg_nc<MODE_BF16, IN_F16, 4>(a, s);
    if (nc == 2) return launch_tg_nc<MODE_BF16, IN_F16, 2>(a, s);
    return launch_tg_nc<MODE_BF16, IN_F16, 1>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tg(int mode, int in_fmt, const TgArgs &a, hipStream_t s) {
  if (in_fmt == IN_C64) {
    switch (mode) {
      case MODE_F32: return launch_tg_mode<MODE_F32, IN_C64>(a, s);
      case MODE_F32S: return launch_tg_mode<MODE_F32S, IN_C64>(a, s);
      case MODE_BF16: return launch_tg_mode<MODE_BF16, IN_C64>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (in_fmt == IN_C64_LAGS) {
    switch (mode) {
      case MODE_F32: return launch_tg_mode<MODE_F32, IN_C64_LAGS>(a, s);
      case MODE_F32S: return launch_tg_mode<MODE_F32S, IN_C64_LAGS>(a, s);
      case MODE_BF16: return launch_tg_mode<MODE_BF16, IN_C64_LAGS>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (in_fmt == IN_BF16) return launch_tg_mode<MODE_BF16, IN_BF16>(a, s);
  if (in_fmt == IN_F16) return launch_tg_mode<MODE_BF16, IN_F16>(a, s);
  if (in_fmt == IN_E4M3) {
    const int nc = pick_nc(a, false);
    if (nc == 4) return launch_fp8_nc<4>(a, s);
    if (nc == 2) return launch_fp8_nc<2>(a, s);
    return launch_fp8_nc<1>(a, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// FP64-accumulating vector kernel: one thread per output element, the sum
// over t in natural order. Used for the FP64 path (c128 in and out) and for
// the final residual of refinement (c64 in and out, FP64 sums).
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void tg64_kernel(Tg64Args a, int cblocks) {
  const long blk = blockIdx.x;
  const long row = blk / cblocks;  // frame * R + antenna
  const int col = (int)(blk - row * cblocks) * 256 + threadIdx.x;
  if (col >= a.c_len) return;
  const int b = (int)(row / a.R);
  const TI *x = (const TI *)a.in + (size_t)row * a.ld_in * 2;
  const int lag = a.seg_lag ? col / a.seg_len * a.seg_lag + col % a.seg_len : col;
  int p = (int)(((long)a.poff - lag % a.N + a.N) % a.N);  // (poff - lag) mod N
  // with reduction blocks, the position jumps by rseg_lag - rseg_len after
  // every block of rseg_len terms
  const int blk_len = a.rseg_lag ? a.rseg_len : a.t_len;
  const int jump = a.rseg_lag ? (a.rseg_lag - a.rseg_len) % a.N : 0;
  int in_blk = 0;
  double re = 0.0, im = 0.0;
  for (int t = 0; t < a.t_len; ++t) {
    const bool neg = (a.bits[p >> 5] >> (p & 31)) & 1u;
    const double xr = (double)x[2 * t], xi = (double)x[2 * t + 1];
    re += neg ? -xr : xr;
    im += neg ? -xi : xi;
    if (++p == a.N) p = 0;
    if (++in_blk == blk_len) {
      in_blk = 0;
      p += jump;
      if (p >= a.N) p -= a.N;
    }
  }
  const double alpha = a.alpha * (a.scales ? (double)a.scales[b] : 1.0);
  re *= alpha;
  im *= alpha;
  const size_t o = ((size_t)row * a.ld_out + col) * 2;
  if (a.beta != 0.0) {
    const TO *c = (const TO *)a.cin;
    re += a.beta * (double)c[o];
    im += a.beta * (double)c[o + 1];
  }
  TO *out = (TO *)a.out;
  out[o] = (TO)re;
  out[o + 1] = (TO)im;
}

hipError_t launch_tg64(const Tg64Args &a, hipStream_t s) {
  const long rows = (long)a.batch * a.R;
  const int cblocks = (a.c_len + 255) / 256;
  const long nblk = rows * cblocks;
  if (nblk <= 0 || nblk > 0x7FFFFFFFL) return hipErrorInvalidValue;
  if (a.in_f64 && a.out_f64)
    hipLaunchKernelGGL((tg64_kernel<double, double>), dim3((unsigned)nblk), dim3(256), 0, s, a,
                       cblocks);
  else if (!a.in_f64 && !a.out_f64)
    hipLaunchKernelGGL((tg64_kernel<float, float>), dim3((unsigned)nblk), dim3(256), 0, s, a,
                       cblocks);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Least-squares correction of correlator rows: one wave per row, FP64 row sum,
// then every element out = c1 * (H + c2 * sum) with c1 = N/(N+1),
// c2 = 1/(N+1-K). The row is read twice (the second time from cache).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void debias_kernel(float *H, long rows, int K, float c1,
                                                     float c2) {
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int lane = threadIdx.x & 63;
  f2a8 *h = (f2a8 *)H + (size_t)row * K;
  double sr = 0.0, si = 0.0;
  for (int k = lane; k < K; k += 64) {
    const f2a8 v = h[k];
    sr += (double)v.x;
    si += (double)v.y;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o);
    si += __shfl_xor(si, o);
  }
  const float ar = (float)(c2 * sr), ai = (float)(c2 * si);
  for (int k = lane; k < K; k += 64) {
    const f2a8 v = h[k];
    h[k] = f2a8{c1 * (v.x + ar), c1 * (v.y + ai)};
  }
}

hipError_t launch_debias(float *H, long rows, int K, int N, hipStream_t s) {
  if (rows <= 0 || K <= 0 || K > N) return hipErrorInvalidValue;
  const long blocks = (rows + 3) / 4;
  if (blocks > 0x7FFFFFFFL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(debias_kernel, dim3((unsigned)blocks), dim3(256), 0, s, H, rows, K,
                     (float)N / (float)(N + 1), 1.0f / (float)(N + 1 - K));
  return hipGetLastError();
}

}  // namespace pnce
