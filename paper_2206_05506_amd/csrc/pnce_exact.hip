// pnce_exact.hip -- the Toeplitz +-1 contraction of Eq. 3 / Eq. 10 (and its
// adjoint) with exact sums, on int8 matrix cores (v_mfma_i32_32x32x32_i8).
//
//   out[r][c] = alpha * sum_t in[r][t] * s'[(t - c) mod N] + beta * cin[r][c]
//
// Every FP32 input row is written in fixed point relative to the row's
// largest magnitude and cut into DG balanced 8-bit digits (the splitting of
// the Ozaki scheme for error-free matrix products, here one-sided: the other
// operand is +-1 and exact in int8):
//   DG = 8: X = rint(x * 2^(62 - e)), |X| < 2^62 (PNCE_PREC_EXACT);
//   DG = 4: X = rint(x * 2^(30 - e)), |X| < 2^30 (PNCE_PREC_EXACT32),
// with 2^e the power of two just above the row's largest |re| or |im|. Each
// digit's contraction is summed exactly in int32 (|digit| <= 128, at most
// 65535 terms, so |sum| < 2^23). Eight digits: the digit sums are combined
// in FP64 (two exact partial sums, one rounding when they are added),
// scaled back, alpha and beta applied in FP64, and the output rounded once
// to FP32. Four digits (no FP64 arithmetic): the digit sums are combined
// exactly in int64, rounded once to FP32 and scaled back, and alpha and
// beta are applied in FP32. Row elements within 2^38 (DG = 8) or 2^6
// (DG = 4) of the row's largest magnitude are represented exactly; smaller
// ones are rounded at 2^(e - 63) or 2^(e - 31).
//
// Tile: 32/DG antennas x DG digits = the 32 rows of the matrix-core A
// operand, by NWV waves x 32*NB output columns (8 waves for outputs wider
// than 512 columns whose rows are long enough to give each workgroup at
// least 4 stages, else 4). A workgroup takes one block of antennas of one
// frame and a share of its column groups (all of them unless the launch
// would be too small to fill the chip). It first finds each row's exponent
// (the first stages' loads already in flight), then streams the rows through
// LDS in stages of 64*NWV samples, one pipeline across its column groups
// (they all read the same rows): each stage is converted into digits between
// the k-steps of the stage before (two stages in flight in registers, one
// barrier per stage). The +-1 operand is expanded from the sequence bit
// stream in LDS through a nibble table; without column segments, block c's
// fragment at k-step i is block 0's at k-step i - c (a block of 32 columns
// is one k-step of 32 terms), so a wave expands one fragment per k-step and
// rotates 2*NB of them.
#include <algorithm>
#include <type_traits>

#include "pnce_device.h"

namespace pnce {

namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

// The digit word of one value: DG bytes.
template <int DG> struct DigitWord { using T = uint64_t; };
template <> struct DigitWord<4> { using T = uint32_t; };

// x (FP32) in fixed point: X = rint(x * 2^k), k = scale - E for a row whose
// largest |re| or |im| has biased exponent field E (E >= 1; scale = 188 for
// DG = 8, 156 for DG = 4), so |X| < 2^(8 DG - 2). x * 2^k is exact (a power
// of two times x; FP32 subnormals are kept) unless it falls below 2^-126,
// where X is 0 either way; exact too are the rounding to an integer (to
// nearest, ties to even), the split of an eight-digit X into
// 32-bit halves (hi = floor(X / 2^32), lo = X - hi 2^32 in [0, 2^32), both
// exact in FP32) and the conversions. The clamp only acts on rows holding
// inf or NaN, whose outputs are NaN anyway. Returned as (X + bias) ^ bias,
// bias = 0x80 in every byte: its bytes, read as signed, are balanced
// base-256 digits of X (X = sum_j digit_j * 256^j, each in [-128, 127]),
// since every byte of X + bias lies in [0, 255] and byte - 128 == byte ^
// 0x80 as a signed byte.
template <int DG>
__device__ __forceinline__ typename DigitWord<DG>::T fixed_digits(float x, int k) {
  constexpr float kLim = DG == 8 ? 0x1p62f : 0x1p30f;
  float f = __builtin_rintf(__builtin_amdgcn_ldexpf(x, k));
  f = __builtin_fminf(__builtin_fmaxf(f, -kLim), kLim);
  if constexpr (DG == 8) {
    const float hi = __builtin_floorf(f * 0x1p-32f);
    const float lo = __builtin_fmaf(hi, -0x1p32f, f);
    const uint64_t X = ((uint64_t)(uint32_t)(int32_t)hi << 32) | (uint64_t)(uint32_t)lo;
    return (X + 0x8080808080808080ull) ^ 0x8080808080808080ull;
  } else {
    const uint32_t X = (uint32_t)(int32_t)f;
    return (X + 0x80808080u) ^ 0x80808080u;
  }
}

// 4x4 byte transpose: out[j] byte s = byte j of in[s].
__device__ __forceinline__ void transpose4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                           uint32_t (&t)[4]) {
  // v_perm_b32(S0, S1, sel): selector bytes 0-3 pick S1's bytes, 4-7 S0's
  const uint32_t ab01 = __builtin_amdgcn_perm(b, a, 0x05010400u);  // a0 b0 a1 b1
  const uint32_t ab23 = __builtin_amdgcn_perm(b, a, 0x07030602u);  // a2 b2 a3 b3
  const uint32_t cd01 = __builtin_amdgcn_perm(d, c, 0x05010400u);  // c0 d0 c1 d1
  const uint32_t cd23 = __builtin_amdgcn_perm(d, c, 0x07030602u);  // c2 d2 c3 d3
  t[0] = __builtin_amdgcn_perm(cd01, ab01, 0x05040100u);  // a0 b0 c0 d0
  t[1] = __builtin_amdgcn_perm(cd01, ab01, 0x07060302u);  // a1 b1 c1 d1
  t[2] = __builtin_amdgcn_perm(cd23, ab23, 0x05040100u);  // a2 b2 c2 d2
  t[3] = __builtin_amdgcn_perm(cd23, ab23, 0x07060302u);  // a3 b3 c3 d3
}

// Digit rows of one thread's samples (SPT = 32 / DG of them): row d
// (d < DG) receives byte d of every sample's word, sample s in byte s.
// DG = 8: 4 samples, one dword per row; DG = 4: 8 samples, two dwords.
template <int DG, int ROW>
__device__ __forceinline__ void store_digits(uint8_t *row0,
                                             const typename DigitWord<DG>::T (&w)[32 / DG]) {
  if constexpr (DG == 8) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      uint32_t t[4];
      transpose4((uint32_t)(w[0] >> (32 * half)), (uint32_t)(w[1] >> (32 * half)),
                 (uint32_t)(w[2] >> (32 * half)), (uint32_t)(w[3] >> (32 * half)), t);
#pragma unroll
      for (int j = 0; j < 4; ++j) *(uint32_t *)(row0 + (4 * half + j) * ROW) = t[j];
    }
  } else {
    uint32_t lo[4], hi[4];
    transpose4(w[0], w[1], w[2], w[3], lo);
    transpose4(w[4], w[5], w[6], w[7], hi);
#pragma unroll
    for (int j = 0; j < 4; ++j) *(uint2 *)(row0 + j * ROW) = uint2{lo[j], hi[j]};
  }
}

// +-1 fragments: 16 sequence bits -> 16 int8 values (bit 1 -> -1 = 0xFF,
// bit 0 -> +1 = 0x01), bit e in byte e, read nibble by nibble from a
// 16-entry table at the start of LDS (16 consecutive dwords: lanes reading
// different entries hit different banks).
__device__ __forceinline__ uint32_t nibble_bytes(uint32_t nib) {
  uint32_t r = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) r |= (((nib >> e) & 1u) ? 0xFFu : 0x01u) << (8 * e);
  return r;
}

__device__ __forceinline__ i32x4 frag_at(const uint32_t *sbits, const uint32_t *lut, int p) {
  const uint32_t w = window32(sbits, p);
  return i32x4{(int)lut[w & 0xFu], (int)lut[(w >> 4) & 0xFu], (int)lut[(w >> 8) & 0xFu],
               (int)lut[(w >> 12) & 0xFu]};
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// One thread's share of a stage: SPT consecutive samples of one antenna, as
// complex pairs.
template <int SPT> struct RawEx {
  f32x4 v[SPT / 2];
};

// Geometry: NWV waves per workgroup (4, or 8 for wide outputs with long
// rows, so that each converted stage feeds twice the matrix work), ANT =
// 32/DG antennas per tile, TPA threads per antenna, each converting SPT =
// 32/DG samples of every stage of CH = 64 NWV samples (KS = CH/32 k-steps
// per barrier). Thread t loads and converts antenna t / TPA, samples
// SPT (t % TPA) .. + SPT - 1 of each stage.
template <int NWV, int DG> struct ExGeom {
  static constexpr int threads = 64 * NWV;
  static constexpr int ant = 32 / DG;
  static constexpr int tpa = threads / ant;
  static constexpr int spt = 32 / DG;
  static constexpr int ch = spt * tpa;
  static constexpr int ks = ch / 32;
  static constexpr int row = ch + 16;  // bytes per digit row in LDS (16 B pad)
  static constexpr int plane = 32 * row;
  static constexpr int stage = 2 * plane;  // re and im planes
  static constexpr int lpg = tpa < 64 ? tpa : 64;  // lanes of one maximum reduction
  static constexpr int gpa = tpa / lpg;            // reductions per antenna
  static constexpr int fin = 16 / DG;  // antennas each lane finishes per column
  static constexpr int scale = 150 + (DG == 8 ? 38 : 6);  // X = rint(x * 2^(scale - E))
};
constexpr int kLutDw = 16;  // LDS: nibble table, sequence bits, row maxima, stages
constexpr int kMaxDw = 16;

template <int DG, int NB, int NWV, bool SB, bool GA>
__global__ __launch_bounds__(64 * NWV, 8 / NWV) void exact_kernel(ExArgs a, int rblocks,
                                                                  int splits, int ngroups,
                                                                  int nbw_pad) {
  using G = ExGeom<NWV, DG>;
  using W = typename DigitWord<DG>::T;
  extern __shared__ __attribute__((aligned(16))) uint32_t smem[];
  constexpr int NW = 2 * NB;  // fragment slots (NW divides the KS k-steps of a stage)
  static_assert(G::ks % NW == 0, "slots must repeat within a stage");
  static_assert(G::ch == 64 * NWV, "one stage size for both digit counts");
  uint32_t *lut = smem;
  uint32_t *sbits = smem + kLutDw;
  uint32_t *mx_tab = smem + kLutDw + nbw_pad;
  uint8_t *stage = (uint8_t *)(smem + kLutDw + nbw_pad + kMaxDw);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m = lane & 31;
  const int kh = lane >> 5;
  const int my_ant = tid / G::tpa;  // the antenna this thread loads and converts
  const int my_idx = tid % G::tpa;
  const int split = blockIdx.x % splits;
  const int rest = blockIdx.x / splits;
  const int rb = rest % rblocks;
  const int b = rest / rblocks;
  const int a0 = rb * G::ant;
  const float *fin = a.in + (size_t)b * a.R * a.ld_in * 2;
  const int row_terms = GA ? a.rseg_n * a.rseg_len : a.t_len;

  const __amdgpu_buffer_rsrc_t rsrc =
      frame_rsrc(fin, ((long long)(a.R - 1) * a.ld_in + row_terms) * 8);
  const uint32_t rowoff = (uint32_t)(a0 + my_ant) * (uint32_t)a.ld_in * 8u;
  const int nchunks = (a.t_len + G::ch - 1) / G::ch;
  const int last = nchunks - 1;
  const int my_n = G::spt * my_idx;  // this thread's first sample in a stage

  // chunk -> registers (past the end: the last chunk again). Pairs cut by
  // the end of the row are read one sample early so that no 16-byte load
  // straddles the end of the frame (t_len >= 2); the conversion shifts them
  // back.
  auto fetch = [&](RawEx<G::spt> &r, int chunk) {
    const int n = (chunk < last ? chunk : last) * G::ch + my_n;
    if constexpr (GA) {
      // rows of lag blocks: position u holds term j*len + l when
      // u = j*step + l, l < len, j < n; other positions read past any frame
      f32x2 x[G::spt];
#pragma unroll
      for (int e = 0; e < G::spt; ++e) {
        const int u = n + e;
        const int j = u / a.rseg_lag;
        const int l = u - j * a.rseg_lag;
        const uint32_t off = (rowoff + 8u * (uint32_t)(j * a.rseg_len + l)) |
                             ((j < a.rseg_n && l < a.rseg_len) ? 0u : 0x80000000u);
        x[e] = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(rsrc, off, 0, 0));
      }
#pragma unroll
      for (int p = 0; p < G::spt / 2; ++p)
        r.v[p] = f32x4{x[2 * p].x, x[2 * p].y, x[2 * p + 1].x, x[2 * p + 1].y};
    } else {
#pragma unroll
      for (int p = 0; p < G::spt / 2; ++p) {
        const int np = n + 2 * p;
        const uint32_t off = rowoff + 8u * (uint32_t)np - (np + 1 == a.t_len ? 8u : 0u);
        r.v[p] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0));
      }
    }
  };
  // The first two stages' loads go out before the rows' exponents are
  // found (they do not depend on them), so their latency overlaps the scan.
  RawEx<G::spt> raw[2];
  fetch(raw[0], 0);
  fetch(raw[1], 1 % nchunks);

  // Largest |re| or |im| bits of each row (exponent field 255: a non-finite
  // value; the row's outputs are then NaN): the TPA threads of an antenna
  // scan its row, reduce over groups of LPG lanes, and the group leaders
  // leave their maxima in LDS.
  {
    uint32_t mx = 0u;
    const int ant = a0 + my_ant;
    if (ant < a.R) {
      const uint2 *row = (const uint2 *)(fin + (size_t)ant * a.ld_in * 2);
      constexpr int step = G::tpa;
      int n = my_idx;
      for (; n + 3 * step < row_terms; n += 4 * step) {
        const uint2 v0 = row[n], v1 = row[n + step], v2 = row[n + 2 * step],
                    v3 = row[n + 3 * step];
        mx = max(mx, max(v0.x & 0x7FFFFFFFu, v0.y & 0x7FFFFFFFu));
        mx = max(mx, max(v1.x & 0x7FFFFFFFu, v1.y & 0x7FFFFFFFu));
        mx = max(mx, max(v2.x & 0x7FFFFFFFu, v2.y & 0x7FFFFFFFu));
        mx = max(mx, max(v3.x & 0x7FFFFFFFu, v3.y & 0x7FFFFFFFu));
      }
      for (; n < row_terms; n += step) {
        const uint2 v = row[n];
        mx = max(mx, max(v.x & 0x7FFFFFFFu, v.y & 0x7FFFFFFFu));
      }
    }
#pragma unroll
    for (int off = G::lpg / 2; off >= 1; off >>= 1)
      mx = max(mx, (uint32_t)__shfl_xor((int)mx, off));
    if (tid % G::lpg == 0) mx_tab[tid / G::lpg] = mx;
  }
  if (tid < kLutDw) lut[tid] = nibble_bytes((uint32_t)tid);
  for (int i = tid; i < a.nbw; i += G::threads) sbits[i] = a.bits[i];
  __syncthreads();
  // exponent field E of antenna j of the tile (E >= 1)
  auto e_of = [&](int j) {
    uint32_t mx = mx_tab[j * G::gpa];
#pragma unroll
    for (int q = 1; q < G::gpa; ++q) mx = max(mx, mx_tab[j * G::gpa + q]);
    return max((int)(mx >> 23), 1);
  };
  const int k_own = G::scale - e_of(my_ant);  // X = rint(x 2^k) for the row this thread converts
  // the rows this lane finishes: antennas 2kh + jj (DG = 8), 2jj + kh (DG = 4)
  int e_fin[G::fin];
#pragma unroll
  for (int jj = 0; jj < G::fin; ++jj) e_fin[jj] = e_of(DG == 8 ? 2 * kh + jj : 2 * jj + kh);

  // registers -> digit planes of LDS stage st, in ten pieces so that they
  // can be spread over the k-steps of the previous stage: pieces 0-3
  // convert the real parts of the thread's samples (samples past the row
  // end read as zero), piece 4 stores their digits, pieces 5-8 convert the
  // imaginary parts and piece 9 stores theirs. The samples are read from
  // the fetch registers, which stay untouched until the stage is converted.
  struct Conv {
    W w[G::spt];
  };
  constexpr int PER = G::spt / 4;  // values converted per piece
  auto conv_piece = [&](auto kp, Conv &cv, uint8_t *st, const RawEx<G::spt> &r, int chunk) {
    constexpr int K = decltype(kp)::value;
    uint8_t *row0 = st + (DG * my_ant) * G::row + my_n;
    if constexpr (K < 4 || (K >= 5 && K < 9)) {
      constexpr bool IM = K >= 5;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int s = (IM ? K - 5 : K) * PER + q;  // sample
        const f32x4 x = r.v[s >> 1];
        float val = IM ? ((s & 1) ? x.w : x.y) : ((s & 1) ? x.z : x.x);
        if constexpr (!GA) {
          // samples left in the row from this thread's first one; a pair
          // cut by the row end was read one sample early
          const int rem = a.t_len - (chunk * G::ch + my_n);
          const float early = (s & 1) ? 0.f : (IM ? x.w : x.z);
          val = s >= rem ? 0.f : ((s | 1) == rem ? early : val);
        }
        cv.w[s] = fixed_digits<DG>(val, k_own);
      }
    } else if constexpr (K == 4) {
      store_digits<DG, G::row>(row0, cv.w);
    } else {
      store_digits<DG, G::row>(row0 + G::plane, cv.w);
    }
  };
  auto land = [&](uint8_t *st, const RawEx<G::spt> &r, int chunk) {
    Conv cv;
    static_for<0, 10>([&](auto kp) { conv_piece(kp, cv, st, r, chunk); });
  };

  // The workgroup's column groups g = split, split + splits, ... all stream
  // the same rows, so the stage pipeline runs straight through them: step s
  // is chunk s % nchunks of group s / nchunks, and the next group's first
  // stage is staged while the last stage of the current one is used.
  const int gw = NWV * 32 * NB;
  const int my_groups = (ngroups - split + splits - 1) / splits;
  const int total = my_groups * nchunks;

  SegPos sp{};
  [[maybe_unused]] SegPos sb[SB ? NB : 1];
  [[maybe_unused]] i32x4 win[SB ? 1 : NW];
  [[maybe_unused]] i32x4 wb[SB ? NB : 1][2];
  [[maybe_unused]] int pb[SB ? NB : 1];
  int p_base = 0;
  i32x16 acc_re[NB], acc_im[NB];
  auto ocol = [&](int c) { return SB ? sb[c].ocol0 : sp.ocol0 + 32 * c; };
  auto nout = [&](int c) { return SB ? sb[c].n_out : sp.n_out - 32 * c; };

  // Group k: this wave's 32*NB columns (lags sp.lag0 + j, stored at
  // sp.ocol0 + j for j < sp.n_out; SB: block c's 32 columns from sb[c]
  // likewise), the B fragments of k-steps -(NB-1) .. 0, zero accumulators.
  // B fragment of lane (m, kh) at k-step i: terms t = 32i + 16kh + e
  // (e < 16) against column lag0 + m: bits p_base + 32i + e with
  // p_base = 16kh - m - lag0 + poff (mod N); positions stay below
  // N + t_len + 600 bits, inside the doubled stream.
  auto start_group = [&](int k) {
    const int v0 = (split + k * splits) * gw + wave * 32 * NB;
    sp = seg_pos(v0, seg_pad(a.seg_len, a.seg_lag, SB ? 32 : 32 * NB), a.seg_len, a.seg_lag,
                 a.c_len);
    if constexpr (SB) {
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        sb[c] = seg_pos(v0 + 32 * c, seg_pad(a.seg_len, a.seg_lag, 32), a.seg_len, a.seg_lag,
                        a.c_len);
        pb[c] = pos_mod(16 * kh - m - sb[c].lag0 + a.poff, a.N);
        wb[c][0] = frag_at(sbits, lut, pb[c]);
      }
    } else {
      p_base = pos_mod(16 * kh - m - sp.lag0 + a.poff, a.N);
      win[0] = frag_at(sbits, lut, p_base);
#pragma unroll
      for (int j = 1; j < NB; ++j)
        win[NW - j] = frag_at(sbits, lut, pos_mod(p_base - 32 * j, a.N));
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        acc_re[c][v] = 0;
        acc_im[c][v] = 0;
      }
    }
  };

  // KS k-steps on one stage; the fragments of k-step i + 1 are built
  // during k-step i (their slot held step i + 1 - 2NB, which no block
  // reads at step i), and so are its A operands. The next stage (registers
  // nr, chunk nchunk) is converted into LDS stage nst in pieces between the
  // k-steps: no wave reads nst until the barrier after this stage.
  constexpr int kPieces = 10;
  constexpr int kPerStep = (kPieces + G::ks - 1) / G::ks;
  auto do_chunk = [&](const uint8_t *st, int chunk, uint8_t *nst, const RawEx<G::spt> &nr,
                      int nchunk) {
    Conv cv;
    i32x4 are[2], aim[2];
    are[0] = *(const i32x4 *)(st + m * G::row + 16 * kh);
    aim[0] = *(const i32x4 *)(st + G::plane + m * G::row + 16 * kh);
    static_for<0, G::ks>([&](auto iu) {
      constexpr int u = decltype(iu)::value;
      const int i = G::ks * chunk + u;
      if constexpr (u + 1 < G::ks) {
        are[(u + 1) & 1] = *(const i32x4 *)(st + m * G::row + 32 * (u + 1) + 16 * kh);
        aim[(u + 1) & 1] = *(const i32x4 *)(st + G::plane + m * G::row + 32 * (u + 1) + 16 * kh);
      }
      if constexpr (SB) {
#pragma unroll
        for (int c = 0; c < NB; ++c)
          wb[c][(u + 1) & 1] = frag_at(sbits, lut, pb[c] + 32 * (i + 1));
      } else {
        win[(u + 1) % NW] = frag_at(sbits, lut, p_base + 32 * (i + 1));
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const i32x4 bw = SB ? wb[c][u & 1] : win[(u - c + NW) % NW];
        acc_re[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(are[u & 1], bw, acc_re[c], 0, 0, 0);
        acc_im[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(aim[u & 1], bw, acc_im[c], 0, 0, 0);
      }
      static_for<u * kPerStep, (u + 1) * kPerStep>([&](auto kp) {
        if constexpr (decltype(kp)::value < kPieces) conv_piece(kp, cv, nst, nr, nchunk);
      });
    });
  };

  // Epilogue. Lane (m, kh) holds, for block c, column ocol(c) + m and
  // accumulator rows 8(v/4) + 4kh + (v%4), i.e. antenna rho / DG, digit
  // rho % DG of row rho:
  //   DG = 8: antenna v/4, digit 4kh + v%4. Q = sum of its four digit sums
  //     times 256^(digit - 4kh) is exact in FP64 (< 2^48); lanes kh = 0 and 1
  //     swap halves so that lane kh finishes antennas 2kh and 2kh + 1:
  //     total = Q_low + 2^32 Q_high;
  //   DG = 4: antenna 2(v/4) + kh, digit v%4: the lane holds all four digit
  //     sums of antennas 2jj + kh (jj < 4), whose total is exact in int64.
  // eight digits: alpha and beta in FP64; four: in FP32 (no FP64 arithmetic)
  [[maybe_unused]] const double alpha =
      DG == 8 ? a.alpha * (a.scales ? (double)a.scales[b] : 1.0) : 0.0;
  [[maybe_unused]] const float alpha_f = a.alpha32 * (a.scales ? a.scales[b] : 1.f);
  const bool use_cin = DG == 8 ? a.beta != 0.0 : a.beta32 != 0.f;
  auto ant_of = [&](int jj) { return a0 + (DG == 8 ? 2 * kh + jj : 2 * jj + kh); };
  // cin of the group's outputs, loaded during its last stage (DG = 8) or
  // at the start of the epilogue (DG = 4: its lanes finish twice the
  // outputs, and the registers are not there to hold them through a stage)
  constexpr bool kPrefetchCin = DG == 8;
  f2a8 cpre[NB][G::fin];
  // this frame's outputs (a frame is below 2 GiB: 32-bit offsets)
  const size_t frame_out = (size_t)b * a.R * a.ld_out * 2;
  const float *cin_f = a.cin ? a.cin + frame_out : nullptr;  // read only when beta != 0
  float *out_f = a.out + frame_out;
  auto load_cin = [&]() {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
#pragma unroll
      for (int jj = 0; jj < G::fin; ++jj) {
        const int ant = ant_of(jj);
        const uint32_t o = (uint32_t)(ant * a.ld_out + ocol(c) + m) * 2u;
        // streaming load: cin is read once and should not evict the rows
        // that the next column groups read again
        cpre[c][jj] = (use_cin && m < nout(c) && ant < a.R)
                          ? __builtin_nontemporal_load((const f2a8 *)(cin_f + o))
                          : f2a8{0.f, 0.f};
      }
    }
  };
  auto finish_group = [&]() {
    if constexpr (!kPrefetchCin) load_cin();
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int col = ocol(c) + m;
      if constexpr (DG == 8) {
        double tot[2][2];  // [antenna ant_of(jj)][re, im]
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
          const i32x16 &acc = ri ? acc_im[c] : acc_re[c];
          double q[4];
#pragma unroll
          for (int j = 0; j < 4; ++j)
            q[j] = (double)acc[4 * j] + 256.0 * (double)acc[4 * j + 1] +
                   65536.0 * (double)acc[4 * j + 2] + 16777216.0 * (double)acc[4 * j + 3];
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const double send = kh ? q[jj] : q[2 + jj];
            const double recv = __shfl_xor(send, 32);
            const double lo = kh ? recv : q[jj];
            const double hi = kh ? q[2 + jj] : recv;
            tot[jj][ri] = lo + 4294967296.0 * hi;
          }
        }
        if (m < nout(c)) {
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const int ant = ant_of(jj);
            if (ant < a.R) {
              const int e = e_fin[jj];
              // 2^(e - scale): X carried scale - e fractional bits
              const double sc =
                  __builtin_bit_cast(double, (uint64_t)(e - G::scale + 1023) << 52);
              double re = alpha * (tot[jj][0] * sc), im = alpha * (tot[jj][1] * sc);
              if (e == 255) re = im = __builtin_nan("");
              const uint32_t o = (uint32_t)(ant * a.ld_out + col) * 2u;
              if (use_cin) {
                re += a.beta * (double)cpre[c][jj].x;
                im += a.beta * (double)cpre[c][jj].y;
              }
              __builtin_nontemporal_store(f2a8{(float)re, (float)im}, (f2a8 *)(out_f + o));
            }
          }
        }
      } else {
        // No FP64: the four digit sums of a row combine exactly in int64
        // (< 2^47), which is rounded once to FP32 and scaled by 2^(e - scale)
        // (exact unless the result leaves FP32's normal range); alpha and
        // beta are applied in FP32.
        if (m < nout(c)) {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int ant = ant_of(jj);
            if (ant < a.R) {
              float v[2];
#pragma unroll
              for (int ri = 0; ri < 2; ++ri) {
                const i32x16 &acc = ri ? acc_im[c] : acc_re[c];
                const int64_t t = (int64_t)acc[4 * jj] + (int64_t)acc[4 * jj + 1] * 256 +
                                  (int64_t)acc[4 * jj + 2] * 65536 +
                                  (int64_t)acc[4 * jj + 3] * 16777216;
                v[ri] = alpha_f * __builtin_amdgcn_ldexpf((float)t, e_fin[jj] - G::scale);
              }
              if (e_fin[jj] == 255) v[0] = v[1] = __builtin_nanf("");
              const uint32_t o = (uint32_t)(ant * a.ld_out + col) * 2u;
              if (use_cin) {
                v[0] = __builtin_fmaf(a.beta32, cpre[c][jj].x, v[0]);
                v[1] = __builtin_fmaf(a.beta32, cpre[c][jj].y, v[1]);
              }
              __builtin_nontemporal_store(f2a8{v[0], v[1]}, (f2a8 *)(out_f + o));
            }
          }
        }
      }
    }
  };

  land(stage, raw[0], 0);
  fetch(raw[0], 2 % nchunks);
  start_group(0);
  __syncthreads();
  for (int s0 = 0; s0 < total; s0 += 2) {
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      const int st = s0 + cc;
      if (st < total) {
        const int chunk = st % nchunks;
        if (kPrefetchCin && chunk == last) load_cin();
        // (after the last step the conversion fills a stage nobody reads)
        do_chunk(stage + cc * G::stage, chunk, stage + (1 - cc) * G::stage, raw[(cc + 1) & 1],
                 (st + 1) % nchunks);
        fetch(raw[(cc + 1) & 1], (st + 3) % nchunks);
        __syncthreads();
        if (chunk == last) {
          finish_group();
          if (st + 1 < total) start_group(st / nchunks + 1);
        }
      }
    }
  }
}

template <int DG, int NB, int NWV>
hipError_t launch_exact_nb(const ExArgs &a, int rblocks, int splits, int ngroups, int nbw_pad,
                           long nt, hipStream_t s) {
  using G = ExGeom<NWV, DG>;
  const size_t lds = (size_t)(kLutDw + nbw_pad + kMaxDw) * 4 + 2 * (size_t)G::stage;
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void *)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)nt), dim3(G::threads), lds, s, a, rblocks, splits,
                       ngroups, nbw_pad);
    return hipGetLastError();
  };
  if (a.seg_lag && a.rseg_lag) return hipErrorInvalidValue;  // never both (one direction each)
  if (a.seg_lag) return go(exact_kernel<DG, NB, NWV, true, false>);
  if (a.rseg_lag) return go(exact_kernel<DG, NB, NWV, false, true>);
  return go(exact_kernel<DG, NB, NWV, false, false>);
}

template <int DG>
hipError_t launch_exact_dg(const ExArgs &a, hipStream_t s) {
  const int vcols = virtual_cols(a.c_len, a.seg_len, a.seg_lag, 32);
  const int nb = vcols > 256 ? 4 : (vcols > 128 ? 2 : 1);
  // 8 waves (one workgroup per compute unit) pay off when each workgroup
  // runs enough stages to hide its fixed latencies (row scan, pipeline
  // start, epilogue); short rows take 4-wave tiles, two workgroups per unit
  const long stages8 = (long)((a.t_len + 511) / 512) * ((vcols + 1023) / 1024);
  const int nwv = (nb == 4 && vcols > 512 && stages8 >= 4) ? 8 : 4;
  const int gw = nwv * 32 * nb;
  const int ngroups = (vcols + gw - 1) / gw;
  constexpr int ant = 32 / DG;
  const int rblocks = (a.R + ant - 1) / ant;
  const long units = (long)a.batch * rblocks;
  // Small launches spread one block's column groups over several
  // workgroups (each finds the rows' exponents itself).
  constexpr long kFill = 2048;
  const int splits = units >= kFill ? 1 : (int)std::min<long>(ngroups, (kFill + units - 1) / units);
  const long nt = units * splits;
  if (nt <= 0 || nt > 0x7FFFFFFFL) return hipErrorInvalidValue;
  const int nbw_pad = (a.nbw + 3) & ~3;
  if (nwv == 8) return launch_exact_nb<DG, 4, 8>(a, rblocks, splits, ngroups, nbw_pad, nt, s);
  if (nb == 4) return launch_exact_nb<DG, 4, 4>(a, rblocks, splits, ngroups, nbw_pad, nt, s);
  if (nb == 2) return launch_exact_nb<DG, 2, 4>(a, rblocks, splits, ngroups, nbw_pad, nt, s);
  return launch_exact_nb<DG, 1, 4>(a, rblocks, splits, ngroups, nbw_pad, nt, s);
}

}  // namespace

hipError_t launch_exact(const ExArgs &a, hipStream_t s) {
  if (a.t_len < 2 || a.t_len > 65535 || a.c_len < 1 || a.R < 1 || a.batch < 1)
    return hipErrorInvalidValue;
  if (a.digits == 8) return launch_exact_dg<8>(a, s);
  if (a.digits == 4) return launch_exact_dg<4>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace pnce
