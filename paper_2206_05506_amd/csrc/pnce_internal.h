// pnce_internal.h -- shared declarations between the C-ABI host code and the
// HIP kernels of libpnce.so. Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pnce {

// Contraction modes of the Toeplitz +-1 kernels (same values as PNCE_PREC_*).
enum Mode { MODE_F32 = 0, MODE_F32S = 1, MODE_BF16 = 2, MODE_F64 = 3 };

// Input encodings of the tiled kernel. IN_C64_LAGS: complex64 rows of
// rseg_n blocks of rseg_len terms, block j's terms sitting at reduction
// positions j * rseg_lag + l (zero between blocks); t_len counts positions.
enum InFmt { IN_C64 = 0, IN_BF16 = 1, IN_F16 = 2, IN_E4M3 = 3, IN_C64_LAGS = 4 };

// One Toeplitz +-1 contraction over a batch of row blocks:
//   out[b][r][c] = alpha_b * sum_{t < t_len} in[b][r][t] * sgn(bits[(t - lag(c) + poff) mod N])
//                  + beta * cin[b][r][c],        c < c_len,
// sgn(0) = +1, sgn(1) = -1, alpha_b = alpha * (scales ? scales[b] : 1).
// lag(c) = c, or with column segments (seg_lag > 0, Eq. 8's lag spacing)
// lag(j * seg_len + l) = j * seg_lag + l for l < seg_len.
// Complex rows are interleaved; packed inputs hold a real plane then an
// imaginary plane per row, each ld_in codes long.
struct TgArgs {
  const void *in;
  float *out;
  const float *cin;
  const uint32_t *bits;
  const float *scales;
  int R, batch;
  int t_len, ld_in;
  int c_len, ld_out;
  int N, nbw;
  float alpha, beta;
  // Nonzero: least-squares rows, out <- N/(N+1) (out + sum(out)/(N+1-c_len))
  // (complex64 input, beta = 0, c_len <= N).
  int ls;
  int seg_len, seg_lag;  // column segments (seg_lag = 0: none)
  int poff;              // shift of every sequence position, in [0, N)
  int rseg_len, rseg_lag, rseg_n;  // reduction blocks of IN_C64_LAGS rows
};

// Columns as the kernels deal them out: segments of seg_len columns are
// padded to a multiple of `gran` (the columns one wave or block holds, so
// none straddles two segments); without segments the layout is the output.
__host__ __device__ inline int seg_pad(int seg_len, int seg_lag, int gran) {
  return seg_lag ? (seg_len + gran - 1) / gran * gran : (1 << 30);
}
inline int virtual_cols(int c_len, int seg_len, int seg_lag, int gran) {
  if (!seg_lag) return c_len;
  return (c_len + seg_len - 1) / seg_len * seg_pad(seg_len, seg_lag, gran);
}

hipError_t launch_tg(int mode, int in_fmt, const TgArgs &a, hipStream_t s);

// Contraction with exact sums (pnce_exact.hip): complex64 rows, int8 matrix
// cores on `digits` (8 or 4) 8-bit fixed-point digits per value, alpha and
// beta in FP64. Same geometry fields as TgArgs; t_len in [2, 65535].
struct ExArgs {
  const float *in;
  float *out;
  const float *cin;
  const uint32_t *bits;
  const float *scales;
  int R, batch;
  int t_len, ld_in;
  int c_len, ld_out;
  int N, nbw;
  double alpha, beta;
  int seg_len, seg_lag;
  int poff;
  int rseg_len, rseg_lag, rseg_n;
  int digits;
  float alpha32, beta32;  // alpha and beta rounded to FP32 (digits == 4)
};
hipError_t launch_exact(const ExArgs &a, hipStream_t s);

// LDS one workgroup needs, at most over the kernels, for a bit stream of
// nbw words, and what a gfx950 workgroup may have.
size_t max_lds_bytes(int nbw);
constexpr size_t kLdsLimitBytes = 160 * 1024;

// In-place least-squares correction of `rows` rows of K complex64 values.
hipError_t launch_debias(float *H, long rows, int K, int N, hipStream_t s);

// Same contraction on complex64 rows with FP64 sums on FP64 matrix cores;
// alpha and beta are applied in FP64 before the single rounding to FP32.
hipError_t launch_f64mm(const TgArgs &a, hipStream_t s);

// FP64-accumulating vector kernel; element types selected by the flags.
struct Tg64Args {
  const void *in;
  void *out;
  const void *cin;
  const uint32_t *bits;
  const float *scales;
  int R, batch;
  int t_len, ld_in;
  int c_len, ld_out;
  int N;
  double alpha, beta;
  bool in_f64, out_f64;
  int seg_len, seg_lag;  // as in TgArgs
  int poff;
  // reduction blocks (rseg_lag = 0: none): term t = j * rseg_len + l of a
  // row sits at position j * rseg_lag + l; t_len counts terms
  int rseg_len, rseg_lag;
};
hipError_t launch_tg64(const Tg64Args &a, hipStream_t s);

// Uneven batch: one persistent launch over a host-built work list.
struct VFrame {           // one frame of the batch (device copy)
  long long y_off;        // first code of the frame in the input buffer
  long long h_off;        // first complex output of the frame
  int R, N, K;
  int bits_off, nbw;      // the frame's bit stream inside the bits table
};
struct VTile {            // one workgroup tile
  int frame, a0, colg, nc;
};
struct VArgs {
  const void *in;         // planar codes of every frame
  float *out;             // complex64 CIRs of every frame
  const float *scales;    // per-frame scale (or null)
  const VFrame *frames;
  const VTile *tiles;
  const int *wg_start;    // tiles of workgroup w: [wg_start[w], wg_start[w+1])
  const uint32_t *bits;   // concatenated bit streams, one per sequence length
  int nbw_max;            // largest bit stream (LDS words)
};
hipError_t launch_varlen(int in_fmt, const VArgs &a, int n_wg, hipStream_t s);
// One frame through the uniform kernel with a forced column width.
hipError_t launch_tg_frame(int in_fmt, int nc, const TgArgs &a, hipStream_t s);

// Quantiser: per-frame scale, then conversion into planar codes.
// Rows of N samples ld complex apart (ld = N: contiguous frames). Batches of
// at least kPackFrameBatch frames (a frame per CU or more) of at most
// kPackFrameMaxBytes each take one launch with a workgroup per frame (the
// frames in flight then fit the Infinity Cache, which serves the second
// read); other batches spread each frame over many workgroups in four
// launches. Both give the same codes and scales.
constexpr int kPackFrameBatch = 256;
constexpr long long kPackFrameMaxBytes = 1LL << 20;
// flag (may be null): a word set to 0 by the launch (the wait flag of the
// workspace path, which these launches do not wait on).
hipError_t launch_pack(const float *y, void *yq, float *scales, int batch,
                       int R, int N, int ld, int fmt, hipStream_t s, uint32_t *flag = nullptr);
// Same codes and scales with a workspace of kPackSyncWords * batch + 1
// words (PNCE_PACK_WORK_BYTES): frames that the one-launch path does not
// take are read from HBM once, in slices held in registers while the frame
// maximum is gathered (one launch after a clear of the workspace). Word
// kPackSyncWords * batch becomes nonzero if a slice's wait for the rest of
// its frame ran past its bound.
constexpr int kPackSyncWords = 1024;
hipError_t launch_pack_ws(const float *y, void *yq, float *scales, uint32_t *work, int batch,
                          int R, int N, int ld, int fmt, hipStream_t s);

}  // namespace pnce
