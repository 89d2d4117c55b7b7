// pnce_internal.h -- shared declarations between the C-ABI host code and the
// HIP kernels of libpnce.so. Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pnce {

// Contraction modes of the Toeplitz +-1 kernels (same values as PNCE_PREC_*).
enum Mode { MODE_F32 = 0, MODE_F32S = 1, MODE_BF16 = 2, MODE_F64 = 3 };

// Input encodings of the tiled kernel.
enum InFmt { IN_C64 = 0, IN_BF16 = 1, IN_F16 = 2, IN_E4M3 = 3 };

// One Toeplitz +-1 contraction over a batch of row blocks:
//   out[b][r][c] = alpha_b * sum_{t < t_len} in[b][r][t] * sgn(bits[(t - c) mod N])
//                  + beta * cin[b][r][c],        c < c_len,
// sgn(0) = +1, sgn(1) = -1, alpha_b = alpha * (scales ? scales[b] : 1).
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
};

hipError_t launch_tg(int mode, int in_fmt, const TgArgs &a, hipStream_t s);

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
};
hipError_t launch_tg64(const Tg64Args &a, hipStream_t s);

// Quantiser: per-frame scale, then conversion into planar codes.
hipError_t launch_pack(const float *y, void *yq, float *scales, int batch,
                       int R, int N, int fmt, hipStream_t s);

}  // namespace pnce
