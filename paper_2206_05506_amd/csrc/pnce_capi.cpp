// pnce_capi.cpp -- host side of libpnce.so: plan construction (m-sequence,
// bit streams), argument validation and the extern "C" entry points declared
// in include/pnce.h.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pnce.h"
#include "pnce_internal.h"

struct pnce_plan {
  int N, T, L, R, K, d;
  int device;
  int nbw;                       // words of each periodic bit stream
  std::vector<signed char> seq;  // +-1, N entries
  uint32_t *d_fwd = nullptr;     // bit p = sequence[p mod N] is -1
  uint32_t *d_rev = nullptr;     // bit p = sequence[(-p) mod N] is -1
};

namespace {

thread_local std::string g_last_error;

pnce_status fail(pnce_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

pnce_status hip_fail(hipError_t e, const char *what) {
  return fail(PNCE_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Feedback masks of one primitive polynomial x^d + sum x^i per degree
// (bit i set for each exponent i < d). Any primitive polynomial gives a
// sequence with the two-level autocorrelation of Eq. 1; this table fixes one
// per degree.
constexpr uint32_t kFeedback[17] = {
    0, 0,
    0x3,     // d=2:  x^2 + x + 1
    0x3,     // d=3:  x^3 + x + 1
    0x3,     // d=4:  x^4 + x + 1
    0x5,     // d=5:  x^5 + x^2 + 1
    0x3,     // d=6:  x^6 + x + 1
    0x3,     // d=7:  x^7 + x + 1
    0x1D,    // d=8:  x^8 + x^4 + x^3 + x^2 + 1
    0x11,    // d=9:  x^9 + x^4 + 1
    0x9,     // d=10: x^10 + x^3 + 1
    0x5,     // d=11: x^11 + x^2 + 1
    0x53,    // d=12: x^12 + x^6 + x^4 + x + 1
    0x1B,    // d=13: x^13 + x^4 + x^3 + x + 1
    0x443,   // d=14: x^14 + x^10 + x^6 + x + 1
    0x3,     // d=15: x^15 + x + 1
    0x100B,  // d=16: x^16 + x^12 + x^3 + x + 1
};

// m-sequence of degree d (Section II-A, Eq. 1). A d-bit window register
// holds bits b[n .. n+d-1] (b[n] in bit 0); the next bit is the parity of the
// window masked by the feedback taps, i.e. b[n+d] = XOR_i b[n+i]. The window
// starts as 1,0,...,0; bit 0 is sent as +1 and bit 1 as -1.
std::vector<signed char> make_sequence(int d) {
  const int N = (1 << d) - 1;
  std::vector<signed char> s(N);
  uint32_t win = 1u;
  for (int n = 0; n < N; ++n) {
    s[n] = (win & 1u) ? -1 : 1;
    const uint32_t fb = (uint32_t)__builtin_parity(win & kFeedback[d]);
    win = (win >> 1) | (fb << (d - 1));
  }
  return s;
}

// Periodic bit stream of `len` bits: bit p = 1 where seq[(sign * p) mod N]
// is -1.
std::vector<uint32_t> bit_stream(const std::vector<signed char> &s, int len_words, int sign) {
  const long N = (long)s.size();
  std::vector<uint32_t> w((size_t)len_words, 0u);
  for (long p = 0; p < 32L * len_words; ++p) {
    long i = (sign * p) % N;
    if (i < 0) i += N;
    if (s[(size_t)i] < 0) w[(size_t)(p >> 5)] |= 1u << (p & 31);
  }
  return w;
}

bool valid_prec(int p) {
  return p == PNCE_PREC_F32 || p == PNCE_PREC_F32S || p == PNCE_PREC_BF16 ||
         p == PNCE_PREC_F64;
}

bool valid_fmt(int f) {
  return f == PNCE_FMT_BF16 || f == PNCE_FMT_F16 || f == PNCE_FMT_E4M3;
}

pnce_status check_plan(const pnce_plan *p) {
  if (!p) return fail(PNCE_E_INVALID, "plan is NULL");
  return PNCE_OK;
}

pnce_status check_batch(const pnce_plan *p, int batch) {
  if (batch <= 0) return fail(PNCE_E_INVALID, "batch must be positive");
  if ((long)batch * p->R > 0x7FFFFFFFL / 2)
    return fail(PNCE_E_INVALID, "batch * R too large");
  return PNCE_OK;
}

// Contraction through the tiled kernels or the FP64 vector kernel.
pnce_status run_tg(const pnce_plan *p, hipStream_t s, int precision, int in_fmt,
                   const void *in, int t_len, int ld_in, void *out, int c_len,
                   const void *cin, const uint32_t *bits, const float *scales,
                   int batch, double alpha, double beta) {
  hipError_t e;
  if (precision == PNCE_PREC_F64) {
    pnce::Tg64Args a{};
    a.in = in;
    a.out = out;
    a.cin = cin;
    a.bits = bits;
    a.scales = scales;
    a.R = p->R;
    a.batch = batch;
    a.t_len = t_len;
    a.ld_in = ld_in;
    a.c_len = c_len;
    a.ld_out = c_len;
    a.N = p->N;
    a.alpha = alpha;
    a.beta = beta;
    a.in_f64 = true;
    a.out_f64 = true;
    e = pnce::launch_tg64(a, s);
  } else {
    pnce::TgArgs a{};
    a.in = in;
    a.out = (float *)out;
    a.cin = (const float *)cin;
    a.bits = bits;
    a.scales = scales;
    a.R = p->R;
    a.batch = batch;
    a.t_len = t_len;
    a.ld_in = ld_in;
    a.c_len = c_len;
    a.ld_out = c_len;
    a.N = p->N;
    a.nbw = p->nbw;
    a.alpha = (float)alpha;
    a.beta = (float)beta;
    e = pnce::launch_tg(precision, in_fmt, a, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return PNCE_OK;
}

}  // namespace

extern "C" {

pnce_status pnce_create(pnce_plan **plan, int N, int T, int L, int R) {
  try {
    if (!plan) return fail(PNCE_E_INVALID, "plan output pointer is NULL");
    *plan = nullptr;
    if (T <= 0 || L <= 0 || R <= 0) return fail(PNCE_E_INVALID, "T, L and R must be positive");
    int d = 0;
    while (d <= 16 && (1 << d) - 1 < N) ++d;
    if (N <= 0 || d < 2 || d > 16 || (1 << d) - 1 != N)
      return fail(PNCE_E_UNSUPPORTED, "N must be 2^d - 1 with 2 <= d <= 16");
    if ((long)T * L > 16L * N) return fail(PNCE_E_INVALID, "T*L exceeds 16*N");
    if (R > 65535) return fail(PNCE_E_INVALID, "R exceeds 65535");
    const int K = T * L;

    pnce_plan *p = new (std::nothrow) pnce_plan();
    if (!p) return fail(PNCE_E_NOMEM, "host allocation failed");
    p->N = N;
    p->T = T;
    p->L = L;
    p->R = R;
    p->K = K;
    p->d = d;
    p->seq = make_sequence(d);
    // Positions read by the kernels stay below N + max(N, K) + 80 bits.
    const long bits = (long)N + (K > N ? K : N) + 160;
    p->nbw = (int)((bits + 31) / 32);
    const std::vector<uint32_t> fwd = bit_stream(p->seq, p->nbw, +1);
    const std::vector<uint32_t> rev = bit_stream(p->seq, p->nbw, -1);

    // Test hook: PNCE_FAULT=alloc makes the device allocation fail.
    const char *fault = std::getenv("PNCE_FAULT");
    if (fault && std::strcmp(fault, "alloc") == 0) {
      delete p;
      return fail(PNCE_E_NOMEM, "device allocation failed (PNCE_FAULT=alloc)");
    }
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
      delete p;
      return hip_fail(e, "hipGetDevice");
    }
    const size_t bytes = (size_t)p->nbw * 4;
    e = hipMalloc((void **)&p->d_fwd, bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_rev, bytes);
    if (e != hipSuccess) {
      (void)hipFree(p->d_fwd);
      delete p;
      return fail(PNCE_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_fwd, fwd.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_rev, rev.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p->d_fwd);
      (void)hipFree(p->d_rev);
      delete p;
      return hip_fail(e, "hipMemcpy");
    }
    *plan = p;
    if (K > N) {
      g_last_error = "T*L > N: lags alias mod N";
      return PNCE_W_LAG_ALIAS;
    }
    return PNCE_OK;
  } catch (...) {
    return fail(PNCE_E_NOMEM, "exception during plan creation");
  }
}

pnce_status pnce_destroy(pnce_plan *plan) {
  if (!plan) return PNCE_OK;
  (void)hipFree(plan->d_fwd);
  (void)hipFree(plan->d_rev);
  delete plan;
  return PNCE_OK;
}

pnce_status pnce_get_sequence(const pnce_plan *plan, signed char *s_host) {
  if (pnce_status st = check_plan(plan)) return st;
  if (!s_host) return fail(PNCE_E_INVALID, "output pointer is NULL");
  std::memcpy(s_host, plan->seq.data(), plan->seq.size());
  return PNCE_OK;
}

pnce_status pnce_get_shape(const pnce_plan *plan, int *N, int *T, int *L, int *R) {
  if (pnce_status st = check_plan(plan)) return st;
  if (N) *N = plan->N;
  if (T) *T = plan->T;
  if (L) *L = plan->L;
  if (R) *R = plan->R;
  return PNCE_OK;
}

pnce_status pnce_estimate(const pnce_plan *plan, void *stream, const void *Y, void *H,
                          int batch, int precision, double alpha, const float *scales,
                          double beta) {
  if (pnce_status st = check_plan(plan)) return st;
  if (!Y || !H) return fail(PNCE_E_INVALID, "Y and H must be non-NULL");
  if (pnce_status st = check_batch(plan, batch)) return st;
  if (!valid_prec(precision)) return fail(PNCE_E_INVALID, "unknown precision");
  return run_tg(plan, (hipStream_t)stream, precision, pnce::IN_C64, Y, plan->N, plan->N, H,
                plan->K, beta != 0.0 ? H : nullptr, plan->d_fwd, scales, batch, alpha, beta);
}

pnce_status pnce_pack(const pnce_plan *plan, void *stream, const void *Y, void *Yq,
                      float *scales, int batch, int format) {
  if (pnce_status st = check_plan(plan)) return st;
  if (!Y || !Yq || !scales) return fail(PNCE_E_INVALID, "Y, Yq and scales must be non-NULL");
  if (pnce_status st = check_batch(plan, batch)) return st;
  if (!valid_fmt(format)) return fail(PNCE_E_INVALID, "unknown format");
  hipError_t e = pnce::launch_pack((const float *)Y, Yq, scales, batch, plan->R, plan->N,
                                   format, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "pack launch");
  return PNCE_OK;
}

pnce_status pnce_estimate_packed(const pnce_plan *plan, void *stream, const void *Yq,
                                 const float *scales, void *H, int batch, int format,
                                 double beta) {
  if (pnce_status st = check_plan(plan)) return st;
  if (!Yq || !H) return fail(PNCE_E_INVALID, "Yq and H must be non-NULL");
  if (pnce_status st = check_batch(plan, batch)) return st;
  if (!valid_fmt(format)) return fail(PNCE_E_INVALID, "unknown format");
  const int in_fmt = format == PNCE_FMT_BF16  ? pnce::IN_BF16
                     : format == PNCE_FMT_F16 ? pnce::IN_F16
                                              : pnce::IN_E4M3;
  const int Np = plan->N + 1;
  // The zero pad sample is part of the reduction (it contributes nothing).
  return run_tg(plan, (hipStream_t)stream, pnce::MODE_BF16, in_fmt, Yq, Np, Np, H, plan->K,
                beta != 0.0 ? H : nullptr, plan->d_fwd, scales, batch, 1.0 / plan->N, beta);
}

pnce_status pnce_adjoint(const pnce_plan *plan, void *stream, const void *G, void *A,
                         const void *C, int batch, int precision, double alpha, double beta) {
  if (pnce_status st = check_plan(plan)) return st;
  if (!G || !A) return fail(PNCE_E_INVALID, "G and A must be non-NULL");
  if (beta != 0.0 && !C) return fail(PNCE_E_INVALID, "C must be non-NULL when beta != 0");
  if (pnce_status st = check_batch(plan, batch)) return st;
  if (!valid_prec(precision)) return fail(PNCE_E_INVALID, "unknown precision");
  return run_tg(plan, (hipStream_t)stream, precision, pnce::IN_C64, G, plan->K, plan->K, A,
                plan->N, beta != 0.0 ? C : nullptr, plan->d_rev, nullptr, batch, alpha, beta);
}

pnce_status pnce_refine(const pnce_plan *plan, void *stream, const void *y, void *X,
                        void *work, int batch, int steps) {
  if (pnce_status st = check_plan(plan)) return st;
  if (!y || !X || (!work && steps > 0)) return fail(PNCE_E_INVALID, "y, X and work must be non-NULL");
  if (pnce_status st = check_batch(plan, batch)) return st;
  if (steps < 0) return fail(PNCE_E_INVALID, "steps must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  for (int j = 0; j < steps; ++j) {
    // r = y - P x   (P x = sum_k x[k] s[(n-k) mod N]: adjoint stream, alpha -1)
    if (j + 1 < steps) {
      if (pnce_status st = run_tg(plan, s, PNCE_PREC_F32S, pnce::IN_C64, X, plan->K, plan->K,
                                  work, plan->N, y, plan->d_rev, nullptr, batch, -1.0, 1.0))
        return st;
    } else {
      pnce::Tg64Args a{};
      a.in = X;
      a.out = work;
      a.cin = y;
      a.bits = plan->d_rev;
      a.scales = nullptr;
      a.R = plan->R;
      a.batch = batch;
      a.t_len = plan->K;
      a.ld_in = plan->K;
      a.c_len = plan->N;
      a.ld_out = plan->N;
      a.N = plan->N;
      a.alpha = -1.0;
      a.beta = 1.0;
      a.in_f64 = false;
      a.out_f64 = false;
      hipError_t e = pnce::launch_tg64(a, s);
      if (e != hipSuccess) return hip_fail(e, "residual launch");
    }
    // x = x + P^T r / N
    if (pnce_status st = run_tg(plan, s, PNCE_PREC_F32S, pnce::IN_C64, work, plan->N, plan->N,
                                X, plan->K, X, plan->d_fwd, nullptr, batch, 1.0 / plan->N, 1.0))
      return st;
  }
  return PNCE_OK;
}

const char *pnce_status_string(pnce_status status) {
  switch (status) {
    case PNCE_OK: return "ok";
    case PNCE_W_LAG_ALIAS: return "warning: T*L > N, lags alias mod N";
    case PNCE_E_INVALID: return "invalid argument";
    case PNCE_E_UNSUPPORTED: return "unsupported configuration";
    case PNCE_E_NOMEM: return "out of memory";
    case PNCE_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char *pnce_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
