// Time-domain signals (Sec. III-F): impulse responses from the spectra (Eqs. 5-6, 9-10, 13:
// h = F^-1[H]) and received signals (Eq. 14: s = h * s_e).
//
// Impulse response of receiver m on t_n = n dt, dt = 1 / (n_t df), n < n_t:
//   h_m(t_n) = 2 df Re[ e^{-j sigma 2 pi f_lo t_n} sum_{k<F} H_m[k] e^{-j sigma 2 pi k n / n_t} ],
// so the inner sum is a length-n_t DFT of the zero-padded spectrum (sign -sigma), then a
// carrier-and-scale pass with the carrier phase reduced in FP64.  The received signal is the
// linear convolution s_m[n] = dt sum_k h_m[k] s_e[n - k] by FFT of length P (zero padding),
// spectral product and inverse FFT.
//
// The FFTs are Stockham autosort transforms of every row (receiver) at once with twiddles from a
// table computed in FP64 once per call.  A row of up to LDS_FFT_MAX points is transformed by
// one workgroup in LDS (one launch for all stages); longer rows run radix-4 stages over global
// memory (plus one radix-2 stage for an odd power of two), each a streaming pass.
#include "internal.hpp"

#include <algorithm>
#include <cmath>

namespace et {

namespace {

constexpr int TB = 256;

inline unsigned tgrid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + TB - 1) / TB, 65536)); }

constexpr int64_t LDS_FFT_MAX = 4096;   // points per row transformed in LDS (two buffers: 64 KB)
constexpr int FB = 256;                  // threads of the LDS transform

// tw[m] = e^{sign j 2 pi m / N}, m < N, from FP64 sincospi rounded to FP32.
__global__ void k_twiddles(float2* __restrict__ tw, int64_t N, int sign) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < N; m += (int64_t)gridDim.x * blockDim.x) {
    double sn, cs;
    sincospi((double)sign * 2.0 * (double)m / (double)N, &sn, &cs);
    tw[m] = make_float2((float)cs, (float)sn);
  }
}

__device__ inline float2 cmulf(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// sign j (a + j b): a quarter turn in the transform's direction
__device__ inline float2 qturn(float2 a, int sign) { return sign > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x); }

// Butterflies of one Stockham stage, sub-transforms of length Ns growing to R Ns (R = 2 or 4):
// for j < N / R with k = j % Ns, v_r = x[j + r N / R] e^{sign j 2 pi r k / (R Ns)}, then the
// R-point DFT of v, y[(j / Ns) R Ns + k + q Ns] = sum_r v_r e^{sign j 2 pi r q / R}.  After
// log2 N stages y is the DFT of the row in natural order.
template <int R>
__device__ inline void stockham_butterfly(const float2* __restrict__ x, float2* __restrict__ y, int64_t N, int64_t Ns,
                                          int64_t j, const float2* __restrict__ tw, int sign) {
  const int64_t k = j % Ns, q0 = (j / Ns) * R * Ns + k;
  const int64_t step = N / (R * Ns);   // table stride of e^{sign j 2 pi k / (R Ns)}
  if (R == 2) {
    const float2 a = x[j], b = cmulf(x[j + N / 2], tw[k * step]);
    y[q0] = make_float2(a.x + b.x, a.y + b.y);
    y[q0 + Ns] = make_float2(a.x - b.x, a.y - b.y);
  } else {
    const int64_t qN = N / 4;
    const float2 v0 = x[j];
    const float2 v1 = cmulf(x[j + qN], tw[k * step]);
    const float2 v2 = cmulf(x[j + 2 * qN], tw[2 * k * step]);
    const float2 v3 = cmulf(x[j + 3 * qN], tw[3 * k * step]);
    const float2 s02 = make_float2(v0.x + v2.x, v0.y + v2.y), d02 = make_float2(v0.x - v2.x, v0.y - v2.y);
    const float2 s13 = make_float2(v1.x + v3.x, v1.y + v3.y), d13 = qturn(make_float2(v1.x - v3.x, v1.y - v3.y), sign);
    y[q0] = make_float2(s02.x + s13.x, s02.y + s13.y);
    y[q0 + Ns] = make_float2(d02.x + d13.x, d02.y + d13.y);
    y[q0 + 2 * Ns] = make_float2(s02.x - s13.x, s02.y - s13.y);
    y[q0 + 3 * Ns] = make_float2(d02.x - d13.x, d02.y - d13.y);
  }
}

// One stage over global memory for `rows` transforms of length N.
template <int R>
__global__ void k_fft_stage(const float2* __restrict__ x, float2* __restrict__ y, int64_t rows, int64_t N, int64_t Ns,
                            const float2* __restrict__ tw, int sign) {
  const int64_t per = N / R;
  const int64_t total = rows * per;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / per, j = t - r * per;
    stockham_butterfly<R>(x + r * N, y + r * N, N, Ns, j, tw, sign);
  }
}

// Every stage of one row (workgroup = row) in LDS: a radix-2 stage first for an odd power of
// two, then radix-4 stages.
__global__ __launch_bounds__(FB) void k_fft_lds(const float2* __restrict__ in, float2* __restrict__ out, int64_t N,
                                                const float2* __restrict__ tw, int sign) {
  __shared__ float2 buf[2][LDS_FFT_MAX];
  const int64_t row = blockIdx.x;
  const float2* src = in + row * N;
  for (int64_t i = threadIdx.x; i < N; i += FB) buf[0][i] = src[i];
  __syncthreads();
  int cur = 0;
  int64_t Ns = 1;
  int lg = 0;
  while ((int64_t(1) << lg) < N) ++lg;
  if (lg & 1) {
    for (int64_t j = threadIdx.x; j < N / 2; j += FB) stockham_butterfly<2>(buf[cur], buf[cur ^ 1], N, Ns, j, tw, sign);
    __syncthreads();
    cur ^= 1;
    Ns = 2;
  }
  for (; Ns < N; Ns *= 4) {
    for (int64_t j = threadIdx.x; j < N / 4; j += FB) stockham_butterfly<4>(buf[cur], buf[cur ^ 1], N, Ns, j, tw, sign);
    __syncthreads();
    cur ^= 1;
  }
  float2* dst = out + row * N;
  for (int64_t i = threadIdx.x; i < N; i += FB) dst[i] = buf[cur][i];
}

// DFT of every row (length N, a power of two) with e^{sign j 2 pi k n / N}: a holds the input;
// returns the buffer holding the result (a or b).  tw: N entries of scratch for the table.
float2* fft_rows(float2* a, float2* b, float2* tw, int64_t rows, int64_t N, int sign, hipStream_t s) {
  k_twiddles<<<tgrid(N), TB, 0, s>>>(tw, N, sign);
  if (N <= LDS_FFT_MAX) {
    if (N > 1) {
      k_fft_lds<<<(unsigned)rows, FB, 0, s>>>(a, b, N, tw, sign);
      ET_HIP(hipGetLastError());
      return b;
    }
    return a;
  }
  float2* x = a;
  float2* y = b;
  int lg = 0;
  while ((int64_t(1) << lg) < N) ++lg;
  int64_t Ns = 1;
  if (lg & 1) {
    k_fft_stage<2><<<tgrid(rows * (N / 2)), TB, 0, s>>>(x, y, rows, N, Ns, tw, sign);
    std::swap(x, y);
    Ns = 2;
  }
  for (; Ns < N; Ns *= 4) {
    k_fft_stage<4><<<tgrid(rows * (N / 4)), TB, 0, s>>>(x, y, rows, N, Ns, tw, sign);
    std::swap(x, y);
  }
  ET_HIP(hipGetLastError());
  return x;
}

__global__ void k_pad_spectra(const float* __restrict__ H, int64_t M, int64_t F, int64_t N, float2* __restrict__ out) {
  const int64_t total = M * N;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = t / N, k = t - m * N;
    out[t] = k < F ? make_float2(H[(m * F + k) * 2], H[(m * F + k) * 2 + 1]) : make_float2(0.f, 0.f);
  }
}

// h[m][n] = 2 df Re(e^{-j sigma 2 pi f_lo n dt} S[m][n]); the carrier phase f_lo n dt is reduced
// to a fraction of a cycle in FP64.
__global__ void k_carrier(const float2* __restrict__ S, int64_t M, int64_t N, double f_lo_dt, int sigma, double scale,
                          float* __restrict__ h) {
  const int64_t total = M * N;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = t % N;
    const double cyc = f_lo_dt * (double)n;
    double sn, cs;
    sincospi(-2.0 * (double)sigma * (cyc - floor(cyc)), &sn, &cs);
    const float2 v = S[t];
    h[t] = (float)(scale * ((double)v.x * cs - (double)v.y * sn));
  }
}

// rows 0..M-1: h zero-padded to P; row M: the emitted call zero-padded to P
__global__ void k_pad_signals(const float* __restrict__ h, int64_t M, int64_t n_t, const float* __restrict__ se,
                              int64_t L, int64_t P, float2* __restrict__ out) {
  const int64_t total = (M + 1) * P;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = t / P, i = t - m * P;
    float v = 0.f;
    if (m < M) v = i < n_t ? h[m * n_t + i] : 0.f;
    else v = i < L ? se[i] : 0.f;
    out[t] = make_float2(v, 0.f);
  }
}

__global__ void k_spectral_product(float2* __restrict__ X, int64_t M, int64_t P) {
  const int64_t total = M * P;
  const float2* E = X + M * P;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const float2 a = X[t], b = E[t % P];
    X[t] = make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
  }
}

__global__ void k_unpack_signal(const float2* __restrict__ Y, int64_t M, int64_t P, int64_t n_out, double scale,
                                float* __restrict__ out) {
  const int64_t total = M * n_out;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = t / n_out, i = t - m * n_out;
    out[t] = (float)(scale * (double)Y[m * P + i].x);
  }
}

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

int64_t conv_length(int64_t n_t, int64_t L) {
  int64_t P = 1;
  while (P < n_t + L - 1) P <<= 1;
  return P;
}

size_t impulse_ws_bytes(int64_t M, int64_t n_t) {
  return 2 * al(sizeof(float2) * (size_t)M * n_t) + al(sizeof(float2) * (size_t)n_t);
}

size_t signal_ws_bytes(int64_t M, int64_t n_t, int64_t L) {
  const int64_t P = conv_length(n_t, L);
  return 2 * al(sizeof(float2) * (size_t)(M + 1) * P) + al(sizeof(float2) * (size_t)P);
}

void impulse_run(int64_t M, int64_t F, double f_lo, double df, int sigma, const float* spectra, int64_t n_t, void* ws,
                 float* h, hipStream_t s) {
  float2* a = (float2*)ws;
  float2* b = (float2*)((char*)ws + al(sizeof(float2) * (size_t)M * n_t));
  float2* tw = (float2*)((char*)ws + 2 * al(sizeof(float2) * (size_t)M * n_t));
  k_pad_spectra<<<tgrid(M * n_t), TB, 0, s>>>(spectra, M, F, n_t, a);
  // sum_k H_k e^{-j sigma 2 pi k n / n_t}: forward DFT for sigma = +1, inverse direction for -1
  float2* S = fft_rows(a, b, tw, M, n_t, -sigma, s);
  const double dt = 1.0 / ((double)n_t * df);
  k_carrier<<<tgrid(M * n_t), TB, 0, s>>>(S, M, n_t, f_lo * dt, sigma, 2.0 * df, h);
  ET_HIP(hipGetLastError());
}

void signal_run(int64_t M, int64_t n_t, const float* h, int64_t L, const float* se, double dt, void* ws, float* out,
                hipStream_t s) {
  const int64_t P = conv_length(n_t, L);
  float2* a = (float2*)ws;
  float2* b = (float2*)((char*)ws + al(sizeof(float2) * (size_t)(M + 1) * P));
  float2* tw = (float2*)((char*)ws + 2 * al(sizeof(float2) * (size_t)(M + 1) * P));
  k_pad_signals<<<tgrid((M + 1) * P), TB, 0, s>>>(h, M, n_t, se, L, P, a);
  float2* X = fft_rows(a, b, tw, M + 1, P, -1, s);
  k_spectral_product<<<tgrid(M * P), TB, 0, s>>>(X, M, P);
  float2* other = X == a ? b : a;
  float2* Y = fft_rows(X, other, tw, M, P, +1, s);   // only the M product rows
  k_unpack_signal<<<tgrid(M * (n_t + L - 1)), TB, 0, s>>>(Y, M, P, n_t + L - 1, dt / (double)P, out);
  ET_HIP(hipGetLastError());
}

}  // namespace et
