// Time-domain signals (Sec. III-F): impulse responses from the spectra (Eqs. 5-6, 9-10, 13:
// h = F^-1[H]) and received signals (Eq. 14: s = h * s_e).
//
// Impulse response of receiver m on t_n = n dt, dt = 1 / (n_t df), n < n_t:
//   h_m(t_n) = 2 df Re[ e^{-j sigma 2 pi f_lo t_n} sum_{k<F} H_m[k] e^{-j sigma 2 pi k n / n_t} ],
// so the inner sum is a length-n_t DFT of the zero-padded spectrum (sign -sigma), done by a
// radix-2 Stockham FFT over global memory (one launch per stage, all receivers together; the
// data are a few MB, so the passes run at HBM/L2 speed), then a carrier-and-scale pass with
// the carrier phase reduced in FP64.  The received signal is the linear convolution
// s_m[n] = dt sum_k h_m[k] s_e[n - k] by FFT of length P (zero padding), spectral product and
// inverse FFT.
#include "internal.hpp"

#include <algorithm>
#include <cmath>

namespace et {

namespace {

constexpr int TB = 256;

inline unsigned tgrid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + TB - 1) / TB, 65536)); }

// One Stockham radix-2 stage over `rows` transforms of length N (Ns = current sub-transform
// length 1, 2, ..., N/2): y[(j / Ns) 2 Ns + j % Ns (+ Ns)] = x[j] +- w x[j + N/2],
// w = e^{sign j pi (j % Ns) / Ns}.  After log2 N stages y is the DFT in natural order.
__global__ void k_fft_stage(const float2* __restrict__ x, float2* __restrict__ y, int64_t rows, int64_t N, int64_t Ns,
                            int sign) {
  const int64_t half = N >> 1;
  const int64_t total = rows * half;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / half, j = t - r * half;
    const float2* xr = x + r * N;
    float2* yr = y + r * N;
    const int64_t k = j % Ns;
    double sn, cs;
    sincospi((double)sign * (double)k / (double)Ns, &sn, &cs);
    const float wr = (float)cs, wi = (float)sn;
    const float2 a = xr[j], b = xr[j + half];
    const float2 bw = make_float2(b.x * wr - b.y * wi, b.x * wi + b.y * wr);
    const int64_t o = (j / Ns) * 2 * Ns + k;
    yr[o] = make_float2(a.x + bw.x, a.y + bw.y);
    yr[o + Ns] = make_float2(a.x - bw.x, a.y - bw.y);
  }
}

// Runs the log2 N stages ping-ponging between a and b; returns the buffer holding the result.
float2* fft_rows(float2* a, float2* b, int64_t rows, int64_t N, int sign, hipStream_t s) {
  float2* x = a;
  float2* y = b;
  for (int64_t Ns = 1; Ns < N; Ns <<= 1) {
    k_fft_stage<<<tgrid(rows * (N >> 1)), TB, 0, s>>>(x, y, rows, N, Ns, sign);
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

size_t impulse_ws_bytes(int64_t M, int64_t n_t) { return 2 * al(sizeof(float2) * (size_t)M * n_t); }

size_t signal_ws_bytes(int64_t M, int64_t n_t, int64_t L) {
  const int64_t P = conv_length(n_t, L);
  return 2 * al(sizeof(float2) * (size_t)(M + 1) * P);
}

void impulse_run(int64_t M, int64_t F, double f_lo, double df, int sigma, const float* spectra, int64_t n_t, void* ws,
                 float* h, hipStream_t s) {
  float2* a = (float2*)ws;
  float2* b = (float2*)((char*)ws + al(sizeof(float2) * (size_t)M * n_t));
  k_pad_spectra<<<tgrid(M * n_t), TB, 0, s>>>(spectra, M, F, n_t, a);
  // sum_k H_k e^{-j sigma 2 pi k n / n_t}: forward DFT for sigma = +1, inverse direction for -1
  float2* S = fft_rows(a, b, M, n_t, -sigma, s);
  const double dt = 1.0 / ((double)n_t * df);
  k_carrier<<<tgrid(M * n_t), TB, 0, s>>>(S, M, n_t, f_lo * dt, sigma, 2.0 * df, h);
  ET_HIP(hipGetLastError());
}

void signal_run(int64_t M, int64_t n_t, const float* h, int64_t L, const float* se, double dt, void* ws, float* out,
                hipStream_t s) {
  const int64_t P = conv_length(n_t, L);
  float2* a = (float2*)ws;
  float2* b = (float2*)((char*)ws + al(sizeof(float2) * (size_t)(M + 1) * P));
  k_pad_signals<<<tgrid((M + 1) * P), TB, 0, s>>>(h, M, n_t, se, L, P, a);
  float2* X = fft_rows(a, b, M + 1, P, -1, s);
  k_spectral_product<<<tgrid(M * P), TB, 0, s>>>(X, M, P);
  float2* other = X == a ? b : a;
  float2* Y = fft_rows(X, other, M, P, +1, s);   // only the M product rows
  k_unpack_signal<<<tgrid(M * (n_t + L - 1)), TB, 0, s>>>(Y, M, P, n_t + L - 1, dt / (double)P, out);
  ET_HIP(hipGetLastError());
}

}  // namespace et
