// Ray sets by the recursive zonal equal-area partition EQ(2, N) of the sphere (Sec. III-C,
// after Leopardi 2006): two polar caps of the region area A = 4 pi / N and n collars of equal
// angular height between them; collar i holds the rounded share of the cumulative ideal
// count, so the first i collars hold M_i = round(Y_i) regions with
// Y_i = N sin^2((theta_c + i delta) / 2) - 1 (rounding each collar's ideal count with the
// error carried into the next one gives these same cumulative counts).  Halves round down,
// and so do values within N 2^-36 above a half: a boundary on the equator has Y exactly
// (N - 2) / 2, which floating point puts on either side of the half.  Every zone
// boundary sits at the colatitude whose cap holds exactly its regions.  Region centres: the
// middle colatitude of the collar and longitudes 2 pi ((j + 1/2) / m + offset_i), where each
// collar is turned against the one above it by Leopardi's twist.
//
// Three launches: the collar table (one thread per collar), the twist prefix (one
// workgroup), the centres (one thread per direction).
#include "internal.hpp"

#include <algorithm>
#include <cmath>

namespace et {

namespace {

constexpr int EB = 256;
constexpr int SCAN_THREADS = 1024;

__device__ inline double cap_angle_of(double frac) {   // colatitude of the cap holding frac of the sphere
  return 2.0 * asin(fmin(1.0, sqrt(frac)));
}

__device__ inline int64_t gcd64(int64_t a, int64_t b) {
  while (b) { const int64_t t = a % b; a = b; b = t; }
  return a;
}

// Mcum[i] for i = 0..n: regions in the first i collars.
__global__ void k_eq_table(int64_t N, int64_t n, double theta_c, double delta, int64_t* __restrict__ Mcum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  int64_t M;
  if (i == 0) M = 0;
  else if (i == n) M = N - 2;
  else {
    const double s = sin(0.5 * (theta_c + (double)i * delta));
    M = (int64_t)floor((double)N * s * s - 1.0 + 0.5 - (double)N * 0x1p-36);
  }
  Mcum[i] = M;
}

// thmid[i]: middle colatitude of collar i (1..n); cut: the last collar whose centres lie
// within the cone (colatitudes increase with i).
__global__ void k_eq_mid(int64_t N, int64_t n, double half_angle, const int64_t* __restrict__ Mcum,
                         double* __restrict__ thmid, unsigned long long* cut) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (i > n) return;
  const double top = cap_angle_of((double)(1 + Mcum[i - 1]) / (double)N);
  const double bot = cap_angle_of((double)(1 + Mcum[i]) / (double)N);
  const double t = 0.5 * (top + bot);
  thmid[i] = t;
  if (t <= half_angle) atomicMax(cut, (unsigned long long)i);
}

// offs[i] = sum over collars l < i of the twist between collars l and l + 1 (offs[1] = 0),
// by one workgroup: each thread sums a run of collars, then a scan over the threads.
__global__ void __launch_bounds__(SCAN_THREADS) k_eq_twist(int64_t n, const int64_t* __restrict__ Mcum,
                                                          double* __restrict__ offs) {
  __shared__ double part[SCAN_THREADS];
  const int tid = threadIdx.x;
  const int64_t per = (n + SCAN_THREADS - 1) / SCAN_THREADS;
  const int64_t lo = 1 + (int64_t)tid * per, hi = std::min<int64_t>(n, lo + per - 1);
  auto twist = [&](int64_t l) {   // collar l (top) against collar l + 1 (bottom)
    const int64_t a = Mcum[l] - Mcum[l - 1], b = Mcum[l + 1] - Mcum[l];
    if (a <= 0 || b <= 0) return 0.0;   // (no collar of EQ(2, N) is empty; kept finite regardless)
    return (1.0 / (double)b - 1.0 / (double)a) / 2.0 + (double)gcd64(a, b) / (2.0 * (double)a * (double)b);
  };
  double s = 0.0;
  for (int64_t l = lo; l <= hi && l < n; ++l) s += twist(l);
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < SCAN_THREADS; d <<= 1) {   // inclusive Hillis-Steele scan
    const double v = tid >= d ? part[tid - d] : 0.0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  double run = tid > 0 ? part[tid - 1] : 0.0;
  for (int64_t l = lo; l <= hi; ++l) {
    offs[l] = run - floor(run);
    if (l < n) run += twist(l);
  }
}

__global__ void k_eq_points(int64_t N, int64_t n, int64_t count, const int64_t* __restrict__ Mcum,
                            const double* __restrict__ thmid, const double* __restrict__ offs,
                            float* __restrict__ dirs) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  double t, p = 0.0;
  if (j == 0) t = 0.0;
  else if (j == N - 1) t = M_PI;
  else {
    int64_t a = 1, b = n;   // smallest collar i with Mcum[i] >= j
    while (a < b) {
      const int64_t c = (a + b) >> 1;
      if (Mcum[c] >= j) b = c; else a = c + 1;
    }
    const int64_t m = Mcum[a] - Mcum[a - 1], jj = j - 1 - Mcum[a - 1];
    t = thmid[a];
    const double u = ((double)jj + 0.5) / (double)m + offs[a];
    p = 2.0 * M_PI * (u - floor(u));
  }
  double st, ct, sp, cp;
  sincos(t, &st, &ct);
  sincos(p, &sp, &cp);
  dirs[3 * j + 0] = (float)ct;
  dirs[3 * j + 1] = (float)(st * cp);
  dirs[3 * j + 2] = (float)(st * sp);
}

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }
inline unsigned grid(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + EB - 1) / EB); }

}  // namespace

EqPlan eq_plan(int64_t N) {
  EqPlan p;
  p.N = N;
  if (N <= 2) return p;   // one region, or two hemispheres: caps only
  const double A = 4.0 * M_PI / (double)N;
  p.theta_c = 2.0 * std::asin(std::sqrt(1.0 / (double)N));
  p.n = std::max<int64_t>(
      1, (int64_t)std::floor((M_PI - 2.0 * p.theta_c) / std::sqrt(A) + 0.5 - (double)N * 0x1p-36));
  p.delta = (M_PI - 2.0 * p.theta_c) / (double)p.n;
  return p;
}

size_t eq_ws_bytes(const EqPlan& p) {
  return al(sizeof(int64_t) * (p.n + 2)) + 2 * al(sizeof(double) * (p.n + 2)) + al(sizeof(unsigned long long));
}

int64_t eq_count(const EqPlan& p, double half_angle, void* ws, hipStream_t s) {
  const int64_t N = p.N;
  if (N == 1) return 1;
  if (N == 2) return half_angle >= M_PI ? 2 : 1;
  char* w = (char*)ws;
  int64_t* Mcum = (int64_t*)w;
  double* thmid = (double*)(w + al(sizeof(int64_t) * (p.n + 2)));
  double* offs = (double*)((char*)thmid + al(sizeof(double) * (p.n + 2)));
  unsigned long long* cut = (unsigned long long*)((char*)offs + al(sizeof(double) * (p.n + 2)));
  k_eq_table<<<grid(p.n + 1), EB, 0, s>>>(N, p.n, p.theta_c, p.delta, Mcum);
  ET_HIP(hipMemsetAsync(cut, 0, sizeof(unsigned long long), s));
  k_eq_mid<<<grid(p.n), EB, 0, s>>>(N, p.n, half_angle, Mcum, thmid, cut);
  k_eq_twist<<<1, SCAN_THREADS, 0, s>>>(p.n, Mcum, offs);
  ET_HIP(hipGetLastError());
  unsigned long long hc = 0;
  int64_t hm = 0;
  ET_HIP(hipMemcpyAsync(&hc, cut, sizeof(hc), hipMemcpyDeviceToHost, s));
  ET_HIP(hipStreamSynchronize(s));
  if (hc > 0) ET_HIP(hipMemcpy(&hm, Mcum + hc, sizeof(int64_t), hipMemcpyDeviceToHost));
  return 1 + hm + (half_angle >= M_PI ? 1 : 0);
}

void eq_points(const EqPlan& p, int64_t count, void* ws, float* dirs, hipStream_t s) {
  char* w = (char*)ws;
  int64_t* Mcum = (int64_t*)w;
  double* thmid = (double*)(w + al(sizeof(int64_t) * (p.n + 2)));
  double* offs = (double*)((char*)thmid + al(sizeof(double) * (p.n + 2)));
  k_eq_points<<<grid(count), EB, 0, s>>>(p.N, p.n, count, Mcum, thmid, offs, dirs);
  ET_HIP(hipGetLastError());
}

}  // namespace et
