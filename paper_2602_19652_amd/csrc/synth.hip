// Echo synthesis (Eqs. 2-4 specular, 7-8 diffraction) and its adjoint.
//
// For record n (point p, path rtot to it, reflected direction d', material q) and receiver
// m at x_m, with r = rtot + |x_m - p| and f_k = f_lo + k df:
//   H_m[k] += A_nmk exp(j 2 pi sigma f_k r / c)
//   A_nmk = r^-p 10^(-(a0 + a1 f_k) r / 20) * I[b(k)] * D_m[bd(k)]
//   I[b] = k_qb exp(-gamma^2 / (2 beta_qb^2)) (specular),  I_d,qb (diffraction)
// where gamma is the angle between d' and the direction from p to x_m.
//
// Precision: the receiver leg, total path and the delay in cycles at f_lo and per bin are
// FP64 (the phase needs the path to ~1e-8 m at 100-200 kHz); sin/cos/exp2 and the
// accumulation are FP32 (v_sin/v_cos take revolutions, so the FP64 reduction hands them
// a fraction of a cycle).
//
// Two kernels compute the same sum:
//  * factorised (MFMA): with k = 64 k1 + k2, amplitude and phase separate as
//      A e^{j phi} = X[n,k1] * Y[n,k2],
//      X = exp2(base + 64 k1 slope + band(k1)) e^{j 2 pi (c0 + 64 k1 cb)},
//      Y = exp2(k2 slope) e^{j 2 pi k2 cb},
//    whenever the material/directivity bands are constant over each run of 64 bins, so
//    H_m[k1, k2] = sum_n X[n,k1] Y[n,k2] is a complex matrix product contracting over the
//    records.  It runs on the FP32 matrix cores (v_mfma_f32_16x16x4f32); only 128
//    transcendental triples per (record, receiver) remain instead of one per bin.
//  * direct: one sin/cos/exp2 per (record, receiver, bin), any band layout.
// Both write per-chunk partial spectra that a final kernel sums in a fixed order
// (bit-reproducible results).
#include "internal.hpp"

#include <algorithm>
#include <cmath>

namespace et {

namespace {

constexpr double LOG2_10 = 3.32192809488736234787;
constexpr float LOG2E_F = 1.44269504088896340736f;
constexpr float PI_F = 3.14159265358979323846f;

struct SynthArgs {
  int32_t M, F, Q, Bk, Bd, El, Az, sigma;
  double f_lo, df, c, A0, A1, ps;
  const double* rx_pos;
  const double* rx_rot;
  const float* refl_k;
  const float* beta;
  const float* dcoef;
  const float* dir;
  int32_t P;               // record chunks
};

SynthArgs make_args(const et_sim_desc* sim, int32_t P) {
  SynthArgs a;
  a.M = sim->M; a.F = sim->F; a.Q = sim->Q; a.Bk = sim->Bk;
  a.Bd = sim->directivity ? sim->Bd : 0;
  a.El = sim->El; a.Az = sim->Az;
  a.sigma = sim->phase_sign;
  a.f_lo = sim->f_lo;
  a.df = sim->F > 1 ? (sim->f_hi - sim->f_lo) / (double)(sim->F - 1) : 0.0;
  a.c = sim->c; a.A0 = sim->atm_a0; a.A1 = sim->atm_a1; a.ps = sim->spreading_p;
  a.rx_pos = sim->rx_pos; a.rx_rot = sim->rx_rot;
  a.refl_k = sim->refl_k; a.beta = sim->lobe_beta; a.dcoef = sim->diff_coef;
  a.dir = sim->directivity;
  a.P = P;
  return a;
}

// Per (record, receiver) quantities shared by every bin.
struct Pair {
  double c0, cb;     // delay in cycles at f_lo and per bin
  float base;        // log2 amplitude at f_lo without band factors
  float slope;       // log2 amplitude change per bin
  double r, l;
  double u[3];
  float gamma;
  int mat;
  int kind;
};

__device__ inline float dir_gain(const float* tab, int El, int Az, float vx, float vy, float vz) {
  const float az = atan2f(vy, vx);
  const float el = atan2f(vz, hypotf(vx, vy));
  float fa = (az + PI_F) / (2.0f * PI_F) * (float)Az - 0.5f;
  float fe = (el + 0.5f * PI_F) / PI_F * (float)El - 0.5f;
  if (!(fa == fa)) fa = 0.f;   // undefined direction (receiver on the point): any cell, indices stay in range
  if (!(fe == fe)) fe = 0.f;
  const float fl = floorf(fa);
  const float ta = fa - fl;
  int i0 = (int)fl % Az;
  if (i0 < 0) i0 += Az;
  const int i1 = (i0 + 1) % Az;
  int j0, j1;
  float te;
  if (fe <= 0.f) { j0 = j1 = 0; te = 0.f; }
  else if (fe >= (float)(El - 1)) { j0 = j1 = El - 1; te = 0.f; }
  else { j0 = min((int)floorf(fe), El - 1); j1 = min(j0 + 1, El - 1); te = fe - (float)j0; }
  const float a0 = (1.f - ta) * tab[j0 * Az + i0] + ta * tab[j0 * Az + i1];
  const float a1 = (1.f - ta) * tab[j1 * Az + i0] + ta * tab[j1 * Az + i1];
  return (1.f - te) * a0 + te * a1;
}

// Returns false if the record does not contribute (not visible).
__device__ inline bool pair_setup(const SynthArgs& a, const et_paths& P, int64_t n, int m, Pair& q) {
  const uint8_t fl = P.flags[n];
  if (!(fl & 1)) return false;
  q.kind = (fl >> 1) & 1;
  const double px = P.p[3 * n], py = P.p[3 * n + 1], pz = P.p[3 * n + 2];
  const double wx = a.rx_pos[3 * m] - px, wy = a.rx_pos[3 * m + 1] - py, wz = a.rx_pos[3 * m + 2] - pz;
  q.l = sqrt(wx * wx + wy * wy + wz * wz);
  q.u[0] = wx / q.l; q.u[1] = wy / q.l; q.u[2] = wz / q.l;
  q.r = P.rtot[n] + q.l;                                   // emitter -> point -> receiver
  const double sc = (double)a.sigma * q.r / a.c;
  q.c0 = sc * a.f_lo;
  q.cb = sc * a.df;
  q.base = (float)(-a.ps * log2(q.r) - (a.A0 + a.A1 * a.f_lo) * q.r / 20.0 * LOG2_10);
  q.slope = (float)(-a.A1 * a.df * q.r / 20.0 * LOG2_10);
  q.mat = P.mat[n];
  q.gamma = 0.f;
  if (q.kind == 0) {
    const float dx = P.dout[3 * n], dy = P.dout[3 * n + 1], dz = P.dout[3 * n + 2];
    const float ux = (float)q.u[0], uy = (float)q.u[1], uz = (float)q.u[2];
    const float cx = dy * uz - dz * uy, cy = dz * ux - dx * uz, cz = dx * uy - dy * ux;
    q.gamma = atan2f(sqrtf(cx * cx + cy * cy + cz * cz), dx * ux + dy * uy + dz * uz);
  }
  return true;
}

__device__ inline float band_log2(const SynthArgs& a, const Pair& q, int b) {
  if (q.kind == 0) {
    const float bt = a.beta[q.mat * a.Bk + b];
    return log2f(a.refl_k[q.mat * a.Bk + b]) - q.gamma * q.gamma / (2.0f * bt * bt) * LOG2E_F;
  }
  return log2f(a.dcoef[q.mat * a.Bk + b]);
}

// direction of arrival in the receiver frame: v = R_m^T (p - x_m) / l = -R_m^T u
__device__ inline void arrival(const SynthArgs& a, const Pair& q, int m, float& vx, float& vy, float& vz) {
  const double ux = -q.u[0], uy = -q.u[1], uz = -q.u[2];
  if (a.rx_rot) {
    const double* R = a.rx_rot + 9 * m;
    vx = (float)(R[0] * ux + R[3] * uy + R[6] * uz);
    vy = (float)(R[1] * ux + R[4] * uy + R[7] * uz);
    vz = (float)(R[2] * ux + R[5] * uy + R[8] * uz);
  } else {
    vx = (float)ux; vy = (float)uy; vz = (float)uz;
  }
}

__device__ inline double frac(double x) { return x - floor(x); }

__device__ inline void chunk_range(int64_t n_rec, int32_t P, int p, int64_t& lo, int64_t& hi) {
  const int64_t per = (n_rec + P - 1) / P;
  lo = std::min<int64_t>((int64_t)p * per, n_rec);
  hi = std::min<int64_t>(lo + per, n_rec);
}

// ------------------------------------------------------------------ factorised MFMA kernel

constexpr int K2 = 64;        // bins per inner run
constexpr int KT1 = 64;       // outer indices per workgroup
constexpr int RB = 32;        // records per batch (contraction depth per batch)
constexpr int XS = 80;        // LDS row stride (floats): 16-lane groups land on distinct banks
constexpr int BMAX = 16;      // band tables per record held in LDS

typedef float floatx4 __attribute__((ext_vector_type(4)));

struct MfmaLds {
  float X[2][RB][XS];         // X real / imag, [record][k1]
  float Y[2][RB][XS];         // Y real / imag, [record][k2]
  double c0[RB], cb[RB];
  float base[RB], slope[RB];
  float band[RB][BMAX];
  float dirl[RB][BMAX];
  int bk[KT1], bd[KT1];
};

__global__ __launch_bounds__(256) void k_synth_mfma(SynthArgs a, et_paths P, const Ctl* ctl, float* __restrict__ part) {
  __shared__ __align__(16) char smem[sizeof(MfmaLds) > 2 * 64 * 64 * 4 ? sizeof(MfmaLds) : 2 * 64 * 64 * 4];
  MfmaLds& L = *reinterpret_cast<MfmaLds*>(smem);
  const int p = blockIdx.x, m = blockIdx.y, k1t = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K1 = a.F / K2;
  const int k1_0 = k1t * KT1;
  const int nk1 = min(KT1, K1 - k1_0);
  int64_t lo, hi;
  chunk_range(ctl->n_rec, a.P, p, lo, hi);
  if (tid < KT1) {
    const int64_t k = (int64_t)(k1_0 + tid) * K2;
    L.bk[tid] = (int)((k * a.Bk) / a.F);
    L.bd[tid] = a.Bd ? (int)((k * a.Bd) / a.F) : 0;
  }
  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // quadrant of this wave: A from X real (waves 0,1) or imag (2,3); B from Y real (0,2) or imag (1,3)
  const int xa = wv >> 1, yb = wv & 1;

  for (int64_t n0 = lo; n0 < hi; n0 += RB) {
    __syncthreads();   // previous batch fully consumed
    if (tid < RB) {
      const int64_t n = n0 + tid;
      Pair q;
      bool ok = n < hi && pair_setup(a, P, n, m, q);
      if (ok) {
        L.c0[tid] = q.c0;
        L.cb[tid] = q.cb;
        L.base[tid] = q.base;
        L.slope[tid] = q.slope;
        for (int b = 0; b < a.Bk; ++b) L.band[tid][b] = band_log2(a, q, b);
        if (a.Bd) {
          float vx, vy, vz;
          arrival(a, q, m, vx, vy, vz);
          const float* tab = a.dir + (size_t)m * a.Bd * a.El * a.Az;
          for (int b = 0; b < a.Bd; ++b) L.dirl[tid][b] = log2f(dir_gain(tab + (size_t)b * a.El * a.Az, a.El, a.Az, vx, vy, vz));
        }
      } else {
        L.c0[tid] = 0.0;
        L.cb[tid] = 0.0;
        L.base[tid] = -INFINITY;
        L.slope[tid] = 0.f;
        for (int b = 0; b < a.Bk; ++b) L.band[tid][b] = 0.f;
        for (int b = 0; b < a.Bd; ++b) L.dirl[tid][b] = 0.f;
      }
    }
    __syncthreads();
    // generate X[n][k1] and Y[n][k2] for the batch: 2 * RB * 64 values, 16 per thread
#pragma unroll 4
    for (int e = tid; e < 2 * RB * 64; e += 256) {
      const int isY = e >= RB * 64;
      const int ee = isY ? e - RB * 64 : e;
      const int r = ee >> 6, k = ee & 63;
      float amp, rev;
      if (!isY) {
        const int kg = (k1_0 + k) * K2;
        const double cyc = L.c0[r] + (double)kg * L.cb[r];
        rev = (float)frac(cyc);
        float lg = L.base[r] + (float)kg * L.slope[r] + L.band[r][L.bk[k]];
        if (a.Bd) lg += L.dirl[r][L.bd[k]];
        amp = (k < nk1) ? exp2f(lg) : 0.f;
      } else {
        rev = (float)frac((double)k * L.cb[r]);
        amp = exp2f((float)k * L.slope[r]);
        if (L.base[r] == -INFINITY) amp = 0.f;
      }
      const float cr = __builtin_amdgcn_cosf(rev) * amp, ci = __builtin_amdgcn_sinf(rev) * amp;
      if (!isY) { L.X[0][r][k] = cr; L.X[1][r][k] = ci; }
      else { L.Y[0][r][k] = cr; L.Y[1][r][k] = ci; }
    }
    __syncthreads();
    // contraction over the batch's records on the matrix cores
#pragma unroll
    for (int kk = 0; kk < RB; kk += 4) {
      const int rr = kk + (lane >> 4), cc = lane & 15;
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = L.X[xa][rr][i * 16 + cc];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = L.Y[yb][rr][j * 16 + cc];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }
  __syncthreads();
  // combine quadrants: Hr = XrYr - XiYi (waves 0, 3), Hi = XrYi + XiYr (waves 1, 2)
  float* sh = reinterpret_cast<float*>(smem);   // [2][64][64]: waves 3 and 2 deposit theirs
  if (wv >= 2) {
    float* dst = sh + (wv == 3 ? 0 : 64 * 64);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(i * 16 + (lane >> 4) * 4 + v) * 64 + j * 16 + (lane & 15)] = acc[i][j][v];
  }
  __syncthreads();
  if (wv < 2) {
    const float* src = sh + (wv == 0 ? 0 : 64 * 64);
    const float sgn = wv == 0 ? -1.f : 1.f;
    float* out = part + (((size_t)p * a.M + m) * a.F) * 2;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k1 = i * 16 + (lane >> 4) * 4 + v, k2 = j * 16 + (lane & 15);
          if (k1 < nk1) {
            const float val = acc[i][j][v] + sgn * src[k1 * 64 + k2];
            out[(size_t)((k1_0 + k1) * K2 + k2) * 2 + wv] = val;
          }
        }
  }
}

// ------------------------------------------------------------------ direct kernel

constexpr int DB = 256;       // threads
constexpr int DPT = 4;        // bins per thread
constexpr int DTILE = DB * DPT;
constexpr int DRB = 64;       // records per batch
constexpr int DBMAX = 64;

struct DirectLds {
  uint32_t a32[DRB], b32[DRB];
  float base[DRB], slope[DRB];
  float band[DRB][DBMAX];
  float dirl[DRB][DBMAX];
};

__global__ __launch_bounds__(DB) void k_synth_direct(SynthArgs a, et_paths P, const Ctl* ctl, float* __restrict__ part) {
  __shared__ DirectLds L;
  const int p = blockIdx.x, m = blockIdx.y;
  const int tid = threadIdx.x;
  const int kbase = blockIdx.z * DTILE + tid * DPT;
  int64_t lo, hi;
  chunk_range(ctl->n_rec, a.P, p, lo, hi);
  int bk[DPT], bd[DPT];
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int64_t k = kbase + i;
    bk[i] = (int)(((k < a.F ? k : a.F - 1) * a.Bk) / a.F);
    bd[i] = a.Bd ? (int)(((k < a.F ? k : a.F - 1) * a.Bd) / a.F) : 0;
  }
  float re[DPT], im[DPT];
#pragma unroll
  for (int i = 0; i < DPT; ++i) re[i] = im[i] = 0.f;
  for (int64_t n0 = lo; n0 < hi; n0 += DRB) {
    __syncthreads();
    if (tid < DRB) {
      const int64_t n = n0 + tid;
      Pair q;
      if (n < hi && pair_setup(a, P, n, m, q)) {
        // integer phase accumulator (Q0.32 cycles): phase_k = a32 + k b32 mod 2^32
        L.a32[tid] = (uint32_t)(uint64_t)llrint(frac(q.c0) * 4294967296.0);
        L.b32[tid] = (uint32_t)(uint64_t)llrint(frac(q.cb) * 4294967296.0);
        L.base[tid] = q.base;
        L.slope[tid] = q.slope;
        for (int b = 0; b < a.Bk; ++b) L.band[tid][b] = band_log2(a, q, b);
        if (a.Bd) {
          float vx, vy, vz;
          arrival(a, q, m, vx, vy, vz);
          const float* tab = a.dir + (size_t)m * a.Bd * a.El * a.Az;
          for (int b = 0; b < a.Bd; ++b) L.dirl[tid][b] = log2f(dir_gain(tab + (size_t)b * a.El * a.Az, a.El, a.Az, vx, vy, vz));
        }
      } else {
        L.a32[tid] = 0; L.b32[tid] = 0;
        L.base[tid] = -INFINITY; L.slope[tid] = 0.f;
        for (int b = 0; b < a.Bk; ++b) L.band[tid][b] = 0.f;
        for (int b = 0; b < a.Bd; ++b) L.dirl[tid][b] = 0.f;
      }
    }
    __syncthreads();
    const int nb = (int)min<int64_t>(DRB, hi - n0);
    for (int r = 0; r < nb; ++r) {
      const uint32_t A32 = L.a32[r], B32 = L.b32[r];
      const float base = L.base[r], slope = L.slope[r];
#pragma unroll
      for (int i = 0; i < DPT; ++i) {
        const int k = kbase + i;
        const uint32_t ph = A32 + (uint32_t)k * B32;
        const float rev = (float)(int32_t)ph * 2.3283064365386963e-10f;   // 2^-32
        float lg = base + (float)k * slope + L.band[r][bk[i]];
        if (a.Bd) lg += L.dirl[r][bd[i]];
        const float amp = exp2f(lg);
        re[i] += amp * __builtin_amdgcn_cosf(rev);
        im[i] += amp * __builtin_amdgcn_sinf(rev);
      }
    }
  }
  float* out = part + (((size_t)p * a.M + m) * a.F) * 2;
#pragma unroll
  for (int i = 0; i < DPT; ++i) {
    const int k = kbase + i;
    if (k < a.F) { out[2 * k] = re[i]; out[2 * k + 1] = im[i]; }
  }
}

__global__ void k_reduce_partials(const float* __restrict__ part, int32_t P, int64_t MF2, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < MF2; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int p = 0; p < P; ++p) s += part[(size_t)p * MF2 + i];
    out[i] = s;
  }
}

// ------------------------------------------------------------------ adjoint

constexpr int GB = 256;
constexpr int GANCHOR = 32;   // bins between exact re-anchoring of the rotation recurrence

__global__ __launch_bounds__(GB) void k_synth_bwd(SynthArgs a, et_paths P, const Ctl* ctl, const float* __restrict__ g,
                                                 double* __restrict__ gpx, double* __restrict__ gpk) {
  extern __shared__ float2 gl[];   // conj-free copy of dL/dH* for this receiver, [F]
  __shared__ double red[GB];
  __shared__ double kval[16][GB];
  __shared__ int kmat[GB];
  __shared__ double kacc[16 * 16];
  const int p = blockIdx.x, m = blockIdx.y, tid = threadIdx.x;
  for (int k = tid; k < a.F; k += GB) gl[k] = make_float2(g[((size_t)m * a.F + k) * 2], g[((size_t)m * a.F + k) * 2 + 1]);
  for (int i = tid; i < a.Q * a.Bk; i += GB) kacc[i] = 0.0;
  int64_t lo, hi;
  chunk_range(ctl->n_rec, a.P, p, lo, hi);
  double gx0 = 0, gx1 = 0, gx2 = 0;
  const double ln10 = 2.30258509299404568402;
  __syncthreads();
  for (int64_t n0 = lo; n0 < hi; n0 += GB) {
    const int64_t n = n0 + tid;
    double sb[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) sb[b] = 0.0;
    int mat = -1;
    Pair q;
    if (n < hi && pair_setup(a, P, n, m, q)) {
      mat = q.kind == 0 ? q.mat : -1;
      // step of the rotation recurrence: exp2(slope) e^{j 2 pi cb}
      const float wrev = (float)frac(q.cb);
      const float wamp = exp2f(q.slope);
      const float wr = wamp * __builtin_amdgcn_cosf(wrev), wi = wamp * __builtin_amdgcn_sinf(wrev);
      float s1r = 0.f, s1i = 0.f;
      const float fdf = (float)a.df;
      for (int b = 0; b < a.Bk; ++b) {
        const int k0 = (int)(((int64_t)b * a.F + a.Bk - 1) / a.Bk);
        const int k1 = (int)(((int64_t)(b + 1) * a.F + a.Bk - 1) / a.Bk);
        const float blog = band_log2(a, q, b);
        float sbr = 0.f;
        for (int ka = k0; ka < k1; ka += GANCHOR) {
          const int ke = min(ka + GANCHOR, k1);
          const float rev = (float)frac(q.c0 + (double)ka * q.cb);
          const float amp = exp2f(q.base + (float)ka * q.slope + blog);
          float tr = amp * __builtin_amdgcn_cosf(rev), ti = amp * __builtin_amdgcn_sinf(rev);
          float f = (float)(a.f_lo + (double)ka * a.df);
          float c1r = 0.f, c1i = 0.f, c0r = 0.f;
          for (int k = ka; k < ke; ++k) {
            const float2 gg = gl[k];
            const float zr = gg.x * tr + gg.y * ti;   // Re(conj(g) T)
            const float zi = gg.x * ti - gg.y * tr;   // Im(conj(g) T)
            c0r += zr;
            c1r += f * zr;
            c1i += f * zi;
            const float nr = tr * wr - ti * wi;
            ti = tr * wi + ti * wr;
            tr = nr;
            f += fdf;
          }
          sbr += c0r;
          s1r += c1r;
          s1i += c1i;
        }
#pragma unroll
        for (int bb = 0; bb < 16; ++bb)
          if (bb == b) sb[bb] = (double)sbr;
      }
      double s0 = 0;
#pragma unroll
      for (int b = 0; b < 16; ++b)
        if (b < a.Bk) s0 += sb[b];
      // d(ln A + j phi)/dx_m = [(-p/r - ln10 (a0 + a1 f)/20) + j sigma 2 pi f / c] u - d(gamma^2)/dx / (2 beta^2)
      const double cu = (-a.ps / q.r - ln10 * a.A0 / 20.0) * s0 - ln10 * a.A1 / 20.0 * (double)s1r -
                        (double)a.sigma * 2.0 * M_PI / a.c * (double)s1i;
      double g0 = 2.0 * cu * q.u[0], g1 = 2.0 * cu * q.u[1], g2 = 2.0 * cu * q.u[2];
      if (q.kind == 0) {
        const double dx = P.dout[3 * n], dy = P.dout[3 * n + 1], dz = P.dout[3 * n + 2];
        const double dnn = sqrt(dx * dx + dy * dy + dz * dz);
        const double hx = dx / dnn, hy = dy / dnn, hz = dz / dnn;
        const double cg = hx * q.u[0] + hy * q.u[1] + hz * q.u[2];
        const double qx = hy * q.u[2] - hz * q.u[1], qy = hz * q.u[0] - hx * q.u[2], qz = hx * q.u[1] - hy * q.u[0];
        const double sg = sqrt(qx * qx + qy * qy + qz * qz);
        const double gam = atan2(sg, cg);
        const double ratio = gam < 1e-8 ? 2.0 : 2.0 * gam / sg;
        // d(gamma^2)/dx = -(2 gamma / sin gamma) (d' - cos(gamma) u) / l
        const double d0 = -ratio * (hx - cg * q.u[0]) / q.l, d1 = -ratio * (hy - cg * q.u[1]) / q.l,
                     d2 = -ratio * (hz - cg * q.u[2]) / q.l;
        double wsum = 0.0;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          if (b < a.Bk) {
            const double bt = (double)a.beta[q.mat * a.Bk + b];
            wsum += sb[b] / (2.0 * bt * bt);
          }
        }
        g0 -= 2.0 * wsum * d0; g1 -= 2.0 * wsum * d1; g2 -= 2.0 * wsum * d2;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          double kv = b < a.Bk ? (double)a.refl_k[q.mat * a.Bk + b] : 0.0;
          sb[b] = kv != 0.0 ? 2.0 * sb[b] / kv : 0.0;
        }
      }
      gx0 += g0; gx1 += g1; gx2 += g2;
    }
    // deterministic per-batch reduction of the band-coefficient gradient by material
    kmat[tid] = mat;
#pragma unroll
    for (int b = 0; b < 16; ++b) kval[b][tid] = sb[b];
    __syncthreads();
    for (int i = tid; i < a.Q * a.Bk; i += GB) {
      const int qq = i / a.Bk, b = i % a.Bk;
      double s = 0.0;
      for (int t = 0; t < GB; ++t)
        if (kmat[t] == qq) s += kval[b][t];
      kacc[i] += s;
    }
    __syncthreads();
  }
  // receiver gradient: block tree reduction
  const double gv[3] = {gx0, gx1, gx2};
  for (int c = 0; c < 3; ++c) {
    red[tid] = gv[c];
    __syncthreads();
    for (int s = GB / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) gpx[((size_t)p * a.M + m) * 3 + c] = red[0];
    __syncthreads();
  }
  for (int i = tid; i < a.Q * a.Bk; i += GB) gpk[((size_t)p * a.M + m) * a.Q * a.Bk + i] = kacc[i];
}

__global__ void k_bwd_reduce(const double* __restrict__ gpx, const double* __restrict__ gpk, int32_t P, int32_t M,
                             int32_t QB, double* __restrict__ grad_k, double* __restrict__ grad_x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < QB) {
    double s = 0.0;
    for (int p = 0; p < P; ++p)
      for (int m = 0; m < M; ++m) s += gpk[((size_t)p * M + m) * QB + i];
    grad_k[i] = s;
  }
  if (i < M * 3) {
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += gpx[(size_t)p * M * 3 + i];
    grad_x[i] = s;
  }
}

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

int choose_P(const et_sim_desc* sim, int64_t cap, bool mfma) {
  // enough workgroups to fill 256 CUs several times over, records per chunk >= a few batches
  const int64_t tiles = mfma ? (int64_t)sim->M * std::max<int64_t>(1, (sim->F / K2 + KT1 - 1) / KT1)
                             : (int64_t)sim->M * ((sim->F + DTILE - 1) / DTILE);
  int64_t P = std::max<int64_t>(1, (2048 + tiles - 1) / tiles);
  P = std::min<int64_t>(P, std::max<int64_t>(1, cap / 256));
  return (int)std::min<int64_t>(P, 256);
}

}  // namespace

bool synth_factorised_ok(const et_sim_desc* sim) {
  if (sim->flags & ET_SYNTH_DIRECT) return false;
  if (sim->F < K2 || sim->F % K2) return false;
  if (sim->Bk > BMAX) return false;
  if (sim->directivity && sim->Bd > BMAX) return false;
  const int K1 = sim->F / K2;
  for (int k1 = 0; k1 < K1; ++k1) {
    const int64_t ka = (int64_t)k1 * K2, kb = ka + K2 - 1;
    if ((ka * sim->Bk) / sim->F != (kb * sim->Bk) / sim->F) return false;
    if (sim->directivity && (ka * sim->Bd) / sim->F != (kb * sim->Bd) / sim->F) return false;
  }
  return true;
}

size_t synth_ws_layout(const et_sim_desc* sim, int64_t cap, char* base, SynthWS* ws) {
  const bool mf = synth_factorised_ok(sim);
  const int P = choose_P(sim, cap, mf);
  size_t off = 0;
  SynthWS w{};
  w.P = P;
  w.partial = (float*)(base ? base + off : nullptr);
  off += al(sizeof(float) * 2 * (size_t)P * sim->M * sim->F);
  if (ws) *ws = w;
  return off;
}

int synth_run(const et_sim_desc* sim, const et_paths* paths, const SynthWS& ws, Ctl* ctl, float* spectra, hipStream_t s) {
  const bool mf = synth_factorised_ok(sim);
  SynthArgs a = make_args(sim, ws.P);
  const et_paths P = *paths;
  if (mf) {
    const int K1 = sim->F / K2;
    dim3 grid(ws.P, sim->M, (K1 + KT1 - 1) / KT1);
    k_synth_mfma<<<grid, 256, 0, s>>>(a, P, ctl, ws.partial);
  } else {
    dim3 grid(ws.P, sim->M, (sim->F + DTILE - 1) / DTILE);
    k_synth_direct<<<grid, DB, 0, s>>>(a, P, ctl, ws.partial);
  }
  const int64_t MF2 = (int64_t)sim->M * sim->F * 2;
  k_reduce_partials<<<(unsigned)std::min<int64_t>((MF2 + 255) / 256, 4096), 256, 0, s>>>(ws.partial, ws.P, MF2, spectra);
  ET_HIP(hipGetLastError());
  return mf ? 1 : 2;
}

size_t synth_bwd_ws_layout(const et_sim_desc* sim, int64_t cap, char* base, SynthWS* ws) {
  const int64_t tiles = sim->M;
  int64_t P = std::max<int64_t>(1, (1024 + tiles - 1) / tiles);
  P = std::min<int64_t>(P, std::max<int64_t>(1, (cap + GB - 1) / GB));
  P = std::min<int64_t>(P, 256);
  size_t off = 0;
  SynthWS w{};
  w.gchunks = (int)P;
  w.gpart_x = (double*)(base ? base + off : nullptr);
  off += al(sizeof(double) * 3 * (size_t)P * sim->M);
  w.gpart_k = (double*)(base ? base + off : nullptr);
  off += al(sizeof(double) * (size_t)P * sim->M * sim->Q * sim->Bk);
  if (ws) *ws = w;
  return off;
}

void synth_bwd_run(const et_sim_desc* sim, const et_paths* paths, const float* grad_spectra, const SynthWS& ws,
                   Ctl* ctl, double* grad_k, double* grad_rx, hipStream_t s) {
  SynthArgs a = make_args(sim, ws.gchunks);
  const et_paths P = *paths;
  dim3 grid(ws.gchunks, sim->M);
  const size_t shm = sizeof(float2) * (size_t)sim->F;
  k_synth_bwd<<<grid, GB, shm, s>>>(a, P, ctl, grad_spectra, ws.gpart_x, ws.gpart_k);
  const int QB = sim->Q * sim->Bk;
  const int n = std::max(QB, sim->M * 3);
  k_bwd_reduce<<<(n + 255) / 256, 256, 0, s>>>(ws.gpart_x, ws.gpart_k, ws.gchunks, sim->M, QB, grad_k, grad_rx);
  ET_HIP(hipGetLastError());
}

}  // namespace et
