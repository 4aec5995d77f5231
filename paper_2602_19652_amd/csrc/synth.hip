// Echo synthesis (Eqs. 2-4 specular, 7-8 diffraction) and its adjoint.
//
// For record n (point p, path rtot to it, reflected direction d', material q) and receiver
// m at x_m, with r = rtot + |x_m - p| and f_k = f_lo + k df:
//   H_m[k] += A_nmk exp(j 2 pi sigma f_k r / c)
//   A_nmk = r^-p 10^(-(a0 + a1 f_k) r / 20) * I[b(k)] * D_m[bd(k)]
//   I[b] = k_qb exp(-gamma^2 / (2 beta_qb^2)) (specular),  I_d,qb (diffraction),  I_p,b (passive)
// where gamma is the angle between d' and the direction from p to x_m.  Records whose
// line-of-sight ray was blocked contribute nothing; a first pass compacts the indices of
// the visible records so that no kernel spends work on the others.  Two alternative
// readings switch per pose: the path product (k_qb replaced by the product of k over the
// ray's reflections so far, through per-record band tables) and per-receiver line of sight
// (a record reaches receiver m only when its bit m is set).
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
//    records.  It runs on the f16 matrix cores (v_mfma_f32_16x16x32_f16) with every FP32
//    operand split into two f16 halves and three half products per real product (FP32
//    accumulation); X and Y themselves come from 32 exp2/sin/cos factors per (record,
//    receiver) (a second 8 x 8 split) plus the band factors (one exp2 per band segment, or
//    folded into the first factor when the band edges fall on groups of 8 outer indices),
//    so only about 40 transcendental triples remain of the 4096 per (record, receiver) of a
//    4096-bin grid.
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
  double kc0, kcb;         // sigma f_lo / c and sigma df / c: cycles per metre of path
  double kbase, kslope;    // log2 absorption per metre at f_lo and per bin
  const float* lk;         // [Q][Bk] log2 k
  const float* lc;         // [Q][Bk] log2(e) / (2 beta^2)
  const float* ld;         // [Q][Bk] log2 I_d
  const float* pcoef;      // [Bk] passive source magnitude I_p (NULL without the passive component)
  const float* lp;         // [Bk] log2 I_p
  const float* lmax;       // [3 Q + 1] per material: max_b log2 k, min_b lobe coefficient, max_b log2 I_d;
                           // then max_b log2 I_p (bounds on the band factors, used with rec_rows 0)
  int32_t rec_rows;        // 1 (path-product reading): lk, lc, ld have a row per record and a
                           // record's `mat` in the kernels is its index; 0: a row per material
  const uint64_t* rxv;     // per-receiver line of sight [records] (NULL: the records' visible bit)
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
  a.kc0 = (double)a.sigma * a.f_lo / a.c;
  a.kcb = (double)a.sigma * a.df / a.c;
  a.kbase = -(a.A0 + a.A1 * a.f_lo) / 20.0 * LOG2_10;
  a.kslope = -a.A1 * a.df / 20.0 * LOG2_10;
  a.pcoef = (sim->flags & ET_PASSIVE) ? sim->passive_coef : nullptr;
  a.lk = a.lc = a.ld = a.lp = a.lmax = nullptr;
  a.rec_rows = 0;
  a.rxv = nullptr;
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
  int mat;           // row of the band tables: the material, or the record (rec_rows)
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

// The gain of dir_gain and its gradient (gx, gy, gz) with respect to the direction v: the
// derivative of the bilinear interpolant inside the cell that holds v, through
// fa = (az + pi) Az / 2pi - 1/2, fe = (el + pi/2) El / pi - 1/2, az = atan2(y, x) and
// el = atan2(z, rho); zero across the clamped elevation rows and on the poles.
__device__ inline float dir_gain_dv(const float* tab, int El, int Az, float vx, float vy, float vz, float& gx,
                                    float& gy, float& gz) {
  const float az = atan2f(vy, vx);
  const float rho2 = vx * vx + vy * vy, rho = sqrtf(rho2);
  const float el = atan2f(vz, rho);
  float fa = (az + PI_F) / (2.0f * PI_F) * (float)Az - 0.5f;
  float fe = (el + 0.5f * PI_F) / PI_F * (float)El - 0.5f;
  if (!(fa == fa)) fa = 0.f;
  if (!(fe == fe)) fe = 0.f;
  const float fl = floorf(fa);
  const float ta = fa - fl;
  int i0 = (int)fl % Az;
  if (i0 < 0) i0 += Az;
  const int i1 = (i0 + 1) % Az;
  int j0, j1;
  float te;
  bool inner = false;
  if (fe <= 0.f) { j0 = j1 = 0; te = 0.f; }
  else if (fe >= (float)(El - 1)) { j0 = j1 = El - 1; te = 0.f; }
  else { j0 = min((int)floorf(fe), El - 1); j1 = min(j0 + 1, El - 1); te = fe - (float)j0; inner = true; }
  const float t00 = tab[j0 * Az + i0], t01 = tab[j0 * Az + i1], t10 = tab[j1 * Az + i0], t11 = tab[j1 * Az + i1];
  const float a0 = (1.f - ta) * t00 + ta * t01;
  const float a1 = (1.f - ta) * t10 + ta * t11;
  const float daz = ((1.f - te) * (t01 - t00) + te * (t11 - t10)) * (float)Az / (2.0f * PI_F);
  const float del = inner ? (a1 - a0) * (float)El / PI_F : 0.f;
  const float n2 = rho2 + vz * vz;
  if (rho2 > 0.f && n2 > 0.f) {
    gx = -daz * vy / rho2 - del * vx * vz / (rho * n2);
    gy = daz * vx / rho2 - del * vy * vz / (rho * n2);
    gz = del * rho / n2;
  } else {
    gx = gy = gz = 0.f;
  }
  return (1.f - te) * a0 + te * a1;
}

// Returns false if the record does not contribute to receiver m (not visible, hidden from
// receiver m under the per-receiver line of sight, or a passive record of another receiver).
__device__ inline bool pair_setup(const SynthArgs& a, const et_paths& P, int64_t n, int m, Pair& q) {
  const uint8_t fl = P.flags[n];
  if (!(fl & 1)) return false;
  if (a.rxv && !((a.rxv[n] >> m) & 1ull)) return false;   // per-receiver line of sight
  q.kind = (fl >> 1) & 3;
  if (q.kind == 2 && P.mat[n] != m) return false;
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
  q.mat = a.rec_rows ? (int)n : P.mat[n];
  q.gamma = 0.f;
  if (q.kind == 0) {
    const float dx = P.dout[3 * n], dy = P.dout[3 * n + 1], dz = P.dout[3 * n + 2];
    const float ux = (float)q.u[0], uy = (float)q.u[1], uz = (float)q.u[2];
    const float cx = dy * uz - dz * uy, cy = dz * ux - dx * uz, cz = dx * uy - dy * ux;
    q.gamma = atan2f(sqrtf(cx * cx + cy * cy + cz * cz), dx * ux + dy * uy + dz * uz);
  }
  return true;
}

// log2 of the band factor: k exp(-gamma^2 / (2 beta^2)) (specular), I_d (diffraction) or
// I_p (passive)
// KFREE: specular records without the factor k (the adjoint's dH/dk, H being linear in k).
template <bool KFREE = false>
__device__ inline float band_log2_v(const SynthArgs& a, int kind, int mat, float gamma, int b) {
  const int64_t i = (int64_t)mat * a.Bk + b;
  return kind == 0 ? (KFREE ? 0.f : a.lk[i]) - gamma * gamma * a.lc[i] : kind == 1 ? a.ld[i] : a.lp[b];
}

__device__ inline void band_table_entry(const SynthArgs& a, int i, float* lk, float* lc, float* ld, float* lp) {
  const float bt = a.beta[i];
  lk[i] = log2f(a.refl_k[i]);
  lc[i] = LOG2E_F / (2.0f * bt * bt);
  ld[i] = log2f(a.dcoef[i]);
  if (i < a.Bk) lp[i] = a.pcoef ? log2f(a.pcoef[i]) : -INFINITY;
}

// Per-material bounds of material q (and, for q = 0, of the passive factors) from the same
// expressions as the table entries, so that each bound equals the extreme of its entries.
__device__ inline void band_bound_entry(const SynthArgs& a, int q, float* lmax) {
  float mk = -INFINITY, mc = INFINITY, md = -INFINITY;
  for (int b = 0; b < a.Bk; ++b) {
    const int i = q * a.Bk + b;
    const float bt = a.beta[i];
    mk = fmaxf(mk, log2f(a.refl_k[i]));
    mc = fminf(mc, LOG2E_F / (2.0f * bt * bt));
    md = fmaxf(md, log2f(a.dcoef[i]));
  }
  lmax[q] = mk;
  lmax[a.Q + q] = mc;
  lmax[2 * a.Q + q] = md;
  if (q == 0) {
    float mp = -INFINITY;
    if (a.pcoef)
      for (int b = 0; b < a.Bk; ++b) mp = fmaxf(mp, log2f(a.pcoef[b]));
    lmax[3 * a.Q] = mp;
  }
}

__global__ void k_band_tables(SynthArgs a, float* lk, float* lc, float* ld, float* lp, float* lmax) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.Q) band_bound_entry(a, i, lmax);
  if (i >= a.Q * a.Bk) return;
  band_table_entry(a, i, lk, lc, ld, lp);
}

__device__ inline float band_log2(const SynthArgs& a, const Pair& q, int b) {
  return band_log2_v(a, q.kind, q.mat, q.gamma, b);
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

__device__ inline void chunk_range(int64_t n, int32_t P, int p, int64_t& lo, int64_t& hi) {
  const int64_t per = (n + P - 1) / P;
  lo = std::min<int64_t>((int64_t)p * per, n);
  hi = std::min<int64_t>(lo + per, n);
}

// Chunks of a fused batch: the visible records are sorted by job, job j owns positions
// [lo[j], hi[j]) and chunks [off[j], off[j + 1]) of at most `per` records each, so no chunk
// mixes jobs.  off[J] is the batch's chunk count.
struct ChunkTab {
  const int64_t* off;   // [J + 1]
  const int64_t* lo;    // [J]
  const int64_t* hi;    // [J]
  const int64_t* per;   // [1]
  int32_t J;
};

// Resolves chunk c to its job and record range; false if c is past the batch's chunks.
__device__ inline bool batch_chunk(const ChunkTab& ct, int64_t c, int& j, int64_t& lo, int64_t& hi) {
  if (c >= ct.off[ct.J]) return false;
  int a = 0, b = ct.J - 1;   // last job with off <= c (jobs without chunks share off with the next)
  while (a < b) {
    const int mid = (a + b + 1) >> 1;
    if (ct.off[mid] <= c) a = mid;
    else b = mid - 1;
  }
  j = a;
  lo = ct.lo[a] + (c - ct.off[a]) * ct.per[0];
  hi = std::min<int64_t>(lo + ct.per[0], ct.hi[a]);
  return true;
}

// Common prologue: the workgroup's arguments and record range, plain or batched.
// Workgroup -> (record chunk, receiver, tile).  Workgroups reach the eight XCDs in turn (linear
// id mod 8).  With a chunk count that is a multiple of 8 the linear id reads as (chunk group,
// receiver and tile, XCD): every XCD works through its chunks one at a time with all receivers
// and tiles of a chunk together, so they share that XCD's L2 for the chunk's records.  Other
// chunk counts keep the grid's own coordinates.
__device__ inline void block_coords(int& p, int& m, int& t) {
  const int64_t nx = gridDim.x, ny = gridDim.y, nz = gridDim.z;
  if (nx % 8 != 0) {
    p = blockIdx.x; m = blockIdx.y; t = blockIdx.z;
    return;
  }
  const int64_t L = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const int64_t q = L >> 3, inner = ny * nz;
  const int64_t mt = q % inner;
  p = (int)((q / inner) * 8 + (L & 7));
  m = (int)(mt % ny);
  t = (int)(mt / ny);
}

#define SYNTH_RESOLVE()                                                      \
  int bp, bm, bt;                                                            \
  block_coords(bp, bm, bt);                                                  \
  SynthArgs a = a0;                                                          \
  int64_t lo, hi;                                                            \
  int jb = 0;                                                                \
  if (BATCH) {                                                               \
    if (!batch_chunk(ct, bp, jb, lo, hi)) return;                            \
    a = jobs[jb];                                                            \
  } else {                                                                   \
    chunk_range(ctl->n_vis, a.P, bp, lo, hi);                                \
  }

// ------------------------------------------------------------------ visible-record list

__global__ void k_vis_flags(et_paths P, const Ctl* ctl, uint64_t* __restrict__ flags) {
  const int64_t n = ctl->n_rec;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = (P.flags[i] & 1) ? 1ull : 0ull;
}

__global__ void k_vis_scatter(const uint64_t* __restrict__ flags, const uint64_t* __restrict__ offs, const Ctl* ctl,
                              int32_t* __restrict__ idx) {
  const int64_t n = ctl->n_rec;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (flags[i]) idx[offs[i]] = (int32_t)i;
}

__global__ void k_vis_count(Ctl* ctl) { ctl->n_vis = (int64_t)ctl->tot[3]; }
__global__ void k_vis_all(Ctl* ctl) { ctl->n_vis = ctl->n_rec; }   // no list: the kernels walk every record

// ------------------------------------------------------------------ factorised MFMA kernel

constexpr int K2 = 64;        // bins per inner run (k = 64 k1 + k2)
constexpr int KT1 = 64;       // outer indices per workgroup
constexpr int RB = 32;        // records per stage (contraction depth per stage)
constexpr int RPW = RB / 4;   // records per wave and stage
constexpr int SMAX = 16;      // band segments (runs of equal material and directivity band) per 64-row tile

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline uint32_t q32(double cyc) {   // fraction of a cycle in Q0.32 (mod 2^32)
  return (uint32_t)((cyc - floor(cyc)) * 4294967296.0);   // in [0, 2^32]; the conversion saturates
}

// Lean per-(record, receiver) setup: FP64 only for the receiver leg, the path and the delay
// reductions.  Phases of the generated values are integer phase accumulators in Q0.32
// (a32 + k1 bx32 for X, k2 by32 for Y), exact mod 1 up to the quantisation of the steps
// (<= 128 * 2^-33 cycles).
struct PairLean {
  uint32_t a32, bx32, by32;
  float base, slope, gamma;
  float vx, vy, vz;
  int mat, kind;         // mat: row of the band tables (the material, or the record: rec_rows)
  float lbm;             // bound on the log2 band factor (with directivity) over every band: the
                         // generating factors carry it, so Xa stays below the record's bound and
                         // the per-segment factors below 1
  // GRAD: receiver-gradient coefficients, d/dx_m of (ln A + j phi) = (c1 + c2 f + j c3 f) u - lobe
  float gux, guy, guz;   // u = (x_m - p) / l
  float gc1;             // -p / r - ln10 a0 / 20
  float glx, gly, glz;   // 2 (gamma / sin gamma) (d' - cos(gamma) u) / l (specular; 0 otherwise)
};

// GRAD: the adjoint's set-up (receiver-gradient coefficients; band factors without k).  dmax: the
// receiver's largest log2 directivity gain (0 without directivity).
template <bool GRAD = false>
__device__ inline void pair_lean(const SynthArgs& a, const et_paths& P, const int32_t* __restrict__ idx, int64_t e,
                                 int64_t hi, int m, PairLean& q, float dmax = 0.f) {
  q.a32 = q.bx32 = q.by32 = 0;
  q.base = -INFINITY;
  q.lbm = 0.f;
  q.slope = q.gamma = q.vx = q.vy = q.vz = 0.f;
  q.mat = q.kind = 0;
  if (GRAD) q.gux = q.guy = q.guz = q.gc1 = q.glx = q.gly = q.glz = 0.f;
  if (e >= hi) return;
  const int64_t n = idx ? (int64_t)idx[e] : e;   // no list: every record (hidden ones skipped here)
  const uint8_t fl = P.flags[n];
  if (!(fl & 1)) return;
  if (a.rxv && !((a.rxv[n] >> m) & 1ull)) return;   // per-receiver line of sight
  const int kind = (fl >> 1) & 3;
  if (kind == 2 && P.mat[n] != m) return;   // a passive record reaches its own receiver only
  q.kind = kind;
  const double wx = a.rx_pos[3 * m] - P.p[3 * n], wy = a.rx_pos[3 * m + 1] - P.p[3 * n + 1],
               wz = a.rx_pos[3 * m + 2] - P.p[3 * n + 2];
  const double l = sqrt(wx * wx + wy * wy + wz * wz);
  const double r = P.rtot[n] + l;                          // emitter -> point -> receiver
  const double cb = r * a.kcb;
  q.a32 = q32(r * a.kc0);
  q.bx32 = q32((double)K2 * cb);
  q.by32 = q32(cb);
  q.base = -(float)a.ps * log2f((float)r) + (float)(r * a.kbase);
  q.slope = (float)(r * a.kslope);
  q.mat = a.rec_rows ? (int)n : P.mat[n];
  const double il = 1.0 / l;
  const float ux = (float)(wx * il), uy = (float)(wy * il), uz = (float)(wz * il);
  if (q.kind == 0) {
    const float dx = P.dout[3 * n], dy = P.dout[3 * n + 1], dz = P.dout[3 * n + 2];
    const float cx = dy * uz - dz * uy, cy = dz * ux - dx * uz, cz = dx * uy - dy * ux;
    const float sc = sqrtf(cx * cx + cy * cy + cz * cz), cc = dx * ux + dy * uy + dz * uz;
    q.gamma = atan2f(sc, cc);
    if (GRAD) {
      // d(gamma^2)/dx_m = -(2 gamma / sin gamma) (h - cos(gamma) u) / l with h = d' / |d'|
      const float idn = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
      const float sg = sc * idn, cg = cc * idn;
      const float ratio = q.gamma < 1e-4f ? 2.0f : 2.0f * q.gamma / sg;
      const float c = ratio * (float)(2.0 * il);
      q.glx = c * (dx * idn - cg * ux);
      q.gly = c * (dy * idn - cg * uy);
      q.glz = c * (dz * idn - cg * uz);
    }
  }
  if (GRAD) {
    q.gux = ux; q.guy = uy; q.guz = uz;
    q.gc1 = (float)(-a.ps / r - 2.30258509299404568402 * a.A0 / 20.0);
  }
  if (a.Bd) {   // direction of arrival in the receiver frame: -R_m^T u
    if (a.rx_rot) {
      const double* R = a.rx_rot + 9 * m;
      q.vx = -(float)(R[0] * ux + R[3] * uy + R[6] * uz);
      q.vy = -(float)(R[1] * ux + R[4] * uy + R[7] * uz);
      q.vz = -(float)(R[2] * ux + R[5] * uy + R[8] * uz);
    } else {
      q.vx = -ux; q.vy = -uy; q.vz = -uz;
    }
  }
  // bound on the record's log2 band factor over every band: from the per-material bounds (at
  // least the largest factor: k and the lobe's coefficient may peak on different bands), or by
  // taking every band with per-record tables
  float bm = -INFINITY;
  if (!a.rec_rows) {
    bm = q.kind == 0   ? (GRAD ? 0.f : a.lmax[q.mat]) - q.gamma * q.gamma * a.lmax[a.Q + q.mat]
         : q.kind == 1 ? a.lmax[2 * a.Q + q.mat]
                       : a.lmax[3 * a.Q];
  } else {
    for (int b = 0; b < a.Bk; ++b) bm = fmaxf(bm, band_log2_v<GRAD>(a, q.kind, q.mat, q.gamma, b));
  }
  q.lbm = bm + dmax;
  if (q.lbm == -INFINITY) {   // every band factor is zero: nothing to add (lbm stays finite)
    q.base = -INFINITY;
    q.lbm = 0.f;
  }
}

// The forward contraction runs on the f16 matrix cores (v_mfma_f32_16x16x32_f16: 32 records per
// instruction, FP32 accumulation).  Each FP32 operand v is split into two halves, hi = f16(v) and
// lo = f16(v - hi), about 22 significant bits together; a real product takes three half
// products, hi hi + hi lo + lo hi (lo lo lies below 2^-22 of it), and the complex product the four
// real ones re re, im im, re im, im re.  The LDS holds the halves k-major: row k (an outer index
// of X, an inner index of Y) holds the stage's 32 records in 4 chunks of 8, the chunk a lane
// hands to an instruction (rows 80 bytes apart, so 16 lanes reading 16 bytes land on distinct
// banks).  f16 has a narrow exponent range: X is scaled by 2^(XTOP - E) with E a workgroup-wide
// bound on log2 |X| over each group of 256 records, taken before the group is generated; when a
// group's bound exceeds E the accumulators are rescaled by a power of two (exact).  A record far
// below the bound loses relative precision in proportion to its negligible share of the sum.
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
constexpr int HROW = 5;          // halfx8 per LDS row: 4 chunks of 8 records and a pad
constexpr float XTOP = 12.f;     // log2 of the largest scaled |X| (|Y| <= 1 for non-negative absorption)
// With SPLIT the Y rows hold no pad: chunk c of row k sits at slot c ^ ((k / 4) % 4), which puts
// 16 lanes reading or writing one chunk of 16 consecutive rows on distinct banks, and the
// workgroup's LDS (about 37 KB) lets four workgroups share a CU.
template <bool SPLIT>
struct H16Buf {
  static constexpr int NA = SPLIT ? KT1 / 2 : KT1;   // rows of X (a tile of at most 32 with SPLIT)
  static constexpr int BROW = SPLIT ? 4 : HROW;
  halfx8 A[4][NA][HROW];         // X halves: [re hi, re lo, im hi, im lo][k1][record chunk]
  halfx8 B[4][K2][BROW];         // Y halves: [re hi, re lo, im hi, im lo][k2][record chunk slot]
  // slot of record chunk c in Y row k
  static __device__ __forceinline__ int bslot(int k, int c) { return SPLIT ? c ^ ((k >> 2) & 3) : c; }
};

typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

// hi = f16(v) two at a time (round to nearest even); lo = f16(v - hi), the difference taken
// exactly by a mixed-precision fma from the f16 hi and the f32 v, written into the low, then
// the high half of one register (the fma leaves the other half as it is).
__device__ inline void split8(const float (&v)[8], halfx8& h, halfx8& l) {
  union { halfx8 h8; uint32_t u[4]; } H, L;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t xu = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){v[2 * i], v[2 * i + 1]}, half2v));
    uint32_t lo;
    asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lo) : "v"(xu), "v"(v[2 * i]));
    asm("v_fma_mixhi_f16 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(lo) : "v"(xu), "v"(v[2 * i + 1]));
    H.u[i] = xu;
    L.u[i] = lo;
  }
  h = H.h8;
  l = L.h8;
}

typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));

// split8 for four values
__device__ inline void split4(const float (&v)[4], halfx4& h, halfx4& l) {
  union { halfx4 h4; uint32_t u[2]; } H, L;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const uint32_t xu = __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){v[2 * i], v[2 * i + 1]}, half2v));
    uint32_t lo;
    asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lo) : "v"(xu), "v"(v[2 * i]));
    asm("v_fma_mixhi_f16 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(lo) : "v"(xu), "v"(v[2 * i + 1]));
    H.u[i] = xu;
    L.u[i] = lo;
  }
  h = H.h4;
  l = L.h4;
}

// Two-level generation: X[8a+b] = Xa[a] Xb[b] bf[seg(8a+b)] and Y[8a+b] = Ya[a] Yb[b]:
// 32 exp2/sin/cos factors per record instead of 128 values, plus one real band factor
// bf = 2^(band + directivity log2) per segment of outer indices with equal bands.
struct WaveScratch {
  float2 xa[RPW][8], xb[RPW][8], ya[RPW][8], yb[RPW][8];
  union {
    float bf[RPW][SMAX + 1];   // [nseg]: zero, for rows past the tile
    float2 xh[RPW][8];         // FOLD: Xa of rows 8 a + 4 .. 8 a + 7 (their half group's band)
  };
};

// Band segments of a tile of outer indices: segment s covers the rows whose material band
// is sb[s] and directivity band sd[s].
struct SegTable {
  int32_t sb[SMAX], sd[SMAX];   // material and directivity band of segment s
  int32_t s0[SMAX], s1[SMAX];   // its rows [s0, s1) within the tile
  int32_t bseg[16];             // segment of material band b, -1 if none (used without directivity)
};

// Band segments of the tile [k1_0, k1_0 + nk1) (the host guarantees bands constant per row
// and at most SMAX segments).  Every thread learns nseg and the segment of its lane's row
// (nseg for a row past the tile).
__device__ inline void seg_init(const SynthArgs& a, int k1_0, int nk1, int tid, SegTable& st, int& nseg, int& myseg) {
  const int lane = tid & 63, wv = tid >> 6;
  const int kr = (k1_0 + min(lane, nk1 - 1)) * K2;
  const int bb = (int)(((int64_t)kr * a.Bk) / a.F), bd = a.Bd ? (int)(((int64_t)kr * a.Bd) / a.F) : 0;
  const int bb_prev = __shfl(bb, lane - 1), bd_prev = __shfl(bd, lane - 1);
  const bool starts = lane < nk1 && (lane == 0 || bb != bb_prev || bd != bd_prev);
  const uint64_t sm = __ballot(starts);
  nseg = __popcll(sm);
  // rows past the tile take the extra segment nseg, whose band factor is zero
  myseg = lane < nk1 ? __popcll(sm & (~0ull >> (63 - lane))) - 1 : nseg;
  if (tid < 16) st.bseg[tid] = -1;
  __syncthreads();
  if (wv == 0 && starts && myseg < SMAX) {
    st.sb[myseg] = bb;
    st.sd[myseg] = bd;
    st.s0[myseg] = lane;
    if (bb < 16) st.bseg[bb] = myseg;
  }
  __syncthreads();
  if (tid < nseg && tid < SMAX) st.s1[tid] = tid + 1 < nseg ? st.s0[tid + 1] : nk1;
  __syncthreads();
}

// 2^lg e^(2 pi j rev) from the hardware exp2, sin and cos (a result below 2^-126 flushes to zero:
// such a value is below 2^-138 of the tile's largest term)
__device__ inline float2 cexp2(float lg, float rev) {
  const float amp = __builtin_amdgcn_exp2f(lg);
  return make_float2(amp * __builtin_amdgcn_cosf(rev), amp * __builtin_amdgcn_sinf(rev));
}
__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// One wave computes the generating factors of RPW records (sub-stage t of its 64 set-up
// records): Xa, Xb, Ya, Yb (8 each) and the band factor of every (record, band segment) of the
// tile, into its WaveScratch.  esh (log2) scales every X of the sub-stage.
// KFREE: the specular band factor leaves out k (see band_log2_v).
// FOLD 4: every band segment is a union of whole half groups of 4 rows (segl, segh: the segments
// of rows 8 j and 8 j + 4 of this lane's group j): the band factor is folded into Xa, one copy
// per half group (Xa for rows 8 j .. 8 j + 3, Xh for 8 j + 4 .. 8 j + 7), and no table is written.
// FOLD 8: whole groups of 8 rows, one copy (Xa).
template <bool KFREE = false, int FOLD = 0>
__device__ inline void gen_factors(const SynthArgs& a, const PairLean& q, int t, int m, int k1_0, int nk1, int lane,
                                   int nseg, const SegTable& st, float esh, WaveScratch& W, int segl = 0,
                                   int segh = 0) {
  const int r = lane >> 3, j = lane & 7;
  const int src = t * RPW + r;                 // lane that set up record r of this sub-stage
  const float base_r = __shfl(q.base, src), slope_r = __shfl(q.slope, src);
  const uint32_t a_r = (uint32_t)__shfl((int)q.a32, src), bx_r = (uint32_t)__shfl((int)q.bx32, src),
                 by_r = (uint32_t)__shfl((int)q.by32, src);
  const float lbm_r = __shfl(q.lbm, src);
  const bool ok = base_r != -INFINITY;
  const uint32_t k1a = (uint32_t)(k1_0 + 8 * j);   // first outer index of group j
  // Xa is zero for a record that adds nothing (and past the tile); then X is zero whatever the
  // other factors (finite for every record: a skipped record has slope 0 and phase steps 0)
  const float S = 2.3283064365386963e-10f;   // 2^-32: Q0.32 cycles to revolutions
  const float lg0 = base_r + (float)(k1a * K2) * slope_r + esh;
  if (FOLD) {
    // the band factors of the two half groups (no record's bound needed: each is its own)
    const float g_r = __shfl(q.gamma, src);
    const int m_r = __shfl(q.mat, src), k_r = __shfl(q.kind, src);
    float ll = band_log2_v<KFREE>(a, k_r, m_r, g_r, st.sb[segl]);
    float lh = FOLD == 4 ? band_log2_v<KFREE>(a, k_r, m_r, g_r, st.sb[segh]) : 0.f;
    if (a.Bd) {
      const float vx = __shfl(q.vx, src), vy = __shfl(q.vy, src), vz = __shfl(q.vz, src);
      const float* tab = a.dir + (size_t)m * a.Bd * a.El * a.Az;
      ll += log2f(dir_gain(tab + (size_t)st.sd[segl] * a.El * a.Az, a.El, a.Az, vx, vy, vz));
      if (FOLD == 4) lh += log2f(dir_gain(tab + (size_t)st.sd[segh] * a.El * a.Az, a.El, a.Az, vx, vy, vz));
    }
    const float rev = (float)(int32_t)(a_r + k1a * bx_r) * S;
    const float c = __builtin_amdgcn_cosf(rev), sn = __builtin_amdgcn_sinf(rev);
    const float al = ok && 8 * j < nk1 ? __builtin_amdgcn_exp2f(lg0 + ll) : 0.f;
    W.xa[r][j] = make_float2(al * c, al * sn);
    if (FOLD == 4) {
      const float ah = ok && 8 * j + 4 < nk1 ? __builtin_amdgcn_exp2f(lg0 + lh) : 0.f;
      W.xh[r][j] = make_float2(ah * c, ah * sn);
    }
  } else {
    // the record's band bound lbm rides on Xa; the band factors (<= 1) go to the table below
    const float lg = ok && 8 * j < nk1 ? lg0 + lbm_r : -INFINITY;
    W.xa[r][j] = cexp2(lg, (float)(int32_t)(a_r + k1a * bx_r) * S);
  }
  W.xb[r][j] = cexp2((float)(j * K2) * slope_r, (float)(int32_t)((uint32_t)j * bx_r) * S);
  W.ya[r][j] = cexp2((float)(8 * j) * slope_r, (float)(int32_t)((uint32_t)(8 * j) * by_r) * S);
  W.yb[r][j] = cexp2((float)j * slope_r, (float)(int32_t)((uint32_t)j * by_r) * S);
  // band factors of every (record, segment), and zero for the segment past the tile
  if (FOLD) {
    // (folded into Xa and Xh)
  } else if (!KFREE) {
    // lane (r, j) takes segments j, j + 8, ... of record r
    const float g_r = __shfl(q.gamma, src);
    const int m_r = __shfl(q.mat, src), k_r = __shfl(q.kind, src);
    float vx = 0.f, vy = 0.f, vz = 0.f;
    if (a.Bd) {
      vx = __shfl(q.vx, src);
      vy = __shfl(q.vy, src);
      vz = __shfl(q.vz, src);
    }
    for (int sg = j; sg < nseg; sg += 8) {
      // (finite for a skipped record too: its Xa is zero)
      float lb = band_log2_v(a, k_r, m_r, g_r, st.sb[sg]);
      if (a.Bd) lb += log2f(dir_gain(a.dir + ((size_t)m * a.Bd + st.sd[sg]) * a.El * a.Az, a.El, a.Az, vx, vy, vz));
      W.bf[r][sg] = __builtin_amdgcn_exp2f(lb - lbm_r);   // <= 1: the record's bound lbm rides on Xa
    }
  } else {
    // the adjoint (no directivity): the pairs enumerated over the wave, each lane fetching its
    // record's data (fewer registers live across the loop: measured faster in that kernel)
    for (int i0 = 0; i0 < RPW * nseg; i0 += 64) {
      const int i = i0 + lane;
      const int rr = min(i / nseg, RPW - 1), sg = i - (i / nseg) * nseg;
      const int sr = t * RPW + rr;
      const float g2 = __shfl(q.gamma, sr), b2 = __shfl(q.base, sr), lm2 = __shfl(q.lbm, sr);
      const int m2 = __shfl(q.mat, sr), k2 = __shfl(q.kind, sr);
      if (i < RPW * nseg) W.bf[rr][sg] = b2 != -INFINITY ? exp2f(band_log2_v<true>(a, k2, m2, g2, st.sb[sg]) - lm2) : 0.f;
    }
  }
  if (!FOLD && j == 7) W.bf[r][nseg] = 0.f;
  // the factors are read back by other lanes of this wave only
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// X and Y values of record rr for this lane's outer and inner index (lane = 8 a + b):
// X[lane] = Xa[a] Xb[b] bf[segment of the lane's row], Y[lane] = Ya[a] Yb[b].
// FOLD 4: the band factor is already on Xa (b < 4) or Xh (b >= 4); FOLD 8: on Xa.
template <int FOLD = 0>
__device__ inline void xy_value(const WaveScratch& W, int rr, int lane, int myseg, float2& x, float2& y) {
  const int ka = lane >> 3, kb = lane & 7;
  y = cmul(W.ya[rr][ka], W.yb[rr][kb]);
  if (FOLD == 8) {
    x = cmul(W.xa[rr][ka], W.xb[rr][kb]);
  } else if (FOLD == 4) {
    x = cmul(kb < 4 ? W.xa[rr][ka] : W.xh[rr][ka], W.xb[rr][kb]);
  } else {
    x = cmul(W.xa[rr][ka], W.xb[rr][kb]);
    const float f = W.bf[rr][myseg];
    x.x *= f;
    x.y *= f;
  }
}

// X of record rr at outer index `row` (as in xy_value; seg: the row's band segment)
template <int FOLD>
__device__ inline float2 x_value(const WaveScratch& W, int rr, int row, int seg) {
  const int ka = row >> 3, kb = row & 7;
  if (FOLD == 8) return cmul(W.xa[rr][ka], W.xb[rr][kb]);
  if (FOLD == 4) return cmul(kb < 4 ? W.xa[rr][ka] : W.xh[rr][ka], W.xb[rr][kb]);
  float2 x = cmul(W.xa[rr][ka], W.xb[rr][kb]);
  const float f = W.bf[rr][seg];
  x.x *= f;
  x.y *= f;
  return x;
}

// The sub-stage's records as f16 halves: X of this lane's outer index into A, Y of its inner
// index into B, chunk wv (the wave's 8 records of the stage).  With a tile of at most 32 rows
// (SPLIT) every lane forms X: lane (row = lane % 32, h = lane / 32) for records 4 h .. 4 h + 3,
// writing its half of the row's 8-record chunk; segx is the band segment of row lane % 32.
template <bool SPLIT, int FOLD>
__device__ inline void write_h16(const WaveScratch& W, int lane, int wv, int myseg, int segx, H16Buf<SPLIT>& buf) {
  if constexpr (SPLIT) {
    const int row = lane & 31, hh = lane >> 5;
    float xr[4], xi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float2 x = x_value<FOLD>(W, 4 * hh + i, row, segx);
      xr[i] = x.x;
      xi[i] = x.y;
    }
    halfx4 h4, l4;
    split4(xr, h4, l4);
    reinterpret_cast<halfx4*>(&buf.A[0][row][wv])[hh] = h4;
    reinterpret_cast<halfx4*>(&buf.A[1][row][wv])[hh] = l4;
    split4(xi, h4, l4);
    reinterpret_cast<halfx4*>(&buf.A[2][row][wv])[hh] = h4;
    reinterpret_cast<halfx4*>(&buf.A[3][row][wv])[hh] = l4;
    const int ka = lane >> 3, kb = lane & 7;
    float yr[RPW], yi[RPW];
#pragma unroll
    for (int rr = 0; rr < RPW; ++rr) {
      const float2 y = cmul(W.ya[rr][ka], W.yb[rr][kb]);
      yr[rr] = y.x;
      yi[rr] = y.y;
    }
    halfx8 h, l;
    const int sl = H16Buf<SPLIT>::bslot(lane, wv);
    split8(yr, h, l);
    buf.B[0][lane][sl] = h;
    buf.B[1][lane][sl] = l;
    split8(yi, h, l);
    buf.B[2][lane][sl] = h;
    buf.B[3][lane][sl] = l;
    return;
  }
  float xr[RPW], xi[RPW], yr[RPW], yi[RPW];
#pragma unroll
  for (int rr = 0; rr < RPW; ++rr) {
    float2 x, y;
    xy_value<FOLD>(W, rr, lane, myseg, x, y);
    xr[rr] = x.x; xi[rr] = x.y; yr[rr] = y.x; yi[rr] = y.y;
  }
  halfx8 h, l;
  if (lane < H16Buf<SPLIT>::NA) {
    split8(xr, h, l);
    buf.A[0][lane][wv] = h;
    buf.A[1][lane][wv] = l;
    split8(xi, h, l);
    buf.A[2][lane][wv] = h;
    buf.A[3][lane][wv] = l;
  }
  split8(yr, h, l);
  buf.B[0][lane][wv] = h;
  buf.B[1][lane][wv] = l;
  split8(yi, h, l);
  buf.B[2][lane][wv] = h;
  buf.B[3][lane][wv] = l;
}

struct BwdBuf;
__device__ inline void write_bwd(const WaveScratch& W, int lane, int wv, BwdBuf& bb);

// Row and column blocks (16 x 16) of a wave: with 64 rows, the quadrant (wv / 2, wv % 2) as 2 x 2
// blocks; with at most 32 rows (SPLIT), row block wv % 2 against the column blocks of half wv / 2.
template <bool SPLIT>
__device__ inline void wave_blocks(int wv, int& rb0, int& cb0) {
  rb0 = SPLIT ? (wv & 1) : 2 * (wv >> 1);
  cb0 = SPLIT ? 2 * (wv >> 1) : 2 * (wv & 1);
}

// One stage (32 records) into the wave's blocks: acc[0] += Xr Yr, acc[1] += Xi Yi,
// acc[2] += Xr Yi + Xi Yr, each real product as three half products.
template <bool SPLIT>
__device__ inline void contract_h16(const H16Buf<SPLIT>& buf, int wv, int lane, floatx4 (&acc)[3][2][2]) {
  constexpr int NRB = SPLIT ? 1 : 2;
  int rb0, cb0;
  wave_blocks<SPLIT>(wv, rb0, cb0);
  const int r16 = lane & 15, ch = lane >> 4;
  halfx8 b[2][4];
#pragma unroll
  for (int jj = 0; jj < 2; ++jj)
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int k2 = 16 * (cb0 + jj) + r16;
      b[jj][f] = buf.B[f][k2][H16Buf<SPLIT>::bslot(k2, ch)];
    }
#pragma unroll
  for (int i = 0; i < NRB; ++i) {
    halfx8 av[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) av[f] = buf.A[f][16 * (rb0 + i) + r16][ch];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      floatx4 rr = acc[0][i][jj], ii = acc[1][i][jj], im = acc[2][i][jj];
      rr = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[0], b[jj][0], rr, 0, 0, 0);
      rr = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[0], b[jj][1], rr, 0, 0, 0);
      rr = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[1], b[jj][0], rr, 0, 0, 0);
      ii = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[2], b[jj][2], ii, 0, 0, 0);
      ii = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[2], b[jj][3], ii, 0, 0, 0);
      ii = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[3], b[jj][2], ii, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[0], b[jj][2], im, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[0], b[jj][3], im, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[1], b[jj][2], im, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[2], b[jj][0], im, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[2], b[jj][1], im, 0, 0, 0);
      im = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[3], b[jj][0], im, 0, 0, 0);
      acc[0][i][jj] = rr;
      acc[1][i][jj] = ii;
      acc[2][i][jj] = im;
    }
  }
}

__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// Upper bound on log2 |X[k1] Y[k2]| over the tile for the record set up in q (-inf for none):
// the amplitude at the tile's first or last row, the record's band bound lbm (at least its
// largest band factor with its lobe, plus the receiver's largest log2 directivity gain), and
// what |Y| can exceed 1 by.
__device__ inline float record_bound(const PairLean& q, int k1_0, int nk1) {
  if (q.base == -INFINITY) return -INFINITY;
  const float s64 = (float)K2 * q.slope;
  return q.base + fmaxf((float)k1_0 * s64, (float)(k1_0 + nk1 - 1) * s64) + fmaxf(0.f, (float)(K2 - 1) * q.slope) +
         q.lbm;
}

// Largest log2 directivity gain of receiver m over every band and cell (the bilinear gain never
// exceeds it); 0 without directivity.  Every thread of the workgroup calls it.
__device__ inline float dir_log2_max(const SynthArgs& a, int m, int tid, float* red) {
  if (!a.Bd) return 0.f;
  const float* tab = a.dir + (size_t)m * a.Bd * a.El * a.Az;
  const int n = a.Bd * a.El * a.Az;
  float v = 0.f;
  for (int i = tid; i < n; i += 256) v = fmaxf(v, tab[i]);
  v = wave_max(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  v = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  __syncthreads();
  return log2f(v);
}

// Workgroup = (record chunk p, receiver m, 64 outer indices).  Every 8 stages each wave sets up
// 64 records (one per lane) and the workgroup bounds their |X|; every stage each wave generates
// 8 of them as f16 halves into LDS, then each wave contracts all 32 records of the stage into
// its blocks of (k1, k2) on the matrix cores.
// FOLD 4 (8): every band edge falls on a multiple of 4 (8) rows and the grid holds whole groups of
// that many rows (bins a multiple of 256, 512): the band factor rides on Xa.
template <bool BATCH, bool SPLIT, int FOLD>
__global__ __launch_bounds__(256, SPLIT ? 4 : 2) void k_synth_mfma(SynthArgs a0, const SynthArgs* __restrict__ jobs,
                                                                   ChunkTab ct, et_paths P,
                                                                   const int32_t* __restrict__ idx, const Ctl* ctl,
                                                                   float* __restrict__ part) {
  SYNTH_RESOLVE();
  __shared__ __align__(16) H16Buf<SPLIT> buf;
  __shared__ WaveScratch wscr[4];
  __shared__ SegTable st;
  __shared__ float red[4];
  const int p = bp, m = bm, k1t = bt;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K1 = a.F / K2;
  const int k1_0 = k1t * KT1;
  const int nk1 = min(KT1, K1 - k1_0);
  int nseg, myseg;
  seg_init(a, k1_0, nk1, tid, st, nseg, myseg);
  // segments of the two half groups of row group lane % 8 (FOLD)
  const int segl = min(__shfl(myseg, 8 * (lane & 7)), nseg - 1), segh = min(__shfl(myseg, 8 * (lane & 7) + 4), nseg - 1);
  const int segx = __shfl(myseg, lane & 31);   // (SPLIT: the band segment of row lane % 32)
  const float dmax = dir_log2_max(a, m, tid, red);
  const int64_t nst = (hi - lo + 8 * RB - 1) / (8 * RB) * 8;   // whole groups of 8 stages (256 records)
  floatx4 acc[3][2][2];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) acc[t][i][jj] = floatx4{0.f, 0.f, 0.f, 0.f};
  float E = -INFINITY;   // current exponent bound (uniform over the workgroup)
  PairLean q;
  for (int64_t s = 0; s < nst; ++s) {
    const int t = (int)(s & 7);
    if (t == 0) {
      // wave w of stage group g owns records [lo + 256 g + 64 w, +64); sub-stage t takes 8 of them
      pair_lean(a, P, idx, lo + (s >> 3) * (8 * RB) + wv * 64 + lane, hi, m, q, dmax);
      const float ub = wave_max(record_bound(q, k1_0, nk1));
      if (lane == 0) red[wv] = ub;
      __syncthreads();
      const float Eg = ceilf(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
      if (Eg > E) {
        if (E != -INFINITY) {
          const float r = exp2f(E - Eg);
#pragma unroll
          for (int tt = 0; tt < 3; ++tt)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int jj = 0; jj < 2; ++jj) acc[tt][i][jj] *= r;
        }
        E = Eg;
      }
    }
    gen_factors<false, FOLD>(a, q, t, m, k1_0, nk1, lane, nseg, st, E != -INFINITY ? XTOP - E : 0.f, wscr[wv], segl,
                             segh);
    write_h16<SPLIT, FOLD>(wscr[wv], lane, wv, myseg, segx, buf);
    __syncthreads();
    contract_h16<SPLIT>(buf, wv, lane, acc);
    __syncthreads();
  }
  // accumulator (i, jj, v) of lane l: row k1 = 16 (rb0 + i) + 4 (l / 16) + v, column k2 = 16 (cb0 + jj) + l % 16
  const float us = E != -INFINITY ? exp2f(E - XTOP) : 0.f;
  int rb0, cb0;
  wave_blocks<SPLIT>(wv, rb0, cb0);
  float* out = part + (((size_t)p * a.M + m) * a.F) * 2;
#pragma unroll
  for (int i = 0; i < (SPLIT ? 1 : 2); ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k1 = 16 * (rb0 + i) + (lane >> 4) * 4 + v, k2 = 16 * (cb0 + jj) + (lane & 15);
        if (k1 < nk1) {
          const size_t o = (size_t)((k1_0 + k1) * K2 + k2) * 2;
          out[o] = (acc[0][i][jj][v] - acc[1][i][jj][v]) * us;
          out[o + 1] = acc[2][i][jj][v] * us;
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

template <bool BATCH>
__global__ __launch_bounds__(DB) void k_synth_direct(SynthArgs a0, const SynthArgs* __restrict__ jobs, ChunkTab ct,
                                                     et_paths P, const int32_t* __restrict__ idx, const Ctl* ctl,
                                                     float* __restrict__ part) {
  SYNTH_RESOLVE();
  __shared__ DirectLds L;
  const int p = bp, m = bm;
  const int tid = threadIdx.x;
  const int kbase = bt * DTILE + tid * DPT;
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
      const int64_t e = n0 + tid;
      Pair q;
      if (e < hi && pair_setup(a, P, idx ? (int64_t)idx[e] : e, m, q)) {
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

template <bool BATCH>
__global__ __launch_bounds__(GB) void k_synth_bwd(SynthArgs a0, const SynthArgs* __restrict__ jobs, ChunkTab ct,
                                                 et_paths P, const int32_t* __restrict__ idx, const Ctl* ctl,
                                                 const float* __restrict__ g, double* __restrict__ gpx,
                                                 double* __restrict__ gpk) {
  SYNTH_RESOLVE();
  if (BATCH) g += (size_t)jb * a.M * a.F * 2;
  extern __shared__ float2 gl[];   // dL/dconj(H) of this receiver, [F]
  __shared__ double red[GB];
  __shared__ double kval[16][GB];
  __shared__ int kmat[GB];
  __shared__ double kacc[16 * 16];
  const int p = bp, m = bm, tid = threadIdx.x;
  for (int k = tid; k < a.F; k += GB) gl[k] = make_float2(g[((size_t)m * a.F + k) * 2], g[((size_t)m * a.F + k) * 2 + 1]);
  for (int i = tid; i < a.Q * a.Bk; i += GB) kacc[i] = 0.0;
  double gx0 = 0, gx1 = 0, gx2 = 0;
  const double ln10 = 2.30258509299404568402;
  __syncthreads();
  for (int64_t n0 = lo; n0 < hi; n0 += GB) {
    const int64_t e = n0 + tid;
    double sb[16];
#pragma unroll
    for (int b = 0; b < 16; ++b) sb[b] = 0.0;
    int mat = -1;
    Pair q;
    int64_t n = -1;
    if (e < hi) n = idx[e];
    if (n >= 0 && pair_setup(a, P, n, m, q)) {
      mat = q.kind == 0 ? q.mat : -1;
      // step of the rotation recurrence: exp2(slope) e^{j 2 pi cb}
      const float wrev = (float)frac(q.cb);
      const float wamp = exp2f(q.slope);
      const float wr = wamp * __builtin_amdgcn_cosf(wrev), wi = wamp * __builtin_amdgcn_sinf(wrev);
      // S_b = sum_{k in band b} conj(g_k) T_k and S1 = sum_k f_k conj(g_k) T_k.  Within a
      // block of GANCHOR bins the FP32 sums carry the small weights (k - ka); blocks combine
      // in FP64 as S1 += f_ka sum z + df sum (k - ka) z.
      double s1r = 0.0, s1i = 0.0;
      // receiver directivity: direction of arrival in the receiver frame, and the sum over
      // directivity bands d of Re(S_d) grad_v ln D_d(v)
      float vx = 0.f, vy = 0.f, vz = 0.f;
      if (a.Bd) arrival(a, q, m, vx, vy, vz);
      double gvx = 0.0, gvy = 0.0, gvz = 0.0;
      for (int b = 0; b < a.Bk; ++b) {
        const int k0 = (int)(((int64_t)b * a.F + a.Bk - 1) / a.Bk);
        const int k1 = (int)(((int64_t)(b + 1) * a.F + a.Bk - 1) / a.Bk);
        // specular records: the band's terms without the factor k (H is linear in k, Eq. 2, so
        // this sum is dH/dk also where k = 0); k multiplies the band's share of the other sums
        const float blog = q.kind == 0 ? -q.gamma * q.gamma * a.lc[(int64_t)q.mat * a.Bk + b] : band_log2(a, q, b);
        const double kf = q.kind == 0 ? (double)a.refl_k[(int64_t)q.mat * a.Bk + b] : 1.0;
        double sbr = 0.0, b1r = 0.0, b1i = 0.0, bgx = 0.0, bgy = 0.0, bgz = 0.0;
        // the band's bins in runs of one directivity band (one run without directivity)
        for (int ks = k0; ks < k1;) {
          int kr = k1;
          float dlog = 0.f, dgx = 0.f, dgy = 0.f, dgz = 0.f;
          if (a.Bd) {
            const int d = (int)(((int64_t)ks * a.Bd) / a.F);
            kr = min(k1, (int)(((int64_t)(d + 1) * a.F + a.Bd - 1) / a.Bd));
            const float D = dir_gain_dv(a.dir + ((size_t)m * a.Bd + d) * a.El * a.Az, a.El, a.Az, vx, vy, vz, dgx,
                                        dgy, dgz);
            dlog = log2f(D);
            const float iD = D > 0.f ? 1.f / D : 0.f;
            dgx *= iD; dgy *= iD; dgz *= iD;
          }
          double srun = 0.0;
          for (int ka = ks; ka < kr; ka += GANCHOR) {
            const int ke = min(ka + GANCHOR, kr);
            const float rev = (float)frac(q.c0 + (double)ka * q.cb);
            const float amp = exp2f(q.base + (float)ka * q.slope + blog + dlog);
            float tr = amp * __builtin_amdgcn_cosf(rev), ti = amp * __builtin_amdgcn_sinf(rev);
            float w = 0.f;
            float c0r = 0.f, c0i = 0.f, c1r = 0.f, c1i = 0.f;
            for (int k = ka; k < ke; ++k) {
              const float2 gg = gl[k];
              const float zr = gg.x * tr + gg.y * ti;   // Re(conj(g) T)
              const float zi = gg.x * ti - gg.y * tr;   // Im(conj(g) T)
              c0r += zr;
              c0i += zi;
              c1r += w * zr;
              c1i += w * zi;
              const float nr = tr * wr - ti * wi;
              ti = tr * wi + ti * wr;
              tr = nr;
              w += 1.f;
            }
            const double fa = a.f_lo + (double)ka * a.df;
            srun += (double)c0r;
            b1r += fa * (double)c0r + a.df * (double)c1r;
            b1i += fa * (double)c0i + a.df * (double)c1i;
          }
          sbr += srun;
          bgx += srun * (double)dgx; bgy += srun * (double)dgy; bgz += srun * (double)dgz;
          ks = kr;
        }
        s1r += kf * b1r;
        s1i += kf * b1i;
        gvx += kf * bgx; gvy += kf * bgy; gvz += kf * bgz;
#pragma unroll
        for (int bb = 0; bb < 16; ++bb)
          if (bb == b) sb[bb] = sbr;
      }
      // sb: band sums without k for specular records; s0 = sum over bands of k * sb
      double s0 = 0;
#pragma unroll
      for (int b = 0; b < 16; ++b)
        if (b < a.Bk) s0 += (q.kind == 0 ? (double)a.refl_k[(int64_t)q.mat * a.Bk + b] : 1.0) * sb[b];
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
            wsum += (double)a.refl_k[q.mat * a.Bk + b] * sb[b] / (2.0 * bt * bt);
          }
        }
        g0 -= 2.0 * wsum * d0; g1 -= 2.0 * wsum * d1; g2 -= 2.0 * wsum * d2;
        // dL/dk of the record's (material, band): 2 Re sum conj(g) dT/dk
#pragma unroll
        for (int b = 0; b < 16; ++b) sb[b] = 2.0 * sb[b];
      }
      if (a.Bd) {
        // v = -R^T u and du/dx_m = (I - u u^T) / l: d ln D / dx_m = -(I - u u^T) R grad_v ln D / l
        double w0 = gvx, w1 = gvy, w2 = gvz;
        if (a.rx_rot) {
          const double* R = a.rx_rot + 9 * m;
          w0 = R[0] * gvx + R[1] * gvy + R[2] * gvz;
          w1 = R[3] * gvx + R[4] * gvy + R[5] * gvz;
          w2 = R[6] * gvx + R[7] * gvy + R[8] * gvz;
        }
        const double uw = q.u[0] * w0 + q.u[1] * w1 + q.u[2] * w2;
        const double c = 2.0 / q.l;
        g0 -= c * (w0 - uw * q.u[0]);
        g1 -= c * (w1 - uw * q.u[1]);
        g2 -= c * (w2 - uw * q.u[2]);
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

// Factorised adjoint.  For record n and receiver m the adjoint needs, per material band b,
//   S_b = sum_{k in b} conj(g_k) T_k   and   S1 = sum_k f_k conj(g_k) T_k,
// with T_k = X[k1] Y[k2] as in the forward kernel and G = conj(g) as a [k1][k2] matrix:
//   S_b = sum_{k1 in b} X[k1] Z[k1],   Z[k1]  = sum_k2 G[k1, k2] Y[k2],
//   S1  = sum_k1 X[k1] Z'[k1],         Z'[k1] = sum_k2 f_k G[k1, k2] Y[k2],
// f_k the frequency of bin k = 64 k1 + k2.  Z and Z' are complex matrix products contracting
// over k2 on the f16 matrix cores with split operands (as in the forward kernel): G = conj(g)
// and f_k G sit in registers as halves, each scaled into the f16 range by a power of two per
// wave, and Y is written as halves, record-major (8 inner indices per lane, 16-byte reads).
// The per-row products go to LDS; per record, band sums and the weighted sum run in FP32 in a
// fixed order, and the chain rule of the direct adjoint turns them into dL/dk and dL/dx_m
// (accumulated over records in FP64).
// LDS record stride of the adjoint's per-row products R0: with 68 = 4 (mod 64) the 16-byte
// writes of four consecutive rows are conflict-free per quarter wave.
constexpr int BS68 = 68;

// Group-major sums (stride 36): the eight threads of each of a wave's eight records reading
// groups 2 j + i fall on 64 distinct banks.
// X carries the band factor without k for specular records: Re(X Z) summed over a band's rows
// is then dH/dk of that band (also where k = 0), and k enters the other sums per row.
constexpr int YROW = 9;     // halfx8 per record row of Y halves: 64 inner indices and a pad (144-byte rows)
struct __align__(16) BwdBuf {
  halfx8 Y[4][RB][YROW];     // Y halves [re hi, re lo, im hi, im lo][record][chunk of 8 inner indices]
  float R0[RB][BS68];        // Re(X Z) per (record, row) (band edges off the 4-row groups)
  float Rg[16][36];          // Re(X Z) summed over a group of 4 rows, per (group, record) (FOLD)
  float2 R1[16][36];         // sum over 4 rows of k X Z' per (row group, record)
  float kv[16][RB];          // 2 S_b of each specular record of the stage (0 for the others), [band][record]
  int32_t kmat[RB];          // the material of each specular record of the stage, -1 for the others
  double dk[4][256];         // per wave: dL/dk of (material, band) over its records so far
  float lobe_w[256];         // per (material, band): 1 / (2 beta^2)
  float kf[256 + 16];        // per (material, band): k; then a row of ones (records of other kinds)
  int32_t recb[RB];          // per record of the stage: its row of kf (mat Bk, or the ones row)
};

// The adjoint's matrix-product operand of the sub-stage's records: Y as f16 halves record-major,
// lane (r, c) = (lane / 8, lane % 8) forming inner indices 8 c .. 8 c + 7 of record r:
// Y[8 c + i] = Ya[c] Yb[i].  (X is formed where it is used, from the factors.)
__device__ inline void write_bwd(const WaveScratch& W, int lane, int wv, BwdBuf& bb) {
  const int row0 = wv * RPW;
  const int r = lane >> 3, c = lane & 7;
  const float2 ya = W.ya[r][c];
  float yr[8], yi[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float2 y = cmul(ya, W.yb[r][i]);
    yr[i] = y.x;
    yi[i] = y.y;
  }
  split8(yr, bb.Y[0][row0 + r][c], bb.Y[1][row0 + r][c]);
  split8(yi, bb.Y[2][row0 + r][c], bb.Y[3][row0 + r][c]);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Sum of v over each group of 8 consecutive lanes, valid in the group's first lane, added as
// ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7)) by lane moves within rows of 16 (no LDS).
template <int CTRL>
__device__ inline float dpp_mov(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
__device__ inline float sum8_first(float v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]: lane ^ 1
  v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]: lane ^ 2
  v += dpp_mov<0x104>(v);   // row_shl 4: lane + 4 within the row
  return v;
}

// dL/dk over the wave's 8 records n of the stage (8 wv .. 8 wv + 7): (material q, band b) adds
// 2 S_b of the specular records of material q.  As a matrix product, kv [band][record] times the
// records' one-hot materials [record][material], on the FP32 matrix cores (the products are
// exact: 0 or the value) in tiles of 16 materials; each lane adds its four sums to the wave's
// FP64 totals in LDS (one lane per (material, band)).  With at most 16 materials the sums stay
// in the FP32 accumulator dkc over a group of 8 stages (64 records) and go to the totals when
// flush is set.  Every lane of the wave calls it.
__device__ inline void dk_wave(BwdBuf& bb, int wv, int lane, int Q, int Bk, floatx4& dkc, bool flush) {
  const int col = lane & 15;   // A: band row; B: material column within the tile
  float av[2];
  int mv[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int n = 8 * wv + 4 * h + (lane >> 4);
    av[h] = col < Bk ? bb.kv[col][n] : 0.f;
    mv[h] = bb.kmat[n];
  }
  if (Q <= 16) {
#pragma unroll
    for (int h = 0; h < 2; ++h) dkc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[h], mv[h] == col ? 1.f : 0.f, dkc, 0, 0, 0);
    if (flush) {
      if (col < Q) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int b = 4 * (lane >> 4) + v;
          if (b < Bk) bb.dk[wv][col * Bk + b] += (double)dkc[v];
        }
      }
      dkc = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    return;
  }
  for (int q0 = 0; q0 < Q; q0 += 16) {
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < 2; ++h) c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[h], mv[h] == q0 + col ? 1.f : 0.f, c, 0, 0, 0);
    // c[v]: band 4 (lane / 16) + v, material q0 + lane % 16
    const int qq = q0 + col;
    if (qq < Q) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int b = 4 * (lane >> 4) + v;
        if (b < Bk) bb.dk[wv][qq * Bk + b] += (double)c[v];
      }
    }
  }
}

// FOLD 4 (8): every band edge of the grid falls on a group of 4 (8) rows (a multiple of 256, 512
// bins) and the grid holds whole groups: each lane's four rows of the matrix-product output belong
// to one band and are summed in registers, and the band factor rides on Xa as in the forward
// kernel.
template <bool BATCH, bool SPLIT, int FOLD>
__global__ __launch_bounds__(256, 2) void k_synth_bwd_mfma(SynthArgs a0, const SynthArgs* __restrict__ jobs,
                                                        ChunkTab ct, et_paths P, const int32_t* __restrict__ idx,
                                                        const Ctl* ctl, const float* __restrict__ g,
                                                        double* __restrict__ gpx, double* __restrict__ gpk) {
  SYNTH_RESOLVE();
  if (BATCH) g += (size_t)jb * a.M * a.F * 2;
  __shared__ __align__(16) BwdBuf bb;
  __shared__ WaveScratch wscr[4];
  __shared__ SegTable st;
  __shared__ double red[256];
  const int p = bp, m = bm, k1t = bt;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K1 = a.F / K2;
  const int k1_0 = k1t * KT1;
  const int nk1 = min(KT1, K1 - k1_0);
  int nseg, myseg;
  seg_init(a, k1_0, nk1, tid, st, nseg, myseg);
  // segments of the two half groups of row group lane % 8 (FOLD)
  const int segl = min(__shfl(myseg, 8 * (lane & 7)), nseg - 1), segh = min(__shfl(myseg, 8 * (lane & 7) + 4), nseg - 1);
  // wave -> block of 16 rows; SPLIT (a tile of at most 32 rows, two blocks) gives each wave
  // pair one block and each wave of a pair one of the stage's two record blocks
  constexpr int NB = SPLIT ? 1 : 2;              // record blocks of 16 per wave and stage
  const int rbw = SPLIT ? (wv & 1) : wv;
  const int nb0 = SPLIT ? (wv >> 1) : 0;
  // A operands: rows k1 = 16 rbw + lane % 16 of G = conj(g) and of f_k G (f_k the bin's
  // frequency), inner indices k2 = 32 h + 8 (lane / 16) + i (h < 2, i < 8), as f16 halves
  // [re hi, re lo, im hi, im lo], scaled by 2^eg and 2^eg2 (per wave) so that the largest
  // magnitude is near 2^12
  halfx8 ga[2][4], gw[2][4];
  float usz, usw;   // 2^-eg, 2^-eg2: undo the scales on Z and Z'
  {
    const int r1g = rbw * 16 + (lane & 15);
    float gr[2][8], gi[2][8], fk[2][8];
    float mz = 0.f, mw = 0.f;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k2 = 32 * h + 8 * (lane >> 4) + i;
        const int k = (k1_0 + r1g) * K2 + k2;
        float vr = 0.f, vi = 0.f;
        if (r1g < nk1) {
          vr = g[((size_t)m * a.F + k) * 2];
          vi = -g[((size_t)m * a.F + k) * 2 + 1];
        }
        gr[h][i] = vr;
        gi[h][i] = vi;
        fk[h][i] = (float)(a.f_lo + (double)k * a.df);
        const float mg = fmaxf(fabsf(vr), fabsf(vi));
        mz = fmaxf(mz, mg);
        mw = fmaxf(mw, mg * fabsf(fk[h][i]));
      }
    mz = wave_max(mz);
    mw = wave_max(mw);
    const float ez = mz > 0.f ? 12.f - ceilf(log2f(mz)) : 0.f, ew = mw > 0.f ? 12.f - ceilf(log2f(mw)) : 0.f;
    const float sz = exp2f(ez), sw = exp2f(ew);
    usz = exp2f(-ez);
    usw = exp2f(-ew);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float zr[8], zi[8], wr[8], wi[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        zr[i] = gr[h][i] * sz;
        zi[i] = gi[h][i] * sz;
        wr[i] = gr[h][i] * fk[h][i] * sw;
        wi[i] = gi[h][i] * fk[h][i] * sw;
      }
      split8(zr, ga[h][0], ga[h][1]);
      split8(zi, ga[h][2], ga[h][3]);
      split8(wr, gw[h][0], gw[h][1]);
      split8(wi, gw[h][2], gw[h][3]);
    }
  }
  const int64_t nst = (hi - lo + 8 * RB - 1) / (8 * RB) * 8;
  const double ln10 = 2.30258509299404568402;
  const double c2 = -ln10 * a.A1 / 20.0, c3 = -(double)a.sigma * 2.0 * M_PI / a.c;
  const int QB = a.Q * a.Bk;
  double gx0 = 0.0, gx1 = 0.0, gx2 = 0.0;
  for (int i = tid; i < QB; i += 256) {
    const double bt = (double)a.beta[i];
    bb.lobe_w[i] = (float)(1.0 / (2.0 * bt * bt));
    bb.kf[i] = a.refl_k[i];
  }
  if (tid < a.Bk) bb.kf[QB + tid] = 1.f;
  for (int i = lane; i < QB; i += 64) bb.dk[wv][i] = 0.0;   // (each wave's own totals)
  // material band and band segment of each of this lane's four epilogue rows (rows past the grid:
  // the last band, and the segment past the tile, whose band factor is zero)
  int rband[4], rseg[4];
  {
    const int r10 = rbw * 16 + (lane >> 4) * 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t kr = (int64_t)min(k1_0 + r10 + v, K1 - 1) * K2;
      rband[v] = (int)((kr * a.Bk) / a.F);
      rseg[v] = __shfl(myseg, r10 + v);
    }
  }
  // rows [br0[h], br1[h]) of the tile in band (tid % 8) + 8 h, the bands this thread sums in the
  // per-record epilogue (empty for a band not in the tile)
  int br0[2], br1[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int b = (tid & 7) + 8 * h, sg = b < a.Bk ? st.bseg[b] : -1;
    br0[h] = sg >= 0 ? st.s0[sg] : 0;
    br1[h] = sg >= 0 ? st.s1[sg] : 0;
  }
  floatx4 dkc = {0.f, 0.f, 0.f, 0.f};
  PairLean q;
  for (int64_t s = 0; s < nst; ++s) {
    const int t = (int)(s & 7);
    if (t == 0) pair_lean<true>(a, P, idx, lo + (s >> 3) * (8 * RB) + wv * 64 + lane, hi, m, q);
    gen_factors<true, FOLD>(a, q, t, m, k1_0, nk1, lane, nseg, st, 0.f, wscr[wv], segl, segh);
    write_bwd(wscr[wv], lane, wv, bb);
    {
      // each generated record's row of k factors
      const int src = t * RPW + (lane & 7);
      const int m_r = __shfl(q.mat, src), k_r = __shfl(q.kind, src);
      if (lane < RPW) bb.recb[wv * RPW + lane] = k_r == 0 ? m_r * a.Bk : QB;
    }
    __syncthreads();
    // acc[0..2]: Z as Gr Yr, Gi Yi, Gr Yi + Gi Yr; acc[3..5]: Z' likewise (f_k G)
    floatx4 acc[6][NB];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int nn = (nb0 + j) * 16 + (lane & 15);
        halfx8 y[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) y[f] = bb.Y[f][nn][4 * h + (lane >> 4)];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const halfx8* A = u ? gw[h] : ga[h];
          floatx4 rr = acc[3 * u][j], ii = acc[3 * u + 1][j], im = acc[3 * u + 2][j];
          rr = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0], y[0], rr, 0, 0, 0);
          rr = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0], y[1], rr, 0, 0, 0);
          rr = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1], y[0], rr, 0, 0, 0);
          ii = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[2], y[2], ii, 0, 0, 0);
          ii = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[2], y[3], ii, 0, 0, 0);
          ii = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[3], y[2], ii, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0], y[2], im, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[0], y[3], im, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[1], y[2], im, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[2], y[0], im, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[2], y[1], im, 0, 0, 0);
          im = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[3], y[0], im, 0, 0, 0);
          acc[3 * u][j] = rr;
          acc[3 * u + 1][j] = ii;
          acc[3 * u + 2][j] = im;
        }
      }
    }
    // accumulator (j, v) of lane l: row 16 rbw + 4 (l / 16) + v, record 16 (nb0 + j) + l % 16
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int nb = nb0 + j;
      const int n = nb * 16 + (lane & 15);
      const int r10 = rbw * 16 + (lane >> 4) * 4;   // this lane's four rows r10 .. r10 + 3
      // X of record n at these rows from its factors (wave n / 8 generated it): Xa (or Xh, the
      // upper half group with FOLD 4) of group r10 / 8 times Xb of r10 % 8 .. + 3, times the
      // row's band factor without FOLD
      float xrv[4], xiv[4];
      {
        const WaveScratch& W = wscr[n >> 3];
        const int rr = n & 7, ga = r10 >> 3, gb = r10 & 7;
        const float2 xa = FOLD == 4 && gb >= 4 ? W.xh[rr][ga] : W.xa[rr][ga];
        const float4 b01 = *reinterpret_cast<const float4*>(&W.xb[rr][gb]);
        const float4 b23 = *reinterpret_cast<const float4*>(&W.xb[rr][gb + 2]);
        const float2 xb[4] = {make_float2(b01.x, b01.y), make_float2(b01.z, b01.w), make_float2(b23.x, b23.y),
                              make_float2(b23.z, b23.w)};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float2 x = cmul(xa, xb[v]);
          if (!FOLD) {
            const float f = W.bf[rr][rseg[v]];
            x.x *= f;
            x.y *= f;
          }
          xrv[v] = x.x;
          xiv[v] = x.y;
        }
      }
      const float* kfr = bb.kf + bb.recb[n];
      float crv[4];
      float s1r = 0.f, s1i = 0.f;
      // Re(X Z) per row (the band sums) and X Z' (the frequency-weighted sum), both before the
      // scales 2^-eg, 2^-eg2, which are applied once per lane below
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float zr = acc[0][j][v] - acc[1][j][v], zi = acc[2][j][v];
        const float wr = acc[3][j][v] - acc[4][j][v], wi = acc[5][j][v];
        const float xr = xrv[v], xi = xiv[v];
        crv[v] = xr * zr - xi * zi;
        const float tr = xr * wr - xi * wi, ti = xr * wi + xi * wr;
        if (FOLD) {   // one band over the four rows: k applies to their sum
          s1r += tr;
          s1i += ti;
        } else {
          const float kv = kfr[rband[v]];
          s1r += kv * tr;
          s1i += kv * ti;
        }
      }
      const int grp = rbw * 4 + (lane >> 4);
      if (FOLD) {
        const float kv = kfr[rband[0]] * usw;
        bb.Rg[grp][n] = ((crv[0] + crv[1]) + (crv[2] + crv[3])) * usz;
        bb.R1[grp][n] = make_float2(kv * s1r, kv * s1i);
      } else {
        *reinterpret_cast<float4*>(&bb.R0[n][r10]) =
            make_float4(crv[0] * usz, crv[1] * usz, crv[2] * usz, crv[3] * usz);
        bb.R1[grp][n] = make_float2(s1r * usw, s1i * usw);
      }
    }
    __syncthreads();
    {
      // eight threads per record: row sums in FP64, bands j and j + 8.  Record n of this stage
      // was set up by lane 8 t + n % 8 of this same wave: its data arrive by shuffle.
      const int n = tid >> 3, j = tid & 7;
      const int src = t * RPW + (n & 7);
      const bool valid = __shfl(q.base, src) != -INFINITY;
      const int mat = __shfl(q.mat, src), kind = __shfl(q.kind, src);
      const float gux = __shfl(q.gux, src), guy = __shfl(q.guy, src), guz = __shfl(q.guz, src);
      const float gc1 = __shfl(q.gc1, src);
      const float glx = __shfl(q.glx, src), gly = __shfl(q.gly, src), glz = __shfl(q.glz, src);
      // partial sums of this thread (row groups 2 j, 2 j + 1; bands j, j + 8) in FP32, combined
      // over the record's eight threads in a fixed order
      float s1r = 0.f, s1i = 0.f;
      const int ngroups = SPLIT ? 8 : 16;   // row groups of 4 written this stage
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        if (2 * j + i >= ngroups) continue;
        const float2 c = bb.R1[2 * j + i][n];
        s1r += c.x;
        s1i += c.y;
      }
      float s0 = 0.f, wl = 0.f;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int b = j + 8 * h;
        float sb = 0.f;
        if (FOLD) {
          for (int gg = br0[h] >> 2; gg < br1[h] >> 2; ++gg) sb += bb.Rg[gg][n];
        } else {
          // the band's rows in four interleaved partial sums (independent LDS reads)
          const int e = br1[h];
          int r1 = br0[h];
          float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
          for (; r1 + 4 <= e; r1 += 4) {
            p0 += bb.R0[n][r1];
            p1 += bb.R0[n][r1 + 1];
            p2 += bb.R0[n][r1 + 2];
            p3 += bb.R0[n][r1 + 3];
          }
          for (; r1 < e; ++r1) p0 += bb.R0[n][r1];
          sb = (p0 + p1) + (p2 + p3);
        }
        // sb leaves out k for specular records: k sb is the band's share of H's sums, 2 sb its dL/dk
        float kvv = 0.f;
        if (b < a.Bk) {
          const float kb = kind == 0 ? bb.kf[mat * a.Bk + b] : 1.f;
          s0 += kb * sb;
          if (valid && kind == 0) {
            wl += kb * sb * bb.lobe_w[mat * a.Bk + b];
            kvv = 2.f * sb;
          }
        }
        if (b < a.Bk) bb.kv[b][n] = kvv;
      }
      s1r = sum8_first(s1r);
      s1i = sum8_first(s1i);
      s0 = sum8_first(s0);
      wl = sum8_first(wl);
      if (j == 0) bb.kmat[n] = valid && kind == 0 ? mat : -1;
      if (j == 0 && valid) {
        // d(ln A + j phi)/dx_m = [(-p/r - ln10 (a0 + a1 f)/20) + j sigma 2 pi f / c] u - d(gamma^2)/dx / (2 beta^2)
        const double cu = (double)gc1 * (double)s0 + c2 * (double)s1r + c3 * (double)s1i;
        const double g0 = 2.0 * cu * (double)gux + (double)wl * (double)glx;
        const double g1 = 2.0 * cu * (double)guy + (double)wl * (double)gly;
        const double g2 = 2.0 * cu * (double)guz + (double)wl * (double)glz;
        gx0 += g0; gx1 += g1; gx2 += g2;
      }
    }
    // the wave's records of this stage into dL/dk (their kv and kmat were written by this wave)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    dk_wave(bb, wv, lane, a.Q, a.Bk, dkc, t == 7);   // (nst is a multiple of 8)
  }
  __syncthreads();
  const size_t slot = ((size_t)p * gridDim.z + k1t) * a.M + m;
  const double gv[3] = {gx0, gx1, gx2};
  for (int c = 0; c < 3; ++c) {
    red[tid] = gv[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) gpx[slot * 3 + c] = red[0];
    __syncthreads();
  }
  // the four waves' totals of each (material, band), in wave order
  if (tid < QB) gpk[slot * QB + tid] = ((bb.dk[0][tid] + bb.dk[1][tid]) + bb.dk[2][tid]) + bb.dk[3][tid];
}

// One workgroup per output value (QB band coefficients, then 3 M receiver coordinates): its
// threads sum fixed strided subsets of the partials in FP64 and a fixed-shape tree in LDS adds
// the 256 sums, so the result does not depend on scheduling.
constexpr int RED_T = 256;
__global__ __launch_bounds__(RED_T) void k_bwd_reduce(const double* __restrict__ gpx, const double* __restrict__ gpk,
                                                      int32_t P, int32_t M, int32_t QB, double* __restrict__ grad_k,
                                                      double* __restrict__ grad_x) {
  __shared__ double red[RED_T];
  const int o = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  if (o < QB) {
    const int64_t n = (int64_t)P * M;   // partial (p, m) at gpk[((p M) + m) QB + o]
    for (int64_t e = tid; e < n; e += RED_T) s += gpk[e * QB + o];
  } else {
    const int i = o - QB;               // coordinate i = 3 m + c at gpx[p 3 M + i]
    for (int64_t p = tid; p < P; p += RED_T) s += gpx[p * M * 3 + i];
  }
  red[tid] = s;
  __syncthreads();
  for (int h = RED_T / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    if (o < QB) grad_k[o] = red[0];
    else grad_x[o - QB] = red[0];
  }
}

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

int choose_P(const et_sim_desc* sim, int64_t cap, bool mfma) {
  // matrix-core kernels: about sixteen workgroups per CU over the launch (measured on the
  // room's 32 x 4096 forward and adjoint: 2048 workgroups 11.20 / 20.16 ms, 3072 10.90 / 20.05,
  // 4096 10.76 / 19.87, 6144 10.75 / 19.98, 8192 10.73 / 19.92 ms).  Chunk count a multiple of 8
  // so that every receiver's workgroups of one chunk share an XCD's L2.
  const int64_t tiles = mfma ? (int64_t)sim->M * std::max<int64_t>(1, (sim->F / K2 + KT1 - 1) / KT1)
                             : (int64_t)sim->M * ((sim->F + DTILE - 1) / DTILE);
  const int64_t target = mfma ? 4096 : 2048;
  int64_t P = std::max<int64_t>(1, (target + tiles - 1) / tiles);
  if (P >= 8) P = (P + 7) / 8 * 8;
  P = std::min<int64_t>(P, std::max<int64_t>(1, cap / 64));
  return (int)std::min<int64_t>(P, 256);
}

size_t vis_ws(int64_t cap, char* base, size_t off, uint64_t** fl, uint64_t** of, int32_t** idx, void** tmp) {
  auto take = [&](size_t b) -> void* { void* p = base ? (void*)(base + off) : nullptr; off += al(b); return p; };
  *fl = (uint64_t*)take(sizeof(uint64_t) * (size_t)cap);
  *of = (uint64_t*)take(sizeof(uint64_t) * (size_t)cap);
  *idx = (int32_t*)take(sizeof(int32_t) * (size_t)cap);
  *tmp = take(scan_temp_bytes(cap));
  return off;
}

void build_tables(SynthArgs& a, const SynthWS& ws, hipStream_t s) {
  a.lk = ws.lk;
  a.lc = ws.lc;
  a.ld = ws.ld;
  a.lp = ws.lp;
  a.lmax = ws.lmax;
  const int n = a.Q * a.Bk;
  k_band_tables<<<(n + 255) / 256, 256, 0, s>>>(a, ws.lk, ws.lc, ws.ld, ws.lp, ws.lmax);
}

// Path-product reading: band tables with a row per record.  Specular record n: the sum of
// log2 k over its ray's specular records up to n (itself and its predecessors through prev)
// and its own lobe coefficient; a diffraction record: its material's log2 I_d.
__global__ void k_path_tables(et_paths P, SynthArgs a, const Ctl* ctl, float* __restrict__ plk,
                              float* __restrict__ plc) {
  const int Bk = a.Bk;
  const int64_t n_rec = ctl->n_rec;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rec * Bk;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = i / Bk;
    const int b = (int)(i - n * Bk);
    const int kind = (P.flags[n] >> 1) & 3;
    const int mat = P.mat[n];
    float s = 0.f, lobe = 0.f;
    if (kind == 0) {
      lobe = a.lc[mat * Bk + b];
      int64_t r = n;
      for (int guard = 0; guard < 256 && r >= 0; ++guard) {   // a ray has at most 255 reflections
        s += a.lk[P.mat[r] * Bk + b];
        const int64_t pr = P.prev[r];
        r = pr < r ? pr : -1;                                    // predecessors have smaller indices
      }
    } else if (kind == 1) {
      s = a.ld[mat * Bk + b];
    }
    plk[i] = s;
    plc[i] = lobe;
  }
}

// Per-receiver line of sight and the path-product reading for one pose's synthesis.
void set_readings(SynthArgs& a, const et_sim_desc* sim, const et_paths& P, const SynthWS& ws, Ctl* ctl,
                  hipStream_t s) {
  a.rxv = (sim->flags & ET_PER_RX_VISIBILITY) ? P.rx_vis : nullptr;
  if (sim->flags & ET_PATH_PRODUCT) {
    const int64_t n = ws.cap * sim->Bk;
    k_path_tables<<<(unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)), 256, 0, s>>>(
        P, a, ctl, ws.plk, ws.plc);
    ET_HIP(hipGetLastError());
    a.lk = ws.plk;
    a.lc = ws.plc;
    a.ld = ws.plk;
    a.rec_rows = 1;
  }
}

size_t table_ws(const et_sim_desc* sim, char* base, size_t off, SynthWS& w) {
  const size_t n = (size_t)sim->Q * sim->Bk;
  w.lk = (float*)(base ? base + off : nullptr);
  off += al(sizeof(float) * n);
  w.lc = (float*)(base ? base + off : nullptr);
  off += al(sizeof(float) * n);
  w.ld = (float*)(base ? base + off : nullptr);
  off += al(sizeof(float) * n);
  w.lp = (float*)(base ? base + off : nullptr);
  off += al(sizeof(float) * sim->Bk);
  w.lmax = (float*)(base ? base + off : nullptr);
  off += al(sizeof(float) * (3 * (size_t)sim->Q + 1));
  return off;
}

void build_vis(const et_paths& P, const SynthWS& ws, int64_t cap, Ctl* ctl, hipStream_t s) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap + 255) / 256, 4096));
  k_vis_flags<<<nb, 256, 0, s>>>(P, ctl, ws.vflags);
  scan_exclusive_u64(ws.vflags, ws.voffs, 0, &ctl->n_rec, cap, &ctl->tot[3], ws.vscan, s);
  k_vis_scatter<<<nb, 256, 0, s>>>(ws.vflags, ws.voffs, ctl, ws.vidx);
  k_vis_count<<<1, 1, 0, s>>>(ctl);
  ET_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ fused batches

constexpr int SJOB_PACK = 16;
struct SynthJobPack {
  SynthArgs j[SJOB_PACK];
  int32_t first, n;
};
static_assert(sizeof(SynthJobPack) <= 4000, "job pack must fit the kernel argument space");

__global__ void k_put_synth_jobs(SynthJobPack pk, SynthArgs* __restrict__ dst) {
  if ((int)threadIdx.x < pk.n) dst[pk.first + threadIdx.x] = pk.j[threadIdx.x];
}

// workgroup j fills job j's band tables (its lk / lc / ld / lp point into the batch's table block)
__global__ void k_band_tables_batch(const SynthArgs* __restrict__ jobs) {
  const SynthArgs a = jobs[blockIdx.x];
  for (int i = threadIdx.x; i < a.Q * a.Bk; i += blockDim.x)
    band_table_entry(a, i, const_cast<float*>(a.lk), const_cast<float*>(a.lc), const_cast<float*>(a.ld),
                     const_cast<float*>(a.lp));
  for (int q = threadIdx.x; q < a.Q; q += blockDim.x) band_bound_entry(a, q, const_cast<float*>(a.lmax));
}

// sort key of each visible record: its job (the ray field of a batch record)
__global__ void k_vis_jobkeys(et_paths P, const int32_t* __restrict__ idx, const Ctl* ctl, uint64_t* __restrict__ keys) {
  const int64_t n = ctl->n_vis;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = (uint64_t)(uint32_t)P.ray[idx[i]];
}

// Per-job ranges of the job-sorted visible list and chunk offsets: chunks of
// per = ceil(n_vis / target) records, never crossing a job.  One workgroup.
__global__ void k_job_chunks(const uint64_t* __restrict__ keys, const Ctl* ctl, int32_t J, int64_t target,
                             int64_t* __restrict__ off, int64_t* __restrict__ lo, int64_t* __restrict__ hi,
                             int64_t* __restrict__ per) {
  const int64_t n = ctl->n_vis;
  const int64_t pc = std::max<int64_t>(1, (n + target - 1) / target);
  for (int j = threadIdx.x; j < J; j += blockDim.x) {
    int64_t a = 0, b = n;   // first position with key >= j
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if (keys[mid] < (uint64_t)j) a = mid + 1;
      else b = mid;
    }
    const int64_t l = a;
    b = n;                  // first position with key >= j + 1
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if (keys[mid] < (uint64_t)j + 1) a = mid + 1;
      else b = mid;
    }
    lo[j] = l;
    hi[j] = a;
    off[j + 1] = (a - l + pc - 1) / pc;   // chunk count, turned into offsets below
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    off[0] = 0;
    for (int j = 0; j < J; ++j) off[j + 1] += off[j];
    per[0] = pc;
  }
}

__global__ void k_reduce_batch(const float* __restrict__ part, ChunkTab ct, int64_t MF2, float* __restrict__ out) {
  const int64_t total = (int64_t)ct.J * MF2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / MF2, r = e - j * MF2;
    float s = 0.f;
    for (int64_t c = ct.off[j]; c < ct.off[j + 1]; ++c) s += part[c * MF2 + r];
    out[e] = s;
  }
}

// per job: dL/dk[Q Bk] and dL/dx[M][3] summed over its chunks, tiles and receivers in a fixed order
__global__ void k_bwd_reduce_batch(const double* __restrict__ gpx, const double* __restrict__ gpk, ChunkTab ct,
                                   int32_t T1, int32_t M, int32_t QB, double* __restrict__ grad_k,
                                   double* __restrict__ grad_x) {
  const int per_job = max(QB, 3 * M);
  const int64_t total = (int64_t)ct.J * per_job;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / per_job;
    const int i = (int)(e - j * per_job);
    if (i < QB) {
      double s = 0.0;
      for (int64_t c = ct.off[j]; c < ct.off[j + 1]; ++c)
        for (int t = 0; t < T1; ++t)
          for (int m = 0; m < M; ++m) s += gpk[(((size_t)c * T1 + t) * M + m) * QB + i];
      grad_k[j * QB + i] = s;
    }
    if (i < 3 * M) {
      double s = 0.0;
      for (int64_t c = ct.off[j]; c < ct.off[j + 1]; ++c)
        for (int t = 0; t < T1; ++t) s += gpx[((size_t)c * T1 + t) * M * 3 + i];
      grad_x[j * 3 * M + i] = s;
    }
  }
}

}  // namespace

// Every material (and directivity) band edge on a multiple of g outer indices (64 g bins) and
// the bins a multiple of 64 g.
bool bands_on_groups(const et_sim_desc* sim, int64_t g) {
  const int64_t F = sim->F, Bk = sim->Bk, Bd = sim->directivity ? sim->Bd : 0, K1 = F / K2;
  if (K1 % g) return false;
  for (int64_t k1 = 1; k1 < K1; ++k1) {
    if (k1 % g == 0) continue;
    const int64_t k = k1 * K2, kp = k - K2;
    if (k * Bk / F != kp * Bk / F) return false;
    if (Bd && k * Bd / F != kp * Bd / F) return false;
  }
  return true;
}

// How the band factor rides on the generating factors (forward and adjoint): 8 when every band
// edge falls on a multiple of 512 bins and the bins are a multiple of 512, 4 for 256, 0 (a table
// of band factors) otherwise.
int bands_fold(const et_sim_desc* sim) { return bands_on_groups(sim, 8) ? 8 : bands_on_groups(sim, 4) ? 4 : 0; }

template <bool BATCH, bool SPLIT>
void launch_fwd_fold(int fold, dim3 grid, hipStream_t s, const SynthArgs& a, const SynthArgs* jobs, const ChunkTab& ct,
                     const et_paths& P, const int32_t* idx, const Ctl* ctl, float* part) {
  if (fold == 8) k_synth_mfma<BATCH, SPLIT, 8><<<grid, 256, 0, s>>>(a, jobs, ct, P, idx, ctl, part);
  else if (fold == 4) k_synth_mfma<BATCH, SPLIT, 4><<<grid, 256, 0, s>>>(a, jobs, ct, P, idx, ctl, part);
  else k_synth_mfma<BATCH, SPLIT, 0><<<grid, 256, 0, s>>>(a, jobs, ct, P, idx, ctl, part);
}

template <bool BATCH>
void launch_fwd_mfma(bool split, int fold, dim3 grid, hipStream_t s, const SynthArgs& a, const SynthArgs* jobs,
                     const ChunkTab& ct, const et_paths& P, const int32_t* idx, const Ctl* ctl, float* part) {
  if (split) launch_fwd_fold<BATCH, true>(fold, grid, s, a, jobs, ct, P, idx, ctl, part);
  else launch_fwd_fold<BATCH, false>(fold, grid, s, a, jobs, ct, P, idx, ctl, part);
}

bool synth_factorised_ok(const et_sim_desc* sim) {
  // needs k = 64 k1 + k2, material / directivity bands constant over each run of 64 bins
  // (the band factor is per outer index), and at most SMAX band segments per tile of KT1
  // outer indices
  if (sim->flags & ET_SYNTH_DIRECT) return false;
  if (sim->F < K2 || sim->F % K2) return false;
  const int64_t F = sim->F, Bk = sim->Bk, Bd = sim->directivity ? sim->Bd : 0;
  int nseg = 0;
  int64_t pb = -1, pd = -1;
  for (int64_t k1 = 0; k1 < F / K2; ++k1) {
    const int64_t ka = k1 * K2, kb = ka + K2 - 1;
    const int64_t b = ka * Bk / F, d = Bd ? ka * Bd / F : 0;
    if (b != kb * Bk / F) return false;
    if (Bd && d != kb * Bd / F) return false;
    if (k1 % KT1 == 0) nseg = 0;
    if (k1 % KT1 == 0 || b != pb || d != pd) ++nseg;
    if (nseg > SMAX) return false;
    pb = b;
    pd = d;
  }
  return true;
}

size_t synth_ws_layout(const et_sim_desc* sim, int64_t cap, char* base, SynthWS* ws) {
  cap = std::max<int64_t>(cap, 1);
  const bool mf = synth_factorised_ok(sim);
  const int P = choose_P(sim, cap, mf);
  size_t off = 0;
  SynthWS w{};
  w.P = P;
  w.cap = cap;
  w.partial = (float*)(base ? base + off : nullptr);
  off += al(sizeof(float) * 2 * (size_t)P * sim->M * sim->F);
  off = vis_ws(cap, base, off, &w.vflags, &w.voffs, &w.vidx, &w.vscan);
  off = table_ws(sim, base, off, w);
  if (sim->flags & ET_PATH_PRODUCT) {
    w.plk = (float*)(base ? base + off : nullptr);
    off += al(sizeof(float) * (size_t)cap * sim->Bk);
    w.plc = (float*)(base ? base + off : nullptr);
    off += al(sizeof(float) * (size_t)cap * sim->Bk);
  }
  if (ws) *ws = w;
  return off;
}

int synth_run(const et_sim_desc* sim, const et_paths* paths, const SynthWS& ws, Ctl* ctl, float* spectra, hipStream_t s,
              hipEvent_t kb, hipEvent_t ke) {
  const bool mf = synth_factorised_ok(sim);
  SynthArgs a = make_args(sim, ws.P);
  const et_paths P = *paths;
  build_vis(P, ws, ws.cap, ctl, s);
  build_tables(a, ws, s);
  set_readings(a, sim, P, ws, ctl, s);
  if (kb) ET_HIP(hipEventRecord(kb, s));
  if (mf) {
    const int K1 = sim->F / K2;
    dim3 grid(ws.P, sim->M, (K1 + KT1 - 1) / KT1);
    launch_fwd_mfma<false>(K1 <= 32, bands_fold(sim), grid, s, a, nullptr, ChunkTab{}, P, ws.vidx, ctl,
                           ws.partial);
  } else {
    dim3 grid(ws.P, sim->M, (sim->F + DTILE - 1) / DTILE);
    k_synth_direct<false><<<grid, DB, 0, s>>>(a, nullptr, ChunkTab{}, P, ws.vidx, ctl, ws.partial);
  }
  if (ke) ET_HIP(hipEventRecord(ke, s));
  const int64_t MF2 = (int64_t)sim->M * sim->F * 2;
  k_reduce_partials<<<(unsigned)std::min<int64_t>((MF2 + 255) / 256, 4096), 256, 0, s>>>(ws.partial, ws.P, MF2, spectra);
  ET_HIP(hipGetLastError());
  return mf ? 1 : 2;
}

int synth_run_noalloc(const et_sim_desc* sim, const et_paths* paths, void* buf, size_t bytes, Ctl* ctl,
                      float* spectra, hipStream_t s, hipEvent_t kb, hipEvent_t ke) {
  ET_CHECK(!(sim->flags & ET_PATH_PRODUCT), ET_E_UNSUPPORTED,
           "ET_PATH_PRODUCT needs per-record tables (a workspace): use et_synthesize");
  const bool mf = synth_factorised_ok(sim);
  const int64_t cap = std::max<int64_t>(paths->capacity, 1);
  SynthWS w{};
  const size_t tables = table_ws(sim, nullptr, 0, w);
  const size_t chunk = al(sizeof(float) * 2 * (size_t)sim->M * sim->F);
  ET_CHECK(tables + chunk <= bytes, ET_E_UNSUPPORTED,
           "receivers x bins too large for the device scratch of the allocation-free call");
  // record chunks: the usual choice, as many as the scratch holds, a multiple of 8 above 8
  int64_t P = std::min<int64_t>(choose_P(sim, cap, mf), (int64_t)((bytes - tables) / chunk));
  if (P > 8) P = P / 8 * 8;
  char* base = (char*)buf;
  table_ws(sim, base, 0, w);
  w.partial = (float*)(base + tables);
  w.P = (int)P;
  w.cap = cap;
  SynthArgs a = make_args(sim, w.P);
  const et_paths Pth = *paths;
  k_vis_all<<<1, 1, 0, s>>>(ctl);
  build_tables(a, w, s);
  a.rxv = (sim->flags & ET_PER_RX_VISIBILITY) ? Pth.rx_vis : nullptr;
  if (kb) ET_HIP(hipEventRecord(kb, s));
  if (mf) {
    const int K1 = sim->F / K2;
    dim3 grid(w.P, sim->M, (K1 + KT1 - 1) / KT1);
    launch_fwd_mfma<false>(K1 <= 32, bands_fold(sim), grid, s, a, nullptr, ChunkTab{}, Pth, nullptr, ctl,
                           w.partial);
  } else {
    dim3 grid(w.P, sim->M, (sim->F + DTILE - 1) / DTILE);
    k_synth_direct<false><<<grid, DB, 0, s>>>(a, nullptr, ChunkTab{}, Pth, nullptr, ctl, w.partial);
  }
  if (ke) ET_HIP(hipEventRecord(ke, s));
  const int64_t MF2 = (int64_t)sim->M * sim->F * 2;
  k_reduce_partials<<<(unsigned)std::min<int64_t>((MF2 + 255) / 256, 4096), 256, 0, s>>>(w.partial, w.P, MF2, spectra);
  ET_HIP(hipGetLastError());
  return mf ? 1 : 2;
}

bool synth_bwd_factorised_ok(const et_sim_desc* sim) { return !sim->directivity && synth_factorised_ok(sim); }

template <bool BATCH, bool SPLIT>
void launch_bwd_fold(int fold, dim3 grid, hipStream_t s, const SynthArgs& a, const SynthArgs* jobs, const ChunkTab& ct,
                     const et_paths& P, const int32_t* idx, const Ctl* ctl, const float* g, double* gpx,
                     double* gpk) {
  if (fold == 8) k_synth_bwd_mfma<BATCH, SPLIT, 8><<<grid, 256, 0, s>>>(a, jobs, ct, P, idx, ctl, g, gpx, gpk);
  else if (fold == 4) k_synth_bwd_mfma<BATCH, SPLIT, 4><<<grid, 256, 0, s>>>(a, jobs, ct, P, idx, ctl, g, gpx, gpk);
  else k_synth_bwd_mfma<BATCH, SPLIT, 0><<<grid, 256, 0, s>>>(a, jobs, ct, P, idx, ctl, g, gpx, gpk);
}

template <bool BATCH>
void launch_bwd_mfma(bool split, int fold, dim3 grid, hipStream_t s, const SynthArgs& a, const SynthArgs* jobs,
                     const ChunkTab& ct, const et_paths& P, const int32_t* idx, const Ctl* ctl, const float* g,
                     double* gpx, double* gpk) {
  if (split) launch_bwd_fold<BATCH, true>(fold, grid, s, a, jobs, ct, P, idx, ctl, g, gpx, gpk);
  else launch_bwd_fold<BATCH, false>(fold, grid, s, a, jobs, ct, P, idx, ctl, g, gpx, gpk);
}

size_t synth_bwd_ws_layout(const et_sim_desc* sim, int64_t cap, char* base, SynthWS* ws) {
  cap = std::max<int64_t>(cap, 1);
  const bool mf = synth_bwd_factorised_ok(sim);
  const int64_t T1 = mf ? (sim->F / K2 + KT1 - 1) / KT1 : 1;
  int64_t P;
  if (mf) {
    P = choose_P(sim, cap, true);
  } else {
    P = std::max<int64_t>(1, (1024 + sim->M - 1) / sim->M);
    P = std::min<int64_t>(P, std::max<int64_t>(1, (cap + GB - 1) / GB));
    P = std::min<int64_t>(P, 256);
  }
  size_t off = 0;
  SynthWS w{};
  w.gchunks = (int)P;
  w.gtiles = (int)T1;
  w.cap = cap;
  w.gpart_x = (double*)(base ? base + off : nullptr);
  off += al(sizeof(double) * 3 * (size_t)P * T1 * sim->M);
  w.gpart_k = (double*)(base ? base + off : nullptr);
  off += al(sizeof(double) * (size_t)P * T1 * sim->M * sim->Q * sim->Bk);
  off = vis_ws(cap, base, off, &w.vflags, &w.voffs, &w.vidx, &w.vscan);
  off = table_ws(sim, base, off, w);
  if (ws) *ws = w;
  return off;
}

int synth_bwd_run(const et_sim_desc* sim, const et_paths* paths, const float* grad_spectra, const SynthWS& ws,
                  Ctl* ctl, double* grad_k, double* grad_rx, hipStream_t s, hipEvent_t kb, hipEvent_t ke) {
  const bool mf = synth_bwd_factorised_ok(sim);
  SynthArgs a = make_args(sim, ws.gchunks);
  const et_paths P = *paths;
  build_vis(P, ws, ws.cap, ctl, s);
  build_tables(a, ws, s);
  a.rxv = (sim->flags & ET_PER_RX_VISIBILITY) ? P.rx_vis : nullptr;   // (no path product in the adjoint)
  if (kb) ET_HIP(hipEventRecord(kb, s));
  if (mf) {
    dim3 grid(ws.gchunks, sim->M, ws.gtiles);
    launch_bwd_mfma<false>(sim->F / K2 <= 32, bands_fold(sim), grid, s, a, nullptr, ChunkTab{}, P, ws.vidx, ctl,
                           grad_spectra, ws.gpart_x, ws.gpart_k);
  } else {
    dim3 grid(ws.gchunks, sim->M);
    const size_t shm = sizeof(float2) * (size_t)sim->F;
    k_synth_bwd<false><<<grid, GB, shm, s>>>(a, nullptr, ChunkTab{}, P, ws.vidx, ctl, grad_spectra, ws.gpart_x,
                                             ws.gpart_k);
  }
  if (ke) ET_HIP(hipEventRecord(ke, s));
  const int QB = sim->Q * sim->Bk;
  k_bwd_reduce<<<QB + 3 * sim->M, RED_T, 0, s>>>(ws.gpart_x, ws.gpart_k, ws.gchunks * ws.gtiles, sim->M, QB, grad_k,
                                                grad_rx);
  ET_HIP(hipGetLastError());
  return mf ? 1 : 2;
}


// ------------------------------------------------------------------ fused batches (host)

namespace {
int chunk_target(const et_sim_desc* s0, bool mf, int32_t wgs) {
  // record chunks over the whole batch for about `wgs` workgroups of the main kernel
  const int64_t per_chunk = mf ? (int64_t)s0->M * std::max<int64_t>(1, (s0->F / K2 + KT1 - 1) / KT1)
                               : (int64_t)s0->M * ((s0->F + DTILE - 1) / DTILE);
  return (int)std::max<int64_t>(1, (wgs + per_chunk - 1) / per_chunk);
}
}  // namespace

bool synth_batch_factorised(int32_t J, const et_job* jobs, bool adjoint) {
  for (int32_t i = 0; i < J; ++i)
    if (!(adjoint ? synth_bwd_factorised_ok(jobs[i].sim) : synth_factorised_ok(jobs[i].sim))) return false;
  return true;
}

size_t synth_batch_ws_layout(int32_t J, const et_job* jobs, int64_t cap, const BatchTune& tune, bool adjoint,
                             char* base, SynthBatchWS* ws) {
  const et_sim_desc* s0 = jobs[0].sim;
  cap = std::max<int64_t>(cap, 1);
  SynthBatchWS w{};
  w.J = J;
  w.cap = cap;
  w.mf = synth_batch_factorised(J, jobs, false);
  w.mf_bwd = adjoint && synth_batch_factorised(J, jobs, true);
  w.fold = 8;   // the coarsest folding every job allows
  for (int32_t i = 0; i < J; ++i) w.fold = std::min(w.fold, bands_fold(jobs[i].sim));
  w.target = chunk_target(s0, w.mf, tune.synth_wgs);
  w.target_bwd = chunk_target(s0, w.mf_bwd, tune.adjoint_wgs);
  // grid size: the chunk count is at most target + J (sum_j ceil(n_j / per)); buffers are
  // sized for the largest target the tuner tries, so that tuning keeps the workspace valid
  w.chunks = w.target + J;
  w.chunks_bwd = w.target_bwd + J;
  const int64_t cmax = chunk_target(s0, w.mf, TUNE_MAX_WGS) + J;
  const int64_t cmax_bwd = chunk_target(s0, w.mf_bwd, TUNE_MAX_WGS) + J;
  w.T1 = w.mf_bwd ? (int)((s0->F / K2 + KT1 - 1) / KT1) : 1;
  size_t off = 0;
  auto take = [&](size_t b) -> void* { void* p = base ? (void*)(base + off) : nullptr; off += al(b); return p; };
  const size_t MF2 = (size_t)s0->M * s0->F * 2;
  w.partial = (float*)take(sizeof(float) * MF2 * (size_t)std::max<int64_t>(cmax, w.chunks));
  if (adjoint) {
    const size_t cb = (size_t)std::max<int64_t>(cmax_bwd, w.chunks_bwd);
    w.gpart_x = (double*)take(sizeof(double) * 3 * cb * w.T1 * s0->M);
    w.gpart_k = (double*)take(sizeof(double) * cb * w.T1 * s0->M * s0->Q * s0->Bk);
  }
  off = vis_ws(cap, base, off, &w.vflags, &w.voffs, &w.vidx, &w.vscan);
  w.keys = (uint64_t*)take(sizeof(uint64_t) * (size_t)cap);
  w.sort_tmp = take(sort_temp_bytes(cap, 8));
  w.tab = (int64_t*)take(sizeof(int64_t) * (size_t)(3 * J + 2) * 2);
  w.jobs = take(sizeof(SynthArgs) * (size_t)J);
  w.tables = (float*)take(sizeof(float) * (size_t)J * (4 * (size_t)s0->Q * s0->Bk + 3 * s0->Q + 1));
  if (ws) *ws = w;
  return off;
}

namespace {
ChunkTab chunk_tab(const SynthBatchWS& w, int which) {
  int64_t* t = w.tab + (size_t)which * (3 * w.J + 2);
  return ChunkTab{t, t + w.J + 1, t + 2 * w.J + 1, t + 3 * w.J + 1, w.J};
}
}  // namespace

int synth_batch_run(int32_t J, const et_job* jobs, const et_paths* paths, const SynthBatchWS& w, Ctl* ctl,
                    float* spectra, const float* grad, double* grad_k, double* grad_rx, int* adjoint_kernel,
                    const hipEvent_t* ev, hipStream_t s) {
  const et_sim_desc* s0 = jobs[0].sim;
  const et_paths P = *paths;
  const int QB = s0->Q * s0->Bk;
  // job table with per-job band tables
  SynthArgs* dj = (SynthArgs*)w.jobs;
  SynthJobPack pk{};
  for (int32_t i = 0; i < J; ++i) {
    SynthArgs a = make_args(jobs[i].sim, 0);
    a.lk = w.tables + (size_t)i * (4 * QB + 3 * s0->Q + 1);
    a.lc = a.lk + QB;
    a.ld = a.lc + QB;
    a.lp = a.ld + QB;
    a.lmax = a.lp + QB;
    pk.j[pk.n++] = a;
    if (pk.n == SJOB_PACK || i + 1 == J) {
      k_put_synth_jobs<<<1, SJOB_PACK, 0, s>>>(pk, dj);
      pk.first += pk.n;
      pk.n = 0;
    }
  }
  k_band_tables_batch<<<J, 256, 0, s>>>(dj);
  // visible records, sorted by job (stable: each job keeps its record order)
  SynthWS vw{};
  vw.vflags = w.vflags; vw.voffs = w.voffs; vw.vidx = w.vidx; vw.vscan = w.vscan;
  build_vis(P, vw, w.cap, ctl, s);
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((w.cap + 255) / 256, 4096));
  k_vis_jobkeys<<<nb, 256, 0, s>>>(P, w.vidx, ctl, w.keys);
  int bits = 0;
  while ((1ll << bits) < (int64_t)J) ++bits;
  if (bits > 0) radix_sort_u64(w.keys, w.vidx, 0, &ctl->n_vis, w.cap, bits, w.sort_tmp, s);
  const int64_t MF2 = (int64_t)s0->M * s0->F * 2;
  // forward
  {
    const ChunkTab ct = chunk_tab(w, 0);
    k_job_chunks<<<1, 256, 0, s>>>(w.keys, ctl, J, w.target, const_cast<int64_t*>(ct.off), const_cast<int64_t*>(ct.lo),
                                   const_cast<int64_t*>(ct.hi), const_cast<int64_t*>(ct.per));
    const SynthArgs a0 = make_args(s0, 0);
    if (ev) ET_HIP(hipEventRecord(ev[0], s));
    if (w.mf) {
      dim3 grid(w.chunks, s0->M, (s0->F / K2 + KT1 - 1) / KT1);
      launch_fwd_mfma<true>(s0->F / K2 <= 32, w.fold, grid, s, a0, dj, ct, P, w.vidx, ctl, w.partial);
    } else {
      dim3 grid(w.chunks, s0->M, (s0->F + DTILE - 1) / DTILE);
      k_synth_direct<true><<<grid, DB, 0, s>>>(a0, dj, ct, P, w.vidx, ctl, w.partial);
    }
    if (ev) ET_HIP(hipEventRecord(ev[1], s));
    k_reduce_batch<<<(unsigned)std::min<int64_t>((J * MF2 + 255) / 256, 8192), 256, 0, s>>>(w.partial, ct, MF2, spectra);
  }
  if (grad) {
    const ChunkTab ct = chunk_tab(w, 1);
    k_job_chunks<<<1, 256, 0, s>>>(w.keys, ctl, J, w.target_bwd, const_cast<int64_t*>(ct.off),
                                   const_cast<int64_t*>(ct.lo), const_cast<int64_t*>(ct.hi), const_cast<int64_t*>(ct.per));
    const SynthArgs a0 = make_args(s0, 0);
    if (ev) ET_HIP(hipEventRecord(ev[2], s));
    if (w.mf_bwd) {
      dim3 grid(w.chunks_bwd, s0->M, w.T1);
      launch_bwd_mfma<true>(s0->F / K2 <= 32, w.fold, grid, s, a0, dj, ct, P, w.vidx, ctl, grad, w.gpart_x,
                            w.gpart_k);
    } else {
      dim3 grid(w.chunks_bwd, s0->M);
      k_synth_bwd<true><<<grid, GB, sizeof(float2) * (size_t)s0->F, s>>>(a0, dj, ct, P, w.vidx, ctl, grad, w.gpart_x,
                                                                         w.gpart_k);
    }
    if (ev) ET_HIP(hipEventRecord(ev[3], s));
    const int64_t n = (int64_t)J * std::max(QB, 3 * s0->M);
    k_bwd_reduce_batch<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(
        w.gpart_x, w.gpart_k, ct, w.T1, s0->M, QB, grad_k, grad_rx);
    if (adjoint_kernel) *adjoint_kernel = w.mf_bwd ? 1 : 2;
  }
  ET_HIP(hipGetLastError());
  return w.mf ? 1 : 2;
}

__global__ void k_sum_spectra(const float* __restrict__ in, int32_t J, int64_t n, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int32_t j = 0; j < J; ++j) acc += in[(size_t)j * n + i];
    out[i] = acc;
  }
}

void sum_spectra(const float* in, int32_t J, int64_t n, float* out, hipStream_t s) {
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384));
  k_sum_spectra<<<grid, 256, 0, s>>>(in, J, n, out);
  ET_HIP(hipGetLastError());
}

}  // namespace et
