// Ray tracing of one pose (Sec. III-C, Algorithm 1) and diffraction sampling (Sec. III-D).
//
// Per bounce j, over the compacted list of active rays:
//   k_bounce   FP32 closest-hit BVH traversal of the FP64 ray rounded to FP32 (which
//              triangle), FP64 plane intersection, specular reflection about the face
//              normal and path-length update (where), FP32 any-hit line-of-sight ray from
//              the hit point toward x_ref
//   scan       exclusive scan of (hit, continue) flags
//   k_scatter  stable compaction: records in ray order after the earlier bounces' records,
//              next-bounce ray state in ray order
// Ray order: a ray set larger than one round of the bounce grid (the threads the chip holds at
// once) is first sorted (stably) by a 16-bit octahedral Morton key of its world direction, so
// that a wave's lanes walk nearby parts of the BVH; the stable compaction keeps that order
// through the bounces, and records carry their ray.  Measured in the room: 2^20 rays trace in
// 3.9 ms sorted against 5.3 ms in seeded order, 2^19 in 2.46 against 2.57 ms; at 2^18 rays,
// which one round holds, the bounce kernel is slower on sorted rays (0.245 against 0.191 ms per
// launch), so such sets keep their given order.
// Traversal: one lane per ray, binary BVH, nearest child first, per-lane stack in LDS
// (spilling to global memory past TRAV_LDS_STACK entries), leaves postponed until a quarter
// of the wave's lanes hold one (after Aila & Laine, HPG 2009), watertight ray-triangle test
// (Woop, Benthin & Wald, JCGT 2013), conservative slab test (Ize 2013).
#include "internal.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>

namespace et {

namespace {

constexpr int BS = TRAV_BLOCK;
constexpr int EMPTY = INT32_MIN;
// Bounce grids of up to 8192 blocks: the room's 2^20 rays run one per thread, so the hardware
// dispatcher balances uneven rays block by block (measured 7% faster than two rays per thread
// on 2048 blocks, whose second round leaves part of the chip idle).
constexpr int MAX_BLOCKS = 8192;

inline unsigned nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + BS - 1) / BS, MAX_BLOCKS)); }
inline unsigned nblk_full(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + BS - 1) / BS); }

struct Ray32 {
  float ox, oy, oz;
  float ix, iy, iz;          // reciprocal direction (tiny components clamped)
  float okx, oky, okz;       // origin permuted for the watertight test
  float Sx, Sy, Sz;          // shear constants
  int kx, ky, kz;
};

__device__ inline float sel3(float a, float b, float c, int k) { return k == 0 ? a : (k == 1 ? b : c); }

__device__ inline float safe_rcp(float d) {
  const float tiny = 1e-30f;
  return 1.0f / (fabsf(d) < tiny ? (d < 0.f ? -tiny : tiny) : d);
}

__device__ inline Ray32 make_ray(double ox, double oy, double oz, double dx, double dy, double dz) {
  Ray32 r;
  r.ox = (float)ox; r.oy = (float)oy; r.oz = (float)oz;
  const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
  r.ix = safe_rcp(fx); r.iy = safe_rcp(fy); r.iz = safe_rcp(fz);
  const float ax = fabsf(fx), ay = fabsf(fy), az = fabsf(fz);
  int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  int kx = kz + 1 == 3 ? 0 : kz + 1;
  int ky = kx + 1 == 3 ? 0 : kx + 1;
  const float dkz = sel3(fx, fy, fz, kz);
  if (dkz < 0.f) { int t = kx; kx = ky; ky = t; }
  r.kx = kx; r.ky = ky; r.kz = kz;
  r.Sx = sel3(fx, fy, fz, kx) / dkz;
  r.Sy = sel3(fx, fy, fz, ky) / dkz;
  r.Sz = 1.0f / dkz;
  r.okx = sel3(r.ox, r.oy, r.oz, kx);
  r.oky = sel3(r.ox, r.oy, r.oz, ky);
  r.okz = sel3(r.ox, r.oy, r.oz, kz);
  return r;
}

// Slab test against both child boxes; far distances widened by 1 + 2*gamma(3) (Ize 2013)
// so that FP32 rounding never rejects a box that the exact ray meets.
__device__ inline void box2(const Node2& n, const Ray32& r, float tmin, float tmax, bool& h0, bool& h1, float& t0,
                            float& t1) {
  const float up = 1.0f + 2.0f * 3.5762786865234375e-7f;   // 1 + 2 * gamma_3, gamma_n = n u / (1 - n u)
  float lx = (n.xy0.x - r.ox) * r.ix, hx = (n.xy0.y - r.ox) * r.ix;
  float ly = (n.xy0.z - r.oy) * r.iy, hy = (n.xy0.w - r.oy) * r.iy;
  float lz = (n.zz.x - r.oz) * r.iz, hz = (n.zz.y - r.oz) * r.iz;
  float tn = fmaxf(fmaxf(fminf(lx, hx), fminf(ly, hy)), fmaxf(fminf(lz, hz), tmin));
  float tf = fminf(fminf(fmaxf(lx, hx), fmaxf(ly, hy)), fmaxf(lz, hz)) * up;
  h0 = tn <= fminf(tf, tmax);
  t0 = tn;
  lx = (n.xy1.x - r.ox) * r.ix; hx = (n.xy1.y - r.ox) * r.ix;
  ly = (n.xy1.z - r.oy) * r.iy; hy = (n.xy1.w - r.oy) * r.iy;
  lz = (n.zz.z - r.oz) * r.iz; hz = (n.zz.w - r.oz) * r.iz;
  tn = fmaxf(fmaxf(fminf(lx, hx), fminf(ly, hy)), fmaxf(fminf(lz, hz), tmin));
  tf = fminf(fminf(fmaxf(lx, hx), fmaxf(ly, hy)), fmaxf(lz, hz)) * up;
  h1 = tn <= fminf(tf, tmax);
  t1 = tn;
}

// Watertight ray-triangle test, two-sided.  Returns t (or a negative value on a miss).
__device__ inline float tri_test(const float4 a, const float4 b, const float4 c, const Ray32& r) {
#pragma clang fp contract(off)
  const float Ax0 = sel3(a.x, a.y, a.z, r.kx) - r.okx, Ay0 = sel3(a.x, a.y, a.z, r.ky) - r.oky,
              Az0 = sel3(a.x, a.y, a.z, r.kz) - r.okz;
  const float Bx0 = sel3(b.x, b.y, b.z, r.kx) - r.okx, By0 = sel3(b.x, b.y, b.z, r.ky) - r.oky,
              Bz0 = sel3(b.x, b.y, b.z, r.kz) - r.okz;
  const float Cx0 = sel3(c.x, c.y, c.z, r.kx) - r.okx, Cy0 = sel3(c.x, c.y, c.z, r.ky) - r.oky,
              Cz0 = sel3(c.x, c.y, c.z, r.kz) - r.okz;
  const float Ax = Ax0 - r.Sx * Az0, Ay = Ay0 - r.Sy * Az0;
  const float Bx = Bx0 - r.Sx * Bz0, By = By0 - r.Sy * Bz0;
  const float Cx = Cx0 - r.Sx * Cz0, Cy = Cy0 - r.Sy * Cz0;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.f || V == 0.f || W == 0.f) {   // exact edge: decide in double (watertightness)
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return -1.f;
  const float det = U + V + W;
  if (det == 0.f) return -1.f;
  const float Az = r.Sz * Az0, Bz = r.Sz * Bz0, Cz = r.Sz * Cz0;
  const float T = U * Az + V * Bz + W * Cz;
  return T / det;
}

struct Stack {
  int* lds;        // this lane's column: entry i at lds[i * BS]
  int* glob;       // this lane's global column: entry i at glob[i * gstride]
  int64_t gstride;
  int sp;
  int cap;         // entries in use: TRAV_STACK (lower only when a test forces overflows)
  int overflow;
  // A push beyond the cap drops the subtree (counted; the traversal still ends normally).
  __device__ inline void push(int v) {
    if (sp >= cap) { ++overflow; return; }
    if (sp < TRAV_LDS_STACK) lds[sp * BS] = v;
    else glob[(int64_t)(sp - TRAV_LDS_STACK) * gstride] = v;
    ++sp;
  }
  // The global part is read as a non-temporal load, so the compiler keeps the two reads apart
  // (an LDS read in the common case) rather than merging them into one generic (flat) load
  // that waits on both memory counters.
  __device__ inline int pop() {
    if (sp == 0) return EMPTY;
    --sp;
    if (sp < TRAV_LDS_STACK) return lds[sp * BS];
    return __builtin_nontemporal_load(glob + (int64_t)(sp - TRAV_LDS_STACK) * gstride);
  }
};

// Closest hit (ANY = false) or any hit (ANY = true) over t in (tmin, tmax), excluding the
// leaf position `excl`.  Closest-hit ties in t go to the smaller original triangle index.
// Boxes are culled against the current best distance widened by 2^-19 relative (about 16
// ulps, more than the rounding of a box entry plus that of a triangle's t): a triangle whose
// computed t ties the best (or lies within rounding of it, as on a shared edge or a box face
// whose slab entry equals the hit distance) is always tested, so the hit does not depend on
// the traversal order, and a refitted tree hits what a rebuilt one hits.
constexpr float T_WIDEN = 1.0f + 1.9073486328125e-6f;   // 1 + 2^-19
template <bool ANY, bool COUNT>
__device__ inline int traverse(const SceneDev& S, const Ray32& r, float tmin, float tmax, int excl, Stack& st,
                               float& t_hit, int64_t& cn, int64_t& ct) {
  int node = S.root;
  st.sp = 0;
  int best = -1, best_orig = INT32_MAX;
  float tb = tmax, tbw = tmax * T_WIDEN;
  while (true) {
    // inner nodes until this lane has none left or a quarter of the active lanes hold a
    // postponed leaf: the first leaf met is set aside and the walk goes on, so the wave tests
    // leaves together (measured against waiting for every lane: room 3.43 -> 3.02 ms, foliage
    // 38.4 -> 27.7 ms; half 3.21 / 31.2, an eighth 3.01 / 27.5 with slower small sets)
    int leaf = EMPTY;
    while (node >= 0) {
      const Node2 n = S.nodes[node];
      if (COUNT) ++cn;
      bool h0, h1;
      float t0, t1;
      box2(n, r, tmin, tbw, h0, h1, t0, t1);
      if (h0 && h1) {
        const bool first0 = t0 <= t1;
        st.push(first0 ? n.ch.y : n.ch.x);
        node = first0 ? n.ch.x : n.ch.y;
      } else if (h0) {
        node = n.ch.x;
      } else if (h1) {
        node = n.ch.y;
      } else {
        node = st.pop();
      }
      if (node < 0 && node != EMPTY && leaf == EMPTY) {
        leaf = node;
        node = st.pop();
      }
      if (__popcll(__ballot(leaf != EMPTY)) * 4 >= __popcll(__ballot(1))) break;
    }
    // the postponed leaf, then any leaf the walk stopped on
    while (leaf != EMPTY) {
      const int pos = ~leaf;
      if (COUNT) ++ct;
      if (pos != excl) {
        const float4 a = S.tri4[3 * (int64_t)pos], b = S.tri4[3 * (int64_t)pos + 1], c = S.tri4[3 * (int64_t)pos + 2];
        const float t = tri_test(a, b, c, r);
        if (t > tmin && t <= tb) {
          if (ANY) {
            if (t < tmax) { t_hit = t; return pos; }
          } else {
            const int orig = __float_as_int(a.w);
            if (t < tb || orig < best_orig) {
              tb = t;
              tbw = t * T_WIDEN;
              best = pos;
              best_orig = orig;
            }
          }
        }
      }
      if (node < 0 && node != EMPTY) {
        leaf = node;
        node = st.pop();
      } else {
        leaf = EMPTY;
      }
    }
    if (node == EMPTY) break;
  }
  t_hit = tb;
  return best;
}

struct PoseArgs {
  double s[3];
  double R[9];
  double xref[3];
  int64_t N;
  int32_t B;
  double maxd;
  double t_eps;
};

// One job of a fused batch: its scene, pose and ray directions.  Rays [ray0, ray0 + a.N) of
// the batch belong to it; in the ray state and the records the ray field holds the job.
struct TraceJob {
  SceneDev S;
  PoseArgs a;
  const float* dirs;
  int64_t ray0;
};

// Job tables reach the device through kernel arguments, a few jobs per launch, so that no
// host buffer has to outlive the call (and graph capture records the values).
constexpr int JOB_PACK = 8;
struct TraceJobPack {
  TraceJob j[JOB_PACK];
  int32_t first, n;
};
static_assert(sizeof(TraceJobPack) <= 4000, "job pack must fit the kernel argument space");

__global__ void k_put_trace_jobs(TraceJobPack pk, TraceJob* __restrict__ dst) {
  if ((int)threadIdx.x < pk.n) dst[pk.first + threadIdx.x] = pk.j[threadIdx.x];
}

__device__ inline double dnorm3(double x, double y, double z) { return sqrt(x * x + y * y + z * z); }

// carry: a later job wave of a batch; the totals of the statistics carry over
__global__ void k_trace_init(Ctl* ctl, int64_t N, int carry) {
  ctl->n_active[0] = N;
  ctl->n_active[1] = 0;
  if (carry) {
    ctl->rec_prev += ctl->rec_base;
  } else {
    ctl->rec_prev = 0;
    ctl->seg = 0;
    ctl->shadow = 0;
    ctl->overflow = 0;
    for (int i = 0; i < 6; ++i) ctl->cnt[i] = 0;
  }
  ctl->rec_base = 0;
  ctl->cmax_bits = 0;
  ctl->n_elig = 0;
  ctl->diff_kept = 0;
  ctl->n_groups = 0;
  ctl->n_draw = 0;
  for (int i = 0; i < 4; ++i) ctl->tot[i] = 0;
}

// The job of batch ray g (the last job with ray0 <= g; jobs without rays share ray0 with the next).
__device__ inline int ray_job(const TraceJob* __restrict__ jobs, int32_t J, int64_t g) {
  int lo = 0, hi = J - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].ray0 <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

constexpr int RAY_KEY_BITS = 16;   // direction cells of the ray sort: 2^16 on the octahedral map

__device__ inline uint32_t spread8(uint32_t v) {   // bit i -> bit 2i
  v = (v | (v << 4)) & 0x0F0Fu;
  v = (v | (v << 2)) & 0x3333u;
  v = (v | (v << 1)) & 0x5555u;
  return v;
}

// Sort key of ray g: Morton code of its world direction on the octahedral map (the top
// RAY_KEY_BITS of 8 + 8 bits), the job above it in a batch.  perm[g] = g (the sort's values).
template <bool BATCH>
__global__ void k_ray_keys(PoseArgs a0, const float* __restrict__ dirs0, const TraceJob* __restrict__ jobs, int32_t J,
                           uint32_t* __restrict__ keys, int32_t* __restrict__ perm) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a0.N) return;
  const float* dirs = dirs0;
  double R[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = a0.R[k];
  int64_t li = g;
  uint32_t hi = 0;
  if (BATCH) {
    const int j = ray_job(jobs, J, g);
    dirs = jobs[j].dirs;
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = jobs[j].a.R[k];
    li = g - jobs[j].ray0;
    hi = (uint32_t)j << RAY_KEY_BITS;
  }
  const float lx = dirs[3 * li], ly = dirs[3 * li + 1], lz = dirs[3 * li + 2];
  float x = (float)(R[0] * lx + R[1] * ly + R[2] * lz);
  float y = (float)(R[3] * lx + R[4] * ly + R[5] * lz);
  float z = (float)(R[6] * lx + R[7] * ly + R[8] * lz);
  const float s = fabsf(x) + fabsf(y) + fabsf(z);
  uint32_t ux = 0, uy = 0;
  if (s > 0.f && s < INFINITY) {
    x /= s; y /= s; z /= s;
    if (z < 0.f) {
      const float tx = (1.f - fabsf(y)) * (x >= 0.f ? 1.f : -1.f), ty = (1.f - fabsf(x)) * (y >= 0.f ? 1.f : -1.f);
      x = tx; y = ty;
    }
    ux = (uint32_t)fminf(fmaxf((x * 0.5f + 0.5f) * 256.f, 0.f), 255.f);
    uy = (uint32_t)fminf(fmaxf((y * 0.5f + 0.5f) * 256.f, 0.f), 255.f);
  }
  keys[g] = hi | ((spread8(ux) | (spread8(uy) << 1)) >> (16 - RAY_KEY_BITS));
  perm[g] = (int32_t)g;
}

// BATCH: a0.N is the batch's total ray count and each ray finds its job in the table.
// Slot i starts ray perm[i] (rays in key order).
template <bool BATCH>
__global__ void k_ray_init(PoseArgs a0, const float* __restrict__ dirs0, const TraceJob* __restrict__ jobs, int32_t J,
                           const int32_t* __restrict__ perm, TraceWS w, Ctl* ctl) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a0.N) return;
  const int64_t g = perm ? perm[i] : i;
  PoseArgs a = a0;
  const float* dirs = dirs0;
  int64_t li = g;
  int32_t tag = (int32_t)g;
  if (BATCH) {
    const int j = ray_job(jobs, J, g);
    a = jobs[j].a;
    dirs = jobs[j].dirs;
    li = g - jobs[j].ray0;
    tag = j;
  }
  const double lx = dirs[3 * li], ly = dirs[3 * li + 1], lz = dirs[3 * li + 2];
  // CalculateWorldDirection: world = R * local, normalised in FP64
  double dx = a.R[0] * lx + a.R[1] * ly + a.R[2] * lz;
  double dy = a.R[3] * lx + a.R[4] * ly + a.R[5] * lz;
  double dz = a.R[6] * lx + a.R[7] * ly + a.R[8] * lz;
  double nrm = dnorm3(dx, dy, dz);
  if (!(nrm > 0.0) || !isfinite(nrm)) {
    atomicOr(&ctl->err, DEV_ERR_RAYDIR);
    nrm = 1.0;
    dx = 1.0; dy = 0.0; dz = 0.0;
  }
  w.st[0][0][i] = a.s[0]; w.st[0][1][i] = a.s[1]; w.st[0][2][i] = a.s[2];
  w.st[0][3][i] = dx / nrm; w.st[0][4][i] = dy / nrm; w.st[0][5][i] = dz / nrm;
  w.st[0][6][i] = 0.0;
  w.prev[0][i] = -1;
  w.ray[0][i] = tag;
  w.prec[0][i] = -1;
}

// BATCH: each ray reads its scene and pose from the job table (the ray field is the job).
// PERRX: one line-of-sight ray from the hit to each of the M receivers at rxp (bit m of the
// result) instead of one toward the pose's reference point.
// Six waves per SIMD (the register budget that asks for, 80, holds the kernel without spills):
// measured 7% faster on the room's trace and 15% on foliage's than five.
template <bool COUNT, bool BATCH, bool PERRX>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(TRAV_WAVES_PER_SIMD))) void k_bounce(
    SceneDev S0, PoseArgs a0, const TraceJob* __restrict__ jobs, TraceWS w, Ctl* ctl, int j,
    const double* __restrict__ rxp, int32_t M) {
  __shared__ int lds_stack[TRAV_LDS_STACK * BS];
  const int cur = j & 1;
  const int64_t n = ctl->n_active[cur];
  const int64_t gtid = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * BS;
  Stack st;
  st.lds = lds_stack + threadIdx.x;
  st.glob = w.gstack + gtid;
  st.gstride = w.gstack_threads;
  st.cap = w.stack_cap;
  st.overflow = 0;
  int64_t cn_c = 0, ct_c = 0, cn_a = 0, ct_a = 0, rays_a = 0;
  for (int64_t i = gtid; i < n; i += stride) {
    int pos;
    float th = INFINITY;
    {
      SceneDev S = S0;
      float teps = (float)a0.t_eps;
      if (BATCH) {
        const TraceJob* tj = jobs + w.ray[cur][i];
        S = tj->S;
        teps = (float)tj->a.t_eps;
      }
      const Ray32 r = make_ray(w.st[cur][0][i], w.st[cur][1][i], w.st[cur][2][i], w.st[cur][3][i], w.st[cur][4][i],
                               w.st[cur][5][i]);
      pos = (!BATCH || S.T > 0) ? traverse<false, COUNT>(S, r, teps, INFINITY, w.prev[cur][i], st, th, cn_c, ct_c) : -1;
    }
    // The FP64 ray state (and a batch ray's job) is read again after the traversal instead of
    // being held in registers through it; the compiler barrier keeps the two reads apart, so
    // the traversal loop runs with fewer live registers (more waves per SIMD).
    __asm__ volatile("" ::: "memory");
    SceneDev S = S0;
    PoseArgs a = a0;
    if (BATCH) {
      const TraceJob* tj = jobs + w.ray[cur][i];
      S = tj->S;
      a = tj->a;
    }
    const float teps = (float)a.t_eps;
    const double ox = w.st[cur][0][i], oy = w.st[cur][1][i], oz = w.st[cur][2][i];
    const double dx = w.st[cur][3][i], dy = w.st[cur][4][i], dz = w.st[cur][5][i];
    const double rtot = w.st[cur][6][i];
    uint64_t flag = 0;
    if (pos >= 0) {
      // FP64 refinement on the chosen triangle: plane intersection, normal, reflection
      const float4 A = S.tri4[3 * (int64_t)pos], Bv = S.tri4[3 * (int64_t)pos + 1], Cv = S.tri4[3 * (int64_t)pos + 2];
      const double e1x = (double)Bv.x - A.x, e1y = (double)Bv.y - A.y, e1z = (double)Bv.z - A.z;
      const double e2x = (double)Cv.x - A.x, e2y = (double)Cv.y - A.y, e2z = (double)Cv.z - A.z;
      double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
      const double nn = dnorm3(nx, ny, nz);
      nx /= nn; ny /= nn; nz /= nn;
      const double dn = dx * nx + dy * ny + dz * nz;
      const double hp = ((double)A.x - ox) * nx + ((double)A.y - oy) * ny + ((double)A.z - oz) * nz;
      const double t = dn != 0.0 ? hp / dn : (double)th;
      const double px = ox + t * dx, py = oy + t * dy, pz = oz + t * dz;
      const double rnew = (j == 0) ? dnorm3(px - a.s[0], py - a.s[1], pz - a.s[2]) : rtot + t;
      const double rx = dx - 2.0 * dn * nx, ry = dy - 2.0 * dn * ny, rz = dz - 2.0 * dn * nz;
      // the bounce's results leave registers before the line-of-sight traversal
      w.rp[0][i] = px; w.rp[1][i] = py; w.rp[2][i] = pz;
      w.rd[0][i] = rx; w.rd[1][i] = ry; w.rd[2][i] = rz;
      w.rr[i] = rnew;
      w.rpos[i] = pos;
      const bool cont = (j + 1 < a.B) && !(rnew >= a.maxd);
      flag = 1ull | ((uint64_t)cont << 32);
      uint64_t vis = 0;
      const int n_los = PERRX ? M : 1;
      for (int m = 0; m < n_los; ++m) {
        // line of sight from the hit point toward the receiver reference point (or receiver m)
        const double tx = PERRX ? rxp[3 * m] : a.xref[0], ty = PERRX ? rxp[3 * m + 1] : a.xref[1],
                     tz = PERRX ? rxp[3 * m + 2] : a.xref[2];
        const double wx = tx - px, wy = ty - py, wz = tz - pz;
        const double L = dnorm3(wx, wy, wz);
        bool v = true;
        if (L > 2.0 * a.t_eps) {
          const Ray32 rv = make_ray(px, py, pz, wx / L, wy / L, wz / L);
          float tv;
          const int blk = traverse<true, COUNT>(S, rv, teps, (float)(L - a.t_eps), pos, st, tv, cn_a, ct_a);
          v = blk < 0;
          ++rays_a;
        }
        if (v) vis |= 1ull << m;
      }
      w.rvis[i] = vis;
    }
    w.flags[i] = flag;
  }
  if (st.overflow) atomicAdd((unsigned long long*)&ctl->overflow, (unsigned long long)st.overflow);
  if (st.overflow) atomicOr(&ctl->err, DEV_ERR_STACK);
  if (COUNT) {
    atomicAdd((unsigned long long*)&ctl->cnt[0], (unsigned long long)cn_c);
    atomicAdd((unsigned long long*)&ctl->cnt[1], (unsigned long long)ct_c);
    atomicAdd((unsigned long long*)&ctl->cnt[2], (unsigned long long)cn_a);
    atomicAdd((unsigned long long*)&ctl->cnt[3], (unsigned long long)ct_a);
    atomicAdd((unsigned long long*)&ctl->cnt[5], (unsigned long long)rays_a);
  }
}

template <bool BATCH>
__global__ void k_scatter(SceneDev S, const TraceJob* __restrict__ jobs, TraceWS w, Ctl* ctl, et_paths P, int j,
                          int perrx) {
  const int cur = j & 1, nxt = cur ^ 1;
  const int64_t n = ctl->n_active[cur];
  const int64_t base = ctl->rec_base;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t f = w.flags[i];
    if (!(f & 1ull)) continue;
    const uint64_t o = w.offs[i];
    const int64_t ri = base + (int64_t)(o & 0xffffffffull);
    const int pos = w.rpos[i];
    const int32_t* tri_orig = S.tri_orig;
    const int32_t* matp = S.mat;
    if (BATCH) {
      const TraceJob* tj = jobs + w.ray[cur][i];
      tri_orig = tj->S.tri_orig;
      matp = tj->S.mat;
    }
    const int orig = tri_orig[pos];
    if (ri < P.capacity) {
      P.p[3 * ri] = w.rp[0][i]; P.p[3 * ri + 1] = w.rp[1][i]; P.p[3 * ri + 2] = w.rp[2][i];
      P.dout[3 * ri] = (float)w.rd[0][i]; P.dout[3 * ri + 1] = (float)w.rd[1][i]; P.dout[3 * ri + 2] = (float)w.rd[2][i];
      P.rtot[ri] = w.rr[i];
      P.tri[ri] = orig;
      P.mat[ri] = matp[orig];
      P.ray[ri] = w.ray[cur][i];
      P.bounce[ri] = (uint8_t)j;
      P.flags[ri] = w.rvis[i] != 0 ? 1 : 0;
      if (P.prev) P.prev[ri] = w.prec[cur][i];
      if (perrx) P.rx_vis[ri] = w.rvis[i];
    } else {
      atomicOr(&ctl->err, DEV_ERR_CAPACITY);
    }
    if (f >> 32) {
      const int64_t k = (int64_t)(o >> 32);
      w.st[nxt][0][k] = w.rp[0][i]; w.st[nxt][1][k] = w.rp[1][i]; w.st[nxt][2][k] = w.rp[2][i];
      w.st[nxt][3][k] = w.rd[0][i]; w.st[nxt][4][k] = w.rd[1][i]; w.st[nxt][5][k] = w.rd[2][i];
      w.st[nxt][6][k] = w.rr[i];
      w.prev[nxt][k] = pos;
      w.ray[nxt][k] = w.ray[cur][i];
      w.prec[nxt][k] = ri;
    }
  }
}

__global__ void k_bounce_epi(Ctl* ctl, int j) {
  const int cur = j & 1;
  const uint64_t t = ctl->tot[0];
  const int64_t hits = (int64_t)(t & 0xffffffffull);
  ctl->seg += ctl->n_active[cur];
  ctl->shadow += hits;
  ctl->rec_base += hits;
  ctl->n_active[cur ^ 1] = (int64_t)(t >> 32);
  ctl->cnt[4] += ctl->n_active[cur];
}

// ------------------------------------------------------------------ diffraction (Sec. III-D)
// Decisions that pick integers (eligibility, weights, CDF search, sample points, incidence
// test) are FP64 without contraction, in a fixed operation order.
#pragma clang fp contract(off)

__device__ inline uint64_t splitmix(uint64_t key, uint64_t counter) {
  uint64_t z = key + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1p-53; }

struct DiffArgs {
  double s[3];
  double axis[3];
  double cone;
  double tau;
  double cos_max;
  uint64_t seed;
  int64_t K;            // draws (per mesh with per_mesh)
  double t_eps;
  int per_mesh;
  int64_t max_meshes;
  uint64_t rx_all;      // per-receiver reading: every receiver's bit (no receiver-side test), else 0
};

__global__ void k_obj_fov(SceneDev S, DiffArgs a, uint8_t* oel) {
  int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= S.n_obj) return;
  const float* b = S.obj_box + 6 * o;
  const double lx = b[0], ly = b[1], lz = b[2], hx = b[3], hy = b[4], hz = b[5];
  if (!(lx <= hx)) { oel[o] = 0; return; }
  const double cx = 0.5 * (lx + hx), cy = 0.5 * (ly + hy), cz = 0.5 * (lz + hz);
  const double ex = hx - lx, ey = hy - ly, ez = hz - lz;
  const double rad = 0.5 * sqrt(ex * ex + ey * ey + ez * ez);
  const double wx = cx - a.s[0], wy = cy - a.s[1], wz = cz - a.s[2];
  const double dist = sqrt(wx * wx + wy * wy + wz * wz);
  if (dist <= rad) { oel[o] = 1; return; }
  const double qx = wy * a.axis[2] - wz * a.axis[1], qy = wz * a.axis[0] - wx * a.axis[2],
               qz = wx * a.axis[1] - wy * a.axis[0];
  const double psi = atan2(sqrt(qx * qx + qy * qy + qz * qz), wx * a.axis[0] + wy * a.axis[1] + wz * a.axis[2]);
  oel[o] = psi <= a.cone + asin(rad / dist);
}

// Largest C_i over the field-of-view objects: positive doubles order as their bit patterns, so
// a wave takes the maximum of the bits by shuffles and issues one atomic.
// Largest C_i over the triangles of eligible objects, as the bit pattern of a non-negative double
// (ordered like the value): a grid-strided maximum per thread, then per wave and per block, and
// one atomic per block (one per wave left the room's 193,212 triangles waiting on about 3000 atomics).
__global__ __launch_bounds__(BS) void k_cmax(SceneDev S, const uint8_t* __restrict__ oel, Ctl* ctl) {
  __shared__ long long wmax[BS / 64];
  long long v = 0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < S.T; t += (int64_t)gridDim.x * blockDim.x) {
    if (oel[S.obj[t]]) {
      const double c = S.C[t];
      if (c > 0.0) {
        const long long b = __double_as_longlong(c);
        v = b > v ? b : v;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const long long o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < BS / 64; ++i) v = wmax[i] > v ? wmax[i] : v;
    if (v > 0) atomicMax((unsigned long long*)&ctl->cmax_bits, (unsigned long long)v);
  }
}

__global__ void k_qweight(SceneDev S, DiffArgs a, const uint8_t* __restrict__ oel, const Ctl* ctl,
                          uint64_t* __restrict__ q, uint64_t* __restrict__ flag) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.T) return;
  const double cmax = __longlong_as_double((long long)ctl->cmax_bits);
  const double c = S.C[t];
  uint64_t qq = 0;
  if (cmax > 0.0 && oel[S.obj[t]] && c > 0.0 && c >= a.tau * cmax) {
    // dithered integer weight: stochastic rounding of (C / Cmax) * 2^32
    const double x = c / cmax * 4294967296.0 + u01(splitmix(a.seed ^ 1ull, (uint64_t)t));
    qq = (uint64_t)floor(x);
  }
  q[t] = qq;
  flag[t] = qq > 0 ? 1ull : 0ull;
}

// Sort keys of the eligible triangles, listed in increasing index: weight descending (one
// CDF), or the mesh first and then weight descending (per mesh).  The radix sort is stable,
// so equal weights keep increasing indices without the index in the key (32 key bits, four
// passes, for one CDF).
__global__ void k_elig_keys(SceneDev S, int per_mesh, const uint64_t* __restrict__ q, const uint64_t* __restrict__ flag,
                            const uint64_t* __restrict__ offs, uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S.T || !flag[t]) return;
  const int64_t p = (int64_t)offs[t];
  keys[p] = per_mesh ? ((uint64_t)S.obj[t] << 32) | (4294967296ull - q[t]) : (4294967296ull - q[t]);
  vals[p] = (int32_t)t;
}

__global__ void k_elig_count(Ctl* ctl) { ctl->n_elig = (int64_t)ctl->tot[1]; }

__global__ void k_sorted_q(const uint64_t* __restrict__ keys, const Ctl* ctl, uint64_t* __restrict__ qs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ctl->n_elig) return;
  qs[i] = 4294967296ull - (keys[i] & 0xffffffffull);
}

// Group starts in the sorted list: a group per mesh (per_mesh), else one group.
__global__ void k_group_flags(const uint64_t* __restrict__ keys, int per_mesh, const Ctl* ctl,
                              uint64_t* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ctl->n_elig) return;
  flag[i] = (i == 0 || (per_mesh && (keys[i] >> 32) != (keys[i - 1] >> 32))) ? 1ull : 0ull;
}

__global__ void k_group_starts(const uint64_t* __restrict__ flag, const uint64_t* __restrict__ rank, const Ctl* ctl,
                               int64_t* __restrict__ gstart) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ctl->n_elig && flag[i]) gstart[rank[i]] = i;
}

// Group count and draws; more meshes than max_meshes keeps the first ones and reports a
// capacity error.  The last kept group ends where the first dropped one starts (its entry of
// gstart is already that start), so only an untruncated list gets the end marker n_elig.
__global__ void k_group_count(Ctl* ctl, DiffArgs a, int64_t* __restrict__ gstart) {
  int64_t g = (int64_t)ctl->tot[2];
  if (a.per_mesh && g > a.max_meshes) {
    atomicOr(&ctl->err, DEV_ERR_CAPACITY);
    g = a.max_meshes;
  } else {
    gstart[g] = ctl->n_elig;
  }
  ctl->n_groups = g;
  ctl->n_draw = a.per_mesh ? a.K * g : (ctl->n_elig > 0 ? a.K : 0);
}

__global__ __launch_bounds__(BS) void k_diff_sample(SceneDev S, DiffArgs a, const uint64_t* __restrict__ W_ex,
                                                    const uint64_t* __restrict__ qs, const int32_t* __restrict__ vals,
                                                    TraceWS w, Ctl* ctl) {
  __shared__ int lds_stack[TRAV_LDS_STACK * BS];
  const int64_t gtid = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * BS;
  Stack st;
  st.lds = lds_stack + threadIdx.x;
  st.glob = w.gstack + gtid;
  st.gstride = w.gstack_threads;
  st.cap = w.stack_cap;
  st.overflow = 0;
  const int64_t n_draw = ctl->n_draw;
  int64_t dummy0 = 0, dummy1 = 0, rays = 0;
  for (int64_t k = gtid; k < n_draw; k += stride) {
    uint64_t keep = 0;
    w.stri[k] = -1;
    {
      // this draw's group (its mesh, or the one CDF) and the group's running sums
      const int64_t g = a.per_mesh ? k / a.K : 0;
      const int64_t j0 = w.gstart[g], j1 = w.gstart[g + 1];
      const uint64_t base = W_ex[j0], total = W_ex[j1 - 1] + qs[j1 - 1] - base;
      const uint64_t ks = a.seed ^ 2ull;
      const uint64_t U = splitmix(ks, 3ull * (uint64_t)k);
      const uint64_t idx = __umul64hi(U, total);
      // first position of the group whose inclusive running sum exceeds idx
      int64_t lo = j0, hi = j1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (W_ex[mid] + qs[mid] - base > idx) hi = mid; else lo = mid + 1;
      }
      const int32_t t = vals[lo];
      const double u1 = u01(splitmix(ks, 3ull * (uint64_t)k + 1ull)), u2 = u01(splitmix(ks, 3ull * (uint64_t)k + 2ull));
      const double su = sqrt(u1);
      const double wa = 1.0 - su, wb = su * (1.0 - u2), wc = su * u2;   // uniform point on the triangle
      const int pos = S.tri_pos[t];
      const float4 A = S.tri4[3 * (int64_t)pos], B = S.tri4[3 * (int64_t)pos + 1], C = S.tri4[3 * (int64_t)pos + 2];
      const double ax = A.x, ay = A.y, az = A.z, bx = B.x, by = B.y, bz = B.z, cx = C.x, cy = C.y, cz = C.z;
      const double ox = wa * ax + wb * bx + wc * cx, oy = wa * ay + wb * by + wc * cy, oz = wa * az + wb * bz + wc * cz;
      double nx = (by - ay) * (cz - az) - (bz - az) * (cy - ay);
      double ny = (bz - az) * (cx - ax) - (bx - ax) * (cz - az);
      double nz = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
      const double nn = sqrt(nx * nx + ny * ny + nz * nz);
      const double inn = 1.0 / nn;
      nx = nx * inn; ny = ny * inn; nz = nz * inn;
      const double wx = a.s[0] - ox, wy = a.s[1] - oy, wz = a.s[2] - oz;
      const double L = sqrt(wx * wx + wy * wy + wz * wz);
      const double iL = 1.0 / L;
      const double vx = wx * iL, vy = wy * iL, vz = wz * iL;
      const double ci = fabs(nx * vx + ny * vy + nz * vz);
      bool ok = ci >= a.cos_max;                                   // incidence-angle constraint
      if (ok) {                                                    // line of sight to the source
        const Ray32 r = make_ray(ox, oy, oz, vx, vy, vz);
        float tv;
        const int blk = traverse<true, false>(S, r, (float)a.t_eps, (float)(L - a.t_eps), pos, st, tv, dummy0, dummy1);
        ok = blk < 0;
        ++rays;
      }
      w.stri[k] = t;
      w.so[3 * k] = ox; w.so[3 * k + 1] = oy; w.so[3 * k + 2] = oz;
      w.sr[k] = L;
      keep = ok ? 1ull : 0ull;
    }
    w.skeep[k] = keep;
  }
  if (st.overflow) {
    atomicAdd((unsigned long long*)&ctl->overflow, (unsigned long long)st.overflow);
    atomicOr(&ctl->err, DEV_ERR_STACK);
  }
  atomicAdd((unsigned long long*)&ctl->shadow, (unsigned long long)rays);
}

__global__ void k_diff_scatter(SceneDev S, DiffArgs a, TraceWS w, Ctl* ctl, et_paths P) {
  const int64_t base = ctl->rec_base;
  const int64_t n_draw = ctl->n_draw;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_draw; k += (int64_t)gridDim.x * blockDim.x) {
    if (!w.skeep[k]) continue;
    const int64_t ri = base + (int64_t)w.soffs[k];
    if (ri >= P.capacity) { atomicOr(&ctl->err, DEV_ERR_CAPACITY); continue; }
    const int32_t t = w.stri[k];
    P.p[3 * ri] = w.so[3 * k]; P.p[3 * ri + 1] = w.so[3 * k + 1]; P.p[3 * ri + 2] = w.so[3 * k + 2];
    P.dout[3 * ri] = 0.f; P.dout[3 * ri + 1] = 0.f; P.dout[3 * ri + 2] = 0.f;
    P.rtot[ri] = w.sr[k];
    P.tri[ri] = t;
    P.mat[ri] = S.mat[t];
    P.ray[ri] = (int32_t)k;
    P.bounce[ri] = 0;
    P.flags[ri] = 3;   // visible | diffraction
    if (P.prev) P.prev[ri] = -1;
    if (a.rx_all) P.rx_vis[ri] = a.rx_all;
  }
}

#pragma clang fp contract(on)

// Passive component: one line-of-sight ray from the emitter to each receiver (no triangle
// excluded) and one record per receiver after the specular and diffraction records: the
// emitter as the point, path 0, the receiver in `mat` and `ray`, kind 2 in the flags.
__global__ __launch_bounds__(BS) void k_passive(SceneDev S, PoseArgs a, const double* __restrict__ rx, int32_t M,
                                                int diff, TraceWS w, Ctl* ctl, et_paths P, int perrx) {
  __shared__ int lds_stack[TRAV_LDS_STACK * BS];
  const int64_t gtid = (int64_t)blockIdx.x * BS + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * BS;
  Stack st;
  st.lds = lds_stack + threadIdx.x;
  st.glob = w.gstack + gtid;
  st.gstride = w.gstack_threads;
  st.cap = w.stack_cap;
  st.overflow = 0;
  const int64_t base = ctl->rec_base + (diff ? (int64_t)ctl->tot[3] : 0);
  int64_t dummy0 = 0, dummy1 = 0, rays = 0;
  for (int64_t m = gtid; m < M; m += stride) {
    const double wx = rx[3 * m] - a.s[0], wy = rx[3 * m + 1] - a.s[1], wz = rx[3 * m + 2] - a.s[2];
    const double L = dnorm3(wx, wy, wz);
    int vis = 1;
    if (L > 2.0 * a.t_eps && S.T > 0) {
      const Ray32 r = make_ray(a.s[0], a.s[1], a.s[2], wx / L, wy / L, wz / L);
      float tv;
      vis = traverse<true, false>(S, r, (float)a.t_eps, (float)(L - a.t_eps), -1, st, tv, dummy0, dummy1) < 0;
      ++rays;
    }
    const int64_t ri = base + m;
    if (ri < P.capacity) {
      P.p[3 * ri] = a.s[0]; P.p[3 * ri + 1] = a.s[1]; P.p[3 * ri + 2] = a.s[2];
      P.dout[3 * ri] = 0.f; P.dout[3 * ri + 1] = 0.f; P.dout[3 * ri + 2] = 0.f;
      P.rtot[ri] = 0.0;
      P.tri[ri] = -1;
      P.mat[ri] = (int32_t)m;
      P.ray[ri] = (int32_t)m;
      P.bounce[ri] = 0;
      P.flags[ri] = (uint8_t)(vis | 4);   // visible | kind 2
      if (P.prev) P.prev[ri] = -1;
      if (perrx) P.rx_vis[ri] = vis && m < 64 ? 1ull << m : 0ull;
    } else {
      atomicOr(&ctl->err, DEV_ERR_CAPACITY);
    }
  }
  if (st.overflow) {
    atomicAdd((unsigned long long*)&ctl->overflow, (unsigned long long)st.overflow);
    atomicOr(&ctl->err, DEV_ERR_STACK);
  }
  if (rays) atomicAdd((unsigned long long*)&ctl->shadow, (unsigned long long)rays);
}

__global__ void k_trace_final(Ctl* ctl, et_paths P, int diff, int32_t n_passive) {
  const int64_t spec = ctl->rec_base;
  const int64_t dk = diff ? (int64_t)ctl->tot[3] : 0;
  ctl->diff_kept = dk;
  const int64_t total = spec + dk + n_passive;
  ctl->n_rec = total;
  P.count[0] = total;
  P.count[1] = spec;
  P.count[2] = dk;
  P.count[3] = ctl->seg;
}

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t trace_ws_layout(int64_t N, int64_t T, int32_t n_obj, int64_t K, char* base, TraceWS* w, int32_t max_blocks) {
  const int64_t Nm = std::max<int64_t>(N, 1), Tm = std::max<int64_t>(T, 1), Km = std::max<int64_t>(K, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)(base + off) : nullptr;
    off += al(bytes);
    return p;
  };
  TraceWS x{};
  for (int b = 0; b < 2; ++b) {
    for (int k = 0; k < 7; ++k) x.st[b][k] = (double*)take(sizeof(double) * Nm);
    x.prev[b] = (int32_t*)take(sizeof(int32_t) * Nm);
    x.ray[b] = (int32_t*)take(sizeof(int32_t) * Nm);
    x.prec[b] = (int64_t*)take(sizeof(int64_t) * Nm);
  }
  for (int k = 0; k < 3; ++k) x.rp[k] = (double*)take(sizeof(double) * Nm);
  for (int k = 0; k < 3; ++k) x.rd[k] = (double*)take(sizeof(double) * Nm);
  x.rr = (double*)take(sizeof(double) * Nm);
  x.rpos = (int32_t*)take(sizeof(int32_t) * Nm);
  x.rvis = (uint64_t*)take(sizeof(uint64_t) * Nm);
  x.flags = (uint64_t*)take(sizeof(uint64_t) * Nm);
  x.offs = (uint64_t*)take(sizeof(uint64_t) * Nm);
  x.scan_tmp = take(scan_temp_bytes(std::max(std::max(Nm, Tm), Km)));
  x.rkeys = (uint32_t*)take(sizeof(uint32_t) * Nm);
  x.rperm = (int32_t*)take(sizeof(int32_t) * Nm);
  x.rsort_tmp = take(sort_temp_bytes(Nm, 4));
  // global stack columns: one per thread of the largest traversing grid (bounces over N rays,
  // diffraction over K draws, the passive rays); a fused batch passes its largest tuned grid
  const int64_t stack_blocks = max_blocks > 0 ? max_blocks
                                              : std::max<int64_t>(nblk(std::max<int64_t>(N, 1)), nblk(std::max<int64_t>(K, 1)));
  x.gstack_threads = stack_blocks * BS;
  x.gstack = (int32_t*)take(sizeof(int32_t) * (size_t)(TRAV_STACK - TRAV_LDS_STACK) * (size_t)x.gstack_threads);
  x.stack_cap = TRAV_STACK;
  if (K > 0) {
    x.oel = (uint8_t*)take((size_t)std::max<int32_t>(n_obj, 1));
    x.dkeys = (uint64_t*)take(sizeof(uint64_t) * Tm);
    x.dvals = (int32_t*)take(sizeof(int32_t) * Tm);
    x.dq = (uint64_t*)take(sizeof(uint64_t) * Tm);
    x.dflags = (uint64_t*)take(sizeof(uint64_t) * Tm);
    x.doffs = (uint64_t*)take(sizeof(uint64_t) * Tm);
    x.sort_tmp = take(sort_temp_bytes(Tm, 8));
    x.stri = (int32_t*)take(sizeof(int32_t) * Km);
    x.so = (double*)take(sizeof(double) * 3 * Km);
    x.sr = (double*)take(sizeof(double) * Km);
    x.skeep = (uint64_t*)take(sizeof(uint64_t) * Km);
    x.soffs = (uint64_t*)take(sizeof(uint64_t) * Km);
    x.goffs = (uint64_t*)take(sizeof(uint64_t) * Tm);
    x.gstart = (int64_t*)take(sizeof(int64_t) * (Tm + 1));
  }
  if (w) *w = x;
  return off;
}

namespace {
// Threads of the bounce kernel that the current device holds at once (blocks per compute unit
// at its occupancy, times the compute units), queried once per device.
int64_t bounce_resident_threads() {
  static std::atomic<int64_t> cache[64];
  int dev = 0;
  ET_HIP(hipGetDevice(&dev));
  std::atomic<int64_t>* slot = (dev >= 0 && dev < 64) ? &cache[dev] : nullptr;
  if (slot) {
    const int64_t v = slot->load(std::memory_order_relaxed);
    if (v > 0) return v;
  }
  int per_cu = 0, cus = 0;
  ET_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bounce<false, false, false>, BS, 0));
  ET_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t v = std::max<int64_t>(1, (int64_t)per_cu * cus) * BS;
  if (slot) slot->store(v, std::memory_order_relaxed);
  return v;
}

PoseArgs pose_args(const et_sim_desc* sim) {
  PoseArgs a;
  for (int k = 0; k < 3; ++k) { a.s[k] = sim->emitter_pos[k]; a.xref[k] = sim->x_ref[k]; }
  for (int k = 0; k < 9; ++k) a.R[k] = sim->emitter_rot[k];
  a.N = (sim->flags & ET_SPECULAR) ? sim->N : 0;
  a.B = sim->max_bounces;
  a.maxd = sim->max_distance;
  a.t_eps = sim->t_eps;
  return a;
}
}  // namespace

size_t trace_batch_jobs_bytes(int32_t J) { return sizeof(TraceJob) * (size_t)std::max(J, 1); }

int64_t trace_batch_rays(int32_t J, const et_job* jobs) {
  int64_t n = 0;
  for (int32_t i = 0; i < J; ++i) n += (jobs[i].sim->flags & ET_SPECULAR) ? jobs[i].sim->N : 0;
  return n;
}

void trace_batch_run(int32_t J, const et_job* jobs, void* dev_jobs, const et_paths* paths, const TraceWS& w,
                     Ctl* ctl, bool counting, int32_t blocks, hipStream_t s, bool carry) {
  TraceJob* dj = (TraceJob*)dev_jobs;
  TraceJobPack pk{};
  int64_t N = 0;
  int B = 0;
  for (int32_t i = 0; i < J; ++i) {
    TraceJob& t = pk.j[pk.n++];
    t.S = jobs[i].scene->d;
    t.a = pose_args(jobs[i].sim);
    t.dirs = jobs[i].sim->ray_dirs;
    t.ray0 = N;
    N += t.a.N;
    B = std::max(B, (int)t.a.B);
    if (pk.n == JOB_PACK || i + 1 == J) {
      k_put_trace_jobs<<<1, JOB_PACK, 0, s>>>(pk, dj);
      pk.first += pk.n;
      pk.n = 0;
    }
  }
  PoseArgs all{};
  all.N = N;
  const et_paths P = *paths;
  k_trace_init<<<1, 1, 0, s>>>(ctl, N, carry ? 1 : 0);
  ET_HIP(hipGetLastError());
  // bounce grid: the tuned block count, within what the workspace's global stacks serve
  const int64_t cap_blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, w.gstack_threads / BS));
  const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + BS - 1) / BS, cap_blocks));
  if (N > 0) {
    const bool sorted = N > (int64_t)gb * BS;
    if (sorted) {
      int jb = 0;
      while ((1ll << jb) < (int64_t)J) ++jb;
      k_ray_keys<true><<<nblk_full(N), BS, 0, s>>>(all, nullptr, dj, J, w.rkeys, w.rperm);
      radix_sort_u32(w.rkeys, w.rperm, N, RAY_KEY_BITS + jb, w.rsort_tmp, s);
    }
    k_ray_init<true><<<nblk_full(N), BS, 0, s>>>(all, nullptr, dj, J, sorted ? w.rperm : nullptr, w, ctl);
    for (int j = 0; j < B; ++j) {
      if (counting) k_bounce<true, true, false><<<gb, BS, 0, s>>>(SceneDev{}, all, dj, w, ctl, j, nullptr, 0);
      else k_bounce<false, true, false><<<gb, BS, 0, s>>>(SceneDev{}, all, dj, w, ctl, j, nullptr, 0);
      scan_exclusive_u64(w.flags, w.offs, 0, &ctl->n_active[j & 1], N, &ctl->tot[0], w.scan_tmp, s);
      k_scatter<true><<<nblk(N), BS, 0, s>>>(SceneDev{}, dj, w, ctl, P, j, 0);
      k_bounce_epi<<<1, 1, 0, s>>>(ctl, j);
      ET_HIP(hipGetLastError());
    }
  }
  k_trace_final<<<1, 1, 0, s>>>(ctl, P, 0, 0);
  ET_HIP(hipGetLastError());
}

void trace_run(const SceneDev& S, const et_sim_desc* sim, const et_paths* paths, const TraceWS& w, Ctl* ctl,
               bool counting, hipStream_t s) {
  const PoseArgs a = pose_args(sim);
  const et_paths P = *paths;
  const bool perrx = (sim->flags & ET_PER_RX_VISIBILITY) != 0;
  k_trace_init<<<1, 1, 0, s>>>(ctl, a.N, 0);
  ET_HIP(hipGetLastError());
  // every traversing grid below stays within the workspace's global stack columns
  auto stack_fits = [&](int64_t n) {
    ET_CHECK((int64_t)nblk(n) * BS <= w.gstack_threads, ET_E_INTERNAL, "trace grid exceeds the workspace's stacks");
  };
  if (a.N > 0 && S.T > 0) {
    stack_fits(a.N);
    const bool sorted = a.N > bounce_resident_threads() || a.N > (int64_t)nblk(a.N) * BS;
    if (sorted) {
      k_ray_keys<false><<<nblk_full(a.N), BS, 0, s>>>(a, sim->ray_dirs, nullptr, 0, w.rkeys, w.rperm);
      radix_sort_u32(w.rkeys, w.rperm, a.N, RAY_KEY_BITS, w.rsort_tmp, s);
    }
    k_ray_init<false><<<nblk_full(a.N), BS, 0, s>>>(a, sim->ray_dirs, nullptr, 0, sorted ? w.rperm : nullptr, w, ctl);
    // bounce grid: whole rounds of resident blocks (no partly filled last round), the rays taken
    // by grid stride (the room's 2^20 rays: 4096 blocks, 2.67 rounds, 2.82 ms per trace; 3072, two
    // rounds, 2.73 ms; 2560 2.79, 2048 3.13, 1536 3.06 ms; foliage's 2^22 rays: 8192 blocks 27.7 ms,
    // 3072 28.7 ms)
    const int64_t res_blocks = std::max<int64_t>(1, bounce_resident_threads() / BS);
    const int64_t nb = nblk(a.N);
    const unsigned gb = (unsigned)(nb > res_blocks ? nb / res_blocks * res_blocks : nb);
    for (int j = 0; j < a.B; ++j) {
      const double* rx = sim->rx_pos;
      const int32_t M = sim->M;
      if (perrx) {
        if (counting) k_bounce<true, false, true><<<gb, BS, 0, s>>>(S, a, nullptr, w, ctl, j, rx, M);
        else k_bounce<false, false, true><<<gb, BS, 0, s>>>(S, a, nullptr, w, ctl, j, rx, M);
      } else {
        if (counting) k_bounce<true, false, false><<<gb, BS, 0, s>>>(S, a, nullptr, w, ctl, j, nullptr, 0);
        else k_bounce<false, false, false><<<gb, BS, 0, s>>>(S, a, nullptr, w, ctl, j, nullptr, 0);
      }
      scan_exclusive_u64(w.flags, w.offs, 0, &ctl->n_active[j & 1], a.N, &ctl->tot[0], w.scan_tmp, s);
      k_scatter<false><<<nblk(a.N), BS, 0, s>>>(S, nullptr, w, ctl, P, j, perrx ? 1 : 0);
      k_bounce_epi<<<1, 1, 0, s>>>(ctl, j);
      ET_HIP(hipGetLastError());
    }
  } else if (a.N > 0) {
    // empty scene: every ray misses at its first segment
    k_bounce_epi<<<1, 1, 0, s>>>(ctl, 0);
  }
  const bool diff = (sim->flags & ET_DIFFRACTION) && sim->diff_K > 0 && S.T > 0;
  if (diff) {
    DiffArgs d;
    for (int k = 0; k < 3; ++k) { d.s[k] = sim->emitter_pos[k]; d.axis[k] = sim->emitter_rot[3 * k]; }
    d.cone = sim->diff_cone_half_angle;
    d.tau = sim->diff_tau;
    d.cos_max = std::cos(sim->diff_max_incidence);
    d.seed = sim->diff_seed;
    d.K = sim->diff_K;
    d.t_eps = sim->t_eps;
    d.per_mesh = (sim->flags & ET_DIFF_PER_MESH) ? 1 : 0;
    d.rx_all = perrx ? (sim->M >= 64 ? ~0ull : (1ull << sim->M) - 1ull) : 0ull;
    d.max_meshes = d.per_mesh ? sim->diff_max_meshes : 1;
    const int64_t max_draw = d.K * d.max_meshes;
    stack_fits(max_draw);
    int obj_bits = 1;
    while (obj_bits < 31 && ((int64_t)1 << obj_bits) < S.n_obj) ++obj_bits;
    k_obj_fov<<<nblk_full(S.n_obj), BS, 0, s>>>(S, d, w.oel);
    k_cmax<<<(unsigned)std::min<int64_t>(nblk_full(S.T), 256), BS, 0, s>>>(S, w.oel, ctl);
    k_qweight<<<nblk_full(S.T), BS, 0, s>>>(S, d, w.oel, ctl, w.dq, w.dflags);
    scan_exclusive_u64(w.dflags, w.doffs, S.T, nullptr, S.T, &ctl->tot[1], w.scan_tmp, s);
    k_elig_keys<<<nblk_full(S.T), BS, 0, s>>>(S, d.per_mesh, w.dq, w.dflags, w.doffs, w.dkeys, w.dvals);
    k_elig_count<<<1, 1, 0, s>>>(ctl);
    radix_sort_u64(w.dkeys, w.dvals, 0, &ctl->n_elig, S.T, d.per_mesh ? 32 + obj_bits : 32, w.sort_tmp, s);
    // weights in sorted order, then their exclusive prefix sums (the CDF) and total
    k_sorted_q<<<nblk_full(S.T), BS, 0, s>>>(w.dkeys, ctl, w.dq);
    scan_exclusive_u64(w.dq, w.doffs, 0, &ctl->n_elig, S.T, nullptr, w.scan_tmp, s);
    // groups of the sorted list (meshes, or one) and the number of draws
    k_group_flags<<<nblk_full(S.T), BS, 0, s>>>(w.dkeys, d.per_mesh, ctl, w.dflags);
    scan_exclusive_u64(w.dflags, w.goffs, 0, &ctl->n_elig, S.T, &ctl->tot[2], w.scan_tmp, s);
    k_group_starts<<<nblk_full(S.T), BS, 0, s>>>(w.dflags, w.goffs, ctl, w.gstart);
    k_group_count<<<1, 1, 0, s>>>(ctl, d, w.gstart);
    k_diff_sample<<<nblk(max_draw), BS, 0, s>>>(S, d, w.doffs, w.dq, w.dvals, w, ctl);
    scan_exclusive_u64(w.skeep, w.soffs, 0, &ctl->n_draw, max_draw, &ctl->tot[3], w.scan_tmp, s);
    k_diff_scatter<<<nblk(max_draw), BS, 0, s>>>(S, d, w, ctl, P);
    ET_HIP(hipGetLastError());
  }
  const int32_t n_passive = (sim->flags & ET_PASSIVE) ? sim->M : 0;
  if (n_passive > 0) stack_fits(n_passive);
  if (n_passive > 0)
    k_passive<<<nblk(n_passive), BS, 0, s>>>(S, a, sim->rx_pos, n_passive, diff ? 1 : 0, w, ctl, P, perrx ? 1 : 0);
  k_trace_final<<<1, 1, 0, s>>>(ctl, P, diff ? 1 : 0, n_passive);
  ET_HIP(hipGetLastError());
}

}  // namespace et
