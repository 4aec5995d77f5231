/*
 * oracle.c -- plain FP64 CPU reference for the echo-simulation hot path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the CPU
 * baseline of the benchmark.  The product library never links or calls it, and it
 * shares no source with the GPU path.  Brute force everywhere (no BVH), IEEE double,
 * built with -ffp-contract=off so every expression rounds exactly as written.
 *
 * Paper: Jansen & Steckel, SonoTraceUE (arXiv 2602.19652).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct { double x, y, z; } v3;

static inline v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static inline v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static inline double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 cross(v3 a, v3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static inline double norm(v3 a) { return sqrt(dot(a, a)); }
static inline double ninf(v3 a) { return fmax(fabs(a.x), fmax(fabs(a.y), fabs(a.z))); }
static inline v3 ld3f(const float* p) { return mk((double)p[0], (double)p[1], (double)p[2]); }
static inline v3 ld3d(const double* p) { return mk(p[0], p[1], p[2]); }
static inline void st3(double* p, v3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }
/* R is row-major 3x3; columns are the local axes expressed in world coordinates. */
static inline v3 rot(const double* R, v3 a) {
  return mk(R[0] * a.x + R[1] * a.y + R[2] * a.z, R[3] * a.x + R[4] * a.y + R[5] * a.z, R[6] * a.x + R[7] * a.y + R[8] * a.z);
}
static inline v3 rotT(const double* R, v3 a) {
  return mk(R[0] * a.x + R[3] * a.y + R[6] * a.z, R[1] * a.x + R[4] * a.y + R[7] * a.z, R[2] * a.x + R[5] * a.y + R[8] * a.z);
}

/* ------------------------------------------------------------------ triangle cache */

typedef struct {
  v3 a, b, c;     /* vertices (FP64, exact promotions of the FP32 input) */
  v3 n;           /* unit face normal (e1 x e2 normalised); zero for a degenerate triangle */
  double cm;      /* max |coordinate| over the three vertices */
} tri_t;

static tri_t* make_tris(int64_t T, const float* verts, const int32_t* tris) {
  tri_t* out = (tri_t*)malloc(sizeof(tri_t) * (size_t)(T > 0 ? T : 1));
  for (int64_t i = 0; i < T; ++i) {
    tri_t* t = &out[i];
    t->a = ld3f(verts + 3 * (int64_t)tris[3 * i + 0]);
    t->b = ld3f(verts + 3 * (int64_t)tris[3 * i + 1]);
    t->c = ld3f(verts + 3 * (int64_t)tris[3 * i + 2]);
    v3 n = cross(sub(t->b, t->a), sub(t->c, t->a));
    double nn = norm(n);
    t->n = nn > 0 ? scl(n, 1.0 / nn) : mk(0, 0, 0);
    t->cm = fmax(ninf(t->a), fmax(ninf(t->b), ninf(t->c)));
  }
  return out;
}

/* Moller & Trumbore (1997) ray-triangle test, two-sided (no back-face culling: the
 * reflection about the face normal is independent of its sign). */
static int mt_hit(v3 o, v3 d, const tri_t* T, double* t_out) {
  v3 e1 = sub(T->b, T->a), e2 = sub(T->c, T->a);
  v3 P = cross(d, e2);
  double det = dot(e1, P);
  if (det == 0.0) return 0;
  double inv = 1.0 / det;
  v3 S = sub(o, T->a);
  double u = dot(S, P) * inv;
  if (u < 0.0 || u > 1.0) return 0;
  v3 Qv = cross(S, e1);
  double v = dot(d, Qv) * inv;
  if (v < 0.0 || u + v > 1.0) return 0;
  *t_out = dot(e2, Qv) * inv;
  return 1;
}

/* Closest hit along (o, d) over t > t_eps, excluding triangle `excl`; ties in t go to
 * the smaller triangle index.  Returns the triangle index or -1. */
static int64_t closest_hit(v3 o, v3 d, const tri_t* tr, int64_t T, int64_t excl, double t_eps, double* t_best) {
  int64_t best = -1;
  double bt = INFINITY;
  for (int64_t j = 0; j < T; ++j) {
    if (j == excl) continue;
    double t;
    if (!mt_hit(o, d, &tr[j], &t)) continue;
    if (!(t > t_eps)) continue;
    if (t < bt) { bt = t; best = j; }
  }
  *t_best = bt;
  return best;
}

/* Any hit over t in (t_lo, t_hi), excluding triangle `excl`. */
static int any_hit(v3 o, v3 d, const tri_t* tr, int64_t T, int64_t excl, double t_lo, double t_hi) {
  for (int64_t j = 0; j < T; ++j) {
    if (j == excl) continue;
    double t;
    if (mt_hit(o, d, &tr[j], &t) && t > t_lo && t < t_hi) return 1;
  }
  return 0;
}

/* ------------------------------------------------------------------ margin predicate
 *
 * The GPU decides which triangle a segment meets in FP32 (rays rounded from FP64).
 * A segment is "marginal" when that decision could differ from the FP64 one: some
 * triangle's edge function (the signed volume d.((a-o)x(b-o)), whose sign decides
 * inside/outside) is within a rounding bound of zero, or two candidate depths are
 * within a rounding bound of each other or of the interval ends, or the accepted hit
 * is grazing.  Bounds scale with kappa * 2^-24 (FP32 unit roundoff) times the operand
 * magnitudes.  A ray whose segments are all non-marginal is "certified".
 */
typedef struct { int cls; double t, et, cosn; } probe_t;  /* cls: 0 miss, 1 certain hit, 2 uncertain */

/* Error model of the FP32 decision.  The sign of the edge function E_ab = d.((a-o)x(b-o))
 * says on which side of the edge line the ray passes; E_ab / |d x (b - a)| is the signed
 * distance between the ray and the edge line measured across the ray.  In FP32 that
 * distance is perturbed by: rounding the FP64 origin (|do| <= u |o|_inf per component),
 * rounding the direction (|dd| <= u, i.e. u |a - o| at the vertex), and the arithmetic of
 * the test (differences a - o are exactly rounded, so relative to |a - o|; shear and
 * products add a few more u |a - o|).  The vertices are FP32 inputs on both sides.  A
 * decision is certain when the distance exceeds kappa * u * (max(|a-o|, |b-o|) + |o|_inf). */
static probe_t probe(v3 o, v3 d, const tri_t* T, double kappa) {
  probe_t r;
  double eps = kappa * 0x1p-24;
  double co = fmax(1.0, ninf(o));
  double dn = dot(T->n, d);
  double h = dot(T->n, sub(T->a, o));
  r.cosn = dn;
  if (dn != 0.0) {
    r.t = h / dn;
    r.et = eps * (co + fabs(r.t)) / fmax(fabs(dn), 1e-12);
  } else {
    r.t = INFINITY;
    r.et = INFINITY;
  }
  v3 A = sub(T->a, o), B = sub(T->b, o), C = sub(T->c, o);
  double la = norm(A), lb = norm(B), lc = norm(C);
  double pab = norm(cross(d, sub(T->b, T->a))), pbc = norm(cross(d, sub(T->c, T->b))),
         pca = norm(cross(d, sub(T->a, T->c)));
  double E[3] = {dot(d, cross(A, B)), dot(d, cross(B, C)), dot(d, cross(C, A))};
  double bnd[3] = {eps * (fmax(la, lb) + co) * pab, eps * (fmax(lb, lc) + co) * pbc, eps * (fmax(lc, la) + co) * pca};
  int pos = 0, neg = 0;
  for (int k = 0; k < 3; ++k) {
    if (E[k] > bnd[k]) ++pos;
    else if (E[k] < -bnd[k]) ++neg;
  }
  if (pos > 0 && neg > 0) r.cls = 0;
  else if (pos == 3 || neg == 3) r.cls = 1;
  else r.cls = 2;
  if (T->n.x == 0 && T->n.y == 0 && T->n.z == 0) r.cls = 0;
  return r;
}

/* Closest-hit segment: hit triangle `h` at t_star (h < 0: miss). */
static int closest_marginal(v3 o, v3 d, const tri_t* tr, int64_t T, int64_t excl, double t_eps, int64_t h,
                            double t_star, double kappa, double mu_g) {
  double eps = kappa * 0x1p-24;
  double hi_star = INFINITY;
  if (h >= 0) {
    probe_t ph = probe(o, d, &tr[h], kappa);
    if (ph.cls != 1) return 1;                     /* hit near an edge of its triangle */
    if (fabs(ph.cosn) < mu_g) return 1;            /* grazing incidence */
    double et = eps * (fmax(1.0, ninf(o)) + t_star) / fmax(fabs(ph.cosn), 1e-12);
    if (t_star - et <= t_eps) return 1;            /* near the self-intersection threshold */
    hi_star = t_star + et;
  }
  for (int64_t j = 0; j < T; ++j) {
    if (j == excl || j == h) continue;
    probe_t p = probe(o, d, &tr[j], kappa);
    if (p.cls == 0 || !isfinite(p.t)) {
      if (p.cls != 0 && fabs(p.cosn) < 1e-12) {
        /* line parallel to a plane it might touch: marginal if it runs within the bound */
        double hgt = fabs(dot(tr[j].n, sub(tr[j].a, o)));
        if (hgt < eps * fmax(1.0, ninf(o))) return 1;
      }
      continue;
    }
    double lo = p.t - p.et, hi = p.t + p.et;
    if (hi <= t_eps) continue;                     /* certainly behind the threshold */
    if (lo <= t_eps) return 1;                     /* straddles the threshold */
    if (lo < hi_star) return 1;                    /* could be (or tie with) the closest */
  }
  return 0;
}

/* Any-hit segment over (t_lo, t_hi). */
static int anyhit_marginal(v3 o, v3 d, const tri_t* tr, int64_t T, int64_t excl, double t_lo, double t_hi,
                           double kappa) {
  double eps = kappa * 0x1p-24;
  for (int64_t j = 0; j < T; ++j) {
    if (j == excl) continue;
    probe_t p = probe(o, d, &tr[j], kappa);
    if (p.cls == 0) continue;
    if (!isfinite(p.t)) {
      double hgt = fabs(dot(tr[j].n, sub(tr[j].a, o)));
      if (hgt < eps * fmax(1.0, ninf(o))) return 1;
      continue;
    }
    double lo = p.t - p.et, hi = p.t + p.et;
    if (hi <= t_lo || lo >= t_hi) continue;
    if (p.cls == 2) return 1;
    if (lo <= t_lo || hi >= t_hi) return 1;
  }
  return 0;
}

/* ------------------------------------------------------------------ Algorithm 1 */

int orc_trace(int64_t V, int64_t T, const float* verts, const int32_t* tris, const int32_t* tri_mat,
              const double* emitter_pos, const double* emitter_rot, int64_t N, const float* dirs,
              int32_t max_bounces, double max_distance, const double* x_ref, double t_eps,
              double kappa, double mu_g, int64_t capacity,
              int64_t* n_rec, int32_t* rec_ray, int32_t* rec_bounce, int32_t* rec_tri, int32_t* rec_mat,
              double* rec_p, double* rec_din, double* rec_dout, double* rec_rtot, uint8_t* rec_vis,
              uint8_t* ray_certified, int32_t* ray_nseg, int32_t M, const double* rx_pos, uint64_t* rec_rxvis) {
  (void)V;
  if (N < 0 || T < 0 || max_bounces < 1 || capacity < N * (int64_t)max_bounces) return -1;
  if (rec_rxvis && (M < 1 || M > 64 || !rx_pos)) return -1;
  tri_t* tr = make_tris(T, verts, tris);
  const int B = max_bounces;
  /* per-ray fixed slots, compacted afterwards in (ray, bounce) order */
  int32_t* s_tri = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N * B + 1));
  double* s_p = (double*)malloc(sizeof(double) * 3 * (size_t)(N * B + 1));
  double* s_din = (double*)malloc(sizeof(double) * 3 * (size_t)(N * B + 1));
  double* s_dout = (double*)malloc(sizeof(double) * 3 * (size_t)(N * B + 1));
  double* s_r = (double*)malloc(sizeof(double) * (size_t)(N * B + 1));
  uint8_t* s_vis = (uint8_t*)malloc((size_t)(N * B + 1));
  uint64_t* s_rxvis = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(N * B + 1));
  int32_t* s_cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N + 1));
  v3 s = ld3d(emitter_pos);
  v3 xr = ld3d(x_ref);
  int certify = kappa > 0;

#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < N; ++i) {
    v3 dw = rot(emitter_rot, ld3f(dirs + 3 * i));         /* CalculateWorldDirection */
    v3 d = scl(dw, 1.0 / norm(dw));
    v3 o = s;
    double rtot = 0.0;
    int64_t prev = -1;
    int cert = 1, cnt = 0, nseg = 0;
    for (int j = 0; j < B; ++j) {
      double t;
      ++nseg;
      int64_t h = closest_hit(o, d, tr, T, prev, t_eps, &t);
      if (certify && cert && closest_marginal(o, d, tr, T, prev, t_eps, h, t, kappa, mu_g)) cert = 0;
      if (h < 0) break;                                     /* miss: stop the ray */
      v3 p = add(o, scl(d, t));
      v3 n = tr[h].n;
      v3 dr = sub(d, scl(n, 2.0 * dot(d, n)));              /* specular reflection */
      rtot = (j == 0) ? norm(sub(p, s)) : rtot + t;         /* path length to the hit */
      int blocked;
      uint64_t bits = 0;
      if (!rec_rxvis) {
        /* line-of-sight ray from the hit point toward the receiver reference point */
        v3 w = sub(xr, p);
        double L = norm(w);
        v3 dv = scl(w, 1.0 / L);
        blocked = any_hit(p, dv, tr, T, h, t_eps, L - t_eps);
        if (certify && cert && anyhit_marginal(p, dv, tr, T, h, t_eps, L - t_eps, kappa)) cert = 0;
      } else {
        /* per-receiver variant: one line-of-sight ray from the hit point to every receiver */
        for (int32_t m = 0; m < M; ++m) {
          v3 w = sub(ld3d(rx_pos + 3 * m), p);
          double L = norm(w);
          v3 dv = scl(w, 1.0 / L);
          int bl = any_hit(p, dv, tr, T, h, t_eps, L - t_eps);
          if (certify && cert && anyhit_marginal(p, dv, tr, T, h, t_eps, L - t_eps, kappa)) cert = 0;
          if (!bl) bits |= 1ull << m;
        }
        blocked = bits == 0;
      }
      int64_t slot = i * B + cnt;
      s_tri[slot] = (int32_t)h;
      st3(s_p + 3 * slot, p);
      st3(s_din + 3 * slot, d);
      st3(s_dout + 3 * slot, dr);
      s_r[slot] = rtot;
      s_vis[slot] = (uint8_t)(!blocked);
      s_rxvis[slot] = bits;
      ++cnt;
      if (isfinite(max_distance) && fabs(rtot - max_distance) < kappa * 0x1p-24 * fmax(1.0, rtot)) cert = 0;
      if (rtot >= max_distance) break;
      o = p;
      d = dr;
      prev = h;
    }
    s_cnt[i] = cnt;
    if (ray_certified) ray_certified[i] = (uint8_t)cert;
    if (ray_nseg) ray_nseg[i] = nseg;
  }
  int64_t w = 0;
  for (int64_t i = 0; i < N; ++i) {
    for (int j = 0; j < s_cnt[i]; ++j) {
      int64_t slot = i * B + j;
      rec_ray[w] = (int32_t)i;
      rec_bounce[w] = j;
      rec_tri[w] = s_tri[slot];
      rec_mat[w] = tri_mat[s_tri[slot]];
      memcpy(rec_p + 3 * w, s_p + 3 * slot, 3 * sizeof(double));
      memcpy(rec_din + 3 * w, s_din + 3 * slot, 3 * sizeof(double));
      memcpy(rec_dout + 3 * w, s_dout + 3 * slot, 3 * sizeof(double));
      rec_rtot[w] = s_r[slot];
      rec_vis[w] = s_vis[slot];
      if (rec_rxvis) rec_rxvis[w] = s_rxvis[slot];
      ++w;
    }
  }
  *n_rec = w;
  free(s_tri); free(s_p); free(s_din); free(s_dout); free(s_r); free(s_vis); free(s_rxvis); free(s_cnt); free(tr);
  return 0;
}

/* ------------------------------------------------------------------ passive component
 *
 * Direct propagation from the emitter to each receiver (the passive component of the
 * method, with its transfer function P(f) = L_geo L_atm I_p e^{j omega r / c}): one
 * line-of-sight test per receiver over the open segment (t_eps, r - t_eps), no triangle
 * excluded.  certified[m] = 0 when that decision is marginal in the FP32 sense. */
int orc_passive(int64_t V, int64_t T, const float* verts, const int32_t* tris, const double* emitter_pos,
                int32_t M, const double* rx_pos, double t_eps, double kappa, uint8_t* vis, uint8_t* certified) {
  if (T < 0 || M < 0 || (T > 0 && (!verts || !tris))) return -1;
  (void)V;
  tri_t* tr = T > 0 ? make_tris(T, verts, tris) : NULL;
  v3 s = ld3d(emitter_pos);
  for (int32_t m = 0; m < M; ++m) {
    v3 w = sub(ld3d(rx_pos + 3 * m), s);
    double r = norm(w);
    int blocked = 0, marg = 0;
    if (r > 2.0 * t_eps && T > 0) {
      v3 d = scl(w, 1.0 / r);
      blocked = any_hit(s, d, tr, T, -1, t_eps, r - t_eps);
      marg = kappa > 0.0 && anyhit_marginal(s, d, tr, T, -1, t_eps, r - t_eps, kappa);
    }
    vis[m] = (uint8_t)!blocked;
    if (certified) certified[m] = (uint8_t)!marg;
  }
  free(tr);
  return 0;
}

/* ------------------------------------------------------------------ synthesis */

/* Receiver directivity: real gain per band, cell-centred az/el grid in the receiver
 * frame (az from -pi, el from -pi/2), bilinear, azimuth periodic, elevation clamped.
 * With dv != NULL also the gradient of the gain with respect to the direction v: the
 * derivative of the bilinear interpolant inside the cell that holds v (zero across the
 * clamped elevation rows; undefined on the poles, where it is set to zero). */
static double directivity_gain_dv(const float* tab, int El, int Az, v3 v, v3* dv) {
  double az = atan2(v.y, v.x);
  double el = atan2(v.z, hypot(v.x, v.y));
  double fa = (az + M_PI) / (2.0 * M_PI) * Az - 0.5;
  double fl = floor(fa);
  double ta = fa - fl;
  long i0 = ((long)fl % Az + Az) % Az, i1 = (i0 + 1) % Az;
  double fe = (el + 0.5 * M_PI) / M_PI * El - 0.5;
  long j0, j1;
  double te;
  int inner = 0;
  if (fe <= 0.0) { j0 = j1 = 0; te = 0.0; }
  else if (fe >= El - 1) { j0 = j1 = El - 1; te = 0.0; }
  else { j0 = (long)floor(fe); j1 = j0 + 1; te = fe - (double)j0; inner = 1; }
  double a0 = (1.0 - ta) * tab[j0 * Az + i0] + ta * tab[j0 * Az + i1];
  double a1 = (1.0 - ta) * tab[j1 * Az + i0] + ta * tab[j1 * Az + i1];
  if (dv) {
    /* dD/daz and dD/del through the cell coordinates fa = (az + pi) Az / 2pi - 1/2 and
     * fe = (el + pi/2) El / pi - 1/2, then az = atan2(y, x) and el = atan2(z, rho) */
    double dfa = (1.0 - te) * ((double)tab[j0 * Az + i1] - tab[j0 * Az + i0]) +
                 te * ((double)tab[j1 * Az + i1] - tab[j1 * Az + i0]);
    double dfe = inner ? a1 - a0 : 0.0;
    double daz = dfa * Az / (2.0 * M_PI), del = dfe * El / M_PI;
    double rho2 = v.x * v.x + v.y * v.y, rho = sqrt(rho2), n2 = rho2 + v.z * v.z;
    if (rho2 > 0.0) {
      dv->x = -daz * v.y / rho2 - del * v.x * v.z / (rho * n2);
      dv->y = daz * v.x / rho2 - del * v.y * v.z / (rho * n2);
      dv->z = del * rho / n2;
    } else {
      *dv = mk(0, 0, 0);
    }
  }
  return (1.0 - te) * a0 + te * a1;
}

static double directivity_gain(const float* tab, int El, int Az, v3 v) {
  return directivity_gain_dv(tab, El, Az, v, NULL);
}

typedef struct {
  double l, r, gamma;   /* receiver leg, total path, deviation angle (specular only) */
  v3 u;                 /* unit vector from the point toward the receiver */
} pair_t;

static pair_t pair_setup(v3 p, v3 dout, double rtot, int kind, v3 xm) {
  pair_t q;
  v3 w = sub(xm, p);
  q.l = norm(w);
  q.u = scl(w, 1.0 / q.l);
  q.r = rtot + q.l;                          /* total path emitter -> point -> receiver */
  q.gamma = 0.0;
  if (kind == 0) q.gamma = atan2(norm(cross(dout, q.u)), dot(dout, q.u));
  return q;
}

/* Path-product reading of the reflection magnitude (the alternative to "k of the hit
 * triangle only"): a specular record at reflection n carries the product of k(T_j, band) over
 * its ray's reflections j <= n.  kp[n][b] for specular records (others unused), from the
 * records' ray and reflection indices: the specular records grouped by ray in increasing
 * reflection order, running products along each ray. */
typedef struct { int32_t ray, bounce; int64_t n; } rb_t;
static int cmp_rb(const void* a, const void* b) {
  const rb_t* x = (const rb_t*)a;
  const rb_t* y = (const rb_t*)b;
  if (x->ray != y->ray) return x->ray < y->ray ? -1 : 1;
  return x->bounce < y->bounce ? -1 : (x->bounce > y->bounce);
}
static double* path_k_products(int64_t n_rec, const uint8_t* kind, const int32_t* mat, const int32_t* ray,
                               const int32_t* bounce, int32_t Bk, const float* refl_k) {
  double* kp = (double*)calloc((size_t)(n_rec > 0 ? n_rec : 1) * Bk, sizeof(double));
  rb_t* list = (rb_t*)malloc(sizeof(rb_t) * (size_t)(n_rec > 0 ? n_rec : 1));
  int64_t ns = 0;
  for (int64_t n = 0; n < n_rec; ++n)
    if (!kind || kind[n] == 0) { list[ns].ray = ray[n]; list[ns].bounce = bounce[n]; list[ns].n = n; ++ns; }
  qsort(list, (size_t)ns, sizeof(rb_t), cmp_rb);
  for (int64_t i = 0; i < ns; ++i) {
    const int64_t n = list[i].n;
    const int first = i == 0 || list[i - 1].ray != list[i].ray;
    for (int b = 0; b < Bk; ++b) {
      const double prev = first ? 1.0 : kp[list[i - 1].n * Bk + b];
      kp[n * Bk + b] = prev * (double)refl_k[mat[n] * Bk + b];
    }
  }
  free(list);
  return kp;
}

int orc_synth(int64_t n_rec, const double* p, const double* dout, const double* rtot, const int32_t* mat,
              const uint8_t* kind, const uint8_t* vis, int32_t M, const double* rx_pos, const double* rx_rot,
              double f_lo, double f_hi, int32_t F, int32_t nk, const int32_t* k_list,
              double c, double A0, double A1, double p_s, int32_t sigma,
              int32_t Q, int32_t Bk, const float* refl_k, const float* beta, const float* diff_coef,
              int32_t Bd, int32_t El, int32_t Az, const float* directivity, const float* passive_coef,
              const int32_t* rx_id, double* out, const uint64_t* rxvis, const int32_t* rec_ray,
              const int32_t* rec_bounce, int path_product) {
  if (M < 1 || F < 1 || nk < 1 || Q < 1 || Bk < 1) return -1;
  if (directivity && (Bd < 1 || El < 1 || Az < 1)) return -1;
  if (path_product && (!rec_ray || !rec_bounce)) return -1;
  for (int64_t n = 0; n < n_rec; ++n)
    if (kind && kind[n] == 2 && !passive_coef) return -1;   /* passive records need I_p */
  double* kp = path_product ? path_k_products(n_rec, kind, mat, rec_ray, rec_bounce, Bk, refl_k) : NULL;
  const double df = F > 1 ? (f_hi - f_lo) / (double)(F - 1) : 0.0;
  const int KB = 64;
  const int nkb = (nk + KB - 1) / KB;
  memset(out, 0, sizeof(double) * 2 * (size_t)M * (size_t)nk);
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
  for (int m = 0; m < M; ++m) {
    for (int kb = 0; kb < nkb; ++kb) {
      int k0 = kb * KB, k1 = k0 + KB < nk ? k0 + KB : nk;
      double acc[2 * 64];
      memset(acc, 0, sizeof(acc));
      v3 xm = ld3d(rx_pos + 3 * m);
      double Dg[64];
      const int gm = rx_id ? rx_id[m] : m;   /* receiver index of the full array */
      for (int64_t n = 0; n < n_rec; ++n) {
        if (rxvis ? !((rxvis[n] >> gm) & 1ull) : (vis && !vis[n])) continue;
        int kd = kind ? kind[n] : 0;
        if (kd == 2 && mat[n] != gm) continue;   /* passive: its own receiver only */
        v3 pn = ld3d(p + 3 * n);
        pair_t q = pair_setup(pn, kd == 0 ? ld3d(dout + 3 * n) : mk(1, 0, 0), rtot[n], kd, xm);
        if (directivity) {
          const double* Rm = rx_rot ? rx_rot + 9 * m : NULL;
          v3 arr = scl(q.u, -1.0);                          /* direction of arrival, world */
          v3 vl = Rm ? rotT(Rm, arr) : arr;
          int nb = Bd < 64 ? Bd : 64;
          for (int b = 0; b < nb; ++b)
            Dg[b] = directivity_gain(directivity + ((size_t)m * Bd + b) * (size_t)El * Az, El, Az, vl);
        }
        double Lgeo = pow(q.r, -p_s);                       /* spherical spreading */
        for (int kk = k0; kk < k1; ++kk) {
          int64_t k = k_list ? k_list[kk] : kk;
          double f = f_lo + (double)k * df;
          int64_t b = (k * Bk) / F;
          double Latm = pow(10.0, -(A0 + A1 * f) * q.r / 20.0);   /* air absorption */
          double I;
          if (kd == 0) {
            double bt = (double)beta[mat[n] * Bk + b];
            double kv = kp ? kp[n * Bk + b] : (double)refl_k[mat[n] * Bk + b];
            I = exp(-(q.gamma * q.gamma) / (2.0 * bt * bt)) * kv;
          } else if (kd == 1) {
            I = (double)diff_coef[mat[n] * Bk + b];
          } else {
            I = (double)passive_coef[b];
          }
          double A = Lgeo * Latm * I;
          if (directivity) A *= Dg[(k * Bd) / F];
          double cyc = (double)sigma * f * q.r / c;         /* delay in cycles at f */
          double ph = 2.0 * M_PI * (cyc - floor(cyc));
          acc[2 * (kk - k0)] += A * cos(ph);
          acc[2 * (kk - k0) + 1] += A * sin(ph);
        }
      }
      for (int kk = k0; kk < k1; ++kk) {
        out[2 * ((size_t)m * nk + kk)] = acc[2 * (kk - k0)];
        out[2 * ((size_t)m * nk + kk) + 1] = acc[2 * (kk - k0) + 1];
      }
    }
  }
  free(kp);
  return 0;
}

/* ------------------------------------------------------------------ adjoint */

int orc_grad(int64_t n_rec, const double* p, const double* dout, const double* rtot, const int32_t* mat,
             const uint8_t* kind, const uint8_t* vis, int32_t M, const double* rx_pos,
             double f_lo, double f_hi, int32_t F, double c, double A0, double A1, double p_s, int32_t sigma,
             int32_t Q, int32_t Bk, const float* refl_k, const float* beta, const float* diff_coef,
             const float* passive_coef, const double* g, double* grad_k, double* grad_x, const uint64_t* rxvis,
             const double* rx_rot, int32_t Bd, int32_t El, int32_t Az, const float* directivity) {
  if (M < 1 || F < 1 || Q < 1 || Bk < 1 || Bk > 64) return -1;
  if (directivity && (Bd < 1 || Bd > 64 || El < 1 || Az < 1)) return -1;
  for (int64_t n = 0; n < n_rec; ++n)
    if (kind && kind[n] == 2 && !passive_coef) return -1;   /* passive records need I_p */
  const double df = F > 1 ? (f_hi - f_lo) / (double)(F - 1) : 0.0;
  const double ln10 = log(10.0);
  double* gk_m = (double*)calloc((size_t)M * Q * Bk, sizeof(double));
  memset(grad_x, 0, sizeof(double) * 3 * (size_t)M);
#pragma omp parallel for schedule(dynamic, 1)
  for (int m = 0; m < M; ++m) {
    v3 xm = ld3d(rx_pos + 3 * m);
    v3 gx = mk(0, 0, 0);
    double* gk = gk_m + (size_t)m * Q * Bk;
    for (int64_t n = 0; n < n_rec; ++n) {
      if (rxvis ? !((rxvis[n] >> m) & 1ull) : (vis && !vis[n])) continue;
      int kd = kind ? kind[n] : 0;
      if (kd == 2 && mat[n] != m) continue;   /* passive: its own receiver only */
      v3 pn = ld3d(p + 3 * n);
      v3 dn = kd == 0 ? ld3d(dout + 3 * n) : mk(1, 0, 0);
      pair_t q = pair_setup(pn, dn, rtot[n], kd, xm);
      double Lgeo = pow(q.r, -p_s);
      double Sb[2 * 64], Sk[64], Sd[64], Dg[64];
      v3 dDg[64];
      memset(Sb, 0, sizeof(double) * 2 * Bk);
      memset(Sk, 0, sizeof(double) * Bk);
      const double* Rm = rx_rot ? rx_rot + 9 * m : NULL;
      if (directivity) {
        /* gain per directivity band and its gradient in the receiver frame (as in orc_synth) */
        v3 vl = Rm ? rotT(Rm, scl(q.u, -1.0)) : scl(q.u, -1.0);
        for (int d = 0; d < Bd; ++d) {
          Dg[d] = directivity_gain_dv(directivity + ((size_t)m * Bd + d) * (size_t)El * Az, El, Az, vl, &dDg[d]);
          Sd[d] = 0.0;
        }
      }
      double S1r = 0, S1i = 0;
      for (int64_t k = 0; k < F; ++k) {
        double f = f_lo + (double)k * df;
        int64_t b = (k * Bk) / F;
        double Latm = pow(10.0, -(A0 + A1 * f) * q.r / 20.0);
        double I, lobe = 0.0;
        if (kd == 0) {
          double bt = (double)beta[mat[n] * Bk + b];
          lobe = exp(-(q.gamma * q.gamma) / (2.0 * bt * bt));
          I = lobe * (double)refl_k[mat[n] * Bk + b];
        } else if (kd == 1) {
          I = (double)diff_coef[mat[n] * Bk + b];
        } else {
          I = (double)passive_coef[b];
        }
        double A = Lgeo * Latm * I;
        if (directivity) A *= Dg[(k * Bd) / F];
        double cyc = (double)sigma * f * q.r / c;
        double ph = 2.0 * M_PI * (cyc - floor(cyc));
        double Tr = A * cos(ph), Ti = A * sin(ph);
        double gr = g[2 * ((size_t)m * F + k)], gi = g[2 * ((size_t)m * F + k) + 1];
        /* conj(g) * T */
        double zr = gr * Tr + gi * Ti, zi = gr * Ti - gi * Tr;
        if (kd == 0) {
          /* H is linear in k (Eq. 2): dT/dk is T with the factor k left out, also where k = 0 */
          double Ak = Lgeo * Latm * lobe;
          if (directivity) Ak *= Dg[(k * Bd) / F];
          Sk[b] += gr * Ak * cos(ph) + gi * Ak * sin(ph);
        }
        Sb[2 * b] += zr;
        Sb[2 * b + 1] += zi;
        if (directivity) Sd[(k * Bd) / F] += zr;
        S1r += f * zr;
        S1i += f * zi;
      }
      double S0r = 0;
      for (int b = 0; b < Bk; ++b) S0r += Sb[2 * b];
      /* d(ln A + j phi)/dx_m = [(-p/r - ln10 (A0 + A1 f)/20) + j sigma 2 pi f / c] u  - dgamma^2/dx / (2 beta^2) */
      double cu = (-p_s / q.r - ln10 * A0 / 20.0) * S0r - ln10 * A1 / 20.0 * S1r - (double)sigma * 2.0 * M_PI / c * S1i;
      v3 grad = scl(q.u, 2.0 * cu);
      if (kd == 0) {
        double sg = norm(cross(dn, q.u)) / norm(dn);
        double cg = dot(dn, q.u) / norm(dn);
        double ratio = (q.gamma < 1e-8) ? 2.0 : 2.0 * q.gamma / sg;
        /* d(gamma^2)/dx = -(2 gamma / sin gamma) (d' - cos(gamma) u) / l, with |d'| = 1 */
        v3 dhat = scl(dn, 1.0 / norm(dn));
        v3 dg2 = scl(sub(dhat, scl(q.u, cg)), -ratio / q.l);
        double wsum = 0;
        for (int b = 0; b < Bk; ++b) {
          double bt = (double)beta[mat[n] * Bk + b];
          wsum += Sb[2 * b] / (2.0 * bt * bt);
          gk[mat[n] * Bk + b] += 2.0 * Sk[b];
        }
        grad = sub(grad, scl(dg2, 2.0 * wsum));
      }
      if (directivity) {
        /* d ln D_d / dx_m: v = -R^T u and du/dx_m = (I - u u^T) / l, so the gradient in x is
         * -(I - u u^T) R (dD_d/dv) / (l D_d) */
        v3 gv = mk(0, 0, 0);
        for (int d = 0; d < Bd; ++d)
          if (Dg[d] != 0.0) gv = add(gv, scl(dDg[d], Sd[d] / Dg[d]));
        v3 w = Rm ? mk(Rm[0] * gv.x + Rm[1] * gv.y + Rm[2] * gv.z, Rm[3] * gv.x + Rm[4] * gv.y + Rm[5] * gv.z,
                       Rm[6] * gv.x + Rm[7] * gv.y + Rm[8] * gv.z)
                  : gv;
        v3 wp = sub(w, scl(q.u, dot(q.u, w)));
        grad = sub(grad, scl(wp, 2.0 / q.l));
      }
      gx = add(gx, grad);
    }
    st3(grad_x + 3 * m, gx);
  }
  memset(grad_k, 0, sizeof(double) * (size_t)Q * Bk);
  for (int m = 0; m < M; ++m)
    for (int64_t i = 0; i < (int64_t)Q * Bk; ++i) grad_k[i] += gk_m[(size_t)m * Q * Bk + i];
  free(gk_m);
  return 0;
}

/* ------------------------------------------------------------------ curvature (Eq. 1) */

int orc_curvature(int64_t V, int64_t T, const float* verts, const int32_t* tris, double a_ref,
                  double* G_v, double* C) {
  if (V < 0 || T < 0) return -1;
  double* K = (double*)calloc(3 * (size_t)(V + 1), sizeof(double));
  double* Am = (double*)calloc((size_t)(V + 1), sizeof(double));
  /* Meyer et al. (2003): K(x_i) = 1/(2 A_mixed) sum_j (cot a_ij + cot b_ij)(x_i - x_j),
   * accumulated triangle by triangle in index order. */
  for (int64_t t = 0; t < T; ++t) {
    int32_t id[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    v3 P[3] = {ld3f(verts + 3 * (int64_t)id[0]), ld3f(verts + 3 * (int64_t)id[1]), ld3f(verts + 3 * (int64_t)id[2])};
    double area2 = norm(cross(sub(P[1], P[0]), sub(P[2], P[0])));
    double area = 0.5 * area2;
    if (area < 1e-20) continue;
    double dotc[3], cot[3];
    for (int c = 0; c < 3; ++c) {
      dotc[c] = dot(sub(P[(c + 1) % 3], P[c]), sub(P[(c + 2) % 3], P[c]));
      cot[c] = dotc[c] / area2;
    }
    int obtuse = dotc[0] < 0.0 || dotc[1] < 0.0 || dotc[2] < 0.0;
    for (int c = 0; c < 3; ++c) {
      int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      v3 ea = sub(P[c], P[c1]), eb = sub(P[c], P[c2]);
      int64_t i = id[c];
      K[3 * i + 0] += cot[c2] * ea.x + cot[c1] * eb.x;
      K[3 * i + 1] += cot[c2] * ea.y + cot[c1] * eb.y;
      K[3 * i + 2] += cot[c2] * ea.z + cot[c1] * eb.z;
      if (!obtuse) Am[i] += (dot(ea, ea) * cot[c2] + dot(eb, eb) * cot[c1]) / 8.0;   /* Voronoi region */
      else if (dotc[c] < 0.0) Am[i] += area / 2.0;
      else Am[i] += area / 4.0;
    }
  }
  for (int64_t v = 0; v < V; ++v) {
    double kn = sqrt(K[3 * v] * K[3 * v] + K[3 * v + 1] * K[3 * v + 1] + K[3 * v + 2] * K[3 * v + 2]);
    G_v[v] = Am[v] > 0.0 ? kn / (4.0 * Am[v]) : 0.0;   /* G = |K|/2 with K = sum / (2 A_mixed) */
  }
  for (int64_t t = 0; t < T; ++t) {
    double g0 = G_v[tris[3 * t]], g1 = G_v[tris[3 * t + 1]], g2 = G_v[tris[3 * t + 2]];
    double dG = fmax(g0, fmax(g1, g2)) - fmin(g0, fmin(g1, g2));
    v3 P0 = ld3f(verts + 3 * (int64_t)tris[3 * t]), P1 = ld3f(verts + 3 * (int64_t)tris[3 * t + 1]),
       P2 = ld3f(verts + 3 * (int64_t)tris[3 * t + 2]);
    double area = 0.5 * norm(cross(sub(P1, P0), sub(P2, P0)));
    double w = a_ref > 0.0 ? fmin(1.0, area / a_ref) : 1.0;
    C[t] = w * dG;
  }
  free(K);
  free(Am);
  return 0;
}

/* ------------------------------------------------------------------ diffraction (Sec. III-D) */

uint64_t orc_splitmix(uint64_t key, uint64_t counter) {
  uint64_t z = key + (counter + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double u01(uint64_t x) { return (double)(x >> 11) * 0x1p-53; }

typedef struct { uint64_t q; int64_t i; int32_t o; } qi_t;
static int cmp_qi(const void* a, const void* b) {
  const qi_t* x = (const qi_t*)a;
  const qi_t* y = (const qi_t*)b;
  if (x->q != y->q) return x->q > y->q ? -1 : 1;   /* weight descending */
  return x->i < y->i ? -1 : (x->i > y->i);          /* index ascending */
}
static int cmp_oqi(const void* a, const void* b) {   /* mesh first, then as cmp_qi */
  const qi_t* x = (const qi_t*)a;
  const qi_t* y = (const qi_t*)b;
  if (x->o != y->o) return x->o < y->o ? -1 : 1;
  return cmp_qi(a, b);
}

int orc_diffraction(int64_t V, int64_t T, const float* verts, const int32_t* tris, const int32_t* tri_obj,
                    int32_t n_obj, const double* C, const double* emitter_pos, const double* emitter_rot,
                    double cone_half_angle, double tau, uint64_t seed, int64_t K, double max_incidence,
                    double t_eps, double kappa, int per_mesh, int64_t max_meshes,
                    uint64_t* q_out, int64_t* n_elig, int64_t* n_samples, int32_t* samp_tri, double* samp_o,
                    double* samp_r, uint8_t* samp_keep, uint8_t* samp_certified) {
  (void)V;
  if (T < 0 || n_obj < 1 || K < 0 || (per_mesh && max_meshes < 1)) return -1;
  v3 s = ld3d(emitter_pos);
  v3 axis = rot(emitter_rot, mk(1, 0, 0));
  /* objects inside the emitter's field of view: bounding sphere of the object's box meets the cone */
  double* lo = (double*)malloc(sizeof(double) * 3 * n_obj);
  double* hi = (double*)malloc(sizeof(double) * 3 * n_obj);
  for (int o = 0; o < n_obj; ++o) { lo[3 * o] = lo[3 * o + 1] = lo[3 * o + 2] = INFINITY; hi[3 * o] = hi[3 * o + 1] = hi[3 * o + 2] = -INFINITY; }
  for (int64_t t = 0; t < T; ++t) {
    int o = tri_obj[t];
    for (int k = 0; k < 3; ++k) {
      const float* v = verts + 3 * (int64_t)tris[3 * t + k];
      for (int a = 0; a < 3; ++a) { lo[3 * o + a] = fmin(lo[3 * o + a], (double)v[a]); hi[3 * o + a] = fmax(hi[3 * o + a], (double)v[a]); }
    }
  }
  uint8_t* oel = (uint8_t*)calloc((size_t)n_obj, 1);
  for (int o = 0; o < n_obj; ++o) {
    if (!(lo[3 * o] <= hi[3 * o])) continue;
    v3 cen = mk(0.5 * (lo[3 * o] + hi[3 * o]), 0.5 * (lo[3 * o + 1] + hi[3 * o + 1]), 0.5 * (lo[3 * o + 2] + hi[3 * o + 2]));
    double rad = 0.5 * norm(sub(mk(hi[3 * o], hi[3 * o + 1], hi[3 * o + 2]), mk(lo[3 * o], lo[3 * o + 1], lo[3 * o + 2])));
    v3 w = sub(cen, s);
    double dist = norm(w);
    if (dist <= rad) { oel[o] = 1; continue; }
    double psi = atan2(norm(cross(w, axis)), dot(w, axis));
    oel[o] = psi <= cone_half_angle + asin(rad / dist);
  }
  double cmax = 0.0;
  for (int64_t t = 0; t < T; ++t)
    if (oel[tri_obj[t]] && C[t] > cmax) cmax = C[t];
  const uint64_t kd = seed ^ 1ull, ks = seed ^ 2ull;
  qi_t* list = (qi_t*)malloc(sizeof(qi_t) * (size_t)(T > 0 ? T : 1));
  int64_t ne = 0;
  for (int64_t t = 0; t < T; ++t) {
    uint64_t q = 0;
    if (cmax > 0.0 && oel[tri_obj[t]] && C[t] > 0.0 && C[t] >= tau * cmax) {
      /* dithered integer weight: stochastic rounding of (C/Cmax) * 2^32 */
      q = (uint64_t)floor(C[t] / cmax * 4294967296.0 + u01(orc_splitmix(kd, (uint64_t)t)));
      if (q > 0) { list[ne].q = q; list[ne].i = t; list[ne].o = tri_obj[t]; ++ne; }
    }
    if (q_out) q_out[t] = q;
  }
  *n_elig = ne;
  /* the triangles sorted by weight (per mesh: grouped by mesh first); one CDF per group,
   * the running sums restarting at every group */
  qsort(list, (size_t)ne, sizeof(qi_t), per_mesh ? cmp_oqi : cmp_qi);
  int64_t* gstart = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ne + 1));
  int64_t ng = 0;
  for (int64_t j = 0; j < ne; ++j)
    if (j == 0 || (per_mesh && list[j].o != list[j - 1].o)) gstart[ng++] = j;
  gstart[ng] = ne;
  int truncated = 0;
  if (per_mesh && ng > max_meshes) { ng = max_meshes; truncated = 1; }
  uint64_t* W = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(ne > 0 ? ne : 1));
  for (int64_t g = 0; g < ng; ++g) {
    uint64_t acc = 0;
    for (int64_t j = gstart[g]; j < gstart[g + 1]; ++j) { acc += list[j].q; W[j] = acc; }
  }
  const int64_t n_draw = per_mesh ? K * ng : K;
  *n_samples = n_draw;
  tri_t* tr = make_tris(T, verts, tris);
  const double cos_max = cos(max_incidence);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < n_draw; ++k) {
    if (ne == 0) { samp_tri[k] = -1; samp_keep[k] = 0; if (samp_certified) samp_certified[k] = 1; continue; }
    const int64_t g = per_mesh ? k / K : 0;   /* the group (mesh) this draw belongs to */
    const int64_t j0 = gstart[g], j1 = gstart[g + 1];
    const uint64_t acc = W[j1 - 1];
    uint64_t U = orc_splitmix(ks, 3 * (uint64_t)k);
    uint64_t idx = (uint64_t)(((unsigned __int128)U * (unsigned __int128)acc) >> 64);
    int64_t a = j0, b = j1;           /* first position of the group with W > idx */
    while (a < b) { int64_t mid = (a + b) / 2; if (W[mid] > idx) b = mid; else a = mid + 1; }
    int64_t t = list[a].i;
    double u1 = u01(orc_splitmix(ks, 3 * (uint64_t)k + 1)), u2 = u01(orc_splitmix(ks, 3 * (uint64_t)k + 2));
    double su = sqrt(u1);
    double wa = 1.0 - su, wb = su * (1.0 - u2), wc = su * u2;   /* uniform point on the triangle */
    v3 o = mk(wa * tr[t].a.x + wb * tr[t].b.x + wc * tr[t].c.x, wa * tr[t].a.y + wb * tr[t].b.y + wc * tr[t].c.y,
              wa * tr[t].a.z + wb * tr[t].b.z + wc * tr[t].c.z);
    v3 w = sub(s, o);
    double L = norm(w);
    v3 dv = scl(w, 1.0 / L);
    double ci = fabs(dot(tr[t].n, dv));
    int keep = ci >= cos_max;                                   /* incidence-angle constraint */
    int cert = fabs(ci - cos_max) > 1e-9;
    if (keep) {
      int blocked = any_hit(o, dv, tr, T, t, t_eps, L - t_eps); /* line of sight to the source */
      if (kappa > 0 && anyhit_marginal(o, dv, tr, T, t, t_eps, L - t_eps, kappa)) cert = 0;
      keep = !blocked;
    }
    samp_tri[k] = (int32_t)t;
    st3(samp_o + 3 * k, o);
    samp_r[k] = L;
    samp_keep[k] = (uint8_t)keep;
    if (samp_certified) samp_certified[k] = (uint8_t)cert;
  }
  free(lo); free(hi); free(oel); free(list); free(W); free(tr); free(gstart);
  return truncated;
}
