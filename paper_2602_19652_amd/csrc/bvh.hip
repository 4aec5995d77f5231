// Scene build on the device:
//  1. triangle boxes, centroid bounds, per-object boxes (field-of-view test of Sec. III-D)
//  2. 30-bit Morton codes of centroids, stable radix sort
//  3. agglomerative clustering over the Morton order (PLOC, Meister & Bittner 2018): each
//     cluster's nearest neighbour within a window is the one whose merged box has the
//     smallest surface area (the surface-area heuristic's cost driver); mutual nearest
//     neighbours merge; repeat until one cluster remains
//  4. packing into 64-byte binary traversal nodes, triangles repacked in leaf order
//  5. curvature metric C_i of Eq. (1) with the Meyer et al. cotangent operator, FP64
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace et {

namespace {

constexpr int BS = 256;

__device__ inline uint32_t f2o(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float o2f(uint32_t u) { return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u); }

__global__ void k_init_bounds(uint32_t* cb, uint32_t* ob, int32_t n_obj) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 6) cb[i] = (i < 3) ? 0xffffffffu : 0u;
  if (i < n_obj * 6) ob[i] = ((i % 6) < 3) ? 0xffffffffu : 0u;
}

// Triangle bounds (centroid bounds, object boxes) and the device checks of the mesh: vertex and
// object indices in range, finite vertex coordinates, materials >= 0 (their largest value goes
// to *mat_max when mat_max is not NULL, for the host's check against a pose's tables).
__global__ void k_tri_bounds(const float* __restrict__ V, const int32_t* __restrict__ tris,
                             const int32_t* __restrict__ obj, const int32_t* __restrict__ mat, int64_t T, int64_t nV,
                             int32_t n_obj, uint32_t* cb, uint32_t* ob, uint32_t* err, int32_t* mat_max) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float c[3] = {INFINITY, INFINITY, INFINITY};
  float cm[3] = {-INFINITY, -INFINITY, -INFINITY};
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int32_t key = -1;   // object of a valid triangle, else -1
  if (i < T && mat_max) {
    const int32_t q = mat[i];
    if (q < 0) atomicOr(err, DEV_ERR_INDEX);
    else atomicMax(mat_max, q);
  }
  if (i < T) {
    int32_t a = tris[3 * i], b = tris[3 * i + 1], cc = tris[3 * i + 2];
    int32_t o = obj[i];
    if (a < 0 || b < 0 || cc < 0 || a >= nV || b >= nV || cc >= nV || o < 0 || o >= n_obj) {
      atomicOr(err, DEV_ERR_INDEX);
    } else {
      key = o;
      bool finite = true;
      for (int k = 0; k < 3; ++k) {
        float x0 = V[3 * (int64_t)a + k], x1 = V[3 * (int64_t)b + k], x2 = V[3 * (int64_t)cc + k];
        finite = finite && isfinite(x0) && isfinite(x1) && isfinite(x2);
        lo[k] = fminf(x0, fminf(x1, x2));
        hi[k] = fmaxf(x0, fmaxf(x1, x2));
        c[k] = cm[k] = 0.5f * (lo[k] + hi[k]);
      }
      if (!finite) {   // a NaN or infinite coordinate: no box, and the call reports it
        atomicOr(err, DEV_ERR_VERTEX);
        key = -1;
        for (int k = 0; k < 3; ++k) {
          c[k] = lo[k] = INFINITY;
          cm[k] = hi[k] = -INFINITY;
        }
      }
    }
  }
  // Object boxes: triangles of an object are usually contiguous, so a wave whose lanes all
  // hold one object reduces its box first and issues 6 atomics instead of 6 per lane.
  const int32_t key0 = __shfl(key, 0);
  if (__all(key == key0) && key0 >= 0) {
    for (int k = 0; k < 3; ++k)
      for (int off = 32; off > 0; off >>= 1) {
        lo[k] = fminf(lo[k], __shfl_xor(lo[k], off));
        hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], off));
      }
    if ((threadIdx.x & 63) == 0)
      for (int k = 0; k < 3; ++k) {
        atomicMin(&ob[6 * key0 + k], f2o(lo[k]));
        atomicMax(&ob[6 * key0 + 3 + k], f2o(hi[k]));
      }
  } else if (key >= 0) {
    for (int k = 0; k < 3; ++k) {
      atomicMin(&ob[6 * key + k], f2o(lo[k]));
      atomicMax(&ob[6 * key + 3 + k], f2o(hi[k]));
    }
  }
  // block reduction of centroid bounds, one atomic per block and axis
  __shared__ float smin[3][BS], smax[3][BS];
  for (int k = 0; k < 3; ++k) { smin[k][threadIdx.x] = c[k]; smax[k][threadIdx.x] = cm[k]; }
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 3; ++k) {
        smin[k][threadIdx.x] = fminf(smin[k][threadIdx.x], smin[k][threadIdx.x + s]);
        smax[k][threadIdx.x] = fmaxf(smax[k][threadIdx.x], smax[k][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) {
      if (smin[k][0] <= smax[k][0]) {
        atomicMin(&cb[k], f2o(smin[k][0]));
        atomicMax(&cb[3 + k], f2o(smax[k][0]));
      }
    }
}

__device__ inline uint32_t spread10(uint32_t x) {
  x &= 0x3ffu;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

__global__ void k_morton(const float* __restrict__ V, const int32_t* __restrict__ tris, int64_t T,
                         const uint32_t* __restrict__ cb, uint32_t* __restrict__ keys, int32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  uint32_t q[3];
  for (int k = 0; k < 3; ++k) {
    float x0 = V[3 * (int64_t)tris[3 * i] + k], x1 = V[3 * (int64_t)tris[3 * i + 1] + k],
          x2 = V[3 * (int64_t)tris[3 * i + 2] + k];
    float c = 0.5f * (fminf(x0, fminf(x1, x2)) + fmaxf(x0, fmaxf(x1, x2)));
    float lo = o2f(cb[k]), hi = o2f(cb[3 + k]);
    float u = hi > lo ? (c - lo) / (hi - lo) : 0.5f;
    u = fminf(fmaxf(u, 0.f), 1.f);
    q[k] = (uint32_t)fminf(u * 1024.f, 1023.f);
  }
  keys[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
  vals[i] = (int32_t)i;
}

__global__ void k_leaves(const float* __restrict__ V, const int32_t* __restrict__ tris, const int32_t* __restrict__ mat,
                         const int32_t* __restrict__ perm, int64_t T, NodeB* __restrict__ nodes,
                         float4* __restrict__ tri4, int32_t* __restrict__ tri_orig, int32_t* __restrict__ tri_pos,
                         int32_t* __restrict__ clusters) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= T) return;
  int32_t t = perm[p];
  float v[3][3];
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < 3; ++k) v[c][k] = V[3 * (int64_t)tris[3 * (int64_t)t + c] + k];
  NodeB n;
  n.lox = fminf(v[0][0], fminf(v[1][0], v[2][0]));
  n.loy = fminf(v[0][1], fminf(v[1][1], v[2][1]));
  n.loz = fminf(v[0][2], fminf(v[1][2], v[2][2]));
  n.hix = fmaxf(v[0][0], fmaxf(v[1][0], v[2][0]));
  n.hiy = fmaxf(v[0][1], fmaxf(v[1][1], v[2][1]));
  n.hiz = fmaxf(v[0][2], fmaxf(v[1][2], v[2][2]));
  n.left = -1;
  n.right = -1;
  nodes[p] = n;
  tri4[3 * p + 0] = make_float4(v[0][0], v[0][1], v[0][2], __int_as_float(t));
  tri4[3 * p + 1] = make_float4(v[1][0], v[1][1], v[1][2], __int_as_float(mat[t]));
  tri4[3 * p + 2] = make_float4(v[2][0], v[2][1], v[2][2], 0.f);
  tri_orig[p] = t;
  tri_pos[t] = (int32_t)p;
  clusters[p] = (int32_t)p;
}

__device__ inline float merged_area(const float* a, const float* b) {
  float dx = fmaxf(a[3], b[3]) - fminf(a[0], b[0]);
  float dy = fmaxf(a[4], b[4]) - fminf(a[1], b[1]);
  float dz = fmaxf(a[5], b[5]) - fminf(a[2], b[2]);
  return dx * dy + dy * dz + dz * dx;   // half the surface area (constant factor is irrelevant)
}

__global__ void k_ploc_nn(const int32_t* __restrict__ cl, const int64_t* __restrict__ n_dev,
                          const NodeB* __restrict__ nodes, int32_t* __restrict__ nn) {
  constexpr int R = PLOC_RADIUS;
  __shared__ float box[BS + 2 * R][6];
  const int64_t n = *n_dev;
  const int64_t base = (int64_t)blockIdx.x * BS;
  if (base >= n) return;
  for (int k = threadIdx.x; k < BS + 2 * R; k += BS) {
    int64_t i = base - R + k;
    if (i >= 0 && i < n) {
      NodeB b = nodes[cl[i]];
      box[k][0] = b.lox; box[k][1] = b.loy; box[k][2] = b.loz;
      box[k][3] = b.hix; box[k][4] = b.hiy; box[k][5] = b.hiz;
    }
  }
  __syncthreads();
  const int64_t i = base + threadIdx.x;
  if (i >= n) return;
  float best = INFINITY;
  int64_t bj = -1;
  for (int d = -R; d <= R; ++d) {
    if (d == 0) continue;
    int64_t j = i + d;
    if (j < 0 || j >= n) continue;
    float a = merged_area(box[threadIdx.x + R], box[threadIdx.x + R + d]);
    if (a < best) { best = a; bj = j; }   // increasing j: ties keep the smaller index
  }
  nn[i] = (int32_t)bj;
}

__global__ void k_ploc_flags(const int32_t* __restrict__ nn, const int64_t* __restrict__ n_dev,
                             uint64_t* __restrict__ flags) {
  const int64_t n = *n_dev;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t j = nn[i];
  bool mutual = (j >= 0) && nn[j] == (int32_t)i;
  uint64_t survive = (mutual && j < i) ? 0u : 1u;
  uint64_t merge = (mutual && i < j) ? 1u : 0u;
  flags[i] = survive | (merge << 32);
}

__global__ void k_ploc_compact(const int32_t* __restrict__ cl, const int32_t* __restrict__ nn,
                               const uint64_t* __restrict__ flags, const uint64_t* __restrict__ offs,
                               int64_t* __restrict__ n_dev, const uint64_t* __restrict__ total,
                               int64_t* __restrict__ next_node, NodeB* __restrict__ nodes, int32_t* __restrict__ out) {
  const int64_t n = *n_dev;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    uint64_t f = flags[i];
    if (f & 0xffffffffu) {
      uint64_t o = offs[i];
      int64_t pos = (int64_t)(o & 0xffffffffu);
      if (f >> 32) {
        int32_t a = cl[i], b = cl[nn[i]];
        int64_t id = *next_node + (int64_t)(o >> 32);
        NodeB x = nodes[a], y = nodes[b];
        NodeB m;
        m.lox = fminf(x.lox, y.lox); m.loy = fminf(x.loy, y.loy); m.loz = fminf(x.loz, y.loz);
        m.hix = fmaxf(x.hix, y.hix); m.hiy = fmaxf(x.hiy, y.hiy); m.hiz = fmaxf(x.hiz, y.hiz);
        m.left = a;
        m.right = b;
        nodes[id] = m;
        out[pos] = (int32_t)id;
      } else {
        out[pos] = cl[i];
      }
    }
  }
}

// updates the counters after compaction (single thread, ordered after k_ploc_compact)
__global__ void k_ploc_update(int64_t* n_dev, const uint64_t* total, int64_t* next_node, int64_t* host_view) {
  uint64_t t = *total;
  *n_dev = (int64_t)(t & 0xffffffffu);
  *next_node += (int64_t)(t >> 32);
  host_view[0] = *n_dev;
  host_view[1] = *next_node;
}

__global__ void k_pack(const NodeB* __restrict__ nb, int64_t T, Node2* __restrict__ out, int32_t* __restrict__ leaf_parent) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T - 1) return;
  NodeB b = nb[T + k];
  NodeB c0 = nb[b.left], c1 = nb[b.right];
  Node2 n;
  n.xy0 = make_float4(c0.lox, c0.hix, c0.loy, c0.hiy);
  n.xy1 = make_float4(c1.lox, c1.hix, c1.loy, c1.hiy);
  n.zz = make_float4(c0.loz, c0.hiz, c1.loz, c1.hiz);
  int e0 = b.left >= T ? (int)(b.left - T) : ~b.left;
  int e1 = b.right >= T ? (int)(b.right - T) : ~b.right;
  n.ch = make_int4(e0, e1, -1, 0);
  out[k] = n;
  if (b.left < T) leaf_parent[b.left] = (int32_t)k;
  if (b.right < T) leaf_parent[b.right] = (int32_t)k;
}

__global__ void k_parents(Node2* __restrict__ nodes, int64_t n_inner) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_inner) return;
  int4 ch = nodes[k].ch;
  if (ch.x >= 0) nodes[ch.x].ch.z = (int)k;
  if (ch.y >= 0) nodes[ch.y].ch.z = (int)k;
}

__global__ void k_depth_sah(const Node2* __restrict__ nodes, const int32_t* __restrict__ leaf_parent, int64_t T,
                            const NodeB* __restrict__ nb, int root_id, int32_t* depth, double* sah) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= T) return;
  int d = 1;
  int node = leaf_parent[p];
  int guard = 0;
  while (node >= 0 && guard < 1 << 20) {
    ++d;
    node = nodes[node].ch.z;
    ++guard;
  }
  atomicMax(depth, d);
  NodeB r = nb[root_id];
  double ra = (double)(r.hix - r.lox) * (r.hiy - r.loy) + (double)(r.hiy - r.loy) * (r.hiz - r.loz) +
              (double)(r.hiz - r.loz) * (r.hix - r.lox);
  NodeB l = nb[p];
  double la = (double)(l.hix - l.lox) * (l.hiy - l.loy) + (double)(l.hiy - l.loy) * (l.hiz - l.loz) +
              (double)(l.hiz - l.loz) * (l.hix - l.lox);
  double s = ra > 0 ? la / ra : 0;
  if (p + 1 < T) {   // inner node T + p
    NodeB x = nb[T + p];
    double xa = (double)(x.hix - x.lox) * (x.hiy - x.loy) + (double)(x.hiy - x.loy) * (x.hiz - x.loz) +
                (double)(x.hiz - x.loz) * (x.hix - x.lox);
    s += ra > 0 ? xa / ra : 0;
  }
  atomicAdd(sah, s);
}

// ------------------------------------------------------------------ curvature (Eq. 1)
// The arithmetic below follows the paper's definition through the Meyer et al. operator
// with the operations in a fixed order and no contraction, so that C_i is reproducible
// to the last bit by any IEEE double implementation evaluating the same expressions.
#pragma clang fp contract(off)

__global__ void k_vcount(const int32_t* __restrict__ tris, int64_t T, uint64_t* __restrict__ cnt) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  for (int c = 0; c < 3; ++c) atomicAdd((unsigned long long*)&cnt[tris[3 * t + c]], 1ull);
}

// (vertex, triangle) pairs in triangle order; a stable sort by vertex leaves each vertex's
// triangles in ascending order, the order in which the operator below sums them.
__global__ void k_vkeys(const int32_t* __restrict__ tris, int64_t n3, uint32_t* __restrict__ key,
                        int32_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  key[i] = (uint32_t)tris[i];
  val[i] = (int32_t)(i / 3);
}

struct d3 { double x, y, z; };
__device__ inline d3 dsub(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline double ddot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline d3 dcross(d3 a, d3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline d3 dload(const float* V, int32_t i) {
  return {(double)V[3 * (int64_t)i], (double)V[3 * (int64_t)i + 1], (double)V[3 * (int64_t)i + 2]};
}

__global__ void k_vertex_curv(const float* __restrict__ V, const int32_t* __restrict__ tris,
                              const uint64_t* __restrict__ offs, const uint64_t* __restrict__ cnt,
                              const int32_t* __restrict__ adj, int64_t nV, double* __restrict__ G) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  double Kx = 0.0, Ky = 0.0, Kz = 0.0, Am = 0.0;
  const int64_t n = (int64_t)cnt[v];
  for (int64_t e = 0; e < n; ++e) {
    const int64_t t = adj[offs[v] + e];
    int32_t id[3] = {tris[3 * t], tris[3 * t + 1], tris[3 * t + 2]};
    d3 P[3] = {dload(V, id[0]), dload(V, id[1]), dload(V, id[2])};
    d3 cr = dcross(dsub(P[1], P[0]), dsub(P[2], P[0]));
    double area2 = sqrt(ddot(cr, cr));
    double area = 0.5 * area2;
    if (area < 1e-20) continue;
    double dotc[3], cot[3];
    for (int c = 0; c < 3; ++c) {
      dotc[c] = ddot(dsub(P[(c + 1) % 3], P[c]), dsub(P[(c + 2) % 3], P[c]));
      cot[c] = dotc[c] / area2;
    }
    bool obtuse = dotc[0] < 0.0 || dotc[1] < 0.0 || dotc[2] < 0.0;
    for (int c = 0; c < 3; ++c) {
      if (id[c] != (int32_t)v) continue;
      int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      d3 ea = dsub(P[c], P[c1]), eb = dsub(P[c], P[c2]);
      Kx += cot[c2] * ea.x + cot[c1] * eb.x;
      Ky += cot[c2] * ea.y + cot[c1] * eb.y;
      Kz += cot[c2] * ea.z + cot[c1] * eb.z;
      if (!obtuse) Am += (ddot(ea, ea) * cot[c2] + ddot(eb, eb) * cot[c1]) / 8.0;   // Voronoi region
      else if (dotc[c] < 0.0) Am += area / 2.0;
      else Am += area / 4.0;
    }
  }
  double kn = sqrt(Kx * Kx + Ky * Ky + Kz * Kz);
  G[v] = Am > 0.0 ? kn / (4.0 * Am) : 0.0;   // G = |K| / 2 with K = sum / (2 A_mixed)
}

__global__ void k_tri_curv(const float* __restrict__ V, const int32_t* __restrict__ tris, int64_t T,
                           const double* __restrict__ G, double a_ref, double* __restrict__ C) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double g0 = G[tris[3 * t]], g1 = G[tris[3 * t + 1]], g2 = G[tris[3 * t + 2]];
  double dG = fmax(g0, fmax(g1, g2)) - fmin(g0, fmin(g1, g2));
  d3 P0 = dload(V, tris[3 * t]), P1 = dload(V, tris[3 * t + 1]), P2 = dload(V, tris[3 * t + 2]);
  d3 cr = dcross(dsub(P1, P0), dsub(P2, P0));
  double area = 0.5 * sqrt(ddot(cr, cr));
  double w = a_ref > 0.0 ? fmin(1.0, area / a_ref) : 1.0;
  C[t] = w * dG;
}

#pragma clang fp contract(on)

__global__ void k_obj_box(const uint32_t* __restrict__ ob, int32_t n_obj, float* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_obj * 6) out[i] = o2f(ob[i]);
}

__global__ void k_single_leaf(Node2* nodes) {
  Node2 n;
  // child 0 is leaf 0 with an infinite box; child 1 is an empty box (never hit)
  n.xy0 = make_float4(-INFINITY, INFINITY, -INFINITY, INFINITY);
  n.xy1 = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
  n.zz = make_float4(-INFINITY, INFINITY, INFINITY, -INFINITY);
  n.ch = make_int4(~0, ~0, -1, 0);
  nodes[0] = n;
}

// ------------------------------------------------------------------ refit (dynamic scenes)
// Same topology, new vertex positions.  The build groups the inner nodes by depth; a refit
// rewrites the repacked triangles, then visits the levels from the deepest up, one launch per
// level: each node forms its two child boxes from its children (a leaf's triangle bounds, or
// the union of an inner child's two slots, final since the previous launch).  Every node
// writes only its own slots, so no thread waits on or fences against another, and every box
// is the exact union of its leaves' FP32 bounds, as the build produces it.

// Clears some bits of the deferred error word (the others keep what earlier calls reported).
__global__ void k_clear_bits(uint32_t* err, uint32_t bits) { atomicAnd(err, ~bits); }

__global__ void k_fill_u32(uint32_t* __restrict__ a, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void k_refit_leaves(const float* __restrict__ V, const int32_t* __restrict__ tris,
                               const int32_t* __restrict__ mat, const int32_t* __restrict__ tri_orig, int64_t T,
                               float4* __restrict__ tri4) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= T) return;
  const int32_t t = tri_orig[p];
  float v[3][3];
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < 3; ++k) v[c][k] = V[3 * (int64_t)tris[3 * (int64_t)t + c] + k];
  tri4[3 * p + 0] = make_float4(v[0][0], v[0][1], v[0][2], __int_as_float(t));
  tri4[3 * p + 1] = make_float4(v[1][0], v[1][1], v[1][2], __int_as_float(mat[t]));
  tri4[3 * p + 2] = make_float4(v[2][0], v[2][1], v[2][2], 0.f);
}

struct Box6 { float lx, hx, ly, hy, lz, hz; };

__device__ inline Box6 child_box(const Node2* nodes, const float4* __restrict__ tri4, int link) {
  if (link < 0) {
    const int64_t p = ~(int64_t)link;
    const float4 a = tri4[3 * p], b = tri4[3 * p + 1], c = tri4[3 * p + 2];
    return {fminf(a.x, fminf(b.x, c.x)), fmaxf(a.x, fmaxf(b.x, c.x)), fminf(a.y, fminf(b.y, c.y)),
            fmaxf(a.y, fmaxf(b.y, c.y)), fminf(a.z, fminf(b.z, c.z)), fmaxf(a.z, fmaxf(b.z, c.z))};
  }
  const Node2 m = nodes[link];
  return {fminf(m.xy0.x, m.xy1.x), fmaxf(m.xy0.y, m.xy1.y), fminf(m.xy0.z, m.xy1.z),
          fmaxf(m.xy0.w, m.xy1.w), fminf(m.zz.x, m.zz.z), fmaxf(m.zz.y, m.zz.w)};
}

__global__ void k_refit_level(const int32_t* __restrict__ level, int64_t n, const float4* __restrict__ tri4,
                              Node2* nodes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = level[i];
  const int4 ch = nodes[k].ch;
  const Box6 b0 = child_box(nodes, tri4, ch.x), b1 = child_box(nodes, tri4, ch.y);
  nodes[k].xy0 = make_float4(b0.lx, b0.hx, b0.ly, b0.hy);
  nodes[k].xy1 = make_float4(b1.lx, b1.hx, b1.ly, b1.hy);
  nodes[k].zz = make_float4(b0.lz, b0.hz, b1.lz, b1.hz);
}

// Depth of every inner node (root 0) by walking its parent links; histogram per depth.
template <int NL>
__global__ void k_node_depth(const Node2* __restrict__ nodes, int64_t n_inner, uint32_t* __restrict__ key,
                             int32_t* __restrict__ val, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[NL + 1];
  for (int i = threadIdx.x; i <= NL; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_inner) {
    int d = 0;
    for (int node = nodes[k].ch.z; node >= 0 && d < NL; node = nodes[node].ch.z) ++d;
    key[k] = (uint32_t)d;
    val[k] = (int32_t)k;
    atomicAdd(&h[d], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= NL; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// SAH cost of the refitted tree (C_node = C_tri = 1, normalised by the root area): the root
// contributes 1 and every other node its box area, read from its parent's child slot.
__device__ inline double slot_area(float lx, float hx, float ly, float hy, float lz, float hz) {
  return (double)(hx - lx) * (hy - ly) + (double)(hy - ly) * (hz - lz) + (double)(hz - lz) * (hx - lx);
}

__global__ void k_refit_sah(const Node2* __restrict__ nodes, int64_t n_inner, int root, double* sah) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Node2 r = nodes[root];
  const double ra = slot_area(fminf(r.xy0.x, r.xy1.x), fmaxf(r.xy0.y, r.xy1.y), fminf(r.xy0.z, r.xy1.z),
                              fmaxf(r.xy0.w, r.xy1.w), fminf(r.zz.x, r.zz.z), fmaxf(r.zz.y, r.zz.w));
  const Node2 n = nodes[k < n_inner ? k : root];
  double s = (k == root) ? 1.0 : 0.0;
  if (ra > 0 && k < n_inner)
    s += (slot_area(n.xy0.x, n.xy0.y, n.xy0.z, n.xy0.w, n.zz.x, n.zz.y) +
          slot_area(n.xy1.x, n.xy1.y, n.xy1.z, n.xy1.w, n.zz.z, n.zz.w)) / ra;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(sah, s);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + BS - 1) / BS > 0 ? (n + BS - 1) / BS : 1); }
inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

// [6] u32 centroid bounds, then a double at byte 64; zero between calls, so that a refit to
// the build's own vertices leaves the whole blob as the build left it
constexpr size_t REFIT_SCRATCH = 256;
constexpr int MAX_LEVEL = TRAV_STACK + 1;

size_t scene_blob_bytes(int64_t T, int64_t V, int32_t n_obj) {
  size_t b = 0;
  b += al(sizeof(Node2) * (size_t)std::max<int64_t>(1, T - 1));
  b += al(sizeof(float4) * 3 * (size_t)std::max<int64_t>(1, T));
  b += 2 * al(sizeof(int32_t) * (size_t)std::max<int64_t>(1, T));   // tri_orig, tri_pos
  b += al(sizeof(double) * (size_t)std::max<int64_t>(1, T));
  b += al(sizeof(double) * (size_t)std::max<int64_t>(1, V));
  b += al(sizeof(float) * 6 * (size_t)std::max<int32_t>(1, n_obj));
  // kept for refits: inner nodes by depth, vertex-triangle lists, refit scratch
  b += al(sizeof(int32_t) * (size_t)std::max<int64_t>(1, T - 1));
  b += 2 * al(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, V));
  b += al(sizeof(int32_t) * 3 * (size_t)std::max<int64_t>(1, T));
  b += al(REFIT_SCRATCH);
  return b;
}

size_t scene_scratch_bytes(int64_t T, int64_t V) {
  const int64_t Tm = std::max<int64_t>(T, 1), Vm = std::max<int64_t>(V, 1);
  size_t b = 0;
  b += al(sizeof(uint32_t) * 6) + al(sizeof(uint32_t) * 6 * 1);   // centroid bounds (object bounds sized below)
  b += al(sizeof(uint32_t) * Tm) + al(sizeof(int32_t) * Tm);       // morton keys / perm
  b += sort_temp_bytes(Tm, 4);
  b += al(sizeof(NodeB) * (size_t)(2 * Tm));                       // build nodes
  b += 2 * al(sizeof(int32_t) * Tm);                               // clusters ping-pong
  b += al(sizeof(int32_t) * Tm);                                   // nn
  b += 2 * al(sizeof(uint64_t) * Tm);                              // flags / offsets
  b += scan_temp_bytes(std::max(Tm, Vm));
  b += al(sizeof(int64_t) * 8) + al(sizeof(uint64_t) * 4);         // counters, totals
  b += al(sizeof(int32_t) * Tm);                                   // leaf parents
  b += al(sizeof(int32_t) * 2) + al(sizeof(double));               // depth, sah
  b += al(sizeof(uint32_t) * 3 * Tm) + sort_temp_bytes(3 * Tm, 4);  // vertex-triangle pair keys, sort
  b += al(sizeof(uint32_t) * (MAX_LEVEL + 1));                     // nodes per depth
  return b;
}

void scene_build(et_scene* sc, const et_mesh_desc* mesh, void* blob, void* scratch, uint32_t* dev_err, hipStream_t s) {
  const int64_t T = mesh->T, V = mesh->V;
  const int32_t n_obj = mesh->n_objects;
  SceneDev& d = sc->d;
  d.T = T; d.V = V; d.n_obj = n_obj;
  d.verts = mesh->vertices; d.tris = mesh->tris; d.mat = mesh->tri_material; d.obj = mesh->tri_object;
  // blob layout
  char* bp = (char*)blob;
  auto takeb = [&](size_t bytes) { char* p = bp; bp += al(bytes); return (void*)p; };
  d.nodes = (Node2*)takeb(sizeof(Node2) * (size_t)std::max<int64_t>(1, T - 1));
  d.tri4 = (float4*)takeb(sizeof(float4) * 3 * (size_t)std::max<int64_t>(1, T));
  d.tri_orig = (int32_t*)takeb(sizeof(int32_t) * (size_t)std::max<int64_t>(1, T));
  d.tri_pos = (int32_t*)takeb(sizeof(int32_t) * (size_t)std::max<int64_t>(1, T));
  d.C = (double*)takeb(sizeof(double) * (size_t)std::max<int64_t>(1, T));
  d.G = (double*)takeb(sizeof(double) * (size_t)std::max<int64_t>(1, V));
  d.obj_box = (float*)takeb(sizeof(float) * 6 * (size_t)std::max<int32_t>(1, n_obj));
  sc->lvl_nodes = (int32_t*)takeb(sizeof(int32_t) * (size_t)std::max<int64_t>(1, T - 1));
  sc->vcnt = (uint64_t*)takeb(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, V));
  sc->voff = (uint64_t*)takeb(sizeof(uint64_t) * (size_t)std::max<int64_t>(1, V));
  sc->adj = (int32_t*)takeb(sizeof(int32_t) * 3 * (size_t)std::max<int64_t>(1, T));
  sc->rscratch = takeb(REFIT_SCRATCH);
  // scratch layout
  const int64_t Tm = std::max<int64_t>(T, 1), Vm = std::max<int64_t>(V, 1);
  char* sp = (char*)scratch;
  auto take = [&](size_t bytes) { char* p = sp; sp += al(bytes); return (void*)p; };
  uint32_t* cb = (uint32_t*)take(sizeof(uint32_t) * 6);
  int32_t* mat_max = (int32_t*)take(sizeof(uint32_t) * 6);   // [0]: largest material index
  uint32_t* keys = (uint32_t*)take(sizeof(uint32_t) * Tm);
  int32_t* perm = (int32_t*)take(sizeof(int32_t) * Tm);
  void* sort_tmp = take(sort_temp_bytes(Tm, 4));
  NodeB* nb = (NodeB*)take(sizeof(NodeB) * (size_t)(2 * Tm));
  int32_t* clA = (int32_t*)take(sizeof(int32_t) * Tm);
  int32_t* clB = (int32_t*)take(sizeof(int32_t) * Tm);
  int32_t* nn = (int32_t*)take(sizeof(int32_t) * Tm);
  uint64_t* flags = (uint64_t*)take(sizeof(uint64_t) * Tm);
  uint64_t* offs = (uint64_t*)take(sizeof(uint64_t) * Tm);
  void* scan_tmp = take(scan_temp_bytes(std::max(Tm, Vm)));
  int64_t* ctr = (int64_t*)take(sizeof(int64_t) * 8);      // [0] n, [1] next node, [2..3] host view
  uint64_t* total = (uint64_t*)take(sizeof(uint64_t) * 4);
  int32_t* leaf_parent = (int32_t*)take(sizeof(int32_t) * Tm);
  int32_t* depth = (int32_t*)take(sizeof(int32_t) * 2);
  double* sah = (double*)take(sizeof(double));
  uint32_t* vkey = (uint32_t*)take(sizeof(uint32_t) * 3 * Tm);
  void* vsort_tmp = take(sort_temp_bytes(3 * Tm, 4));
  uint32_t* lvl_hist = (uint32_t*)take(sizeof(uint32_t) * (MAX_LEVEL + 1));
  uint64_t* vcnt = sc->vcnt;
  uint64_t* voff = sc->voff;
  int32_t* adj = sc->adj;
  // object boxes live in the blob as floats; build them as ordered uints in the blob memory
  uint32_t* ob = (uint32_t*)d.obj_box;

  hipEvent_t e0, e1;
  ET_HIP(hipEventCreate(&e0));
  ET_HIP(hipEventCreate(&e1));
  ET_HIP(hipEventRecord(e0, s));

  k_init_bounds<<<nblk(6 * (int64_t)std::max(n_obj, 1)), BS, 0, s>>>(cb, ob, n_obj);
  k_fill_u32<<<1, 1, 0, s>>>((uint32_t*)mat_max, 1, 0u);
  if (T > 0) {
    k_tri_bounds<<<nblk(T), BS, 0, s>>>(d.verts, d.tris, d.obj, d.mat, T, V, n_obj, cb, ob, dev_err, mat_max);
  }
  k_obj_box<<<nblk(6 * (int64_t)std::max(n_obj, 1)), BS, 0, s>>>(ob, n_obj, d.obj_box);
  ET_HIP(hipGetLastError());
  // the index check must pass before any kernel dereferences triangle indices
  uint32_t herr = 0;
  int32_t hmat = 0;
  ET_HIP(hipMemcpyAsync(&herr, dev_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  ET_HIP(hipMemcpyAsync(&hmat, mat_max, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  ET_HIP(hipStreamSynchronize(s));
  ET_CHECK(!(herr & DEV_ERR_INDEX), ET_E_INVALID,
           "mesh index out of range (triangle vertex or object index, or a negative material)");
  ET_CHECK(!(herr & DEV_ERR_VERTEX), ET_E_INVALID, "non-finite vertex coordinate in a triangle");
  sc->max_mat = T > 0 ? hmat : -1;

  int64_t h_ctr[2] = {0, 0};
  if (T >= 1) {
    k_morton<<<nblk(T), BS, 0, s>>>(d.verts, d.tris, T, cb, keys, perm);
    radix_sort_u32(keys, perm, T, 30, sort_tmp, s);
    k_leaves<<<nblk(T), BS, 0, s>>>(d.verts, d.tris, d.mat, perm, T, nb, d.tri4, d.tri_orig, d.tri_pos, clA);
    ET_HIP(hipGetLastError());
  }
  int root_id = 0;
  if (T >= 2) {
    // agglomerative clustering; the cluster count lives on the device, the host reads it
    // once per iteration to decide whether to continue
    h_ctr[0] = T;
    h_ctr[1] = T;
    ET_HIP(hipMemcpyAsync(ctr, h_ctr, sizeof(int64_t) * 2, hipMemcpyHostToDevice, s));
    int64_t n = T;
    int iter = 0;
    int32_t* cin = clA;
    int32_t* cout = clB;
    while (n > 1) {
      ET_CHECK(++iter < 100000, ET_E_INTERNAL, "BVH clustering did not converge");
      k_ploc_nn<<<nblk(n), BS, 0, s>>>(cin, ctr, nb, nn);
      k_ploc_flags<<<nblk(n), BS, 0, s>>>(nn, ctr, flags);
      scan_exclusive_u64(flags, offs, n, nullptr, n, total, scan_tmp, s);
      k_ploc_compact<<<nblk(n), BS, 0, s>>>(cin, nn, flags, offs, ctr, total, ctr + 1, nb, cout);
      k_ploc_update<<<1, 1, 0, s>>>(ctr, total, ctr + 1, ctr + 2);
      ET_HIP(hipGetLastError());
      int64_t hv[2];
      ET_HIP(hipMemcpyAsync(hv, ctr + 2, sizeof(int64_t) * 2, hipMemcpyDeviceToHost, s));
      ET_HIP(hipStreamSynchronize(s));
      ET_CHECK(hv[0] < n && hv[0] >= 1, ET_E_INTERNAL, "BVH clustering made no progress");
      n = hv[0];
      std::swap(cin, cout);
      h_ctr[1] = hv[1];
    }
    ET_CHECK(h_ctr[1] == 2 * T - 1, ET_E_INTERNAL, "BVH node count mismatch");
    root_id = (int)(2 * T - 2);
    k_pack<<<nblk(T - 1), BS, 0, s>>>(nb, T, d.nodes, leaf_parent);
    k_parents<<<nblk(T - 1), BS, 0, s>>>(d.nodes, T - 1);
    ET_HIP(hipMemsetAsync(depth, 0, sizeof(int32_t), s));
    ET_HIP(hipMemsetAsync(sah, 0, sizeof(double), s));
    k_depth_sah<<<nblk(T), BS, 0, s>>>(d.nodes, leaf_parent, T, nb, root_id, depth, sah);
    // inner nodes grouped by depth for refits (stable sort: the order is deterministic)
    k_fill_u32<<<1, BS, 0, s>>>(lvl_hist, MAX_LEVEL + 1, 0u);
    k_node_depth<MAX_LEVEL><<<nblk(T - 1), BS, 0, s>>>(d.nodes, T - 1, keys, sc->lvl_nodes, lvl_hist);
    radix_sort_u32(keys, sc->lvl_nodes, T - 1, 7, sort_tmp, s);
    ET_HIP(hipGetLastError());
    d.root = (int)(T - 2);   // the last node created is the root; packed index = id - T
    sc->n_nodes = T - 1;
  } else {
    k_single_leaf<<<1, 1, 0, s>>>(d.nodes);
    d.root = 0;
    sc->n_nodes = 1;
  }

  k_fill_u32<<<1, BS, 0, s>>>((uint32_t*)sc->rscratch, REFIT_SCRATCH / 4, 0u);
  // curvature (Eq. 1)
  if (T > 0 && V > 0) {
    k_fill_u32<<<nblk(2 * V), BS, 0, s>>>((uint32_t*)vcnt, 2 * V, 0u);
    k_vcount<<<nblk(T), BS, 0, s>>>(d.tris, T, vcnt);
    scan_exclusive_u64(vcnt, voff, V, nullptr, V, nullptr, scan_tmp, s);
    k_vkeys<<<nblk(3 * T), BS, 0, s>>>(d.tris, 3 * T, vkey, adj);
    int vbits = 1;
    while (vbits < 32 && ((int64_t)1 << vbits) < V) ++vbits;
    radix_sort_u32(vkey, adj, 3 * T, vbits, vsort_tmp, s);
    k_vertex_curv<<<nblk(V), BS, 0, s>>>(d.verts, d.tris, voff, vcnt, adj, V, d.G);
    k_tri_curv<<<nblk(T), BS, 0, s>>>(d.verts, d.tris, T, d.G, mesh->area_ref, d.C);
    ET_HIP(hipGetLastError());
  }
  ET_HIP(hipEventRecord(e1, s));
  ET_HIP(hipEventSynchronize(e1));
  float ms = 0;
  ET_HIP(hipEventElapsedTime(&ms, e0, e1));
  sc->build_ms = ms;
  ET_HIP(hipEventDestroy(e0));
  ET_HIP(hipEventDestroy(e1));
  if (T >= 2) {
    int32_t hd = 0;
    double hs = 0;
    ET_HIP(hipMemcpy(&hd, depth, sizeof(int32_t), hipMemcpyDeviceToHost));
    ET_HIP(hipMemcpy(&hs, sah, sizeof(double), hipMemcpyDeviceToHost));
    sc->depth = hd;
    sc->sah = hs;
    std::vector<uint32_t> hist(MAX_LEVEL + 1);
    ET_HIP(hipMemcpy(hist.data(), lvl_hist, sizeof(uint32_t) * hist.size(), hipMemcpyDeviceToHost));
    int levels = MAX_LEVEL + 1;
    while (levels > 0 && hist[levels - 1] == 0) --levels;
    sc->lvl_off.assign(1, 0);
    for (int l = 0; l < levels; ++l) sc->lvl_off.push_back(sc->lvl_off.back() + hist[l]);
    ET_CHECK(sc->lvl_off.back() == T - 1, ET_E_INTERNAL, "BVH level grouping lost nodes");
  } else {
    sc->depth = T;
    sc->sah = T;
  }
  ET_CHECK(sc->depth <= TRAV_STACK, ET_E_UNSUPPORTED, "BVH deeper than the traversal stack");
}

}  // namespace et

namespace et {

void scene_refit(et_scene* sc, const float* vertices, double area_ref, uint32_t* dev_err, hipStream_t s) {
  SceneDev& d = sc->d;
  const int64_t T = d.T, V = d.V;
  const int32_t n_obj = d.n_obj;
  d.verts = vertices;
  uint32_t* cb = (uint32_t*)sc->rscratch;
  double* sah = (double*)((char*)sc->rscratch + 64);
  uint32_t* ob = (uint32_t*)d.obj_box;
  hipEvent_t e0, e1;
  ET_HIP(hipEventCreate(&e0));
  ET_HIP(hipEventCreate(&e1));
  ET_HIP(hipEventRecord(e0, s));
  k_clear_bits<<<1, 1, 0, s>>>(dev_err, DEV_ERR_VERTEX);
  k_init_bounds<<<nblk(6 * (int64_t)std::max(n_obj, 1)), BS, 0, s>>>(cb, ob, n_obj);
  if (T > 0) k_tri_bounds<<<nblk(T), BS, 0, s>>>(d.verts, d.tris, d.obj, d.mat, T, V, n_obj, cb, ob, dev_err, nullptr);
  k_obj_box<<<nblk(6 * (int64_t)std::max(n_obj, 1)), BS, 0, s>>>(ob, n_obj, d.obj_box);
  if (T > 0) k_refit_leaves<<<nblk(T), BS, 0, s>>>(d.verts, d.tris, d.mat, d.tri_orig, T, d.tri4);
  if (T >= 2) {
    for (int l = (int)sc->lvl_off.size() - 2; l >= 0; --l) {
      const int64_t a = sc->lvl_off[l], n = sc->lvl_off[l + 1] - a;
      k_refit_level<<<nblk(n), BS, 0, s>>>(sc->lvl_nodes + a, n, d.tri4, d.nodes);
    }
    k_fill_u32<<<1, BS, 0, s>>>((uint32_t*)sah, 2, 0u);
    k_refit_sah<<<nblk(T - 1), BS, 0, s>>>(d.nodes, T - 1, d.root, sah);
  }
  if (T > 0 && V > 0) {   // the vertex-triangle lists depend on the topology only
    k_vertex_curv<<<nblk(V), BS, 0, s>>>(d.verts, d.tris, sc->voff, sc->vcnt, sc->adj, V, d.G);
    k_tri_curv<<<nblk(T), BS, 0, s>>>(d.verts, d.tris, T, d.G, area_ref, d.C);
  }
  ET_HIP(hipGetLastError());
  ET_HIP(hipEventRecord(e1, s));
  ET_HIP(hipEventSynchronize(e1));
  float ms = 0;
  ET_HIP(hipEventElapsedTime(&ms, e0, e1));
  sc->refit_ms = ms;
  ET_HIP(hipEventDestroy(e0));
  ET_HIP(hipEventDestroy(e1));
  if (T >= 2) ET_HIP(hipMemcpyAsync(&sc->sah, sah, sizeof(double), hipMemcpyDeviceToHost, s));
  k_fill_u32<<<1, BS, 0, s>>>((uint32_t*)sc->rscratch, REFIT_SCRATCH / 4, 0u);
  ET_HIP(hipGetLastError());
  uint32_t herr = 0;
  ET_HIP(hipMemcpyAsync(&herr, dev_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  k_clear_bits<<<1, 1, 0, s>>>(dev_err, DEV_ERR_VERTEX);   // reported by this call's status only
  ET_HIP(hipGetLastError());
  ET_HIP(hipStreamSynchronize(s));
  ET_CHECK(!(herr & DEV_ERR_VERTEX), ET_E_INVALID,
           "non-finite vertex coordinate in a triangle (refit again with finite vertices before tracing)");
}

}  // namespace et
