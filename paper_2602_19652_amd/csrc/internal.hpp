// Internal declarations shared by the HIP translation units of the echotrace library.
// Not part of the ABI (include/echotrace.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/echotrace.h"

namespace et {

// ------------------------------------------------------------------ errors

struct Error {
  int code;
  std::string msg;
};

#define ET_HIP(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::et::Error{ET_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define ET_CHECK(cond, code, msg)                          \
  do {                                                     \
    if (!(cond)) throw ::et::Error{(code), std::string(msg)}; \
  } while (0)

// deferred device-side error bits (et_stats.status)
enum : uint32_t {
  DEV_ERR_INDEX = 1u << 0,      // triangle index out of range
  DEV_ERR_STACK = 1u << 1,      // traversal stack overflow
  DEV_ERR_CAPACITY = 1u << 2,   // record capacity exceeded
  DEV_ERR_RAYDIR = 1u << 3,     // zero / non-finite ray direction
  DEV_ERR_BUILD = 1u << 4,      // BVH build invariant broken
  DEV_ERR_VERTEX = 1u << 5,     // non-finite coordinate of a vertex that a triangle uses
};

// ------------------------------------------------------------------ BVH layout

// Traversal node of the binary BVH (64 bytes, one cache line pair): the two child boxes
// stored side by side so that one node fetch tests both children.
struct __align__(16) Node2 {
  float4 xy0;  // child 0: lo.x hi.x lo.y hi.y
  float4 xy1;  // child 1: lo.x hi.x lo.y hi.y
  float4 zz;   // child 0 lo.z hi.z, child 1 lo.z hi.z
  int4 ch;     // child 0, child 1 (>= 0 inner node, < 0 leaf ~position), parent, unused
};

// Build-time node: box + children (leaves 0..T-1 are triangles in Morton order,
// inner nodes T..2T-2 are created by the agglomerative clustering).
struct __align__(16) NodeB {
  float lox, loy, loz;
  int left;
  float hix, hiy, hiz;
  int right;
};

// per-lane stack entries held in LDS: 26 KB per 256-thread block, so six blocks (six waves
// per SIMD) fit the compute unit's 160 KB
constexpr int TRAV_LDS_STACK = 26;
constexpr int TRAV_WAVES_PER_SIMD = 6;
constexpr int TRAV_STACK = 64;         // total per-lane entries (rest in global memory)
constexpr int TRAV_BLOCK = 256;
constexpr int PLOC_RADIUS = 16;

struct SceneDev {
  int64_t T = 0, V = 0;
  int32_t n_obj = 0;
  const float* verts = nullptr;
  const int32_t* tris = nullptr;
  const int32_t* mat = nullptr;
  const int32_t* obj = nullptr;
  Node2* nodes = nullptr;       // [max(1, T-1)]
  float4* tri4 = nullptr;       // [T][3]: v0 (w = original index bits), v1 (w = material bits), v2
  int32_t* tri_orig = nullptr;  // [T] original triangle index per leaf position
  int32_t* tri_pos = nullptr;   // [T] leaf position per original triangle index
  double* C = nullptr;          // [T] curvature metric per original triangle
  double* G = nullptr;          // [V] per-vertex mean curvature magnitude
  float* obj_box = nullptr;     // [n_obj][6] lo xyz, hi xyz
  int root = 0;                 // root node index (T == 1: node 0 with a single leaf)
};

}  // namespace et

struct et_scene {
  et::SceneDev d;
  int64_t n_nodes = 0;
  int32_t depth = 0;
  double sah = 0;
  double build_ms = 0;
  double refit_ms = 0;
  int device = 0;
  int32_t max_mat = -1;            // largest material index of the mesh (-1: no triangles)
  // what a refit reads besides the tree (device arrays in the blob; level offsets on the host)
  int32_t* lvl_nodes = nullptr;    // [T-1] inner nodes grouped by depth, root first
  std::vector<int64_t> lvl_off;    // [levels + 1] start of each depth in lvl_nodes
  uint64_t* vcnt = nullptr;        // [V] triangles around each vertex
  uint64_t* voff = nullptr;        // [V] start of each vertex's list in adj
  int32_t* adj = nullptr;          // [3T] triangles around each vertex, ascending
  void* rscratch = nullptr;        // refit scratch: centroid bounds, SAH accumulator
};

namespace et {

// ------------------------------------------------------------------ device prims (prims.hip)

// Exclusive scan of n elements (n read from device memory if n_dev != nullptr, else n_host).
// temp must hold scan_temp_bytes(n_max) bytes.  total (device, optional) receives the sum.
size_t scan_temp_bytes(int64_t n_max);
void scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n_host, const int64_t* n_dev, int64_t n_max,
                        uint64_t* total, void* temp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the key.
size_t sort_temp_bytes(int64_t n, int key_bytes);
void radix_sort_u32(uint32_t* keys, int32_t* vals, int64_t n, int bits, void* temp, hipStream_t s);
void radix_sort_u64(uint64_t* keys, int32_t* vals, int64_t n_host, const int64_t* n_dev, int64_t n_max, int bits,
                    void* temp, hipStream_t s);

// ------------------------------------------------------------------ scene build (bvh.hip)
size_t scene_blob_bytes(int64_t T, int64_t V, int32_t n_obj);
size_t scene_scratch_bytes(int64_t T, int64_t V);
// Builds the BVH and curvature; returns host-side info.  Throws et::Error.
void scene_build(et_scene* sc, const et_mesh_desc* mesh, void* blob, void* scratch, uint32_t* dev_err,
                 hipStream_t s);
// New vertex positions, same topology: BVH refit (structure kept, boxes recomputed bottom-up),
// triangle repack, object boxes and curvature.  Throws et::Error.
void scene_refit(et_scene* sc, const float* vertices, double area_ref, uint32_t* dev_err,
                 hipStream_t s);

}  // namespace et

namespace et {

// ------------------------------------------------------------------ per-context control block
// A small device struct (one per context) holding counters that kernels update and later
// kernels read, so that no phase needs a host round trip.
struct Ctl {
  uint32_t err;              // DEV_ERR_* bits
  uint32_t pad0;
  int64_t n_active[2];       // active rays of the current / next bounce
  int64_t rec_base;          // specular records produced so far (may exceed capacity)
  int64_t rec_prev;          // specular records of the earlier job waves of a batch
  int64_t seg;               // closest-hit segments traced
  int64_t shadow;            // line-of-sight rays traced
  int64_t overflow;          // traversal stack overflows
  uint64_t tot[4];           // scan totals
  uint64_t cmax_bits;        // max C_i over eligible objects (bit pattern of a non-negative double)
  int64_t n_elig;            // triangles in the diffraction CDF
  int64_t diff_kept;         // kept diffraction samples
  int64_t cnt[6];            // traversal work counters (nodes/tris closest, nodes/tris any, rays c/a)
  int64_t n_rec;             // records to synthesise
  int64_t n_vis;             // of which visible (compacted index list)
  int64_t n_groups;          // diffraction CDF groups (1, or the meshes with eligible triangles)
  int64_t n_draw;            // diffraction draws (K, or K per mesh)
};

struct TraceWS {
  // ray state ping-pong (FP64 origin/direction, path length, previous leaf position, ray id)
  double* st[2][7];
  int32_t* prev[2];
  int32_t* ray[2];
  int64_t* prec[2];          // record index of the ray's previous reflection (-1 before the first)
  // per-slot bounce results
  double* rp[3];
  double* rd[3];
  double* rr;
  int32_t* rpos;
  uint64_t* rvis;            // line of sight: 0/1, or receiver bits (per-receiver reading)
  uint64_t* flags;
  uint64_t* offs;
  void* scan_tmp;
  uint32_t* rkeys;           // ray order: direction keys (job in the high bits in a batch)
  int32_t* rperm;            // ray index per slot after sorting by key
  void* rsort_tmp;
  int32_t* gstack;           // global part of the traversal stacks
  int64_t gstack_threads;
  int32_t stack_cap;         // per-lane stack entries in use (TRAV_STACK; lower only to test overflows)
  // diffraction
  uint8_t* oel;
  uint64_t* dkeys;
  int32_t* dvals;
  uint64_t* dq;
  uint64_t* dflags;
  uint64_t* doffs;
  void* sort_tmp;
  int32_t* stri;
  double* so;
  double* sr;
  uint64_t* skeep;
  uint64_t* soffs;
  uint64_t* goffs;    // [T] group ranks (per-mesh CDFs)
  int64_t* gstart;    // [T + 1] first sorted position of each group
};

// Workspace layout of et_trace.  base == nullptr: only computes the size.
// max_blocks: largest bounce-kernel grid the workspace serves (0: the single-pose default)
size_t trace_ws_layout(int64_t N, int64_t T, int32_t n_obj, int64_t K, char* base, TraceWS* ws,
                       int32_t max_blocks = 0);
// Fused batch (specular jobs): all jobs' rays share the bounce kernels; records carry the
// job index in their ray field.  dev_jobs holds trace_batch_jobs_bytes(J) bytes.
size_t trace_batch_jobs_bytes(int32_t J);
int64_t trace_batch_rays(int32_t J, const et_job* jobs);
// carry: a later job wave of one batch (segment, line-of-sight and record totals carry over)
void trace_batch_run(int32_t J, const et_job* jobs, void* dev_jobs, const et_paths* paths, const TraceWS& w,
                     Ctl* ctl, bool counting, int32_t blocks, hipStream_t s, bool carry = false);
void trace_run(const SceneDev& S, const et_sim_desc* sim, const et_paths* paths, const TraceWS& ws, Ctl* ctl,
               bool counting, hipStream_t s);

// ------------------------------------------------------------------ synthesis (synth.hip)
struct SynthWS {
  float* partial;            // [P][M][F][2]
  int32_t P;
  double* gpart_x;           // [chunks][tiles][M][3]
  double* gpart_k;           // [chunks][tiles][M][Q][Bk]
  int32_t gchunks;           // adjoint record chunks
  int32_t gtiles;            // adjoint tiles of outer indices (factorised kernel)
  int64_t cap;               // record capacity
  uint64_t* vflags;          // visible-record compaction: flags, offsets, index list, scan scratch
  uint64_t* voffs;
  int32_t* vidx;
  void* vscan;
  float* lk;                 // per (material, band): log2 k, log2(e)/(2 beta^2), log2 I_d
  float* lc;
  float* ld;
  float* lp;                 // [Bk] log2 I_p (passive component)
  float* lmax;               // [3 Q + 1] per material: max log2 k, min lobe coefficient, max log2 I_d; max log2 I_p
  float* plk;                // [cap][Bk] path-product reading: log2 k over each record's path (or log2 I_d)
  float* plc;                // [cap][Bk] path-product reading: each record's lobe coefficient
};
size_t synth_ws_layout(const et_sim_desc* sim, int64_t cap, char* base, SynthWS* ws);
// returns 1 for the factorised MFMA kernel, 2 for the direct kernel
// kb/ke (optional) are recorded around the main synthesis kernel alone
int synth_run(const et_sim_desc* sim, const et_paths* paths, const SynthWS& ws, Ctl* ctl, float* spectra,
              hipStream_t s, hipEvent_t kb = nullptr, hipEvent_t ke = nullptr);
size_t synth_bwd_ws_layout(const et_sim_desc* sim, int64_t cap, char* base, SynthWS* ws);
// returns 1 (factorised MFMA adjoint) or 2 (direct adjoint)
int synth_bwd_run(const et_sim_desc* sim, const et_paths* paths, const float* grad_spectra, const SynthWS& ws,
                  Ctl* ctl, double* grad_k, double* grad_rx, hipStream_t s, hipEvent_t kb = nullptr,
                  hipEvent_t ke = nullptr);
bool synth_factorised_ok(const et_sim_desc* sim);
bool synth_bwd_factorised_ok(const et_sim_desc* sim);

// Synthesis without a workspace (et_synthesize_noalloc): band tables and partial spectra in
// `buf` (bytes), every record walked (no visible-record list).  Throws ET_E_UNSUPPORTED when the
// tables and one record chunk's partial spectra do not fit.
int synth_run_noalloc(const et_sim_desc* sim, const et_paths* paths, void* buf, size_t bytes, Ctl* ctl,
                      float* spectra, hipStream_t s, hipEvent_t kb = nullptr, hipEvent_t ke = nullptr);

// ------------------------------------------------------------------ device scratch (noalloc.hip)
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
// Takes the scratch array's address on `device` (current) once; called at context creation.
void noalloc_init(int device);
// The scratch address on `device` (noalloc_init must have run there).
void* noalloc_scratch(int device);

// ------------------------------------------------------------------ time domain (timedomain.hip)
// out[i] = sum over j < J (in order) of in[j][i], i < n (synth.hip)
void sum_spectra(const float* in, int32_t J, int64_t n, float* out, hipStream_t s);

// ------------------------------------------------------------------ EQ ray sets (eq.hip)

struct EqPlan {
  int64_t N = 0, n = 0;       // regions, collars
  double theta_c = 0, delta = 0;   // polar cap colatitude, collar height
};
EqPlan eq_plan(int64_t N);
size_t eq_ws_bytes(const EqPlan& p);
// Builds the collar table in ws and returns the number of region centres within the cone
// (synchronises the stream).
int64_t eq_count(const EqPlan& p, double half_angle, void* ws, hipStream_t s);
void eq_points(const EqPlan& p, int64_t count, void* ws, float* dirs, hipStream_t s);

int64_t conv_length(int64_t n_t, int64_t L);
size_t impulse_ws_bytes(int64_t M, int64_t n_t);
size_t signal_ws_bytes(int64_t M, int64_t n_t, int64_t L);
void impulse_run(int64_t M, int64_t F, double f_lo, double df, int sigma, const float* spectra, int64_t n_t, void* ws,
                 float* h, hipStream_t s);
void signal_run(int64_t M, int64_t n_t, const float* h, int64_t L, const float* se, double dt, void* ws, float* out,
                hipStream_t s);

// Launch shapes of the fused batch (the autotuner's knobs): workgroups of the main synthesis
// and adjoint kernels the record chunks aim at.
struct BatchTune {
  int32_t synth_wgs = 4096;       // (the autotuner's choice for the 320-job batch of 2048-bin jobs)
  int32_t adjoint_wgs = 4096;
  int32_t trace_blocks = 4096;    // grid of the bounce kernels (grid-stride over the active rays)
  int64_t wave_rays = 1ll << 23;  // rays of a job wave: jobs run in waves whose rays add up to this
};
constexpr int64_t MIN_WAVE_RAYS = 1024;
// Largest values the autotuner tries; workspaces are sized for them.
constexpr int32_t TUNE_MAX_WGS = 16384;
constexpr int32_t TUNE_MAX_TRACE_BLOCKS = 8192;

// Fused batch synthesis: the visible records of all jobs, sorted by job, in chunks that never
// mix jobs; one launch of the synthesis (and adjoint) kernel for the whole batch.
struct SynthBatchWS {
  int32_t J;
  int64_t cap;
  bool mf, mf_bwd;
  int fold;    // 8 / 4: every band edge on a multiple of 512 / 256 bins, and the bins, in every job; else 0
  int32_t target, target_bwd;   // chunk count the batch aims at
  int32_t chunks, chunks_bwd;   // grid size: target + J bounds the chunk count
  int32_t T1;                   // adjoint tiles of outer indices
  float* partial;               // [chunks][M][F][2]
  double* gpart_x;              // [chunks][T1][M][3]
  double* gpart_k;              // [chunks][T1][M][Q][Bk]
  uint64_t* vflags;
  uint64_t* voffs;
  int32_t* vidx;
  void* vscan;
  uint64_t* keys;               // job of each visible record (sort keys)
  void* sort_tmp;
  int64_t* tab;                 // chunk tables (forward, adjoint)
  void* jobs;                   // device job table
  float* tables;                // [J][4 Q Bk + 3 Q + 1] band tables and their per-material bounds
};
bool synth_batch_factorised(int32_t J, const et_job* jobs, bool adjoint);
size_t synth_batch_ws_layout(int32_t J, const et_job* jobs, int64_t cap, const BatchTune& tune, bool adjoint,
                             char* base, SynthBatchWS* ws);
// returns the forward kernel (1 MFMA, 2 direct); *adjoint_kernel likewise when grad != nullptr
// ev (optional): 4 events recorded around the synthesis kernel and the adjoint kernel
int synth_batch_run(int32_t J, const et_job* jobs, const et_paths* paths, const SynthBatchWS& w, Ctl* ctl,
                    float* spectra, const float* grad, double* grad_k, double* grad_rx, int* adjoint_kernel,
                    const hipEvent_t* ev, hipStream_t s);

}  // namespace et
