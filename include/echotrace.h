/*
 * echotrace.h -- C ABI of the MI355X (gfx950) echo-simulation hot path.
 *
 * Computes what the SonoTraceUE paper (Jansen & Steckel, arXiv 2602.19652) computes per
 * frame: rays emitted from a sensor pose are traced through a triangle-mesh scene with
 * specular bounces (Sec. III-C, Algorithm 1), curvature-importance Monte Carlo
 * diffraction points are drawn (Sec. III-D), the direct emitter-receiver paths of the
 * passive component are tested (Sec. III-E), and every path becomes a complex
 * contribution to each receiver's transfer function (Eqs. 2-4 specular, 7-8 diffraction,
 * 11-13 passive).  Scene in, per-receiver spectra out; then impulse responses and received
 * signals (Sec. III-F).  Around that: batches of poses and scenes, several emitters, the
 * adjoint of the synthesis, equal-area ray sets and BVH refits for dynamic scenes.
 *
 * Conventions
 *  - Every call returns an int status (et_status); no exception crosses the ABI.
 *    et_last_error() gives a message for the last failing call on a context.
 *  - Pointers documented as "device" are HIP device pointers (e.g. torch CUDA tensors on
 *    ROCm); "host" pointers are read during the call only.  The caller owns every buffer:
 *    scene blob, scratch, workspace, inputs and outputs.  Apart from two small control
 *    blocks per context (counters and error word, allocated by et_create, freed by
 *    et_destroy) the library allocates no device memory.
 *  - Calls enqueue work on the context's stream and return; outputs are valid once the
 *    stream has completed the work (the Python binding uses torch's current stream).
 *    et_get_stats() synchronises the stream.  A fused batch of several job waves also uses a
 *    second stream of the context's own (default priority, created by the first such call,
 *    destroyed by et_destroy), forked from and joined back into the context's stream within
 *    the call.
 *  - A context is used by one host thread at a time.  Scenes are immutable after build
 *    and may be shared by contexts on the same device.
 *  - Host-side validation (shapes, null pointers, ranges of scalar parameters) runs
 *    before any launch; array contents on the device are trusted, except that the mesh is
 *    checked on the device during scene build (vertex and object indices in range, materials
 *    >= 0, finite coordinates of the vertices that triangles use; otherwise ET_E_INVALID) and
 *    a trace refuses a pose whose band tables have fewer rows (Q) than the scene's largest
 *    material index needs (ET_E_INVALID).
 *  - Angles are radians, lengths metres, frequencies Hz.  Rotation matrices are 3x3
 *    row-major, their columns are the local axes expressed in world coordinates
 *    (world = R * local).
 */
#ifndef ECHOTRACE_H
#define ECHOTRACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ET_ABI_VERSION 4

typedef enum {
  ET_OK = 0,
  ET_E_INVALID = -1,     /* bad argument: null pointer, shape, range, NaN pose */
  ET_E_WORKSPACE = -2,   /* caller buffer smaller than the queried size */
  ET_E_CAPACITY = -3,    /* path buffer too small for the records produced (true count in stats) */
  ET_E_DEVICE = -4,      /* HIP runtime error */
  ET_E_UNSUPPORTED = -5, /* valid request outside what the library implements */
  ET_E_INTERNAL = -6     /* device-side invariant broken (e.g. traversal stack overflow) */
} et_status;

typedef struct et_ctx et_ctx;
typedef struct et_scene et_scene;

int et_abi_version(void);
const char* et_status_string(int status);

/* Context bound to a HIP device and stream (stream may be NULL: the null stream). */
int et_create(int device, void* hip_stream, et_ctx** out);
int et_destroy(et_ctx* ctx);
int et_set_stream(et_ctx* ctx, void* hip_stream);
const char* et_last_error(const et_ctx* ctx);

/* ------------------------------------------------------------------ scene (Sec. III-B)
 * Scene mesh: world-space triangles welded per object, with a material (acoustic
 * profile) per triangle (per-object granularity, Sec. III-B) and an object id used by
 * the emitter field-of-view test of the diffraction sampler (Sec. III-D). */
typedef struct {
  int64_t V, T;
  const float* vertices;        /* device [V][3] */
  const int32_t* tris;          /* device [T][3], indices in [0, V) */
  const int32_t* tri_material;  /* device [T], in [0, Q) of the simulation tables */
  const int32_t* tri_object;    /* device [T], in [0, n_objects) */
  int32_t n_objects;
  double area_ref;              /* reference area of the curvature metric's area weight
                                   w(A) = min(1, A / area_ref), Eq. (1); <= 0 gives w = 1 */
} et_mesh_desc;

/* Byte sizes of the scene blob (kept for the scene's lifetime: BVH nodes, repacked
 * triangles, curvature C_i, object boxes, and what et_scene_refit reads) and of the build
 * scratch (free after build). */
int et_scene_size(et_ctx* ctx, const et_mesh_desc* mesh, size_t* blob_bytes, size_t* scratch_bytes);

/* Builds the device acceleration structure (surface-area-driven agglomerative BVH over
 * Morton-sorted triangles) and the per-triangle curvature metric C_i of Eq. (1) (Meyer
 * et al. cotangent operator).  The handle borrows `blob` and copies the mesh pointers
 * (the mesh arrays must outlive the scene). */
int et_scene_build(et_ctx* ctx, const et_mesh_desc* mesh, void* blob, size_t blob_bytes, void* scratch,
                   size_t scratch_bytes, et_scene** out);
int et_scene_free(et_scene* scene);

typedef struct {
  int64_t T, V, n_nodes;
  int32_t depth;          /* BVH depth (root = 1) */
  double sah_cost;        /* SAH cost with C_node = 1, C_tri = 1, normalised by the root area */
  double build_ms;        /* device time of the build (event-timed) */
  double refit_ms;        /* device time of the last et_scene_refit (0 before any) */
} et_scene_info;
int et_scene_get_info(et_ctx* ctx, const et_scene* scene, et_scene_info* info);   /* synchronises */

/* Device copies of the curvature outputs of the build: C [T] (Eq. 1) and G_v [V]
 * (half the norm of the mean-curvature normal).  Either pointer may be NULL. */
int et_scene_curvature(et_ctx* ctx, const et_scene* scene, double* C_out, double* G_out);

/* Dynamic scenes (objects moved or meshes animated between frames, Sec. III-A/III-B; the
 * paper computes curvature offline and so leaves animated meshes out of the diffraction
 * component, Sec. VI): new vertex positions for the same triangles, materials and objects.
 *   vertices   device [V][3] FP32, same V as the build; it replaces the mesh's vertex
 *              pointer and must outlive the scene (or the next refit)
 *   area_ref   as in et_mesh_desc, for the recomputed curvature C_i of Eq. (1)
 * Recomputes the repacked triangles, the object boxes, the curvature G_v and C_i, and every
 * BVH box bottom-up, one depth level per launch, over the topology of the last build.  It
 * takes no workspace: what it needs beyond the tree (nodes by depth, the triangles around each
 * vertex, a few bytes of scratch) was kept in the blob by the build.  The boxes are exact
 * unions of the FP32 triangle bounds, so refitting to the build's own vertices reproduces the
 * blob bit for bit and traces of a refitted scene hit what a fresh build hits.  Large
 * deformations keep a valid but looser tree: sah_cost of et_scene_get_info is recomputed
 * (rebuild when it grows).  Ordered on the context's stream; returns after the refit
 * finished; refits of one scene must not overlap.  Errors: ET_E_INVALID for NULL pointers and
 * for a non-finite coordinate of a vertex that a triangle uses (the scene must then be refitted
 * to finite vertices before it is traced again), ET_E_DEVICE for device failures (the scene is
 * then unusable and must be rebuilt). */
int et_scene_refit(et_ctx* ctx, et_scene* scene, const float* vertices, double area_ref);

/* ------------------------------------------------------------------ one pose (one emitter) */
enum {
  ET_SPECULAR = 1u << 0,      /* trace rays (Algorithm 1) and synthesise their records */
  ET_DIFFRACTION = 1u << 1,   /* draw diff_K curvature-importance samples (Sec. III-D) */
  ET_SYNTH_DIRECT = 1u << 2,  /* force the per-term synthesis and adjoint kernels (no factorised MFMA path) */
  ET_PASSIVE = 1u << 3,       /* passive component: direct emitter -> receiver path per receiver,
                                 P(f) = L_geo L_atm I_p e^{j omega r / c} (Eqs. 11-13), with a
                                 line-of-sight test from the emitter to each receiver */
  ET_DIFF_PER_MESH = 1u << 4, /* with ET_DIFFRACTION: diff_K candidates for every mesh (object)
                                 with eligible triangles, each from the mesh's own curvature CDF
                                 (Sec. III-D); meshes in increasing object order, draws numbered
                                 mesh-major; at most diff_max_meshes meshes (more: the first ones,
                                 and ET_E_CAPACITY at et_get_stats) */
  ET_PATH_PRODUCT = 1u << 5,  /* alternative reading of Eq. (2): a specular record's magnitude uses
                                 the product of k over its ray's reflections up to it (the default
                                 uses its own triangle's k).  et_trace fills paths->prev; synthesis
                                 needs it.  Not differentiable here (the adjoint reports
                                 ET_E_UNSUPPORTED).  Records of one pose < 2^31. */
  ET_PER_RX_VISIBILITY = 1u << 6  /* alternative reading of Algorithm 1's visibility ray: one line of
                                 sight from every hit to every receiver (M <= 64) instead of one
                                 toward x_ref; et_trace fills paths->rx_vis (bit m: receiver m sees
                                 the point); synthesis and adjoint pair a record with receiver m
                                 only when its bit is set.  Diffraction records have every bit set
                                 (no receiver-side test), passive ones their own receiver's. */
};

typedef struct {
  double emitter_pos[3];
  double emitter_rot[9];
  int32_t M;                    /* receivers */
  const double* rx_pos;         /* device [M][3] */
  const double* rx_rot;         /* device [M][9] or NULL (identity frames) */
  double x_ref[3];              /* target of the per-hit line-of-sight ray (Algorithm 1) */
  int64_t N;                    /* rays */
  const float* ray_dirs;        /* device [N][3], emitter frame (normalised in FP64) */
  int32_t max_bounces;          /* reflection points (hit records) per ray, >= 1 */
  double max_distance;          /* stop a ray once its path reaches this (after recording) */
  double t_eps;                 /* self-intersection threshold: hits need t > t_eps */
  double f_lo, f_hi;            /* inclusive linear frequency grid of F bins */
  int32_t F;
  double c;                     /* speed of sound (343 m/s in the paper) */
  double atm_a0, atm_a1;        /* air absorption A(f) = a0 + a1 f in dB/m: L_atm = 10^(-A r / 20) */
  double spreading_p;           /* spreading L_geo = r^-p (p = 2 in the paper) */
  int32_t phase_sign;           /* +1: exp(+j 2 pi f r / c) as printed in Eq. (4); -1 conjugates */
  int32_t Q, Bk;                /* materials x frequency bands; band of bin k is floor(k Bk / F) */
  const float* refl_k;          /* device [Q][Bk] reflection magnitude k (Eq. 2), >= 0; the kernels
                                   take log2 k, so a negative entry gives NaN spectra (device data
                                   are not inspected on the host) */
  const float* lobe_beta;       /* device [Q][Bk] lobe opening angle beta, radians (Eq. 2), > 0 */
  const float* diff_coef;       /* device [Q][Bk] diffraction coefficient I_d (Eq. 7), >= 0 */
  int32_t Bd, El, Az;           /* directivity bands, elevation and azimuth cells */
  const float* directivity;     /* device [M][Bd][El][Az] real gain or NULL */
  int64_t diff_K;               /* diffraction samples */
  uint64_t diff_seed;
  double diff_tau;              /* eligibility: C_i >= tau * max C */
  double diff_max_incidence;    /* incidence limit between normal and source direction */
  double diff_cone_half_angle;  /* emitter field of view for object eligibility */
  uint32_t flags;               /* ET_SPECULAR | ET_DIFFRACTION | ET_SYNTH_DIRECT | ET_PASSIVE | ET_DIFF_PER_MESH |
                                   ET_PATH_PRODUCT | ET_PER_RX_VISIBILITY */
  const float* passive_coef;    /* device [Bk] source magnitude I_p per band (ET_PASSIVE), >= 0 */
  int64_t diff_max_meshes;      /* ET_DIFF_PER_MESH: meshes that may receive candidates (sizes the
                                   records and workspace: diff_K * diff_max_meshes draws) */
} et_sim_desc;

/* Path records (hit buffer B of Algorithm 1 plus diffraction points and the passive
 * component), caller-owned device SoA arrays of `capacity` entries.  Order: specular
 * records bounce-major (all bounce-0 hits, then bounce 1, ...); within a bounce the rays
 * follow the library's traversal order (ray order, or sorted by direction when there are
 * more rays than the device holds threads of the traversal kernel at once; deterministic
 * either way; `ray` names each record's ray).  Kept diffraction samples follow in sample order, then with ET_PASSIVE one
 * record per receiver m (the emitter as the point, rtot 0, mat = ray = m) that reaches
 * receiver m only.  count (device int64[4]) = {records, specular, diffraction, segments};
 * passive records = records - specular - diffraction. */
typedef struct {
  int64_t capacity;
  double* p;          /* [cap][3] hit / diffraction point */
  float* dout;        /* [cap][3] reflected direction (specular) */
  double* rtot;       /* [cap] path length emitter -> point */
  int32_t* tri;       /* [cap] original triangle index */
  int32_t* mat;       /* [cap] material of the triangle */
  int32_t* ray;       /* [cap] ray index (specular) or sample index (diffraction) */
  uint8_t* bounce;    /* [cap] reflection index within the ray */
  uint8_t* flags;     /* [cap] bit0 visible (line of sight; with ET_PER_RX_VISIBILITY: seen by
                         any receiver); bits 1-2 kind: 0 specular, 1 diffraction, 2 passive */
  int64_t* count;     /* device int64[4] */
  int64_t* prev;      /* [cap] or NULL: index of the same ray's previous specular record, -1 at
                         its first reflection (written when not NULL; ET_PATH_PRODUCT needs it) */
  uint64_t* rx_vis;   /* [cap] or NULL: per-receiver line-of-sight bits (ET_PER_RX_VISIBILITY) */
} et_paths;

/* Workspace bytes for et_trace / et_synthesize / et_simulate with this descriptor. */
int et_workspace_size(et_ctx* ctx, const et_scene* scene, const et_sim_desc* sim, size_t* bytes);

/* Algorithm 1 (+ diffraction sampling if ET_DIFFRACTION, + the passive component if
 * ET_PASSIVE): fills `paths` (and paths->prev when not NULL, paths->rx_vis with
 * ET_PER_RX_VISIBILITY).  Records beyond capacity are dropped and the call reports
 * ET_E_CAPACITY at the next et_get_stats. */
int et_trace(et_ctx* ctx, const et_scene* scene, const et_sim_desc* sim, void* ws, size_t ws_bytes,
             const et_paths* paths);

/* Eqs. (2)-(4), (7)-(8): spectra[m][k] = sum over visible records of M(f_k) e^{j sigma 2 pi f_k r / c}
 * with r = rtot + |p - x_m|.  Output device float [M][F][2] (complex64), overwritten.
 * Reads the record count from paths->count[0]. */
int et_synthesize(et_ctx* ctx, const et_sim_desc* sim, const et_paths* paths, void* ws, size_t ws_bytes,
                  float* spectra);

/* For callers that cannot allocate device memory or hand over a workspace (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): et_synthesize with the
 * same inputs and output, but no workspace.  Its band tables and per-chunk partial spectra live
 * in a 64 MiB scratch array that the library keeps in each GPU's memory from the first
 * et_create on that device until the process ends, and its kernels walk every record (hidden
 * ones contribute nothing) instead of a compacted list of the visible ones.  The call allocates
 * nothing.  Limits: the tables (4 Q Bk + Bk floats) and one record chunk's partial spectra
 * (8 M F bytes) must fit in the scratch (ET_E_UNSUPPORTED otherwise, e.g. beyond M F = 8 M);
 * ET_PATH_PRODUCT is refused (ET_E_UNSUPPORTED: it needs per-record tables).  Every call on a
 * device uses that device's one scratch and leaves its contents there: calls that overlap on
 * one GPU (other streams, contexts or threads) race and must be serialised by the caller.
 * Results equal et_synthesize's up to the FP32 order of the per-chunk sums. */
int et_synthesize_noalloc(et_ctx* ctx, const et_sim_desc* sim, const et_paths* paths, float* spectra);

/* et_trace followed by et_synthesize. */
int et_simulate(et_ctx* ctx, const et_scene* scene, const et_sim_desc* sim, const et_paths* paths, void* ws,
                size_t ws_bytes, float* spectra);

/* Adjoint of et_synthesize over fixed records: given grad_spectra = dL/dH* as complex64
 * [M][F][2] (for L = sum |H - H_target|^2 this is H - H_target), writes dL/d refl_k as
 * double [Q][Bk] and dL/d rx_pos as double [M][3] (device, overwritten).  Records keep
 * their hit points and visibility ("fixed ray paths").  With receiver directivity the
 * receiver gradient includes the change of each band's gain with the direction of arrival
 * (the gradient of the bilinear table inside the cell that holds the direction; the receiver
 * orientations rx_rot are not differentiated); such calls run the per-term kernel.
 * ET_E_UNSUPPORTED for ET_PATH_PRODUCT, Bk > 16, Q*Bk > 256 or F > 12288. */
int et_synthesize_backward(et_ctx* ctx, const et_sim_desc* sim, const et_paths* paths, const float* grad_spectra,
                           void* ws, size_t ws_bytes, double* grad_k, double* grad_rx);

/* ------------------------------------------------------------------ batches of poses */
typedef struct {
  const et_scene* scene;
  const et_sim_desc* sim;       /* per-job descriptor (M, F, B, Q, Bk equal across jobs) */
} et_job;

/* Workspace for a batch: fused (specular-only) batches run in job waves (et_tuning.wave_rays) and
 * need one wave's rays and synthesis scratch and, with several waves, two waves' records (the
 * next wave traces into one buffer while the synthesis reads the other); other batches run job
 * after job and need the largest job's scratch plus every job's records. */
int et_batch_workspace_size(et_ctx* ctx, int32_t J, const et_job* jobs, size_t* bytes);

/* Traces and synthesises J jobs (poses and scenes may all differ; M, F, Q and Bk are shared).
 * When every job is specular-only the batch runs fused: one ray-state array holds all jobs'
 * rays and each bounce is one launch over all of them (every ray reads its scene and pose
 * from a device job table); the visible records of all jobs are sorted by job (stably) and
 * cut into chunks that never mix jobs, so one synthesis launch (and one adjoint launch)
 * covers the batch, followed by a per-job reduction in a fixed order.  With several job waves
 * the traces run on the context's second stream, each wave's synthesis (and adjoint) on the
 * context's stream once its trace is done, so that a wave's synthesis runs beside the next
 * wave's trace; the waves alternate between two record buffers and two control blocks, and
 * the call's work ends on the context's stream (not when the stream is being captured into a
 * graph: then the waves run in order on that stream).  Launch shapes come from the context's
 * tuning (et_autotune_batch).  Batches with diffraction jobs run job after
 * job.  spectra is device float [J][M][F][2].  grad_spectra (optional, same shape, dL/dconj(H)
 * per job) makes the call also write every job's adjoint into grad_k [J][Q][Bk] and
 * grad_rx [J][M][3] (device double).  Results are bit-reproducible for a given tuning. */
int et_simulate_batch(et_ctx* ctx, int32_t J, const et_job* jobs, void* ws, size_t ws_bytes, float* spectra,
                      const float* grad_spectra, double* grad_k, double* grad_rx);

/* Captures et_simulate_batch into a HIP graph owned by the context and replays it
 * (the first call captures; later calls with the same arguments replay). */
int et_simulate_batch_graph(et_ctx* ctx, int32_t J, const et_job* jobs, void* ws, size_t ws_bytes,
                            float* spectra, const float* grad_spectra, double* grad_k, double* grad_rx);
int et_graph_reset(et_ctx* ctx);

/* ------------------------------------------------------------------ several emitters
 * Simultaneous sources (the paper's multi-emitter scenes): S emitters in one scene heard by
 * one receiver array.  Propagation is linear, so the received spectrum is the sum of every
 * emitter's (Eq. 6 summed over the sources): H_m = sum_s H_m^(s).  sims is an array of S
 * descriptors that share rx_pos (the same device pointer), M, F, f_lo, f_hi and phase_sign;
 * poses, rays, bounces, components (ET_SPECULAR, ET_DIFFRACTION, ET_PASSIVE) and materials may
 * differ.  The emitters run as the jobs of a batch (fused when all are specular-only), each
 * into its own spectra in the workspace, then one kernel sums them in emitter order, so the
 * result is bit-reproducible.  spectra: device float [M][F][2]. */
int et_emitters_workspace_size(et_ctx* ctx, const et_scene* scene, int32_t S, const et_sim_desc* sims,
                               size_t* bytes);
int et_simulate_emitters(et_ctx* ctx, const et_scene* scene, int32_t S, const et_sim_desc* sims, void* ws,
                         size_t ws_bytes, float* spectra);

/* ------------------------------------------------------------------ time domain
 * The step after the path: impulse responses from the spectra (Eqs. 5-6, 9-10, 13:
 * h = F^-1[H]) and received signals (Eq. 14: s = h * s_e).
 *
 * Impulse response of receiver m from its spectrum on the grid f_k = f_lo + k df (df =
 * (f_hi - f_lo) / (F - 1)), sampled at t_n = n dt with dt = 1 / (n_t df), n < n_t:
 *   h_m(t_n) = 2 df Re sum_k H_m[k] exp(-j phase_sign 2 pi f_k t_n),
 * the real signal of the one-sided band spectrum; a path of delay tau peaks at t = tau for
 * either phase sign.  The band-limited response repeats every 1/df (c/df of path length);
 * n_t sets the sampling (fs = n_t df, at least 2 f_hi for a Nyquist-sampled signal).
 * spectra: device float [M][F][2]; h: device float [M][n_t]; n_t a power of two with
 * F <= n_t <= 2^22; *dt_out (host, may be NULL) receives dt.  ET_E_WORKSPACE if ws_bytes is
 * below et_impulse_response_workspace_size. */
int et_impulse_response_workspace_size(int32_t M, int32_t n_t, size_t* bytes);
int et_impulse_response(et_ctx* ctx, int32_t M, int32_t F, double f_lo, double f_hi, int32_t phase_sign,
                        const float* spectra, int32_t n_t, void* ws, size_t ws_bytes, float* h, double* dt_out);

/* Received signal of every receiver for the emitted call s_e (L samples at the same dt):
 *   s_m[n] = dt sum_k h_m[k] s_e[n - k],  n < n_t + L - 1,
 * computed by FFT of length P = the power of two >= n_t + L - 1 (P <= 2^23).
 * h: device float [M][n_t]; s_e: device float [L]; out: device float [M][n_t + L - 1]. */
int et_receiver_signal_workspace_size(int32_t M, int32_t n_t, int64_t L, size_t* bytes);
int et_receiver_signal(et_ctx* ctx, int32_t M, int32_t n_t, const float* h, int64_t L, const float* s_e, double dt,
                       void* ws, size_t ws_bytes, float* out);

/* ------------------------------------------------------------------ ray sets (Sec. III-C)
 * The paper spreads each emitter's rays by the recursive zonal equal-area partition of the
 * sphere (Leopardi 2006).  EQ(2, N): two polar caps of area A = 4 pi / N, n collars of equal
 * angular height between them (n = round((pi - 2 theta_c) / sqrt(A))), collar i holding the
 * rounded share of the cumulative ideal count, every zone boundary at the colatitude whose cap
 * holds exactly its regions.  A direction is a region centre: the middle colatitude of its
 * collar, longitudes 2 pi ((j + 1/2) / m_i + offset_i) with each collar turned against the one
 * above by Leopardi's twist (1/m_{i+1} - 1/m_i)/2 + gcd(m_i, m_{i+1}) / (2 m_i m_{i+1}) turns.
 * Counts round to the nearest integer with halves (and values within N 2^-36 above a half)
 * rounded down: a boundary on the equator has an ideal count of exactly (N - 2) / 2.
 * Directions are in the emitter frame with the polar axis on the boresight +x:
 * (cos t, sin t cos p, sin t sin p).  Order: the boresight, then collar by collar outward in
 * increasing longitude, then the backward pole; a cone keeps a prefix of this order.
 *   N                regions of the whole sphere, 1 <= N <= 2^28
 *   cone_half_angle  radians in (0, pi]: keep the centres with colatitude <= it
 *   ws               device workspace of et_eq_directions_workspace_size(N) bytes (collar table)
 *   dirs             device [capacity][3] FP32, or NULL with capacity 0 to query the count
 *   count            host out: the number of directions in the cone
 * Synchronises the stream (the count comes back to the host).  ET_E_CAPACITY (count still
 * set, nothing written) when dirs is given and the count exceeds capacity. */
int et_eq_directions_workspace_size(int64_t N, size_t* bytes);
int et_eq_directions(et_ctx* ctx, int64_t N, double cone_half_angle, void* ws, size_t ws_bytes, float* dirs,
                     int64_t capacity, int64_t* count);

/* ------------------------------------------------------------------ tuning of fused batches
 * Launch shapes kept per context: the workgroups that the record chunks of the synthesis and
 * adjoint kernels aim at, and the grid of the bounce kernels (grid-stride over the active
 * rays).  Workspaces from et_batch_workspace_size serve every allowed value. */
typedef struct {
  int32_t synth_wgs;      /* 64 .. 16384 (default 4096) */
  int32_t adjoint_wgs;    /* 64 .. 16384 (default 4096) */
  int32_t trace_blocks;   /* 64 .. 8192 (default 4096) */
  int32_t wave_rays;      /* rays per job wave of a fused batch: >= 1024, or 0 for the default 2^23.
                             Jobs run in waves of consecutive jobs whose rays add up to at most this
                             (a larger job forms its own wave); the workspace holds one wave's rays
                             and records, so et_batch_workspace_size depends on it */
  double ms_trace, ms_synth, ms_adjoint;   /* event times of the chosen shape (et_autotune_batch),
                                              summed over the waves */
} et_tuning;
int et_get_tuning(et_ctx* ctx, et_tuning* out);
int et_set_tuning(et_ctx* ctx, const et_tuning* t);   /* ET_E_INVALID outside the ranges */

/* Autotuner: runs the fused batch (as et_simulate_batch, with the adjoint when grad_spectra
 * is given) once per candidate shape (synthesis and adjoint workgroups 1024, 2048, 4096, 8192,
 * 16384; bounce grids 1024, 2048, 4096, 6144, 8192 blocks), times the trace phase, the synthesis
 * kernel and the adjoint kernel with events, keeps for each knob its fastest candidate in
 * the context (its runs take the job waves in order on the context's stream, so that the
 * phases do not interact) and returns the choice with its times.  The outputs hold the
 * results of the last run.  ET_E_UNSUPPORTED for batches that do not run
 * fused (jobs with diffraction). */
int et_autotune_batch(et_ctx* ctx, int32_t J, const et_job* jobs, void* ws, size_t ws_bytes, float* spectra,
                      const float* grad_spectra, double* grad_k, double* grad_rx, et_tuning* out);

/* ------------------------------------------------------------------ statistics */
typedef struct {
  int64_t records, specular, diffraction, segments;  /* of the last trace */
  int64_t shadow_rays;                               /* visibility / line-of-sight rays */
  int64_t diff_eligible;                             /* triangles in the diffraction CDF */
  int64_t stack_overflows;                           /* traversal stack overflows (must be 0) */
  int64_t dropped;                                   /* records beyond capacity */
  int32_t synth_kernel;                              /* 1 factorised MFMA, 2 direct per-term */
  int32_t status;                                    /* deferred device-side status */
  double ms_trace, ms_diffraction, ms_synth;         /* event-timed phases of the last calls (summed
                                                        over job waves; pipelined waves overlap) */
  double ms_adjoint;                                 /* event-timed et_synthesize_backward */
  double ms_synth_kernel, ms_adjoint_kernel;         /* the main synthesis / adjoint kernel alone */
  int32_t adjoint_kernel;                            /* 1 factorised MFMA, 2 direct per-term */
  int32_t reserved0;
  int64_t passive;                                   /* passive records of the last trace */
} et_stats;
int et_get_stats(et_ctx* ctx, et_stats* out);   /* synchronises the context stream */

/* Traversal work counters (node and triangle fetches of closest-hit and any-hit queries)
 * for the roofline's algorithmic bytes: enables counting in the next et_trace.  0/1. */
int et_set_counting(et_ctx* ctx, int enable);
typedef struct { int64_t nodes_closest, tris_closest, nodes_any, tris_any, rays_closest, rays_any; } et_counters;
int et_get_counters(et_ctx* ctx, et_counters* out);

/* Test hook for the overflow path of the traversal stack (normally unreachable: 64 entries per
 * lane hold any tree this library builds for up to 2^31 triangles in practice).  Limits the
 * per-lane stack of later traces on this context to `entries` (1 .. 64; 0 restores 64).  A
 * traversal that needs more drops the subtrees that do not fit, so those rays may miss their
 * true hits; every kernel still completes, and et_get_stats reports the dropped pushes in
 * stack_overflows with status ET_E_INTERNAL.  ET_E_INVALID outside [0, 64]. */
int et_set_stack_limit(et_ctx* ctx, int32_t entries);

#ifdef __cplusplus
}
#endif
#endif
