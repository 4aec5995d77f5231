// C ABI entry points (include/echotrace.h): argument validation, workspace planning,
// launch sequencing on the context stream, statistics and graph capture.
#include "internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

using namespace et;

// which of the context's event pairs hold times of the last calls
enum : uint32_t { TM_TRACE = 1, TM_SYNTH = 2, TM_ADJ = 4, TM_SYNTH_K = 8, TM_ADJ_K = 16, TM_WAVES = 32 };

struct et_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  Ctl* ctl = nullptr;                 // device control block (with ctl2, the only library allocations)
  Ctl* ctl2 = nullptr;                // control block of the odd job waves of a pipelined batch
  hipStream_t aux = nullptr;          // a batch's trace stream (default priority) beside `stream`,
                                      // created by the first pipelined batch
  hipEvent_t pev[5] = {};             // pipelined batch: fork, trace done (2), synthesis done (2)
  bool serial_waves = false;          // the autotuner's runs: job waves in order on one stream
  bool counting = false;
  int32_t stack_cap = TRAV_STACK;     // per-lane traversal stack entries (et_set_stack_limit)
  hipEvent_t ev[12] = {};
  uint32_t timed = 0;   // event pairs holding the last calls' times (TM_* bits)
  std::vector<hipEvent_t> wave_ev;   // fused batches: per job wave, trace / synthesis / adjoint pairs
  int32_t waves_timed = 0;           // waves of the last timed fused batch (TM_WAVES)
  int synth_kernel = 0;
  et::BatchTune tune;
  int adjoint_kernel = 0;
  const int64_t* last_count = nullptr;   // device count array of the last traced paths
  // graph replay of a batch
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint64_t> graph_key;
};

namespace {

int fail(et_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

template <typename F>
int guarded(et_ctx* ctx, F&& f) {
  if (!ctx) return ET_E_INVALID;
  try {
    ET_HIP(hipSetDevice(ctx->device));
    f();
    ctx->last_error.clear();
    return ET_OK;
  } catch (const Error& e) {
    return fail(ctx, e.code, e.msg);
  } catch (const std::exception& e) {
    return fail(ctx, ET_E_INTERNAL, e.what());
  }
}

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

void validate_mesh(const et_mesh_desc* m) {
  ET_CHECK(m, ET_E_INVALID, "mesh descriptor is NULL");
  ET_CHECK(m->T >= 0 && m->V >= 0, ET_E_INVALID, "negative mesh sizes");
  ET_CHECK(m->T < (int64_t)1 << 31 && m->V < (int64_t)1 << 31, ET_E_UNSUPPORTED, "mesh larger than 2^31 elements");
  ET_CHECK(m->T == 0 || (m->vertices && m->tris && m->tri_material && m->tri_object), ET_E_INVALID,
           "mesh array pointer is NULL");
  ET_CHECK(m->n_objects >= 1, ET_E_INVALID, "n_objects must be >= 1");
  ET_CHECK(std::isfinite(m->area_ref), ET_E_INVALID, "area_ref is not finite");
}

void validate_sim(const et_sim_desc* s, bool need_rays) {
  ET_CHECK(s, ET_E_INVALID, "simulation descriptor is NULL");
  ET_CHECK(finite3(s->emitter_pos) && finite3(s->x_ref), ET_E_INVALID, "emitter position or x_ref not finite");
  for (int i = 0; i < 9; ++i) ET_CHECK(std::isfinite(s->emitter_rot[i]), ET_E_INVALID, "emitter rotation not finite");
  ET_CHECK(s->M >= 1 && s->rx_pos, ET_E_INVALID, "need M >= 1 receivers and rx_pos");
  ET_CHECK(s->F >= 1, ET_E_INVALID, "need F >= 1 frequency bins");
  ET_CHECK(std::isfinite(s->f_lo) && std::isfinite(s->f_hi) && s->f_lo >= 0 && s->f_hi >= s->f_lo, ET_E_INVALID,
           "frequency grid must satisfy 0 <= f_lo <= f_hi");
  ET_CHECK(std::isfinite(s->c) && s->c > 0, ET_E_INVALID, "speed of sound must be positive");
  ET_CHECK(std::isfinite(s->atm_a0) && std::isfinite(s->atm_a1) && std::isfinite(s->spreading_p), ET_E_INVALID,
           "absorption / spreading parameters not finite");
  ET_CHECK(s->phase_sign == 1 || s->phase_sign == -1, ET_E_INVALID, "phase_sign must be +1 or -1");
  ET_CHECK(s->Q >= 1 && s->Bk >= 1 && s->Bk <= 64, ET_E_INVALID, "need Q >= 1 and 1 <= Bk <= 64");
  ET_CHECK(s->refl_k && s->lobe_beta && s->diff_coef, ET_E_INVALID, "material tables are NULL");
  if (s->directivity) {
    ET_CHECK(s->Bd >= 1 && s->Bd <= 64 && s->El >= 1 && s->Az >= 1, ET_E_INVALID, "directivity shape invalid");
  }
  ET_CHECK(!(s->flags & ET_PASSIVE) || s->passive_coef, ET_E_INVALID, "ET_PASSIVE needs passive_coef");
  if (need_rays) {
    ET_CHECK(s->N >= 0, ET_E_INVALID, "negative ray count");
    ET_CHECK(s->N == 0 || s->ray_dirs || !(s->flags & ET_SPECULAR), ET_E_INVALID, "ray_dirs is NULL");
    ET_CHECK(s->N < (int64_t)1 << 31, ET_E_UNSUPPORTED, "more than 2^31 rays in one pose");
    ET_CHECK(s->max_bounces >= 1 && s->max_bounces <= 255, ET_E_INVALID, "max_bounces must be in [1, 255]");
    ET_CHECK(!std::isnan(s->max_distance) && s->max_distance > 0, ET_E_INVALID, "max_distance must be > 0");
    ET_CHECK(std::isfinite(s->t_eps) && s->t_eps >= 0, ET_E_INVALID, "t_eps must be finite and >= 0");
    if (s->flags & ET_DIFFRACTION) {
      ET_CHECK(s->diff_K >= 0 && s->diff_K < (int64_t)1 << 31, ET_E_INVALID, "diff_K out of range");
      if (s->flags & ET_DIFF_PER_MESH)
        ET_CHECK(s->diff_max_meshes >= 1 && s->diff_max_meshes < (int64_t)1 << 31 &&
                     s->diff_K * s->diff_max_meshes < (int64_t)1 << 31,
                 ET_E_INVALID, "per-mesh diffraction needs 1 <= diff_max_meshes and diff_K * diff_max_meshes < 2^31");
      ET_CHECK(std::isfinite(s->diff_tau) && std::isfinite(s->diff_max_incidence) &&
                   std::isfinite(s->diff_cone_half_angle),
               ET_E_INVALID, "diffraction parameters not finite");
    }
  }
}

void validate_paths(const et_paths* p) {
  ET_CHECK(p, ET_E_INVALID, "paths descriptor is NULL");
  ET_CHECK(p->capacity >= 0, ET_E_INVALID, "negative path capacity");
  ET_CHECK(p->count, ET_E_INVALID, "paths->count is NULL");
  ET_CHECK(p->capacity == 0 || (p->p && p->dout && p->rtot && p->tri && p->mat && p->ray && p->bounce && p->flags),
           ET_E_INVALID, "a path array is NULL");
}

// The arrays the alternative readings need, for calls that write or read them.
void validate_readings(const et_sim_desc* s, const et_paths* p) {
  if (s->flags & ET_PATH_PRODUCT) {
    ET_CHECK(p->capacity == 0 || p->prev, ET_E_INVALID, "ET_PATH_PRODUCT needs paths->prev");
    ET_CHECK(p->capacity < ((int64_t)1 << 31), ET_E_UNSUPPORTED, "ET_PATH_PRODUCT needs fewer than 2^31 records");
  }
  if (s->flags & ET_PER_RX_VISIBILITY) {
    ET_CHECK(p->capacity == 0 || p->rx_vis, ET_E_INVALID, "ET_PER_RX_VISIBILITY needs paths->rx_vis");
    ET_CHECK(s->M <= 64, ET_E_UNSUPPORTED, "ET_PER_RX_VISIBILITY supports at most 64 receivers");
  }
}

// Diffraction draws at most: diff_K, or diff_K per mesh for at most diff_max_meshes meshes.
int64_t diff_draws_max(const et_sim_desc* s) {
  if (!(s->flags & ET_DIFFRACTION)) return 0;
  return s->diff_K * ((s->flags & ET_DIFF_PER_MESH) ? s->diff_max_meshes : 1);
}

int64_t records_upper_bound(const et_sim_desc* s) {
  int64_t n = 0;
  if (s->flags & ET_SPECULAR) n += s->N * (int64_t)s->max_bounces;
  n += diff_draws_max(s);
  if (s->flags & ET_PASSIVE) n += s->M;
  return n;
}

size_t al(size_t b) { return (b + 255) / 256 * 256; }

size_t paths_bytes(int64_t cap) {   // the arrays of carve_paths, each aligned to 256 bytes
  return al(cap * (24 + 12 + 8 + 4 + 4 + 4 + 1 + 1 + 8 + 8)) + al(8 * sizeof(int64_t)) + 10 * 256;
}

// A batch runs fused (all rays in shared bounce kernels, all records in shared synthesis
// kernels) when every job is specular-only; otherwise jobs run one after another.
bool batch_fused(int32_t J, const et_job* jobs) {
  if (J > 65536) return false;   // the ray sort keys hold the job in 16 bits
  for (int32_t j = 0; j < J; ++j)
    if (jobs[j].sim->flags & (ET_DIFFRACTION | ET_PASSIVE | ET_PATH_PRODUCT | ET_PER_RX_VISIBILITY)) return false;
  return true;
}

struct WsPlan {
  size_t trace = 0, synth = 0, bwd = 0;
  size_t total() const { return trace + synth + bwd; }
};

WsPlan plan(const et_scene* sc, const et_sim_desc* s, int64_t cap) {
  WsPlan w;
  const int64_t N = (s->flags & ET_SPECULAR) ? s->N : 0;
  const int64_t K = diff_draws_max(s);
  if (sc) w.trace = al(trace_ws_layout(N, sc->d.T, sc->d.n_obj, K, nullptr, nullptr));
  w.synth = al(synth_ws_layout(s, cap, nullptr, nullptr));
  w.bwd = al(synth_bwd_ws_layout(s, cap, nullptr, nullptr));
  return w;
}

// Workspace of a fused batch: trace job table, ray state of all jobs, records of all jobs,
// synthesis scratch (visible list sorted by job, chunk tables, partial spectra, gradients).
// Job waves of a fused batch: consecutive jobs whose rays add up to at most wave_rays (a job
// with more rays forms a wave of its own).  Each wave is traced, synthesised and differentiated
// by the fused kernels in the same workspace, so the workspace holds one wave's rays and records.
struct Wave {
  int32_t j0, n;
  int64_t N, cap;
};

std::vector<Wave> job_waves(int32_t J, const et_job* jobs, int64_t wave_rays) {
  std::vector<Wave> w;
  Wave cur{0, 0, 0, 0};
  for (int32_t j = 0; j < J; ++j) {
    const int64_t nr = (jobs[j].sim->flags & ET_SPECULAR) ? jobs[j].sim->N : 0;
    if (cur.n > 0 && cur.N + nr > wave_rays) {
      w.push_back(cur);
      cur = Wave{j, 0, 0, 0};
    }
    ++cur.n;
    cur.N += nr;
    cur.cap += records_upper_bound(jobs[j].sim);
  }
  w.push_back(cur);
  return w;
}

// Workspace of a fused batch: each part sized for the largest wave.
struct FusedPlan {
  std::vector<Wave> waves;
  int64_t N = 0, cap = 0;
  size_t tj = 0, tw = 0, pp = 0, sy = 0, total = 0;
};

FusedPlan fused_plan(et_ctx* ctx, int32_t J, const et_job* jobs) {
  FusedPlan f;
  f.waves = job_waves(J, jobs, ctx->tune.wave_rays);
  for (const Wave& w : f.waves) {
    const int64_t cap = std::max<int64_t>(w.cap, 1);
    f.N = std::max(f.N, w.N);
    f.cap = std::max(f.cap, cap);
    f.tj = std::max(f.tj, al(trace_batch_jobs_bytes(w.n)));
    f.sy = std::max(f.sy, al(synth_batch_ws_layout(w.n, jobs + w.j0, cap, ctx->tune, true, nullptr, nullptr)));
  }
  f.tw = al(trace_ws_layout(f.N, 0, 0, 0, nullptr, nullptr, TUNE_MAX_TRACE_BLOCKS));
  f.pp = al(paths_bytes(f.cap));
  // with several waves, two record buffers: the next wave's trace fills one while the
  // synthesis reads the other
  f.total = f.tj + f.tw + (f.waves.size() > 1 ? 2 : 1) * f.pp + f.sy;
  return f;
}

// Workspace of a batch run job after job: the largest job's scratch plus every job's records.
size_t sequential_bytes(int32_t J, const et_job* jobs) {
  size_t mx = 0, paths = 0;
  for (int j = 0; j < J; ++j) {
    const int64_t cap = std::max<int64_t>(records_upper_bound(jobs[j].sim), 1);
    mx = std::max(mx, plan(jobs[j].scene, jobs[j].sim, cap).total());
    paths += paths_bytes(cap);
  }
  return mx + paths;
}

void check_scene(const et_scene* sc) { ET_CHECK(sc, ET_E_INVALID, "scene is NULL"); }

// Phase times of the last timed fused batch, summed over its job waves: trace, synthesis
// kernel, adjoint kernel (ms; the stream must have completed the batch).
void wave_phase_ms(et_ctx* ctx, double* t) {
  t[0] = t[1] = t[2] = 0.0;
  for (int32_t w = 0; w < ctx->waves_timed; ++w) {
    const hipEvent_t* e = ctx->wave_ev.data() + 6 * w;
    float ms = 0.f;
    for (int p = 0; p < 3; ++p) {
      if (p == 2 && !(ctx->timed & TM_ADJ_K)) break;
      ET_HIP(hipEventElapsedTime(&ms, e[2 * p], e[2 * p + 1]));
      t[p] += ms;
    }
  }
}

// The scene's materials index the pose's band tables.
void check_materials(const et_scene* sc, const et_sim_desc* sim) {
  ET_CHECK(sc->max_mat < sim->Q, ET_E_INVALID, "a triangle's material is >= Q (the band tables' rows)");
}

void trace_impl(et_ctx* ctx, const et_scene* sc, const et_sim_desc* sim, void* ws, size_t ws_bytes, const et_paths* paths) {
  check_scene(sc);
  validate_sim(sim, true);
  check_materials(sc, sim);
  validate_paths(paths);
  validate_readings(sim, paths);
  const WsPlan w = plan(sc, sim, std::max<int64_t>(paths->capacity, records_upper_bound(sim)));
  ET_CHECK(ws || w.trace == 0, ET_E_INVALID, "workspace is NULL");
  ET_CHECK(ws_bytes >= w.trace, ET_E_WORKSPACE, "workspace too small for et_trace");
  TraceWS tw;
  trace_ws_layout((sim->flags & ET_SPECULAR) ? sim->N : 0, sc->d.T, sc->d.n_obj, diff_draws_max(sim), (char*)ws,
                  &tw);
  tw.stack_cap = ctx->stack_cap;
  ET_HIP(hipEventRecord(ctx->ev[0], ctx->stream));
  trace_run(sc->d, sim, paths, tw, ctx->ctl, ctx->counting, ctx->stream);
  ET_HIP(hipEventRecord(ctx->ev[1], ctx->stream));
  ctx->timed |= TM_TRACE;
  ctx->last_count = paths->count;
}

void synth_impl(et_ctx* ctx, const et_sim_desc* sim, const et_paths* paths, void* ws, size_t ws_bytes, float* spectra,
                bool from_trace) {
  validate_sim(sim, false);
  validate_paths(paths);
  validate_readings(sim, paths);
  ET_CHECK(spectra, ET_E_INVALID, "spectra is NULL");
  SynthWS sw;
  const size_t need = synth_ws_layout(sim, std::max<int64_t>(paths->capacity, 1), nullptr, nullptr);
  ET_CHECK(ws_bytes >= need, ET_E_WORKSPACE, "workspace too small for et_synthesize");
  synth_ws_layout(sim, std::max<int64_t>(paths->capacity, 1), (char*)ws, &sw);
  (void)from_trace;
  ET_HIP(hipEventRecord(ctx->ev[4], ctx->stream));
  ctx->synth_kernel = synth_run(sim, paths, sw, ctx->ctl, spectra, ctx->stream, ctx->ev[8], ctx->ev[9]);
  ET_HIP(hipEventRecord(ctx->ev[5], ctx->stream));
  ctx->timed |= TM_SYNTH | TM_SYNTH_K;
}

// number of records to synthesise = min(paths count, capacity); written into the control block
__global__ void k_set_nrec(Ctl* ctl, const int64_t* count, int64_t cap) {
  int64_t n = count[0];
  ctl->n_rec = n < cap ? n : cap;
}

// A pipelined batch's second control block starts without a deferred error.
__global__ void k_ctl_clear_err(Ctl* c) { c->err = 0; }

// The odd waves' statistics and deferred errors join the even waves' (every field the
// statistics read that a batch accumulates).
__global__ void k_ctl_merge(Ctl* a, const Ctl* b) {
  a->err |= b->err;
  a->rec_prev += b->rec_prev + b->rec_base;
  a->seg += b->seg;
  a->shadow += b->shadow;
  a->overflow += b->overflow;
  for (int i = 0; i < 6; ++i) a->cnt[i] += b->cnt[i];
}

}  // namespace

extern "C" {

int et_abi_version(void) { return ET_ABI_VERSION; }

const char* et_status_string(int status) {
  switch (status) {
    case ET_OK: return "ok";
    case ET_E_INVALID: return "invalid argument";
    case ET_E_WORKSPACE: return "workspace too small";
    case ET_E_CAPACITY: return "path capacity exceeded";
    case ET_E_DEVICE: return "HIP runtime error";
    case ET_E_UNSUPPORTED: return "unsupported request";
    case ET_E_INTERNAL: return "internal device-side error";
    default: return "unknown status";
  }
}

int et_create(int device, void* hip_stream, et_ctx** out) {
  if (!out) return ET_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ET_E_DEVICE;
  et_ctx* c = new et_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  try {
    ET_HIP(hipSetDevice(device));
    ET_HIP(hipMalloc(&c->ctl, sizeof(Ctl)));
    ET_HIP(hipMemset(c->ctl, 0, sizeof(Ctl)));
    ET_HIP(hipMalloc(&c->ctl2, sizeof(Ctl)));
    ET_HIP(hipMemset(c->ctl2, 0, sizeof(Ctl)));
    for (auto& e : c->ev) ET_HIP(hipEventCreate(&e));
    for (auto& e : c->pev) ET_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    noalloc_init(device);   // this device's address of the allocation-free calls' scratch
  } catch (const Error& e) {
    et_destroy(c);
    return e.code;
  }
  *out = c;
  return ET_OK;
}

int et_destroy(et_ctx* ctx) {
  if (!ctx) return ET_E_INVALID;
  (void)hipSetDevice(ctx->device);
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->wave_ev) (void)hipEventDestroy(e);
  for (auto& e : ctx->pev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
  if (ctx->ctl2) (void)hipFree(ctx->ctl2);
  if (ctx->ctl) (void)hipFree(ctx->ctl);
  delete ctx;
  return ET_OK;
}

int et_set_stream(et_ctx* ctx, void* hip_stream) {
  if (!ctx) return ET_E_INVALID;
  ctx->stream = (hipStream_t)hip_stream;
  return ET_OK;
}

const char* et_last_error(const et_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "NULL context"; }

int et_scene_size(et_ctx* ctx, const et_mesh_desc* mesh, size_t* blob_bytes, size_t* scratch_bytes) {
  return guarded(ctx, [&] {
    validate_mesh(mesh);
    ET_CHECK(blob_bytes && scratch_bytes, ET_E_INVALID, "output pointer is NULL");
    *blob_bytes = scene_blob_bytes(mesh->T, mesh->V, mesh->n_objects);
    *scratch_bytes = scene_scratch_bytes(mesh->T, mesh->V);
  });
}

int et_scene_build(et_ctx* ctx, const et_mesh_desc* mesh, void* blob, size_t blob_bytes, void* scratch,
                   size_t scratch_bytes, et_scene** out) {
  return guarded(ctx, [&] {
    validate_mesh(mesh);
    ET_CHECK(out, ET_E_INVALID, "output pointer is NULL");
    *out = nullptr;
    ET_CHECK(blob && scratch, ET_E_INVALID, "blob or scratch is NULL");
    ET_CHECK(blob_bytes >= scene_blob_bytes(mesh->T, mesh->V, mesh->n_objects), ET_E_WORKSPACE, "scene blob too small");
    ET_CHECK(scratch_bytes >= scene_scratch_bytes(mesh->T, mesh->V), ET_E_WORKSPACE, "scene scratch too small");
    et_scene* sc = new et_scene();
    sc->device = ctx->device;
    try {
      ET_HIP(hipMemsetAsync(&ctx->ctl->err, 0, sizeof(uint32_t), ctx->stream));
      scene_build(sc, mesh, blob, scratch, &ctx->ctl->err, ctx->stream);
    } catch (...) {
      delete sc;
      throw;
    }
    *out = sc;
  });
}

int et_scene_free(et_scene* scene) {
  if (!scene) return ET_E_INVALID;
  delete scene;
  return ET_OK;
}

int et_scene_refit(et_ctx* ctx, et_scene* scene, const float* vertices, double area_ref) {
  return guarded(ctx, [&] {
    check_scene(scene);
    ET_CHECK(vertices || scene->d.V == 0, ET_E_INVALID, "vertices is NULL");
    ET_CHECK(std::isfinite(area_ref), ET_E_INVALID, "area_ref is not finite");
    ET_CHECK(scene->device == ctx->device, ET_E_INVALID, "scene lives on another device");
    scene_refit(scene, vertices, area_ref, &ctx->ctl->err, ctx->stream);
  });
}

int et_scene_get_info(et_ctx* ctx, const et_scene* scene, et_scene_info* info) {
  return guarded(ctx, [&] {
    check_scene(scene);
    ET_CHECK(info, ET_E_INVALID, "info is NULL");
    info->T = scene->d.T;
    info->V = scene->d.V;
    info->n_nodes = scene->n_nodes;
    info->depth = scene->depth;
    info->sah_cost = scene->sah;
    info->build_ms = scene->build_ms;
    info->refit_ms = scene->refit_ms;
  });
}

int et_scene_curvature(et_ctx* ctx, const et_scene* scene, double* C_out, double* G_out) {
  return guarded(ctx, [&] {
    check_scene(scene);
    if (C_out && scene->d.T > 0)
      ET_HIP(hipMemcpyAsync(C_out, scene->d.C, sizeof(double) * scene->d.T, hipMemcpyDeviceToDevice, ctx->stream));
    if (G_out && scene->d.V > 0)
      ET_HIP(hipMemcpyAsync(G_out, scene->d.G, sizeof(double) * scene->d.V, hipMemcpyDeviceToDevice, ctx->stream));
  });
}

int et_workspace_size(et_ctx* ctx, const et_scene* scene, const et_sim_desc* sim, size_t* bytes) {
  return guarded(ctx, [&] {
    ET_CHECK(bytes, ET_E_INVALID, "bytes is NULL");
    validate_sim(sim, scene != nullptr);
    *bytes = plan(scene, sim, std::max<int64_t>(records_upper_bound(sim), 1)).total();
  });
}

int et_trace(et_ctx* ctx, const et_scene* scene, const et_sim_desc* sim, void* ws, size_t ws_bytes,
             const et_paths* paths) {
  return guarded(ctx, [&] {
    ctx->timed = 0;
    trace_impl(ctx, scene, sim, ws, ws_bytes, paths);
  });
}

int et_synthesize(et_ctx* ctx, const et_sim_desc* sim, const et_paths* paths, void* ws, size_t ws_bytes,
                  float* spectra) {
  return guarded(ctx, [&] {
    validate_paths(paths);
    ctx->timed = 0;
    k_set_nrec<<<1, 1, 0, ctx->stream>>>(ctx->ctl, paths->count, paths->capacity);
    ET_HIP(hipGetLastError());
    synth_impl(ctx, sim, paths, ws, ws_bytes, spectra, false);
  });
}

int et_synthesize_noalloc(et_ctx* ctx, const et_sim_desc* sim, const et_paths* paths, float* spectra) {
  return guarded(ctx, [&] {
    validate_paths(paths);
    validate_sim(sim, false);
    validate_readings(sim, paths);
    ET_CHECK(spectra, ET_E_INVALID, "spectra is NULL");
    ctx->timed = 0;
    void* buf = noalloc_scratch(ctx->device);
    k_set_nrec<<<1, 1, 0, ctx->stream>>>(ctx->ctl, paths->count, paths->capacity);
    ET_HIP(hipGetLastError());
    ET_HIP(hipEventRecord(ctx->ev[4], ctx->stream));
    ctx->synth_kernel = synth_run_noalloc(sim, paths, buf, NOALLOC_SCRATCH_BYTES, ctx->ctl, spectra, ctx->stream,
                                          ctx->ev[8], ctx->ev[9]);
    ET_HIP(hipEventRecord(ctx->ev[5], ctx->stream));
    ctx->timed |= TM_SYNTH | TM_SYNTH_K;
  });
}

int et_simulate(et_ctx* ctx, const et_scene* scene, const et_sim_desc* sim, const et_paths* paths, void* ws,
                size_t ws_bytes, float* spectra) {
  return guarded(ctx, [&] {
    check_scene(scene);
    validate_sim(sim, true);
    validate_paths(paths);
    ctx->timed = 0;
    const WsPlan w = plan(scene, sim, std::max<int64_t>(paths->capacity, 1));
    ET_CHECK(ws, ET_E_INVALID, "workspace is NULL");
    ET_CHECK(ws_bytes >= w.trace + w.synth, ET_E_WORKSPACE, "workspace too small for et_simulate");
    trace_impl(ctx, scene, sim, ws, w.trace, paths);
    k_set_nrec<<<1, 1, 0, ctx->stream>>>(ctx->ctl, paths->count, paths->capacity);
    synth_impl(ctx, sim, paths, (char*)ws + w.trace, ws_bytes - w.trace, spectra, true);
  });
}

int et_synthesize_backward(et_ctx* ctx, const et_sim_desc* sim, const et_paths* paths, const float* grad_spectra,
                           void* ws, size_t ws_bytes, double* grad_k, double* grad_rx) {
  return guarded(ctx, [&] {
    validate_sim(sim, false);
    validate_paths(paths);
    validate_readings(sim, paths);
    ET_CHECK(grad_spectra && grad_k && grad_rx, ET_E_INVALID, "gradient pointer is NULL");
    ET_CHECK(!(sim->flags & ET_PATH_PRODUCT), ET_E_UNSUPPORTED, "the adjoint does not support ET_PATH_PRODUCT");
    ET_CHECK(sim->Bk <= 16 && sim->Q * sim->Bk <= 256, ET_E_UNSUPPORTED, "adjoint needs Bk <= 16 and Q*Bk <= 256");
    ET_CHECK(sim->F <= 12288, ET_E_UNSUPPORTED, "adjoint keeps dL/dH of one receiver in LDS: F <= 12288");
    SynthWS sw;
    const size_t need = synth_bwd_ws_layout(sim, std::max<int64_t>(paths->capacity, 1), nullptr, nullptr);
    ET_CHECK(ws && ws_bytes >= need, ET_E_WORKSPACE, "workspace too small for et_synthesize_backward");
    synth_bwd_ws_layout(sim, std::max<int64_t>(paths->capacity, 1), (char*)ws, &sw);
    k_set_nrec<<<1, 1, 0, ctx->stream>>>(ctx->ctl, paths->count, paths->capacity);
    ET_HIP(hipEventRecord(ctx->ev[6], ctx->stream));
    ctx->adjoint_kernel = synth_bwd_run(sim, paths, grad_spectra, sw, ctx->ctl, grad_k, grad_rx, ctx->stream,
                                        ctx->ev[10], ctx->ev[11]);
    ET_HIP(hipEventRecord(ctx->ev[7], ctx->stream));
    ctx->timed = TM_ADJ | TM_ADJ_K;
  });
}

int et_batch_workspace_size(et_ctx* ctx, int32_t J, const et_job* jobs, size_t* bytes) {
  return guarded(ctx, [&] {
    ET_CHECK(J >= 1 && jobs && bytes, ET_E_INVALID, "need J >= 1, jobs and bytes");
    for (int j = 0; j < J; ++j) {
      check_scene(jobs[j].scene);
      validate_sim(jobs[j].sim, true);
    }
    *bytes = batch_fused(J, jobs) ? fused_plan(ctx, J, jobs).total : sequential_bytes(J, jobs);
  });
}

}  // extern "C"

namespace {

// Carves per-job path buffers from the batch workspace (after the shared scratch).
et_paths carve_paths(char*& p, int64_t cap) {
  auto take = [&](size_t b) { char* r = p; p += al(b); return (void*)r; };
  et_paths P;
  P.capacity = cap;
  P.p = (double*)take(sizeof(double) * 3 * cap);
  P.dout = (float*)take(sizeof(float) * 3 * cap);
  P.rtot = (double*)take(sizeof(double) * cap);
  P.tri = (int32_t*)take(sizeof(int32_t) * cap);
  P.mat = (int32_t*)take(sizeof(int32_t) * cap);
  P.ray = (int32_t*)take(sizeof(int32_t) * cap);
  P.bounce = (uint8_t*)take(cap);
  P.flags = (uint8_t*)take(cap);
  P.count = (int64_t*)take(8 * sizeof(int64_t));
  P.prev = (int64_t*)take(sizeof(int64_t) * cap);
  P.rx_vis = (uint64_t*)take(sizeof(uint64_t) * cap);
  return P;
}

// timed: record the phase events (trace, synthesis kernel, adjoint kernel) of a fused batch
void batch_impl(et_ctx* ctx, int32_t J, const et_job* jobs, void* ws, size_t ws_bytes, float* spectra,
                const float* grad_spectra, double* grad_k, double* grad_rx, bool timed = false) {
  ET_CHECK(J >= 1 && jobs, ET_E_INVALID, "need J >= 1 jobs");
  ET_CHECK(spectra, ET_E_INVALID, "spectra is NULL");
  const et_sim_desc* s0 = jobs[0].sim;
  for (int j = 0; j < J; ++j) {
    check_scene(jobs[j].scene);
    validate_sim(jobs[j].sim, true);
    check_materials(jobs[j].scene, jobs[j].sim);
    const et_sim_desc* s = jobs[j].sim;
    ET_CHECK(s->M == s0->M && s->F == s0->F && s->Q == s0->Q && s->Bk == s0->Bk, ET_E_INVALID,
             "jobs of a batch must share M, F, Q and Bk");
    if (grad_spectra)
      ET_CHECK(!(s->flags & ET_PATH_PRODUCT) && s->Bk <= 16 && s->Q * s->Bk <= 256 &&
                   s->F <= 12288,
               ET_E_UNSUPPORTED, "adjoint limits exceeded");
    if (s->flags & ET_PER_RX_VISIBILITY) ET_CHECK(s->M <= 64, ET_E_UNSUPPORTED, "ET_PER_RX_VISIBILITY: M <= 64");
  }
  if (grad_spectra) ET_CHECK(grad_k && grad_rx, ET_E_INVALID, "gradient outputs are NULL");
  size_t need = 0;
  ET_CHECK(et_batch_workspace_size(ctx, J, jobs, &need) == ET_OK, ET_E_INVALID, "batch workspace query failed");
  ET_CHECK(ws && ws_bytes >= need, ET_E_WORKSPACE, "workspace too small for et_simulate_batch");
  ctx->last_count = nullptr;
  if (batch_fused(J, jobs)) {
    const FusedPlan f = fused_plan(ctx, J, jobs);
    const size_t nw = f.waves.size();
    char* base = (char*)ws;
    void* dj = base;
    base += f.tj;
    char* twb = base;
    base += f.tw;
    char* ppb = base;
    base += (nw > 1 ? 2 : 1) * f.pp;
    char* syb = base;
    const size_t MF2 = (size_t)s0->M * s0->F * 2;
    const size_t QB = (size_t)s0->Q * s0->Bk;
    // timed: three event pairs per wave (trace, synthesis kernel, adjoint kernel)
    if (timed)
      while (ctx->wave_ev.size() < 6 * nw) {
        hipEvent_t e;
        ET_HIP(hipEventCreate(&e));
        ctx->wave_ev.push_back(e);
      }
    // Pipelined waves (several waves, and the stream not being captured into a graph): the
    // traces run on the context's second stream, each wave's synthesis on the caller's stream
    // once its trace is done, so that wave w's synthesis runs beside wave w + 1's trace.  Waves
    // alternate between two record buffers and two control blocks; a trace waits until the
    // synthesis that last read its buffer is done, and the caller's stream ends after both.
    hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
    ET_HIP(hipStreamIsCapturing(ctx->stream, &cap_status));
    const bool pipe = nw > 1 && cap_status == hipStreamCaptureStatusNone && !ctx->serial_waves;
    if (pipe && !ctx->aux) ET_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    hipStream_t ts = pipe ? ctx->aux : ctx->stream;   // trace stream
    if (pipe) {
      ET_HIP(hipEventRecord(ctx->pev[0], ctx->stream));
      ET_HIP(hipStreamWaitEvent(ts, ctx->pev[0], 0));
      k_ctl_clear_err<<<1, 1, 0, ts>>>(ctx->ctl2);
    }
    for (size_t wi = 0; wi < nw; ++wi) {
      const Wave& wv = f.waves[wi];
      const et_job* wj = jobs + wv.j0;
      const int64_t cap = std::max<int64_t>(wv.cap, 1);
      const int k = pipe ? (int)(wi & 1) : 0;   // record buffer and control block of this wave
      Ctl* ctl = k ? ctx->ctl2 : ctx->ctl;
      TraceWS tw;
      trace_ws_layout(wv.N, 0, 0, 0, twb, &tw, TUNE_MAX_TRACE_BLOCKS);
      tw.stack_cap = ctx->stack_cap;
      char* pp = ppb + k * f.pp;
      et_paths P = carve_paths(pp, cap);
      SynthBatchWS sw;
      synth_batch_ws_layout(wv.n, wj, cap, ctx->tune, true, syb, &sw);
      hipEvent_t* ev = timed ? ctx->wave_ev.data() + 6 * wi : nullptr;
      if (pipe && wi >= 2) ET_HIP(hipStreamWaitEvent(ts, ctx->pev[3 + k], 0));   // buffer k read by wave wi - 2
      if (ev) ET_HIP(hipEventRecord(ev[0], ts));
      // a control block carries its statistics from its earlier waves
      trace_batch_run(wv.n, wj, dj, &P, tw, ctl, ctx->counting, ctx->tune.trace_blocks, ts,
                      pipe ? wi >= 2 : wi > 0);
      if (ev) ET_HIP(hipEventRecord(ev[1], ts));
      if (pipe) {
        ET_HIP(hipEventRecord(ctx->pev[1 + k], ts));
        ET_HIP(hipStreamWaitEvent(ctx->stream, ctx->pev[1 + k], 0));
      }
      k_set_nrec<<<1, 1, 0, ctx->stream>>>(ctl, P.count, P.capacity);
      int ak = 0;
      const hipEvent_t kev[4] = {ev ? ev[2] : nullptr, ev ? ev[3] : nullptr, ev ? ev[4] : nullptr,
                                 ev ? ev[5] : nullptr};
      ctx->synth_kernel =
          synth_batch_run(wv.n, wj, &P, sw, ctl, spectra + (size_t)wv.j0 * MF2,
                          grad_spectra ? grad_spectra + (size_t)wv.j0 * MF2 : nullptr,
                          grad_spectra ? grad_k + (size_t)wv.j0 * QB : nullptr,
                          grad_spectra ? grad_rx + (size_t)wv.j0 * s0->M * 3 : nullptr, &ak, ev ? kev : nullptr,
                          ctx->stream);
      if (grad_spectra) ctx->adjoint_kernel = ak;
      if (pipe) ET_HIP(hipEventRecord(ctx->pev[3 + k], ctx->stream));
    }
    if (pipe) k_ctl_merge<<<1, 1, 0, ctx->stream>>>(ctx->ctl, ctx->ctl2);
    ctx->waves_timed = timed ? (int32_t)nw : 0;
    ctx->timed = timed ? (TM_WAVES | TM_TRACE | TM_SYNTH_K | (grad_spectra ? TM_ADJ_K : 0u)) : 0u;
    return;
  }
  size_t mx = 0;
  for (int j = 0; j < J; ++j) {
    const int64_t cap = std::max<int64_t>(records_upper_bound(jobs[j].sim), 1);
    mx = std::max(mx, plan(jobs[j].scene, jobs[j].sim, cap).total());
  }
  char* pp = (char*)ws + mx;
  const size_t MF2 = (size_t)s0->M * s0->F * 2;
  for (int j = 0; j < J; ++j) {
    const et_sim_desc* s = jobs[j].sim;
    const int64_t cap = std::max<int64_t>(records_upper_bound(s), 1);
    et_paths P = carve_paths(pp, cap);
    const WsPlan w = plan(jobs[j].scene, s, cap);
    TraceWS tw;
    trace_ws_layout((s->flags & ET_SPECULAR) ? s->N : 0, jobs[j].scene->d.T, jobs[j].scene->d.n_obj,
                    diff_draws_max(s), (char*)ws, &tw);
    tw.stack_cap = ctx->stack_cap;
    trace_run(jobs[j].scene->d, s, &P, tw, ctx->ctl, false, ctx->stream);
    k_set_nrec<<<1, 1, 0, ctx->stream>>>(ctx->ctl, P.count, P.capacity);
    SynthWS sw;
    synth_ws_layout(s, cap, (char*)ws + w.trace, &sw);
    ctx->synth_kernel = synth_run(s, &P, sw, ctx->ctl, spectra + (size_t)j * MF2, ctx->stream);
    if (grad_spectra) {
      SynthWS bw;
      synth_bwd_ws_layout(s, cap, (char*)ws + w.trace + w.synth, &bw);
      ctx->adjoint_kernel = synth_bwd_run(s, &P, grad_spectra + (size_t)j * MF2, bw, ctx->ctl,
                                          grad_k + (size_t)j * s->Q * s->Bk, grad_rx + (size_t)j * s->M * 3,
                                          ctx->stream);
    }
  }
}

}  // namespace

extern "C" {

int et_simulate_batch(et_ctx* ctx, int32_t J, const et_job* jobs, void* ws, size_t ws_bytes, float* spectra,
                      const float* grad_spectra, double* grad_k, double* grad_rx) {
  return guarded(ctx, [&] {
    ctx->timed = 0;
    batch_impl(ctx, J, jobs, ws, ws_bytes, spectra, grad_spectra, grad_k, grad_rx, true);
  });
}

int et_simulate_batch_graph(et_ctx* ctx, int32_t J, const et_job* jobs, void* ws, size_t ws_bytes, float* spectra,
                            const float* grad_spectra, double* grad_k, double* grad_rx) {
  return guarded(ctx, [&] {
    ET_CHECK(ctx->stream, ET_E_INVALID, "graph capture needs a non-null context stream");
    ET_CHECK(J >= 1 && jobs, ET_E_INVALID, "need J >= 1 jobs");
    // the graph bakes in every pointer and scalar: key on all of them
    std::vector<uint64_t> key;
    key.push_back((uint64_t)J);
    key.push_back((uint64_t)(uintptr_t)ws);
    key.push_back((uint64_t)ws_bytes);
    key.push_back((uint64_t)(uintptr_t)spectra);
    key.push_back((uint64_t)(uintptr_t)grad_spectra);
    key.push_back((uint64_t)(uintptr_t)grad_k);
    key.push_back((uint64_t)(uintptr_t)grad_rx);
    key.push_back(((uint64_t)(uint32_t)ctx->tune.synth_wgs << 32) | (uint32_t)ctx->tune.adjoint_wgs);
    key.push_back((uint64_t)(uint32_t)ctx->tune.trace_blocks);
    key.push_back((uint64_t)ctx->tune.wave_rays);
    key.push_back(((uint64_t)(uint32_t)ctx->stack_cap << 1) | (ctx->counting ? 1u : 0u));
    for (int j = 0; j < J; ++j) {
      key.push_back((uint64_t)(uintptr_t)jobs[j].scene);
      const uint64_t* w = reinterpret_cast<const uint64_t*>(jobs[j].sim);
      for (size_t i = 0; i < sizeof(et_sim_desc) / 8; ++i) key.push_back(w[i]);
    }
    if (!ctx->graph_exec || key != ctx->graph_key) {
      if (ctx->graph_exec) { ET_HIP(hipGraphExecDestroy(ctx->graph_exec)); ctx->graph_exec = nullptr; }
      if (ctx->graph) { ET_HIP(hipGraphDestroy(ctx->graph)); ctx->graph = nullptr; }
      ET_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      try {
        batch_impl(ctx, J, jobs, ws, ws_bytes, spectra, grad_spectra, grad_k, grad_rx);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(ctx->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      ET_HIP(hipStreamEndCapture(ctx->stream, &ctx->graph));
      ET_HIP(hipGraphInstantiate(&ctx->graph_exec, ctx->graph, nullptr, nullptr, 0));
      ctx->graph_key = key;
    }
    ctx->timed = 0;
    ET_HIP(hipGraphLaunch(ctx->graph_exec, ctx->stream));
  });
}

// Several simultaneous emitters over one scene and one receiver array: the emitters run as
// the jobs of a batch (fused when all are specular-only) into per-emitter spectra in the
// workspace, which one kernel sums in emitter order.
size_t emitters_batch_bytes(et_ctx* ctx, int32_t S, const et_job* jobs) {
  return batch_fused(S, jobs) ? fused_plan(ctx, S, jobs).total : sequential_bytes(S, jobs);
}

void emitters_check(const et_scene* scene, int32_t S, const et_sim_desc* sims) {
  check_scene(scene);
  ET_CHECK(S >= 1 && sims, ET_E_INVALID, "need S >= 1 emitters");
  for (int e = 0; e < S; ++e) {
    validate_sim(&sims[e], true);
    check_materials(scene, &sims[e]);
    const et_sim_desc& a = sims[0];
    const et_sim_desc& b = sims[e];
    ET_CHECK(b.M == a.M && b.F == a.F && b.f_lo == a.f_lo && b.f_hi == a.f_hi && b.phase_sign == a.phase_sign &&
                 b.rx_pos == a.rx_pos,
             ET_E_INVALID, "emitters must share the receivers (rx_pos), M, F, the frequency grid and the phase sign");
  }
}

int et_emitters_workspace_size(et_ctx* ctx, const et_scene* scene, int32_t S, const et_sim_desc* sims,
                               size_t* bytes) {
  return guarded(ctx, [&] {
    emitters_check(scene, S, sims);
    ET_CHECK(bytes, ET_E_INVALID, "bytes is NULL");
    std::vector<et_job> jobs(S);
    for (int e = 0; e < S; ++e) jobs[e] = et_job{scene, &sims[e]};
    *bytes = al(sizeof(float) * 2 * (size_t)S * sims[0].M * sims[0].F) + emitters_batch_bytes(ctx, S, jobs.data());
  });
}

int et_simulate_emitters(et_ctx* ctx, const et_scene* scene, int32_t S, const et_sim_desc* sims, void* ws,
                         size_t ws_bytes, float* spectra) {
  return guarded(ctx, [&] {
    emitters_check(scene, S, sims);
    ET_CHECK(spectra, ET_E_INVALID, "spectra is NULL");
    std::vector<et_job> jobs(S);
    for (int e = 0; e < S; ++e) jobs[e] = et_job{scene, &sims[e]};
    const size_t per = al(sizeof(float) * 2 * (size_t)S * sims[0].M * sims[0].F);
    const size_t need = per + emitters_batch_bytes(ctx, S, jobs.data());
    ET_CHECK(ws && ws_bytes >= need, ET_E_WORKSPACE, "workspace too small for et_simulate_emitters");
    ctx->timed = 0;
    float* each = (float*)ws;
    batch_impl(ctx, S, jobs.data(), (char*)ws + per, ws_bytes - per, each, nullptr, nullptr, nullptr, false);
    sum_spectra(each, S, (int64_t)2 * sims[0].M * sims[0].F, spectra, ctx->stream);
  });
}

int et_graph_reset(et_ctx* ctx) {
  return guarded(ctx, [&] {
    if (ctx->graph_exec) { ET_HIP(hipGraphExecDestroy(ctx->graph_exec)); ctx->graph_exec = nullptr; }
    if (ctx->graph) { ET_HIP(hipGraphDestroy(ctx->graph)); ctx->graph = nullptr; }
    ctx->graph_key.clear();
  });
}

int et_get_stats(et_ctx* ctx, et_stats* out) {
  int rc = guarded(ctx, [&] {
    ET_CHECK(out, ET_E_INVALID, "stats is NULL");
    ET_HIP(hipStreamSynchronize(ctx->stream));
    Ctl h;
    ET_HIP(hipMemcpy(&h, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->records = h.rec_prev + h.rec_base + h.diff_kept;
    out->specular = h.rec_prev + h.rec_base;
    out->diffraction = h.diff_kept;
    out->segments = h.seg;
    out->shadow_rays = h.shadow;
    out->diff_eligible = h.n_elig;
    out->stack_overflows = h.overflow;
    out->synth_kernel = ctx->synth_kernel;
    if (ctx->last_count) {
      int64_t cnt[4];
      ET_HIP(hipMemcpy(cnt, ctx->last_count, sizeof(cnt), hipMemcpyDeviceToHost));
      out->records = cnt[0];
      out->passive = cnt[0] - cnt[1] - cnt[2];
    }
    float ms = 0;
    if (ctx->timed & TM_WAVES) {
      double t[3];
      wave_phase_ms(ctx, t);
      out->ms_trace = t[0];
      out->ms_synth_kernel = t[1];
      out->ms_adjoint_kernel = t[2];
    } else {
      auto pair = [&](uint32_t bit, int a, int b, double& dst) {
        if ((ctx->timed & bit) && hipEventElapsedTime(&ms, ctx->ev[a], ctx->ev[b]) == hipSuccess) dst = ms;
      };
      pair(TM_TRACE, 0, 1, out->ms_trace);
      pair(TM_SYNTH, 4, 5, out->ms_synth);
      pair(TM_SYNTH_K, 8, 9, out->ms_synth_kernel);
      pair(TM_ADJ, 6, 7, out->ms_adjoint);
      if ((ctx->timed & TM_ADJ_K) && hipEventElapsedTime(&ms, ctx->ev[10], ctx->ev[11]) == hipSuccess)
        out->ms_adjoint_kernel = ms;
    }
    out->adjoint_kernel = ctx->adjoint_kernel;
    uint32_t err = h.err;
    out->status = ET_OK;
    if (err & DEV_ERR_CAPACITY) {
      out->status = ET_E_CAPACITY;
      out->dropped = 1;
    }
    if (err & (DEV_ERR_STACK | DEV_ERR_BUILD)) out->status = ET_E_INTERNAL;
    if (err & (DEV_ERR_INDEX | DEV_ERR_RAYDIR)) out->status = ET_E_INVALID;
    // clear the deferred error word for the next call
    ET_HIP(hipMemset(&ctx->ctl->err, 0, sizeof(uint32_t)));
  });
  if (rc == ET_OK && out->status != ET_OK) {
    ctx->last_error = "deferred device-side error";
    return out->status;
  }
  return rc;
}

namespace {
void check_time_shape(int32_t M, int32_t n_t) {
  ET_CHECK(M >= 1, ET_E_INVALID, "need M >= 1 receivers");
  ET_CHECK(n_t >= 1 && n_t <= (1 << 22) && (n_t & (n_t - 1)) == 0, ET_E_INVALID,
           "n_t must be a power of two in [1, 2^22]");
}
}  // namespace

int et_impulse_response_workspace_size(int32_t M, int32_t n_t, size_t* bytes) {
  try {
    if (!bytes) return ET_E_INVALID;
    check_time_shape(M, n_t);
    *bytes = impulse_ws_bytes(M, n_t);
    return ET_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

int et_impulse_response(et_ctx* ctx, int32_t M, int32_t F, double f_lo, double f_hi, int32_t phase_sign,
                        const float* spectra, int32_t n_t, void* ws, size_t ws_bytes, float* h, double* dt_out) {
  return guarded(ctx, [&] {
    check_time_shape(M, n_t);
    ET_CHECK(F >= 2 && F <= n_t, ET_E_INVALID, "need 2 <= F <= n_t");
    ET_CHECK(std::isfinite(f_lo) && std::isfinite(f_hi) && f_hi > f_lo && f_lo >= 0, ET_E_INVALID,
             "frequency grid must satisfy 0 <= f_lo < f_hi");
    ET_CHECK(phase_sign == 1 || phase_sign == -1, ET_E_INVALID, "phase_sign must be +1 or -1");
    ET_CHECK(spectra && h, ET_E_INVALID, "spectra or h is NULL");
    ET_CHECK(ws && ws_bytes >= impulse_ws_bytes(M, n_t), ET_E_WORKSPACE, "workspace too small for et_impulse_response");
    const double df = (f_hi - f_lo) / (double)(F - 1);
    impulse_run(M, F, f_lo, df, phase_sign, spectra, n_t, ws, h, ctx->stream);
    if (dt_out) *dt_out = 1.0 / ((double)n_t * df);
  });
}

int et_receiver_signal_workspace_size(int32_t M, int32_t n_t, int64_t L, size_t* bytes) {
  try {
    if (!bytes) return ET_E_INVALID;
    check_time_shape(M, n_t);
    if (L < 1 || conv_length(n_t, L) > ((int64_t)1 << 23)) return ET_E_INVALID;
    *bytes = signal_ws_bytes(M, n_t, L);
    return ET_OK;
  } catch (const Error& e) {
    return e.code;
  }
}

int et_receiver_signal(et_ctx* ctx, int32_t M, int32_t n_t, const float* h, int64_t L, const float* s_e, double dt,
                       void* ws, size_t ws_bytes, float* out) {
  return guarded(ctx, [&] {
    check_time_shape(M, n_t);
    ET_CHECK(L >= 1 && conv_length(n_t, L) <= ((int64_t)1 << 23), ET_E_INVALID, "need L >= 1 and n_t + L - 1 <= 2^23");
    ET_CHECK(std::isfinite(dt) && dt > 0, ET_E_INVALID, "dt must be positive");
    ET_CHECK(h && s_e && out, ET_E_INVALID, "h, s_e or out is NULL");
    ET_CHECK(ws && ws_bytes >= signal_ws_bytes(M, n_t, L), ET_E_WORKSPACE, "workspace too small for et_receiver_signal");
    signal_run(M, n_t, h, L, s_e, dt, ws, out, ctx->stream);
  });
}

int et_eq_directions_workspace_size(int64_t N, size_t* bytes) {
  if (!bytes || N < 1 || N > ((int64_t)1 << 28)) return ET_E_INVALID;
  *bytes = eq_ws_bytes(eq_plan(N));
  return ET_OK;
}

int et_eq_directions(et_ctx* ctx, int64_t N, double cone_half_angle, void* ws, size_t ws_bytes, float* dirs,
                     int64_t capacity, int64_t* count) {
  return guarded(ctx, [&] {
    ET_CHECK(N >= 1 && N <= ((int64_t)1 << 28), ET_E_INVALID, "need 1 <= N <= 2^28");
    ET_CHECK(std::isfinite(cone_half_angle) && cone_half_angle > 0 && cone_half_angle <= M_PI, ET_E_INVALID,
             "cone half-angle must lie in (0, pi]");
    ET_CHECK(count, ET_E_INVALID, "count is NULL");
    ET_CHECK(dirs || capacity == 0, ET_E_INVALID, "dirs is NULL");
    ET_CHECK(capacity >= 0, ET_E_INVALID, "negative capacity");
    const EqPlan p = eq_plan(N);
    ET_CHECK(ws && ws_bytes >= eq_ws_bytes(p), ET_E_WORKSPACE, "workspace too small for et_eq_directions");
    const int64_t c = eq_count(p, cone_half_angle, ws, ctx->stream);
    *count = c;
    if (!dirs) return;
    ET_CHECK(c <= capacity, ET_E_CAPACITY, "more directions than capacity");
    eq_points(p, c, ws, dirs, ctx->stream);
  });
}

int et_get_tuning(et_ctx* ctx, et_tuning* out) {
  return guarded(ctx, [&] {
    ET_CHECK(out, ET_E_INVALID, "tuning is NULL");
    std::memset(out, 0, sizeof(*out));
    out->synth_wgs = ctx->tune.synth_wgs;
    out->adjoint_wgs = ctx->tune.adjoint_wgs;
    out->trace_blocks = ctx->tune.trace_blocks;
    out->wave_rays = (int32_t)ctx->tune.wave_rays;
  });
}

int et_set_tuning(et_ctx* ctx, const et_tuning* t) {
  return guarded(ctx, [&] {
    ET_CHECK(t, ET_E_INVALID, "tuning is NULL");
    auto in = [](int32_t v, int32_t hi) { return v >= 64 && v <= hi; };
    ET_CHECK(in(t->synth_wgs, TUNE_MAX_WGS) && in(t->adjoint_wgs, TUNE_MAX_WGS) &&
                 in(t->trace_blocks, TUNE_MAX_TRACE_BLOCKS),
             ET_E_INVALID, "tuning values must lie in 64 .. 4096");
    ET_CHECK(t->wave_rays == 0 || t->wave_rays >= MIN_WAVE_RAYS, ET_E_INVALID, "wave_rays must be 0 or >= 1024");
    ctx->tune.synth_wgs = t->synth_wgs;
    ctx->tune.adjoint_wgs = t->adjoint_wgs;
    ctx->tune.trace_blocks = t->trace_blocks;
    ctx->tune.wave_rays = t->wave_rays == 0 ? BatchTune{}.wave_rays : (int64_t)t->wave_rays;
  });
}

int et_autotune_batch(et_ctx* ctx, int32_t J, const et_job* jobs, void* ws, size_t ws_bytes, float* spectra,
                      const float* grad_spectra, double* grad_k, double* grad_rx, et_tuning* out) {
  return guarded(ctx, [&] {
    ET_CHECK(out, ET_E_INVALID, "tuning is NULL");
    ET_CHECK(J >= 1 && jobs, ET_E_INVALID, "need J >= 1 jobs");
    for (int j = 0; j < J; ++j) {
      check_scene(jobs[j].scene);
      validate_sim(jobs[j].sim, true);
    }
    ET_CHECK(batch_fused(J, jobs), ET_E_UNSUPPORTED, "autotuning applies to fused (specular-only) batches");
    const int32_t cw[5] = {1024, 2048, 4096, 8192, 16384};
    const int32_t cb[5] = {1024, 2048, 4096, 6144, 8192};
    // each phase is timed alone: the job waves run in order, not pipelined over two streams
    struct Serial {
      et_ctx* c;
      ~Serial() { c->serial_waves = false; }
    } serial{ctx};
    ctx->serial_waves = true;
    auto run = [&](double* t) {
      batch_impl(ctx, J, jobs, ws, ws_bytes, spectra, grad_spectra, grad_k, grad_rx, true);
      ET_HIP(hipStreamSynchronize(ctx->stream));
      wave_phase_ms(ctx, t);
    };
    double t[3], best[3] = {INFINITY, INFINITY, INFINITY};
    BatchTune pick = ctx->tune;
    run(t);   // warm-up
    for (int i = 0; i < 5; ++i) {
      ctx->tune.synth_wgs = ctx->tune.adjoint_wgs = cw[i];
      ctx->tune.trace_blocks = cb[i];
      run(t);
      if (t[0] < best[0]) { best[0] = t[0]; pick.trace_blocks = cb[i]; }
      if (t[1] < best[1]) { best[1] = t[1]; pick.synth_wgs = cw[i]; }
      if (grad_spectra && t[2] < best[2]) { best[2] = t[2]; pick.adjoint_wgs = cw[i]; }
    }
    ctx->tune = pick;
    run(t);
    std::memset(out, 0, sizeof(*out));
    out->synth_wgs = pick.synth_wgs;
    out->adjoint_wgs = pick.adjoint_wgs;
    out->trace_blocks = pick.trace_blocks;
    out->wave_rays = (int32_t)pick.wave_rays;
    out->ms_trace = t[0];
    out->ms_synth = t[1];
    out->ms_adjoint = t[2];
  });
}

int et_set_counting(et_ctx* ctx, int enable) {
  if (!ctx) return ET_E_INVALID;
  ctx->counting = enable != 0;
  return ET_OK;
}

int et_set_stack_limit(et_ctx* ctx, int32_t entries) {
  return guarded(ctx, [&] {
    ET_CHECK(entries >= 0 && entries <= TRAV_STACK, ET_E_INVALID, "stack limit must be in [0, 64]");
    ctx->stack_cap = entries == 0 ? TRAV_STACK : entries;
  });
}

int et_get_counters(et_ctx* ctx, et_counters* out) {
  return guarded(ctx, [&] {
    ET_CHECK(out, ET_E_INVALID, "counters is NULL");
    ET_HIP(hipStreamSynchronize(ctx->stream));
    Ctl h;
    ET_HIP(hipMemcpy(&h, ctx->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    out->nodes_closest = h.cnt[0];
    out->tris_closest = h.cnt[1];
    out->nodes_any = h.cnt[2];
    out->tris_any = h.cnt[3];
    out->rays_closest = h.cnt[4];
    out->rays_any = h.cnt[5];
  });
}

}  // extern "C"
