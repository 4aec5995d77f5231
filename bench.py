"""Benchmark of the echo-simulation hot path on one MI355X.

Workload (room scene): a 10x8x3 m room with 100 boxes and 100 cylinders (193,212
triangles, 16 materials x 8 bands), 2^20 rays over the frontal hemisphere, <= 4 reflection
points per ray, 32 receivers in a 12 cm planar aperture, 4096 bins over 20-100 kHz, 65,536
curvature-importance diffraction samples.  Seeded synthetic inputs (no dataset).

One step = one et_simulate call: ray init, 4 bounces of closest-hit + line-of-sight
traversal, diffraction sampling and filtering, synthesis of every record into the 32 x
4096 complex spectra.  The scene (BVH, curvature) is built once before timing, like the
paper's offline pre-processing.

Printed: one JSON line.  value = closest-hit segments (ray-bounces, hits plus the final
misses) per second of the whole step, in millions.  Extra keys give the tracing-stage and
synthesis-stage throughputs (the metric's second half, G(record.receiver.bin)/s), the
roofline of the dominant kernel and the FP64 oracle on the host cores as a baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays·bounces/s + G(hit·mic·bin)/s synthesis; batched fwd+adjoint vs plain"
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_F16_TFLOPS = 2500.0    # dense fp16 matrix cores: the synthesis products' operand type
PEAK_MFMA_F32_TFLOPS = 157.3     # dense fp32 matrix cores: the ceiling of an fp32-operand contraction
SYNTH_FLOP_PER_TERM = 8          # one complex multiply-accumulate (4 mul + 4 add)
ADJ_FLOP_PER_TERM = 16           # two: the band sum conj(g) T and the frequency-weighted sum
# executed on the matrix cores: every fp32 factor is split into two f16 halves and each real
# product taken as three half products (hi hi, hi lo, lo hi); a complex multiply-accumulate
# is four real products, so 12 half products of 2 flop each per term (twice that in the adjoint)
SYNTH_EXEC_FLOP_PER_TERM = 24
ADJ_EXEC_FLOP_PER_TERM = 48
FLOP_PER_MFMA_F16 = 2 * 16 * 16 * 32   # v_mfma_f32_16x16x32_f16
NODE_BYTES, TRI_BYTES, RAY_IO_BYTES = 64, 48, 128
# traversal arithmetic per unit, one VALU lane operation each (an FMA counts once): a node visit
# is the slab test of both child boxes (per box 6 FMA, 6 min/max per axis, 4 for the entry and
# exit reductions, the widening multiply, 1 min and 1 compare); a triangle test is the watertight
# test (9 translations, 6 shears, 6 for the edge functions, 6 sign tests, 2 for the determinant,
# 3 scalings, 3 for T, 1 division); a ray its set-up (reciprocals, axis choice, shear constants)
NODE_OPS, TRI_OPS, RAY_OPS = 38, 36, 25
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # lane operations per second: 256 CUs x 4 SIMDs x 16 lanes


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rays", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=32768, help="rays of the oracle's bounded sample (about 10 s of host work)")
    ap.add_argument("--profile-only", action="store_true", help="a few steps, no baselines (for rocprofv3)")
    ap.add_argument("--profile-workload", choices=("room", "foliage"), default="room",
                    help="the step --profile-only runs: the room (with one adjoint call) or the foliage scene")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="skip the dynamic-scene and other-workload legs (a kernel trace then holds only the "
                         "room step's synthesis launches)")
    ap.add_argument("--batch-poses", type=int, default=256, help="poses of the batch leg (0 with 0 scenes skips it)")
    ap.add_argument("--batch-scenes", type=int, default=64)
    ap.add_argument("--batch-rays", type=int, default=1 << 18)
    return ap.parse_args()


def source_hash(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def counter_for(kernel: str, key: str = "bytes_per_launch"):
    """A per-launch figure from rocprofv3 counters (HBM bytes, matrix-core instructions), if
    taken on the current source of the kernel; None otherwise."""
    f = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    e = d.get(kernel)
    if not e or key not in e:
        return None
    src = os.path.join(ROOT, "paper_2602_19652_amd", "csrc", e["source"])
    if source_hash(src) != e["source_sha"]:
        return None
    return e[key]


def traffic_for(kernel: str):
    return counter_for(kernel, "bytes_per_launch")


def mfma_roofline(kname: str, terms: int, ms: float, flop_per_term: int, exec_flop_per_term: int) -> dict:
    """Roofline of a synthesis kernel on the fp16 matrix cores: algorithmic flop (the complex
    multiply-accumulates of the plain sum) and executed flop (from the matrix-core instruction
    counter when it was taken on this source, else from the kernel's structure)."""
    alg = terms * flop_per_term
    achieved = alg / (ms * 1e-3) / 1e12
    n_mfma = counter_for(kname, "mfma_insts_per_launch")
    exec_flop = n_mfma * FLOP_PER_MFMA_F16 if n_mfma else terms * exec_flop_per_term
    exec_tf = exec_flop / (ms * 1e-3) / 1e12
    return {"kernel": kname, "bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_F16_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_MFMA_F16_TFLOPS, "traffic": traffic_for(kname), "kernel_ms": ms,
            "algorithmic_flop_per_launch": alg,
            "per_unit": f"{flop_per_term} flop per (visible record, receiver, bin)",
            "executed": {"flop_per_launch": exec_flop, "achieved": exec_tf, "frac": exec_tf / PEAK_MFMA_F16_TFLOPS,
                         "source": "SQ_INSTS_MFMA x 16384" if n_mfma else
                         f"{exec_flop_per_term} flop per term (three f16 half products per real product)"},
            "algorithmic_over_f32_mfma_peak": achieved / PEAK_MFMA_F32_TFLOPS}


def host_cpu():
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def _oracle_sample(O, scene, sim, n_rays: int, M: int, F: int, seg_total: int, terms_total: int, seed: int):
    g = np.random.Generator(np.random.PCG64(seed))
    sub = np.sort(g.choice(len(sim["ray_dirs"]), n_rays, replace=False))
    t0 = time.perf_counter()
    rec = O.trace(scene, sim, dirs=sim["ray_dirs"][sub], certify=False)
    t1 = time.perf_counter()
    bins = np.arange(0, F, 16, dtype=np.int32)        # 1/16 of the bins, all receivers
    O.synth(rec, sim, bins=bins)
    t2 = time.perf_counter()
    seg = int(rec["nseg"].sum())
    terms = len(rec["rtot"]) * M * len(bins)
    t_seg = (t1 - t0) / max(seg, 1)
    t_term = (t2 - t1) / max(terms, 1)
    job_s = seg_total * t_seg + terms_total * t_term
    return {"value": seg_total / job_s / 1e6,
            "sample": f"{n_rays} seeded rays traced by brute force ({seg} segments, {t1 - t0:.1f} s) and their "
                      f"{len(rec['rtot'])} records synthesised on every 16th bin ({terms:.3g} terms, {t2 - t1:.1f} s); "
                      f"whole-job time extrapolated linearly in segments and terms",
            "sec_per_segment": t_seg, "sec_per_term": t_term}


def cpu_baseline(scene, sim, n_rays: int, M: int, F: int, seg_total: int, terms_total: int):
    """The oracle (FP64 brute force, OpenMP over rays and receivers) on a bounded sample of
    the same workload, scaled to the whole job: time per segment (trace, with the per-hit
    line-of-sight rays) and per term (synthesis) measured on the sample, then the job's
    segment and term counts.  Once with every host thread the process may use, once on one
    thread over an eighth of the sample."""
    import oracle as O
    L = O.lib()
    model, avail = host_cpu()
    L.omp_set_num_threads(avail)
    threads = int(L.omp_get_max_threads())
    full = _oracle_sample(O, scene, sim, n_rays, M, F, seg_total, terms_total, 4242)
    L.omp_set_num_threads(1)
    one = _oracle_sample(O, scene, sim, max(n_rays // 8, 256), M, F, seg_total, terms_total, 4243)
    L.omp_set_num_threads(avail)
    one["cores"] = 1
    return dict(full, unit="Mrays·bounces/s", cores=threads, kind="oracle", host_cpu=model, one_core=one)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library runs each pose, batch and "
              f"adjoint on a single GPU and does not shard across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2602_19652_amd as et
    import workloads as W

    assert torch.cuda.is_available(), "bench needs the GPU"
    torch.cuda.set_device(0)
    if args.profile_only and args.profile_workload == "foliage":
        scene, sim = W.foliage_scene()
        sim["area_ref"] = W.median_triangle_area(scene)
    else:
        scene, sim = W.room_scene(n_rays=args.rays)
    ctx = et.Context(0)
    sc = et.Scene(ctx, scene, area_ref=sim["area_ref"])
    info = sc.info()
    s = et.Sim(sim)
    P = et.Paths(s.capacity())
    ws = et.Workspace()
    out = torch.empty(s.M, s.F, 2, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        et.simulate(ctx, sc, s, paths=P, ws=ws, out=out)
    torch.cuda.synchronize()
    st = ctx.stats()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        et.simulate(ctx, sc, s, paths=P, ws=ws, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    st = ctx.stats()
    seg = st.segments
    n_rec = st.records
    n_vis = int((P.flags[:n_rec] & 1).sum().item())      # blocked records contribute nothing
    terms = n_vis * s.M * s.F
    if args.profile_only:
        if args.profile_workload == "room":
            # one adjoint call over the step's paths, for the counter runs
            gen = torch.Generator(device="cuda").manual_seed(2024)
            et.synthesize_backward(ctx, s, P, torch.randn(s.M, s.F, dtype=torch.complex64, device="cuda",
                                                          generator=gen), ws=ws)
            torch.cuda.synchronize()
        # calibration for hardware byte counters: one plain device copy of a known size
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_only": True, "ms_per_step": ms_step, "segments": seg, "records": n_rec,
                          "calibration_copy_bytes": a.numel()}))
        return

    # stage timings on the same stream: tracing (with diffraction) and synthesis alone
    reps = max(3, args.steps)
    e0.record(stream)
    for _ in range(reps):
        et.trace(ctx, sc, s, paths=P, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_trace = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        et.synthesize(ctx, s, P, ws=ws, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_synth = e0.elapsed_time(e1) / reps
    kern = ctx.stats().synth_kernel
    # the synthesis kernel alone: HIP events the library records around its launch, on the same stream
    ms_synth_kernel = 0.0
    for _ in range(reps):
        et.synthesize(ctx, s, P, ws=ws, out=out)
        ms_synth_kernel += ctx.stats().ms_synth_kernel / reps

    # time domain of the step's spectra: impulse responses at fs = n_t df (16384 samples, 320 kHz)
    # and received signals for a 2 ms 20-100 kHz chirp
    Hc = torch.view_as_complex(out)
    n_t = 16384
    td_ws = et.Workspace()
    h_t, dt = et.impulse_response(ctx, s, Hc, n_t, ws=td_ws)
    L_call = int(round(2e-3 / dt))
    tt = torch.arange(L_call, dtype=torch.float64, device="cuda") * dt
    chirp = (torch.sin(2 * math.pi * (20e3 * tt + 0.5 * (80e3 / (L_call * dt)) * tt * tt))
             * torch.hann_window(L_call, periodic=False, dtype=torch.float64, device="cuda")).float()
    sig_ws = et.Workspace()
    et.receiver_signal(ctx, h_t, chirp, dt, ws=sig_ws)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        et.impulse_response(ctx, s, Hc, n_t, ws=td_ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_ir = e0.elapsed_time(e1) / reps
    e0.record(stream)
    for _ in range(reps):
        et.receiver_signal(ctx, h_t, chirp, dt, ws=sig_ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_sig = e0.elapsed_time(e1) / reps
    del td_ws, sig_ws

    # per-mesh diffraction allocation (Sec. III-D): 1024 candidates for each eligible mesh
    sim_pm = dict(sim, diff_K=1024, diff_per_mesh=True, diff_max_meshes=int(scene["n_objects"]))
    s_pm = et.Sim(sim_pm, flags=et.ET_DIFFRACTION | et.ET_DIFF_PER_MESH)
    P_pm = et.Paths(s_pm.capacity())
    et.trace(ctx, sc, s_pm, paths=P_pm, ws=ws)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        et.trace(ctx, sc, s_pm, paths=P_pm, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_pm = e0.elapsed_time(e1) / reps
    st_pm = ctx.stats()
    draws_pm = int(P_pm.count[2].item())
    del P_pm, s_pm

    # EQ ray set of the step's size over the whole sphere (collar table, count, centres)
    eq_ws = et.Workspace()
    et.eq_directions(ctx, s.desc.N, ws=eq_ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        et.eq_directions(ctx, s.desc.N, ws=eq_ws)
    torch.cuda.synchronize()
    ms_eq = (time.perf_counter() - t0) * 1e3 / reps
    del eq_ws

    # adjoint over the fixed paths of the step (32 receivers x 4096 bins): seeded dL/dconj(H)
    gen = torch.Generator(device="cuda").manual_seed(2024)
    gH = torch.randn(s.M, s.F, dtype=torch.complex64, device="cuda", generator=gen)
    et.synthesize_backward(ctx, s, P, gH, ws=ws)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        et.synthesize_backward(ctx, s, P, gH, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_adj = e0.elapsed_time(e1) / reps
    ms_adj_kernel = 0.0
    for _ in range(reps):
        et.synthesize_backward(ctx, s, P, gH, ws=ws)
        sta = ctx.stats()
        ms_adj_kernel += sta.ms_adjoint_kernel / reps
    adj_kern = sta.adjoint_kernel

    # achievable HBM bandwidth: a plain 1 GiB device copy (bytes read + written over its time)
    src_b = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
    dst_b = torch.empty_like(src_b)
    dst_b.copy_(src_b)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        dst_b.copy_(src_b)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src_b.numel() / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del src_b, dst_b

    # traversal work counters (separate counting pass, outside the timed region)
    ctx.set_counting(True)
    et.trace(ctx, sc, s, paths=P, ws=ws)
    cnt = ctx.counters()
    ctx.set_counting(False)

    dynamic = None if args.no_extra_legs else dynamic_leg(ctx, et, W, scene, sim, sc, s, P, ws, out, reps)
    pipelined = None if args.no_extra_legs else pipelined_leg(ctx, et, sc, s, P, ws, out, reps)
    other_configs = None if args.no_extra_legs else configs_leg(ctx, et, W, reps)

    adj_tflops = terms * ADJ_FLOP_PER_TERM / (ms_adj_kernel * 1e-3) / 1e12
    # kernel instantiation names as the profiler reports them
    adj_name = adj_kernel_name(s) if adj_kern == 1 else "k_synth_bwd<false>"
    if ms_synth >= ms_trace and kern == 1:
        roof = mfma_roofline(fwd_kernel_name(s), terms, ms_synth_kernel, SYNTH_FLOP_PER_TERM,
                             SYNTH_EXEC_FLOP_PER_TERM)
    else:
        roof = trace_roofline(cnt, ms_trace)
    adj_roof = (mfma_roofline(adj_name, terms, ms_adj_kernel, ADJ_FLOP_PER_TERM, ADJ_EXEC_FLOP_PER_TERM)
                if adj_kern == 1 else None)
    line = {
        "metric": METRIC,
        "value": seg / (ms_step * 1e-3) / 1e6,
        "unit": "Mrays·bounces/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64+f16x3", "data": "synthetic",
        "config": {"workload": "room scene: 10x8x3 m room + 100 boxes + 100 cylinders (193,212 tris), 2^20 rays, "
                               "<=4 reflection points, 32 mics, 4096 bins 20-100 kHz, 65,536 diffraction samples",
                   "rays": s.desc.N, "triangles": info.T, "receivers": s.M, "bins": s.F, "max_bounces": s.desc.max_bounces,
                   "diff_samples": s.desc.diff_K},
        "segments": seg, "records": n_rec, "visible_records": n_vis, "shadow_rays": st.shadow_rays,
        "trace_ms": ms_trace, "trace_mrays_bounces_per_s": seg / (ms_trace * 1e-3) / 1e6,
        "synth_ms": ms_synth, "synth_kernel_ms": ms_synth_kernel,
        "synth_g_terms_per_s": terms / (ms_synth * 1e-3) / 1e9, "synth_kernel": kern,
        "time_domain": {"workload": f"impulse responses of the step's spectra, n_t = {n_t} samples at "
                                    f"{1 / dt / 1e3:.1f} kHz; received signals for a {L_call}-sample 20-100 kHz chirp",
                        "impulse_ms": ms_ir, "signal_ms": ms_sig},
        "diffraction_per_mesh": {"workload": "room scene, diffraction only, 1024 candidates per eligible mesh",
                                 "ms": ms_pm, "kept": draws_pm, "eligible_triangles": st_pm.diff_eligible},
        "ray_set": {"workload": f"EQ sphere partition, {s.desc.N} region centres (two calls: count, then centres)",
                    "wall_ms": ms_eq},
        "adjoint": {"workload": "fixed paths of the step, 32 receivers x 4096 bins, seeded dL/dconj(H)",
                    "ms": ms_adj, "kernel_ms": ms_adj_kernel, "kernel": adj_kern,
                    "g_terms_per_s": terms / (ms_adj * 1e-3) / 1e9,
                    "kernel_tflops_algorithmic": adj_tflops, "roofline": adj_roof},
        "bvh": {"nodes": info.n_nodes, "depth": info.depth, "sah_cost": info.sah_cost, "build_ms": info.build_ms},
        "dynamic_scene": dynamic,
        "pipelined_poses": pipelined,
        "other_configs": other_configs,
        "traversal": {"nodes_per_segment": (cnt.nodes_closest) / max(cnt.rays_closest, 1),
                      "tris_per_segment": cnt.tris_closest / max(cnt.rays_closest, 1),
                      "nodes_per_shadow_ray": cnt.nodes_any / max(cnt.rays_any, 1),
                      "roofline": trace_roofline(cnt, ms_trace), "achievable_hbm_GBs": copy_gbs},
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(scene, sim, args.cpu_rays, s.M, s.F, seg, terms)
    if args.batch_poses + args.batch_scenes > 0:
        del P, ws
        torch.cuda.empty_cache()
        line["batched"] = batched_leg(ctx, args)
    print(json.dumps(line))


def bands_on_groups(F: int, bands, g: int, whole: bool) -> bool:
    """Every band edge (of each band count in `bands`) on a multiple of 64 g bins, and with
    `whole` the bins a multiple of 64 g: the grouped-row instantiations of the synthesis kernels."""
    K1 = F // 64
    if whole and K1 % g:
        return False
    return all(k1 % g == 0 or (k1 * 64 * B) // F == ((k1 - 1) * 64 * B) // F
               for B in bands if B for k1 in range(1, K1))


def fold_mode(F: int, bands) -> int:
    """How the synthesis kernels fold the band factor: 8 (band edges on 512 bins), 4 (256), 0."""
    return 8 if bands_on_groups(F, bands, 8, True) else 4 if bands_on_groups(F, bands, 4, True) else 0


def fwd_kernel_name(s) -> str:
    """The forward matrix-core kernel's instantiation, as the profiler names it."""
    Bd = s.desc.Bd if s.desc.directivity else 0
    return f"k_synth_mfma<false, {'true' if s.F // 64 <= 32 else 'false'}, {fold_mode(s.F, [s.desc.Bk, Bd])}>"


def adj_kernel_name(s) -> str:
    return f"k_synth_bwd_mfma<false, {'true' if s.F // 64 <= 32 else 'false'}, {fold_mode(s.F, [s.desc.Bk])}>"


def trace_roofline(cnt, ms_trace: float, traffic_key: str = "k_bounce<false, false, false>") -> dict:
    """The traversal against HBM bandwidth: the node, triangle and ray bytes its visits touch
    (counting pass) over the trace time of the step.  Caches serve most of them, so they can
    exceed what HBM delivers; the measured HBM bytes of the bounce kernel are `traffic`.  The
    arithmetic of the same visits against the vector-ALU lane rate is reported beside it."""
    nodes, tris = cnt.nodes_closest + cnt.nodes_any, cnt.tris_closest + cnt.tris_any
    rays = cnt.rays_closest + cnt.rays_any
    trav_bytes = nodes * NODE_BYTES + tris * TRI_BYTES + rays * RAY_IO_BYTES
    gbs = trav_bytes / (ms_trace * 1e-3) / 1e9
    ops = nodes * NODE_OPS + tris * TRI_OPS + rays * RAY_OPS
    tops = ops / (ms_trace * 1e-3) / 1e12
    return {"kernel": "k_bounce<false, false, false>", "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": counter_for(traffic_key),
            "algorithmic_bytes": trav_bytes,
            "per_unit": f"{NODE_BYTES} B per node visit, {TRI_BYTES} B per triangle test, {RAY_IO_BYTES} B per ray "
                        f"(closest-hit and line-of-sight traversals)",
            "alu": {"achieved": tops, "peak": PEAK_VALU_TOPS, "unit": "Top/s", "frac": tops / PEAK_VALU_TOPS,
                    "algorithmic_ops": ops,
                    "per_unit": f"{NODE_OPS} ops per node visit, {TRI_OPS} per triangle test, {RAY_OPS} per ray"}}


def configs_leg(ctx, et, W, reps):
    """The step on the other single-pose workloads: the tiny wall + sphere scene (16,384
    rays, <=3 reflection points, 2 receivers, 1024 bins) and the foliage scene (1M
    triangles, 2^22 rays, <=6 reflection points, 2 receivers with directivity, 8192 bins)."""
    import torch
    res = {}
    for name, (scene_c, sim_c) in (("tiny", W.tiny_scene()), ("foliage", W.foliage_scene())):
        sc_c = et.Scene(ctx, scene_c, area_ref=W.median_triangle_area(scene_c))
        s_c = et.Sim(sim_c)
        P_c = et.Paths(s_c.capacity())
        ws_c = et.Workspace()
        out_c = torch.empty(s_c.M, s_c.F, 2, dtype=torch.float32, device="cuda")
        et.simulate(ctx, sc_c, s_c, paths=P_c, ws=ws_c, out=out_c)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            et.simulate(ctx, sc_c, s_c, paths=P_c, ws=ws_c, out=out_c)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        st = ctx.stats()
        n_vis = int((P_c.flags[:st.records] & 1).sum().item())
        terms_c = n_vis * s_c.M * s_c.F
        # traversal work of the same trace (separate counting pass, outside the timed region)
        ctx.set_counting(True)
        et.trace(ctx, sc_c, s_c, paths=P_c, ws=ws_c)
        cnt = ctx.counters()
        ctx.set_counting(False)
        if st.ms_synth_kernel > st.ms_trace and st.synth_kernel == 1:
            roof = mfma_roofline(fwd_kernel_name(s_c), terms_c, st.ms_synth_kernel, SYNTH_FLOP_PER_TERM,
                                 SYNTH_EXEC_FLOP_PER_TERM)
        else:
            roof = trace_roofline(cnt, st.ms_trace, f"k_bounce<false, false, false> [{name}]")
        res[name] = {"triangles": len(scene_c["tris"]), "rays": s_c.desc.N, "receivers": s_c.M, "bins": s_c.F,
                     "ms_per_step": ms, "mrays_bounces_per_s": st.segments / (ms * 1e-3) / 1e6,
                     "trace_ms": st.ms_trace, "synth_kernel_ms": st.ms_synth_kernel, "synth_kernel": st.synth_kernel,
                     "g_terms_per_s": terms_c / (ms * 1e-3) / 1e9, "build_ms": sc_c.info().build_ms,
                     "traversal": {"nodes_per_segment": cnt.nodes_closest / max(cnt.rays_closest, 1),
                                   "tris_per_segment": cnt.tris_closest / max(cnt.rays_closest, 1),
                                   "nodes_per_shadow_ray": cnt.nodes_any / max(cnt.rays_any, 1)},
                     "roofline": roof}
        del P_c, ws_c, sc_c
        torch.cuda.empty_cache()
    return res


def dynamic_leg(ctx, et, W, scene, sim, sc, s, P, ws, out, reps):
    """Animated room: one frame in which the 200 objects turn and move (every fourth also
    deforms).  The tree is refitted (et_scene_refit) or rebuilt; the step then runs on it."""
    import torch
    a_ref = sim["area_ref"]
    V0 = torch.as_tensor(scene["vertices"]).cuda()
    V1 = torch.as_tensor(W.animate_objects(scene, W.rng(31))).cuda()
    dev_ms, n = 0.0, 2 * reps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n):
        sc.refit(V1 if i % 2 == 0 else V0, area_ref=a_ref)
        dev_ms += sc.info().refit_ms
    wall_ms = (time.perf_counter() - t0) * 1e3 / n
    sc.refit(V1, area_ref=a_ref)
    refit_sah = sc.info().sah_cost
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def step_ms(scn):
        et.simulate(ctx, scn, s, paths=P, ws=ws, out=out)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            et.simulate(ctx, scn, s, paths=P, ws=ws, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_refitted = step_ms(sc)
    moved = dict(scene, vertices=V1.cpu().numpy())
    fresh = et.Scene(ctx, moved, area_ref=a_ref)
    fi = fresh.info()
    ms_fresh = step_ms(fresh)
    del fresh
    sc.refit(V0, area_ref=a_ref)
    return {"workload": "room scene, one animation frame: 200 objects turned by up to 0.15 rad and moved by up "
                        "to 10 cm, every fourth deformed (1 cm radial ripple); same topology",
            "refit_ms": dev_ms / n, "refit_wall_ms": wall_ms, "build_ms": fi.build_ms,
            "sah_refit": refit_sah, "sah_rebuilt": fi.sah_cost,
            "step_ms_refitted": ms_refitted, "step_ms_rebuilt": ms_fresh,
            "frame_ms_refit": dev_ms / n + ms_refitted, "frame_ms_rebuild": fi.build_ms + ms_fresh}


def pipelined_leg(ctx, et, sc, s, P, ws, out, reps):
    """Room poses handed alternately to two contexts, each on a stream of its own (default
    priority): the calls are asynchronous and the contexts share only the scene, so one pose's
    synthesis runs while the next pose's trace does.  Wall time per pose over 2 reps poses,
    against the same loop on one context and stream."""
    import torch
    ctx2 = et.Context(0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ctxs = [ctx, ctx2]
    Ps = [P, et.Paths(s.capacity())]
    wss = [ws, et.Workspace()]
    outs = [out, torch.empty_like(out)]

    def run(n, two):
        for i in range(n):
            k = i % 2 if two else 0
            with torch.cuda.stream(streams[k]):
                et.simulate(ctxs[k], sc, s, paths=Ps[k], ws=wss[k], out=outs[k])

    def per_pose(two):
        run(2, two)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(2 * reps, two)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / (2 * reps)

    one, two = per_pose(False), per_pose(True)
    del ctx2
    return {"workload": "room step per pose, poses alternating between two contexts on two streams",
            "ms_per_pose_one_stream": one, "ms_per_pose_two_streams": two}


def batched_leg(ctx, args):
    """Batch workload: poses along a spline through the room plus uneven independent scenes
    (2^18 rays, <= 4 reflection points, 8 receivers, 2048 bins each).  Jobs per second of
    (a) separate single-pose forward calls, (b) one fused batched forward call, (c) one
    fused batched forward + adjoint call (seeded synthetic dL/dconj(H) per job), (d) (c)
    replayed from a captured HIP graph, and (b), (c) again with the autotuner's launch
    shapes.  The ratio reported is the throughput of (c) over that of (a)."""
    import torch
    import paper_2602_19652_amd as et
    import workloads as W
    t0 = time.perf_counter()
    b = W.batched_workload(n_poses=args.batch_poses, n_scenes=args.batch_scenes, n_rays=args.batch_rays)
    gen_s = time.perf_counter() - t0
    scenes = [et.Scene(ctx, sc) for sc in b.scenes]
    sims = [et.Sim(j.sim, flags=et.ET_SPECULAR) for j in b.jobs]
    J = len(b.jobs)
    ws = et.Workspace()
    paths = et.Paths(max(s.capacity() for s in sims))
    out = torch.empty(sims[0].M, sims[0].F, 2, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def plain():
        for i, j in enumerate(b.jobs):
            et.simulate(ctx, scenes[j.scene_index], sims[i], paths=paths, ws=ws, out=out)
    ms_plain = timed(plain, 2)
    batch = et.Batch(ctx, [(scenes[j.scene_index], sims[i]) for i, j in enumerate(b.jobs)])
    g = torch.Generator(device="cuda").manual_seed(1004)
    grad = torch.randn(J, sims[0].M, sims[0].F, dtype=torch.complex64, device="cuda", generator=g) * 1e-3
    ms_fwd = timed(lambda: batch.run(), 2)
    ms_fwd_adj = timed(lambda: batch.run(grad_spectra=grad), 2)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        batch.run(grad_spectra=grad, graph=True)          # capture
        torch.cuda.synchronize()
        e0.record(side)
        for _ in range(2):
            batch.run(grad_spectra=grad, graph=True)
        e1.record(side)
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / 2
    # launch shapes from the autotuner, then the same legs again
    tune = batch.autotune(grad_spectra=grad)
    ms_fwd_t = timed(lambda: batch.run(), 2)
    ms_fwd_adj_t = timed(lambda: batch.run(grad_spectra=grad), 2)
    batch.run(grad_spectra=grad)
    st = ctx.stats()
    jobs_s = lambda ms: J / (ms * 1e-3)
    ws_gb = batch.ws.numel() / 1e9
    tuned = {"synth_wgs": tune.synth_wgs, "adjoint_wgs": tune.adjoint_wgs, "trace_blocks": tune.trace_blocks,
             "batched_fwd_ms": ms_fwd_t, "batched_fwd_adj_ms": ms_fwd_adj_t,
             "phase_ms": {"trace": tune.ms_trace, "synth_kernel": tune.ms_synth, "adjoint_kernel": tune.ms_adjoint},
             "phase_ms_note": "each phase alone (the autotuner's runs take the job waves in order)",
             "phase_ms_pipelined": {"trace": st.ms_trace, "synth_kernel": st.ms_synth_kernel,
                                    "adjoint_kernel": st.ms_adjoint_kernel},
             "ratio_batched_fwd_adj_vs_plain_fwd": ms_plain / ms_fwd_adj_t}
    return {"jobs": J, "poses": args.batch_poses, "scenes": args.batch_scenes, "rays_per_job": args.batch_rays,
            "receivers": sims[0].M, "bins": sims[0].F, "scene_triangles": [int(len(sc["tris"])) for sc in b.scenes],
            "plain_fwd_ms": ms_plain, "batched_fwd_ms": ms_fwd, "batched_fwd_adj_ms": ms_fwd_adj,
            "batched_fwd_adj_graph_ms": ms_graph,
            "plain_fwd_jobs_per_s": jobs_s(ms_plain), "batched_fwd_jobs_per_s": jobs_s(ms_fwd),
            "batched_fwd_adj_jobs_per_s": jobs_s(ms_fwd_adj), "batched_fwd_adj_graph_jobs_per_s": jobs_s(ms_graph),
            "ratio_batched_fwd_adj_vs_plain_fwd": ms_plain / ms_fwd_adj,
            "ratio_graph_fwd_adj_vs_plain_fwd": ms_plain / ms_graph, "autotuned": tuned, "workspace_gb": ws_gb,
            "input_generation_s": gen_s}


if __name__ == "__main__":
    main()
