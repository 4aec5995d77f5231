"""GPU parity on the other workload configurations: foliage (receiver directivity, 1M
triangles, 8192 bins, 6 reflection points), batches of poses and scenes (plain vs batched
vs graph replay), and the differentiation workload (autograd, finite differences,
gradient-descent recovery of hidden band coefficients)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import check_spectra

pytestmark = pytest.mark.gpu
TOL = 1e-4


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.fixture(scope="module")
def ctx(et):
    return et.Context(0)


# ----------------------------------------------------------------------------- foliage

@pytest.fixture(scope="module")
def foliage():
    scene, sim = W.foliage_scene(n_rays=1 << 22)
    sub = np.sort(W.rng(91).choice(len(sim["ray_dirs"]), 512, replace=False))
    return scene, sim, sub


def test_foliage_trace_parity(et, ctx, foliage):
    """1M leaf triangles, 6 reflection points: hit sequences on certified rays of a sample."""
    scene, sim, sub = foliage
    dirs = sim["ray_dirs"][sub]
    ref = O.trace(scene, sim, dirs=dirs)
    sc = et.Scene(ctx, scene)
    info = sc.info()
    s = et.Sim(sim, flags=et.ET_SPECULAR, ray_dirs=dirs)
    P = et.trace(ctx, sc, s)
    st = ctx.stats()
    gpu = P.to_host()
    from test_gpu_parity import compare_traces
    mism = compare_traces(gpu, ref, ref["certified"])
    print(f"foliage: BVH depth {info.depth}, records gpu {st.records} oracle {len(ref['rtot'])}, "
          f"certified {ref['certified'].mean():.4f}, mismatches {mism}")
    assert mism == 0 and st.stack_overflows == 0


@pytest.mark.parametrize("direct", [False, True])
def test_foliage_synthesis_with_directivity(et, ctx, foliage, direct):
    """2 receivers with a 16-band x 32 el x 64 az directivity table, 8192 bins 20-200 kHz."""
    scene, sim, sub = foliage
    ref = O.trace(scene, sim, dirs=sim["ray_dirs"][sub], certify=False)
    flags = et.ET_SPECULAR | (et.ET_SYNTH_DIRECT if direct else 0)
    s = et.Sim(sim, flags=flags)
    P = et.Paths.from_records(ref)
    H = et.synthesize(ctx, s, P).cpu().numpy()
    st = ctx.stats()
    assert st.synth_kernel == (2 if direct else 1)
    bins = np.sort(W.rng(6).choice(sim["F"], 128, replace=False))
    H_ref = O.synth(ref, sim, bins=bins)
    check_spectra(H[:, bins], H_ref, f"foliage synthesis ({'direct' if direct else 'factorised'}, directivity), "
                  f"{len(ref['rtot'])} records, 128 sampled bins")
    # every bin of both receivers for 256 of the records
    rec = {k: v[:256] for k, v in ref.items() if k not in ("certified", "nseg")}
    H = et.synthesize(ctx, s, et.Paths.from_records(rec)).cpu().numpy()
    check_spectra(H, O.synth(rec, sim), f"foliage synthesis, all 8192 bins, {len(rec['rtot'])} records")


# ----------------------------------------------------------------------------- batches

@pytest.fixture(scope="module")
def batch_small():
    """A reduced batch: 6 poses along the spline in the room + 4 uneven scenes."""
    return W.batched_workload(n_poses=6, n_scenes=4, n_rays=1 << 11, M=8, F=2048, tmax=2e4)


def _batch_sims(et, b, extra_flags=0):
    """Uneven jobs: job i keeps its first 2^11 - 97 i rays."""
    sims = []
    for i, j in enumerate(b.jobs):
        n = max(64, (1 << 11) - 97 * i)
        sims.append(et.Sim(j.sim, flags=et.ET_SPECULAR | extra_flags, ray_dirs=j.sim["ray_dirs"][:n]))
    return sims


def test_batch_fused_matches_plain_and_graph(et, ctx, batch_small):
    """Fused batch (all rays in shared bounce kernels, records sorted by job into shared
    synthesis launches) vs one plain simulation per job: same segments, spectra equal up to
    the FP32 summation order; repeated runs and graph replays bit-identical."""
    import torch
    b = batch_small
    scenes = [et.Scene(ctx, s) for s in b.scenes]
    sims = _batch_sims(et, b)
    plain, seg = [], 0
    for i, j in enumerate(b.jobs):
        plain.append(et.simulate(ctx, scenes[j.scene_index], sims[i]).cpu().numpy())
        seg += ctx.stats().segments
    batch = et.Batch(ctx, [(scenes[j.scene_index], sims[i]) for i, j in enumerate(b.jobs)])
    Hb = batch.run().cpu().numpy()
    st = ctx.stats()
    assert st.segments == seg
    errs = [rel_l2(Hb[i], plain[i]) for i in range(len(b.jobs))]
    print(f"fused batch of {len(b.jobs)} jobs: segments {st.segments}, max rel L2 vs plain {max(errs):.3e}")
    assert max(errs) <= 1e-5
    # in job waves of at most 4096 rays: the same segments and records in total, a smaller workspace
    t0 = ctx.tuning()
    ctx.set_tuning(t0.synth_wgs, t0.adjoint_wgs, t0.trace_blocks, 4096)
    try:
        bw = et.Batch(ctx, [(scenes[j.scene_index], sims[i]) for i, j in enumerate(b.jobs)])
        Hw = bw.run().cpu().numpy()
        stw = ctx.stats()
        ew = [rel_l2(Hw[i], plain[i]) for i in range(len(b.jobs))]
        print(f"in waves of <= 4096 rays: workspace {bw.ws.numel() / 1e6:.1f} MB against {batch.ws.numel() / 1e6:.1f} "
              f"MB, segments {stw.segments}, records {stw.records} (one wave {st.records}), max rel L2 vs plain "
              f"{max(ew):.3e}")
        assert stw.segments == seg and stw.records == st.records
        assert bw.ws.numel() < batch.ws.numel()
        assert max(ew) <= 1e-5
        # several waves run pipelined over two streams; repeated runs and a captured graph (whose
        # waves run in order on one stream) give the same bits
        assert np.array_equal(bw.run().cpu().numpy(), Hw), "pipelined waves not deterministic"
        sw = torch.cuda.Stream()
        with torch.cuda.stream(sw):
            Hwg = bw.run(graph=True).cpu().numpy()
            torch.cuda.synchronize()
        assert np.array_equal(Hwg, Hw), "pipelined waves differ from the waves in order"
    finally:
        ctx.set_tuning(t0.synth_wgs, t0.adjoint_wgs, t0.trace_blocks, 0)
    assert np.array_equal(batch.run().cpu().numpy(), Hb), "fused batch not deterministic"
    # graph capture on a side stream, replayed several times with eager work in between
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(3):
            Hg = batch.run(graph=True).cpu().numpy()
            torch.cuda.synchronize()
            assert np.array_equal(Hg, Hb), f"graph replay {rep} differs"
            et.simulate(ctx, scenes[0], sims[0])          # unrelated eager work between replays
            torch.cuda.synchronize()


def _certified_records(rec):
    """The records of the rays the oracle certified (record arrays only)."""
    keep = rec["certified"][rec["ray"]]
    return {k: v[keep] for k, v in rec.items() if k not in ("certified", "nseg")}


@pytest.mark.parametrize("wave_rays", [0, 1024])
def test_batch_fused_matches_oracle_per_job(et, ctx, batch_small, wave_rays):
    """Every job of a fused batch (6 poses in the room and the 4 uneven scenes, uneven ray
    counts) on its oracle-certified rays: the fused forward's spectra (eager, and graph replays
    with eager work between them) against the oracle's per job and per receiver, and the fused
    adjoint's dL/dk and dL/dx_m per job against the oracle gradient for a seeded dL/dconj(H).
    Once as one job wave and once in waves of at most 1024 rays (four waves here), which reuse
    one wave's workspace."""
    import torch
    t0 = ctx.tuning()
    ctx.set_tuning(t0.synth_wgs, t0.adjoint_wgs, t0.trace_blocks, wave_rays)
    try:
        _batch_vs_oracle(et, ctx, batch_small)
    finally:
        ctx.set_tuning(t0.synth_wgs, t0.adjoint_wgs, t0.trace_blocks, 0)


def _batch_vs_oracle(et, ctx, batch_small):
    import torch
    b = batch_small
    scenes = [et.Scene(ctx, s) for s in b.scenes]
    sims, recs, psims = [], [], []
    for i, j in enumerate(b.jobs):
        n = 384 - 29 * i
        sim = dict(j.sim, ray_dirs=j.sim["ray_dirs"][:n])
        ref = O.trace(b.scenes[j.scene_index], sim)
        dirs = sim["ray_dirs"][ref["certified"]]
        recs.append(_certified_records(ref))
        psims.append(sim)
        sims.append(et.Sim(sim, flags=et.ET_SPECULAR, ray_dirs=dirs))
    batch = et.Batch(ctx, [(scenes[j.scene_index], sims[i]) for i, j in enumerate(b.jobs)])
    print(f"batch of {len(b.jobs)} jobs, {sum(s.desc.N for s in sims)} rays, wave_rays {ctx.tuning().wave_rays}: "
          f"workspace {batch.ws.numel() / 1e6:.1f} MB")
    J, M, F = len(b.jobs), sims[0].M, sims[0].F
    gen = np.random.default_rng(44)
    g = (gen.normal(size=(J, M, F)) + 1j * gen.normal(size=(J, M, F))).astype(np.complex64)
    gd = torch.as_tensor(g).cuda()
    Hb = batch.run(grad_spectra=gd).cpu().numpy()
    assert ctx.stats().adjoint_kernel == 1
    gk_b, gx_b = batch.grad_k.cpu().numpy(), batch.grad_rx.cpu().numpy()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for rep in range(2):
            Hg = batch.run(grad_spectra=gd, graph=True).cpu().numpy()
            torch.cuda.synchronize()
            assert np.array_equal(Hg, Hb), f"graph replay {rep} differs from the eager batch"
            assert np.array_equal(batch.grad_k.cpu().numpy(), gk_b) and np.array_equal(batch.grad_rx.cpu().numpy(), gx_b)
            et.simulate(ctx, scenes[0], sims[0])
            torch.cuda.synchronize()
    worst = 0.0
    for i, j in enumerate(b.jobs):
        H_ref = O.synth(recs[i], psims[i])
        e = check_spectra(Hb[i], H_ref, f"batch job {i} (scene {j.scene_index}, {len(recs[i]['rtot'])} records)")
        gk_ref, gx_ref = O.grad(recs[i], psims[i], g[i].astype(np.complex128))
        ek, ex = rel_l2(gk_b[i], gk_ref), rel_l2(gx_b[i], gx_ref)
        print(f"batch job {i}: adjoint dL/dk {ek:.3e}, dL/dx {ex:.3e}")
        assert ek <= TOL and ex <= TOL
        worst = max(worst, e, ek, ex)
    print(f"fused batch vs oracle: worst relative error over {J} jobs {worst:.3e}")


def test_batch_fused_adjoint_matches_per_job(et, ctx, batch_small):
    """Batched forward + adjoint: every job's dL/dk and dL/dx vs its own adjoint call."""
    import torch
    b = batch_small
    scenes = [et.Scene(ctx, s) for s in b.scenes]
    sims = _batch_sims(et, b)
    batch = et.Batch(ctx, [(scenes[j.scene_index], sims[i]) for i, j in enumerate(b.jobs)])
    g = torch.Generator(device="cuda").manual_seed(5)
    J, M, F = len(b.jobs), sims[0].M, sims[0].F
    grad = torch.randn(J, M, F, dtype=torch.complex64, device="cuda", generator=g)
    batch.run(grad_spectra=grad)
    gk_b, gx_b = batch.grad_k.cpu().numpy(), batch.grad_rx.cpu().numpy()
    assert ctx.stats().adjoint_kernel == 1
    ek, ex = [], []
    for i, j in enumerate(b.jobs):
        P = et.trace(ctx, scenes[j.scene_index], sims[i])
        gk, gx = et.synthesize_backward(ctx, sims[i], P, grad[i])
        ek.append(rel_l2(gk_b[i], gk.cpu().numpy()))
        ex.append(rel_l2(gx_b[i], gx.cpu().numpy()))
    print(f"batched adjoint vs per job: max rel dL/dk {max(ek):.3e}, dL/dx {max(ex):.3e}")
    assert max(ek) <= 1e-5 and max(ex) <= 1e-5


def test_batch_fused_adjoint_with_directivity(et, ctx, batch_small):
    """A fused batch whose receivers have directivity (four bands, 16 x 32 cells, each job its
    own table): the forward runs factorised, the adjoint per term; every job's spectra and
    gradients against its own calls."""
    import torch
    b = batch_small
    scenes = [et.Scene(ctx, s) for s in b.scenes]
    g = W.rng(41)
    sims = []
    for i, j in enumerate(b.jobs):
        n = max(64, (1 << 11) - 97 * i)
        tab = np.ascontiguousarray(g.uniform(0.2, 1.0, (8, 4, 16, 32)).astype(np.float32))
        sims.append(et.Sim(dict(j.sim, directivity=tab), flags=et.ET_SPECULAR, ray_dirs=j.sim["ray_dirs"][:n]))
    batch = et.Batch(ctx, [(scenes[j.scene_index], sims[i]) for i, j in enumerate(b.jobs)])
    tg = torch.Generator(device="cuda").manual_seed(6)
    J, M, F = len(b.jobs), sims[0].M, sims[0].F
    grad = torch.randn(J, M, F, dtype=torch.complex64, device="cuda", generator=tg)
    Hb = batch.run(grad_spectra=grad).cpu().numpy()
    st = ctx.stats()
    assert st.synth_kernel == 1 and st.adjoint_kernel == 2
    gk_b, gx_b = batch.grad_k.cpu().numpy(), batch.grad_rx.cpu().numpy()
    eh, ek, ex = [], [], []
    for i, j in enumerate(b.jobs):
        P = et.trace(ctx, scenes[j.scene_index], sims[i])
        eh.append(rel_l2(Hb[i], et.synthesize(ctx, sims[i], P).cpu().numpy()))
        gk, gx = et.synthesize_backward(ctx, sims[i], P, grad[i])
        ek.append(rel_l2(gk_b[i], gk.cpu().numpy()))
        ex.append(rel_l2(gx_b[i], gx.cpu().numpy()))
    print(f"batch with directivity: max rel H {max(eh):.3e}, dL/dk {max(ek):.3e}, dL/dx {max(ex):.3e}")
    assert max(eh) <= 1e-5 and max(ek) <= 1e-5 and max(ex) <= 1e-5


def test_batch_autotune(et, ctx, batch_small):
    """The autotuner picks candidate launch shapes with measured phase times; results under
    the new shapes agree with the default ones (same records, other summation chunks)."""
    import torch
    b = batch_small
    scenes = [et.Scene(ctx, s) for s in b.scenes]
    sims = _batch_sims(et, b)
    batch = et.Batch(ctx, [(scenes[j.scene_index], sims[i]) for i, j in enumerate(b.jobs)])
    H0 = batch.run().cpu().numpy()
    g = torch.Generator(device="cuda").manual_seed(6)
    grad = torch.randn(len(b.jobs), sims[0].M, sims[0].F, dtype=torch.complex64, device="cuda", generator=g)
    try:
        t = batch.autotune(grad_spectra=grad)
        print(f"autotune: synth {t.synth_wgs} wgs ({t.ms_synth:.3f} ms), adjoint {t.adjoint_wgs} wgs "
              f"({t.ms_adjoint:.3f} ms), bounce grid {t.trace_blocks} ({t.ms_trace:.3f} ms)")
        assert t.synth_wgs in (1024, 2048, 4096, 8192, 16384) and t.adjoint_wgs in (1024, 2048, 4096, 8192, 16384)
        assert t.trace_blocks in (1024, 2048, 4096, 6144, 8192)
        assert t.ms_trace > 0 and t.ms_synth > 0 and t.ms_adjoint > 0
        cur = ctx.tuning()
        assert (cur.synth_wgs, cur.adjoint_wgs, cur.trace_blocks) == (t.synth_wgs, t.adjoint_wgs, t.trace_blocks)
        H1 = batch.run().cpu().numpy()
        assert rel_l2(H1, H0) <= 1e-5
        with pytest.raises(et.EchoError):
            ctx.set_tuning(32, 1024, 2048)
    finally:
        ctx.set_tuning(2048, 1024, 2048)


def test_batch_with_diffraction_runs_job_by_job(et, ctx, batch_small):
    """Jobs with diffraction sampling take the sequential path: bit-identical to plain calls."""
    b = batch_small
    jobs = b.jobs[:3]
    scenes = [et.Scene(ctx, s, area_ref=W.median_triangle_area(s)) for s in b.scenes]
    sims = [et.Sim(dict(j.sim, diff_K=1024, diff_seed=9 + i), flags=et.ET_SPECULAR | et.ET_DIFFRACTION)
            for i, j in enumerate(jobs)]
    plain = [et.simulate(ctx, scenes[j.scene_index], sims[i]).cpu().numpy() for i, j in enumerate(jobs)]
    batch = et.Batch(ctx, [(scenes[j.scene_index], sims[i]) for i, j in enumerate(jobs)])
    Hb = batch.run().cpu().numpy()
    for i in range(len(jobs)):
        assert np.array_equal(Hb[i], plain[i]), f"job {i} differs from its plain simulation"


# ----------------------------------------------------------------------------- differentiation

@pytest.fixture(scope="module")
def diff_paths(et, ctx):
    """Fixed specular paths of the room scene (a seeded ray subset), 32 receivers, 64 bins."""
    scene, sim = W.room_scene(n_rays=1 << 20, F=64, diff_K=0)
    sub = np.sort(W.rng(55).choice(len(sim["ray_dirs"]), 1024, replace=False))
    rec = O.trace(scene, sim, dirs=sim["ray_dirs"][sub], certify=False)
    return scene, sim, rec


def test_spectra_fn_autograd_matches_oracle(et, ctx, diff_paths):
    import torch
    scene, sim, rec = diff_paths
    g = W.rng(13)
    k_star = g.uniform(0.3, 0.99, (16, 8)).astype(np.float32)
    H_star = O.synth(rec, dict(sim, refl_k=k_star))
    k0 = np.full((16, 8), 0.5, np.float32)
    s = et.Sim(dict(sim, refl_k=k0), flags=et.ET_SPECULAR)
    P = et.Paths.from_records(rec)
    k = torch.tensor(k0, device="cuda", requires_grad=True)
    x = torch.tensor(sim["rx_pos"], device="cuda", requires_grad=True)
    H = et.SpectraFn.apply(k, x, ctx, s, P)
    L = (H - torch.as_tensor(H_star, dtype=torch.complex64, device="cuda")).abs().pow(2).sum()
    L.backward()
    H_ref = O.synth(rec, dict(sim, refl_k=k0))
    gk_ref, gx_ref = O.grad(rec, dict(sim, refl_k=k0), H_ref - H_star)
    ek = rel_l2(k.grad.cpu().numpy(), gk_ref)
    ex = rel_l2(x.grad.cpu().numpy(), gx_ref)
    eL = abs(L.item() - np.sum(np.abs(H_ref - H_star) ** 2)) / np.sum(np.abs(H_ref - H_star) ** 2)
    print(f"autograd: loss rel {eL:.2e}, dL/dk rel {ek:.2e}, dL/dx rel {ex:.2e}")
    assert eL <= 1e-5 and ek <= TOL and ex <= TOL


def test_gpu_gradient_directional_fd(et, ctx, diff_paths):
    """Directional derivatives of the GPU loss along random directions in (k, x) against
    central differences of the FP64 oracle loss (h = 1e-6)."""
    import torch
    scene, sim, rec = diff_paths
    g = W.rng(14)
    k_star = g.uniform(0.3, 0.99, (16, 8)).astype(np.float32)
    H_star = O.synth(rec, dict(sim, refl_k=k_star))
    k0 = g.uniform(0.4, 0.8, (16, 8)).astype(np.float32)
    s = et.Sim(dict(sim, refl_k=k0), flags=et.ET_SPECULAR)
    P = et.Paths.from_records(rec)
    H = et.synthesize(ctx, s, P)
    gk, gx = et.synthesize_backward(ctx, s, P, H - torch.as_tensor(H_star, dtype=torch.complex64, device="cuda"))
    gk, gx = gk.cpu().numpy(), gx.cpu().numpy()

    def loss(k, x):
        return float(np.sum(np.abs(O.synth(rec, dict(sim, refl_k=k, rx_pos=x)) - H_star) ** 2))
    h = 1e-6
    Hk = O.synth(rec, dict(sim, refl_k=k0))
    for t in range(4):
        dk = g.normal(size=k0.shape).astype(np.float32)
        dx = g.normal(size=sim["rx_pos"].shape) * 0.01
        fd_x = (loss(k0, sim["rx_pos"] + h * dx) - loss(k0, sim["rx_pos"] - h * dx)) / (2 * h)
        an_x = float(np.sum(gx * dx))
        # H is linear in k: the directional derivative along dk is exact with the table dk
        dH = O.synth(rec, dict(sim, refl_k=dk))
        ex_k = float(np.sum(2 * np.real(np.conj(Hk - H_star) * dH)))
        an_k = float(np.sum(gk * dk.astype(np.float64)))
        print(f"direction {t}: x analytic {an_x:.6e} FD {fd_x:.6e}; k analytic {an_k:.6e} exact {ex_k:.6e}")
        assert abs(an_x - fd_x) <= 1e-3 * abs(fd_x) + 1e-12
        assert abs(an_k - ex_k) <= 1e-4 * abs(ex_k) + 1e-12


def test_gradient_descent_recovers_hidden_coefficients(et, ctx, diff_paths):
    """L is quadratic in k (the reflection coefficient of the n-th triangle only): projected
    gradient descent with the GPU adjoint converges to the FP64 normal-equation solution,
    which recovers the hidden coefficients on the identifiable (material, band) entries."""
    import torch
    scene, sim, rec = diff_paths
    g = W.rng(15)
    k_star = g.uniform(0.3, 0.99, (16, 8)).astype(np.float32)
    H_star = O.synth(rec, dict(sim, refl_k=k_star))
    # basis responses (FP64 oracle): H(k) = sum_qb k_qb E_qb
    E = []
    for i in range(128):
        e = np.zeros((16, 8), np.float32)
        e.flat[i] = 1
        E.append(O.synth(rec, dict(sim, refl_k=e)).ravel())
    E = np.stack(E, 1)
    # entries the data observe: the Gauss-Newton diagonal within 12 decades of the largest
    # (deeply attenuated entries reach 1e-76, whose reciprocal step overflows FP32)
    diag = 2 * np.sum(np.abs(E) ** 2, axis=0)
    used = diag > 1e-12 * diag.max()
    Ar = np.concatenate([E.real, E.imag])[:, used]
    br = np.concatenate([H_star.real.ravel(), H_star.imag.ravel()])
    k_ne = np.linalg.lstsq(Ar, br, rcond=None)[0]
    # identifiable entries: the FP64 data determine them (normal equations recover k*)
    ident = np.zeros(128, bool)
    ident[np.nonzero(used)[0]] = np.abs(k_ne - k_star.ravel()[used]) < 1e-6
    assert ident.sum() >= 0.8 * used.sum()
    # gradient descent on the GPU, preconditioned by the diagonal of the Gauss-Newton matrix
    s = et.Sim(dict(sim, refl_k=np.full((16, 8), 0.5, np.float32)), flags=et.ET_SPECULAR)
    P = et.Paths.from_records(rec)
    k = torch.full((16, 8), 0.5, device="cuda", dtype=torch.float32)
    x = torch.tensor(sim["rx_pos"], device="cuda")
    Hs = torch.as_tensor(H_star, dtype=torch.complex64, device="cuda")
    step = torch.as_tensor(np.where(used, 1.0 / np.where(used, diag, 1.0), 0.0).reshape(16, 8), device="cuda",
                           dtype=torch.float32)
    for it in range(200):
        kk = k.clone().requires_grad_(True)
        H = et.SpectraFn.apply(kk, x, ctx, s, P)
        L = (H - Hs).abs().pow(2).sum()
        L.backward()
        # projected onto physical coefficients (the band factor is taken in the log domain)
        k = (k - 0.5 * step * kk.grad).detach().clamp_(1e-3, 1.0)
    kg = k.cpu().numpy().astype(np.float64).ravel()
    # (a) the descent reaches the target spectra (FP64 residual of the linear model)
    res = np.linalg.norm(E @ kg - H_star.ravel()) / np.linalg.norm(H_star)
    # (b) coefficients are recovered where the data pin them: entries that a relative spectral
    # error of 1e-5 (the FP32 forward/adjoint sit near 1e-6) moves by < 1e-3 at most
    sens = np.linalg.norm(np.linalg.pinv(Ar), axis=1) * np.linalg.norm(br) * 1e-5
    well = np.zeros(128, bool)
    well[np.nonzero(used)[0]] = sens < 1e-3
    well &= ident
    err_w = np.max(np.abs(kg[well] - k_star.ravel()[well]))
    err_i = np.max(np.abs(kg[ident] - k_star.ravel()[ident]))
    print(f"GD recovery: {ident.sum()} of {used.sum()} observed coefficients identifiable, {well.sum()} well "
          f"determined; spectra residual {res:.2e}, max abs error {err_w:.2e} (well determined), "
          f"{err_i:.2e} (all identifiable), final loss {L.item():.3e}")
    assert well.sum() >= 0.5 * ident.sum()
    assert res <= 1e-5
    assert err_w <= 1e-3


# ----------------------------------------------------------------------------- differentiation at the stated sizes

@pytest.fixture(scope="module")
def d_instance(et, ctx):
    """The differentiation workload: the room scene's fixed specular paths (diffraction off),
    traced on the GPU, 32 receivers; hidden band coefficients from the workload's seed."""
    scene, sim = W.room_scene(n_rays=1 << 20, diff_K=0)
    sc = et.Scene(ctx, scene, area_ref=sim["area_ref"])
    k_star = W.rng(1005).uniform(0.3, 0.99, (16, 8)).astype(np.float32)
    return scene, sim, sc, k_star


def test_d_reduced_instance_all_parameters(et, ctx, d_instance):
    """Reduced instance: 2^14 of the room's rays, 256 bins, all 224 parameters (16 x 8 band
    coefficients and 32 x 3 receiver coordinates).  The GPU adjoint against the FP64 oracle's
    gradient, and that gradient against central differences of the FP64 loss for every
    parameter: for k exact (H is linear in k, so the difference needs only the band's bins and
    the material's records), for x_m with h = 1e-6 m over receiver m's spectrum."""
    import torch
    scene, sim, sc, k_star = d_instance
    sim = dict(sim, F=256)
    sub = np.sort(W.rng(1006).choice(len(sim["ray_dirs"]), 1 << 14, replace=False))
    k0 = np.full((16, 8), 0.5, np.float32)
    simk = dict(sim, refl_k=k0)
    s = et.Sim(simk, flags=et.ET_SPECULAR, ray_dirs=sim["ray_dirs"][sub])
    P = et.trace(ctx, sc, s)
    rec = P.to_host()
    H_star = O.synth(rec, dict(sim, refl_k=k_star))
    H = O.synth(rec, simk)
    gR = H - H_star
    gk_ref, gx_ref = O.grad(rec, simk, gR)
    gk, gx = et.synthesize_backward(ctx, s, P, torch.as_tensor(gR.astype(np.complex64)).cuda())
    gk, gx = gk.cpu().numpy(), gx.cpu().numpy()
    ek, ex = rel_l2(gk, gk_ref), rel_l2(gx, gx_ref)
    wk = float(np.max(np.abs(gk - gk_ref)) / np.max(np.abs(gk_ref)))
    wx = float(np.max(np.abs(gx - gx_ref)) / np.max(np.abs(gx_ref)))
    print(f"D reduced ({len(rec['rtot'])} records, 32 x 256): GPU vs oracle gradient dL/dk {ek:.3e} (worst entry "
          f"{wk:.3e} of the largest), dL/dx {ex:.3e} (worst {wx:.3e})")
    assert ek <= TOL and ex <= TOL and wk <= TOL and wx <= TOL
    # the oracle gradient against central differences, all 224 parameters
    h = 1e-6
    F, Bk = sim["F"], 8
    worst_k = worst_x = 0.0
    for q in range(16):
        sel = rec["mat"] == q
        recq = {kk: v[sel] for kk, v in rec.items() if hasattr(v, "__len__") and len(v) == len(sel)}
        for b in range(Bk):
            bins = np.arange(F)[(np.arange(F) * Bk) // F == b].astype(np.int32)
            e = np.zeros((16, Bk), np.float32)
            e[q, b] = 1.0
            E = O.synth(recq, dict(simk, refl_k=e), bins=bins) if sel.any() else np.zeros((32, len(bins)))
            Lp = np.sum(np.abs(gR[:, bins] + h * E) ** 2)
            Lm = np.sum(np.abs(gR[:, bins] - h * E) ** 2)
            fd = (Lp - Lm) / (2 * h)
            worst_k = max(worst_k, abs(fd - gk_ref[q, b]) / np.max(np.abs(gk_ref)))
    for m in range(32):
        for a in range(3):
            Ls = []
            for sgn in (1, -1):
                xp = simk["rx_pos"].copy()
                xp[m, a] += sgn * h
                Hm = O.synth(rec, dict(simk, rx_pos=xp), M_subset=[m])
                Ls.append(np.sum(np.abs(Hm[0] - H_star[m]) ** 2))
            fd = (Ls[0] - Ls[1]) / (2 * h)
            worst_x = max(worst_x, abs(fd - gx_ref[m, a]) / np.max(np.abs(gx_ref)))
    print(f"D reduced: oracle gradient vs central differences, worst over 128 k entries {worst_k:.2e}, over 96 "
          f"receiver coordinates {worst_x:.2e} (of the largest entry)")
    assert worst_k <= 1e-6 and worst_x <= 1e-5


def test_d_full_instance_directional_derivatives(et, ctx, d_instance):
    """Full instance: the room step's fixed specular paths (2^20 rays), 32 receivers x 4096
    bins.  The oracle evaluates the loss on a seeded subset of 16 bins (the full sum is 5.5e11
    FP64 terms), so the loss is L = sum over those bins of |H - H*|^2, and the GPU adjoint is fed
    dL/dconj(H) = H - H* on them and zero elsewhere.  The GPU forward matches the oracle on the
    16 bins; 8 directional derivatives (4 along receiver coordinates, central differences with
    h = 1e-6 m; 4 along band coefficients, exact by linearity) match the adjoint's."""
    import torch
    scene, sim, sc, k_star = d_instance
    g = W.rng(1007)
    k0 = g.uniform(0.4, 0.8, (16, 8)).astype(np.float32)
    simk = dict(sim, refl_k=k0)
    s = et.Sim(simk, flags=et.ET_SPECULAR)
    P = et.trace(ctx, sc, s)
    rec = P.to_host()
    bins = np.sort(g.choice(sim["F"], 16, replace=False)).astype(np.int32)
    H_gpu = et.synthesize(ctx, s, P).cpu().numpy()
    H = O.synth(rec, simk, bins=bins)
    check_spectra(H_gpu[:, bins], H, f"D full ({len(rec['rtot'])} records): GPU forward vs oracle on 16 bins")
    H_star = O.synth(rec, dict(simk, refl_k=k_star), bins=bins)
    gR = H - H_star
    gfull = np.zeros((32, sim["F"]), np.complex64)
    gfull[:, bins] = gR
    gk, gx = et.synthesize_backward(ctx, s, P, torch.as_tensor(gfull).cuda())
    gk, gx = gk.cpu().numpy(), gx.cpu().numpy()

    def loss(k, x):
        return float(np.sum(np.abs(O.synth(rec, dict(simk, refl_k=k, rx_pos=x), bins=bins) - H_star) ** 2))
    h = 1e-6
    x0 = simk["rx_pos"]
    for t in range(4):
        dx = g.normal(size=x0.shape) * 0.01
        fd = (loss(k0, x0 + h * dx) - loss(k0, x0 - h * dx)) / (2 * h)
        an = float(np.sum(gx * dx))
        print(f"D full, receiver direction {t}: adjoint {an:.6e}, central difference {fd:.6e}")
        assert abs(an - fd) <= 1e-3 * abs(fd)
    for t in range(4):
        dk = g.normal(size=k0.shape).astype(np.float32)
        dH = O.synth(rec, dict(simk, refl_k=dk), bins=bins)
        ex = float(np.sum(2 * np.real(np.conj(gR) * dH)))   # exact: L is quadratic in k
        an = float(np.sum(gk * dk.astype(np.float64)))
        print(f"D full, coefficient direction {t}: adjoint {an:.6e}, exact {ex:.6e}")
        assert abs(an - ex) <= 1e-4 * abs(ex)


def test_two_contexts_on_two_streams(et, ctx):
    """Two contexts, each on a stream of its own, run alternate poses of the room concurrently
    (one pose's synthesis beside the other's trace): every call's spectra equal, bit for bit,
    those of the same pose run alone on one context."""
    import torch
    scene, sim = W.room_scene(n_rays=1 << 16, M=4, F=1024, diff_K=4096)
    simB = dict(sim, emitter_pos=np.asarray(sim["emitter_pos"]) + np.array([0.3, 0.0, 0.0]))
    sc = et.Scene(ctx, scene, area_ref=sim["area_ref"])
    sims = [et.Sim(sim), et.Sim(simB)]
    ref = [et.simulate(ctx, sc, s).clone() for s in sims]
    torch.cuda.synchronize()
    assert not torch.equal(ref[0], ref[1])
    ctxs = [ctx, et.Context(0)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    paths = [et.Paths(s.capacity()) for s in sims]
    wss = [et.Workspace(), et.Workspace()]
    outs = [torch.empty(s.M, s.F, 2, dtype=torch.float32, device="cuda") for s in sims]
    for k in range(2):   # workspaces sized before the concurrent calls
        et.simulate(ctxs[k], sc, sims[k], paths=paths[k], ws=wss[k], out=outs[k])
    torch.cuda.synchronize()
    for rep in range(4):
        got = []
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                got.append(et.simulate(ctxs[k], sc, sims[k], paths=paths[k], ws=wss[k], out=outs[k]))
        torch.cuda.synchronize()
        for k in range(2):
            assert torch.equal(got[k], ref[k]), (rep, k)
