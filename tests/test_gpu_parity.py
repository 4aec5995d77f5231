"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Protocol:
  * hit triangles and visibility bits match bit-exactly on certified rays (rays none of
    whose segments is marginal under the oracle's FP32-rounding margin predicate);
  * spectra match within 1e-4 relative L2 (complex, over all receivers and bins): the
    synthesis fed the oracle's own records, and end to end on the certified rays;
  * diffraction sample lists match exactly (integer CDF, shared counter-based RNG);
  * the adjoint matches the oracle's analytic gradient within 1e-4 relative.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-4


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def spectra_err(H, H_ref):
    """Relative L2 over all receivers and bins, and the worst receiver's own relative L2
    (value, receiver index); spectra are [M, bins]."""
    H, H_ref = np.asarray(H), np.asarray(H_ref)
    per = [rel_l2(H[m], H_ref[m]) for m in range(H_ref.shape[0])]
    w = int(np.argmax(per))
    return rel_l2(H, H_ref), per[w], w


def check_spectra(H, H_ref, what, tol=TOL):
    """Asserts the global and every receiver's relative L2 against the oracle; prints both."""
    e, ew, w = spectra_err(H, H_ref)
    print(f"{what}: rel L2 {e:.3e}, worst receiver {w}: {ew:.3e}")
    assert e <= tol and ew <= tol, f"{what}: rel L2 {e:.3e}, receiver {w} {ew:.3e}"
    return e


def by_ray(rec, n_rays):
    """{ray: [(bounce, tri, vis, rtot, p)]} sorted by bounce."""
    out = {i: [] for i in range(n_rays)}
    for k in range(len(rec["rtot"])):
        out[int(rec["ray"][k])].append((int(rec["bounce"][k]), int(rec["tri"][k]), int(rec["vis"][k]),
                                        float(rec["rtot"][k]), np.asarray(rec["p"][k])))
    for v in out.values():
        v.sort(key=lambda x: x[0])
    return out


def compare_traces(gpu, orc, certified):
    g = by_ray(gpu, len(certified))
    o = by_ray(orc, len(certified))
    mism = 0
    for i in np.nonzero(certified)[0]:
        a, b = g[i], o[i]
        if [(x[0], x[1], x[2]) for x in a] != [(x[0], x[1], x[2]) for x in b]:
            mism += 1
            continue
        for x, y in zip(a, b):
            assert abs(x[3] - y[3]) <= 1e-9 * max(1.0, y[3])
            assert np.max(np.abs(x[4] - y[4])) <= 1e-9
    return mism


@pytest.fixture(scope="module")
def ctx(et):
    return et.Context(0)


@pytest.fixture(scope="module")
def tiny():
    scene, sim = W.tiny_scene()
    ref = O.trace(scene, sim)
    return scene, sim, ref


# ----------------------------------------------------------------------------- scene build

def test_scene_build_tiny(et, ctx, tiny):
    scene, sim, _ = tiny
    sc = et.Scene(ctx, scene, area_ref=W.median_triangle_area(scene))
    info = sc.info()
    assert info.T == len(scene["tris"]) and info.n_nodes == info.T - 1
    assert 1 < info.depth <= 64
    print(f"tiny BVH: depth {info.depth} SAH {info.sah_cost:.2f} build {info.build_ms:.2f} ms")


def test_curvature_bitwise_matches_oracle(et, ctx):
    """C_i and G_v: same definition, same operation order, IEEE double on both sides."""
    g = W.rng(21)
    scene = W.room_geometry(g, n_boxes=20, n_cyl=20)
    a_ref = W.median_triangle_area(scene)
    G_ref, C_ref = O.curvature(scene, a_ref)
    sc = et.Scene(ctx, scene, area_ref=a_ref)
    Cg, Gg = sc.curvature()
    Cg, Gg = Cg.cpu().numpy(), Gg.cpu().numpy()
    np.testing.assert_allclose(Gg, G_ref, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Cg, C_ref, rtol=1e-12, atol=1e-14)
    exact = float(np.mean(Cg == C_ref))
    print(f"curvature: bitwise-equal fraction {exact:.6f}")
    assert exact == 1.0


# ----------------------------------------------------------------------------- tracing

def test_trace_parity_tiny(et, ctx, tiny):
    scene, sim, ref = tiny
    sc = et.Scene(ctx, scene)
    s = et.Sim(sim)
    P = et.trace(ctx, sc, s)
    st = ctx.stats()
    gpu = P.to_host()
    cert = ref["certified"]
    mism = compare_traces(gpu, ref, cert)
    print(f"tiny: records gpu {st.records} oracle {len(ref['rtot'])}, certified {cert.mean():.4f}, mismatches {mism}")
    assert st.stack_overflows == 0
    assert mism == 0
    assert st.segments == int(ref["nseg"].sum())


SYNTH_LAYOUTS = {
    # name: (material bands, directivity bands or 0, forced direct, kernel expected)
    "bands8": (8, 0, False, 1),          # 128-bin bands: one band per two 64-bin rows
    "bands16": (16, 0, False, 1),        # 64-bin bands: a segment per row
    "bands2": (2, 0, False, 1),
    "bands12": (12, 0, False, 2),        # band edges inside 64-bin rows: only the direct kernel applies
    "bands16_dir4": (16, 4, False, 1),   # receiver directivity with its own band split
    "bands8_dir4_direct": (8, 4, True, 2),
    "bands8_direct": (8, 0, True, 2),
}


# name: (bins, material bands, directivity bands or 0): the factorised kernel's ways of carrying
# the band factor: edges on 512 bins (folded per group of 8 rows), on 256 bins (folded per half
# group of 4 rows, also with a last group that holds 4 rows), and off both (a table of band
# factors; 3072 bins, 192-bin bands)
FOLD_LAYOUTS = {
    "F4096_bands8_fold8": (4096, 8, 0),
    "F4096_bands16_fold4": (4096, 16, 0),
    "F4096_bands16_dir8_fold4": (4096, 16, 8),
    "F3072_bands16_table": (3072, 16, 0),
    "F1280_bands5_fold4_partial_group": (1280, 5, 0),   # 20 rows: the last group of 8 holds 4
}


@pytest.mark.parametrize("layout", list(FOLD_LAYOUTS))
def test_synthesis_band_folding(et, ctx, tiny, layout):
    """The factorised kernel under each band-factor layout (tiles of 20, 48 and 64 rows), every
    bin, against the oracle's spectra of 2048 of the tiny scene's records."""
    scene, sim, ref = tiny
    F, Bk, Bd = FOLD_LAYOUTS[layout]
    g = W.rng(13)
    sim = dict(sim, F=F, refl_k=g.uniform(0.3, 0.99, (1, Bk)).astype(np.float32),
               lobe_beta=g.uniform(0.05, 0.3, (1, Bk)).astype(np.float32),
               diff_coef=np.full((1, Bk), 0.1, np.float32))
    if Bd:
        sim["directivity"] = g.uniform(0.2, 1.0, (len(sim["rx_pos"]), Bd, 8, 16)).astype(np.float32)
    sub = {k: (v[:2048] if isinstance(v, np.ndarray) and len(v) == len(ref["rtot"]) else v) for k, v in ref.items()}
    H = et.synthesize(ctx, et.Sim(sim, flags=et.ET_SPECULAR), et.Paths.from_records(sub)).cpu().numpy()
    st = ctx.stats()
    check_spectra(H, O.synth(sub, sim), f"band folding {layout} (kernel {st.synth_kernel}, {len(sub['rtot'])} records)")
    assert st.synth_kernel == 1


@pytest.mark.parametrize("layout", list(SYNTH_LAYOUTS))
def test_synthesis_isolation_tiny(et, ctx, tiny, layout):
    """GPU synthesis of the oracle's own records vs the oracle's spectra, over band layouts
    that select the factorised or the direct kernel."""
    scene, sim, ref = tiny
    Bk, Bd, direct, kernel = SYNTH_LAYOUTS[layout]
    g = W.rng(12)
    sim = dict(sim, refl_k=g.uniform(0.3, 0.99, (1, Bk)).astype(np.float32),
               lobe_beta=g.uniform(0.05, 0.3, (1, Bk)).astype(np.float32),
               diff_coef=np.full((1, Bk), 0.1, np.float32))
    if Bd:
        sim["directivity"] = g.uniform(0.2, 1.0, (len(sim["rx_pos"]), Bd, 8, 16)).astype(np.float32)
    flags = et.ET_SPECULAR | (et.ET_SYNTH_DIRECT if direct else 0)
    s = et.Sim(sim, flags=flags)
    P = et.Paths.from_records(ref)
    H = et.synthesize(ctx, s, P).cpu().numpy()
    st = ctx.stats()
    H_ref = O.synth(ref, sim)
    check_spectra(H, H_ref, f"tiny synthesis {layout} (kernel {st.synth_kernel})")
    assert st.synth_kernel == kernel


def test_end_to_end_tiny_certified(et, ctx, tiny):
    scene, sim, ref = tiny
    dirs = sim["ray_dirs"][ref["certified"]]
    ref_c = O.trace(scene, sim, dirs=dirs)
    H_ref = O.synth(ref_c, sim)
    sc = et.Scene(ctx, scene)
    s = et.Sim(sim, ray_dirs=dirs)
    H = et.simulate(ctx, sc, s).cpu().numpy()
    check_spectra(H, H_ref, "tiny end to end (certified rays)")


def test_determinism(et, ctx, tiny):
    scene, sim, _ = tiny
    sc = et.Scene(ctx, scene)
    s = et.Sim(sim)
    H1 = et.simulate(ctx, sc, s).cpu().numpy()
    H2 = et.simulate(ctx, sc, s).cpu().numpy()
    assert np.array_equal(H1, H2)


@pytest.fixture(scope="module")
def room_small():
    """Room scene geometry (full 193,212 triangles), a seeded subset of its rays."""
    scene, sim = W.room_scene(n_rays=1 << 20)
    g = W.rng(77)
    sub = np.sort(g.choice(len(sim["ray_dirs"]), 2048, replace=False))
    return scene, sim, sub


def test_trace_parity_room_subset(et, ctx, room_small):
    scene, sim, sub = room_small
    dirs = sim["ray_dirs"][sub]
    ref = O.trace(scene, sim, dirs=dirs)
    sc = et.Scene(ctx, scene, area_ref=sim["area_ref"])
    info = sc.info()
    print(f"room BVH: nodes {info.n_nodes} depth {info.depth} SAH {info.sah_cost:.1f} build {info.build_ms:.1f} ms")
    s = et.Sim(sim, flags=et.ET_SPECULAR, ray_dirs=dirs)
    P = et.trace(ctx, sc, s)
    st = ctx.stats()
    gpu = P.to_host()
    cert = ref["certified"]
    mism = compare_traces(gpu, ref, cert)
    print(f"room subset: records gpu {st.records} oracle {len(ref['rtot'])}, certified {cert.mean():.4f}, mismatches {mism}")
    assert mism == 0
    assert st.stack_overflows == 0


@pytest.mark.parametrize("direct", [False, True])
def test_synthesis_isolation_room(et, ctx, room_small, direct):
    """32 receivers x 4096 bins; the oracle evaluates a seeded sample of 96 bins."""
    scene, sim, sub = room_small
    ref = O.trace(scene, sim, dirs=sim["ray_dirs"][sub[:1024]], certify=False)
    flags = et.ET_SPECULAR | (et.ET_SYNTH_DIRECT if direct else 0)
    s = et.Sim(sim, flags=flags)
    P = et.Paths.from_records(ref)
    H = et.synthesize(ctx, s, P).cpu().numpy()
    bins = np.sort(W.rng(5).choice(sim["F"], 96, replace=False))
    bins[0], bins[-1] = 0, sim["F"] - 1
    H_ref = O.synth(ref, sim, bins=bins)
    check_spectra(H[:, bins], H_ref, f"room synthesis ({'direct' if direct else 'factorised'}), "
                  f"{len(ref['rtot'])} records, 96 sampled bins")


@pytest.mark.parametrize("direct", [False, True])
def test_synthesis_room_all_bins(et, ctx, room_small, direct):
    """Every one of the 4096 bins of all 32 receivers, for 256 records of the room."""
    scene, sim, sub = room_small
    ref = O.trace(scene, sim, dirs=sim["ray_dirs"][sub[1024:1088]], certify=False)
    rec = {k: v[:256] for k, v in ref.items() if k not in ("certified", "nseg")}
    s = et.Sim(sim, flags=et.ET_SPECULAR | (et.ET_SYNTH_DIRECT if direct else 0))
    H = et.synthesize(ctx, s, et.Paths.from_records(rec)).cpu().numpy()
    check_spectra(H, O.synth(rec, sim), f"room synthesis, all bins ({'direct' if direct else 'factorised'}), "
                  f"{len(rec['rtot'])} records")


# ----------------------------------------------------------------------------- diffraction

def _diffraction_case(per_mesh, max_meshes=None):
    g = W.rng(31)
    scene = W.room_geometry(g, n_boxes=30, n_cyl=30)
    a_ref = W.median_triangle_area(scene)
    sim = W.make_sim(emitter_pos=[1.0, 4.0, 1.2], emitter_rot=np.eye(3), rx_pos=[[1.0, 4.02, 1.2]],
                     ray_dirs=np.zeros((0, 3)), max_bounces=1, f_lo=20e3, f_hi=100e3, F=256,
                     refl_k=np.full((16, 8), 0.8), lobe_beta=np.full((16, 8), 0.1), diff_coef=np.full((16, 8), 0.2),
                     diff_K=512 if per_mesh else 8192, diff_seed=1234, diff_tau=0.1, diff_max_incidence_deg=80.0,
                     diff_cone_half_angle_deg=90.0, diff_per_mesh=per_mesh,
                     diff_max_meshes=max_meshes or scene["n_objects"])
    return scene, sim, a_ref


@pytest.mark.parametrize("per_mesh", [False, True])
def test_diffraction_samples_match(et, ctx, per_mesh):
    """One CDF (diff_K draws) or a CDF per mesh (diff_K draws for each of the meshes with
    eligible triangles, Sec. III-D): the GPU's kept samples against the oracle's."""
    scene, sim, a_ref = _diffraction_case(per_mesh)
    _, C_ref = O.curvature(scene, a_ref)
    ref = O.diffraction(scene, sim, C_ref)
    sc = et.Scene(ctx, scene, area_ref=a_ref)
    s = et.Sim(sim, flags=et.ET_DIFFRACTION | (et.ET_DIFF_PER_MESH if per_mesh else 0))
    P = et.trace(ctx, sc, s)
    st = ctx.stats()
    gpu = P.to_host()
    assert st.diff_eligible == ref["n_elig"]
    if per_mesh:
        print(f"per-mesh: {len(ref['tri']) // sim['diff_K']} meshes x {sim['diff_K']} draws")
        assert len(ref["tri"]) > sim["diff_K"] and not ref["truncated"]
    kept = np.nonzero(ref["keep"])[0]
    # GPU records: kept samples in sample order, ray field = sample index
    g_idx = gpu["ray"]
    cert = ref["certified"]
    g_set = set(g_idx.tolist())
    flips = [k for k in range(len(cert)) if cert[k] and ((k in g_set) != bool(ref["keep"][k]))]
    print(f"diffraction: eligible {st.diff_eligible}, kept gpu {len(g_idx)} oracle {len(kept)}, "
          f"certified {cert.mean():.4f}, keep mismatches on certified {len(flips)}")
    assert not flips
    common = np.intersect1d(g_idx, kept)
    pos = {k: i for i, k in enumerate(g_idx)}
    for k in common:
        i = pos[k]
        assert gpu["tri"][i] == ref["tri"][k]
        assert np.array_equal(gpu["p"][i], ref["o"][k])          # same FP64 operations: bit-equal
        assert gpu["rtot"][i] == ref["r_src"][k]


def test_diffraction_per_mesh_cap(et, ctx):
    """More eligible meshes than diff_max_meshes: the first meshes keep their draws (the same
    as without the cap, the last kept mesh's CDF ending at its own last triangle) and the trace
    reports a capacity error.  Four kept meshes: the fourth keeps 70 of its draws."""
    MM = 4
    scene, sim, a_ref = _diffraction_case(True, max_meshes=MM)
    _, C_ref = O.curvature(scene, a_ref)
    ref = O.diffraction(scene, sim, C_ref)
    K = sim["diff_K"]
    assert ref["truncated"] and len(ref["tri"]) == MM * K
    sc = et.Scene(ctx, scene, area_ref=a_ref)
    s = et.Sim(sim, flags=et.ET_DIFFRACTION | et.ET_DIFF_PER_MESH)
    P = et.trace(ctx, sc, s)
    with pytest.raises(et.EchoError) as e:
        ctx.stats()
    assert e.value.status == -3
    gpu = P.to_host()
    g_idx = gpu["ray"]
    assert g_idx.max() < MM * K
    # every certified draw of the kept meshes: same keep decision, triangle, point and path as
    # the oracle's
    cert = ref["certified"]
    g_set = set(g_idx.tolist())
    flips = [k for k in range(len(cert)) if cert[k] and ((k in g_set) != bool(ref["keep"][k]))]
    assert not flips
    pos = {k: i for i, k in enumerate(g_idx)}
    common = np.intersect1d(g_idx, np.nonzero(ref["keep"])[0])
    last = 0
    for k in common:
        i = pos[k]
        assert gpu["tri"][i] == ref["tri"][k]
        assert np.array_equal(gpu["p"][i], ref["o"][k])
        assert gpu["rtot"][i] == ref["r_src"][k]
        last += k >= (MM - 1) * K
    # the oracle's draws of each group stay on that group's mesh
    obj = np.asarray(scene["tri_object"])
    meshes = [len(set(obj[ref["tri"][g * K:(g + 1) * K]].tolist())) for g in range(MM)]
    print(f"capped per-mesh: {len(common)} kept draws compared, {last} of the last kept mesh; meshes per group {meshes}")
    assert last > 0 and meshes == [1] * MM


# ----------------------------------------------------------------------------- adjoint

ADJOINT_CASES = {
    # name: (bins, material bands, forced direct, diffraction records added, kernel expected)
    "factorised_F512": (512, 8, False, False, 1),
    "factorised_F8192_two_tiles": (8192, 16, False, False, 1),
    "factorised_F1024_bands_on_256_bins": (1024, 4, False, False, 1),   # 16 outer indices, band edges on 4 of them
    "factorised_F3072_bands_off_256_bins": (3072, 16, False, False, 1),  # 48 outer indices, 3 per band
    "factorised_F4096_bands_on_256_bins": (4096, 16, False, False, 1),   # a full 64-row tile, 4 per band
    "factorised_F1280_partial_group": (1280, 5, False, False, 1),        # 20 rows, 4 per band
    "factorised_F512_diffraction": (512, 8, False, True, 1),
    "direct_F512": (512, 8, True, False, 2),
    "direct_F500": (500, 4, False, False, 2),      # bins not a multiple of 64
}


@pytest.mark.parametrize("case", list(ADJOINT_CASES))
def test_adjoint_matches_oracle_gradient(et, ctx, tiny, case):
    """dL/dk and dL/dx_m of L = sum |H - H*|^2 from the GPU adjoint vs the FP64 oracle gradient."""
    scene, sim, ref = tiny
    F, Bk, direct, diffraction, kernel = ADJOINT_CASES[case]
    g = W.rng(8)
    sim = dict(sim, F=F, refl_k=g.uniform(0.3, 0.99, (1, Bk)).astype(np.float32),
               lobe_beta=g.uniform(0.05, 0.3, (1, Bk)).astype(np.float32),
               diff_coef=g.uniform(0.05, 0.3, (1, Bk)).astype(np.float32))
    if F > 4096:   # keep the FP64 oracle to seconds: a ray subset
        ref = O.trace(scene, sim, dirs=sim["ray_dirs"][:2048], certify=False)
    if diffraction:
        _, C_ref = O.curvature(scene, W.median_triangle_area(scene))
        smp = O.diffraction(scene, dict(sim, diff_K=4096, diff_seed=77), C_ref)
        ref = O.concat_records(ref, O.diffraction_records(scene, smp))
    hidden = dict(sim, refl_k=g.uniform(0.3, 0.99, (1, Bk)).astype(np.float32),
                  diff_coef=g.uniform(0.05, 0.3, (1, Bk)).astype(np.float32))
    H_star = O.synth(ref, hidden)
    H = O.synth(ref, sim)
    gk_ref, gx_ref = O.grad(ref, sim, H - H_star)
    import torch
    s = et.Sim(sim, flags=et.ET_SPECULAR | (et.ET_SYNTH_DIRECT if direct else 0))
    P = et.Paths.from_records(ref)
    gk, gx = et.synthesize_backward(ctx, s, P, torch.as_tensor(H - H_star).to("cuda"))
    st = ctx.stats()
    gk, gx = gk.cpu().numpy(), gx.cpu().numpy()
    ek, ex = rel_l2(gk, gk_ref), rel_l2(gx, gx_ref)
    print(f"adjoint {case} (kernel {st.adjoint_kernel}, {len(ref['rtot'])} records): rel err dL/dk {ek:.3e}, "
          f"dL/dx {ex:.3e}")
    assert st.adjoint_kernel == kernel
    assert ek <= TOL and ex <= TOL


@pytest.mark.parametrize("direct", [False, True])
def test_adjoint_at_zero_coefficients(et, ctx, tiny, direct):
    """dL/dk where some band coefficients are exactly zero: H is linear in k, so the gradient
    there is the sum over the band's terms without k (not zero), and the other coefficients and
    the receiver gradient are unaffected; both adjoint kernels against the oracle gradient."""
    import torch
    scene, sim, ref = tiny
    g = W.rng(9)
    k = g.uniform(0.3, 0.99, (1, 8)).astype(np.float32)
    k[0, 1] = 0.0
    k[0, 6] = 0.0
    sim = dict(sim, F=512, refl_k=k, lobe_beta=g.uniform(0.05, 0.3, (1, 8)).astype(np.float32))
    H_star = O.synth(ref, dict(sim, refl_k=g.uniform(0.3, 0.99, (1, 8)).astype(np.float32)))
    H = O.synth(ref, sim)
    gk_ref, gx_ref = O.grad(ref, sim, H - H_star)
    s = et.Sim(sim, flags=et.ET_SPECULAR | (et.ET_SYNTH_DIRECT if direct else 0))
    gk, gx = et.synthesize_backward(ctx, s, et.Paths.from_records(ref), torch.as_tensor(H - H_star).to("cuda"))
    st = ctx.stats()
    gk, gx = gk.cpu().numpy(), gx.cpu().numpy()
    ek, ex = rel_l2(gk, gk_ref), rel_l2(gx, gx_ref)
    ez = rel_l2(gk[0, [1, 6]], gk_ref[0, [1, 6]])
    print(f"adjoint with k = 0 bands (kernel {st.adjoint_kernel}): dL/dk {ek:.3e} (zero bands {ez:.3e}), dL/dx {ex:.3e}")
    assert st.adjoint_kernel == (2 if direct else 1)
    assert np.all(np.abs(gk_ref[0, [1, 6]]) > 1e-3 * np.max(np.abs(gk_ref)))
    assert ek <= TOL and ex <= TOL and ez <= TOL


def test_adjoint_with_directivity_matches_oracle_gradient(et, ctx, tiny):
    """Receiver directivity (a rough 32 x 64 table per band and receiver, four bands, rotated
    receiver frames): the per-term adjoint's dL/dk and dL/dx_m, whose direction-of-arrival term
    moves the receivers' gradient, against the FP64 oracle gradient."""
    scene, sim, ref = tiny
    g = W.rng(31)
    M = len(sim["rx_pos"])
    rot = []
    for i in range(M):
        a, b = 0.5 + 0.7 * i, 0.2 - 0.4 * i
        rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
        ry = np.array([[np.cos(b), 0, np.sin(b)], [0, 1, 0], [-np.sin(b), 0, np.cos(b)]])
        rot.append(rz @ ry)
    sim = dict(sim, F=512, refl_k=g.uniform(0.3, 0.99, (1, 8)).astype(np.float32),
               lobe_beta=g.uniform(0.05, 0.3, (1, 8)).astype(np.float32), rx_rot=np.stack(rot),
               directivity=np.ascontiguousarray(g.uniform(0.2, 1.0, (M, 4, 32, 64)).astype(np.float32)))
    hidden = dict(sim, refl_k=g.uniform(0.3, 0.99, (1, 8)).astype(np.float32),
                  rx_pos=sim["rx_pos"] + g.normal(0, 2e-3, sim["rx_pos"].shape))
    H_star = O.synth(ref, hidden)
    H = O.synth(ref, sim)
    gk_ref, gx_ref = O.grad(ref, sim, H - H_star)
    _, gx_plain = O.grad(ref, dict(sim, directivity=None), H - H_star)
    import torch
    s = et.Sim(sim, flags=et.ET_SPECULAR)
    P = et.Paths.from_records(ref)
    gk, gx = et.synthesize_backward(ctx, s, P, torch.as_tensor(H - H_star).to("cuda"))
    st = ctx.stats()
    gk, gx = gk.cpu().numpy(), gx.cpu().numpy()
    ek, ex = rel_l2(gk, gk_ref), rel_l2(gx, gx_ref)
    print(f"adjoint with directivity (kernel {st.adjoint_kernel}, {len(ref['rtot'])} records): rel err dL/dk "
          f"{ek:.3e}, dL/dx {ex:.3e}; the directivity term moves dL/dx by {rel_l2(gx_plain, gx_ref):.2e}")
    assert st.adjoint_kernel == 2
    assert rel_l2(gx_plain, gx_ref) > 100 * TOL
    assert ek <= TOL and ex <= TOL


# ----------------------------------------------------------------------------- passive component

def _passive_sim(sim, rx):
    g = W.rng(21)
    return dict(sim, rx_pos=np.asarray(rx, float), rx_rot=np.repeat(np.eye(3)[None], len(rx), axis=0),
                x_ref=np.asarray(rx, float).mean(axis=0),
                passive_coef=g.uniform(0.2, 1.0, sim["refl_k"].shape[1]).astype(np.float32))


@pytest.mark.parametrize("direct", [False, True])
def test_passive_component_matches_oracle(et, ctx, tiny, direct):
    """Receivers in front of and behind the wall (x = 4): the GPU's line-of-sight decisions
    match the oracle's, the passive records follow the others, and the spectra (specular on
    certified rays + passive) match the oracle's."""
    scene, sim, _ = tiny
    sim = _passive_sim(sim, [[0.0, 0.3, 0.1], [0.2, -0.4, 0.0], [5.0, 0.3, 0.1], [4.5, -1.0, 0.5]])
    vis_ref, cert = O.passive(scene, sim)
    assert cert.all() and list(vis_ref) == [True, True, False, False]
    ref = O.trace(scene, sim)
    dirs = sim["ray_dirs"][ref["certified"]]
    ref_c = O.trace(scene, sim, dirs=dirs)
    rec_ref = O.concat_records(ref_c, O.passive_records(sim, vis_ref))
    sc = et.Scene(ctx, scene)
    flags = et.ET_SPECULAR | et.ET_PASSIVE | (et.ET_SYNTH_DIRECT if direct else 0)
    s = et.Sim(sim, flags=flags, ray_dirs=dirs)
    P = et.trace(ctx, sc, s)
    st = ctx.stats()
    gpu = P.to_host()
    assert st.passive == 4 and st.records == len(rec_ref["rtot"])
    tail = slice(len(gpu["rtot"]) - 4, None)
    assert list(gpu["kind"][tail]) == [2, 2, 2, 2] and list(gpu["mat"][tail]) == [0, 1, 2, 3]
    assert list(gpu["vis"][tail].astype(bool)) == list(vis_ref)
    H = et.synthesize(ctx, s, P).cpu().numpy()
    assert ctx.stats().synth_kernel == (2 if direct else 1)
    H_ref = O.synth(rec_ref, sim)
    check_spectra(H, H_ref, f"passive ({'direct' if direct else 'factorised'}; receivers behind the wall keep "
                  f"only echoes)")


def test_passive_adjoint_matches_oracle(et, ctx, tiny):
    """Adjoint over specular + passive records: the direct path's receiver gradient included."""
    import torch
    scene, sim, ref = tiny
    sim = _passive_sim(dict(sim, F=512), [[0.3, 0.4, 0.1], [0.2, -0.5, -0.1]])
    ref = O.trace(scene, sim, certify=False)
    rec = O.concat_records(ref, O.passive_records(sim, [True, True]))
    g = W.rng(22)
    H_star = O.synth(rec, dict(sim, rx_pos=sim["rx_pos"] + g.normal(0, 1e-3, (2, 3))))
    H = O.synth(rec, sim)
    gk_ref, gx_ref = O.grad(rec, sim, H - H_star)
    s = et.Sim(sim, flags=et.ET_SPECULAR | et.ET_PASSIVE)
    P = et.Paths.from_records(rec)
    gk, gx = et.synthesize_backward(ctx, s, P, torch.as_tensor(H - H_star).to("cuda"))
    ek, ex = rel_l2(gk.cpu().numpy(), gk_ref), rel_l2(gx.cpu().numpy(), gx_ref)
    print(f"passive adjoint (kernel {ctx.stats().adjoint_kernel}): rel err dL/dk {ek:.3e}, dL/dx {ex:.3e}")
    assert ek <= TOL and ex <= TOL


# ----------------------------------------------------------------------------- time domain

@pytest.mark.parametrize("sigma,n_t", [(1, 4096), (-1, 4096), (1, 1024), (1, 65536), (-1, 32768)])
def test_impulse_response_matches_oracle(et, ctx, tiny, sigma, n_t):
    """h = F^-1[H] of the tiny scene's spectra (1024 bins 20-100 kHz; n_t = 4096 samples at
    320 kHz, the minimum n_t = F, and rows too long for one workgroup's LDS: radix-4 passes
    over global memory, with a radix-2 pass first for an odd power of two) against the
    oracle's definition."""
    import torch
    scene, sim, ref = tiny
    sim = dict(sim, phase_sign=sigma)
    H = O.synth(ref, sim)
    s = et.Sim(sim)
    h, dt = et.impulse_response(ctx, s, torch.as_tensor(H, dtype=torch.complex64, device="cuda"), n_t)
    h_ref, dt_ref = O.impulse_response(H.astype(np.complex64), sim, n_t)
    e = rel_l2(h.cpu().numpy(), h_ref)
    print(f"impulse response (sigma {sigma}, n_t {n_t}): rel L2 {e:.3e}, dt {dt:.3e} s")
    assert dt == pytest.approx(dt_ref, rel=1e-15)
    assert e <= 1e-5


def test_receiver_signal_matches_oracle(et, ctx, tiny):
    """s = h * s_e for a 20-100 kHz chirp of an odd length (the FFT length pads to a power of two)."""
    import torch
    scene, sim, ref = tiny
    H = O.synth(ref, sim)
    s = et.Sim(sim)
    h, dt = et.impulse_response(ctx, s, torch.as_tensor(H, dtype=torch.complex64, device="cuda"), 4096)
    L = 641
    t = np.arange(L) * dt
    T = L * dt
    s_e = np.sin(2 * np.pi * (20e3 * t + 0.5 * (80e3 / T) * t * t)) * np.hanning(L)
    out = et.receiver_signal(ctx, h, torch.as_tensor(s_e, dtype=torch.float32, device="cuda"), dt)
    ref_s = O.receiver_signal(h.cpu().numpy().astype(np.float64), s_e.astype(np.float32), dt)
    e = rel_l2(out.cpu().numpy(), ref_s)
    print(f"receiver signal: {out.shape[1]} samples, rel L2 {e:.3e}")
    assert out.shape == (2, 4096 + L - 1)
    assert e <= 1e-5


def test_time_domain_rejects_bad_shapes(et, ctx, tiny):
    import torch
    scene, sim, ref = tiny
    s = et.Sim(sim)
    H = torch.zeros(2, sim["F"], dtype=torch.complex64, device="cuda")
    for n_t in (3000, 512):              # not a power of two; shorter than F
        with pytest.raises(et.EchoError) as e:
            et.impulse_response(ctx, s, H, n_t)
        assert e.value.status == -1


# ----------------------------------------------------------------------------- errors

def test_invalid_arguments_report_status(et, ctx, tiny):
    import ctypes
    scene, sim, _ = tiny
    sc = et.Scene(ctx, scene)
    s = et.Sim(sim)
    bad = et.Sim(sim)
    bad.desc.max_bounces = 0
    with pytest.raises(et.EchoError) as e:
        et.trace(ctx, sc, bad)
    assert e.value.status == -1
    P = et.Paths(4)
    n = ctypes.c_size_t()
    buf = et.Workspace().get(16)
    rc = et.lib().et_trace(ctx.h, sc.h, ctypes.byref(s.desc), ctypes.c_void_p(buf.data_ptr()), 16, ctypes.byref(P.desc))
    assert rc == -2                                            # workspace too small
    # capacity: 4 records for 16384 rays -> deferred ET_E_CAPACITY
    ws = et.Workspace()
    et.trace(ctx, sc, s, paths=P, ws=ws)
    with pytest.raises(et.EchoError) as e:
        ctx.stats()
    assert e.value.status == -3
    assert P.count[0].item() > 4


# ----------------------------------------------------------------------------- EQ ray sets

@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 10, 33, 100, 1000, 4097, 65536, 1 << 20])
def test_eq_directions_match_oracle(et, ctx, N):
    """Region centres of EQ(2, N): the collar counts decide integers, so the sets must have
    the same size and order; values agree to FP32 rounding of FP64 arithmetic."""
    D = et.eq_directions(ctx, N).cpu().numpy().astype(np.float64)
    R = O.eq_directions(N)
    assert D.shape == R.shape
    err = float(np.max(np.abs(D - R)))
    print(f"EQ N={N}: max |diff| {err:.2e}, bitwise-equal fraction {np.mean(D == R.astype(np.float32)):.6f}")
    assert err <= 1.2e-7


def test_eq_cone_and_errors(et, ctx):
    import ctypes
    N, a = 1 << 20, math.radians(30.0)
    R = O.eq_directions(N, a)
    b, z = O.eq_zones(N)
    mids = [(b[k] + b[k + 1]) / 2 for k in range(1, len(z) - 1)]
    assert min(abs(t - a) for t in mids) > 1e-9   # the cone's edge is clear of every collar's centre
    D = et.eq_directions(ctx, N, a).cpu().numpy()
    assert D.shape == R.shape
    assert float(np.max(np.abs(D - R))) <= 1.2e-7
    n = ctypes.c_size_t()
    assert et.lib().et_eq_directions_workspace_size(0, ctypes.byref(n)) == -1
    assert et.lib().et_eq_directions_workspace_size(N, ctypes.byref(n)) == 0
    ws = et.Workspace().get(n.value)
    cnt = ctypes.c_int64()
    out = et.Workspace().get(64)
    args = (ctypes.c_void_p(ws.data_ptr()), n.value)
    assert et.lib().et_eq_directions(ctx.h, N, 0.0, *args, None, 0, ctypes.byref(cnt)) == -1
    assert et.lib().et_eq_directions(ctx.h, N, a, *args, None, 0, None) == -1
    assert et.lib().et_eq_directions(ctx.h, N, a, ctypes.c_void_p(ws.data_ptr()), 8, None, 0, ctypes.byref(cnt)) == -2
    rc = et.lib().et_eq_directions(ctx.h, N, a, *args, ctypes.c_void_p(out.data_ptr()), 5, ctypes.byref(cnt))
    assert rc == -3 and cnt.value == len(R)


def test_trace_with_eq_directions(et, ctx, tiny):
    """The tiny scene traced with the EQ ray set of its 60-degree cone (about 16k rays)."""
    scene, sim, _ = tiny
    N, a = 245760, math.radians(30.0)
    R = O.eq_directions(N, a)
    D = et.eq_directions(ctx, N, a)
    assert np.array_equal(D.cpu().numpy(), R.astype(np.float32))
    ref = O.trace(scene, sim, dirs=R.astype(np.float32))
    sc = et.Scene(ctx, scene)
    gpu = et.trace(ctx, sc, et.Sim(sim, ray_dirs=D)).to_host()
    mism = compare_traces(gpu, ref, ref["certified"])
    print(f"EQ rays {len(R)}: certified {ref['certified'].mean():.4f}, mismatches {mism}")
    assert mism == 0


# ----------------------------------------------------------------------------- several emitters

def _emitter_sims(sim, scene_rot_deg=(0.0, 12.0, -8.0), pos=((0, 0, 0), (0.0, 0.4, 0.15), (0.2, -0.3, -0.1))):
    out = []
    for a, p in zip(scene_rot_deg, pos):
        c, s = math.cos(math.radians(a)), math.sin(math.radians(a))
        out.append(dict(sim, emitter_pos=np.array(p, float), emitter_rot=np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])))
    return out


def test_emitters_sum_matches_oracle(et, ctx, tiny):
    """Three simultaneous emitters (specular, fused batch): the spectra equal the sum of the
    oracle's per-emitter spectra on each emitter's certified rays."""
    scene, sim, _ = tiny
    sims = _emitter_sims(sim)
    H_ref = 0
    gs = []
    for se in sims:
        ref = O.trace(scene, se)
        dirs = se["ray_dirs"][ref["certified"]]
        H_ref = H_ref + O.synth(O.trace(scene, se, dirs=dirs), se)
        gs.append(et.Sim(se, ray_dirs=dirs))
    for g in gs[1:]:
        g.rx_pos = gs[0].rx_pos
        g.refresh()
    sc = et.Scene(ctx, scene)
    H = et.simulate_emitters(ctx, sc, gs).cpu().numpy()
    check_spectra(H, H_ref, "3 emitters vs oracle")
    each = sum(et.simulate(ctx, sc, g).cpu().numpy().astype(np.complex128) for g in gs)
    print(f"3 emitters vs sum of single-emitter calls {rel_l2(H, each):.3e}")
    assert rel_l2(H, each) <= 1e-6


def test_emitters_with_diffraction_and_passive(et, ctx, tiny):
    """Emitters with diffraction and the passive component run job after job; the sum equals
    the single-emitter calls, and mismatched receivers are rejected."""
    scene, sim, _ = tiny
    sims = _emitter_sims(dict(sim, diff_K=4096, diff_seed=3, diff_tau=0.05, passive_coef=np.full(8, 0.5, np.float32)))
    gs = [et.Sim(se) for se in sims]
    for g in gs[1:]:
        g.rx_pos = gs[0].rx_pos
        g.refresh()
    sc = et.Scene(ctx, scene, area_ref=W.median_triangle_area(scene))
    H = et.simulate_emitters(ctx, sc, gs).cpu().numpy()
    each = sum(et.simulate(ctx, sc, g).cpu().numpy().astype(np.complex128) for g in gs)
    print(f"3 emitters with diffraction + passive: rel L2 vs single calls {rel_l2(H, each):.3e}")
    assert rel_l2(H, each) <= 1e-6
    other = et.Sim(sims[1])
    with pytest.raises(et.EchoError) as e:
        et.simulate_emitters(ctx, sc, [gs[0], other])
    assert e.value.status == -1


# ----------------------------------------------------------------------------- alternative readings

def _screen_scene():
    """A wall 4 m ahead and a small screen that hides part of it from the receiver at +y."""
    mb = W.MeshBuilder()
    mb.add(np.array([[4, -3, -2], [4, 3, -2], [4, 3, 2], [4, -3, 2]], float), np.array([[0, 1, 2], [0, 2, 3]]), 0)
    mb.add(np.array([[1.5, 0.05, -0.6], [1.5, 0.8, -0.6], [1.5, 0.8, 0.6], [1.5, 0.05, 0.6]], float),
           np.array([[0, 1, 2], [0, 2, 3]]), 1)
    return mb.build()


@pytest.mark.parametrize("direct", [False, True])
def test_path_product_matches_oracle(et, ctx, direct):
    """Path-product reading (k multiplied over every reflection of the ray): records chain
    through prev, and the spectra match the oracle's on certified rays, both kernels."""
    scene = _screen_scene()
    g = W.rng(12)
    k = np.array([[0.9, 0.8, 0.85, 0.7, 0.95, 0.6, 0.75, 0.5], [0.4, 0.5, 0.6, 0.7, 0.3, 0.9, 0.2, 0.8]], np.float32)
    sim = W.make_sim(emitter_pos=[0, 0, 0], emitter_rot=np.eye(3), rx_pos=[[0, 0.3, 0], [0, -0.3, 0]],
                     ray_dirs=W.cone_directions(g, 8192, math.radians(35)), max_bounces=4, f_lo=20e3, f_hi=100e3,
                     F=1024, refl_k=k, lobe_beta=np.full((2, 8), 0.3, np.float32),
                     diff_coef=np.full((2, 8), 0.1, np.float32), path_product=True)
    ref = O.trace(scene, sim)
    dirs = sim["ray_dirs"][ref["certified"]]
    ref_c = O.trace(scene, sim, dirs=dirs)
    H_ref = O.synth(ref_c, sim)
    assert np.any(ref_c["bounce"] > 0)
    sc = et.Scene(ctx, scene)
    s = et.Sim(sim, ray_dirs=dirs, flags=et.ET_SPECULAR | et.ET_PATH_PRODUCT | (et.ET_SYNTH_DIRECT if direct else 0))
    P = et.trace(ctx, sc, s)
    H = et.synthesize(ctx, s, P).cpu().numpy()
    h = P.to_host()
    # every record after a ray's first reflection points at that ray's previous reflection
    for i in np.nonzero(h["bounce"] > 0)[0][:2000]:
        j = h["prev"][i]
        assert 0 <= j < i and h["ray"][j] == h["ray"][i] and h["bounce"][j] == h["bounce"][i] - 1
    assert np.all(h["prev"][h["bounce"] == 0] == -1)
    lit = O.synth(ref_c, dict(sim, path_product=False))
    check_spectra(H, H_ref, f"path product ({'direct' if direct else 'factorised'}; literal reading differs by "
                  f"{rel_l2(lit, H_ref):.2e})")
    assert ctx.stats().synth_kernel == (2 if direct else 1)
    with pytest.raises(et.EchoError) as ex:
        et.synthesize_backward(ctx, s, P, torch_randn_like(H))
    assert ex.value.status == -5


def torch_randn_like(H):
    import torch
    g = torch.Generator(device="cuda").manual_seed(3)
    return torch.randn(H.shape, dtype=torch.complex64, device="cuda", generator=g)


def test_per_receiver_visibility_matches_oracle(et, ctx):
    """Per-receiver line of sight: the receiver bits of every certified ray's records, the
    spectra and the adjoint match the oracle's; a fused batch of such jobs equals single calls."""
    scene = _screen_scene()
    g = W.rng(13)
    sim = W.make_sim(emitter_pos=[0, 0, 0], emitter_rot=np.eye(3), rx_pos=[[0, 0.3, 0], [0, -0.3, 0]],
                     ray_dirs=W.cone_directions(g, 8192, math.radians(35)), max_bounces=3, f_lo=20e3, f_hi=100e3,
                     F=512, refl_k=np.full((2, 8), 0.9, np.float32), lobe_beta=np.full((2, 8), 0.3, np.float32),
                     diff_coef=np.full((2, 8), 0.1, np.float32), per_rx_visibility=True)
    ref = O.trace(scene, sim)
    dirs = sim["ray_dirs"][ref["certified"]]
    ref_c = O.trace(scene, sim, dirs=dirs)
    b = ref_c["rxvis"]
    assert np.any((b & np.uint64(1)) != ((b >> np.uint64(1)) & np.uint64(1)))
    sc = et.Scene(ctx, scene)
    s = et.Sim(sim, ray_dirs=dirs)
    assert s.desc.flags & et.ET_PER_RX_VISIBILITY
    P = et.trace(ctx, sc, s)
    h = P.to_host()
    order_g = np.lexsort((h["bounce"], h["ray"]))
    order_o = np.lexsort((ref_c["bounce"], ref_c["ray"]))
    assert np.array_equal(h["ray"][order_g], ref_c["ray"][order_o])
    assert np.array_equal(h["rxvis"][order_g], ref_c["rxvis"][order_o])
    H = et.synthesize(ctx, s, P).cpu().numpy()
    H_ref = O.synth(ref_c, sim)
    e = check_spectra(H, H_ref, "per-receiver visibility spectra")
    # the adjoint over the same records
    rng = np.random.default_rng(5)
    gH = (rng.normal(size=H.shape) + 1j * rng.normal(size=H.shape)).astype(np.complex64)
    import torch
    gk, gx = et.synthesize_backward(ctx, s, P, torch.as_tensor(gH).cuda())
    gk_ref, gx_ref = O.grad(ref_c, sim, gH.astype(np.complex128))
    ek, ex = rel_l2(gk.cpu().numpy(), gk_ref), rel_l2(gx.cpu().numpy(), gx_ref)
    print(f"per-receiver visibility: spectra rel L2 {e:.3e}, dL/dk {ek:.3e}, dL/dx {ex:.3e}")
    assert e <= TOL and ek <= TOL and ex <= TOL
    # two such emitters run as batch jobs (job after job): their sum equals single calls
    s2 = et.Sim(dict(sim, emitter_pos=np.array([0.1, 0.0, 0.05])), ray_dirs=dirs)
    s2.rx_pos = s.rx_pos
    s2.refresh()
    Hs = et.simulate_emitters(ctx, sc, [s, s2]).cpu().numpy()
    each = et.simulate(ctx, sc, s).cpu().numpy().astype(np.complex128) + et.simulate(ctx, sc, s2).cpu().numpy()
    assert rel_l2(Hs, each) <= 1e-6
