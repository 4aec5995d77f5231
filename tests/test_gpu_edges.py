"""Edge cases of the path against the FP64 oracle: an empty scene, no rays, scenes of one and
two triangles (the smallest trees), ragged and single-bin frequency grids, a large grid over
several tiles, and rays that bounce up to the 255-record limit in a closed room."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import check_spectra, compare_traces, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def ctx(et):
    return et.Context(0)


def _empty_scene():
    return {"vertices": np.zeros((0, 3), np.float32), "tris": np.zeros((0, 3), np.int32),
            "tri_material": np.zeros(0, np.int32), "tri_object": np.zeros(0, np.int32), "n_objects": 1}


def test_empty_scene(et, ctx):
    """No triangles: every ray misses at its first segment; the passive component alone
    reaches the receivers."""
    _, sim = W.tiny_scene(n_rays=256)
    sim = dict(sim, passive_coef=np.full(8, 0.7, np.float32))
    scene = _empty_scene()
    sc = et.Scene(ctx, scene)
    assert sc.info().T == 0
    s = et.Sim(sim, flags=et.ET_SPECULAR | et.ET_PASSIVE)
    P = et.trace(ctx, sc, s)
    st = ctx.stats()
    assert st.specular == 0 and st.passive == s.M and st.segments == 256
    vis, _ = O.passive(scene, sim)
    H_ref = O.synth(O.passive_records(sim, vis), sim)
    H = et.synthesize(ctx, s, P).cpu().numpy()
    check_spectra(H, H_ref, "empty scene, passive component")


def test_zero_rays(et, ctx):
    scene, sim = W.tiny_scene(n_rays=16)
    sc = et.Scene(ctx, scene)
    s = et.Sim(sim, ray_dirs=np.zeros((0, 3), np.float32))
    H = et.simulate(ctx, sc, s).cpu().numpy()
    st = ctx.stats()
    assert st.records == 0 and st.segments == 0
    assert not np.any(H)


@pytest.mark.parametrize("T", [1, 2])
def test_smallest_trees(et, ctx, T):
    """One triangle (a single leaf, no inner node) and two (one inner node)."""
    mb = W.MeshBuilder()
    mb.add(np.array([[3, -1, -1], [3, 1, -1], [3, 0, 1.5]], float), np.array([[0, 1, 2]]), 0)
    if T == 2:
        mb.add(np.array([[5, -3, -3], [5, 3, -3], [5, 0, 3]], float), np.array([[0, 1, 2]]), 0)
    scene = mb.build()
    _, sim = W.tiny_scene(n_rays=4096)
    ref = O.trace(scene, sim)
    sc = et.Scene(ctx, scene)
    gpu = et.trace(ctx, sc, et.Sim(sim)).to_host()
    mism = compare_traces(gpu, ref, ref["certified"])
    print(f"T={T}: records gpu {len(gpu['rtot'])} oracle {len(ref['rtot'])}, certified {ref['certified'].mean():.4f}")
    assert mism == 0


@pytest.fixture(scope="module")
def tiny_records():
    scene, sim = W.tiny_scene()
    ref = O.trace(scene, sim, certify=False)
    return scene, sim, ref


@pytest.mark.parametrize("F", [1, 63, 65, 1000])
def test_ragged_bin_counts(et, ctx, tiny_records, F):
    """Grids that are not a multiple of 64 bins (the per-term kernel) and a single bin."""
    _, sim, ref = tiny_records
    s_f = dict(sim, F=F, f_hi=sim["f_lo"] if F == 1 else sim["f_hi"])
    H_ref = O.synth(ref, s_f)
    s = et.Sim(s_f)
    P = et.Paths.from_records(ref)
    H = et.synthesize(ctx, s, P).cpu().numpy()
    check_spectra(H, H_ref, f"F={F}: kernel {ctx.stats().synth_kernel}")


def test_large_grid_many_tiles(et, ctx, tiny_records):
    """16384 bins 20-200 kHz: the factorised kernel over four tiles of 64 rows; 128 sampled bins
    against the oracle."""
    _, sim, ref = tiny_records
    s_f = dict(sim, F=16384, f_hi=200e3)
    bins = np.sort(W.rng(5).choice(16384, 128, replace=False))
    H_ref = O.synth(ref, s_f, bins=bins)
    s = et.Sim(s_f)
    H = et.synthesize(ctx, s, et.Paths.from_records(ref)).cpu().numpy()
    assert ctx.stats().synth_kernel == 1
    check_spectra(H[:, bins], H_ref, "F=16384, sampled bins")


def test_255_bounces_in_a_closed_room(et, ctx):
    """Rays inside a closed 10 x 8 x 3 m box reflect until the 255-record limit or the
    maximum path length; every certified ray's hits match the oracle's."""
    mb = W.MeshBuilder()
    v, t = W.quad_grid_box([0, 0, 0], [10.0, 8.0, 3.0], 1)
    mb.add(v, t, 0)
    scene = mb.build()
    g = W.rng(8)
    d = g.normal(size=(256, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    _, base = W.tiny_scene(n_rays=16)
    sim = dict(base, emitter_pos=np.array([3.0, 4.0, 1.5]), ray_dirs=d.astype(np.float32), max_bounces=255,
               max_distance=5000.0, rx_pos=np.array([[3.0, 4.02, 1.5]]), rx_rot=np.eye(3)[None],
               x_ref=np.array([3.0, 4.02, 1.5]))
    ref = O.trace(scene, sim)
    sc = et.Scene(ctx, scene)
    gpu = et.trace(ctx, sc, et.Sim(sim)).to_host()
    per_ray = np.bincount(ref["ray"], minlength=256)
    mism = compare_traces(gpu, ref, ref["certified"])
    print(f"closed room: records per ray up to {per_ray.max()}, certified {ref['certified'].mean():.4f}, "
          f"mismatches {mism}")
    assert per_ray.max() == 255
    assert mism == 0


def _distance_stops(ray, rtot, rays, n_rays, B, md):
    """Rays among `rays` whose last record is the one at which the path reached md before B
    records were made."""
    sel = np.isin(ray, rays)
    cnt = np.bincount(ray[sel], minlength=n_rays)
    last = np.full(n_rays, -np.inf)
    np.maximum.at(last, ray[sel], rtot[sel])
    return int(np.sum((cnt < B) & (last >= md)))


@pytest.mark.parametrize("case", ["closed_box_12m", "room_8m"])
def test_max_distance_cuts_paths(et, ctx, case):
    """Algorithm 1's MaxDistance: a hit is recorded, then the ray stops once its path has
    reached the limit.  Closed 10 x 8 x 3 m box with 20 reflection points and a 12 m limit, and
    the room scene's rays (a seeded subset) with an 8 m limit: records of every certified ray
    equal the oracle's, including the record at the crossing, and some rays stop by distance."""
    if case == "closed_box_12m":
        mb = W.MeshBuilder()
        v, t = W.quad_grid_box([0, 0, 0], [10.0, 8.0, 3.0], 1)
        mb.add(v, t, 0)
        scene = mb.build()
        g = W.rng(18)
        d = g.normal(size=(1024, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        _, base = W.tiny_scene(n_rays=16)
        md, B = 12.0, 20
        sim = dict(base, emitter_pos=np.array([3.0, 4.0, 1.5]), ray_dirs=d.astype(np.float32), max_bounces=B,
                   max_distance=md, rx_pos=np.array([[3.0, 4.02, 1.5]]), rx_rot=np.eye(3)[None],
                   x_ref=np.array([3.0, 4.02, 1.5]))
    else:
        scene, sim = W.room_scene(n_rays=1 << 20)
        sub = np.sort(W.rng(78).choice(len(sim["ray_dirs"]), 2048, replace=False))
        md, B = 8.0, sim["max_bounces"]
        sim = dict(sim, ray_dirs=sim["ray_dirs"][sub], max_distance=md)
    ref = O.trace(scene, sim)
    n = len(sim["ray_dirs"])
    sc = et.Scene(ctx, scene)
    gpu = et.trace(ctx, sc, et.Sim(sim, flags=et.ET_SPECULAR)).to_host()
    st = ctx.stats()
    cert = ref["certified"]
    mism = compare_traces(gpu, ref, cert)
    rays_c = np.nonzero(cert)[0]
    stops_g = _distance_stops(gpu["ray"], gpu["rtot"], rays_c, n, B, md)
    stops_o = _distance_stops(ref["ray"], ref["rtot"], rays_c, n, B, md)
    print(f"{case}: {n} rays, certified {cert.mean():.4f}, records gpu {st.records} oracle {len(ref['rtot'])}, "
          f"certified rays stopped by distance: gpu {stops_g} oracle {stops_o}, mismatches {mism}")
    assert mism == 0 and st.stack_overflows == 0
    assert stops_g == stops_o and stops_o > 0.1 * len(rays_c)


# ----------------------------------------------------------------------------- maximum sizes

def _tiny_materials(scene, sim, Q, Bk, F, n_rays, seed):
    """The tiny scene with Q materials drawn per triangle and Bk bands."""
    g = W.rng(seed)
    scene = dict(scene, tri_material=g.integers(0, Q, len(scene["tris"])).astype(np.int32))
    sim = dict(sim, F=F, ray_dirs=sim["ray_dirs"][:n_rays],
               refl_k=g.uniform(0.3, 0.99, (Q, Bk)).astype(np.float32),
               lobe_beta=g.uniform(0.05, 0.3, (Q, Bk)).astype(np.float32),
               diff_coef=g.uniform(0.05, 0.3, (Q, Bk)).astype(np.float32))
    return scene, sim, g


def test_adjoint_at_its_limits(et, ctx):
    """The adjoint at the largest accepted shape (12288 bins, 16 bands, 16 materials, so
    Q Bk = 256) against the oracle gradient; one step past each limit is refused with
    ET_E_UNSUPPORTED."""
    import torch
    base_scene, base_sim = W.tiny_scene(n_rays=1024)
    scene, sim, g = _tiny_materials(base_scene, base_sim, 16, 16, 12288, 1024, 51)
    ref = O.trace(scene, sim, certify=False)
    hidden = dict(sim, refl_k=g.uniform(0.3, 0.99, (16, 16)).astype(np.float32))
    H_star = O.synth(ref, hidden)
    H = O.synth(ref, sim)
    gk_ref, gx_ref = O.grad(ref, sim, H - H_star)
    P = et.Paths.from_records(ref)
    gk, gx = et.synthesize_backward(ctx, et.Sim(sim), P, torch.as_tensor(H - H_star).to("cuda"))
    st = ctx.stats()
    ek, ex = rel_l2(gk.cpu().numpy(), gk_ref), rel_l2(gx.cpu().numpy(), gx_ref)
    print(f"adjoint at F=12288, Q=Bk=16 (kernel {st.adjoint_kernel}, {len(ref['rtot'])} records): "
          f"dL/dk {ek:.3e}, dL/dx {ex:.3e}")
    assert st.adjoint_kernel == 1
    assert ek <= TOL and ex <= TOL
    over = [dict(sim, F=12352),                                                        # F > 12288
            dict(sim, refl_k=np.full((16, 17), 0.5, np.float32), lobe_beta=np.full((16, 17), 0.2, np.float32),
                 diff_coef=np.full((16, 17), 0.1, np.float32)),                      # Bk > 16
            dict(sim, refl_k=np.full((17, 16), 0.5, np.float32), lobe_beta=np.full((17, 16), 0.2, np.float32),
                 diff_coef=np.full((17, 16), 0.1, np.float32))]                      # Q Bk > 256
    for bad in over:
        s = et.Sim(bad)
        gb = torch.zeros(s.M, s.F, dtype=torch.complex64, device="cuda")
        with pytest.raises(et.EchoError) as err:
            et.synthesize_backward(ctx, s, P, gb)
        assert err.value.status == -5


@pytest.mark.parametrize("Q,Bk,F", [(64, 4, 4096), (40, 3, 4608), (256, 1, 2048), (17, 15, 1920), (51, 5, 960)])
def test_adjoint_with_many_materials(et, ctx, Q, Bk, F):
    """dL/dk with more than 16 materials (the factorised adjoint sums it per tile of 16
    materials): Q Bk up to 256, bands of whole 64-bin rows with edges on the 4-row groups
    (4096, 4608 bins) and off them (1920, 960), a last material tile partly filled, tiles of
    at most 32 rows (2048, 1920, 960 bins) and a grid of two tiles (4608).  Against the
    oracle gradient."""
    import torch
    base_scene, base_sim = W.tiny_scene(n_rays=2048)
    scene, sim, g = _tiny_materials(base_scene, base_sim, Q, Bk, F, 2048, 53 + Q)
    ref = O.trace(scene, sim, certify=False)
    hidden = dict(sim, refl_k=g.uniform(0.3, 0.99, (Q, Bk)).astype(np.float32))
    H_star = O.synth(ref, hidden)
    H = O.synth(ref, sim)
    gk_ref, gx_ref = O.grad(ref, sim, H - H_star)
    P = et.Paths.from_records(ref)
    gk, gx = et.synthesize_backward(ctx, et.Sim(sim), P, torch.as_tensor(H - H_star).to("cuda"))
    st = ctx.stats()
    gk = gk.cpu().numpy()
    ek, ex = rel_l2(gk, gk_ref), rel_l2(gx.cpu().numpy(), gx_ref)
    used = np.unique(ref["mat"][ref["kind"] == 0])
    print(f"adjoint, Q={Q}, Bk={Bk}, F={F} (kernel {st.adjoint_kernel}, {len(ref['rtot'])} records, "
          f"{len(used)} materials hit): dL/dk {ek:.3e}, dL/dx {ex:.3e}")
    assert st.adjoint_kernel == 1
    assert ek <= TOL and ex <= TOL
    assert len(used) > 16
    # per material: a material that no record reflects from has a zero gradient, the others
    # agree to TOL of the largest entry
    scale = np.abs(gk_ref).max()
    for qq in range(Q):
        if qq not in used:
            assert np.all(gk[qq] == 0), qq
        else:
            assert np.abs(gk[qq] - gk_ref[qq]).max() <= TOL * scale, qq


@pytest.mark.parametrize("F", [4096, 65536])
def test_synthesis_with_64_bands(et, ctx, F):
    """The largest band tables: 64 material bands and a 64-band receiver directivity.  At
    4096 bins every 64-bin row is its own band (more segments per tile than the factorised
    kernel holds, so the per-term kernel runs); at 65536 bins the bands span 1024 bins and the
    factorised kernel runs over 16 tiles.  Sampled bins against the oracle."""
    base_scene, base_sim = W.tiny_scene(n_rays=2048)
    scene, sim, g = _tiny_materials(base_scene, base_sim, 3, 64, F, 2048, 52)
    sim = dict(sim, directivity=W.directivity_table(g, len(sim["rx_pos"]), Bd=64, El=16, Az=32), f_hi=200e3)
    ref = O.trace(scene, sim, certify=False)
    bins = np.sort(W.rng(9).choice(F, 96, replace=False))
    H_ref = O.synth(ref, sim, bins=bins)
    H = et.synthesize(ctx, et.Sim(sim), et.Paths.from_records(ref)).cpu().numpy()
    st = ctx.stats()
    check_spectra(H[:, bins], H_ref, f"64 bands, F={F}: kernel {st.synth_kernel}")
    assert st.synth_kernel == (2 if F == 4096 else 1)


def test_per_receiver_visibility_at_64_receivers(et, ctx):
    """Per-receiver line of sight at its limit of 64 receivers (a ring of 64 around the
    emitter, the screen scene hiding part of the wall from some of them): every certified
    record's 64 receiver bits equal the oracle's; 65 receivers are refused."""
    from test_gpu_parity import _screen_scene
    import math
    scene = _screen_scene()
    g = W.rng(14)
    ang = np.linspace(0, 2 * math.pi, 64, endpoint=False)
    rx = np.stack([np.zeros(64), 0.35 * np.cos(ang), 0.35 * np.sin(ang)], 1)
    sim = W.make_sim(emitter_pos=[0, 0, 0], emitter_rot=np.eye(3), rx_pos=rx,
                     ray_dirs=W.cone_directions(g, 4096, math.radians(35)), max_bounces=3, f_lo=20e3, f_hi=100e3,
                     F=256, refl_k=np.full((2, 8), 0.9, np.float32), lobe_beta=np.full((2, 8), 0.3, np.float32),
                     diff_coef=np.full((2, 8), 0.1, np.float32), per_rx_visibility=True)
    ref = O.trace(scene, sim)
    dirs = sim["ray_dirs"][ref["certified"]]
    ref_c = O.trace(scene, sim, dirs=dirs)
    bits = ref_c["rxvis"]
    assert np.any(bits != bits[0]) and np.any(bits >> np.uint64(63))
    sc = et.Scene(ctx, scene)
    P = et.trace(ctx, sc, et.Sim(sim, ray_dirs=dirs))
    h = P.to_host()
    order_g = np.lexsort((h["bounce"], h["ray"]))
    order_o = np.lexsort((ref_c["bounce"], ref_c["ray"]))
    assert np.array_equal(h["ray"][order_g], ref_c["ray"][order_o])
    assert np.array_equal(h["rxvis"][order_g], ref_c["rxvis"][order_o])
    print(f"64 receivers: {len(bits)} records, {np.mean([bin(int(b)).count('1') for b in bits]):.1f} receivers "
          f"in sight per record")
    rx65 = np.concatenate([rx, [[0.0, 0.0, 0.5]]])
    s65 = et.Sim(dict(sim, rx_pos=rx65, rx_rot=np.repeat(np.eye(3)[None], 65, axis=0),
                      x_ref=rx65.mean(0)), ray_dirs=dirs)
    with pytest.raises(et.EchoError) as err:
        et.trace(ctx, sc, s65)
    assert err.value.status == -5
