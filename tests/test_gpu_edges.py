"""Edge cases of the path against the FP64 oracle: an empty scene, no rays, scenes of one and
two triangles (the smallest trees), ragged and single-bin frequency grids, a large grid over
several tiles, and rays that bounce up to the 255-record limit in a closed room."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import compare_traces, rel_l2

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
    assert rel_l2(H, H_ref) <= TOL


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
    e = rel_l2(H, H_ref)
    print(f"F={F}: kernel {ctx.stats().synth_kernel}, rel L2 {e:.3e}")
    assert e <= TOL


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
    e = rel_l2(H[:, bins], H_ref)
    print(f"F=16384: rel L2 on sampled bins {e:.3e}")
    assert e <= TOL


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
