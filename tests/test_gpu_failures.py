"""Failure handling through the C ABI: malformed meshes (indices out of range, negative or
too large materials, non-finite vertices) are refused with ET_E_INVALID, a refit to
non-finite vertices is refused and a later refit recovers, and a traversal stack held below
what the tree needs (the test hook et_set_stack_limit) drops subtrees, finishes every kernel
and reports the overflow count with ET_E_INTERNAL."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_gpu_parity import compare_traces

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(et):
    return et.Context(0)


def _tiny():
    return W.tiny_scene(n_rays=1024)


def _build_status(et, ctx, scene):
    try:
        et.Scene(ctx, scene)
    except et.EchoError as e:
        return e.status
    return 0


def test_mesh_index_errors(et, ctx):
    scene, _ = _tiny()
    T = len(scene["tris"])
    for what, mutate in [
        ("vertex index = V", lambda s: s["tris"].__setitem__((T // 2, 1), len(s["vertices"]))),
        ("negative vertex index", lambda s: s["tris"].__setitem__((3, 0), -1)),
        ("object index = n_objects", lambda s: s["tri_object"].__setitem__(T - 1, s["n_objects"])),
        ("negative object index", lambda s: s["tri_object"].__setitem__(0, -2)),
        ("negative material", lambda s: s["tri_material"].__setitem__(7, -1)),
    ]:
        bad = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
        mutate(bad)
        st = _build_status(et, ctx, bad)
        print(f"{what}: status {st}")
        assert st == -1, what
    # the context still works afterwards
    assert _build_status(et, ctx, scene) == 0


def test_material_beyond_tables_refused_at_trace(et, ctx):
    scene, sim = _tiny()
    bad = dict(scene, tri_material=scene["tri_material"].copy())
    bad["tri_material"][5] = 1          # the pose's tables have Q = 1 row
    sc = et.Scene(ctx, bad)
    with pytest.raises(et.EchoError) as e:
        et.trace(ctx, sc, et.Sim(sim))
    assert e.value.status == -1


@pytest.mark.parametrize("value", [np.nan, np.inf])
def test_non_finite_vertices(et, ctx, value):
    """Build refuses a non-finite coordinate of a used vertex; a refit to such vertices is
    refused and a refit back to finite ones restores a scene that traces like a fresh build."""
    scene, sim = _tiny()
    bad = dict(scene, vertices=scene["vertices"].copy())
    bad["vertices"][int(scene["tris"][10, 2]), 1] = value
    assert _build_status(et, ctx, bad) == -1
    sc = et.Scene(ctx, scene)
    with pytest.raises(et.EchoError) as e:
        sc.refit(bad["vertices"])
    assert e.value.status == -1
    sc.refit(scene["vertices"])
    s = et.Sim(sim)
    ref = O.trace(scene, sim)
    gpu = et.trace(ctx, sc, s).to_host()
    st = ctx.stats()
    assert st.stack_overflows == 0
    assert compare_traces(gpu, ref, ref["certified"]) == 0


def test_stack_overflow_is_reported(et, ctx):
    """A 3-entry traversal stack cannot hold the room's tree: kernels finish, et_get_stats
    reports the dropped pushes and ET_E_INTERNAL; the full stack traces normally again."""
    scene, sim = W.room_scene(n_rays=1 << 20)
    sc = et.Scene(ctx, scene, area_ref=sim["area_ref"])
    s = et.Sim(sim, flags=et.ET_SPECULAR, ray_dirs=sim["ray_dirs"][:65536])
    with pytest.raises(et.EchoError):
        ctx.set_stack_limit(65)
    try:
        ctx.set_stack_limit(3)
        et.trace(ctx, sc, s)
        with pytest.raises(et.EchoError) as e:
            ctx.stats()
        assert e.value.status == -6
        print(f"stack limit 3: {e.value.stats.stack_overflows} dropped pushes, {e.value.stats.segments} segments")
        assert e.value.stats.stack_overflows > 0
    finally:
        ctx.set_stack_limit(0)
    et.trace(ctx, sc, s)
    st = ctx.stats()
    assert st.stack_overflows == 0 and st.segments > 0


def test_stack_overflow_in_pipelined_batch(et, ctx):
    """A fused batch in four job waves (pipelined over two streams, two control blocks) with a
    3-entry traversal stack: the overflows of every wave reach et_get_stats (ET_E_INTERNAL), as
    many as when the same batch runs its waves in order (a captured graph); with the full stack
    again the replay is clean (the graph is keyed on the stack limit)."""
    import torch
    scene, sim = W.room_scene(n_rays=1 << 16, M=2, F=256, diff_K=0)
    sc = et.Scene(ctx, scene, area_ref=sim["area_ref"])
    sims = [et.Sim(dict(sim, emitter_pos=np.asarray(sim["emitter_pos"]) + np.array([0.1 * i, 0.0, 0.0])),
                   flags=et.ET_SPECULAR) for i in range(4)]
    t0 = ctx.tuning()
    ctx.set_tuning(t0.synth_wgs, t0.adjoint_wgs, t0.trace_blocks, 1 << 16)   # one job per wave
    side = torch.cuda.Stream()
    try:
        batch = et.Batch(ctx, [(sc, s) for s in sims])
        ctx.set_stack_limit(3)
        batch.run()
        with pytest.raises(et.EchoError) as e:
            ctx.stats()
        assert e.value.status == -6
        n_pipe = e.value.stats.stack_overflows
        with torch.cuda.stream(side):
            batch.run(graph=True)
            torch.cuda.synchronize()
        with pytest.raises(et.EchoError) as e2:
            ctx.stats()
        print(f"4 waves, stack limit 3: {n_pipe} dropped pushes pipelined, {e2.value.stats.stack_overflows} in order")
        assert n_pipe > 0 and e2.value.stats.stack_overflows == n_pipe
        ctx.set_stack_limit(0)
        with torch.cuda.stream(side):
            batch.run(graph=True)
            torch.cuda.synchronize()
        assert ctx.stats().stack_overflows == 0
        batch.run()
        assert ctx.stats().stack_overflows == 0
    finally:
        ctx.set_stack_limit(0)
        ctx.set_tuning(t0.synth_wgs, t0.adjoint_wgs, t0.trace_blocks, 0)
