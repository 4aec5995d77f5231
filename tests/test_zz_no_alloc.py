"""et_synthesize_noalloc (no workspace: the library's per-device scratch, every record walked)
against et_synthesize on the same records, through the C ABI: two calls in a row, the first on
the room scene's records (32 receivers x 4096 bins), the second with a smaller input (the tiny
scene: 2 receivers x 1024 bins, fewer records), then the per-term kernel; each within the
1e-4 relative L2 bar, over all receivers and per receiver."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import check_spectra

pytestmark = pytest.mark.gpu


def _records(et, ctx, scene, sim, n_rays):
    sc = et.Scene(ctx, scene, area_ref=sim.get("area_ref", 0.0))
    s = et.Sim(sim, ray_dirs=sim["ray_dirs"][:n_rays])
    return s, et.trace(ctx, sc, s)


def test_noalloc_synthesis_matches_workspace_call(et):
    import torch
    ctx = et.Context(0)
    room, rsim = W.room_scene(n_rays=1 << 20)
    tiny, tsim = W.tiny_scene()
    s1, P1 = _records(et, ctx, room, rsim, 1 << 16)
    s2, P2 = _records(et, ctx, tiny, tsim, 4096)
    s3 = et.Sim(tsim, flags=et.ET_SPECULAR | et.ET_SYNTH_DIRECT, ray_dirs=tsim["ray_dirs"][:4096])
    cases = [("room, 32 x 4096", s1, P1), ("tiny, 2 x 1024 (smaller input)", s2, P2), ("tiny, per-term kernel", s3, P2)]
    outs = [torch.empty(s.M, s.F, 2, dtype=torch.float32, device="cuda") for _, s, _ in cases]
    torch.cuda.synchronize()
    for (what, s, P), out in zip(cases, outs):
        ref = et.synthesize(ctx, s, P).cpu().numpy()
        kref = ctx.stats().synth_kernel
        H = et.synthesize_noalloc(ctx, s, P, out).cpu().numpy()
        st = ctx.stats()
        print(f"{what}: {P.n()} records, kernel {st.synth_kernel}")
        assert st.synth_kernel == kref
        assert np.all(np.isfinite(H)) and np.linalg.norm(ref) > 0
        check_spectra(H, ref, f"allocation-free synthesis vs workspace call ({what})")
    # the scratch keeps the last call's contents: a repeated call still starts from zero
    H = et.synthesize_noalloc(ctx, s1, P1, outs[0]).cpu().numpy()
    check_spectra(H, et.synthesize(ctx, s1, P1).cpu().numpy(), "room again after smaller calls")
