"""Python binding of the echotrace C ABI (include/echotrace.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels of
libechotrace.so.  PyTorch supplies device memory (caller-owned tensors) and the stream
(torch's current HIP stream); no computation of the method happens here.  Importing this
module without the built library, or calling it without a GPU, raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libechotrace.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "echotrace.h")

ET_SPECULAR, ET_DIFFRACTION, ET_SYNTH_DIRECT, ET_PASSIVE, ET_DIFF_PER_MESH = 1, 2, 4, 8, 16
ET_PATH_PRODUCT, ET_PER_RX_VISIBILITY = 32, 64
STATUS = {0: "ET_OK", -1: "ET_E_INVALID", -2: "ET_E_WORKSPACE", -3: "ET_E_CAPACITY", -4: "ET_E_DEVICE",
          -5: "ET_E_UNSUPPORTED", -6: "ET_E_INTERNAL"}


class EchoError(RuntimeError):
    def __init__(self, status: int, msg: str, stats=None):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.stats = stats     # the statistics of a failing et_get_stats (deferred device-side status)


# ------------------------------------------------------------------ ABI structs

class MeshDesc(C.Structure):
    _fields_ = [("V", C.c_int64), ("T", C.c_int64), ("vertices", C.c_void_p), ("tris", C.c_void_p),
                ("tri_material", C.c_void_p), ("tri_object", C.c_void_p), ("n_objects", C.c_int32),
                ("area_ref", C.c_double)]


class SimDesc(C.Structure):
    _fields_ = [("emitter_pos", C.c_double * 3), ("emitter_rot", C.c_double * 9), ("M", C.c_int32),
                ("rx_pos", C.c_void_p), ("rx_rot", C.c_void_p), ("x_ref", C.c_double * 3), ("N", C.c_int64),
                ("ray_dirs", C.c_void_p), ("max_bounces", C.c_int32), ("max_distance", C.c_double),
                ("t_eps", C.c_double), ("f_lo", C.c_double), ("f_hi", C.c_double), ("F", C.c_int32),
                ("c", C.c_double), ("atm_a0", C.c_double), ("atm_a1", C.c_double), ("spreading_p", C.c_double),
                ("phase_sign", C.c_int32), ("Q", C.c_int32), ("Bk", C.c_int32), ("refl_k", C.c_void_p),
                ("lobe_beta", C.c_void_p), ("diff_coef", C.c_void_p), ("Bd", C.c_int32), ("El", C.c_int32),
                ("Az", C.c_int32), ("directivity", C.c_void_p), ("diff_K", C.c_int64), ("diff_seed", C.c_uint64),
                ("diff_tau", C.c_double), ("diff_max_incidence", C.c_double), ("diff_cone_half_angle", C.c_double),
                ("flags", C.c_uint32), ("passive_coef", C.c_void_p), ("diff_max_meshes", C.c_int64)]


class PathsDesc(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("p", C.c_void_p), ("dout", C.c_void_p), ("rtot", C.c_void_p),
                ("tri", C.c_void_p), ("mat", C.c_void_p), ("ray", C.c_void_p), ("bounce", C.c_void_p),
                ("flags", C.c_void_p), ("count", C.c_void_p), ("prev", C.c_void_p), ("rx_vis", C.c_void_p)]


class SceneInfo(C.Structure):
    _fields_ = [("T", C.c_int64), ("V", C.c_int64), ("n_nodes", C.c_int64), ("depth", C.c_int32),
                ("sah_cost", C.c_double), ("build_ms", C.c_double), ("refit_ms", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("records", C.c_int64), ("specular", C.c_int64), ("diffraction", C.c_int64), ("segments", C.c_int64),
                ("shadow_rays", C.c_int64), ("diff_eligible", C.c_int64), ("stack_overflows", C.c_int64),
                ("dropped", C.c_int64), ("synth_kernel", C.c_int32), ("status", C.c_int32), ("ms_trace", C.c_double),
                ("ms_diffraction", C.c_double), ("ms_synth", C.c_double), ("ms_adjoint", C.c_double),
                ("ms_synth_kernel", C.c_double), ("ms_adjoint_kernel", C.c_double),
                ("adjoint_kernel", C.c_int32), ("reserved0", C.c_int32), ("passive", C.c_int64)]


class Counters(C.Structure):
    _fields_ = [("nodes_closest", C.c_int64), ("tris_closest", C.c_int64), ("nodes_any", C.c_int64),
                ("tris_any", C.c_int64), ("rays_closest", C.c_int64), ("rays_any", C.c_int64)]


class Job(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("sim", C.POINTER(SimDesc))]


class Tuning(C.Structure):
    _fields_ = [("synth_wgs", C.c_int32), ("adjoint_wgs", C.c_int32), ("trace_blocks", C.c_int32),
                ("wave_rays", C.c_int32), ("ms_trace", C.c_double), ("ms_synth", C.c_double),
                ("ms_adjoint", C.c_double)]


_lib = None


def declared_symbols() -> list[str]:
    """Entry points declared in include/echotrace.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(et_\w+)\s*\(", txt, re.M)))


def lib():
    """The loaded product library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2602_19652_amd.build` first")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "et_abi_version": ([], C.c_int),
            "et_status_string": ([C.c_int], C.c_char_p),
            "et_create": ([C.c_int, vp, C.POINTER(vp)], C.c_int),
            "et_destroy": ([vp], C.c_int),
            "et_set_stream": ([vp, vp], C.c_int),
            "et_last_error": ([vp], C.c_char_p),
            "et_scene_size": ([vp, C.POINTER(MeshDesc), C.POINTER(sz), C.POINTER(sz)], C.c_int),
            "et_scene_build": ([vp, C.POINTER(MeshDesc), vp, sz, vp, sz, C.POINTER(vp)], C.c_int),
            "et_scene_free": ([vp], C.c_int),
            "et_scene_get_info": ([vp, vp, C.POINTER(SceneInfo)], C.c_int),
            "et_scene_curvature": ([vp, vp, vp, vp], C.c_int),
            "et_scene_refit": ([vp, vp, vp, C.c_double], C.c_int),
            "et_eq_directions_workspace_size": ([i64, C.POINTER(sz)], C.c_int),
            "et_emitters_workspace_size": ([vp, vp, i32, vp, C.POINTER(sz)], C.c_int),
            "et_simulate_emitters": ([vp, vp, i32, vp, vp, sz, vp], C.c_int),
            "et_eq_directions": ([vp, i64, C.c_double, vp, sz, vp, i64, C.POINTER(i64)], C.c_int),
            "et_workspace_size": ([vp, vp, C.POINTER(SimDesc), C.POINTER(sz)], C.c_int),
            "et_trace": ([vp, vp, C.POINTER(SimDesc), vp, sz, C.POINTER(PathsDesc)], C.c_int),
            "et_synthesize": ([vp, C.POINTER(SimDesc), C.POINTER(PathsDesc), vp, sz, vp], C.c_int),
            "et_simulate": ([vp, vp, C.POINTER(SimDesc), C.POINTER(PathsDesc), vp, sz, vp], C.c_int),
            "et_synthesize_noalloc": ([vp, C.POINTER(SimDesc), C.POINTER(PathsDesc), vp], C.c_int),
            "et_synthesize_backward": ([vp, C.POINTER(SimDesc), C.POINTER(PathsDesc), vp, vp, sz, vp, vp], C.c_int),
            "et_batch_workspace_size": ([vp, i32, C.POINTER(Job), C.POINTER(sz)], C.c_int),
            "et_simulate_batch": ([vp, i32, C.POINTER(Job), vp, sz, vp, vp, vp, vp], C.c_int),
            "et_simulate_batch_graph": ([vp, i32, C.POINTER(Job), vp, sz, vp, vp, vp, vp], C.c_int),
            "et_graph_reset": ([vp], C.c_int),
            "et_get_stats": ([vp, C.POINTER(Stats)], C.c_int),
            "et_set_counting": ([vp, C.c_int], C.c_int),
            "et_get_counters": ([vp, C.POINTER(Counters)], C.c_int),
            "et_set_stack_limit": ([vp, i32], C.c_int),
            "et_get_tuning": ([vp, C.POINTER(Tuning)], C.c_int),
            "et_set_tuning": ([vp, C.POINTER(Tuning)], C.c_int),
            "et_autotune_batch": ([vp, i32, C.POINTER(Job), vp, sz, vp, vp, vp, vp, C.POINTER(Tuning)], C.c_int),
            "et_impulse_response_workspace_size": ([i32, i32, C.POINTER(sz)], C.c_int),
            "et_impulse_response": ([vp, i32, i32, C.c_double, C.c_double, i32, vp, i32, vp, sz, vp,
                                     C.POINTER(C.c_double)], C.c_int),
            "et_receiver_signal_workspace_size": ([i32, i32, i64, C.POINTER(sz)], C.c_int),
            "et_receiver_signal": ([vp, i32, i32, vp, i64, vp, C.c_double, vp, sz, vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev() -> torch.device:
    if not torch.cuda.is_available():
        raise RuntimeError("echotrace needs a HIP GPU (torch.cuda is not available)")
    return torch.device("cuda", torch.cuda.current_device())


def _to_dev(a, dtype):
    if isinstance(a, torch.Tensor):
        return a.to(device=_dev(), dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=_dev(), dtype=dtype).contiguous()


# ------------------------------------------------------------------ context

class Context:
    """An et_ctx bound to the current device; every call runs on torch's current stream."""

    def __init__(self, device: int | None = None):
        dev = _dev() if device is None else torch.device("cuda", device)
        self.device = dev.index
        h = C.c_void_p()
        self._check(lib().et_create(self.device, C.c_void_p(torch.cuda.current_stream(dev).cuda_stream), C.byref(h)),
                    "et_create")
        self.h = h

    def _check(self, rc: int, what: str):
        if rc != 0:
            msg = lib().et_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise EchoError(rc, f"{what}: {msg}")

    def call(self, name: str, *args):
        lib().et_set_stream(self.h, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        rc = getattr(lib(), name)(self.h, *args)
        self._check(rc, name)
        return rc

    def stats(self) -> Stats:
        st = Stats()
        rc = lib().et_get_stats(self.h, C.byref(st))
        if rc != 0:
            raise EchoError(rc, f"et_get_stats: {lib().et_last_error(self.h).decode()} (status {st.status})", st)
        return st

    def counters(self) -> Counters:
        c = Counters()
        self.call("et_get_counters", C.byref(c))
        return c

    def set_counting(self, on: bool):
        self.call("et_set_counting", 1 if on else 0)

    def set_stack_limit(self, entries: int):
        """Test hook: per-lane traversal stack entries for later traces (0 restores the full stack)."""
        self.call("et_set_stack_limit", int(entries))

    def tuning(self) -> Tuning:
        t = Tuning()
        self.call("et_get_tuning", C.byref(t))
        return t

    def set_tuning(self, synth_wgs: int, adjoint_wgs: int, trace_blocks: int, wave_rays: int = 0):
        t = Tuning(synth_wgs=synth_wgs, adjoint_wgs=adjoint_wgs, trace_blocks=trace_blocks, wave_rays=wave_rays)
        self.call("et_set_tuning", C.byref(t))

    def close(self):
        if getattr(self, "h", None):
            lib().et_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ scene

class Scene:
    """Device copy of a scene mesh plus its BVH/curvature blob (built by et_scene_build)."""

    def __init__(self, ctx: Context, scene: dict, area_ref: float = 0.0):
        self.ctx = ctx
        self.vertices = _to_dev(scene["vertices"], torch.float32)
        self.tris = _to_dev(scene["tris"], torch.int32)
        self.tri_material = _to_dev(scene["tri_material"], torch.int32)
        self.tri_object = _to_dev(scene["tri_object"], torch.int32)
        self.T, self.V = len(scene["tris"]), len(scene["vertices"])
        self.desc = MeshDesc(self.V, self.T, _ptr(self.vertices).value, _ptr(self.tris).value,
                             _ptr(self.tri_material).value, _ptr(self.tri_object).value, int(scene["n_objects"]),
                             float(area_ref))
        blob, scratch = C.c_size_t(), C.c_size_t()
        ctx.call("et_scene_size", C.byref(self.desc), C.byref(blob), C.byref(scratch))
        self.blob = torch.empty(blob.value, dtype=torch.uint8, device=_dev())
        tmp = torch.empty(scratch.value, dtype=torch.uint8, device=_dev())
        h = C.c_void_p()
        ctx.call("et_scene_build", C.byref(self.desc), _ptr(self.blob), blob.value, _ptr(tmp), scratch.value, C.byref(h))
        torch.cuda.synchronize()
        del tmp
        self.h = h

    def refit(self, vertices, area_ref: float = 0.0):
        """New vertex positions [V][3] for the same topology (et_scene_refit); keeps the
        device copy alive as the scene's vertex array."""
        v = _to_dev(vertices, torch.float32)
        if tuple(v.shape) != (self.V, 3):
            raise ValueError(f"vertices must have shape ({self.V}, 3), got {tuple(v.shape)}")
        self.ctx.call("et_scene_refit", self.h, _ptr(v), float(area_ref))
        self.vertices = v

    def info(self) -> SceneInfo:
        i = SceneInfo()
        self.ctx.call("et_scene_get_info", self.h, C.byref(i))
        return i

    def curvature(self):
        Cc = torch.empty(max(self.T, 1), dtype=torch.float64, device=_dev())
        G = torch.empty(max(self.V, 1), dtype=torch.float64, device=_dev())
        self.ctx.call("et_scene_curvature", self.h, _ptr(Cc), _ptr(G))
        return Cc[:self.T], G[:self.V]

    def close(self):
        if getattr(self, "h", None):
            lib().et_scene_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ per-pose descriptor

class Sim:
    """Device arrays + et_sim_desc for one pose, from a workload settings dict."""

    def __init__(self, sim: dict, flags: int | None = None, ray_dirs=None):
        self.src = sim
        rays = sim["ray_dirs"] if ray_dirs is None else ray_dirs
        self.ray_dirs = _to_dev(rays, torch.float32).reshape(-1, 3)
        self.rx_pos = _to_dev(sim["rx_pos"], torch.float64).reshape(-1, 3)
        self.rx_rot = _to_dev(sim["rx_rot"], torch.float64).reshape(-1, 9)
        self.refl_k = _to_dev(sim["refl_k"], torch.float32)
        self.lobe_beta = _to_dev(sim["lobe_beta"], torch.float32)
        self.diff_coef = _to_dev(sim["diff_coef"], torch.float32)
        D = sim.get("directivity")
        self.directivity = None if D is None else _to_dev(D, torch.float32)
        pc = sim.get("passive_coef")
        self.passive_coef = None if pc is None else _to_dev(pc, torch.float32)
        if flags is None:
            flags = (ET_SPECULAR | (ET_DIFFRACTION if sim.get("diff_K", 0) > 0 else 0)
                     | (ET_PASSIVE if pc is not None else 0)
                     | (ET_DIFF_PER_MESH if sim.get("diff_per_mesh", False) else 0)
                     | (ET_PATH_PRODUCT if sim.get("path_product", False) else 0)
                     | (ET_PER_RX_VISIBILITY if sim.get("per_rx_visibility", False) else 0))
        d = SimDesc()
        d.emitter_pos[:] = [float(x) for x in np.asarray(sim["emitter_pos"], float)]
        d.emitter_rot[:] = [float(x) for x in np.asarray(sim["emitter_rot"], float).ravel()]
        d.M = self.rx_pos.shape[0]
        d.x_ref[:] = [float(x) for x in np.asarray(sim["x_ref"], float)]
        d.N = self.ray_dirs.shape[0]
        d.max_bounces = int(sim["max_bounces"])
        d.max_distance = float(sim["max_distance"])
        d.t_eps = float(sim["t_eps"])
        d.f_lo, d.f_hi, d.F = float(sim["f_lo"]), float(sim["f_hi"]), int(sim["F"])
        d.c, d.atm_a0, d.atm_a1 = float(sim["c"]), float(sim["atm_a0"]), float(sim["atm_a1"])
        d.spreading_p, d.phase_sign = float(sim["spreading_p"]), int(sim["phase_sign"])
        d.Q, d.Bk = self.refl_k.shape
        if self.directivity is not None:
            _, d.Bd, d.El, d.Az = self.directivity.shape
        d.diff_K = int(sim.get("diff_K", 0))
        d.diff_seed = int(sim.get("diff_seed", 0))
        d.diff_tau = float(sim.get("diff_tau", 0.1))
        d.diff_max_incidence = float(np.radians(sim.get("diff_max_incidence_deg", 80.0)))
        d.diff_cone_half_angle = float(np.radians(sim.get("diff_cone_half_angle_deg", 90.0)))
        d.flags = int(flags)
        d.diff_max_meshes = int(sim.get("diff_max_meshes", 1))
        self.desc = d
        self.refresh()

    def refresh(self):
        """Re-point the descriptor at the (possibly replaced) device tensors."""
        d = self.desc
        d.rx_pos, d.rx_rot, d.ray_dirs = _ptr(self.rx_pos).value, _ptr(self.rx_rot).value, _ptr(self.ray_dirs).value
        d.refl_k, d.lobe_beta, d.diff_coef = _ptr(self.refl_k).value, _ptr(self.lobe_beta).value, _ptr(self.diff_coef).value
        d.directivity = None if self.directivity is None else _ptr(self.directivity).value
        d.passive_coef = None if self.passive_coef is None else _ptr(self.passive_coef).value

    @property
    def M(self):
        return self.desc.M

    @property
    def F(self):
        return self.desc.F

    def capacity(self) -> int:
        """Records a trace can produce at most (sizes Paths)."""
        d = self.desc
        n = 0
        if d.flags & ET_SPECULAR:
            n += d.N * d.max_bounces
        if d.flags & ET_DIFFRACTION:
            n += d.diff_K * (d.diff_max_meshes if d.flags & ET_DIFF_PER_MESH else 1)
        if d.flags & ET_PASSIVE:
            n += d.M
        return max(n, 1)


# ------------------------------------------------------------------ path records

class Paths:
    """Caller-owned device record buffers (et_paths)."""

    def __init__(self, capacity: int):
        dev = _dev()
        cap = max(int(capacity), 1)
        self.capacity = cap
        self.p = torch.zeros(cap, 3, dtype=torch.float64, device=dev)
        self.dout = torch.zeros(cap, 3, dtype=torch.float32, device=dev)
        self.rtot = torch.zeros(cap, dtype=torch.float64, device=dev)
        self.tri = torch.zeros(cap, dtype=torch.int32, device=dev)
        self.mat = torch.zeros(cap, dtype=torch.int32, device=dev)
        self.ray = torch.zeros(cap, dtype=torch.int32, device=dev)
        self.bounce = torch.zeros(cap, dtype=torch.uint8, device=dev)
        self.flags = torch.zeros(cap, dtype=torch.uint8, device=dev)
        self.count = torch.zeros(8, dtype=torch.int64, device=dev)
        self.prev = torch.full((cap,), -1, dtype=torch.int64, device=dev)
        self.rx_vis = torch.zeros(cap, dtype=torch.int64, device=dev)   # uint64 bits
        self.desc = PathsDesc(cap, *[_ptr(t).value for t in (self.p, self.dout, self.rtot, self.tri, self.mat, self.ray,
                                                             self.bounce, self.flags, self.count, self.prev,
                                                             self.rx_vis)])

    @classmethod
    def from_records(cls, rec: dict) -> "Paths":
        """Uploads host records (e.g. produced by another implementation) for synthesis."""
        n = len(rec["rtot"])
        P = cls(n)
        if n:
            P.p[:n] = torch.as_tensor(np.asarray(rec["p"], np.float64))
            P.dout[:n] = torch.as_tensor(np.asarray(rec["dout"], np.float32))
            P.rtot[:n] = torch.as_tensor(np.asarray(rec["rtot"], np.float64))
            P.mat[:n] = torch.as_tensor(np.asarray(rec["mat"], np.int32))
            if "tri" in rec:
                P.tri[:n] = torch.as_tensor(np.asarray(rec["tri"], np.int32))
            vis = np.asarray(rec.get("vis", np.ones(n)), np.uint8) & 1
            kind = np.asarray(rec.get("kind", np.zeros(n)), np.uint8) & 3
            P.flags[:n] = torch.as_tensor(vis | (kind << 1))
            if "rxvis" in rec:
                P.rx_vis[:n] = torch.as_tensor(np.asarray(rec["rxvis"], np.uint64).view(np.int64))
        P.count[0] = n
        P.count[1] = n
        return P

    def n(self) -> int:
        return int(min(self.count[0].item(), self.capacity))

    def to_host(self) -> dict:
        n = self.n()
        fl = self.flags[:n].cpu().numpy()
        return {"p": self.p[:n].cpu().numpy(), "dout": self.dout[:n].cpu().numpy().astype(np.float64),
                "rtot": self.rtot[:n].cpu().numpy(), "tri": self.tri[:n].cpu().numpy(), "mat": self.mat[:n].cpu().numpy(),
                "ray": self.ray[:n].cpu().numpy(), "bounce": self.bounce[:n].cpu().numpy().astype(np.int32),
                "vis": (fl & 1).astype(np.uint8), "kind": ((fl >> 1) & 3).astype(np.uint8),
                "prev": self.prev[:n].cpu().numpy(), "rxvis": self.rx_vis[:n].cpu().numpy().view(np.uint64),
                "count": self.count[:4].cpu().numpy()}


# ------------------------------------------------------------------ calls

class Workspace:
    def __init__(self):
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=_dev())
        return self.buf


def workspace_size(ctx: Context, scene: Scene | None, sim: Sim) -> int:
    n = C.c_size_t()
    ctx.call("et_workspace_size", None if scene is None else scene.h, C.byref(sim.desc), C.byref(n))
    return n.value


def trace(ctx: Context, scene: Scene, sim: Sim, paths: Paths | None = None, ws: Workspace | None = None) -> Paths:
    paths = paths or Paths(sim.capacity())
    ws = ws or Workspace()
    buf = ws.get(workspace_size(ctx, scene, sim))
    ctx.call("et_trace", scene.h, C.byref(sim.desc), _ptr(buf), buf.numel(), C.byref(paths.desc))
    return paths


def synthesize(ctx: Context, sim: Sim, paths: Paths, ws: Workspace | None = None, out: torch.Tensor | None = None):
    """Spectra as complex64 [M, F] (a view of a float32 [M, F, 2] tensor)."""
    ws = ws or Workspace()
    buf = ws.get(workspace_size(ctx, None, sim))
    out = out if out is not None else torch.empty(sim.M, sim.F, 2, dtype=torch.float32, device=_dev())
    ctx.call("et_synthesize", C.byref(sim.desc), C.byref(paths.desc), _ptr(buf), buf.numel(), _ptr(out))
    return torch.view_as_complex(out)


def synthesize_noalloc(ctx: Context, sim: Sim, paths: Paths, out: torch.Tensor):
    """et_synthesize_noalloc: spectra into the caller's float32 [M, F, 2] tensor `out` without a
    workspace (the library's per-device scratch); returns the complex64 [M, F] view."""
    ctx.call("et_synthesize_noalloc", C.byref(sim.desc), C.byref(paths.desc), _ptr(out))
    return torch.view_as_complex(out)


def simulate(ctx: Context, scene: Scene, sim: Sim, paths: Paths | None = None, ws: Workspace | None = None,
             out: torch.Tensor | None = None):
    """Algorithm 1 + diffraction + synthesis: spectra complex64 [M, F]."""
    paths = paths or Paths(sim.capacity())
    ws = ws or Workspace()
    buf = ws.get(workspace_size(ctx, scene, sim))
    out = out if out is not None else torch.empty(sim.M, sim.F, 2, dtype=torch.float32, device=_dev())
    ctx.call("et_simulate", scene.h, C.byref(sim.desc), C.byref(paths.desc), _ptr(buf), buf.numel(), _ptr(out))
    return torch.view_as_complex(out)


def synthesize_backward(ctx: Context, sim: Sim, paths: Paths, grad_spectra: torch.Tensor, ws: Workspace | None = None):
    """Adjoint over fixed records: grad_spectra is dL/dconj(H) (complex [M, F]);
    returns (dL/d refl_k [Q, Bk] float64, dL/d rx_pos [M, 3] float64)."""
    ws = ws or Workspace()
    buf = ws.get(workspace_size(ctx, None, sim))
    g = torch.view_as_real(grad_spectra.to(torch.complex64).contiguous()).contiguous()
    gk = torch.empty(sim.desc.Q, sim.desc.Bk, dtype=torch.float64, device=_dev())
    gx = torch.empty(sim.M, 3, dtype=torch.float64, device=_dev())
    ctx.call("et_synthesize_backward", C.byref(sim.desc), C.byref(paths.desc), _ptr(g), _ptr(buf), buf.numel(),
             _ptr(gk), _ptr(gx))
    return gk, gx


def impulse_response(ctx: Context, sim: Sim, spectra: torch.Tensor, n_t: int, ws: Workspace | None = None):
    """Impulse responses h [M, n_t] (float32) of spectra (complex [M, F] on the sim's grid) and
    their sample spacing dt: h_m(n dt) = 2 df Re sum_k H_m[k] exp(-j sigma 2 pi f_k n dt)."""
    ws = ws or Workspace()
    d = sim.desc
    H = torch.view_as_real(spectra.to(torch.complex64).contiguous()).contiguous() if spectra.is_complex() \
        else spectra.contiguous()
    n = C.c_size_t()
    rc = lib().et_impulse_response_workspace_size(d.M, n_t, C.byref(n))
    if rc != 0:
        raise EchoError(rc, "et_impulse_response_workspace_size")
    buf = ws.get(n.value)
    h = torch.empty(d.M, n_t, dtype=torch.float32, device=_dev())
    dt = C.c_double()
    ctx.call("et_impulse_response", d.M, d.F, d.f_lo, d.f_hi, d.phase_sign, _ptr(H), n_t, _ptr(buf), buf.numel(),
             _ptr(h), C.byref(dt))
    return h, dt.value


def receiver_signal(ctx: Context, h: torch.Tensor, s_e: torch.Tensor, dt: float, ws: Workspace | None = None):
    """Received signals s [M, n_t + L - 1] (float32): s_m[n] = dt sum_k h_m[k] s_e[n - k]."""
    ws = ws or Workspace()
    h = h.to(torch.float32).contiguous()
    s_e = s_e.to(device=h.device, dtype=torch.float32).contiguous()
    M, n_t = h.shape
    L = s_e.numel()
    n = C.c_size_t()
    rc = lib().et_receiver_signal_workspace_size(M, n_t, L, C.byref(n))
    if rc != 0:
        raise EchoError(rc, "et_receiver_signal_workspace_size")
    buf = ws.get(n.value)
    out = torch.empty(M, n_t + L - 1, dtype=torch.float32, device=_dev())
    ctx.call("et_receiver_signal", M, n_t, _ptr(h), L, _ptr(s_e), float(dt), _ptr(buf), buf.numel(), _ptr(out))
    return out


def simulate_emitters(ctx: Context, scene: Scene, sims: list, ws: Workspace | None = None,
                      out: torch.Tensor | None = None):
    """Spectra complex64 [M, F] of several simultaneous emitters (et_simulate_emitters): the
    sum over the emitters of each one's spectra.  The Sim objects must share their receiver
    tensor (rx_pos), M, F and the frequency grid."""
    ws = ws or Workspace()
    arr = (SimDesc * len(sims))(*[s.desc for s in sims])
    n = C.c_size_t()
    ctx.call("et_emitters_workspace_size", scene.h, len(sims), C.cast(arr, C.c_void_p), C.byref(n))
    buf = ws.get(n.value)
    M, F = sims[0].M, sims[0].F
    out = out if out is not None else torch.empty(M, F, 2, dtype=torch.float32, device=_dev())
    ctx.call("et_simulate_emitters", scene.h, len(sims), C.cast(arr, C.c_void_p), _ptr(buf), buf.numel(), _ptr(out))
    return torch.view_as_complex(out)


def eq_directions(ctx: Context, N: int, cone_half_angle: float = math.pi, ws: Workspace | None = None) -> torch.Tensor:
    """Ray directions [count, 3] (float32, emitter frame, boresight +x): the centres of the
    regions of the equal-area partition EQ(2, N) of the sphere within the cone."""
    ws = ws or Workspace()
    n = C.c_size_t()
    rc = lib().et_eq_directions_workspace_size(int(N), C.byref(n))
    if rc != 0:
        raise EchoError(rc, "et_eq_directions_workspace_size")
    buf = ws.get(n.value)
    count = C.c_int64()
    ctx.call("et_eq_directions", int(N), float(cone_half_angle), _ptr(buf), buf.numel(), None, 0, C.byref(count))
    out = torch.empty(max(count.value, 1), 3, dtype=torch.float32, device=_dev())
    ctx.call("et_eq_directions", int(N), float(cone_half_angle), _ptr(buf), buf.numel(), _ptr(out), count.value,
             C.byref(count))
    return out[:count.value]


class SpectraFn(torch.autograd.Function):
    """H = synth(refl_k, rx_pos) over fixed path records, differentiable in both inputs.

    forward(refl_k [Q, Bk] float32, rx_pos [M, 3] float64, ctx, sim, paths) -> complex64 [M, F].
    The backward pass calls the hand-written adjoint kernel (et_synthesize_backward)."""

    @staticmethod
    def forward(fctx, refl_k, rx_pos, ctx: Context, sim: Sim, paths: Paths):
        sim.refl_k = refl_k.detach().to(torch.float32).contiguous()
        sim.rx_pos = rx_pos.detach().to(torch.float64).contiguous()
        sim.refresh()
        fctx.save_for_backward(refl_k, rx_pos)
        fctx.et = (ctx, sim, paths)
        return synthesize(ctx, sim, paths).clone()

    @staticmethod
    def backward(fctx, grad_out):
        ctx, sim, paths = fctx.et
        refl_k, rx_pos = fctx.saved_tensors
        sim.refl_k = refl_k.detach().to(torch.float32).contiguous()
        sim.rx_pos = rx_pos.detach().to(torch.float64).contiguous()
        sim.refresh()
        # torch passes 2 dL/dconj(H) for a real loss; the adjoint takes dL/dconj(H)
        gk, gx = synthesize_backward(ctx, sim, paths, grad_out * 0.5)
        return gk.to(refl_k.dtype), gx.to(rx_pos.dtype), None, None, None


# ------------------------------------------------------------------ batches

class Batch:
    """Jobs (scene, pose) sharing M, F, Q, Bk; one et_simulate_batch call runs them all."""

    def __init__(self, ctx: Context, jobs: list[tuple[Scene, Sim]]):
        self.ctx = ctx
        self.jobs = jobs
        self.arr = (Job * len(jobs))(*[Job(s.h, C.pointer(m.desc)) for s, m in jobs])
        n = C.c_size_t()
        ctx.call("et_batch_workspace_size", len(jobs), self.arr, C.byref(n))
        self.ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=_dev())
        M, F = jobs[0][1].M, jobs[0][1].F
        self.spectra = torch.empty(len(jobs), M, F, 2, dtype=torch.float32, device=_dev())
        Q, Bk = jobs[0][1].desc.Q, jobs[0][1].desc.Bk
        self.grad_k = torch.zeros(len(jobs), Q, Bk, dtype=torch.float64, device=_dev())
        self.grad_rx = torch.zeros(len(jobs), M, 3, dtype=torch.float64, device=_dev())

    def run(self, grad_spectra: torch.Tensor | None = None, graph: bool = False):
        g = None if grad_spectra is None else torch.view_as_real(grad_spectra.to(torch.complex64).contiguous())
        name = "et_simulate_batch_graph" if graph else "et_simulate_batch"
        self.ctx.call(name, len(self.jobs), self.arr, _ptr(self.ws), self.ws.numel(), _ptr(self.spectra), _ptr(g),
                      _ptr(self.grad_k) if g is not None else None, _ptr(self.grad_rx) if g is not None else None)
        return torch.view_as_complex(self.spectra)

    def autotune(self, grad_spectra: torch.Tensor | None = None) -> Tuning:
        """Times the batch over the library's candidate launch shapes and keeps the fastest
        (per knob) in the context; returns the choice and its phase times."""
        g = None if grad_spectra is None else torch.view_as_real(grad_spectra.to(torch.complex64).contiguous())
        t = Tuning()
        self.ctx.call("et_autotune_batch", len(self.jobs), self.arr, _ptr(self.ws), self.ws.numel(),
                      _ptr(self.spectra), _ptr(g), _ptr(self.grad_k) if g is not None else None,
                      _ptr(self.grad_rx) if g is not None else None, C.byref(t))
        return t
