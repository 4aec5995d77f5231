"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only builds input arrays: triangle meshes (welded per object), poses,
ray-direction sets, material band tables and receiver directivity tables.  It holds
none of the method's arithmetic (no tracing, no spectra, no curvature).

Every scene is a dict of numpy arrays plus scalar simulation settings:

  vertices      float32 [V, 3]   world-space positions (metres)
  tris          int32   [T, 3]   vertex indices, welded within an object
  tri_material  int32   [T]      acoustic profile index (per-object granularity)
  tri_object    int32   [T]      object index (0 .. n_objects-1)

and a simulation dict (``make_sim``) with emitter/receiver poses (float64, the phase
needs them), ray directions in the emitter frame (float32), the frequency grid,
material band tables and optional directivity.

The workloads stand in for the paper's scenes (a bat with one emitter and two
receivers, an office lobby with a 32-microphone planar array, a dense forest, a
closed-loop trajectory); their recipes follow the configuration list of the
benchmark (tiny wall+sphere, room, foliage, batched, differentiation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_SOUND = 343.0          # speed of sound used by the paper's synthesis equations (m/s)
A1_DB_PER_M_HZ = 3.5e-5  # synthetic linear air-absorption slope: 0.7/3.5/7 dB/m at 20/100/200 kHz


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------- meshes

class MeshBuilder:
    """Accumulates welded objects into one scene mesh."""

    def __init__(self):
        self.verts: list[np.ndarray] = []
        self.tris: list[np.ndarray] = []
        self.mats: list[np.ndarray] = []
        self.objs: list[np.ndarray] = []
        self.nv = 0
        self.nobj = 0

    def add(self, verts: np.ndarray, tris: np.ndarray, material: int) -> int:
        verts = np.asarray(verts, dtype=np.float64)
        tris = np.asarray(tris, dtype=np.int64)
        self.verts.append(verts)
        self.tris.append(tris + self.nv)
        self.mats.append(np.full(len(tris), material, dtype=np.int32))
        self.objs.append(np.full(len(tris), self.nobj, dtype=np.int32))
        self.nv += len(verts)
        self.nobj += 1
        return self.nobj - 1

    def build(self) -> dict:
        return {
            "vertices": np.ascontiguousarray(np.concatenate(self.verts).astype(np.float32)),
            "tris": np.ascontiguousarray(np.concatenate(self.tris).astype(np.int32)),
            "tri_material": np.ascontiguousarray(np.concatenate(self.mats)),
            "tri_object": np.ascontiguousarray(np.concatenate(self.objs)),
            "n_objects": self.nobj,
        }


def quad_grid_box(lo, hi, n: int):
    """Closed axis-aligned box surface, each face an n x n grid of quads (2 tris each).

    Vertices on shared edges are welded (one lattice point, one index)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    index = {}
    verts = []

    def vid(i, j, k):
        key = (i, j, k)
        if key not in index:
            index[key] = len(verts)
            verts.append(lo + (hi - lo) * np.array([i, j, k], float) / n)
        return index[key]

    tris = []
    # each face: fixed axis a at value 0 or n; (u, v) the other two axes, oriented outward
    for a in range(3):
        u, v = [x for x in range(3) if x != a]
        for side in (0, n):
            for i in range(n):
                for j in range(n):
                    def lat(ii, jj):
                        c = [0, 0, 0]
                        c[a] = side
                        c[u] = ii
                        c[v] = jj
                        return vid(*c)
                    q00, q10, q11, q01 = lat(i, j), lat(i + 1, j), lat(i + 1, j + 1), lat(i, j + 1)
                    if (side == n) == ((a == 1)):
                        tris.append((q00, q11, q10)); tris.append((q00, q01, q11))
                    else:
                        tris.append((q00, q10, q11)); tris.append((q00, q11, q01))
    return np.array(verts), np.array(tris, dtype=np.int64)


def cylinder(radius: float, height: float, segments: int, rings: int):
    """Closed z-aligned cylinder at the origin (base z=0): side split into `rings` stacks,
    fan caps with a centre vertex.  Rim vertices are shared by side and caps."""
    verts = []
    for r in range(rings + 1):
        z = height * r / rings
        for s in range(segments):
            ang = 2 * math.pi * s / segments
            verts.append((radius * math.cos(ang), radius * math.sin(ang), z))
    cb = len(verts); verts.append((0.0, 0.0, 0.0))
    ct = len(verts); verts.append((0.0, 0.0, height))
    tris = []
    for r in range(rings):
        for s in range(segments):
            a = r * segments + s
            b = r * segments + (s + 1) % segments
            c = (r + 1) * segments + (s + 1) % segments
            d = (r + 1) * segments + s
            tris.append((a, b, c)); tris.append((a, c, d))
    top = rings * segments
    for s in range(segments):
        tris.append((cb, (s + 1) % segments, s))
        tris.append((ct, top + s, top + (s + 1) % segments))
    return np.array(verts), np.array(tris, dtype=np.int64)


def icosphere(subdiv: int, radius: float = 1.0):
    """Icosahedron subdivided `subdiv` times by edge midpoints, projected to the sphere.
    subdiv=3 gives 642 vertices and 1280 triangles."""
    t = (1 + 5 ** 0.5) / 2
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, float) / np.linalg.norm(p) for p in v]
    for _ in range(subdiv):
        cache = {}
        nf = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    return np.array(verts) * radius, np.array(f, dtype=np.int64)


def disc_fan(centre, normal, radius: float, n_rim: int = 16):
    """A flat leaf disc: centre vertex + n_rim rim vertices, n_rim triangles."""
    normal = np.asarray(normal, float)
    normal = normal / np.linalg.norm(normal)
    helper = np.array([1.0, 0, 0]) if abs(normal[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = np.cross(normal, helper); e1 /= np.linalg.norm(e1)
    e2 = np.cross(normal, e1)
    ang = 2 * np.pi * np.arange(n_rim) / n_rim
    rim = centre + radius * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2)
    verts = np.vstack([centre[None, :], rim])
    tris = np.array([(0, 1 + s, 1 + (s + 1) % n_rim) for s in range(n_rim)], dtype=np.int64)
    return verts, tris


def rot_z(angle: float) -> np.ndarray:
    c, s = math.cos(angle), math.sin(angle)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


def frame_from_forward(fwd) -> np.ndarray:
    """Rotation whose first column is the horizontal forward direction (boresight = local +x),
    third column = world +z (upright sensor)."""
    f = np.array([fwd[0], fwd[1], 0.0], float)
    f /= np.linalg.norm(f)
    z = np.array([0, 0, 1.0])
    y = np.cross(z, f)
    return np.stack([f, y, z], axis=1)


# --------------------------------------------------------------------------- rays

def cone_directions(g: np.random.Generator, n: int, half_angle_rad: float) -> np.ndarray:
    """Directions uniform over the solid angle of a cone about local +x: cos(theta) ~ U[cos a, 1]."""
    ct = g.uniform(math.cos(half_angle_rad), 1.0, n)
    ph = g.uniform(0.0, 2 * math.pi, n)
    st = np.sqrt(np.maximum(0.0, 1 - ct * ct))
    d = np.stack([ct, st * np.cos(ph), st * np.sin(ph)], axis=1)
    return np.ascontiguousarray(d.astype(np.float32))


def disc_mics(g: np.random.Generator, m: int, diameter: float, centre, rot) -> np.ndarray:
    """m receivers uniform over a disc in the sensor's local y-z plane."""
    rad = 0.5 * diameter * np.sqrt(g.uniform(0, 1, m))
    ang = g.uniform(0, 2 * math.pi, m)
    local = np.stack([np.zeros(m), rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    return np.ascontiguousarray(np.asarray(centre, float)[None, :] + local @ np.asarray(rot).T)


def band_tables(g: np.random.Generator, q: int, b: int):
    k = g.uniform(0.3, 0.99, (q, b)).astype(np.float32)
    beta = g.uniform(0.05, 0.3, (q, b)).astype(np.float32)
    d = g.uniform(0.05, 0.3, (q, b)).astype(np.float32)
    return np.ascontiguousarray(k), np.ascontiguousarray(beta), np.ascontiguousarray(d)


# --------------------------------------------------------------------------- sim settings

def make_sim(*, emitter_pos, emitter_rot, rx_pos, ray_dirs, max_bounces, f_lo, f_hi, F,
             refl_k, lobe_beta, diff_coef, rx_rot=None, directivity=None, max_distance=math.inf,
             c=C_SOUND, atm_a0=0.0, atm_a1=A1_DB_PER_M_HZ, spreading_p=2.0, phase_sign=1,
             diff_K=0, diff_seed=0, diff_tau=0.1, diff_max_incidence_deg=80.0,
             diff_cone_half_angle_deg=90.0, x_ref=None, t_eps=1e-5, passive_coef=None, diff_per_mesh=False,
             diff_max_meshes=1, path_product=False, per_rx_visibility=False) -> dict:
    rx_pos = np.ascontiguousarray(np.asarray(rx_pos, dtype=np.float64).reshape(-1, 3))
    M = len(rx_pos)
    if rx_rot is None:
        rx_rot = np.repeat(np.eye(3)[None], M, axis=0)
    rx_rot = np.ascontiguousarray(np.asarray(rx_rot, dtype=np.float64).reshape(M, 3, 3))
    if x_ref is None:
        x_ref = rx_pos.mean(axis=0)
    return {
        "emitter_pos": np.asarray(emitter_pos, dtype=np.float64).reshape(3).copy(),
        "emitter_rot": np.ascontiguousarray(np.asarray(emitter_rot, dtype=np.float64).reshape(3, 3)),
        "rx_pos": rx_pos, "rx_rot": rx_rot,
        "ray_dirs": np.ascontiguousarray(np.asarray(ray_dirs, dtype=np.float32).reshape(-1, 3)),
        "max_bounces": int(max_bounces), "max_distance": float(max_distance),
        "x_ref": np.asarray(x_ref, dtype=np.float64).reshape(3).copy(), "t_eps": float(t_eps),
        "f_lo": float(f_lo), "f_hi": float(f_hi), "F": int(F),
        "c": float(c), "atm_a0": float(atm_a0), "atm_a1": float(atm_a1),
        "spreading_p": float(spreading_p), "phase_sign": int(phase_sign),
        "refl_k": np.ascontiguousarray(np.asarray(refl_k, np.float32)),
        "lobe_beta": np.ascontiguousarray(np.asarray(lobe_beta, np.float32)),
        "diff_coef": np.ascontiguousarray(np.asarray(diff_coef, np.float32)),
        "directivity": None if directivity is None else np.ascontiguousarray(np.asarray(directivity, np.float32)),
        "diff_K": int(diff_K), "diff_seed": int(diff_seed), "diff_tau": float(diff_tau),
        "diff_max_incidence_deg": float(diff_max_incidence_deg),
        "diff_cone_half_angle_deg": float(diff_cone_half_angle_deg),
        "diff_per_mesh": bool(diff_per_mesh), "diff_max_meshes": int(diff_max_meshes),
        "path_product": bool(path_product), "per_rx_visibility": bool(per_rx_visibility),
        "passive_coef": None if passive_coef is None else np.ascontiguousarray(np.asarray(passive_coef, np.float32)),
    }


def median_triangle_area(scene: dict) -> float:
    """Reference area for the curvature metric's area weighting (an input, chosen by the caller)."""
    v = scene["vertices"].astype(np.float64)
    t = scene["tris"]
    a = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1)
    return float(np.median(a))


# --------------------------------------------------------------------------- configurations

def tiny_scene(seed: int = 1001, n_rays: int = 16384, F: int = 1024, bounces: int = 3):
    """Plain method, tiny: a 4x4 m wall (2 tris) at x=4 and an icosphere (r=0.5, 1280 tris)
    3 m away; one emitter, 2 receivers 5 cm apart; rays seeded uniform in a 60 degree cone
    (half-angle 30 degrees); one flat material R=0.9; 20-100 kHz."""
    g = rng(seed)
    mb = MeshBuilder()
    mb.add(np.array([[4, -2, -2], [4, 2, -2], [4, 2, 2], [4, -2, 2]], float), np.array([[0, 1, 2], [0, 2, 3]]), 0)
    sv, st = icosphere(3, 0.5)
    ang = math.radians(15)
    mb.add(sv + 3 * np.array([math.cos(ang), math.sin(ang), 0.0]), st, 0)
    scene = mb.build()
    k = np.full((1, 8), 0.9, np.float32)
    beta = np.full((1, 8), 0.1, np.float32)
    dcoef = np.full((1, 8), 0.1, np.float32)
    sim = make_sim(emitter_pos=[0, 0, 0], emitter_rot=np.eye(3), rx_pos=[[0, 0.025, 0], [0, -0.025, 0]],
                   ray_dirs=cone_directions(g, n_rays, math.radians(30)), max_bounces=bounces,
                   f_lo=20e3, f_hi=100e3, F=F, refl_k=k, lobe_beta=beta, diff_coef=dcoef)
    return scene, sim


def room_geometry(g: np.random.Generator, n_boxes=100, n_cyl=100, sensor=(1.0, 4.0, 1.2), box_subdiv=9,
                  cyl_segments=120, cyl_rings=3, room=(10.0, 8.0, 3.0), keepout=0.75, n_mat=16):
    """10x8x3 m box room (12 tris) + seeded boxes and cylinders; material 0 for the room,
    1 + (i mod 15) for object i."""
    mb = MeshBuilder()
    rv, rt = quad_grid_box([0, 0, 0], list(room), 1)
    mb.add(rv, rt, 0)
    sensor = np.asarray(sensor, float)
    placed = 0
    i = 0
    while placed < n_boxes + n_cyl:
        is_box = placed < n_boxes
        cx, cy = g.uniform(0.5, room[0] - 0.5), g.uniform(0.5, room[1] - 0.5)
        if is_box:
            sx, sy, sz = g.uniform(0.2, 1.5, 3)
            yaw = g.uniform(0, 2 * math.pi)
            v, t = quad_grid_box([-sx / 2, -sy / 2, 0], [sx / 2, sy / 2, sz], box_subdiv)
            v = v @ rot_z(yaw).T
            reach = 0.5 * math.hypot(sx, sy)
        else:
            r = g.uniform(0.1, 0.5)
            h = g.uniform(0.3, 2.5)
            v, t = cylinder(r, h, cyl_segments, cyl_rings)
            reach = r
        v = v + np.array([cx, cy, 0.001])
        if math.hypot(cx - sensor[0], cy - sensor[1]) < keepout + reach:
            continue
        mb.add(v, t, 1 + (i % (n_mat - 1)))
        placed += 1
        i += 1
    return mb.build()


def animate_objects(scene: dict, g: np.random.Generator, shift=0.1, yaw=0.15, bulge=0.01, bulge_every=4):
    """One animation frame of a scene: every object except object 0 (the room shell) turns
    about the vertical through its centroid by U[-yaw, yaw] rad and moves by U[-shift, shift]
    m in x and y; every `bulge_every`-th of them also deforms non-rigidly (its vertices move
    radially by bulge * sin(2 pi z / 0.5 m)).  Returns new vertices [V][3] (same topology)."""
    V = np.asarray(scene["vertices"], np.float64).copy()
    tris = np.asarray(scene["tris"])
    vobj = np.full(len(V), -1, np.int64)
    for c in range(3):
        vobj[tris[:, c]] = scene["tri_object"]
    for o in range(1, int(scene["n_objects"])):
        idx = np.nonzero(vobj == o)[0]
        if len(idx) == 0:
            continue
        cen = V[idx].mean(axis=0)
        p = V[idx] - np.array([cen[0], cen[1], 0.0])
        if bulge and o % bulge_every == 0:
            r = np.hypot(p[:, 0], p[:, 1])
            scale = 1.0 + bulge * np.sin(2 * math.pi * p[:, 2] / 0.5) / np.maximum(r, 1e-6)
            p[:, 0] *= scale
            p[:, 1] *= scale
        p = p @ rot_z(g.uniform(-yaw, yaw)).T
        V[idx] = p + np.array([cen[0] + g.uniform(-shift, shift), cen[1] + g.uniform(-shift, shift), 0.0])
    return np.ascontiguousarray(V.astype(np.float32))


def room_scene(seed: int = 1002, n_rays: int = 1 << 20, M: int = 32, F: int = 4096, bounces: int = 4,
               diff_K: int = 65536, n_boxes=100, n_cyl=100):
    """Room scene: 10x8x3 m room + 100 boxes + 100 cylinders (193,212 tris), 16 materials x 8
    bands; 2^20 rays over the frontal hemisphere; <=4 bounces; 32-mic planar array in a 12 cm
    aperture; 4096 bins 20-100 kHz; curvature-threshold diffraction with 65,536 MC samples."""
    g = rng(seed)
    scene = room_geometry(g, n_boxes=n_boxes, n_cyl=n_cyl)
    k, beta, dcoef = band_tables(g, 16, 8)
    s = np.array([1.0, 4.0, 1.2])
    R = np.eye(3)
    mics = disc_mics(g, M, 0.12, s, R)
    sim = make_sim(emitter_pos=s, emitter_rot=R, rx_pos=mics, ray_dirs=cone_directions(g, n_rays, math.pi / 2),
                   max_bounces=bounces, f_lo=20e3, f_hi=100e3, F=F, refl_k=k, lobe_beta=beta,
                   diff_coef=dcoef, diff_K=diff_K, diff_seed=seed, diff_tau=0.1,
                   diff_max_incidence_deg=80.0, diff_cone_half_angle_deg=90.0)
    sim["area_ref"] = median_triangle_area(scene)
    return scene, sim


def directivity_table(g: np.random.Generator, M: int, Bd=16, El=32, Az=64) -> np.ndarray:
    """Synthetic receiver directivity in the receiver frame (boresight local +x):
    ((1 + cos el cos az)/2)^(1 + b/2) * (1 + 0.05 xi), xi ~ U[-1, 1] per cell; cell-centred grid."""
    az = -math.pi + (np.arange(Az) + 0.5) * 2 * math.pi / Az
    el = -math.pi / 2 + (np.arange(El) + 0.5) * math.pi / El
    base = (1 + np.cos(el)[:, None] * np.cos(az)[None, :]) / 2
    tab = np.empty((M, Bd, El, Az), np.float64)
    for m in range(M):
        for b in range(Bd):
            tab[m, b] = base ** (1 + b / 2) * (1 + 0.05 * g.uniform(-1, 1, (El, Az)))
    return np.ascontiguousarray(tab.astype(np.float32))


def foliage_scene(seed: int = 1003, n_leaves: int = 62500, n_rays: int = 1 << 22, F: int = 8192, bounces: int = 6):
    """Foliage: 62,500 seeded leaf discs (r 1-5 cm, 16 tris each: 1M tris) in a 4 m cube;
    2 receivers with a 64x32 az/el x 16-band directivity table; 2^22 rays (cone half-angle
    60 degrees); <=6 bounces; 8192 bins 20-200 kHz."""
    g = rng(seed)
    mb = MeshBuilder()
    s = np.array([2.0, 2.0, 2.0])
    placed = 0
    while placed < n_leaves:
        c = g.uniform(0, 4, 3)
        r = g.uniform(0.01, 0.05)
        n = g.normal(size=3)
        if np.linalg.norm(c - s) < 0.15 + r:
            continue
        v, t = disc_fan(c, n, r)
        mb.add(v, t, placed % 16)
        placed += 1
    scene = mb.build()
    k, beta, dcoef = band_tables(g, 16, 8)
    R = np.eye(3)
    rx = np.array([s + [0, 0.025, 0], s - [0, 0.025, 0]])
    rx_rot = np.stack([rot_z(math.radians(20)), rot_z(math.radians(-20))])
    sim = make_sim(emitter_pos=s, emitter_rot=R, rx_pos=rx, rx_rot=rx_rot,
                   ray_dirs=cone_directions(g, n_rays, math.radians(60)), max_bounces=bounces,
                   f_lo=20e3, f_hi=200e3, F=F, refl_k=k, lobe_beta=beta, diff_coef=dcoef,
                   directivity=directivity_table(g, 2))
    return scene, sim


def catmull_rom(pts: np.ndarray, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Positions and tangents at n uniform parameters along a Catmull-Rom spline through pts."""
    P = np.vstack([pts[:1], pts, pts[-1:]])
    segs = len(pts) - 1
    us = np.linspace(0, segs, n, endpoint=False)
    pos, tan = [], []
    for u in us:
        i = int(u)
        t = u - i
        p0, p1, p2, p3 = P[i], P[i + 1], P[i + 2], P[i + 3]
        pos.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t * t + (-p0 + 3 * p1 - 3 * p2 + p3) * t ** 3))
        tan.append(0.5 * ((-p0 + p2) + 2 * (2 * p0 - 5 * p1 + 4 * p2 - p3) * t + 3 * (-p0 + 3 * p1 - 3 * p2 + p3) * t * t))
    return np.array(pos), np.array(tan)


@dataclass
class Job:
    scene_index: int
    sim: dict


@dataclass
class Batch:
    scenes: list = field(default_factory=list)
    jobs: list = field(default_factory=list)


def _point_clear(scene, p, margin):
    v = scene["vertices"]
    obj = scene["tri_object"]
    t = scene["tris"]
    for o in range(1, scene["n_objects"]):
        idx = np.unique(t[obj == o])
        lo = v[idx].min(0) - margin
        hi = v[idx].max(0) + margin
        if np.all(p >= lo) and np.all(p <= hi):
            return False
    return True


def batched_workload(seed: int = 1004, n_poses: int = 256, n_scenes: int = 64, n_rays: int = 1 << 18,
                     M: int = 8, F: int = 2048, bounces: int = 4, room_kwargs=None, tmin=1e3, tmax=5e4):
    """Batched: n_poses sensor poses along a seeded spline through the room scene, plus
    n_scenes independent scenes of log-uniform size (box room + tessellated boxes/cylinders)
    with one free pose each."""
    g = rng(seed)
    room_kwargs = room_kwargs or {}
    room, room_sim = room_scene(1002, n_rays=8, M=8, F=16, diff_K=0, **room_kwargs)
    batch = Batch()
    batch.scenes.append(room)
    ctrl = []
    while len(ctrl) < 8:
        p = np.array([g.uniform(1.5, 8.5), g.uniform(1.5, 6.5), g.uniform(0.8, 1.8)])
        if _point_clear(room, p, 0.3):
            ctrl.append(p)
    pos, tan = catmull_rom(np.array(ctrl), n_poses)

    def job_sim(scene, p, fwd, tables):
        R = frame_from_forward(fwd)
        mics = disc_mics(g, M, 0.12, p, R)
        return make_sim(emitter_pos=p, emitter_rot=R, rx_pos=mics, ray_dirs=cone_directions(g, n_rays, math.pi / 2),
                        max_bounces=bounces, f_lo=20e3, f_hi=100e3, F=F, refl_k=tables[0], lobe_beta=tables[1],
                        diff_coef=tables[2])
    room_tables = (room_sim["refl_k"], room_sim["lobe_beta"], room_sim["diff_coef"])
    for i in range(n_poses):
        batch.jobs.append(Job(0, job_sim(room, pos[i], tan[i], room_tables)))
    for s_i in range(n_scenes):
        target = int(round(math.exp(g.uniform(math.log(tmin), math.log(tmax)))))
        dims = (g.uniform(3, 10), g.uniform(3, 8), g.uniform(2.5, 4))
        sensor = np.array([dims[0] * 0.3, dims[1] * 0.5, 1.2])
        # objects: 300-tri boxes (5x5 faces) and 400-tri cylinders, about half the triangles each,
        # so that the scene lands within 200 triangles of the target size
        nb = max(1, int(round((target - 12) * 0.5 / 300)))
        nc = max(0, int(round((target - 12 - 300 * nb) / 400)))
        sub = rng(seed * 1000 + s_i)
        scene = room_geometry(sub, n_boxes=nb, n_cyl=nc, sensor=sensor, box_subdiv=5,
                              cyl_segments=40, cyl_rings=4, room=dims, keepout=0.6)
        batch.scenes.append(scene)
        tables = band_tables(g, 16, 8)
        fwd = np.array([math.cos(g.uniform(0, 2 * math.pi)), math.sin(g.uniform(0, 2 * math.pi)), 0.0])
        if np.linalg.norm(fwd) < 1e-3:
            fwd = np.array([1.0, 0, 0])
        batch.jobs.append(Job(len(batch.scenes) - 1, job_sim(scene, sensor, fwd, tables)))
    return batch
