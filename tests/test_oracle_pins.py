"""Pins of the FP64 oracle against facts fixed by geometry, the paper's definitions and
published algorithms -- never against the oracle itself or the GPU path.

Each test names what pins it: the image-source construction of a planar wall, the
unfolding of an empty box room, the reciprocity of a single reflection point, the pure
delay of a unit-amplitude path, the textbook mean curvature of a sphere and of a plane,
the published SplitMix64 outputs, sampling statistics, and finite differences.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sim(**kw):
    base = dict(emitter_pos=[0, 0, 0], emitter_rot=np.eye(3), rx_pos=[[0, 0, 0]], ray_dirs=[[1, 0, 0]],
                max_bounces=1, f_lo=20e3, f_hi=100e3, F=257, refl_k=np.full((1, 8), 0.9),
                lobe_beta=np.full((1, 8), 0.1), diff_coef=np.full((1, 8), 0.1))
    base.update(kw)
    return W.make_sim(**base)


def wall_scene(d=3.0, h=5.0):
    """Planar wall x = d; its diagonal does not pass through (d, 0, 0)."""
    mb = W.MeshBuilder()
    mb.add(np.array([[d, -h, -2 * h], [d, h, -2 * h], [d, h, h], [d, -h, h]], float), np.array([[0, 1, 2], [0, 2, 3]]), 0)
    return mb.build()


def box_room(L=(5.0, 4.0, 3.0)):
    mb = W.MeshBuilder()
    v, t = W.quad_grid_box([0, 0, 0], list(L), 1)
    mb.add(v, t, 0)
    return mb.build()


# ---------------------------------------------------------------------------------------- IS-1

@pytest.mark.parametrize("p_s", [1.0, 2.0])
def test_image_source_single_wall(p_s):
    """On-axis ray at a planar wall x = d, receiver at the emitter: the echo is the image
    source at 2d -- delay 2d/c, spreading (2d)^-p, absorption over 2d, no lobe loss."""
    d = 3.0
    scene = wall_scene(d)
    sim = _sim(spreading_p=p_s)
    rec = O.trace(scene, sim)
    assert len(rec["rtot"]) == 1 and rec["vis"][0] == 1
    np.testing.assert_allclose(rec["p"][0], [d, 0, 0], atol=1e-12)
    np.testing.assert_allclose(rec["dout"][0], [-1, 0, 0], atol=1e-12)
    H = O.synth(rec, sim)[0]
    f = np.linspace(20e3, 100e3, 257)
    r = 2 * d
    atten = 10 ** (-(3.5e-5 * f) * r / 20)
    k32 = float(np.float32(0.9))   # the tables are FP32 inputs
    expect = k32 * r ** (-p_s) * atten * np.exp(1j * 2 * np.pi * f * r / 343.0)
    np.testing.assert_allclose(H, expect, rtol=1e-11, atol=1e-14)
    # the delay is 2d/c: the phase advances by 2 pi df (2d/c) per bin
    ratio = H[1:] / H[:-1]
    np.testing.assert_allclose(np.angle(ratio), np.angle(np.exp(1j * 2 * np.pi * (f[1] - f[0]) * r / 343.0)), atol=1e-9)


def test_single_wall_offset_receiver():
    """Receiver off axis: the method's path is emitter -> hit (d) -> receiver (sqrt(d^2+y^2)),
    deviation angle atan(y/d) between the mirror direction (-1,0,0) and the receiver."""
    d, y = 2.0, 0.3
    scene = wall_scene(d)
    sim = _sim(rx_pos=[[0, y, 0]])
    rec = O.trace(scene, sim)
    H = O.synth(rec, sim)[0]
    f = np.linspace(20e3, 100e3, 257)
    r = d + math.hypot(d, y)
    gam = math.atan2(y, d)
    k32, b32 = float(np.float32(0.9)), float(np.float32(0.1))
    expect = k32 * r ** -2 * 10 ** (-(3.5e-5 * f) * r / 20) * math.exp(-gam ** 2 / (2 * b32 ** 2)) * np.exp(
        1j * 2 * np.pi * f * r / 343.0)
    np.testing.assert_allclose(H, expect, rtol=1e-11, atol=1e-16)


# ---------------------------------------------------------------------------------------- IS-2

def test_single_wall_many_rays_geometry():
    """Every ray of a cone hitting the wall x = d lands at s + (d / cos theta) d, with
    path d / cos theta and the mirror direction (-dx, dy, dz)."""
    d = 3.0
    scene = wall_scene(d, h=20.0)
    g = W.rng(5)
    dirs = W.cone_directions(g, 500, math.radians(40))
    sim = _sim(ray_dirs=dirs)
    rec = O.trace(scene, sim)
    assert len(rec["rtot"]) == 500
    dd = dirs.astype(np.float64)
    dd /= np.linalg.norm(dd, axis=1, keepdims=True)
    tt = d / dd[:, 0]
    np.testing.assert_allclose(rec["rtot"], tt, rtol=1e-13)
    np.testing.assert_allclose(rec["p"], dd * tt[:, None], atol=1e-12)
    np.testing.assert_allclose(rec["dout"], dd * np.array([-1, 1, 1]), atol=1e-13)


# ---------------------------------------------------------------------------------------- IS-4

def _unfold(s, d, L, n):
    """First n wall crossings of the straight line s + t d in the unfolded box lattice."""
    cross = []
    for a in range(3):
        if d[a] == 0:
            continue
        if d[a] > 0:
            ks = np.arange(1, n + 2)
        else:
            ks = -np.arange(0, n + 1)
        for k in ks:
            cross.append(((k * L[a] - s[a]) / d[a], a))
    cross.sort()
    cross = cross[:n]
    out = []
    flips = np.zeros(3, int)
    for t, a in cross:
        q = s + t * d
        p = np.empty(3)
        for b in range(3):
            m = np.mod(q[b], 2 * L[b])
            p[b] = m if m <= L[b] else 2 * L[b] - m
        din = d * (-1.0) ** flips
        flips[a] += 1
        out.append((t, a, p, din))
    return out, cross


def test_box_room_unfolding():
    """In an empty axis-aligned box, the n-th hit is the n-th lattice-plane crossing of the
    unfolded straight line: path t_n, point fold(s + t_n d), incoming direction with one
    sign flip per earlier crossing of that axis."""
    L = np.array([5.0, 4.0, 3.0])
    scene = box_room(tuple(L))
    s = np.array([1.3, 1.7, 1.1])
    g = W.rng(7)
    v = g.normal(size=(200, 3))
    dirs = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    B = 6
    sim = _sim(emitter_pos=s, ray_dirs=dirs, max_bounces=B, rx_pos=[s + [0, 0.02, 0]])
    rec = O.trace(scene, sim)
    checked = 0
    for i in range(len(dirs)):
        d = dirs[i].astype(np.float64)
        d /= np.linalg.norm(d)
        exp, cr = _unfold(s, d, L, B)
        ts = [c[0] for c in cr]
        if min(np.diff(ts)) < 1e-6:
            continue                                   # corner / edge crossing: ambiguous order
        sel = rec["ray"] == i
        assert sel.sum() == B
        for j, (t, a, p, din) in enumerate(exp):
            k = np.nonzero(sel)[0][j]
            assert rec["bounce"][k] == j
            np.testing.assert_allclose(rec["rtot"][k], t, rtol=1e-12)
            np.testing.assert_allclose(rec["p"][k], p, atol=1e-10)
            np.testing.assert_allclose(rec["din"][k], din, atol=1e-12)
            # the hit triangle lies in the crossed wall plane
            tri = scene["tris"][rec["tri"][k]]
            wall = scene["vertices"][tri][:, a]
            assert np.all(np.abs(wall - p[a]) < 1e-9)
        checked += 1
    assert checked > 180


def test_max_distance_between_parallel_walls():
    """Algorithm 1 records a hit and then stops the ray once its path reaches MaxDistance.
    Between walls x = 0 and x = D with the emitter at x = e, a ray at angle theta to the x axis
    reaches its n-th wall after r_n = ((D - e) + (n - 1) D) / cos(theta); the ray keeps exactly
    the records up to the first r_n >= MaxDistance (or max_bounces of them)."""
    D, e = 3.0, 1.0
    mb = W.MeshBuilder()
    for x in (0.0, D):
        mb.add(np.array([[x, -50, -50], [x, 50, -50], [x, 50, 50], [x, -50, 50]], float),
               np.array([[0, 1, 2], [0, 2, 3]]), 0)
    scene = mb.build()
    th = np.radians([0.0, 17.0, 41.0])
    dirs = np.stack([np.cos(th), np.sin(th) * 0.6, np.sin(th) * 0.8], 1).astype(np.float32)
    B = 8
    for md in (0.5, 4.0, 6.5, 13.9, 40.0, math.inf):
        sim = _sim(emitter_pos=[e, 0.1, -0.2], ray_dirs=dirs, max_bounces=B, max_distance=md,
                   rx_pos=[[e, 0.12, -0.2]])
        rec = O.trace(scene, sim)
        for i in range(len(dirs)):
            d = dirs[i].astype(np.float64)
            c = d[0] / np.linalg.norm(d)
            r = ((D - e) + np.arange(B) * D) / c
            n = int(np.argmax(r >= md)) + 1 if np.any(r >= md) else B
            sel = rec["ray"] == i
            assert sel.sum() == n, (md, i)
            np.testing.assert_allclose(rec["rtot"][sel], r[:n], rtol=1e-12)
            assert rec["certified"][i]
    # a path that reaches MaxDistance within the FP32 margin is not certified
    sim = _sim(emitter_pos=[e, 0.1, -0.2], ray_dirs=dirs[:1], max_bounces=B, max_distance=5.0 * (1 + 1e-9),
               rx_pos=[[e, 0.12, -0.2]])
    rec = O.trace(scene, sim)
    assert not rec["certified"][0]
    # an exact tie stops the ray (r >= MaxDistance): along the axis the paths 2 and 5 are exact
    sim = _sim(emitter_pos=[e, 0.1, -0.2], ray_dirs=dirs[:1], max_bounces=B, max_distance=5.0,
               rx_pos=[[e, 0.12, -0.2]])
    rec = O.trace(scene, sim)
    assert list(rec["rtot"]) == [2.0, 5.0]


# ---------------------------------------------------------------------------------------- reciprocity

def test_reciprocity_single_point():
    """Swapping emitter and receiver about one reflection point leaves the path length and
    the deviation angle unchanged, hence the spectrum (R(a).b = a.R(b) for a mirror R)."""
    scene = wall_scene(2.0)
    A = np.array([0.0, 0.0, 0.0])
    Bp = np.array([0.0, 2.0, 0.5])
    p = np.array([2.0, 1.0, 0.25])
    # exact FP32 directions (the oracle normalises in FP64): toward p from A and from B
    simAB = _sim(emitter_pos=A, rx_pos=[Bp], ray_dirs=[[2.0, 1.0, 0.25]], x_ref=Bp)
    simBA = _sim(emitter_pos=Bp, rx_pos=[A], ray_dirs=[[2.0, -1.0, -0.25]], x_ref=A)
    rAB = O.trace(scene, simAB)
    rBA = O.trace(scene, simBA)
    np.testing.assert_allclose(rAB["p"][0], p, atol=1e-13)
    np.testing.assert_allclose(rBA["p"][0], p, atol=1e-13)
    HAB = O.synth(rAB, simAB)
    HBA = O.synth(rBA, simBA)
    np.testing.assert_allclose(HAB, HBA, rtol=1e-12, atol=0)
    # the off-specular case: same point, different receiver heights still reciprocal
    C2 = np.array([0.0, 2.3, -0.4])
    s1 = _sim(emitter_pos=A, rx_pos=[C2], ray_dirs=[[2.0, 1.0, 0.25]], x_ref=C2)
    r1 = O.trace(scene, s1)
    dC = (p - C2).astype(np.float32)
    s2 = _sim(emitter_pos=C2, rx_pos=[A], ray_dirs=[dC], x_ref=A)
    r2 = O.trace(scene, s2)
    assert np.linalg.norm(r2["p"][0] - p) < 1e-6            # FP32 direction from C2 is rounded
    H1, H2 = O.synth(r1, s1), O.synth(r2, s2)
    np.testing.assert_allclose(np.abs(H1), np.abs(H2), rtol=1e-5)


# ---------------------------------------------------------------------------------------- synthesis

def test_pure_delay_special_case():
    """alpha = 0, beta -> inf, p = 0, k = 1: each bin is exp(j 2 pi f r / c); the spectrum is a
    geometric sequence in k and its forward DFT peaks at bin F df r / c (delay r / c)."""
    F = 1024
    sim = _sim(F=F, atm_a1=0.0, spreading_p=0.0, refl_k=np.ones((1, 8)), lobe_beta=np.full((1, 8), 1e6))
    r_tot, ell = 1.5, 1.0
    rec = {"p": np.array([[1.0, 0, 0]]), "dout": np.array([[-1.0, 0, 0]]), "rtot": np.array([r_tot]),
           "mat": np.array([0], np.int32)}
    H = O.synth(rec, sim)[0]
    r = r_tot + ell
    np.testing.assert_allclose(np.abs(H), 1.0, atol=1e-12)
    df = (100e3 - 20e3) / (F - 1)
    ratio = H[1:] / H[:-1]
    np.testing.assert_allclose(ratio, np.exp(1j * 2 * np.pi * df * r / 343.0), atol=1e-10)
    h = np.fft.fft(H)
    assert np.argmax(np.abs(h)) == int(round(F * df * r / 343.0)) % F


def test_spectrum_is_linear_in_records():
    """Eq. (6): the total response is the sum of per-point responses."""
    scene, sim = W.tiny_scene(n_rays=64, F=64)
    rec = O.trace(scene, sim)
    H = O.synth(rec, sim)
    parts = sum(O.synth({k: v[i:i + 1] for k, v in rec.items() if k not in ("certified", "nseg")}, sim)
                for i in range(len(rec["rtot"])))
    np.testing.assert_allclose(H, parts, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------------------- curvature

def test_curvature_sphere():
    """Mean curvature of a sphere of radius r is 1/r: the Meyer operator on an icosphere
    (subdivision 3) reproduces it within its O(h^2) discretisation error."""
    v, t = W.icosphere(3, 0.5)
    scene = {"vertices": v.astype(np.float32), "tris": t.astype(np.int32)}
    G, C = O.curvature(scene, 1.0)
    np.testing.assert_allclose(G, 2.0, rtol=2e-3)
    # scaling by s divides curvature by s
    scene2 = {"vertices": (2 * v).astype(np.float32), "tris": t.astype(np.int32)}
    G2, _ = O.curvature(scene2, 1.0)
    np.testing.assert_allclose(G2, G / 2, rtol=1e-6)


def test_curvature_flat_plane():
    """The cotangent Laplacian reproduces linear functions: interior vertices of a flat
    mesh have K = 0; so does every triangle with only interior vertices."""
    n = 8
    xs, ys = np.meshgrid(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1) ** 1.3, indexing="ij")
    v = np.stack([xs.ravel(), ys.ravel(), np.zeros(xs.size)], 1).astype(np.float32)
    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = i * (n + 1) + j, (i + 1) * (n + 1) + j, (i + 1) * (n + 1) + j + 1, i * (n + 1) + j + 1
            tris += [(a, b, c), (a, c, d)]
    t = np.array(tris, np.int32)
    G, C = O.curvature({"vertices": v, "tris": t}, 1.0)
    interior = np.ones((n + 1, n + 1), bool)
    interior[0, :] = interior[-1, :] = interior[:, 0] = interior[:, -1] = False
    interior = interior.ravel()
    assert np.all(np.abs(G[interior]) < 1e-12)
    assert np.all(G[~interior] > 1e-3)                    # open boundary: one-sided cotangents
    inner_tri = interior[t].all(1)
    assert np.all(C[inner_tri] == 0)


def _fan(apex, rim):
    """One-ring of the vertex `apex` (index 0): triangles (apex, rim[i], rim[i + 1]), closed."""
    v = np.vstack([apex, rim]).astype(np.float32)
    n = len(rim)
    t = np.array([[0, 1 + i, 1 + (i + 1) % n] for i in range(n)], np.int32)
    return v, t


def _ring_area(v, t, apex):
    w = np.asarray(v, np.float64).copy()
    w[0] = apex
    a = w[t[:, 1]] - w[t[:, 0]]
    b = w[t[:, 2]] - w[t[:, 0]]
    return 0.5 * np.sum(np.linalg.norm(np.cross(a, b), axis=1))


def _angles(v, t):
    """Interior angles [T][3] (radians) at the triangles' three corners, FP64."""
    w = np.asarray(v, np.float64)
    out = np.zeros((len(t), 3))
    for c in range(3):
        a = w[t[:, (c + 1) % 3]] - w[t[:, c]]
        b = w[t[:, (c + 2) % 3]] - w[t[:, c]]
        out[:, c] = np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1))
    return out


def test_curvature_regular_pyramid_apex_closed_forms():
    """Apex of a regular pyramid (n rim vertices at radius R, apex height h): the cotangent
    operator of Eq. (1) (Meyer et al.) gives |K| = |grad of the one-ring area| / A_mixed.
    Non-obtuse one-ring (n = 6): the Voronoi areas give G = 2h / (R^2 + h^2).  Obtuse apex
    (n = 3, h^2 < R^2 / 2): A_mixed = half the ring's area, G = h / (R^2 cos^2(pi/3) + h^2)."""
    R = 1.0
    for n, h, expect in ((6, 0.45, lambda h: 2 * h / (R * R + h * h)),
                         (3, 0.30, lambda h: h / (R * R * math.cos(math.pi / 3) ** 2 + h * h))):
        ang = 2 * math.pi * np.arange(n) / n
        rim = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros(n)], 1)
        v, t = _fan([0, 0, h], rim)
        h32 = float(v[0, 2])   # the FP32 apex the oracle sees (the rim is exact in FP32 up to rounding)
        G, _ = O.curvature({"vertices": v, "tris": t}, 1.0)
        A = _angles(v, t)
        if n == 3:
            assert np.all(A[:, 0] > math.pi / 2)            # obtuse at the apex
        else:
            assert np.all(A < math.pi / 2)
        # closed form on the FP32 geometry: rim radius and apex height as stored
        R32 = float(np.mean(np.linalg.norm(v[1:, :2].astype(np.float64), axis=1)))
        if n == 6:
            want = 2 * h32 / (R32 * R32 + h32 * h32)
        else:
            want = h32 / (R32 * R32 * math.cos(math.pi / 3) ** 2 + h32 * h32)
        np.testing.assert_allclose(G[0], want, rtol=1e-6)
        assert abs(want - expect(h)) < 1e-6 * want


def test_curvature_obtuse_one_ring_mixed_area():
    """A one-ring whose triangles are all obtuse, some at the centre vertex and some at a rim
    vertex.  Meyer et al.'s mixed area is then area/2 for a triangle obtuse at the vertex and
    area/4 for one obtuse elsewhere; the cotangent sum is twice the gradient of the ring's area
    with respect to the vertex (central differences of plain triangle areas here), so
    G = |grad A_ring| / (2 A_mixed).  Swapping the two weights changes G by far more than the
    tolerance."""
    phi = np.radians([0.0, 140.0, 195.0, 250.0, 305.0])
    r = np.array([1.0, 1.0, 0.3, 1.0, 0.3])
    rim = np.stack([r * np.cos(phi), r * np.sin(phi), np.array([0.0, 0.02, -0.01, 0.03, -0.02])], 1)
    v, t = _fan([0.0, 0.0, 0.05], rim)
    A = _angles(v, t)
    obt_c = A[:, 0] > math.pi / 2
    obt_o = (A[:, 1:] > math.pi / 2).any(1)
    assert np.all(obt_c | obt_o) and obt_c.any() and obt_o.any()
    assert np.min(np.abs(A - math.pi / 2)) > 0.1          # clear of right angles
    w = np.asarray(v, np.float64)
    area = 0.5 * np.linalg.norm(np.cross(w[t[:, 1]] - w[t[:, 0]], w[t[:, 2]] - w[t[:, 0]]), axis=1)
    a_mixed = np.sum(np.where(obt_c, area / 2, area / 4))
    hd = 1e-6
    grad = np.array([(_ring_area(v, t, w[0] + hd * e) - _ring_area(v, t, w[0] - hd * e)) / (2 * hd) for e in np.eye(3)])
    want = np.linalg.norm(grad) / (2 * a_mixed)
    G, _ = O.curvature({"vertices": v, "tris": t}, 1.0)
    swapped = np.linalg.norm(grad) / (2 * np.sum(np.where(obt_c, area / 4, area / 2)))
    assert abs(swapped - want) > 0.05 * want
    np.testing.assert_allclose(G[0], want, rtol=1e-7)


def test_curvature_box_edges():
    """A subdivided box is flat except along its edges: C_i > 0 exactly on triangles that
    touch an edge or corner of the box."""
    v, t = W.quad_grid_box([0, 0, 0], [1.0, 0.7, 0.4], 5)
    G, C = O.curvature({"vertices": v.astype(np.float32), "tris": t.astype(np.int32)}, 1.0)
    lo, hi = v.min(0), v.max(0)
    on_edge = ((np.abs(v - lo) < 1e-9) | (np.abs(v - hi) < 1e-9)).sum(1) >= 2
    assert np.all(G[~on_edge] < 1e-9)
    assert np.all(G[on_edge] > 1e-3)
    touches = on_edge[t].any(1)
    # triangles whose vertices all sit on edges can still have dG = 0 (equal G); never the reverse
    assert np.all(C[~touches] < 1e-12)              # rounding noise of a flat one-ring only
    assert (C[touches] > 0).mean() > 0.5


# ---------------------------------------------------------------------------------------- RNG

def test_splitmix_published_outputs():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if l.strip() and not l.startswith("#")]
    for c, hexv in rows:
        assert O.splitmix(0, int(c)) == int(hexv, 16)


# ---------------------------------------------------------------------------------------- diffraction

def _boxes_scene():
    mb = W.MeshBuilder()
    g = W.rng(11)
    for i in range(6):
        v, t = W.quad_grid_box([0, 0, 0], list(g.uniform(0.3, 0.8, 3)), 4)
        mb.add(v + np.array([2.0 + i * 0.9, g.uniform(-1, 1), g.uniform(-0.5, 0.5)]), t, i % 3)
    return mb.build()


def test_diffraction_sampler_statistics():
    """Samples are drawn with probability q_i / sum(q): chi-square of the triangle histogram;
    every sample lies on its triangle; only edge triangles of the boxes carry weight."""
    from scipy.stats import chisquare
    scene = _boxes_scene()
    G, C = O.curvature(scene, W.median_triangle_area(scene))
    sim = _sim(diff_K=200000, diff_seed=99, diff_tau=0.0, diff_cone_half_angle_deg=90.0)
    s = O.diffraction(scene, sim, C, certify=False)
    q = s["q"].astype(np.float64)
    assert s["n_elig"] == int((q > 0).sum())
    assert np.all(C[q > 0] > 0)
    # dithered weights: q = floor(x) or floor(x) + 1 with x = C / Cmax * 2^32
    x = C / C.max() * 2.0 ** 32
    sel = q > 0
    assert np.all((q[sel] == np.floor(x[sel])) | (q[sel] == np.floor(x[sel]) + 1))
    tri = s["tri"]
    assert np.all(q[tri] > 0)
    counts = np.bincount(tri, minlength=len(q))[sel]
    expect = q[sel] / q[sel].sum() * len(tri)
    big = expect >= 5
    obs, exp = counts[big], expect[big]
    if (~big).any():
        obs, exp = np.append(obs, counts[~big].sum()), np.append(exp, expect[~big].sum())
    assert chisquare(obs, exp).pvalue > 1e-3
    # each sample point lies on its triangle (barycentric coordinates in [0, 1])
    V = scene["vertices"].astype(np.float64)
    T = scene["tris"][tri]
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    o = s["o"]
    n = np.cross(b - a, c - a)
    area = np.linalg.norm(n, axis=1)
    wa = np.einsum("ij,ij->i", np.cross(b - o, c - o), n) / area ** 2
    wb = np.einsum("ij,ij->i", np.cross(c - o, a - o), n) / area ** 2
    assert np.all(wa > -1e-9) and np.all(wb > -1e-9) and np.all(wa + wb < 1 + 1e-9)
    assert np.all(np.abs(np.einsum("ij,ij->i", o - a, n / area[:, None])) < 1e-12)


def test_diffraction_filters():
    """Kept samples satisfy the incidence constraint and see the source; the field-of-view
    test removes objects behind the emitter."""
    scene = _boxes_scene()
    G, C = O.curvature(scene, W.median_triangle_area(scene))
    sim = _sim(diff_K=4000, diff_seed=5, diff_tau=0.1, diff_max_incidence_deg=60.0, diff_cone_half_angle_deg=90.0)
    s = O.diffraction(scene, sim, C, certify=False)
    V = scene["vertices"].astype(np.float64)
    T = scene["tris"][s["tri"]]
    n = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    w = -s["o"]
    cosi = np.abs(np.einsum("ij,ij->i", n, w)) / np.linalg.norm(w, axis=1)
    assert np.all(cosi[s["keep"]] >= math.cos(math.radians(60)) - 1e-12)
    np.testing.assert_allclose(s["r_src"], np.linalg.norm(s["o"], axis=1), rtol=1e-14)
    # rear-facing emitter: boxes sit at x > 1.5, a cone about -x with half-angle 30 deg sees none
    sim_back = _sim(diff_K=100, diff_seed=5, emitter_rot=np.diag([-1.0, -1.0, 1.0]), diff_cone_half_angle_deg=30.0)
    s2 = O.diffraction(scene, sim_back, C, certify=False)
    assert s2["n_elig"] == 0 and not s2["keep"].any()


def test_diffraction_per_mesh_allocation():
    """Sec. III-D, a fixed number of candidates per mesh: every mesh with eligible triangles
    gets K draws from its own CDF (chi-square per mesh), in increasing object order; one mesh
    alone reproduces the global sampler draw for draw; a cap on the meshes truncates."""
    from scipy.stats import chisquare
    scene = _boxes_scene()
    G, C = O.curvature(scene, W.median_triangle_area(scene))
    K = 30000
    sim = _sim(diff_K=K, diff_seed=99, diff_tau=0.0, diff_cone_half_angle_deg=90.0, diff_per_mesh=True,
               diff_max_meshes=scene["n_objects"])
    s = O.diffraction(scene, sim, C, certify=False)
    q = s["q"].astype(np.float64)
    obj = scene["tri_object"]
    meshes = sorted(set(obj[q > 0].tolist()))
    assert len(meshes) == scene["n_objects"] == 6 and not s["truncated"]
    assert len(s["tri"]) == K * len(meshes)
    for r, o in enumerate(meshes):
        tri = s["tri"][r * K:(r + 1) * K]
        assert np.all(obj[tri] == o)
        sel = (q > 0) & (obj == o)
        counts = np.bincount(tri, minlength=len(q))[sel]
        expect = q[sel] / q[sel].sum() * K
        big = expect >= 5
        ob, ex = counts[big], expect[big]
        if (~big).any():
            ob, ex = np.append(ob, counts[~big].sum()), np.append(ex, expect[~big].sum())
        assert chisquare(ob, ex).pvalue > 1e-4
    # a single mesh: the per-mesh sampler is the global one
    one = dict(scene, tri_object=np.zeros_like(obj), n_objects=1)
    a = O.diffraction(one, sim, C, certify=False)
    b = O.diffraction(one, dict(sim, diff_per_mesh=False), C, certify=False)
    assert np.array_equal(a["tri"], b["tri"]) and np.array_equal(a["o"], b["o"])
    # at most two meshes: the first two by object id
    c = O.diffraction(scene, dict(sim, diff_max_meshes=2), C, certify=False)
    assert c["truncated"] and len(c["tri"]) == 2 * K
    assert np.array_equal(c["tri"], s["tri"][:2 * K])


# ---------------------------------------------------------------------------------------- adjoint

def _loss(rec, sim, Hstar):
    H = O.synth(rec, sim)
    return float(np.sum(np.abs(H - Hstar) ** 2))


def test_adjoint_matches_finite_differences():
    """Central differences (h = 1e-6, FP64) of L = sum |H - H*|^2 with respect to every band
    coefficient and every receiver coordinate match the analytic adjoint."""
    scene, sim = W.tiny_scene(n_rays=48, F=64)
    g = W.rng(3)
    sim["refl_k"] = np.ascontiguousarray(g.uniform(0.3, 0.99, (1, 8)).astype(np.float32))
    sim["lobe_beta"] = np.ascontiguousarray(g.uniform(0.1, 0.3, (1, 8)).astype(np.float32))
    rec = O.trace(scene, sim)
    assert len(rec["rtot"]) > 20
    hidden = dict(sim)
    hidden["refl_k"] = np.ascontiguousarray(g.uniform(0.3, 0.99, (1, 8)).astype(np.float32))
    Hstar = O.synth(rec, hidden)
    H = O.synth(rec, sim)
    gk, gx = O.grad(rec, sim, H - Hstar)
    # k is FP32 in the ABI; differentiate in FP64 through a float64 table (the oracle promotes exactly)
    h = 1e-6
    for b in range(8):
        kp = sim["refl_k"].astype(np.float64).copy(); kp[0, b] += h
        km = sim["refl_k"].astype(np.float64).copy(); km[0, b] -= h
        # H is linear in k: evaluate with unit tables to stay in FP64
        e = np.zeros((1, 8), np.float32); e[0, b] = 1.0
        Hb = O.synth(rec, dict(sim, refl_k=e))
        Lp = np.sum(np.abs(H + h * Hb - Hstar) ** 2)
        Lm = np.sum(np.abs(H - h * Hb - Hstar) ** 2)
        np.testing.assert_allclose(gk[0, b], (Lp - Lm) / (2 * h), rtol=1e-6, atol=1e-12 * abs(Lp))
    for m in range(2):
        for a in range(3):
            sp = dict(sim); sp["rx_pos"] = sim["rx_pos"].copy(); sp["rx_pos"][m, a] += h
            sm = dict(sim); sm["rx_pos"] = sim["rx_pos"].copy(); sm["rx_pos"][m, a] -= h
            fd = (_loss(rec, sp, Hstar) - _loss(rec, sm, Hstar)) / (2 * h)
            np.testing.assert_allclose(gx[m, a], fd, rtol=1e-5, atol=1e-9 * max(1.0, abs(fd)))


def test_adjoint_at_zero_coefficients_matches_finite_differences():
    """H is linear in k (Eq. 2), so dL/dk_qb does not vanish where k_qb = 0: central
    differences of L in FP64 (k - h < 0 included, the magnitude is linear through zero) match
    the analytic gradient at bands whose coefficient is exactly zero and at the others."""
    scene, sim = W.tiny_scene(n_rays=48, F=64)
    g = W.rng(33)
    k = g.uniform(0.3, 0.99, (1, 8)).astype(np.float32)
    k[0, 2] = 0.0
    k[0, 5] = 0.0
    sim = dict(sim, refl_k=k, lobe_beta=np.ascontiguousarray(g.uniform(0.1, 0.3, (1, 8)).astype(np.float32)))
    rec = O.trace(scene, sim)
    Hstar = O.synth(rec, dict(sim, refl_k=g.uniform(0.3, 0.99, (1, 8)).astype(np.float32)))
    gk, _ = O.grad(rec, sim, O.synth(rec, sim) - Hstar)
    h = 1e-3
    for b in range(8):
        kp = k.copy(); kp[0, b] += h
        km = k.copy(); km[0, b] -= h
        dk = float(kp[0, b]) - float(km[0, b])      # the FP32 steps actually taken
        fd = (_loss(rec, dict(sim, refl_k=kp), Hstar) - _loss(rec, dict(sim, refl_k=km), Hstar)) / dk
        np.testing.assert_allclose(gk[0, b], fd, rtol=1e-6, atol=1e-12)
    assert abs(gk[0, 2]) > 1e-3 * np.max(np.abs(gk)) and abs(gk[0, 5]) > 1e-3 * np.max(np.abs(gk))


def test_directivity_adjoint_matches_finite_differences():
    """With receiver directivity (a rough random 64 x 32 table per band and receiver, rotated
    receiver frames), central differences of L with respect to every receiver coordinate match
    the analytic gradient, whose direction-of-arrival term is not small here (it changes the
    gradient by more than the tolerance)."""
    scene, sim = W.tiny_scene(n_rays=48, F=64)
    g = W.rng(7)
    sim = dict(sim, directivity=np.ascontiguousarray(g.uniform(0.2, 1.0, (2, 4, 32, 64)).astype(np.float32)))
    rot = []
    for ang in (0.4, -0.9):
        c, s_ = np.cos(ang), np.sin(ang)
        rz = np.array([[c, -s_, 0], [s_, c, 0], [0, 0, 1]])
        rx = np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)], [0, np.sin(0.3), np.cos(0.3)]])
        rot.append(rz @ rx)
    sim["rx_rot"] = np.ascontiguousarray(np.stack(rot))
    rec = O.trace(scene, sim)
    assert len(rec["rtot"]) > 20
    Hstar = O.synth(rec, dict(sim, rx_pos=sim["rx_pos"] + g.normal(0, 2e-3, sim["rx_pos"].shape)))
    H = O.synth(rec, sim)
    _, gx = O.grad(rec, sim, H - Hstar)
    # the same records and target without the directivity term in the gradient (but with it in
    # H) must disagree: the term is exercised
    plain = dict(sim, directivity=None)
    _, gx0 = O.grad(rec, plain, O.synth(rec, sim) - Hstar)
    assert np.max(np.abs(gx - gx0)) > 1e-3 * np.max(np.abs(gx))
    h = 1e-6
    for m in range(2):
        for a in range(3):
            sp = dict(sim); sp["rx_pos"] = sim["rx_pos"].copy(); sp["rx_pos"][m, a] += h
            sm = dict(sim); sm["rx_pos"] = sim["rx_pos"].copy(); sm["rx_pos"][m, a] -= h
            fd = (_loss(rec, sp, Hstar) - _loss(rec, sm, Hstar)) / (2 * h)
            np.testing.assert_allclose(gx[m, a], fd, rtol=1e-5, atol=1e-9 * max(1.0, abs(fd)))


def _directivity_probe(table, v_local, rx, R):
    """|H| of one secondary-source record seen by a receiver at rx with frame R, arriving from
    the receiver-frame direction v_local: with no spreading, no absorption and I_d = 1 every
    bin's magnitude is the receiver gain of its directivity band (F = Bd bins, one per band)."""
    M, Bd, El, Az = table.shape
    v = np.asarray(v_local, np.float64)
    p = np.asarray(rx, np.float64) + 1.7 * (np.asarray(R) @ (v / np.linalg.norm(v)))
    rec = {"p": p[None], "dout": np.zeros((1, 3)), "rtot": np.array([0.3]), "mat": np.zeros(1, np.int32),
           "kind": np.ones(1, np.uint8), "vis": np.ones(1, np.uint8)}
    sim = _sim(rx_pos=[rx], rx_rot=np.asarray(R)[None], F=Bd, f_lo=40e3, f_hi=41e3, spreading_p=0.0, atm_a1=0.0,
               diff_coef=np.ones((1, 1)), refl_k=np.ones((1, 1)), lobe_beta=np.ones((1, 1)), directivity=table)
    return np.abs(O.synth(rec, sim)[0])


def _cell_dir(az, el):
    return [math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)]


def test_directivity_lookup_cell_centres_and_between():
    """Receiver directivity (the receiver transfer function of the signal-generation section,
    read as a real gain on a cell-centred azimuth/elevation grid in the receiver frame, bilinear,
    periodic in azimuth, clamped in elevation), seen through a receiver turned by a known yaw and
    pitch:
      * at the centre of cell (i, j) (az = -pi + (i + 1/2) 2pi/Az, el = -pi/2 + (j + 1/2) pi/El)
        the gain is the table entry itself;
      * a table linear in the cell-centre angles is reproduced exactly in between;
      * across the azimuth seam (between the last and the first centre) it interpolates the two;
      * beyond the outermost elevation centre it keeps that row's value."""
    El, Az, Bd = 8, 16, 2
    yaw, pitch = 0.7, -0.4
    rz = np.array([[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0], [0, 0, 1]])
    ry = np.array([[math.cos(pitch), 0, math.sin(pitch)], [0, 1, 0], [-math.sin(pitch), 0, math.cos(pitch)]])
    R = rz @ ry
    rx = [0.3, -0.2, 0.5]
    da, de = 2 * math.pi / Az, math.pi / El
    az_c = -math.pi + (np.arange(Az) + 0.5) * da
    el_c = -math.pi / 2 + (np.arange(El) + 0.5) * de
    g = W.rng(17)
    rough = g.uniform(0.2, 1.0, (1, Bd, El, Az)).astype(np.float32)
    for (i, j) in [(0, 0), (3, 5), (15, 7), (8, 2), (11, 4)]:
        got = _directivity_probe(rough, _cell_dir(az_c[i], el_c[j]), rx, R)
        np.testing.assert_allclose(got, rough[0, :, j, i], rtol=1e-9)
    # a table linear in the centre angles: D = a + b az + c el (band 1 with other coefficients)
    coef = [(1.5, 0.05, 0.1), (2.0, -0.07, 0.2)]
    lin = np.zeros((1, Bd, El, Az), np.float32)
    for b, (a0, a1, a2) in enumerate(coef):
        lin[0, b] = a0 + a1 * az_c[None, :] + a2 * el_c[:, None]
    for az, el in [(0.3, 0.2), (-1.1, -0.9), (2.5, 1.1), (-2.9, 0.05)]:
        got = _directivity_probe(lin, _cell_dir(az, el), rx, R)
        # bilinear interpolation of the stored FP32 samples of a linear function is that function
        # (up to the FP32 rounding of the samples)
        want = np.array([a0 + a1 * az + a2 * el for (a0, a1, a2) in coef])
        np.testing.assert_allclose(got, want, rtol=3e-7)
    # azimuth seam: a quarter of the way from the last centre (pi - da/2) to the first (-pi + da/2)
    saw = np.zeros((1, Bd, El, Az), np.float32)
    saw[0, :, :, :] = np.arange(Az, dtype=np.float32)[None, None, :] + 100 * np.arange(El, dtype=np.float32)[None, :, None]
    got = _directivity_probe(saw, _cell_dir(math.pi - da / 4, el_c[3]), rx, R)
    np.testing.assert_allclose(got, 0.75 * (Az - 1) + 0.25 * 0 + 300, rtol=1e-9)
    got = _directivity_probe(saw, _cell_dir(-math.pi + da / 4, el_c[3]), rx, R)
    np.testing.assert_allclose(got, 0.25 * (Az - 1) + 0.75 * 0 + 300, rtol=1e-9)
    # elevation beyond the top and bottom centres: clamped to those rows
    got = _directivity_probe(lin, _cell_dir(0.4, math.pi / 2 - de / 5), rx, R)
    np.testing.assert_allclose(got, [a0 + a1 * 0.4 + a2 * el_c[-1] for (a0, a1, a2) in coef], rtol=3e-7)
    got = _directivity_probe(lin, _cell_dir(-0.6, -math.pi / 2 + de / 3), rx, R)
    np.testing.assert_allclose(got, [a0 - a1 * 0.6 + a2 * el_c[0] for (a0, a1, a2) in coef], rtol=3e-7)


def test_spectrum_linear_in_band_coefficients():
    """With the reflection coefficient of the hit triangle only, H is linear in k:
    H(k) = sum_{q,b} k_qb H(e_qb)."""
    scene, sim = W.tiny_scene(n_rays=64, F=32)
    rec = O.trace(scene, sim)
    g = W.rng(4)
    k = g.uniform(0.3, 0.99, (1, 8)).astype(np.float32)
    H = O.synth(rec, dict(sim, refl_k=k))
    acc = 0
    for b in range(8):
        e = np.zeros((1, 8), np.float32); e[0, b] = 1
        acc = acc + float(k[0, b]) * O.synth(rec, dict(sim, refl_k=e))
    np.testing.assert_allclose(H, acc, rtol=1e-12, atol=1e-16)


# ---------------------------------------------------------------------------------------- invariants

def test_closed_sphere_never_missed_from_inside():
    """Rays from the centre of a closed icosphere all hit it (brute force, FP64)."""
    v, t = W.icosphere(3, 0.5)
    mb = W.MeshBuilder(); mb.add(v, t, 0)
    scene = mb.build()
    g = W.rng(9)
    d = g.normal(size=(2000, 3)).astype(np.float32)
    sim = _sim(ray_dirs=d, max_bounces=1, rx_pos=[[0.01, 0, 0]])
    rec = O.trace(scene, sim)
    assert len(rec["rtot"]) == 2000
    np.testing.assert_allclose(np.linalg.norm(rec["p"], axis=1), 0.5, rtol=0.01)


def test_margin_predicate_flags_edge_hits():
    """Rays aimed exactly at the shared diagonal of a two-triangle wall are marginal;
    rays through triangle interiors are certified."""
    d = 3.0
    mb = W.MeshBuilder()
    mb.add(np.array([[d, -2, -2], [d, 2, -2], [d, 2, 2], [d, -2, 2]], float), np.array([[0, 1, 2], [0, 2, 3]]), 0)
    scene = mb.build()
    dirs = np.array([[3, 0, 0], [3, 1, 1], [3, 0.5, -1.2], [3, -1, 0.9]], np.float32)
    sim = _sim(ray_dirs=dirs, rx_pos=[[0, 0.01, 0]])
    rec = O.trace(scene, sim)
    assert list(rec["certified"]) == [False, False, True, True]


# ---------------------------------------------------------------------------------------- passive component

def test_passive_equals_mirror_image_echo():
    """A perfect mirror (k = 1, lobe wide enough to be 1 to 1e-12) makes the traced specular
    echo s -> p -> A equal to the direct (passive) term from s to A's mirror image A':
    same path |A' - s|, same spreading, absorption and phase.  The two go through different
    parts of the oracle (tracing + specular synthesis vs the passive record)."""
    d = 2.0
    scene = wall_scene(d=d)
    A = np.array([0.0, 0.3, 0.1])
    A_img = np.array([2 * d, 0.3, 0.1])
    p_spec = A_img * 0.5                                  # the specular point on x = d
    dirs = (p_spec / np.linalg.norm(p_spec)).reshape(1, 3)
    ones = np.ones((1, 8), np.float32)
    sim = _sim(rx_pos=[A], ray_dirs=dirs, refl_k=ones, lobe_beta=np.full((1, 8), 1e6, np.float32),
               passive_coef=np.ones(8, np.float32))
    rec = O.trace(scene, sim, dirs=dirs.astype(np.float32), certify=False)
    assert len(rec["rtot"]) == 1 and rec["vis"][0] == 1
    H_spec = O.synth(rec, sim)
    sim_img = dict(sim, rx_pos=A_img.reshape(1, 3), x_ref=A_img)
    H_pass = O.synth(O.passive_records(sim_img, [True]), sim_img)
    # the ray direction is FP32: compare against the echo of the traced point itself
    r_traced = rec["rtot"][0] + np.linalg.norm(A - rec["p"][0])
    assert abs(r_traced - np.linalg.norm(A_img)) < 1e-6
    sim_img2 = dict(sim_img, rx_pos=(A_img * r_traced / np.linalg.norm(A_img)).reshape(1, 3))
    H_pass2 = O.synth(O.passive_records(sim_img2, [True]), sim_img2)
    np.testing.assert_allclose(H_pass2, H_spec, rtol=1e-9, atol=1e-12 * np.abs(H_spec).max())
    assert np.abs(H_pass).max() > 0


def test_passive_line_of_sight():
    """The wall blocks the emitter's view of the mirror image behind it, not of a receiver in
    front of it; blocked passive records contribute nothing."""
    scene = wall_scene(d=2.0)
    sim = _sim(rx_pos=[[0.0, 0.3, 0.1], [4.0, 0.3, 0.1]], passive_coef=np.ones(8, np.float32))
    vis, cert = O.passive(scene, sim)
    assert list(vis) == [True, False] and cert.all()
    H = O.synth(O.passive_records(sim, vis), sim)
    assert np.abs(H[0]).min() > 0 and np.abs(H[1]).max() == 0


def test_passive_adjoint_matches_finite_differences():
    """The receiver gradient of the passive term (r = |x_m - s|) by central differences.
    Receivers half a metre from the emitter: at 2.5 cm the 1/r^2 curvature of the direct
    term makes the differences, not the gradient, the inaccurate side."""
    scene, sim = W.tiny_scene(n_rays=24, F=48)
    sim = dict(sim, rx_pos=np.array([[0.3, 0.4, 0.1], [0.2, -0.5, -0.1]]), x_ref=np.array([0.25, -0.05, 0.0]))
    sim["passive_coef"] = np.ascontiguousarray(W.rng(4).uniform(0.2, 1.0, 8).astype(np.float32))
    rec = O.concat_records(O.trace(scene, sim), O.passive_records(sim, [True, True]))
    g = W.rng(5)
    Hstar = O.synth(rec, dict(sim, rx_pos=sim["rx_pos"] + g.normal(0, 1e-3, sim["rx_pos"].shape)))
    H = O.synth(rec, sim)
    _, gx = O.grad(rec, sim, H - Hstar)
    h = 1e-6
    for m in range(2):
        for a in range(3):
            sp = dict(sim); sp["rx_pos"] = sim["rx_pos"].copy(); sp["rx_pos"][m, a] += h
            sm = dict(sim); sm["rx_pos"] = sim["rx_pos"].copy(); sm["rx_pos"][m, a] -= h
            fd = (_loss(rec, sp, Hstar) - _loss(rec, sm, Hstar)) / (2 * h)
            np.testing.assert_allclose(gx[m, a], fd, rtol=1e-5, atol=1e-9 * max(1.0, abs(fd)))


# ---------------------------------------------------------------------------------------- time domain

@pytest.mark.parametrize("sigma", [1, -1])
def test_impulse_response_of_a_pure_delay(sigma):
    """A unit-amplitude path of delay tau has H_k = exp(j sigma 2 pi f_k tau); its impulse
    response is the closed-form geometric series 2 df Re[e^{j s 2pi f_lo x} (1 - e^{j s 2pi F df x})
    / (1 - e^{j s 2pi df x})] with x = tau - t, which peaks at t = tau."""
    sim = _sim(F=256, phase_sign=sigma)
    F, df = 256, (sim["f_hi"] - sim["f_lo"]) / 255
    n_t = 1024
    dt = 1.0 / (n_t * df)
    tau = 137 * dt                                    # on the sample grid
    f = sim["f_lo"] + df * np.arange(F)
    H = np.exp(1j * sigma * 2 * np.pi * f * tau)[None, :]
    h, dt_o = O.impulse_response(H, sim, n_t)
    assert dt_o == pytest.approx(dt, rel=1e-15)
    x = tau - dt * np.arange(n_t)
    num = 1 - np.exp(1j * sigma * 2 * np.pi * F * df * x)
    den = 1 - np.exp(1j * sigma * 2 * np.pi * df * x)
    with np.errstate(invalid="ignore", divide="ignore"):
        geo = np.where(np.abs(den) > 1e-12, num / den, F)
    closed = 2 * df * np.real(np.exp(1j * sigma * 2 * np.pi * sim["f_lo"] * x) * geo)
    np.testing.assert_allclose(h[0], closed, atol=1e-9 * 2 * df * F)
    assert int(np.argmax(h[0])) == 137
    assert h[0, 137] == pytest.approx(2 * df * F, rel=1e-12)


def test_receiver_signal_is_a_convolution():
    """Convolving with a sampled delta returns the impulse response; with a delayed delta,
    the response shifted; and the result is linear in the emitted call."""
    g = W.rng(31)
    h = g.normal(size=(3, 64))
    dt = 1e-6
    d0 = np.zeros(5); d0[0] = 1 / dt
    np.testing.assert_allclose(O.receiver_signal(h, d0, dt)[:, :64], h, rtol=1e-14)
    d2 = np.zeros(5); d2[2] = 1 / dt
    np.testing.assert_allclose(O.receiver_signal(h, d2, dt)[:, 2:66], h, rtol=1e-14)
    a, b = g.normal(size=9), g.normal(size=9)
    np.testing.assert_allclose(O.receiver_signal(h, 2 * a - b, dt),
                               2 * O.receiver_signal(h, a, dt) - O.receiver_signal(h, b, dt), atol=1e-18)


# ----------------------------------------------------------------------------- EQ ray sets (Sec. III-C)

def test_eq_small_sets_closed_forms():
    """EQ(2, N) worked by hand: N = 1 is the boresight; N = 2 the two hemispheres' poles; for
    N = 3, 4, 6 the band between the caps (colatitude acos(1 - 2/N)) is lower than the ideal
    region size sqrt(4 pi / N), so it forms one equatorial collar of N - 2 regions whose
    centres sit at longitudes 2 pi (j + 1/2) / (N - 2)."""
    h = math.sqrt(0.5)
    want = {1: [[1, 0, 0]],
            2: [[1, 0, 0], [-1, 0, 0]],
            3: [[1, 0, 0], [0, -1, 0], [-1, 0, 0]],
            4: [[1, 0, 0], [0, 0, 1], [0, 0, -1], [-1, 0, 0]],
            6: [[1, 0, 0], [0, h, h], [0, -h, h], [0, -h, -h], [0, h, -h], [-1, 0, 0]]}
    for N, w in want.items():
        np.testing.assert_allclose(O.eq_directions(N), np.array(w, float), atol=1e-15)


@pytest.mark.parametrize("N", list(range(1, 400)) + [997, 4096, 65537, 1 << 20])
def test_eq_zones_equal_area_and_carry(N):
    """Every zone's area (from its boundary colatitudes) is its region count times 4 pi / N,
    and each collar boundary's cap differs from the cap of the equal-height grid line by at
    most half a region (the carried rounding)."""
    b, z = O.eq_zones(N)
    assert sum(z) == N and min(z) >= 1 and z[0] == 1 and (N == 1 or z[-1] == 1)
    A = 4 * math.pi / N
    areas = np.array([2 * math.pi * (math.cos(b[k]) - math.cos(b[k + 1])) for k in range(len(z))])
    np.testing.assert_allclose(areas, np.array(z) * A, rtol=1e-8, atol=1e-13)
    if N > 2:
        tc = math.acos(1 - 2 / N)
        n = len(z) - 2
        d = (math.pi - 2 * tc) / n
        for k in range(1, n + 1):   # boundary k closes zone k - 1
            grid = 2 * math.pi * (1 - math.cos(tc + (k - 1) * d))
            cap = 2 * math.pi * (1 - math.cos(b[k]))
            assert abs(cap - grid) / A <= 0.5 + 1e-6


def test_eq_twist_and_order():
    """Twist closed forms; centres ordered by colatitude with a cone keeping a prefix."""
    for n in (1, 2, 7, 40):
        assert O.eq_circle_offset(n, n) == pytest.approx(1 / (2 * n), abs=1e-15)
    assert O.eq_circle_offset(6, 12) == pytest.approx((1 / 12 - 1 / 6) / 2 + 6 / (2 * 72), abs=1e-15)
    D = O.eq_directions(5000)
    assert np.all(np.diff(D[:, 0]) <= 1e-15)
    for a in (0.3, 1.0, 2.5):
        C = O.eq_directions(5000, a)
        k = int(np.sum(D[:, 0] >= math.cos(a) - 1e-12))
        assert len(C) == k and np.array_equal(C, D[:k])
    np.testing.assert_allclose(np.linalg.norm(D, axis=1), 1.0, atol=1e-15)


@pytest.mark.parametrize("N", [2000, 20000])
def test_eq_cap_discrepancy(N):
    """Equal-area regions make every spherical cap hold its share of centres to
    O(N^-1/2) with a small constant (seeded random caps: <= 0.35 / sqrt(N); seeded random
    point sets reach about 1 / sqrt(N))."""
    D = O.eq_directions(N)
    g = np.random.default_rng(5)
    worst = 0.0
    for _ in range(300):
        ax = g.normal(size=3)
        ax /= np.linalg.norm(ax)
        a = g.uniform(0.05, math.pi - 0.05)
        share = float(np.sum(D @ ax >= math.cos(a))) / N
        worst = max(worst, abs(share - (1 - math.cos(a)) / 2))
    assert worst <= 0.35 / math.sqrt(N)


# ----------------------------------------------------------------------------- alternative readings

def test_path_product_between_parallel_walls():
    """Path-product reading of the reflection magnitude: a ray bouncing along x between the
    walls x = 10 (material 1, hit first) and x = 0 (material 0) carries, at its n-th record,
    k1^ceil(n/2) k0^floor(n/2) times the literal value (k of the hit triangle only)."""
    mb = W.MeshBuilder()
    v, t = W.quad_grid_box([0, 0, 0], [10.0, 8.0, 3.0], 1)
    xs = v[t].mean(axis=1)[:, 0]
    for tri, xc in zip(t, xs):   # one object per triangle: material by the wall it lies on
        mb.add(v[tri], np.array([[0, 1, 2]]), 1 if abs(xc - 10.0) < 1e-9 else 0)
    scene = mb.build()
    k0, k1 = 0.8, 0.55
    sim = _sim(emitter_pos=[5.0, 4.3, 1.1], x_ref=[5.0, 4.3, 1.1], rx_pos=[[4.0, 4.3, 1.1]],
               ray_dirs=[[1, 0, 0]], max_bounces=6, F=64,
               refl_k=np.array([[k0] * 8, [k1] * 8]), lobe_beta=np.full((2, 8), 1e6),
               diff_coef=np.full((2, 8), 0.1))
    rec = O.trace(scene, sim)
    assert len(rec["rtot"]) == 6 and list(rec["mat"]) == [1, 0, 1, 0, 1, 0]
    for i in range(6):
        one = {k: v[i:i + 1] for k, v in rec.items() if k not in ("certified", "nseg")}
        one["vis"] = np.ones(1, np.uint8)
        lit = O.synth(one, sim)
        pp = O.synth(one, dict(sim, path_product=True))
        # a single record alone has no earlier reflections of its ray in the list: literal value
        np.testing.assert_allclose(pp, lit, rtol=1e-13)
    full = {k: v for k, v in rec.items() if k not in ("certified", "nseg")}
    full["vis"] = np.ones(6, np.uint8)
    for n in range(6):
        # spectra of the first n + 1 records minus the first n: record n alone, in context
        def part(s, upto):
            sub = {k: v[:upto] for k, v in full.items()}
            return O.synth(sub, s) if upto else 0
        lit_n = part(sim, n + 1) - part(sim, n)
        pp_n = part(dict(sim, path_product=True), n + 1) - part(dict(sim, path_product=True), n)
        kf0, kf1 = float(np.float32(k0)), float(np.float32(k1))   # the tables are FP32
        want = kf1 ** math.ceil(n / 2) * kf0 ** (n // 2)
        np.testing.assert_allclose(pp_n, want * lit_n, rtol=1e-10, atol=1e-18)


def test_per_receiver_visibility_equals_reference_point_tests():
    """Per-receiver line of sight: bit m of a record equals the reference-point test with
    x_ref placed at receiver m; a screen in front of one receiver makes the bits differ, and the
    spectrum of receiver m uses exactly the records its bit admits."""
    mb = W.MeshBuilder()
    mb.add(np.array([[4, -3, -2], [4, 3, -2], [4, 3, 2], [4, -3, 2]], float), np.array([[0, 1, 2], [0, 2, 3]]), 0)
    mb.add(np.array([[1.5, 0.05, -0.6], [1.5, 0.8, -0.6], [1.5, 0.8, 0.6], [1.5, 0.05, 0.6]], float),
           np.array([[0, 1, 2], [0, 2, 3]]), 0)
    scene = mb.build()
    g = W.rng(4)
    rx = np.array([[0.0, 0.3, 0.0], [0.0, -0.3, 0.0]])
    sim = _sim(emitter_pos=[0, 0, 0], rx_pos=rx, ray_dirs=W.cone_directions(g, 4000, math.radians(30)),
               max_bounces=2, F=64, refl_k=np.full((1, 8), 0.9), lobe_beta=np.full((1, 8), 0.3),
               diff_coef=np.full((1, 8), 0.1), per_rx_visibility=True)
    per = O.trace(scene, sim)
    bits = per["rxvis"]
    for m in range(2):
        lit = O.trace(scene, dict(sim, per_rx_visibility=False, x_ref=rx[m]))
        assert np.array_equal(lit["ray"], per["ray"]) and np.array_equal(lit["bounce"], per["bounce"])
        assert np.array_equal(((bits >> np.uint64(m)) & np.uint64(1)).astype(np.uint8), lit["vis"])
        H_per = O.synth(per, sim, M_subset=[m])
        H_lit = O.synth(lit, dict(sim, per_rx_visibility=False), M_subset=[m])
        np.testing.assert_allclose(H_per, H_lit, rtol=1e-12, atol=1e-20)
    b0, b1 = bits & np.uint64(1), (bits >> np.uint64(1)) & np.uint64(1)
    assert np.any(b0 != b1)
    assert np.array_equal(per["vis"], ((b0 | b1) > 0).astype(np.uint8))
