"""FP64 CPU oracle for the echo-simulation hot path (ctypes wrapper over oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by tests/, the smoke check and the CPU-baseline leg
of the benchmark; the product library never imports it and shares no code with it.
The C source is plain brute force in IEEE double (see oracle.c); this module only
marshals numpy arrays.

Pins (tests/test_oracle_*.py): single-wall image source, box-room unfolding, reciprocity
of the single-point path, the sphere and flat-plane curvature values, the SplitMix64
published outputs, chi-square of the diffraction sampler, finite differences of the
adjoint.  Parts with no external pin ("parity unpinned"): the area weighting w(A) and
scale eta of the curvature metric, the eligibility threshold tau, the dither of the
CDF, the visibility target x_ref, the air-absorption constants.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

KAPPA = 32.0      # margin bound in units of FP32 unit roundoff (2^-24)
MU_G = 1e-3       # grazing threshold on |d . n| at an accepted hit


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB_PATH)
        _lib.orc_splitmix.restype = C.c_uint64
        _lib.orc_splitmix.argtypes = [C.c_uint64, C.c_uint64]
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def trace(scene: dict, sim: dict, dirs=None, certify: bool = True, kappa: float = KAPPA, mu_g: float = MU_G) -> dict:
    """Algorithm 1 by brute force in FP64.  Returns records in (ray, bounce) order plus the
    per-ray certification flag and closest-hit segment count."""
    L = lib()
    dirs = _f32(sim["ray_dirs"] if dirs is None else dirs)
    N = len(dirs)
    B = int(sim["max_bounces"])
    cap = max(1, N * B)
    out = {
        "ray": np.zeros(cap, np.int32), "bounce": np.zeros(cap, np.int32), "tri": np.zeros(cap, np.int32),
        "mat": np.zeros(cap, np.int32), "p": np.zeros((cap, 3)), "din": np.zeros((cap, 3)),
        "dout": np.zeros((cap, 3)), "rtot": np.zeros(cap), "vis": np.zeros(cap, np.uint8),
    }
    cert = np.zeros(max(N, 1), np.uint8)
    nseg = np.zeros(max(N, 1), np.int32)
    n = C.c_int64(0)
    v = _f32(scene["vertices"]); t = _i32(scene["tris"]); m = _i32(scene["tri_material"])
    ep = _f64(sim["emitter_pos"]); er = _f64(sim["emitter_rot"]); xr = _f64(sim["x_ref"])
    per_rx = bool(sim.get("per_rx_visibility", False))
    rx = _f64(sim["rx_pos"])
    rxvis = np.zeros(cap, np.uint64) if per_rx else None
    rc = L.orc_trace(C.c_int64(len(v)), C.c_int64(len(t)), _p(v), _p(t), _p(m), _p(ep), _p(er), C.c_int64(N), _p(dirs),
                     C.c_int32(B), C.c_double(sim["max_distance"]), _p(xr), C.c_double(sim["t_eps"]),
                     C.c_double(kappa if certify else 0.0), C.c_double(mu_g), C.c_int64(cap), C.byref(n),
                     _p(out["ray"]), _p(out["bounce"]), _p(out["tri"]), _p(out["mat"]), _p(out["p"]), _p(out["din"]),
                     _p(out["dout"]), _p(out["rtot"]), _p(out["vis"]), _p(cert), _p(nseg),
                     C.c_int32(len(rx)), _p(rx), _p(rxvis))
    if rc != 0:
        raise ValueError(f"orc_trace failed ({rc})")
    k = n.value
    res = {key: val[:k].copy() for key, val in out.items()}
    if per_rx:
        res["rxvis"] = rxvis[:k].copy()
    res["kind"] = np.zeros(k, np.uint8)
    res["certified"] = cert[:N].astype(bool)
    res["nseg"] = nseg[:N].copy()
    return res


def synth(rec: dict, sim: dict, bins=None, M_subset=None) -> np.ndarray:
    """Eqs. (2)-(4) and (7)-(8): complex spectra [M, nk] (complex128) by direct summation.
    `bins` selects frequency indices (default all F); `M_subset` selects receivers.
    sim["per_rx_visibility"]: per-receiver line of sight from rec["rxvis"] (bit m: receiver
    m); sim["path_product"]: specular magnitudes as the product of k over the ray's
    reflections so far (rec["ray"], rec["bounce"])."""
    L = lib()
    F = int(sim["F"])
    k_list = np.arange(F, dtype=np.int32) if bins is None else _i32(bins)
    rx = _f64(sim["rx_pos"]); rr = _f64(sim["rx_rot"])
    D = sim.get("directivity")
    rx_id = np.arange(len(rx), dtype=np.int32)
    if M_subset is not None:
        rx_id = _i32(rx_id[M_subset])
        rx = _f64(rx[M_subset]); rr = _f64(rr[M_subset])
        if D is not None:
            D = D[M_subset]
    M = len(rx)
    Bd = El = Az = 0
    if D is not None:
        D = _f32(D)
        _, Bd, El, Az = D.shape
    n = len(rec["rtot"])
    p = _f64(rec["p"]) if n else np.zeros((1, 3))
    dout = _f64(rec.get("dout", np.zeros((n, 3)))) if n else np.zeros((1, 3))
    rt = _f64(rec["rtot"]) if n else np.zeros(1)
    mat = _i32(rec["mat"]) if n else np.zeros(1, np.int32)
    kind = np.ascontiguousarray(rec.get("kind", np.zeros(n, np.uint8)), np.uint8) if n else np.zeros(1, np.uint8)
    vis = np.ascontiguousarray(rec.get("vis", np.ones(n, np.uint8)), np.uint8) if n else np.zeros(1, np.uint8)
    k = _f32(sim["refl_k"]); b = _f32(sim["lobe_beta"]); dc = _f32(sim["diff_coef"])
    Q, Bk = k.shape
    pc = sim.get("passive_coef")
    pc = None if pc is None else _f32(pc)
    rxvis = None
    if sim.get("per_rx_visibility", False):
        rxvis = np.ascontiguousarray(rec["rxvis"], np.uint64) if n else np.zeros(1, np.uint64)
    pp = bool(sim.get("path_product", False))
    rray = _i32(rec["ray"]) if (pp and n) else (np.zeros(1, np.int32) if pp else None)
    rbnc = _i32(rec["bounce"]) if (pp and n) else (np.zeros(1, np.int32) if pp else None)
    out = np.zeros((M, len(k_list), 2))
    rc = L.orc_synth(C.c_int64(n), _p(p), _p(dout), _p(rt), _p(mat), _p(kind), _p(vis), C.c_int32(M), _p(rx), _p(rr),
                     C.c_double(sim["f_lo"]), C.c_double(sim["f_hi"]), C.c_int32(F), C.c_int32(len(k_list)), _p(k_list),
                     C.c_double(sim["c"]), C.c_double(sim["atm_a0"]), C.c_double(sim["atm_a1"]),
                     C.c_double(sim["spreading_p"]), C.c_int32(sim["phase_sign"]), C.c_int32(Q), C.c_int32(Bk),
                     _p(k), _p(b), _p(dc), C.c_int32(Bd), C.c_int32(El), C.c_int32(Az), _p(D), _p(pc), _p(rx_id),
                     _p(out), _p(rxvis), _p(rray), _p(rbnc), C.c_int(int(pp)))
    if rc != 0:
        raise ValueError(f"orc_synth failed ({rc})")
    return out[..., 0] + 1j * out[..., 1]


def grad(rec: dict, sim: dict, g: np.ndarray):
    """Analytic gradient of L = sum |H - H*|^2 with g = H - H* (complex [M, F]):
    returns (dL/d refl_k [Q, Bk], dL/d rx_pos [M, 3])."""
    L = lib()
    if sim.get("path_product", False):
        raise ValueError("gradient with the path-product reading is not defined here")
    F = int(sim["F"])
    rx = _f64(sim["rx_pos"]); rr = _f64(sim["rx_rot"])
    M = len(rx)
    n = len(rec["rtot"])
    D = sim.get("directivity")
    Bd = El = Az = 0
    if D is not None:
        D = _f32(D)
        _, Bd, El, Az = D.shape
    gg = np.ascontiguousarray(np.stack([g.real, g.imag], -1), np.float64)
    k = _f32(sim["refl_k"]); b = _f32(sim["lobe_beta"]); dc = _f32(sim["diff_coef"])
    Q, Bk = k.shape
    gk = np.zeros((Q, Bk)); gx = np.zeros((M, 3))
    kind = np.ascontiguousarray(rec.get("kind", np.zeros(n, np.uint8)), np.uint8)
    vis = np.ascontiguousarray(rec.get("vis", np.ones(n, np.uint8)), np.uint8)
    pc = sim.get("passive_coef")
    pc = None if pc is None else _f32(pc)
    rxvis = np.ascontiguousarray(rec["rxvis"], np.uint64) if sim.get("per_rx_visibility", False) else None
    rc = L.orc_grad(C.c_int64(n), _p(_f64(rec["p"])), _p(_f64(rec["dout"])), _p(_f64(rec["rtot"])), _p(_i32(rec["mat"])),
                    _p(kind), _p(vis), C.c_int32(M), _p(rx), C.c_double(sim["f_lo"]), C.c_double(sim["f_hi"]),
                    C.c_int32(F), C.c_double(sim["c"]), C.c_double(sim["atm_a0"]), C.c_double(sim["atm_a1"]),
                    C.c_double(sim["spreading_p"]), C.c_int32(sim["phase_sign"]), C.c_int32(Q), C.c_int32(Bk),
                    _p(k), _p(b), _p(dc), _p(pc), _p(gg), _p(gk), _p(gx), _p(rxvis), _p(rr), C.c_int32(Bd),
                    C.c_int32(El), C.c_int32(Az), _p(D))
    if rc != 0:
        raise ValueError(f"orc_grad failed ({rc})")
    return gk, gx


def curvature(scene: dict, a_ref: float):
    """Eq. (1): per-vertex G_v and per-triangle C_i (FP64)."""
    L = lib()
    v = _f32(scene["vertices"]); t = _i32(scene["tris"])
    G = np.zeros(len(v)); Ci = np.zeros(len(t))
    rc = L.orc_curvature(C.c_int64(len(v)), C.c_int64(len(t)), _p(v), _p(t), C.c_double(a_ref), _p(G), _p(Ci))
    if rc != 0:
        raise ValueError("orc_curvature failed")
    return G, Ci


def splitmix(key: int, counter: int) -> int:
    return int(lib().orc_splitmix(C.c_uint64(key), C.c_uint64(counter)))


def diffraction(scene: dict, sim: dict, Ci: np.ndarray, certify: bool = True, kappa: float = KAPPA) -> dict:
    """Section III-D sampler: K candidates drawn from the dithered integer CDF of C_i,
    filtered by incidence angle and line of sight to the emitter.  With sim["diff_per_mesh"]
    every mesh (object) with eligible triangles gets its own K candidates from its own CDF
    (at most sim["diff_max_meshes"] meshes, in increasing object order)."""
    L = lib()
    v = _f32(scene["vertices"]); t = _i32(scene["tris"]); o = _i32(scene["tri_object"])
    K = int(sim["diff_K"])
    per_mesh = bool(sim.get("diff_per_mesh", False))
    mm = int(sim.get("diff_max_meshes", 1)) if per_mesh else 1
    cap = max(K * mm, 1)
    T = len(t)
    q = np.zeros(max(T, 1), np.uint64)
    ne = C.c_int64(0)
    ns = C.c_int64(0)
    st = np.zeros(cap, np.int32); so = np.zeros((cap, 3)); sr = np.zeros(cap)
    sk = np.zeros(cap, np.uint8); sc = np.zeros(cap, np.uint8)
    Ci = _f64(Ci)
    rc = L.orc_diffraction(C.c_int64(len(v)), C.c_int64(T), _p(v), _p(t), _p(o), C.c_int32(int(scene["n_objects"])),
                           _p(Ci), _p(_f64(sim["emitter_pos"])), _p(_f64(sim["emitter_rot"])),
                           C.c_double(math.radians(sim["diff_cone_half_angle_deg"])), C.c_double(sim["diff_tau"]),
                           C.c_uint64(sim["diff_seed"]), C.c_int64(K),
                           C.c_double(math.radians(sim["diff_max_incidence_deg"])), C.c_double(sim["t_eps"]),
                           C.c_double(kappa if certify else 0.0), C.c_int(int(per_mesh)), C.c_int64(mm), _p(q),
                           C.byref(ne), C.byref(ns), _p(st), _p(so), _p(sr), _p(sk), _p(sc))
    if rc < 0:
        raise ValueError("orc_diffraction failed")
    n = ns.value
    return {"q": q[:T], "n_elig": ne.value, "tri": st[:n], "o": so[:n], "r_src": sr[:n], "keep": sk[:n].astype(bool),
            "certified": sc[:n].astype(bool), "truncated": rc == 1}


def diffraction_records(scene: dict, samples: dict) -> dict:
    """Kept diffraction samples as synthesis records (kind 1: omnidirectional secondary source)."""
    keep = samples["keep"]
    tri = samples["tri"][keep]
    n = int(keep.sum())
    return {"p": samples["o"][keep].copy(), "dout": np.zeros((n, 3)), "rtot": samples["r_src"][keep].copy(),
            "mat": scene["tri_material"][tri].astype(np.int32), "kind": np.ones(n, np.uint8),
            "vis": np.ones(n, np.uint8), "tri": tri.astype(np.int32)}


def passive(scene: dict, sim: dict, certify: bool = True, kappa: float = KAPPA):
    """Passive component: line of sight from the emitter to every receiver (vis[M]) and the
    certification of each decision against FP32 traversal."""
    L = lib()
    v = _f32(scene["vertices"]); t = _i32(scene["tris"])
    rx = _f64(sim["rx_pos"])
    M = len(rx)
    vis = np.zeros(max(M, 1), np.uint8); cert = np.zeros(max(M, 1), np.uint8)
    rc = L.orc_passive(C.c_int64(len(v)), C.c_int64(len(t)), _p(v), _p(t), _p(_f64(sim["emitter_pos"])), C.c_int32(M),
                       _p(rx), C.c_double(sim["t_eps"]), C.c_double(kappa if certify else 0.0), _p(vis), _p(cert))
    if rc != 0:
        raise ValueError("orc_passive failed")
    return vis[:M].astype(bool), cert[:M].astype(bool)


def passive_records(sim: dict, vis) -> dict:
    """One passive record per receiver m: the emitter as the point, path 0 so far, the
    receiver index in the material field, kind 2."""
    M = len(sim["rx_pos"])
    s = np.asarray(sim["emitter_pos"], np.float64).reshape(1, 3)
    return {"p": np.repeat(s, M, axis=0), "dout": np.zeros((M, 3)), "rtot": np.zeros(M),
            "mat": np.arange(M, dtype=np.int32), "kind": np.full(M, 2, np.uint8),
            "vis": np.asarray(vis, np.uint8), "tri": np.full(M, -1, np.int32)}


def concat_records(a: dict, b: dict) -> dict:
    keys = ["p", "dout", "rtot", "mat", "kind", "vis"]
    return {k: np.concatenate([np.asarray(a[k]), np.asarray(b[k])]) for k in keys}


# ------------------------------------------------------------------ time domain

def impulse_response(H: np.ndarray, sim: dict, n_t: int):
    """Impulse response per receiver from its spectrum on the grid f_k = f_lo + k df (Eqs. 5-6,
    9-10, 13: h = F^-1[H]).  Under the e^{-i omega t} convention of the phase (sigma = +1), a
    delay e^{+j sigma omega tau} becomes a peak at t = tau:
        h(t) = 2 df Re sum_k H_k exp(-j sigma 2 pi f_k t),   t_n = n / (n_t df), n < n_t,
    the real signal of the one-sided band spectrum.  The sum over k is a length-n_t DFT of the
    zero-padded spectrum (numpy's FFT as the step), times the carrier exp(-j sigma 2 pi f_lo t).
    Returns (h [M, n_t] float64, dt)."""
    H = np.asarray(H, np.complex128)
    M, F = H.shape
    if n_t < F:
        raise ValueError("n_t must be >= F")
    sigma = int(sim["phase_sign"])
    df = (sim["f_hi"] - sim["f_lo"]) / (F - 1) if F > 1 else 0.0
    dt = 1.0 / (n_t * df)
    pad = np.zeros((M, n_t), np.complex128)
    pad[:, :F] = H
    S = np.fft.fft(pad, axis=1) if sigma > 0 else np.fft.ifft(pad, axis=1) * n_t
    n = np.arange(n_t)
    cyc = sim["f_lo"] * n * dt                     # carrier phase in cycles, reduced before the exponential
    carrier = np.exp(-1j * sigma * 2.0 * np.pi * (cyc - np.floor(cyc)))
    return 2.0 * df * np.real(carrier[None, :] * S), dt


def receiver_signal(h: np.ndarray, s_e: np.ndarray, dt: float) -> np.ndarray:
    """Eq. 14: s(t) = (h * s_e)(t), sampled: s[n] = dt sum_k h[k] s_e[n - k], length
    n_t + L - 1 (direct summation)."""
    h = np.asarray(h, np.float64)
    s_e = np.asarray(s_e, np.float64)
    return dt * np.stack([np.convolve(row, s_e) for row in np.atleast_2d(h)])


# ------------------------------------------------------------------ EQ sphere partition (ray set)

def _cap_area(theta: float) -> float:
    """Area of the spherical cap of angular radius theta on the unit sphere."""
    return 2.0 * math.pi * (1.0 - math.cos(theta))


def _cap_angle(area: float) -> float:
    """Angular radius of the cap of the given area (inverse of _cap_area)."""
    return 2.0 * math.asin(min(1.0, math.sqrt(area / (4.0 * math.pi))))


def _round(x: float, N: int) -> int:
    """Nearest integer to x >= 0, with halves rounded down.  A collar boundary on the equator
    has an ideal cumulative count of exactly (N - 2) / 2, a half for odd N, which floating
    point lands on either side of: values within N * 2^-36 above a half count as the half, so
    that every evaluation order rounds them the same way."""
    return int(math.floor(x + 0.5 - N * 2.0 ** -36))


def eq_zones(N: int):
    """Recursive zonal equal-area partition EQ(2, N) of the unit sphere (Leopardi 2006; the
    ray set of Sec. III-C).  Returns (zone boundaries theta_0 = 0 < ... < theta_Z = pi,
    regions per zone) from the north cap to the south cap.  Steps: two polar caps of the
    region area A = 4 pi / N; the band between them is cut into n collars of equal angular
    height, n the rounded ratio of the band's height to the ideal region size sqrt(A); each
    collar's ideal region count (its area over A) is rounded in order with the rounding error
    carried into the next collar; the zone boundaries are then placed so that every zone's
    area is exactly its region count times A."""
    if N < 1:
        raise ValueError("N must be >= 1")
    if N > 1 << 28:
        raise ValueError("N must be <= 2^28")
    if N == 1:
        return [0.0, math.pi], [1]
    A = 4.0 * math.pi / N
    theta_c = _cap_angle(A)
    if N == 2:
        return [0.0, theta_c, math.pi], [1, 1]
    delta_i = math.sqrt(A)
    n = max(1, _round((math.pi - 2.0 * theta_c) / delta_i, N))
    delta_f = (math.pi - 2.0 * theta_c) / n
    counts = []
    carry = 0.0
    for i in range(1, n + 1):
        ideal = (_cap_area(theta_c + i * delta_f) - _cap_area(theta_c + (i - 1) * delta_f)) / A
        m = _round(ideal + carry, N)
        carry += ideal - m
        counts.append(m)
    zones = [1] + counts + [1]
    bounds = [0.0]
    acc = 0
    for m in zones[:-1]:
        acc += m
        bounds.append(_cap_angle(acc * A))
    bounds.append(math.pi)
    return bounds, zones


def eq_circle_offset(n_top: int, n_bot: int) -> float:
    """Rotation (in turns) of a collar of n_bot regions against the collar of n_top regions
    above it that keeps the region centres of the two collars apart (Leopardi's twist)."""
    return (1.0 / n_bot - 1.0 / n_top) / 2.0 + math.gcd(n_top, n_bot) / (2.0 * n_top * n_bot)


def eq_directions(N: int, cone_half_angle: float = math.pi) -> np.ndarray:
    """Centres of the regions of EQ(2, N) as unit vectors about the boresight +x:
    (cos t, sin t cos p, sin t sin p) with t the colatitude.  Order: north cap, then every
    collar by increasing longitude, then the south cap.  A collar's centres sit at the
    middle colatitude of the collar and at longitudes 2 pi ((j + 1/2) / m + offset), the
    offset of the first collar 0 and each next one turned by eq_circle_offset.  Only the
    centres with colatitude <= cone_half_angle are returned (a prefix of the order)."""
    bounds, zones = eq_zones(N)
    thetas, phis = [0.0], [0.0]
    offset = 0.0
    Z = len(zones)
    for z in range(1, Z):
        m = zones[z]
        if z == Z - 1:
            thetas.append(math.pi)
            phis.append(0.0)
            break
        t = 0.5 * (bounds[z] + bounds[z + 1])
        for j in range(m):
            thetas.append(t)
            phis.append(2.0 * math.pi * (((j + 0.5) / m + offset) % 1.0))
        if z + 1 < Z - 1:
            offset = (offset + eq_circle_offset(m, zones[z + 1])) % 1.0
    th = np.array(thetas)
    ph = np.array(phis)
    keep = th <= cone_half_angle
    th, ph = th[keep], ph[keep]
    return np.stack([np.cos(th), np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph)], axis=1)
