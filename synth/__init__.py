"""Seeded synthetic inputs for the template-bank search (shared by tests and bench).

This module holds none of the search's arithmetic: it draws noise, builds
segment times, detector velocities, sky vectors, weights and template grids.
Injected tracks are added by the caller from bins computed elsewhere (the
CPU oracle in tests, the library's own injection call in the benchmark).

Workloads stand in for the paper's data (8-s Hann-windowed SFTs of 24 h in
Gaussian noise, Sec. 2-3): under Gaussian noise the normalised power of a
pixel is Exp(1), so spectrograms are Exp(1) draws in FP64 rounded to FP32,
with additive power along injected tracks.  The detector velocity replaces a
solar-system ephemeris by a circular orbit plus diurnal rotation.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0
V_ORBIT = 29.8e3           # m/s, mean orbital speed of the Earth
P_ORBIT = 3.156e7          # s, one year
V_ROT_EQ = 0.465e3         # m/s, equatorial rotation speed
P_SIDEREAL = 86164.0       # s, sidereal day
OBLIQUITY = math.radians(23.4393)

# detector sites (latitude, longitude) in degrees
SITE_H = (46.455, -119.408)
SITE_L = (30.563, -90.774)


# azimuth of the first arm in degrees east of north (the second is 90 degrees
# further east), approximately those of the two LIGO sites
ARM_AZ_H = 324.0
ARM_AZ_L = 252.3


def earth_rotation_angle(t):
    """Rotation angle of the Earth-fixed frame about z at times t (rad): the
    same rotation that carries the site in `velocity` (longitude 0 on the
    equatorial x axis at t = 0)."""
    return 2.0 * np.pi * np.asarray(t, dtype=np.float64) / P_SIDEREAL


def site_arms(lat_deg, lon_deg, azimuth_deg, opening_deg=90.0):
    """Unit vectors [2][3] of the two arms of a detector at a site, in the
    Earth-fixed frame (z on the rotation axis, x at longitude 0): the first
    arm at `azimuth_deg` east of north in the local horizontal plane, the
    second `opening_deg` further east."""
    la, lo = math.radians(lat_deg), math.radians(lon_deg)
    north = np.array([-math.sin(la) * math.cos(lo), -math.sin(la) * math.sin(lo), math.cos(la)])
    east = np.array([-math.sin(lo), math.cos(lo), 0.0])
    out = []
    for az in (azimuth_deg, azimuth_deg + opening_deg):
        a = math.radians(az)
        v = math.cos(a) * north + math.sin(a) * east
        out.append(v / np.linalg.norm(v))
    return np.ascontiguousarray(out)


def exp_noise(n_seg, n_bins, seed):
    """FP32 Exp(1) spectrogram by inverse CDF in FP64 (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((n_seg, n_bins))          # [0, 1)
    x = -np.log1p(-u)                        # -ln(1 - u), u in [0,1) -> (0, inf)
    return x.astype(np.float32)


def segment_times(n_seg, t_sft, t_start=0.0):
    """Segment mid-times t_j = t_start + (j + 1/2) T_sft."""
    return t_start + (np.arange(n_seg, dtype=np.float64) + 0.5) * float(t_sft)


def velocity(t, lat_deg=0.0, lon_deg=0.0):
    """Detector velocity [n, 3] in m/s, equatorial frame: circular orbit plus rotation."""
    t = np.asarray(t, dtype=np.float64)
    phi = 2.0 * np.pi * t / P_ORBIT
    v_orb = V_ORBIT * np.stack([-np.sin(phi), np.cos(phi) * math.cos(OBLIQUITY),
                                np.cos(phi) * math.sin(OBLIQUITY)], axis=-1)
    psi = 2.0 * np.pi * t / P_SIDEREAL + math.radians(lon_deg)
    vr = V_ROT_EQ * math.cos(math.radians(lat_deg))
    v_rot = vr * np.stack([-np.sin(psi), np.cos(psi), np.zeros_like(psi)], axis=-1)
    return np.ascontiguousarray(v_orb + v_rot)


def sky_vector(alpha, delta):
    """Unit vector (cos d cos a, cos d sin a, sin d) for right ascension a, declination d."""
    return np.array([math.cos(delta) * math.cos(alpha), math.cos(delta) * math.sin(alpha),
                     math.sin(delta)], dtype=np.float64)


def fibonacci_cap(n, center, half_angle_rad):
    """n quasi-uniform unit vectors in a spherical cap around `center` (Fibonacci lattice)."""
    golden = (1.0 + 5.0 ** 0.5) / 2.0
    i = np.arange(n, dtype=np.float64)
    cos_min = math.cos(half_angle_rad)
    z = 1.0 - (1.0 - cos_min) * (i + 0.5) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    ph = 2.0 * np.pi * i / golden
    pts = np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=-1)
    c = np.asarray(center, dtype=np.float64)
    c = c / np.linalg.norm(c)
    # rotate +z onto c (Rodrigues)
    zax = np.array([0.0, 0.0, 1.0])
    ax = np.cross(zax, c)
    s = np.linalg.norm(ax)
    if s < 1e-15:
        out = pts if c[2] > 0 else pts * np.array([1.0, 1.0, -1.0])
    else:
        ax = ax / s
        cth = float(np.dot(zax, c))
        K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        R = np.eye(3) + s * K + (1 - cth) * (K @ K)
        out = pts @ R.T
    return out / np.linalg.norm(out, axis=1, keepdims=True)


class Workload:
    """A detector set plus a lattice grid and injection list (numpy arrays only)."""

    def __init__(self, name, dets, grid, injections, rho_th=1.6):
        self.name = name
        self.dets = dets            # list of dicts: rho, t_seg, v, k_lo, t_sft, weights
        self.grid = grid            # dict: f0_min, f0_step, n_f0, tau, brake, sky, t0
        self.injections = injections  # list of dicts: f0, tau, brake, sky, amp
        self.rho_th = np.float32(rho_th)

    @property
    def n_templates(self):
        g = self.grid
        return g["n_f0"] * len(g["tau"]) * len(g["brake"]) * len(g["sky"])

    @property
    def n_evals(self):
        return self.n_templates * sum(d["rho"].shape[0] for d in self.dets)


def tiny(seed=1, with_noise=True):
    """The small workload: one detector, T_obs = 4096 s in 1024 segments of 4 s,
    400-600 Hz at 0.25 Hz (800 bins, k_lo = 1600), FP32 Exp(1) power, one
    injection (f0 = 550, tau = 7000, n = 5, +4.0), one sky point
    (alpha, delta) = (1.0, 0.3); grid f0 500-600 step 0.25 (400) x tau
    {3500, 7000, 14000, 35000} x n {3, 5, 7} = 4800 templates."""
    n_seg, n_bins, t_sft, k_lo = 1024, 800, 4.0, 1600
    rho = exp_noise(n_seg, n_bins, seed) if with_noise else np.zeros((n_seg, n_bins), np.float32)
    t_seg = segment_times(n_seg, t_sft)
    det = dict(rho=rho, t_seg=t_seg, v=velocity(t_seg, 0.0, 0.0), k_lo=k_lo, t_sft=t_sft,
               weights=None)
    sky = sky_vector(1.0, 0.3)[None, :]
    grid = dict(f0_min=500.0, f0_step=0.25, n_f0=400,
                tau=np.array([3500.0, 7000.0, 14000.0, 35000.0]),
                brake=np.array([3.0, 5.0, 7.0]), sky=sky, t0=0.0)
    inj = [dict(f0=550.0, tau=7000.0, brake=5.0, sky=sky[0], amp=4.0)]
    return Workload("tiny-1024seg-800bin-4800tpl", [det], grid, inj)


def realistic(seed=2, weight_seed=3, inj_seed=4, n_seg=10800, n_bins=8000, n_f0=8000):
    """The realistic single search: T_obs = 86400 s in 10800 segments of 8 s,
    500-1500 Hz at 0.125 Hz (8000 bins, k_lo = 4000), FP32 Exp(1) power,
    per-segment noise-floor weights U[0.5, 2], 20 injections with amplitude
    U[0.5, 3] (times w_j), off-grid parameters; grid f0 = 500 + 0.125 i
    (8000) x tau geomspace(3500, 35000, 32) x n linspace(3, 7, 9) x 1 sky.
    Smaller n_seg / n_bins / n_f0 give the same recipe at reduced size."""
    t_sft, k_lo = 8.0, 4000
    rho = exp_noise(n_seg, n_bins, seed)
    w = np.random.Generator(np.random.PCG64(weight_seed)).uniform(0.5, 2.0, n_seg).astype(np.float32)
    t_seg = segment_times(n_seg, t_sft)
    det = dict(rho=rho, t_seg=t_seg, v=velocity(t_seg, 0.0, 0.0), k_lo=k_lo, t_sft=t_sft,
               weights=w)
    sky = sky_vector(1.0, 0.3)[None, :]
    grid = dict(f0_min=500.0, f0_step=0.125, n_f0=n_f0,
                tau=np.geomspace(3500.0, 35000.0, 32), brake=np.linspace(3.0, 7.0, 9),
                sky=sky, t0=0.0)
    r = np.random.Generator(np.random.PCG64(inj_seed))
    f_hi = 500.0 + (n_bins - 1) * 0.125
    inj = []
    for _ in range(20):
        amp = r.uniform(0.5, 3.0)
        f0 = r.uniform(500.0, f_hi)
        tau = math.exp(r.uniform(math.log(3500.0), math.log(35000.0)))
        brake = r.uniform(3.0, 7.0)
        inj.append(dict(f0=f0, tau=tau, brake=brake, sky=sky[0], amp=amp))
    return Workload(f"realistic-{n_seg}seg-{n_bins}bin-{grid['n_f0'] * 288}tpl", [det], grid, inj)


def batch_searches(seed=5, n_searches=64, t_sft=8.0):
    """The batch of uneven searches: T_obs ~ U[2 h, 48 h] (whole segments of
    8 s), band width ~ U[100, 1000] Hz placed in 500-3000 Hz on the 0.125-Hz
    grid, two detectors (the H and L site rotations), a sky patch of N_sky ~
    log-uniform integer [16, 1024] Fibonacci points in a 10-degree cap around a
    random centre, and a lattice of f0 at every bin of the band x tau {3500,
    7000, 14000, 35000} x n {3, 5, 7} from the data start.  Returns a list of
    dicts (geometry and grid; the power itself is generated on the device)."""
    r = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_searches):
        t_obs = r.uniform(2 * 3600.0, 48 * 3600.0)
        n_seg = max(1, int(round(t_obs / t_sft)))
        width = r.uniform(100.0, 1000.0)
        n_bins = int(round(width / 0.125))
        f_lo = 500.0 + 0.125 * int(r.integers(0, int((3000.0 - 500.0 - n_bins * 0.125) / 0.125) + 1))
        k_lo = int(round(f_lo * t_sft))
        n_sky = int(round(math.exp(r.uniform(math.log(16.0), math.log(1024.0)))))
        centre = sky_vector(r.uniform(0.0, 2.0 * math.pi), math.asin(r.uniform(-1.0, 1.0)))
        sky = fibonacci_cap(n_sky, centre, math.radians(10.0))
        t_seg = segment_times(n_seg, t_sft)
        dets = [dict(t_seg=t_seg, v=velocity(t_seg, *site), k_lo=k_lo, t_sft=t_sft, n_seg=n_seg, n_bins=n_bins)
                for site in (SITE_H, SITE_L)]
        grid = dict(f0_min=f_lo, f0_step=0.125, n_f0=n_bins, tau=np.array([3500.0, 7000.0, 14000.0, 35000.0]),
                    brake=np.array([3.0, 5.0, 7.0]), sky=sky, t0=0.0)
        out.append(dict(dets=dets, grid=grid, n_templates=n_bins * 12 * n_sky,
                        n_evals=n_bins * 12 * n_sky * 2 * n_seg))
    return out


POOL_SIZE = 1 << 24


def exp_pool(seed=5, size=POOL_SIZE):
    """A pool of `size` FP32 Exp(1) values (exp_noise) from which the rows of
    the many-search workload are cut."""
    return exp_noise(1, size, seed)[0]


def pool_offsets(search, det, n_seg, n_bins, seed=5, size=POOL_SIZE):
    """Start of each row's window in the pool for detector `det` of search
    `search`: independent uniform integers in [0, size - n_bins]."""
    r = np.random.Generator(np.random.PCG64([seed, 1000 + search, det]))
    return r.integers(0, size - n_bins + 1, n_seg)


def pool_rows(pool, offsets, n_bins):
    """The spectrogram whose row j is pool[offsets[j] : offsets[j] + n_bins]:
    every pixel is one of the pool's Exp(1) values, and rows are windows at
    independent random positions.  Works on numpy arrays and on torch tensors
    (a device pool gives a device spectrogram with the same values)."""
    if hasattr(pool, "unfold"):
        return pool.unfold(0, int(n_bins), 1)[offsets].contiguous()
    return np.lib.stride_tricks.sliding_window_view(pool, int(n_bins))[np.asarray(offsets)]


def random_bank(n, f0_range, tau_range, brake_range, sky, seed=11):
    """The uniform random template bank of Sec. 2: n templates drawn uniformly
    (linearly) in f0, tau and the braking index over the given closed ranges,
    all at one sky direction (the search's sky point is fixed).  Returns the
    [n][6] rows (f0, tau, n, sky x, y, z) that the explicit-template
    evaluation takes."""
    r = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((int(n), 6), np.float64)
    out[:, 0] = r.uniform(f0_range[0], f0_range[1], n)
    out[:, 1] = r.uniform(tau_range[0], tau_range[1], n)
    out[:, 2] = r.uniform(brake_range[0], brake_range[1], n)
    k = np.asarray(sky, np.float64).reshape(3)
    out[:, 3:] = k / np.linalg.norm(k)
    return out
