"""Synthetic participating media in the character of the paper's datasets.

The paper's renders use a noise-displaced cloud with vacuum around it, a CT
scan with per-channel albedo over one extinction field, and single-scattered
light from a directional source (Sec. 6).  Those datasets are not available,
so the media here are generated from seeds:

* ``value_noise``: SplitMix64-hashed lattice values in [0, 1), octave o has
  4*2**o cells per unit length and amplitude 0.5**o (lacunarity 2, gain 0.5),
  trilinear interpolation with smoothstep fade, sampled at voxel centres
  (i + 0.5)/n, normalised by the amplitude sum.
* ``cloud_extinction``: sigma_t = sigma_max * smoothstep(clamp((v - e0)/(e1 - e0)))
  with e1 = max v and e0 placed so that exactly a fraction p_vac of the voxels
  get sigma_t < 0.01 (near-vacuum).
* ``beer_lambert_source``: single-scatter source q = L * sigma_s * T for a
  directional light of unit radiance entering at the z = 0 face travelling +z,
  T = exp(-h * (sum_{k'<k} sigma_t + sigma_t/2)) (midpoint rule on the raw
  extinction), sigma_s = albedo * sigma_t.
* ``point_source``: homogeneous medium with one emitting voxel of power 1
  (j = 1/h^3), the paper's point-source validation set-up (Sec. 6.1).

Every array is float64, shape (nx, ny, nz), z fastest.
"""
from __future__ import annotations

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _lattice(seed: int, octave: int, m: int) -> np.ndarray:
    """Uniform [0,1) values on an (m+1)^3 lattice."""
    a = np.arange(m + 1, dtype=np.uint64)
    key = ((np.uint64(seed) << np.uint64(54)) | (np.uint64(octave) << np.uint64(48)))
    key = (key | (a[:, None, None] << np.uint64(32)) | (a[None, :, None] << np.uint64(16))
           | a[None, None, :])
    u = (_splitmix64(key) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return u


def _axis_weights(n: int, f: int):
    t = (np.arange(n) + 0.5) / n * f
    i0 = np.floor(t).astype(np.int64)
    fr = t - i0
    w = fr * fr * (3.0 - 2.0 * fr)
    return i0, w


def value_noise(n, octaves: int, seed: int, chunk: int = 32) -> np.ndarray:
    """Fractal value noise in [0,1) on an n^3 (or (nx,ny,nz)) voxel grid."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    out = np.zeros((nx, ny, nz))
    amp_sum = 0.0
    for o in range(octaves):
        f = 4 * 2 ** o
        amp = 0.5 ** o
        amp_sum += amp
        V = _lattice(seed, o, f)
        xi, xw = _axis_weights(nx, f)
        yi, yw = _axis_weights(ny, f)
        zi, zw = _axis_weights(nz, f)
        for x0 in range(0, nx, chunk):
            x1 = min(nx, x0 + chunk)
            a = xi[x0:x1]
            w = xw[x0:x1, None, None]
            t = (1.0 - w) * V[a] + w * V[a + 1]
            w = yw[None, :, None]
            t = (1.0 - w) * t[:, yi] + w * t[:, yi + 1]
            w = zw[None, None, :]
            t = (1.0 - w) * t[:, :, zi] + w * t[:, :, zi + 1]
            out[x0:x1] += amp * t
    return out / amp_sum


def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def _smoothstep_inv(y: float) -> float:
    return 0.5 - np.sin(np.arcsin(1.0 - 2.0 * y) / 3.0)


def cloud_extinction(v: np.ndarray, sigma_max: float, p_vac: float) -> np.ndarray:
    e1 = float(v.max())
    q = float(np.quantile(v, p_vac))
    delta = _smoothstep_inv(0.01 / sigma_max)
    e0 = (q - delta * e1) / (1.0 - delta)
    t = np.clip((v - e0) / (e1 - e0), 0.0, 1.0)
    return sigma_max * _smoothstep(t)


def beer_lambert_source(sigma_t: np.ndarray, albedo, h: float, light: float = 1.0) -> np.ndarray:
    """q = L * albedo * sigma_t * T with the light travelling +z from the z = 0 face."""
    tau_before = np.cumsum(sigma_t, axis=2) - sigma_t          # sum over k' < k
    T = np.exp(-h * (tau_before + 0.5 * sigma_t))
    return light * np.asarray(albedo) * sigma_t * T


def point_source(n: int = 32, sigma_t: float = 10.0, albedo: float = 0.9, h: float | None = None,
                 centre=None):
    """Homogeneous medium, unit-power source in one voxel (default (n//2,)*3)."""
    h = 1.0 / n if h is None else h
    st = np.full((n, n, n), float(sigma_t))
    al = np.full((n, n, n), float(albedo))
    Q = np.zeros((n, n, n))
    c = (n // 2,) * 3 if centre is None else tuple(centre)
    Q[c] = 1.0 / h ** 3
    return st, al, Q, h


def sphere_cloud(n, sigma_t: float = 10.0, albedo: float = 0.9, radius: float = 0.4,
                 octaves: int = 3, seed: int = 7):
    """The convergence test case of Sec. 5 (Fig. 3): a sphere of constant
    extinction centred in the unit cube, vacuum (sigma_t = 0) outside, and an
    emission field of fractal value noise inside the sphere only.  The paper
    gives neither the extinction, the albedo nor the radius; these defaults
    put about 8 optical depths across the sphere.  h = 1/n."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    h = 1.0 / max(nx, ny, nz)
    x = (np.arange(nx) + 0.5) * h - 0.5 * nx * h
    y = (np.arange(ny) + 0.5) * h - 0.5 * ny * h
    z = (np.arange(nz) + 0.5) * h - 0.5 * nz * h
    r2 = x[:, None, None] ** 2 + y[None, :, None] ** 2 + z[None, None, :] ** 2
    inside = r2 <= radius * radius
    st = np.where(inside, float(sigma_t), 0.0)
    al = np.full_like(st, float(albedo))
    Q = np.where(inside, value_noise((nx, ny, nz), octaves, seed), 0.0)
    return st, al, Q, h


def cloud_medium(n, octaves: int, sigma_max: float, p_vac: float, albedo: float, seed: int):
    """Heterogeneous cloud: (sigma_t, albedo, Q, h) with h = 1/n (unit cube)."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    h = 1.0 / max(nx, ny, nz)
    v = value_noise((nx, ny, nz), octaves, seed)
    st = cloud_extinction(v, sigma_max, p_vac)
    al = np.full_like(st, float(albedo))
    Q = beer_lambert_source(st, al, h)
    return st, al, Q, h


# Workloads named by what they are.
CONFIGS = {
    "point32": dict(kind="point", n=32, sigma_t=10.0, albedo=0.9),
    "cloud128": dict(kind="cloud", n=128, octaves=5, sigma_max=200.0, p_vac=0.40, albedo=0.99,
                     seed=1),
    "cloud256": dict(kind="cloud", n=256, octaves=5, sigma_max=200.0, p_vac=0.40, albedo=0.99,
                     seed=2),
    "cloud512": dict(kind="cloud", n=512, octaves=7, sigma_max=500.0, p_vac=0.60, albedo=0.995,
                     seed=4),
}


def config(name: str, n: int | None = None):
    """Inputs (sigma_t, albedo, Q, h) of a named workload; ``n`` overrides its size."""
    c = dict(CONFIGS[name])
    if n is not None:
        c["n"] = n
    if c.pop("kind") == "point":
        return point_source(c["n"], c["sigma_t"], c["albedo"])
    return cloud_medium(c["n"], c["octaves"], c["sigma_max"], c["p_vac"], c["albedo"], c["seed"])


def batch_config(nvol: int = 16, sizes=(64, 96, 128, 160, 192), albedos=(0.99, 0.95, 0.9),
                 seed: int = 3, size_scale: float = 1.0):
    """Batched workload: nvol cloud volumes of seeded uneven sizes, one shared
    extinction per volume and one albedo per colour channel.

    Returns a list of dicts {sigma_t, h, albedo: [per channel], Q: [per channel]}.
    ``size_scale`` shrinks every size (rounded to a multiple of 8) for quick tests.
    """
    rng = np.random.default_rng(seed)
    picks = rng.choice(np.asarray(sizes), size=nvol)
    vols = []
    for v, s in enumerate(picks):
        s = int(s)
        if size_scale != 1.0:
            s = max(16, int(round(s * size_scale / 8.0)) * 8)
        vols.append(batch_volume(s, v, albedos))
    return vols


def batch_volume(s: int, v: int, albedos=(0.99, 0.95, 0.9)):
    """Volume v of the batched workload at size s^3 (h = 1/s): 5-octave cloud
    of seed 300 + v, sigma_t in [0, 200] with 40 % near-vacuum, one albedo and
    single-scatter source per colour channel."""
    h = 1.0 / s
    st = cloud_extinction(value_noise(s, 5, 300 + v), 200.0, 0.40)
    chans_a = [np.full_like(st, a) for a in albedos]
    chans_q = [beer_lambert_source(st, a, h) for a in chans_a]
    return dict(sigma_t=st, h=h, albedo=chans_a, Q=chans_q, n=s)
