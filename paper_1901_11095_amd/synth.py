"""Seeded synthetic seismic volumes (inputs only; none of the saliency arithmetic lives here).

The paper evaluates on a real 3D survey (the F3 block, Sec. 3) that is not available
here; these volumes stand in for it with the same character: layered reflectors with gentle
dips, normal faults, chaotic (salt-like) bodies and noise, convolved with a seismic
wavelet along the time axis.

Recipe (all random numbers from ``numpy.random.default_rng``, PCG64):
  * layer thicknesses ~ 1 + Geometric(p = 1/(mean-1)) samples, mean ``thickness_mean``;
  * reflection coefficient of each boundary ~ N(0, ``refl_sigma``);
  * a regional dip (magnitude U(0, max_dip), azimuth U(0, 2 pi)) shared by all boundaries
    plus a per-boundary perturbation, total dip <= ``max_dip_deg``; the boundary depth is
    split linearly between the two nearest samples;
  * ``n_faults`` planar normal faults (dip U(60, 75) deg, random strike, through a random
    interior point); the hanging wall is shifted down by ``throw`` samples;
  * ``n_chaotic`` boxes of side ``chaotic_size`` whose reflectivity is replaced by i.i.d.
    N(0, 1) samples;
  * convolution along axis 0 with a Ricker wavelet of peak ``f_peak`` Hz sampled at ``dt``
    seconds, taps |k| <= ceil(1 / (f_peak dt));
  * white Gaussian noise at ``snr_db`` (10 log10 of the signal-to-noise variance ratio);
  * finally (v - mean) / std, stored as float32 C-order [n0][n1][n2].
Per-voxel random fields (chaotic reflectivity, noise) are drawn per slab of 32 rows of
axis 1 from ``default_rng([seed, tag, slab])`` so the result does not depend on memory
chunking.
"""
from __future__ import annotations

import math

import numpy as np

_SLAB = 32


def ricker(f_peak: float = 30.0, dt: float = 0.004) -> np.ndarray:
    """Ricker wavelet (1 - 2 pi^2 f^2 t^2) exp(-pi^2 f^2 t^2) at t = k dt."""
    K = int(math.ceil(1.0 / (f_peak * dt)))
    t = np.arange(-K, K + 1) * dt
    a = (math.pi * f_peak * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float64)


def _slab_rng(seed: int, tag: int, slab: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(tag), int(slab)])


def make_volume(shape=(64, 64, 64), seed: int = 0, n_faults: int = 1, throw: int = 4,
                n_chaotic: int = 0, chaotic_size: int = 64, snr_db: float = 10.0,
                thickness_mean: float = 6.0, refl_sigma: float = 0.1,
                max_dip_deg: float = 5.0, f_peak: float = 30.0, dt: float = 0.004) -> np.ndarray:
    n0, n1, n2 = (int(s) for s in shape)
    rng = np.random.default_rng(int(seed))
    wav = ricker(f_peak, dt)
    K = (len(wav) - 1) // 2

    # --- global structure -------------------------------------------------------------
    reg_dip = math.radians(rng.uniform(0.0, max_dip_deg * 0.7))
    reg_az = rng.uniform(0.0, 2.0 * math.pi)
    lat = max(n1, n2)
    pad = int(math.ceil(math.tan(math.radians(max_dip_deg)) * lat)) + throw * n_faults + K + 2
    t_lo, t_hi = -pad, n0 + pad
    depths, coeffs, gx, gy = [], [], [], []
    z = float(t_lo)
    p = 1.0 / max(thickness_mean - 1.0, 1e-6)
    while z < t_hi:
        z += 1.0 + float(rng.geometric(min(p, 1.0)) - 1)
        depths.append(z)
        coeffs.append(rng.normal(0.0, refl_sigma))
        dd = math.radians(rng.uniform(0.0, max_dip_deg * 0.3))
        da = rng.uniform(0.0, 2.0 * math.pi)
        gx.append(math.tan(reg_dip) * math.cos(reg_az) + math.tan(dd) * math.cos(da))
        gy.append(math.tan(reg_dip) * math.sin(reg_az) + math.tan(dd) * math.sin(da))
    depths = np.asarray(depths)
    coeffs = np.asarray(coeffs)
    gx = np.asarray(gx)
    gy = np.asarray(gy)

    faults = []
    for _ in range(n_faults):
        dip = math.radians(rng.uniform(60.0, 75.0))
        strike = rng.uniform(0.0, 2.0 * math.pi)
        # plane normal in (t, x, y) sample units: horizontal part along the dip direction
        nrm = np.array([math.sin(dip), math.cos(dip) * math.cos(strike),
                        math.cos(dip) * math.sin(strike)])
        p0 = np.array([rng.uniform(0.25, 0.75) * n0, rng.uniform(0.25, 0.75) * n1,
                       rng.uniform(0.25, 0.75) * n2])
        faults.append((nrm, p0))

    boxes = []
    for _ in range(n_chaotic):
        c = min(chaotic_size, n0, n1, n2)
        boxes.append((int(rng.integers(0, n0 - c + 1)), int(rng.integers(0, n1 - c + 1)),
                      int(rng.integers(0, n2 - c + 1)), c))

    snr_lin = 10.0 ** (snr_db / 10.0)
    out = np.empty((n0, n1, n2), np.float32)
    nt = t_hi - t_lo
    yy = np.arange(n2, dtype=np.float64)

    # --- per slab of axis-1 rows: reflectivity, faults, chaotic boxes, wavelet ---------
    for s0 in range(0, n1, _SLAB):
        s1 = min(n1, s0 + _SLAB)
        xs = np.arange(s0, s1, dtype=np.float64)
        refl = np.zeros((nt, s1 - s0, n2), np.float64)
        X = (xs[:, None] - n1 / 2.0)
        Y = (yy[None, :] - n2 / 2.0)
        cols = np.arange((s1 - s0) * n2)
        for b in range(len(depths)):
            zb = depths[b] + gx[b] * X + gy[b] * Y - t_lo
            i0 = np.floor(zb).astype(np.int64)
            fr = zb - i0
            for off, wgt in ((0, 1.0 - fr), (1, fr)):
                it = (i0 + off).ravel()
                ok = (it >= 0) & (it < nt)
                flat = refl.reshape(nt, -1)
                # one entry per column in each call, so plain fancy-index accumulation is exact
                flat[it[ok], cols[ok]] += coeffs[b] * wgt.ravel()[ok]
        tt = (np.arange(nt, dtype=np.float64) + t_lo)[:, None, None]
        for nrm, p0 in faults:
            side = (nrm[0] * (tt - p0[0]) + nrm[1] * (xs[None, :, None] - p0[1]) +
                    nrm[2] * (yy[None, None, :] - p0[2])) > 0.0
            shifted = np.zeros_like(refl)
            shifted[throw:] = refl[:-throw] if throw > 0 else refl
            refl = np.where(side, shifted, refl)
        for ib, (bt, bx, by, c) in enumerate(boxes):
            lo_x, hi_x = max(bx, s0), min(bx + c, s1)
            if lo_x >= hi_x:
                continue
            r = _slab_rng(seed, 10 + ib, s0 // _SLAB)
            blk = r.standard_normal((c, hi_x - lo_x, c))
            refl[bt - t_lo:bt - t_lo + c, lo_x - s0:hi_x - s0, by:by + c] = blk
        trace = np.zeros((n0, s1 - s0, n2), np.float64)
        for k in range(-K, K + 1):
            # trace[t] = sum_k wav[k] refl[t - k]
            trace += wav[k + K] * refl[(0 - t_lo) - k:(n0 - t_lo) - k]
        out[:, s0:s1, :] = trace.astype(np.float32)

    # --- noise at the requested SNR, then unit variance ---------------------------------
    sig_var = float(np.var(out, dtype=np.float64))
    nstd = math.sqrt(sig_var / snr_lin) if sig_var > 0 else 0.0
    for s0 in range(0, n1, _SLAB):
        s1 = min(n1, s0 + _SLAB)
        r = _slab_rng(seed, 2, s0 // _SLAB)
        out[:, s0:s1, :] += (nstd * r.standard_normal((n0, s1 - s0, n2))).astype(np.float32)
    mean = float(np.mean(out, dtype=np.float64))
    std = float(np.std(out, dtype=np.float64))
    out -= np.float32(mean)
    if std > 0:
        out *= np.float32(1.0 / std)
    return out


# Named workloads (sizes, seeds and structure of the benchmark volumes)
WORKLOADS = {
    # 64^3, one normal fault, 10 dB
    "vol64": dict(shape=(64, 64, 64), seed=0, n_faults=1, n_chaotic=0, snr_db=10.0),
    # 256 x 512 x 512, three faults and one 64^3 chaotic body
    "survey256x512x512": dict(shape=(256, 512, 512), seed=1, n_faults=3, n_chaotic=1,
                              chaotic_size=64, snr_db=10.0),
    # 512^3 held-out volume for the learned surrogate
    "vol512": dict(shape=(512, 512, 512), seed=99, n_faults=3, n_chaotic=1, chaotic_size=64,
                   snr_db=10.0),
    # 512 x 1024 x 1024, six faults, two chaotic bodies, 5 dB
    "survey512x1024x1024": dict(shape=(512, 1024, 1024), seed=7, n_faults=6, n_chaotic=2,
                                chaotic_size=64, snr_db=5.0),
}


def workload(name: str) -> np.ndarray:
    return make_volume(**WORKLOADS[name])


def integer_volume(shape, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Small random integers in [lo, hi] as float32 (exactness checks)."""
    rng = np.random.default_rng(int(seed))
    return rng.integers(lo, hi + 1, size=shape).astype(np.float32)


def random_volume(shape, seed: int) -> np.ndarray:
    rng = np.random.default_rng(int(seed))
    return rng.standard_normal(shape).astype(np.float32)
