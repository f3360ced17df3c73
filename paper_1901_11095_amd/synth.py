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
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_SLAB = 32


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


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
    # slabs are independent (their random fields come from per-slab generators), so they
    # are filled by a thread pool; the result does not depend on the number of workers
    def fill(s0):
        s1 = min(n1, s0 + _SLAB)
        xs = np.arange(s0, s1, dtype=np.float64)
        X = (xs[:, None] - n1 / 2.0)
        Y = (yy[None, :] - n2 / 2.0)
        ncol = (s1 - s0) * n2
        # every boundary adds to the two samples around its depth in each column; the adds
        # are applied in boundary order (then upper sample first), as np.bincount sums its
        # weights in the order of its index list
        zb = (depths[:, None, None] + gx[:, None, None] * X[None] + gy[:, None, None] * Y[None]
              - t_lo).reshape(len(depths), 1, ncol)
        i0 = np.floor(zb).astype(np.int64)
        fr = zb - i0
        it = np.concatenate([i0, i0 + 1], axis=1)
        val = coeffs[:, None, None] * np.concatenate([1.0 - fr, fr], axis=1)
        lin = it * ncol + np.arange(ncol)
        ok = (it >= 0) & (it < nt)
        refl = np.bincount(lin[ok], weights=val[ok], minlength=nt * ncol).reshape(nt, s1 - s0, n2)
        tt = np.arange(nt, dtype=np.float64) + t_lo
        rows = np.arange(nt)[:, None, None]
        for nrm, p0 in faults:
            # hanging wall: nrm . (p - p0) > 0, summed in the order t, x, y.  With nrm[0] > 0
            # the partial sum over t and x never decreases down a column, and a rounded sum
            # of two doubles is positive exactly when the exact sum is, so the wall of each
            # column is the rows from the first one whose t+x part exceeds minus the y part
            tx = (nrm[0] * (tt - p0[0]))[:, None] + nrm[1] * (xs - p0[1])[None, :]
            my = -(nrm[2] * (yy - p0[2]))
            first = np.stack([np.searchsorted(tx[:, j], my, side="right")
                              for j in range(s1 - s0)])
            if throw > 0:
                wall = rows >= first[None]
                src = refl[:-throw].copy()
                np.copyto(refl[throw:], src, where=wall[throw:])
                refl[:throw][wall[:throw]] = 0.0
        for ib, (bt, bx, by, c) in enumerate(boxes):
            lo_x, hi_x = max(bx, s0), min(bx + c, s1)
            if lo_x >= hi_x:
                continue
            r = _slab_rng(seed, 10 + ib, s0 // _SLAB)
            blk = r.standard_normal((c, hi_x - lo_x, c))
            refl[bt - t_lo:bt - t_lo + c, lo_x - s0:hi_x - s0, by:by + c] = blk
        # trace[t] = sum_k wav[k] refl[t - k], in blocks of rows that stay in cache
        tb = max(1, (1 << 18) // ((s1 - s0) * n2))
        tmp = np.empty((tb, s1 - s0, n2), np.float64)
        for a in range(0, n0, tb):
            b = min(n0, a + tb)
            trace = np.zeros((b - a, s1 - s0, n2), np.float64)
            for k in range(-K, K + 1):
                np.multiply(refl[a - t_lo - k:b - t_lo - k], wav[k + K], out=tmp[:b - a])
                trace += tmp[:b - a]
            out[a:b, s0:s1, :] = trace

    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(fill, range(0, n1, _SLAB)))

    # --- noise at the requested SNR, then unit variance ---------------------------------
    sig_var = float(np.var(out, dtype=np.float64))
    nstd = math.sqrt(sig_var / snr_lin) if sig_var > 0 else 0.0

    def noise(s0):
        s1 = min(n1, s0 + _SLAB)
        r = _slab_rng(seed, 2, s0 // _SLAB)
        out[:, s0:s1, :] += (nstd * r.standard_normal((n0, s1 - s0, n2))).astype(np.float32)

    with ThreadPoolExecutor(max_workers=_workers()) as ex:
        list(ex.map(noise, range(0, n1, _SLAB)))
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
