#!/usr/bin/env python3
"""Benchmark of the saliency hot path on one MI355X.

One step = one sal_saliency pass (local 3D DFT spectra -> plane projections -> spectral
energies -> directional comparisons -> FP64 normalisation and combination) over the
512 x 1024 x 1024 synthetic survey volume (2 GiB, six faults, two chaotic bodies, 5 dB)
with a 16^3 cube, FP32 contractions.  On the same volume the split-BF16 form and the
learned surrogate (with its tile checks and exact fallback) are timed too, each with its
error against the FP32 map and the oracle.  Prints one JSON line (see the "metric" field).
Inputs are resident in HBM before timing starts.

Per-kernel durations come from HIP events the library records around each of its kernels
on the launch stream.  The roofline of a fused kernel that contracts every window is its
algorithmic flop count (the separable DFT contraction per voxel with the first two axes
shared between windows and the Hermitian half along t: 4hL + 8hL^2 + 8hL^3 with
h = L/2 + 1) over its measured average duration, against the matrix-core peak of its operand
type.  At cube 8 and 16 in FP32 the windows slide along t (one 2-D plane DFT and one complex
multiply-add per bin per window, then the magnitudes and projections): its roofline counts
the flops of that method against the FP32 vector peak, and the direct kernel is timed beside
it as the form "fp32_direct".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "saliency voxels/sec (plain FP32 vs BF16-split vs surrogate) at stated max error"
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2516.6, "f16": 2516.6, "f32_vector": 78.6}
HBM_PEAK_TBPS = 8.0  # MI355X HBM3E
PROFILES = os.path.join(ROOT, "profiles")


def dft_flops_per_voxel(L: int) -> int:
    h = L // 2 + 1
    return 4 * h * L + 8 * h * L * L + 8 * h * L ** 3


def dft_flops_per_voxel_min(L: int) -> int:
    """The same contraction with real rows at real cost and conjugate rows skipped: stage A
    real input (rows mu = 0, L/2 with real twiddles); stage B keeps nu <= L/2 for mu = 0, L/2
    (real input); stage C computes omega <= L/2 only for the four real rows.  This is the
    least work any separable form of the definition does."""
    h = L // 2 + 1
    a = 4 * L * (h - 1)
    b = 4 * L * L + 8 * L * L * (h - 2)
    c = 8 * L * L + 8 * L * L * (L - 2) + 8 * L ** 3 * (h - 2)
    return a + b + c


def slide_flops_per_voxel(L: int = 16) -> int:
    """Flops per window of the kernel whose windows slide along t (cube 8 or 16): the packed
    real DFT along x of one position of the entering-minus-leaving plane (L rows of L taps,
    real: 2 L^2), the complex DFT along y of its L/2 columns (8 L^2 L/2), the update of the
    L^3/2 stored bins (complex multiply 6 + add 2), their magnitudes (3, the square root
    counted as 1) and the three weighted sums (2 each): 53,760 at L = 16, 6,784 at L = 8."""
    nb = L ** 3 // 2
    return 2 * L * L + 8 * L * L * (L // 2) + 8 * nb + 4 * nb + 6 * nb


def pair_dft_flops(L: int) -> int:
    """Real flops of one L-point complex DFT with its terms and outputs in conjugate pairs
    (sums and differences of the inputs r and L - r times the real and imaginary twiddle
    parts; an FMA counts 2): 8M^2 + 10M for odd L (M = (L - 1)/2), 8M^2 + 18M + 6 for even L
    (M = L/2 - 1, the self-paired term and output L/2 added)."""
    if L % 2:
        m = (L - 1) // 2
        return 8 * m * m + 10 * m
    m = L // 2 - 1
    return 8 * m * m + 18 * m + 6


def gen_flops_per_voxel(L: int) -> int:
    """Flops per voxel of the vector-ALU kernel of cube sides 2..7: the real DFT along t into
    h = L/2 + 1 bins (4hL), the paired L-point DFTs along x (h per voxel), and per row (mu,
    nu) of the y stage, with the conjugate rows of the real mu = 0 (and L/2) taken once: its
    paired DFT, L magnitudes (3 each, the square root counted as 1), the sums of the bins om
    and L - om that share weights, three weighted sums per weight group om <= L/2 (2 each)
    and the row's three products into E (2 each): 1,490 at L = 5, where the direct
    contraction counts 3,660."""
    h = L // 2 + 1
    real_rows = 1 + (L % 2 == 0)
    rows = h * L - real_rows * (L - (L // 2 + 1))
    per_row = pair_dft_flops(L) + 4 * L + (L - 1) // 2 + 6 * (L // 2 + 1) + 6
    return 4 * h * L + h * pair_dft_flops(L) + rows * per_row


# What a committed counter record covers: the kernel template's own text, the device helpers
# and the box geometry it reads (a launcher or host-side change leaves the record valid).
KERNEL_TEXT = {
    "k_energy_slide": ("sal_energy_slide.hip", "k_energy_slide"),
    "k_energy_f32": ("sal_kernels.hip", "k_energy_f32"),
    "k_energy_h": ("sal_energy16.hip", "k_energy_h"),
    "k_conv3": ("sal_net.hip", "k_conv3"),
}
CSRC = os.path.join(ROOT, "paper_1901_11095_amd", "csrc")
SURROGATE_FLOPS = 2 * 47952  # multiply-adds of the five convolutions per voxel


def _function_text(path: str, name: str) -> str:
    """The definition of the __global__ function `name` in `path`: from its declarator to the
    brace that closes its body."""
    with open(path) as fh:
        src = fh.read()
    i = src.find("void %s(" % name)
    if i < 0:
        raise KeyError(name)
    j = src.index("{", i)
    depth = 0
    for k in range(j, len(src)):
        if src[k] == "{":
            depth += 1
        elif src[k] == "}":
            depth -= 1
            if depth == 0:
                return src[i:k + 1]
    raise ValueError("unbalanced braces in %s" % path)


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    fname, func = KERNEL_TEXT[kernel]
    h.update(_function_text(os.path.join(CSRC, fname), func).encode())
    with open(os.path.join(CSRC, "sal_device.h"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(CSRC, "sal_internal.h")) as fh:
        txt = fh.read()
    a, b = txt.find("struct ebox {"), txt.find("// ------------------------------------------------------------------ launchers")
    h.update(txt[a:b].encode())
    return h.hexdigest()[:16]


def counters_from_profiles(kernel_tag: str, kernel: str):
    """The committed rocprofv3 counter summary of the kernel (HBM bytes per launch scaled by
    a copy-kernel calibration, MFMA busy fraction), if it was taken on the current kernel
    text; else None."""
    path = os.path.join(PROFILES, "traffic_%s.json" % kernel_tag)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash(kernel):
        return None
    return rec


def roofline_block(kernel: str, ms: float, nvox: int, flops_per_voxel: int, peak_key: str, tag: str,
                   kernel_fn: str, min_flops_per_voxel=None, bound: str = "mfma"):
    """Roofline of one kernel: algorithmic flops per launch over the measured launch time."""
    achieved = flops_per_voxel * nvox / (ms * 1e-3) / 1e12
    prof = counters_from_profiles(tag, kernel_fn) or {}
    rec = {"bound": bound, "achieved": achieved, "peak": PEAK_TFLOPS[peak_key], "unit": "TFLOP/s",
           "frac": achieved / PEAK_TFLOPS[peak_key], "traffic": prof.get("bytes_per_launch"),
           "kernel": kernel, "kernel_ms": ms, "flops_per_voxel": flops_per_voxel,
           "mfma_busy": prof.get("mfma_busy"), "counters": "profiles/traffic_%s.json" % tag if prof else None}
    if min_flops_per_voxel:
        rec["flops_per_voxel_min"] = min_flops_per_voxel
        rec["frac_min"] = rec["frac"] * min_flops_per_voxel / flops_per_voxel
    if prof.get("algorithmic_bytes_per_launch"):
        rec["algorithmic_bytes"] = prof["algorithmic_bytes_per_launch"]
    if rec["traffic"]:
        # HBM rate of the measured traffic at this launch time, against the 8 TB/s peak
        rec["hbm_gbps"] = rec["traffic"] / (ms * 1e-3) / 1e9
        rec["hbm_frac"] = rec["hbm_gbps"] / (HBM_PEAK_TBPS * 1e3)
    return rec


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(V, L: int, shape_all=(64, 96, 96), shape_one=(24, 32, 48)):
    """The FP64 oracle (unmodified) on centred crops of the same volume, each computed as a
    volume of its own (every voxel's window DFT, projections, Eq. (5), Eq. (6)): the same
    per-voxel work as the GPU step.  Once with every OpenMP thread, once with one."""
    import ctypes
    import numpy as np
    import oracle as O
    O.lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    nmax = int(gomp.omp_get_max_threads())

    def run(shape, threads):
        gomp.omp_set_num_threads(int(threads))
        lo = tuple((n - s) // 2 for n, s in zip(V.shape, shape))
        crop = np.ascontiguousarray(V[lo[0]:lo[0] + shape[0], lo[1]:lo[1] + shape[1], lo[2]:lo[2] + shape[2]])
        t0 = time.perf_counter()
        O.saliency(crop, O.Params(L=L))
        dt = time.perf_counter() - t0
        return crop.size / dt, dt, lo

    try:
        v_all, dt_all, lo_all = run(shape_all, nmax)
        v_one, dt_one, lo_one = run(shape_one, 1)
    finally:
        gomp.omp_set_num_threads(nmax)
    return {"value": v_all, "unit": "voxels/s", "cores": nmax, "kind": "oracle",
            "value_1_thread": v_one, "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "FP64 oracle, the whole method at cube %d on a %dx%dx%d crop at %s of the "
                      "same volume (%.1f s, %d threads) and on a %dx%dx%d crop at %s (%.1f s, 1 "
                      "thread), each crop computed as a volume" % ((L,) + tuple(shape_all) + (lo_all, dt_all, nmax)
                                                                    + tuple(shape_one) + (lo_one, dt_one))}


def parity_sample(V, S, E, Sr, stats, L: int, seed: int = 7, b: int = 24, keep=None):
    """Max relative error of the GPU maps against the oracle on a seeded b^3 sub-block
    (the oracle's raw maps of the block are stored in `keep` when given)."""
    import numpy as np
    import oracle as O
    rng = np.random.default_rng(seed)
    lo = tuple(int(rng.integers(0, n - b + 1)) for n in V.shape)
    sl = tuple(slice(a, a + b) for a in lo)
    Eo, So = O.raw_box(V, O.Params(L=L), lo, (b, b, b))
    st = stats.cpu().numpy()
    Sref = O.combine_with_stats(So, st[:6], vmax=st[6])
    if keep is not None:
        keep["S_raw"], keep["S"] = So, Sref

    def rel(g, r):
        return float(np.abs(g - r).max() / np.abs(r).max())
    Eg = E[(slice(None),) + sl].cpu().numpy()
    Sg = Sr[(slice(None),) + sl].cpu().numpy()
    return {"E": max(rel(Eg[m], Eo[m]) for m in range(3)),
            "S_raw": max(rel(Sg[m], So[m]) for m in range(3)),
            "S": rel(S[sl].cpu().numpy(), Sref), "block": [list(lo), [b, b, b]]}


def time_form(ctx, Vg, steps, warmup):
    """Average ms per sal_saliency pass and per-kernel ms (HIP events) for one context."""
    import torch
    S = torch.empty_like(Vg)
    ws = ctx.workspace(Vg.shape)
    for _ in range(warmup):
        ctx.saliency(Vg, S=S, workspace=ws)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.saliency(Vg, S=S, workspace=ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kms, n = ctx.profile_read(reset=True)
    ctx.profile(False)
    return 1e3 * elapsed / steps, {k: v / max(n, 1) for k, v in kms.items()}


def sampled_error(ctx, V, Vg, L, seed=7, b=24):
    import torch
    dev = Vg.device
    shp = (3,) + tuple(Vg.shape)
    E = torch.empty(shp, dtype=torch.float32, device=dev)
    Sr = torch.empty(shp, dtype=torch.float32, device=dev)
    st = torch.empty(8, dtype=torch.float64, device=dev)
    S = ctx.saliency(Vg, E_out=E, S_raw_out=Sr, stats_out=st)
    torch.cuda.synchronize()
    err = parity_sample(V, S, E, Sr, st, L, seed=seed, b=b)
    del E, Sr
    return err


def surrogate_same_volume(V, Vg, S_ref, Sr_ref, st_ref, ms_fp32, ms_split, steps, warmup):
    """The learned surrogate on the headline volume (resident): inference, the seeded 2 %
    tile check, the check of the 5 % of tiles with the highest predicted saliency and of the
    tiles holding each map's extremes, split-BF16 fallback on tiles over the bound, exact
    FP64 normalisation.  Errors against the plain FP32 map everywhere, split by checked and
    unchecked tiles (the bound holds on checked tiles by construction; unchecked tiles are
    not verified)."""
    import numpy as np
    import torch
    from paper_1901_11095_amd import sal, surrogate
    dev = Vg.device
    N = Vg.numel()
    net = surrogate.load()
    ctx_fb = sal.Saliency(L=16, precision=sal.BF16_SPLIT)
    S_raw = torch.empty((3,) + tuple(Vg.shape), dtype=torch.float32, device=dev)
    for _ in range(max(1, warmup)):
        res = surrogate.infer_with_fallback(net, ctx_fb, Vg, S_raw=S_raw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = surrogate.infer_with_fallback(net, ctx_fb, Vg, S_raw=S_raw)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / steps
    # the network alone (five convolution launches on the current stream)
    pred = torch.empty_like(S_raw)
    net.infer(Vg, out=pred)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(3):
        net.infer(Vg, out=pred)
    ev[1].record()
    torch.cuda.synchronize()
    t_net = ev[0].elapsed_time(ev[1]) / 3
    # errors against the plain FP32 GPU map, per 32^3 tile
    t = 32
    n0, n1, n2 = Vg.shape
    rng = (st_ref[1:6:2] - st_ref[0:6:2]).float().reshape(3, 1, 1, 1)

    def tile_max(x):
        return x.reshape(n0 // t, t, n1 // t, t, n2 // t, t).amax(dim=(1, 3, 5)).flatten()
    raw_pre = tile_max(((pred - Sr_ref).abs() / rng).amax(0))
    raw_post = tile_max(((res["S_raw"] - Sr_ref).abs() / rng).amax(0))
    dS = (res["S"] - S_ref).abs()
    dS_tile = tile_max(dS)
    nt1, nt2 = n1 // t, n2 // t
    checked = torch.zeros(dS_tile.numel(), dtype=torch.bool, device=dev)
    idx = [(lo[0] // t * nt1 + lo[1] // t) * nt2 + lo[2] // t for lo, _ in res["tiles"]]
    checked[torch.tensor(idx, dtype=torch.long, device=dev)] = True
    S_pre = sal.normalize_combine(ctx_fb, pred, Vg)
    dS_pre = (S_pre - S_ref).abs()
    unchecked = ~checked
    tcfg = surrogate.training_config()
    out = {
        "training": {"volumes": tcfg["n_volumes"], "shape": tcfg["shape"], "pairs_per_epoch": tcfg["pairs_per_epoch"],
                     "epochs": tcfg["epochs"], "mixed_structure_and_snr": tcfg["mix"],
                     "deviation": "trained on 32 seeded 256^3 volumes of mixed structure and SNR (3-12 dB) "
                                  "instead of 8 at one noise level, which did not generalise to the 5 dB survey"},
        "voxels_per_s": N / t_sur, "ms": 1e3 * t_sur, "speedup_vs_plain_fp32": ms_fp32 / (1e3 * t_sur),
        "speedup_vs_plain_bf16_split": ms_split / (1e3 * t_sur), "tile": t, "bound": 0.02,
        "bound_scope": "raw maps within 2% of each map's range on every checked tile (exact "
                       "replacement); unchecked tiles are not verified",
        "checked_tiles": int(checked.sum()), "n_tiles": int(checked.numel()),
        "checked_over_bound_replaced": int((res["tile_err"] > 0.02).sum()),
        "tiles_within_bound_vs_plain_fp32": {"before_fallback": float((raw_pre <= 0.02).float().mean()),
                                             "after_fallback": float((raw_post <= 0.02).float().mean()),
                                             "unchecked_over_bound": int(((raw_post > 0.02) & unchecked).sum())},
        "S_abs_err_vs_plain_fp32": {"max": float(dS.max()), "mean": float(dS.mean()),
                                    "max_on_checked_tiles": float(dS_tile[checked].max()),
                                    "max_on_unchecked_tiles": float(dS_tile[unchecked].max()),
                                    "max_before_fallback": float(dS_pre.max()),
                                    "mean_before_fallback": float(dS_pre.mean())},
        "net_inference_ms": t_net,
        "roofline": roofline_block("k_conv3 x 5 (network inference, sum of the five launches)", t_net, N,
                                   SURROGATE_FLOPS, "bf16", "conv3_survey512x1024x1024", "k_conv3"),
    }
    out["roofline"]["bound"] = "mfma"
    del res, pred, S_raw, dS, S_pre, dS_pre
    return out


def surrogate_leg(args, dev):
    """Learned surrogate on the held-out 512^3 volume (cube 16): inference, seeded 2% tile
    check with split-BF16 fallback, exact normalisation; against the plain FP32 method."""
    import numpy as np
    import torch
    from paper_1901_11095_amd import sal, surrogate, synth
    print("# surrogate: generating held-out %d^3 volume" % args.sur_n, file=sys.stderr, flush=True)
    V = torch.from_numpy(synth.make_volume(**surrogate.volume_kwargs(99, (args.sur_n,) * 3))).to(dev)
    N = V.numel()
    net = surrogate.load()
    ctx_plain = sal.Saliency(L=16)
    ctx_fb = sal.Saliency(L=16, precision=sal.BF16_SPLIT)
    S_raw = torch.empty((3,) + tuple(V.shape), dtype=torch.float32, device=dev)
    for _ in range(max(1, args.warmup // 2)):
        res = surrogate.infer_with_fallback(net, ctx_fb, V, S_raw=S_raw)
    torch.cuda.synchronize()
    steps = max(2, args.steps // 4)
    print("# surrogate: timing %d passes" % steps, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = surrogate.infer_with_fallback(net, ctx_fb, V, S_raw=S_raw)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / steps
    # the plain method on the same volume, FP32 and split-BF16
    print("# surrogate: plain method on the same volume", file=sys.stderr, flush=True)
    ms_plain, _ = time_form(ctx_plain, V, 2, 1)
    ms_fb, _ = time_form(ctx_fb, V, 2, 1)
    st_ref = torch.zeros(8, dtype=torch.float64, device=dev)
    Sr_ref = torch.empty_like(S_raw)
    S_ref = ctx_plain.saliency(V, S_raw_out=Sr_ref, stats_out=st_ref)
    pred = net.infer(V)
    rng = (st_ref[1:6:2] - st_ref[0:6:2]).float().reshape(3, 1, 1, 1)
    raw_err = ((pred - Sr_ref).abs() / rng).amax(0)
    t = 32
    n0, n1, n2 = V.shape
    tmax = raw_err.reshape(n0 // t, t, n1 // t, t, n2 // t, t).amax(dim=(1, 3, 5))
    S_pre = sal.normalize_combine(ctx_plain, pred.contiguous(), V)
    dS_pre = (S_pre - S_ref).abs()
    dS = (res["S"] - S_ref).abs()
    # the exact map of the checked tiles is within the bound by construction; report it
    checked_err = []
    for lo, td in res["tiles"]:
        sl = tuple(slice(a, a + d) for a, d in zip(lo, td))
        checked_err.append(float(dS[sl].max()))
    # the same pipeline without the check of the 5% of tiles with the highest predicted
    # saliency (where the network's largest errors sit): faster, larger worst-case error
    for _ in range(2):
        res_t = surrogate.infer_with_fallback(net, ctx_fb, V, S_raw=S_raw, top_frac=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res_t = surrogate.infer_with_fallback(net, ctx_fb, V, S_raw=S_raw, top_frac=0.0)
    torch.cuda.synchronize()
    t_top = (time.perf_counter() - t0) / steps
    dS_t = (res_t["S"] - S_ref).abs()
    top5 = {"ms": 1e3 * t_top, "voxels_per_s": N / t_top, "speedup_vs_plain_fp32": ms_plain / (1e3 * t_top),
            "checked_tiles": len(res_t["tiles"]),
            "S_abs_err_vs_plain_fp32": {"max": float(dS_t.max()), "mean": float(dS_t.mean())}}
    del res_t, dS_t
    # the plain method on the stride-2 window lattice (split-BF16): the other fast
    # approximation of the same map
    ctx_s2 = sal.Saliency(L=16, precision=sal.BF16_SPLIT, stride=2)
    ms_s2, _ = time_form(ctx_s2, V, 3, 1)
    dS_s2 = (ctx_s2.saliency(V) - S_ref).abs()
    stride2 = {"ms": ms_s2, "speedup_vs_plain_fp32": ms_plain / ms_s2,
               "S_abs_err_vs_plain_fp32": {"max": float(dS_s2.max()), "mean": float(dS_s2.mean())}}
    del ctx_s2, dS_s2
    flops = 2 * 47952  # multiply-adds of the five convolutions per voxel
    net.infer(V, out=pred)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        net.infer(V, out=pred)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t0) / 3
    net_tf = flops * N / t_net / 1e12
    return {
        "voxels_per_s": N / t_sur, "ms": 1e3 * t_sur, "L": 16, "volume": [args.sur_n] * 3,
        "tile": 32, "checked_tiles": len(res["tiles"]), "n_tiles": res["n_tiles"],
        "checked_over_bound": int((res["tile_err"] > 0.02).sum()), "bound": 0.02,
        "speedup_vs_plain_fp32": ms_plain / (1e3 * t_sur), "plain_fp32_ms": ms_plain,
        "speedup_vs_plain_bf16_split": ms_fb / (1e3 * t_sur), "plain_bf16_split_ms": ms_fb,
        "tiles_within_bound_before_fallback": float((tmax <= 0.02).float().mean()),
        "S_abs_err_vs_plain_fp32": {"max": float(dS.max()), "mean": float(dS.mean()),
                                    "max_on_checked_tiles": max(checked_err),
                                    "max_before_fallback": float(dS_pre.max()),
                                    "mean_before_fallback": float(dS_pre.mean())},
        "net_inference_ms": 1e3 * t_net,
        "top_saliency_check_frac": 0.05,
        "without_top_saliency_check": top5,
        "plain_bf16_split_stride2": stride2,
        "roofline": {"bound": "mfma", "achieved": net_tf, "peak": PEAK_TFLOPS["bf16"],
                     "unit": "TFLOP/s", "frac": net_tf / PEAK_TFLOPS["bf16"],
                     "kernel": "k_conv3 (five layers, network inference only)",
                     "flops_per_voxel": flops},
    }


def small_cube_leg(args, V, Vg, L=5):
    """The paper's own cube (5 x 5 x 5, Sec. 2) on the same volume: FP32 on the vector ALUs
    (2L = 10 rows would fill 10/16 of a matrix-core tile).  Roofline: the kernel's own flops
    (gen_flops_per_voxel) against the FP32 vector peak without packed instructions
    (78.6 TFLOP/s: 256 CUs x 64 lanes x 2 flops x 2.4 GHz), the rate of the direct
    contraction's count beside it."""
    from paper_1901_11095_amd import sal
    ctx = sal.Saliency(L=L)
    ms, km = time_form(ctx, Vg, max(3, args.steps // 2), 2)
    fpv = gen_flops_per_voxel(L)
    ach = fpv * V.size / (km["energy"] * 1e-3) / 1e12
    return {"L": L, "voxels_per_s": V.size / (ms * 1e-3), "ms_per_step": ms, "kernels_ms": km,
            "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_TFLOPS["f32_vector"],
                         "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS["f32_vector"],
                         "kernel": "k_energy_gen<%d, 1>" % L, "flops_per_voxel": fpv,
                         "direct_equivalent_tflops": dft_flops_per_voxel(L) * V.size / (km["energy"] * 1e-3) / 1e12},
            "max_rel_err_vs_oracle": None if args.no_check else sampled_error(ctx, V, Vg, L)}


def strided_leg(args, V, Vg):
    """Windows on the stride-2 lattice (Sec. 2 first step allows any overlap above one half)
    with the energies interpolated back to every voxel: speed against stride 1 and the
    difference of the final map from the stride-1 map (what the lattice gives up)."""
    import torch
    from paper_1901_11095_amd import sal
    out = {}
    for L, prec in ((args.L, sal.FP32), (args.L, sal.BF16_SPLIT)):
        c1 = sal.Saliency(L=L, precision=prec)
        c2 = sal.Saliency(L=L, precision=prec, stride=2)
        ms1, _ = time_form(c1, Vg, max(3, args.steps // 4), 2)
        ms2, km2 = time_form(c2, Vg, max(3, args.steps // 4), 2)
        S1 = c1.saliency(Vg)
        S2 = c2.saliency(Vg)
        d = (S2 - S1).abs()
        out["L%d_%s" % (L, sal.PRECISION_NAMES[prec])] = {
            "voxels_per_s": V.size / (ms2 * 1e-3), "ms_per_step": ms2, "kernels_ms": km2,
            "speedup_vs_stride1": ms1 / ms2,
            "S_abs_diff_vs_stride1": {"max": float(d.max()), "mean": float(d.mean())}}
        del c1, c2, S1, S2, d
        torch.cuda.empty_cache()
    return out


def precision_table(dev):
    """Every precision form against the FP64 oracle on the whole 64^3 volume at cube 8 and
    16: max and mean of |GPU - oracle| / max|oracle| for E_t, E_x, E_y, S_t, S_x, S_y (raw
    maps of Eq. (5)) and the combined S of Eq. (6)."""
    import numpy as np
    import torch
    import oracle as O
    from paper_1901_11095_amd import sal, synth
    V = synth.workload("vol64")
    Vg = torch.from_numpy(V).to(dev)
    names = ("E_t", "E_x", "E_y", "S_t", "S_x", "S_y")
    table = {}
    for L in (8, 16):
        print("# precision table: oracle at cube %d" % L, file=sys.stderr, flush=True)
        ref = O.saliency(V, O.Params(L=L))
        maps_ref = [ref["E"][m] for m in range(3)] + [ref["S_raw"][m] for m in range(3)]
        for prec in sorted(sal.PRECISION_NAMES):
            c = sal.Saliency(L=L, precision=prec)
            S, E, Sr, _ = c.saliency_maps(Vg)
            got = [E[m] for m in range(3)] + [Sr[m] for m in range(3)]
            row = {}
            for n, g, r in zip(names + ("S",), got + [S], maps_ref + [ref["S"]]):
                d = np.abs(g.double().cpu().numpy() - r)
                den = float(np.abs(r).max())
                row[n] = {"max": float(d.max()) / den, "mean": float(d.mean()) / den}
            table["L%d_%s" % (L, sal.PRECISION_NAMES[prec])] = row
            del c
    return {"volume": "vol64 (64^3, seed 0)", "metric": "|GPU - FP64 oracle| / max|oracle|",
            "maps": table}


def stream_leg(args, dev, V=None):
    """The 512 x 1024 x 1024 survey (2 GiB, cube 16) from pinned host memory: the surrogate
    streamed through HBM in t-slabs with split-BF16 fallback tiles, against the plain method
    resident and streamed; errors against the plain FP32 GPU map and the oracle."""
    import numpy as np
    import torch
    from paper_1901_11095_amd import sal, stream, surrogate, synth
    name = "survey512x1024x1024"
    if V is None:
        print("# stream: generating %s" % name, file=sys.stderr, flush=True)
        V = synth.workload(name)
    N = V.size
    Vh = stream.pinned(V)
    net = surrogate.load()
    ctx32 = sal.Saliency(L=16)
    ctxb = sal.Saliency(L=16, precision=sal.BF16_SPLIT)
    slab = args.slab

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, 1e3 * (time.perf_counter() - t0) / reps

    print("# stream: host-to-device copy", file=sys.stderr, flush=True)
    Vg = torch.empty(V.shape, dtype=torch.float32, device=dev)
    Vg.copy_(Vh, non_blocking=True)
    _, ms_h2d = timed(lambda: Vg.copy_(Vh, non_blocking=True), 2)

    print("# stream: surrogate streamed (slab %d)" % slab, file=sys.stderr, flush=True)
    sur = lambda: stream.surrogate_streamed(net, ctxb, Vh, slab=slab)  # noqa: E731
    sur()
    res, ms_sur = timed(sur, 2)
    print("# stream: surrogate resident", file=sys.stderr, flush=True)
    Sr_buf = torch.empty((3,) + V.shape, dtype=torch.float32, device=dev)
    res_dev, ms_sur_dev = timed(
        lambda: surrogate.infer_with_fallback(net, ctxb, Vg, S_raw=Sr_buf), 2)
    del res_dev, Sr_buf
    print("# stream: plain FP32 and split-BF16 resident, FP32 streamed", file=sys.stderr, flush=True)
    ms_fp32, _ = time_form(ctx32, Vg, 1, 1)
    ms_bf, _ = time_form(ctxb, Vg, 1, 1)
    _, ms_fp32_st = timed(lambda: stream.plain_streamed(ctx32, Vh, slab=slab), 1)

    # the plain FP32 GPU map with every intermediate (reference for the surrogate's errors)
    S_ref, E_ref, Sr_ref, st_ref = ctx32.saliency_maps(Vg)
    dS = (res["S"] - S_ref).abs()
    rng = (st_ref[1:6:2] - st_ref[0:6:2]).float().reshape(3, 1, 1, 1)
    t = 32
    n0, n1, n2 = V.shape
    P = net.infer(Vg)
    raw_pre = ((P - Sr_ref).abs() / rng).amax(0)
    tmax_pre = raw_pre.reshape(n0 // t, t, n1 // t, t, n2 // t, t).amax(dim=(1, 3, 5))
    del P, raw_pre
    raw_err = ((res["S_raw"] - Sr_ref).abs() / rng).amax(0)
    tmax = raw_err.reshape(n0 // t, t, n1 // t, t, n2 // t, t).amax(dim=(1, 3, 5))
    del raw_err
    checked = [float(dS[tuple(slice(a, a + d) for a, d in zip(lo, td))].max())
               for lo, td in res["tiles"]]

    blocks = []
    if not args.no_check:
        print("# stream: oracle on a seeded 32^3 sub-block", file=sys.stderr, flush=True)
        b = 32
        ref = {}
        plain = parity_sample(V, S_ref, E_ref, Sr_ref, st_ref, 16, seed=5, b=b, keep=ref)
        So, Sref_o = ref["S_raw"], ref["S"]
        sl = tuple(slice(a, a + b) for a in plain["block"][0])
        st = st_ref.cpu().numpy()
        rng_o = (st[1:6:2] - st[0:6:2]).reshape(3, 1, 1, 1)
        Ssur = res["S_raw"][(slice(None),) + sl].cpu().numpy()
        blocks.append({"block": plain["block"], "plain_fp32_max_rel_err": plain,
                       "surrogate_raw_err_over_range": float((np.abs(Ssur - So) / rng_o).max()),
                       "surrogate_S_abs_err": float(np.abs(res["S"][sl].cpu().numpy() - Sref_o).max())})
    del E_ref
    return {
        "workload": name, "shape": list(V.shape), "L": 16, "slab": slab, "tile": 32,
        "bound": 0.02, "data": "synthetic, pinned host memory",
        "surrogate_streamed": {"voxels_per_s": N / (ms_sur * 1e-3), "ms": ms_sur,
                               "checked_tiles": len(res["tiles"]), "n_tiles": res["n_tiles"],
                               "checked_over_bound": int((res["tile_err"] > 0.02).sum())},
        "surrogate_resident": {"voxels_per_s": N / (ms_sur_dev * 1e-3), "ms": ms_sur_dev},
        "plain_fp32_resident": {"voxels_per_s": N / (ms_fp32 * 1e-3), "ms": ms_fp32},
        "plain_fp32_streamed": {"voxels_per_s": N / (ms_fp32_st * 1e-3), "ms": ms_fp32_st},
        "plain_bf16_split_resident": {"voxels_per_s": N / (ms_bf * 1e-3), "ms": ms_bf},
        "host_to_device_GBps": V.nbytes / (ms_h2d * 1e-3) / 1e9,
        "speedup_surrogate_streamed_vs_plain_fp32_resident": ms_fp32 / ms_sur,
        "tiles_within_bound": {"before_fallback": float((tmax_pre <= 0.02).float().mean()),
                               "after_fallback": float((tmax <= 0.02).float().mean())},
        "S_abs_err_vs_plain_fp32": {"max": float(dS.max()), "mean": float(dS.mean()),
                                    "max_on_checked_tiles": max(checked)},
        "oracle_blocks": blocks,
    }


def strides_same_volume(Vg, S_ref, ms_fp32, L, strides=(2, 3, 4, 7, 8, 16)):
    """Windows on the stride-s lattice of the headline volume (FP32), energies interpolated
    back to every voxel: speed against stride 1 and the difference of the final map from the
    stride-1 map.  At cube 8 and 16 the strides below L/2 run on the kernel whose windows
    slide along t, the non-overlapping s = L on the window-by-window kernel."""
    import torch
    from paper_1901_11095_amd import sal
    out = {}
    N = Vg.numel()
    for st in strides:
        if st != L and 2 * st >= L:
            continue
        print("# stride %d" % st, file=sys.stderr, flush=True)
        c = sal.Saliency(L=L, stride=st)
        ms, km = time_form(c, Vg, 3, 1)
        S = c.saliency(Vg)
        d = (S - S_ref).abs()
        out["s%d" % st] = {"voxels_per_s": N / (ms * 1e-3), "ms_per_step": ms, "kernels_ms": km,
                           "speedup_vs_stride1": ms_fp32 / ms,
                           "kernel": "k_energy_slide<%d, %d>" % (L, st) if L in (8, 16) and 2 * st < L else (
                               "k_energy_f32<%d, 2>" % L if st == 2 else
                               "k_energy_win_mfma" if L == 16 else "k_energy_win<%d>" % L),
                           "S_abs_diff_vs_stride1": {"max": float(d.max()), "mean": float(d.mean())}}
        del c, S, d
        torch.cuda.empty_cache()
    return out


def survey_L8_leg(args, dev):
    """The 256 x 512 x 512 survey volume at cube 8 (FP32 and every 16-bit form, the paper's
    5^3 cube, stride-2 windows): the smaller survey configuration."""
    import torch
    from paper_1901_11095_amd import sal, synth
    name, L = "survey256x512x512", 8
    print("# %s: generating" % name, file=sys.stderr, flush=True)
    V = synth.workload(name)
    N = V.size
    Vg = torch.from_numpy(V).to(dev)
    ctx = sal.Saliency(L=L)
    steps = max(3, args.steps // 2)
    ms, km = time_form(ctx, Vg, steps, 2)
    fpv = dft_flops_per_voxel(L)
    roof = roofline_block("k_energy_slide<%d, 1> (windows sliding along t)" % L, km["energy"], N,
                          slide_flops_per_voxel(L), "f32_vector", "energy_slide_L%d_%s" % (L, name),
                          "k_energy_slide", bound="alu")
    roof["direct_equivalent_tflops"] = fpv * N / (km["energy"] * 1e-3) / 1e12
    out = {"workload": name, "shape": list(V.shape), "L": L, "voxels_per_s": N / (ms * 1e-3),
           "ms_per_step": ms, "kernels_ms": km, "roofline": roof,
           "max_rel_err_vs_oracle": None if args.no_check else sampled_error(ctx, V, Vg, L)}
    forms = {}
    if not args.no_forms:
        print("# %s: form fp32_direct" % name, file=sys.stderr, flush=True)
        c = sal.Saliency(L=L, t_direct=True)
        ms_d, kmd = time_form(c, Vg, steps, 2)
        forms["fp32_direct"] = {
            "voxels_per_s": N / (ms_d * 1e-3), "ms_per_step": ms_d, "speedup_vs_fp32": ms / ms_d,
            "kernels_ms": kmd,
            "roofline": roofline_block("k_energy_f32<%d, 1>" % L, kmd["energy"], N, fpv, "f32",
                                       "energy_f32_L%d_%s" % (L, name), "k_energy_f32",
                                       dft_flops_per_voxel_min(L)),
            "max_rel_err_vs_oracle": None if args.no_check else sampled_error(c, V, Vg, L)}
        del c
        for prec in (sal.BF16_SPLIT, sal.FP16_SPLITW, sal.FP16_SPLIT, sal.BF16, sal.FP16):
            pname = sal.PRECISION_NAMES[prec]
            print("# %s: form %s" % (name, pname), file=sys.stderr, flush=True)
            c = sal.Saliency(L=L, precision=prec)
            ms_f, kmf = time_form(c, Vg, max(3, args.steps // 4), 2)
            forms[pname] = {
                "voxels_per_s": N / (ms_f * 1e-3), "ms_per_step": ms_f, "speedup_vs_fp32": ms / ms_f,
                "kernels_ms": kmf,
                "roofline": roofline_block("k_energy_h<%d>" % L, kmf["energy"], N, fpv,
                                           "bf16" if "bf16" in pname else "f16",
                                           "energy_h_%s_L%d_%s" % (pname, L, name), "k_energy_h",
                                           dft_flops_per_voxel_min(L)),
                "max_rel_err_vs_oracle": None if args.no_check else sampled_error(c, V, Vg, L)}
            del c
        print("# %s: paper cube 5^3" % name, file=sys.stderr, flush=True)
        forms["fp32_paper_cube_L5"] = small_cube_leg(args, V, Vg, 5)
        print("# %s: stride-2 windows" % name, file=sys.stderr, flush=True)
        args_l8 = argparse.Namespace(**vars(args))
        args_l8.L = L
        forms["stride2"] = strided_leg(args_l8, V, Vg)
    out["forms"] = forms
    del Vg, ctx
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="survey512x1024x1024")
    ap.add_argument("--L", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle checks")
    ap.add_argument("--no-forms", action="store_true", help="only the FP32 form")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned surrogate legs")
    ap.add_argument("--no-l8", action="store_true", help="skip the 256x512x512 cube-8 leg")
    ap.add_argument("--no-vol512", action="store_true", help="skip the held-out 512^3 surrogate leg")
    ap.add_argument("--sur-n", type=int, default=512, help="side of the held-out surrogate volume")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the 512x1024x1024 host-streamed leg")
    ap.add_argument("--slab", type=int, default=128, help="t-rows per streamed slab")
    ap.add_argument("--no-table", action="store_true",
                    help="skip the per-map error table of every form on the 64^3 volume")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        return 2

    import torch
    from paper_1901_11095_amd import build as B
    from paper_1901_11095_amd import sal, synth

    dev = torch.device("cuda", 0)
    if args.copy_calib:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "launches": 5}))
        return 0

    if not B.is_built():
        B.build()
    print("# generating %s" % args.workload, file=sys.stderr, flush=True)
    V = synth.workload(args.workload)
    N = V.size
    Vg = torch.from_numpy(V).to(dev)
    ctx = sal.Saliency(L=args.L)
    print("# fp32: timing %d steps" % args.steps, file=sys.stderr, flush=True)
    ms_step, kms = time_form(ctx, Vg, args.steps, args.warmup)
    value = N / (ms_step * 1e-3)
    fpv = dft_flops_per_voxel(args.L)
    slide = args.L in (8, 16)
    if slide:
        # the windows slide along t: the flops of that method against the FP32 vector peak
        # (packed FP32 instructions are not used: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz)
        roof = roofline_block("k_energy_slide<%d, 1> (windows sliding along t)" % args.L, kms["energy"], N,
                              slide_flops_per_voxel(args.L), "f32_vector",
                              "energy_slide_L%d_%s" % (args.L, args.workload), "k_energy_slide", bound="alu")
        roof["flops_convention"] = (
            "per window: 2L^2 (packed real DFT along x of one position of the plane difference) + "
            "8L^2 L/2 (complex DFT along y of the L/2 packed columns) + 8 per stored bin (complex "
            "multiply-add of the update, L^3/2 bins) + 4 per bin (magnitude, square root as 1) + "
            "6 per bin (three weighted sums) = %d; adds and square roots count one flop, so the "
            "vector-issue use is higher than frac" % slide_flops_per_voxel(args.L))
        roof["direct_equivalent_tflops"] = fpv * N / (kms["energy"] * 1e-3) / 1e12
    else:
        roof = roofline_block("k_energy_f32<%d>" % args.L, kms["energy"], N, fpv, "f32",
                              "energy_f32_L%d_%s" % (args.L, args.workload), "k_energy_f32",
                              dft_flops_per_voxel_min(args.L))
        roof["flops_convention"] = ("4hL + 8hL^2 + 8hL^3 per voxel, h = L/2 + 1: the separable DFT "
                                    "contraction with real rows counted at complex cost; frac_min uses "
                                    "the count with real rows at real cost and conjugate rows skipped")
    roof["kernels_ms"] = kms

    # the plain FP32 map with every intermediate: reference of the other forms' errors
    S_ref, E_ref, Sr_ref, st_ref = ctx.saliency_maps(Vg)
    torch.cuda.synchronize()
    err = None
    if not args.no_check:
        print("# fp32: sampled oracle check", file=sys.stderr, flush=True)
        err = parity_sample(V, S_ref, E_ref, Sr_ref, st_ref, args.L)
    del E_ref
    torch.cuda.empty_cache()

    forms = {}
    ms_split = None
    if not args.no_forms and slide:
        print("# form fp32_direct", file=sys.stderr, flush=True)
        c = sal.Saliency(L=args.L, t_direct=True)
        ms_d, km = time_form(c, Vg, max(3, args.steps // 4), 2)
        Sd = c.saliency(Vg)
        forms["fp32_direct"] = {
            "voxels_per_s": N / (ms_d * 1e-3), "ms_per_step": ms_d, "speedup_vs_fp32": ms_step / ms_d,
            "kernels_ms": km,
            "roofline": roofline_block("k_energy_f32<%d, 1>" % args.L, km["energy"], N, fpv, "f32",
                                       "energy_f32_L%d_%s" % (args.L, args.workload), "k_energy_f32",
                                       dft_flops_per_voxel_min(args.L)),
            "S_abs_err_vs_plain_fp32": float((Sd - S_ref).abs().max()),
        }
        del c, Sd
        torch.cuda.empty_cache()
    if not args.no_forms:
        print("# form bf16_split", file=sys.stderr, flush=True)
        c = sal.Saliency(L=args.L, precision=sal.BF16_SPLIT)
        ms_split, km = time_form(c, Vg, max(3, args.steps // 4), 2)
        Ssp = c.saliency(Vg)
        forms["bf16_split"] = {
            "voxels_per_s": N / (ms_split * 1e-3), "ms_per_step": ms_split,
            "speedup_vs_fp32": ms_step / ms_split, "kernels_ms": km,
            "roofline": roofline_block("k_energy_h<%d, bf16, split>" % args.L, km["energy"], N, fpv, "bf16",
                                       "energy_h_bf16_split_L%d_%s" % (args.L, args.workload),
                                       "k_energy_h", dft_flops_per_voxel_min(args.L)),
            "S_abs_err_vs_plain_fp32": float((Ssp - S_ref).abs().max()),
            "max_rel_err_vs_oracle": None if args.no_check else sampled_error(c, V, Vg, args.L),
        }
        del c, Ssp
        torch.cuda.empty_cache()
    if not args.no_surrogate and args.L == 16:
        print("# surrogate on the same volume", file=sys.stderr, flush=True)
        forms["surrogate"] = surrogate_same_volume(V, Vg, S_ref, Sr_ref, st_ref, ms_step,
                                                   ms_split if ms_split else float("nan"),
                                                   max(2, args.steps // 5), 1)
        torch.cuda.empty_cache()
    if not args.no_forms:
        forms["strides"] = strides_same_volume(Vg, S_ref, ms_step, args.L)
    del S_ref, Sr_ref, ctx
    torch.cuda.empty_cache()

    legs = {}
    if not args.no_l8:
        legs["survey256x512x512_L8"] = survey_L8_leg(args, dev)
    if not args.no_surrogate and not args.no_vol512:
        legs["surrogate_vol512"] = surrogate_leg(args, dev)
        torch.cuda.empty_cache()
    table = None
    if not args.no_table and not args.no_check:
        table = precision_table(dev)
    streamed = None
    if not args.no_stream:
        del Vg
        torch.cuda.empty_cache()
        streamed = stream_leg(args, dev, V if args.workload == "survey512x1024x1024" else None)

    cpu = None
    if not args.no_cpu:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(V, args.L)

    line = {
        "metric": METRIC, "value": value, "unit": "voxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "shape": list(V.shape), "L": args.L,
                   "form": "fp32", "rays": "+-t,+-x,+-y", "sigma": args.L / 4.0,
                   "parallelism": "none (1 GPU)"},
        "max_rel_err_vs_oracle": err,
        "roofline": roof,
        "forms": forms,
        "legs": legs,
        "streamed": streamed,
        "precision_table": table,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
