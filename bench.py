#!/usr/bin/env python3
"""Benchmark of the saliency hot path on one MI355X.

One step = one sal_saliency pass (local 3D DFT spectra -> plane projections -> spectral
energies -> directional comparisons -> FP64 normalisation and combination) over the
256 x 512 x 512 synthetic survey volume with an 8^3 cube, FP32 contractions.  Prints one
JSON line (see the "metric" field).  Inputs are resident in HBM before timing starts.

Per-kernel durations come from HIP events the library records around each of its kernels
on the launch stream; the roofline of the dominant kernel (the fused steps 1-3 kernel) is
its algorithmic flop count (separable DFT contraction per voxel: 4hL + 8hL^2 + 8hL^3 with
h = L/2 + 1) over its measured average duration, against the FP32 MFMA peak.
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
PROFILES = os.path.join(ROOT, "profiles")


def dft_flops_per_voxel(L: int) -> int:
    h = L // 2 + 1
    return 4 * h * L + 8 * h * L * L + 8 * h * L ** 3


# sources that define the FP32 fused kernel (its code, device helpers and launch set-up)
ENERGY_F32_SOURCES = ("sal_kernels.hip", "sal_device.h", "sal_internal.h")


def kernel_source_hash(files=ENERGY_F32_SOURCES) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1901_11095_amd", "csrc")
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters_from_profiles(kernel_tag: str):
    """The committed rocprofv3 counter summary of the kernel (HBM bytes per launch scaled by
    a copy-kernel calibration, MFMA busy fraction), if it was taken on the current kernel
    sources; else None."""
    path = os.path.join(PROFILES, "traffic_%s.json" % kernel_tag)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def cpu_baseline(V, L: int, sample_shape=(160, 192, 192)):
    """The FP64 oracle (unmodified) on a bounded sub-block of the same volume: energies on
    the block plus the comparison halo, Eq. (5) and the normalised combination."""
    import numpy as np
    import oracle as O
    p = O.Params(L=L)
    lo = tuple((n - s) // 2 for n, s in zip(V.shape, sample_shape))
    t0 = time.perf_counter()
    E, Sr = O.raw_box(V, p, lo, sample_shape)
    S, _ = O.combine(Sr, vmax=float(np.abs(V).max()))
    dt = time.perf_counter() - t0
    nvox = int(np.prod(sample_shape))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": nvox / dt, "unit": "voxels/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, %dx%dx%d sub-block at %s of the same volume (energies on "
                      "the block plus an r-voxel halo, Eq. (5), normalised Eq. (6)); %.1f s"
                      % (sample_shape + (lo, dt))}


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
    (2L = 10 rows would fill 10/16 of a matrix-core tile).  Roofline against the FP32 vector
    peak without packed instructions (78.6 TFLOP/s: 256 CUs x 128 lanes x 2 flops x 2.4 GHz)."""
    from paper_1901_11095_amd import sal
    ctx = sal.Saliency(L=L)
    ms, km = time_form(ctx, Vg, max(3, args.steps // 2), 2)
    fpv = dft_flops_per_voxel(L)
    ach = fpv * V.size / (km["energy"] * 1e-3) / 1e12
    return {"L": L, "voxels_per_s": V.size / (ms * 1e-3), "ms_per_step": ms, "kernels_ms": km,
            "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_TFLOPS["f32_vector"],
                         "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS["f32_vector"],
                         "kernel": "k_energy_gen<%d>" % L, "flops_per_voxel": fpv},
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


def stream_leg(args, dev):
    """The 512 x 1024 x 1024 survey (2 GiB, cube 16) from pinned host memory: the surrogate
    streamed through HBM in t-slabs with split-BF16 fallback tiles, against the plain method
    resident and streamed; errors against the plain FP32 GPU map and the oracle."""
    import numpy as np
    import torch
    from paper_1901_11095_amd import sal, stream, surrogate, synth
    name = "survey512x1024x1024"
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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="survey256x512x512")
    ap.add_argument("--L", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled oracle checks")
    ap.add_argument("--no-forms", action="store_true", help="only the FP32 form")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned surrogate leg")
    ap.add_argument("--sur-n", type=int, default=512, help="side of the surrogate's volume")
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
    e_ms = kms["energy"]
    achieved = fpv * N / (e_ms * 1e-3) / 1e12
    tag = "energy_f32_L%d_%s" % (args.L, args.workload)
    prof = counters_from_profiles(tag) or {}
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS["f32"], "traffic": prof.get("bytes_per_launch"),
            "kernel": "k_energy_f32<%d>" % args.L, "kernel_ms": e_ms, "flops_per_voxel": fpv,
            "mfma_busy": prof.get("mfma_busy"), "kernels_ms": kms}

    err = None
    if not args.no_check:
        print("# fp32: sampled oracle check", file=sys.stderr, flush=True)
        err = sampled_error(ctx, V, Vg, args.L)

    forms = {}
    if not args.no_forms:
        for prec in (sal.BF16_SPLIT, sal.FP16_SPLITW, sal.FP16_SPLIT, sal.BF16, sal.FP16):
            name = sal.PRECISION_NAMES[prec]
            print("# form %s" % name, file=sys.stderr, flush=True)
            c = sal.Saliency(L=args.L, precision=prec)
            ms_f, km = time_form(c, Vg, max(3, args.steps // 4), 2)
            dt = "bf16" if "bf16" in name else "f16"
            ach = fpv * N / (km["energy"] * 1e-3) / 1e12
            forms[name] = {
                "voxels_per_s": N / (ms_f * 1e-3), "ms_per_step": ms_f,
                "speedup_vs_fp32": ms_step / ms_f, "kernels_ms": km,
                "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[dt],
                             "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS[dt],
                             "kernel": "k_energy_h<%d>" % args.L},
                "max_rel_err_vs_oracle": None if args.no_check else sampled_error(c, V, Vg, args.L),
            }
            del c
    if not args.no_forms:
        print("# paper cube 5^3", file=sys.stderr, flush=True)
        forms["fp32_paper_cube_L5"] = small_cube_leg(args, V, Vg, 5)
        print("# stride-2 windows", file=sys.stderr, flush=True)
        forms["stride2"] = strided_leg(args, V, Vg)
    if not args.no_surrogate:
        forms["surrogate"] = surrogate_leg(args, dev)
    table = None
    if not args.no_table and not args.no_check:
        table = precision_table(dev)
    streamed = None
    if not args.no_stream:
        del Vg
        torch.cuda.empty_cache()
        streamed = stream_leg(args, dev)

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
        "streamed": streamed,
        "precision_table": table,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
