"""Learned surrogate of the saliency method: training driver, checkpoints, and inference
with tile checks and exact fallback.  The arithmetic runs in libsal's HIP kernels
(sal_net_*, sal_saliency, sal_tile_merge, sal_normalize_combine); this module only
selects windows and tiles and moves tensors.

Training pairs.  The plain method (cube L = 16, FP32) gives the raw directional maps
S_t, S_x, S_y of seeded synthetic volumes.  A pair is a voxel v with its label S_m(v) and
the 16^3 window around it.  The network is run on 16^3 windows; its output at a voxel
depends on the 11^3 neighbourhood (five 3^3 layers), so the 6^3 centre of every window is
labelled and each window carries 216 pairs.  Targets are divided by the per-component
standard deviation over the training volumes; inference multiplies it back.

Fallback.  After inference a seeded sample of tiles is recomputed by the plain method on a
crop (tile plus L voxels of context, which holds every sample the tile's exact values
depend on) and any tile whose error exceeds the bound (max |pred - exact| over the
component's range) is replaced by the exact values before the exact FP64 normalisation
and Eq. (6).  Tiles outside the sample are not verified.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass, field
from typing import Optional

import numpy as np
import torch

from . import sal, synth

WINDOW = 16
MARGIN = 5
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                       "surrogate_L16.safetensors")


@dataclass
class TrainConfig:
    """Defaults: the configuration of the committed weights (32 volumes whose faults, chaotic
    bodies and SNR come from their seeds, 2M labelled voxels per epoch, 96 epochs, cosine
    learning rate 1e-3 -> 1e-4).  n_volumes=8, seeds 10..17, mix=False is the 8-volume set at
    one noise level, which does not generalise to the 5 dB survey volume."""
    L: int = 16
    n_volumes: int = 32
    shape: tuple = (256, 256, 256)
    seeds: tuple = tuple(range(10, 42))
    pairs_per_epoch: int = 2_000_000
    epochs: int = 96
    batch: int = 64
    lr: float = 1e-3
    lr_min: float = 1e-4
    window_seed: int = 18
    init_seed: int = 0
    mix: bool = True           # draw each training volume's structure and SNR from its seed
    history: list = field(default_factory=list)


def volume_kwargs(seed: int, shape, mix: bool = False) -> dict:
    """Training/held-out volumes: faults, a chaotic body and noise, sized to the shape.
    With `mix` the structure is drawn from the seed as well (1-6 faults, 0-2 chaotic bodies
    of side/8 to side/4, SNR 3-12 dB), so a training set spans the noise levels and
    structure counts of the survey-scale volumes."""
    side = min(shape)
    if not mix:
        return dict(shape=tuple(shape), seed=int(seed), n_faults=3, n_chaotic=1,
                    chaotic_size=max(8, side // 4), snr_db=10.0)
    r = np.random.default_rng([int(seed), 77])
    return dict(shape=tuple(shape), seed=int(seed), n_faults=int(r.integers(1, 7)),
                n_chaotic=int(r.integers(0, 3)),
                chaotic_size=max(8, int(r.integers(side // 8, side // 4 + 1))),
                snr_db=float(r.uniform(3.0, 12.0)))


def exact_raw_maps(ctx: sal.Saliency, V: torch.Tensor) -> torch.Tensor:
    """Plain-method raw maps [3, n0, n1, n2] of a device volume."""
    Sr = torch.empty((3,) + tuple(V.shape), dtype=torch.float32, device=V.device)
    ctx.saliency(V, S_raw_out=Sr)
    return Sr


def make_training_set(cfg: TrainConfig, device="cuda"):
    """Volumes and their exact raw maps, on the device."""
    ctx = sal.Saliency(L=cfg.L)
    vols, labels = [], []
    for s in cfg.seeds[:cfg.n_volumes]:
        V = torch.from_numpy(synth.make_volume(**volume_kwargs(s, cfg.shape, cfg.mix))).to(device)
        vols.append(V)
        labels.append(exact_raw_maps(ctx, V))
    torch.cuda.synchronize()
    return vols, labels


def _windows(vols, labels, pos, scale):
    """Gather windows (X [B, W, W, W]) and channel-last targets (T [B, W, W, W, 3])."""
    X, T = [], []
    for (i, t, x, y) in pos:
        X.append(vols[i][t:t + WINDOW, x:x + WINDOW, y:y + WINDOW])
        T.append(labels[i][:, t:t + WINDOW, x:x + WINDOW, y:y + WINDOW])
    X = torch.stack(X).contiguous()
    T = (torch.stack(T).permute(0, 2, 3, 4, 1) / scale).contiguous()
    return X, T


def train(cfg: TrainConfig, net: Optional[sal.Net] = None, log=print):
    """Train the network; returns (net, cfg with the loss history and scale)."""
    vols, labels = make_training_set(cfg)
    scale = torch.stack([torch.cat([lb[m].flatten() for lb in labels]).std() for m in range(3)])
    scale = scale.reshape(1, 1, 1, 1, 3).float()
    net = net or sal.Net(seed=cfg.init_seed)
    net.set_output_scale(scale.flatten().tolist())
    per_window = (WINDOW - 2 * MARGIN) ** 3
    n_windows = math.ceil(cfg.pairs_per_epoch / per_window)
    steps_per_epoch = math.ceil(n_windows / cfg.batch)
    total = steps_per_epoch * cfg.epochs
    rng = np.random.default_rng(cfg.window_seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    step = 0
    t0 = time.time()
    for ep in range(cfg.epochs):
        acc = 0.0
        for it in range(steps_per_epoch):
            pos = [(int(rng.integers(0, len(vols))),) +
                   tuple(int(rng.integers(0, n - WINDOW + 1)) for n in cfg.shape)
                   for _ in range(cfg.batch)]
            X, T = _windows(vols, labels, pos, scale)
            lr = cfg.lr_min + 0.5 * (cfg.lr - cfg.lr_min) * (1 + math.cos(math.pi * step / total))
            net.train_step(X, T, MARGIN, lr, loss_out=loss)
            acc += float(loss.item()) if it % 16 == 0 else 0.0
            step += 1
        mean = acc / max(1, (steps_per_epoch + 15) // 16)
        cfg.history.append(mean)
        log("epoch %d/%d  loss %.4f  (%.1f s)" % (ep + 1, cfg.epochs, mean, time.time() - t0))
    return net, cfg


def save(net: sal.Net, cfg: TrainConfig, path: str = WEIGHTS):
    from safetensors.numpy import save_file
    os.makedirs(os.path.dirname(path), exist_ok=True)
    meta = {"config": json.dumps({k: v for k, v in asdict(cfg).items()})}
    save_file({"params": net.get_params(), "out_scale": np.asarray(net.out_scale, np.float32)},
              path, metadata=meta)


def training_config(path: str = WEIGHTS) -> dict:
    """The training configuration stored with the weights (loss history left out)."""
    from safetensors import safe_open
    with safe_open(path, "np") as f:
        cfg = json.loads(f.metadata()["config"])
    cfg.pop("history", None)
    return cfg


def load(path: str = WEIGHTS, device: int = 0) -> sal.Net:
    from safetensors.numpy import load_file
    d = load_file(path)
    net = sal.Net(seed=0, device=device)
    net.set_params(d["params"])
    net.set_output_scale(d["out_scale"].tolist())
    return net


def tiles_of(shape, tile: int):
    return [(t, x, y) for t in range(0, shape[0], tile) for x in range(0, shape[1], tile)
            for y in range(0, shape[2], tile)]


class TileCheck:
    """Checks tiles of predicted raw maps against the plain method and replaces those over
    the bound.  `source(lo, hi)` returns (volume, origin): a device volume holding at least
    the samples of the box [lo, hi) of the full volume, and the full-volume position of its
    first sample (the resident volume itself with origin 0, or a crop copied from host
    memory); it serves `check`, one tile at a time.  `volumes(tiles)` yields
    (volume, origin, subset) groups covering the given tile indices, each subset with its
    halos inside its device volume; it serves `check_many`, which checks a group's tiles in
    batched passes (sal_check_tiles).  A tile is checked at most once."""

    def __init__(self, ctx: sal.Saliency, S_raw: torch.Tensor, stats: torch.Tensor, source,
                 tile: int, bound: float, capacity: int, volumes=None, chunk: int = 256):
        self.ctx, self.S_raw, self.stats, self.source = ctx, S_raw, stats, source
        self.volumes, self.chunk = volumes, chunk
        self.shape = tuple(S_raw.shape[1:])
        self.tile, self.bound = tile, bound
        self.nt = [(n + tile - 1) // tile for n in self.shape]
        self.errs = torch.zeros(capacity, dtype=torch.float32, device=S_raw.device)
        self.done = {}      # tile index -> slot in errs
        self.tiles = []     # (lo, dims) in check order
        self.exact = torch.empty((3, tile, tile, tile), dtype=torch.float32, device=S_raw.device)
        self._ws = None

    def n_tiles(self) -> int:
        return self.nt[0] * self.nt[1] * self.nt[2]

    def tile_lo(self, ti: int):
        a, rest = divmod(ti, self.nt[1] * self.nt[2])
        b, c = divmod(rest, self.nt[2])
        return (a * self.tile, b * self.tile, c * self.tile)

    def tile_of_voxel(self, flat: int) -> int:
        t, x, y = np.unravel_index(flat, self.shape)
        return int((t // self.tile * self.nt[1] + x // self.tile) * self.nt[2] + y // self.tile)

    def check(self, ti: int) -> bool:
        if ti in self.done or len(self.done) >= len(self.errs):
            return False
        j = len(self.done)
        self.done[ti] = j
        lo = self.tile_lo(ti)
        td = tuple(min(self.tile, n - a) for a, n in zip(lo, self.shape))
        halo = self.ctx.L  # floor(L/2) window + floor(d/2) comparison reach, d = L
        clo = tuple(max(0, a - halo) for a in lo)
        chi = tuple(min(n, a + d + halo) for a, d, n in zip(lo, td, self.shape))
        V, org = self.source(clo, chi)
        exact = self.exact[:, :td[0], :td[1], :td[2]]
        if td != (self.tile,) * 3:
            exact = torch.empty((3,) + td, dtype=torch.float32, device=self.S_raw.device)
        self.ctx.raw_box(V, tuple(a - o for a, o in zip(lo, org)), td, out=exact)
        sal.tile_merge(self.ctx, self.S_raw, exact, lo, lo, td, self.stats, self.bound,
                       self.errs[j:j + 1])
        self.tiles.append((lo, td))
        return True

    def tile_dims(self, ti: int):
        return tuple(min(self.tile, n - a) for a, n in zip(self.tile_lo(ti), self.shape))

    def check_many(self, tis) -> int:
        """Check the given tiles not checked yet (up to the capacity) in batched passes;
        returns how many were checked."""
        new = [t for t in dict.fromkeys(int(t) for t in tis) if t not in self.done]
        new = new[:max(0, len(self.errs) - len(self.done))]
        if not new:
            return 0
        if self.volumes is None:
            for ti in new:
                self.check(ti)
            return len(new)
        for V, org, sub in self.volumes(new):
            by_dims = {}
            for ti in sub:
                by_dims.setdefault(self.tile_dims(ti), []).append(ti)
            for td, group in by_dims.items():
                for c0 in range(0, len(group), self.chunk):
                    part = group[c0:c0 + self.chunk]
                    j0 = len(self.done)
                    los = [self.tile_lo(ti) for ti in part]
                    for k, ti in enumerate(part):
                        self.done[ti] = j0 + k
                        self.tiles.append((los[k], td))
                    need = sal.check_tiles_workspace_size(self.ctx, V.shape, len(part), td)
                    if self._ws is None or self._ws.numel() < need:
                        self._ws = torch.empty(need, dtype=torch.uint8, device=V.device)
                    box = [tuple(a - o for a, o in zip(lo, org)) for lo in los]
                    sal.check_tiles(self.ctx, V, box, self.S_raw, los, td, self.stats, self.bound,
                                    self.errs[j0:j0 + len(part)], workspace=self._ws)
        return len(new)

    def verify_extremes(self, max_rounds: int = 8, per_round: int = 32) -> int:
        """The volume-wide minimum and maximum of each map set the normalisation of Eq. (6).
        Check every unchecked tile whose values pass the extremes of the checked tiles by
        more than the bound (as a fraction of the checked range; a smaller excess moves the
        normalised map by less than the bound), up to `per_round` per extreme and round,
        most extreme first, until no unchecked tile does.  Returns the rounds used."""
        for r in range(max_rounds):
            mm = sal.tile_minmax(self.ctx, self.S_raw, self.tile).cpu().numpy()
            done = np.zeros(len(mm), dtype=bool)
            done[list(self.done)] = True
            new = []
            for m in range(3):
                lo, hi = mm[done, 2 * m].min(), mm[done, 2 * m + 1].max()
                tol = self.bound * (hi - lo)
                col = mm[:, 2 * m + 1]
                cand = np.nonzero(~done & (col > hi + tol))[0]
                new.extend(int(t) for t in cand[np.argsort(-col[cand], kind="stable")][:per_round])
                col = mm[:, 2 * m]
                cand = np.nonzero(~done & (col < lo - tol))[0]
                new.extend(int(t) for t in cand[np.argsort(col[cand], kind="stable")][:per_round])
            new = list(dict.fromkeys(new))
            if not new:
                return r
            self.check_many(new)
        return max_rounds

    def check_top(self, frac: float, abc=(1 / 3, 1 / 3, 1 / 3)) -> int:
        """Check the `frac` of the tiles with the highest predicted saliency: the upper bound
        sum_m a_m (max_m - lo_m) / (hi_m - lo_m) of Eq. (6) over the tile, with the predicted
        volume-wide ranges.  The surrogate's largest errors sit in such tiles (edges of
        chaotic bodies).  Returns the number of tiles checked."""
        k = int(math.ceil(frac * self.n_tiles()))
        if k <= 0:
            return 0
        mm = sal.tile_minmax(self.ctx, self.S_raw, self.tile).cpu().numpy().astype(np.float64)
        st = self.stats.cpu().numpy()
        score = np.zeros(len(mm))
        for m in range(3):
            rng = st[2 * m + 1] - st[2 * m]
            if rng > 0:
                score += abc[m] * (mm[:, 2 * m + 1] - st[2 * m]) / rng
        return self.check_many(np.argsort(-score, kind="stable")[:k])

    def errors(self) -> torch.Tensor:
        return self.errs[:len(self.done)]


def seeded_tiles(n_tiles: int, frac: float, seed: int):
    k = max(1, int(round(frac * n_tiles)))
    return sorted(np.random.default_rng(seed).choice(n_tiles, size=k, replace=False).tolist())


def infer_with_fallback(net: sal.Net, ctx_exact: sal.Saliency, V: torch.Tensor, tile: int = 32,
                        frac: float = 0.02, bound: float = 0.02, seed: int = 0,
                        S_raw: Optional[torch.Tensor] = None, check_extremes: bool = True,
                        max_rounds: int = 8, per_round: int = 32, top_frac: float = 0.05):
    """Surrogate maps, a seeded check of `frac` of the tiles against the plain method with
    exact replacement of the tiles over `bound`, optionally the `top_frac` of the tiles with
    the highest predicted saliency, then (with `check_extremes`) the tiles that hold each
    map's extremes until all of them are checked, then the exact FP64 normalisation and
    Eq. (6).
    Returns a dict with S, S_raw, stats, the checked tiles and their errors."""
    dev = V.device
    S_raw = net.infer(V, out=S_raw)
    stats = torch.zeros(8, dtype=torch.float64, device=dev)
    S = sal.normalize_combine(ctx_exact, S_raw, V, stats_out=stats)
    n_all = len(tiles_of(tuple(V.shape), tile))
    sample = seeded_tiles(n_all, frac, seed)
    cap = len(sample) + int(math.ceil(top_frac * n_all)) + (6 * per_round * max_rounds if check_extremes else 0)
    chk = TileCheck(ctx_exact, S_raw, stats, lambda lo, hi: (V, (0, 0, 0)), tile, bound, cap,
                    volumes=lambda tis: [(V, (0, 0, 0), tis)])
    chk.check_many(sample)
    chk.check_top(top_frac)
    rounds = chk.verify_extremes(max_rounds, per_round) if check_extremes else 0
    S = sal.normalize_combine(ctx_exact, S_raw, V, S=S, stats_out=stats)
    return {"S": S, "S_raw": S_raw, "stats": stats, "tiles": chk.tiles, "tile_err": chk.errors(),
            "n_tiles": chk.n_tiles(), "extreme_rounds": rounds}
