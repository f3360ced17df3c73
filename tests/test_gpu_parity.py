"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar: max|gpu - oracle| / max|oracle| <= 1e-5 for every FP32 map; bit-exact where the
arithmetic is exact (integer windows, unweighted comparisons, min/max statistics).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def relmax(got, ref):
    """max |got - ref| / max |ref| (complex values compared as complex numbers)."""
    dt = np.complex128 if (np.iscomplexobj(got) or np.iscomplexobj(ref)) else np.float64
    got = np.asarray(got, dt)
    ref = np.asarray(ref, dt)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def ctx8():
    return sal.Saliency(L=8)


@pytest.fixture(scope="module")
def ctx16():
    return sal.Saliency(L=16)


def gpu(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


# ------------------------------------------------------------------ step 1 ------------

@pytest.mark.parametrize("L", [8, 16])
def test_local_spectra_vs_oracle(dev, L):
    ctx = sal.Saliency(L=L)
    V = synth.random_volume((20, 19, 23), seed=L)
    for lo, bn in [((0, 0, 0), (2, 3, 4)), ((17, 15, 19), (3, 4, 4)), ((8, 7, 9), (2, 2, 3))]:
        print("local_spectra L=%d lo=%s bn=%s" % (L, lo, bn), flush=True)
        F = ctx.local_spectra(gpu(V, dev), lo, bn)
        torch.cuda.synchronize()
        ref = O.local_spectra(V, L, lo, bn)
        got = F.cpu().numpy().astype(np.complex128)
        assert relmax(got, ref) <= TOL


@pytest.mark.parametrize("L", [8, 16])
def test_local_spectra_dc_bit_exact(dev, L):
    """Integer windows: the DC bin is an integer sum times 2^-3k, exact in any order."""
    ctx = sal.Saliency(L=L)
    V = synth.integer_volume((19, 18, 21), seed=3)
    lo, bn = (0, 0, 0), (19, 18, 21) if L == 8 else (10, 18, 21)
    F = ctx.local_spectra(gpu(V, dev), lo, bn).cpu().numpy()
    dc_gpu = F[..., 0, 0, 0]
    ref = O.local_spectra(V, L, lo, (bn[0], bn[1], bn[2]))[..., 0, 0, 0]
    assert np.array_equal(dc_gpu.real.astype(np.float64), ref.real)
    assert np.all(dc_gpu.imag == 0.0)


# --------------------------------------------------------------- steps 2-3 -----------

@pytest.mark.parametrize("L", [8, 16])
def test_project_vs_oracle(dev, L):
    ctx = sal.Saliency(L=L)
    V = synth.random_volume((18, 17, 19), seed=5)
    spec = O.local_spectra(V, L, (1, 2, 3), (3, 2, 4)).astype(np.complex64)
    E = ctx.project(gpu(spec, dev)).cpu().numpy()
    flat = spec.reshape(-1, L, L, L)
    ref = np.stack([O.project(f.astype(np.complex128)) for f in flat], 1)
    assert relmax(E, ref) <= TOL


# ------------------------------------------------------------------ step 4 -----------

def test_dcs_vs_oracle(dev, ctx8):
    E = (np.abs(synth.random_volume((3, 21, 22, 23), seed=8)) + 0.1).astype(np.float32)
    S = ctx8.directional_compare(gpu(E, dev)).cpu().numpy()
    ref = O.dcs(E.astype(np.float64), 4, 2.0, O.RAYS_AXIS)
    assert relmax(S, ref) <= TOL


def test_dcs_all_rays_vs_oracle(dev):
    ctx = sal.Saliency(L=8, rays=sal.RAYS_ALL)
    E = (np.abs(synth.random_volume((3, 12, 11, 13), seed=9)) + 0.1).astype(np.float32)
    S = ctx.directional_compare(gpu(E, dev)).cpu().numpy()
    ref = O.dcs(E.astype(np.float64), 4, 2.0, O.RAYS_ALL)
    assert relmax(S, ref) <= TOL


def test_dcs_bit_exact_unweighted(dev):
    """sigma = inf: integer E, Q = 2r = 8, every partial sum exact -> bit-exact."""
    ctx = sal.Saliency(L=8, sigma=math.inf)
    E = np.abs(synth.integer_volume((3, 9, 10, 11), seed=4)).astype(np.float32)
    S = ctx.directional_compare(gpu(E, dev)).cpu().numpy().astype(np.float64)
    ref = O.dcs(E.astype(np.float64), 4, math.inf, O.RAYS_AXIS)
    assert np.array_equal(S, ref)


# ----------------------------------------------------------------- whole path ----------

def _check_full(ctx, V, L, dev, rays=O.RAYS_AXIS, sigma=None):
    p = O.Params(L=L, rays=rays, sigma=sigma)
    ref = O.saliency(V, p)
    S, E, Sr, st = ctx.saliency_maps(gpu(V, dev))
    torch.cuda.synchronize()
    E, Sr, S, st = E.cpu().numpy(), Sr.cpu().numpy(), S.cpu().numpy(), st.cpu().numpy()
    for m in range(3):
        assert relmax(E[m], ref["E"][m]) <= TOL, ("E", m, relmax(E[m], ref["E"][m]))
        assert relmax(Sr[m], ref["S_raw"][m]) <= TOL, ("S_raw", m)
    assert relmax(S, ref["S"]) <= TOL, ("S", relmax(S, ref["S"]))
    # statistics: exact min/max of the GPU's own raw maps and of |V|
    for m in range(3):
        assert st[2 * m] == Sr[m].min() and st[2 * m + 1] == Sr[m].max()
    assert st[6] == np.abs(V).max()
    return E, Sr, S, st


@pytest.mark.parametrize("shape", [(24, 20, 40), (33, 17, 45), (9, 9, 9), (40, 5, 70)])
def test_saliency_small_L8(dev, ctx8, shape):
    print("saliency L=8 shape", shape, flush=True)
    V = synth.make_volume(shape, seed=sum(shape), n_faults=1)
    _check_full(ctx8, V, 8, dev)


@pytest.mark.parametrize("shape", [(20, 18, 33), (17, 40, 9)])
def test_saliency_small_L16(dev, ctx16, shape):
    print("saliency L=16 shape", shape, flush=True)
    V = synth.make_volume(shape, seed=sum(shape), n_faults=1)
    _check_full(ctx16, V, 16, dev)


def test_saliency_all_rays(dev):
    ctx = sal.Saliency(L=8, rays=sal.RAYS_ALL)
    V = synth.make_volume((21, 22, 35), seed=2)
    _check_full(ctx, V, 8, dev, rays=O.RAYS_ALL)


def test_saliency_vol64_full(dev, ctx8):
    """64^3 volume, one fault, 10 dB: the whole volume against the oracle."""
    V = synth.workload("vol64")
    _check_full(ctx8, V, 8, dev)


@pytest.mark.parametrize("L", [8, 16])
def test_saliency_survey_subblock(dev, L):
    """256 x 512 x 512 survey volume on the GPU; oracle on seeded 32^3 sub-blocks (raw maps
    with the halo the comparison needs; the final map with the GPU's volume statistics)."""
    ctx = sal.Saliency(L=L)
    V = synth.workload("survey256x512x512")
    Vg = gpu(V, dev)
    S, E, Sr, st = ctx.saliency_maps(Vg)
    torch.cuda.synchronize()
    stats = st.cpu().numpy()
    rng = np.random.default_rng(1234 + L)
    los = [(0, 0, 0), (V.shape[0] - 32, V.shape[1] - 32, V.shape[2] - 32)]
    los.append(tuple(int(rng.integers(0, n - 32 + 1)) for n in V.shape))
    p = O.Params(L=L)
    for lo in los:
        print("sub-block", lo, flush=True)
        sl = tuple(slice(a, a + 32) for a in lo)
        Eo, So = O.raw_box(V, p, lo, (32, 32, 32))
        Eg = E[(slice(None),) + sl].cpu().numpy()
        Sg = Sr[(slice(None),) + sl].cpu().numpy()
        for m in range(3):
            assert relmax(Eg[m], Eo[m]) <= TOL
            assert relmax(Sg[m], So[m]) <= TOL
        Sref = O.combine_with_stats(So, stats[:6], vmax=stats[6])
        assert relmax(S[sl].cpu().numpy(), Sref) <= TOL
    # statistics are the exact min/max of the GPU raw maps
    Srn = Sr.cpu().numpy()
    for m in range(3):
        assert stats[2 * m] == Srn[m].min() and stats[2 * m + 1] == Srn[m].max()
    assert stats[6] == np.abs(V).max()


PARAM_CASES = [
    # (L, d, sigma, abc, normalize): Eq. (5) line length and Gaussian width, Eq. (6) weights
    (8, 6, 1.3, (0.5, 0.3, 0.2), 1),
    (8, None, None, (0.2, 0.7, 0.1), 0),
    (16, 10, 3.0, (1.0, 0.0, 0.0), 1),
    (5, 4, None, (0.25, 0.25, 0.5), 1),
]


@pytest.mark.parametrize("L,d,sigma,abc,normalize", PARAM_CASES)
def test_saliency_parameters_vs_oracle(dev, L, d, sigma, abc, normalize):
    """Non-default parameters of the method (the top-down tuning of Sec. 2: line length,
    Gaussian width, unequal weights of Eq. (6), raw combination) on the GPU against the
    oracle."""
    print("parameters", L, d, sigma, abc, normalize, flush=True)
    shape = (21, 23, 34) if L < 16 else (20, 22, 33)
    V = synth.make_volume(shape, seed=17, n_faults=1)
    ctx = sal.Saliency(L=L, d=d, sigma=sigma, abc=abc, normalize=bool(normalize))
    ref = O.saliency(V, O.Params(L=L, d=d, sigma=sigma, abc=abc, normalize=normalize))
    S, E, Sr, st = ctx.saliency_maps(gpu(V, dev))
    torch.cuda.synchronize()
    for m in range(3):
        assert relmax(Sr[m].cpu().numpy(), ref["S_raw"][m]) <= TOL, ("S_raw", m)
    assert relmax(S.cpu().numpy(), ref["S"]) <= TOL


def test_zero_contrast_guard_threshold(dev, ctx8):
    """zero_range placed between the smallest and the middle component range (relative
    to max|V|): exactly one component is treated as having no contrast, on both sides."""
    V = synth.make_volume((22, 20, 35), seed=23, n_faults=1)
    ref = O.saliency(V, O.Params(L=8))
    st = ref["stats"]
    vmax = float(np.abs(V).max())
    rel = sorted((st[2 * m + 1] - st[2 * m]) / vmax for m in range(3))
    zr = 0.5 * (rel[0] + rel[1])
    ctx = sal.Saliency(L=8, zero_range=zr)
    ref = O.saliency(V, O.Params(L=8, zero_range=zr))
    S, E, Sr, st_g = ctx.saliency_maps(gpu(V, dev))
    assert relmax(S.cpu().numpy(), ref["S"]) <= TOL
    # the dropped component leaves S in [0, 2/3]
    assert float(S.max()) <= 2.0 / 3.0 + 1e-6


# ------------------------------------------------------------ invariants on GPU --------

def test_constant_volume(dev, ctx8):
    V = np.full((20, 21, 33), 2.5, np.float32)
    S, E, Sr, st = ctx8.saliency_maps(gpu(V, dev))
    assert float(E.abs().max()) <= 1e-6 * 2.5
    assert torch.all(S == 0)


def test_dc_shift(dev, ctx8):
    V = (synth.integer_volume((20, 19, 35), seed=6) / 8.0).astype(np.float32)
    _, E0, S0, _ = ctx8.saliency_maps(gpu(V, dev))
    _, E1, S1, _ = ctx8.saliency_maps(gpu(V + 3.0, dev))
    assert relmax(E1.cpu().numpy(), E0.cpu().numpy()) <= TOL
    assert relmax(S1.cpu().numpy(), S0.cpu().numpy()) <= TOL


def test_axis_permutation(dev, ctx8):
    V = synth.random_volume((18, 26, 37), seed=12)
    _, E, Sr, _ = ctx8.saliency_maps(gpu(V, dev))
    Vp = np.ascontiguousarray(V.transpose(1, 0, 2))
    _, Ep, Srp, _ = ctx8.saliency_maps(gpu(Vp, dev))
    E, Ep = E.cpu().numpy(), Ep.cpu().numpy()
    for m, mp in [(0, 1), (1, 0), (2, 2)]:
        assert relmax(Ep[mp], E[m].transpose(1, 0, 2)) <= TOL


# ------------------------------------------------------------------ errors -------------

def test_error_paths(dev, ctx8):
    V = torch.zeros((4, 20, 20), device=dev)
    with pytest.raises(sal.SalError) as ei:
        ctx8.saliency(V)
    assert ei.value.status == sal.SAL_E_INVAL
    V = torch.zeros((20, 20, 20), device=dev)
    ws = torch.empty(16, dtype=torch.uint8, device=dev)
    with pytest.raises(sal.SalError) as ei:
        ctx8.saliency(V, workspace=ws)
    assert ei.value.status == sal.SAL_E_WORKSPACE
    big = torch.zeros(20 * 20 * 20 + 1, device=dev)
    with pytest.raises(sal.SalError) as ei:
        ctx8.saliency(big[1:].view(20, 20, 20))
    assert ei.value.status == sal.SAL_E_INVAL
    with pytest.raises(sal.SalError) as ei:
        sal.Saliency(L=21)
    assert ei.value.status == sal.SAL_E_UNSUPPORTED
    with pytest.raises(sal.SalError) as ei:
        sal.Saliency(L=5, precision=sal.BF16_SPLIT)
    assert ei.value.status == sal.SAL_E_UNSUPPORTED


def test_saliency_full_survey_subblocks(dev):
    """The 512 x 1024 x 1024 survey (2 GiB, six faults, two chaotic bodies, 5 dB) at cube
    16, in the launch configuration of the benchmark: the oracle on 16^3 sub-blocks at a
    corner, at the far corner and inside (energies on the block plus the comparison halo)."""
    ctx = sal.Saliency(L=16)
    V = synth.workload("survey512x1024x1024")
    Vg = gpu(V, dev)
    S, E, Sr, st = ctx.saliency_maps(Vg)
    torch.cuda.synchronize()
    stats = st.cpu().numpy()
    b = 16
    los = [(0, 0, 0), (V.shape[0] - b, V.shape[1] - b, V.shape[2] - b), (250, 600, 301)]
    p = O.Params(L=16)
    for lo in los:
        print("survey sub-block", lo, flush=True)
        sl = tuple(slice(a, a + b) for a in lo)
        Eo, So = O.raw_box(V, p, lo, (b, b, b))
        for m in range(3):
            assert relmax(E[(m,) + sl].cpu().numpy(), Eo[m]) <= TOL
            assert relmax(Sr[(m,) + sl].cpu().numpy(), So[m]) <= TOL
        Sref = O.combine_with_stats(So, stats[:6], vmax=stats[6])
        assert relmax(S[sl].cpu().numpy(), Sref) <= TOL
    for m in range(3):
        assert stats[2 * m] == float(Sr[m].min()) and stats[2 * m + 1] == float(Sr[m].max())


def test_size_limits(dev, ctx8):
    """Smallest accepted volume (every side max(floor(L/2), r) + 1) against the oracle; a
    volume of 2^31 voxels or more is rejected before any launch."""
    V = synth.random_volume((5, 5, 5), seed=1)
    _check_full(ctx8, V, 8, dev)
    with pytest.raises(sal.SalError) as ei:
        ctx8.workspace_size((2048, 1024, 1024))
    assert ei.value.status == sal.SAL_E_INVAL
    with pytest.raises(sal.SalError) as ei:
        ctx8.workspace_size((4, 100, 100))
    assert ei.value.status == sal.SAL_E_INVAL


def test_profile_counts_and_reset(dev, ctx8):
    """sal_profile_*: every timed saliency() call adds to the four kernel timers and the call
    count; a read with reset starts them again from zero."""
    V = gpu(synth.make_volume((20, 21, 33), seed=2), dev)
    ctx8.profile(True)
    ctx8.profile_read(reset=True)
    for _ in range(3):
        ctx8.saliency(V)
    torch.cuda.synchronize()
    ms, n = ctx8.profile_read(reset=True)
    assert n == 3 and all(v > 0.0 for v in ms.values()), (ms, n)
    ms, n = ctx8.profile_read(reset=True)
    assert n == 0 and all(v == 0.0 for v in ms.values()), (ms, n)
    ctx8.profile(False)
    ctx8.saliency(V)
    torch.cuda.synchronize()
    assert ctx8.profile_read(reset=True)[1] == 0
