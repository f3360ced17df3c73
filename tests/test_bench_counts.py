"""The flop counts the benchmark's rooflines divide by, checked against an operation-counting
run of the arithmetic they describe (CPU only).

pair_dft_flops(L): an L-point complex DFT with the terms r, L - r and the outputs om, L - om
taken in conjugate pairs.  The counting version below performs exactly that arithmetic on
Python complex numbers, tallies its real adds and FMAs (an FMA counts 2), and must also
reproduce the plain DFT sum_r b[r] w^(om r)."""
import numpy as np
import pytest

import bench


class Tally:
    def __init__(self):
        self.flops = 0

    def add(self, a, b):          # complex add: 2 real adds
        self.flops += 2
        return a + b

    def sub(self, a, b):
        self.flops += 2
        return a - b

    def fma_real(self, a, s, c):  # complex a times real s plus complex c: 2 real FMAs
        self.flops += 4
        return a * s + c


def paired_dft(b, w, L, t):
    M, ev = (L - 1) // 2, L % 2 == 0
    u = {r: t.add(b[r], b[L - r]) for r in range(1, M + 1)}
    d = {r: t.sub(b[r], b[L - r]) for r in range(1, M + 1)}
    f0 = b[0]
    for r in range(1, M + 1):
        f0 = t.add(f0, u[r])
    if ev:
        f0 = t.add(f0, b[L // 2])
    F = [0j] * L
    F[0] = f0
    for om in range(1, M + 1):
        P, Q = b[0], 0j
        for r in range(1, M + 1):
            k = (om * r) % L
            P = t.fma_real(u[r], w[k].real, P)
            Q = t.fma_real(d[r], w[k].imag, Q)
        if ev:
            P = t.fma_real(b[L // 2], -1.0 if om & 1 else 1.0, P)
        F[om] = t.add(P, 1j * Q)       # (P.x - Q.y, P.y + Q.x): 2 real adds
        F[L - om] = t.sub(P, 1j * Q)
    if ev:
        fh = b[0]
        for r in range(1, M + 1):
            fh = t.fma_real(u[r], -1.0 if r & 1 else 1.0, fh)
        F[L // 2] = t.fma_real(b[L // 2], -1.0 if (L // 2) & 1 else 1.0, fh)
    return np.array(F)


@pytest.mark.parametrize("L", range(2, 8))
@pytest.mark.parametrize("sign", [-1, 1])
def test_pair_dft_count_and_value(L, sign):
    rng = np.random.default_rng(L)
    b = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    w = np.exp(sign * 2j * np.pi * np.arange(L) / L)
    t = Tally()
    got = paired_dft(list(b), w, L, t)
    ref = np.array([sum(b[r] * w[(om * r) % L] for r in range(L)) for om in range(L)])
    assert np.abs(got - ref).max() <= 1e-12
    assert t.flops == bench.pair_dft_flops(L)


def test_flop_counts_per_voxel():
    # paper's cube: 4hL + h x-DFTs of 52 flops + 13 y rows (rows 3, 4 of mu = 0 skipped), each
    # a DFT (52), 5 magnitudes (20), 2 pair sums, 3 weight groups (18) and the row factor (6)
    assert bench.gen_flops_per_voxel(5) == 4 * 3 * 5 + 3 * 52 + 13 * (52 + 20 + 2 + 18 + 6) == 1490
    assert bench.dft_flops_per_voxel(5) == 3660
    assert bench.slide_flops_per_voxel(16) == 53760 and bench.slide_flops_per_voxel(8) == 6784
    assert bench.dft_flops_per_voxel(16) == 313920 and bench.dft_flops_per_voxel(8) == 23200
