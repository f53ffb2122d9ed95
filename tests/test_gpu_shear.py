"""Simple shear (Eq. btum): tumbling times and extension along the flow.

FP64 GPU against the oracle: the same Philox streams and FP64 arithmetic give
trajectories equal to ~1e-13, so every orientation decision, hence every
tumble, its time and its histogram bin, must agree exactly, and the summed
extension to rounding.  The reduced-precision paths are compared with the
FP64 GPU path statistically: mean extension within 2%, number of tumbles and
mean tumbling time within 10% (tumbles are rare, noise-triggered events, so
paired trajectories that differ by rounding may tumble a sample apart).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1411_3487_amd import Context, inputs

pytestmark = pytest.mark.gpu

NU, TS = 0.35, 0.034
B_FAC = 1.0 / (1.0 - 2.0 * NU)


def zeta1(M):
    return 16 * NU * math.sin(math.pi / (2 * M)) ** 4


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def gpu_shear(prec, pos, M, dtau, gdot, n_steps, se, seed=5, graphs=False):
    with Context(pos, seed=seed, precision=prec) as ctx:
        ctx.set_params([M], [dtau], T_star=TS, nu=NU, gamma_dot=gdot, sample_every=se,
                       use_graphs=graphs)
        ctx.step_modes(n_steps)
        return ctx.accumulators()[0]


def test_fp64_tumbling_matches_oracle():
    """8 chains of 16 beads at Wi = 100 (gamma_dot = 100 zeta_1), dtau = 1,
    10^4 steps sampled every 20."""
    B, M, dtau, se, nblk = 8, 16, 1.0, 20, 500
    gdot = 100 * zeta1(M)
    pos = inputs.straight_chains(B, M, B_FAC, seed=1, random_orientation=True)
    acc = gpu_shear("fp64", pos, M, dtau, gdot, se * nblk, se)

    R = oracle.modes_from_positions(pos)
    Lx, Ly, xspan = [], [], 0.0
    for k in range(nblk):
        R = oracle.step_modes(R, NU, TS, dtau, se, seed=5, step0=k * se,
                              chain_ids=np.arange(B), gamma_dot=gdot)
        o = oracle.chain_observables(oracle.positions_from_modes(R))
        Lx.append(o[:, 2])
        Ly.append(o[:, 3])
        xspan += o[:, 14].sum()
    Lx, Ly = np.array(Lx), np.array(Ly)
    steps = se * np.arange(1, nblk + 1)
    n_tot, times = 0, []
    for c in range(B):
        n, t = oracle.tumbles(Lx[:, c], Ly[:, c], steps)
        n_tot += n
        times += t
    print(f"tumbles {n_tot}, times {len(times)}, mean {np.mean(times):.0f} steps; "
          f"GPU {acc['tumbles']:.0f}, {acc['n_tau']:.0f}")
    assert n_tot >= 20 and len(times) >= 10
    assert acc["tumbles"] == n_tot
    assert acc["n_tau"] == len(times)
    assert acc["tau"] == sum(times)
    assert acc["tau2"] == sum(t * t for t in times)
    assert np.array_equal(acc["tumble_hist"], oracle.tumble_histogram(times))
    assert abs(acc["xspan"] / xspan - 1) < 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_reduced_precision_shear_statistics(prec):
    """250 chains of 16 beads, Wi = 100, 10^4 steps; paired with FP64."""
    B, M, dtau, se, n = 250, 16, 1.0, 20, 10000
    gdot = 100 * zeta1(M)
    pos = inputs.straight_chains(B, M, B_FAC, seed=1, random_orientation=True)
    a = gpu_shear("fp64", pos, M, dtau, gdot, n, se)
    b = gpu_shear(prec, pos, M, dtau, gdot, n, se, graphs=True)
    ext = [x["xspan"] / x["n_samples"] / x["n_chains"] / ((M - 1) * B_FAC) for x in (a, b)]
    mtau = [x["tau"] / x["n_tau"] for x in (a, b)]
    print(f"{prec}: extension {ext[0]:.4f} vs {ext[1]:.4f}; tumbles {a['tumbles']:.0f} vs "
          f"{b['tumbles']:.0f}; mean tumbling time {mtau[0]:.0f} vs {mtau[1]:.0f} steps")
    assert a["tumbles"] > 500
    assert abs(ext[1] / ext[0] - 1) < 0.02
    assert abs(b["tumbles"] / a["tumbles"] - 1) < 0.10
    assert abs(mtau[1] / mtau[0] - 1) < 0.10


def test_extension_grows_with_shear_rate():
    """At fixed Wi the chain stretches along the flow: the mean extension at
    Wi = 100 exceeds that at Wi = 1 (FP64, 64 chains of 32 beads)."""
    B, M, dtau, se, n = 64, 32, 1.0, 20, 10000
    pos = inputs.straight_chains(B, M, B_FAC, seed=3, random_orientation=True)
    ext = []
    for wi in (1.0, 100.0):
        acc = gpu_shear("fp64", pos, M, dtau, wi * zeta1(M), n, se)
        ext.append(acc["xspan"] / acc["n_samples"] / B)
    assert ext[1] > ext[0]
