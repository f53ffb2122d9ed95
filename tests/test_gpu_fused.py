"""Reduced-precision fused path (FP32 MFMA and split-BF16) against the FP64
CPU oracle and the FP64 GPU path.

Tolerances follow from the arithmetic.  One step moves a chain by
C_p dH_p + W_p eta_p; FP32 rounding of the state (2^-24 of |R|), of the
transforms (~2^-22 of the bond vector) and the single-precision Box-Muller
noise give a position error per step of a few 1e-7 of the contour length for
FP32; split BF16 carries 2^-17 relative products, a few 1e-6.  The bounds
below are 10-30x those estimates.  Over many steps the dynamics is
contractive, so the paired trajectories stay close, and the statistics must
agree with the FP64 GPU path within 2% (the target for reduced precision).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1411_3487_amd import Context, DMError, inputs, _lib

pytestmark = pytest.mark.gpu

NU, TS = 0.35, 0.034
B_FAC = 1.0 / (1.0 - 2.0 * NU)
ONE_STEP_TOL = {"fp32": 1e-5, "bf16x3": 1e-4}
MANY_STEP_TOL = {"fp32": 1e-3, "bf16x3": 1e-2}
DTAU = {64: 10.0, 96: 10.0, 128: 50.0, 192: 50.0, 256: 100.0, 384: 100.0, 512: 100.0}


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def rel_pos_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    M = a.shape[-1]
    return float(np.abs(a - b).reshape(a.shape[0], -1).max(axis=1).max() / ((M - 1) * B_FAC))


def run(prec, pos, M, n, seed=3, **kw):
    with Context(pos, seed=seed, precision=prec) as ctx:
        ctx.set_params([M], [kw.pop("dtau", DTAU.get(M, 10.0))], T_star=TS, nu=NU, **kw)
        ctx.step_modes(n)
        return ctx.positions(), ctx.modes()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("M", [2, 4, 64, 96, 128, 192, 256, 384, 512])
def test_fused_single_step_matches_oracle(prec, M):
    B = 7                      # two tiles of 5 chains, the second one ragged
    pos = inputs.straight_chains(B, M, B_FAC, seed=M + 1)
    dtau = DTAU.get(M, 1.0)
    got, _ = run(prec, pos, M, 1, dtau=dtau)
    R = oracle.step_modes(oracle.modes_from_positions(pos), NU, TS, dtau, 1, seed=3)
    err = rel_pos_err(got, oracle.positions_from_modes(R))
    print(f"{prec} M={M}: one-step rel err {err:.3e}")
    assert err < ONE_STEP_TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("M", [64, 256])
def test_fused_trajectory_stays_close_to_oracle(prec, M):
    B = 5
    pos = inputs.straight_chains(B, M, B_FAC, seed=M + 2)
    got, _ = run(prec, pos, M, 300)
    R = oracle.step_modes(oracle.modes_from_positions(pos), NU, TS, DTAU[M], 300, seed=3)
    err = rel_pos_err(got, oracle.positions_from_modes(R))
    print(f"{prec} M={M}: 300-step rel err {err:.3e}")
    assert err < MANY_STEP_TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_free_modes_and_shear(prec):
    """Coupling off: the update and the noise alone (with shear)."""
    B, M = 6, 64
    pos = inputs.straight_chains(B, M, B_FAC, seed=5)
    got, _ = run(prec, pos, M, 50, nonlinear=False, gamma_dot=1e-3)
    R = oracle.step_modes(oracle.modes_from_positions(pos), NU, TS, 10.0, 50, seed=3,
                          gamma_dot=1e-3, nonlinear=False)
    err = rel_pos_err(got, oracle.positions_from_modes(R))
    print(f"{prec}: free-mode 50-step rel err {err:.3e}")
    assert err < ONE_STEP_TOL[prec] * 10


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_centre_of_mass_is_fp64_random_walk(prec):
    """R_0 is advanced in FP64; its increments equal the FP64 path's to the
    single-precision noise (relative 1e-6)."""
    B, M = 10, 128
    pos = inputs.straight_chains(B, M, B_FAC, seed=7)
    _, R = run(prec, pos, M, 200)
    _, R64 = run("fp64", pos, M, 200)
    d = np.abs(R[:, :, 0] - R64[:, :, 0]).max()
    spread = np.abs(R64[:, :, 0] - oracle.modes_from_positions(pos)[:, :, 0]).max()
    assert d < 1e-5 * spread


def test_fused_rejects_odd_and_long_chains():
    for M in (63, 514):
        pos = inputs.straight_chains(1, M, B_FAC, seed=1)
        with pytest.raises(DMError):
            Context(pos, precision="bf16x3")


def msd_sum_theory(D, dtau, s, ns):
    """Mean and standard deviation, per chain, of the sum over ns samples
    (every s steps of dtau) of |r_cm(t_k) - r_cm(0)|^2 for a free 3-D random
    walk with diffusion coefficient D: E = 6 D sum_k t_k and, since
    Cov(|W(t_i)|^2, |W(t_j)|^2) = 6 (2 D min(t_i, t_j))^2 for Brownian W,
    Var = 24 D^2 sum_ij min(t_i, t_j)^2."""
    t = dtau * s * np.arange(1, ns + 1)
    mn = np.minimum.outer(t, t)
    return 6 * D * t.sum(), np.sqrt(24 * D * D * (mn * mn).sum())


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("B,M,dtau,n,s", [(1024, 128, 50.0, 2000, 20),
                                          (1024, 256, 100.0, 3000, 30),
                                          (256, 512, 100.0, 2000, 20)])
def test_statistics_match_fp64_within_two_percent(prec, B, M, dtau, n, s):
    """Shapes of the batched configurations (128 bp at dtau 50; 256 and 512
    bp at dtau 100), reduced in chains and steps; paired runs on identical
    Philox streams from the same random-orientation start.  Mean bond
    length, mean squared bond length, <L^2>, the middle bead's squared
    distance from the centre of mass and every mode variance <|R_p|^2>
    within 2% of the FP64 GPU path.  The centre of mass is FP64 on both
    paths, driven by the same Philox bits (FP64 normals on the plain form,
    the FP32 ones widened on the fused path), so its MSD agrees by
    construction to about 1e-7; instead both are checked against
    free-draining diffusion D = T*/M (Sec. VII.B) within five standard
    deviations of the sampled estimate."""
    pos = inputs.straight_chains(B, M, B_FAC, seed=1, random_orientation=True)
    acc = {}
    for p in ("fp64", prec):
        with Context(pos, seed=1, precision=p) as ctx:
            ctx.set_params([M], [dtau], T_star=TS, nu=NU, sample_every=s)
            ctx.step_modes(n)
            acc[p] = ctx.accumulators()[0]
    a, b = acc["fp64"], acc[prec]
    assert a["n_samples"] == b["n_samples"] == n // s
    for key in ("bond", "bond2", "L2", "dmid2"):
        rel = abs(b[key] / a[key] - 1)
        print(f"{prec} {B}x{M} {key}: rel diff {rel:.2e}")
        assert rel < 0.02, key
    rel_modes = np.abs(b["modes"][1:] / a["modes"][1:] - 1)
    print(f"{prec} {B}x{M} modes: max rel diff {rel_modes.max():.2e}")
    assert rel_modes.max() < 0.02
    mean, sd = msd_sum_theory(TS / M, dtau, s, n // s)
    for p, x in acc.items():
        z = (x["msd_cm"] / B - mean) / (sd / np.sqrt(B))
        print(f"{p} {B}x{M} msd_cm: {x['msd_cm'] / B / mean:.4f} of 6 D t, z = {z:.2f}")
        assert abs(z) < 5, (p, z)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_full_size_sampled_chains(prec):
    """The benchmark workload (4096 x 256 bp) in its launch shape; sampled
    chains recomputed by the oracle one by one."""
    B, M, n = 4096, 256, 10
    pos = inputs.straight_chains(B, M, B_FAC, seed=1)
    got, _ = run(prec, pos, M, n, seed=1)
    for c in [0, 4, 5, 2048, 4095]:
        R = oracle.step_modes(oracle.modes_from_positions(pos[c][None]), NU, TS, 100.0, n,
                              seed=1, chain_ids=[c])
        err = rel_pos_err(got[c][None], oracle.positions_from_modes(R))
        assert err < ONE_STEP_TOL[prec] * n, (c, err)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_uneven_ensemble(prec):
    lens = [64, 96, 128, 192, 256, 384, 512]
    beads = inputs.mixed_lengths(40, lens, seed=2)
    chains = inputs.mixed_chains(beads, B_FAC, seed=2)
    with Context(chains, seed=2, precision=prec) as ctx:
        ctx.set_params(lens, [DTAU[m] for m in lens], T_star=TS, nu=NU)
        ctx.step_modes(3)
        got = ctx.positions()
    for c in range(0, 40, 3):
        M = int(beads[c])
        R = oracle.step_modes(oracle.modes_from_positions(chains[c][None]), NU, TS, DTAU[M], 3,
                              seed=2, chain_ids=[c])
        err = rel_pos_err(got[c][None], oracle.positions_from_modes(R))
        assert err < 3 * ONE_STEP_TOL[prec], (c, M, err)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("M", [2, 64, 96, 256, 512])
def test_fused_observables_match_fp64_of_the_same_state(prec, M):
    """The fused observation kernel (FP32 MFMA positions from the FP32 state)
    against the oracle's observables of the FP64 positions and amplitudes of
    the same state: FP32 rounding of positions of size ~M b."""
    B = 12
    pos = inputs.straight_chains(B, M, B_FAC, seed=M + 7, random_orientation=True)
    with Context(pos, seed=4, precision=prec) as ctx:
        ctx.set_params([M], [DTAU.get(M, 10.0)], T_star=TS, nu=NU)
        ctx.step_modes(30)
        got = ctx.chain_observables()
        m2 = ctx.observables(_lib.DM_OBS_MODES).reshape(B, M)
        p64, R64 = ctx.positions(), ctx.modes()
    want = oracle.chain_observables(p64)
    scale = (M - 1) * B_FAC
    for k, name in enumerate(oracle.OBS_NAMES):
        unit = {"L2": scale ** 2, "bond2_mean": B_FAC ** 2}.get(name, scale)
        err = np.abs(got[:, k] - want[:, k]).max() / unit
        assert err < 2e-6, (name, err)
    want_m2 = (R64 ** 2).sum(axis=1)
    assert np.allclose(m2, want_m2, rtol=2e-6, atol=1e-12 * want_m2.max())


@pytest.mark.parametrize("B,M,dtau,n", [(4096, 256, 100.0, 300), (1024, 128, 50.0, 300),
                                        (1024, 512, 100.0, 200)])
def test_benchmark_launch_configuration_at_full_size(B, M, dtau, n):
    """Split BF16 in the launch configuration the benchmark times: autotuned
    tile shapes (4-tile workgroups at 4096 x 256, split tiles at 1024
    chains), sampling blocks of 100 steps replayed as graphs with the
    observables of each block taken beside the next launch where CUs are
    spare.  Afterwards sampled chains are recomputed by the oracle one by
    one: positions, and the per-chain observables of the final state, which
    the last (eager) observation wrote."""
    pos = inputs.straight_chains(B, M, B_FAC, seed=1, random_orientation=True)
    with Context(pos, seed=1, precision="bf16x3") as ctx:
        ctx.set_params([M], [dtau], T_star=TS, nu=NU, sample_every=100, use_graphs=True,
                       autotune=True)
        print(ctx.tiling()[0])
        ctx.step_modes(n)
        got = ctx.positions()
        obs = ctx.chain_observables()
        acc = ctx.accumulators()[0]
    assert acc["n_samples"] == n // 100 and acc["n_chains"] == B
    for c in [0, 4, 5, B // 4 + 3, B // 2, B - 1]:
        R = oracle.step_modes(oracle.modes_from_positions(pos[c][None]), NU, TS, dtau, n,
                              seed=1, chain_ids=[c])
        want = oracle.positions_from_modes(R)
        err = rel_pos_err(got[c][None], want)
        print(f"chain {c}: {n}-step rel err {err:.2e}")
        assert err < 1e-4, (c, err)
        o = oracle.chain_observables(want)[0]
        L = (M - 1) * B_FAC
        assert abs(obs[c, 1] - o[1]) < 1e-3 * L * L, c       # L^2
        assert abs(obs[c, 0] - o[0]) < 1e-4 * B_FAC, c       # mean bond length
