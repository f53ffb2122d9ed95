"""GPU parity of the HIP library against the FP64 CPU oracle (through the C ABI).

FP64 plain form: trajectories must agree to 1e-10 relative over 1e3 steps on
identical Philox streams.  The error measure is the largest bead-position
difference divided by the chain's contour length (M-1) b, per chain.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1411_3487_amd import Context, DMError, inputs, _lib

pytestmark = pytest.mark.gpu

NU, TS = 0.35, 0.034
B_FAC = 1.0 / (1.0 - 2.0 * NU)
FP64_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def rel_pos_err(a, b):
    """max over chains of max |r_a - r_b| / ((M-1) b)."""
    a, b = np.asarray(a), np.asarray(b)
    M = a.shape[-1]
    return float(np.max(np.abs(a - b).reshape(a.shape[0], -1).max(axis=1)) / ((M - 1) * B_FAC))


def oracle_positions(pos0, dtau, n, seed, ids=None, step0=0, gamma_dot=0.0, nonlinear=True):
    R = oracle.modes_from_positions(pos0)
    R = oracle.step_modes(R, NU, TS, dtau, n, seed=seed, chain_ids=ids, step0=step0,
                          gamma_dot=gamma_dot, nonlinear=nonlinear)
    return oracle.positions_from_modes(R)


# ----------------------------------------------------------------- FP64 path
@pytest.mark.parametrize("B,M,dtau,n", [(1, 64, 10.0, 1000), (7, 100, 10.0, 300),
                                        (3, 255, 100.0, 100), (2, 2, 0.5, 200),
                                        (4, 3, 0.2, 200), (5, 17, 1.0, 300),
                                        (2, 2047, 100.0, 10), (2, 2048, 100.0, 10)])
def test_fp64_mode_steps_match_oracle(B, M, dtau, n):
    """Lengths from the smallest (2 beads) to the largest the FP64 path takes
    (2048), with and without the multiple-of-16 GEMM pipeline."""
    pos = inputs.straight_chains(B, M, B_FAC, seed=M, random_orientation=True)
    with Context(pos, seed=11, precision="fp64") as ctx:
        ctx.set_params([M], [dtau], T_star=TS, nu=NU)
        ctx.step_modes(n)
        got = ctx.positions()
        modes = ctx.modes()
    ref = oracle_positions(pos, dtau, n, seed=11)
    err = rel_pos_err(got, ref)
    print(f"B={B} M={M} dtau={dtau} n={n}: rel err {err:.3e}")
    assert err < FP64_TOL
    Rref = oracle.modes_from_positions(ref)
    assert np.abs(modes - Rref).max() <= 1e-9 * np.abs(Rref).max()


@pytest.mark.parametrize("B,M,dtau,ids", [(1024, 128, 50.0, [0, 1, 2, 3, 511, 512, 1000, 1023]),
                                          (4096, 256, 100.0, [0, 1337, 2048, 4095]),
                                          (1024, 512, 100.0, [5, 1023])])
def test_fp64_thousand_steps_on_the_batched_configurations(B, M, dtau, ids):
    """1e3 FP64 mode steps of the whole batched ensemble (1024 x 128 bp at
    dtau 50; 4096 x 256 and 1024 x 512 bp at dtau 100; random orientation,
    seed 1) on the GPU; the oracle advances the sampled chains with their
    ensemble chain indices (same Philox streams) and must agree to 1e-10 of
    the contour length."""
    n = 1000
    pos = inputs.straight_chains(B, M, B_FAC, seed=1, random_orientation=True)
    with Context(pos, seed=1, precision="fp64") as ctx:
        ctx.set_params([M], [dtau], T_star=TS, nu=NU)
        ctx.step_modes(n)
        got = ctx.positions()
    ref = oracle_positions(pos[ids], dtau, n, seed=1, ids=ids)
    err = rel_pos_err(got[ids], ref)
    print(f"B={B} M={M} dtau={dtau} n={n} chains {ids}: rel err {err:.3e}")
    assert err < FP64_TOL
    assert np.all(np.isfinite(got))


def test_fp64_uneven_lengths_in_one_context():
    beads = [64, 17, 2, 64, 100, 3, 17]
    chains = [inputs.straight_chains(1, m, B_FAC, seed=10 + i)[0] for i, m in enumerate(beads)]
    lengths, dts = [2, 3, 17, 64, 100], [0.5, 0.3, 1.0, 10.0, 10.0]
    with Context(chains, seed=5, precision="fp64") as ctx:
        ctx.set_params(lengths, dts, T_star=TS, nu=NU)
        ctx.step_modes(150)
        got = ctx.positions()
    for c, m in enumerate(beads):
        ref = oracle_positions(chains[c][None], dts[lengths.index(m)], 150, seed=5, ids=[c])
        assert rel_pos_err(got[c][None], ref) < FP64_TOL, (c, m)


def test_fp64_shear_matches_oracle():
    B, M, dtau, gdot = 3, 64, 10.0, 2e-3
    pos = inputs.straight_chains(B, M, B_FAC, seed=8)
    with Context(pos, seed=2, precision="fp64") as ctx:
        ctx.set_params([M], [dtau], T_star=TS, nu=NU, gamma_dot=gdot)
        ctx.step_modes(400)
        got = ctx.positions()
    ref = oracle_positions(pos, dtau, 400, seed=2, gamma_dot=gdot)
    assert rel_pos_err(got, ref) < FP64_TOL


def test_fp64_free_modes_match_oracle():
    B, M = 4, 32
    pos = inputs.straight_chains(B, M, B_FAC, seed=9)
    with Context(pos, seed=4, precision="fp64") as ctx:
        ctx.set_params([M], [3.0], T_star=TS, nu=NU, nonlinear=False)
        ctx.step_modes(200)
        got = ctx.positions()
    ref = oracle_positions(pos, 3.0, 200, seed=4, nonlinear=False)
    assert rel_pos_err(got, ref) < FP64_TOL


@pytest.mark.parametrize("M", [2, 5, 64, 130, 2048])
def test_euler_matches_oracle(M):
    B, dtau, n = 5, 0.1, (500 if M < 1000 else 50)
    pos = inputs.straight_chains(B, M, B_FAC, seed=20 + M)
    with Context(pos, seed=7, precision="fp64") as ctx:
        ctx.set_params([M], [10.0], T_star=TS, nu=NU, gamma_dot=1e-3)
        ctx.step_euler(n, dtau)
        got = ctx.positions()
        assert ctx.step == n
    ref = oracle.step_euler(pos, NU, TS, dtau, n, seed=7, gamma_dot=1e-3)
    assert rel_pos_err(got, ref) < FP64_TOL


def test_mode_and_euler_steps_share_the_step_counter():
    B, M = 3, 48
    pos = inputs.straight_chains(B, M, B_FAC, seed=31)
    with Context(pos, seed=9, precision="fp64") as ctx:
        ctx.set_params([M], [5.0], T_star=TS, nu=NU)
        ctx.step_modes(10)
        ctx.step_euler(20, 0.05)
        ctx.step_modes(10)
        got = ctx.positions()
        assert ctx.step == 40
    R = oracle.modes_from_positions(pos)
    R = oracle.step_modes(R, NU, TS, 5.0, 10, seed=9)
    x = oracle.step_euler(oracle.positions_from_modes(R), NU, TS, 0.05, 20, seed=9, step0=10)
    R = oracle.step_modes(oracle.modes_from_positions(x), NU, TS, 5.0, 10, seed=9, step0=30)
    assert rel_pos_err(got, oracle.positions_from_modes(R)) < FP64_TOL


def test_chain_observables_match_oracle():
    beads = [64, 64, 31, 128]
    chains = [inputs.straight_chains(1, m, B_FAC, seed=40 + i)[0] for i, m in enumerate(beads)]
    with Context(chains, seed=1, precision="fp64") as ctx:
        ctx.set_params([31, 64, 128], [5.0, 10.0, 50.0], T_star=TS, nu=NU)
        ctx.step_modes(50)
        pos = ctx.positions()
        obs = ctx.chain_observables()
        m2 = ctx.observables(_lib.DM_OBS_MODES)
        R = ctx.modes()
    for c in range(len(beads)):
        ref = oracle.chain_observables(pos[c][None])[0]
        assert np.allclose(obs[c], ref, rtol=1e-12, atol=1e-12), c
    flat = np.concatenate([(r ** 2).sum(axis=0) for r in R])
    assert np.allclose(m2, flat, rtol=1e-12)


def test_accumulators_sum_sampled_observables():
    B, M, s = 6, 64, 25
    pos = inputs.straight_chains(B, M, B_FAC, seed=50)
    with Context(pos, seed=3, precision="fp64") as ctx:
        ctx.set_params([M], [10.0], T_star=TS, nu=NU, sample_every=s)
        cm0 = ctx.chain_observables()[:, 5:8].copy()
        want = np.zeros(4)
        want_modes = np.zeros(M)
        for _ in range(4):
            ctx.step_modes(s)
            o = ctx.chain_observables()
            want += [o[:, 0].sum(), o[:, 15].sum(), o[:, 1].sum(),
                     ((o[:, 5:8] - cm0) ** 2).sum()]
            want_modes += ctx.observables(_lib.DM_OBS_MODES).reshape(B, M).sum(axis=0)
        acc = ctx.accumulators()[0]
    assert acc["M"] == M and acc["n_chains"] == B and acc["n_samples"] == 4
    got = np.array([acc["bond"], acc["bond2"], acc["L2"], acc["msd_cm"]])
    assert np.allclose(got, want, rtol=1e-12)
    assert np.allclose(acc["modes"], want_modes, rtol=1e-12)


def test_full_size_sampled_chains_fp64():
    """The 256-bp workload (4096 chains) in the benchmark's launch shape;
    sampled chains are recomputed by the oracle one by one."""
    B, M, n = 4096, 256, 20
    pos = inputs.straight_chains(B, M, B_FAC, seed=1)
    with Context(pos, seed=1, precision="fp64") as ctx:
        ctx.set_params([M], [100.0], T_star=TS, nu=NU)
        ctx.step_modes(n)
        got = ctx.positions()
    for c in [0, 1, 2047, 4095]:
        ref = oracle_positions(pos[c][None], 100.0, n, seed=1, ids=[c])
        assert rel_pos_err(got[c][None], ref) < FP64_TOL, c


# ----------------------------------------------------------------- errors
def test_invalid_parameters_are_rejected():
    pos = inputs.straight_chains(2, 16, B_FAC, seed=1)
    with Context(pos, seed=0, precision="fp64") as ctx:
        with pytest.raises(DMError) as e:
            ctx.step_modes(1)
        assert e.value.code == _lib.DM_ESTATE
        for bad in [dict(nu=0.5, T_star=TS), dict(nu=-0.1, T_star=TS), dict(nu=NU, T_star=0.0)]:
            with pytest.raises(DMError) as e:
                ctx.set_params([16], [1.0], **bad)
            assert e.value.code == _lib.DM_EINVAL
        with pytest.raises(DMError):
            ctx.set_params([17], [1.0], T_star=TS, nu=NU)
        with pytest.raises(DMError):
            ctx.set_params([16], [-1.0], T_star=TS, nu=NU)
        ctx.set_params([16], [1.0], T_star=TS, nu=NU)
        ctx.step_modes(0)
        assert ctx.step == 0
        with pytest.raises(DMError):
            ctx.step_euler(1, 0.0)


def test_unstable_euler_reports_nonfinite_state():
    """Sec. III.A: Euler blows up above dtau ~ 0.3; the finite check reports it."""
    pos = inputs.straight_chains(2, 32, B_FAC, seed=3)
    with Context(pos, seed=0, precision="fp64") as ctx:
        ctx.set_params([32], [1.0], T_star=TS, nu=NU, check_finite=True)
        ctx.step_euler(100, 0.05)
        with pytest.raises(DMError) as e:
            ctx.step_euler(3000, 0.35)
        assert e.value.code == _lib.DM_ENONFINITE


def test_save_load_resume_is_bit_identical():
    pos = inputs.straight_chains(6, 64, B_FAC, seed=12)
    with Context(pos, seed=6, precision="fp64") as a:
        a.set_params([64], [10.0], T_star=TS, nu=NU, sample_every=10)
        a.step_modes(100)
        blob = a.save_state()
        a.step_modes(100)
        ref = a.modes()
        ref_acc = a.accumulators()[0]
    with Context(pos, seed=6, precision="fp64") as b:
        b.set_params([64], [10.0], T_star=TS, nu=NU, sample_every=10)
        b.load_state(blob)
        assert b.step == 100
        b.step_modes(100)
        assert np.array_equal(b.modes(), ref)
        assert np.array_equal(b.accumulators()[0]["modes"], ref_acc["modes"])


def test_runs_are_deterministic():
    pos = inputs.straight_chains(9, 96, B_FAC, seed=13)
    outs = []
    for _ in range(2):
        with Context(pos, seed=8, precision="fp64") as ctx:
            ctx.set_params([96], [10.0], T_star=TS, nu=NU)
            ctx.step_modes(50)
            outs.append(ctx.modes())
    assert np.array_equal(outs[0], outs[1])


def test_positions_to_device_buffer():
    beads = [16, 40, 16]
    chains = [inputs.straight_chains(1, m, B_FAC, seed=60 + i)[0] for i, m in enumerate(beads)]
    with Context(chains, seed=0, precision="fp64") as ctx:
        ctx.set_params([16, 40], [1.0, 2.0], T_star=TS, nu=NU)
        ctx.step_modes(5)
        host = ctx.positions()
        dev = torch.zeros(3 * sum(beads), dtype=torch.float64, device="cuda")
        ctx.positions_to_device(dev.data_ptr())
        torch.cuda.synchronize()
        flat = np.concatenate([h.ravel() for h in host])
        assert np.array_equal(dev.cpu().numpy(), flat)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_library_initial_state_matches_oracle(prec):
    """A context created without positions builds the batched workloads'
    initial state itself (straight chains, Philox-uniform directions, 0.01 b
    jitter; Philox tags 5 and 4) at its first dm_set_params: the positions
    equal the oracle's generator of the same recipe, and 100 mode steps from
    them follow the oracle.  Before dm_set_params the state cannot be read."""
    B, M, dtau, n = 12, 128, 50.0, 100
    with Context(None, seed=1, precision=prec, beads=[M] * B) as ctx:
        with pytest.raises(DMError):
            ctx.positions()
        ctx.set_params([M], [dtau], T_star=TS, nu=NU)
        x0 = ctx.positions()
        ctx.step_modes(n)
        x = ctx.positions()
    want0 = oracle.config_chains(M, B, NU, seed=1)
    err0 = rel_pos_err(x0, want0)
    ref = oracle_positions(want0, dtau, n, seed=1)
    err = rel_pos_err(x, ref)
    print(f"{prec}: initial state err {err0:.2e}, after {n} steps {err:.2e}")
    assert err0 < (1e-13 if prec == "fp64" else 1e-6)
    assert err < (FP64_TOL if prec == "fp64" else 1e-3)


def test_library_initial_state_of_an_uneven_ensemble():
    beads = [64, 128, 64, 256, 128]
    with Context(None, seed=3, precision="fp64", beads=beads) as ctx:
        ctx.set_params([64, 128, 256], [10.0, 50.0, 100.0], T_star=TS, nu=NU)
        got = ctx.positions()
    for c, M in enumerate(beads):
        want = oracle.config_chains(M, 1, NU, seed=3, chain_ids=[c])
        assert rel_pos_err(got[c][None], want) < 1e-13, c
