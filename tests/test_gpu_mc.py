"""Metropolis Monte Carlo in the mode representation (dm_step_mc).

FP64 GPU against the oracle on identical Philox streams: every accept/reject
decision compares U1 with exp(-dH'/T*) where both sides' dH' agree to ~1e-13,
so the decisions, the accepted counts and the final amplitudes agree (the
latter to rounding).  Then the use the paper makes of the sampler: its
equilibrium values Q(0) (end-to-end vector, middle bond, middle bead about
the centre of mass) against the mode dynamics at a small time step, within
the paper's 5 %.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1411_3487_amd import Context, inputs, _lib

pytestmark = pytest.mark.gpu

NU, TS = 0.35, 0.034
B_FAC = 1.0 / (1.0 - 2.0 * NU)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("M", [2, 3, 16, 70])
def test_mc_fp64_matches_oracle(M):
    B, n, scale = 6, 30, 3.0
    pos = inputs.straight_chains(B, M, B_FAC, seed=M, random_orientation=True, jitter=0.05)
    with Context(pos, seed=3, precision="fp64") as ctx:
        ctx.set_params([M], [1.0], T_star=TS, nu=NU)
        ctx.step_modes(2)                  # the step counter is shared: start at 2
        R0 = ctx.modes()
        acc = ctx.step_mc(n, scale)
        got = ctx.modes()
        assert ctx.step == 2 + n
    want, want_acc = oracle.mc_sweeps(R0, NU, TS, scale, n, seed=3, step0=2)
    print(f"M={M}: accepted {acc} (oracle {want_acc.sum()}) of {B * n * 3 * (M - 1)}")
    assert acc == want_acc.sum()
    err = np.abs(got - want).max() / max(1.0, np.abs(want).max())
    assert err < 1e-10, err


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mc_on_fused_contexts(prec):
    """The fused state is converted to FP64 for the sweeps and back; the
    centre of mass is untouched and about 56 % of the proposals pass at
    step_scale = 3."""
    B, M, n = 20, 64, 40
    pos = inputs.straight_chains(B, M, B_FAC, seed=2, random_orientation=True)
    with Context(pos, seed=5, precision=prec) as ctx:
        ctx.set_params([M], [10.0], T_star=TS, nu=NU)
        R0 = ctx.modes()
        acc = ctx.step_mc(n)
        R = ctx.modes()
    frac = acc / (B * n * 3 * (M - 1))
    assert 0.45 < frac < 0.65, frac
    assert np.allclose(R[:, :, 0], R0[:, :, 0], rtol=0, atol=1e-12)
    assert np.all(np.isfinite(R))


def test_mc_equilibrium_values_match_mode_dynamics():
    """Q(0) of Sec. V.B for 32-bead chains: <L^2>, <|u_mid|^2> and
    <|r_mid - r_cm|^2> from the sampler and from FP64 mode dynamics at
    dtau = 1 (well below the time steps of Table 1), within 5 %."""
    B, M = 256, 32
    pos = inputs.straight_chains(B, M, B_FAC, seed=11, random_orientation=True)
    q = {}
    with Context(pos, seed=21, precision="fp64") as ctx:
        ctx.set_params([M], [1.0], T_star=TS, nu=NU, sample_every=10)
        ctx.step_mc(2000)
        ctx.accumulators(reset=True)
        ctx.step_mc(4000)
        q["mc"] = ctx.accumulators()[0]
    with Context(pos, seed=22, precision="fp64") as ctx:
        ctx.set_params([M], [1.0], T_star=TS, nu=NU, sample_every=50)
        ctx.step_modes(100000)
        ctx.accumulators(reset=True)
        ctx.step_modes(300000)
        q["dyn"] = ctx.accumulators()[0]
    for key in ("L2", "dmid2", "bond", "bond2"):
        a, b = (q[s][key] / q[s]["n_samples"] for s in ("mc", "dyn"))
        print(f"{key}: MC {a:.5g}  dynamics {b:.5g}  ratio {b / a:.4f}")
        assert abs(b / a - 1) < 0.05, key


def test_coarse_grained_chain_keeps_the_end_to_end_distance():
    """Sec. VI: a 128-bp chain as 129 beads (k = 1) or as 65 beads of two
    basepairs (k = 2) with the parameters of Eq. (x4) (r = 120, y = 12000):
    Monte Carlo <L^2> in units of a^2 agree within 5 %, and both lie within
    10 % of the wormlike-chain value 2 l_p L_c [1 - (l_p/L_c)(1 - e^{-L_c/l_p})]."""
    r, y, B = 120.0, 12000.0, 256
    L2 = {}
    for k, M in ((1, 129), (2, 65)):
        T, nu = _lib.coarse_grain(r, y, k)
        b = 1.0 / (1.0 - 2.0 * nu)
        pos = inputs.straight_chains(B, M, b, seed=30 + k, random_orientation=True)
        with Context(pos, seed=40 + k, precision="fp64") as ctx:
            ctx.set_params([M], [1.0], T_star=T, nu=nu, sample_every=20)
            ctx.step_mc(6000)
            ctx.accumulators(reset=True)
            ctx.step_mc(12000)
            a = ctx.accumulators()[0]
        d = k / b                      # reduced length unit in basepairs
        L2[k] = a["L2"] / a["n_samples"] / B * d * d
    Lc, lp = 128.0, r
    wlc = 2 * lp * Lc * (1 - lp / Lc * (1 - np.exp(-Lc / lp)))
    print(f"<L^2>/a^2: k=1 {L2[1]:.1f}, k=2 {L2[2]:.1f}, wormlike chain {wlc:.1f}")
    assert abs(L2[2] / L2[1] - 1) < 0.05
    for k in (1, 2):
        assert abs(L2[k] / wlc - 1) < 0.10
