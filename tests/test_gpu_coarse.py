"""Sec. VI, Fig. 5 at a reduced size: the end-to-end vector's mean square
displacement against real time of a chain of k = 1 beads per basepair and of
the same chain as dimers (k = 2), each with its parameters of Eq. (x4)
(r = 120, y = 12000) and its time unit of Eq. (g2) (a_k = k a, xi_k = k xi).
64 bp (64 beads, dtau = 10, Table 1) against 32 dimers (32 beads, the time
step giving the same real time per step), 512 chains each, relaxed for
4 / zeta_1 from straight chains, then 4096 samples every 100 steps.  The msd
is 2 (<L.L>(0) - <L.L>(lag)) from the lag correlators, in units of a^2.
The paper shows the two curves on top of each other (full-size run:
bench.py --workload coarse, 5 %); here, with about 4000 independent
samples of L per curve, they must agree within 10 % up to lag 512 samples
(about one relaxation time), and <L^2> within 5 %."""
import numpy as np
import pytest
import torch

from paper_1411_3487_amd import Context, coarse_grain
from paper_1411_3487_amd._lib import coarse_grain_time

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def msd_curve(k, M, dtau, B=512, K=11, nsamp=4096, se=100, prec="bf16x3"):
    T, nu = coarse_grain(120.0, 12000.0, k)
    z1 = 16 * nu * np.sin(np.pi / (2 * M)) ** 4
    relax = int(round(4.0 / z1 / dtau / se)) * se
    with Context(None, seed=8, precision=prec, beads=[M] * B) as ctx:
        ctx.set_params([M], [dtau], T_star=T, nu=nu, sample_every=se, corr_lags=K,
                       use_graphs=True)
        ctx.step_modes(relax)
        ctx.accumulators(reset=True)
        ctx.step_modes(nsamp * se)
        a = ctx.accumulators()[0]
    d2 = (k * (1.0 - 2.0 * nu)) ** 2
    c = a["corr"][:K]
    LL = c[:, 0] / np.maximum(c[:, 3], 1)
    return 2.0 * (LL[0] - LL) * d2, a["L2"] / a["n_samples"] / B * d2


def test_dimerised_chain_follows_the_basepair_chain_in_real_time():
    dtau1 = 10.0
    dtau2 = dtau1 * coarse_grain_time(120.0, 12000.0, 1) / coarse_grain_time(120.0, 12000.0, 2)
    m1, L1 = msd_curve(1, 64, dtau1)
    m2, L2 = msd_curve(2, 32, dtau2)
    ratio = m2[1:] / m1[1:]
    print("msd ratio k=2 / k=1 at lags 1..512 samples:", np.round(ratio, 4))
    print(f"<L^2>/a^2: k=1 {L1:.2f}, k=2 {L2:.2f}")
    assert np.all(np.abs(ratio - 1) < 0.10)
    assert abs(L2 / L1 - 1) < 0.05
    # the msd grows with the lag (the curve is resolved, not noise)
    assert np.all(np.diff(m1[1:]) > 0)
