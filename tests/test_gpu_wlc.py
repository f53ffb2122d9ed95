"""The nu -> 0 (inextensible wormlike chain) limit on the GPU, dm_step_wlc,
against the oracle on identical Philox streams (FP64 both: trajectories agree
to rounding; the cyclic-reduction tension solve rounds differently from the
oracle's Thomas sweep, by ~1e-15 relative), and the unit bond lengths it
maintains."""
import numpy as np
import pytest
import torch

import oracle
from paper_1411_3487_amd import Context
from paper_1411_3487_amd.inputs import unit_chains

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("midpoint", [True, False])
@pytest.mark.parametrize("M", [2, 3, 17, 64, 65, 66, 100, 341, 342])
def test_wlc_matches_oracle(M, midpoint):
    """Up to M = 64 one wavefront per chain with the chain in registers (bond
    n in lane n); up to M = 341 one wavefront per chain with the chain in LDS
    (several bonds per lane from M = 66); both solve for the tensions by
    cyclic reduction.  From M = 342 one thread per chain runs the Thomas
    sweep.  Both forms of the cycle: forces at the midpoint bonds and at
    the bonds of the start of the step."""
    B, T, dt, n = 7, 0.2, 2e-3, 150
    pos = unit_chains(B, M, M)
    with Context(pos, seed=12, precision="fp64") as ctx:
        ctx.step_wlc(n, dt, T, iters=8, midpoint=midpoint)
        got = ctx.positions()
    want = oracle.step_wlc(pos, T, dt, n, iters=8, seed=12, midpoint=midpoint)
    err = np.abs(got - want).max() / max(1.0, M - 1)
    print(f"M={M}: max |dr| / (M-1) = {err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("M", [64, 100, 342])
def test_wlc_converged_cycles_match_oracle(M):
    """The cycle stopped at convergence (tol 1e-12, at most 16 passes) on both
    sides: a pass count that differs near the threshold moves a bond by at
    most ~tol, far inside the parity bound."""
    B, T, dt, n = 9, 1.0 / 114.4, 1e-3, 200
    pos = unit_chains(B, M, 3 * M, T_bar=T)
    with Context(pos, seed=4, precision="fp64") as ctx:
        ctx.step_wlc(n, dt, T, iters=16, tol=1e-12)
        got = ctx.positions()
    want = oracle.step_wlc(pos, T, dt, n, iters=16, seed=4, tol=1e-12)
    err = np.abs(got - want).max() / max(1.0, M - 1)
    print(f"M={M}: max |dr| / (M-1) = {err:.2e}")
    assert err < 1e-10


def test_wlc_unit_bonds_and_fused_context():
    B, M = 20, 64
    pos = unit_chains(B, M, 5, T_bar=0.05)
    with Context(pos * 3.0, seed=3, precision="bf16x3") as ctx:   # bonds rescaled
        ctx.step_wlc(500, 1e-4, 0.05, iters=8)
        x = ctx.positions()
    ell = np.linalg.norm(np.diff(x, axis=2), axis=1)
    assert np.abs(ell - 1).max() < 1e-5          # FP32 state after the call
