"""The allocation-free FP64 mode step (dm_step_modes_f64_static), called
through the C ABI on caller-owned device amplitudes, against the context's
dm_step_modes on the same chains and Philox streams: two calls in a row, the
second with a smaller input (fewer chains of an odd length, from chain index
3, with shear, split over two calls at consecutive steps).  The step's
tables are built on the device, so the bar is that of the FP64 plain form
against the oracle: 1e-10 relative."""
import numpy as np
import pytest
import torch

from paper_1411_3487_amd import Context, inputs, _lib

pytestmark = pytest.mark.gpu

NU, TS = 0.35, 0.034
B_FAC = 1.0 / (1.0 - 2.0 * NU)
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def static_step(R_dev, B, M, dtau, seed, chain0, step0, n, gdot=0.0, nonlinear=True):
    lib = _lib.load()
    stream = torch.cuda.current_stream()
    rc = lib.dm_step_modes_f64_static(R_dev.data_ptr(), B, M, TS, NU, dtau, gdot,
                                      1 if nonlinear else 0, seed, chain0, step0, n,
                                      stream.cuda_stream)
    assert rc == _lib.DM_OK, lib.dm_last_error(None).decode()


def context_run(pos, M, dtau, seed, n, gdot=0.0):
    with Context(pos, seed=seed, precision="fp64") as ctx:
        ctx.set_params([M], [dtau], T_star=TS, nu=NU, gamma_dot=gdot)
        R0 = ctx.modes()
        ctx.step_modes(n)
        return R0, ctx.modes()


def rel(got, want):
    """Largest difference of the internal modes (p >= 1) and of the centre of
    mass mode, each relative to its own largest magnitude."""
    internal = np.abs(got[..., 1:] - want[..., 1:]).max() / np.abs(want[..., 1:]).max()
    com = np.abs(got[..., 0] - want[..., 0]).max() / np.abs(want[..., 0]).max()
    return max(internal, com)


def test_static_step_matches_the_context_on_two_calls():
    B, M, dtau, n = 512, 256, 100.0, 200
    pos = inputs.straight_chains(B, M, B_FAC, seed=1, random_orientation=True)
    R0, want = context_run(pos, M, dtau, 7, n)
    R = torch.tensor(R0, dtype=torch.float64, device="cuda").contiguous()
    print(f"call 1: {B} x {M}, {n} steps", flush=True)
    static_step(R, B, M, dtau, 7, 0, 0, n)
    torch.cuda.synchronize()
    err = rel(R.cpu().numpy(), want)
    print(f"call 1: rel err {err:.2e}")
    assert err < TOL

    # second, smaller input: chains 3..9 of a 10-chain ensemble of 63 beads
    # (odd length: the other update kernel), shear on, in two calls
    B2, M2, dtau2, gdot = 10, 63, 10.0, 1e-3
    pos2 = inputs.straight_chains(B2, M2, B_FAC, seed=2, random_orientation=True)
    R0b, wantb = context_run(pos2, M2, dtau2, 9, 300, gdot=gdot)
    R2 = torch.tensor(R0b[3:], dtype=torch.float64, device="cuda").contiguous()
    print(f"call 2: {B2 - 3} x {M2}, 120 + 180 steps", flush=True)
    static_step(R2, B2 - 3, M2, dtau2, 9, 3, 0, 120, gdot=gdot)
    static_step(R2, B2 - 3, M2, dtau2, 9, 3, 120, 180, gdot=gdot)
    torch.cuda.synchronize()
    err = rel(R2.cpu().numpy(), wantb[3:])
    print(f"call 2: rel err {err:.2e}")
    assert err < TOL


def test_static_step_rejects_sizes_beyond_the_array():
    lib = _lib.load()
    R = torch.zeros(8, dtype=torch.float64, device="cuda")
    rc = lib.dm_step_modes_f64_static(R.data_ptr(), 100000, 256, TS, NU, 100.0, 0.0, 1, 0, 0,
                                      0, 1, torch.cuda.current_stream().cuda_stream)
    assert rc == _lib.DM_EINVAL
    assert b"DM_STATIC_SCRATCH_BYTES" in lib.dm_last_error(None)
