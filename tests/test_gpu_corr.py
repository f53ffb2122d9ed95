"""Time correlations of Sec. V.B in the accumulators (corr_lags).

Per lag l_j (0, 1, 2, 4, ... samples) the sums over chains and sample pairs
(t, t - l_j) of L(t).L(t - l_j), u_m(t).u_m(t - l_j) and
|d(t) - d(t - l_j)|^2 (d = r_mid - r_cm), and the pair counts.  The FP64 path
is compared with the same sums over the oracle's trajectory, sampled at the
same steps; the fused paths with the FP64 path on the same Philox streams;
replayed graphs with eager runs, bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1411_3487_amd import Context, inputs

pytestmark = pytest.mark.gpu

NU, TS = 0.35, 0.034
B_FAC = 1.0 / (1.0 - 2.0 * NU)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def oracle_corr(pos, M, dtau, se, ns, K, seed):
    R = oracle.modes_from_positions(pos)
    B = pos.shape[0]
    v = []
    for s in range(ns):
        R = oracle.step_modes(R, NU, TS, dtau, se, seed=seed, step0=s * se,
                              chain_ids=np.arange(B))
        o = oracle.chain_observables(oracle.positions_from_modes(R))
        v.append(np.concatenate([o[:, 2:5], o[:, 8:11], o[:, 11:14]], axis=1))
    v = np.array(v)                                   # (ns, B, 9)
    out = np.zeros((K, 4))
    for j in range(K):
        lag = 0 if j == 0 else 2 ** (j - 1)
        if lag >= ns:
            continue
        a, b = v[lag:], v[:ns - lag]
        out[j, 0] = (a[..., 0:3] * b[..., 0:3]).sum()
        out[j, 1] = (a[..., 3:6] * b[..., 3:6]).sum()
        out[j, 2] = ((a[..., 6:9] - b[..., 6:9]) ** 2).sum()
        out[j, 3] = (ns - lag) * B
    return out


def gpu_corr(prec, pos, M, dtau, se, ns, K, seed, graphs=False):
    with Context(pos, seed=seed, precision=prec) as ctx:
        ctx.set_params([M], [dtau], T_star=TS, nu=NU, sample_every=se, corr_lags=K,
                       use_graphs=graphs)
        ctx.step_modes(se * ns)
        return ctx.accumulators()[0]["corr"]


@pytest.mark.parametrize("M", [16, 64])
def test_fp64_correlations_match_oracle(M):
    B, dtau, se, ns, K = 6, 10.0, 5, 70, 8
    pos = inputs.straight_chains(B, M, B_FAC, seed=M + 3, random_orientation=True)
    got = gpu_corr("fp64", pos, M, dtau, se, ns, K, seed=6)
    want = oracle_corr(pos, M, dtau, se, ns, K, seed=6)
    assert np.array_equal(got[:K, 3], want[:, 3])
    assert np.allclose(got[:K, :3], want[:, :3], rtol=1e-9, atol=0)
    assert not np.any(got[K:])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_correlations_match_fp64(prec):
    B, M, dtau, se, ns, K = 40, 64, 10.0, 10, 100, 8
    pos = inputs.straight_chains(B, M, B_FAC, seed=8, random_orientation=True)
    a = gpu_corr("fp64", pos, M, dtau, se, ns, K, seed=9)
    b = gpu_corr(prec, pos, M, dtau, se, ns, K, seed=9, graphs=True)
    assert np.array_equal(a[:, 3], b[:, 3])
    assert np.all(a[0, 2] == 0) and np.all(b[0, 2] == 0)   # |d - d|^2 at lag 0
    rel = np.abs(b[:K, :3] - a[:K, :3]) / np.maximum(np.abs(a[:K, :3]), 1e-300)
    rel[0, 2] = 0.0
    print(prec, rel.max())
    assert rel.max() < 1e-3
