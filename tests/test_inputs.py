"""The seeded input generators: the equilibrium wormlike-chain sampler must
reproduce the closed forms of the discrete wormlike chain (independent bond
angles with density ~ exp(cos(theta) / T-bar))."""
import numpy as np

from paper_1411_3487_amd import inputs


def test_unit_chains_random_directions():
    x = inputs.unit_chains(4000, 5, seed=1)
    u = np.diff(x, axis=2)
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-14)
    assert np.allclose(x[:, :, 0], 0.0)
    # independent uniform directions: <u_n . u_m> = 0, <L^2> = N
    assert abs((u[:, :, 1:] * u[:, :, :-1]).sum(axis=1).mean()) < 0.03
    L = x[:, :, -1]
    assert abs((L * L).sum(axis=1).mean() / 4 - 1) < 0.05


def test_unit_chains_wormlike_closed_forms():
    B, M, T = 20000, 12, 0.1
    x = inputs.unit_chains(B, M, seed=2, T_bar=T)
    u = np.diff(x, axis=2)
    c = 1 / np.tanh(1 / T) - T                 # <cos theta> for density ~ exp(cos / T)
    cs = (u[:, :, 1:] * u[:, :, :-1]).sum(axis=1)
    assert abs(cs.mean() / c - 1) < 1e-3
    # second moment: <cos^2> = 1 - 2 T <cos> for this density
    assert abs((cs * cs).mean() / (1 - 2 * T * c) - 1) < 1e-3
    # bond correlations decay as c^k (independent angles, uniform azimuth)
    for k in (2, 5):
        ck = (u[:, :, k:] * u[:, :, :-k]).sum(axis=1).mean()
        assert abs(ck / c ** k - 1) < 5e-3, k
    N = M - 1
    L2 = N + 2 * sum((N - k) * c ** k for k in range(1, N))
    L = x[:, :, -1]
    assert abs((L * L).sum(axis=1).mean() / L2 - 1) < 5e-3


def test_unit_chains_degenerate_lengths():
    assert inputs.unit_chains(3, 1, seed=0).shape == (3, 3, 1)
    x = inputs.unit_chains(3, 2, seed=0, T_bar=0.05)
    assert np.allclose(np.linalg.norm(x[:, :, 1] - x[:, :, 0], axis=1), 1.0)
