"""Seeded synthetic inputs shared by the tests, the bench and the smoke run.

This module holds none of the method's arithmetic: it only draws initial
conformations and chain lengths with numpy's default generator, so that the
HIP library and the CPU oracle can be started from identical inputs.

Recipe (the paper's workloads are single dsDNA chains of 64-512 basepairs,
one bead per basepair, Sec. II.A and Sec. V.B):
  * a chain of M beads starts straight, with consecutive beads ``spacing``
    apart (the mean bond length a = b d, i.e. b in reduced units), along x
    or along a direction drawn uniformly on the unit sphere;
  * every bead coordinate gets Gaussian jitter of standard deviation
    ``jitter * spacing`` (0.01 a by default);
  * uneven ensembles draw each chain's length uniformly from a list.
"""
from __future__ import annotations

import numpy as np


def straight_chains(n_chains: int, M: int, spacing: float, seed: int,
                    random_orientation: bool = True,
                    jitter: float = 0.01) -> np.ndarray:
    """Positions (n_chains, 3, M) float64 in units of d."""
    rng = np.random.default_rng(seed)
    if random_orientation:
        cos_t = rng.uniform(-1.0, 1.0, n_chains)
        ang = rng.uniform(0.0, 2.0 * np.pi, n_chains)
        sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
        e = np.stack([sin_t * np.cos(ang), sin_t * np.sin(ang), cos_t], axis=1)
    else:
        e = np.tile(np.array([1.0, 0.0, 0.0]), (n_chains, 1))
    n = np.arange(M, dtype=np.float64) * spacing
    pos = e[:, :, None] * n[None, None, :]
    pos += jitter * spacing * rng.standard_normal((n_chains, 3, M))
    return pos


def mixed_lengths(n_chains: int, lengths, seed: int) -> np.ndarray:
    """Chain lengths (beads) drawn uniformly from ``lengths``, int32."""
    rng = np.random.default_rng(seed)
    lengths = np.asarray(lengths, dtype=np.int32)
    return lengths[rng.integers(0, len(lengths), n_chains)].astype(np.int32)


def mixed_chains(beads: np.ndarray, spacing: float, seed: int,
                 jitter: float = 0.01) -> list:
    """One (3, M_c) array per chain for an uneven ensemble."""
    rng = np.random.default_rng(seed + 1000003)
    out = []
    for M in beads:
        cos_t = rng.uniform(-1.0, 1.0)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        sin_t = np.sqrt(max(0.0, 1.0 - cos_t * cos_t))
        e = np.array([sin_t * np.cos(ang), sin_t * np.sin(ang), cos_t])
        n = np.arange(int(M), dtype=np.float64) * spacing
        p = e[:, None] * n[None, :] + jitter * spacing * rng.standard_normal((3, int(M)))
        out.append(p)
    return out


def unit_chains(n_chains: int, M: int, seed: int, T_bar: float | None = None) -> np.ndarray:
    """Chains of M beads joined by unit bonds, (n_chains, 3, M), first bead at
    the origin.  With T_bar None the bond directions are independent and
    uniform; otherwise the chain is a discrete wormlike chain in equilibrium
    at reduced temperature T_bar: each bond angle to the previous bond is
    independent with density ~ exp(cos(theta) / T_bar), sampled by inverting
    its distribution in cos(theta), and the azimuth is uniform."""
    if M < 2:
        return np.zeros((n_chains, 3, M))
    rng = np.random.default_rng(seed)
    u = np.zeros((n_chains, 3, M - 1))
    v = rng.standard_normal((n_chains, 3))
    u[:, :, 0] = v / np.linalg.norm(v, axis=1, keepdims=True)
    for n in range(1, M - 1):
        if T_bar is None:
            v = rng.standard_normal((n_chains, 3))
            u[:, :, n] = v / np.linalg.norm(v, axis=1, keepdims=True)
            continue
        x = rng.random(n_chains)
        ct = 1 + T_bar * np.log(x + (1 - x) * np.exp(-2 / T_bar))
        ph = 2 * np.pi * rng.random(n_chains)
        p = u[:, :, n - 1]
        a = np.where(np.abs(p[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
        e1 = np.cross(p, a)
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(p, e1)
        st = np.sqrt(np.maximum(0, 1 - ct ** 2))
        u[:, :, n] = ct[:, None] * p + st[:, None] * (np.cos(ph)[:, None] * e1 +
                                                      np.sin(ph)[:, None] * e2)
    pos = np.zeros((n_chains, 3, M))
    pos[:, :, 1:] = np.cumsum(u, axis=2)
    return pos
