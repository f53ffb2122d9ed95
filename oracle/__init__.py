"""FP64 CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

Plain, slow, obviously-correct reference for the mode-amplitude Langevin step
of Panja, Barkema & van Leeuwen (arXiv:1411.3487), Secs. II–IV, and the
bead-space Euler scheme of Sec. III (Eqs. b3-b5).  The arithmetic lives in
``dm_oracle.c`` (plain C, FP64, OpenMP over chains); this module only
compiles it with gcc and marshals numpy arrays through ctypes.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this package.  The product library never does.

Layout: one chain is a (3, M) float64 array, component-major (x, y, z rows,
bead or mode index along the row); several chains are (B, 3, M).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_i64 = ctypes.c_int64
_p = ctypes.c_void_p

TAG_MODE = 0
TAG_EULER = 1


def build() -> str:
    """Compile dm_oracle.c into liboracle.so with gcc (always rebuilds)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    sig = {
        "orc_philox4x32_10": (None, [_p, _p, _p]),
        "orc_gauss4": (None, [_u64, _u32, _u32, _i64, _u32, _u32, _p]),
        "orc_normal": (_d, [_u64, _u32, _u32, _i64, _u32, _u32]),
        "orc_reduced_params": (None, [_d, _d, _d, _d, _d, _p, _p, _p, _p, _p]),
        "orc_tables": (None, [_i, _d, _d, _d, _p, _p, _p, _p, _p, _p]),
        "orc_modes_from_positions": (None, [_i, _p, _p, _p]),
        "orc_positions_from_modes": (None, [_i, _p, _p, _p]),
        "orc_delta_h": (None, [_i, _d, _p, _p]),
        "orc_step_modes": (None, [_i, _i, _p, _p, _d, _d, _d, _d, _i, _u64, _i64, _i64]),
        "orc_bead_force": (None, [_i, _d, _p, _p]),
        "orc_step_euler": (None, [_i, _i, _p, _p, _d, _d, _d, _d, _u64, _i64, _i64]),
        "orc_energy": (_d, [_i, _d, _p]),
        "orc_set_threads": (None, [_i]),
        "orc_mc_sweeps": (None, [_i, _i, _p, _p, _d, _d, _d, _u64, _i64, _i64, _p]),
        "orc_step_wlc": (None, [_i, _i, _p, _p, _d, _d, _i, _d, _i, _u64, _i64, _i64]),
        "orc_chain_observables": (None, [_i, _p, _p]),
        "orc_config_chains": (None, [_i, _i, _p, _d, _u64, _p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def philox4x32_10(ctr, key) -> np.ndarray:
    """Raw Philox4x32-10 block for a 4-word counter and 2-word key."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gauss4(seed, block, chain, step, comp, tag) -> np.ndarray:
    lib = _load()
    z = np.zeros(4)
    lib.orc_gauss4(seed, block, chain, step, comp, tag, _ptr(z))
    return z


def normal(seed, index, chain, step, comp, tag) -> float:
    return _load().orc_normal(seed, index, chain, step, comp, tag)


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops over chains (timing only)."""
    _load().orc_set_threads(int(n))


def reduced_params(lam, kappa, kT, a, xi) -> dict:
    """Physical (lambda, kappa, kT, a, xi) -> reduced T*, nu, b, d, xi/lambda."""
    lib = _load()
    vals = [ctypes.c_double() for _ in range(5)]
    lib.orc_reduced_params(lam, kappa, kT, a, xi, *[ctypes.addressof(v) for v in vals])
    return dict(zip(["T_star", "nu", "b", "d", "time_unit"], [v.value for v in vals]))


def tables(M: int, nu: float, T_star: float, dtau: float) -> dict:
    """phi (M, M) row-major phi[n, p]; zeta_l, zeta, E, C, W (M,)."""
    lib = _load()
    phi = np.zeros((M, M))
    arrs = [np.zeros(M) for _ in range(5)]
    lib.orc_tables(M, nu, T_star, dtau, _ptr(phi), *[_ptr(a) for a in arrs])
    out = dict(zip(["zeta_l", "zeta", "E", "C", "W"], arrs))
    out["phi"] = phi
    return out


def modes_from_positions(pos: np.ndarray) -> np.ndarray:
    """pos (..., 3, M) -> R (..., 3, M), Eq. (c1)."""
    lib = _load()
    pos = _f64(pos)
    M = pos.shape[-1]
    phi = tables(M, 0.25, 1.0, 1.0)["phi"]
    flat = pos.reshape(-1, 3, M)
    out = np.zeros_like(flat)
    for c in range(flat.shape[0]):
        lib.orc_modes_from_positions(M, _ptr(phi), _ptr(flat[c]), _ptr(out[c]))
    return out.reshape(pos.shape)


def positions_from_modes(R: np.ndarray) -> np.ndarray:
    """R (..., 3, M) -> pos (..., 3, M), all modes, Eq. (c1)."""
    lib = _load()
    R = _f64(R)
    M = R.shape[-1]
    phi = tables(M, 0.25, 1.0, 1.0)["phi"]
    flat = R.reshape(-1, 3, M)
    out = np.zeros_like(flat)
    for c in range(flat.shape[0]):
        lib.orc_positions_from_modes(M, _ptr(phi), _ptr(flat[c]), _ptr(out[c]))
    return out.reshape(R.shape)


def delta_h(R: np.ndarray, nu: float) -> np.ndarray:
    """Delta H_p of Eq. (e11) for one chain's mode amplitudes R (3, M)."""
    lib = _load()
    R = _f64(R)
    M = R.shape[-1]
    out = np.zeros_like(R)
    lib.orc_delta_h(M, nu, _ptr(R), _ptr(out))
    return out


def step_modes(R, nu, T_star, dtau, n_steps, seed=0, step0=0, chain_ids=None,
               gamma_dot=0.0, nonlinear=True) -> np.ndarray:
    """Advance mode amplitudes R (B, 3, M) by n_steps mode steps; returns a copy."""
    lib = _load()
    R = _f64(R).copy()
    B, _, M = R.shape
    ids = np.arange(B, dtype=np.uint32) if chain_ids is None else \
        np.ascontiguousarray(chain_ids, dtype=np.uint32)
    lib.orc_step_modes(M, B, _ptr(ids), _ptr(R), nu, T_star, dtau, gamma_dot,
                       1 if nonlinear else 0, seed, step0, n_steps)
    return R


def bead_force(pos, nu) -> np.ndarray:
    """-dH'/dr_n for one chain (3, M)."""
    lib = _load()
    pos = _f64(pos)
    out = np.zeros_like(pos)
    lib.orc_bead_force(pos.shape[-1], nu, _ptr(pos), _ptr(out))
    return out


def step_euler(pos, nu, T_star, dtau, n_steps, seed=0, step0=0, chain_ids=None,
               gamma_dot=0.0) -> np.ndarray:
    """Advance bead positions (B, 3, M) by n_steps Euler steps; returns a copy."""
    lib = _load()
    pos = _f64(pos).copy()
    B, _, M = pos.shape
    ids = np.arange(B, dtype=np.uint32) if chain_ids is None else \
        np.ascontiguousarray(chain_ids, dtype=np.uint32)
    lib.orc_step_euler(M, B, _ptr(ids), _ptr(pos), nu, T_star, dtau, gamma_dot,
                       seed, step0, n_steps)
    return pos


def step_wlc(pos, T_bar, dt, n_steps, iters=3, seed=0, step0=0, chain_ids=None,
             tol=0.0, midpoint=True) -> np.ndarray:
    """Advance positions (B, 3, M) of unit-bond chains by n_steps steps of the
    nu -> 0 (inextensible) limit, Eqs. (y2)-(y14); returns a copy.  The
    tension cycle runs at most `iters` times, and with tol > 0 stops once a
    cycle changes no bond component by more than tol."""
    lib = _load()
    pos = _f64(pos).copy()
    B, _, M = pos.shape
    ids = np.arange(B, dtype=np.uint32) if chain_ids is None else \
        np.ascontiguousarray(chain_ids, dtype=np.uint32)
    lib.orc_step_wlc(M, B, _ptr(ids), _ptr(pos), T_bar, dt, iters, tol,
                     1 if midpoint else 0, seed, step0, n_steps)
    return pos


def mc_sweeps(R, nu, T_star, scale, n_sweeps, seed=0, step0=0, chain_ids=None):
    """Metropolis sweeps of the mode amplitudes R (B, 3, M) (see
    orc_mc_sweeps); returns (R after the sweeps, accepted proposals per chain)."""
    lib = _load()
    R = _f64(R).copy()
    B, _, M = R.shape
    ids = np.arange(B, dtype=np.uint32) if chain_ids is None else \
        np.ascontiguousarray(chain_ids, dtype=np.uint32)
    acc = np.zeros(B, dtype=np.int64)
    lib.orc_mc_sweeps(M, B, _ptr(ids), _ptr(R), nu, T_star, scale, seed, step0, n_sweeps,
                      _ptr(acc))
    return R, acc


def energy(pos, nu) -> float:
    pos = _f64(pos)
    return _load().orc_energy(pos.shape[-1], nu, _ptr(pos))


def config_chains(M: int, n_chains: int, nu: float, seed: int, chain_ids=None) -> np.ndarray:
    """Initial state of the batched workloads, (B, 3, M): straight chains of
    bond length b = 1/(1 - 2 nu) along a direction uniform on the sphere,
    jittered by 0.01 b per coordinate (Philox tags 5 and 4, step 0)."""
    lib = _load()
    ids = np.arange(n_chains, dtype=np.uint32) if chain_ids is None else \
        np.ascontiguousarray(chain_ids, dtype=np.uint32)
    out = np.zeros((len(ids), 3, M))
    lib.orc_config_chains(M, len(ids), _ptr(ids), 1.0 / (1.0 - 2.0 * nu), seed, _ptr(out))
    return out


OBS_NAMES = ["bond_mean", "L2", "Lx", "Ly", "Lz", "cmx", "cmy", "cmz",
             "umx", "umy", "umz", "dmx", "dmy", "dmz", "xspan", "bond2_mean"]


def chain_observables(pos) -> np.ndarray:
    """Per-chain observables (B, 16) from positions (B, 3, M); see OBS_NAMES."""
    lib = _load()
    pos = _f64(pos)
    flat = pos.reshape(-1, 3, pos.shape[-1])
    out = np.zeros((flat.shape[0], 16))
    for c in range(flat.shape[0]):
        lib.orc_chain_observables(flat.shape[-1], _ptr(flat[c]), _ptr(out[c]))
    return out


TUMBLE_BINS = 32


def tumbles(Lx, Ly, steps):
    """Tumbles of one chain under simple shear (Sec. VIII) from its in-plane
    end-to-end vector (Lx, Ly) sampled at the given steps.

    The paper shows tumbling without defining it; the reading used here: the
    chain points along +x once Lx > |(Lx, Ly)|/2 and along -x once
    Lx < -|(Lx, Ly)|/2, and keeps its previous orientation in between
    (hysteresis, so thermal jitter about the y axis is not counted).  Every
    change of orientation is one tumble (half a turn); a tumbling time is the
    number of steps between two consecutive tumbles.

    Returns (number of tumbles, list of tumbling times in steps)."""
    state, last, n, times = 0, None, 0, []
    for lx, ly, k in zip(Lx, Ly, steps):
        rho = math.sqrt(lx * lx + ly * ly)
        new = 1 if lx > 0.5 * rho else (-1 if lx < -0.5 * rho else state)
        if state != 0 and new != state:
            n += 1
            if last is not None:
                times.append(k - last)
            last = k
        state = new
    return n, times


def tumble_histogram(times) -> np.ndarray:
    """Counts of tumbling times in octaves: bin j holds 2^j <= tau < 2^(j+1)
    steps (the last bin also everything longer)."""
    h = np.zeros(TUMBLE_BINS)
    for t in times:
        h[min(TUMBLE_BINS - 1, int(math.floor(math.log2(t))))] += 1
    return h
