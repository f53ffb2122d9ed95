"""ctypes binding of libdnamodes.so: argument marshalling only.

Every function keeps the C name of include/dnamodes.h; all simulation work
runs in the library's HIP kernels.  The binding raises DMError on any
non-zero status and refuses to run without the compiled library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdnamodes.so")

DM_OK = 0
DM_EINVAL = -1
DM_ENOMEM = -2
DM_EHIP = -3
DM_ENONFINITE = -4
DM_ESTATE = -5

DM_FP64 = 0
DM_FP32 = 1
DM_BF16X3 = 2
PRECISIONS = {"fp64": DM_FP64, "fp32": DM_FP32, "bf16x3": DM_BF16X3}

DM_OBS_CHAIN = 1
DM_OBS_MODES = 2
DM_OBS_ACCUM = 4
DM_OBS_RESET = 8
DM_NCHAIN_OBS = 16
DM_NACC_HEAD = 13
DM_NTUMBLE_BINS = 32
DM_NCORR = 16
CHAIN_OBS_NAMES = ["bond_mean", "L2", "Lx", "Ly", "Lz", "cmx", "cmy", "cmz",
                   "umx", "umy", "umz", "dmx", "dmy", "dmz", "xspan", "bond2_mean"]
ACC_NAMES = ["M", "n_chains", "n_samples", "bond", "bond2", "L2", "msd_cm", "dmid2", "xspan",
             "tumbles", "tau", "tau2", "n_tau"]
DM_NTILING = 9
TILING_NAMES = ["M", "n_chains", "RT", "JC", "resident", "tpw", "items", "item_us", "split"]


class DMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dnamodes error {code}: {msg}")
        self.code = code


class dm_params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("kappa", ctypes.c_double),
                ("kT", ctypes.c_double), ("a", ctypes.c_double), ("xi", ctypes.c_double),
                ("T_star", ctypes.c_double), ("nu", ctypes.c_double),
                ("gamma_dot", ctypes.c_double), ("nonlinear", ctypes.c_int32),
                ("n_lengths", ctypes.c_int32),
                ("lengths", ctypes.POINTER(ctypes.c_int32)),
                ("dt", ctypes.POINTER(ctypes.c_double)),
                ("sample_every", ctypes.c_int32), ("check_finite", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("tiles_per_wg", ctypes.c_int32), ("table_mode", ctypes.c_int32),
                ("corr_lags", ctypes.c_int32)]


EXPORTS = ["dm_init_chains", "dm_set_params", "dm_step_modes", "dm_step_euler", "dm_step_mc",
           "dm_step_wlc",
           "dm_observables", "dm_observables_size", "dm_get_positions", "dm_get_modes",
           "dm_save_state", "dm_load_state", "dm_get_step", "dm_get_tiling",
           "dm_tuning_report", "dm_coarse_grain", "dm_coarse_grain_time", "dm_sync", "dm_destroy",
           "dm_last_error", "dm_step_modes_f64_static"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: run paper_1411_3487_amd/build.py "
                          "(the HIP library is required; there is no fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                             ctypes.c_uint64, ctypes.c_size_t)
    sigs = {
        "dm_init_chains": ([ctypes.POINTER(vp), i32, vp, vp, u64, i32, vp], ctypes.c_int),
        "dm_set_params": ([vp, ctypes.POINTER(dm_params)], ctypes.c_int),
        "dm_step_modes": ([vp, i64], ctypes.c_int),
        "dm_step_euler": ([vp, i64, ctypes.c_double], ctypes.c_int),
        "dm_step_mc": ([vp, i64, ctypes.c_double, ctypes.POINTER(i64)], ctypes.c_int),
        "dm_step_wlc": ([vp, i64, ctypes.c_double, ctypes.c_double, i32, ctypes.c_double, i32],
                        ctypes.c_int),
        "dm_observables": ([vp, i32, vp, sz], ctypes.c_int),
        "dm_observables_size": ([vp, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "dm_get_positions": ([vp, vp, i32], ctypes.c_int),
        "dm_get_modes": ([vp, vp], ctypes.c_int),
        "dm_save_state": ([vp, vp, ctypes.POINTER(sz)], ctypes.c_int),
        "dm_load_state": ([vp, vp, sz], ctypes.c_int),
        "dm_get_step": ([vp, ctypes.POINTER(i64)], ctypes.c_int),
        "dm_get_tiling": ([vp, vp, sz, ctypes.POINTER(i32)], ctypes.c_int),
        "dm_tuning_report": ([vp], ctypes.c_char_p),
        "dm_coarse_grain_time": ([ctypes.c_double, ctypes.c_double, i32,
                                  ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "dm_coarse_grain": ([ctypes.c_double, ctypes.c_double, i32, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "dm_sync": ([vp], ctypes.c_int),
        "dm_destroy": ([vp], ctypes.c_int),
        "dm_last_error": ([vp], ctypes.c_char_p),
        "dm_step_modes_f64_static": ([vp, i32, i32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, i32, u64,
                                      ctypes.c_uint32, i64, i64, vp], ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def coarse_grain(r: float, y: float, k: int):
    """(T*_k, nu_k) of a chain with one bead per k basepairs (dm_coarse_grain)."""
    lib = load()
    t, n = ctypes.c_double(), ctypes.c_double()
    rc = lib.dm_coarse_grain(r, y, k, ctypes.byref(t), ctypes.byref(n))
    if rc != DM_OK:
        raise DMError(rc, lib.dm_last_error(None).decode())
    return t.value, n.value


def coarse_grain_time(r: float, y: float, k: int) -> float:
    """Time unit c_k of that chain in units of a^2 xi / kT (dm_coarse_grain_time)."""
    lib = load()
    c = ctypes.c_double()
    rc = lib.dm_coarse_grain_time(r, y, k, ctypes.byref(c))
    if rc != DM_OK:
        raise DMError(rc, lib.dm_last_error(None).decode())
    return c.value


class Context:
    """One dm_ctx: a batch of chains on the current HIP device.

    pos0 is a list of (3, M_c) arrays, or a (B, 3, M) array for equal lengths,
    in units of d; or None with ``beads`` (chain lengths): then the library
    builds its own initial state at the first set_params (see dm_init_chains).  stream is a torch.cuda.Stream (or None for the null stream).
    """

    def __init__(self, pos0, seed: int = 0, precision="fp64", stream=None, beads=None):
        self.lib = load()
        if pos0 is None:
            # the library builds the initial state at the first set_params
            self.beads = np.ascontiguousarray(beads, dtype=np.int32)
            chains, flat = range(len(self.beads)), None
        else:
            if isinstance(pos0, np.ndarray) and pos0.ndim == 3:
                chains = [pos0[i] for i in range(pos0.shape[0])]
            else:
                chains = list(pos0)
            self.beads = np.array([c.shape[-1] for c in chains], dtype=np.int32)
            flat = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float64).ravel()
                                                        for c in chains]))
        self.offsets = np.concatenate([[0], np.cumsum(3 * self.beads.astype(np.int64))])
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.precision = prec
        self._stream = stream
        sptr = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        h = ctypes.c_void_p()
        rc = self.lib.dm_init_chains(ctypes.byref(h), len(chains), self.beads.ctypes.data,
                                     None if flat is None else flat.ctypes.data, seed, prec,
                                     sptr)
        if rc != DM_OK:
            raise DMError(rc, self.lib.dm_last_error(None).decode())
        self.h = h

    # ------------------------------------------------------------------ utils
    def _check(self, rc):
        if rc != DM_OK:
            raise DMError(rc, self.lib.dm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ API
    def set_params(self, lengths, dt, T_star=None, nu=None, gamma_dot=0.0, nonlinear=True,
                   sample_every=0, check_finite=False, physical=None, autotune=False,
                   use_graphs=False, tiles_per_wg=0, table_mode=0, corr_lags=0):
        """Reduced units by default; physical=dict(lambda_, kappa, kT, a, xi)."""
        p = dm_params()
        if physical:
            for k, v in physical.items():
                setattr(p, k, v)
        else:
            p.T_star, p.nu = T_star, nu
        lens = np.ascontiguousarray(lengths, dtype=np.int32)
        dts = np.ascontiguousarray(dt, dtype=np.float64)
        p.gamma_dot = gamma_dot
        p.nonlinear = 1 if nonlinear else 0
        p.n_lengths = len(lens)
        p.lengths = lens.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        p.dt = dts.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.sample_every = sample_every
        p.check_finite = 1 if check_finite else 0
        p.autotune = 1 if autotune else 0
        p.use_graphs = 1 if use_graphs else 0
        p.tiles_per_wg = tiles_per_wg
        p.corr_lags = corr_lags
        p.table_mode = {"auto": 0, "resident": 1, "streamed": 2, "split": 3,
                        "split8": 4}.get(table_mode, table_mode)
        self._check(self.lib.dm_set_params(self.h, ctypes.byref(p)))

    def tiling(self) -> list:
        """Per length bucket: dict of the fused launch's tile shape."""
        nb = ctypes.c_int32()
        self._check(self.lib.dm_get_tiling(self.h, None, 0, ctypes.byref(nb)))
        out = np.zeros(DM_NTILING * nb.value)
        self._check(self.lib.dm_get_tiling(self.h, out.ctypes.data, out.size, ctypes.byref(nb)))
        return [dict(zip(TILING_NAMES, out[i * DM_NTILING:(i + 1) * DM_NTILING]))
                for i in range(nb.value)]

    def tuning_report(self) -> str:
        return self.lib.dm_tuning_report(self.h).decode()

    def step_modes(self, n_steps: int):
        self._check(self.lib.dm_step_modes(self.h, n_steps))

    def step_euler(self, n_steps: int, dtau: float):
        self._check(self.lib.dm_step_euler(self.h, n_steps, dtau))

    def step_wlc(self, n_steps: int, dt_bar: float, T_bar: float, iters: int = 8,
                 tol: float = 0.0, midpoint: bool = True):
        self._check(self.lib.dm_step_wlc(self.h, n_steps, dt_bar, T_bar, iters, tol,
                                         1 if midpoint else 0))

    def step_mc(self, n_sweeps: int, step_scale: float = 3.0) -> int:
        """Metropolis sweeps; returns the number of accepted proposals."""
        acc = ctypes.c_int64()
        self._check(self.lib.dm_step_mc(self.h, n_sweeps, step_scale, ctypes.byref(acc)))
        return acc.value

    def observables_size(self, which: int) -> int:
        n = ctypes.c_size_t()
        self._check(self.lib.dm_observables_size(self.h, which, ctypes.byref(n)))
        return n.value

    def observables(self, which: int) -> np.ndarray:
        out = np.zeros(self.observables_size(which))
        self._check(self.lib.dm_observables(self.h, which, out.ctypes.data, out.size))
        return out

    def chain_observables(self) -> np.ndarray:
        return self.observables(DM_OBS_CHAIN).reshape(-1, DM_NCHAIN_OBS)

    def accumulators(self, reset=False) -> list:
        """Per length bucket: dict of the head sums, 'modes' (sum |R_p|^2) and
        'tumble_hist' (counts of tumbling times in octaves of steps) and 'corr'
        (DM_NCORR x 4: per lag 0, 1, 2, 4, ... samples the sums of L.L', u_m.u_m',
        |d - d'|^2 and the pair count)."""
        flat = self.observables(DM_OBS_ACCUM | (DM_OBS_RESET if reset else 0))
        out, i = [], 0
        while i < flat.size:
            M = int(flat[i])
            d = dict(zip(ACC_NAMES, flat[i:i + DM_NACC_HEAD]))
            j = i + DM_NACC_HEAD
            d["modes"] = flat[j:j + M].copy()
            d["tumble_hist"] = flat[j + M:j + M + DM_NTUMBLE_BINS].copy()
            c0 = j + M + DM_NTUMBLE_BINS
            d["corr"] = flat[c0:c0 + 4 * DM_NCORR].reshape(DM_NCORR, 4).copy()
            out.append(d)
            i = c0 + 4 * DM_NCORR
        return out

    def _split(self, flat):
        chains = [flat[self.offsets[c]:self.offsets[c + 1]].reshape(3, -1)
                  for c in range(len(self.beads))]
        if np.all(self.beads == self.beads[0]):
            return np.stack(chains)
        return chains

    def positions(self):
        out = np.zeros(int(self.offsets[-1]))
        self._check(self.lib.dm_get_positions(self.h, out.ctypes.data, 0))
        return self._split(out)

    def positions_to_device(self, dst_ptr: int):
        self._check(self.lib.dm_get_positions(self.h, ctypes.c_void_p(dst_ptr), 1))

    def modes(self):
        out = np.zeros(int(self.offsets[-1]))
        self._check(self.lib.dm_get_modes(self.h, out.ctypes.data))
        return self._split(out)

    def save_state(self) -> bytes:
        n = ctypes.c_size_t()
        self._check(self.lib.dm_save_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.lib.dm_save_state(self.h, buf, ctypes.byref(n)))
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.dm_load_state(self.h, buf, len(blob)))

    @property
    def step(self) -> int:
        k = ctypes.c_int64()
        self._check(self.lib.dm_get_step(self.h, ctypes.byref(k)))
        return k.value

    def sync(self):
        self._check(self.lib.dm_sync(self.h))
