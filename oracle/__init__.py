"""CPU oracle for PTHR on the 3D Gaussian Edwards-Anderson model.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  The C
sources here (``pthr_oracle.c``, ``exact_enum.c``) share no code with the GPU
library under ``paper_2605_25872_amd/``.

``Oracle`` wraps the plain sequential reference of one elementary Monte Carlo
step (paper Sec. 3); ``exact_enumerate`` wraps the brute-force enumeration of
L=2 and L=3 lattices that pins it (paper Sec. 2, Eqs. 1-4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_ORACLE = os.path.join(HERE, "liboracle.so")
LIB_EXACT = os.path.join(HERE, "libexact.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]

FP64, FP32 = 0, 1
ACU, SINGLE_NEG = 0, 1
SWEEP_PT, SWEEP_ER = 1, 2
METROPOLIS, HEAT_BATH, MICSA = 0, 1, 2
NOBS = 6
OBS_NAMES = ("e", "e2", "q2", "q4", "ql", "sdy")


def build() -> None:
    """Compile both oracle libraries with gcc (always recompiles)."""
    for src, out in (("pthr_oracle.c", LIB_ORACLE), ("exact_enum.c", LIB_EXACT)):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, os.path.join(HERE, src), "-o", tmp, "-lm"])
        os.replace(tmp, out)


_libs: dict[str, ctypes.CDLL] = {}


def _load(path: str) -> ctypes.CDLL:
    if path not in _libs:
        if not os.path.exists(path):
            build()
        _libs[path] = ctypes.CDLL(path)
    return _libs[path]


class OracleParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("first_sample", ctypes.c_int32), ("n_replicas", ctypes.c_int32),
                ("n_temps", ctypes.c_int32), ("n_reservoir", ctypes.c_int32),
                ("sweeps_per_emcs", ctypes.c_int32), ("er_sweeps_per_emcs", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("houdayer_mode", ctypes.c_int32),
                ("t_acu", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("local_update", ctypes.c_int32), ("micsa_refresh", ctypes.c_int32)]


def _lib() -> ctypes.CDLL:
    lib = _load(LIB_ORACLE)
    if getattr(lib, "_typed", False):
        return lib
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.oracle_create.restype = vp
    lib.oracle_create.argtypes = [ctypes.POINTER(OracleParams), ctypes.c_char_p, ctypes.c_size_t]
    lib.oracle_destroy.argtypes = [vp]
    lib.oracle_init_samples.argtypes = [vp, vp, vp]
    lib.oracle_sweep.argtypes = [vp, i32, i32]
    lib.oracle_houdayer.argtypes = [vp]
    lib.oracle_pt_swap.argtypes = [vp, i32]
    lib.oracle_measure.argtypes = [vp, vp, vp, vp]
    lib.oracle_run.argtypes = [vp, i64, vp, vp, vp]
    lib.oracle_cluster_labels.argtypes = [vp, i32, i32, i32, vp]
    for name in ("oracle_spins", "oracle_clone_at", "oracle_er_head", "oracle_pt_last",
                 "oracle_pt_count", "oracle_pt_energy", "oracle_rt_state", "oracle_rt_count",
                 "oracle_walker"):
        getattr(lib, name).restype = vp
        getattr(lib, name).argtypes = [vp]
    lib.oracle_t.restype = i64
    lib.oracle_t.argtypes = [vp]
    lib.oracle_m.argtypes = [vp, i32]
    lib.oracle_philox4x32_10.argtypes = [vp, vp, vp]
    lib.oracle_pexp.restype = ctypes.c_double
    lib.oracle_pexp.argtypes = [ctypes.c_double]
    lib.oracle_plog.restype = ctypes.c_double
    lib.oracle_plog.argtypes = [ctypes.c_double]
    lib.oracle_uniform53.restype = ctypes.c_double
    lib.oracle_uniform53.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_uniform32.restype = ctypes.c_float
    lib.oracle_uniform32.argtypes = [ctypes.c_uint32]
    lib.oracle_pexp2_32.restype = ctypes.c_float
    lib.oracle_pexp2_32.argtypes = [ctypes.c_float]
    lib.oracle_pexp2_32_coef.restype = ctypes.c_float
    lib.oracle_pexp2_32_coef.argtypes = [ctypes.c_int]
    lib.oracle_heat_bath_flip.restype = i32
    lib.oracle_heat_bath_flip.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.oracle_heat_bath_flip32.restype = i32
    lib.oracle_heat_bath_flip32.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_float]
    lib.oracle_round_trip_step.restype = i32
    lib.oracle_round_trip_step.argtypes = [vp, vp, i32]
    lib.oracle_energy.restype = ctypes.c_double
    lib.oracle_energy.argtypes = [vp, i32, i32]
    lib.oracle_delta_e.restype = ctypes.c_double
    lib.oracle_delta_e.argtypes = [vp, i32, i32, i32]
    lib._typed = True
    return lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def pexp(x: float) -> float:
    return float(_lib().oracle_pexp(float(x)))


def plog(u: float) -> float:
    """ln(u) for 0 < u <= 1, the routine the MicSA walker refresh uses."""
    return float(_lib().oracle_plog(float(u)))


def uniform53(lo: int, hi: int) -> float:
    return float(_lib().oracle_uniform53(lo, hi))


def uniform32(w: int) -> np.float32:
    return np.float32(_lib().oracle_uniform32(w))


def pexp2_32(t: float) -> np.float32:
    """FP32 form of the Metropolis exponential: 2^t (IEEE overflow to +inf,
    gradual underflow to 0)."""
    return np.float32(_lib().oracle_pexp2_32(float(np.float32(t))))


def pexp2_32_coefficients() -> list[float]:
    """Coefficients c0..c6 of the polynomial pexp2_32 evaluates for 2^f."""
    return [float(_lib().oracle_pexp2_32_coef(n)) for n in range(7)]


def heat_bath_flip(u: float, a: float, dE: float, fp32: bool = False) -> bool:
    """Heat-bath test given a = exp(-beta |dE|) (FP32 form if fp32)."""
    if fp32:
        return bool(_lib().oracle_heat_bath_flip32(float(np.float32(u)), float(np.float32(a)),
                                                   float(np.float32(dE))))
    return bool(_lib().oracle_heat_bath_flip(float(u), float(a), float(dE)))


def round_trip_step(rt_state: np.ndarray, at: np.ndarray) -> int:
    """Round-trip bookkeeping of one replica group after its PT step (updates
    rt_state, uint8 indexed by clone, in place); returns the trips completed."""
    assert rt_state.dtype == np.uint8 and rt_state.flags["C_CONTIGUOUS"]
    a = np.ascontiguousarray(at, dtype=np.int32)
    return int(_lib().oracle_round_trip_step(_ptr(rt_state), _ptr(a), len(a)))


class Observables:
    """Accumulators filled by ``measure``: acc [S][N_T][6] (sum e, e^2, q^2, q^4,
    q_l, S), the pooled overlap histogram hist [N_T][V+1] and the count."""

    def __init__(self, n_samples: int, n_temps: int, V: int):
        self.acc = np.zeros((n_samples, n_temps, NOBS), dtype=np.float64)
        self.hist = np.zeros((n_temps, V + 1), dtype=np.uint64)
        self.n_meas = np.zeros(1, dtype=np.uint64)


class Oracle:
    """Plain sequential PTHR over ``n_samples`` samples (global ids start at
    ``first_sample``), following paper Sec. 3 step by step."""

    def __init__(self, L, n_samples=1, n_replicas=2, n_temps=8, n_reservoir=0,
                 sweeps_per_emcs=10, er_sweeps_per_emcs=240, precision=FP64,
                 houdayer_mode=ACU, t_acu=1.0, seed=1, first_sample=0, local_update=METROPOLIS,
                 micsa_refresh=0):
        self.lib = _lib()
        self.params = OracleParams(L, n_samples, first_sample, n_replicas, n_temps, n_reservoir,
                                   sweeps_per_emcs, er_sweeps_per_emcs, precision, houdayer_mode,
                                   t_acu, seed, local_update, micsa_refresh)
        err = ctypes.create_string_buffer(256)
        self.ctx = self.lib.oracle_create(ctypes.byref(self.params), err, 256)
        if not self.ctx:
            raise ValueError(err.value.decode())
        self.L, self.S, self.NR, self.NT = L, n_samples, n_replicas, n_temps
        self.NER = n_reservoir
        self.V = L ** 3
        self.NPT = n_replicas * n_temps
        self.C = self.NPT + n_replicas * n_reservoir
        self._J = None

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            self.lib.oracle_destroy(ctx)
            self.ctx = None

    def _check(self, rc: int, what: str) -> None:
        if rc != 0:
            raise RuntimeError(f"oracle {what} failed ({rc})")

    def init(self, J: np.ndarray, T: np.ndarray) -> None:
        self._J = np.ascontiguousarray(J, dtype=np.float64).reshape(self.S, 3, self.V)
        self._T = np.ascontiguousarray(T, dtype=np.float64)
        self._check(self.lib.oracle_init_samples(self.ctx, _ptr(self._J), _ptr(self._T)), "init")

    def sweep(self, n: int, which: int = SWEEP_PT | SWEEP_ER) -> None:
        self._check(self.lib.oracle_sweep(self.ctx, n, which), "sweep")

    def houdayer(self) -> None:
        self._check(self.lib.oracle_houdayer(self.ctx), "houdayer")

    def pt_swap(self, do_reservoir: bool = True) -> None:
        self._check(self.lib.oracle_pt_swap(self.ctx, int(do_reservoir)), "pt_swap")

    def new_observables(self) -> Observables:
        return Observables(self.S, self.NT, self.V)

    def measure(self, obs: Observables) -> None:
        self._check(self.lib.oracle_measure(self.ctx, _ptr(obs.acc), _ptr(obs.hist),
                                            _ptr(obs.n_meas)), "measure")

    def run(self, n_emcs: int, obs: Observables | None = None) -> None:
        if obs is None:
            rc = self.lib.oracle_run(self.ctx, n_emcs, None, None, None)
        else:
            rc = self.lib.oracle_run(self.ctx, n_emcs, _ptr(obs.acc), _ptr(obs.hist),
                                     _ptr(obs.n_meas))
        self._check(rc, "run")

    def emcs(self, obs: Observables | None = None) -> None:
        """One EMCS through the step-wise calls (same bits as ``run(1)``)."""
        self.sweep(self.params.sweeps_per_emcs, SWEEP_PT)
        if self.NER:
            self.sweep(self.params.er_sweeps_per_emcs, SWEEP_ER)
        self.houdayer()
        self.pt_swap(True)
        if obs is not None:
            self.measure(obs)

    def _view(self, fn, dtype, shape):
        addr = getattr(self.lib, fn)(self.ctx)
        n = int(np.prod(shape))
        buf = (ctypes.c_char * (n * np.dtype(dtype).itemsize)).from_address(addr)
        return np.frombuffer(buf, dtype=dtype, count=n).reshape(shape)

    @property
    def spins(self) -> np.ndarray:
        return self._view("oracle_spins", np.int8, (self.S, self.C, self.V))

    @property
    def clone_at(self) -> np.ndarray:
        return self._view("oracle_clone_at", np.int32, (self.S, self.NR, self.NT))

    @property
    def er_head(self) -> np.ndarray:
        return self._view("oracle_er_head", np.int32, (self.S, self.NR))

    @property
    def pt_last(self) -> np.ndarray:
        return self._view("oracle_pt_last", np.uint8, (self.S, self.NR, self.NT - 1))

    @property
    def pt_count(self) -> np.ndarray:
        return self._view("oracle_pt_count", np.uint32, (self.S, self.NR, self.NT - 1))

    @property
    def pt_energy(self) -> np.ndarray:
        return self._view("oracle_pt_energy", np.float64, (self.S, self.NPT))

    @property
    def walker(self) -> np.ndarray:
        """MicSA walker energy of every PT clone, [S][N_r*N_T] (writable view)."""
        return self._view("oracle_walker", np.float64, (self.S, self.NPT))

    @property
    def rt_state(self) -> np.ndarray:
        return self._view("oracle_rt_state", np.uint8, (self.S, self.NPT))

    @property
    def rt_count(self) -> np.ndarray:
        return self._view("oracle_rt_count", np.uint64, (self.S,))

    @property
    def t(self) -> int:
        return int(self.lib.oracle_t(self.ctx))

    def m(self, cls: int) -> int:
        return int(self.lib.oracle_m(self.ctx, cls))

    def labels(self, s: int, p: int, k: int) -> np.ndarray:
        out = np.zeros(self.V, dtype=np.int32)
        self._check(self.lib.oracle_cluster_labels(self.ctx, s, p, k, _ptr(out)), "labels")
        return out

    def energy(self, s: int, clone: int) -> float:
        return float(self.lib.oracle_energy(self.ctx, s, clone))

    def delta_e(self, s: int, clone: int, site: int) -> float:
        return float(self.lib.oracle_delta_e(self.ctx, s, clone, site))


def exact_enumerate(L: int, J: np.ndarray, betas) -> dict:
    """Exact <H>/V, <(H/V)^2>, <q_l> and P(Q) for one sample of size L=2 or 3."""
    lib = _load(LIB_EXACT)
    vp = ctypes.c_void_p
    lib.exact_enumerate.argtypes = [ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, vp, vp]
    V = L ** 3
    Jc = np.ascontiguousarray(J, dtype=np.float64).reshape(3, V)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    nb = len(b)
    e = np.zeros(nb)
    e2 = np.zeros(nb)
    ql = np.zeros(nb)
    pq = np.zeros((nb, V + 1))
    rc = lib.exact_enumerate(L, _ptr(Jc), nb, _ptr(b), _ptr(e), _ptr(e2), _ptr(ql), _ptr(pq))
    if rc != 0:
        raise RuntimeError("exact_enumerate failed")
    return {"e": e, "e2": e2, "ql": ql, "pq": pq}
