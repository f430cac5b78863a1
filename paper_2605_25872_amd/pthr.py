"""Python binding of the PTHR C ABI (include/pthr.h).

Argument marshalling only: every step of the method runs in the HIP library
``libpthr.so`` (built in-tree by ``paper_2605_25872_amd.build``).  PyTorch
provides the device memory (uint8 tensors) and the current HIP stream.  If the
library is missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpthr.so")

PTHR_OK, PTHR_EINVAL, PTHR_EUNSUPPORTED, PTHR_EHIP, PTHR_ESTATE, PTHR_EDEVICE = 0, -1, -2, -3, -4, -5
FP64, FP32 = 0, 1
ACU, SINGLE_NEG = 0, 1
METROPOLIS, HEAT_BATH, MICSA = 0, 1, 2
NOBS = 6
OBS_NAMES = ("e", "e2", "q2", "q4", "ql", "sdy")

EXPORTED = (
    "pthr_create", "pthr_destroy", "pthr_last_error", "pthr_create_error", "pthr_state_bytes",
    "pthr_obs_bytes", "pthr_obs_acc_offset", "pthr_obs_hist_offset", "pthr_init_samples",
    "pthr_sweep", "pthr_houdayer", "pthr_pt_swap", "pthr_measure", "pthr_obs_clear", "pthr_run",
    "pthr_cluster_labels", "pthr_read_spins", "pthr_read_pt", "pthr_counters", "pthr_check",
    "pthr_blob_bytes", "pthr_get_state", "pthr_set_state", "pthr_get_schedule",
    "pthr_set_schedule", "pthr_autotune", "pthr_lds_bytes", "pthr_group_create",
    "pthr_group_destroy", "pthr_group_last_error", "pthr_group_run", "pthr_cluster_stats",
    "pthr_write_spins", "pthr_read_walkers", "pthr_autotune_noalloc", "pthr_autotune_results",
)


class PthrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pthr error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("n_replicas", ctypes.c_int32), ("n_temps", ctypes.c_int32),
                ("n_reservoir", ctypes.c_int32), ("sweeps_per_emcs", ctypes.c_int32),
                ("er_sweeps_per_emcs", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("houdayer_mode", ctypes.c_int32), ("local_update", ctypes.c_int32),
                ("t_acu", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("micsa_refresh", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("threads_per_sample", ctypes.c_int32), ("samples_per_launch", ctypes.c_int32),
                ("exp_early_out", ctypes.c_int32), ("graph_window", ctypes.c_int32),
                ("clone_split", ctypes.c_int32), ("exp_filter", ctypes.c_int32),
                ("sample_split", ctypes.c_int32), ("overlap_reservoir", ctypes.c_int32)]


_lib = None


def library() -> ctypes.CDLL:
    """Load libpthr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; load it first so that libpthr.so binds to
    # the same runtime instance as the tensors and streams it is handed
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_2605_25872_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER(Params)
    sig = {
        "pthr_create": (i32, [P, ctypes.POINTER(vp)]),
        "pthr_destroy": (i32, [vp]),
        "pthr_last_error": (ctypes.c_char_p, [vp]),
        "pthr_create_error": (ctypes.c_char_p, []),
        "pthr_state_bytes": (sz, [P]),
        "pthr_lds_bytes": (sz, [P]),
        "pthr_obs_bytes": (sz, [P]),
        "pthr_obs_acc_offset": (sz, [P]),
        "pthr_obs_hist_offset": (sz, [P]),
        "pthr_init_samples": (i32, [vp, vp, vp, vp, vp]),
        "pthr_sweep": (i32, [vp, i32, i32, vp]),
        "pthr_houdayer": (i32, [vp, vp]),
        "pthr_pt_swap": (i32, [vp, i32, vp]),
        "pthr_measure": (i32, [vp, vp, vp]),
        "pthr_obs_clear": (i32, [vp, vp, vp]),
        "pthr_run": (i32, [vp, i64, vp, vp]),
        "pthr_cluster_labels": (i32, [vp, vp, vp]),
        "pthr_cluster_stats": (i32, [vp, vp, vp]),
        "pthr_read_spins": (i32, [vp, vp, vp]),
        "pthr_write_spins": (i32, [vp, vp, vp]),
        "pthr_read_walkers": (i32, [vp, vp, vp]),
        "pthr_read_pt": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "pthr_counters": (i32, [vp, vp, vp, vp]),
        "pthr_check": (i32, [vp, vp]),
        "pthr_blob_bytes": (sz, [vp]),
        "pthr_get_state": (i32, [vp, vp, sz, vp]),
        "pthr_set_state": (i32, [vp, vp, sz, vp]),
        "pthr_get_schedule": (i32, [vp, ctypes.POINTER(Schedule)]),
        "pthr_set_schedule": (i32, [vp, ctypes.POINTER(Schedule)]),
        "pthr_autotune": (i32, [vp, vp, i32, vp, vp]),
        "pthr_autotune_noalloc": (i32, [vp, i32, vp, vp]),
        "pthr_autotune_results": (i32, [vp, ctypes.POINTER(Schedule), vp, i32]),
        "pthr_group_create": (i32, [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]),
        "pthr_group_destroy": (i32, [vp]),
        "pthr_group_last_error": (ctypes.c_char_p, [vp]),
        "pthr_group_run": (i32, [vp, i64, ctypes.POINTER(vp), i32, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _np_ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def make_params(L, n_samples, n_replicas, n_temps, n_reservoir, sweeps_per_emcs=10,
                er_sweeps_per_emcs=240, precision=FP64, houdayer_mode=ACU, t_acu=1.0, seed=1,
                local_update=METROPOLIS, micsa_refresh=0) -> Params:
    if isinstance(precision, str):
        precision = {"fp64": FP64, "fp32": FP32}[precision]
    if isinstance(houdayer_mode, str):
        houdayer_mode = {"acu": ACU, "single": SINGLE_NEG}[houdayer_mode]
    if isinstance(local_update, str):
        local_update = {"metropolis": METROPOLIS, "heatbath": HEAT_BATH, "micsa": MICSA}[local_update]
    return Params(L, n_samples, n_replicas, n_temps, n_reservoir, sweeps_per_emcs,
                  er_sweeps_per_emcs, precision, houdayer_mode, local_update, t_acu, seed, micsa_refresh)


class Pthr:
    """One PTHR context: a batch of samples resident in a caller-owned device
    buffer (a torch uint8 tensor), advanced by the library's HIP kernels."""

    def __init__(self, L, n_samples, n_replicas=4, n_temps=8, n_reservoir=4, sweeps_per_emcs=10,
                 er_sweeps_per_emcs=240, precision=FP64, houdayer_mode=ACU, t_acu=1.0, seed=1,
                 device="cuda:0", local_update=METROPOLIS, micsa_refresh=0):
        import torch

        self.torch = torch
        self.lib = library()
        self.params = make_params(L, n_samples, n_replicas, n_temps, n_reservoir, sweeps_per_emcs,
                                  er_sweeps_per_emcs, precision, houdayer_mode, t_acu, seed, local_update,
                                  micsa_refresh)
        ctx = ctypes.c_void_p()
        rc = self.lib.pthr_create(ctypes.byref(self.params), ctypes.byref(ctx))
        if rc != PTHR_OK:
            raise PthrError(rc, self.lib.pthr_create_error().decode())
        self.ctx = ctx
        self.device = torch.device(device)
        self.L, self.S, self.NR, self.NT, self.NERG = L, n_samples, n_replicas, n_temps, n_reservoir
        self.V = L ** 3
        self.NPT = n_replicas * n_temps
        self.C = self.NPT + n_replicas * n_reservoir
        self.state_bytes = self.lib.pthr_state_bytes(ctypes.byref(self.params))
        self.state = torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)
        self.K_acu = 0

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.pthr_destroy(ctx)
            self.ctx = None

    # ------------------------------------------------------------ plumbing
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, rc: int) -> None:
        if rc != PTHR_OK:
            raise PthrError(rc, self.lib.pthr_last_error(self.ctx).decode())

    # ------------------------------------------------------------ the method
    def init_samples(self, J: np.ndarray, T: np.ndarray) -> None:
        Jh = np.ascontiguousarray(J, dtype=np.float64).reshape(self.S, 3, self.V)
        Th = np.ascontiguousarray(T, dtype=np.float64)
        self.T = Th.copy()
        self.K_acu = int(np.sum(Th < self.params.t_acu))
        with self.torch.cuda.device(self.device):
            self._check(self.lib.pthr_init_samples(self.ctx, _np_ptr(Jh), _np_ptr(Th),
                                                   ctypes.c_void_p(self.state.data_ptr()),
                                                   self._stream()))

    def sweep(self, n_pt: int, n_er: int = 0) -> None:
        """n_pt sweeps of the PT clones and n_er of the reservoir clones, one launch."""
        self._check(self.lib.pthr_sweep(self.ctx, n_pt, n_er, self._stream()))

    def houdayer(self) -> None:
        self._check(self.lib.pthr_houdayer(self.ctx, self._stream()))

    def pt_swap(self, do_reservoir: bool = True) -> None:
        self._check(self.lib.pthr_pt_swap(self.ctx, int(do_reservoir), self._stream()))

    def new_obs(self):
        n = self.lib.pthr_obs_bytes(ctypes.byref(self.params))
        obs = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        self._check(self.lib.pthr_obs_clear(self.ctx, ctypes.c_void_p(obs.data_ptr()), self._stream()))
        return obs

    def measure(self, obs) -> None:
        self._check(self.lib.pthr_measure(self.ctx, ctypes.c_void_p(obs.data_ptr()), self._stream()))

    def run(self, n_emcs: int, obs=None) -> None:
        ptr = ctypes.c_void_p(obs.data_ptr()) if obs is not None else None
        self._check(self.lib.pthr_run(self.ctx, n_emcs, ptr, self._stream()))

    def emcs(self, obs=None) -> None:
        """One EMCS through the step-wise calls."""
        self.sweep(self.params.sweeps_per_emcs, self.params.er_sweeps_per_emcs if self.NERG else 0)
        self.houdayer()
        self.pt_swap(True)
        if obs is not None:
            self.measure(obs)

    # ------------------------------------------------------------ read-back
    def obs_arrays(self, obs) -> dict:
        raw = obs.cpu().numpy()
        acc_off = self.lib.pthr_obs_acc_offset(ctypes.byref(self.params))
        hist_off = self.lib.pthr_obs_hist_offset(ctypes.byref(self.params))
        n_acc = self.S * self.NT * NOBS
        return {
            "n_meas": int(raw[:8].view(np.uint64)[0]),
            "acc": raw[acc_off:acc_off + 8 * n_acc].view(np.float64).reshape(self.S, self.NT, NOBS),
            "hist": raw[hist_off:hist_off + 8 * self.NT * (self.V + 1)].view(np.uint64)
            .reshape(self.NT, self.V + 1),
        }

    def read_spins(self) -> np.ndarray:
        out = np.empty((self.S, self.C, self.V), dtype=np.int8)
        self._check(self.lib.pthr_read_spins(self.ctx, _np_ptr(out), self._stream()))
        return out

    def write_spins(self, spins: np.ndarray) -> None:
        """Replace every clone's spins: int8 [S][C][V] of +1/-1."""
        a = np.ascontiguousarray(spins, dtype=np.int8).reshape(self.S, self.C, self.V)
        self._check(self.lib.pthr_write_spins(self.ctx, _np_ptr(a), self._stream()))

    def read_walkers(self) -> np.ndarray:
        """MicSA walker energy of every PT clone, [S][N_r*N_T] by clone id."""
        out = np.empty((self.S, self.NPT), dtype=np.float64)
        self._check(self.lib.pthr_read_walkers(self.ctx, _np_ptr(out), self._stream()))
        return out

    def read_pt(self) -> dict:
        S, NR, NT = self.S, self.NR, self.NT
        d = {
            "clone_at": np.empty((S, NR, NT), np.int32), "er_head": np.empty((S, NR), np.int32),
            "pt_last": np.empty((S, NR, NT - 1), np.uint8),
            "pt_count": np.empty((S, NR, NT - 1), np.uint32),
            "pt_energy": np.empty((S, self.NPT), np.float64),
            "rt_state": np.empty((S, self.NPT), np.uint8), "rt_count": np.empty((S,), np.uint64),
        }
        self._check(self.lib.pthr_read_pt(self.ctx, *(_np_ptr(d[k]) for k in (
            "clone_at", "er_head", "pt_last", "pt_count", "pt_energy", "rt_state", "rt_count")),
            self._stream()))
        return d

    def labels(self) -> np.ndarray:
        K = self.K_acu
        out = self.torch.empty((self.S, self.NR // 2, max(K, 1), self.V), dtype=self.torch.int32,
                               device=self.device)
        self._check(self.lib.pthr_cluster_labels(self.ctx, ctypes.c_void_p(out.data_ptr()),
                                                 self._stream()))
        return out.cpu().numpy()[:, :, :K]

    def cluster_stats(self) -> np.ndarray:
        """[S][N_r/2][K][2][6] sizes of the six largest majority (index 0) and
        minority (index 1) clusters of every Houdayer pair and T_k < t_acu."""
        K = self.K_acu
        out = self.torch.zeros((self.S, self.NR // 2, max(K, 1), 2, 6), dtype=self.torch.int32,
                               device=self.device)
        self._check(self.lib.pthr_cluster_stats(self.ctx, ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out.cpu().numpy()[:, :, :K]

    def counters(self) -> tuple[int, int, int]:
        t, mp, me = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.pthr_counters(self.ctx, ctypes.byref(t), ctypes.byref(mp), ctypes.byref(me)))
        return t.value, mp.value, me.value

    def check(self) -> None:
        self._check(self.lib.pthr_check(self.ctx, self._stream()))

    def get_state(self) -> bytes:
        n = self.lib.pthr_blob_bytes(self.ctx)
        buf = ctypes.create_string_buffer(n)
        self._check(self.lib.pthr_get_state(self.ctx, buf, n, self._stream()))
        return buf.raw

    def set_state(self, blob: bytes) -> None:
        self._check(self.lib.pthr_set_state(self.ctx, blob, len(blob), self._stream()))

    def schedule(self) -> Schedule:
        sch = Schedule()
        self._check(self.lib.pthr_get_schedule(self.ctx, ctypes.byref(sch)))
        return sch

    def set_schedule(self, threads_per_sample=None, samples_per_launch=None, exp_early_out=None,
                     graph_window=None, clone_split=None, exp_filter=None, sample_split=None,
                     overlap_reservoir=None) -> None:
        sch = self.schedule()
        if overlap_reservoir is not None:
            sch.overlap_reservoir = int(overlap_reservoir)
        if sample_split is not None:
            sch.sample_split = sample_split
        if exp_filter is not None:
            sch.exp_filter = int(exp_filter)
        if clone_split is not None:
            sch.clone_split = clone_split
        if graph_window is not None:
            sch.graph_window = graph_window
        if threads_per_sample is not None:
            sch.threads_per_sample = threads_per_sample
        if samples_per_launch is not None:
            sch.samples_per_launch = samples_per_launch
        if exp_early_out is not None:
            sch.exp_early_out = int(exp_early_out)
        self._check(self.lib.pthr_set_schedule(self.ctx, ctypes.byref(sch)))

    def autotune(self, n_emcs: int = 2) -> float:
        scratch = self.torch.empty(self.state_bytes, dtype=self.torch.uint8, device=self.device)
        best = ctypes.c_double()
        self._check(self.lib.pthr_autotune(self.ctx, ctypes.c_void_p(scratch.data_ptr()), n_emcs,
                                           ctypes.byref(best), self._stream()))
        return best.value

    def autotune_results(self) -> list[tuple[Schedule, float]]:
        """(candidate schedule, ms per EMCS) of every candidate the last autotuning timed."""
        n = self.lib.pthr_autotune_results(self.ctx, None, None, 0)
        sch = (Schedule * max(n, 1))()
        ms = np.zeros(max(n, 1), dtype=np.float64)
        self.lib.pthr_autotune_results(self.ctx, sch, _np_ptr(ms), n)
        return [(sch[i], float(ms[i])) for i in range(n)]

    def autotune_noalloc(self, n_emcs: int = 2) -> float:
        """pthr_autotune_noalloc: the same tuning with no device allocation (the
        scratch state lives in the library's static workspace)."""
        best = ctypes.c_double()
        self._check(self.lib.pthr_autotune_noalloc(self.ctx, n_emcs, ctypes.byref(best), self._stream()))
        return best.value


class Group:
    """Several contexts (e.g. lattices of different sizes) advanced together:
    each context's EMCS chain on its own HIP stream, windows of EMCS captured
    into one graph with a branch per context."""

    def __init__(self, members: list):
        self.members = list(members)
        self.lib = library()
        self.torch = self.members[0].torch
        arr = (ctypes.c_void_p * len(self.members))(*(m.ctx.value for m in self.members))
        grp = ctypes.c_void_p()
        rc = self.lib.pthr_group_create(arr, len(self.members), ctypes.byref(grp))
        if rc != PTHR_OK:
            raise PthrError(rc, self.lib.pthr_create_error().decode())
        self.grp = grp

    def __del__(self):
        grp = getattr(self, "grp", None)
        if grp is not None and grp.value:
            self.lib.pthr_group_destroy(grp)
            self.grp = None

    def run(self, n_emcs: int, obs: list | None = None, graph_window: int = 16) -> None:
        """n_emcs EMCS of every member; obs: None or one buffer (or None) per member."""
        ptrs = None
        if obs is not None:
            if len(obs) != len(self.members):
                raise ValueError("one observable buffer (or None) per member")
            ptrs = (ctypes.c_void_p * len(obs))(*(o.data_ptr() if o is not None else None for o in obs))
        stream = ctypes.c_void_p(self.torch.cuda.current_stream(self.members[0].device).cuda_stream)
        rc = self.lib.pthr_group_run(self.grp, n_emcs, ptrs, graph_window, stream)
        if rc != PTHR_OK:
            raise PthrError(rc, self.lib.pthr_group_last_error(self.grp).decode())
