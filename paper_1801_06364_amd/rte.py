"""ctypes binding of librte.so (the C-ABI declared in include/rte.h).

Argument marshalling only: every step of the transport solve runs in the
HIP library. PyTorch supplies the device workspace and the HIP stream.
The functions ``rte_*`` mirror the C entry points one to one; ``Solver``
bundles a handle with the torch workspace that backs it.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librte.so")

RTE_OK, RTE_EINVAL, RTE_ENOMEM, RTE_EUNSTABLE, RTE_EDEVICE = 0, -1, -2, -3, -4
RTE_FP32, RTE_FP64 = 0, 1
RTE_RK4, RTE_EULER = 0, 1
RTE_FLUENCE_NOW, RTE_FLUENCE_INTEGRATED = 0, 1

EXPORTS = (
    "rte_workspace_bytes", "rte_create", "rte_step", "rte_run", "rte_fluence",
    "rte_readings", "rte_residuals", "rte_steps_done", "rte_get_state",
    "rte_set_state", "rte_coupling_dense", "rte_profile_kernels", "rte_destroy",
    "rte_strerror", "rte_adjoint_workspace_bytes", "rte_forward_checkpointed",
    "rte_adjoint", "rte_krylov_workspace_bytes", "rte_steady_gmres", "rte_expo_advance",
    "rte_profile_expo", "rte_set_source_profile", "rte_snapshot_bytes", "rte_snapshot",
    "rte_restore", "rte_batch_slot_bytes", "rte_batch_create", "rte_batch_admit", "rte_batch_step",
    "rte_batch_poll", "rte_batch_handle", "rte_batch_release", "rte_batch_destroy",
    "rte_static_scratch_bytes", "rte_steady_gmres_static", "rte_set_medium_device",
    "rte_set_state_device", "rte_readings_device", "rte_adjoint_device",
)
RTE_SLOT_FREE, RTE_SLOT_STAGING, RTE_SLOT_STAGED, RTE_SLOT_RUNNING, RTE_SLOT_DONE, RTE_SLOT_FAILED = range(6)
KERNEL_CLASSES = ("fwd_plane", "zderiv", "couple", "inv_plane", "end_step",
                  "fwd_rows", "y_fwd", "y_inv", "inv_rows", "z_fwd", "expo", "z_inv", "expo_table")


class RteError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class rte_config(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("order_N", C.c_int32), ("precision", C.c_int32),
        ("pml_width", C.c_int32), ("dx_mm", C.c_double), ("c_mm_ps", C.c_double),
        ("dt_ps", C.c_double), ("pml_mu0", C.c_double), ("pml_mu1", C.c_double),
        ("n_det", C.c_int32), ("scheme", C.c_int32),
        ("det_index", C.POINTER(C.c_int64)), ("record_steps", C.c_int64),
    ]


class rte_medium(C.Structure):
    _fields_ = [
        ("mu_a", C.POINTER(C.c_double)), ("mu_s", C.POINTER(C.c_double)),
        ("g", C.POINTER(C.c_double)), ("psi0", C.POINTER(C.c_double)),
        ("q", C.POINTER(C.c_double)), ("psi0_moments", C.c_int32),
        ("q_moments", C.c_int32),
    ]


_lib = None


def lib():
    """Load librte.so; raise if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1801_06364_amd.build` (there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i64p, dp = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)
        L.rte_workspace_bytes.argtypes = [C.POINTER(rte_config)]
        L.rte_workspace_bytes.restype = C.c_size_t
        L.rte_create.argtypes = [C.POINTER(rte_config), C.POINTER(rte_medium), vp,
                                 C.c_size_t, vp, C.POINTER(vp)]
        L.rte_create.restype = C.c_int
        L.rte_step.argtypes = [vp, C.c_int64]
        L.rte_step.restype = C.c_int
        L.rte_run.argtypes = [vp, C.c_int64, C.c_double, i64p]
        L.rte_run.restype = C.c_int
        L.rte_fluence.argtypes = [vp, C.c_int, dp, C.c_size_t]
        L.rte_fluence.restype = C.c_int
        L.rte_readings.argtypes = [vp, dp, C.c_size_t, i64p]
        L.rte_readings.restype = C.c_int
        L.rte_residuals.argtypes = [vp, dp, C.c_size_t, i64p]
        L.rte_residuals.restype = C.c_int
        L.rte_steps_done.argtypes = [vp, i64p]
        L.rte_steps_done.restype = C.c_int
        L.rte_get_state.argtypes = [vp, dp, C.c_size_t]
        L.rte_get_state.restype = C.c_int
        L.rte_set_state.argtypes = [vp, dp, C.c_size_t]
        L.rte_set_state.restype = C.c_int
        L.rte_coupling_dense.argtypes = [C.c_int32, dp, dp, dp]
        L.rte_coupling_dense.restype = C.c_int
        L.rte_profile_kernels.argtypes = [vp, C.c_int64, dp, i64p]
        L.rte_profile_kernels.restype = C.c_int
        L.rte_adjoint_workspace_bytes.argtypes = [C.POINTER(rte_config), C.c_int64, C.c_int64]
        L.rte_adjoint_workspace_bytes.restype = C.c_size_t
        L.rte_forward_checkpointed.argtypes = [vp, C.c_int64, C.c_int64, vp, C.c_size_t]
        L.rte_forward_checkpointed.restype = C.c_int
        L.rte_adjoint.argtypes = [vp, C.c_int64, C.c_int64, vp, C.c_size_t, dp, dp, dp]
        L.rte_adjoint.restype = C.c_int
        L.rte_adjoint_device.argtypes = [vp, C.c_int64, C.c_int64, vp, C.c_size_t, vp, vp, vp]
        L.rte_adjoint_device.restype = C.c_int
        L.rte_set_medium_device.argtypes = [vp, vp, vp]
        L.rte_set_medium_device.restype = C.c_int
        L.rte_set_state_device.argtypes = [vp, vp, C.c_int32]
        L.rte_set_state_device.restype = C.c_int
        L.rte_readings_device.argtypes = [vp, vp, C.c_size_t, i64p]
        L.rte_readings_device.restype = C.c_int
        L.rte_krylov_workspace_bytes.argtypes = [C.POINTER(rte_config), C.c_int32]
        L.rte_krylov_workspace_bytes.restype = C.c_size_t
        L.rte_steady_gmres.argtypes = [vp, C.c_int32, C.c_int64, C.c_double, C.c_int32, vp, C.c_size_t,
                                       i64p, dp]
        L.rte_steady_gmres.restype = C.c_int
        L.rte_static_scratch_bytes.argtypes = []
        L.rte_static_scratch_bytes.restype = C.c_size_t
        L.rte_steady_gmres_static.argtypes = [vp, C.c_int32, C.c_int64, C.c_double, C.c_int32, i64p, dp]
        L.rte_steady_gmres_static.restype = C.c_int
        L.rte_expo_advance.argtypes = [vp, C.c_double]
        L.rte_expo_advance.restype = C.c_int
        L.rte_set_source_profile.argtypes = [vp, dp, C.c_int64, C.c_double, C.c_int64, vp, C.c_size_t]
        L.rte_set_source_profile.restype = C.c_int
        L.rte_profile_expo.argtypes = [vp, C.c_double, dp, C.POINTER(C.c_int64)]
        L.rte_profile_expo.restype = C.c_int
        L.rte_snapshot_bytes.argtypes = [vp]
        L.rte_snapshot_bytes.restype = C.c_size_t
        L.rte_snapshot.argtypes = [vp, vp, C.c_size_t]
        L.rte_snapshot.restype = C.c_int
        L.rte_restore.argtypes = [vp, vp, C.c_size_t]
        L.rte_restore.restype = C.c_int
        L.rte_batch_slot_bytes.argtypes = [C.POINTER(rte_config)]
        L.rte_batch_slot_bytes.restype = C.c_size_t
        L.rte_batch_create.argtypes = [C.POINTER(rte_config), C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.rte_batch_create.restype = C.c_int
        L.rte_batch_admit.argtypes = [vp, C.c_int32, C.POINTER(rte_medium), C.POINTER(C.c_int64), C.c_int64]
        L.rte_batch_admit.restype = C.c_int
        L.rte_batch_step.argtypes = [vp, C.c_int64]
        L.rte_batch_step.restype = C.c_int
        L.rte_batch_poll.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.rte_batch_poll.restype = C.c_int
        L.rte_batch_handle.argtypes = [vp, C.c_int32, C.POINTER(vp)]
        L.rte_batch_handle.restype = C.c_int
        L.rte_batch_release.argtypes = [vp, C.c_int32]
        L.rte_batch_release.restype = C.c_int
        L.rte_batch_destroy.argtypes = [vp]
        L.rte_batch_destroy.restype = None
        L.rte_destroy.argtypes = [vp]
        L.rte_destroy.restype = None
        L.rte_strerror.argtypes = [C.c_int]
        L.rte_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().rte_strerror(code).decode()


def _check(code: int, what: str):
    if code != RTE_OK:
        raise RteError(code, what)


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def make_config(n, N, precision, dx, c, dt, W, mu0, mu1, det_index=None,
                record_steps=0, scheme=RTE_RK4):
    det = np.ascontiguousarray(det_index if det_index is not None else [], np.int64)
    cfg = rte_config(n=n, order_N=N, precision=precision, pml_width=W, dx_mm=dx,
                     c_mm_ps=c, dt_ps=dt, pml_mu0=mu0, pml_mu1=mu1,
                     n_det=int(det.size), scheme=int(scheme),
                     det_index=det.ctypes.data_as(C.POINTER(C.c_int64)) if det.size else None,
                     record_steps=int(record_steps))
    return cfg, det


# ---------------------------------------------------- raw entry points ---

def rte_workspace_bytes(cfg: rte_config) -> int:
    return int(lib().rte_workspace_bytes(C.byref(cfg)))


def rte_coupling_dense(N: int):
    M = (N + 1) ** 2
    out = [np.zeros((M, M)) for _ in range(3)]
    _check(lib().rte_coupling_dense(N, *[_dptr(o) for o in out]), "rte_coupling_dense")
    return out


class Solver:
    """One device-resident solve behind an ``rte_handle``.

    The torch tensor ``self.workspace`` owns the device memory; the handle
    runs on ``self.stream`` (a torch stream, the current one by default).
    """

    def __init__(self, n, N, dx, c, dt, mu_a, mu_s, g, psi0=None, q=None, W=0,
                 mu0=0.01, mu1=1.0, precision="f32", det_index=None,
                 record_steps=0, stream=None, device="cuda", scheme="rk4"):
        """psi0 / q: arrays of shape (K, n, n, n) holding the K leading
        real-basis moments (K <= M; the rest are zero), or None."""
        import torch
        self.n, self.N, self.M = n, N, (N + 1) ** 2
        prec = RTE_FP64 if precision in ("f64", RTE_FP64) else RTE_FP32
        self.precision = prec
        sch = RTE_EULER if scheme in ("euler", RTE_EULER) else RTE_RK4
        self.cfg, self._det = make_config(n, N, prec, dx, c, dt, W, mu0, mu1,
                                          det_index, record_steps, sch)
        self.n_det = int(self._det.size)
        nbytes = rte_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise RteError(RTE_EINVAL, "rte_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        arrs = [_f64(mu_a), _f64(mu_s), _f64(g), _f64(psi0), _f64(q)]
        pm = 0 if psi0 is None else arrs[3].size // n ** 3
        qm = 0 if q is None else arrs[4].size // n ** 3
        if (psi0 is not None and (pm * n ** 3 != arrs[3].size or pm > self.M)) or \
                (q is not None and (qm * n ** 3 != arrs[4].size or qm > self.M)):
            raise RteError(RTE_EINVAL, "psi0 / q must hold whole leading moments")
        med = rte_medium(*[_dptr(a) for a in arrs], pm, qm)
        self._keep = arrs
        h = C.c_void_p()
        rc = lib().rte_create(C.byref(self.cfg), C.byref(med),
                              C.c_void_p(self.workspace.data_ptr()), nbytes,
                              C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._keep = None
        _check(rc, "rte_create")
        self.h = h

    @classmethod
    def from_workload(cls, wl, **kw):
        args = dict(n=wl.n, N=wl.N, dx=wl.dx, c=wl.c, dt=wl.dt, mu_a=wl.mu_a,
                    mu_s=wl.mu_s, g=wl.g, psi0=wl.psi0, q=wl.q, W=wl.W,
                    mu0=wl.mu0, mu1=wl.mu1, precision=wl.precision,
                    det_index=wl.det_index, record_steps=wl.steps,
                    scheme=getattr(wl, "scheme", "rk4"))
        args.update(kw)
        return cls(**args)

    # -- C-ABI wrappers ---------------------------------------------------
    def step(self, k: int = 1):
        _check(lib().rte_step(self.h, int(k)), "rte_step")

    def run(self, max_steps: int, tol: float) -> int:
        taken = C.c_int64(0)
        rc = lib().rte_run(self.h, int(max_steps), float(tol), C.byref(taken))
        _check(rc, "rte_run")
        return int(taken.value)

    def fluence(self, which: int = RTE_FLUENCE_NOW) -> np.ndarray:
        out = np.zeros(self.n ** 3)
        _check(lib().rte_fluence(self.h, which, _dptr(out), out.size), "rte_fluence")
        return out.reshape(self.n, self.n, self.n)

    def readings(self) -> np.ndarray:
        cap = max(1, int(self.cfg.record_steps) * max(self.n_det, 1))
        out = np.zeros(cap)
        rows = C.c_int64(0)
        _check(lib().rte_readings(self.h, _dptr(out), out.size, C.byref(rows)), "rte_readings")
        return out[: rows.value * self.n_det].reshape(rows.value, self.n_det)

    def residuals(self) -> np.ndarray:
        out = np.zeros(max(1, int(self.cfg.record_steps)))
        rows = C.c_int64(0)
        _check(lib().rte_residuals(self.h, _dptr(out), out.size, C.byref(rows)), "rte_residuals")
        return out[: rows.value].copy()

    def steps_done(self) -> int:
        s = C.c_int64(0)
        _check(lib().rte_steps_done(self.h, C.byref(s)), "rte_steps_done")
        return int(s.value)

    def get_state(self) -> np.ndarray:
        out = np.zeros(self.M * self.n ** 3)
        _check(lib().rte_get_state(self.h, _dptr(out), out.size), "rte_get_state")
        return out.reshape(self.M, self.n, self.n, self.n)

    def set_state(self, psi: np.ndarray):
        a = _f64(psi).ravel()
        _check(lib().rte_set_state(self.h, _dptr(a), a.size), "rte_set_state")

    def snapshot(self) -> bytes:
        """Checkpoint of the run (state, step count, integrated fluence,
        record, flags) as host bytes."""
        nb = int(lib().rte_snapshot_bytes(self.h))
        buf = (C.c_ubyte * nb)()
        _check(lib().rte_snapshot(self.h, C.cast(buf, C.c_void_p), nb), "rte_snapshot")
        return bytes(buf)

    def restore(self, snap: bytes):
        """Resume from a snapshot taken on a solver with the same
        configuration, detectors, maps and source."""
        buf = C.create_string_buffer(bytes(snap), len(snap))
        _check(lib().rte_restore(self.h, C.cast(buf, C.c_void_p), len(snap)), "rte_restore")

    # -- time-dependent source ---------------------------------------------
    def set_source_profile(self, samples, delta_ps: float, rows: int):
        """Source q(r) s(t), s linear between samples spaced delta_ps apart
        (t from step 0); the library tabulates per-step weights for `rows`
        steps into a device table owned by this solver. samples=None
        returns to a constant source."""
        import torch
        if samples is None:
            _check(lib().rte_set_source_profile(self.h, None, 0, 1.0, 0, None, 0), "rte_set_source_profile")
            self._qw = None
            return
        sm = _f64(samples).ravel()
        cols = 1 if self.cfg.scheme == RTE_EULER else 4
        table = torch.empty(max(1, int(rows)) * cols, dtype=torch.float64, device=self.workspace.device)
        _check(lib().rte_set_source_profile(self.h, _dptr(sm), sm.size, float(delta_ps), int(rows),
                                            C.c_void_p(table.data_ptr()), table.numel() * 8),
               "rte_set_source_profile")
        self._qw = table

    # -- exact propagation (homogeneous media) -----------------------------
    def expo_advance(self, t_ps: float):
        """Advance the state by t_ps exactly (per-mode matrix exponential);
        homogeneous medium without boundary layer only."""
        _check(lib().rte_expo_advance(self.h, float(t_ps)), "rte_expo_advance")

    # -- steady state by GMRES --------------------------------------------
    def steady_gmres(self, tol: float = 1e-6, restart: int = 16, max_iters: int = 2000,
                     steps_per_apply: int = 0):
        """Solve for the steady state in place (u <- solution of (S + Sigma)
        u = q), by GMRES on that operator (steps_per_apply = 0) or on
        I - P^K with P one time step (steps_per_apply = K); returns (Arnoldi
        steps, final relative residual of the steady-state equation)."""
        import torch
        nbytes = int(lib().rte_krylov_workspace_bytes(C.byref(self.cfg), int(restart)))
        if nbytes == 0:
            raise RteError(RTE_EINVAL, "rte_krylov_workspace_bytes")
        kws = torch.empty(nbytes, dtype=torch.uint8, device=self.workspace.device)
        it = C.c_int64(0)
        res = C.c_double(0.0)
        rc = lib().rte_steady_gmres(self.h, int(restart), int(max_iters), float(tol), int(steps_per_apply),
                                    C.c_void_p(kws.data_ptr()), nbytes, C.byref(it), C.byref(res))
        self.stream.synchronize()
        del kws
        _check(rc, "rte_steady_gmres")
        return int(it.value), float(res.value)

    def steady_gmres_static(self, tol: float = 1e-6, restart: int = 16, max_iters: int = 2000,
                            steps_per_apply: int = 0):
        """steady_gmres with the Krylov workspace in the library's static
        device array (rte_steady_gmres_static: no device allocation); the
        Krylov workspace of (n, N, restart) must fit rte_static_scratch_bytes()."""
        it = C.c_int64(0)
        res = C.c_double(0.0)
        rc = lib().rte_steady_gmres_static(self.h, int(restart), int(max_iters), float(tol),
                                           int(steps_per_apply), C.byref(it), C.byref(res))
        _check(rc, "rte_steady_gmres_static")
        return int(it.value), float(res.value)

    # -- discrete adjoint ---------------------------------------------------
    def forward_checkpointed(self, steps: int, every: int = 0):
        """Run ``steps`` steps keeping checkpoints every ``every`` steps
        (default ceil(sqrt(steps))) in a torch-owned device workspace."""
        import math
        import torch
        every = int(every) or max(1, math.ceil(math.sqrt(steps)))
        nbytes = int(lib().rte_adjoint_workspace_bytes(C.byref(self.cfg), int(steps), every))
        if nbytes == 0:
            raise RteError(RTE_EINVAL, "rte_adjoint_workspace_bytes")
        self.adj_ws = torch.empty(nbytes, dtype=torch.uint8, device=self.workspace.device)
        self.adj_steps, self.adj_every = int(steps), every
        _check(lib().rte_forward_checkpointed(self.h, int(steps), every,
                                              C.c_void_p(self.adj_ws.data_ptr()), nbytes),
               "rte_forward_checkpointed")

    def adjoint(self, dj_dr):
        """dJ/dmu_a, dJ/dmu_s (each (n, n, n), FP64) for adjoint sources
        ``dj_dr[step][det]`` of the last checkpointed forward run."""
        n = self.n
        ga = np.zeros(n ** 3)
        gs = np.zeros(n ** 3)
        d = np.ascontiguousarray(dj_dr, np.float64).reshape(self.adj_steps, self.n_det)
        _check(lib().rte_adjoint(self.h, self.adj_steps, self.adj_every,
                                 C.c_void_p(self.adj_ws.data_ptr()), self.adj_ws.numel(),
                                 _dptr(d), _dptr(ga), _dptr(gs)), "rte_adjoint")
        return ga.reshape(n, n, n), gs.reshape(n, n, n)

    # -- device-resident inputs and outputs ----------------------------------
    @staticmethod
    def _dev_f64(t, numel, what):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == numel):
            raise RteError(RTE_EINVAL, f"{what}: a contiguous FP64 CUDA tensor of {numel} elements")
        return C.c_void_p(t.data_ptr())

    def set_medium_device(self, mu_a, mu_s):
        """New mu_a, mu_s from FP64 CUDA tensors (n^3 each), loss maps rebuilt on the device."""
        n3 = self.n ** 3
        _check(lib().rte_set_medium_device(self.h, self._dev_f64(mu_a, n3, "mu_a"),
                                           self._dev_f64(mu_s, n3, "mu_s")), "rte_set_medium_device")

    def set_state_device(self, psi):
        """State from an FP64 CUDA tensor holding K leading moments (K n^3 elements)."""
        n3 = self.n ** 3
        k = psi.numel() // n3
        if k * n3 != psi.numel() or k > self.M:
            raise RteError(RTE_EINVAL, "psi must hold whole leading moments")
        _check(lib().rte_set_state_device(self.h, self._dev_f64(psi, k * n3, "psi"), k),
               "rte_set_state_device")

    def readings_device(self):
        """Readings [rows][n_det] as an FP64 CUDA tensor (device-to-device copy)."""
        import torch
        cap = int(self.cfg.record_steps)
        out = torch.empty((max(cap, 1), max(self.n_det, 1)), dtype=torch.float64, device=self.workspace.device)
        rows = C.c_int64(0)
        _check(lib().rte_readings_device(self.h, C.c_void_p(out.data_ptr()), cap * self.n_det, C.byref(rows)),
               "rte_readings_device")
        return out[:int(rows.value), :self.n_det]

    def adjoint_device(self, dj_dr):
        """dJ/dmu_a, dJ/dmu_s as FP64 CUDA tensors (n, n, n) for adjoint
        sources dj_dr[step][det] given as an FP64 CUDA tensor."""
        import torch
        n = self.n
        dev = self.workspace.device
        ga = torch.empty(n ** 3, dtype=torch.float64, device=dev)
        gs = torch.empty(n ** 3, dtype=torch.float64, device=dev)
        d = dj_dr.to(device=dev, dtype=torch.float64).contiguous()
        _check(lib().rte_adjoint_device(self.h, self.adj_steps, self.adj_every,
                                        C.c_void_p(self.adj_ws.data_ptr()), self.adj_ws.numel(),
                                        self._dev_f64(d, self.adj_steps * self.n_det, "dj_dr"),
                                        C.c_void_p(ga.data_ptr()), C.c_void_p(gs.data_ptr())),
               "rte_adjoint_device")
        return ga.view(n, n, n), gs.view(n, n, n)

    def profile_kernels(self, nsteps: int):
        """Per-kernel-class milliseconds (summed) and launch counts over
        ``nsteps`` steps timed with HIP events on the handle's stream."""
        ms = np.zeros(len(KERNEL_CLASSES))
        cnt = np.zeros(len(KERNEL_CLASSES), np.int64)
        _check(lib().rte_profile_kernels(self.h, int(nsteps), _dptr(ms),
                                         cnt.ctypes.data_as(C.POINTER(C.c_int64))),
               "rte_profile_kernels")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES) if cnt[i]}

    def profile_expo(self, t_ps: float):
        """expo_advance(t_ps) with per-kernel-class event timing."""
        ms = np.zeros(len(KERNEL_CLASSES))
        cnt = np.zeros(len(KERNEL_CLASSES), np.int64)
        _check(lib().rte_profile_expo(self.h, float(t_ps), _dptr(ms),
                                      cnt.ctypes.data_as(C.POINTER(C.c_int64))),
               "rte_profile_expo")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES) if cnt[i]}

    def close(self):
        if getattr(self, "h", None):
            self.stream.synchronize()
            lib().rte_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many solves of one configuration advanced together (``rte_batch_*``):
    ``slots`` slots in one torch-owned workspace, stepped in chunks on
    ``self.stream``; requests are admitted into free slots (from any
    thread), polled, read and released."""

    def __init__(self, n, N, dx, c, dt, W, slots, mu0=0.01, mu1=1.0, precision="f32",
                 n_det=0, record_steps=0, scheme="rk4", stream=None, device="cuda"):
        import torch
        self.n, self.N, self.M, self.slots = n, N, (N + 1) ** 2, int(slots)
        prec = RTE_FP64 if precision in ("f64", RTE_FP64) else RTE_FP32
        sch = RTE_EULER if scheme in ("euler", RTE_EULER) else RTE_RK4
        self.cfg, _ = make_config(n, N, prec, dx, c, dt, W, mu0, mu1, None, record_steps, sch)
        self.cfg.n_det = int(n_det)
        self.n_det = int(n_det)
        self.slot_bytes = int(lib().rte_batch_slot_bytes(C.byref(self.cfg)))
        if self.slot_bytes == 0:
            raise RteError(RTE_EINVAL, "rte_batch_slot_bytes")
        self.workspace = torch.empty(self.slot_bytes * self.slots, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        b = C.c_void_p()
        _check(lib().rte_batch_create(C.byref(self.cfg), self.slots, C.c_void_p(self.workspace.data_ptr()),
                                      self.workspace.numel(), C.c_void_p(self.stream.cuda_stream), C.byref(b)),
               "rte_batch_create")
        self.b = b
        self._steps = np.zeros(self.slots, np.int64)
        self._status = np.zeros(self.slots, np.int32)

    def admit(self, slot, mu_a, mu_s, g, steps, psi0=None, q=None, det_index=None):
        n = self.n
        arrs = [_f64(mu_a), _f64(mu_s), _f64(g), _f64(psi0), _f64(q)]
        pm = 0 if psi0 is None else arrs[3].size // n ** 3
        qm = 0 if q is None else arrs[4].size // n ** 3
        med = rte_medium(*[_dptr(a) for a in arrs], pm, qm)
        det = np.ascontiguousarray(det_index if det_index is not None else [], np.int64)
        if det.size != self.n_det:
            raise RteError(RTE_EINVAL, "detector count differs from the batch configuration")
        dp = det.ctypes.data_as(C.POINTER(C.c_int64)) if det.size else None
        _check(lib().rte_batch_admit(self.b, int(slot), C.byref(med), dp, int(steps)), "rte_batch_admit")

    def step(self, k: int):
        _check(lib().rte_batch_step(self.b, int(k)), "rte_batch_step")

    def poll(self):
        """(steps_done[slots], status[slots], chunks in flight) from the
        newest completed chunk."""
        fl = C.c_int32(0)
        _check(lib().rte_batch_poll(self.b, self._steps.ctypes.data_as(C.POINTER(C.c_int64)),
                                    self._status.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(fl)),
               "rte_batch_poll")
        return self._steps.copy(), self._status.copy(), int(fl.value)

    def _handle(self, slot):
        h = C.c_void_p()
        _check(lib().rte_batch_handle(self.b, int(slot), C.byref(h)), "rte_batch_handle")
        return h

    def fluence(self, slot, which: int = RTE_FLUENCE_NOW) -> np.ndarray:
        out = np.zeros(self.n ** 3)
        _check(lib().rte_fluence(self._handle(slot), which, _dptr(out), out.size), "rte_fluence")
        return out.reshape(self.n, self.n, self.n)

    def get_state(self, slot) -> np.ndarray:
        out = np.zeros(self.M * self.n ** 3)
        _check(lib().rte_get_state(self._handle(slot), _dptr(out), out.size), "rte_get_state")
        return out.reshape(self.M, self.n, self.n, self.n)

    def readings(self, slot) -> np.ndarray:
        cap = max(1, int(self.cfg.record_steps) * max(self.n_det, 1))
        out = np.zeros(cap)
        rows = C.c_int64(0)
        _check(lib().rte_readings(self._handle(slot), _dptr(out), out.size, C.byref(rows)), "rte_readings")
        return out[: rows.value * self.n_det].reshape(rows.value, self.n_det)

    def steps_done(self, slot) -> int:
        s = C.c_int64(0)
        _check(lib().rte_steps_done(self._handle(slot), C.byref(s)), "rte_steps_done")
        return int(s.value)

    def release(self, slot):
        _check(lib().rte_batch_release(self.b, int(slot)), "rte_batch_release")

    def close(self):
        if getattr(self, "b", None):
            lib().rte_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
