"""Python binding of the HGKS C ABI (include/hgks.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels
of libhgks.so.  PyTorch supplies device memory (the state and the workspace
are torch tensors) and the HIP stream.  Importing works without a GPU; any
call that needs the library raises if libhgks.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhgks.so")

ABI_VERSION = 2
HGKS_FLAG_CONSTANT_MASS_FLUX = 1
HGKS_OK, HGKS_E_INVALID, HGKS_E_NOMEM, HGKS_E_DEVICE, HGKS_E_NONFINITE, HGKS_E_NEGATIVE_STATE, HGKS_E_UNSUPPORTED = range(7)
BC_PERIODIC, BC_ISOTHERMAL_WALL = 0, 1
FP64, MIXED, FP32 = 0, 1, 2

EXPORTED = [
    "hgks_workspace_size", "hgks_init", "hgks_step", "hgks_stats", "hgks_dt", "hgks_residual",
    "hgks_destroy", "hgks_status_string", "hgks_last_error", "hgks_profile", "hgks_profile_read",
    "hgks_batch_workspace_size", "hgks_batch_init", "hgks_batch_step", "hgks_batch_stats", "hgks_batch_info",
    "hgks_residual_static", "hgks_fma_probe",
]
STATIC_SCRATCH_BYTES = 64 << 20
PROFILE_CLASSES = ("recon", "flux", "update", "other")


class hgks_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("bc", ctypes.c_int32 * 3),
        ("y_stretch", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
        ("mu_ref", ctypes.c_double),
        ("T_ref", ctypes.c_double),
        ("mu_exp", ctypes.c_double),
        ("T_wall", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("cfl", ctypes.c_double),
        ("rho_ref", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
    ]


class hgks_stats_t(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("dt_last", ctypes.c_double),
        ("steps", ctypes.c_int64),
        ("Ek", ctypes.c_double),
        ("eps_sol", ctypes.c_double),
        ("eps_dil", ctypes.c_double),
        ("eps_com", ctypes.c_double),
        ("total", ctypes.c_double * 5),
        ("max_abs", ctypes.c_double * 5),
        ("min_p", ctypes.c_double),
        ("min_rho", ctypes.c_double),
        ("nonfinite", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("body_force_x", ctypes.c_double),
    ]


class HGKSError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"hgks status {status}: {msg}")


_lib = None


def lib():
    """Load libhgks.so (fails loudly when the HIP library is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2207_01173_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, d = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
        C = ctypes.POINTER(hgks_config)
        L.hgks_workspace_size.argtypes = [C, ctypes.POINTER(sz)]
        L.hgks_init.argtypes = [C, vp, vp, sz, vp, d, ctypes.POINTER(vp)]
        L.hgks_step.argtypes = [vp, i32, d]
        L.hgks_stats.argtypes = [vp, ctypes.POINTER(hgks_stats_t)]
        L.hgks_dt.argtypes = [vp, ctypes.POINTER(d)]
        L.hgks_residual.argtypes = [vp, vp, d, vp, vp]
        L.hgks_residual_static.argtypes = [C, vp, d, vp, vp, vp]
        L.hgks_fma_probe.argtypes = [vp, i32, i32, vp]
        L.hgks_destroy.argtypes = [vp]
        L.hgks_batch_workspace_size.argtypes = [i32, C, ctypes.POINTER(sz)]
        L.hgks_batch_init.argtypes = [i32, C, ctypes.POINTER(vp), vp, sz, vp, ctypes.POINTER(vp)]
        L.hgks_batch_step.argtypes = [vp, i32]
        L.hgks_batch_stats.argtypes = [vp, i32, ctypes.POINTER(hgks_stats_t)]
        L.hgks_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.hgks_profile.argtypes = [vp, i32]
        L.hgks_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.hgks_status_string.argtypes = [i32]
        L.hgks_status_string.restype = ctypes.c_char_p
        L.hgks_last_error.argtypes = [vp]
        L.hgks_last_error.restype = ctypes.c_char_p
        for f in ("hgks_workspace_size", "hgks_init", "hgks_step", "hgks_stats", "hgks_dt", "hgks_residual",
                  "hgks_residual_static", "hgks_fma_probe",
                  "hgks_destroy", "hgks_profile", "hgks_profile_read", "hgks_batch_workspace_size",
                  "hgks_batch_init", "hgks_batch_step", "hgks_batch_stats", "hgks_batch_info"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def make_config(p: dict, precision: int = FP64) -> hgks_config:
    """Fill hgks_config from a workload parameter dict (see workloads.py)."""
    c = hgks_config()
    c.abi_version = ABI_VERSION
    for a in range(3):
        c.n[a] = int(p["n"][a])
        c.lo[a] = float(p["lo"][a])
        c.hi[a] = float(p["hi"][a])
        c.bc[a] = int(p.get("bc", (0, 0, 0))[a])
        c.body_force[a] = float(p.get("body_force", (0.0, 0.0, 0.0))[a])
    c.y_stretch = float(p.get("y_stretch", 0.0))
    c.gamma = float(p.get("gamma", 1.4))
    c.prandtl = float(p.get("prandtl", 1.0))
    c.mu_ref = float(p.get("mu_ref", 0.0))
    c.T_ref = float(p.get("T_ref", 1.0))
    c.mu_exp = float(p.get("mu_exp", 0.0))
    c.T_wall = float(p.get("T_wall", 1.0))
    c.cfl = float(p.get("cfl", 0.5))
    c.rho_ref = float(p.get("rho0", 1.0))
    c.precision = int(precision)
    c.flags = HGKS_FLAG_CONSTANT_MASS_FLUX if p.get("mass_flux_control") else 0
    return c


def _check(st, ctx=None):
    if st != HGKS_OK:
        msg = lib().hgks_status_string(st).decode()
        if ctx is not None:
            msg += " | " + (lib().hgks_last_error(ctx) or b"").decode()
        raise HGKSError(st, msg)


# ---- thin wrappers with the C names ------------------------------------------

def hgks_workspace_size(cfg: hgks_config) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().hgks_workspace_size(ctypes.byref(cfg), ctypes.byref(n)))
    return int(n.value)


def hgks_init(cfg, q_ptr: int, ws_ptr: int, ws_bytes: int, stream_ptr: int, t0: float = 0.0):
    ctx = ctypes.c_void_p(0)
    _check(lib().hgks_init(ctypes.byref(cfg), ctypes.c_void_p(q_ptr), ctypes.c_void_p(ws_ptr), ws_bytes,
                           ctypes.c_void_p(stream_ptr), float(t0), ctypes.byref(ctx)))
    return ctx


def hgks_step(ctx, nsteps: int, dt_fixed: float = 0.0):
    _check(lib().hgks_step(ctx, int(nsteps), float(dt_fixed)), ctx)


def _stats_dict(s: hgks_stats_t) -> dict:
    return {
        "t": s.t, "dt_last": s.dt_last, "steps": s.steps, "Ek": s.Ek, "eps_sol": s.eps_sol,
        "eps_dil": s.eps_dil, "eps_com": s.eps_com, "total": np.array(s.total[:]),
        "max_abs": np.array(s.max_abs[:]), "min_p": s.min_p, "min_rho": s.min_rho, "nonfinite": s.nonfinite,
        "body_force_x": s.body_force_x,
    }


def hgks_stats(ctx) -> dict:
    s = hgks_stats_t()
    _check(lib().hgks_stats(ctx, ctypes.byref(s)), ctx)
    return _stats_dict(s)


def hgks_dt(ctx) -> float:
    d = ctypes.c_double(0.0)
    _check(lib().hgks_dt(ctx, ctypes.byref(d)), ctx)
    return float(d.value)


def hgks_residual(ctx, q_ptr: int, dt: float, L_ptr: int, dL_ptr: int):
    _check(lib().hgks_residual(ctx, ctypes.c_void_p(q_ptr), float(dt), ctypes.c_void_p(L_ptr),
                               ctypes.c_void_p(dL_ptr)), ctx)


def hgks_residual_static(cfg, q_ptr: int, dt: float, L_ptr: int, dL_ptr: int, stream_ptr: int):
    """L and dL/dt with no context and no workspace (the library's static
    device array); asynchronous on the stream."""
    L = lib()
    st = L.hgks_residual_static(ctypes.byref(cfg), ctypes.c_void_p(q_ptr), float(dt), ctypes.c_void_p(L_ptr),
                                ctypes.c_void_p(dL_ptr), ctypes.c_void_p(stream_ptr))
    if st != HGKS_OK:
        raise HGKSError(st, L.hgks_last_error(None).decode())


def hgks_fma_probe(out_ptr: int, blocks: int, iters: int, stream_ptr: int):
    """Enqueue the FP64 FMA-rate probe (16 * iters operations per thread,
    blocks * 256 threads) on the stream."""
    _check(lib().hgks_fma_probe(ctypes.c_void_p(out_ptr), int(blocks), int(iters), ctypes.c_void_p(stream_ptr)), None)


def hgks_profile(ctx, enable: bool):
    _check(lib().hgks_profile(ctx, 1 if enable else 0), ctx)


def hgks_profile_read(ctx) -> dict:
    """{class: (total_ms, launches)} since the last read."""
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    _check(lib().hgks_profile_read(ctx, ms, n), ctx)
    return {PROFILE_CLASSES[c]: (float(ms[c]), int(n[c])) for c in range(4)}


def _cfg_array(cfgs):
    arr = (hgks_config * len(cfgs))()
    for i, c in enumerate(cfgs):
        arr[i] = c
    return arr


def hgks_batch_workspace_size(cfgs) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().hgks_batch_workspace_size(len(cfgs), _cfg_array(cfgs), ctypes.byref(n)))
    return int(n.value)


def hgks_batch_init(cfgs, q_ptrs, ws_ptr: int, ws_bytes: int, stream_ptr: int):
    ctx = ctypes.c_void_p(0)
    qs = (ctypes.c_void_p * len(q_ptrs))(*[ctypes.c_void_p(p) for p in q_ptrs])
    _check(lib().hgks_batch_init(len(cfgs), _cfg_array(cfgs), qs, ctypes.c_void_p(ws_ptr), ws_bytes,
                                 ctypes.c_void_p(stream_ptr), ctypes.byref(ctx)))
    return ctx


def hgks_batch_step(ctx, nsteps: int):
    _check(lib().hgks_batch_step(ctx, int(nsteps)), ctx)


def hgks_batch_stats(ctx, i: int) -> dict:
    s = hgks_stats_t()
    _check(lib().hgks_batch_stats(ctx, int(i), ctypes.byref(s)), ctx)
    return _stats_dict(s)


BATCH_INFO_KEYS = ("instances", "flux_tile_x", "group_mib", "groups", "flux_tiles", "tune_source",
                   "recon_tiles", "cell_blocks")


def hgks_batch_info(ctx) -> dict:
    info = (ctypes.c_int64 * 8)()
    _check(lib().hgks_batch_info(ctx, info), ctx)
    return dict(zip(BATCH_INFO_KEYS, [int(x) for x in info]))


def hgks_destroy(ctx):
    _check(lib().hgks_destroy(ctx))


# ---- convenience object over torch tensors -----------------------------------

class Solver:
    """One simulation: state q (torch float64 [5, nz, ny, nx] on the GPU),
    workspace and stream owned by torch; every step runs in libhgks.so."""

    def __init__(self, params: dict, q0, precision: int = FP64, t0: float = 0.0, device: str = "cuda:0",
                 stream=None):
        import torch

        self.params = params
        self.cfg = make_config(params, precision)
        nx, ny, nz = params["n"]
        q = torch.as_tensor(np.ascontiguousarray(q0) if isinstance(q0, np.ndarray) else q0,
                            dtype=torch.float64, device=device)
        self.q = q.contiguous().clone()
        assert tuple(self.q.shape) == (5, nz, ny, nx), self.q.shape
        self.ws_bytes = hgks_workspace_size(self.cfg)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.q.device)
        # the copies above ran on the current stream; the library's work on its own
        self.stream.wait_stream(torch.cuda.current_stream(self.q.device))
        self.ctx = hgks_init(self.cfg, self.q.data_ptr(), self.ws_ptr, self.ws_bytes, self.stream.cuda_stream, t0)

    def step(self, nsteps: int = 1, dt_fixed: float = 0.0):
        hgks_step(self.ctx, nsteps, dt_fixed)

    def stats(self) -> dict:
        return hgks_stats(self.ctx)

    def dt(self) -> float:
        return hgks_dt(self.ctx)

    def residual(self, q, dt: float):
        import torch

        qd = torch.as_tensor(q, dtype=torch.float64, device=self.q.device).contiguous()
        L = torch.empty_like(qd)
        dL = torch.empty_like(qd)
        self.stream.wait_stream(torch.cuda.current_stream(self.q.device))
        hgks_residual(self.ctx, qd.data_ptr(), dt, L.data_ptr(), dL.data_ptr())
        return L, dL

    def state(self) -> np.ndarray:
        self.stream.synchronize()
        return self.q.cpu().numpy()

    def close(self):
        if getattr(self, "ctx", None) is not None:
            hgks_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """An ensemble of independent instances advanced together (one launch per
    kernel over all instances' tiles, each step a replayed HIP graph, each
    instance with its own CFL time step).  States are torch float64 tensors;
    the workspace and a dedicated stream come from torch."""

    def __init__(self, params_list, q0_list, precision: int = FP64, device: str = "cuda:0"):
        import torch

        self.params = list(params_list)
        self.cfgs = [make_config(p, precision) for p in self.params]
        self.q = []
        for p, q0 in zip(self.params, q0_list):
            nx, ny, nz = p["n"]
            t = torch.as_tensor(np.ascontiguousarray(q0) if isinstance(q0, np.ndarray) else q0,
                                dtype=torch.float64, device=device).contiguous().clone()
            assert tuple(t.shape) == (5, nz, ny, nx), t.shape
            self.q.append(t)
        self.ws_bytes = hgks_batch_workspace_size(self.cfgs)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255
        self.stream = torch.cuda.Stream(device=device)
        torch.cuda.synchronize(device)
        self.ctx = hgks_batch_init(self.cfgs, [t.data_ptr() for t in self.q], self.ws_ptr, self.ws_bytes,
                                   self.stream.cuda_stream)

    def step(self, nsteps: int = 1):
        hgks_batch_step(self.ctx, nsteps)

    def stats(self, i: int) -> dict:
        return hgks_batch_stats(self.ctx, i)

    def info(self) -> dict:
        return hgks_batch_info(self.ctx)

    def synchronize(self):
        self.stream.synchronize()

    def state(self, i: int) -> np.ndarray:
        self.stream.synchronize()
        return self.q[i].cpu().numpy()

    def close(self):
        if getattr(self, "ctx", None) is not None:
            hgks_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
