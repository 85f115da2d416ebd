"""MI355X (gfx950) HSMA reaction potential: thin Python binding over libhsma.so.

Argument marshalling only: every step of the computation runs in the HIP kernels of
``libhsma.so`` (C ABI declared in ``include/hsma.h``).  PyTorch supplies device memory
and streams.  Importing works without a GPU; every compute call requires the built
library and a GPU and raises otherwise (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsma.so")

HSMA_PAIR_FP32 = 0
HSMA_PAIR_FP32_COMP = 1
HSMA_PAIR_FP64 = 2
PAIR_PREC = {"fp32": HSMA_PAIR_FP32, "fp32c": HSMA_PAIR_FP32_COMP, "fp64": HSMA_PAIR_FP64}

STATUS = {0: "HSMA_OK", 1: "HSMA_EINVAL", 2: "HSMA_EDOMAIN", 3: "HSMA_ENOMEM", 4: "HSMA_EBUSY",
          5: "HSMA_EDEVICE", 6: "HSMA_ESTATE"}


class HsmaError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


class TreeOpts(C.Structure):
    _fields_ = [("theta", C.c_double), ("order", C.c_int), ("depth", C.c_int)]


class PlanOpts(C.Structure):
    _fields_ = [("p", C.c_int), ("tau", C.c_double), ("rc_over_a", C.c_double), ("F1", C.c_int),
                ("pair_prec", C.c_int), ("check_set", C.c_int), ("dipole", C.c_int), ("dy_over_Rtau", C.c_double)]


class PlanInfo(C.Structure):
    _fields_ = [("a", C.c_double), ("eps1", C.c_double), ("eps2", C.c_double), ("kappa", C.c_double),
                ("tau", C.c_double), ("R_tau", C.c_double), ("rc", C.c_double), ("gamma", C.c_double),
                ("sigma", C.c_double), ("dbar", C.c_double), ("p", C.c_int), ("K", C.c_int), ("P", C.c_int),
                ("M", C.c_int), ("F1", C.c_int), ("F2", C.c_int), ("pair_prec", C.c_int), ("device", C.c_int),
                ("check_set", C.c_int), ("dipole", C.c_int), ("dy_over_Rtau", C.c_double)]


class Request(C.Structure):
    _fields_ = [("type", C.c_int), ("sys", C.c_int), ("commit", C.c_int), ("k", C.c_int64), ("x", C.c_double),
                ("y", C.c_double), ("z", C.c_double), ("tag", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("type", C.c_int), ("sys", C.c_int), ("status", C.c_int), ("value", C.c_double),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("memory_budget", C.c_size_t), ("max_systems", C.c_int), ("max_batch", C.c_int),
                ("delta_slots", C.c_int), ("energy_slots", C.c_int), ("energy_workgroups", C.c_int),
                ("move_priority", C.c_int)]


class LaunchSettings(C.Structure):
    _fields_ = [("persistent", C.c_int), ("target_items", C.c_int), ("symmetric", C.c_int), ("sym_order", C.c_int),
                ("fit", C.c_int), ("energy_block", C.c_int), ("energy_workgroups", C.c_int)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class TuneTrial(C.Structure):
    _fields_ = [("s", LaunchSettings), ("ms", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("chosen", LaunchSettings), ("ms_start", C.c_double), ("ms_tuned", C.c_double), ("timed", C.c_int),
                ("cached", C.c_int), ("trials", TuneTrial * 32)]


class ServerInfo(C.Structure):
    _fields_ = [("memory_used", C.c_size_t), ("memory_budget", C.c_size_t), ("pending", C.c_int64),
                ("completed", C.c_uint64), ("batches", C.c_uint64), ("batched_requests", C.c_uint64),
                ("systems", C.c_int), ("now", C.c_double)]


REQ_DELTA = 0
REQ_ENERGY = 1

_lib = None
_VP = C.c_void_p
_DP = C.POINTER(C.c_double)


def load_library(path: str | None = None):
    """Load libhsma.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"libhsma.so not built at {path}: run paper_1907_01724_amd/build.py "
                           f"(or __graft_entry__.build())")
    L = C.CDLL(path)
    L.hsma_plan_opts_default.restype = PlanOpts
    L.hsma_plan.argtypes = [C.c_double] * 4 + [C.c_int, C.c_int, C.POINTER(_VP)]
    L.hsma_plan_ex.argtypes = [C.c_double] * 4 + [C.c_int, C.c_int, C.POINTER(PlanOpts), C.POINTER(_VP)]
    L.hsma_plan_destroy.argtypes = [_VP]
    L.hsma_plan_get_info.argtypes = [_VP, C.POINTER(PlanInfo)]
    L.hsma_workspace_bytes.argtypes = [_VP, C.c_int64]
    L.hsma_workspace_bytes.restype = C.c_size_t
    L.hsma_potential.argtypes = [_VP, C.c_int64] + [_VP] * 5 + [_VP, C.c_size_t, _VP]
    L.hsma_energy.argtypes = [_VP, C.c_int64] + [_VP] * 6 + [_VP, C.c_size_t, _VP]
    L.hsma_energy_noalloc.argtypes = [_VP, C.c_int64] + [_VP] * 6 + [_VP]
    L.hsma_debug_intermediates.argtypes = [_VP, C.c_int64, _VP, _VP, _DP, _DP, _DP, _DP]
    L.hsma_stream_check.argtypes = [_VP, _VP]
    L.hsma_status_string.argtypes = [C.c_int]
    L.hsma_status_string.restype = C.c_char_p
    L.hsma_version.restype = C.c_int
    L.hsma_profile_enable.argtypes = [_VP, C.c_int]
    L.hsma_profile_read.argtypes = [_VP, _DP, C.POINTER(C.c_int64)]
    L.hsma_group_create.argtypes = [C.c_int, C.POINTER(_VP), C.POINTER(_VP)]
    L.hsma_group_destroy.argtypes = [_VP]
    L.hsma_plan_group.argtypes = [_VP]
    L.hsma_plan_group.restype = _VP
    L.hsma_batched_workspace_bytes.argtypes = [_VP, C.c_int, C.c_int64, C.c_int64]
    L.hsma_batched_workspace_bytes.restype = C.c_size_t
    L.hsma_energy_batched.argtypes = [_VP, C.c_int, _VP, _VP, C.c_int64, C.c_int64] + [_VP] * 6 + [_VP, C.c_size_t,
                                                                                                   _VP]
    L.hsma_group_stream_check.argtypes = [_VP, _VP]
    L.hsma_group_tune.argtypes = [_VP, C.c_int, C.c_int]
    L.hsma_group_set_symmetric.argtypes = [_VP, C.c_int]
    L.hsma_group_eval_kernel.argtypes = [_VP, C.c_int, C.c_int64, C.c_int64]
    L.hsma_group_eval_kernel.restype = C.c_int
    L.hsma_group_set_fit.argtypes = [_VP, C.c_int]
    L.hsma_group_set_sym_order.argtypes = [_VP, C.c_int]
    L.hsma_group_set_energy_launch.argtypes = [_VP, C.c_int, C.c_int]
    L.hsma_group_autotune_workspace_bytes.argtypes = [_VP, C.c_int, C.c_int64, C.c_int64]
    L.hsma_group_autotune_workspace_bytes.restype = C.c_size_t
    L.hsma_group_get_settings.argtypes = [_VP, C.POINTER(LaunchSettings)]
    L.hsma_group_apply_settings.argtypes = [_VP, C.POINTER(LaunchSettings)]
    L.hsma_group_autotune.argtypes = [_VP, C.c_int, _VP, _VP, C.c_int64, C.c_int64] + [_VP] * 6 + [
        _VP, C.c_size_t, _VP, C.c_int, C.POINTER(TuneResult)]
    L.hsma_system_create_ex.argtypes = [_VP, C.c_int64] + [_VP] * 4 + [C.c_int, _VP, C.POINTER(_VP)]
    L.hsma_kirkwood_workspace_bytes.argtypes = [C.c_int, C.c_int64]
    L.hsma_kirkwood_workspace_bytes.restype = C.c_size_t
    L.hsma_kirkwood.argtypes = [_VP, C.c_int, C.c_int64] + [_VP] * 6 + [_VP, C.c_size_t, _VP]
    L.hsma_tree_workspace_bytes.argtypes = [_VP, C.c_int64, C.POINTER(TreeOpts)]
    L.hsma_tree_workspace_bytes.restype = C.c_size_t
    L.hsma_energy_tree.argtypes = [_VP, C.c_int64] + [_VP] * 6 + [C.POINTER(TreeOpts), _VP, C.c_size_t, _VP]
    L.hsma_field_workspace_bytes.argtypes = [_VP, C.c_int64]
    L.hsma_field_workspace_bytes.restype = C.c_size_t
    L.hsma_field.argtypes = [_VP, C.c_int64] + [_VP] * 9 + [_VP, C.c_size_t, _VP]
    L.hsma_field_batched_workspace_bytes.argtypes = [_VP, C.c_int, C.c_int64, C.c_int64]
    L.hsma_field_batched_workspace_bytes.restype = C.c_size_t
    L.hsma_field_batched.argtypes = [_VP, C.c_int, _VP, _VP, C.c_int64, C.c_int64] + [_VP] * 9 + [_VP, C.c_size_t,
                                                                                                   _VP]
    L.hsma_group_fit_route.argtypes = [_VP, C.c_int]
    L.hsma_group_fit_route.restype = C.c_int
    L.hsma_system_create.argtypes = [_VP, C.c_int64] + [_VP] * 4 + [_VP, C.POINTER(_VP)]
    L.hsma_delta_energy.argtypes = [_VP, C.c_int64, C.c_double, C.c_double, C.c_double, _VP, _VP]
    L.hsma_system_commit.argtypes = [_VP, C.c_int64, C.c_double, C.c_double, C.c_double, _VP]
    L.hsma_system_energy.argtypes = [_VP, _VP, _VP]
    L.hsma_system_positions.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.hsma_system_destroy.argtypes = [_VP]
    L.hsma_system_workspace_bytes.argtypes = [_VP]
    L.hsma_system_workspace_bytes.restype = C.c_size_t
    L.hsma_system_full_energy.argtypes = [_VP, _VP, _VP, C.c_size_t, _VP]
    L.hsma_server_opts_default.restype = ServerOpts
    L.hsma_server_create.argtypes = [C.POINTER(ServerOpts), C.POINTER(_VP)]
    L.hsma_server_destroy.argtypes = [_VP]
    L.hsma_server_add_system.argtypes = [_VP, _VP, C.c_int64] + [_VP] * 4 + [C.POINTER(C.c_int)]
    L.hsma_server_remove_system.argtypes = [_VP, C.c_int]
    L.hsma_server_submit.argtypes = [_VP, C.POINTER(Request), C.c_int]
    L.hsma_server_poll.argtypes = [_VP, C.POINTER(Result), C.c_int]
    L.hsma_server_poll.restype = C.c_int
    L.hsma_server_stats.argtypes = [_VP, C.POINTER(ServerInfo)]
    L.hsma_server_run_load.argtypes = [_VP, C.POINTER(Request), C.POINTER(C.c_double), C.c_int, C.POINTER(Result)]
    for name in ("hsma_plan", "hsma_plan_ex", "hsma_plan_destroy", "hsma_plan_get_info", "hsma_potential",
                 "hsma_energy", "hsma_energy_noalloc", "hsma_debug_intermediates", "hsma_stream_check", "hsma_profile_enable",
                 "hsma_profile_read", "hsma_group_create", "hsma_group_destroy", "hsma_energy_batched",
                 "hsma_group_stream_check", "hsma_group_tune", "hsma_group_set_symmetric", "hsma_group_eval_kernel",
                 "hsma_group_set_fit", "hsma_group_set_sym_order", "hsma_group_set_energy_launch",
                 "hsma_group_get_settings", "hsma_group_apply_settings", "hsma_group_autotune", "hsma_field",
                 "hsma_field_batched",
                 "hsma_kirkwood", "hsma_energy_tree", "hsma_system_create_ex", "hsma_system_create", "hsma_delta_energy",
                 "hsma_system_commit", "hsma_system_energy", "hsma_system_positions", "hsma_system_destroy",
                 "hsma_system_full_energy", "hsma_server_create", "hsma_server_destroy", "hsma_server_add_system",
                 "hsma_server_remove_system", "hsma_server_submit", "hsma_server_stats", "hsma_server_run_load"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(code: int, where: str):
    if code != 0:
        raise HsmaError(code, where)


def _torch():
    import torch  # imported lazily: the binding itself only needs ctypes
    return torch


def _dev_ptr(t, name: str, n: int | None = None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t.data_ptr()


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Workspace:
    """A 256-byte aligned device buffer of at least nbytes (backed by a uint8 tensor)."""

    def __init__(self, nbytes: int, device=None):
        torch = _torch()
        self.nbytes = int(nbytes)
        self.buf = torch.empty(max(self.nbytes, 1) + 256, dtype=torch.uint8, device=device or "cuda")
        p = self.buf.data_ptr()
        self.ptr = p + (-p) % 256


def workspace(nbytes: int, device=None) -> Workspace:
    return Workspace(nbytes, device)


def _ensure(cache: dict, key, nbytes: int, device) -> Workspace:
    w = cache.get(key)
    if w is None or w.nbytes < nbytes:
        w = Workspace(nbytes, device)
        cache[key] = w
    return w


class Plan:
    """One cavity (a, eps1, eps2, kappa) discretised with P surface nodes and M check points.

    check_set: 0 golden-angle lattice, 1 the Gauss-Legendre grid (M = 2p (2p + 1));
    dipole: 0 exact surface dipoles, 1 the +-dy/2 point pairs, 2 a single layer (monopoles only)."""

    def __init__(self, a: float, eps1: float, eps2: float, kappa: float, P: int, M: int, p: int | None = None,
                 tau: float = 0.1, rc_over_a: float | None = None, F1: int | None = None,
                 pair_prec: str | int = "fp32c", check_set: int = 0, dipole: int = 0,
                 dy_over_Rtau: float | None = None):
        L = load_library()
        o = L.hsma_plan_opts_default()
        if p is not None:
            o.p = int(p)
        o.tau = float(tau)
        if rc_over_a is not None:
            o.rc_over_a = float(rc_over_a)
        if F1 is not None:
            o.F1 = int(F1)
        o.pair_prec = PAIR_PREC[pair_prec] if isinstance(pair_prec, str) else int(pair_prec)
        o.check_set = int(check_set)
        o.dipole = int(dipole)
        if dy_over_Rtau is not None:
            o.dy_over_Rtau = float(dy_over_Rtau)
        h = _VP()
        _check(L.hsma_plan_ex(float(a), float(eps1), float(eps2), float(kappa), int(P), int(M), C.byref(o),
                              C.byref(h)), "hsma_plan_ex")
        self._h = h
        self._ws = {}
        inf = PlanInfo()
        _check(L.hsma_plan_get_info(h, C.byref(inf)), "hsma_plan_get_info")
        self.info = {k: getattr(inf, k) for k, _ in PlanInfo._fields_}

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load_library().hsma_plan_destroy(self._h)
            self._h = None
            self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, N: int) -> int:
        return int(load_library().hsma_workspace_bytes(self._h, int(N)))

    def _workspace(self, N: int, device) -> Workspace:
        return _ensure(self._ws, (int(N), str(device)), self.workspace_bytes(N), device)

    def potential(self, x, y, z, q, phi=None, stream=None, ws: Workspace | None = None):
        torch = _torch()
        N = x.numel()
        if phi is None:
            phi = torch.empty(N, dtype=torch.float64, device=x.device)
        w = ws if ws is not None else self._workspace(N, x.device)
        _check(load_library().hsma_potential(self._h, N, _dev_ptr(x, "x", N), _dev_ptr(y, "y", N),
                                             _dev_ptr(z, "z", N), _dev_ptr(q, "q", N), _dev_ptr(phi, "phi", N),
                                             w.ptr, w.nbytes, _stream_ptr(stream)), "hsma_potential")
        return phi

    def energy_noalloc(self, x, y, z, q, phi=None, E=None, stream=None):
        """hsma_energy on the library's own device scratch (no workspace, nothing allocated by
        the library); E must be given for the call to allocate nothing here either."""
        torch = _torch()
        N = x.numel()
        if E is None:
            E = torch.empty(1, dtype=torch.float64, device=x.device)
        _check(load_library().hsma_energy_noalloc(self._h, N, _dev_ptr(x, "x", N), _dev_ptr(y, "y", N),
                                                  _dev_ptr(z, "z", N), _dev_ptr(q, "q", N),
                                                  _dev_ptr(phi, "phi", N) if phi is not None else None,
                                                  _dev_ptr(E, "E", 1), _stream_ptr(stream)),
               "hsma_energy_noalloc")
        return E

    def energy(self, x, y, z, q, phi=None, E=None, stream=None, ws: Workspace | None = None):
        torch = _torch()
        N = x.numel()
        if E is None:
            E = torch.empty(1, dtype=torch.float64, device=x.device)
        w = ws if ws is not None else self._workspace(N, x.device)
        _check(load_library().hsma_energy(self._h, N, _dev_ptr(x, "x", N), _dev_ptr(y, "y", N),
                                          _dev_ptr(z, "z", N), _dev_ptr(q, "q", N),
                                          _dev_ptr(phi, "phi", N) if phi is not None else None,
                                          _dev_ptr(E, "E", 1), w.ptr, w.nbytes, _stream_ptr(stream)),
               "hsma_energy")
        return E

    def field_workspace_bytes(self, N: int) -> int:
        return int(load_library().hsma_field_workspace_bytes(self._h, int(N)))

    def field(self, x, y, z, q, phi=None, E=None, stream=None, ws: Workspace | None = None):
        """Potential and field E = -grad Phi_RF at every ion (images held fixed).
        Returns (phi, field) with field an (N, 3) float64 device tensor."""
        torch = _torch()
        N = x.numel()
        if phi is None:
            phi = torch.empty(N, dtype=torch.float64, device=x.device)
        f = torch.empty((3, N), dtype=torch.float64, device=x.device)
        w = ws if ws is not None else _ensure(self._ws, ("field", N, str(x.device)), self.field_workspace_bytes(N),
                                              x.device)
        _check(load_library().hsma_field(self._h, N, _dev_ptr(x, "x", N), _dev_ptr(y, "y", N), _dev_ptr(z, "z", N),
                                         _dev_ptr(q, "q", N), _dev_ptr(phi, "phi", N), f[0].data_ptr(),
                                         f[1].data_ptr(), f[2].data_ptr(),
                                         _dev_ptr(E, "E", 1) if E is not None else None, w.ptr, w.nbytes,
                                         _stream_ptr(stream)), "hsma_field")
        return phi, f.t()

    def kirkwood(self, x, y, z, q, order: int = 40, phi=None, E=None, stream=None, ws: Workspace | None = None):
        """The truncated Kirkwood series (Sec. 2.2) for this plan's cavity, in FP64: potentials
        at the ions (and the energy when E is given).  Returns phi."""
        torch = _torch()
        N = x.numel()
        if phi is None:
            phi = torch.empty(N, dtype=torch.float64, device=x.device)
        lib = load_library()
        w = ws if ws is not None else _ensure(self._ws, ("kirkwood", int(order), N, str(x.device)),
                                              int(lib.hsma_kirkwood_workspace_bytes(int(order), N)), x.device)
        _check(lib.hsma_kirkwood(self._h, int(order), N, _dev_ptr(x, "x", N), _dev_ptr(y, "y", N), _dev_ptr(z, "z", N),
                                 _dev_ptr(q, "q", N), _dev_ptr(phi, "phi", N),
                                 _dev_ptr(E, "E", 1) if E is not None else None, w.ptr, w.nbytes,
                                 _stream_ptr(stream)), "hsma_kirkwood")
        return phi

    def tree_workspace_bytes(self, N: int, theta: float = 0.5, order: int = 4, depth: int = 0) -> int:
        o = TreeOpts(float(theta), int(order), int(depth))
        return int(load_library().hsma_tree_workspace_bytes(self._h, int(N), C.byref(o)))

    def energy_tree(self, x, y, z, q, theta: float = 0.5, order: int = 4, depth: int = 0, phi=None, E=None,
                    stream=None, ws: Workspace | None = None):
        """Potentials (and the energy when E is given) with the Kelvin-image sum by the treecode
        (opening angle theta, multipole order 2, 4, 6, 8 or 10; depth 0 = from N).  Returns phi."""
        torch = _torch()
        N = x.numel()
        if phi is None:
            phi = torch.empty(N, dtype=torch.float64, device=x.device)
        lib = load_library()
        o = TreeOpts(float(theta), int(order), int(depth))
        nb = int(lib.hsma_tree_workspace_bytes(self._h, N, C.byref(o)))
        if nb == 0:
            raise RuntimeError("hsma_tree_workspace_bytes: invalid arguments")
        w = ws if ws is not None else _ensure(self._ws, ("tree", N, float(theta), int(order), int(depth),
                                                         str(x.device)), nb, x.device)
        _check(lib.hsma_energy_tree(self._h, N, _dev_ptr(x, "x", N), _dev_ptr(y, "y", N), _dev_ptr(z, "z", N),
                                    _dev_ptr(q, "q", N), _dev_ptr(phi, "phi", N),
                                    _dev_ptr(E, "E", 1) if E is not None else None, C.byref(o), w.ptr, w.nbytes,
                                    _stream_ptr(stream)), "hsma_energy_tree")
        return phi

    def intermediates(self, N: int, device, stream=None):
        """Check fields u, v and surface strengths Q', D' of the last call with this workspace."""
        import numpy as np
        inf = self.info
        u = np.zeros(inf["M"])
        v = np.zeros(inf["M"])
        Q = np.zeros(inf["P"])
        D = np.zeros(inf["P"])
        ws_ptr = self._workspace(N, device).ptr
        p = lambda a: a.ctypes.data_as(_DP)  # noqa: E731
        _check(load_library().hsma_debug_intermediates(self._h, int(N), ws_ptr, _stream_ptr(stream), p(u), p(v),
                                                       p(Q), p(D)), "hsma_debug_intermediates")
        return u, v, Q, D

    @property
    def group(self):
        """Handle of the one-plan group this plan owns (for profiling)."""
        return load_library().hsma_plan_group(self._h)

    def tune(self, persistent: bool = False, target_items: int = 65536):
        _check(load_library().hsma_group_tune(self.group, 1 if persistent else 0, int(target_items)),
               "hsma_group_tune")

    def set_symmetric(self, mode: int = 1):
        """Symmetric Kelvin kernel: 0 never, 1 for large launches (default), 2 / 3 always with ion
        blocks of 256 / 512."""
        _check(load_library().hsma_group_set_symmetric(self.group, int(mode)), "hsma_group_set_symmetric")

    def set_sym_order(self, mode: int = 0):
        """Item order of the symmetric kernel: 0 automatic, 1 each system's surface items after
        its block pairs, 2 all block pairs first (bit-identical results)."""
        _check(load_library().hsma_group_set_sym_order(self.group, int(mode)), "hsma_group_set_sym_order")

    def eval_kernel(self, N: int) -> int:
        return int(load_library().hsma_group_eval_kernel(self.group, 1, int(N), int(N)))

    def set_fit(self, mode: int = 0):
        """Fit apply: 0 automatic, 1 GEMV, 2 FP32 MFMA, 3 split-BF16x3 MFMA, 4 split-BF16x6 MFMA
        (FP32 pair modes)."""
        _check(load_library().hsma_group_set_fit(self.group, int(mode)), "hsma_group_set_fit")

    def fit_route(self) -> int:
        """1 GEMV, 2 FP32 MFMA, 3 split-BF16x3 MFMA, 4 split-BF16x6 MFMA."""
        return int(load_library().hsma_group_fit_route(self.group, 1))

    def profile(self, on: bool = True):
        _profile(self.group, on)

    def profile_read(self) -> dict:
        return _profile_read(self.group)

    def stream_check(self, stream=None) -> int:
        """Synchronise; return 0 or the status code (2 = an ion outside the cavity)."""
        return int(load_library().hsma_stream_check(self._h, _stream_ptr(stream)))


STAGES = ("pack", "check", "fit", "eval", "finish")


def _profile(group_handle, on: bool):
    _check(load_library().hsma_profile_enable(group_handle, 1 if on else 0), "hsma_profile_enable")


def _profile_read(group_handle) -> dict:
    ms = (C.c_double * 5)()
    cnt = (C.c_int64 * 5)()
    _check(load_library().hsma_profile_read(group_handle, ms, cnt), "hsma_profile_read")
    return {s: (ms[i], cnt[i]) for i, s in enumerate(STAGES)}


class Group:
    """Plans sharing one discretisation, evaluated together over many ion configurations."""

    def __init__(self, plans):
        L = load_library()
        self.plans = list(plans)
        arr = (_VP * len(self.plans))(*[p.handle for p in self.plans])
        h = _VP()
        _check(L.hsma_group_create(len(self.plans), arr, C.byref(h)), "hsma_group_create")
        self._h = h
        self._ws = {}

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            load_library().hsma_group_destroy(self._h)
            self._h = None
            self._ws = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, nsys: int, total_n: int, max_n: int) -> int:
        return int(load_library().hsma_batched_workspace_bytes(self._h, int(nsys), int(total_n), int(max_n)))

    def energy(self, offsets, x, y, z, q, total_n: int, max_n: int, plan_of=None, phi=None, E=None, stream=None,
               ws=None):
        """Potentials and energies of nsys systems; offsets: int64 device tensor of nsys + 1."""
        torch = _torch()
        nsys = offsets.numel() - 1
        if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
            raise TypeError("offsets must be a contiguous int64 device tensor")
        if plan_of is not None and (plan_of.dtype != torch.int32 or not plan_of.is_cuda or plan_of.numel() != nsys):
            raise TypeError("plan_of must be an int32 device tensor of nsys entries")
        if E is None:
            E = torch.empty(nsys, dtype=torch.float64, device=x.device)
        w = ws if ws is not None else _ensure(self._ws, (nsys, int(total_n), int(max_n), str(x.device)),
                                              self.workspace_bytes(nsys, total_n, max_n), x.device)
        _check(load_library().hsma_energy_batched(
            self._h, nsys, offsets.data_ptr(), plan_of.data_ptr() if plan_of is not None else None, int(total_n),
            int(max_n), _dev_ptr(x, "x", total_n), _dev_ptr(y, "y", total_n), _dev_ptr(z, "z", total_n),
            _dev_ptr(q, "q", total_n), _dev_ptr(phi, "phi", total_n) if phi is not None else None,
            _dev_ptr(E, "E", nsys), w.ptr, w.nbytes, _stream_ptr(stream)), "hsma_energy_batched")
        return E

    def potential(self, offsets, x, y, z, q, total_n: int, max_n: int, plan_of=None, phi=None, stream=None,
                  ws=None):
        """Potentials alone (hsma_energy_batched with E = NULL: the launch in the group's pair
        precision, no energy launch).  Returns phi."""
        torch = _torch()
        nsys = offsets.numel() - 1
        if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
            raise TypeError("offsets must be a contiguous int64 device tensor")
        if plan_of is not None and (plan_of.dtype != torch.int32 or not plan_of.is_cuda or plan_of.numel() != nsys):
            raise TypeError("plan_of must be an int32 device tensor of nsys entries")
        if phi is None:
            phi = torch.empty(int(total_n), dtype=torch.float64, device=x.device)
        w = ws if ws is not None else _ensure(self._ws, (nsys, int(total_n), int(max_n), str(x.device)),
                                              self.workspace_bytes(nsys, total_n, max_n), x.device)
        _check(load_library().hsma_energy_batched(
            self._h, nsys, offsets.data_ptr(), plan_of.data_ptr() if plan_of is not None else None, int(total_n),
            int(max_n), _dev_ptr(x, "x", total_n), _dev_ptr(y, "y", total_n), _dev_ptr(z, "z", total_n),
            _dev_ptr(q, "q", total_n), _dev_ptr(phi, "phi", total_n), None, w.ptr, w.nbytes,
            _stream_ptr(stream)), "hsma_energy_batched")
        return phi

    def field(self, offsets, x, y, z, q, total_n: int, max_n: int, plan_of=None, phi=None, E=None, stream=None,
              ws=None):
        """Potentials, fields (total_n x 3) and energies of nsys systems (E=False: no energies, so no
        energy launch)."""
        torch = _torch()
        nsys = offsets.numel() - 1
        if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
            raise TypeError("offsets must be a contiguous int64 device tensor")
        if plan_of is not None and (plan_of.dtype != torch.int32 or not plan_of.is_cuda or plan_of.numel() != nsys):
            raise TypeError("plan_of must be an int32 device tensor of nsys entries")
        if E is None:
            E = torch.empty(nsys, dtype=torch.float64, device=x.device)
        if phi is None:
            phi = torch.empty(int(total_n), dtype=torch.float64, device=x.device)
        f = torch.empty((3, int(total_n)), dtype=torch.float64, device=x.device)
        e_ptr = None if E is False else _dev_ptr(E, "E", nsys)
        lib = load_library()
        w = ws if ws is not None else _ensure(
            self._ws, ("field", nsys, int(total_n), int(max_n), str(x.device)),
            int(lib.hsma_field_batched_workspace_bytes(self._h, nsys, int(total_n), int(max_n))), x.device)
        _check(lib.hsma_field_batched(
            self._h, nsys, offsets.data_ptr(), plan_of.data_ptr() if plan_of is not None else None, int(total_n),
            int(max_n), _dev_ptr(x, "x", total_n), _dev_ptr(y, "y", total_n), _dev_ptr(z, "z", total_n),
            _dev_ptr(q, "q", total_n), _dev_ptr(phi, "phi", total_n), f[0].data_ptr(), f[1].data_ptr(),
            f[2].data_ptr(), e_ptr, w.ptr, w.nbytes, _stream_ptr(stream)), "hsma_field_batched")
        return phi, f.t(), (None if E is False else E)

    def tune(self, persistent: bool = False, target_items: int = 65536):
        _check(load_library().hsma_group_tune(self._h, 1 if persistent else 0, int(target_items)), "hsma_group_tune")

    def set_symmetric(self, mode: int = 1):
        """Symmetric Kelvin kernel: 0 never, 1 for large launches (default), 2 / 3 always with ion
        blocks of 256 / 512."""
        _check(load_library().hsma_group_set_symmetric(self._h, int(mode)), "hsma_group_set_symmetric")

    def set_sym_order(self, mode: int = 0):
        """Item order of the symmetric kernel: 0 automatic, 1 each system's surface items after
        its block pairs, 2 all block pairs first (bit-identical results)."""
        _check(load_library().hsma_group_set_sym_order(self._h, int(mode)), "hsma_group_set_sym_order")

    def eval_kernel(self, nsys: int, total_n: int, max_n: int) -> int:
        """Ion-block size of the symmetric Kelvin kernel these sizes would use, or 0."""
        return int(load_library().hsma_group_eval_kernel(self._h, int(nsys), int(total_n), int(max_n)))

    def set_fit(self, mode: int = 0):
        """Fit apply: 0 automatic, 1 GEMV, 2 FP32 MFMA, 3 split-BF16x3 MFMA, 4 split-BF16x6 MFMA
        (FP32 pair modes)."""
        _check(load_library().hsma_group_set_fit(self._h, int(mode)), "hsma_group_set_fit")

    def fit_route(self, nsys: int) -> int:
        """1 GEMV, 2 FP32 MFMA, 3 split-BF16x3 MFMA, 4 split-BF16x6 MFMA."""
        return int(load_library().hsma_group_fit_route(self._h, int(nsys)))

    def autotune_workspace_bytes(self, nsys: int, total_n: int, max_n: int) -> int:
        return int(load_library().hsma_group_autotune_workspace_bytes(self._h, int(nsys), int(total_n), int(max_n)))

    def set_energy_launch(self, block: int = 0, workgroups: int = 0):
        """Energy launch: ions per block (0 automatic, 128, 256, 512) and grid (0: one item per wave;
        > 0: persistent grid of that many workgroups)."""
        _check(load_library().hsma_group_set_energy_launch(self._h, int(block), int(workgroups)),
               "hsma_group_set_energy_launch")

    def settings(self) -> dict:
        s = LaunchSettings()
        _check(load_library().hsma_group_get_settings(self._h, C.byref(s)), "hsma_group_get_settings")
        return s.as_dict()

    def apply_settings(self, settings: dict):
        s = LaunchSettings(**{k: int(settings[k]) for k, _ in LaunchSettings._fields_})
        _check(load_library().hsma_group_apply_settings(self._h, C.byref(s)), "hsma_group_apply_settings")

    def autotune(self, offsets, x, y, z, q, total_n: int, max_n: int, plan_of=None, phi=None, E=None, stream=None,
                 ws=None, force: bool = False) -> dict:
        """Times the call energy(..., phi=phi, E=E) (E None: potentials alone) under candidate launch
        settings and leaves the fastest on the group (hsma_group_autotune); overwrites phi, E, ws."""
        torch = _torch()
        nsys = offsets.numel() - 1
        if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
            raise TypeError("offsets must be a contiguous int64 device tensor")
        if plan_of is not None and (plan_of.dtype != torch.int32 or not plan_of.is_cuda or plan_of.numel() != nsys):
            raise TypeError("plan_of must be an int32 device tensor of nsys entries")
        w = ws if ws is not None else _ensure(self._ws, ("tune", nsys, int(total_n), int(max_n), str(x.device)),
                                              self.autotune_workspace_bytes(nsys, total_n, max_n), x.device)
        r = TuneResult()
        _check(load_library().hsma_group_autotune(
            self._h, nsys, offsets.data_ptr(), plan_of.data_ptr() if plan_of is not None else None, int(total_n),
            int(max_n), _dev_ptr(x, "x", total_n), _dev_ptr(y, "y", total_n), _dev_ptr(z, "z", total_n),
            _dev_ptr(q, "q", total_n), _dev_ptr(phi, "phi", total_n) if phi is not None else None,
            _dev_ptr(E, "E", nsys) if E is not None else None, w.ptr, w.nbytes, _stream_ptr(stream),
            1 if force else 0, C.byref(r)), "hsma_group_autotune")
        return {"chosen": r.chosen.as_dict(), "ms_start": r.ms_start, "ms_tuned": r.ms_tuned, "timed": r.timed,
                "cached": bool(r.cached),
                "trials": [{"settings": r.trials[i].s.as_dict(), "ms": r.trials[i].ms} for i in range(min(r.timed, 32))]}

    def profile(self, on: bool = True):
        _profile(self._h, on)

    def profile_read(self) -> dict:
        return _profile_read(self._h)

    def stream_check(self, stream=None) -> int:
        return int(load_library().hsma_group_stream_check(self._h, _stream_ptr(stream)))


class System:
    """A resident ion configuration for single-ion-move energy changes (Monte Carlo)."""

    def __init__(self, plan: Plan, x, y, z, q, stream=None, coulomb: bool = False):
        """coulomb: the energy (and every move's change) also holds the direct Coulomb energy
        of the ions in the cavity."""
        L = load_library()
        self.plan = plan
        self.n = x.numel()
        h = _VP()
        _check(L.hsma_system_create_ex(plan.handle, self.n, _dev_ptr(x, "x", self.n), _dev_ptr(y, "y", self.n),
                                       _dev_ptr(z, "z", self.n), _dev_ptr(q, "q", self.n), 1 if coulomb else 0,
                                       _stream_ptr(stream), C.byref(h)), "hsma_system_create_ex")
        self._h = h
        self.device = x.device

    @property
    def handle(self):
        return self._h

    def delta_energy(self, k: int, pos, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        _check(load_library().hsma_delta_energy(self._h, int(k), float(pos[0]), float(pos[1]), float(pos[2]),
                                                _dev_ptr(out, "dE"), _stream_ptr(stream)), "hsma_delta_energy")
        return out

    def commit(self, k: int, pos, stream=None):
        _check(load_library().hsma_system_commit(self._h, int(k), float(pos[0]), float(pos[1]), float(pos[2]),
                                                 _stream_ptr(stream)), "hsma_system_commit")

    def energy(self, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        _check(load_library().hsma_system_energy(self._h, _dev_ptr(out, "E"), _stream_ptr(stream)),
               "hsma_system_energy")
        return out

    def workspace_bytes(self) -> int:
        return int(load_library().hsma_system_workspace_bytes(self._h))

    def full_energy(self, out=None, stream=None, ws: Workspace | None = None):
        """A fresh FP64 full evaluation of the current energy (state unchanged); synchronises."""
        torch = _torch()
        L = load_library()
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        if ws is None:
            ws = Workspace(int(L.hsma_system_workspace_bytes(self._h)), self.device)
        _check(L.hsma_system_full_energy(self._h, _dev_ptr(out, "E"), ws.ptr, ws.nbytes, _stream_ptr(stream)),
               "hsma_system_full_energy")
        torch.cuda.synchronize()
        return out

    def positions(self, stream=None):
        torch = _torch()
        xyz = [torch.empty(self.n, dtype=torch.float64, device=self.device) for _ in range(3)]
        _check(load_library().hsma_system_positions(self._h, *[t.data_ptr() for t in xyz], _stream_ptr(stream)),
               "hsma_system_positions")
        return xyz

    def close(self):
        if self._h:
            load_library().hsma_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def requests_array(reqs) -> "C.Array":
    """reqs: iterable of (type, sys, commit, k, x, y, z) tuples -> ctypes array of Request."""
    reqs = list(reqs)
    arr = (Request * max(len(reqs), 1))()
    for i, r in enumerate(reqs):
        t, sys_id, commit, k, x, y, z = r
        arr[i] = Request(int(t), int(sys_id), int(commit), int(k), float(x), float(y), float(z), i)
    return arr


class Server:
    """Continuous-batching request server over resident systems (see hsma_server_* in hsma.h)."""

    def __init__(self, memory_budget: int = 0, max_systems: int = 1024, max_batch: int = 256, delta_slots: int = 1,
                 energy_slots: int = 2, energy_workgroups: int = 0, move_priority: int = 1):
        L = load_library()
        o = ServerOpts(int(memory_budget), int(max_systems), int(max_batch), int(delta_slots), int(energy_slots),
                       int(energy_workgroups), int(move_priority))
        h = _VP()
        _check(L.hsma_server_create(C.byref(o), C.byref(h)), "hsma_server_create")
        self._h = h
        self._plans = []

    def add_system(self, plan: Plan, x, y, z, q) -> int:
        n = x.numel()
        i = C.c_int(-1)
        _check(load_library().hsma_server_add_system(self._h, plan.handle, n, _dev_ptr(x, "x", n), _dev_ptr(y, "y", n),
                                                     _dev_ptr(z, "z", n), _dev_ptr(q, "q", n), C.byref(i)),
               "hsma_server_add_system")
        self._plans.append(plan)  # plans must outlive the server's systems
        return i.value

    def remove_system(self, sys_id: int):
        _check(load_library().hsma_server_remove_system(self._h, int(sys_id)), "hsma_server_remove_system")

    def submit(self, reqs):
        n = len(reqs)
        if n == 0:
            return
        arr = reqs if isinstance(reqs, C.Array) else requests_array(reqs)
        _check(load_library().hsma_server_submit(self._h, arr, n), "hsma_server_submit")

    def poll(self, max_results: int = 4096):
        buf = (Result * max_results)()
        n = load_library().hsma_server_poll(self._h, buf, max_results)
        return [buf[i] for i in range(n)]

    def stats(self) -> dict:
        inf = ServerInfo()
        _check(load_library().hsma_server_stats(self._h, C.byref(inf)), "hsma_server_stats")
        return {k: getattr(inf, k) for k, _ in ServerInfo._fields_}

    def run_load(self, reqs, arrival):
        """Open-loop load: request i submitted at arrival[i] s; returns the results in order."""
        arr = requests_array(reqs)
        n = len(reqs)
        times = (C.c_double * max(n, 1))(*[float(t) for t in arrival])
        out = (Result * max(n, 1))()
        _check(load_library().hsma_server_run_load(self._h, arr, times, n, out), "hsma_server_run_load")
        return [out[i] for i in range(n)]

    def close(self):
        if self._h:
            load_library().hsma_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def status_string(code: int) -> str:
    return load_library().hsma_status_string(int(code)).decode()
