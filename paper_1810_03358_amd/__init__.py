"""MI355X force-field energy/gradient and local minimization (arXiv 1810.03358).

Thin Python binding of the C ABI in ``include/ff.h``: argument marshalling
only.  Every evaluation and every optimizer step runs in the HIP kernels of
``libff_mi355x.so``; PyTorch supplies device memory and the stream.  Nothing
here computes the force field or takes an optimizer decision, and there is no
CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from ._native import (  # noqa: F401
    FF_GD, FF_FGM, FF_CG, FF_LBFGS, FF_HB, FF_OGM, FF_FP64, FF_FP32_ACC64,
    FF_CONVERGED, FF_MAX_ITER, FF_LS_FAILED, FF_NONFINITE_START, FF_DIVERGED,
    FF_LS_DEFAULT, FF_LS_PAR, FF_LS_H, FF_MIN_RESUME, FF_MIN_NO_CERTIFY,
    FF_OK, FF_ERR_ARG, FF_ERR_HIP, FF_ERR_WORKSPACE, FF_ERR_UNSUPPORTED,
    FF_CG_PRP, FF_CG_FR, FF_CG_HS, FF_CG_PRP_PLUS, FF_CG_CD, FF_CG_LS, FF_CG_DY,
)
CG_BETAS = {"prp": FF_CG_PRP, "fr": FF_CG_FR, "hs": FF_CG_HS, "prp+": FF_CG_PRP_PLUS, "cd": FF_CG_CD,
            "ls": FF_CG_LS, "dy": FF_CG_DY}

METHODS = {"gd": FF_GD, "fgm": FF_FGM, "cg": FF_CG, "lbfgs": FF_LBFGS, "hb": FF_HB, "ogm": FF_OGM}
PRECISIONS = {"fp64": FF_FP64, "fp32": FF_FP32_ACC64}
TERMS = {FF_CONVERGED: "converged", FF_MAX_ITER: "max_iter", FF_LS_FAILED: "ls_failed",
         FF_NONFINITE_START: "nonfinite_start", FF_DIVERGED: "diverged"}


class FFError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where} failed with status {status}: {N.last_error()}")
        self.status = status


def _check(status: int, where: str):
    if status != FF_OK:
        raise FFError(status, where)


class HostSystem:
    """ff_system view of a system dict (host arrays kept alive here)."""

    def __init__(self, d: dict):
        f64 = lambda k: np.ascontiguousarray(d[k], dtype=np.float64).ravel()  # noqa: E731
        i32 = lambda k: np.ascontiguousarray(d[k], dtype=np.int32).ravel()  # noqa: E731
        self.arrays = dict(q=f64("q"), sigma=f64("sigma"), eps=f64("eps"),
                           bond=i32("bonds"), bond_k=f64("bond_k"), bond_r0=f64("bond_r0"),
                           angle=i32("angles"), angle_k=f64("angle_k"), angle_t0=f64("angle_t0"),
                           dihedral=i32("dihedrals"), dihedral_v=f64("dihedral_v"))
        a = self.arrays
        dp = lambda v: v.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        ip = lambda v: v.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
        self.n = int(d["n_atoms"])
        self.c = N.FFSystem(self.n, dp(a["q"]), dp(a["sigma"]), dp(a["eps"]),
                            len(a["bond_k"]), ip(a["bond"]), dp(a["bond_k"]), dp(a["bond_r0"]),
                            len(a["angle_k"]), ip(a["angle"]), dp(a["angle_k"]), dp(a["angle_t0"]),
                            len(a["dihedral"]) // 4, ip(a["dihedral"]), dp(a["dihedral_v"]),
                            float(d["coulomb_c"]))


def workspace_bytes(system: dict, m_max: int = 10) -> int:
    return int(N.load().ff_workspace_bytes(C.byref(HostSystem(system).c), m_max))


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def tile_configs() -> list:
    """Shapes of the pair-kernel tile configurations:
    (block, waves32, ipl32, waves64, ipl64) per index."""
    lib = N.load()
    out = []
    for k in range(int(lib.ff_num_tile_configs())):
        v = [C.c_int32() for _ in range(5)]
        _check(lib.ff_tile_config_info(k, *[C.byref(x) for x in v]), "ff_tile_config_info")
        out.append(tuple(x.value for x in v))
    return out


def autotune(system, x: torch.Tensor, precision: str | int = "fp32", reps: int = 5, device="cuda", stream=None):
    """Time every tile configuration and chunk length on E+grad evaluations of
    ``system`` (one dict or a list) at ``x`` and return
    ((tile_config, chunk), ms_per_eval) of the fastest."""
    lib = N.load()
    systems = list(system) if isinstance(system, (list, tuple)) else [system]
    hosts = [HostSystem(d) for d in systems]
    arr = (N.FFSystem * len(hosts))(*[h.c for h in hosts])
    nbytes = int(lib.ff_autotune_workspace_bytes(arr, len(hosts)))
    if nbytes == 0:
        raise FFError(FF_ERR_ARG, "ff_autotune_workspace_bytes")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=torch.device(device))
    ptr = (ws.data_ptr() + 255) // 256 * 256
    if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.is_cuda and x.is_contiguous()):
        raise ValueError("coordinates must be a contiguous float64 CUDA tensor")
    cfg, ch, ms = C.c_int32(), C.c_int32(), C.c_double()
    _check(lib.ff_autotune(arr, len(hosts), C.c_void_p(x.data_ptr()), C.c_void_p(ptr), nbytes,
                           int(PRECISIONS.get(precision, precision)), int(reps), _stream_ptr(stream), C.byref(cfg), C.byref(ch),
                           C.byref(ms)), "ff_autotune")
    del ws
    return (cfg.value, ch.value), ms.value


def _out_tensor(t, numel: int, x: torch.Tensor, name: str) -> torch.Tensor:
    """An output buffer the kernels write numel float64 values into: checked
    like the coordinates x (already checked to be a CUDA tensor), since the
    kernels write through its raw pointer."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64, not {t.dtype}")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, {numel} needed")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != x.device:
        raise ValueError(f"{name} is on {t.device}, the coordinates on {x.device}")
    return t


def energy_grad_noalloc(system: dict, x: torch.Tensor, out_e: torch.Tensor, out_g: torch.Tensor | None = None,
                        precision: str | int = "fp64", stream=None):
    """E and grad E of one system at x through ff_energy_grad_noalloc: no
    context, no workspace; the library's static device scratch instead.  The
    caller passes the outputs (out_e: >= 1 float64 entry, out_g: like x or
    None).  Blocks until the packed system is on the device, then returns with
    the evaluation enqueued on the stream."""
    hs = HostSystem(system)
    if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.is_cuda and x.is_contiguous()
            and x.numel() == 3 * hs.n):
        raise ValueError("coordinates must be a contiguous float64 CUDA tensor with 3*n_atoms elements")
    _out_tensor(out_e, 1, x, "out_e")
    if out_g is not None:
        _out_tensor(out_g, x.numel(), x, "out_g")
    _check(N.load().ff_energy_grad_noalloc(C.byref(hs.c), C.c_void_p(x.data_ptr()), C.c_void_p(out_e.data_ptr()),
                                           C.c_void_p(out_g.data_ptr()) if out_g is not None else None,
                                           int(PRECISIONS.get(precision, precision)), _stream_ptr(stream)),
           "ff_energy_grad_noalloc")
    return out_e, out_g


class Context:
    """Prepared system(s) on one GPU: workspace (torch uint8 tensor) + ff_ctx.

    ``system`` is one system dict or a list of them (a batch, minimized
    together; coordinates are then concatenated in list order)."""

    def __init__(self, system, m_max: int = 10, device="cuda", stream=None, tiling=None):
        """``tiling`` = (tile_config, chunk) or (tile_config, chunk,
        chunk64) names the pair-kernel tiling (chunk64: the FP64 kernel's
        chunk length, else `chunk`; e.g. from :func:`autotune`); None lets
        the library choose.  ``self.tiling`` is the (tile_config, chunk,
        chunk64) in use."""
        lib = N.load()
        self.is_batch = isinstance(system, (list, tuple))
        systems = list(system) if self.is_batch else [system]
        self.hosts = [HostSystem(d) for d in systems]
        self.host = self.hosts[0]
        self.n_sys = len(self.hosts)
        self.sizes = [h.n for h in self.hosts]
        self.n = sum(self.sizes)
        self.device = torch.device(device)
        self._sys_array = (N.FFSystem * self.n_sys)(*[h.c for h in self.hosts])
        if tiling is None:
            nbytes = int(lib.ff_workspace_bytes_batch(self._sys_array, self.n_sys, m_max))
        else:
            tiling = tuple(int(v) for v in tiling)
            if len(tiling) not in (2, 3):
                raise ValueError("tiling must be (tile_config, chunk) or (tile_config, chunk, chunk64)")
            tiling = tiling if len(tiling) == 3 else tiling + (tiling[1],)
            nbytes = int(lib.ff_workspace_bytes_tiled(self._sys_array, self.n_sys, m_max, *tiling))
        if nbytes == 0:
            raise FFError(FF_ERR_ARG, "ff_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        ctx = C.c_void_p()
        if tiling is None:
            _check(lib.ff_create_batch(self._sys_array, self.n_sys, C.c_void_p(self._ws_ptr), nbytes, m_max,
                                       _stream_ptr(stream), C.byref(ctx)), "ff_create_batch")
        else:
            _check(lib.ff_create_tiled(self._sys_array, self.n_sys, C.c_void_p(self._ws_ptr), nbytes, m_max,
                                       *tiling, _stream_ptr(stream), C.byref(ctx)),
                   "ff_create_tiled")
        self._ctx = ctx
        self.m_max = m_max
        cfg, ch, ch64 = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib.ff_get_tiling(self._ctx, C.byref(cfg), C.byref(ch), C.byref(ch64)), "ff_get_tiling")
        self.tiling = (cfg.value, ch.value, ch64.value)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            N.load().ff_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _coords(self, x) -> torch.Tensor:
        if not (isinstance(x, torch.Tensor) and x.dtype == torch.float64 and x.is_cuda and x.is_contiguous()
                and x.numel() == 3 * self.n):
            raise ValueError("coordinates must be a contiguous float64 CUDA tensor with 3*n_atoms elements")
        return x

    def energy_grad(self, x: torch.Tensor, precision: str | int = "fp64", want_grad: bool = True,
                    out_e: torch.Tensor | None = None, out_g: torch.Tensor | None = None, stream=None):
        """E and grad E at x (device tensor [n_atoms, 3], float64).  Asynchronous
        on the current stream; returns device tensors (out_e: n_sys float64
        entries, out_g: like x, if given)."""
        x = self._coords(x)
        prec = PRECISIONS.get(precision, precision)
        e = _out_tensor(out_e, self.n_sys, x, "out_e") if out_e is not None else \
            torch.empty(self.n_sys, dtype=torch.float64, device=x.device)
        g = None
        if want_grad:
            g = _out_tensor(out_g, x.numel(), x, "out_g") if out_g is not None else torch.empty_like(x)
        _check(N.load().ff_energy_grad(self._ctx, C.c_void_p(x.data_ptr()), C.c_void_p(e.data_ptr()),
                                       C.c_void_p(g.data_ptr()) if g is not None else None, int(prec),
                                       _stream_ptr(stream)), "ff_energy_grad")
        return e, g

    def minimize(self, x: torch.Tensor, method: str | int = "lbfgs", m: int = 10, tol: float = 1e-3,
                 max_iter: int = 2000, precision: str | int = "fp64", linesearch: int = FF_LS_DEFAULT,
                 ls_K: int = 2, h_init: float = 0.1, k_plus: float = 2.0, k_minus: float = 0.5,
                 eps_h: float = 1e-10, cg_restart: int = 0, cg_beta: str | int = "prp", ls_par_g0: bool = True,
                 fgm_restart: bool = False, hb_alpha: float = 0.0, hb_beta: float = 0.0, resume: bool = False,
                 certify: bool = True, stream=None) -> dict:
        """Minimize in place (x is overwritten with the result point(s)); blocks.
        Returns a result dict (a list of them for a batch)."""
        x = self._coords(x)
        p = N.FFMinParams()
        N.load().ff_default_params(C.byref(p))
        p.method = METHODS.get(method, method)
        p.m, p.tol, p.max_iter = m, tol, max_iter
        p.precision = PRECISIONS.get(precision, precision)
        p.linesearch, p.ls_K = linesearch, ls_K
        p.h_init, p.k_plus, p.k_minus, p.eps_h = h_init, k_plus, k_minus, eps_h
        p.cg_restart = cg_restart
        p.cg_beta = CG_BETAS.get(cg_beta, cg_beta)
        p.ls_par_g0 = 1 if ls_par_g0 else 0
        p.fgm_restart = 1 if fgm_restart else 0
        p.hb_alpha, p.hb_beta = hb_alpha, hb_beta
        p.flags = (FF_MIN_RESUME if resume else 0) | (0 if certify else FF_MIN_NO_CERTIFY)
        res = (N.FFMinResult * self.n_sys)()
        _check(N.load().ff_minimize(self._ctx, C.c_void_p(x.data_ptr()), C.byref(p), res,
                                    _stream_ptr(stream)), "ff_minimize")
        out = [dict(term=r.term, term_name=TERMS.get(r.term, str(r.term)), iters=r.iters, evals=r.evals,
                    evals_fp64=r.evals_fp64, energy=r.energy, grad_inf=r.grad_inf, grad_2=r.grad_2) for r in res]
        return out if self.is_batch else out[0]

    def energy_profile(self, x: torch.Tensor, t, precision: str | int = "fp64", stream=None) -> np.ndarray:
        """E(x + t u) along the unit antigradient u at x for every t:
        array [len(t)] (a batch: [len(t), n_sys])."""
        x = self._coords(x)
        tv = np.ascontiguousarray(np.asarray(t, dtype=np.float64).ravel())
        out = np.empty((len(tv), self.n_sys), dtype=np.float64)
        dp = C.POINTER(C.c_double)
        _check(N.load().ff_energy_profile(self._ctx, C.c_void_p(x.data_ptr()), tv.ctypes.data_as(dp), len(tv),
                                          out.ctypes.data_as(dp), int(PRECISIONS.get(precision, precision)),
                                          _stream_ptr(stream)), "ff_energy_profile")
        return out if self.is_batch else out[:, 0]

    def time_pair(self, x: torch.Tensor, precision: str | int = "fp32", reps: int = 20, stream=None) -> float:
        """Average duration (ms) of the pair kernel alone at x, HIP-event timed."""
        x = self._coords(x)
        ms = C.c_double()
        _check(N.load().ff_time_pair(self._ctx, C.c_void_p(x.data_ptr()), int(PRECISIONS.get(precision, precision)),
                                     reps, _stream_ptr(stream), C.byref(ms)), "ff_time_pair")
        return ms.value

    def trace(self, max_entries: int = 4096, stream=None) -> np.ndarray:
        """(E, h, evals) after each iteration of the last minimize call."""
        buf = np.zeros(3 * max_entries)
        n = N.load().ff_get_trace(self._ctx, buf.ctypes.data_as(C.POINTER(C.c_double)), max_entries,
                                  _stream_ptr(stream))
        if n < 0:
            raise FFError(n, "ff_get_trace")
        return buf[: 3 * n].reshape(n, 3)
