"""ctypes binding of the C-ABI in include/hz.h (argument marshalling only).

Every array argument is a torch CUDA tensor (complex128 / float64); the
binding passes its device pointer.  Nothing here computes: all steps run in
the HIP kernels of ``libhz.so``.  Loading fails loudly when the library has not
been built (run ``python -m paper_1510_01831_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhz.so")

HZ_OK, HZ_EINVAL, HZ_ENOMEM, HZ_ESTATE, HZ_ENOCONV, HZ_ESINGULAR, HZ_EDEVICE = 0, -1, -2, -3, -4, -5, -6
HZ_FP64, HZ_MIXED, HZ_MIXED_REFINE = 0, 1, 2
HZ_MODEL_VELOCITY, HZ_MODEL_SLOWNESS2 = 0, 1
HZ_PRECOND_GS, HZ_PRECOND_JACOBI = 0, 1
HZ_KRYLOV_GMRES, HZ_KRYLOV_BICGSTAB = 0, 1
HZ_INNER_LU, HZ_INNER_PT = 0, 1

EXPORTED = [
    "hz_setup", "hz_factor", "hz_solve", "hz_adjoint", "hz_solve_ext", "hz_adjoint_ext",
    "hz_misfit_gradient", "hz_misfit", "hz_misfit_noalloc", "hz_update_model", "hz_update_model_local",
    "hz_set_stream", "hz_get_info", "hz_get_timing",
    "hz_destroy", "hz_strerror", "hz_last_error", "hz_apply_layer", "hz_apply_sie",
    "hz_apply_precond", "hz_sie_rhs", "hz_cell_solve", "hz_cell_shape", "hz_residual",
    "hz_profile", "hz_profile_read",
]


class Params(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int), ("n_z", ctypes.c_int), ("h", ctypes.c_double),
                ("omega", ctypes.c_double), ("n_pml", ctypes.c_int),
                ("pml_beta", ctypes.c_double), ("layers", ctypes.c_int),
                ("cells", ctypes.c_int), ("precision", ctypes.c_int),
                ("model_kind", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("precond", ctypes.c_int), ("krylov", ctypes.c_int),
                ("inner", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("plr", ctypes.c_int), ("plr_eps", ctypes.c_double)]


class RhsStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_resid", ctypes.c_double),
                ("vol_resid", ctypes.c_double), ("refine_steps", ctypes.c_int),
                ("err_est", ctypes.c_double)]


class Timing(ctypes.Structure):
    _fields_ = [("t_setup", ctypes.c_double), ("t_factor", ctypes.c_double),
                ("t_rhs", ctypes.c_double), ("t_gmres", ctypes.c_double),
                ("t_recon", ctypes.c_double), ("t_solve", ctypes.c_double),
                ("gmres_iters", ctypes.c_int), ("inner_iters", ctypes.c_int)]


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("n_pml", ctypes.c_int), ("W", ctypes.c_int),
                ("layers", ctypes.c_int), ("cells", ctypes.c_int),
                ("trace_len", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("device_bytes", ctypes.c_longlong), ("plr_bytes", ctypes.c_longlong),
                ("plr_dense_bytes", ctypes.c_longlong), ("min_pivot_ratio", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libhz.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1510_01831_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.hz_setup.argtypes = [vp, ctypes.POINTER(Params), ctypes.POINTER(vp)]
        L.hz_factor.argtypes = [vp]
        for name in ("hz_solve", "hz_solve_ext"):
            getattr(L, name).argtypes = [vp, vp, i, vp, d, i, ctypes.POINTER(RhsStats),
                                         ctypes.POINTER(Timing)]
        for name in ("hz_adjoint", "hz_adjoint_ext"):
            getattr(L, name).argtypes = [vp, vp, i, vp, d, i, ctypes.POINTER(RhsStats)]
        L.hz_misfit_gradient.argtypes = [vp, vp, vp, i, vp]
        L.hz_misfit.argtypes = [vp, vp, vp, i, i, vp, ctypes.POINTER(d)]
        L.hz_misfit_noalloc.argtypes = [vp, vp, vp, i, i, vp, vp]
        L.hz_update_model.argtypes = [vp, vp]
        L.hz_update_model_local.argtypes = [vp, vp, ctypes.POINTER(i)]
        L.hz_set_stream.argtypes = [vp, vp]
        L.hz_get_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.hz_get_timing.argtypes = [vp, ctypes.POINTER(Timing)]
        L.hz_destroy.argtypes = [vp]
        L.hz_destroy.restype = None
        L.hz_strerror.argtypes = [i]
        L.hz_strerror.restype = ctypes.c_char_p
        L.hz_last_error.argtypes = []
        L.hz_last_error.restype = ctypes.c_char_p
        L.hz_apply_layer.argtypes = [vp, i, vp, vp, i, vp, i]
        L.hz_apply_sie.argtypes = [vp, vp, vp, i]
        L.hz_apply_precond.argtypes = [vp, vp, vp, i]
        L.hz_sie_rhs.argtypes = [vp, vp, vp, i]
        L.hz_cell_solve.argtypes = [vp, i, i, vp, vp, i]
        L.hz_cell_shape.argtypes = [vp, i, i, ctypes.POINTER(i), ctypes.POINTER(i)]
        L.hz_residual.argtypes = [vp, vp, vp, vp, i]
        L.hz_profile.argtypes = [vp, i]
        L.hz_profile_read.argtypes = [vp, ctypes.POINTER(KStat), i, ctypes.POINTER(i)]
        for name in EXPORTED:
            if name not in ("hz_destroy", "hz_strerror", "hz_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


class HzError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        super().__init__(f"{where}: {L.hz_strerror(status).decode()} "
                         f"({L.hz_last_error().decode()})")
        self.status = status


def _check(status: int, where: str, allow=()):
    if status != HZ_OK and status not in allow:
        raise HzError(status, where)
    return status


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One context of the C library: setup, factor, solve, adjoint."""

    def __init__(self, model, omega: float, n_pml: int, layers: int, cells: int,
                 precision: int = HZ_FP64, model_kind: int = HZ_MODEL_VELOCITY,
                 pml_beta: float = 2.0, max_batch: int = 1, factor: bool = True,
                 precond: int = HZ_PRECOND_GS, krylov: int = HZ_KRYLOV_GMRES,
                 inner: int = HZ_INNER_LU, inner_tol: float = 0.0, plr: int = 0,
                 plr_eps: float = 0.0):
        import torch

        self.torch = torch
        n = model.shape[-1]
        self.n = n
        self.model = model.to(device="cuda", dtype=torch.float64).contiguous()
        self.prm = Params(n, n, 1.0 / (n + 1), float(omega), int(n_pml), float(pml_beta),
                          int(layers), int(cells), int(precision), int(model_kind),
                          int(max_batch), int(precond), int(krylov), int(inner),
                          float(inner_tol), int(plr), float(plr_eps))
        self.ctx = ctypes.c_void_p()
        self._stats_raw = None
        self._stats_list = None
        L = lib()
        _check(L.hz_setup(_ptr(self.model), ctypes.byref(self.prm), ctypes.byref(self.ctx)),
               "hz_setup")
        info = Info()
        _check(L.hz_get_info(self.ctx, ctypes.byref(info)), "hz_get_info")
        self.info = info
        if factor:
            self.factor()

    # ------------------------------------------------------------------
    def factor(self):
        _check(lib().hz_factor(self.ctx), "hz_factor")
        info = Info()
        _check(lib().hz_get_info(self.ctx, ctypes.byref(info)), "hz_get_info")
        self.info = info

    def update_model(self, model):
        self.model = model.to(device="cuda", dtype=self.torch.float64).contiguous()
        _check(lib().hz_update_model(self.ctx, _ptr(self.model)), "hz_update_model")

    def update_model_local(self, model) -> int:
        """New model and re-factorisation of the cells it changes (the context
        must be factored); returns the number of cells redone."""
        self.model = model.to(device="cuda", dtype=self.torch.float64).contiguous()
        n = ctypes.c_int(0)
        _check(lib().hz_update_model_local(self.ctx, _ptr(self.model), ctypes.byref(n)),
               "hz_update_model_local")
        info = Info()
        _check(lib().hz_get_info(self.ctx, ctypes.byref(info)), "hz_get_info")
        self.info = info
        return int(n.value)

    def _solve(self, fn, f, tol, max_iter, ext, allow_noconv):
        torch = self.torch
        f = f.to(device="cuda", dtype=torch.complex128).contiguous()
        if f.dim() == 2:
            f = f.unsqueeze(0)
        B = f.shape[0]
        side = self.info.W if ext else self.n
        u = torch.empty((B, side, side), dtype=torch.complex128, device="cuda")
        stats = (RhsStats * B)()
        args = [self.ctx, _ptr(f), B, _ptr(u), float(tol), int(max_iter), stats]
        if fn in ("hz_solve", "hz_solve_ext"):
            timing = Timing()
            args.append(ctypes.byref(timing))
        st = getattr(lib(), fn)(*args)
        _check(st, fn, allow=(HZ_ENOCONV,) if allow_noconv else ())
        self.last_status = st
        self._stats_raw = stats            # converted on first access of last_stats
        self._stats_list = None
        return u

    @property
    def last_stats(self):
        """Per-RHS statistics of the last solve or adjoint (list of dicts)."""
        if self._stats_list is None and self._stats_raw is not None:
            self._stats_list = [dict(iters=s.iters, rel_resid=s.rel_resid, vol_resid=s.vol_resid,
                                     refine_steps=s.refine_steps, err_est=s.err_est)
                                for s in self._stats_raw]
        return self._stats_list

    def solve(self, f, tol=1e-10, max_iter=100, ext=False, allow_noconv=False):
        return self._solve("hz_solve_ext" if ext else "hz_solve", f, tol, max_iter, ext,
                           allow_noconv)

    def adjoint(self, f, tol=1e-10, max_iter=100, ext=False, allow_noconv=False):
        return self._solve("hz_adjoint_ext" if ext else "hz_adjoint", f, tol, max_iter, ext,
                           allow_noconv)

    def misfit_gradient(self, u_ext, lam_ext):
        torch = self.torch
        g = torch.empty((self.n, self.n), dtype=torch.float64, device="cuda")
        _check(lib().hz_misfit_gradient(self.ctx, _ptr(u_ext.contiguous()),
                                        _ptr(lam_ext.contiguous()), u_ext.shape[0], _ptr(g)),
               "hz_misfit_gradient")
        return g

    def misfit(self, u_ext, d_obs, rec_row):
        """(J, adjoint source P^T (P u - d)) for receivers on depth row rec_row."""
        torch = self.torch
        B = u_ext.shape[0]
        adj = torch.empty((B, self.n, self.n), dtype=torch.complex128, device="cuda")
        J = ctypes.c_double()
        _check(lib().hz_misfit(self.ctx, _ptr(u_ext.contiguous()),
                               _ptr(d_obs.to(device="cuda", dtype=torch.complex128).contiguous()),
                               int(rec_row), B, _ptr(adj), ctypes.byref(J)), "hz_misfit")
        return J.value, adj

    def misfit_noalloc(self, u_ext, d_obs, rec_row, adj_out, J_out):
        """hz_misfit_noalloc into caller-owned outputs (adj_out: B x n x n
        complex128, J_out: one float64 on the device); returns without
        waiting for the context's stream."""
        _check(lib().hz_misfit_noalloc(self.ctx, _ptr(u_ext), _ptr(d_obs), int(rec_row),
                                       u_ext.shape[0], _ptr(adj_out), _ptr(J_out)),
               "hz_misfit_noalloc")

    def profile(self, on: bool):
        _check(lib().hz_profile(self.ctx, int(bool(on))), "hz_profile")

    def profile_read(self) -> list:
        arr = (KStat * 256)()
        cnt = ctypes.c_int()
        _check(lib().hz_profile_read(self.ctx, arr, 256, ctypes.byref(cnt)), "hz_profile_read")
        return [dict(name=k.name.decode(), launches=k.launches, ms=k.ms, bytes=k.bytes,
                     flops=k.flops) for k in arr[:min(cnt.value, 256)]]

    def timing(self) -> dict:
        t = Timing()
        _check(lib().hz_get_timing(self.ctx, ctypes.byref(t)), "hz_get_timing")
        return {k: getattr(t, k) for k, _ in Timing._fields_}

    # ---------------------------------------------------------- blocks
    def apply_layer(self, layer, top, bot, side, B):
        torch = self.torch
        W = self.info.W
        out = torch.empty((2, W, B), dtype=torch.complex128, device="cuda")
        _check(lib().hz_apply_layer(self.ctx, layer, _ptr(top), _ptr(bot), side, _ptr(out), B),
               "hz_apply_layer")
        return out

    def apply_sie(self, x):
        y = self.torch.empty_like(x)
        _check(lib().hz_apply_sie(self.ctx, _ptr(x), _ptr(y), x.shape[-1]), "hz_apply_sie")
        return y

    def apply_precond(self, x):
        y = self.torch.empty_like(x)
        _check(lib().hz_apply_precond(self.ctx, _ptr(x), _ptr(y), x.shape[-1]),
               "hz_apply_precond")
        return y

    def sie_rhs(self, f):
        torch = self.torch
        f = f.to(device="cuda", dtype=torch.complex128).contiguous()
        B = f.shape[0]
        y = torch.empty((self.info.trace_len, B), dtype=torch.complex128, device="cuda")
        _check(lib().hz_sie_rhs(self.ctx, _ptr(f), _ptr(y), B), "hz_sie_rhs")
        return y

    def cell_shape(self, layer, cell):
        HL, Wc = ctypes.c_int(), ctypes.c_int()
        _check(lib().hz_cell_shape(self.ctx, layer, cell, ctypes.byref(HL), ctypes.byref(Wc)),
               "hz_cell_shape")
        return HL.value, Wc.value

    def cell_solve(self, layer, cell, g):
        x = self.torch.empty_like(g)
        _check(lib().hz_cell_solve(self.ctx, layer, cell, _ptr(g), _ptr(x), g.shape[-1]),
               "hz_cell_solve")
        return x

    def residual(self, u_ext, f_ext):
        r = self.torch.empty_like(u_ext)
        _check(lib().hz_residual(self.ctx, _ptr(u_ext), _ptr(f_ext), _ptr(r), u_ext.shape[0]),
               "hz_residual")
        return r

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().hz_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
