"""Python binding of the C ABI (argument marshalling only).

Every call forwards to libehelm.so; PyTorch only provides device memory
(complex128 / float64 CUDA tensors) and the current HIP stream.  Names
follow include/ehelm.h.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _native as N


class EhelmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ehelm status {status}: {msg}")
        self.status = status


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _check_dev(t: torch.Tensor, dtype, numel, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def default_abc_sides(dim: int) -> int:
    """All sides but the top (low side of the depth axis)."""
    return ((1 << (2 * dim)) - 1) & ~(1 << (2 * (dim - 1)))


class ElasticHelmholtz:
    """Context of the block-acoustic preconditioned elastic Helmholtz solver
    (eh_create ... eh_destroy)."""

    def __init__(self, n, h, vp, vs, rho, omega, *, levels=3, cycle="V",
                 nu=(1, 2), damping=(0.8, 0.8, 0.3), alpha=0.1,
                 mg_precision=32, restart=20, abc_width=20, abc_sides=None,
                 gamma0=0.01 * math.pi, intergrid="full", graphs=True, autotune=True, fused=True,
                 ap_variant="A_p", coarse_solver="auto", drop_converged=True,
                 stream=None):
        L = N.lib()
        self._lib = L
        self.dim = len(n)
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        opts = N.EhOpts()
        L.eh_default_opts(ctypes.byref(opts))
        opts.levels = int(levels)
        opts.cycle = {"V": 0, "W": 1}[cycle] if isinstance(cycle, str) else int(cycle)
        opts.nu_pre, opts.nu_post = int(nu[0]), int(nu[1])
        opts.n_damping = len(damping)
        for i, v in enumerate(damping):
            opts.damping[i] = float(v)
        opts.alpha = float(alpha)
        opts.mg_precision = int(mg_precision)
        opts.restart = int(restart)
        opts.abc_width = int(abc_width)
        opts.abc_sides = default_abc_sides(self.dim) if abc_sides is None else int(abc_sides)
        opts.gamma0 = float(gamma0)
        opts.intergrid = {"full": 0, "mixed": 1}[intergrid] if isinstance(intergrid, str) else int(intergrid)
        opts.graphs = 1 if graphs else 0
        opts.autotune = 1 if autotune else 0
        opts.fused = 1 if fused else 0
        opts.ap_variant = {"A_p": 0, "tilde": 1}[ap_variant] if isinstance(ap_variant, str) else int(ap_variant)
        opts.coarse_solver = ({"auto": 0, "dense": 1, "bt": 2}[coarse_solver] if isinstance(coarse_solver, str)
                              else int(coarse_solver))
        opts.drop_converged = 1 if drop_converged else 0
        self.opts = opts
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel()) for a in (vp, vs, rho)]
        ncell = int(np.prod(self.n))
        for a in arrs:
            if a.size != ncell:
                raise ValueError("medium arrays must have n[0]*...*n[d-1] entries")
        n64 = (ctypes.c_int64 * 3)(*(list(self.n) + [1] * (3 - self.dim)))
        h64 = (ctypes.c_double * 3)(*(list(self.h) + [1.0] * (3 - self.dim)))
        dp = ctypes.POINTER(ctypes.c_double)
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        ctx = ctypes.c_void_p()
        st = L.eh_create(ctypes.byref(ctx), self.dim, n64, h64,
                         arrs[0].ctypes.data_as(dp), arrs[1].ctypes.data_as(dp),
                         arrs[2].ctypes.data_as(dp), float(omega), ctypes.byref(opts),
                         ctypes.c_void_p(stream))
        if st != N.EH_OK:
            raise EhelmError(st, L.eh_last_error(None).decode())
        self._ctx = ctx
        self.omega = float(omega)
        self.ndof = int(L.eh_ndof(ctx))
        self.ncell = ncell
        sizes = []
        for k in range(self.dim):
            m = list(self.n)
            m[k] += 1
            sizes.append(int(np.prod(m)))
        sizes.append(ncell)
        self.field_sizes = sizes
        self.offsets = np.concatenate([[0], np.cumsum(sizes)])[:-1].tolist()

    # -- plumbing -------------------------------------------------------------
    def _check(self, st):
        if st not in (N.EH_OK, N.EH_NOT_CONVERGED):
            raise EhelmError(st, self._lib.eh_last_error(self._ctx).decode())
        return st

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.eh_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_stream(self, stream):
        self._check(self._lib.eh_set_stream(self._ctx, ctypes.c_void_p(stream)))

    # -- calls ------------------------------------------------------------------
    def _nrhs(self, t, per):
        if t.numel() % per:
            raise ValueError("buffer size is not a multiple of the vector length")
        return t.numel() // per

    def apply_operator(self, x, y=None):
        nrhs = self._nrhs(x, self.ndof)
        _check_dev(x, torch.complex128, nrhs * self.ndof, "x")
        y = torch.empty_like(x) if y is None else y
        _check_dev(y, torch.complex128, nrhs * self.ndof, "y")
        self._check(self._lib.eh_apply_operator(self._ctx, _ptr(x), _ptr(y), nrhs))
        return y

    def apply_preconditioner(self, r, z=None):
        nrhs = self._nrhs(r, self.ndof)
        _check_dev(r, torch.complex128, nrhs * self.ndof, "r")
        z = torch.empty_like(r) if z is None else z
        _check_dev(z, torch.complex128, nrhs * self.ndof, "z")
        self._check(self._lib.eh_apply_preconditioner(self._ctx, _ptr(r), _ptr(z), nrhs))
        return z

    def block_dims(self, block, level=0):
        out = (ctypes.c_int64 * 3)()
        self._check(self._lib.eh_block_dims(self._ctx, int(block), int(level), out))
        return tuple(int(v) for v in out)

    def block_cycle(self, block, f):
        np_ = int(np.prod(self.block_dims(block, 0)))
        nrhs = self._nrhs(f, np_)
        _check_dev(f, torch.complex128, nrhs * np_, "f")
        e = torch.empty_like(f)
        self._check(self._lib.eh_block_cycle(self._ctx, int(block), _ptr(f), _ptr(e), nrhs))
        return e

    def block_apply(self, block, level, x):
        np_ = int(np.prod(self.block_dims(block, level)))
        nrhs = self._nrhs(x, np_)
        _check_dev(x, torch.complex128, nrhs * np_, "x")
        y = torch.empty_like(x)
        self._check(self._lib.eh_block_apply(self._ctx, int(block), int(level), _ptr(x), _ptr(y), nrhs))
        return y

    def solve(self, b, tol=1e-6, maxit=1000, x=None):
        nrhs = self._nrhs(b, self.ndof)
        _check_dev(b, torch.complex128, nrhs * self.ndof, "b")
        x = torch.empty_like(b) if x is None else x
        _check_dev(x, torch.complex128, nrhs * self.ndof, "x")
        info = (N.EhInfo * nrhs)()
        self._check(self._lib.eh_solve(self._ctx, _ptr(b), _ptr(x), nrhs, float(tol), int(maxit), info))
        return x, [dict(iters=i.iters, converged=bool(i.converged), relres_true=i.relres_true,
                        relres_est=i.relres_est) for i in info]

    def block_solve(self, block, f, tol=1e-10, maxit=1000):
        """Solve one shifted acoustic block alone (eh_block_solve)."""
        np_ = int(np.prod(self.block_dims(block, 0)))
        nrhs = self._nrhs(f, np_)
        _check_dev(f, torch.complex128, nrhs * np_, "f")
        x = torch.empty_like(f)
        info = (N.EhInfo * nrhs)()
        self._check(self._lib.eh_block_solve(self._ctx, int(block), _ptr(f), _ptr(x), nrhs, float(tol),
                                             int(maxit), info))
        return x, [dict(iters=i.iters, converged=bool(i.converged), relres_true=i.relres_true) for i in info]

    def apply_Z(self, v, tol=1e-10, maxit=1000):
        """y = Z(alpha) v for one cell vector (eh_apply_Z)."""
        _check_dev(v, torch.complex128, self.ncell, "v")
        y = torch.empty_like(v)
        st = self._check(self._lib.eh_apply_Z(self._ctx, _ptr(v), _ptr(y), float(tol), int(maxit)))
        if st == N.EH_NOT_CONVERGED:
            raise EhelmError(st, self._lib.eh_last_error(self._ctx).decode())
        return y

    def power_Z(self, v0, iters, tol=1e-10, maxit=1000):
        """Power-method estimates ||Z v_k|| of rho(Z(alpha)) (eh_power_Z);
        v0 (one cell vector) is copied, not modified."""
        _check_dev(v0, torch.complex128, self.ncell, "v0")
        v = v0.clone()
        est = (ctypes.c_double * int(iters))()
        st = self._check(self._lib.eh_power_Z(self._ctx, _ptr(v), int(iters), float(tol), int(maxit), est))
        if st == N.EH_NOT_CONVERGED:
            raise EhelmError(st, self._lib.eh_last_error(self._ctx).decode())
        return np.array(est[:]), v

    def misfit(self, u, rec, d):
        nrhs = self._nrhs(u, self.ndof)
        _check_dev(u, torch.complex128, nrhs * self.ndof, "u")
        _check_dev(rec, torch.int64, rec.numel(), "rec")
        _check_dev(d, torch.complex128, nrhs * rec.numel(), "d")
        g = torch.empty_like(u)
        phi = ctypes.c_double()
        self._check(self._lib.eh_misfit(self._ctx, _ptr(u), _ptr(rec), rec.numel(), _ptr(d), nrhs,
                                        _ptr(g), ctypes.byref(phi)))
        return phi.value, g

    def misfit_noalloc(self, u, rec, d, g, phi):
        """eh_misfit_noalloc: writes g and phi (a one-element float64 CUDA
        tensor) on the context's stream without allocating or waiting."""
        nrhs = self._nrhs(u, self.ndof)
        _check_dev(u, torch.complex128, nrhs * self.ndof, "u")
        _check_dev(rec, torch.int64, rec.numel(), "rec")
        _check_dev(d, torch.complex128, nrhs * rec.numel(), "d")
        _check_dev(g, torch.complex128, nrhs * self.ndof, "g")
        _check_dev(phi, torch.float64, 1, "phi")
        self._check(self._lib.eh_misfit_noalloc(self._ctx, _ptr(u), _ptr(rec), rec.numel(), _ptr(d), nrhs,
                                                _ptr(g), _ptr(phi)))

    def timer_enable(self, classes):
        """Select kernel classes (names of _native.KERNEL_CLASSES) to time."""
        mask = 0
        for c in classes:
            mask |= 1 << N.KERNEL_CLASSES[c]
        self._check(self._lib.eh_timer_enable(self._ctx, mask))

    def timer_read(self, cls):
        """(launches, milliseconds, algorithmic bytes) since the last read."""
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.eh_timer_read(self._ctx, N.KERNEL_CLASSES[cls], ctypes.byref(n),
                                            ctypes.byref(ms), ctypes.byref(by)))
        return n.value, ms.value, by.value

    def gradient(self, u, w):
        nrhs = self._nrhs(u, self.ndof)
        _check_dev(u, torch.complex128, nrhs * self.ndof, "u")
        _check_dev(w, torch.complex128, nrhs * self.ndof, "w")
        out = [torch.empty(self.ncell, dtype=torch.float64, device=u.device) for _ in range(3)]
        self._check(self._lib.eh_gradient(self._ctx, _ptr(u), _ptr(w), nrhs, *(_ptr(t) for t in out)))
        return tuple(out)
