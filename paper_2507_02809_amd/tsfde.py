"""ctypes binding of libtsfde.so (include/tsfde.h).  Argument marshalling only: every step
of the solver runs in the library's HIP kernels.  Device arrays are torch tensors on a ROCm
device; host arrays are numpy arrays.  Raises RuntimeError when the library is missing."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_LIBPATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtsfde.so")
_lib = None

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ENONFINITE, ENOTIMPL = range(7)
FP64, MIXED, PREC_F32 = 0, 1, 2
BLOCK_CG, BLOCK_TAU, BLOCK_STRANG = 0, 1, 2
WARM_PREVIOUS, WARM_LINEAR, WARM_QUADRATIC, WARM_HALF = 0, 1, 2, 3
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOCONV", 5: "ENONFINITE", 6: "ENOTIMPL"}

EXPORTED = [
    "tsfde_default_opts", "tsfde_create_problem", "tsfde_create_problem_ex", "tsfde_set_mu", "tsfde_set_gamma2", "tsfde_set_alpha",
    "tsfde_destroy_problem", "tsfde_vector_length", "tsfde_device_bytes", "tsfde_problem_scalars", "tsfde_get_stencil",
    "tsfde_compute_stencil", "tsfde_apply_A", "tsfde_apply_A_f32", "tsfde_apply_P_inv",
    "tsfde_apply_P_inv_f32", "tsfde_apply_P_inv_noalloc", "tsfde_gmres_solve", "tsfde_recover_f", "tsfde_recover_f_batch",
    "tsfde_forward_solve", "tsfde_apply_AT", "tsfde_apply_PT_inv", "tsfde_adjoint_solve",
    "tsfde_recover_f_vjp", "tsfde_recover_f_vjp_batch", "tsfde_arnoldi", "tsfde_ritz_values",
    "tsfde_singular_value_estimates", "tsfde_discrepancy", "tsfde_gmres_solve_block", "tsfde_recover_f_block",
    "tsfde_autotune", "tsfde_recover_f_multi", "tsfde_last_error",
]


class Tuning(C.Structure):
    _fields_ = [("mv_variant", C.c_int), ("n_mv", C.c_int), ("mv_ids", C.c_int * 8), ("mv_ms", C.c_double * 8),
                ("pinv_blocks", C.c_int), ("n_pinv", C.c_int), ("pinv_cand", C.c_int * 8),
                ("pinv_ms", C.c_double * 8), ("restart", C.c_int), ("inner_tol", C.c_double),
                ("warm_start", C.c_int), ("solve_s", C.c_double), ("solves", C.c_int)]

    def as_dict(self) -> dict:
        return {"mv_variant": self.mv_variant,
                "mv_ms": {int(self.mv_ids[i]): float(self.mv_ms[i]) for i in range(self.n_mv)},
                "pinv_blocks": self.pinv_blocks,
                "pinv_ms": {int(self.pinv_cand[i]): float(self.pinv_ms[i]) for i in range(self.n_pinv)},
                "restart": self.restart, "inner_tol": self.inner_tol, "warm_start": self.warm_start,
                "solve_s": self.solve_s, "solves": self.solves}


class Opts(C.Structure):
    _fields_ = [("restart", C.c_int), ("maxit", C.c_int), ("tol", C.c_double), ("precision", C.c_int),
                ("use_precond", C.c_int), ("inner_tol", C.c_double), ("inner_maxit", C.c_int),
                ("refine_tol", C.c_double), ("max_refine", C.c_int), ("block_solver", C.c_int),
                ("warm_start", C.c_int), ("max_device_bytes", C.c_longlong), ("recompute_z", C.c_int),
                ("graph", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("refinements", C.c_int), ("converged", C.c_int),
                ("inner_iters", C.c_longlong), ("rel_res", C.c_double), ("t_total", C.c_double),
                ("t_precond", C.c_double), ("t_matvec", C.c_double), ("t_ortho", C.c_double),
                ("history_len", C.c_int), ("history_ptr", C.POINTER(C.c_double))]

    def history(self) -> list:
        """The solve's relative residual history (copied out of the problem's host buffer)."""
        return [self.history_ptr[i] for i in range(self.history_len)] if self.history_len > 0 else []

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "history_ptr"}
        d["history"] = self.history()
        return d


class TsfdeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """Load libtsfde.so (built in-tree by paper_2507_02809_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise RuntimeError(f"{_LIBPATH} is missing: build it with python -m paper_2507_02809_amd.build")
    L = C.CDLL(_LIBPATH)
    dp, fp, vp = C.POINTER(C.c_double), C.POINTER(C.c_float), C.c_void_p
    i, d = C.c_int, C.c_double
    pp = C.POINTER(C.c_void_p)
    L.tsfde_default_opts.argtypes = [C.POINTER(Opts)]
    L.tsfde_default_opts.restype = None
    L.tsfde_create_problem.argtypes = [i, i, i, d, d, d, d, dp, dp, dp, dp, dp, pp]
    L.tsfde_create_problem_ex.argtypes = [i, i, i, d, d, d, d, dp, dp, dp, dp, dp, d, dp, pp]
    L.tsfde_set_mu.argtypes = [vp, dp]
    L.tsfde_set_gamma2.argtypes = [vp, dp]
    L.tsfde_set_alpha.argtypes = [vp, d]
    L.tsfde_destroy_problem.argtypes = [vp]
    L.tsfde_destroy_problem.restype = None
    L.tsfde_vector_length.argtypes = [vp]
    L.tsfde_vector_length.restype = C.c_size_t
    L.tsfde_device_bytes.argtypes = [vp]
    L.tsfde_device_bytes.restype = C.c_size_t
    L.tsfde_problem_scalars.argtypes = [vp, dp]
    L.tsfde_get_stencil.argtypes = [vp, dp]
    L.tsfde_compute_stencil.argtypes = [i, i, d, dp]
    L.tsfde_apply_A.argtypes = [vp, vp, vp, vp]
    L.tsfde_apply_A_f32.argtypes = [vp, vp, vp, vp]
    L.tsfde_apply_P_inv.argtypes = [vp, vp, vp, C.POINTER(Opts), vp]
    L.tsfde_apply_P_inv_f32.argtypes = [vp, vp, vp, C.POINTER(Opts), vp]
    L.tsfde_apply_P_inv_noalloc.argtypes = [vp, vp, vp, C.POINTER(Opts), vp]
    L.tsfde_gmres_solve.argtypes = [vp, vp, vp, C.POINTER(Opts), C.POINTER(Stats), vp]
    L.tsfde_recover_f.argtypes = [vp, vp, vp, C.POINTER(Opts), C.POINTER(Stats), vp]
    L.tsfde_forward_solve.argtypes = [vp, vp, vp, C.POINTER(Opts), vp]
    L.tsfde_recover_f_batch.argtypes = [pp, i, pp, C.POINTER(Opts), C.POINTER(Stats), i, vp]
    L.tsfde_apply_AT.argtypes = [vp, vp, vp, vp]
    L.tsfde_arnoldi.argtypes = [vp, vp, i, dp, C.POINTER(C.c_int), C.POINTER(Opts), vp]
    L.tsfde_ritz_values.argtypes = [dp, i, i, dp, dp]
    L.tsfde_singular_value_estimates.argtypes = [vp, i, i, dp, dp, C.POINTER(C.c_int), C.POINTER(Opts), vp]
    L.tsfde_discrepancy.argtypes = [vp, vp, dp, C.POINTER(Opts), vp]
    L.tsfde_recover_f_vjp_batch.argtypes = [pp, i, pp, pp, pp, dp, pp, C.POINTER(Opts), C.POINTER(Stats), i, vp]
    L.tsfde_apply_PT_inv.argtypes = [vp, vp, vp, C.POINTER(Opts), vp]
    L.tsfde_adjoint_solve.argtypes = [vp, vp, vp, C.POINTER(Opts), C.POINTER(Stats), vp]
    L.tsfde_recover_f_vjp.argtypes = [vp, vp, vp, vp, dp, vp, C.POINTER(Opts), C.POINTER(Stats), vp]
    L.tsfde_gmres_solve_block.argtypes = [vp, i, vp, vp, dp, C.POINTER(Opts), C.POINTER(Stats), vp]
    L.tsfde_recover_f_block.argtypes = [vp, i, vp, vp, dp, C.POINTER(Opts), C.POINTER(Stats), vp]
    L.tsfde_autotune.argtypes = [vp, C.POINTER(Opts), i, C.POINTER(Tuning), vp]
    L.tsfde_recover_f_multi.argtypes = [pp, i, pp, C.POINTER(Opts), C.POINTER(Stats), vp]
    L.tsfde_last_error.argtypes = []
    L.tsfde_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("tsfde_default_opts", "tsfde_destroy_problem", "tsfde_vector_length", "tsfde_device_bytes",
                        "tsfde_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def last_error() -> str:
    return lib().tsfde_last_error().decode()


def _check(status: int, allow=()):
    if status != OK and status not in allow:
        raise TsfdeError(status, last_error())
    return status


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().tsfde_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _host(a, n: int, name: str):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if arr.size != n:
        raise ValueError(f"{name}: expected {n} values, got {arr.size}")
    return arr, arr.ctypes.data_as(C.POINTER(C.c_double))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(t, dtype, n: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a device tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor of {n} elements")
    return C.c_void_p(t.data_ptr())


def compute_stencil(d: int, N: int, omega: float) -> np.ndarray:
    """The library's stencil a_l, 0 <= l_i < N (host computation, no device needed)."""
    out = np.empty(N ** d)
    _check(lib().tsfde_compute_stencil(d, N, omega, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out.reshape((N,) * d)


class Problem:
    """A problem on the current ROCm device (tsfde_create_problem_ex)."""

    def __init__(self, d, N, M, T, beta, omega, alpha, gamma1, gamma2, q, rho=None, mu=None,
                 length: float = 1.0, stencil=None):
        L = lib()
        Nd = N ** d
        self.d, self.N, self.M = d, N, M
        self.Nd = Nd
        keep = []
        args = []
        for a, n, name in ((gamma1, M * Nd, "gamma1"), (gamma2, M * Nd, "gamma2"), (q, M, "q"),
                           (rho, Nd, "rho"), (mu, Nd, "mu")):
            arr, ptr = _host(a, n, name)
            keep.append(arr)
            args.append(ptr)
        st_arr, st_ptr = _host(stencil, Nd, "stencil")
        h = C.c_void_p()
        _check(L.tsfde_create_problem_ex(d, N, M, T, beta, omega, alpha, *args, length, st_ptr, C.byref(h)))
        self._h = h
        self.n_tot = int(L.tsfde_vector_length(h))
        self.mu_host = np.zeros(Nd) if mu is None else np.asarray(mu, dtype=np.float64).reshape(-1).copy()

    @classmethod
    def from_inputs(cls, inp, mu=None, stencil=None):
        return cls(inp.d, inp.N, inp.M, inp.T, inp.beta, inp.omega, inp.alpha, inp.gamma1, inp.gamma2,
                   inp.q, inp.rho, mu, inp.length, stencil)

    def close(self):
        if getattr(self, "_h", None):
            lib().tsfde_destroy_problem(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_mu(self, mu):
        arr, ptr = _host(mu, self.Nd, "mu")
        _check(lib().tsfde_set_mu(self._h, ptr))
        self.mu_host = arr

    def set_gamma2(self, gamma2):
        """Replace the gamma2 samples ([M, N^d] host values, > 0)."""
        arr, ptr = _host(gamma2, self.M * self.Nd, "gamma2")
        _check(lib().tsfde_set_gamma2(self._h, ptr))

    def set_alpha(self, alpha: float):
        _check(lib().tsfde_set_alpha(self._h, float(alpha)))

    def device_bytes(self) -> int:
        """Device bytes the problem holds (arrays, work buffers allocated so far, Krylov basis)."""
        return int(lib().tsfde_device_bytes(self._h))

    def scalars(self) -> dict:
        out = (C.c_double * 6)()
        _check(lib().tsfde_problem_scalars(self._h, out))
        return dict(zip(["h", "dt", "eta", "c_t", "c_f", "L"], list(out)))

    def stencil(self) -> np.ndarray:
        out = np.empty(self.Nd)
        _check(lib().tsfde_get_stencil(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape((self.N,) * self.d)

    def apply_A(self, y, z=None, stream=None):
        import torch
        f32 = y.dtype == torch.float32
        if z is None:
            z = torch.empty_like(y)
        fn = lib().tsfde_apply_A_f32 if f32 else lib().tsfde_apply_A
        _check(fn(self._h, _dptr(y, y.dtype, self.n_tot, "y"), _dptr(z, y.dtype, self.n_tot, "z"), _stream(stream)))
        return z

    def apply_P_inv(self, z, y=None, opts: Optional[Opts] = None, stream=None):
        import torch
        f32 = z.dtype == torch.float32
        if y is None:
            y = torch.empty_like(z)
        fn = lib().tsfde_apply_P_inv_f32 if f32 else lib().tsfde_apply_P_inv
        _check(fn(self._h, _dptr(z, z.dtype, self.n_tot, "z"), _dptr(y, z.dtype, self.n_tot, "y"),
                  C.byref(opts) if opts is not None else None, _stream(stream)))
        return y

    def apply_P_inv_noalloc(self, z, y, opts: Optional[Opts] = None, stream=None):
        """y = P^{-1} z (FP64) with the library's static device scratch: no device allocation, y given."""
        import torch
        _check(lib().tsfde_apply_P_inv_noalloc(self._h, _dptr(z, torch.float64, self.n_tot, "z"),
                                               _dptr(y, torch.float64, self.n_tot, "y"),
                                               C.byref(opts) if opts is not None else None, _stream(stream)))
        return y

    def gmres_solve(self, b=None, x=None, opts: Optional[Opts] = None, stream=None, raise_noconv=False):
        import torch
        if x is None:
            x = torch.zeros(self.n_tot, dtype=torch.float64, device="cuda")
        bp = _dptr(b, torch.float64, self.n_tot, "b") if b is not None else None
        st = Stats()
        rc = lib().tsfde_gmres_solve(self._h, bp, _dptr(x, torch.float64, self.n_tot, "x"),
                                     C.byref(opts) if opts is not None else None, C.byref(st), _stream(stream))
        _check(rc, allow=() if raise_noconv else (ENOCONV,))
        return x, st

    def recover_f(self, opts: Optional[Opts] = None, work=None, stream=None, raise_noconv=False):
        import torch
        f = torch.empty(self.Nd, dtype=torch.float64, device="cuda")
        wp = _dptr(work, torch.float64, self.n_tot, "work") if work is not None else None
        st = Stats()
        rc = lib().tsfde_recover_f(self._h, _dptr(f, torch.float64, self.Nd, "f"), wp,
                                   C.byref(opts) if opts is not None else None, C.byref(st), _stream(stream))
        _check(rc, allow=() if raise_noconv else (ENOCONV,))
        return f, st

    def autotune(self, opts: Optional[Opts] = None, what: int = 3, stream=None):
        """tsfde_autotune: returns (tuned opts, Tuning); the kernel choices stay with the problem."""
        o = opts if opts is not None else default_opts()
        o = Opts.from_buffer_copy(o)
        t = Tuning()
        _check(lib().tsfde_autotune(self._h, C.byref(o), what, C.byref(t), _stream(stream)))
        return o, t

    def gmres_solve_block(self, B, X=None, opts: Optional[Opts] = None, stream=None, raise_noconv=False):
        """Block FGMRES on the columns of B (nrhs x n_tot device tensor); returns (X, stats, rel_res)."""
        import torch
        k = B.shape[0] if B.dim() == 2 else 1
        if X is None:
            X = torch.zeros(k, self.n_tot, dtype=torch.float64, device="cuda")
        rel = np.zeros(k)
        st = Stats()
        rc = lib().tsfde_gmres_solve_block(self._h, k, _dptr(B, torch.float64, k * self.n_tot, "B"),
                                           _dptr(X, torch.float64, k * self.n_tot, "X"),
                                           rel.ctypes.data_as(C.POINTER(C.c_double)),
                                           C.byref(opts) if opts is not None else None, C.byref(st), _stream(stream))
        _check(rc, allow=() if raise_noconv else (ENOCONV,))
        return X, st, rel

    def recover_f_block(self, mus, opts: Optional[Opts] = None, stream=None, raise_noconv=False):
        """f~ for each data set mu_c (rows of mus, nrhs x N^d device tensor) in one block solve;
        returns (F (nrhs x N^d), stats, rel_res)."""
        import torch
        k = mus.shape[0]
        F = torch.empty(k, self.Nd, dtype=torch.float64, device="cuda")
        rel = np.zeros(k)
        st = Stats()
        rc = lib().tsfde_recover_f_block(self._h, k, _dptr(mus, torch.float64, k * self.Nd, "mus"),
                                         _dptr(F, torch.float64, k * self.Nd, "F"),
                                         rel.ctypes.data_as(C.POINTER(C.c_double)),
                                         C.byref(opts) if opts is not None else None, C.byref(st), _stream(stream))
        _check(rc, allow=() if raise_noconv else (ENOCONV,))
        return F, st, rel

    def apply_AT(self, lam, z=None, stream=None):
        import torch
        if z is None:
            z = torch.empty_like(lam)
        _check(lib().tsfde_apply_AT(self._h, _dptr(lam, torch.float64, self.n_tot, "lam"),
                                    _dptr(z, torch.float64, self.n_tot, "z"), _stream(stream)))
        return z

    def apply_PT_inv(self, g, lam=None, opts: Optional[Opts] = None, stream=None):
        import torch
        if lam is None:
            lam = torch.empty_like(g)
        _check(lib().tsfde_apply_PT_inv(self._h, _dptr(g, torch.float64, self.n_tot, "g"),
                                        _dptr(lam, torch.float64, self.n_tot, "lam"),
                                        C.byref(opts) if opts is not None else None, _stream(stream)))
        return lam

    def adjoint_solve(self, g, lam=None, opts: Optional[Opts] = None, stream=None, raise_noconv=False):
        import torch
        if lam is None:
            lam = torch.zeros_like(g)
        st = Stats()
        rc = lib().tsfde_adjoint_solve(self._h, _dptr(g, torch.float64, self.n_tot, "g"),
                                       _dptr(lam, torch.float64, self.n_tot, "lam"),
                                       C.byref(opts) if opts is not None else None, C.byref(st), _stream(stream))
        _check(rc, allow=() if raise_noconv else (ENOCONV,))
        return lam, st

    def recover_f_vjp(self, y, gf, opts: Optional[Opts] = None, stream=None, raise_noconv=False,
                      gamma2=False):
        """(grad_mu, grad_alpha, stats) of L(f~) with dL/df~ = gf, given the solution y of A y = z;
        with gamma2=True, (grad_mu, grad_alpha, grad_gamma2 [M, N^d], stats)."""
        import torch
        gmu = torch.empty(self.Nd, dtype=torch.float64, device="cuda")
        gg2 = torch.empty(self.M * self.Nd, dtype=torch.float64, device="cuda") if gamma2 else None
        ga = C.c_double(0.0)
        st = Stats()
        rc = lib().tsfde_recover_f_vjp(self._h, _dptr(y, torch.float64, self.n_tot, "y"),
                                       _dptr(gf, torch.float64, self.Nd, "gf"), _dptr(gmu, torch.float64, self.Nd, "gmu"),
                                       C.byref(ga), _dptr(gg2, torch.float64, self.M * self.Nd, "gg2") if gamma2 else None,
                                       C.byref(opts) if opts is not None else None, C.byref(st), _stream(stream))
        _check(rc, allow=() if raise_noconv else (ENOCONV,))
        if gamma2:
            return gmu, ga.value, gg2.view(self.M, self.Nd), st
        return gmu, ga.value, st

    def arnoldi(self, k: int, b=None, opts: Optional[Opts] = None, stream=None):
        """(H, steps): the (steps+1) x steps Hessenberg matrix of Arnoldi on A P^{-1} from b (default z)."""
        import torch
        H = np.zeros((k + 1) * k)
        steps = C.c_int(0)
        bp = _dptr(b, torch.float64, self.n_tot, "b") if b is not None else None
        _check(lib().tsfde_arnoldi(self._h, bp, int(k), H.ctypes.data_as(C.POINTER(C.c_double)), C.byref(steps),
                                   C.byref(opts) if opts is not None else None, _stream(stream)))
        m = steps.value
        return H.reshape(k + 1, k)[:m + 1, :m], m

    def singular_value_estimates(self, precond: bool, iters: int = 200, opts: Optional[Opts] = None, stream=None):
        """(sigma_max, sigma_min, (power steps, inverse steps)) of A or P^{-1} A (tsfde_singular_value_estimates);
        sigma_max / sigma_min estimates the 2-norm condition number."""
        smax, smin = C.c_double(0.0), C.c_double(0.0)
        used = (C.c_int * 2)()
        _check(lib().tsfde_singular_value_estimates(self._h, 1 if precond else 0, int(iters), C.byref(smax),
                                                    C.byref(smin), used, C.byref(opts) if opts is not None else None,
                                                    _stream(stream)))
        return smax.value, smin.value, (used[0], used[1])

    def discrepancy(self, f, opts: Optional[Opts] = None, stream=None) -> float:
        """||v^(M)(f) - mu_eps||_2 for the direct problem solved with source f (tsfde_discrepancy)."""
        import torch
        r = C.c_double(0.0)
        _check(lib().tsfde_discrepancy(self._h, _dptr(f, torch.float64, self.Nd, "f"), C.byref(r),
                                       C.byref(opts) if opts is not None else None, _stream(stream)))
        return r.value

    def forward_solve(self, f, opts: Optional[Opts] = None, stream=None):
        import torch
        v = torch.empty(self.M * self.Nd, dtype=torch.float64, device="cuda")
        _check(lib().tsfde_forward_solve(self._h, _dptr(f, torch.float64, self.Nd, "f"),
                                         _dptr(v, torch.float64, self.M * self.Nd, "v"),
                                         C.byref(opts) if opts is not None else None, _stream(stream)))
        return v


def recover_f_batch(problems, opts: Optional[Opts] = None, max_inflight: int = 2, stream=None,
                    raise_noconv=False):
    """tsfde_recover_f_batch: f~ of every problem, up to max_inflight solved side by side.
    Returns a list of (f, stats)."""
    import torch
    n = len(problems)
    fs = [torch.empty(p.Nd, dtype=torch.float64, device="cuda") for p in problems]
    hs = (C.c_void_p * max(n, 1))(*[p._h.value for p in problems])
    fp = (C.c_void_p * max(n, 1))(*[f.data_ptr() for f in fs])
    st = (Stats * max(n, 1))()
    rc = lib().tsfde_recover_f_batch(hs, n, fp, C.byref(opts) if opts is not None else None, st, max_inflight,
                                     _stream(stream))
    _check(rc, allow=() if raise_noconv else (ENOCONV,))
    return [(fs[i], st[i]) for i in range(n)]


def recover_f_multi(problems, opts: Optional[Opts] = None, stream=None, raise_noconv=False):
    """tsfde_recover_f_multi: f~ of every problem, solved in lockstep with shared P^{-1} launches.
    Returns a list of (f, stats)."""
    import torch
    n = len(problems)
    fs = [torch.empty(p.Nd, dtype=torch.float64, device="cuda") for p in problems]
    hs = (C.c_void_p * max(n, 1))(*[p._h.value for p in problems])
    fp = (C.c_void_p * max(n, 1))(*[f.data_ptr() for f in fs])
    st = (Stats * max(n, 1))()
    rc = lib().tsfde_recover_f_multi(hs, n, fp, C.byref(opts) if opts is not None else None, st, _stream(stream))
    _check(rc, allow=() if raise_noconv else (ENOCONV,))
    return [(fs[i], st[i]) for i in range(n)]


def recover_f_autograd(problem: "Problem", mu, opts: Optional[Opts] = None, adjoint_opts: Optional[Opts] = None,
                       log_alpha=None, gamma2=None):
    """f~ as a differentiable function of the final-time data mu_eps (a device FP64 tensor of N^d
    values) and, optionally, of log alpha (a 0-d FP64 tensor) and the gamma2 samples (a device FP64
    tensor [M, N^d]; any differentiable parameterisation, e.g. an interpolated coarse field, can
    produce them).  The forward pass sets the inputs and runs tsfde_recover_f; the backward pass runs
    tsfde_recover_f_vjp (one adjoint solve) and returns dL/dmu, dL/dlog alpha = alpha dL/dalpha and
    dL/dgamma2.  The alpha gradient of the last backward pass is also left in problem.last_grad_alpha."""
    import math

    import torch

    class _RecoverF(torch.autograd.Function):
        @staticmethod
        def forward(ctx, m, la, g2):
            problem.set_mu(m.detach().cpu().numpy())
            if la is not None:
                problem.set_alpha(math.exp(float(la)))
            if g2 is not None:
                problem.set_gamma2(g2.detach().cpu().numpy())
            y = torch.empty(problem.n_tot, dtype=torch.float64, device="cuda")
            f, _ = problem.recover_f(opts, work=y, raise_noconv=True)
            ctx.save_for_backward(y)
            ctx.alpha = math.exp(float(la)) if la is not None else None
            ctx.has = (la is not None, g2 is not None)
            ctx.g2shape = g2.shape if g2 is not None else None
            return f

        @staticmethod
        def backward(ctx, gf):
            (y,) = ctx.saved_tensors
            want_g2 = ctx.has[1] and ctx.needs_input_grad[2]
            out = problem.recover_f_vjp(y, gf.contiguous().to(torch.float64), adjoint_opts, raise_noconv=True,
                                        gamma2=want_g2)
            gmu, ga = out[0], out[1]
            problem.last_grad_alpha = ga
            gla = torch.tensor(ga * ctx.alpha, dtype=torch.float64, device=gmu.device) if ctx.has[0] else None
            gg2 = out[2].reshape(ctx.g2shape) if want_g2 else None
            return gmu, gla, gg2

    return _RecoverF.apply(mu, log_alpha, gamma2)


def discrepancy_curve(problem: "Problem", alphas, opts: Optional[Opts] = None, fwd_opts: Optional[Opts] = None):
    """Morozov's discrepancy of the quasi-boundary-value reconstruction for each alpha: f_alpha
    recovered from the problem's data mu_eps (tsfde_recover_f after tsfde_set_alpha), then
    tsfde_discrepancy (the direct problem solved for f_alpha, ||v^(M)(f_alpha) - mu_eps||_2).
    The problem keeps the last alpha of the sweep.  Returns (residuals, list of f_alpha)."""
    res, fs = [], []
    for a in alphas:
        problem.set_alpha(a)
        f, _ = problem.recover_f(opts, raise_noconv=True)
        res.append(problem.discrepancy(f, opts=fwd_opts))
        fs.append(f)
    return res, fs


def select_alpha(alphas, residuals, delta: float, tau: float = 1.1):
    """The discrepancy principle: the largest alpha whose residual is at most tau * delta (delta the
    noise norm ||mu_eps - mu||); None if no alpha of the grid qualifies."""
    ok = [a for a, r in zip(alphas, residuals) if r <= tau * delta]
    return max(ok) if ok else None


def recover_f_vjp_batch(problems, gfs, ys=None, opts: Optional[Opts] = None, max_inflight: int = 2,
                        gamma2=False, stream=None, raise_noconv=False):
    """tsfde_recover_f_vjp_batch: per problem (grad_mu, grad_alpha[, grad_gamma2], stats); ys None uses
    each problem's solution from its last recover_f without a work buffer."""
    import torch
    n = len(problems)
    gmu = [torch.empty(p.Nd, dtype=torch.float64, device="cuda") for p in problems]
    gg2 = [torch.empty(p.M * p.Nd, dtype=torch.float64, device="cuda") for p in problems] if gamma2 else None
    ga = np.zeros(max(n, 1))
    arr = lambda ptrs: (C.c_void_p * max(n, 1))(*ptrs)
    hs = arr([p._h.value for p in problems])
    yp = arr([_dptr(y, torch.float64, p.n_tot, "y").value for y, p in zip(ys, problems)]) if ys is not None else None
    gp = arr([_dptr(g, torch.float64, p.Nd, "gf").value for g, p in zip(gfs, problems)])
    mp = arr([t.data_ptr() for t in gmu])
    g2p = arr([t.data_ptr() for t in gg2]) if gamma2 else None
    st = (Stats * max(n, 1))()
    rc = lib().tsfde_recover_f_vjp_batch(hs, n, yp, gp, mp, ga.ctypes.data_as(C.POINTER(C.c_double)), g2p,
                                         C.byref(opts) if opts is not None else None, st, max_inflight,
                                         _stream(stream))
    _check(rc, allow=() if raise_noconv else (ENOCONV,))
    if gamma2:
        return [(gmu[i], float(ga[i]), gg2[i].view(problems[i].M, problems[i].Nd), st[i]) for i in range(n)]
    return [(gmu[i], float(ga[i]), st[i]) for i in range(n)]


def ritz_values(H):
    """Eigenvalues of the leading square block of an Arnoldi Hessenberg matrix (tsfde_ritz_values)."""
    m = H.shape[1]
    A = np.ascontiguousarray(np.asarray(H, dtype=np.float64)[:m, :m])
    re, im = np.empty(m), np.empty(m)
    _check(lib().tsfde_ritz_values(A.ctypes.data_as(C.POINTER(C.c_double)), m, m,
                                   re.ctypes.data_as(C.POINTER(C.c_double)), im.ctypes.data_as(C.POINTER(C.c_double))))
    return re + 1j * im
