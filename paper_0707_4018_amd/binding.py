"""ctypes binding of include/amg.h (argument marshalling only).

Device tensors are torch tensors on the current HIP device; calls are
enqueued on torch's current stream.  Field layouts are the canonical ones of
the C ABI: complex psi[rhs][site][spin][colour] (x_1 fastest), links
U[mu][site][a][b], coarse fields psi[rhs][site][t].
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch

F64 = 0
F32 = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib_path() -> str:
    return os.path.join(_HERE, "libamg.so")


class AMGError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class _Lattice(C.Structure):
    _fields_ = [("nd", C.c_int), ("dims", C.c_int * 4)]


class _Params(C.Structure):
    _fields_ = [
        ("nlevels", C.c_int), ("block", (C.c_int * 4) * 3), ("nvec", C.c_int * 3),
        ("nu_pre", C.c_int), ("nu_post", C.c_int), ("omega", C.c_double),
        ("coarse_tol", C.c_double), ("coarse_maxiter", C.c_int), ("coarse_restart", C.c_int),
        ("outer_restart", C.c_int), ("inner_prec", C.c_int), ("p_bf16", C.c_int),
        ("kcycle_tol", C.c_double), ("kcycle_maxiter", C.c_int), ("coarse_dense_max", C.c_int),
        ("coarse_jacobi", C.c_int), ("coarse_eo", C.c_int),
    ]


class _Info(C.Structure):
    _fields_ = [
        ("iters", C.c_int), ("converged", C.c_int), ("true_rel_res", C.c_double),
        ("n_fine_D", C.c_longlong), ("n_fine_Ddag", C.c_longlong), ("n_coarse", C.c_longlong),
        ("t_ms", C.c_double),
    ]


class _NParams(C.Structure):
    _fields_ = [
        ("nlevels", C.c_int), ("block", (C.c_int * 2) * 3), ("nvec", C.c_int * 3), ("omega", C.c_double),
        ("sa_factor", C.c_double), ("power_steps", C.c_int), ("coarse_dense_max", C.c_int),
        ("fine_box", C.c_int), ("setup_dense_max", C.c_int), ("setup_coarse_tol", C.c_double),
        ("setup_coarse_maxiter", C.c_int),
    ]


class _NInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int), ("converged", C.c_int), ("restarts", C.c_int), ("rel_res_normal", C.c_double),
        ("rel_res_D", C.c_double), ("n_fine_D", C.c_longlong), ("n_fine_Ddag", C.c_longlong), ("t_ms", C.c_double),
    ]


_P = C.c_void_p
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
_SIGS = {
    "amg_set_allocator": (C.c_int, [_ALLOC_FN, _RELEASE_FN, _P]),
    "amg_status_str": (C.c_char_p, [C.c_int]),
    "amg_last_error": (C.c_char_p, []),
    "amg_default_params": (None, [C.POINTER(_Params)]),
    "amg_gauge_create": (C.c_int, [C.POINTER(_Lattice), _P, C.c_double, _P, C.POINTER(_P)]),
    "amg_gauge_set_mass": (C.c_int, [_P, C.c_double]),
    "amg_gauge_info": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "amg_gauge_destroy": (C.c_int, [_P]),
    "amg_apply": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, C.c_int, _P]),
    "amg_apply_internal": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, _P]),
    "amg_apply_noalloc": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, C.c_int, _P]),
    "amg_cgnr_solve": (C.c_int, [_P, _P, _P, C.c_double, C.c_int, C.POINTER(_Info), _P]),
    "amg_setup": (C.c_int, [_P, C.POINTER(_Params), C.POINTER(_P), _P, C.POINTER(_P)]),
    "amg_setup_adaptive": (C.c_int, [_P, C.POINTER(_Params), C.POINTER(_P), C.c_int, C.c_int, _P,
                                     C.POINTER(_P)]),
    "amg_solver_set_mass": (C.c_int, [_P, C.c_double]),
    "amg_solver_destroy": (C.c_int, [_P]),
    "amg_solve": (C.c_int, [_P, _P, _P, C.c_int, C.c_double, C.c_int, C.POINTER(_Info), _P]),
    "amg_get_nullvecs": (C.c_int, [_P, C.c_int, _P, _P]),
    "amg_get_coarse_op": (C.c_int, [_P, C.c_int, _P, _P]),
    "amg_level_apply": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P, C.c_int, _P]),
    "amg_transfer": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P, C.c_int, _P]),
    "amg_get_prolongator": (C.c_int, [_P, C.c_int, C.c_int, _P, _P]),
    "amg_vcycle": (C.c_int, [_P, _P, _P, C.c_int, _P]),
    "amg_mr": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P, C.c_int, _P]),
    "amg_level_info": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(C.c_longlong)]),
    "amg_profile_enable": (C.c_int, [_P, C.c_int, C.c_int, C.c_int]),
    "amg_batch_create": (C.c_int, [C.POINTER(_P), C.POINTER(C.c_int), C.c_int, C.c_int, _P, C.POINTER(_P)]),
    "amg_batch_solve": (C.c_int, [_P, C.POINTER(_P), C.POINTER(_P), C.c_double, C.c_int, C.POINTER(_Info), _P]),
    "amg_batch_info": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "amg_batch_destroy": (C.c_int, [_P]),
    "amg_batch_info2": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "amg_batch_tuning": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_float)]),
    "amg_profile_read": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    "amg_profile_read_kind": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]),
    "amg_setup_adaptive_levels": (C.c_int, [_P, C.POINTER(_Params), C.POINTER(_P), C.POINTER(C.c_int),
                                            C.POINTER(C.c_int), _P, C.POINTER(_P)]),
    "amg_setup_refined": (C.c_int, [_P, C.POINTER(_Params), _P, C.c_int, C.c_int, C.c_int, C.POINTER(_P), C.c_int,
                                    C.c_int, _P, C.POINTER(_P)]),
    "amg_mg_convergence": (C.c_int, [_P, _P, C.c_int, C.POINTER(C.c_double), _P]),
    "amg_cnn_num_params": (C.c_longlong, []),
    "amg_cnn_create": (C.c_int, [C.POINTER(C.c_float), C.c_int, C.POINTER(_P)]),
    "amg_cnn_destroy": (C.c_int, [_P]),
    "amg_cnn_get_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "amg_cnn_set_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "amg_cnn_forward": (C.c_int, [_P, _P, C.c_int, C.c_int, C.c_int, _P, _P]),
    "amg_cnn_loss_grad": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                    C.POINTER(C.c_float), _P]),
    "amg_cnn_train_step": (C.c_int, [_P, _P, _P, C.c_int, C.c_int, C.c_int, C.c_float, C.POINTER(C.c_double), _P]),
    "amg_cnn_propose": (C.c_int, [_P, _P, C.c_int, C.c_int, _P, _P]),
    "amg_normal_default_params": (None, [C.POINTER(_NParams)]),
    "amg_normal_setup": (C.c_int, [_P, C.POINTER(_NParams), C.POINTER(_P), C.POINTER(_P), _P, C.POINTER(_P)]),
    "amg_normal_setup_adaptive": (C.c_int, [_P, C.POINTER(_NParams), C.POINTER(_P), C.POINTER(_P),
                                            C.POINTER(C.c_int), C.POINTER(C.c_int), _P, C.POINTER(_P)]),
    "amg_normal_set_mass": (C.c_int, [_P, C.c_double, _P]),
    "amg_normal_solve": (C.c_int, [_P, _P, _P, C.c_double, C.c_int, C.c_int, C.POINTER(_NInfo), _P]),
    "amg_normal_vcycle": (C.c_int, [_P, _P, _P, _P]),
    "amg_normal_level_apply": (C.c_int, [_P, C.c_int, _P, _P, _P]),
    "amg_normal_export": (C.c_int, [_P, C.c_int, C.c_int, _P, _P]),
    "amg_normal_level_info": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "amg_normal_destroy": (C.c_int, [_P]),
    "amg_setup_learned": (C.c_int, [_P, C.POINTER(_Params), _P, C.POINTER(_P), C.c_int, C.c_int, C.c_int,
                                    C.c_double, C.c_int, C.c_int, C.c_int, _P, C.POINTER(_P), C.POINTER(C.c_int),
                                    C.POINTER(C.c_double)]),
}


def load_library(path: str | None = None):
    """Load libamg.so (built in-tree by paper_0707_4018_amd.build); raise if absent."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or lib_path()
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} is missing: build it with python -m paper_0707_4018_amd.build")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _LIB = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        lib = load_library()
        raise AMGError(status, where, f"{lib.amg_status_str(status).decode()}: {lib.amg_last_error().decode()}")


def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes))
    except Exception:  # out of memory: the library reports AMG_ERR_NOMEM
        return None


def _torch_release(ptr, stream, ctx):
    torch.cuda.caching_allocator_delete(ptr)


# kept for the life of the process: buffers taken from torch are released
# through these even after the default allocator is restored
_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_RELEASE = _RELEASE_FN(_torch_release)


def use_torch_allocator(enable: bool = True) -> None:
    """amg_set_allocator: take the handles' internal device buffers from torch's
    caching allocator (enable) or from hipMalloc again (disable).  Handles
    created while enabled should be destroyed before the interpreter exits."""
    lib = load_library()
    if enable:
        _check(lib.amg_set_allocator(_TORCH_ALLOC, _TORCH_RELEASE, None), "amg_set_allocator")
    else:
        _check(lib.amg_set_allocator(_ALLOC_FN(), _RELEASE_FN(), None), "amg_set_allocator")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor, dtype=torch.complex128) -> C.c_void_p:
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


@dataclass
class MGParams:
    """Multigrid parameters; defaults are the paper's where it gives one."""
    blocks: list = field(default_factory=lambda: [(4, 4)])
    nvec: list = field(default_factory=lambda: [8])
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.8
    coarse_tol: float = 0.1
    coarse_maxiter: int = 64
    coarse_restart: int = 16
    outer_restart: int = 16
    inner_prec: int = F64
    p_bf16: bool = False
    kcycle_tol: float = 0.1
    kcycle_maxiter: int = 0
    coarse_dense_max: int = 4096
    coarse_jacobi: bool = False
    coarse_eo: bool = False

    def to_c(self) -> _Params:
        p = _Params()
        load_library().amg_default_params(C.byref(p))
        p.nlevels = len(self.blocks) + 1
        for l, b in enumerate(self.blocks):
            for mu in range(4):
                p.block[l][mu] = int(b[mu]) if mu < len(b) else 1
            p.nvec[l] = int(self.nvec[l])
        p.nu_pre, p.nu_post, p.omega = self.nu_pre, self.nu_post, self.omega
        p.coarse_tol, p.coarse_maxiter, p.coarse_restart = self.coarse_tol, self.coarse_maxiter, self.coarse_restart
        p.outer_restart, p.inner_prec, p.p_bf16 = self.outer_restart, self.inner_prec, int(self.p_bf16)
        p.kcycle_tol, p.kcycle_maxiter = self.kcycle_tol, self.kcycle_maxiter
        p.coarse_dense_max = self.coarse_dense_max
        p.coarse_jacobi = int(self.coarse_jacobi)
        p.coarse_eo = int(self.coarse_eo)
        return p


@dataclass
class SolveInfo:
    iters: int
    converged: bool
    true_rel_res: float
    n_fine_D: int
    n_fine_Ddag: int
    n_coarse: int
    t_ms: float

    @staticmethod
    def from_c(i: _Info) -> "SolveInfo":
        return SolveInfo(i.iters, bool(i.converged), i.true_rel_res, i.n_fine_D, i.n_fine_Ddag, i.n_coarse, i.t_ms)


class Gauge:
    """A gauge field handle with the fine Wilson-Dirac operator at mass m."""

    def __init__(self, links: torch.Tensor, mass: float):
        lib = load_library()
        nd = links.shape[0]
        lat = _Lattice()
        lat.nd = nd
        self.dims = tuple(int(d) for d in reversed(links.shape[1:1 + nd]))
        for mu in range(4):
            lat.dims[mu] = self.dims[mu] if mu < nd else 1
        self.nd = nd
        self.nc = 1 if nd == 2 else 3
        self.ns = 2 if nd == 2 else 4
        self.V = 1
        for d in self.dims:
            self.V *= d
        self._links = links.contiguous()
        h = C.c_void_p()
        _check(lib.amg_gauge_create(C.byref(lat), _ptr(self._links), float(mass), _stream(), C.byref(h)),
               "amg_gauge_create")
        self._h = h
        self.mass = float(mass)

    @property
    def handle(self):
        return self._h

    def set_mass(self, m: float):
        _check(load_library().amg_gauge_set_mass(self._h, float(m)), "amg_gauge_set_mass")
        self.mass = float(m)

    @property
    def links_compressed(self) -> bool:
        """True when the 4d stencil reads two-row (12-real) SU(3) links."""
        c = C.c_int()
        _check(load_library().amg_gauge_info(self._h, None, None, C.byref(c)), "amg_gauge_info")
        return bool(c.value)

    def apply(self, psi: torch.Tensor, dagger: bool = False, prec: int = F64) -> torch.Tensor:
        """D psi (or D^dagger psi) for psi of shape (nrhs, V, ns, nc) or (V, ns, nc)."""
        dt = torch.complex128 if prec == F64 else torch.complex64
        x = psi.contiguous()
        nrhs = x.shape[0] if x.dim() == 4 else 1
        out = torch.empty_like(x)
        _check(load_library().amg_apply(self._h, int(dagger), prec, _ptr(x, dt), _ptr(out, dt), nrhs, _stream()),
               "amg_apply")
        return out

    def apply_noalloc(self, psi: torch.Tensor, out: torch.Tensor, dagger: bool = False, prec: int = F64) -> None:
        """amg_apply_noalloc into a caller-provided `out` (no device allocation by the library)."""
        dt = torch.complex128 if prec == F64 else torch.complex64
        nrhs = psi.shape[0] if psi.dim() == 4 else 1
        _check(load_library().amg_apply_noalloc(self._h, int(dagger), prec, _ptr(psi, dt), _ptr(out, dt), nrhs,
                                                 _stream()), "amg_apply_noalloc")

    def apply_internal(self, dagger: bool, prec: int, nrhs: int, iters: int):
        _check(load_library().amg_apply_internal(self._h, int(dagger), prec, nrhs, iters, _stream()),
               "amg_apply_internal")

    def cgnr(self, chi: torch.Tensor, tol: float = 1e-10, max_iter: int = 100000):
        x = chi.contiguous()
        psi = torch.empty_like(x)
        info = _Info()
        st = load_library().amg_cgnr_solve(self._h, _ptr(x), _ptr(psi), float(tol), int(max_iter), C.byref(info),
                                           _stream())
        if st not in (0, 7):
            _check(st, "amg_cgnr_solve")
        return psi, SolveInfo.from_c(info)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                load_library().amg_gauge_destroy(self._h)
                self._h = None
        except Exception:
            pass


class Solver:
    """Multigrid hierarchy + FGCR solver bound to a Gauge."""

    def __init__(self, gauge: Gauge, params: MGParams, nullvecs=None, init=None, nu0=20, ncyc=2):
        """Setup from given near-null vectors, or adaptive from random `init`
        (nu0 / ncyc: one count for every level or a list per level)."""
        lib = load_library()
        self.gauge = gauge
        self.params = params
        self._p = params.to_c()
        h = C.c_void_p()
        if nullvecs is not None:
            vs = [v.contiguous() for v in nullvecs]
            arr = (C.c_void_p * len(vs))(*[_ptr(v).value for v in vs])
            _check(lib.amg_setup(gauge.handle, C.byref(self._p), arr, _stream(), C.byref(h)), "amg_setup")
            self._keep = vs
        elif init is not None:
            vs = [v.contiguous() for v in init]
            arr = (C.c_void_p * len(vs))(*[_ptr(v).value for v in vs])
            if isinstance(nu0, (list, tuple)) or isinstance(ncyc, (list, tuple)):
                nl = len(vs)
                n0 = list(nu0) if isinstance(nu0, (list, tuple)) else [nu0] * nl
                nc = list(ncyc) if isinstance(ncyc, (list, tuple)) else [ncyc] * nl
                _check(lib.amg_setup_adaptive_levels(gauge.handle, C.byref(self._p), arr, (C.c_int * nl)(*n0),
                                                     (C.c_int * nl)(*nc), _stream(), C.byref(h)),
                       "amg_setup_adaptive_levels")
            else:
                _check(lib.amg_setup_adaptive(gauge.handle, C.byref(self._p), arr, int(nu0), int(ncyc), _stream(),
                                              C.byref(h)), "amg_setup_adaptive")
            self._keep = vs
        else:
            raise ValueError("give nullvecs (setup) or init (adaptive setup)")
        self._h = h
        self.mass = gauge.mass

    def set_mass(self, m: float):
        _check(load_library().amg_solver_set_mass(self._h, float(m)), "amg_solver_set_mass")
        self.mass = float(m)

    def level_info(self, level: int):
        dims = (C.c_int * 4)()
        dof = C.c_int()
        V = C.c_longlong()
        _check(load_library().amg_level_info(self._h, level, dims, C.byref(dof), C.byref(V)), "amg_level_info")
        return tuple(dims), dof.value, V.value

    def solve(self, chi: torch.Tensor, tol: float = 1e-10, max_iter: int = 1000, raise_noconv: bool = True):
        """psi with |chi - D psi| <= tol |chi|; chi of shape (nrhs, V, ns, nc)."""
        x = chi.contiguous()
        nrhs = x.shape[0] if x.dim() == 4 else 1
        psi = torch.empty_like(x)
        infos = (_Info * nrhs)()
        st = load_library().amg_solve(self._h, _ptr(x), _ptr(psi), nrhs, float(tol), int(max_iter), infos, _stream())
        if st != 0 and (raise_noconv or st != 7):
            _check(st, "amg_solve")
        return psi, [SolveInfo.from_c(i) for i in infos]

    def vcycle(self, b: torch.Tensor) -> torch.Tensor:
        x = b.contiguous()
        nrhs = x.shape[0] if x.dim() == 4 else 1
        out = torch.empty_like(x)
        _check(load_library().amg_vcycle(self._h, _ptr(x), _ptr(out), nrhs, _stream()), "amg_vcycle")
        return out

    def mr(self, level: int, nu: int, b: torch.Tensor, nrhs: int = 1, prec: int = F64) -> torch.Tensor:
        dt = torch.complex128 if prec == F64 else torch.complex64
        x = b.contiguous()
        out = torch.empty_like(x)
        _check(load_library().amg_mr(self._h, level, prec, nu, _ptr(x, dt), _ptr(out, dt), nrhs, _stream()), "amg_mr")
        return out

    def level_apply(self, level: int, x: torch.Tensor, dagger: bool = False, prec: int = F64, nrhs: int = 1):
        dt = torch.complex128 if prec == F64 else torch.complex64
        xi = x.contiguous()
        out = torch.empty_like(xi)
        _check(load_library().amg_level_apply(self._h, level, int(dagger), prec, _ptr(xi, dt), _ptr(out, dt), nrhs,
                                              _stream()), "amg_level_apply")
        return out

    def restrict(self, level: int, r: torch.Tensor, nrhs: int = 1, prec: int = F64) -> torch.Tensor:
        dt = torch.complex128 if prec == F64 else torch.complex64
        dims, dof, V = self.level_info(level + 1)
        out = torch.empty((nrhs, V, dof), dtype=dt, device=r.device)
        _check(load_library().amg_transfer(self._h, level, 0, prec, _ptr(r.contiguous(), dt), _ptr(out, dt), nrhs,
                                           _stream()), "amg_transfer")
        return out

    def prolong(self, level: int, e: torch.Tensor, nrhs: int = 1, prec: int = F64) -> torch.Tensor:
        dt = torch.complex128 if prec == F64 else torch.complex64
        dims, dof, V = self.level_info(level)
        out = torch.empty((nrhs, V, dof), dtype=dt, device=e.device)
        _check(load_library().amg_transfer(self._h, level, 1, prec, _ptr(e.contiguous(), dt), _ptr(out, dt), nrhs,
                                           _stream()), "amg_transfer")
        return out

    def prolongator(self, level: int, prec: int = F64) -> torch.Tensor:
        """P of coarsening `level` as stored: (V_l, dof_l, 2 nvec_l) complex128."""
        dims, dof, V = self.level_info(level)
        nc = 2 * self.params.nvec[level]
        out = torch.empty((V, dof, nc), dtype=torch.complex128, device="cuda")
        _check(load_library().amg_get_prolongator(self._h, level, prec, _ptr(out), _stream()), "amg_get_prolongator")
        return out

    def coarse_op(self, level: int) -> torch.Tensor:
        dims, dof, V = self.level_info(level)
        ndir = 2 * self.gauge.nd + 1
        out = torch.empty((V, ndir, dof, dof), dtype=torch.complex128, device="cuda")
        _check(load_library().amg_get_coarse_op(self._h, level, _ptr(out), _stream()), "amg_get_coarse_op")
        return out

    def nullvecs(self, level: int) -> torch.Tensor:
        dims, dof, V = self.level_info(level)
        nv = self.params.nvec[level]
        out = torch.empty((nv, V, dof), dtype=torch.complex128, device="cuda")
        _check(load_library().amg_get_nullvecs(self._h, level, _ptr(out), _stream()), "amg_get_nullvecs")
        return out

    @classmethod
    def _bare(cls, gauge: Gauge, params: MGParams):
        self = cls.__new__(cls)
        self.gauge = gauge
        self.params = params
        self._p = params.to_c()
        self.mass = gauge.mass
        return self

    @classmethod
    def refined(cls, gauge: Gauge, params: MGParams, start, n_start=None, nu_ref: int = 0, ncyc_ref: int = 2,
                init=None, nu0: int = 20, ncyc: int = 2):
        """Level 0 from the first n_start vectors of `start` (each relaxed by
        nu_ref MR steps) plus nvec[0] - n_start adaptive iterations from
        init[0]; deeper levels adaptive from init[l]."""
        self = cls._bare(gauge, params)
        st0 = start.contiguous()
        n_start = params.nvec[0] if n_start is None else int(n_start)
        vs = [v.contiguous() for v in (init or [st0])]
        arr = (C.c_void_p * len(vs))(*[_ptr(v).value for v in vs])
        h = C.c_void_p()
        _check(load_library().amg_setup_refined(gauge.handle, C.byref(self._p), _ptr(st0), n_start, int(nu_ref),
                                                 int(ncyc_ref), arr, int(nu0), int(ncyc), _stream(), C.byref(h)),
               "amg_setup_refined")
        self._keep = vs + [st0]
        self._h = h
        return self

    @classmethod
    def learned(cls, gauge: Gauge, params: MGParams, net: "Cnn", init, n_start=None, nu_ref: int = 0,
                ncyc_ref: int = 2, rho_max: float = 0.5, rho_iters: int = 0, nu0: int = 20, ncyc: int = 2):
        """amg_setup_learned: the network's proposals (n_start of them) plus
        adaptive iterations for the rest, falling back to the plain adaptive
        setup from `init`.  Returns (solver, fell_back, rho)."""
        self = cls._bare(gauge, params)
        n_start = params.nvec[0] if n_start is None else int(n_start)
        vs = [v.contiguous() for v in init]
        arr = (C.c_void_p * len(vs))(*[_ptr(v).value for v in vs])
        h = C.c_void_p()
        fb = C.c_int()
        rho = C.c_double()
        _check(load_library().amg_setup_learned(gauge.handle, C.byref(self._p), net.handle, arr, n_start,
                                                 int(nu_ref), int(ncyc_ref), float(rho_max), int(rho_iters),
                                                 int(nu0), int(ncyc), _stream(), C.byref(h), C.byref(fb),
                                                 C.byref(rho)), "amg_setup_learned")
        self._keep = vs
        self._h = h
        return self, bool(fb.value), rho.value

    def convergence(self, e0: torch.Tensor, iters: int = 3) -> float:
        """Convergence factor of e <- e - V(D e) from the fine field e0."""
        rho = C.c_double()
        _check(load_library().amg_mg_convergence(self._h, _ptr(e0.contiguous()), int(iters), C.byref(rho),
                                                  _stream()), "amg_mg_convergence")
        return rho.value

    PROF_FINE, PROF_COARSE, PROF_RESTRICT, PROF_PROLONG, PROF_COARSE_MR = 0, 1, 2, 3, 4

    def profile(self, kind: int, level: int, enable: bool = True):
        """Time every launch of kernel `kind` on `level` with HIP events."""
        _check(load_library().amg_profile_enable(self._h, kind, level, int(enable)), "amg_profile_enable")

    def profile_read(self, kind: int | None = None, level: int | None = None):
        """(summed kernel milliseconds, launches) since profile(); synchronises.
        With kind and level: the part of one (kind, level) of an all-kinds profile."""
        ms = C.c_double()
        n = C.c_longlong()
        if kind is None:
            _check(load_library().amg_profile_read(self._h, C.byref(ms), C.byref(n)), "amg_profile_read")
        else:
            _check(load_library().amg_profile_read_kind(self._h, int(kind), int(level), C.byref(ms), C.byref(n)),
                   "amg_profile_read_kind")
        return ms.value, n.value

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                load_library().amg_solver_destroy(self._h)
                self._h = None
        except Exception:
            pass


class Batch:
    """Independent solvers advanced together, one launch per stage over all of them."""

    def __init__(self, solvers, nrhs, autotune: bool = True):
        lib = load_library()
        self.solvers = list(solvers)
        self.nrhs = [int(k) for k in nrhs]
        n = len(self.solvers)
        hs = (C.c_void_p * n)(*[s._h.value for s in self.solvers])
        nr = (C.c_int * n)(*self.nrhs)
        h = C.c_void_p()
        _check(lib.amg_batch_create(hs, nr, n, int(autotune), _stream(), C.byref(h)), "amg_batch_create")
        self._h = h

    def info(self):
        """The launch shapes in use (autotuned or default) and, after an
        autotune, every candidate the tuner timed."""
        lib = load_library()
        cap, mrhs, stages = C.c_int(), C.c_int(), C.c_int()
        _check(lib.amg_batch_info2(self._h, C.byref(cap), C.byref(mrhs), C.byref(stages)), "amg_batch_info2")
        n = lib.amg_batch_tuning(self._h, 0, None, None, None)
        caps, mr, ms = (C.c_int * max(n, 1))(), (C.c_int * max(n, 1))(), (C.c_float * max(n, 1))()
        lib.amg_batch_tuning(self._h, n, caps, mr, ms)
        return {"red_block_cap": cap.value, "coarse_mrhs_mfma": bool(mrhs.value),
                "launches_per_outer_step": stages.value,
                "tuning": [{"red_block_cap": caps[i], "coarse_mrhs_mfma": bool(mr[i]), "ms_per_outer_step": ms[i]}
                           for i in range(n)]}

    def solve(self, chis, tol: float = 1e-10, max_iter: int = 1000, raise_noconv: bool = True):
        """chis[i]: (nrhs[i], V_i, 2, 1) complex128 on the GPU; returns (psis, infos per rhs)."""
        lib = load_library()
        xs = [c.contiguous() for c in chis]
        psis = [torch.empty_like(c) for c in xs]
        n = len(xs)
        cp = (C.c_void_p * n)(*[_ptr(c).value for c in xs])
        pp = (C.c_void_p * n)(*[_ptr(p).value for p in psis])
        infos = (_Info * sum(self.nrhs))()
        st = lib.amg_batch_solve(self._h, cp, pp, float(tol), int(max_iter), infos, _stream())
        if st != 0 and (raise_noconv or st != 7):
            _check(st, "amg_batch_solve")
        return psis, [SolveInfo.from_c(i) for i in infos]

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                load_library().amg_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Cnn:
    """The near-null-vector proposal network (two-dimensional U(1)).

    Parameters travel as one flat float32 vector: per layer W[c_out][c_in][3][3]
    then b[c_out].  Links: (B, 2, V) or (2, V) complex128 on the GPU; target
    vectors (B, 8, V, 2) complex128 (level-0 near-null vectors)."""

    CHANNELS = (4, 64, 64, 64, 32)

    def __init__(self, params, bf16: bool = True):
        import numpy as np
        lib = load_library()
        flat = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        if flat.size != self.num_params():
            raise ValueError(f"expected {self.num_params()} parameters, got {flat.size}")
        h = C.c_void_p()
        _check(lib.amg_cnn_create(_fptr(flat), int(bf16), C.byref(h)), "amg_cnn_create")
        self._h = h
        self.bf16 = bool(bf16)

    @staticmethod
    def num_params() -> int:
        return int(load_library().amg_cnn_num_params())

    @property
    def handle(self):
        return self._h

    def params(self):
        import numpy as np
        out = np.empty(self.num_params(), dtype=np.float32)
        _check(load_library().amg_cnn_get_params(self._h, _fptr(out)), "amg_cnn_get_params")
        return out

    def set_params(self, params):
        import numpy as np
        flat = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        if flat.size != self.num_params():
            raise ValueError("wrong parameter count")
        _check(load_library().amg_cnn_set_params(self._h, _fptr(flat)), "amg_cnn_set_params")

    @staticmethod
    def _shape(links: torch.Tensor, L1: int, L2: int):
        B = links.shape[0] if links.dim() == 3 else 1
        if links.shape[-1] != L1 * L2 or links.shape[-2] != 2:
            raise ValueError("links must be (B, 2, L1*L2)")
        return B

    def forward(self, links: torch.Tensor, L1: int, L2: int) -> torch.Tensor:
        B = self._shape(links, L1, L2)
        out = torch.empty((B, 32, L2, L1), dtype=torch.float32, device="cuda")
        _check(load_library().amg_cnn_forward(self._h, _ptr(links.contiguous()), B, L1, L2,
                                               _ptr(out, torch.float32), _stream()), "amg_cnn_forward")
        return out

    def loss_grad(self, links: torch.Tensor, vecs: torch.Tensor, L1: int, L2: int, grads: bool = True):
        import numpy as np
        B = self._shape(links, L1, L2)
        loss = C.c_double()
        g = np.empty(self.num_params(), dtype=np.float32) if grads else None
        _check(load_library().amg_cnn_loss_grad(self._h, _ptr(links.contiguous()), _ptr(vecs.contiguous()), B, L1,
                                                 L2, C.byref(loss), _fptr(g) if grads else None, _stream()),
               "amg_cnn_loss_grad")
        return loss.value, g

    def train_step(self, links: torch.Tensor, vecs: torch.Tensor, L1: int, L2: int, lr: float) -> float:
        B = self._shape(links, L1, L2)
        loss = C.c_double()
        _check(load_library().amg_cnn_train_step(self._h, _ptr(links.contiguous()), _ptr(vecs.contiguous()), B, L1,
                                                  L2, float(lr), C.byref(loss), _stream()), "amg_cnn_train_step")
        return loss.value

    def propose(self, links: torch.Tensor, L1: int, L2: int) -> torch.Tensor:
        self._shape(links, L1, L2)
        out = torch.empty((8, L1 * L2, 2), dtype=torch.complex128, device="cuda")
        _check(load_library().amg_cnn_propose(self._h, _ptr(links.contiguous()), L1, L2, _ptr(out), _stream()),
               "amg_cnn_propose")
        return out

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                load_library().amg_cnn_destroy(self._h)
                self._h = None
        except Exception:
            pass


@dataclass
class NormalParams:
    """Multigrid for the normal equations D^dag D (the paper's own variant):
    defaults are the paper's (4x4 blocks twice, M = 8, omega = 0.8) and the
    classical smoothing factor 4/3."""
    blocks: list = field(default_factory=lambda: [(4, 4), (4, 4)])
    nvec: list = field(default_factory=lambda: [8, 8])
    omega: float = 0.8
    sa_factor: float = 4.0 / 3.0
    power_steps: int = 20
    coarse_dense_max: int = 4096
    fine_box: bool = True
    setup_dense_max: int = 1024
    setup_coarse_tol: float = 1e-6
    setup_coarse_maxiter: int = 20000

    def to_c(self) -> _NParams:
        p = _NParams()
        load_library().amg_normal_default_params(C.byref(p))
        p.nlevels = len(self.blocks) + 1
        for l, b in enumerate(self.blocks):
            p.block[l][0], p.block[l][1] = int(b[0]), int(b[1])
            p.nvec[l] = int(self.nvec[l])
        p.omega, p.sa_factor, p.power_steps = self.omega, self.sa_factor, self.power_steps
        p.coarse_dense_max, p.setup_dense_max = self.coarse_dense_max, self.setup_dense_max
        p.fine_box = int(self.fine_box)
        p.setup_coarse_tol, p.setup_coarse_maxiter = self.setup_coarse_tol, self.setup_coarse_maxiter
        return p


@dataclass
class NormalInfo:
    iters: int
    converged: bool
    restarts: int
    rel_res_normal: float
    rel_res_D: float
    n_fine_D: int
    n_fine_Ddag: int
    t_ms: float


class NormalMG:
    """amg_normal_*: MG on A = D^dag D with the Galerkin hierarchy, the frozen
    two-step smoother and (MG-)CG, bound to a 2d Gauge."""

    def __init__(self, gauge: Gauge, params: NormalParams, smoother_b, vecs=None, init=None, nu0=20, ncyc=2):
        """From given near-null vectors `vecs` ([M, V_l, dof_l] per coarsening)
        or adaptively from `init` (nu0 / ncyc: a count or one per coarsening);
        smoother_b: one field per coarsening level ([V_l, dof_l])."""
        lib = load_library()
        self.gauge = gauge
        self.params = params
        self._p = params.to_c()
        sbs = [v.contiguous() for v in smoother_b]
        sarr = (C.c_void_p * len(sbs))(*[_ptr(v).value for v in sbs])
        h = C.c_void_p()
        if vecs is not None:
            vs = [v.contiguous() for v in vecs]
            arr = (C.c_void_p * len(vs))(*[_ptr(v).value for v in vs])
            _check(lib.amg_normal_setup(gauge.handle, C.byref(self._p), arr, sarr, _stream(), C.byref(h)),
                   "amg_normal_setup")
        else:
            vs = [v.contiguous() for v in init]
            arr = (C.c_void_p * len(vs))(*[_ptr(v).value for v in vs])
            nl = len(vs)
            n0 = list(nu0) if isinstance(nu0, (list, tuple)) else [nu0] * nl
            nc = list(ncyc) if isinstance(ncyc, (list, tuple)) else [ncyc] * nl
            _check(lib.amg_normal_setup_adaptive(gauge.handle, C.byref(self._p), arr, sarr, (C.c_int * nl)(*n0),
                                                 (C.c_int * nl)(*nc), _stream(), C.byref(h)),
                   "amg_normal_setup_adaptive")
        self._keep = (vs, sbs)
        self._h = h
        self.nlevels = len(params.blocks) + 1

    def set_mass(self, m: float):
        _check(load_library().amg_normal_set_mass(self._h, float(m), _stream()), "amg_normal_set_mass")

    def solve(self, chi: torch.Tensor, tol: float = 1e-10, max_iter: int = 100000, precond: bool = True):
        """psi with D^dag D psi = D^dag chi by MG-CG (precond) or CG."""
        x = chi.contiguous()
        psi = torch.empty_like(x)
        info = _NInfo()
        st = load_library().amg_normal_solve(self._h, _ptr(x), _ptr(psi), float(tol), int(max_iter), int(precond),
                                             C.byref(info), _stream())
        if st not in (0, 7):
            _check(st, "amg_normal_solve")
        return psi, NormalInfo(info.iters, bool(info.converged), info.restarts, info.rel_res_normal, info.rel_res_D,
                               info.n_fine_D, info.n_fine_Ddag, info.t_ms)

    def vcycle(self, x: torch.Tensor) -> torch.Tensor:
        x = x.contiguous()
        out = torch.empty_like(x)
        _check(load_library().amg_normal_vcycle(self._h, _ptr(x), _ptr(out), _stream()), "amg_normal_vcycle")
        return out

    def level_apply(self, level: int, x: torch.Tensor) -> torch.Tensor:
        x = x.contiguous()
        out = torch.empty_like(x)
        _check(load_library().amg_normal_level_apply(self._h, int(level), _ptr(x), _ptr(out), _stream()),
               "amg_normal_level_apply")
        return out

    def level_info(self, level: int) -> dict:
        dims, dof = (C.c_int * 2)(), C.c_int()
        taus, lo = (C.c_double * 2)(), (C.c_double * 2)()
        _check(load_library().amg_normal_level_info(self._h, int(level), dims, C.byref(dof), taus, lo),
               "amg_normal_level_info")
        return {"dims": (dims[0], dims[1]), "dof": dof.value, "taus": (taus[0], taus[1]),
                "lambda": lo[0], "sa_omega": lo[1]}

    def export(self, level: int, what: int) -> torch.Tensor:
        """0: P of coarsening `level` (dense), 1: A_level (dense), 2: the
        near-null vectors of coarsening `level`."""
        lib = load_library()
        if what == 0:
            f, c = self.level_info(level), self.level_info(level + 1)
            shape = (f["dims"][0] * f["dims"][1] * f["dof"], c["dims"][0] * c["dims"][1] * c["dof"])
        elif what == 1:
            i = self.level_info(level)
            n = i["dims"][0] * i["dims"][1] * i["dof"]
            shape = (n, n)
        else:
            f, c = self.level_info(level), self.level_info(level + 1)
            shape = (c["dof"], f["dims"][0] * f["dims"][1], f["dof"])
        out = torch.empty(shape, dtype=torch.complex128, device="cuda")
        _check(lib.amg_normal_export(self._h, int(level), int(what), _ptr(out), _stream()), "amg_normal_export")
        return out

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                load_library().amg_normal_destroy(self._h)
                self._h = None
        except Exception:
            pass
