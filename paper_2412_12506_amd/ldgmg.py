"""Thin ctypes binding of libldgmg.so (the C-ABI declared in include/ldgmg.h).

Argument marshalling only: every step of the solver runs in the library.
Device vectors are passed as torch tensors (their data_ptr) or raw integer
addresses; streams as torch streams, raw hipStream_t integers or None.
The library must have been built (paper_2412_12506_amd/build.py); importing
this module does not load it, the first call does and raises if it is absent.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldgmg.so")

# enums (include/ldgmg.h)
OK, EINVAL, ENOMEM, EHIP, ENOCONV, ESINGULAR, ESTATE = 0, -1, -2, -3, -4, -5, -6
POISSON, STOKES = 0, 1
BASIS = {"legendre": 0, "gl_nodal": 1}
BC = {"D": 0, "N": 1, "P": 2}
SMOOTHER = {"jacobi": 0, "gs": 1, "sai": 2}
ORDER = {"OO": 0, "OI": 1, "IO": 2, "II": 3}
PRECISION = {"fp64": 0, "fp32": 1, "bf16s": 2}
STORAGE = {"auto": 0, "expanded": 1, "pooled": 2, "tiled": 3}
KRYLOV = {"cg": 0, "gmres": 1}
OP = {"residual": 0, "apply_a": 1, "apply_s": 2, "apply_st": 3, "smooth_fwd": 4,
      "smooth_rev": 5, "restrict": 6, "prolong_add": 7, "bottom": 8, "apply_a64": 9}
EXPORT = {"A": 0, "S": 1, "PINV": 2}


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int), ("p", C.c_int), ("basis", C.c_int),
                ("system", C.c_int), ("gamma", C.c_int), ("bc", C.c_int * 6),
                ("mu", C.POINTER(C.c_double)), ("tau0", C.c_double), ("cp", C.c_double),
                ("smoother", C.c_int), ("sai_level", C.c_int), ("order", C.c_int),
                ("nu1", C.c_int), ("nu2", C.c_int), ("omega", C.c_double), ("zeta", C.c_double),
                ("precision", C.c_int), ("nthreads", C.c_int), ("hbm_budget", C.c_size_t),
                ("storage", C.c_int), ("rho", C.POINTER(C.c_double)), ("delta", C.c_double),
                ("setup_device", C.c_int),
                ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p),
                ("alloc_ctx", C.c_void_p)]


# dev_alloc / dev_free callback types of ldgmg_problem
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class TorchAllocator:
    """dev_alloc / dev_free backed by torch's caching allocator, so that a
    hierarchy's device memory is counted by torch (memory_allocated) and
    returned to its cache on unload.  Allocations are associated with
    `stream` (torch's current stream when None) on `device`."""

    def __init__(self, device=None, stream=None):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = stream
        self.live = 0

        def _alloc(nbytes, ctx):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:
                return None
            self.live += 1
            return ptr

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)
            self.live -= 1

        self._alloc = ALLOC_FN(_alloc)      # kept alive as long as this object
        self._free = FREE_FN(_free)

    def install(self, problem: "Problem"):
        problem.dev_alloc = C.cast(self._alloc, C.c_void_p)
        problem.dev_free = C.cast(self._free, C.c_void_p)
        problem.alloc_ctx = None


class Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("rel_res_true", C.c_double),
                ("rel_res_krylov", C.c_double), ("eta", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int),
                ("history_len", C.c_int), ("vcycles", C.c_int)]


# callbacks of ldgmg_solve_stream
NEXT_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                      C.POINTER(C.c_longlong))
DONE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_longlong, C.c_int, C.POINTER(Info))


class LdgmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ldgmg error {code}: {msg}")
        self.code = code


_lib = None

SYMBOLS = ["ldgmg_problem_default", "ldgmg_estimate_bytes", "ldgmg_setup_host", "ldgmg_rebuild_smoother",
           "ldgmg_upload",
           "ldgmg_setup", "ldgmg_sizes", "ldgmg_level_info", "ldgmg_rhs_volume", "ldgmg_vcycle",
           "ldgmg_solve", "ldgmg_solve_batch", "ldgmg_vcycle_batch", "ldgmg_level_op", "ldgmg_export", "ldgmg_export_colours",
           "ldgmg_setup_stats", "ldgmg_profile", "ldgmg_profile_read", "ldgmg_unload", "ldgmg_cg_guard", "ldgmg_fp32_products", "ldgmg_device_bytes", "ldgmg_upload_bytes", "ldgmg_level_storage",
           "ldgmg_rhs_check", "ldgmg_kernel", "ldgmg_solve_stream", "ldgmg_vcycle_batch_noalloc",
           "ldgmg_setup_stats_device", "ldgmg_cg_graph", "ldgmg_destroy",
           "ldgmg_last_error"]


def lib():
    """Load libldgmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2412_12506_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
    H = C.c_void_p
    L.ldgmg_problem_default.argtypes = [C.POINTER(Problem)]
    L.ldgmg_estimate_bytes.argtypes = [C.POINTER(Problem), C.POINTER(C.c_size_t)]
    L.ldgmg_setup_host.argtypes = [C.POINTER(Problem), C.POINTER(H)]
    L.ldgmg_rebuild_smoother.argtypes = [H, C.POINTER(Problem), C.POINTER(H)]
    L.ldgmg_upload.argtypes = [H, vp]
    L.ldgmg_setup.argtypes = [C.POINTER(Problem), vp, C.POINTER(H)]
    L.ldgmg_sizes.argtypes = [H, C.POINTER(C.c_longlong), ip, ip]
    L.ldgmg_level_info.argtypes = [H, C.c_int, ip, ip, ip, ip, ip]
    L.ldgmg_rhs_volume.argtypes = [H, dp, C.c_int, vp, vp]
    L.ldgmg_vcycle.argtypes = [H, vp, vp, vp]
    L.ldgmg_solve.argtypes = [H, vp, vp, C.c_int, C.c_double, C.c_int, C.POINTER(Info), vp]
    L.ldgmg_level_op.argtypes = [H, C.c_int, C.c_int, vp, vp, vp, vp]
    L.ldgmg_solve_batch.argtypes = [C.POINTER(H), C.POINTER(vp), C.POINTER(vp), C.c_int, C.c_int, C.c_double,
                                    C.c_int, C.POINTER(Info), vp]
    L.ldgmg_rhs_check.argtypes = [H, C.c_double]
    L.ldgmg_solve_stream.argtypes = [H, C.c_int, C.c_double, C.c_int, NEXT_FN, DONE_FN, vp, vp]
    L.ldgmg_kernel.argtypes = [H, ip, dp]
    L.ldgmg_vcycle_batch.argtypes = [H, C.POINTER(vp), C.POINTER(vp), C.c_int, vp]
    L.ldgmg_vcycle_batch_noalloc.argtypes = [H, C.POINTER(vp), C.POINTER(vp), C.c_int, vp]
    L.ldgmg_export.argtypes = [H, C.c_int, C.c_int, ip, ip, dp, ip, ip]
    L.ldgmg_export_colours.argtypes = [H, C.c_int, ip]
    L.ldgmg_setup_stats.argtypes = [H, C.c_int, ip, dp]
    L.ldgmg_setup_stats_device.argtypes = [H, C.c_int, ip, ip, dp]
    L.ldgmg_profile.argtypes = [H, C.c_int]
    L.ldgmg_profile_read.argtypes = [H, C.c_int, ip, dp]
    L.ldgmg_unload.argtypes = [H]
    L.ldgmg_cg_guard.argtypes = [H, C.c_int]
    L.ldgmg_cg_graph.argtypes = [H, C.c_int]
    L.ldgmg_fp32_products.argtypes = [H, C.c_int]
    L.ldgmg_device_bytes.argtypes = [H, C.POINTER(C.c_size_t)]
    L.ldgmg_upload_bytes.argtypes = [H, C.POINTER(C.c_size_t)]
    L.ldgmg_level_storage.argtypes = [H, C.c_int, ip, ip, ip]
    L.ldgmg_destroy.argtypes = [H]
    L.ldgmg_last_error.argtypes = []
    L.ldgmg_last_error.restype = C.c_char_p
    for s in SYMBOLS[:-1]:
        getattr(L, s).restype = C.c_int
    _lib = L
    return L


def _check(rc: int, allow=()):
    if rc != OK and rc not in allow:
        raise LdgmgError(rc, lib().ldgmg_last_error().decode())
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s, *tensors) -> Optional[int]:
    """hipStream_t of `s`; with s None, torch's current stream on the device
    of the first torch tensor among `tensors` (so that the library's work is
    ordered after torch's producers of b and before its consumers of x), else
    the null stream."""
    if s is None:
        for t in tensors:
            if getattr(t, "is_cuda", False):
                import torch
                return torch.cuda.current_stream(t.device).cuda_stream
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def ldgmg_problem_default() -> Problem:
    p = Problem()
    _check(lib().ldgmg_problem_default(C.byref(p)))
    return p


def make_problem(dim: int, n: int, p: int, system: str = "poisson", basis: str = "legendre",
                 gamma: int = 1, bc=None, mu=None, tau0: float = 1.0, cp: float = 0.1,
                 smoother: str = "sai", sai_level: int = 1, order: str = "OI", nu1: int = 3,
                 nu2: int = 3, omega: float = 0.0, zeta: float = 0.0, precision: str = "fp32",
                 nthreads: int = 0, hbm_budget: int = 0, storage: str = "auto", allocator=None,
                 rho=None, delta: float = 0.0, setup_device: bool = False):
    """Problem struct plus the numpy array that backs `mu` (keep both alive).
    allocator: None (hipMalloc) or an object with install(problem), such as
    TorchAllocator (keep it alive as long as the handle)."""
    pr = ldgmg_problem_default()
    pr.dim, pr.n, pr.p = dim, n, p
    pr.system = POISSON if system == "poisson" else STOKES
    pr.basis = BASIS[basis]
    pr.gamma = gamma
    bc = bc or ["D"] * (2 * dim)
    for i in range(6):
        pr.bc[i] = BC[bc[i]] if i < len(bc) else 0
    mu_arr = None
    if mu is not None:
        mu_arr = np.ascontiguousarray(mu, dtype=np.float64)
        if mu_arr.size != n ** dim:
            raise ValueError("mu must have n^dim entries")
        pr.mu = mu_arr.ctypes.data_as(C.POINTER(C.c_double))
    pr.tau0, pr.cp = tau0, cp
    pr.smoother = SMOOTHER[smoother]
    pr.sai_level = sai_level
    pr.order = ORDER[order]
    pr.nu1, pr.nu2 = nu1, nu2
    pr.omega, pr.zeta = omega, zeta
    pr.precision = PRECISION[precision]
    pr.nthreads = nthreads
    pr.hbm_budget = hbm_budget
    pr.storage = STORAGE[storage]
    pr.delta = delta
    pr.setup_device = 1 if setup_device else 0
    if rho is not None:
        rho_arr = np.ascontiguousarray(rho, dtype=np.float64)
        if rho_arr.size != n ** dim:
            raise ValueError("rho must have n^dim entries")
        pr.rho = rho_arr.ctypes.data_as(C.POINTER(C.c_double))
        mu_arr = (mu_arr, rho_arr)        # keep both arrays alive with the struct
    if allocator is not None:
        allocator.install(pr)
    return pr, mu_arr


def ldgmg_estimate_bytes(problem: Problem) -> int:
    out = C.c_size_t(0)
    _check(lib().ldgmg_estimate_bytes(C.byref(problem), C.byref(out)))
    return out.value


def ldgmg_setup_host(problem: Problem) -> int:
    h = C.c_void_p()
    _check(lib().ldgmg_setup_host(C.byref(problem), C.byref(h)))
    return h.value


def ldgmg_rebuild_smoother(src: int, problem: Problem) -> int:
    h = C.c_void_p()
    _check(lib().ldgmg_rebuild_smoother(src, C.byref(problem), C.byref(h)))
    return h.value


def ldgmg_upload(h: int, stream=None):
    _check(lib().ldgmg_upload(h, _stream(stream)))


def ldgmg_setup(problem: Problem, stream=None) -> int:
    h = C.c_void_p()
    _check(lib().ldgmg_setup(C.byref(problem), _stream(stream), C.byref(h)))
    return h.value


def ldgmg_sizes(h: int):
    nd, bs, nl = C.c_longlong(), C.c_int(), C.c_int()
    _check(lib().ldgmg_sizes(h, C.byref(nd), C.byref(bs), C.byref(nl)))
    return nd.value, bs.value, nl.value


def ldgmg_level_info(h: int, level: int):
    v = [C.c_int() for _ in range(5)]
    _check(lib().ldgmg_level_info(h, level, *[C.byref(x) for x in v]))
    return dict(zip(["n", "nelem", "nnzb_A", "nnzb_S", "ncolours"], [x.value for x in v]))


def ldgmg_rhs_volume(h: int, f_qp: np.ndarray, nq: int, b, stream=None):
    f = np.ascontiguousarray(f_qp, dtype=np.float64)
    _check(lib().ldgmg_rhs_volume(h, f.ctypes.data_as(C.POINTER(C.c_double)), nq, _ptr(b),
                                  _stream(stream, b)))


def ldgmg_vcycle(h: int, b, x, stream=None):
    _check(lib().ldgmg_vcycle(h, _ptr(b), _ptr(x), _stream(stream, b, x)))


def ldgmg_solve(h: int, b, x, krylov: str = "cg", rtol: float = 1e-10, maxit: int = 200,
                stream=None, history_cap: int = 256) -> dict:
    hist = np.zeros(history_cap)
    info = Info()
    info.history = hist.ctypes.data_as(C.POINTER(C.c_double))
    info.history_cap = history_cap
    rc = _check(lib().ldgmg_solve(h, _ptr(b), _ptr(x), KRYLOV[krylov], rtol, maxit,
                                  C.byref(info), _stream(stream, b, x)), allow=(ENOCONV,))
    return {"iters": info.iters, "converged": bool(info.converged),
            "rel_res_true": info.rel_res_true, "rel_res_krylov": info.rel_res_krylov,
            "eta": info.eta, "history": hist[: info.history_len].copy(),
            "vcycles": info.vcycles, "status": rc}


MAX_BATCH = 16


def _ptr_array(ts):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t)
    return arr


def ldgmg_solve_batch(hs, bs, xs, rtol: float = 1e-10, maxit: int = 200, stream=None,
                      history_cap: int = 256, krylov: str = "cg") -> list:
    """Batched solve of k = len(bs) right-hand sides; hs is one handle (for
    all of them) or a list of k handles (right-hand side q on hs[q])."""
    k = len(bs)
    hl = [hs] * k if isinstance(hs, int) else list(hs)
    if len(hl) != k:
        raise ValueError("one handle per right-hand side")
    harr = (C.c_void_p * k)(*hl)
    hists = [np.zeros(history_cap) for _ in range(k)]
    infos = (Info * k)()
    for i in range(k):
        infos[i].history = hists[i].ctypes.data_as(C.POINTER(C.c_double))
        infos[i].history_cap = history_cap
    rc = _check(lib().ldgmg_solve_batch(harr, _ptr_array(bs), _ptr_array(xs), k, KRYLOV[krylov], rtol, maxit,
                                        infos, _stream(stream, *bs)), allow=(ENOCONV,))
    return [{"iters": infos[i].iters, "converged": bool(infos[i].converged),
             "rel_res_true": infos[i].rel_res_true, "rel_res_krylov": infos[i].rel_res_krylov,
             "eta": infos[i].eta, "history": hists[i][: infos[i].history_len].copy(),
             "vcycles": infos[i].vcycles, "status": rc} for i in range(k)]


def _info_dict(info, hist, rc):
    return {"iters": info.iters, "converged": bool(info.converged), "rel_res_true": info.rel_res_true,
            "rel_res_krylov": info.rel_res_krylov, "eta": info.eta,
            "history": hist[: info.history_len].copy() if hist is not None else None,
            "vcycles": info.vcycles, "status": rc}


def ldgmg_solve_stream(h: int, slots: int, next_rhs, on_done, rtol: float = 1e-10, maxit: int = 200,
                       stream=None) -> int:
    """Continuous batching (ldgmg_solve_stream).  next_rhs() returns None or
    (b, x, tag) with b, x device tensors (kept alive by the caller until
    on_done(tag, info) has been called for that tag).  Returns the status."""
    held = {}
    err = []

    def _next(ctx, pb, px, ptag):
        try:
            item = next_rhs()
        except Exception as ex:          # stop feeding; reported after the call
            err.append(ex)
            return 0
        if item is None:
            return 0
        b, x, tag = item
        held[int(tag)] = (b, x)
        pb[0] = _ptr(b)
        px[0] = _ptr(x)
        ptag[0] = int(tag)
        return 1

    def _done(ctx, tag, status, pinfo):
        try:
            on_done(int(tag), _info_dict(pinfo.contents, None, status))
        except Exception as ex:
            err.append(ex)
        held.pop(int(tag), None)

    nf, df = NEXT_FN(_next), DONE_FN(_done)
    rc = _check(lib().ldgmg_solve_stream(h, slots, rtol, maxit, nf, df, None, _stream(stream)),
                allow=(ENOCONV,))
    if err:
        raise err[0]
    return rc


def ldgmg_rhs_check(h: int, tol: float):
    _check(lib().ldgmg_rhs_check(h, tol))


def ldgmg_kernel(h: int, with_vectors: bool = False):
    """Number of kernel vectors of the fine operator (and the vectors,
    [count, ndofs], if asked)."""
    cnt = C.c_int(0)
    _check(lib().ldgmg_kernel(h, C.byref(cnt), None))
    if not with_vectors:
        return cnt.value
    nd, _, _ = ldgmg_sizes(h)
    out = np.zeros((cnt.value, nd))
    if cnt.value:
        _check(lib().ldgmg_kernel(h, C.byref(cnt), out.ctypes.data_as(C.POINTER(C.c_double))))
    return cnt.value, out


def ldgmg_vcycle_batch(h: int, bs, xs, stream=None):
    _check(lib().ldgmg_vcycle_batch(h, _ptr_array(bs), _ptr_array(xs), len(bs), _stream(stream, *bs)))


def ldgmg_vcycle_batch_noalloc(h: int, bs, xs, stream=None):
    """ldgmg_vcycle_batch with the library's static scratch array (no allocation)."""
    _check(lib().ldgmg_vcycle_batch_noalloc(h, _ptr_array(bs), _ptr_array(xs), len(bs), _stream(stream, *bs)))


def ldgmg_level_op(h: int, level: int, op: str, in1, in2, out, stream=None):
    _check(lib().ldgmg_level_op(h, level, OP[op], _ptr(in1), _ptr(in2), _ptr(out),
                                _stream(stream, in1, in2, out)))


def ldgmg_export(h: int, level: int, what: str):
    """Host FP64 export: (row_ptr, col, blocks[nnzb, bs, bs]) or a dense array (PINV)."""
    L = lib()
    nnzb, dn = C.c_int(0), C.c_int(0)
    _check(L.ldgmg_export(h, level, EXPORT[what], None, None, None, C.byref(nnzb), C.byref(dn)))
    if what == "PINV":
        N = dn.value
        out = np.zeros((N, N))
        _check(L.ldgmg_export(h, level, EXPORT[what], None, None,
                              out.ctypes.data_as(C.POINTER(C.c_double)), None, C.byref(dn)))
        return out
    _, bs, _ = ldgmg_sizes(h)
    info = ldgmg_level_info(h, level)
    ne = info["nelem"]
    bs = bs  # same block size on every level
    rp = np.zeros(ne + 1, dtype=np.int32)
    ci = np.zeros(nnzb.value, dtype=np.int32)
    blocks = np.zeros((nnzb.value, bs, bs))
    _check(L.ldgmg_export(h, level, EXPORT[what], rp.ctypes.data_as(C.POINTER(C.c_int)),
                          ci.ctypes.data_as(C.POINTER(C.c_int)),
                          blocks.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nnzb), None))
    return rp, ci, blocks


def ldgmg_export_colours(h: int, level: int) -> np.ndarray:
    ne = ldgmg_level_info(h, level)["nelem"]
    out = np.zeros(ne, dtype=np.int32)
    _check(lib().ldgmg_export_colours(h, level, out.ctypes.data_as(C.POINTER(C.c_int))))
    return out


def ldgmg_setup_stats(h: int, level: int):
    u, s = C.c_int(), C.c_double()
    _check(lib().ldgmg_setup_stats(h, level, C.byref(u), C.byref(s)))
    return u.value, s.value


def ldgmg_setup_stats_device(h: int, level: int):
    """(SAI problems solved on the device, by host QR, seconds of the level's SAI solves)."""
    d, q, t = C.c_int(), C.c_int(), C.c_double()
    _check(lib().ldgmg_setup_stats_device(h, level, C.byref(d), C.byref(q), C.byref(t)))
    return d.value, q.value, t.value


PROFILE_KIND = {"A": 0, "S": 1, "ST": 2, "A64": 3, "FUSED": 4}


def ldgmg_profile(h: int, enable: bool):
    _check(lib().ldgmg_profile(h, 1 if enable else 0))


def ldgmg_profile_read(h: int, kind: str):
    """(launch count, summed milliseconds) of one kind of fine-level launch."""
    cnt, ms = C.c_int(), C.c_double()
    _check(lib().ldgmg_profile_read(h, PROFILE_KIND[kind], C.byref(cnt), C.byref(ms)))
    return cnt.value, ms.value


def ldgmg_unload(h: int):
    _check(lib().ldgmg_unload(h))


def ldgmg_cg_guard(h: int, enable: bool = True):
    _check(lib().ldgmg_cg_guard(h, 1 if enable else 0))


def ldgmg_cg_graph(h: int, check_every: int = 4):
    """CG solves of the handle replay one captured iteration check_every times
    between host checks (0: eager)."""
    _check(lib().ldgmg_cg_graph(h, int(check_every)))


def ldgmg_fp32_products(h: int, enable: bool = True):
    _check(lib().ldgmg_fp32_products(h, 1 if enable else 0))


def ldgmg_device_bytes(h: int) -> int:
    out = C.c_size_t(0)
    _check(lib().ldgmg_device_bytes(h, C.byref(out)))
    return out.value


def ldgmg_upload_bytes(h: int) -> int:
    out = C.c_size_t(0)
    _check(lib().ldgmg_upload_bytes(h, C.byref(out)))
    return out.value


def ldgmg_level_storage(h: int, level: int) -> dict:
    a, b, t = C.c_int(0), C.c_int(0), C.c_int(0)
    _check(lib().ldgmg_level_storage(h, level, C.byref(a), C.byref(b), C.byref(t)))
    return {"pool_A": a.value, "pool_S": b.value, "tiled_A": bool(t.value & 1), "tiled_S": bool(t.value & 2)}


def ldgmg_destroy(h: int):
    if h:
        lib().ldgmg_destroy(h)


def export_bsr(h: int, level: int, what: str = "A"):
    """Export as a scipy BSR matrix (test helper)."""
    import scipy.sparse as sp
    rp, ci, blocks = ldgmg_export(h, level, what)
    ne = rp.size - 1
    bs = blocks.shape[1]
    return sp.bsr_matrix((blocks, ci, rp), shape=(ne * bs, ne * bs))


class Solver:
    """Owns one handle.  Example:
        s = Solver(dim=3, n=16, p=3); s.upload(); info = s.solve(b, x)
    """

    def __init__(self, host_only: bool = False, stream=None, fp32_products: bool = False, **kw):
        self._allocator = kw.get("allocator")
        self.problem, self._mu = make_problem(**kw)
        self.handle = ldgmg_setup_host(self.problem)
        self.ndofs, self.bs, self.nlevels = ldgmg_sizes(self.handle)
        if fp32_products:
            ldgmg_fp32_products(self.handle, True)
        if not host_only:
            self.upload(stream)

    def upload(self, stream=None):
        ldgmg_upload(self.handle, stream)

    def resmoothed(self, **kw) -> "Solver":
        """A host-only Solver for the same problem with another smoother (kw as
        for the constructor), reusing this hierarchy's operators and bottom."""
        new = Solver.__new__(Solver)
        new._allocator = kw.get("allocator")
        new.problem, new._mu = make_problem(**kw)
        new.handle = ldgmg_rebuild_smoother(self.handle, new.problem)
        new.ndofs, new.bs, new.nlevels = ldgmg_sizes(new.handle)
        return new

    def unload(self):
        ldgmg_unload(self.handle)

    @property
    def device_bytes(self) -> int:
        return ldgmg_device_bytes(self.handle)

    @property
    def upload_bytes(self) -> int:
        return ldgmg_upload_bytes(self.handle)

    def vcycle(self, b, x, stream=None):
        ldgmg_vcycle(self.handle, b, x, stream)

    def solve(self, b, x, krylov="cg", rtol=1e-10, maxit=200, stream=None):
        return ldgmg_solve(self.handle, b, x, krylov, rtol, maxit, stream)

    def close(self):
        if getattr(self, "handle", None):
            ldgmg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
