"""ctypes binding of the C ABI in include/bddc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbddc.so")

BDDC_OK, BDDC_EINVAL, BDDC_ENOMEM, BDDC_ENOCONV, BDDC_EBREAKDOWN, BDDC_EFACTOR, BDDC_EDEVICE, BDDC_EBUSY = \
    0, -1, -2, -3, -4, -5, -6, -7
BDDC_FP64, BDDC_MIXED = 0, 1
BDDC_ALL_CONSTRAINED = 1
BDDC_MULTISCALE = 4
BDDC_STIFFNESS_SCALING = 8
BDDC_AUTOTUNE = 16
BDDC_DEVICE_PTRS = 1
BDDC_EAGER = 2
BDDC_STEP1_ONLY = 4
BDDC_STEP12_ONLY = 8
X_SCHUR, X_FACE_EIG, X_FACE_K, X_DSCALE, X_GAMMA, X_OMEGA, X_T, X_PSI, X_COARSE_INV = 1, 2, 3, 4, 5, 6, 7, 8, 9
OP_SYSTEM, OP_PRECOND = 1, 2

EXPORTED = ["bddc_setup", "bddc_solve", "bddc_stats", "bddc_set_stream", "bddc_destroy", "bddc_last_error",
            "bddc_sizes", "bddc_export", "bddc_apply", "bddc_time_kernel", "bddc_estimate_bytes",
            "bddc_solve_batch", "bddc_solve_block", "bddc_solve_noalloc", "bddc_set_allocator",
            "bddc_server_create", "bddc_server_submit", "bddc_server_poll", "bddc_server_stats",
            "bddc_server_destroy"]
K_SCHUR_APPLY, K_PRECOND_APPLY, K_PRECOND_FULL = 1, 2, 3
K_BLOCK_SCHUR, K_BLOCK_PRECOND_APPLY, K_BLOCK_PRECOND_FULL = 4, 5, 6


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double * 3)]


class Partition(C.Structure):
    _fields_ = [("nsub", C.c_int32 * 3), ("cuts", C.POINTER(C.c_int32) * 3)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_it", C.c_int32), ("flags", C.c_uint32), ("coarse_leaf", C.c_int32),
                ("coarse_top", C.c_int32), ("t_workgroups", C.c_int32), ("ms_source", C.POINTER(C.c_double)),
                ("bflux", C.POINTER(C.c_double)), ("coarse_subtree", C.c_int32),
                ("sweep_single", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("it", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double), ("kappa", C.c_double),
                ("lambda_min", C.c_double), ("lambda_max", C.c_double), ("omega_tilde", C.c_double),
                ("n_adaptive", C.c_int32), ("n_coarse_flux", C.c_int32), ("n_coarse", C.c_int32),
                ("n_sub", C.c_int32), ("n_gamma", C.c_int32), ("n_faces", C.c_int32), ("precision", C.c_int32),
                ("coarse_levels", C.c_int32), ("coarse_fronts", C.c_int32), ("coarse_dense", C.c_int32),
                ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("t_pcg_ms", C.c_double), ("bytes_per_iter", C.c_double), ("bytes_prec", C.c_double),
                ("device_bytes", C.c_double), ("sweep_wide4", C.c_int32), ("sweep_wide16", C.c_int32),
                ("t_workgroups", C.c_int32), ("t_tune_ms", C.c_double), ("tune_coarse_ms", C.c_double * 4),
                ("tune_precond_ms", C.c_double * 4), ("bytes_prec_block", C.c_double),
                ("flops_block_local", C.c_double), ("sweep_subtree_levels", C.c_int32), ("sweep_wide1", C.c_int32),
                ("tune_subtree_ms", C.c_double * 7), ("tune_wide1_ms", C.c_double * 4)]


class ServerOptions(C.Structure):
    _fields_ = [("mem_cap", C.c_double), ("max_active", C.c_int32), ("setup_workers", C.c_int32),
                ("precision", C.c_int32), ("flags", C.c_uint32)]


class Request(C.Structure):
    _fields_ = [("grid", Grid), ("perm", C.POINTER(C.c_double)), ("part", Partition), ("tau", C.c_double),
                ("rhs", C.POINTER(C.c_double)), ("rtol", C.c_double), ("max_it", C.c_int32),
                ("problem_key", C.c_uint64)]


class RequestStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("it", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("kappa", C.c_double), ("n_sub", C.c_int32), ("n_coarse", C.c_int32), ("queue_ms", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("latency_ms", C.c_double),
                ("est_bytes", C.c_double), ("device_bytes", C.c_double), ("peak_bytes", C.c_double),
                ("batch", C.c_int32), ("reused", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("queued", C.c_int64),
                ("active", C.c_int64), ("peak_active", C.c_int32), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("solves_per_s", C.c_double), ("peak_bytes", C.c_double), ("mem_cap", C.c_double)]


class BddcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bddc error {code}: {msg}")
        self.code = code


_lib = None

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_allocator_keep = None


def set_allocator(alloc=None, free=None):
    """Route the device allocations of handles created afterwards through
    alloc(nbytes) -> int address and free(address); None for both restores
    hipMalloc / hipFree.  The Python callables must stay thread-safe."""
    global _allocator_keep
    lib = load_library()
    if (alloc is None) != (free is None):
        raise ValueError("give both routines or neither")
    if alloc is None:
        _check(lib, lib.bddc_set_allocator(ALLOC_FN(), FREE_FN(), None))
        _allocator_keep = None
        return
    a = ALLOC_FN(lambda n, ctx: alloc(int(n)))
    f = FREE_FN(lambda p, ctx: free(int(p)))
    _check(lib, lib.bddc_set_allocator(a, f, None))
    _allocator_keep = (a, f)          # the C side holds these pointers


def load_library(path=LIB_PATH):
    """Load libbddc.so; raises if it was not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_1901_02090_amd.build.build()")
    lib = C.CDLL(path)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    lib.bddc_setup.argtypes = [C.POINTER(Grid), dp, C.POINTER(Partition), C.c_double, C.POINTER(Options),
                               C.POINTER(P)]
    lib.bddc_setup.restype = C.c_int
    lib.bddc_solve.argtypes = [P, P, C.c_double, P, P, C.c_uint32]
    lib.bddc_solve.restype = C.c_int
    lib.bddc_stats.argtypes = [P, C.POINTER(Stats)]
    lib.bddc_stats.restype = C.c_int
    lib.bddc_set_stream.argtypes = [P, P]
    lib.bddc_set_stream.restype = C.c_int
    lib.bddc_destroy.argtypes = [P]
    lib.bddc_destroy.restype = C.c_int
    lib.bddc_last_error.argtypes = []
    lib.bddc_last_error.restype = C.c_char_p
    lib.bddc_sizes.argtypes = [P, C.POINTER(C.c_int64)]
    lib.bddc_sizes.restype = C.c_int
    lib.bddc_export.argtypes = [P, C.c_int32, C.c_int32, P, C.c_int64]
    lib.bddc_export.restype = C.c_int64
    lib.bddc_apply.argtypes = [P, C.c_int32, dp, dp, dp, dp]
    lib.bddc_apply.restype = C.c_int
    lib.bddc_time_kernel.argtypes = [P, C.c_int32, C.c_int32, dp, dp]
    lib.bddc_time_kernel.restype = C.c_int
    lib.bddc_solve_batch.argtypes = [P, C.c_int32, P, C.c_double, P, P, C.c_uint32, C.POINTER(C.c_int32)]
    lib.bddc_solve_batch.restype = C.c_int
    lib.bddc_solve_block.argtypes = [P, C.c_int32, P, C.c_double, P, P, C.c_uint32, C.POINTER(C.c_int32)]
    lib.bddc_solve_block.restype = C.c_int
    lib.bddc_solve_noalloc.argtypes = [P, P, C.c_double, P, P]
    lib.bddc_solve_noalloc.restype = C.c_int
    lib.bddc_set_allocator.argtypes = [ALLOC_FN, FREE_FN, C.c_void_p]
    lib.bddc_set_allocator.restype = C.c_int
    lib.bddc_estimate_bytes.argtypes = [C.POINTER(Grid), C.POINTER(Partition), C.c_double, C.POINTER(Options), dp]
    lib.bddc_estimate_bytes.restype = C.c_int
    lib.bddc_server_create.argtypes = [C.POINTER(ServerOptions), C.POINTER(P)]
    lib.bddc_server_create.restype = C.c_int
    lib.bddc_server_submit.argtypes = [P, C.POINTER(Request), C.POINTER(C.c_uint64)]
    lib.bddc_server_submit.restype = C.c_int
    lib.bddc_server_poll.argtypes = [P, C.c_uint64, C.c_double, dp, dp, C.POINTER(RequestStats)]
    lib.bddc_server_poll.restype = C.c_int
    lib.bddc_server_stats.argtypes = [P, C.POINTER(ServerStats)]
    lib.bddc_server_stats.restype = C.c_int
    lib.bddc_server_destroy.argtypes = [P]
    lib.bddc_server_destroy.restype = C.c_int
    _lib = lib
    return lib


def _check(lib, rc, allow=()):
    if rc != BDDC_OK and rc not in allow:
        raise BddcError(rc, lib.bddc_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _grid_part(n, h, cuts):
    """ctypes grid and partition; the cut arrays are returned to keep them alive."""
    dim = len(n)
    n = tuple(int(v) for v in n)
    g = Grid(dim, (C.c_int32 * 3)(*(list(n) + [1] * (3 - dim))),
             (C.c_double * 3)(*(list(map(float, h)) + [1.0] * (3 - dim))))
    keep = [np.ascontiguousarray(c, dtype=np.int32) for c in cuts]
    cp = (C.POINTER(C.c_int32) * 3)(*[c.ctypes.data_as(C.POINTER(C.c_int32)) for c in keep] +
                                    [C.POINTER(C.c_int32)()] * (3 - dim))
    part = Partition((C.c_int32 * 3)(*([len(c) - 1 for c in keep] + [1] * (3 - dim))), cp)
    return g, part, keep


def _scaling_flag(scaling):
    if scaling == "multiplicity":
        return 0
    if scaling == "stiffness":
        return BDDC_STIFFNESS_SCALING
    raise ValueError("scaling must be 'multiplicity' or 'stiffness'")


def _steps_flag(steps):
    if steps is None:
        return 0
    if steps == 1:
        return BDDC_STEP1_ONLY
    if steps == 12:
        return BDDC_STEP12_ONLY
    raise ValueError("steps must be None, 1 or 12")


def _tau(tau):
    return float(tau) if (tau is not None and math.isfinite(tau)) else 0.0


def estimate_bytes(n, h, cuts, tau=math.inf, precision="fp64", all_constrained=False, multiscale=False):
    """Device bytes a problem may hold at the peak of its setup (host-only)."""
    lib = load_library()
    g, part, _keep = _grid_part(n, h, cuts)
    opt = Options(BDDC_MIXED if precision == "mixed" else BDDC_FP64, 0,
                  (BDDC_ALL_CONSTRAINED if all_constrained else 0) | (BDDC_MULTISCALE if multiscale else 0),
                  0, 0, 0)
    out = C.c_double()
    _check(lib, lib.bddc_estimate_bytes(C.byref(g), C.byref(part), _tau(tau), C.byref(opt), C.byref(out)))
    return out.value


class Solver:
    """One problem resident on the GPU: setup once, solve many right-hand sides."""

    def __init__(self, n, h, perm, cuts, tau=math.inf, precision="fp64", max_it=10000, all_constrained=False,
                 coarse_leaf=0, coarse_top=0, t_workgroups=0, multiscale=False,
                 scaling="multiplicity", ms_source=None, autotune=False, bflux=None, coarse_subtree=0,
                 sweep_single=0):
        """ms_source: with multiscale=True, the cell-integrated well source that
        shapes the multiscale sources of the subdomains holding a well.
        bflux: [n_faces_all] prescribed normal fluxes of the boundary faces
        (global face numbering; interior entries ignored), None: no flow."""
        self.lib = lib = load_library()
        self.n = tuple(int(v) for v in n)
        g, part, self._cuts = _grid_part(n, h, cuts)
        opt = Options(BDDC_MIXED if precision == "mixed" else BDDC_FP64, int(max_it),
                      (BDDC_ALL_CONSTRAINED if all_constrained else 0) |
                      (BDDC_MULTISCALE if multiscale else 0) | _scaling_flag(scaling) |
                      (BDDC_AUTOTUNE if autotune else 0),
                      int(coarse_leaf), int(coarse_top), int(t_workgroups))
        opt.coarse_subtree = int(coarse_subtree)
        opt.sweep_single = int(sweep_single)
        ms = None
        if ms_source is not None:
            ms = np.ascontiguousarray(ms_source, dtype=np.float64).reshape(-1)
            if ms.size != int(np.prod(self.n)):
                raise ValueError("ms_source must hold one value per cell")
            opt.ms_source = _dptr(ms)
        bf = None
        if bflux is not None:
            nn = list(self.n) + [1] * (3 - len(self.n))
            nfa = sum(int(np.prod([nn[e] + (e == d) for e in range(3)])) for d in range(len(self.n)))
            bf = np.ascontiguousarray(bflux, dtype=np.float64).reshape(-1)
            if bf.size != nfa:
                raise ValueError("bflux must hold one value per grid face")
            opt.bflux = _dptr(bf)
        perm = np.ascontiguousarray(perm, dtype=np.float64).reshape(-1)
        t = _tau(tau)
        self.h = C.c_void_p()
        _check(lib, lib.bddc_setup(C.byref(g), _dptr(perm), C.byref(part), t, C.byref(opt), C.byref(self.h)))
        sz = (C.c_int64 * 8)()
        _check(lib, lib.bddc_sizes(self.h, sz))
        (self.N, self.n_gamma, self.n_faces, self.n_coarse_flux, self.n_cells, self.n_faces_all,
         self.n_adaptive, self.max_gamma_local) = [int(v) for v in sz]

    # -- solves ----------------------------------------------------------------
    def solve(self, source, rtol=1e-8, allow_noconv=False, eager=False, steps=None):
        """steps=1 / 12: return u_0 of step 1 / u^* of steps 1-2 instead of the solution."""
        src = np.ascontiguousarray(source, dtype=np.float64)
        flux = np.empty(self.n_faces_all)
        pres = np.empty(self.n_cells)
        rc = self.lib.bddc_solve(self.h, src.ctypes.data, float(rtol), flux.ctypes.data, pres.ctypes.data,
                                 (BDDC_EAGER if eager else 0) | _steps_flag(steps))
        _check(self.lib, rc, allow=(BDDC_ENOCONV,) if allow_noconv else ())
        return flux, pres

    def solve_batch(self, sources, rtol=1e-8):
        """Solve several sources ([k, n_cells]) on the resident problem; returns (flux, pressure, iterations)."""
        src = np.ascontiguousarray(sources, dtype=np.float64).reshape(-1, self.n_cells)
        k = src.shape[0]
        flux = np.empty((k, self.n_faces_all))
        pres = np.empty((k, self.n_cells))
        its = (C.c_int32 * max(k, 1))()
        rc = self.lib.bddc_solve_batch(self.h, k, src.ctypes.data, float(rtol), flux.ctypes.data, pres.ctypes.data, 0,
                                       its)
        _check(self.lib, rc, allow=(BDDC_ENOCONV,))
        return flux, pres, np.array(its[:k], dtype=np.int32)

    def solve_block(self, sources, rtol=1e-8, eager=False):
        """Solve several sources ([k, n_cells]) with the block CG (blocks of 16
        sources per iteration); returns (flux, pressure, iterations)."""
        src = np.ascontiguousarray(sources, dtype=np.float64).reshape(-1, self.n_cells)
        k = src.shape[0]
        flux = np.empty((k, self.n_faces_all))
        pres = np.empty((k, self.n_cells))
        its = (C.c_int32 * max(k, 1))()
        rc = self.lib.bddc_solve_block(self.h, k, src.ctypes.data, float(rtol), flux.ctypes.data, pres.ctypes.data,
                                       BDDC_EAGER if eager else 0, its)
        _check(self.lib, rc, allow=(BDDC_ENOCONV,))
        return flux, pres, np.array(its[:k], dtype=np.int32)

    def solve_block_device(self, k, src_ptr, rtol, flux_ptr, pres_ptr):
        """Device-pointer block solve of k sources ([k][n_cells] at src_ptr, outputs likewise);
        returns the iterations."""
        its = (C.c_int32 * max(k, 1))()
        rc = self.lib.bddc_solve_block(self.h, int(k), C.c_void_p(src_ptr), float(rtol), C.c_void_p(flux_ptr),
                                       C.c_void_p(pres_ptr), BDDC_DEVICE_PTRS, its)
        _check(self.lib, rc, allow=(BDDC_ENOCONV,))
        return np.array(its[:k], dtype=np.int32)

    def solve_device(self, src_ptr, rtol, flux_ptr, pres_ptr, eager=False, steps=None):
        """Device-pointer solve (e.g. torch tensor data_ptr()); no host copies."""
        rc = self.lib.bddc_solve(self.h, C.c_void_p(src_ptr), float(rtol), C.c_void_p(flux_ptr),
                                 C.c_void_p(pres_ptr),
                                 BDDC_DEVICE_PTRS | (BDDC_EAGER if eager else 0) | _steps_flag(steps))
        return _check(self.lib, rc, allow=(BDDC_ENOCONV,))

    def solve_noalloc(self, src_ptr, rtol, flux_ptr, pres_ptr):
        """Device-pointer solve through bddc_solve_noalloc (no device allocation;
        CG scratch in the library's static device array)."""
        rc = self.lib.bddc_solve_noalloc(self.h, C.c_void_p(src_ptr), float(rtol), C.c_void_p(flux_ptr),
                                         C.c_void_p(pres_ptr))
        return _check(self.lib, rc, allow=(BDDC_ENOCONV,))

    def set_stream(self, stream_ptr):
        _check(self.lib, self.lib.bddc_set_stream(self.h, C.c_void_p(stream_ptr)))

    def stats(self):
        s = Stats()
        _check(self.lib, self.lib.bddc_stats(self.h, C.byref(s)))
        return {k: (list(getattr(s, k)) if isinstance(getattr(s, k), C.Array) else getattr(s, k))
                for k, _ in Stats._fields_}

    # -- diagnostics -------------------------------------------------------------
    def _export(self, what, index, count, dtype):
        out = np.empty(max(count, 1), dtype=dtype)
        rc = self.lib.bddc_export(self.h, what, index, out.ctypes.data, out.size)
        if rc < 0:
            _check(self.lib, int(rc))
        return out[:rc]

    def schur(self, i):
        n = self._export(X_SCHUR, i, self.max_gamma_local ** 2, np.float64)
        m = int(round(math.sqrt(len(n))))
        return n.reshape(m, m, order="F")

    def T(self, i):
        n = self._export(X_T, i, self.max_gamma_local ** 2, np.float64)
        m = int(round(math.sqrt(len(n))))
        return n.reshape(m, m, order="F")

    def psi(self, i):
        out = self._export(X_PSI, i, self.max_gamma_local * 1024, np.float64)
        nG = self.schur(i).shape[0]        # interface size of subdomain i
        return out.reshape(nG, -1, order="F")

    def coarse_inverse(self):
        n = self._export(X_COARSE_INV, 0, self.n_coarse_flux ** 2, np.float64)
        return n.reshape(self.n_coarse_flux, self.n_coarse_flux, order="F")

    def face_eigs(self, f):
        return self._export(X_FACE_EIG, f, 4096, np.float64)

    def face_k(self):
        return self._export(X_FACE_K, 0, self.n_faces, np.int32)

    def face_omega(self):
        return self._export(X_OMEGA, 0, self.n_faces, np.float64)

    def dscale(self):
        return self._export(X_DSCALE, 0, self.N, np.float64)

    def gamma(self):
        return self._export(X_GAMMA, 0, self.n_gamma, np.int32)

    def apply(self, which, xu, xp=None):
        xu = np.ascontiguousarray(xu, dtype=np.float64)
        xp = np.zeros(self.N) if xp is None else np.ascontiguousarray(xp, dtype=np.float64)
        yu = np.empty(self.n_gamma)
        yp = np.empty(self.N)
        _check(self.lib, self.lib.bddc_apply(self.h, which, _dptr(xu), _dptr(xp), _dptr(yu), _dptr(yp)))
        return yu, yp

    def apply_system(self, xu, xp):
        return self.apply(OP_SYSTEM, xu, xp)

    def apply_precond(self, xu):
        return self.apply(OP_PRECOND, xu)

    def time_kernel(self, which, reps=50):
        """Mean duration (ms) and algorithmic bytes of one CG kernel (or of the whole preconditioner)."""
        ms, by = C.c_double(), C.c_double()
        _check(self.lib, self.lib.bddc_time_kernel(self.h, which, int(reps), C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.bddc_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop with continuous batching over independent problems (bddc_server_*)."""

    def __init__(self, precision="fp64", mem_cap=0.0, max_active=4, setup_workers=1, all_constrained=False):
        self.lib = lib = load_library()
        opt = ServerOptions(float(mem_cap), int(max_active), int(setup_workers),
                            BDDC_MIXED if precision == "mixed" else BDDC_FP64,
                            BDDC_ALL_CONSTRAINED if all_constrained else 0)
        self.h = C.c_void_p()
        _check(lib, lib.bddc_server_create(C.byref(opt), C.byref(self.h)))
        self._sizes = {}

    def submit(self, n, h, perm, cuts, source, tau=math.inf, rtol=1e-8, max_it=10000, key=0):
        """Queue one problem; returns its ticket at once (inputs are copied).  key: nonzero for a
        problem that stays resident and is shared (and its solves batched) by the requests of that key."""
        g, part, keep = _grid_part(n, h, cuts)
        perm = np.ascontiguousarray(perm, dtype=np.float64).reshape(-1)
        src = np.ascontiguousarray(source, dtype=np.float64).reshape(-1)
        req = Request(g, _dptr(perm), part, _tau(tau), _dptr(src), float(rtol), int(max_it), int(key))
        t = C.c_uint64()
        _check(self.lib, self.lib.bddc_server_submit(self.h, C.byref(req), C.byref(t)))
        dim = len(n)
        nn = [int(v) for v in n] + [1] * (3 - dim)
        ncells = int(np.prod(nn))
        nfaces = sum(int(np.prod([nn[e] + (1 if e == d else 0) for e in range(3)])) for d in range(dim))
        self._sizes[t.value] = (nfaces, ncells)
        return t.value

    def poll(self, ticket, wait_ms=0.0):
        """None while pending; else (flux, pressure, stats dict) once done (raises on a failed request)."""
        nfaces, ncells = self._sizes[ticket]
        flux = np.empty(nfaces)
        pres = np.empty(ncells)
        st = RequestStats()
        rc = self.lib.bddc_server_poll(self.h, C.c_uint64(ticket), float(wait_ms), _dptr(flux), _dptr(pres),
                                       C.byref(st))
        if rc == BDDC_EBUSY:
            return None
        del self._sizes[ticket]
        _check(self.lib, rc, allow=(BDDC_ENOCONV,))
        return flux, pres, {k: getattr(st, k) for k, _ in RequestStats._fields_}

    def result(self, ticket):
        return self.poll(ticket, wait_ms=-1.0)

    def stats(self):
        s = ServerStats()
        _check(self.lib, self.lib.bddc_server_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.bddc_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
