"""ctypes binding of ``libsem.so`` (argument marshalling only).

Every computation happens in the C/HIP library.  Device vectors are torch
tensors on a HIP device; they are passed as raw pointers together with
torch's current stream.  The module raises at import time when the library
has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1506_05996_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

SEM_OK, SEM_EINVAL, SEM_ENOMEM, SEM_EMESH, SEM_ENOCONV, SEM_EBREAKDOWN, SEM_EHIP, SEM_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7)
SEM_F64, SEM_F32 = 0, 1
PC_NONE, PC_FINE, PC_COARSE, PC_TWOSCALE = 0, 1, 2, 3
SOLVE_FP64, SOLVE_FP32_REFINED = 0, 1

STATUS_NAMES = {0: "SEM_OK", -1: "SEM_EINVAL", -2: "SEM_ENOMEM", -3: "SEM_EMESH", -4: "SEM_ENOCONV",
                -5: "SEM_EBREAKDOWN", -6: "SEM_EHIP", -7: "SEM_EUNSUPPORTED"}

# every symbol declared in include/sem.h
EXPORTS = [
    "sem_default_setup_opts", "sem_default_solve_opts", "sem_mesh_setup", "sem_mesh_destroy",
    "sem_mesh_sizes", "sem_mesh_numbering", "sem_mesh_gs_csr", "sem_mesh_patch_table",
    "sem_mesh_node_coords", "sem_mesh_lumped_mass", "sem_mesh_boundary_mask", "sem_mesh_geometry",
    "sem_mesh_set_dirichlet", "sem_apply_A", "sem_precond", "sem_coarse_solve", "sem_pcg_solve",
    "sem_time_apply_A", "sem_mesh_tile", "sem_mesh_set_tile", "sem_mesh_coarse_factor_size", "sem_last_error", "sem_batch_setup", "sem_batch_sizes", "sem_batch_solve",
    "sem_batch_destroy", "sem_mesh_set_coefficients", "sem_mesh_coefficients", "sem_heat_step",
    "sem_mesh_set_element_coefficients", "sem_mesh_set_node_coefficients", "sem_mesh_boundary_face_mass", "sem_mesh_set_coarse_solver",
    "sem_mesh_amg_hierarchy", "sem_pcg_solve_noalloc", "sem_stream_bench",
]


class SetupOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("host_only", ctypes.c_int), ("build_fp32", ctypes.c_int),
                ("autotune", ctypes.c_int), ("tune_cache", ctypes.c_char_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("pc", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("use_x0", ctypes.c_int), ("inner_rtol", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("check_every", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer_iterations", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int),
                ("history_len", ctypes.c_int)]


_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_lib.sem_default_setup_opts.argtypes = [ctypes.POINTER(SetupOpts)]
_lib.sem_default_setup_opts.restype = None
_lib.sem_default_solve_opts.argtypes = [ctypes.POINTER(SolveOpts)]
_lib.sem_default_solve_opts.restype = None
_lib.sem_mesh_setup.argtypes = [_p, _i64, _p, _i64, ctypes.c_int, ctypes.POINTER(SetupOpts), ctypes.POINTER(_p)]
_lib.sem_mesh_destroy.argtypes = [_p]
_lib.sem_mesh_sizes.argtypes = [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
for name in ["sem_mesh_numbering", "sem_mesh_patch_table", "sem_mesh_node_coords", "sem_mesh_lumped_mass",
             "sem_mesh_boundary_mask", "sem_mesh_set_dirichlet"]:
    getattr(_lib, name).argtypes = [_p, _p]
_lib.sem_mesh_gs_csr.argtypes = [_p, _p, _p]
_lib.sem_mesh_geometry.argtypes = [_p, _p, _p]
_lib.sem_apply_A.argtypes = [_p, _p, _p, ctypes.c_int, _p]
_lib.sem_precond.argtypes = [_p, _p, _p, ctypes.c_int, ctypes.c_int, _p]
_lib.sem_coarse_solve.argtypes = [_p, _p, _p, _p]
_lib.sem_pcg_solve.argtypes = [_p, _p, _p, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), _p]
_lib.sem_stream_bench.argtypes = [_p, _p, _p, ctypes.c_int64, ctypes.c_int, _p, ctypes.POINTER(ctypes.c_double)]
_lib.sem_pcg_solve_noalloc.argtypes = [_p, _p, _p, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveStats), _p]
_lib.sem_time_apply_A.argtypes = [_p, _p, _p, ctypes.c_int, ctypes.c_int, _p, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
_lib.sem_last_error.restype = ctypes.c_char_p
_lib.sem_batch_setup.argtypes = [ctypes.c_int, _p, _p, _p, _p, _p, ctypes.POINTER(SetupOpts), ctypes.POINTER(_p)]
_lib.sem_batch_sizes.argtypes = [_p, _p]
_lib.sem_batch_solve.argtypes = [_p, _p, _p, ctypes.POINTER(SolveOpts), _p, _p]
_lib.sem_batch_destroy.argtypes = [_p]
_lib.sem_mesh_tile.argtypes = [_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
_lib.sem_mesh_coarse_factor_size.argtypes = [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
_lib.sem_mesh_set_coefficients.argtypes = [_p, ctypes.c_double, ctypes.c_double]
_lib.sem_mesh_coefficients.argtypes = [_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.sem_mesh_set_element_coefficients.argtypes = [_p, _p, _p]
_lib.sem_mesh_set_node_coefficients.argtypes = [_p, _p, _p]
_lib.sem_mesh_boundary_face_mass.argtypes = [_p, _p, _i64, _p]
_lib.sem_mesh_set_coarse_solver.argtypes = [_p, ctypes.c_int]
_lib.sem_mesh_amg_hierarchy.argtypes = [_p, _p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _p]
_lib.sem_heat_step.argtypes = [_p, ctypes.c_double, ctypes.c_double, _p, _p, _p, ctypes.POINTER(SolveOpts),
                               ctypes.POINTER(SolveStats), _p]
_lib.sem_mesh_set_tile.argtypes = [_p, ctypes.c_int, ctypes.c_int]
TILE_MFMA = 16
COARSE_EXACT, COARSE_AMG = 0, 1  # sem_coarse_solver
TILE_GEO = 32  # operator tile that rebuilds the geometric factors from the vertices
TILE_LINE_GEO = 64  # line-phase operator kernel, factors rebuilt from the vertices
TILE_LINE = 48  # line-phase operator kernel, stored factors
TILE_MFMA = 16  # matrix-core operator kernel (N = 15)


class SemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def last_error() -> str:
    return _lib.sem_last_error().decode()


def _check(status):
    if status != SEM_OK:
        raise SemError(status, last_error())
    return status


def _no_alias(a, b, na, nb):
    """Reject two tensors whose storage ranges overlap (the library forbids it)."""
    a0, b0 = a.data_ptr(), b.data_ptr()
    a1, b1 = a0 + a.numel() * a.element_size(), b0 + b.numel() * b.element_size()
    if a0 < b1 and b0 < a1:
        raise ValueError(f"{na} and {nb} must not overlap")


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_solve_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    _lib.sem_default_solve_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Mesh:
    """Owning wrapper of a ``sem_mesh`` handle."""

    def __init__(self, vtx, hexes, order, host_only=False, device=0, build_fp32=True, autotune=True,
                 tune_cache=None):
        vtx = np.ascontiguousarray(vtx, dtype=np.float64)
        hexes = np.ascontiguousarray(hexes, dtype=np.int64)
        if vtx.ndim != 2 or vtx.shape[1] != 3 or hexes.ndim != 2 or hexes.shape[1] != 8:
            raise ValueError("vtx must be [V,3] and hexes [E,8]")
        opts = SetupOpts(device=device, host_only=int(host_only), build_fp32=int(build_fp32),
                         autotune=int(autotune), tune_cache=tune_cache.encode() if tune_cache else None)
        h = ctypes.c_void_p()
        _check(_lib.sem_mesh_setup(_ptr(vtx), vtx.shape[0], _ptr(hexes), hexes.shape[0], int(order),
                                   ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.order = int(order)
        self.n_elem = hexes.shape[0]
        ng, nl, nv = _i64(), _i64(), _i64()
        _check(_lib.sem_mesh_sizes(h, ctypes.byref(ng), ctypes.byref(nl), ctypes.byref(nv)))
        self.n_global, self.n_local, self.n_vertices = ng.value, nl.value, nv.value
        self.host_only = host_only
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sem_mesh_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def handle(self):
        return self._h

    # --- host tables -------------------------------------------------------
    def numbering(self) -> np.ndarray:
        n1 = self.order + 1
        out = np.empty((self.n_elem, n1, n1, n1), dtype=np.int32)
        _check(_lib.sem_mesh_numbering(self._h, _ptr(out)))
        return out

    def gs_csr(self):
        off = np.empty(self.n_global + 1, dtype=np.int64)
        idx = np.empty(self.n_local, dtype=np.int32)
        _check(_lib.sem_mesh_gs_csr(self._h, _ptr(off), _ptr(idx)))
        return off, idx

    def patch_table(self) -> np.ndarray:
        m = self.order + 3
        out = np.empty((self.n_elem, m, m, m), dtype=np.int32)
        _check(_lib.sem_mesh_patch_table(self._h, _ptr(out)))
        return out

    def node_coords(self) -> np.ndarray:
        out = np.empty((self.n_global, 3))
        _check(_lib.sem_mesh_node_coords(self._h, _ptr(out)))
        return out

    def lumped_mass(self) -> np.ndarray:
        out = np.empty(self.n_global)
        _check(_lib.sem_mesh_lumped_mass(self._h, _ptr(out)))
        return out

    def boundary_mask(self) -> np.ndarray:
        out = np.empty(self.n_global, dtype=np.uint8)
        _check(_lib.sem_mesh_boundary_mask(self._h, _ptr(out)))
        return out

    def geometry(self):
        n1 = self.order + 1
        G = np.empty((self.n_elem, 6, n1, n1, n1))
        mass = np.empty((self.n_elem, n1, n1, n1))
        _check(_lib.sem_mesh_geometry(self._h, _ptr(G), _ptr(mass)))
        return G, mass

    def set_dirichlet(self, mask):
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mask.shape == (self.n_global,)
        _check(_lib.sem_mesh_set_dirichlet(self._h, _ptr(mask)))

    # --- device calls ------------------------------------------------------
    @staticmethod
    def _dtype_code(t):
        import torch
        if t.dtype == torch.float64:
            return SEM_F64
        if t.dtype == torch.float32:
            return SEM_F32
        raise TypeError("vectors must be float64 or float32")

    def _check_vecs(self, *specs):
        """specs: (tensor, name, dtype or None, length or None).  Each must be a
        contiguous 1D tensor of `length` entries (default n_global) on this
        handle's device, float64 or float32 (or exactly `dtype`).  Types are
        checked for every argument first, then sizes and devices; TypeError /
        ValueError are raised before anything reaches the library."""
        import torch
        for t, name, dtype, _ in specs:
            if not isinstance(t, torch.Tensor):
                raise TypeError(f"{name} must be a torch tensor")
            if dtype is not None and t.dtype != dtype:
                raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
            if t.dtype not in (torch.float64, torch.float32):
                raise TypeError(f"{name} must be float64 or float32, got {t.dtype}")
        for t, name, _, n in specs:
            n = self.n_global if n is None else n
            if not t.is_contiguous() or t.numel() != n:
                raise ValueError(f"{name} must be a contiguous tensor of {n} entries")
            if not t.is_cuda or t.device.index != self.device:
                raise ValueError(f"{name} must live on cuda:{self.device}")

    def _check_vec(self, t, n=None, dtype=None, name="vector"):
        self._check_vecs((t, name, dtype, n))

    def apply_A(self, u, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty_like(u) if isinstance(u, torch.Tensor) else None
        self._check_vecs((u, "u", None, None), (y, "y", getattr(u, "dtype", None), None))
        _no_alias(u, y, "u", "y")
        _check(_lib.sem_apply_A(self._h, _dptr(u), _dptr(y), self._dtype_code(u), _stream(stream)))
        return y

    def tile(self, dtype=SEM_F64) -> int:
        """Elements per workgroup the operator kernel uses for dtype."""
        v = ctypes.c_int()
        _check(_lib.sem_mesh_tile(self._h, int(dtype), ctypes.byref(v)))
        return v.value

    def coarse_factor_size(self):
        """(forward, backward) FP64 entries one exact coarse solve reads."""
        f, b = _i64(), _i64()
        _check(_lib.sem_mesh_coarse_factor_size(self._h, ctypes.byref(f), ctypes.byref(b)))
        return f.value, b.value

    def set_tile(self, epb, dtype=SEM_F64):
        _check(_lib.sem_mesh_set_tile(self._h, int(dtype), int(epb)))

    def time_apply_A(self, u, y, reps, stream=None):
        """Mean (element kernel, gather kernel) durations in ms over `reps` applies."""
        self._check_vecs((u, "u", None, None), (y, "y", getattr(u, "dtype", None), None))
        _no_alias(u, y, "u", "y")
        te, tg = ctypes.c_double(), ctypes.c_double()
        _check(_lib.sem_time_apply_A(self._h, _dptr(u), _dptr(y), self._dtype_code(u), int(reps), _stream(stream),
                                     ctypes.byref(te), ctypes.byref(tg)))
        return te.value, tg.value

    def precond(self, r, z=None, pc=PC_TWOSCALE, stream=None):
        import torch
        if z is None:
            z = torch.empty_like(r) if isinstance(r, torch.Tensor) else None
        self._check_vecs((r, "r", None, None), (z, "z", getattr(r, "dtype", None), None))
        _no_alias(r, z, "r", "z")
        _check(_lib.sem_precond(self._h, _dptr(r), _dptr(z), self._dtype_code(r), int(pc), _stream(stream)))
        return z

    def coarse_solve(self, R, Z=None, stream=None):
        import torch
        if Z is None:
            Z = torch.empty_like(R) if isinstance(R, torch.Tensor) else None
        self._check_vecs((R, "R", torch.float64, self.n_vertices), (Z, "Z", torch.float64, self.n_vertices))
        _check(_lib.sem_coarse_solve(self._h, _dptr(R), _dptr(Z), _stream(stream)))
        return Z

    def set_coefficients(self, kappa=1.0, c=0.0):
        """Constant kappa and c of c u - div(kappa grad u) = s for the operator,
        the preconditioner and the coarse matrix (refactorised on change)."""
        _check(_lib.sem_mesh_set_coefficients(self._h, float(kappa), float(c)))

    def set_element_coefficients(self, kappa=None, c=None):
        """One kappa_e and c_e per element (arrays [n_elem], None: 1 resp. 0)."""
        import numpy as np
        arrs = []
        for v in (kappa, c):
            if v is None:
                arrs.append(None)
            else:
                a = np.ascontiguousarray(v, dtype=np.float64)
                if a.shape != (self.n_elem,):
                    raise ValueError(f"expected shape ({self.n_elem},), got {a.shape}")
                arrs.append(a)
        _check(_lib.sem_mesh_set_element_coefficients(
            self._h, *(a.ctypes.data_as(ctypes.c_void_p) if a is not None else None for a in arrs)))

    def set_node_coefficients(self, kappa=None, c=None):
        """kappa and c at every local node (arrays [n_elem, (N+1)^3] or
        [n_elem, N+1, N+1, N+1] indexed [e, k, j, i]; None: 1 resp. 0)."""
        import numpy as np
        n1 = self.order + 1
        arrs = []
        for v in (kappa, c):
            if v is None:
                arrs.append(None)
            else:
                a = np.ascontiguousarray(v, dtype=np.float64)
                if a.size != self.n_elem * n1 ** 3 or a.shape[0] != self.n_elem:
                    raise ValueError(f"expected {self.n_elem} x {n1 ** 3} values, got shape {a.shape}")
                arrs.append(a)
        _check(_lib.sem_mesh_set_node_coefficients(
            self._h, *(a.ctypes.data_as(ctypes.c_void_p) if a is not None else None for a in arrs)))

    def boundary_face_mass(self, faces):
        """Lumped surface mass ws[n_global] of the listed boundary faces
        ((element, local face) pairs) for the Neumann term kappa g ws."""
        import numpy as np
        f = np.ascontiguousarray(faces, dtype=np.int64).reshape(-1, 2)
        ws = np.empty(self.n_global, dtype=np.float64)
        _check(_lib.sem_mesh_boundary_face_mass(self._h, f.ctypes.data_as(ctypes.c_void_p), int(f.shape[0]),
                                                ws.ctypes.data_as(ctypes.c_void_p)))
        return ws

    def set_coarse_solver(self, solver):
        """P_0: COARSE_EXACT (nested-dissection inverse) or COARSE_AMG (one K-cycle)."""
        _check(_lib.sem_mesh_set_coarse_solver(self._h, int(solver)))

    def amg_hierarchy(self, cap=32):
        """(level sizes, aggregates of the level-0 unknowns or None), built on the host."""
        sizes = np.zeros(cap, dtype=np.int64)
        nl = ctypes.c_int()
        _check(_lib.sem_mesh_amg_hierarchy(self._h, sizes.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(nl),
                                           None))
        sizes = sizes[:min(nl.value, cap)]
        agg = None
        if nl.value >= 2:
            agg = np.empty(int(sizes[0]), dtype=np.int32)
            _check(_lib.sem_mesh_amg_hierarchy(self._h, sizes.ctypes.data_as(ctypes.c_void_p), 0, ctypes.byref(nl),
                                               agg.ctypes.data_as(ctypes.c_void_p)))
        return sizes, agg

    def coefficients(self):
        k, c = ctypes.c_double(), ctypes.c_double()
        _check(_lib.sem_mesh_coefficients(self._h, ctypes.byref(k), ctypes.byref(c)))
        return k.value, c.value

    def heat_step(self, u_prev, dt, kappa, q=None, u_next=None, mode=SOLVE_FP64, pc=PC_TWOSCALE, rtol=1e-10,
                  max_iter=1000, inner_rtol=3e-3, max_outer=20, check_every=1, stream=None, raise_on_noconv=True):
        """One backward Euler step of the heat equation: (kappa A + M/dt) u_next =
        M (u_prev/dt + q), started from u_prev.  Returns (u_next, info)."""
        import torch
        if u_next is None:
            u_next = torch.empty_like(u_prev) if isinstance(u_prev, torch.Tensor) else None
        specs = [(u_prev, "u_prev", torch.float64, None), (u_next, "u_next", torch.float64, None)]
        if q is not None:
            specs.append((q, "q", torch.float64, None))
        self._check_vecs(*specs)
        if q is not None:
            _no_alias(q, u_next, "q", "u_next")
        opts = default_solve_opts(mode=mode, pc=pc, rtol=rtol, max_iter=max_iter, inner_rtol=inner_rtol,
                                  max_outer=max_outer, check_every=check_every, use_x0=1)
        st = SolveStats()
        status = _lib.sem_heat_step(self._h, float(kappa), float(dt), _dptr(u_prev),
                                    _dptr(q) if q is not None else None, _dptr(u_next), ctypes.byref(opts),
                                    ctypes.byref(st), _stream(stream))
        info = dict(status=status, iterations=st.iterations, outer=st.outer_iterations,
                    rel_residual=st.rel_residual, solve_ms=st.solve_ms)
        if status != SEM_OK and (status != SEM_ENOCONV or raise_on_noconv):
            raise SemError(status, last_error() + f" ({info})")
        return u_next, info

    def solve(self, b, x=None, mode=SOLVE_FP64, pc=PC_TWOSCALE, rtol=1e-8, max_iter=1000, inner_rtol=1e-3,
              max_outer=20, check_every=1, use_x0=False, history=0, stream=None, raise_on_noconv=True,
              noalloc=False):
        """sem_pcg_solve, or with noalloc=True sem_pcg_solve_noalloc (work in the
        library's static scratch array; pass x to keep this call free of allocation)."""
        import torch
        if x is None:
            x = torch.zeros_like(b) if isinstance(b, torch.Tensor) else None
        self._check_vecs((b, "b", torch.float64, None), (x, "x", torch.float64, None))
        _no_alias(b, x, "b", "x")
        opts = default_solve_opts(mode=mode, pc=pc, rtol=rtol, max_iter=max_iter, inner_rtol=inner_rtol,
                                  max_outer=max_outer, check_every=check_every, use_x0=int(use_x0))
        st = SolveStats()
        hist = None
        if history:
            hist = (ctypes.c_double * history)()
            st.history = hist
            st.history_cap = history
        fn = _lib.sem_pcg_solve_noalloc if noalloc else _lib.sem_pcg_solve
        status = fn(self._h, _dptr(b), _dptr(x), ctypes.byref(opts), ctypes.byref(st), _stream(stream))
        info = dict(status=status, iterations=st.iterations, outer=st.outer_iterations,
                    rel_residual=st.rel_residual, solve_ms=st.solve_ms,
                    history=list(hist[:st.history_len]) if hist is not None else None)
        if status != SEM_OK and (status != SEM_ENOCONV or raise_on_noconv):
            raise SemError(status, last_error() + f" ({info})")
        return x, info


class Batch:
    """Owning wrapper of a ``sem_batch`` handle: independent meshes solved together."""

    def __init__(self, meshes, device=0, build_fp32=True, autotune=True, tune_cache=None):
        """meshes: list of (vtx [V,3], hexes [E,8], order)."""
        self._keep = []
        n = len(meshes)
        vp, hp = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
        nv, nh, orders = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int * n)()
        for i, (vtx, hexes, order) in enumerate(meshes):
            vtx = np.ascontiguousarray(vtx, dtype=np.float64)
            hexes = np.ascontiguousarray(hexes, dtype=np.int64)
            self._keep += [vtx, hexes]
            vp[i], hp[i] = vtx.ctypes.data, hexes.ctypes.data
            nv[i], nh[i], orders[i] = vtx.shape[0], hexes.shape[0], int(order)
        opts = SetupOpts(device=device, host_only=0, build_fp32=int(build_fp32), autotune=int(autotune),
                         tune_cache=tune_cache.encode() if tune_cache else None)
        h = ctypes.c_void_p()
        self.device = int(device)
        _check(_lib.sem_batch_setup(n, ctypes.cast(vp, _p), ctypes.cast(nv, _p), ctypes.cast(hp, _p),
                                    ctypes.cast(nh, _p), ctypes.cast(orders, _p), ctypes.byref(opts),
                                    ctypes.byref(h)))
        self._h = h
        self.n = n
        ng = (ctypes.c_int64 * n)()
        _check(_lib.sem_batch_sizes(h, ctypes.cast(ng, _p)))
        self.n_global = list(ng)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.sem_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def solve(self, bs, xs=None, mode=SOLVE_FP64, pc=PC_TWOSCALE, rtol=1e-8, max_iter=1000, inner_rtol=1e-3,
              max_outer=20, check_every=1, stream=None, raise_on_noconv=True):
        import torch
        if len(bs) != self.n:
            raise ValueError("one right-hand side per instance")
        if xs is None:
            xs = [torch.zeros_like(b) for b in bs]
        if len(xs) != self.n:
            raise ValueError("one solution vector per instance")
        bp, xp = (ctypes.c_void_p * self.n)(), (ctypes.c_void_p * self.n)()
        for i, (b, x) in enumerate(zip(bs, xs)):
            for name, t in (("b", b), ("x", x)):
                if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
                    raise TypeError(f"instance {i}: {name} must be a float64 tensor")
                if (not t.is_cuda or t.device.index != self.device or not t.is_contiguous()
                        or t.numel() != self.n_global[i]):
                    raise ValueError(f"instance {i}: {name} must be a contiguous float64 vector of "
                                     f"{self.n_global[i]} entries on cuda:{self.device}")
            _no_alias(b, x, f"b[{i}]", f"x[{i}]")
            bp[i], xp[i] = b.data_ptr(), x.data_ptr()
        opts = default_solve_opts(mode=mode, pc=pc, rtol=rtol, max_iter=max_iter, inner_rtol=inner_rtol,
                                  max_outer=max_outer, check_every=check_every)
        st = (SolveStats * self.n)()
        status = _lib.sem_batch_solve(self._h, ctypes.cast(bp, _p), ctypes.cast(xp, _p), ctypes.byref(opts),
                                      ctypes.cast(st, _p), _stream(stream))
        infos = [dict(iterations=s.iterations, outer=s.outer_iterations, rel_residual=s.rel_residual,
                      solve_ms=s.solve_ms) for s in st]
        if status != SEM_OK and (status != SEM_ENOCONV or raise_on_noconv):
            raise SemError(status, last_error())
        return xs, infos, status


def stream_bench(n=1 << 28, reps=10, device=0):
    """Copy, triad and read bandwidth (GB/s) of the library's streaming probes
    over three fresh FP64 arrays of n entries on `device`."""
    import torch
    dev = torch.device("cuda", device)
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b, c = torch.empty_like(a), torch.empty_like(a)
    out = (ctypes.c_double * 3)()
    _check(_lib.sem_stream_bench(_dptr(a), _dptr(b), _dptr(c), int(n), int(reps), _stream(None), out))
    return {"copy_gbs": out[0], "triad_gbs": out[1], "read_gbs": out[2]}


def library_symbols():
    """Names of the C-ABI symbols the loaded library exports (for checks)."""
    out = {}
    for name in EXPORTS:
        try:
            out[name] = getattr(_lib, name) is not None
        except AttributeError:
            out[name] = False
    return out
