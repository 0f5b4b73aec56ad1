"""Python binding of libhipsso (argument marshalling only).

Every step of the analysis runs in the HIP kernels of ``libhipsso.so``; this module converts
torch tensors (device memory, streams) into the plain pointers and sizes of the C ABI declared
in ``include/hipsso.h`` and back.  The names follow the C entry points (``sso_problem_create``,
``sso_solve`` ...); :class:`Problem` bundles them for convenience.

There is no CPU fallback: importing the binding without the built library, or calling it
without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhipsso.so")

SSO_OK, SSO_EINVAL, SSO_ENOMEM, SSO_EHIP, SSO_ENOTCONV, SSO_EBREAKDOWN = 0, -1, -2, -3, -4, -5
SSO_ESIZE = -6
NOALLOC_MAX_QUADS = 139673   # SSO_NOALLOC_MAX_QUADS
OBJ_COMPLIANCE, OBJ_STRAIN_ENERGY, OBJ_LINEAR, OBJ_USER = 0, 1, 2, 3
PREC_FP64, PREC_MIXED, PREC_AUTO = 0, 1, 2
SOLVER_AUTO, SOLVER_STANDARD, SOLVER_FUSED, SOLVER_WG = 0, 1, 2, 3

OBJECTIVES = {"compliance": OBJ_COMPLIANCE, "strain_energy": OBJ_STRAIN_ENERGY,
              "linear": OBJ_LINEAR, "user": OBJ_USER}

_vp = ctypes.c_void_p


class sso_mesh(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("xyz", _vp), ("fixed", _vp), ("f_nodal", _vp),
                ("n_beams", ctypes.c_int32), ("beam_nodes", _vp), ("beam_prop", _vp),
                ("n_quads", ctypes.c_int32), ("quad_nodes", _vp), ("quad_prop", _vp),
                ("quad_scale", _vp), ("unit_weight", ctypes.c_double),
                ("surface_load", ctypes.c_double), ("u_prescribed", _vp)]


class sso_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("max_it", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("profile_every", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("solver", ctypes.c_int32), ("inner_max_it", ctypes.c_int32)]


class sso_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("t_elem_us", ctypes.c_double), ("t_asm_us", ctypes.c_double),
                ("t_solve_us", ctypes.c_double), ("t_adj_us", ctypes.c_double),
                ("bytes_moved", ctypes.c_double), ("spmv_us", ctypes.c_double),
                ("spmv_samples", ctypes.c_int32), ("spmv_bytes", ctypes.c_double),
                ("refine_steps", ctypes.c_int32), ("solver", ctypes.c_int32),
                ("sym_products", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ("sso_problem_create", "sso_problem_create_like", "sso_problem_update", "sso_set_options", "sso_solve",
           "sso_solve_begin", "sso_solve_end", "sso_batch_create", "sso_batch_iterate",
           "sso_batch_destroy", "sso_objective", "sso_adjoint", "sso_pattern", "sso_matrix",
           "sso_sizes", "sso_strerror", "sso_problem_destroy", "sso_size_objective",
           "sso_size_objective_noalloc", "sso_size_penalty_update", "sso_hat_filter",
           "sso_problem_bytes", "sso_batch_launch", "sso_batch_wait", "sso_problem_set_stream",
           "sso_pool_trim", "sso_batch_profile", "sso_batch_timing")

_lib = None
_hip = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhipsso.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2407_20026_amd/build.py")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    lib.sso_problem_create.argtypes = [P(sso_mesh), P(sso_options), _vp, P(_vp)]
    lib.sso_problem_create_like.argtypes = [_vp, P(sso_mesh), P(sso_options), _vp, P(_vp)]
    lib.sso_problem_update.argtypes = [_vp, _vp, _vp, _vp]
    lib.sso_set_options.argtypes = [_vp, P(sso_options)]
    lib.sso_solve.argtypes = [_vp, _vp, P(sso_stats)]
    lib.sso_objective.argtypes = [_vp, ctypes.c_int, _vp, P(ctypes.c_double)]
    lib.sso_adjoint.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, P(sso_stats)]
    lib.sso_pattern.argtypes = [_vp, P(_vp), P(_vp), P(_vp), P(_vp), P(ctypes.c_int64),
                                P(ctypes.c_int64)]
    lib.sso_matrix.argtypes = [_vp, _vp, _vp]
    lib.sso_sizes.argtypes = [_vp, P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64)]
    lib.sso_pool_trim.argtypes = [ctypes.c_int, ctypes.c_uint64]
    lib.sso_problem_bytes.argtypes = [_vp, P(ctypes.c_int64)]
    lib.sso_solve_begin.argtypes = [_vp]
    lib.sso_solve_end.argtypes = [_vp, _vp, P(sso_stats)]
    lib.sso_batch_create.argtypes = [_vp, P(_vp)]
    lib.sso_batch_iterate.argtypes = [_vp, P(_vp), ctypes.c_int, ctypes.c_int,
                                      P(ctypes.c_int32)]
    lib.sso_size_objective.argtypes = [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       P(ctypes.c_double), _vp, _vp, P(sso_stats)]
    lib.sso_size_objective_noalloc.argtypes = lib.sso_size_objective.argtypes
    lib.sso_size_penalty_update.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                            P(ctypes.c_double)]
    lib.sso_hat_filter.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_double, _vp]
    lib.sso_batch_launch.argtypes = [_vp, P(_vp), ctypes.c_int, ctypes.c_int]
    lib.sso_batch_wait.argtypes = [_vp, P(_vp), ctypes.c_int, P(ctypes.c_int32)]
    lib.sso_problem_set_stream.argtypes = [_vp, _vp]
    lib.sso_batch_profile.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
    lib.sso_batch_timing.argtypes = [_vp, P(ctypes.c_double), P(ctypes.c_int64),
                                     P(ctypes.c_double), P(ctypes.c_double)]
    lib.sso_batch_destroy.argtypes = [_vp]
    lib.sso_batch_destroy.restype = None
    lib.sso_strerror.argtypes = [ctypes.c_int]
    lib.sso_strerror.restype = ctypes.c_char_p
    lib.sso_problem_destroy.argtypes = [_vp]
    lib.sso_problem_destroy.restype = None
    for name in EXPORTS:
        if name not in ("sso_strerror", "sso_problem_destroy", "sso_batch_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _hiprt():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


class SSOError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load_library().sso_strerror(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")


def pool_trim(device=0, keep_bytes: int = 0) -> None:
    """Release the library's cached device memory beyond keep_bytes (sso_pool_trim)."""
    dev = torch.device(device) if not isinstance(device, int) else torch.device("cuda", device)
    _check(load_library().sso_pool_trim(dev.index or 0, keep_bytes), "sso_pool_trim")


def _check(status: int, where: str) -> int:
    if status != SSO_OK:
        raise SSOError(status, where)
    return status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(a, dtype, device):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dtype).contiguous()


def _stream_handle(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class Options:
    precision: int = PREC_FP64
    rtol: float = 1e-8
    max_it: int = 200000
    refine_steps: int = 20
    profile_every: int = 0
    inner_rtol: float = 0.0
    solver: int = SOLVER_AUTO
    inner_max_it: int = 0

    def c(self) -> sso_options:
        return sso_options(self.precision, self.rtol, self.max_it, self.refine_steps,
                           self.profile_every, self.inner_rtol, self.solver, self.inner_max_it)


class Problem:
    """One structure on one GPU: owns the library handle and the device copies of the mesh.

    ``mesh`` is a :class:`meshgen.Mesh`-like object (numpy or torch arrays with the C-ABI
    layout).  All work runs on ``stream`` (default: torch's current stream).  ``like``: a live
    problem of the same topology whose pattern is shared (sso_problem_create_like)."""

    def __init__(self, mesh, options: Options | None = None, device="cuda", stream=None,
                 like: "Problem | None" = None):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("hipsso needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n_nodes = int(mesh.xyz.shape[0])
        self.n_beams = int(mesh.beam_nodes.shape[0])
        self.n_quads = int(mesh.quad_nodes.shape[0])
        d = self.device
        with torch.cuda.stream(self.stream):
            # uploads run on the problem's stream, so the library's copies are ordered after them
            self._xyz = _dev(mesh.xyz, torch.float64, d)
            self._fixed = _dev(mesh.fixed, torch.uint8, d)
            self._f = _dev(mesh.f_nodal, torch.float64, d)
            self._bn = _dev(mesh.beam_nodes, torch.int32, d)
            self._bp = _dev(mesh.beam_prop, torch.float64, d)
            self._qn = _dev(mesh.quad_nodes, torch.int32, d)
            self._qp = _dev(mesh.quad_prop, torch.float64, d)
            self._qs = _dev(getattr(mesh, "quad_scale", None), torch.float64, d)
            self._up = _dev(getattr(mesh, "u_prescribed", None), torch.float64, d)
        cm = sso_mesh(self.n_nodes, _ptr(self._xyz), _ptr(self._fixed), _ptr(self._f),
                      self.n_beams, _ptr(self._bn), _ptr(self._bp),
                      self.n_quads, _ptr(self._qn), _ptr(self._qp), _ptr(self._qs),
                      float(mesh.unit_weight), float(mesh.surface_load), _ptr(self._up))
        self.options = options or Options()
        opts = self.options.c()
        h = ctypes.c_void_p()
        if like is not None:
            _check(lib.sso_problem_create_like(like.handle, ctypes.byref(cm), ctypes.byref(opts),
                                               _stream_handle(self.stream), ctypes.byref(h)),
                   "sso_problem_create_like")
        else:
            _check(lib.sso_problem_create(ctypes.byref(cm), ctypes.byref(opts),
                                          _stream_handle(self.stream), ctypes.byref(h)),
                   "sso_problem_create")
        self.handle = h
        self.n_dof = 6 * self.n_nodes
        nd, nb, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.sso_sizes(h, ctypes.byref(nd), ctypes.byref(nb), ctypes.byref(nz)),
               "sso_sizes")
        self.n_blocks, self.nnz = nb.value, nz.value
        self.last_stats = None
        # bumped by every call that changes the design or the solution (update, options, solves)
        self.generation = 0

    def _new(self, shape, dtype):
        with torch.cuda.stream(self.stream):
            return torch.empty(shape, dtype=dtype, device=self.device)

    # -- lifecycle --------------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            load_library().sso_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- C entry points ---------------------------------------------------------------
    def update(self, xyz=None, quad_t=None, quad_scale=None):
        d = self.device
        # inputs may come from work queued on the caller's stream
        self.stream.wait_stream(torch.cuda.current_stream(d))
        with torch.cuda.stream(self.stream):
            self._upd = [_dev(a, torch.float64, d) for a in (xyz, quad_t, quad_scale)]
        self.generation += 1
        _check(load_library().sso_problem_update(self.handle, *[_ptr(a) for a in self._upd]),
               "sso_problem_update")

    def set_options(self, options: Options):
        self.options = options
        self.generation += 1
        o = options.c()
        _check(load_library().sso_set_options(self.handle, ctypes.byref(o)), "sso_set_options")

    def solve(self, u_out: torch.Tensor | None = None, check: bool = True):
        """Forward analysis; returns (u [n_nodes, 6] float64 device tensor, stats dict)."""
        if u_out is None:
            u_out = self._new((self.n_nodes, 6), torch.float64)
        st = sso_stats()
        self.generation += 1
        status = load_library().sso_solve(self.handle, _ptr(u_out), ctypes.byref(st))
        self.last_stats = st.as_dict()
        self.last_status = status
        if check:
            _check(status, "sso_solve")
        return u_out, self.last_stats

    def set_stream(self, stream):
        """Move the problem's work to `stream` (sso_problem_set_stream): ordered after the work
        already enqueued on its old stream."""
        _check(load_library().sso_problem_set_stream(self.handle, _stream_handle(stream)),
               "sso_problem_set_stream")
        self.stream = stream

    def solve_begin(self):
        """Everything up to the first PCG iteration; then iterate with :class:`Batch`."""
        self.generation += 1
        _check(load_library().sso_solve_begin(self.handle), "sso_solve_begin")

    def solve_end(self, u_out: torch.Tensor | None = None, check: bool = True):
        if u_out is None:
            u_out = self._new((self.n_nodes, 6), torch.float64)
        st = sso_stats()
        status = load_library().sso_solve_end(self.handle, _ptr(u_out), ctypes.byref(st))
        self.last_stats = st.as_dict()
        self.last_status = status
        if check:
            _check(status, "sso_solve_end")
        return u_out, self.last_stats

    def objective(self, kind="compliance", a=None) -> float:
        g = ctypes.c_double()
        with torch.cuda.stream(self.stream):
            at = _dev(a, torch.float64, self.device)
        _check(load_library().sso_objective(self.handle, OBJECTIVES.get(kind, kind), _ptr(at),
                                            ctypes.byref(g)), "sso_objective")
        return g.value

    def adjoint(self, kind="compliance", dg_du=None, want_t=True, want_scale=True):
        """Gradient of the objective: dict with dg_dxyz [n_nodes, 3], dg_dt [n_quads],
        dg_dscale [n_quads] (float64 device tensors) and the stats."""
        d = self.device
        gx = self._new((self.n_nodes, 3), torch.float64)
        gt = self._new(self.n_quads, torch.float64) if want_t else None
        gs = self._new(self.n_quads, torch.float64) if want_scale else None
        if dg_du is not None:
            self.stream.wait_stream(torch.cuda.current_stream(d))
        with torch.cuda.stream(self.stream):
            du = _dev(dg_du, torch.float64, d)
        st = sso_stats()
        _check(load_library().sso_adjoint(self.handle, OBJECTIVES.get(kind, kind), _ptr(du),
                                          _ptr(gx), _ptr(gt) if self.n_quads else None,
                                          _ptr(gs) if self.n_quads else None, ctypes.byref(st)),
               "sso_adjoint")
        return dict(dg_dxyz=gx, dg_dt=gt, dg_dscale=gs, stats=st.as_dict())

    def size_objective(self, eps1, u_max, t_min, want_t=True, noalloc=False, out=None):
        """Penalised material volume g = (1 + eps1 c) W of the last solve (sso_size_objective,
        or sso_size_objective_noalloc with noalloc=True): dict with g, c, W, dg_dxyz
        [n_nodes, 3], dg_dt [n_quads] and the stats.  ``out`` = (dg_dxyz, dg_dt) preallocated
        device tensors (dg_dt may be None), else allocated here."""
        if out is None:
            gx = self._new((self.n_nodes, 3), torch.float64)
            gt = self._new(self.n_quads, torch.float64) if want_t and self.n_quads else None
        else:
            gx, gt = out
        res = (ctypes.c_double * 3)()
        st = sso_stats()
        lib = load_library()
        fn = lib.sso_size_objective_noalloc if noalloc else lib.sso_size_objective
        _check(fn(self.handle, float(eps1), float(u_max), float(t_min), res, _ptr(gx), _ptr(gt),
                  ctypes.byref(st)),
               "sso_size_objective_noalloc" if noalloc else "sso_size_objective")
        return dict(g=res[0], c=res[1], W=res[2], dg_dxyz=gx, dg_dt=gt, stats=st.as_dict())

    def hat_filter(self, g, radius, nodes=None):
        """Hat-filtered nodal sensitivities (sso_hat_filter): g [n] for the design nodes
        (int indices, or None for nodes 0..n-1), weights max(0, radius - distance)."""
        d = self.device
        self.stream.wait_stream(torch.cuda.current_stream(d))
        with torch.cuda.stream(self.stream):
            gd = _dev(g, torch.float64, d)
            nd = _dev(nodes, torch.int32, d)
        n = int(gd.numel())
        out = self._new(n, torch.float64)
        _check(load_library().sso_hat_filter(self.handle, n, _ptr(nd), _ptr(gd), float(radius),
                                             _ptr(out)), "sso_hat_filter")
        return out

    @staticmethod
    def update_eps1(eps1, violated, kappa=1.015):
        """Self-adaptive penalty coefficient for the next size-optimisation step
        (sso_size_penalty_update)."""
        out = ctypes.c_double()
        _check(load_library().sso_size_penalty_update(float(eps1), int(bool(violated)),
                                                      float(kappa), ctypes.byref(out)),
               "sso_size_penalty_update")
        return out.value

    def pattern(self):
        """Copies of the scalar CSR view and the scatter permutation (int32 device tensors)."""
        rp, col, perm, seg = (ctypes.c_void_p() for _ in range(4))
        nnz, ncoo = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().sso_pattern(self.handle, ctypes.byref(rp), ctypes.byref(col),
                                          ctypes.byref(perm), ctypes.byref(seg),
                                          ctypes.byref(nnz), ctypes.byref(ncoo)), "sso_pattern")
        out = {}
        for name, src, n in (("row_ptr", rp, self.n_dof + 1), ("col", col, nnz.value),
                             ("perm", perm, ncoo.value), ("seg", seg, nnz.value + 1)):
            t = self._new(max(n, 1), torch.int32)[:n]
            if n:
                self.stream.synchronize()
                if _hiprt().hipMemcpy(_ptr(t), src, 4 * n, 3) != 0:
                    raise RuntimeError("hipMemcpy failed")
            out[name] = t
        return out

    def device_bytes(self) -> int:
        """Device memory the problem holds (sso_problem_bytes)."""
        b = ctypes.c_int64()
        _check(load_library().sso_problem_bytes(self.handle, ctypes.byref(b)), "sso_problem_bytes")
        return b.value

    def matrix(self):
        """(K values in scalar CSR order [nnz], masked load vector [n_nodes, 6])."""
        vals = self._new(self.nnz, torch.float64)
        f = self._new((self.n_nodes, 6), torch.float64)
        _check(load_library().sso_matrix(self.handle, _ptr(vals), _ptr(f)), "sso_matrix")
        return vals, f


class Batch:
    """Multi-problem PCG launcher on one stream (``sso_batch_*``)."""

    def __init__(self, stream=None, device="cuda"):
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        _check(load_library().sso_batch_create(_stream_handle(self.stream), ctypes.byref(h)),
               "sso_batch_create")
        self.handle = h

    def iterate(self, problems, n_iter: int):
        """Advance every begun, unfinished problem by n_iter iterations; returns done flags."""
        n = len(problems)
        arr = (ctypes.c_void_p * max(n, 1))(*[p.handle for p in problems])
        done = (ctypes.c_int32 * max(n, 1))()
        _check(load_library().sso_batch_iterate(self.handle, arr, n, n_iter, done),
               "sso_batch_iterate")
        return [bool(done[i]) for i in range(n)]

    def launch(self, problems, n_iter: int):
        """Enqueue n_iter iterations of every begun, unfinished problem and return at once
        (sso_batch_launch); wait(problems) with the same list collects the done flags."""
        n = len(problems)
        arr = (ctypes.c_void_p * max(n, 1))(*[p.handle for p in problems])
        _check(load_library().sso_batch_launch(self.handle, arr, n, n_iter), "sso_batch_launch")

    def wait(self, problems):
        n = len(problems)
        arr = (ctypes.c_void_p * max(n, 1))(*[p.handle for p in problems])
        done = (ctypes.c_int32 * max(n, 1))()
        _check(load_library().sso_batch_wait(self.handle, arr, n, done), "sso_batch_wait")
        return [bool(done[i]) for i in range(n)]

    def profile(self, every: int, span: int = 8):
        """Time the first span iterations of every every-th launch of FP64 standard problems
        with HIP events (sso_batch_profile; every = 0 stops); resets the sums."""
        _check(load_library().sso_batch_profile(self.handle, int(every), int(span)),
               "sso_batch_profile")

    def timing(self) -> dict:
        """Sums of the timed spans (sso_batch_timing): event time, iterations, the problem-
        iterations' algorithmic bytes with all of K counted and as the products read K."""
        us, bt, br = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        it = ctypes.c_int64()
        _check(load_library().sso_batch_timing(self.handle, ctypes.byref(us), ctypes.byref(it),
                                               ctypes.byref(bt), ctypes.byref(br)),
               "sso_batch_timing")
        return {"us": us.value, "iters": it.value, "bytes": bt.value, "bytes_read": br.value}

    def close(self):
        if getattr(self, "handle", None):
            load_library().sso_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
