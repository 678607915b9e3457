"""Python binding of libblr (the MI355X collision hot path of the adaptive
dynamical low-rank Boltzmann method).

Argument marshalling only: every step of the computation runs in the HIP
library ``libblr.so`` built from ``csrc/`` (see ``build.py``).  PyTorch
supplies device memory and the stream.  Loading fails loudly when the library
is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblr.so")

BLR_FP32, BLR_FP64 = 0, 1
BLR_NO_CONSERVE = 0x1
BLR_PLAIN_SCHEDULE = 0x2
BLR_GENERIC_FFT = 0x4
BLR_CARLEMAN = 0x8
BLR_DEALIAS = 0x10
BLR_STEP_ADD = 0x1
BLR_STEP_DROP = 0x2
BLR_STEP_FP64_COLLISION = 0x4
BLR_STEP_HOUSEHOLDER_ADD = 0x8
BLR_STEP_HOUSEHOLDER_QR = 0x10
BLR_STEP_EAGER = 0x20
BLR_STEP_FP64_DEFECT = 0x40
BLR_STEP_DEFECT_REFRESH = 0x80

(BLR_OK, BLR_ERR_ARG, BLR_ERR_NOMEM, BLR_ERR_HIP, BLR_ERR_UNSUPPORTED, BLR_ERR_NUMERIC,
 BLR_ERR_NOT_CONVERGED) = range(7)
STATUS = {0: "BLR_OK", 1: "BLR_ERR_ARG", 2: "BLR_ERR_NOMEM", 3: "BLR_ERR_HIP",
          4: "BLR_ERR_UNSUPPORTED", 5: "BLR_ERR_NUMERIC", 6: "BLR_ERR_NOT_CONVERGED"}

EXPORTS = ["blr_create", "blr_destroy", "blr_last_error", "blr_workspace_bytes",
           "blr_collision_pairs", "blr_collision_pairs_noalloc", "blr_state_from_full", "blr_dlr_step", "blr_steady_solve",
           "blr_full_step", "blr_server_create", "blr_server_submit", "blr_server_wait",
           "blr_server_load", "blr_server_clock", "blr_server_last_error", "blr_server_destroy"]


class BlrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class VGrid(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n", ctypes.c_int32), ("L", ctypes.c_double),
                ("R", ctypes.c_double), ("C", ctypes.c_double), ("gamma", ctypes.c_double),
                ("m_rho", ctypes.c_int32), ("m_sigma", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("aniso_n", ctypes.c_int32), ("aniso", ctypes.c_double * 5)]


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
                ("f_left", ctypes.c_void_p), ("f_right", ctypes.c_void_p), ("v", VGrid),
                ("wall_left", ctypes.c_int32), ("wall_right", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("y_lo", ctypes.c_double), ("y_hi", ctypes.c_double),
                ("f_bottom", ctypes.c_void_p), ("f_top", ctypes.c_void_p),
                ("wall_bottom", ctypes.c_int32), ("wall_top", ctypes.c_int32),
                ("face_rows", ctypes.c_int32), ("solid", ctypes.c_void_p),
                ("f_obstacle", ctypes.c_void_p)]


class State(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("r_cap", ctypes.c_int32), ("X", ctypes.c_void_p),
                ("S", ctypes.c_void_p), ("V", ctypes.c_void_p), ("step", ctypes.c_int64),
                ("seed", ctypes.c_uint64)]


class StepParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("c_drop", ctypes.c_double), ("add_tol", ctypes.c_double),
                ("r_min", ctypes.c_int32), ("r_max", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class StepInfo(ctypes.Structure):
    _fields_ = [("err", ctypes.c_double), ("err_ada", ctypes.c_double), ("drop_tol", ctypes.c_double),
                ("r_in", ctypes.c_int32), ("r_added", ctypes.c_int32), ("r_out", ctypes.c_int32),
                ("ms_collision", ctypes.c_float), ("ms_step", ctypes.c_float)]


class SolveParams(ctypes.Structure):
    _fields_ = [("step", StepParams), ("res_tol", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("defect_every", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("err_ada", ctypes.c_double), ("r", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("ms_wall", ctypes.c_double),
                ("pair_evals", ctypes.c_int64)]


class ServerParams(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("hbm_budget", ctypes.c_int64),
                ("batch_collisions", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("problem", Problem), ("state", ctypes.POINTER(State)), ("solve", SolveParams),
                ("tag", ctypes.c_int64)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("info", SolveInfo), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("bytes", ctypes.c_int64),
                ("message", ctypes.c_char * 128)]


_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libblr.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"libblr.so not built at {path}; run __graft_entry__.build() "
                          f"or python paper_2112_02695_amd/build.py")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.blr_create.argtypes = [ctypes.c_int, P, ctypes.POINTER(P)]
    lib.blr_destroy.argtypes = [P]
    lib.blr_last_error.argtypes = [P]
    lib.blr_last_error.restype = ctypes.c_char_p
    lib.blr_workspace_bytes.argtypes = [P, ctypes.POINTER(VGrid), ctypes.c_int32, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_size_t)]
    lib.blr_collision_pairs.argtypes = [P, ctypes.POINTER(VGrid), ctypes.c_int, P, ctypes.c_int32,
                                        P, ctypes.c_int32, P]
    if hasattr(lib, "blr_collision_pairs_noalloc"):
        lib.blr_collision_pairs_noalloc.argtypes = lib.blr_collision_pairs.argtypes
    if hasattr(lib, "blr_dlr_step"):
        lib.blr_state_from_full.argtypes = [P, ctypes.POINTER(Problem), P, ctypes.c_int32,
                                            ctypes.POINTER(State)]
        lib.blr_svd_small.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, P]
        lib.blr_dlr_step.argtypes = [P, ctypes.POINTER(Problem), ctypes.POINTER(State),
                                     ctypes.POINTER(StepParams), ctypes.POINTER(StepInfo)]
        lib.blr_steady_solve.argtypes = [P, ctypes.POINTER(Problem), ctypes.POINTER(State),
                                         ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo)]
    if hasattr(lib, "blr_full_step"):
        lib.blr_full_step.argtypes = [P, ctypes.POINTER(Problem), ctypes.c_int, P, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)]
    if hasattr(lib, "blr_server_create"):
        lib.blr_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(ServerParams),
                                          ctypes.POINTER(P)]
        lib.blr_server_submit.argtypes = [P, ctypes.POINTER(Request)]
        lib.blr_server_wait.argtypes = [P, ctypes.c_int32, ctypes.c_double,
                                        ctypes.POINTER(Completion), ctypes.POINTER(ctypes.c_int32)]
        lib.blr_server_load.argtypes = [P, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]
        lib.blr_server_clock.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
        lib.blr_server_batch_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int64)]
        lib.blr_server_last_error.argtypes = [P]
        lib.blr_server_destroy.argtypes = [P]
    for name in EXPORTS:
        if hasattr(lib, name):
            getattr(lib, name).restype = (ctypes.c_char_p if name.endswith("last_error")
                                          else ctypes.c_int)
    _LIB = lib
    return lib


def make_vgrid(d: int, n: int, L: float, C: float = 1.0, gamma: float = 0.0, m_rho: int = 16,
               m_sigma: int = 0, R: float = 0.0, flags: int = 0, aniso=None) -> VGrid:
    """aniso: the coefficients of the kernel's angular factor (Legendre in 3D,
    Chebyshev in 2D), at most 5; None for the isotropic kernel."""
    co = [float(x) for x in (aniso or ())]
    if len(co) > 5:
        raise ValueError("at most 5 angular coefficients")
    arr = (ctypes.c_double * 5)(*(co + [0.0] * (5 - len(co))))
    return VGrid(d, n, float(L), float(R), float(C), float(gamma), m_rho, m_sigma, flags,
                 len(co), arr)


def vgrid_from_spec(spec, flags: int = 0, aniso=None) -> VGrid:
    return make_vgrid(spec.d, spec.n, spec.L, spec.C, spec.gamma, spec.m_rho, spec.m_sigma,
                      flags=flags, aniso=aniso)


class Context:
    """A libblr context bound to one device and one HIP stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.blr_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise BlrError(rc, "blr_create failed")
        self.h = h

    def _check(self, rc):
        if rc != 0:
            msg = self.lib.blr_last_error(self.h)
            raise BlrError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.blr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, vg: VGrid, r_max: int, precision: int) -> int:
        out = ctypes.c_size_t()
        self._check(self.lib.blr_workspace_bytes(self.h, ctypes.byref(vg), r_max, precision,
                                                 ctypes.byref(out)))
        return out.value

    def collision_pairs(self, vg: VGrid, V, pairs, out=None, noalloc: bool = False):
        """Q_s(V_i, V_j) for each row (i, j) of ``pairs``; V is a CUDA tensor
        (r, n^d) of float32 or float64.  Returns (npairs, n^d) on the stream.
        noalloc: call blr_collision_pairs_noalloc (workspace in the library's
        fixed device array; ``out`` must then be given)."""
        import torch
        if not (V.is_cuda and V.dim() == 2 and V.is_contiguous()):
            raise ValueError("V must be a contiguous 2-D CUDA tensor (r, n^d)")
        prec = {torch.float32: BLR_FP32, torch.float64: BLR_FP64}[V.dtype]
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        npairs = pr.shape[0]
        if out is None:
            out = torch.empty((npairs, V.shape[1]), dtype=V.dtype, device=V.device)
        assert out.is_contiguous() and out.dtype == V.dtype and out.shape[0] >= npairs
        fn = self.lib.blr_collision_pairs_noalloc if noalloc else self.lib.blr_collision_pairs
        self._check(fn(
            self.h, ctypes.byref(vg), prec, ctypes.c_void_p(V.data_ptr()), V.shape[0],
            pr.ctypes.data_as(ctypes.c_void_p), npairs, ctypes.c_void_p(out.data_ptr())))
        return out

    # -------------------------------------------------------------- DLR --
    def make_problem(self, vg: VGrid, nx: int, x_lo: float, x_hi: float, fL, fR,
                     wall_left: bool = False, wall_right: bool = False) -> Problem:
        """fL / fR: float64 CUDA tensors of n^d values, the inflow Maxwellians, or
        the wall Maxwellians' shapes where wall_left / wall_right is set
        (Maxwell diffusive walls)."""
        assert fL.dtype.itemsize == 8 and fR.dtype.itemsize == 8
        pb = Problem(nx, float(x_lo), float(x_hi), ctypes.c_void_p(fL.data_ptr()),
                     ctypes.c_void_p(fR.data_ptr()), vg, int(bool(wall_left)),
                     int(bool(wall_right)))
        pb._keep = (fL, fR)
        return pb

    def make_problem2d(self, vg: VGrid, nx: int, ny: int, x_lo: float, x_hi: float, y_lo: float,
                       y_hi: float, faces, solid=None, obstacle=None) -> Problem:
        """Rectangle with nx x ny cells (cell ix ny + iy).  faces: four (f, wall)
        pairs for x_lo, x_hi, y_lo, y_hi; f a float64 CUDA tensor of n^d values
        (one row for the face) or (face cells, n^d) (one row per face cell:
        ny on an x face, nx on a y face); wall=True: a Maxwell diffusive wall
        whose Maxwellian shape f is.  solid: optional host array of nx ny
        cells (nonzero = solid); obstacle: the float64 CUDA tensor of n^d
        values giving the shape of the obstacle walls' Maxwellian."""
        assert len(faces) == 4
        rows = 0
        for k, (f, _) in enumerate(faces):
            assert f.dtype.itemsize == 8 and f.is_contiguous()
            if f.dim() == 2:
                assert f.shape[0] == (ny if k < 2 else nx)
                rows |= 1 << k
        f = [ctypes.c_void_p(t.data_ptr()) for t, _ in faces]
        w = [int(bool(x)) for _, x in faces]
        keep = [t for t, _ in faces]
        sp, op = None, None
        if solid is not None:
            import numpy as np
            sm = np.ascontiguousarray(np.asarray(solid).reshape(-1) != 0, dtype=np.uint8)
            assert sm.size == nx * ny
            keep.append(sm)
            sp = ctypes.c_void_p(sm.ctypes.data)
        if obstacle is not None:
            assert obstacle.dtype.itemsize == 8 and obstacle.is_contiguous()
            keep.append(obstacle)
            op = ctypes.c_void_p(obstacle.data_ptr())
        pb = Problem(nx, float(x_lo), float(x_hi), f[0], f[1], vg, w[0], w[1], ny, float(y_lo),
                     float(y_hi), f[2], f[3], w[2], w[3], rows, sp, op)
        pb._keep = tuple(keep)
        return pb

    def make_state(self, X, S, V, r: int, seed: int = 0) -> State:
        """X (r_cap, nx), S (r_cap, r_cap), V (r_cap, n^d): float64 CUDA tensors."""
        r_cap = X.shape[0]
        assert S.shape == (r_cap, r_cap) and V.shape[0] == r_cap
        st = State(r, r_cap, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(S.data_ptr()),
                   ctypes.c_void_p(V.data_ptr()), 0, seed)
        st._keep = (X, S, V)
        return st

    def svd_small(self, A, trans: bool = False, complete: bool = True):
        """A = U diag(sig) W^T (of A^T when trans) for a square float64 CUDA
        tensor of at most 64 x 64; returns (U, sig, W) on the stream."""
        import torch
        assert A.is_cuda and A.dtype == torch.float64 and A.is_contiguous() and A.dim() == 2
        r = A.shape[0]
        assert A.shape[1] == r
        U = torch.empty((r, r), dtype=torch.float64, device=A.device)
        W = torch.empty((r, r), dtype=torch.float64, device=A.device)
        sig = torch.empty((r,), dtype=torch.float64, device=A.device)
        self._check(self.lib.blr_svd_small(self.h, ctypes.c_void_p(A.data_ptr()), r, int(bool(trans)),
                                           int(bool(complete)), ctypes.c_void_p(U.data_ptr()),
                                           ctypes.c_void_p(sig.data_ptr()),
                                           ctypes.c_void_p(W.data_ptr())))
        return U, sig, W

    def state_from_full(self, pb: Problem, f0, r: int, st: State):
        self._check(self.lib.blr_state_from_full(self.h, ctypes.byref(pb),
                                                 ctypes.c_void_p(f0.data_ptr()), r, ctypes.byref(st)))
        return st

    def dlr_step(self, pb: Problem, st: State, sp: StepParams) -> StepInfo:
        info = StepInfo()
        self._check(self.lib.blr_dlr_step(self.h, ctypes.byref(pb), ctypes.byref(st),
                                          ctypes.byref(sp), ctypes.byref(info)))
        return info

    def steady_solve(self, pb: Problem, st: State, p: SolveParams, allow_unconverged=False):
        info = SolveInfo()
        rc = self.lib.blr_steady_solve(self.h, ctypes.byref(pb), ctypes.byref(st), ctypes.byref(p),
                                       ctypes.byref(info))
        if rc == 6 and allow_unconverged:
            return info
        self._check(rc)
        return info

    # ------------------------------------------------------ full tensor --
    def full_step(self, pb: Problem, F, dt: float, prec: int = BLR_FP32) -> float:
        """One full-tensor step of F (float64 CUDA tensor of nx (nx ny on a
        rectangle) rows of n^d values, updated in place); returns err_full."""
        cells = pb.nx * (pb.ny if pb.ny >= 2 else 1)
        assert F.dtype.itemsize == 8 and F.is_contiguous() and F.shape[0] == cells
        err = ctypes.c_double()
        self._check(self.lib.blr_full_step(self.h, ctypes.byref(pb), prec,
                                           ctypes.c_void_p(F.data_ptr()), float(dt),
                                           ctypes.byref(err)))
        return err.value


class Server:
    """Steady solves served on one device (``blr_server_*``): ``slots`` solves
    at once, each on its own context, stream and host thread, admitted first
    in, first out as slots and the device-memory budget allow.

    ``submit`` keeps the problem, the state and their tensors alive until the
    request's completion has been returned by ``wait``.  batch_collisions: the
    FP32 pair collisions of all live solves on the fused grids run together,
    one launch sequence per step (see blr_server_params)."""

    def __init__(self, device: int = 0, slots: int = 4, hbm_budget: int = 0,
                 batch_collisions: bool = False):
        self.lib = load_library()
        h = ctypes.c_void_p()
        rc = self.lib.blr_server_create(
            device, ctypes.byref(ServerParams(slots, hbm_budget, int(bool(batch_collisions)))),
            ctypes.byref(h))
        if rc != 0:
            raise BlrError(rc, "blr_server_create failed")
        self.h = h
        self._live = {}

    def batch_stats(self):
        """(batches run, step collisions they held) with batch_collisions."""
        r, j = ctypes.c_int64(), ctypes.c_int64()
        rc = self.lib.blr_server_batch_stats(self.h, ctypes.byref(r), ctypes.byref(j))
        if rc != 0:
            raise BlrError(rc, "blr_server_batch_stats failed")
        return r.value, j.value

    def submit(self, pb: Problem, st: State, sp: SolveParams, tag: int):
        if tag in self._live:
            raise ValueError(f"tag {tag} is already in flight")
        req = Request(pb, ctypes.pointer(st), sp, tag)
        rc = self.lib.blr_server_submit(self.h, ctypes.byref(req))
        if rc != 0:
            msg = self.lib.blr_server_last_error(self.h)
            raise BlrError(rc, msg.decode() if msg else "")
        self._live[tag] = (pb, st, req)

    def wait(self, max_out: int = 64, timeout: float | None = None):
        """Completions finished since the last call (at least one unless the
        timeout passed or nothing is queued or running)."""
        buf = (Completion * max(1, max_out))()
        n = ctypes.c_int32()
        rc = self.lib.blr_server_wait(self.h, max_out, -1.0 if timeout is None else float(timeout),
                                      buf, ctypes.byref(n))
        if rc != 0:
            raise BlrError(rc, "blr_server_wait failed")
        out = [buf[i] for i in range(n.value)]
        for c in out:
            self._live.pop(c.tag, None)
        return out

    def load(self):
        q, r = ctypes.c_int64(), ctypes.c_int64()
        self.lib.blr_server_load(self.h, ctypes.byref(q), ctypes.byref(r))
        return q.value, r.value

    def clock(self) -> float:
        t = ctypes.c_double()
        self.lib.blr_server_clock(self.h, ctypes.byref(t))
        return t.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.blr_server_destroy(self.h)
            self.h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def upper_pairs(r: int):
    return [(i, j) for i in range(r) for j in range(i, r)]
