"""Python binding of libpgcp (ctypes): argument marshalling only.

Every stage runs inside the C-ABI library (host C++ for the partition and the
weld, HIP kernels on gfx950 for everything else).  PyTorch provides device
memory and the stream.  If the built library is missing, importing the
binding's entry points raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import time
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PGCP_LIB names another build of the same library (the host-sanitizer build
# libpgcp_asan.so in the sanitizer test)
LIB_PATH = os.environ.get("PGCP_LIB") or os.path.join(HERE, "libpgcp.so")

PGCP_FREE, PGCP_DISK, PGCP_SPHERE = 0, 1, 2
MODES = {"free": PGCP_FREE, "disk": PGCP_DISK, "sphere": PGCP_SPHERE}
PGCP_FP64, PGCP_FP32_REFINE = 0, 1
STATUS = {0: "OK", -1: "INVALID", -2: "TOPOLOGY", -3: "DEGENERATE", -4: "NOCONV", -5: "BREAKDOWN",
          -6: "WELD", -7: "HIP", -8: "NOMEM"}


class PGCPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pgcp {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("stall_iters", ctypes.c_int32), ("tol", ctypes.c_double), ("inner_tol", ctypes.c_double),
                ("precond", ctypes.c_int32), ("reserved", ctypes.c_int32), ("lpc", ctypes.c_void_p)]


class SolveStats(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("total_iters", ctypes.c_int64),
                ("iters", ctypes.POINTER(ctypes.c_int32)), ("relres", ctypes.POINTER(ctypes.c_double)),
                ("status", ctypes.POINTER(ctypes.c_int32)), ("seconds", ctypes.c_double),
                ("cg_kernel_ms", ctypes.c_double), ("cg_bytes", ctypes.c_double), ("cg_launches", ctypes.c_int32),
                ("rows_per_thread", ctypes.c_int32), ("cg_workgroups", ctypes.c_int32), ("cg_block", ctypes.c_int32),
                ("cg_stream", ctypes.c_int32), ("n_fallback", ctypes.c_int32), ("cg_single", ctypes.c_int32),
                ("cg_bytes_native", ctypes.c_double)]


class DistStats(ctypes.Structure):
    _fields_ = [("mean_abs_d", ctypes.c_double), ("sd_abs_d", ctypes.c_double), ("max_abs_d", ctypes.c_double),
                ("median_abs_d", ctypes.c_double), ("iqr_abs_d", ctypes.c_double), ("max_mu", ctypes.c_double),
                ("n_flipped", ctypes.c_int64), ("n_mu_ge1", ctypes.c_int64)]


class FoldStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("pieces_repaired", ctypes.c_int32), ("flips_before", ctypes.c_int64),
                ("flips_after", ctypes.c_int64), ("total_iters", ctypes.c_int64), ("cg_kernel_ms", ctypes.c_double),
                ("pieces_stopped", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PartInfo(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("nf", ctypes.c_int64), ("n_sub", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("n_rows", ctypes.c_int64), ("n_bdy", ctypes.c_int64), ("n_seam", ctypes.c_int64),
                ("nnz_offdiag", ctypes.c_int64), ("sell_elems", ctypes.c_int64), ("weld_rounds", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


EXPORTS = ["pgcp_ctx_create", "pgcp_ctx_destroy", "pgcp_last_error", "pgcp_ctx_set_stream", "pgcp_partition",
           "pgcp_part_query", "pgcp_part_export", "pgcp_part_destroy", "pgcp_laplacian_export",
           "pgcp_assemble_cotan", "pgcp_local_param", "pgcp_weld", "pgcp_harmonic_solve", "pgcp_distortion",
           "pgcp_lpc_num_params", "pgcp_lpc_create", "pgcp_lpc_get_params", "pgcp_lpc_destroy", "pgcp_lpc_infer",
           "pgcp_lpc_export", "pgcp_lpc_grad", "pgcp_lpc_train_step", "pgcp_part_rows",
           "pgcp_part_row_vertices", "pgcp_area_distortion", "pgcp_area_objective", "pgcp_area_mobius_opt",
           "pgcp_lpc_save", "pgcp_lpc_load", "pgcp_lpc_step", "pgcp_part_solution", "pgcp_distortion_noalloc",
           "pgcp_distortion_noalloc_max_faces", "pgcp_fold_repair"]
PGCP_PC_JACOBI, PGCP_PC_LEARNED = 0, 1
SYSTEMS = {"dncp": 0, "harmonic": 1}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpgcp.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libpgcp.so not built ({path}); run `python -m paper_1903_12359_amd.build`")
    # torch's HIP runtime must enumerate the devices before the library's first
    # HIP call: in the other order the library's runtime finds no device
    import torch
    torch.cuda.is_available()
    L = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "pgcp_ctx_create": (I32, [ctypes.POINTER(P), ctypes.c_int, P]),
        "pgcp_ctx_destroy": (None, [P]),
        "pgcp_last_error": (ctypes.c_char_p, [P]),
        "pgcp_ctx_set_stream": (I32, [P, P]),
        "pgcp_partition": (I32, [P, P, I64, P, I64, P, I32, ctypes.POINTER(P)]),
        "pgcp_part_query": (I32, [P, ctypes.POINTER(PartInfo)]),
        "pgcp_part_export": (I32, [P, P, P, P, P, P]),
        "pgcp_part_destroy": (None, [P]),
        "pgcp_laplacian_export": (I32, [P, P, I32, P, P, P]),
        "pgcp_assemble_cotan": (I32, [P, P, P]),
        "pgcp_local_param": (I32, [P, P, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveStats)]),
        "pgcp_weld": (I32, [P, P, P, P]),
        "pgcp_harmonic_solve": (I32, [P, P, P, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveStats)]),
        "pgcp_distortion": (I32, [P, P, I64, P, I64, P, I32, P, P, P, I32, ctypes.POINTER(DistStats)]),
        "pgcp_fold_repair": (I32, [P, P, P, P, P, D, I32, ctypes.POINTER(SolveOpts), ctypes.POINTER(FoldStats)]),
        "pgcp_distortion_noalloc": (I32, [P, P, I64, P, I64, P, I32, P, P, P, ctypes.POINTER(DistStats)]),
        "pgcp_distortion_noalloc_max_faces": (I64, []),
        "pgcp_lpc_save": (I32, [P, P, ctypes.c_char_p]),
        "pgcp_lpc_load": (I32, [P, ctypes.c_char_p, ctypes.POINTER(P)]),
        "pgcp_lpc_step": (I32, [P, ctypes.POINTER(I64)]),
        "pgcp_part_solution": (I32, [P, P, ctypes.POINTER(I32), P]),
        "pgcp_lpc_num_params": (I64, []),
        "pgcp_lpc_create": (I32, [P, P, ctypes.POINTER(P)]),
        "pgcp_lpc_get_params": (I32, [P, P, P]),
        "pgcp_lpc_destroy": (None, [P]),
        "pgcp_lpc_infer": (I32, [P, P, P, I32]),
        "pgcp_lpc_export": (I32, [P, P, I32, P, P, P, P]),
        "pgcp_lpc_grad": (I32, [P, P, P, I32, P, I32, ctypes.POINTER(D), P]),
        "pgcp_lpc_train_step": (I32, [P, P, P, I32, P, I32, ctypes.c_float, ctypes.POINTER(D)]),
        "pgcp_part_rows": (I32, [P, P]),
        "pgcp_part_row_vertices": (I32, [P, P]),
        "pgcp_area_distortion": (I32, [P, P, I64, P, I64, P, I32, P, P]),
        "pgcp_area_objective": (I32, [P, P, I64, P, I64, P, I32, I32, P, P]),
        "pgcp_area_mobius_opt": (I32, [P, P, I64, P, I64, P, I32, I32, I32, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _opts(precision="fp64", tol=1e-10, inner_tol=0.0, max_iter=0, max_refine=0, stall_iters=0, lpc=None):
    o = SolveOpts()
    o.stall_iters = stall_iters
    if lpc is not None:
        o.precond = PGCP_PC_LEARNED
        o.lpc = lpc.h
    o.precision = PGCP_FP32_REFINE if precision in ("fp32", "fp32_refine", PGCP_FP32_REFINE) else PGCP_FP64
    o.tol = tol
    o.inner_tol = inner_tol
    o.max_iter = max_iter
    o.max_refine = max_refine
    return o


@dataclass
class SolveReport:
    n_sub: int
    refine_steps: int
    total_iters: int
    iters: np.ndarray
    relres: np.ndarray
    status: np.ndarray
    seconds: float
    cg_kernel_ms: float = 0.0
    cg_bytes: float = 0.0
    cg_launches: int = 0
    rows_per_thread: int = 0
    cg_workgroups: int = 0
    cg_block: int = 0
    cg_stream: int = 0
    n_fallback: int = 0
    cg_single: int = 0
    cg_bytes_native: float = 0.0


class Context:
    """A libpgcp context bound to a device and torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.pgcp_ctx_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            msg = self.lib.pgcp_last_error(None)
            raise PGCPError(rc, "context creation failed: " + (msg.decode() if msg else ""))
        self.h = h

    def check(self, rc):
        if rc != 0:
            msg = self.lib.pgcp_last_error(self.h)
            raise PGCPError(rc, msg.decode() if msg else "")

    def close(self):
        for lc in getattr(self, "_lane_ctxs", []):
            lc.close()
        self._lane_ctxs = []
        if getattr(self, "h", None):
            self.lib.pgcp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HostOnly:
    """Stand-in context for host-only plans (partition and weld without a GPU)."""

    def __init__(self):
        self.lib = load_library()
        self.h = None

    def check(self, rc):
        if rc != 0:
            raise PGCPError(rc, "host-only call failed")


class Plan:
    """A partition plan (pgcp_part) built on the host and mirrored on the device.

    ctx=None builds a host-only plan (partition, export and weld only).
    """

    def __init__(self, ctx, V, F, label, mode="free"):
        if ctx is None:
            ctx = HostOnly()
        self.ctx = ctx
        V = np.ascontiguousarray(V, dtype=np.float64)
        F = np.ascontiguousarray(F, dtype=np.int32)
        label = np.ascontiguousarray(label, dtype=np.int32)
        self.mode = MODES[mode] if isinstance(mode, str) else int(mode)
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.pgcp_partition(ctx.h, _ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(label),
                                         self.mode, ctypes.byref(h)))
        self.h = h
        info = PartInfo()
        ctx.check(ctx.lib.pgcp_part_query(h, ctypes.byref(info)))
        self.info = info
        self.nv, self.nf, self.K = info.nv, info.nf, info.n_sub
        self.n_bdy, self.n_seam = info.n_bdy, info.n_seam

    def export(self):
        face_sub = np.empty(self.nf, np.int32)
        sub_nv = np.empty(self.K, np.int32)
        loop_ptr = np.empty(self.K + 1, np.int32)
        loop_gv = np.empty(self.n_bdy, np.int32)
        seam_gv = np.empty(self.n_seam, np.int32)
        self.ctx.check(self.ctx.lib.pgcp_part_export(self.h, _ptr(face_sub), _ptr(sub_nv), _ptr(loop_ptr),
                                                     _ptr(loop_gv), _ptr(seam_gv)))
        return dict(face_sub=face_sub, sub_nv=sub_nv, loop_ptr=loop_ptr, loop_gv=loop_gv, seam_gv=seam_gv)

    def laplacian(self, piece: int):
        """Assembled FP64 Laplacian of one piece as scipy CSR (local order)."""
        import scipy.sparse as sp
        n = int(self.export()["sub_nv"][piece])
        rowptr = np.empty(n + 1, np.int32)
        self.ctx.check(self.ctx.lib.pgcp_laplacian_export(self.ctx.h, self.h, piece, _ptr(rowptr), None, None))
        col = np.empty(rowptr[-1], np.int32)
        val = np.empty(rowptr[-1], np.float64)
        self.ctx.check(self.ctx.lib.pgcp_laplacian_export(self.ctx.h, self.h, piece, _ptr(rowptr), _ptr(col),
                                                          _ptr(val)))
        return sp.csr_matrix((val, col, rowptr), shape=(n, n))

    def rows(self):
        """Packed-row ranges of the pieces ([K+1]) and the total row count."""
        row0 = np.empty(self.K + 1, np.int64)
        self.ctx.check(self.ctx.lib.pgcp_part_rows(self.h, _ptr(row0)))
        return row0

    def row_vertices(self):
        """Global vertex of every packed row ([row0[K]]), -1 on padding rows."""
        gv = np.empty(int(self.rows()[-1]), np.int32)
        self.ctx.check(self.ctx.lib.pgcp_part_row_vertices(self.h, _ptr(gv)))
        return gv

    def solution(self, out=None):
        """Packed-row iterate of the last solve on this plan ([rows][2] float64
        on the device) and which system it was ("dncp" or "harmonic")."""
        import torch
        if out is None:
            out = torch.empty((int(self.rows()[-1]), 2), dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        sysv = ctypes.c_int32()
        self.ctx.check(self.ctx.lib.pgcp_part_solution(self.ctx.h, self.h, ctypes.byref(sysv), _ptr(out)))
        return out, ("dncp" if sysv.value == 0 else "harmonic")

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.pgcp_part_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



class LPC:
    """The learned SPAI preconditioner network (pgcp_lpc) on a context's device.

    LPC(ctx, params) starts from a parameter vector (None: all zeros, i.e.
    Jacobi); LPC.load(ctx, path) from a training-state file written by save()."""

    def __init__(self, ctx: Context, params: np.ndarray | None = None, _handle=None):
        self.ctx = ctx
        self.n_params = int(ctx.lib.pgcp_lpc_num_params())
        if _handle is not None:
            self.h = _handle
            return
        p = None
        if params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            if p.size != self.n_params:
                raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.pgcp_lpc_create(ctx.h, _ptr(p), ctypes.byref(h)))
        self.h = h

    @classmethod
    def load(cls, ctx: Context, path: str) -> "LPC":
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.pgcp_lpc_load(ctx.h, os.fsencode(path), ctypes.byref(h)))
        return cls(ctx, _handle=h)

    def save(self, path: str):
        """Parameters, Adam moments and step to `path` (pgcp_lpc_save)."""
        self.ctx.check(self.ctx.lib.pgcp_lpc_save(self.ctx.h, self.h, os.fsencode(path)))

    @property
    def step(self) -> int:
        v = ctypes.c_int64()
        self.ctx.check(self.ctx.lib.pgcp_lpc_step(self.h, ctypes.byref(v)))
        return int(v.value)

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        self.ctx.check(self.ctx.lib.pgcp_lpc_get_params(self.ctx.h, self.h, _ptr(out)))
        return out

    def infer(self, plan: Plan, system="harmonic"):
        self.ctx.check(self.ctx.lib.pgcp_lpc_infer(self.ctx.h, plan.h, self.h, SYSTEMS[system]))

    def export(self, plan: Plan, piece: int):
        """(o_off, o_diag, m_off, m_diag) of one piece after infer(), CSR order without the diagonal."""
        nv = int(plan.export()["sub_nv"][piece])
        L = plan.laplacian(piece)
        nnz = L.nnz - nv
        o_off, m_off = np.empty(nnz), np.empty(nnz)
        o_diag, m_diag = np.empty(nv), np.empty(nv)
        self.ctx.check(self.ctx.lib.pgcp_lpc_export(self.ctx.h, plan.h, piece, _ptr(o_off), _ptr(o_diag),
                                                    _ptr(m_off), _ptr(m_diag)))
        return o_off, o_diag, m_off, m_diag

    def grad(self, plan: Plan, probes_dev, system="harmonic"):
        loss = ctypes.c_double()
        g = np.empty(self.n_params, np.float32)
        self.ctx.check(self.ctx.lib.pgcp_lpc_grad(self.ctx.h, plan.h, self.h, SYSTEMS[system], _ptr(probes_dev),
                                                  int(probes_dev.shape[0]), ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def train_step(self, plan: Plan, probes_dev, lr: float, system="harmonic") -> float:
        loss = ctypes.c_double()
        self.ctx.check(self.ctx.lib.pgcp_lpc_train_step(self.ctx.h, plan.h, self.h, SYSTEMS[system],
                                                        _ptr(probes_dev), int(probes_dev.shape[0]), float(lr),
                                                        ctypes.byref(loss)))
        return loss.value

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.pgcp_lpc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stats_struct(K):
    st = SolveStats()
    it = np.zeros(K, np.int32)
    rr = np.zeros(2 * K, np.float64)
    ss = np.zeros(K, np.int32)
    st.iters = it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    st.relres = rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    st.status = ss.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    return st, (it, rr, ss)


def _report(st, keep):
    it, rr, ss = keep
    return SolveReport(st.n_sub, st.refine_steps, st.total_iters, it.copy(), rr.reshape(-1, 2).copy(),
                       ss.copy(), st.seconds, st.cg_kernel_ms, st.cg_bytes, st.cg_launches, st.rows_per_thread,
                       st.cg_workgroups, st.cg_block, st.cg_stream, st.n_fallback, st.cg_single,
                       st.cg_bytes_native)


def assemble_cotan(ctx: Context, plan: Plan, V_dev):
    ctx.check(ctx.lib.pgcp_assemble_cotan(ctx.h, plan.h, _ptr(V_dev)))


def local_param(ctx: Context, plan: Plan, out=None, stats=True, allow_noconv=False, **opts):
    import torch
    if out is None:
        out = torch.empty((plan.n_bdy, 2), dtype=torch.float64, device=f"cuda:{ctx.device}")
    o = _opts(**opts)
    rep = None
    if stats:
        st, keep = _stats_struct(plan.K)
        rc = ctx.lib.pgcp_local_param(ctx.h, plan.h, ctypes.byref(o), _ptr(out), ctypes.byref(st))
        rep = _report(st, keep)
    else:
        rc = ctx.lib.pgcp_local_param(ctx.h, plan.h, ctypes.byref(o), _ptr(out), None)
    if not (allow_noconv and rc == -4):
        ctx.check(rc)
    return out, rep


def weld(ctx, plan: Plan, bdy_host: np.ndarray, out=None):
    """Host weld; ctx may be None (host-only plans)."""
    if ctx is None:
        ctx = plan.ctx
    bdy_host = np.ascontiguousarray(bdy_host, dtype=np.float64)
    if out is None:
        out = np.empty((plan.n_seam, 2), np.float64)
    ctx.check(ctx.lib.pgcp_weld(ctx.h, plan.h, _ptr(bdy_host), _ptr(out)))
    return out


def harmonic_solve(ctx: Context, plan: Plan, welded_dev, out=None, stats=True, allow_noconv=False, **opts):
    import torch
    dim = 3 if plan.mode == PGCP_SPHERE else 2
    if out is None:
        out = torch.empty((plan.nv, dim), dtype=torch.float64, device=f"cuda:{ctx.device}")
    o = _opts(**opts)
    rep = None
    if stats:
        st, keep = _stats_struct(plan.K)
        rc = ctx.lib.pgcp_harmonic_solve(ctx.h, plan.h, _ptr(welded_dev), ctypes.byref(o), _ptr(out),
                                         ctypes.byref(st))
        rep = _report(st, keep)
    else:
        rc = ctx.lib.pgcp_harmonic_solve(ctx.h, plan.h, _ptr(welded_dev), ctypes.byref(o), _ptr(out), None)
    if not (allow_noconv and rc == -4):
        ctx.check(rc)
    return out, rep


def fold_repair(ctx: Context, plan: Plan, V_dev, F_dev, param_dev, delta=0.1, max_passes=5, **opts):
    """pgcp_fold_repair: quasi-conformal fold repair of a planar map in place;
    returns the report as a dict."""
    o = _opts(**opts)
    st = FoldStats()
    ctx.check(ctx.lib.pgcp_fold_repair(ctx.h, plan.h, _ptr(V_dev), _ptr(F_dev), _ptr(param_dev), float(delta),
                                       int(max_passes), ctypes.byref(o), ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in FoldStats._fields_}


def distortion(ctx: Context, V_dev, F_dev, param_dev, want_arrays=False, quantiles=False, stats=True):
    import torch
    nv, nf = V_dev.shape[0], F_dev.shape[0]
    dim = param_dev.shape[1]
    dev = f"cuda:{ctx.device}"
    d = mu = flip = None
    if want_arrays:
        d = torch.empty((nf, 3), dtype=torch.float64, device=dev)
        mu = torch.empty(nf, dtype=torch.float64, device=dev)
        flip = torch.empty(nf, dtype=torch.uint8, device=dev)
    st = DistStats()
    ctx.check(ctx.lib.pgcp_distortion(ctx.h, _ptr(V_dev), nv, _ptr(F_dev), nf, _ptr(param_dev), dim, _ptr(d),
                                      _ptr(mu), _ptr(flip), 1 if quantiles else 0,
                                      ctypes.byref(st) if stats else None))
    out = {k: getattr(st, k) for k, _ in DistStats._fields_} if stats else None
    return out, d, mu, flip


def distortion_noalloc(ctx: Context, V_dev, F_dev, param_dev, d=None, mu=None, flip=None, stats=True):
    """pgcp_distortion_noalloc: the distortion check without any allocation in
    the library (outputs d [nf][3], mu [nf], flip [nf] are the caller's, or None)."""
    nv, nf = V_dev.shape[0], F_dev.shape[0]
    st = DistStats()
    ctx.check(ctx.lib.pgcp_distortion_noalloc(ctx.h, _ptr(V_dev), nv, _ptr(F_dev), nf, _ptr(param_dev),
                                              param_dev.shape[1], _ptr(d), _ptr(mu), _ptr(flip),
                                              ctypes.byref(st) if stats else None))
    return {k: getattr(st, k) for k, _ in DistStats._fields_} if stats else None


def area_distortion(ctx: Context, V_dev, F_dev, param_dev, want_d=False):
    """Section 6: mean |d_area| of the parameterization (and d_area per face)."""
    import torch
    nf = F_dev.shape[0]
    d = torch.empty(nf, dtype=torch.float64, device=f"cuda:{ctx.device}") if want_d else None
    m = ctypes.c_double()
    ctx.check(ctx.lib.pgcp_area_distortion(ctx.h, _ptr(V_dev), V_dev.shape[0], _ptr(F_dev), nf, _ptr(param_dev),
                                           param_dev.shape[1], _ptr(d), ctypes.byref(m)))
    return m.value, d


def area_objective(ctx: Context, V_dev, F_dev, param_dev, mode, mobius):
    """Section 6: mean |d_area| of the parameterization composed with a Moebius map."""
    p = np.ascontiguousarray(mobius, dtype=np.float64)
    v = ctypes.c_double()
    ctx.check(ctx.lib.pgcp_area_objective(ctx.h, _ptr(V_dev), V_dev.shape[0], _ptr(F_dev), F_dev.shape[0],
                                          _ptr(param_dev), param_dev.shape[1], MODES[mode], _ptr(p),
                                          ctypes.byref(v)))
    return v.value


def area_mobius_opt(ctx: Context, V_dev, F_dev, param_dev, mode, max_evals=400, want_map=False):
    """Section 6: the Moebius map minimising mean |d_area| (Nelder-Mead on the device's objective).

    Returns (parameters, before, after, evaluations, composed map or None)."""
    import torch
    p = np.zeros(2 if mode == "disk" else 8, np.float64)
    b, a, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    Y = torch.empty_like(param_dev) if want_map else None
    ctx.check(ctx.lib.pgcp_area_mobius_opt(ctx.h, _ptr(V_dev), V_dev.shape[0], _ptr(F_dev), F_dev.shape[0],
                                           _ptr(param_dev), param_dev.shape[1], MODES[mode], int(max_evals),
                                           _ptr(p), ctypes.byref(b), ctypes.byref(a), ctypes.byref(n), _ptr(Y)))
    return p, b.value, a.value, n.value, Y


def run_stream(ctx: Context, cases, lanes: int = 1, **kw):
    """Algorithm 3 over a sequence of meshes, overlapping host and device work.

    `cases` is an iterable of dicts with keys V, F, label and optionally mode,
    V_dev, F_dev (the device copies must be complete before the call).  Every
    mesh goes through every stage; yields run()'s (phi_dev, dist_stats,
    reports) per mesh, in input order.  Remaining keyword arguments go to run().

    lanes=1: while the device runs the stages of one mesh, a worker thread
    partitions the next one on the host (pgcp_partition releases the
    interpreter lock; its plan upload is ordered on the context's stream).
    reports["times"]["partition"] is the time spent waiting for the prefetched
    plan and ["partition_overlapped"] the worker's partition time.

    lanes=n>1: n meshes are in flight.  A worker thread partitions meshes (up
    to n + 1 ahead) on a context of its own; each lane is a host thread with a
    context of its own on a stream of its own (all kept on `ctx` for later
    calls) that takes the next plan and runs the stages.  The library runs one
    batched-CG kernel at a time on a device (they take the whole device); the
    partition, a lane's weld and solve host steps, and its other kernels
    overlap the solves of the other lanes.  phi_dev is on the lane's stream,
    which has finished with it when it is yielded.  Batches that need the
    streaming CG kernel (pieces too large for the register kernel, e.g. the
    2048^2 field) have lost workgroups at the first barrier of a launch with
    several lanes in flight; the launch then gives up and the call raises
    PGCPError ("batched CG barrier timed out ..."); run them with lanes=1.
    """
    if lanes > 1:
        yield from _run_lanes(ctx, cases, lanes, kw)
        return
    from concurrent.futures import ThreadPoolExecutor

    def build(c):
        t = time.perf_counter()
        p = Plan(ctx, c["V"], c["F"], c["label"], c.get("mode", "free"))
        return p, time.perf_counter() - t

    it = iter(cases)
    with ThreadPoolExecutor(max_workers=1) as ex:
        nxt = next(it, None)
        fut = ex.submit(build, nxt) if nxt is not None else None
        while fut is not None:
            cur = nxt
            t = time.perf_counter()
            plan, t_build = fut.result()
            wait = time.perf_counter() - t
            nxt = next(it, None)
            fut = ex.submit(build, nxt) if nxt is not None else None
            times = {}
            try:
                out = run(ctx, cur["V"], cur["F"], cur["label"], cur.get("mode", "free"), V_dev=cur.get("V_dev"),
                          F_dev=cur.get("F_dev"), plan=plan, times=times, **kw)
            finally:
                plan.close()
            times["partition"] = wait
            times["partition_overlapped"] = t_build
            yield out


def _run_lanes(ctx: Context, cases, lanes: int, kw):
    import threading
    from collections import deque

    import torch
    from concurrent.futures import ThreadPoolExecutor
    pool = getattr(ctx, "_lane_ctxs", None)
    if pool is None:
        pool = ctx._lane_ctxs = []
    while len(pool) < lanes + 1:
        pool.append(Context(ctx.device, torch.cuda.Stream(ctx.device)))
    part_ctx = pool[lanes]            # the partition worker's context (plan uploads)
    free = list(pool[:lanes])
    free_lock = threading.Lock()
    torch.cuda.current_stream(ctx.device).synchronize()   # inputs made on the caller's stream

    def build(c):
        t = time.perf_counter()
        p = Plan(part_ctx, c["V"], c["F"], c["label"], c.get("mode", "free"))   # upload finished on return
        return p, time.perf_counter() - t

    def work(c, pf):
        with free_lock:
            lc = free.pop()
        try:
            t = time.perf_counter()
            plan, t_build = pf.result()
            wait = time.perf_counter() - t
            with torch.cuda.stream(lc.stream):
                times = {}
                try:
                    out = run(lc, c["V"], c["F"], c["label"], c.get("mode", "free"), V_dev=c.get("V_dev"),
                              F_dev=c.get("F_dev"), plan=plan, times=times, **kw)
                finally:
                    plan.close()
                times["partition"] = wait
                times["partition_overlapped"] = t_build
                return out
        finally:
            with free_lock:
                free.append(lc)

    it = iter(cases)
    plans, running = deque(), deque()
    with ThreadPoolExecutor(max_workers=1) as pex, ThreadPoolExecutor(max_workers=lanes) as lex:
        def fill():
            # partitions run up to lanes + 1 meshes ahead of the lanes
            while len(plans) + len(running) < 2 * lanes + 1:
                c = next(it, None)
                if c is None:
                    break
                plans.append((c, pex.submit(build, c)))
            while plans and len(running) < lanes:
                c, pf = plans.popleft()
                running.append(lex.submit(work, c, pf))

        try:
            fill()
            while running:
                out = running.popleft().result()
                fill()
                yield out
        finally:
            for _, pf in plans:   # plans built for meshes that were not run
                if pf.cancel():
                    continue
                try:
                    pf.result()[0].close()
                except Exception:
                    pass


def run(ctx: Context, V, F, label, mode="free", precision="fp64", tol=1e-10, inner_tol=0.0,
        V_dev=None, F_dev=None, quantiles=False, plan=None, times=None, dncp_precision="fp64", lpc=None,
        repair_folds=True):
    """Algorithm 3 end to end; returns (phi_dev, dist_stats, reports).

    V, F, label are host arrays (the partition runs on the host); V_dev/F_dev
    are their device copies (made here if not given).  `precision` is the
    inner-solve precision of the harmonic solve; the DNCP solve uses
    `dncp_precision` (FP64 by default: its free-boundary system has a
    near-null space that FP32 CG cannot resolve).  With `lpc` (an LPC) both
    solves use the learned sparse approximate inverse instead of Jacobi; the
    network runs on the device right before each solve (inside the timing).
    With repair_folds (planar modes), the harmonic maps then go through the
    quasi-conformal fold repair (pgcp_fold_repair), which costs one flip count
    when no face is flipped; its report is reports["fold"].
    """
    import torch
    dev = f"cuda:{ctx.device}"
    if times is None:
        times = {}
    sync = ctx.stream.synchronize
    t = time.perf_counter()
    if V_dev is None:
        V_dev = torch.from_numpy(np.ascontiguousarray(V, np.float64)).to(dev)
    if F_dev is None:
        F_dev = torch.from_numpy(np.ascontiguousarray(F, np.int32)).to(dev)
    own_plan = plan is None
    if plan is None:
        plan = Plan(ctx, V, F, label, mode)
    times["partition"] = time.perf_counter() - t
    t = time.perf_counter()
    assemble_cotan(ctx, plan, V_dev)
    bdy, rep1 = local_param(ctx, plan, precision=dncp_precision, tol=tol, inner_tol=inner_tol, lpc=lpc)
    bdy_h = bdy.cpu().numpy()
    times["assemble+dncp"] = time.perf_counter() - t
    t = time.perf_counter()
    welded = weld(ctx, plan, bdy_h)
    times["weld"] = time.perf_counter() - t
    t = time.perf_counter()
    welded_dev = torch.from_numpy(welded).to(dev)
    phi, rep2 = harmonic_solve(ctx, plan, welded_dev, precision=precision, tol=tol, inner_tol=inner_tol,
                               lpc=lpc)
    sync()
    times["harmonic"] = time.perf_counter() - t
    fold = None
    if repair_folds and plan.mode != PGCP_SPHERE:
        t = time.perf_counter()
        fold = fold_repair(ctx, plan, V_dev, F_dev, phi, precision=precision, tol=tol, inner_tol=inner_tol)
        times["fold_repair"] = time.perf_counter() - t
    t = time.perf_counter()
    st, _, _, _ = distortion(ctx, V_dev, F_dev, phi, quantiles=quantiles)
    times["distortion"] = time.perf_counter() - t
    if own_plan:
        plan.close()
    return phi, st, dict(dncp=rep1, harmonic=rep2, times=times, bdy=bdy_h, welded=welded, fold=fold)
