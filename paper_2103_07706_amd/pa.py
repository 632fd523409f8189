"""ctypes binding of libpa.so (C ABI in include/pa.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory (tensors) and the stream.  A missing
library is an error; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpa.so")

PA_FP64, PA_FP32_REFINED = 0, 1
PA_BACKWARD_PER_TERM, PA_BACKWARD_CLENSHAW = 0, 1
PA_SOLVER_CG, PA_SOLVER_CHEBYSHEV = 0, 1
PA_EXP_CHEBYSHEV, PA_EXP_REXI = 0, 1
PA_BDM2_APPLY_L, PA_BDM2_EXPL, PA_BDM2_NONLINEAR, PA_BDM2_PHASE_AVG, PA_BDM2_STEP = range(5)
PA_OK, PA_EINVAL, PA_ENOMEM, PA_EHIP, PA_ENOCONV, PA_ENOTSUP, PA_EGROWTH = range(7)
_STATUS = {0: "PA_OK", 1: "PA_EINVAL", 2: "PA_ENOMEM", 3: "PA_EHIP", 4: "PA_ENOCONV",
           5: "PA_ENOTSUP", 6: "PA_EGROWTH"}


class PAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class MeshInfo(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("nv", ctypes.c_int32), ("ne", ctypes.c_int32),
                ("nc", ctypes.c_int32), ("radius", ctypes.c_double)]


class Phys(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("H", ctypes.c_double), ("omega", ctypes.c_double),
                ("b_cell", ctypes.POINTER(ctypes.c_double)), ("lambda_bar", ctypes.c_double)]


class SolveCfg(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("backward", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("growth_guard", ctypes.c_int32),
                ("cg_rtol", ctypes.c_double), ("cheb_tol", ctypes.c_double),
                ("weight_cut", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("solver", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("exponential", ctypes.c_int32),
                ("rexi_nodes", ctypes.c_int32), ("rexi_eta0", ctypes.c_double)]


PA_PRECOND_JACOBI, PA_PRECOND_LEARNED = 0, 1
PA_KERNEL_NONE, PA_KERNEL_CG_ITER, PA_KERNEL_CHEB_ITER, PA_KERNEL_CHEB_LP_ITER = 0, 1, 2, 3
PA_KERNEL_CHEB_FUSED = 4
PA_KERNEL_CHEB3_ITER = 5
PA_KERNEL_CHEB32_ITER = 6
PA_KERNEL_B2_STEP = 7


class TrainCfg(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("probes", ctypes.c_int32), ("lr", ctypes.c_double),
                ("bf16", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class TrainStats(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("ms", ctypes.c_double), ("steps", ctypes.c_int32)]


class LpInfo(ctypes.Structure):
    _fields_ = [("eig_min", ctypes.c_double), ("eig_max", ctypes.c_double),
                ("jacobi_eig_min", ctypes.c_double), ("jacobi_eig_max", ctypes.c_double),
                ("width_p", ctypes.c_int32), ("width_pm", ctypes.c_int32)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("work_launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("units", ctypes.c_double)]


class LaunchTune(ctypes.Structure):
    _fields_ = [("narrow_rows_per_thread", ctypes.c_int32), ("wide_max_wg", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("lp_min_cols", ctypes.c_int32),
                ("mixed_min_cols", ctypes.c_int32), ("fused_steps", ctypes.c_int32)]


TUNE_FIELDS = ("narrow_rows_per_thread", "wide_max_wg", "lp_min_cols", "mixed_min_cols",
               "fused_steps")
TUNE_DEFAULTS = {"lp_min_cols": 8, "mixed_min_cols": 8, "fused_steps": 6}


def _tune_dict(t) -> dict:
    return {k: getattr(t, k) for k in TUNE_FIELDS}


def _tune_struct(d) -> "LaunchTune":
    t = LaunchTune()
    for k in TUNE_FIELDS:
        setattr(t, k, d[k] if k in d else TUNE_DEFAULTS[k])
    return t


class Stats(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("cg_iters_max", ctypes.c_int32), ("kmax", ctypes.c_int32),
                ("ksum", ctypes.c_int32), ("terms", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("guard_trips", ctypes.c_int32),
                ("resid_max", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("graph", ctypes.c_int32), ("budget", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("lp_solves", ctypes.c_int32),
                ("fallbacks", ctypes.c_int32), ("graph_captured", ctypes.c_int32),
                ("rexi_nodes", ctypes.c_int32), ("rexi_solves", ctypes.c_int32),
                ("rexi_iters", ctypes.c_int32), ("rexi_iters_max", ctypes.c_int32),
                ("rexi_restarts", ctypes.c_int32), ("rexi_pad", ctypes.c_int32),
                ("rexi_eta0", ctypes.c_double), ("rexi_resid_max", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
_V = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)
_SZ = ctypes.c_size_t

EXPORTS = {
    "pa_last_error": (ctypes.c_char_p, []),
    "pa_ctx_create": (ctypes.c_int, [ctypes.c_int, _V, ctypes.POINTER(_V)]),
    "pa_ctx_set_stream": (ctypes.c_int, [_V, _V]),
    "pa_ctx_destroy": (ctypes.c_int, [_V]),
    "pa_ctx_profile": (ctypes.c_int, [_V, ctypes.c_int]),
    "pa_ctx_profile_read": (ctypes.c_int, [_V, ctypes.POINTER(KernelProfile)]),
    "pa_ctx_set_cg_budget": (ctypes.c_int, [_V, ctypes.c_double, ctypes.c_int]),
    "pa_mesh_icosahedral": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.POINTER(_V)]),
    "pa_mesh_get_info": (ctypes.c_int, [_V, ctypes.POINTER(MeshInfo)]),
    "pa_mesh_export": (ctypes.c_int, [_V, _D, _I, _I, _I, _I]),
    "pa_mesh_destroy": (ctypes.c_int, [_V]),
    "pa_mesh_from_arrays": (ctypes.c_int, [ctypes.c_int, _D, ctypes.c_int, _I, ctypes.c_int, _I, _I,
                                           _I, ctypes.c_double, ctypes.POINTER(_V)]),
    "pa_bdm2_create": (ctypes.c_int, [_V, ctypes.POINTER(Phys), ctypes.POINTER(_V)]),
    "pa_bdm2_info": (ctypes.c_int, [_V, _I, _I, _D, _D]),
    "pa_bdm2_tables": (ctypes.c_int, [_V, _I, _D, _D, _I, _D, _I, _D]),
    "pa_bdm2_device_size": (ctypes.c_int, [_V, ctypes.POINTER(_SZ)]),
    "pa_bdm2_bind": (ctypes.c_int, [_V, _V, _V]),
    "pa_bdm2_set_lambda": (ctypes.c_int, [_V, ctypes.c_double]),
    "pa_bdm2_set_bottom": (ctypes.c_int, [_V, _D]),
    "pa_bdm2_estimate_lambda": (ctypes.c_int, [_V, _V, ctypes.c_int, ctypes.c_double, _V, _SZ,
                                               _D]),
    "pa_bdm2_workspace_size": (ctypes.c_int, [_V, ctypes.c_int, ctypes.c_int, _D, _V,
                                              ctypes.POINTER(SolveCfg), ctypes.POINTER(_SZ)]),
    "pa_bdm2_nonlinear": (ctypes.c_int, [_V, _V, ctypes.c_int, _V, _V, _V, _SZ,
                                         ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_bdm2_phase_avg_rhs": (ctypes.c_int, [_V, _V, _V, ctypes.c_int, _V, _V, _V, _SZ,
                                             ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_bdm2_apply_L": (ctypes.c_int, [_V, _V, ctypes.c_int, _V, _V, _V, _SZ,
                                       ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_bdm2_expL_apply": (ctypes.c_int, [_V, _V, ctypes.c_int, _D, _V, _V, _V, _SZ,
                                          ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_bdm2_step": (ctypes.c_int, [_V, _V, _V, ctypes.c_double, ctypes.c_int, _V, _V, _SZ,
                                    ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_bdm2_destroy": (ctypes.c_int, [_V]),
    "pa_ops_create": (ctypes.c_int, [_V, ctypes.POINTER(Phys), ctypes.POINTER(_V)]),
    "pa_ops_device_size": (ctypes.c_int, [_V, ctypes.POINTER(_SZ)]),
    "pa_ops_bind": (ctypes.c_int, [_V, _V, _V]),
    "pa_ops_estimate_lambda": (ctypes.c_int, [_V, _V, ctypes.c_int, ctypes.c_double, _V, _SZ,
                                              _D]),
    "pa_ops_set_lambda": (ctypes.c_int, [_V, ctypes.c_double]),
    "pa_ops_get_lambda": (ctypes.c_int, [_V, _D]),
    "pa_ops_destroy": (ctypes.c_int, [_V]),
    "pa_avg_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.POINTER(_V)]),
    "pa_avg_create_nodes": (ctypes.c_int, [ctypes.c_int, _D, _D, ctypes.POINTER(_V)]),
    "pa_avg_nodes": (ctypes.c_int, [_V, _D, _D]),
    "pa_avg_destroy": (ctypes.c_int, [_V]),
    "pa_solve_cfg_default": (None, [ctypes.POINTER(SolveCfg)]),
    "pa_workspace_size": (ctypes.c_int, [_V, _V, ctypes.c_int, ctypes.POINTER(SolveCfg),
                                         ctypes.POINTER(_SZ)]),
    "pa_expL_apply": (ctypes.c_int, [_V, _V, ctypes.c_int, _D, _V, _V, _V, _SZ,
                                     ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_swe_nonlinear": (ctypes.c_int, [_V, _V, ctypes.c_int, _V, _V, _V, _SZ,
                                        ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_phase_avg_rhs": (ctypes.c_int, [_V, _V, _V, ctypes.c_int, _V, _V, _V, _SZ,
                                        ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_step": (ctypes.c_int, [_V, _V, _V, ctypes.c_double, ctypes.c_int, _V, _V, _SZ,
                               ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_diagnostics": (ctypes.c_int, [_V, _V, ctypes.c_int, _V, _V, _SZ, _D]),
    "pa_get_launch_tune": (ctypes.c_int, [ctypes.POINTER(LaunchTune)]),
    "pa_set_launch_tune": (ctypes.c_int, [ctypes.POINTER(LaunchTune)]),
    "pa_phase_avg_rhs_noalloc": (ctypes.c_int, [_V, _V, _V, ctypes.c_int, _V, _V,
                                                ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_ops_set_tune": (ctypes.c_int, [_V, ctypes.POINTER(LaunchTune)]),
    "pa_ops_get_tune": (ctypes.c_int, [_V, ctypes.POINTER(LaunchTune), ctypes.POINTER(ctypes.c_int)]),
    "pa_autotune": (ctypes.c_int, [_V, _V, _V, ctypes.c_int, _V, _V, _V, _SZ,
                                   ctypes.POINTER(SolveCfg), ctypes.POINTER(LaunchTune)]),
    "pa_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_V), _I, _V,
                                       ctypes.POINTER(_V)]),
    "pa_batch_workspace_size": (ctypes.c_int, [_V, ctypes.POINTER(SolveCfg), ctypes.POINTER(_SZ)]),
    "pa_batch_run": (ctypes.c_int, [_V, _V, ctypes.POINTER(_V), ctypes.POINTER(_V), _V, _SZ,
                                    ctypes.POINTER(SolveCfg), ctypes.POINTER(Stats)]),
    "pa_batch_set_tune": (ctypes.c_int, [_V, ctypes.c_int, ctypes.POINTER(LaunchTune)]),
    "pa_batch_get_tune": (ctypes.c_int, [_V, ctypes.c_int, ctypes.POINTER(LaunchTune)]),
    "pa_batch_autotune": (ctypes.c_int, [_V, _V, ctypes.POINTER(_V), ctypes.POINTER(_V), _V, _SZ,
                                         ctypes.POINTER(SolveCfg), ctypes.POINTER(LaunchTune)]),
    "pa_batch_destroy": (ctypes.c_int, [_V]),
    "pa_lp_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                    ctypes.POINTER(_V)]),
    "pa_lp_param_count": (ctypes.c_int, [_V, ctypes.POINTER(ctypes.c_int)]),
    "pa_lp_get_params": (ctypes.c_int, [_V, ctypes.POINTER(ctypes.c_float)]),
    "pa_lp_set_params": (ctypes.c_int, [_V, ctypes.POINTER(ctypes.c_float)]),
    "pa_lp_save": (ctypes.c_int, [_V, ctypes.c_char_p]),
    "pa_lp_load": (ctypes.c_int, [_V, ctypes.c_char_p]),
    "pa_lp_destroy": (ctypes.c_int, [_V]),
    "pa_lp_workspace_size": (ctypes.c_int, [ctypes.POINTER(_V), ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.POINTER(_SZ)]),
    "pa_lp_train": (ctypes.c_int, [_V, _V, ctypes.POINTER(_V), ctypes.c_int,
                                   ctypes.POINTER(TrainCfg), _V, _SZ, ctypes.POINTER(TrainStats)]),
    "pa_lp_loss_grad": (ctypes.c_int, [_V, _V, _V, ctypes.c_int, _D, ctypes.c_int, _V, _SZ, _D,
                                       _D]),
    "pa_lp_ghat": (ctypes.c_int, [_V, _V, _V, ctypes.c_int, _V, _SZ, _D, _D]),
    "pa_ops_lp_attach": (ctypes.c_int, [_V, _V, _V, ctypes.c_int, _V, _SZ,
                                        ctypes.POINTER(LpInfo)]),
    "pa_ops_lp_device_size": (ctypes.c_int, [_V, ctypes.POINTER(_SZ)]),
    "pa_ops_lp_bind": (ctypes.c_int, [_V, _V, _V]),
}


def lib():
    """Open libpa.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        # Share PyTorch's HIP runtime: initialise it before the library binds
        # libamdhip64, so that one runtime serves both (on a machine without a
        # GPU only the host-side entry points are usable).
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise PAError(code, lib().pa_last_error().decode())


def _ptr(t):
    """Device pointer of a torch tensor."""
    return ctypes.c_void_p(t.data_ptr())


def _dp(a):
    return a.ctypes.data_as(_D)


def get_launch_tune() -> dict:
    """Process-wide launch shape (pa_get_launch_tune)."""
    t = LaunchTune()
    _check(lib().pa_get_launch_tune(ctypes.byref(t)))
    return _tune_dict(t)


def set_launch_tune(**changes):
    """Change fields of the process-wide launch shape (pa_set_launch_tune)."""
    cur = get_launch_tune()
    cur.update(changes)
    _check(lib().pa_set_launch_tune(ctypes.byref(_tune_struct(cur))))


def solve_cfg(precision=None, backward=None, maxit=None, cg_rtol=None, cheb_tol=None,
              weight_cut=None, inner_rtol=None, use_graph=None, solver=None, precond=None,
              growth_guard=None, exponential=None, rexi_nodes=None,
              rexi_eta0=None) -> SolveCfg:
    """A solve configuration: the library's defaults (pa_solve_cfg_default:
    FP64, Chebyshev exponential, Clenshaw backward sum, Chebyshev mass
    solves, graph replay, Jacobi preconditioning, cg_rtol 1e-10, Chebyshev
    threshold 1e-6) with the given fields changed."""
    c = SolveCfg()
    lib().pa_solve_cfg_default(ctypes.byref(c))
    for name, v in (("precision", precision), ("backward", backward), ("maxit", maxit),
                    ("cg_rtol", cg_rtol), ("cheb_tol", cheb_tol), ("weight_cut", weight_cut),
                    ("inner_rtol", inner_rtol), ("solver", solver), ("precond", precond),
                    ("growth_guard", growth_guard), ("exponential", exponential),
                    ("rexi_nodes", rexi_nodes), ("rexi_eta0", rexi_eta0)):
        if v is not None:
            setattr(c, name, v)
    if use_graph is not None:
        c.use_graph = 1 if use_graph else 0
    return c


class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = _V()
        _check(lib().pa_ctx_create(device, _V(stream), ctypes.byref(h)))
        self._h = h

    def profile(self, kernel: int):
        """Start timing every launch of one kernel (PA_KERNEL_NONE: off)."""
        _check(lib().pa_ctx_profile(self._h, kernel))

    def set_cg_budget(self, cg_rtol: float, iters: int):
        _check(lib().pa_ctx_set_cg_budget(self._h, cg_rtol, iters))

    def profile_read(self):
        p = KernelProfile()
        _check(lib().pa_ctx_profile_read(self._h, ctypes.byref(p)))
        return {f: getattr(p, f) for f, _ in p._fields_}

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pa_ctx_destroy(self._h)
            self._h = None


class Mesh:
    """Icosahedral mesh (host)."""

    def __init__(self, level: int, radius: float = 6.37122e6, _handle=None):
        h = _V()
        if _handle is None:
            _check(lib().pa_mesh_icosahedral(level, radius, ctypes.byref(h)))
        else:
            h = _handle
        self._h = h
        info = MeshInfo()
        _check(lib().pa_mesh_get_info(h, ctypes.byref(info)))
        self.level, self.nv, self.ne, self.nc = info.level, info.nv, info.ne, info.nc
        self.radius = info.radius
        self.verts = np.zeros((self.nv, 3))
        self.cell_verts = np.zeros((self.nc, 3), np.int32)
        self.cell_edges = np.zeros((self.nc, 3), np.int32)
        self.edge_cells = np.zeros((self.ne, 2), np.int32)
        self.edge_verts = np.zeros((self.ne, 2), np.int32)
        _check(lib().pa_mesh_export(h, _dp(self.verts), self.cell_verts.ctypes.data_as(_I),
                                    self.cell_edges.ctypes.data_as(_I),
                                    self.edge_cells.ctypes.data_as(_I),
                                    self.edge_verts.ctypes.data_as(_I)))

    @classmethod
    def from_arrays(cls, verts, cell_verts, cell_edges, edge_cells, edge_verts,
                    radius: float = 6.37122e6):
        """pa_mesh_from_arrays: a mesh from host arrays in the layout of
        pa_mesh_export (checked against the library's mesh conventions)."""
        v = np.ascontiguousarray(verts, np.float64)
        cv, ce, ec, ev = (np.ascontiguousarray(a, np.int32)
                          for a in (cell_verts, cell_edges, edge_cells, edge_verts))
        h = _V()
        _check(lib().pa_mesh_from_arrays(len(v), _dp(v), len(cv), cv.ctypes.data_as(_I), len(ec),
                                         ce.ctypes.data_as(_I), ec.ctypes.data_as(_I),
                                         ev.ctypes.data_as(_I), radius, ctypes.byref(h)))
        return cls(-1, radius, _handle=h)

    @property
    def n(self):
        return self.ne + self.nc

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pa_mesh_destroy(self._h)
            self._h = None


class Avg:
    """Averaging nodes and weights (Sec. 2.2)."""

    def __init__(self, M: int = None, T: float = None, s=None, w=None):
        h = _V()
        if s is not None:
            s = np.ascontiguousarray(s, np.float64)
            w = np.ascontiguousarray(w, np.float64)
            _check(lib().pa_avg_create_nodes(len(s), _dp(s), _dp(w), ctypes.byref(h)))
            M = len(s)
        else:
            _check(lib().pa_avg_create(M, T, ctypes.byref(h)))
        self._h = h
        self.M = M
        self.T = T  # None for explicit nodes
        self.s = np.zeros(M)
        self.w = np.zeros(M)
        _check(lib().pa_avg_nodes(h, _dp(self.s), _dp(self.w)))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pa_avg_destroy(self._h)
            self._h = None


class Ops:
    """Operators bound to a device buffer, with a workspace cache."""

    def __init__(self, ctx: Context, mesh: Mesh, g=9.80616, H=1000.0, omega=7.292e-5, b=None,
                 lambda_bar=0.0):
        import torch
        self.ctx, self.mesh = ctx, mesh
        self.g, self.H, self.omega = g, H, omega
        self._b = None if b is None else np.ascontiguousarray(b, np.float64)
        ph = Phys(g, H, omega, None if self._b is None else _dp(self._b), lambda_bar)
        h = _V()
        _check(lib().pa_ops_create(mesh._h, ctypes.byref(ph), ctypes.byref(h)))
        self._h = h
        self._ws = None
        self.rebind()

    def rebind(self):
        """Upload the operators into a newly allocated device buffer
        (pa_ops_bind); the previous buffer may then be freed."""
        import torch
        sz = _SZ()
        _check(lib().pa_ops_device_size(self._h, ctypes.byref(sz)))
        buf = torch.empty(sz.value + 256, dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        base = buf.data_ptr()
        off = (-base) % 256
        _check(lib().pa_ops_bind(self.ctx._h, self._h, _V(base + off)))
        self._buf = buf

    @property
    def n(self):
        return self.mesh.n

    @property
    def lambda_bar(self):
        v = ctypes.c_double()
        _check(lib().pa_ops_get_lambda(self._h, ctypes.byref(v)))
        return v.value

    @lambda_bar.setter
    def lambda_bar(self, value):
        _check(lib().pa_ops_set_lambda(self._h, float(value)))

    def workspace(self, avg=None, batch=1, cfg=None):
        import torch
        cfg = cfg or solve_cfg()
        sz = _SZ()
        _check(lib().pa_workspace_size(self._h, None if avg is None else avg._h, batch,
                                       ctypes.byref(cfg), ctypes.byref(sz)))
        if self._ws is None or self._ws.numel() < sz.value + 256:
            self._ws = None
            self._ws = torch.empty(sz.value + 256, dtype=torch.uint8,
                                   device=f"cuda:{self.ctx.device}")
        base = self._ws.data_ptr()
        off = (-base) % 256
        return _V(base + off), self._ws.numel() - off

    def estimate_lambda(self, iters=200, safety=1.05):
        ws, nb = self.workspace()
        v = ctypes.c_double()
        _check(lib().pa_ops_estimate_lambda(self.ctx._h, self._h, iters, safety, ws, nb,
                                            ctypes.byref(v)))
        return v.value

    # ---- the hot path -------------------------------------------------------
    def expL_apply(self, t, U, cfg=None, out=None):
        cfg = cfg or solve_cfg()
        B = U.shape[0]
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, np.float64), (B,)))
        out = U.new_empty(U.shape) if out is None else out
        ws, nb = self.workspace(None, B, cfg)
        st = Stats()
        _check(lib().pa_expL_apply(self.ctx._h, self._h, B, _dp(t), _ptr(U), _ptr(out), ws, nb,
                                   ctypes.byref(cfg), ctypes.byref(st)))
        return out, st.as_dict()

    def swe_nonlinear(self, U, cfg=None, out=None):
        cfg = cfg or solve_cfg()
        B = U.shape[0]
        out = U.new_empty(U.shape) if out is None else out
        ws, nb = self.workspace(None, B, cfg)
        st = Stats()
        _check(lib().pa_swe_nonlinear(self.ctx._h, self._h, B, _ptr(U), _ptr(out), ws, nb,
                                      ctypes.byref(cfg), ctypes.byref(st)))
        return out, st.as_dict()

    def phase_avg_rhs(self, avg: Avg, U, cfg=None, out=None):
        cfg = cfg or solve_cfg()
        members = U.shape[0]
        out = U.new_empty(U.shape) if out is None else out
        ws, nb = self.workspace(avg, members, cfg)
        st = Stats()
        _check(lib().pa_phase_avg_rhs(self.ctx._h, self._h, avg._h, members, _ptr(U), _ptr(out),
                                      ws, nb, ctypes.byref(cfg), ctypes.byref(st)))
        return out, st.as_dict()

    def phase_avg_rhs_noalloc(self, avg: Avg, U, cfg=None, out=None):
        """pa_phase_avg_rhs_noalloc: the library's static device scratch
        instead of a workspace (no device allocation by the call)."""
        cfg = cfg or solve_cfg()
        out = U.new_empty(U.shape) if out is None else out
        st = Stats()
        _check(lib().pa_phase_avg_rhs_noalloc(self.ctx._h, self._h, avg._h, U.shape[0], _ptr(U),
                                              _ptr(out), ctypes.byref(cfg), ctypes.byref(st)))
        return out, st.as_dict()

    def step(self, avg: Avg, dt: float, U, cfg=None):
        cfg = cfg or solve_cfg()
        members = U.shape[0]
        ws, nb = self.workspace(avg, members, cfg)
        st = Stats()
        _check(lib().pa_step(self.ctx._h, self._h, avg._h, dt, members, _ptr(U), ws, nb,
                             ctypes.byref(cfg), ctypes.byref(st)))
        return U, st.as_dict()

    def autotune(self, avg: Avg, U, cfg=None, cache=None):
        """Pick the launch shape for this problem (pa_autotune).  With a
        cache file (JSON), a shape stored for the same problem key is applied
        instead of searching, and a new search result is stored."""
        import json
        cfg = cfg or solve_cfg()
        members = U.shape[0]
        key = (f"level{self.mesh.level}_members{members}_M{avg.M}_rtol{cfg.cg_rtol:g}_"
               f"tol{cfg.cheb_tol:g}_bw{cfg.backward}_prec{cfg.precision}_graph{cfg.use_graph}_"
               f"solver{cfg.solver}_precond{cfg.precond}")
        table = {}
        if cache and os.path.exists(cache):
            table = json.load(open(cache))
            if key in table:
                self.set_tune(**{k: table[key][k] for k in TUNE_FIELDS})
                return dict(table[key], cached=True)
        out = U.new_empty(U.shape)
        ws, nb = self.workspace(avg, members, cfg)
        t = LaunchTune()
        _check(lib().pa_autotune(self.ctx._h, self._h, avg._h, members, _ptr(U), _ptr(out), ws,
                                 nb, ctypes.byref(cfg), ctypes.byref(t)))
        res = dict(_tune_dict(t), best_ms=t.best_ms)
        if cache:
            table[key] = res
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return dict(res, cached=False)

    def set_tune(self, **fields):
        """Give these operators their own launch shape (pa_ops_set_tune):
        the fields given, the others from the shape in use now.  With no
        fields, drop the own shape (calls take the process default)."""
        if not fields:
            _check(lib().pa_ops_set_tune(self._h, None))
            return
        cur = self.get_tune()
        cur.update(fields)
        _check(lib().pa_ops_set_tune(self._h, ctypes.byref(_tune_struct(cur))))

    def get_tune(self):
        """The launch shape calls on these operators use (pa_ops_get_tune)."""
        t = LaunchTune()
        own = ctypes.c_int()
        _check(lib().pa_ops_get_tune(self._h, ctypes.byref(t), ctypes.byref(own)))
        return _tune_dict(t)

    def has_own_tune(self):
        t = LaunchTune()
        own = ctypes.c_int()
        _check(lib().pa_ops_get_tune(self._h, ctypes.byref(t), ctypes.byref(own)))
        return bool(own.value)

    def diagnostics(self, U):
        B = U.shape[0]
        ws, nb = self.workspace(None, B)
        out = np.zeros(5 * B)
        _check(lib().pa_diagnostics(self.ctx._h, self._h, B, _ptr(U), ws, nb, _dp(out)))
        return out.reshape(B, 5)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pa_ops_destroy(self._h)
            self._h = None


class BDM2:
    """The BDM2 x P1DG linear operator and its Chebyshev exponential
    (pa_bdm2_*).  Assembled on the host at construction; bind(ctx) uploads
    the tables before the device calls."""

    def __init__(self, mesh: Mesh, g=9.80616, H=1000.0, omega=7.292e-5, lambda_bar=0.0):
        self.mesh = mesh
        ph = Phys(g, H, omega, None, lambda_bar)
        h = _V()
        _check(lib().pa_bdm2_create(mesh._h, ctypes.byref(ph), ctypes.byref(h)))
        self._h = h
        nu, nh = ctypes.c_int32(), ctypes.c_int32()
        lo, hi = ctypes.c_double(), ctypes.c_double()
        _check(lib().pa_bdm2_info(h, ctypes.byref(nu), ctypes.byref(nh), ctypes.byref(lo),
                                  ctypes.byref(hi)))
        self.nu, self.nh = nu.value, nh.value
        self.n = self.nu + self.nh
        self.eig_bounds = (lo.value, hi.value)
        self.ctx = None
        self._buf = None
        self._ws = None

    def tables(self):
        nu, nc = self.nu, self.mesh.nc
        t = dict(col=np.zeros(21 * nu, np.int32), mass=np.zeros(21 * nu), cor=np.zeros(21 * nu),
                 bcol=np.zeros(6 * nu, np.int32), bval=np.zeros(6 * nu),
                 cdof=np.zeros(12 * nc, np.int32), q=np.zeros(36 * nc))
        ip = lambda a: a.ctypes.data_as(_I)  # noqa: E731
        _check(lib().pa_bdm2_tables(self._h, ip(t["col"]), _dp(t["mass"]), _dp(t["cor"]),
                                    ip(t["bcol"]), _dp(t["bval"]), ip(t["cdof"]), _dp(t["q"])))
        return t

    def bind(self, ctx: Context):
        import torch
        sz = _SZ()
        _check(lib().pa_bdm2_device_size(self._h, ctypes.byref(sz)))
        buf = torch.empty(sz.value + 256, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        base = buf.data_ptr()
        _check(lib().pa_bdm2_bind(ctx._h, self._h, _V(base + (-base) % 256)))
        self.ctx, self._buf = ctx, buf
        return self

    def set_lambda(self, lambda_bar):
        _check(lib().pa_bdm2_set_lambda(self._h, float(lambda_bar)))

    def set_bottom(self, b):
        """pa_bdm2_set_bottom (before bind): P1DG bottom heights, or None."""
        if b is None:
            _check(lib().pa_bdm2_set_bottom(self._h, None))
            return self
        self._bot = np.ascontiguousarray(b, np.float64)
        if self._bot.shape != (self.nh,):
            raise ValueError("bottom needs nh values")
        _check(lib().pa_bdm2_set_bottom(self._h, _dp(self._bot)))
        return self

    def estimate_lambda(self, iters=200, safety=1.05):
        """pa_bdm2_estimate_lambda: sets and returns lambda_bar."""
        cfg = solve_cfg(cg_rtol=1e-12)
        ws, nb = self._workspace(PA_BDM2_APPLY_L, 1, None, cfg)
        v = ctypes.c_double()
        _check(lib().pa_bdm2_estimate_lambda(self.ctx._h, self._h, iters, safety, ws, nb,
                                             ctypes.byref(v)))
        return v.value

    def workspace_size(self, call, B, t=None, avg=None, cfg=None):
        cfg = cfg or solve_cfg()
        sz = _SZ()
        _check(lib().pa_bdm2_workspace_size(self._h, call, B, None if t is None else _dp(t),
                                            None if avg is None else avg._h, ctypes.byref(cfg),
                                            ctypes.byref(sz)))
        return sz.value

    def _workspace(self, call, B, t, cfg, avg=None):
        import torch
        need = self.workspace_size(call, B, t, avg, cfg)
        if self._ws is None or self._ws.numel() < need + 256:
            self._ws = None
            self._ws = torch.empty(need + 256, dtype=torch.uint8,
                                   device=f"cuda:{self.ctx.device}")
        base = self._ws.data_ptr()
        off = (-base) % 256
        return _V(base + off), self._ws.numel() - off

    def apply_L(self, U, cfg=None, out=None):
        cfg = cfg or solve_cfg()
        B = U.shape[0]
        out = U.new_empty(U.shape) if out is None else out
        ws, nb = self._workspace(PA_BDM2_APPLY_L, B, None, cfg)
        st = Stats()
        _check(lib().pa_bdm2_apply_L(self.ctx._h, self._h, B, _ptr(U), _ptr(out), ws, nb,
                                     ctypes.byref(cfg), ctypes.byref(st)))
        return out, st.as_dict()

    def expL_apply(self, t, U, cfg=None, out=None):
        cfg = cfg or solve_cfg()
        B = U.shape[0]
        t = np.ascontiguousarray(np.broadcast_to(np.asarray(t, np.float64), (B,)))
        out = U.new_empty(U.shape) if out is None else out
        ws, nb = self._workspace(PA_BDM2_EXPL, B, t, cfg)
        st = Stats()
        _check(lib().pa_bdm2_expL_apply(self.ctx._h, self._h, B, _dp(t), _ptr(U), _ptr(out), ws,
                                        nb, ctypes.byref(cfg), ctypes.byref(st)))
        return out, st.as_dict()

    def nonlinear(self, U, cfg=None, out=None):
        cfg = cfg or solve_cfg()
        B = U.shape[0]
        out = U.new_empty(U.shape) if out is None else out
        ws, nb = self._workspace(PA_BDM2_NONLINEAR, B, None, cfg)
        st = Stats()
        _check(lib().pa_bdm2_nonlinear(self.ctx._h, self._h, B, _ptr(U), _ptr(out), ws, nb,
                                       ctypes.byref(cfg), ctypes.byref(st)))
        return out, st.as_dict()

    def phase_avg_rhs(self, avg: Avg, U, cfg=None, out=None):
        cfg = cfg or solve_cfg()
        members = U.shape[0]
        out = U.new_empty(U.shape) if out is None else out
        ws, nb = self._workspace(PA_BDM2_PHASE_AVG, members, None, cfg, avg)
        st = Stats()
        _check(lib().pa_bdm2_phase_avg_rhs(self.ctx._h, self._h, avg._h, members, _ptr(U),
                                           _ptr(out), ws, nb, ctypes.byref(cfg),
                                           ctypes.byref(st)))
        return out, st.as_dict()

    def step(self, avg: Avg, dt: float, U, cfg=None):
        """pa_bdm2_step: one averaged RK4 step, U updated in place."""
        cfg = cfg or solve_cfg()
        members = U.shape[0]
        dtv = np.array([dt], np.float64)
        ws, nb = self._workspace(PA_BDM2_STEP, members, dtv, cfg, avg)
        st = Stats()
        _check(lib().pa_bdm2_step(self.ctx._h, self._h, avg._h, float(dt), members, _ptr(U), ws,
                                  nb, ctypes.byref(cfg), ctypes.byref(st)))
        return U, st.as_dict()

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pa_bdm2_destroy(self._h)
            self._h = None


class Batch:
    """Several averaged right-hand-side problems (meshes and ensembles) run
    together (pa_batch_*): items[i] = (ops, members)."""

    def __init__(self, ctx: Context, items, avg: Avg):
        self.ctx, self.avg = ctx, avg
        self.items = list(items)
        n = len(self.items)
        self._ops = [o for o, _ in self.items]  # keep the operators alive
        opsv = (_V * n)(*[o._h for o in self._ops])
        mem = np.ascontiguousarray([m for _, m in self.items], np.int32)
        h = _V()
        _check(lib().pa_batch_create(n, opsv, mem.ctypes.data_as(_I), avg._h, ctypes.byref(h)))
        self._h = h
        self._ws = None

    def __len__(self):
        return len(self.items)

    def workspace(self, cfg=None):
        import torch
        cfg = cfg or solve_cfg()
        sz = _SZ()
        _check(lib().pa_batch_workspace_size(self._h, ctypes.byref(cfg), ctypes.byref(sz)))
        if self._ws is None or self._ws.numel() < sz.value + 256:
            self._ws = None
            self._ws = torch.empty(sz.value + 256, dtype=torch.uint8,
                                   device=f"cuda:{self.ctx.device}")
        base = self._ws.data_ptr()
        off = (-base) % 256
        return _V(base + off), self._ws.numel() - off

    def _ptrs(self, Us, outs):
        n = len(self.items)
        if len(Us) != n or len(outs) != n:
            raise ValueError(f"need {n} inputs and outputs")
        for (o, m), U, out in zip(self.items, Us, outs):
            if tuple(U.shape) != (m, o.n) or tuple(out.shape) != (m, o.n):
                raise ValueError(f"state shape must be ({m}, {o.n})")
        return (_V * n)(*[U.data_ptr() for U in Us]), (_V * n)(*[x.data_ptr() for x in outs])

    def run(self, Us, cfg=None, outs=None):
        """Nbar of every item; returns (outputs, per-item stats)."""
        cfg = cfg or solve_cfg()
        outs = [U.new_empty(U.shape) for U in Us] if outs is None else outs
        up, op = self._ptrs(Us, outs)
        ws, nb = self.workspace(cfg)
        st = (Stats * len(self.items))()
        _check(lib().pa_batch_run(self.ctx._h, self._h, up, op, ws, nb, ctypes.byref(cfg), st))
        return outs, [s.as_dict() for s in st]

    def set_tune(self, item, narrow_rows_per_thread, wide_max_wg, lp_min_cols=8,
                 mixed_min_cols=8, fused_steps=6):
        t = _tune_struct(dict(narrow_rows_per_thread=narrow_rows_per_thread,
                              wide_max_wg=wide_max_wg, lp_min_cols=lp_min_cols,
                              mixed_min_cols=mixed_min_cols, fused_steps=fused_steps))
        _check(lib().pa_batch_set_tune(self._h, item, ctypes.byref(t)))

    def get_tune(self, item):
        t = LaunchTune()
        _check(lib().pa_batch_get_tune(self._h, item, ctypes.byref(t)))
        return _tune_dict(t)

    def autotune(self, Us, cfg=None, cache=None):
        """Per-item launch shapes (pa_batch_autotune).  With a JSON cache, an
        item whose key (level, members, M, configuration) is stored takes the
        stored shape; the others are searched and stored."""
        import json
        cfg = cfg or solve_cfg()
        keys = [f"level{o.mesh.level}_members{m}_M{self.avg.M}_rtol{cfg.cg_rtol:g}_"
                f"tol{cfg.cheb_tol:g}_bw{cfg.backward}_prec{cfg.precision}_"
                f"solver{cfg.solver}_precond{cfg.precond}_batch" for o, m in self.items]
        table = {}
        if cache and os.path.exists(cache):
            table = json.load(open(cache))
        if all(k in table for k in keys):
            for i, k in enumerate(keys):
                _check(lib().pa_batch_set_tune(self._h, i, ctypes.byref(_tune_struct(table[k]))))
            return [dict(table[k], cached=True) for k in keys]
        outs = [U.new_empty(U.shape) for U in Us]
        up, op = self._ptrs(Us, outs)
        ws, nb = self.workspace(cfg)
        t = (LaunchTune * len(self.items))()
        _check(lib().pa_batch_autotune(self.ctx._h, self._h, up, op, ws, nb, ctypes.byref(cfg), t))
        res = [dict(_tune_dict(x), best_ms=x.best_ms) for x in t]
        if cache:
            table.update(dict(zip(keys, res)))
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return [dict(r, cached=False) for r in res]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pa_batch_destroy(self._h)
            self._h = None


def _dev_buffer(nbytes, device):
    """256-byte aligned device buffer: (tensor keeping it alive, address)."""
    import torch
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{device}")
    base = t.data_ptr()
    return t, base + ((-base) % 256)


class LearnedPrecond:
    """Parameters of the learned mass-matrix preconditioner (pa_lp_*)."""

    def __init__(self, seed: int = 0):
        h = _V()
        _check(lib().pa_lp_create(3, 32, seed, ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int()
        _check(lib().pa_lp_param_count(h, ctypes.byref(n)))
        self.n_params = n.value

    @property
    def params(self):
        out = np.zeros(self.n_params, np.float32)
        _check(lib().pa_lp_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    @params.setter
    def params(self, value):
        v = np.ascontiguousarray(value, np.float32)
        assert v.size == self.n_params
        _check(lib().pa_lp_set_params(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def save(self, path):
        _check(lib().pa_lp_save(self._h, str(path).encode()))

    def load(self, path):
        _check(lib().pa_lp_load(self._h, str(path).encode()))

    @staticmethod
    def _ops_array(ops_list):
        return (_V * len(ops_list))(*[o._h for o in ops_list])

    def _workspace(self, ops_list, probes, steps, device):
        sz = _SZ()
        _check(lib().pa_lp_workspace_size(self._ops_array(ops_list), len(ops_list), probes, steps,
                                          ctypes.byref(sz)))
        return _dev_buffer(sz.value, device) + (sz.value,)

    def train(self, ops_list, steps=300, probes=8, lr=3e-3, bf16=True, seed=1):
        """Train on the GPU over the given operators; returns the statistics."""
        ctx = ops_list[0].ctx
        buf, ws, nb = self._workspace(ops_list, probes, steps, ctx.device)
        cfg = TrainCfg(steps, probes, lr, 1 if bf16 else 0, seed)
        st = TrainStats()
        _check(lib().pa_lp_train(ctx._h, self._h, self._ops_array(ops_list), len(ops_list),
                                 ctypes.byref(cfg), _V(ws), nb, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def loss_grad(self, ops, probes, bf16=False):
        """Loss and gradient for host probes [n_e][P] (library numbering)."""
        Z = np.ascontiguousarray(probes, np.float64)
        buf, ws, nb = self._workspace([ops], Z.shape[1], 1, ops.ctx.device)
        loss = ctypes.c_double()
        grad = np.zeros(self.n_params)
        _check(lib().pa_lp_loss_grad(ops.ctx._h, self._h, ops._h, Z.shape[1], _dp(Z),
                                     1 if bf16 else 0, _V(ws), nb, ctypes.byref(loss), _dp(grad)))
        return loss.value, grad

    def ghat(self, ops, bf16=False):
        """(diagonal [n_e], off-diagonal [n_e][4] in mass-pattern slot order)."""
        buf, ws, nb = self._workspace([ops], 1, 1, ops.ctx.device)
        gd = np.zeros(ops.mesh.ne)
        go = np.zeros((ops.mesh.ne, 4))
        _check(lib().pa_lp_ghat(ops.ctx._h, self._h, ops._h, 1 if bf16 else 0, _V(ws), nb,
                                _dp(gd), _dp(go)))
        return gd, go

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pa_lp_destroy(self._h)
            self._h = None


def attach_learned(ops, lp: LearnedPrecond, bf16=True):
    """Inference on ops' graph, P = G G^T and P M on the host, bound to a
    device buffer owned by ops; returns the spectral information."""
    buf, ws, nb = lp._workspace([ops], 1, 1, ops.ctx.device)
    info = LpInfo()
    _check(lib().pa_ops_lp_attach(ops.ctx._h, ops._h, lp._h, 1 if bf16 else 0, _V(ws), nb,
                                  ctypes.byref(info)))
    del buf
    sz = _SZ()
    _check(lib().pa_ops_lp_device_size(ops._h, ctypes.byref(sz)))
    ops._lp_buf, addr = _dev_buffer(sz.value, ops.ctx.device)
    _check(lib().pa_ops_lp_bind(ops.ctx._h, ops._h, _V(addr)))
    return {f: getattr(info, f) for f, _ in info._fields_}
