"""Oracle: plain single-threaded FP64 CPU implementation of the method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2103_07706_amd``) and neither imports the
other.  The arithmetic lives in the C sources next to this file (see
``oracle.h`` for what each function follows in the paper and what pins it);
this module only builds the shared object and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["om_mesh.c", "om_ops.c", "om_cheb.c", "om_rexi.c", "om_nonlin.c", "om_avg.c"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (portable flags, no -march=native, since
    the object may run on another host)."""
    if force or not os.path.exists(_SO):
        srcs = [os.path.join(_HERE, s) for s in _SOURCES]
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-o", tmp] + srcs + ["-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)
_V = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        sig = {
            "om_mesh_create": (_V, [ctypes.c_int, ctypes.c_double]),
            "om_mesh_destroy": (None, [_V]),
            "om_mesh_counts": (None, [_V, _I, _I, _I]),
            "om_mesh_export": (None, [_V, _D, _I, _I, _I, _I, _I]),
            "om_ops_create": (_V, [_V, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]),
            "om_ops_destroy": (None, [_V]),
            "om_ops_export": (ctypes.c_int, [_V, _I, _I, _D, _D, _D]),
            "om_mass_solve": (ctypes.c_int, [_V, _D, _D, ctypes.c_double, ctypes.c_int]),
            "om_apply_L": (ctypes.c_int, [_V, _D, _D, ctypes.c_double]),
            "om_power_rho": (ctypes.c_double, [_V, _D, ctypes.c_int, ctypes.c_double]),
            "om_cheb_coeffs": (None, [ctypes.c_double, ctypes.c_int, _D]),
            "om_cheb_truncate": (ctypes.c_int, [_D, ctypes.c_int, ctypes.c_double]),
            "om_expL": (ctypes.c_int, [_V, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _D, _D]),
            "om_nonlinear": (ctypes.c_int, [_V, _D, _D, ctypes.c_double]),
            "om_rexi_coeffs": (None, [ctypes.c_double, ctypes.c_int, ctypes.c_double, _D, _D]),
            "om_rexi_expL": (ctypes.c_int, [_V, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            _D, _D]),
            "om_avg_nodes": (None, [ctypes.c_int, ctypes.c_double, _D, _D]),
            "om_phase_avg_rhs": (ctypes.c_int, [_V, ctypes.c_double, ctypes.c_int, _D, _D,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                _D, _D]),
            "om_step": (ctypes.c_int, [_V, ctypes.c_double, ctypes.c_int, _D, _D,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, _D]),
            "om_rexi_phase_avg_rhs": (ctypes.c_int, [_V, ctypes.c_double, ctypes.c_int, _D, _D,
                                                     ctypes.c_int, ctypes.c_double,
                                                     ctypes.c_double, ctypes.c_double,
                                                     ctypes.c_int, _D, _D]),
            "om_rexi_step": (ctypes.c_int, [_V, ctypes.c_double, ctypes.c_int, _D, _D,
                                            ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            _D]),
            "om_diagnostics": (None, [_V, _D, _D]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _ip(a):
    return a.ctypes.data_as(_I)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


class Mesh:
    """Icosahedral mesh of flat triangles (paper Sec. 3 mesh description)."""

    def __init__(self, level: int, radius: float = 6.37122e6):
        lib = _load()
        self.level = level
        self.radius = radius
        self._h = lib.om_mesh_create(level, radius)
        if not self._h:
            raise OracleError("mesh level out of range")
        nv, ne, nc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        lib.om_mesh_counts(self._h, ctypes.byref(nv), ctypes.byref(ne), ctypes.byref(nc))
        self.nv, self.ne, self.nc = nv.value, ne.value, nc.value
        self.verts = np.zeros((self.nv, 3))
        self.cell_verts = np.zeros((self.nc, 3), np.int32)
        self.cell_edges = np.zeros((self.nc, 3), np.int32)
        self.cell_sign = np.zeros((self.nc, 3), np.int32)
        self.edge_cells = np.zeros((self.ne, 2), np.int32)
        self.edge_verts = np.zeros((self.ne, 2), np.int32)
        lib.om_mesh_export(self._h, _dp(self.verts), _ip(self.cell_verts), _ip(self.cell_edges),
                           _ip(self.cell_sign), _ip(self.edge_cells), _ip(self.edge_verts))

    @property
    def n(self) -> int:
        return self.ne + self.nc

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.om_mesh_destroy(self._h)
            self._h = None


class Ops:
    """RT0/P0 discrete operators on a mesh (paper Sec. 2.5)."""

    def __init__(self, mesh: Mesh, g: float = 9.80616, H: float = 1000.0,
                 Omega: float = 7.292e-5, b=None):
        lib = _load()
        self.mesh = mesh
        self.g, self.H, self.Omega = g, H, Omega
        self._b = None if b is None else _f64(b)
        self._h = lib.om_ops_create(mesh._h, g, H, Omega,
                                    None if self._b is None else _dp(self._b))

    @property
    def n(self) -> int:
        return self.mesh.n

    def export(self):
        lib = _load()
        nnz = lib.om_ops_export(self._h, None, None, None, None, None)
        rowptr = np.zeros(self.mesh.ne + 1, np.int32)
        cols = np.zeros(nnz, np.int32)
        mass = np.zeros(nnz)
        cor = np.zeros(nnz)
        area = np.zeros(self.mesh.nc)
        lib.om_ops_export(self._h, _ip(rowptr), _ip(cols), _dp(mass), _dp(cor), _dp(area))
        return dict(rowptr=rowptr, cols=cols, mass=mass, cor=cor, area=area)

    def mass_solve(self, b, rtol=1e-14, maxit=1000):
        b = _f64(b)
        x = np.zeros_like(b)
        it = _load().om_mass_solve(self._h, _dp(b), _dp(x), rtol, maxit)
        if it < 0:
            raise OracleError("mass solve did not converge")
        return x, it

    def apply_L(self, U, rtol=1e-14):
        U = _f64(U)
        out = np.zeros_like(U)
        if _load().om_apply_L(self._h, _dp(U), _dp(out), rtol) < 0:
            raise OracleError("mass solve did not converge")
        return out

    def power_rho(self, v0, iters=400, rtol=1e-12):
        v0 = _f64(v0)
        return _load().om_power_rho(self._h, _dp(v0), iters, rtol)

    def expL(self, lambda_bar, t, U, tol=1e-13, rtol=1e-14):
        U = _f64(U)
        out = np.zeros_like(U)
        K = _load().om_expL(self._h, lambda_bar, t, tol, rtol, _dp(U), _dp(out))
        if K < 0:
            raise OracleError("exponential failed")
        return out, K

    def rexi_expL(self, lambda_bar, t, U, N, eta0, gm_rtol=1e-13, rtol=1e-14):
        """exp(t L) U by the rational (REXI) sum with N nodes on the ellipse
        of parameter eta0; returns (result, largest GMRES iteration count)."""
        U = _f64(U)
        out = np.zeros_like(U)
        it = _load().om_rexi_expL(self._h, lambda_bar, t, N, eta0, gm_rtol, rtol, _dp(U),
                                  _dp(out))
        if it < 0:
            raise OracleError("rational exponential failed")
        return out, it

    def nonlinear(self, U, rtol=1e-14):
        U = _f64(U)
        out = np.zeros_like(U)
        if _load().om_nonlinear(self._h, _dp(U), _dp(out), rtol) < 0:
            raise OracleError("mass solve did not converge")
        return out

    def phase_avg_rhs(self, lambda_bar, s, w, U, tol=1e-13, rtol=1e-14, which=0):
        U, s, w = _f64(U), _f64(s), _f64(w)
        out = np.zeros_like(U)
        st = _load().om_phase_avg_rhs(self._h, lambda_bar, len(s), _dp(s), _dp(w), tol, rtol,
                                      which, _dp(U), _dp(out))
        if st < 0:
            raise OracleError("averaged RHS failed")
        return out

    def step(self, lambda_bar, s, w, dt, U, tol=1e-13, rtol=1e-14, which=0):
        U = _f64(U).copy()
        s, w = _f64(s), _f64(w)
        st = _load().om_step(self._h, lambda_bar, len(s), _dp(s), _dp(w), dt, tol, rtol, which,
                             _dp(U))
        if st < 0:
            raise OracleError("step failed")
        return U

    def rexi_phase_avg_rhs(self, lambda_bar, s, w, U, N, eta0, gm_rtol=1e-13, rtol=1e-14,
                           which=0):
        """Nbar with every exponential the rational (REXI) sum of rexi_expL."""
        U, s, w = _f64(U), _f64(s), _f64(w)
        out = np.zeros_like(U)
        st = _load().om_rexi_phase_avg_rhs(self._h, lambda_bar, len(s), _dp(s), _dp(w), N, eta0,
                                           gm_rtol, rtol, which, _dp(U), _dp(out))
        if st < 0:
            raise OracleError("rational averaged RHS failed")
        return out

    def rexi_step(self, lambda_bar, s, w, dt, U, N, eta0, gm_rtol=1e-13, rtol=1e-14, which=0):
        """One averaged RK4 step with every exponential the REXI sum."""
        U = _f64(U).copy()
        s, w = _f64(s), _f64(w)
        st = _load().om_rexi_step(self._h, lambda_bar, len(s), _dp(s), _dp(w), dt, N, eta0,
                                  gm_rtol, rtol, which, _dp(U))
        if st < 0:
            raise OracleError("rational step failed")
        return U

    def diagnostics(self, U):
        U = _f64(U)
        out = np.zeros(5)
        _load().om_diagnostics(self._h, _dp(U), _dp(out))
        return dict(mass=out[0], energy_linear=out[1], energy_nonlinear=out[2],
                    hdiv_u=out[3], l2_eta=out[4])

    def wnorm(self, U):
        """Energy norm ||U||_W^2 = H u'M u + g sum |c| eta^2 (L is W-skew)."""
        U = _f64(U)
        d = self.diagnostics(U)
        return np.sqrt(2.0 * d["energy_linear"])

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.om_ops_destroy(self._h)
            self._h = None


def cheb_coeffs(Lbar: float, npts: int):
    """Complex Chebyshev coefficients of exp(i Lbar x) on [-1, 1] (DCT)."""
    a = np.zeros(2 * (npts + 1))
    _load().om_cheb_coeffs(Lbar, npts, _dp(a))
    return a[0::2] + 1j * a[1::2]


def cheb_truncate(a, tol: float) -> int:
    a = np.asarray(a)
    buf = np.zeros(2 * len(a))
    buf[0::2], buf[1::2] = a.real, a.imag
    return _load().om_cheb_truncate(_dp(buf), len(a) - 1, tol)


def rexi_coeffs(theta: float, N: int, eta0: float):
    """Nodes X_j and coefficients c_j (complex arrays) of the rational
    approximation r(x) = sum_j c_j / (X_j - x) of exp(i theta x)."""
    X = np.zeros(2 * N)
    c = np.zeros(2 * N)
    _load().om_rexi_coeffs(theta, N, eta0, _dp(X), _dp(c))
    return X[0::2] + 1j * X[1::2], c[0::2] + 1j * c[1::2]


def avg_nodes(M: int, T: float):
    s = np.zeros(M)
    w = np.zeros(M)
    _load().om_avg_nodes(M, T, _dp(s), _dp(w))
    return s, w


def lambda_bar(ops: Ops, iters: int = 400, seed: int = 12345, factor: float = 1.05,
               rtol: float = 1e-12) -> float:
    """Upper estimate of the spectral radius of L: factor x power iteration
    from a seeded start vector (the start vector is an input, not part of the
    method's arithmetic)."""
    v0 = np.random.default_rng(seed).standard_normal(ops.n)
    return factor * ops.power_rho(v0, iters, rtol)
