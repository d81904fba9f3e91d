"""Oracle: plain serial FP64 CPU implementation of the parareal-with-splitting
hot path (arXiv 2502.08370), used as the parity reference.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product
library (``paper_2502_08370_amd``) never imports it and shares no code with
it. The arithmetic lives in ``oracle.c`` (see its header for the paper passages
each routine follows); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

_dp = C.POINTER(C.c_double)


class OrProblem(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("T", C.c_double),
        ("n_slices", C.c_int), ("fine_steps", C.c_int), ("coarse_steps", C.c_int),
        ("split", C.c_int), ("fine_method", C.c_int),
        ("c", C.c_double),
        ("ax", _dp), ("ay", _dp),
        ("n_colors", C.c_int), ("rho", _dp),
        ("n_forcing", C.c_int), ("fS", _dp), ("fg_fine", _dp), ("fg_coarse", _dp),
    ]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (contraction off for reproducibility)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER(OrProblem)
        L.or_faces_from_theta.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
        L.or_faces_from_theta_1d.argtypes = [C.c_int, _dp, _dp]
        L.or_apply_A.argtypes = [P, _dp, _dp]
        L.or_apply_Aj.argtypes = [P, C.c_int, _dp, _dp]
        L.or_fie_step.argtypes = [P, C.c_double, _dp, _dp]
        L.or_dr_step.argtypes = [P, C.c_double, _dp, _dp]
        L.or_fine.argtypes = [P, C.c_int, _dp]
        L.or_coarse.argtypes = [P, C.c_int, _dp]
        L.or_fine_batch.argtypes = [P, C.c_int, _dp, _dp]
        L.or_sequential_fine.argtypes = [P, _dp, _dp]
        L.or_coarse_sweep.argtypes = [P, _dp, _dp, _dp]
        L.or_coarse_sweep.restype = C.c_double
        L.or_parareal.argtypes = [P, _dp, C.c_int, C.c_double, _dp, _dp]
        L.or_parareal.restype = C.c_int
        L.or_adjoint.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.or_theta_grad.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "float64 C-contiguous array required"
    return a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class Problem:
    """Problem description mirrored from the paper's model (section 2).

    dim: 1 or 2; nx, ny: interior nodes; T, n_slices (N_c), fine_steps (s),
    coarse_steps; split: 'dim' or 'dd'; fine: 'fie' or 'dr'; c: reaction;
    ax (ny, nx+1) / ay (ny+1, nx): face coefficients; rho: partition of unity
    of the domain-decomposition split, (M, nx+1) face weights in 1D, (M, 2nx+1)
    half-grid samples in x in 2D (vertical strips, see oracle.h); forcing:
    None or (S, g_fine, g_coarse) with S (m, ny, nx) the spatial factors of the
    source F(t) = sum_m g_m(t) S_m and g_fine (m, N*s), g_coarse (m, N*cs) its
    time factors at the fine / coarse step end times (see oracle.h).
    """

    def __init__(self, *, dim, nx, ny, T, n_slices, fine_steps, coarse_steps=1, split="dim",
                 fine="fie", c=0.0, ax, ay=None, rho=None, forcing=None):
        self.dim, self.nx, self.ny = int(dim), int(nx), int(ny)
        if self.dim == 1:
            self.ny = 1
        self.T, self.n_slices = float(T), int(n_slices)
        self.fine_steps, self.coarse_steps = int(fine_steps), int(coarse_steps)
        self.split, self.fine_method, self.c = split, fine, float(c)
        self.ax = _f64(ax).reshape(self.ny, self.nx + 1)
        self.ay = None if ay is None else _f64(ay).reshape(self.ny + 1, self.nx)
        rw = 2 * self.nx + 1 if self.dim == 2 else self.nx + 1
        self.rho = None if rho is None else _f64(rho).reshape(-1, rw)
        self.fS = self.fgf = self.fgc = None
        nf = 0
        if forcing is not None:
            S, gf, gc = forcing
            nf = int(np.asarray(S).shape[0])
            self.fS = _f64(S).reshape(nf, self.nx * self.ny)
            self.fgf = _f64(gf).reshape(nf, self.n_slices * self.fine_steps)
            self.fgc = _f64(gc).reshape(nf, self.n_slices * self.coarse_steps)
        self._s = OrProblem(
            self.dim, self.nx, self.ny, self.T, self.n_slices, self.fine_steps, self.coarse_steps,
            1 if split == "dd" else 0, 1 if fine == "dr" else 0, self.c,
            _ptr(self.ax), _ptr(self.ay),
            0 if self.rho is None else self.rho.shape[0], _ptr(self.rho),
            nf, _ptr(self.fS), _ptr(self.fgf), _ptr(self.fgc))

    @property
    def npts(self):
        return self.nx * self.ny

    @property
    def shape(self):
        return (self.ny, self.nx) if self.dim == 2 else (self.nx,)

    def _p(self):
        return C.byref(self._s)

    def state(self, u):
        return np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape).copy()

    def apply_A(self, u):
        u = self.state(u)
        out = np.empty_like(u)
        lib().or_apply_A(self._p(), _ptr(u), _ptr(out))
        return out

    def apply_Aj(self, j, u):
        u = self.state(u)
        out = np.empty_like(u)
        lib().or_apply_Aj(self._p(), int(j), _ptr(u), _ptr(out))
        return out

    def fie_step(self, u, tau, F=None):
        u = self.state(u)
        lib().or_fie_step(self._p(), float(tau), _ptr(None if F is None else self.state(F)), _ptr(u))
        return u

    def dr_step(self, u, tau, F=None):
        u = self.state(u)
        lib().or_dr_step(self._p(), float(tau), _ptr(None if F is None else self.state(F)), _ptr(u))
        return u

    def fine(self, u, n=0):
        """Fine propagator over coarse interval n."""
        u = self.state(u)
        lib().or_fine(self._p(), int(n), _ptr(u))
        return u

    def coarse(self, u, n=0):
        """Coarse propagator over coarse interval n."""
        u = self.state(u)
        lib().or_coarse(self._p(), int(n), _ptr(u))
        return u

    def fine_batch(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        n = U.shape[0]
        out = np.empty_like(U)
        lib().or_fine_batch(self._p(), n, _ptr(U), _ptr(out))
        return out

    def sequential_fine(self, u0):
        out = np.empty((self.n_slices + 1,) + self.shape)
        lib().or_sequential_fine(self._p(), _ptr(self.state(u0)), _ptr(out))
        return out

    def coarse_sweep(self, F, G_old, U):
        """In-place on G_old and U (numpy float64 arrays); returns the increment."""
        return lib().or_coarse_sweep(self._p(), _ptr(_f64(F)) if F is not None else None,
                                     _ptr(G_old), _ptr(U))

    def parareal(self, u0, k_max, tol=0.0):
        U = np.empty((self.n_slices + 1,) + self.shape)
        hist = np.zeros(max(k_max, 1))
        k = lib().or_parareal(self._p(), _ptr(self.state(u0)), int(k_max), float(tol), _ptr(U),
                              _ptr(hist))
        return U, k, hist[:k].copy()

    def adjoint(self, u0, lam_T):
        g0 = np.empty(self.shape)
        gax = np.empty((self.ny, self.nx + 1))
        gay = np.empty((self.ny + 1, self.nx)) if self.dim == 2 else None
        lib().or_adjoint(self._p(), _ptr(self.state(u0)), _ptr(self.state(lam_T)), _ptr(g0),
                         _ptr(gax), _ptr(gay))
        return g0, gax, gay


def faces_from_theta(nx, ny, theta, dim=2):
    """Face coefficients (mean of e^theta over the face's two nodes) from nodal theta."""
    if dim == 1:
        theta = _f64(theta).reshape(nx + 2)
        ax = np.empty((1, nx + 1))
        lib().or_faces_from_theta_1d(nx, _ptr(theta), _ptr(ax))
        return ax, None
    theta = _f64(theta).reshape(ny + 2, nx + 2)
    ax = np.empty((ny, nx + 1))
    ay = np.empty((ny + 1, nx))
    lib().or_faces_from_theta(nx, ny, _ptr(theta), _ptr(ax), _ptr(ay))
    return ax, ay


def theta_grad(nx, ny, theta, gax, gay):
    theta = _f64(theta).reshape(ny + 2, nx + 2)
    out = np.empty_like(theta)
    lib().or_theta_grad(nx, ny, _ptr(theta), _ptr(_f64(gax)), _ptr(_f64(gay)) if gay is not None else None,
                        _ptr(out))
    return out
