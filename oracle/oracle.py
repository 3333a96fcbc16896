"""ctypes wrapper of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product library never does.

The oracle computes, in plain FP64 loops, the spectral-difference residual
and SSPRK(5,3) step of the paper (arXiv 2502.17805, sections "MHD Governing
Equations", "Spectral Difference Method", "Problem Formulation and Boundary
Conditions"); see ``sdmhd_oracle.c`` for the step-by-step citations.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sdmhd_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class Params(C.Structure):
    """Mirror of ``or_params``."""
    _fields_ = [(n, C.c_double) for n in ("gamma", "Rgas", "GM", "Omega", "nu", "kappa", "eta",
                                          "kr_scale", "kr_c0", "kr_c1", "kr_c2", "kr_omega_per_r",
                                          "c_h", "glm_a")] + [
        ("powell", C.c_int32),
        ("wall_kind", C.c_int32 * 2), ("wall_mag", C.c_int32 * 2), ("wall_th", C.c_int32 * 2),
        ("q_wall", C.c_double * 2), ("T_wall", C.c_double * 2)]


def make_params(**kw) -> Params:
    """Params from keyword arguments; 2-element fields take sequences."""
    p = Params()
    defaults = dict(gamma=5.0 / 3.0, Rgas=1.0, GM=0.0, Omega=0.0, nu=0.0, kappa=0.0, eta=0.0,
                    kr_scale=0.0, kr_c0=0.0, kr_c1=0.0, kr_c2=0.0, kr_omega_per_r=0.0,
                    c_h=0.0, glm_a=0.0, powell=0, wall_kind=(0, 0), wall_mag=(0, 0),
                    wall_th=(0, 0), q_wall=(0.0, 0.0), T_wall=(0.0, 0.0))
    defaults.update(kw)
    for k, v in defaults.items():
        if k in ("wall_kind", "wall_mag", "wall_th"):
            getattr(p, k)[0], getattr(p, k)[1] = int(v[0]), int(v[1])
        elif k in ("q_wall", "T_wall"):
            getattr(p, k)[0], getattr(p, k)[1] = float(v[0]), float(v[1])
        elif k == "powell":
            p.powell = int(v)
        else:
            setattr(p, k, float(v))
    return p


_lib = None


def _configure(L):
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
    L.or_shell_new.restype = vp
    L.or_shell_new.argtypes = [ip, ip, ip, C.c_double, C.c_double]
    L.or_box_new.restype = vp
    L.or_box_new.argtypes = [ip, ip, ip, ip, C.c_double, C.c_double, C.c_double, ip, C.c_double]
    L.or_mesh_free.argtypes = [vp]
    L.or_mesh_sizes.argtypes = [vp, C.POINTER(C.c_int64)]
    L.or_mesh_get.argtypes = [vp, C.c_char_p, vp]
    L.or_mesh_get.restype = ip
    L.or_residual.argtypes = [vp, C.POINTER(Params), vp, vp, vp, vp, vp]
    L.or_residual.restype = ip
    L.or_ssprk53_step.argtypes = [vp, C.POINTER(Params), vp, vp, C.c_double]
    L.or_ssprk53_step.restype = ip
    L.or_ssprk53_table.argtypes = [vp, vp, vp]
    L.or_diagnostics.argtypes = [vp, C.POINTER(Params), vp, vp, vp]
    L.or_diagnostics.restype = ip
    L.or_sph_profiles.argtypes = [vp, vp, C.c_double, C.c_double, ip, ip, vp]
    L.or_sph_profiles.restype = ip
    L.or_tables.argtypes = [ip, vp, vp, vp, vp, vp]
    L.or_tables.restype = ip
    L.or_threads.restype = ip
    L.or_point_flux.argtypes = [vp, vp, C.c_double, vp, C.POINTER(Params), vp, vp]
    L.or_point_rusanov.argtypes = [vp, vp, vp, C.POINTER(Params), vp]
    L.or_point_cf.argtypes = [vp, vp, C.POINTER(Params)]
    L.or_point_cf.restype = C.c_double
    L.or_point_wall_flux.argtypes = [vp, vp, C.c_double, vp, ip, C.POINTER(Params), vp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = _configure(C.CDLL(_SO))
    return _lib


def build_variant(source_text: str, path: str) -> str:
    """Compile a modified copy of the oracle source into `path` (the tests use
    it to plant a mistake and check that a pin catches it)."""
    src = path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-fPIC", "-shared", "-I", _HERE, "-o", path, src, "-lm"], check=True)
    return path


def source_text() -> str:
    """The oracle's C source with its pointwise-physics include inlined."""
    with open(_SRC) as f:
        src = f.read()
    inc = '#include "sdmhd_oracle_point.inc"'
    with open(os.path.join(_HERE, "sdmhd_oracle_point.inc")) as f:
        return src.replace(inc, f.read())


def swap_library(path):
    """Make every call of this module use the library at `path` (None: the
    built oracle); returns the previous library object for swap_back."""
    global _lib
    prev = _lib
    _lib = None if path is None else _configure(C.CDLL(path))
    return prev


def swap_back(prev):
    global _lib
    _lib = prev


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def tables(N: int):
    """(xs, xf, I[(N+1),N], D[N,(N+1)], W) of the oracle."""
    xs, xf = np.zeros(N), np.zeros(N + 1)
    I, D, W = np.zeros((N + 1, N)), np.zeros((N, N + 1)), np.zeros(N)
    if lib().or_tables(N, _ptr(xs), _ptr(xf), _ptr(I), _ptr(D), _ptr(W)):
        raise ValueError("unsupported N")
    return xs, xf, I, D, W


def ssprk53_table():
    a, b, c = np.zeros((6, 6)), np.zeros((6, 6)), np.zeros(5)
    lib().or_ssprk53_table(_ptr(a), _ptr(b), _ptr(c))
    return a, b, c


def point_flux(prm, q, G, n, kr=0.0):
    """(F_inv . n, F_vis . n) at one point; G[v*3+j] = dQ_v/dx_j."""
    q, G, n = (np.ascontiguousarray(a, dtype=np.float64) for a in (q, G, n))
    Fi, Fv = np.zeros(9), np.zeros(9)
    lib().or_point_flux(_ptr(q), _ptr(G), float(kr), _ptr(n), C.byref(prm), _ptr(Fi), _ptr(Fv))
    return Fi, Fv


def point_rusanov(prm, qL, qR, n):
    qL, qR, n = (np.ascontiguousarray(a, dtype=np.float64) for a in (qL, qR, n))
    F = np.zeros(9)
    lib().or_point_rusanov(_ptr(qL), _ptr(qR), _ptr(n), C.byref(prm), _ptr(F))
    return F


def point_cf(prm, q, nh):
    q, nh = (np.ascontiguousarray(a, dtype=np.float64) for a in (q, nh))
    return float(lib().or_point_cf(_ptr(q), _ptr(nh), C.byref(prm)))


def point_wall_flux(prm, q, G, n, group, kr=0.0):
    q, G, n = (np.ascontiguousarray(a, dtype=np.float64) for a in (q, G, n))
    F = np.zeros(9)
    lib().or_point_wall_flux(_ptr(q), _ptr(G), float(kr), _ptr(n), int(group), C.byref(prm), _ptr(F))
    return F


def threads() -> int:
    return int(lib().or_threads())


class Mesh:
    """An oracle mesh (shell or box) with its metrics and face table."""

    def __init__(self, handle, N):
        if not handle:
            raise ValueError("mesh construction failed")
        self._h = handle
        self._L = lib()  # the library that made the handle serves every call on it
        s = (C.c_int64 * 4)()
        self._L.or_mesh_sizes(handle, s)
        self.E, self.F, self.NB, self.N = int(s[0]), int(s[1]), int(s[2]), int(s[3])

    @classmethod
    def shell(cls, N, Nz, Nr, rb=0.70, rt=0.98):
        return cls(lib().or_shell_new(N, Nz, Nr, rb, rt), N)

    @classmethod
    def box(cls, N, nx, ny, nz, L=(1.0, 1.0, 1.0), periodic=7, warp=0.0):
        return cls(lib().or_box_new(N, nx, ny, nz, L[0], L[1], L[2], periodic, warp), N)

    def __del__(self):
        try:
            if self._h:
                self._L.or_mesh_free(self._h)
                self._h = None
        except Exception:
            pass

    def get(self, name):
        N, E = self.N, self.E
        N3, NF = N ** 3, (N + 1) * N * N
        shapes = {"x_sp": ((E, 3, N3), np.float64), "detJ_sp": ((E, N3), np.float64),
                  "S_sp": ((E, 3, 3, N3), np.float64), "S_fp": ((E, 3, 3, NF), np.float64),
                  "faces": ((self.F, 5), np.int32), "nbr": ((E, 6, 3), np.int32),
                  "W3detJ": ((E, N3), np.float64), "x_bfp": ((self.NB, 3, N * N), np.float64)}
        shp, dt = shapes[name]
        out = np.zeros(shp, dtype=dt)
        if self._L.or_mesh_get(self._h, name.encode(), _ptr(out)):
            raise KeyError(name)
        return out

    def residual(self, prm, Q, ghost=None, with_scale=False, with_divB=False):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        R = np.empty_like(Q)
        ts = np.zeros(9)
        dB = np.zeros((self.E, self.N ** 3)) if with_divB else None
        g = None if ghost is None else np.ascontiguousarray(ghost, dtype=np.float64)
        rc = self._L.or_residual(self._h, C.byref(prm), _ptr(Q), _ptr(g), _ptr(R), _ptr(ts), _ptr(dB))
        if rc:
            raise RuntimeError("oracle residual failed (Dirichlet face without ghost data)")
        out = [R]
        if with_scale:
            out.append(ts)
        if with_divB:
            out.append(dB)
        return out[0] if len(out) == 1 else tuple(out)

    def step(self, prm, Q, dt, ghost=None):
        Q = np.array(Q, dtype=np.float64, copy=True, order="C")
        g = None if ghost is None else np.ascontiguousarray(ghost, dtype=np.float64)
        if self._L.or_ssprk53_step(self._h, C.byref(prm), _ptr(Q), _ptr(g), float(dt)):
            raise RuntimeError("oracle step failed")
        return Q

    def sph_profiles(self, Q, n_r, n_th, rb=0.70, rt=0.98):
        """Per (r, theta) bin: sums of w, w V_phi, w V_mer, w (B_r^2 + B_theta^2)/2,
        w B_phi^2/2 over the SPs in the bin, shape (n_r, n_th, 5)."""
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        out = np.zeros((n_r, n_th, 5))
        if self._L.or_sph_profiles(self._h, _ptr(Q), float(rb), float(rt), int(n_r), int(n_th), _ptr(out)):
            raise ValueError("bad bin counts or radii")
        return out

    def diagnostics(self, prm, Q, ghost=None):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        out = np.zeros(16)
        g = None if ghost is None else np.ascontiguousarray(ghost, dtype=np.float64)
        if self._L.or_diagnostics(self._h, C.byref(prm), _ptr(Q), _ptr(g), _ptr(out)):
            raise RuntimeError("oracle diagnostics failed")
        return out
