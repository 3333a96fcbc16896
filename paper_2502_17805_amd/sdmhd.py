"""Python binding of the gfx950 spectral-difference GLM-MHD library (libsdmhd.so).

Argument marshalling only: every step of the residual and Runge-Kutta stage
runs in the library's HIP kernels.  PyTorch provides device memory and streams.
If the compiled library is missing this module raises at import time -- there
is no CPU fallback.

Entry points mirror include/sdmhd.h:
  shell(Nz, Nr, p)/box(...)        host mesh, metrics and neighbour table
  Solver(mesh, arith)              context + device copies of the mesh
  Solver.residual(prm, Q)          R = dQ/dt                 (sdm_residual)
  Solver.stage(prm, regs, st, dt)  one fused Shu-Osher stage (sdm_rk_stage)
  Solver.step(prm, dt)             one SSPRK(5,3) step     (sdm_ssprk53_step)
  Solver.step_noalloc(prm, dt)     the same without a workspace (sdm_ssprk53_step_noalloc)
  Solver.diagnostics(prm, Q)       volume, mass, energy, KE, E_B, div B, ...
  sph_bins / Solver.sph_profiles   spherical-component sums per (r, theta) bin
  background_profile(r, ...)       polytrope / flux-balanced initial background
  ssp53_stages()                   the SSPRK(5,3) stages (sdm_ssprk53_stages)
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdmhd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2502_17805_amd/build.py "
                      "(or __graft_entry__.build()) first -- there is no fallback path")

# torch is loaded first so that the library binds to the same HIP runtime
# (by soname) as the torch that allocates its memory and streams; two HIP
# runtimes in one process do not share devices.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

SDM_OK = 0


class Params(C.Structure):
    """Mirror of sdm_params."""
    _fields_ = [(n, C.c_double) for n in ("gamma", "Rgas", "GM", "Omega", "nu", "kappa", "eta",
                                          "kr_scale", "kr_c0", "kr_c1", "kr_c2", "kr_omega_per_r",
                                          "c_h", "glm_a")] + [
        ("powell", C.c_int32), ("wall_kind", C.c_int32 * 2), ("wall_mag", C.c_int32 * 2),
        ("wall_th", C.c_int32 * 2), ("q_wall", C.c_double * 2), ("T_wall", C.c_double * 2),
        ("ghost", C.c_void_p), ("import_q", C.c_void_p), ("import_v", C.c_void_p)]


class Stage(C.Structure):
    """Mirror of sdm_stage."""
    _fields_ = [("n_in", C.c_int32), ("in_idx", C.c_int32 * 4), ("alpha", C.c_double * 4),
                ("cur", C.c_int32), ("out", C.c_int32), ("beta", C.c_double),
                ("traces_valid", C.c_int32)]


class BatchItem(C.Structure):
    """Mirror of sdm_batch_item."""
    _fields_ = [("ctx", C.c_void_p), ("prm", C.POINTER(Params)), ("regs", C.POINTER(C.c_void_p)),
                ("n_regs", C.c_int32), ("stage", Stage), ("dt", C.c_double), ("ws", C.c_void_p)]


class BackgroundDesc(C.Structure):
    """Mirror of sdm_background."""
    _fields_ = [(n, C.c_double) for n in ("GM", "Rgas", "gamma", "rb", "rt", "rho_b", "N_rho", "L", "kappa",
                                          "kr_scale", "kr_c0", "kr_c1", "kr_c2", "kr_omega_per_r")] + [
        ("flux_balanced", C.c_int32)]


class MeshDesc(C.Structure):
    """Mirror of sdm_mesh."""
    _fields_ = [("n_elem", C.c_int64), ("n_bfaces", C.c_int64), ("x_sp", C.c_void_p),
                ("detJ", C.c_void_p), ("S_fp", C.c_void_p), ("Sj_sp", C.c_void_p), ("nbr", C.c_void_p),
                ("n_face", C.c_void_p)]


_vp, _i64p = C.c_void_p, C.POINTER(C.c_int64)
_lib.sdm_last_error.restype = C.c_char_p
_lib.sdm_version.restype = C.c_char_p
_lib.sdm_shell_sizes.argtypes = [C.c_int, C.c_int, _i64p, _i64p]
_lib.sdm_shell_build.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double] + [_vp] * 6
_lib.sdm_box_sizes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _i64p, _i64p]
_lib.sdm_box_build.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                               C.c_int, C.c_double, C.c_int] + [_vp] * 6
_lib.sdm_tables.argtypes = [C.c_int] + [_vp] * 5
_lib.sdm_create.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]
_lib.sdm_destroy.argtypes = [_vp]
_lib.sdm_mesh_bind.argtypes = [_vp, C.POINTER(MeshDesc)]
_lib.sdm_workspace_size.argtypes = [_vp, C.POINTER(C.c_size_t)]
_lib.sdm_workspace_traces.argtypes = [_vp, _vp, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]
_lib.sdm_residual.argtypes = [_vp, C.POINTER(Params), _vp, _vp, _vp, _vp]
_lib.sdm_rk_stage.argtypes = [_vp, C.POINTER(Params), C.POINTER(C.c_void_p), C.c_int,
                              C.POINTER(Stage), C.c_double, _vp, _vp]
_lib.sdm_rk_stage_volume.argtypes = _lib.sdm_rk_stage.argtypes
_lib.sdm_rk_stage_finish.argtypes = _lib.sdm_rk_stage.argtypes
_lib.sdm_diagnostics.argtypes = [_vp, C.POINTER(Params), _vp, _vp, _vp, _vp]
_lib.sdm_sph_bins.argtypes = [C.c_int64, C.c_int, _vp, C.c_double, C.c_double, C.c_int, C.c_int, _vp, _vp]
_lib.sdm_sph_profiles.argtypes = [_vp, _vp, _vp, _vp, C.c_int, _vp, _vp]
_lib.sdm_background_profile.argtypes = [C.POINTER(BackgroundDesc), C.c_int64, _vp, _vp, _vp, _vp]
_lib.sdm_ssprk53_stages.argtypes = [C.POINTER(Stage), C.POINTER(C.c_double)]
_lib.sdm_ssprk53_step.argtypes = [_vp, C.POINTER(Params), C.POINTER(C.c_void_p), C.c_double, C.c_int, _vp, _vp]
_lib.sdm_ssprk53_step_noalloc.argtypes = [_vp, C.POINTER(Params), C.POINTER(C.c_void_p), C.c_double, _vp]
_lib.sdm_batch_workspace_size.argtypes = [C.c_int, C.POINTER(C.c_size_t)]
_lib.sdm_batch_stage.argtypes = [C.POINTER(BatchItem), C.c_int, _vp, C.c_size_t, C.c_int, _vp]
_lib.sdm_profile_enable.argtypes = [_vp, C.c_int]
_lib.sdm_profile_read.argtypes = [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
for _f in ("sdm_shell_sizes", "sdm_shell_build", "sdm_box_sizes", "sdm_box_build", "sdm_tables",
           "sdm_create", "sdm_destroy", "sdm_mesh_bind", "sdm_workspace_size", "sdm_residual",
           "sdm_rk_stage", "sdm_diagnostics", "sdm_profile_enable", "sdm_profile_read",
           "sdm_batch_workspace_size", "sdm_batch_stage", "sdm_workspace_traces", "sdm_rk_stage_volume",
           "sdm_rk_stage_finish", "sdm_sph_bins", "sdm_sph_profiles", "sdm_ssprk53_stages", "sdm_ssprk53_step",
           "sdm_ssprk53_step_noalloc", "sdm_background_profile"):
    getattr(_lib, _f).restype = C.c_int

EXPORTED = ("sdm_last_error", "sdm_version", "sdm_shell_sizes", "sdm_shell_build", "sdm_box_sizes",
            "sdm_box_build", "sdm_tables", "sdm_create", "sdm_destroy", "sdm_mesh_bind",
            "sdm_workspace_size", "sdm_residual", "sdm_rk_stage", "sdm_diagnostics",
            "sdm_profile_enable", "sdm_profile_read", "sdm_batch_workspace_size", "sdm_batch_stage",
            "sdm_workspace_traces", "sdm_rk_stage_volume", "sdm_rk_stage_finish", "sdm_sph_bins",
            "sdm_sph_profiles", "sdm_ssprk53_stages", "sdm_ssprk53_step", "sdm_ssprk53_step_noalloc",
            "sdm_background_profile")
KERNELS = ("traces", "volume", "volume_diag", "finish_residual", "finish_stage")


class SdmError(RuntimeError):
    pass


def _check(rc):
    if rc != SDM_OK:
        raise SdmError(f"status {rc}: {_lib.sdm_last_error().decode()}")


def _p(a):
    return C.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else C.c_void_p(a.data_ptr())


def make_params(ghost=None, import_q=None, import_v=None, **kw) -> Params:
    """sdm_params from keyword values; ghost / import_q / import_v are device
    tensors (or None) that must outlive the calls using the parameters."""
    p = Params()
    d = dict(gamma=5.0 / 3.0, Rgas=1.0, GM=0.0, Omega=0.0, nu=0.0, kappa=0.0, eta=0.0,
             kr_scale=0.0, kr_c0=0.0, kr_c1=0.0, kr_c2=0.0, kr_omega_per_r=0.0, c_h=0.0, glm_a=0.0,
             powell=0, wall_kind=(0, 0), wall_mag=(0, 0), wall_th=(0, 0), q_wall=(0.0, 0.0),
             T_wall=(0.0, 0.0))
    d.update(kw)
    for k, v in d.items():
        if k in ("wall_kind", "wall_mag", "wall_th"):
            arr = getattr(p, k)
            arr[0], arr[1] = int(v[0]), int(v[1])
        elif k in ("q_wall", "T_wall"):
            arr = getattr(p, k)
            arr[0], arr[1] = float(v[0]), float(v[1])
        elif k == "powell":
            p.powell = int(v)
        else:
            setattr(p, k, float(v))
    p.ghost = None if ghost is None else ghost.data_ptr()
    p.import_q = None if import_q is None else import_q.data_ptr()
    p.import_v = None if import_v is None else import_v.data_ptr()
    return p


@dataclasses.dataclass
class Mesh:
    """Host arrays of one mesh (layouts of include/sdmhd.h)."""
    p: int
    E: int
    NB: int
    x_sp: np.ndarray
    detJ: np.ndarray
    S_fp: np.ndarray
    Sj_sp: np.ndarray
    nbr: np.ndarray
    n_face: np.ndarray

    @property
    def N(self):
        return self.p + 1


def _alloc(p, E, NB):
    N = p + 1
    N3, NF = N ** 3, (N + 1) * N * N
    return Mesh(p, E, NB, np.zeros((E, 3, N3)), np.zeros((E, N3)), np.zeros((E, 3, 3, NF)),
                np.zeros((E, 3, 3, N3)), np.zeros((E, 6), dtype=np.int32), np.zeros((E, 6, 3, N * N)))


def shell(Nz: int, Nr: int, p: int, rb: float = 0.70, rt: float = 0.98) -> Mesh:
    E, NB = C.c_int64(), C.c_int64()
    _check(_lib.sdm_shell_sizes(Nz, Nr, C.byref(E), C.byref(NB)))
    m = _alloc(p, E.value, NB.value)
    _check(_lib.sdm_shell_build(Nz, Nr, p, rb, rt, _p(m.x_sp), _p(m.detJ), _p(m.S_fp), _p(m.Sj_sp),
                                _p(m.nbr), _p(m.n_face)))
    return m


def box(nx, ny, nz, p, L=(1.0, 1.0, 1.0), periodic=7, warp=0.0) -> Mesh:
    E, NB = C.c_int64(), C.c_int64()
    _check(_lib.sdm_box_sizes(nx, ny, nz, periodic, C.byref(E), C.byref(NB)))
    m = _alloc(p, E.value, NB.value)
    _check(_lib.sdm_box_build(nx, ny, nz, L[0], L[1], L[2], periodic, warp, p, _p(m.x_sp), _p(m.detJ),
                              _p(m.S_fp), _p(m.Sj_sp), _p(m.nbr), _p(m.n_face)))
    return m


@dataclasses.dataclass
class SphBins:
    """(r, theta) bins of a mesh's solution points (sdm_sph_bins): host order
    and offsets; device copies are made on first use by a Solver."""
    n_r: int
    n_th: int
    rb: float
    rt: float
    order: np.ndarray    # int32 [E N^3]
    offsets: np.ndarray  # int64 [n_r n_th + 1]
    _dev: tuple = None


def sph_bins(mesh: Mesh, n_r: int, n_th: int, rb: float = 0.70, rt: float = 0.98) -> SphBins:
    n = mesh.E * mesh.N ** 3
    order = np.zeros(n, dtype=np.int32)
    offsets = np.zeros(n_r * n_th + 1, dtype=np.int64)
    _check(_lib.sdm_sph_bins(mesh.E, mesh.p, _p(mesh.x_sp), rb, rt, n_r, n_th, _p(order), _p(offsets)))
    return SphBins(n_r, n_th, rb, rt, order, offsets)


def background_profile(r, GM=1.0, Rgas=1.0, gamma=5.0 / 3.0, rb=0.70, rt=0.98, rho_b=1.0, N_rho=3.0,
                       L=0.0, kappa=0.0, kr_scale=0.0, kr_c0=0.0, kr_c1=0.0, kr_c2=0.0, kr_omega_per_r=0.0,
                       flux_balanced=True):
    """(rho, p, T) of the initial background at radii r (sdm_background_profile):
    the flux-balanced profile, or the polytrope with flux_balanced=False."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    d = BackgroundDesc(GM, Rgas, gamma, rb, rt, rho_b, N_rho, L, kappa, kr_scale, kr_c0, kr_c1, kr_c2,
                       kr_omega_per_r, 1 if flux_balanced else 0)
    out = [np.empty_like(r) for _ in range(3)]
    _check(_lib.sdm_background_profile(C.byref(d), r.size, _p(r), *[_p(o) for o in out]))
    return tuple(out)


def face_point_map(N: int) -> np.ndarray:
    """[8][N^2]: for orientation code o, the neighbour's face-point index
    a' + N b' of this side's face point a + N b (the map of include/sdmhd.h)."""
    out = np.zeros((8, N * N), dtype=np.int64)
    for o in range(8):
        for b in range(N):
            for a in range(N):
                p, q = (b, a) if o & 4 else (a, b)
                a2 = N - 1 - p if o & 1 else p
                b2 = N - 1 - q if o & 2 else q
                out[o, a + N * b] = a2 + N * b2
    return out


@dataclasses.dataclass
class Shard:
    """One partition of a mesh, as one GPU of a split run holds it.

    mesh     the partition's own arrays; faces whose neighbour lies in another
             partition are boundary faces of group 3 (import faces)
    elems    [E_local] global index of each local element
    bface    [NB_local] global boundary-face index of each local boundary
             face, -1 for import faces (re-indexes ghost rows)
    imports  [n_imp][4] local boundary-face index, neighbour's global element,
             its face, orientation code: where each import face's data comes from
    """
    mesh: Mesh
    elems: np.ndarray
    bface: np.ndarray
    imports: np.ndarray


def make_shard(mesh: Mesh, elems) -> Shard:
    """The partition of `mesh` made of the (global) elements `elems`.  The
    metrics and face normals are the full mesh's rows, so the symmetric face
    normals of partition faces are those of the unsplit mesh."""
    elems = np.asarray(elems, dtype=np.int64)
    E = len(elems)
    loc = -np.ones(mesh.E, dtype=np.int64)
    loc[elems] = np.arange(E)
    nbr = np.zeros((E, 6), dtype=np.int32)
    bface, imports = [], []
    for le, ge in enumerate(elems):
        for f in range(6):
            code = int(mesh.nbr[ge, f])
            if code >= 0 and loc[code >> 6] >= 0:
                nbr[le, f] = (int(loc[code >> 6]) << 6) | (code & 63)
                continue
            bf = len(bface)
            if code >= 0:  # neighbour in another partition: import face
                group, gbf = 3, -1
                imports.append((bf, code >> 6, (code >> 3) & 7, code & 7))
            else:
                group, gbf = (-code - 1) & 3, (-code - 1) >> 2
            nbr[le, f] = -(1 + group + 4 * bf)
            bface.append(gbf)
    m = Mesh(mesh.p, E, len(bface), mesh.x_sp[elems].copy(), mesh.detJ[elems].copy(), mesh.S_fp[elems].copy(),
             mesh.Sj_sp[elems].copy(), nbr, mesh.n_face[elems].copy())
    return Shard(m, elems, np.asarray(bface, dtype=np.int64), np.asarray(imports, dtype=np.int64).reshape(-1, 4))


def gather_imports(shard: Shard, q_traces, v_traces):
    """Import buffers of a partition from the neighbours' workspace traces
    (torch tensors [E_global][6][9][N^2] and [E_global][6][7][N^2], e.g. the
    views of a run over the whole mesh): each import face gets its
    neighbour's trace and viscous flux in this face's point order."""
    import torch
    N2 = q_traces.shape[-1]
    pm = torch.as_tensor(face_point_map(shard.mesh.N), device=q_traces.device)
    imp = torch.as_tensor(shard.imports, device=q_traces.device)
    out_q = torch.zeros((shard.mesh.NB, 9, N2), dtype=q_traces.dtype, device=q_traces.device)
    out_v = torch.zeros((shard.mesh.NB, 7, N2), dtype=v_traces.dtype, device=v_traces.device)
    if len(imp):
        e, f, pts = imp[:, 1, None, None], imp[:, 2, None, None], pm[imp[:, 3]][:, None, :]
        out_q[imp[:, 0]] = q_traces[e, f, torch.arange(9, device=pm.device)[None, :, None], pts]
        out_v[imp[:, 0]] = v_traces[e, f, torch.arange(7, device=pm.device)[None, :, None], pts]
    return out_q, out_v


def tables(p: int):
    N = p + 1
    xs, xf, I, D, W = np.zeros(N), np.zeros(N + 1), np.zeros((N + 1, N)), np.zeros((N, N + 1)), np.zeros(N)
    _check(_lib.sdm_tables(p, _p(xs), _p(xf), _p(I), _p(D), _p(W)))
    return xs, xf, I, D, W


def ssp53_stages():
    """The five SSPRK(5,3) stages on four registers as the library defines
    them (sdm_ssprk53_stages): a list of (cur, [(input register, alpha)],
    beta, out)."""
    st = (Stage * 5)()
    _check(_lib.sdm_ssprk53_stages(st, None))
    return [(x.cur, [(x.in_idx[k], x.alpha[k]) for k in range(x.n_in)], x.beta, x.out) for x in st]


def ssp53_stage_times():
    """Time of each stage's input state in units of dt (sdm_ssprk53_stages)."""
    st = (Stage * 5)()
    c = (C.c_double * 5)()
    _check(_lib.sdm_ssprk53_stages(st, c))
    return list(c)


class Solver:
    """A device context with one bound mesh, four FP64 state registers and
    the workspace, all allocated through torch on the current device."""

    def __init__(self, mesh: Mesh, arith: int = 0, device: int = 0):
        import torch
        self.torch = torch
        self.mesh = mesh
        self.dev = torch.device("cuda", device)
        self.arith = arith
        h = C.c_void_p()
        _check(_lib.sdm_create(device, mesh.p, arith, C.byref(h)))
        self._h = h
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)  # noqa: E731
        self.x_sp, self.detJ, self.S_fp, self.nbr = t(mesh.x_sp), t(mesh.detJ), t(mesh.S_fp), t(mesh.nbr)
        self.n_face, self.Sj_sp = t(mesh.n_face), t(mesh.Sj_sp)
        md = MeshDesc(mesh.E, mesh.NB, self.x_sp.data_ptr(), self.detJ.data_ptr(), self.S_fp.data_ptr(),
                      self.Sj_sp.data_ptr(), self.nbr.data_ptr(), self.n_face.data_ptr())
        _check(_lib.sdm_mesh_bind(h, C.byref(md)))
        nb = C.c_size_t()
        _check(_lib.sdm_workspace_size(h, C.byref(nb)))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.dev)
        shp = (mesh.E, 9, mesh.N ** 3)
        self.regs = [torch.zeros(shp, dtype=torch.float64, device=self.dev) for _ in range(4)]
        self._traces_of = None  # register whose traces the workspace holds
        self.diag_out = torch.zeros(16, dtype=torch.float64, device=self.dev)

    def __del__(self):
        try:
            if self._h:
                _lib.sdm_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def trace_views(self):
        """(q_traces [E][6][9][N^2], v_traces [E][6][7][N^2]) as tensors viewing
        the workspace (residual arithmetic type): what this partition sends to
        its neighbours (sdm_workspace_traces)."""
        q, v = C.c_void_p(), C.c_void_p()
        _check(_lib.sdm_workspace_traces(self._h, self.ws.data_ptr(), C.byref(q), C.byref(v)))
        dt = self.torch.float64 if self.arith == 0 else self.torch.float32
        isz = 8 if self.arith == 0 else 4
        E, N2 = self.mesh.E, self.mesh.N ** 2
        base = self.ws.data_ptr()

        def view(ptr, nvar):
            off = ptr - base
            return self.ws[off:off + E * 6 * nvar * N2 * isz].view(dt).view(E, 6, nvar, N2)
        return view(q.value, 9), view(v.value, 7)

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.dev).cuda_stream)

    def set_state(self, Q):
        self.regs[0].copy_(self.torch.as_tensor(Q, dtype=self.torch.float64).to(self.dev))
        self._traces_of = None

    @property
    def state(self):
        return self.regs[0]

    def residual(self, prm: Params, Q=None, out=None):
        Q = self.regs[0] if Q is None else Q
        R = self.torch.empty_like(Q) if out is None else out
        _check(_lib.sdm_residual(self._h, C.byref(prm), Q.data_ptr(), R.data_ptr(), self.ws.data_ptr(),
                                 self._stream()))
        self._traces_of = None
        return R

    def stage(self, prm: Params, cur: int, inputs, beta: float, out: int, dt: float, regs=None, part="all"):
        """regs[out] = sum alpha regs[in] + beta dt R(regs[cur]).  part = "all"
        (sdm_rk_stage), or "volume" then "finish" (its two halves, with a
        halo exchange in between for a split mesh)."""
        regs = self.regs if regs is None else regs
        st = Stage()
        st.n_in = len(inputs)
        for k, (idx, al) in enumerate(inputs):
            st.in_idx[k] = idx
            st.alpha[k] = al
        st.cur, st.out, st.beta = cur, out, beta
        st.traces_valid = 1 if (self._traces_of == cur and regs is self.regs) else 0
        arr = (C.c_void_p * len(regs))(*[r.data_ptr() for r in regs])
        fn = {"all": _lib.sdm_rk_stage, "volume": _lib.sdm_rk_stage_volume, "finish": _lib.sdm_rk_stage_finish}[part]
        _check(fn(self._h, C.byref(prm), arr, len(regs), C.byref(st), dt, self.ws.data_ptr(), self._stream()))
        if part == "volume":
            self._traces_of = cur if regs is self.regs else None
        else:
            self._traces_of = out if regs is self.regs else None

    def step(self, prm: Params, dt: float):
        """One SSPRK(5,3) step of the state in register 0 (sdm_ssprk53_step)."""
        arr = (C.c_void_p * 4)(*[r.data_ptr() for r in self.regs[:4]])
        _check(_lib.sdm_ssprk53_step(self._h, C.byref(prm), arr, dt, 1 if self._traces_of == 0 else 0,
                                     self.ws.data_ptr(), self._stream()))
        self._traces_of = 0

    def step_noalloc(self, prm: Params, dt: float, regs=None):
        """One SSPRK(5,3) step of regs[0] with the library's static face-trace
        scratch instead of the workspace (sdm_ssprk53_step_noalloc)."""
        regs = self.regs if regs is None else regs
        arr = (C.c_void_p * 4)(*[r.data_ptr() for r in regs[:4]])
        _check(_lib.sdm_ssprk53_step_noalloc(self._h, C.byref(prm), arr, dt, self._stream()))
        if regs is self.regs:
            self._traces_of = None  # the workspace was not touched

    def profile(self, enable: bool):
        _check(_lib.sdm_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """{kernel: (total ms, launches)} of the launches since profile(True)."""
        ms = (C.c_double * 8)()
        cnt = (C.c_int64 * 8)()
        _check(_lib.sdm_profile_read(self._h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNELS) if cnt[i]}

    def sph_profiles(self, bins: SphBins, Q=None):
        """Per (r, theta) bin: sums of w, w V_phi, w V_mer, w (B_r^2 + B_theta^2)/2,
        w B_phi^2/2 over its solution points (sdm_sph_profiles), as a host
        array (n_r, n_th, 5)."""
        torch = self.torch
        Q = self.regs[0] if Q is None else Q
        if bins._dev is None or bins._dev[0] != self.dev:
            bins._dev = (self.dev, torch.from_numpy(bins.order).to(self.dev),
                         torch.from_numpy(bins.offsets).to(self.dev))
        nb = bins.n_r * bins.n_th
        out = torch.empty((nb, 5), dtype=torch.float64, device=self.dev)
        _check(_lib.sdm_sph_profiles(self._h, Q.data_ptr(), bins._dev[1].data_ptr(), bins._dev[2].data_ptr(),
                                     nb, out.data_ptr(), self._stream()))
        return out.cpu().numpy().reshape(bins.n_r, bins.n_th, 5)

    def diagnostics(self, prm: Params, Q=None):
        Q = self.regs[0] if Q is None else Q
        _check(_lib.sdm_diagnostics(self._h, C.byref(prm), Q.data_ptr(), self.diag_out.data_ptr(),
                                    self.ws.data_ptr(), self._stream()))
        self._traces_of = None
        return self.diag_out.cpu().numpy()
