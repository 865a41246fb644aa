"""FP64 CPU oracle of the explicit residual evaluation (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2609_07387_amd``) and does not import it: both consume the same
seeded input arrays and nothing else.

The C sources (``oracle_mesh.c``, ``oracle_solver.c``) follow the paper's
Sec. 2.2 step by step; this module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = ["oracle_mesh.c", "oracle_solver.c"]

QM = 16     # max quadrature points per face (4 x 4 at P4)
MAXF = 6    # max faces per cell
MAXMD = 32  # directional stencil stride
MAXC = 128  # central stencil cap


def build(verbose: bool = False, out: str | None = None, tuned: bool = False) -> str:
    """Compile the oracle with gcc and OpenMP.  The checker (default, into
    oracle/liboracle.so) is plain -O2 with no -march tuning and no FMA
    contraction, so its results do not depend on the host; tuned=True builds
    -O3 -march=native (for timing on the host that runs it) into `out`."""
    out = out or _LIB
    opt = ["-O3", "-march=native"] if tuned else ["-O2", "-ffp-contract=off"]
    cmd = ["gcc", *opt, "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", "-o", out]
    cmd += [os.path.join(_HERE, s) for s in _SRC] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


def use_library(path: str) -> None:
    """Load the oracle from another build of the same sources (e.g. a tuned
    build for timing); call before any other use of this module."""
    global _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _lib = C.CDLL(path)
    _declare(_lib)


class MeshIn(C.Structure):
    _fields_ = [
        ("n_vert", C.c_int64), ("xyz", C.c_void_p), ("n_cell", C.c_int64), ("type", C.c_void_p),
        ("cell_ptr", C.c_void_p), ("cell_vtx", C.c_void_p), ("period", C.c_double * 3),
        ("n_bface", C.c_int64), ("bface_ptr", C.c_void_p), ("bface_vtx", C.c_void_p), ("bface_tag", C.c_void_p),
    ]


class Opts(C.Structure):
    _fields_ = [("order", C.c_int), ("tri_qp", C.c_int), ("lambda_c", C.c_double), ("eps", C.c_double),
                ("max_layers", C.c_int), ("stencil_factor", C.c_double)]


class Phys(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mach", C.c_double), ("reynolds", C.c_double), ("prandtl", C.c_double),
                ("viscous", C.c_int), ("flux", C.c_int), ("grad", C.c_int)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int * 8), ("state", (C.c_double * 5) * 8)]


def _declare(L):
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
    L.oracle_last_error.restype = C.c_char_p
    L.oracle_build.argtypes = [C.POINTER(MeshIn), C.POINTER(Opts), vp, i32, C.POINTER(vp)]
    L.oracle_free.argtypes = [vp]
    L.oracle_free.restype = None
    L.oracle_info.argtypes = [vp, vp]
    L.oracle_cell_faces.argtypes = [vp, vp, vp]
    L.oracle_face_data.argtypes = [vp] * 8
    L.oracle_cell_data.argtypes = [vp] * 4
    L.oracle_stencil.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.oracle_operators.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.oracle_cell_quadrature.argtypes = [vp, i64, vp, vp, i32]
    L.oracle_reconstruct.argtypes = [vp, C.POINTER(Phys), vp, vp, vp, vp, vp]
    L.oracle_gradients.argtypes = [vp, C.POINTER(Phys), vp, vp, vp]
    L.oracle_gradients_lsq.argtypes = [vp, C.POINTER(Phys), vp, vp, vp]
    L.oracle_face_flux.argtypes = [vp, C.POINTER(Phys), vp, vp, vp, vp, vp]
    L.oracle_residual.argtypes = [vp, vp, vp]
    L.oracle_dt.argtypes = [vp, C.POINTER(Phys), vp, dbl, vp]
    L.oracle_rk_stage.argtypes = [vp, i32, dbl, vp, vp, vp]
    L.oracle_ssp54_stage.argtypes = [vp, i32, dbl, vp, vp, vp]
    L.oracle_run_ssp54.argtypes = [vp, C.POINTER(Phys), vp, vp, dbl, i32, vp, vp, vp]
    L.oracle_kinetic_energy.argtypes = [vp, vp, vp]
    L.oracle_dissipation.argtypes = [vp, C.POINTER(Phys), vp, vp, vp, vp]
    L.oracle_run.argtypes = [vp, C.POINTER(Phys), vp, vp, dbl, i32, vp, vp, vp]
    L.oracle_gate_features.argtypes = [vp, C.POINTER(Phys), vp, vp]
    L.oracle_point_flux.argtypes = [C.POINTER(Phys), vp, vp, vp, vp]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}: {lib().oracle_last_error().decode()}")


def phys(gamma=1.4, mach=0.1, reynolds=1600.0, prandtl=0.72, viscous=False, flux="hllc",
         gradients="green_gauss") -> Phys:
    if gradients not in ("green_gauss", "least_squares"):
        raise ValueError(f"gradients: {gradients!r}")
    return Phys(gamma, mach, reynolds, prandtl, int(bool(viscous)), 1 if flux == "hllc" else 0,
                1 if gradients == "least_squares" else 0)


def point_flux(ph, uL, uR, n):
    """Convective numerical flux of one state pair across unit normal n."""
    uL, uR, n = (np.ascontiguousarray(a, np.float64) for a in (uL, uR, n))
    F = np.zeros(5)
    _check(lib().oracle_point_flux(C.byref(ph), _p(uL), _p(uR), _p(n), _p(F)))
    return F


def bc(entries=None) -> BC:
    """entries: {tag: (kind, state5 or None)}; kinds 1 Dirichlet, 2 copy, 3 wall."""
    b = BC()
    for t, (kind, state) in (entries or {}).items():
        b.kind[t] = kind
        if state is not None:
            for v in range(5):
                b.state[t][v] = float(state[v])
    return b


class OracleMesh:
    """Oracle-side mesh: geometry, faces, stencils and operators built by the
    oracle's own code from the raw mesh arrays."""

    def __init__(self, mesh, order=2, need=None, lambda_c=1000.0, eps=1e-12, max_layers=3, stencil_factor=2.0):
        L = lib()
        self._keep = [np.ascontiguousarray(mesh.xyz, np.float64), np.ascontiguousarray(mesh.ctype, np.uint8),
                      np.ascontiguousarray(mesh.cell_ptr, np.int64), np.ascontiguousarray(mesh.cell_vtx, np.int64),
                      np.ascontiguousarray(mesh.bface_ptr, np.int64), np.ascontiguousarray(mesh.bface_vtx, np.int64),
                      np.ascontiguousarray(mesh.bface_tag, np.int32)]
        xyz, ty, cp, cv, bp, bv, bt = self._keep
        mi = MeshIn(xyz.shape[0], _p(xyz), ty.shape[0], _p(ty), _p(cp), _p(cv),
                    (C.c_double * 3)(*[float(x) for x in mesh.period]), bt.shape[0], _p(bp), _p(bv), _p(bt))
        op = Opts(order, 3, lambda_c, eps, max_layers, stencil_factor)
        self._need = None if need is None else np.ascontiguousarray(need, np.uint8)
        h = C.c_void_p()
        _check(L.oracle_build(C.byref(mi), C.byref(op), _p(self._need), 0, C.byref(h)))
        self.h = h
        info = np.zeros(11, np.int64)
        L.oracle_info(self.h, _p(info))
        (self.n_cell, self.n_face, self.K, self.nq_max, self.nfc_max, self.mc_max, self.md_max, self.mc_min,
         self.n_bnd, self.n_dropped, self.kd) = (int(x) for x in info)
        self.order = order

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_free(self.h)
            self.h = None

    # ---- mesh data
    def cell_faces(self):
        c2f = np.zeros((self.n_cell, MAXF), np.int64)
        side = np.zeros((self.n_cell, MAXF), np.int8)
        lib().oracle_cell_faces(self.h, _p(c2f), _p(side))
        return c2f, side

    def face_data(self):
        nf = self.n_face
        d = dict(cells=np.zeros((nf, 2), np.int64), nq=np.zeros(nf, np.int32), area=np.zeros(nf),
                 nrm=np.zeros((nf, 3)), qp=np.zeros((nf, QM, 3)), qw=np.zeros((nf, QM)), shift=np.zeros((nf, 3)))
        lib().oracle_face_data(self.h, *[_p(d[k]) for k in ("cells", "nq", "area", "nrm", "qp", "qw", "shift")])
        return d

    def cell_data(self):
        vol, cen, hb = np.zeros(self.n_cell), np.zeros((self.n_cell, 3)), np.zeros(self.n_cell)
        lib().oracle_cell_data(self.h, _p(vol), _p(cen), _p(hb))
        return vol, cen, hb

    def stencil(self, cell):
        cen = np.zeros(MAXC, np.int64)
        nce = np.zeros(1, np.int32)
        d = np.zeros((MAXF, MAXMD), np.int64)
        nd = np.zeros(MAXF, np.int32)
        df = np.zeros(MAXF, np.int32)
        rc = lib().oracle_stencil(self.h, int(cell), _p(cen), _p(nce), _p(d), _p(nd), _p(df))
        if rc < 0:
            _check(rc)
        return cen[:nce[0]].copy(), [d[s, :nd[s]].copy() for s in range(rc)], df[:rc].copy()

    def operators(self, cell):
        cen, dirs, _ = self.stencil(cell)
        K = self.K
        Bc = np.zeros((K, len(cen)))
        kd = self.kd
        Bd = np.zeros((MAXF, kd, MAXMD))
        O = np.zeros((K, K))
        Phi = np.zeros((MAXF, QM, K))
        mean = np.zeros(K)
        _check(lib().oracle_operators(self.h, int(cell), _p(Bc), _p(Bd), _p(O), _p(Phi), _p(mean)))
        Bd_list = [np.ascontiguousarray(Bd.reshape(-1)[s * kd * MAXMD: s * kd * MAXMD + kd * len(dirs[s])]
                                        .reshape(kd, len(dirs[s]))) for s in range(len(dirs))]
        return dict(Bc=Bc, Bd=Bd_list, O=O, Phi=Phi, mean=mean)

    def cell_quadrature(self, cell, cap=4000):
        x = np.zeros((cap, 3))
        w = np.zeros(cap)
        n = lib().oracle_cell_quadrature(self.h, int(cell), _p(x), _p(w), cap)
        if n < 0:
            raise RuntimeError("quadrature capacity")
        return x[:n].copy(), w[:n].copy()

    # ---- solver steps
    def reconstruct(self, U, ph, gate_mask=None, with_flags=False):
        U = np.ascontiguousarray(U, np.float64)
        fs = np.full((self.n_face, 2, QM, 5), np.nan)
        flags = np.zeros(self.n_cell, np.uint8)
        label = np.zeros(self.n_cell)
        gm = None if gate_mask is None else np.ascontiguousarray(gate_mask, np.uint8)
        _check(lib().oracle_reconstruct(self.h, C.byref(ph), _p(U), _p(gm), _p(fs), _p(flags), _p(label)))
        return (fs, flags, label) if with_flags else fs

    def gradients(self, U, ph, bcs=None):
        """Cell gradients of (u, v, w, T) by the method ph.grad selects."""
        U = np.ascontiguousarray(U, np.float64)
        g = np.zeros((12, self.n_cell))
        fn = lib().oracle_gradients_lsq if ph.grad == 1 else lib().oracle_gradients
        _check(fn(self.h, C.byref(ph), None if bcs is None else C.byref(bcs), _p(U), _p(g)))
        return g

    def face_flux(self, U, fs, ph, gradW=None, bcs=None):
        ff = np.zeros((self.n_face, 5))
        gw = None if gradW is None else np.ascontiguousarray(gradW)
        _check(lib().oracle_face_flux(self.h, C.byref(ph), None if bcs is None else C.byref(bcs),
                                      _p(np.ascontiguousarray(U, np.float64)), _p(np.ascontiguousarray(fs)),
                                      _p(gw), _p(ff)))
        return ff

    def residual(self, ff):
        R = np.zeros((5, self.n_cell))
        _check(lib().oracle_residual(self.h, _p(np.ascontiguousarray(ff)), _p(R)))
        return R

    def dt(self, U, ph, cfl):
        out = np.zeros(1)
        _check(lib().oracle_dt(self.h, C.byref(ph), _p(np.ascontiguousarray(U)), float(cfl), _p(out)))
        return float(out[0])

    def rk_stage(self, stage, dt, U0, R, U):
        _check(lib().oracle_rk_stage(self.h, int(stage), float(dt), _p(U0), _p(R), _p(U)))

    def ssp54_stage(self, stage, dt, W, R, U):
        _check(lib().oracle_ssp54_stage(self.h, int(stage), float(dt), _p(W), _p(R), _p(U)))

    def rhs(self, U, ph, bcs=None, gate_mask=None):
        fs = self.reconstruct(U, ph, gate_mask)
        g = self.gradients(U, ph, bcs) if ph.viscous else None
        ff = self.face_flux(U, fs, ph, g, bcs)
        return self.residual(ff)

    def kinetic_energy(self, U):
        out = np.zeros(1)
        lib().oracle_kinetic_energy(self.h, _p(np.ascontiguousarray(U)), _p(out))
        return float(out[0])

    def dissipation(self, U, ph, bcs=None):
        a, b = np.zeros(1), np.zeros(1)
        lib().oracle_dissipation(self.h, C.byref(ph), None if bcs is None else C.byref(bcs),
                                 _p(np.ascontiguousarray(U)), _p(a), _p(b))
        return float(a[0]), float(b[0])

    def run(self, U, ph, cfl, n_steps, bcs=None, gate_mask=None, integrator="ssp3"):
        """n_steps SSP-RK3 (or, integrator="ssp54", five-stage fourth-order
        SSP-RK) steps; returns (U_new, ke_history, dt_history)."""
        U = np.array(U, np.float64, order="C", copy=True)
        ke = np.zeros(n_steps + 1)
        dts = np.zeros(max(n_steps, 1))
        gm = None if gate_mask is None else np.ascontiguousarray(gate_mask, np.uint8)
        fn = lib().oracle_run_ssp54 if integrator == "ssp54" else lib().oracle_run
        _check(fn(self.h, C.byref(ph), None if bcs is None else C.byref(bcs), _p(U), float(cfl),
                  int(n_steps), _p(gm), _p(ke), _p(dts)))
        return U, ke, dts[:n_steps]

    def gate_features(self, U, ph):
        f = np.zeros((self.n_cell, 12))
        _check(lib().oracle_gate_features(self.h, C.byref(ph), _p(np.ascontiguousarray(U)), _p(f)))
        return f
