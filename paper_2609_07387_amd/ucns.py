"""Thin Python binding of libucns (argument marshalling only).

Every step of the residual evaluation runs in the library's HIP kernels;
PyTorch only provides device memory and the stream.  The names follow the C
ABI in ``include/ucns.h``.  Importing this module does not need a GPU; the
compute calls do, and they fail loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libucns.so")

F64, F32 = 0, 1
RUSANOV, HLLC = 0, 1
GRADIENTS = {"green_gauss": 0, "least_squares": 1}  # ucns_phys.grad
BC_NONE, BC_DIRICHLET, BC_TRANSMISSIVE, BC_WALL, BC_SYMMETRY = 0, 1, 2, 3, 4
MAX_FACES, MAX_DIR, MAX_CENTRAL = 6, 32, 128

# Names declared in include/ucns.h (checked by the test-suite against the
# library's exports).
EXPORTS = [
    "ucns_last_error", "ucns_mesh_build", "ucns_mesh_free", "ucns_mesh_info", "ucns_mesh_arena_bytes",
    "ucns_mesh_upload", "ucns_mesh_faces", "ucns_mesh_cell_geometry", "ucns_mesh_stencil", "ucns_mesh_operators",
    "ucns_workspace_elems", "ucns_dt", "ucns_reconstruct", "ucns_gradients", "ucns_face_flux", "ucns_residual",
    "ucns_rk_stage", "ucns_residual_rk_stage", "ucns_diag_ke", "ucns_gate_features", "ucns_mlp_forward",
    "ucns_gate_mask", "ucns_mlp_train_step", "ucns_mlp_pack", "ucns_residual_rk_final",
    "ucns_residual_ssp54_stage", "ucns_mesh_gradient_weights", "ucns_recon_span_bytes",
    "ucns_check", "ucns_residual_rk_final_noalloc", "ucns_mesh_release", "ucns_diag_dissipation",
    "ucns_reconstruct_gradients",
]


class MeshDesc(C.Structure):
    _fields_ = [
        ("n_vert", C.c_int64), ("xyz", C.c_void_p), ("n_cell", C.c_int64), ("type", C.c_void_p),
        ("cell_ptr", C.c_void_p), ("cell_vtx", C.c_void_p), ("period", C.c_double * 3),
        ("n_bface", C.c_int64), ("bface_ptr", C.c_void_p), ("bface_vtx", C.c_void_p), ("bface_tag", C.c_void_p),
    ]


class ReconOpts(C.Structure):
    _fields_ = [("order", C.c_int), ("lambda_c", C.c_double), ("eps", C.c_double), ("max_layers", C.c_int),
                ("stencil_factor", C.c_double)]


class Phys(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mach", C.c_double), ("reynolds", C.c_double), ("prandtl", C.c_double),
                ("viscous", C.c_int), ("flux", C.c_int), ("grad", C.c_int)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int * 8), ("state", (C.c_double * 5) * 8)]


class Gate(C.Structure):
    _fields_ = [("mask", C.c_void_p), ("mlp_image", C.c_void_p), ("mask_out", C.c_void_p)]


# gate network parameter block (float32) offsets, as in include/ucns.h
MLP_OFF = {"mu": 0, "isig": 16, "W1": 32, "b1": 1056, "W2": 1120, "b2": 5216, "w3": 5280, "b3": 5344, "theta": 5345}
MLP_NPARAM = 5348
MLP_IMAGE_BYTES = 13312


_lib = None


def lib():
    """The loaded libucns (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libucns.so not found at {LIB_PATH}; build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dbl, flt = C.c_void_p, C.c_int64, C.c_int, C.c_double, C.c_float
        L.ucns_last_error.restype = C.c_char_p
        L.ucns_mesh_build.argtypes = [C.POINTER(MeshDesc), C.POINTER(ReconOpts), i32, C.POINTER(vp)]
        L.ucns_mesh_free.argtypes = [vp]
        L.ucns_mesh_free.restype = None
        L.ucns_mesh_info.argtypes = [vp, vp]
        L.ucns_mesh_arena_bytes.argtypes = [vp, i32, C.POINTER(C.c_size_t)]
        L.ucns_mesh_upload.argtypes = [vp, i32, vp, C.c_size_t, vp]
        L.ucns_mesh_release.argtypes = [vp, i32]
        L.ucns_mesh_faces.argtypes = [vp, vp, vp, vp, vp]
        L.ucns_mesh_cell_geometry.argtypes = [vp, vp, vp, vp]
        L.ucns_mesh_stencil.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.ucns_mesh_operators.argtypes = [vp, i64, vp, vp, vp, vp]
        L.ucns_mesh_gradient_weights.argtypes = [vp, i64, vp]
        L.ucns_workspace_elems.argtypes = [vp, vp, vp, vp, vp]
        L.ucns_recon_span_bytes.argtypes = [i64, i32, i32, i32, C.POINTER(C.c_uint64)]
        L.ucns_check.argtypes = [vp, vp]
        L.ucns_residual_rk_final_noalloc.argtypes = [vp, C.POINTER(Phys), vp, i32, vp, vp, vp, dbl, vp, vp, vp]
        L.ucns_dt.argtypes = [vp, C.POINTER(Phys), vp, dbl, vp, vp, vp]
        L.ucns_reconstruct.argtypes = [vp, C.POINTER(Phys), vp, i32, vp, vp, vp, vp, vp]
        L.ucns_gradients.argtypes = [vp, C.POINTER(Phys), vp, vp, i32, vp, vp]
        L.ucns_reconstruct_gradients.argtypes = [vp, C.POINTER(Phys), vp, vp, i32, vp, vp, vp, vp, vp]
        L.ucns_face_flux.argtypes = [vp, C.POINTER(Phys), vp, vp, vp, vp, i32, vp, vp]
        L.ucns_residual.argtypes = [vp, vp, i32, vp, vp]
        L.ucns_rk_stage.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.ucns_residual_rk_stage.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp]
        L.ucns_diag_ke.argtypes = [vp, vp, vp, vp, vp]
        L.ucns_diag_dissipation.argtypes = [vp, C.POINTER(Phys), vp, i32, vp, vp, vp]
        L.ucns_residual_ssp54_stage.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp]
        L.ucns_residual_rk_final.argtypes = [vp, C.POINTER(Phys), vp, i32, vp, vp, vp, dbl, vp, vp, vp, vp]
        L.ucns_gate_features.argtypes = [vp, vp, i32, vp, vp]
        L.ucns_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.ucns_gate_mask.argtypes = [vp, vp, i64, vp, vp]
        L.ucns_mlp_pack.argtypes = [vp, vp, vp]
        L.ucns_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, i64, flt, flt, i32, vp, vp]
        _lib = L
    return _lib


class UcnsError(RuntimeError):
    pass


def check(rc):
    if rc != 0:
        raise UcnsError(f"libucns error {rc}: {lib().ucns_last_error().decode()}")


def _np(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _dp(t):
    """Device pointer of a torch tensor (or None)."""
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def phys(gamma=1.4, mach=0.1, reynolds=1600.0, prandtl=0.72, viscous=False, flux="hllc",
         gradients="green_gauss") -> Phys:
    """gradients: "green_gauss" or "least_squares" (the viscous cell gradients)."""
    if gradients not in GRADIENTS:
        raise ValueError(f"gradients: {gradients!r}")
    return Phys(gamma, mach, reynolds, prandtl, int(bool(viscous)), HLLC if flux == "hllc" else RUSANOV,
                GRADIENTS[gradients])


def bc(entries=None) -> BC:
    """entries: {tag: (kind, state5 or None)}."""
    b = BC()
    for t in range(8):
        b.kind[t] = BC_TRANSMISSIVE
    for t, (kind, state) in (entries or {}).items():
        b.kind[t] = kind
        if state is not None:
            for v in range(5):
                b.state[t][v] = float(state[v])
    return b


class Mesh:
    """Library mesh handle (host build) plus its device arenas."""

    def __init__(self, mesh, order=2, lambda_c=1000.0, eps=1e-12, max_layers=3, n_threads=0, stencil_factor=2.0):
        L = lib()
        self._keep = [np.ascontiguousarray(mesh.xyz, np.float64), np.ascontiguousarray(mesh.ctype, np.uint8),
                      np.ascontiguousarray(mesh.cell_ptr, np.int64), np.ascontiguousarray(mesh.cell_vtx, np.int64),
                      np.ascontiguousarray(mesh.bface_ptr, np.int64), np.ascontiguousarray(mesh.bface_vtx, np.int64),
                      np.ascontiguousarray(mesh.bface_tag, np.int32)]
        xyz, ty, cp, cv, bp, bv, bt = self._keep
        d = MeshDesc(xyz.shape[0], _np(xyz), ty.shape[0], _np(ty), _np(cp), _np(cv),
                     (C.c_double * 3)(*[float(x) for x in mesh.period]), bt.shape[0], _np(bp), _np(bv), _np(bt))
        o = ReconOpts(order, lambda_c, eps, max_layers, stencil_factor)
        h = C.c_void_p()
        check(L.ucns_mesh_build(C.byref(d), C.byref(o), int(n_threads), C.byref(h)))
        self.h = h
        self._keep = None
        info = np.zeros(16, np.int64)
        check(L.ucns_mesh_info(self.h, _np(info)))
        (self.n_cell, self.n_face, self.K, self.qmax, self.nfmax, self.mc_pad, self.nd_max, self.md_pad,
         self.n_bnd, self.n_dropped, self.mc_min, _, self.order, self.kd) = (int(x) for x in info[:14])
        fs, ff, gw, rs = (np.zeros(1, np.int64) for _ in range(4))
        check(L.ucns_workspace_elems(self.h, _np(fs), _np(ff), _np(gw), _np(rs)))
        self.n_face_state, self.n_face_flux, self.n_grad, self.n_reduce = int(fs[0]), int(ff[0]), int(gw[0]), int(rs[0])
        self.arenas = {}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ucns_mesh_free(self.h)
            self.h = None

    # ---- host inspection
    def arena_bytes(self, precision):
        n = C.c_size_t()
        check(lib().ucns_mesh_arena_bytes(self.h, precision, C.byref(n)))
        return int(n.value)

    def faces(self):
        c2f = np.zeros((self.n_cell, MAX_FACES), np.int32)
        fcell = np.zeros((self.n_face, 2), np.int64)
        qp = np.zeros((self.n_face, self.qmax, 3))
        shift = np.zeros((self.n_face, 3))
        check(lib().ucns_mesh_faces(self.h, _np(c2f), _np(fcell), _np(qp), _np(shift)))
        return c2f, fcell, qp, shift

    def cell_geometry(self):
        vol, cen, hb = np.zeros(self.n_cell), np.zeros((self.n_cell, 3)), np.zeros(self.n_cell)
        check(lib().ucns_mesh_cell_geometry(self.h, _np(vol), _np(cen), _np(hb)))
        return vol, cen, hb

    def stencil(self, cell):
        cen = np.zeros(MAX_CENTRAL, np.int64)
        n = np.zeros(1, np.int32)
        d = np.zeros((MAX_FACES, MAX_DIR), np.int64)
        nd = np.zeros(MAX_FACES, np.int32)
        df = np.zeros(MAX_FACES, np.int32)
        rc = lib().ucns_mesh_stencil(self.h, int(cell), _np(cen), _np(n), _np(d), _np(nd), _np(df))
        if rc < 0:
            check(rc)
        return cen[:n[0]].copy(), [d[s, :nd[s]].copy() for s in range(rc)], df[:rc].copy()

    def operators(self, cell):
        cen, dirs, _ = self.stencil(cell)
        K = self.K
        Bc = np.zeros((K, len(cen)))
        Bd = np.zeros((MAX_FACES, self.kd, MAX_DIR))
        O = np.zeros((K, K))
        Phi = np.zeros((self.nfmax, self.qmax, K))
        check(lib().ucns_mesh_operators(self.h, int(cell), _np(Bc), _np(Bd), _np(O), _np(Phi)))
        return dict(Bc=Bc, Bd=[Bd[s, :, :len(dirs[s])].copy() for s in range(len(dirs))], O=O, Phi=Phi)

    def gradient_weights(self, cell):
        """Least-squares gradient weights G[6][3] of one cell by local face slot."""
        G = np.zeros((MAX_FACES, 3))
        check(lib().ucns_mesh_gradient_weights(self.h, int(cell), _np(G)))
        return G

    # ---- device
    def upload(self, precision, device="cuda"):
        import torch

        nbytes = self.arena_bytes(precision)
        arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        check(lib().ucns_mesh_upload(self.h, precision, _dp(arena), nbytes, _stream()))
        self.arenas[precision] = arena
        return arena

    def release(self, precision=None):
        """Forget the device arena of one precision (both if None) in the
        library, then drop it (the library must never keep a freed arena)."""
        for p in ([F64, F32] if precision is None else [precision]):
            check(lib().ucns_mesh_release(self.h, p))
            self.arenas.pop(p, None)


def _t(precision):
    import torch

    return torch.float64 if precision == F64 else torch.float32


class Workspace:
    """Caller-owned device workspaces of one precision."""

    def __init__(self, mesh: Mesh, precision, viscous, device="cuda"):
        import torch

        dt = _t(precision)
        self.face_state = torch.empty(mesh.n_face_state, dtype=dt, device=device)
        self.face_flux = torch.empty(mesh.n_face_flux, dtype=dt, device=device)
        self.gradW = torch.empty(mesh.n_grad, dtype=dt, device=device) if viscous else None
        self.reduce = torch.empty(mesh.n_reduce, dtype=torch.float64, device=device)
        self.flags = torch.zeros(mesh.n_cell, dtype=torch.uint8, device=device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        self.ke = torch.zeros(1, dtype=torch.float64, device=device)
        self.U0 = None
        self.R = None


# ------------------------------------------------------------ entry points

def recon_span_bytes(n_cell, precision, n_unknowns, n_face_slots):
    """Largest byte span of one reconstruction buffer descriptor (host query)."""
    out = C.c_uint64()
    check(lib().ucns_recon_span_bytes(int(n_cell), int(precision), int(n_unknowns), int(n_face_slots),
                                      C.byref(out)))
    return int(out.value)


def dt(mesh, ph, U, cfl, scratch, dt_dev, stream=None):
    check(lib().ucns_dt(mesh.h, C.byref(ph), _dp(U), float(cfl), _dp(scratch), _dp(dt_dev), _stream(stream)))


def mlp_pack(params, image=None, stream=None):
    """Packed network image (uint8 [MLP_IMAGE_BYTES]) of a parameter block."""
    import torch

    if image is None:
        image = torch.empty(MLP_IMAGE_BYTES, dtype=torch.uint8, device=params.device)
    check(lib().ucns_mlp_pack(_dp(params), _dp(image), _stream(stream)))
    return image


def reconstruct(mesh, ph, U, precision, face_state, gate_mask=None, flags=None, label=None, stream=None,
                mlp_image=None, mask_out=None):
    """gate_mask (uint8, 1 = smooth) or mlp_image (see mlp_pack) selects the gate."""
    g = None
    if gate_mask is not None or mlp_image is not None:
        g = Gate(None if gate_mask is None else C.c_void_p(gate_mask.data_ptr()),
                 None if mlp_image is None else C.c_void_p(mlp_image.data_ptr()),
                 None if mask_out is None else C.c_void_p(mask_out.data_ptr()))
    check(lib().ucns_reconstruct(mesh.h, C.byref(ph), _dp(U), precision, None if g is None else C.byref(g),
                                 _dp(face_state), _dp(flags), _dp(label), _stream(stream)))


def bc_device(bcs, device="cuda"):
    """A boundary table (BC, or None for all transmissive) copied to device
    memory, for reconstruct_gradients."""
    import torch

    b = bc() if bcs is None else bcs
    raw = torch.frombuffer(bytearray(bytes(b)), dtype=torch.uint8)
    return raw.to(device)


def reconstruct_gradients(mesh, ph, bc_dev, U, precision, face_state, flags, gradW, gate_mask=None, mlp_image=None,
                          mask_out=None, stream=None):
    """reconstruct() and the gradients() of the same U in one pass (order 2,
    either gradient method); bc_dev from bc_device()."""
    g = None
    if gate_mask is not None or mlp_image is not None:
        g = Gate(None if gate_mask is None else C.c_void_p(gate_mask.data_ptr()),
                 None if mlp_image is None else C.c_void_p(mlp_image.data_ptr()),
                 None if mask_out is None else C.c_void_p(mask_out.data_ptr()))
    check(lib().ucns_reconstruct_gradients(mesh.h, C.byref(ph), _dp(bc_dev), _dp(U), precision,
                                           None if g is None else C.byref(g), _dp(face_state), _dp(flags),
                                           _dp(gradW), _stream(stream)))


def gate_features(mesh, U, precision, out, stream=None):
    check(lib().ucns_gate_features(mesh.h, _dp(U), precision, _dp(out), _stream(stream)))


def mlp_forward(params, feats, prob, stream=None):
    check(lib().ucns_mlp_forward(_dp(params), _dp(feats), int(feats.shape[0]), _dp(prob), _stream(stream)))


def gate_mask(params, feats, mask, stream=None):
    check(lib().ucns_gate_mask(_dp(params), _dp(feats), int(feats.shape[0]), _dp(mask), _stream(stream)))


def mlp_train_step(params, grads, adam_state, feats, labels, pos_weight, lr, t, loss, stream=None):
    check(lib().ucns_mlp_train_step(_dp(params), _dp(grads), _dp(adam_state), _dp(feats), _dp(labels),
                                    int(feats.shape[0]), float(pos_weight), float(lr), int(t), _dp(loss),
                                    _stream(stream)))


def gradients(mesh, ph, bcs, U, precision, gradW, stream=None):
    check(lib().ucns_gradients(mesh.h, C.byref(ph), None if bcs is None else C.byref(bcs), _dp(U), precision,
                               _dp(gradW), _stream(stream)))


def face_flux(mesh, ph, bcs, U, face_state, gradW, precision, ff, stream=None):
    check(lib().ucns_face_flux(mesh.h, C.byref(ph), None if bcs is None else C.byref(bcs), _dp(U), _dp(face_state),
                               _dp(gradW), precision, _dp(ff), _stream(stream)))


def residual(mesh, ff, precision, R, stream=None):
    check(lib().ucns_residual(mesh.h, _dp(ff), precision, _dp(R), _stream(stream)))


def rk_stage(mesh, stage, dt_dev, U0, R, U, stream=None):
    check(lib().ucns_rk_stage(mesh.h, int(stage), _dp(dt_dev), _dp(U0), _dp(R), _dp(U), _stream(stream)))


def residual_rk_stage(mesh, ff, precision, stage, dt_dev, U0, U, stream=None):
    check(lib().ucns_residual_rk_stage(mesh.h, _dp(ff), precision, int(stage), _dp(dt_dev), _dp(U0), _dp(U),
                                       _stream(stream)))


def residual_rk_final(mesh, ph, ff, precision, dt_dev, U0, U, cfl, scratch, dt_next, ke_dev, stream=None):
    """Last RK stage with the next step's dt and the new state's kinetic energy."""
    check(lib().ucns_residual_rk_final(mesh.h, C.byref(ph), _dp(ff), precision, _dp(dt_dev), _dp(U0), _dp(U),
                                       float(cfl), _dp(scratch), _dp(dt_next), _dp(ke_dev), _stream(stream)))


def residual_rk_final_noalloc(mesh, ph, ff, precision, dt_dev, U0, U, cfl, dt_next, ke_dev, stream=None):
    """residual_rk_final with the library's static reduction scratch (no workspace)."""
    check(lib().ucns_residual_rk_final_noalloc(mesh.h, C.byref(ph), _dp(ff), precision, _dp(dt_dev), _dp(U0),
                                               _dp(U), float(cfl), _dp(dt_next), _dp(ke_dev), _stream(stream)))


def residual_ssp54_stage(mesh, ff, precision, stage, dt_dev, W, U, stream=None):
    """Residual fused with stage 0..4 of the five-stage fourth-order SSP-RK;
    W (float64 [4][5][n_cell]) carries the stage states between calls."""
    check(lib().ucns_residual_ssp54_stage(mesh.h, _dp(ff), precision, int(stage), _dp(dt_dev), _dp(W), _dp(U),
                                          _stream(stream)))


def check_state(dt_dev, stream=None):
    """Raises UcnsError (code UCNS_ENUM = -7) when the device time step is
    NaN, infinite or not positive, i.e. the state has gone bad (synchronous)."""
    check(lib().ucns_check(_dp(dt_dev), _stream(stream)))


def diag_ke(mesh, U, scratch, ke_dev, stream=None):
    check(lib().ucns_diag_ke(mesh.h, _dp(U), _dp(scratch), _dp(ke_dev), _stream(stream)))


def diag_dissipation(mesh, ph, gradW, precision, scratch, eps_dev, stream=None):
    """eps_dev (device double [2]) <- (solenoidal, dilatational) dissipation
    from the cell gradients gradW of a preceding gradients() call."""
    check(lib().ucns_diag_dissipation(mesh.h, C.byref(ph), _dp(gradW), precision, _dp(scratch), _dp(eps_dev),
                                      _stream(stream)))


class Solver:
    """SSP-RK3 driver over the C-ABI calls (one stream, no host syncs)."""

    def __init__(self, mesh: Mesh, ph: Phys, precision=F64, bcs=None, cfl=0.5, gate_mask=None, device="cuda",
                 mlp=None, label=False, integrator="ssp3"):
        """gate_mask: fixed per-cell mask (1 = smooth); mlp: gate network
        parameters (device float32) evaluated inside every reconstruction;
        label: also record max |omega - lambda| per cell (ws.label);
        integrator: "ssp3" (Shu-Osher SSP-RK3) or "ssp54" (five-stage
        fourth-order SSP-RK)."""
        import torch

        self.mesh, self.ph, self.precision, self.bcs, self.cfl = mesh, ph, precision, bcs, cfl
        if precision not in mesh.arenas:
            mesh.upload(precision, device)
        self.ws = Workspace(mesh, precision, bool(ph.viscous), device)
        self.ws.label = torch.zeros(mesh.n_cell, dtype=torch.float32, device=device) if label else None
        self.ws.mask_out = torch.zeros(mesh.n_cell, dtype=torch.uint8, device=device) if mlp is not None else None
        self.U0 = torch.empty((5, mesh.n_cell), dtype=torch.float64, device=device)
        self.gate_mask = gate_mask
        self.mlp = mlp
        self.mlp_image = mlp_pack(mlp) if mlp is not None else None
        self._dt_key = None  # (data pointer, version) of the U whose dt ws.dt holds
        assert integrator in ("ssp3", "ssp54"), integrator
        self.integrator = integrator
        self.W = (torch.empty((4, 5, mesh.n_cell), dtype=torch.float64, device=device)
                  if integrator == "ssp54" else None)
        # viscous P2: one pass forms the point states and the gradients (the
        # boundary table then lives on the device)
        self.fused = bool(ph.viscous) and mesh.order == 2 and not label
        self.bc_dev = bc_device(bcs, device) if self.fused else None
        # a list here collects, for every reconstruction call, a (start, end)
        # HIP-event pair recorded on the launch stream and, with the network,
        # the call's count of cells taken as smooth (a device scalar); timing only
        self.recon_events = None

    def rhs_stage(self, U):
        ws = self.ws
        ev = self.recon_events
        if ev is not None:
            import torch

            s = torch.cuda.current_stream()
            ev.append([torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True), None])
            ev[-1][0].record(s)
        if self.fused:
            reconstruct_gradients(self.mesh, self.ph, self.bc_dev, U, self.precision, ws.face_state, ws.flags,
                                  ws.gradW, self.gate_mask, mlp_image=self.mlp_image, mask_out=ws.mask_out)
        else:
            reconstruct(self.mesh, self.ph, U, self.precision, ws.face_state, self.gate_mask, ws.flags, ws.label,
                        mlp_image=self.mlp_image, mask_out=ws.mask_out)
        if ev is not None:
            ev[-1][1].record(s)
            if ws.mask_out is not None:
                ev[-1][2] = ws.mask_out.sum()
        if self.ph.viscous and not self.fused:
            gradients(self.mesh, self.ph, self.bcs, U, self.precision, ws.gradW)
        face_flux(self.mesh, self.ph, self.bcs, U, ws.face_state, ws.gradW, self.precision, ws.face_flux)

    def ensure_dt(self, U):
        """ws.dt = the time step of U (kept from the previous step when valid)."""
        if self._dt_key != (U.data_ptr(), U._version):
            dt(self.mesh, self.ph, U, self.cfl, self.ws.reduce, self.ws.dt)
            self._dt_key = (U.data_ptr(), U._version)

    def step(self, U, ke=False):
        """One SSP-RK3 step of U in place.  The last stage also leaves the
        next step's dt in ws.dt and the kinetic energy of the new U in ws.ke
        (whatever ke says), so a step that follows on the same, unmodified U
        skips its own dt pass (a change to U through torch bumps its version
        and forces one)."""
        ws = self.ws
        self.ensure_dt(U)
        if self.integrator == "ssp54":
            for s in range(5):
                self.rhs_stage(U)
                residual_ssp54_stage(self.mesh, ws.face_flux, self.precision, s, ws.dt, self.W, U)
            diag_ke(self.mesh, U, ws.reduce, ws.ke)
            self._dt_key = None  # the next step takes its own dt pass
            return
        self._step_ssp3(U)
        self._dt_key = (U.data_ptr(), U._version)

    def _step_ssp3(self, U):
        """The three stages; the last also leaves the next dt and the kinetic
        energy in ws.dt and ws.ke (launches only: no host logic that a graph
        capture would freeze)."""
        ws = self.ws
        for s in range(2):  # stage 0 stores U^n into U0
            self.rhs_stage(U)
            residual_rk_stage(self.mesh, ws.face_flux, self.precision, s, ws.dt, self.U0, U)
        self.rhs_stage(U)
        residual_rk_final(self.mesh, self.ph, ws.face_flux, self.precision, ws.dt, self.U0, U, self.cfl, ws.reduce,
                          ws.dt, ws.ke)

    def check(self):
        """Raises UcnsError if the last computed time step flags a NaN/Inf or
        non-positive state (one host round trip)."""
        check_state(self.ws.dt)

    def dissipation(self, U, eps_dev=None):
        """Device double [2]: solenoidal and dilatational dissipation of U
        (cell gradients by the solver's gradient method, then the reduction);
        stays on the device."""
        import torch

        if eps_dev is None:
            eps_dev = torch.empty(2, dtype=torch.float64, device=U.device)
        gw = self.ws.gradW
        if gw is None:
            gw = self.ws.gradW = torch.empty(self.mesh.n_grad, dtype=_t(self.precision), device=U.device)
        gradients(self.mesh, self.ph, self.bcs, U, self.precision, gw)
        diag_dissipation(self.mesh, self.ph, gw, self.precision, self.ws.reduce, eps_dev)
        return eps_dev

    def capture(self, U):
        """Records one SSP-RK3 step of U (this tensor, in place) as a HIP
        graph: the same library calls on the capture stream, replayed by
        step_graph() with one launch.  The step reads the time step the
        previous step's last stage left in ws.dt, so U must be the state the
        solver last stepped (or one whose dt was just computed); capture
        itself runs no kernel.  SSP-RK3 only; no reconstruction timing
        events inside the graph."""
        import torch

        assert self.integrator == "ssp3" and self.recon_events is None
        self.ensure_dt(U)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            self._step_ssp3(U)
        torch.cuda.current_stream().wait_stream(side)
        self._graph, self._graph_U = g, U
        return g

    def step_graph(self, U):
        """One step by replaying the captured graph (same U tensor)."""
        assert U is self._graph_U, "the graph steps the tensor it was captured with"
        self._graph.replay()
        self._dt_key = (U.data_ptr(), U._version)

    def run(self, U, n_steps, ke_history=False, check_every=0):
        """n_steps steps of U in place; with check_every > 0 the state is
        checked (check()) every that many steps, and always at the end."""
        import torch

        hist, dts = [], []
        if ke_history:
            diag_ke(self.mesh, U, self.ws.reduce, self.ws.ke)
            hist.append(self.ws.ke.clone())
        for i in range(n_steps):
            if ke_history:
                self.ensure_dt(U)
                dts.append(self.ws.dt.clone())
            self.step(U)
            if ke_history:
                hist.append(self.ws.ke.clone())
            if check_every > 0 and (i + 1) % check_every == 0:
                self.ensure_dt(U)
                self.check()
        if n_steps > 0:
            self.ensure_dt(U)   # the SSP-RK3 step already left the new state's dt
            self.check()
        if ke_history:
            return torch.cat(hist).cpu().numpy(), torch.cat(dts).cpu().numpy()
        return None
