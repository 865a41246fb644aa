"""Helpers shared by the GPU parity tests: run one stage / n steps through the
C-ABI and through the oracle on the same seeded inputs, and align face data."""
import numpy as np

import oracle
from paper_2609_07387_amd import ucns


def grouped_rel_linf(A, B):
    """Relative L-inf per group {rho}, {rho u, rho v, rho w}, {rho E}; the max
    over groups (error of A against the reference B)."""
    out = 0.0
    for g in ([0], [1, 2, 3], [4]):
        den = np.abs(B[g]).max()
        out = max(out, np.abs(A[g] - B[g]).max() / (den if den > 0 else 1.0))
    return out


def face_maps(lm, om):
    """Aligned (library face, oracle face, side) triples over every (cell, local face)."""
    c2f_l, _, _, _ = lm.faces()
    c2f_o, side_o = om.cell_faces()
    ok = c2f_o >= 0
    fl = (c2f_l[ok] >> 1).astype(np.int64)
    sl = (c2f_l[ok] & 1).astype(np.int64)
    fo = c2f_o[ok]
    assert np.array_equal(sl, side_o[ok].astype(np.int64))
    return fl, fo, sl


def lib_arrays(lm, precision, device="cuda"):
    import torch

    dt = torch.float64 if precision == ucns.F64 else torch.float32
    fs = torch.full((lm.n_face_state,), float("nan"), dtype=dt, device=device)
    ff = torch.zeros(lm.n_face_flux, dtype=dt, device=device)
    gw = torch.zeros(lm.n_grad, dtype=dt, device=device)
    R = torch.zeros((5, lm.n_cell), dtype=torch.float64, device=device)
    return fs, ff, gw, R


def point_states(lm, fs):
    """Library point states [NFMAX][Q][n_pad][5] (one row per point slot, the
    cell count padded to whole 64-cell tiles) as [NFMAX][Q][5][n_cell]; numpy
    or torch."""
    NF, Q, nc = lm.nfmax, lm.qmax, lm.n_cell
    npad = -(-nc // 64) * 64
    g = fs.reshape(NF, Q, npad, 5)[:, :, :nc, :]
    return g.transpose(2, 3) if hasattr(g, "contiguous") else g.transpose(0, 1, 3, 2)


def face_major(lm, fs_cells):
    """Library point states as [n_face][2][Q][5] (NaN where a face has no such
    side)."""
    c2f, _, _, _ = lm.faces()
    NF, Q = lm.nfmax, lm.qmax
    fsc = point_states(lm, np.asarray(fs_cells))
    out = np.full((lm.n_face, 2, Q, 5), np.nan)
    for lf in range(NF):
        f2 = c2f[:, lf].astype(np.int64)
        ok = f2 >= 0
        out[f2[ok] >> 1, f2[ok] & 1] = fsc[lf].transpose(2, 0, 1)[ok]
    return out


def gpu_stage(lm, ph, U_np, precision, bcs=None, gate_mask=None, device="cuda", fused=False):
    """One residual evaluation on the GPU; returns host copies of
    (face_state [nf,2,Q,5], gradW [12,nc] or None, face_flux [nf,5], R [5,nc], flags).
    fused: the point states and the gradients from the one-pass call."""
    import torch

    if precision not in lm.arenas:
        lm.upload(precision, device)
    U = torch.tensor(U_np, dtype=torch.float64, device=device).contiguous()
    fs, ff, gw, R = lib_arrays(lm, precision, device)
    flags = torch.zeros(lm.n_cell, dtype=torch.uint8, device=device)
    gm = None if gate_mask is None else torch.tensor(gate_mask, dtype=torch.uint8, device=device)
    if fused:
        ucns.reconstruct_gradients(lm, ph, ucns.bc_device(bcs, device), U, precision, fs, flags, gw, gm)
    else:
        ucns.reconstruct(lm, ph, U, precision, fs, gm, flags)
        if ph.viscous:
            ucns.gradients(lm, ph, bcs, U, precision, gw)
    ucns.face_flux(lm, ph, bcs, U, fs, gw if ph.viscous else None, precision, ff)
    ucns.residual(lm, ff, precision, R)
    torch.cuda.synchronize()
    return (face_major(lm, fs.double().cpu().numpy()),
            gw.double().cpu().numpy().reshape(12, lm.n_cell) if ph.viscous else None,
            ff.double().cpu().numpy().reshape(lm.n_face, 5), R.cpu().numpy(), flags.cpu().numpy())


def gpu_run(lm, ph, U_np, precision, n_steps, cfl, bcs=None, gate_mask=None, device="cuda", integrator="ssp3"):
    import torch

    gm = None if gate_mask is None else torch.tensor(gate_mask, dtype=torch.uint8, device=device)
    s = ucns.Solver(lm, ph, precision, bcs, cfl, gm, device, integrator=integrator)
    U = torch.tensor(U_np, dtype=torch.float64, device=device).contiguous()
    ke, dts = s.run(U, n_steps, ke_history=True)
    torch.cuda.synchronize()
    return U.cpu().numpy(), ke, dts


def oracle_stage(om, ph, U, bcs=None, gate_mask=None):
    fs, flags, label = om.reconstruct(U, ph, gate_mask, with_flags=True)
    g = om.gradients(U, ph, bcs) if ph.viscous else None
    ff = om.face_flux(U, fs, ph, g, bcs)
    R = om.residual(ff)
    return fs, g, ff, R, flags, label


def as_oracle_phys(ph):
    return oracle.Phys(ph.gamma, ph.mach, ph.reynolds, ph.prandtl, ph.viscous, ph.flux, ph.grad)


def as_oracle_bc(b):
    if b is None:
        return None
    o = oracle.BC()
    for t in range(8):
        o.kind[t] = b.kind[t]
        for v in range(5):
            o.state[t][v] = b.state[t][v]
    return o
