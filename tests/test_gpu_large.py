"""GPU parity at a mesh size where the reconstruction's face-point offsets
once spanned more than the 4 GiB a buffer descriptor addresses with 32-bit
offsets (FP64 P2 hexahedra beyond 7.46M cells): the point states of sampled
cells, every face point of each, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2609_07387_amd import inputs, ucns
from parity_helpers import as_oracle_phys, point_states

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1500)
def test_large_hex_mesh_fp64_point_states_sampled():
    """196^3 = 7,529,536 periodic hexahedra, P2, FP64, one reconstruction:
    sampled cells (random, plus the first and last 64 of the cell range,
    whose lanes carry the largest offsets) against the oracle within 1e-12
    of each variable group's scale.  The state is the Taylor-Green field
    sampled at the cell centroids (cell averages by quadrature would take
    minutes of host time at this size; both sides read the same array)."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = 196
    print(f"[gpu] large mesh {n}^3 FP64: host builds", flush=True)
    m = inputs.periodic_hex_mesh(n)
    nc = m.n_cell
    cen = m.cell_vertex_coords().mean(axis=1)
    U = np.ascontiguousarray(inputs.tgv_conserved(cen).T)
    del cen
    lm = ucns.Mesh(m, order=2)
    assert ucns.recon_span_bytes(nc, ucns.F64, lm.K, lm.nfmax) < 2 ** 32
    # (the old single face-point stream: 72 rows of 8 nc bytes)
    assert lm.nfmax * lm.qmax * 3 * 8 * nc > 2 ** 32
    rng = np.random.default_rng(11)
    sample = np.unique(np.concatenate([rng.choice(nc, 3000, replace=False), np.arange(64),
                                       np.arange(nc - 64, nc)]))
    need = np.zeros(nc, np.uint8)
    need[sample] = 1
    om = oracle.OracleMesh(m, order=2, need=need)
    ph = ucns.phys(flux="hllc", viscous=False)
    print("[gpu]   reconstruction on the device", flush=True)
    lm.upload(ucns.F64)
    Ud = torch.tensor(U, dtype=torch.float64, device="cuda")
    fs = torch.full((lm.n_face_state,), float("nan"), dtype=torch.float64, device="cuda")
    flags = torch.zeros(nc, dtype=torch.uint8, device="cuda")
    ucns.reconstruct(lm, ph, Ud, ucns.F64, fs, None, flags)
    torch.cuda.synchronize()
    NF, Q = lm.nfmax, lm.qmax
    g = point_states(lm, fs)[:, :, :, torch.as_tensor(sample, device="cuda")].cpu().numpy()  # [NF][Q][5][s]
    del fs, Ud
    lm.release()
    torch.cuda.empty_cache()
    print("[gpu]   oracle at the sampled cells", flush=True)
    ofs = om.reconstruct(U, as_oracle_phys(ph))  # [n_face][2][QM][5]
    c2f_o, side_o = om.cell_faces()
    c2f_l, _, _, _ = lm.faces()
    au = np.abs(U).max(axis=1)
    scale = np.array([au[0], au[1:4].max(), au[1:4].max(), au[1:4].max(), au[4]])
    err = 0.0
    for lf in range(NF):
        fo = c2f_o[sample, lf]
        so = side_o[sample, lf].astype(np.int64)
        assert np.array_equal(c2f_l[sample, lf] & 1, so)
        b = ofs[fo, so, :Q, :]          # [s][Q][5]
        a = g[lf].transpose(2, 0, 1)    # [s][Q][5]
        assert not np.isnan(a).any() and not np.isnan(b).any()
        err = max(err, (np.abs(a - b) / scale[None, None, :]).max())
    print(f"[gpu]   {len(sample)} cells, point-state err {err:.2e}", flush=True)
    assert err < 1e-12, err
