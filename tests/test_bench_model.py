"""CPU checks of the benchmark's algorithmic byte model (the numerator of the
reported roofline) and of the names that tie it to the measured-traffic
records.  The per-cell figures are those of the P2 CWENOZ reconstruction on a
hexahedral lattice: 26-cell central stencil, six 9-cell directional
stencils, 2 x 2 Gauss points per face."""
import json
import os

import pytest

import bench
from paper_2609_07387_amd import inputs, ucns

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hex_mesh():
    if not os.path.exists(ucns.LIB_PATH):
        pytest.skip("libucns.so not built")
    return ucns.Mesh(inputs.periodic_hex_mesh(6), order=2)


def test_reconstruction_bytes_per_cell_hex_p2(hex_mesh):
    lm = hex_mesh
    assert (lm.K, lm.mc_pad, lm.md_pad, lm.nd_max, lm.nfmax, lm.qmax) == (9, 26, 9, 6, 6, 4)
    # operators: 9 x 26 central + 6 x 4 x 3 point offsets + 9 basis means
    # + 45 indicator entries + 6 x 3 x 9 directional = 522 values; 80 indices
    assert bench.recon_bytes_per_cell(lm, ucns.F64) == 8 * 522 + 4 * 80 + 6 + 1 + 40 + 8 * 120 + 1 == 5504
    assert bench.recon_bytes_per_cell(lm, ucns.F32) == 4 * 522 + 4 * 80 + 6 + 1 + 40 + 4 * 120 + 1 == 2936
    # a cell taken as smooth reads no directional operators, indices or
    # indicator matrix; the network adds its inputs and the mask
    lin = bench.recon_bytes_per_cell(lm, ucns.F32, linear=True, gate=True)
    assert lin == 4 * 315 + 4 * 26 + 6 + 1 + 40 + 4 * 120 + 1 + (4 * 6 + 3 * 6 * 4 + 4 + 2) == 1994
    # the fused Green-Gauss gradients: 6 x 3 slot weights and 12 values
    # written, plus the 6 neighbour ids when the gate has not read them
    assert bench.recon_bytes_per_cell(lm, ucns.F32, linear=True, gate=True, grad=True) == 1994 + 4 * 18 + 4 * 12
    assert bench.recon_bytes_per_cell(lm, ucns.F64, grad=True) == 5504 + 4 * 6 + 8 * 18 + 8 * 12
    # and the separate gradient pass drops out of the stage's bytes
    full = bench.step_bytes_per_cell(lm, ucns.F64, recon=5504)
    fused = bench.step_bytes_per_cell(lm, ucns.F64, recon=5504 + 4 * 6 + 8 * 18 + 8 * 12, fused=True)
    assert full - fused == (40 + 4 * 6 + 8 * 12 + 3 * (8 + 4 * 8)) - (4 * 6 + 8 * 18 + 8 * 12)


def test_traffic_records_name_the_timed_kernels():
    """Each variant's record lists every kernel of the reconstruction call the
    benchmark times (otherwise the benchmark reports no traffic)."""
    for head, name in bench.TRAFFIC.items():
        with open(os.path.join(ROOT, "profiles", name)) as f:
            text = f.read()
        i = text.index("```json")
        rec = json.loads(text[i + 7:text.index("```", i + 7)])
        for k in bench.recon_kernels(head, 1).split("|"):
            assert k in rec["kernel"], (head, k)
