"""A captured SSP-RK3 step (HIP graph of the library's launches) replayed
against eager steps: every replay bitwise equal to the eager step it stands
for, with the program's own eager work and synchronisations in between."""
import numpy as np
import pytest

from paper_2609_07387_amd import gate, inputs, ucns

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", ["fp64", "fp32_gate"])
def test_graph_replay_matches_eager_steps(variant):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    m = inputs.periodic_hex_mesh(12)
    U0 = inputs.tgv_initial(m)
    ph = ucns.phys(flux="hllc", viscous=True)
    lm = ucns.Mesh(m, order=2)
    prec = ucns.F64 if variant == "fp64" else ucns.F32
    mlp = None
    if variant == "fp32_gate":
        import os

        if not os.path.exists(gate.WEIGHTS):
            pytest.skip("no trained network")
        mlp = torch.tensor(np.load(gate.WEIGHTS).astype(np.float32), device="cuda")
    steps = 4
    eager = ucns.Solver(lm, ph, prec, cfl=0.5, mlp=mlp)
    Ue = torch.tensor(U0, device="cuda")
    ref, dts = [], []
    for _ in range(steps):
        eager.step(Ue)
        ref.append(Ue.clone())
        dts.append(eager.ws.dt.clone())
    torch.cuda.synchronize()
    solver = ucns.Solver(lm, ph, prec, cfl=0.5, mlp=mlp)
    Ug = torch.tensor(U0, device="cuda")
    solver.capture(Ug)
    torch.cuda.synchronize()
    assert torch.equal(Ug, torch.tensor(U0, device="cuda"))  # capture runs nothing
    for k in range(steps):
        solver.step_graph(Ug)
        torch.cuda.synchronize()
        assert torch.equal(Ug, ref[k]), k
        assert torch.equal(solver.ws.dt, dts[k]), k
        # eager work of the program between replays
        _ = float((Ug * 2.0).sum().item())
        torch.cuda.synchronize()
    solver.check()
