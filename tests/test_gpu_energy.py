"""Energy budget on the GPU (pf_energies) against the oracle's energies."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.step import Sim as OSim, run as orun
from tests.gpu_common import random_state, to_oracle

pytestmark = pytest.mark.gpu

SPLITS = ["none", "spectral", "voldev", "starconvex"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("plane", ["strain", "stress"])
@pytest.mark.parametrize("model", [1, 2])
def test_energies_match_oracle(dtype, split, plane, model):
    from paper_2606_23458_amd import Simulator, State
    p = w.small_plate(23, 13, jitter=0.2, seed=3, split=split, plane=plane, gamma_star=0.8, model=model,
                      random_diag=True)
    osim = OSim(p)
    sim = Simulator(p, dtype=dtype, dt=[osim.dt])
    st = random_state(p, seed=21)
    got = sim.energies(State.from_user(sim.mesh, [st]))[0]
    ref = osim.energies(to_oracle(st))
    tol = 1e-11 if dtype == "f64" else 2e-5
    for g, r, name in zip(got, ref, ("kin", "el", "frac")):
        assert abs(g - r) <= tol * abs(r), (name, g, r)


def test_energy_history_of_a_trajectory():
    """Energies of a 60-step FP64 trajectory, every 10 steps, against the oracle's states."""
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(32, 16, seed=3).with_(steps=60)
    osim = OSim(p)
    _, rec, _ = orun(p, steps=60, sim=osim, record_every=10)
    sim = Simulator(p, dtype="f64", dt=[osim.dt])
    for k in range(6):
        sim.step(10)
        got = sim.energies()[0]
        o = rec[k]
        ost = to_oracle({"u": o["u"], "v": o["v"], "a": o["a"], "d": o["d"], "H": o["H"]})
        ref = osim.energies(ost)
        for g, r in zip(got, ref):
            assert abs(g - r) <= 1e-8 * max(abs(r), 1e-30), (k, got, ref)
