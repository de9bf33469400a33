"""Damage subcycling on the GPU (Sec. 2.3) against the oracle's schedule."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.constitutive import subcycle_limit
from oracle.step import Sim as OSim, run as orun
from tests.gpu_common import rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nu,plane", [(0.2, "strain"), (0.25, "strain"), (0.35, "stress"), (0.3, "stress")])
def test_subcycle_limit_matches_oracle(nu, plane):
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(12, 6).with_(nu=nu, plane=plane)
    sim = Simulator(p, dtype="f64")
    assert sim.n_max == [subcycle_limit(p.E, nu, p.rho, plane)]


def test_n_sub_beyond_limit_is_refused():
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(12, 6)
    with pytest.raises(ValueError, match="N_max"):
        Simulator(p, dtype="f64", n_sub=5)


@pytest.mark.parametrize("n_sub", [2, 3])
def test_subcycled_trajectory_matches_oracle(n_sub):
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(32, 16, seed=3).with_(steps=24)
    osim = OSim(p)
    ref, _, _ = orun(p, steps=24, sim=osim, n_sub=n_sub)
    sim = Simulator(p, dtype="f64", dt=[osim.dt], n_sub=n_sub, allow_beyond_limit=True)
    sim.step(24)
    torch.cuda.synchronize()
    got = sim.state.to_user()[0]
    for f, o in (("u", ref.u), ("v", ref.v), ("d", ref.d), ("H", ref.H)):
        assert rel_err(got[f], o.numpy()) < 1e-9, f


def test_subcycled_windowed_run_equals_step():
    from paper_2606_23458_amd import Simulator
    p = w.small_plate(32, 16, seed=3)
    a = Simulator(p, dtype="f64", n_sub=2)
    b = Simulator(p, dtype="f64", n_sub=2, dt=list(a.dt))
    a.step(17)
    b.run(17, window=6)
    torch.cuda.synchronize()
    assert torch.equal(a.state.nodes, b.state.nodes) and torch.equal(a.state.H, b.state.H)
    assert torch.equal(a.active, b.active)
