"""pf_damage_pass_repeat: back-to-back damage passes of a solve stopped mid-iteration."""
import pytest
import torch

import workloads as w
from paper_2606_23458_amd import CgConfig, Simulator
from paper_2606_23458_amd import _lib as L

pytestmark = pytest.mark.gpu


def _stopped_solve(sim: Simulator, rounds: int):
    """One explicit step, then a damage solve cut after `rounds` CG rounds."""
    c = sim.cg
    cg = CgConfig(c.tol, c.max_iter, 0, c.start, c.monotone, rounds, 0, 0)
    s_in, s_out = sim.state, sim._next
    sim.explicit(s_in, s_out)
    sim.damage(s_out.H, s_in.d, s_out.d, sim._active_next, sim.active, cg=cg)
    torch.cuda.synchronize()
    return s_out


def test_repeat_keeps_the_damage_array_and_needs_a_cg_iteration():
    p = w.config0()
    sim = Simulator(p, dtype="f32", tile_nodes=128)
    sim.step(40)
    # set-up, first pass, then iterations: the solve is in a CG iteration
    s_out = _stopped_solve(sim, 4)
    st = sim.cg_stats()[0]
    assert st["flags"] & L.PF_FLAG_NOT_CONVERGED, st
    d0 = s_out.d.clone()
    arrays = (s_out.H, sim.state.d, s_out.d)
    sim.repeat_damage_pass(5, *arrays)
    torch.cuda.synchronize()
    assert torch.equal(s_out.d, d0)
    # a solve that finished is refused
    sim.damage(s_out.H, sim.state.d, s_out.d, sim._active_next, sim.active)
    torch.cuda.synchronize()
    with pytest.raises(L.PfError, match="CG iteration"):
        sim.repeat_damage_pass(1, *arrays)
    with pytest.raises(L.PfError, match="n_passes"):
        sim.repeat_damage_pass(0, *arrays)


def test_repeat_refuses_the_polynomial_preconditioner():
    p = w.config0()
    sim = Simulator(p, dtype="f32", tile_nodes=128)
    sim.step(5)
    c = sim.cg
    cg = CgConfig(c.tol, c.max_iter, 0, c.start, c.monotone, 4, 0, 3)
    sim.explicit(sim.state, sim._next)
    sim.damage(sim._next.H, sim.state.d, sim._next.d, sim._active_next, sim.active, cg=cg)
    torch.cuda.synchronize()
    with pytest.raises(L.PfError, match="Jacobi"):
        sim.repeat_damage_pass(1, sim._next.H, sim.state.d, sim._next.d)
