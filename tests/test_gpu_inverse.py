"""Toughness inversion (Sec. 4, material parameter inversion) with the GPU forward map
and reverse sweep, on targets the oracle computes from a known toughness."""
import numpy as np
import pytest
import torch

import workloads as w
from oracle.step import Sim as OSim, run as orun

pytestmark = pytest.mark.gpu


def test_batched_gc_inversion_recovers_the_oracle_toughness():
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.inverse import invert_gc
    probs = [w.small_plate(24, 12, jitter=0.1, seed=s).with_(steps=30) for s in (1, 2, 3)]
    targets, dts = [], []
    for p in probs:
        osim = OSim(p)
        targets.append(orun(p, steps=30, Gc=3.0, sim=osim)[0].d.numpy())
        dts.append(osim.dt)
    sim = Simulator(probs, dtype="f64", tile_nodes=64, dt=dts)
    tgt = torch.tensor(sim.mesh.nodes_to_internal(targets), dtype=torch.float64, device="cuda")
    out = invert_gc(sim, tgt, steps=30, gc0=[2.0, 4.5, 2.6], checkpoint_every=10)
    assert np.all(np.abs(out["Gc"] - 3.0) < 1e-4 * 3.0), out
    assert np.all(out["loss"] < 1e-3 * out["history"][0][1]), out["loss"]


def test_two_region_field_inversion_recovers_the_oracle_field():
    """phi = 1.3 on elements above the crack line, 0.8 below: recovered from the final damage."""
    from paper_2606_23458_amd import Simulator
    from paper_2606_23458_amd.inverse import invert_gc_field
    p = w.small_plate(24, 12, jitter=0.1, seed=5).with_(steps=30)
    cy = p.xy[p.tri].mean(axis=1)[:, 1]
    upper = (cy > np.median(cy)).astype(np.float64)
    basis = np.stack([upper, 1.0 - upper], axis=1)
    theta_star = np.array([1.3, 0.8])
    osim = OSim(p, gc_scale=basis @ theta_star)
    target = orun(p, steps=30, sim=osim)[0].d.numpy()
    sim = Simulator(p, dtype="f64", tile_nodes=64, dt=[osim.dt])
    tgt = torch.tensor(sim.mesh.nodes_to_internal([target]), dtype=torch.float64, device="cuda")
    out = invert_gc_field(sim, tgt, steps=30, basis=basis, theta0=[1.0, 1.0], checkpoint_every=10)
    assert np.all(np.abs(out["theta"] - theta_star) < 1e-3 * theta_star), out
