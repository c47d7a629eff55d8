"""Gravity-only leap-frog (steps 1, 2, 7, 8, 9 of Sec. 5) around the device force.

CPU: the Plummer velocity sampler is in virial equilibrium (2K = -W, with W
from the oracle's direct sum).  GPU: energy is conserved over a short run at
a small opening angle, and at theta = 0 the trajectory follows an FP64
leap-frog on the oracle's direct sum.
"""
import numpy as np
import pytest

import oracle
import synth


def test_plummer_velocities_virial():
    from paper_1206_1199_amd.integrate import plummer_velocities
    pos, m = synth.plummer(8192, seed=11)
    v = plummer_velocities(pos, seed=12)
    _, pot = oracle.direct(pos, m, 1e-3)
    k = 0.5 * np.sum(m * np.sum(v * v, axis=1))
    w = 0.5 * np.sum(m * pot)
    assert 2 * k / abs(w) == pytest.approx(1.0, abs=0.05)
    np.testing.assert_allclose((m[:, None] * v).sum(0), 0, atol=1e-12)


@pytest.mark.gpu
@pytest.mark.parametrize("batches,use_graph", [(1, False), (6, False), (1, True)])
def test_leapfrog_energy_conservation(batches, use_graph):
    from paper_1206_1199_amd.integrate import LeapFrog, plummer_velocities
    pos, m = synth.plummer(8192, seed=13)
    v = plummer_velocities(pos, seed=14)
    lf = LeapFrog(pos, v, m, eps=0.01, theta=0.4, g_max=64, batches=batches, use_graph=use_graph)
    e0 = lf.energy()[2]
    for _ in range(25):
        lf.step(2e-3)
    e1 = lf.energy()[2]
    print(f"energy {e0:.8f} -> {e1:.8f}, rel drift {abs(e1 - e0) / abs(e0):.2e}", flush=True)
    assert abs(e1 - e0) / abs(e0) < 2e-4
    assert np.abs(lf.momentum()).max() < 1e-5


@pytest.mark.gpu
def test_leapfrog_theta0_follows_direct_sum():
    from paper_1206_1199_amd.integrate import LeapFrog
    rng = np.random.default_rng(15)
    pos = rng.normal(size=(512, 3))
    vel = rng.normal(size=(512, 3)) * 0.1
    m = np.full(512, 1 / 512)
    lf = LeapFrog(pos, vel, m, eps=0.05, theta=0.0, g_max=64)
    x, v = pos.copy(), vel.copy()
    a, _ = oracle.direct(x, m, 0.05)
    dt = 0.01
    for _ in range(5):
        lf.step(dt)
        v += 0.5 * dt * a
        x += dt * v
        a, _ = oracle.direct(x, m, 0.05)
        v += 0.5 * dt * a
    np.testing.assert_allclose(lf.x, x, rtol=0, atol=1e-6)
    np.testing.assert_allclose(lf.v, v, rtol=0, atol=1e-6)


@pytest.mark.gpu
def test_pipelined_and_graph_forces_match_plain_bitwise():
    """Walking in batches overlapped with the device force, or replaying a
    captured graph, gives bitwise the forces of one plain force call."""
    import paper_1206_1199_amd as otoo
    from paper_1206_1199_amd.integrate import LeapFrog
    pos, m = synth.plummer(30000, seed=16)
    v = np.zeros_like(pos)
    ctx = otoo.Context(0)
    ref = LeapFrog(pos, v, m, eps=0.01, theta=0.6, g_max=64, ctx=ctx)
    for batches, use_graph in ((7, False), (1, True), (200, False)):
        lf = LeapFrog(pos, v, m, eps=0.01, theta=0.6, g_max=64, ctx=ctx, batches=batches, use_graph=use_graph)
        np.testing.assert_array_equal(lf.a, ref.a)
        np.testing.assert_array_equal(lf.phi, ref.phi)
    print(f"step times: tree {ref.times.tree_ms[-1]:.1f} ms, walk {ref.times.walk_ms[-1]:.1f} ms, "
          f"eval {ref.times.eval_ms[-1]:.1f} ms; batched eval {lf.times.eval_ms[-1]:.1f} ms", flush=True)
