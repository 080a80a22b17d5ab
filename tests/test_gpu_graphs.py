"""Graph mode of tmd_integrate: whole rebuild intervals run as captured HIP
graphs must leave the state of the eager run bit for bit, on every replay.

Each test advances two identical systems, one eagerly and one in graph mode,
by the same sequence of integrate calls of uneven lengths (so intervals
start at different points of a call), does other eager work and a
synchronisation between the calls, and compares positions, velocities and
forces exactly after every call.
"""

import numpy as np
import pytest

import oracle
from workloads import md_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_2009_07400_amd import System  # noqa: E402

CHUNKS = [45, 20, 61, 7, 40, 19, 41]


def _pair(make):
    a, b = make(), make()
    b.set_graphs(True)
    return a, b


def _same(a, b, label):
    pa, va, sa = a.get_state()
    pb, vb, sb = b.get_state()
    fa, _ = a.compute_forces(energy=False)
    fb, _ = b.compute_forces(energy=False)
    torch.cuda.synchronize()
    assert sa == sb, label
    assert torch.equal(pa, pb), label
    assert torch.equal(va, vb), label
    assert torch.equal(fa, fb), label


def _single():
    s = md_system(10, seed=21)  # 4,000 atoms, 5 cells per axis
    g = System(s.n, s.L)
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    return g


def _batch():
    specs = [(4, 0.80, 0.9, 31), (6, 0.8442, 1.44, 32), (9, 0.85, 1.0, 33), (12, 0.78, 1.3, 34)]
    states = [md_system(n, rho, T, seed=seed) for n, rho, T, seed in specs]
    g = System.batch([s.n for s in states], [s.L for s in states], {"max_neighbors": 160})
    g.set_state(torch.from_numpy(np.concatenate([s.pos() for s in states])),
                torch.from_numpy(np.concatenate([s.vel() for s in states])))
    return g


@pytest.mark.parametrize("make", [_single, _batch], ids=["single", "batch"])
def test_graph_replays_equal_eager_runs(make):
    a, b = _pair(make)
    try:
        for k, n in enumerate(CHUNKS):
            a.integrate(n)
            b.integrate(n)
            _same(a, b, f"after call {k} ({n} steps)")
            # eager work on the graph-mode system between replays
            b.get_neighbors()
            b.sync()
            a.sync()
        info = b.info()
        # intervals flip the double-buffered copies: two graphs, replayed since
        assert info["graph_captures"] == 2
        assert info["graph_launches"] >= 5
        assert a.info()["graph_launches"] == 0
    finally:
        a.close()
        b.close()


def test_graph_recaptured_after_schedule_change_and_off_again():
    a, b = _pair(_single)
    try:
        for g in (a, b):
            g.integrate(60)
        _same(a, b, "first schedule")
        for g in (a, b):
            g.set_schedule(threads=128, block_edge=2, lanes_per_atom=2)
            g.integrate(60)
        _same(a, b, "second schedule")
        assert b.info()["graph_captures"] == 4
        b.set_graphs(False)
        for g in (a, b):
            g.integrate(45)
        _same(a, b, "graphs off")
        assert b.info()["graph_captures"] == 4
    finally:
        a.close()
        b.close()


def test_graph_mode_with_thermo_output_runs_eagerly():
    a, b = _pair(_single)
    try:
        ta = a.integrate(80, thermo_every=10)
        tb = b.integrate(80, thermo_every=10)
        torch.cuda.synchronize()
        assert torch.equal(ta, tb)
        _same(a, b, "thermo run")
        assert b.info()["graph_captures"] == 0
    finally:
        a.close()
        b.close()


def test_graph_mode_trajectory_matches_oracle():
    s = md_system(8, seed=22)  # 2,048 atoms
    g = System(s.n, s.L)
    g.set_graphs(True)
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    g.integrate(100)
    p, v, _ = g.get_state()
    torch.cuda.synchronize()
    assert g.info()["graph_launches"] >= 3
    g.close()
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 100, thermo=False)
    L = s.L
    d = p.cpu().numpy() - r["x"]
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(v.cpu().numpy() - r["v"]).max() < 1e-9


def test_graph_mode_across_set_state_and_adjoint():
    a, b = _pair(_single)
    try:
        for g in (a, b):
            g.integrate(50)
        p, v, _ = a.get_state()
        lam = torch.linspace(-1.0, 1.0, 3 * a.n, dtype=torch.float64, device="cuda").reshape(a.n, 3)
        grads = []
        for g in (a, b):
            g.set_state(p, v)
            g.adjoint_forward(40)
            grads.append(g.adjoint_backward(lam))
        torch.cuda.synchronize()
        for x, y in zip(*grads):
            assert torch.equal(x, y)
        # (the adjoint leaves the list stale, so no force comparison here)
        (pa, va, sa), (pb, vb, sb) = a.get_state(), b.get_state()
        torch.cuda.synchronize()
        assert sa == sb and torch.equal(pa, pb) and torch.equal(va, vb)
        for g in (a, b):
            g.integrate(63)
        _same(a, b, "graphs after set_state and the adjoint")
        assert b.info()["graph_launches"] >= 2
    finally:
        a.close()
        b.close()
