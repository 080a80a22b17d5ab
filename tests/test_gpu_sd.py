"""Spring-Dashpot contact model (Sec. 3.2, Eq. 3) on the GPU against the CPU
oracle, through the C ABI.

Bars as for Lennard-Jones: lists bit-exact (sorted rows, original ids);
every sphere's force within 1e-12 of its conditioning scale sum_j |F_ij| at
identical positions and velocities; elastic energy and virial within 1e-12;
positions and velocities within 1e-9 after 200 steps of the damped dynamics
(the damping takes the half-step velocities, as in the oracle).
"""

import numpy as np
import pytest

import oracle
from workloads import sd_half_domain, sd_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_2009_07400_amd import System, TmdError  # noqa: E402

FORCE_TOL = 1e-12
POS_TOL = 1e-9


def _say(msg):
    print(msg, flush=True)


def _params(s, **kw):
    p = dict(model="spring_dashpot", stiffness=s.k, damping=s.gamma, sigma=s.sigma, cutoff=s.cutoff, skin=s.skin,
             dt=s.dt, max_neighbors=64)
    p.update(kw)
    return p


def _mic(d, L):
    return d - L * np.round(d / L)


def _gpu(s, sched=None, **kw):
    g = System(s.n, s.L, **_params(s, **kw))
    if sched:
        g.set_schedule(**sched)
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    return g


@pytest.mark.parametrize("ncell,sched", [(6, None), (6, dict(block_edge=3)), (6, dict(lds_atoms=64)),
                                         (10, None), (10, dict(block_edge=3)), (10, dict(build_lanes=2)),
                                         (3, None)])
def test_lists_forces_energy_match_oracle(ncell, sched):
    s = sd_system(ncell, seed=40 + ncell)
    _say(f"spring-dashpot forces: {s.n} spheres, L {s.L:.3f}, schedule {sched}")
    g = _gpu(s, sched)
    try:
        g.build_neighbors()
        counts, ids = g.get_neighbors()
        F, ev = g.compute_forces()
        g.sync()
        x, v = s.pos(), s.vel()
        c_o, n_o, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], s.L, s.cutoff + s.skin, maxnb=64)
        assert np.array_equal(counts.cpu().numpy(), c_o)
        assert np.array_equal(ids.cpu().numpy(), n_o)
        Fo, sc, Uo, Wo = oracle.sd_forces(x, v, s.L, c_o, n_o, s.k, s.gamma, s.sigma)
        F = F.cpu().numpy()
        err = np.linalg.norm(F - Fo, axis=1)
        assert (err <= FORCE_TOL * np.maximum(sc, 1e-300)).all(), float((err / np.maximum(sc, 1e-300)).max())
        U, W = ev.cpu().numpy()
        assert U == pytest.approx(Uo, rel=FORCE_TOL) and W == pytest.approx(Wo, rel=FORCE_TOL)
        assert (sc > 0).mean() > 0.9  # a dense packing: nearly every sphere is in contact
    finally:
        g.close()


@pytest.mark.parametrize("ncell,sched", [(6, None), (8, dict(block_edge=3)), (8, dict(lds_atoms=64))])
def test_damped_trajectory_matches_oracle(ncell, sched):
    s = sd_system(ncell, seed=60 + ncell)
    steps = 200
    _say(f"spring-dashpot trajectory: {s.n} spheres, {steps} steps, schedule {sched}")
    g = _gpu(s, sched)
    try:
        th = g.integrate(steps, thermo_every=50)
        p, vel, step = g.get_state()
        g.sync()
        r = oracle.sd_run(s.pos(), s.vel(), s.L, steps, s.k, s.gamma, sigma=s.sigma, cutoff=s.cutoff, skin=s.skin,
                          dt=s.dt)
        assert step == steps
        assert np.abs(_mic(p.cpu().numpy() - r["x"], s.L)).max() < POS_TOL
        assert np.abs(vel.cpu().numpy() - r["v"]).max() < POS_TOL
        th = th.cpu().numpy()
        for row, k in zip(th, range(50, steps + 1, 50)):
            assert row == pytest.approx(r["thermo"][k], rel=1e-9, abs=1e-12)
        # the dashpot dissipates
        assert r["thermo"][steps][4] < r["thermo"][0][4]
    finally:
        g.close()


def test_split_integrate_and_graph_mode_are_bitwise_identical():
    s = sd_system(6, seed=71)
    a = _gpu(s)
    a.integrate(60)
    pa, va, _ = a.get_state()
    b = _gpu(s)
    b.integrate(7)
    b.set_graphs(True)
    b.integrate(53)
    pb, vb, _ = b.get_state()
    a.sync()
    b.sync()
    assert torch.equal(pa, pb) and torch.equal(va, vb)
    a.close()
    b.close()


def test_batch_of_sphere_boxes_matches_oracle():
    boxes = [sd_system(4, seed=80, k=800.0, gamma=3.0), sd_system(7, seed=81, k=1200.0, gamma=8.0),
             sd_system(5, seed=82, k=1000.0, gamma=0.0)]
    g = System.batch([b.n for b in boxes], [b.L for b in boxes], [_params(b) for b in boxes])
    g.set_state(torch.from_numpy(np.concatenate([b.pos() for b in boxes])),
                torch.from_numpy(np.concatenate([b.vel() for b in boxes])))
    g.integrate(100)
    p, v, _ = g.get_state()
    g.sync()
    p, v = p.cpu().numpy(), v.cpu().numpy()
    off = 0
    for b in boxes:
        r = oracle.sd_run(b.pos(), b.vel(), b.L, 100, b.k, b.gamma, sigma=b.sigma, cutoff=b.cutoff, skin=b.skin,
                          dt=b.dt)
        assert np.abs(_mic(p[off:off + b.n] - r["x"], b.L)).max() < POS_TOL
        assert np.abs(v[off:off + b.n] - r["v"]).max() < POS_TOL
        off += b.n
    g.close()


def test_half_filled_domain_at_rest():
    """The load-balancing geometry of Sec. 6 (half of the box filled along a
    diagonal plane) with zero stiffness and damping: spheres at rest, every
    force zero, lists equal to the oracle's."""
    pos, L = sd_half_domain(16)
    g = System(pos.shape[0], L, model="spring_dashpot", stiffness=0.0, damping=0.0, sigma=1.0, cutoff=1.0, skin=0.3,
               dt=1e-3, max_neighbors=32)
    g.set_state(torch.from_numpy(pos), torch.zeros(pos.shape[0], 3, dtype=torch.float64))
    g.integrate(40)
    p, v, _ = g.get_state()
    counts, ids = g.get_neighbors()
    g.sync()
    assert np.array_equal(p.cpu().numpy(), pos) and not v.cpu().numpy().any()
    c_o, n_o, _ = oracle.build_list(pos[:, 0], pos[:, 1], pos[:, 2], L, 1.3, maxnb=32)
    assert np.array_equal(counts.cpu().numpy(), c_o) and np.array_equal(ids.cpu().numpy(), n_o)
    g.close()


def test_spring_dashpot_rejections():
    s = sd_system(4, seed=90)
    g = _gpu(s)
    with pytest.raises(TmdError):
        g.set_schedule(lanes_per_atom=2)
    with pytest.raises(TmdError):
        g.adjoint_forward(20)
    with pytest.raises(TmdError):
        g.set_lj_params([1.0], [1.0])
    g.close()
