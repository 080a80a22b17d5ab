"""Position layouts (the particle layouts of Sec. 4.2: SoA, AoS, clustered
AoSoA) on the GPU, through the C ABI.  The kernels compute the same values
in the same order whatever the layout, so every layout gives the SoA run's
results bit for bit - lists, forces, energies and whole trajectories, also
when the layout changes mid-run - and the SoA run is checked against the
oracle (lists bit-exact, forces within 1e-12 of each atom's scale)."""

import numpy as np
import pytest

import oracle
from workloads import SplitMix64, md_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_2009_07400_amd import System, TmdError  # noqa: E402

LAYOUTS = ("aos", "aosoa")


def _say(msg):
    print(msg, flush=True)


def _mic(d, L):
    return d - L * np.round(d / L)


CASES = {
    "liquid10": lambda: (lambda s: (s.pos(), s.vel(), s.L))(md_system(10, seed=91)),
    "nc3_6": lambda: (lambda s: (s.pos(), s.vel(), s.L))(md_system(6, seed=92)),
    # 1001 atoms: the last AoSoA cluster is partly padding
    "ragged_uniform": lambda: (SplitMix64(93).next_double(3 * 1001).reshape(1001, 3) * 12.5,
                               np.zeros((1001, 3)), 12.5),
}


def _system(pos, vel, L, layout=None, sched=None, **kw):
    g = System(pos.shape[0], L, max_neighbors=256, **kw)
    if layout:
        g.set_layout(layout)  # before the state: nothing to convert
    g.set_state(torch.from_numpy(pos), torch.from_numpy(vel))
    if sched:
        g.set_schedule(**sched)
    return g


def _lists_forces(g):
    g.build_neighbors()
    counts, ids = g.get_neighbors()
    F, ev = g.compute_forces()
    g.sync()
    return counts.cpu().numpy(), ids.cpu().numpy(), F.cpu().numpy(), ev.cpu().numpy()


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("sched", [dict(), dict(block_edge=3, build_lanes=2), dict(lds_atoms=256)])
def test_layouts_give_the_soa_lists_and_forces(case, sched):
    pos, vel, L = CASES[case]()
    _say(f"layouts: {case}, schedule {sched}")
    ref = _system(pos, vel, L, sched=sched)
    c0, n0, F0, ev0 = _lists_forces(ref)
    ref.close()
    co, no, _ = oracle.build_list(pos[:, 0], pos[:, 1], pos[:, 2], L, 2.8, maxnb=256)
    assert np.array_equal(c0, co) and np.array_equal(n0, no)
    Fo, sc, Uo, Wo = oracle.forces(pos[:, 0], pos[:, 1], pos[:, 2], L, co, no)
    assert (np.linalg.norm(F0 - Fo, axis=1) <= 1e-12 * np.maximum(sc, 1e-300)).all()
    for lay in LAYOUTS:
        g = _system(pos, vel, L, layout=lay, sched=sched)
        assert g.info()["layout"] == System.LAYOUTS[lay]
        c, n, F, ev = _lists_forces(g)
        g.close()
        assert np.array_equal(c, c0) and np.array_equal(n, n0), lay
        assert np.array_equal(F, F0) and np.array_equal(ev, ev0), lay


@pytest.mark.parametrize("lay", LAYOUTS)
def test_layout_trajectory_is_the_soa_trajectory(lay):
    s = md_system(10, seed=94)
    runs = []
    for layout in (None, lay):
        g = _system(s.pos(), s.vel(), s.L, layout=layout)
        th = g.integrate(100, thermo_every=20)
        p, v, _ = g.get_state()
        g.sync()
        runs.append((p.cpu().numpy(), v.cpu().numpy(), th.cpu().numpy()))
        g.close()
    (p0, v0, t0), (p1, v1, t1) = runs
    assert np.array_equal(p0, p1) and np.array_equal(v0, v1) and np.array_equal(t0, t1)
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 100, thermo=False)
    assert np.abs(_mic(p1 - r["x"], s.L)).max() < 1e-9


def test_layout_change_mid_run_and_in_graph_mode():
    s = md_system(9, seed=95)
    a = _system(s.pos(), s.vel(), s.L)
    a.integrate(90)
    pa, va, _ = a.get_state()
    b = _system(s.pos(), s.vel(), s.L)
    b.integrate(13)
    b.set_layout("aos")
    b.integrate(27)
    b.set_graphs(True)
    b.set_layout("aosoa")
    b.integrate(30)
    b.set_layout("soa")
    b.integrate(20)
    pb, vb, _ = b.get_state()
    a.sync()
    b.sync()
    assert torch.equal(pa, pb) and torch.equal(va, vb)
    a.close()
    b.close()


def test_layout_with_half_lists_and_batch():
    specs = [(5, 0.80, 1.0, 96), (8, 0.85, 1.2, 97), (4, 0.9, 0.8, 98)]
    boxes = [md_system(n, rho, T, seed=sd) for n, rho, T, sd in specs]
    for half in (False, True):
        g = System.batch([b.n for b in boxes], [b.L for b in boxes], dict(max_neighbors=128))
        g.set_layout("aosoa")
        g.set_state(torch.from_numpy(np.concatenate([b.pos() for b in boxes])),
                    torch.from_numpy(np.concatenate([b.vel() for b in boxes])))
        g.set_half_list(half)
        g.integrate(50)
        p, v, _ = g.get_state()
        g.sync()
        p = p.cpu().numpy()
        off = 0
        for b in boxes:
            r = oracle.run(b.x, b.y, b.z, b.vx, b.vy, b.vz, b.L, 50, thermo=False)
            assert np.abs(_mic(p[off:off + b.n] - r["x"], b.L)).max() < 1e-9
            off += b.n
        g.close()


def test_layout_rejections_and_autotune():
    s = md_system(8, seed=99)
    g = _system(s.pos(), s.vel(), s.L, layout="aos")
    with pytest.raises(TmdError):
        g.adjoint_forward(20)
    with pytest.raises(TmdError):
        g.set_layout(5)
    sched = g.autotune(repeats=2)
    assert sched["layout"] in (0, 1, 2) and g.info()["layout"] == sched["layout"]
    g.integrate(20)  # runs in the picked layout
    p, _, _ = g.get_state()
    g.sync()
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 20, thermo=False)
    assert np.abs(_mic(p.cpu().numpy() - r["x"], s.L)).max() < 1e-9
    # tuned for the adjoint: full lists and SoA positions, which it runs with
    sched = g.autotune(repeats=2, for_adjoint=True)
    assert sched["layout"] == 0 and sched["half_list"] == 0
    g.adjoint_forward(20)
    g.sync()
    g.close()


def test_repeated_layout_changes_keep_every_position():
    """Layout conversions back and forth leave the state bit for bit, the
    NaN sentinel included (a later step would report a non-finite value)."""
    s = md_system(9, seed=97)
    g = _system(s.pos(), s.vel(), s.L)
    p0, v0, _ = g.get_state()
    for lay in ("aosoa", "aos", "soa", "aosoa", "soa", "aos", "aosoa", "aos", "soa") * 3:
        g.set_layout(lay)
    p1, v1, _ = g.get_state()
    g.integrate(25)
    g.sync()
    assert torch.equal(p0, p1) and torch.equal(v0, v1)
    g.close()
