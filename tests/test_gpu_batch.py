"""Batched replicas and work schedules against the CPU oracle.

Boxes of different sizes (2 to 7 cells per axis, odd counts give blocks one
cell thick), densities, temperatures and LJ parameters are advanced in the
same launches; each box must match the oracle run on that box alone, and
the batch must match separate single-box runs bit for bit.
"""

import numpy as np
import pytest

import oracle
from workloads import batched_box_specs, md_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_2009_07400_amd import System  # noqa: E402

# (ncell, rho, T, seed, eps, sigma): cells per axis 2, 3, 4, 5, 7
BOXES = [(4, 0.80, 0.9, 11, 1.0, 1.0), (6, 0.8442, 1.44, 12, 1.05, 0.98), (8, 0.75, 1.2, 13, 1.0, 1.0),
         (9, 0.85, 1.0, 14, 0.9, 1.02), (12, 0.78, 1.3, 15, 1.0, 1.0)]


def _states():
    out = []
    for ncell, rho, T, seed, eps, sig in BOXES:
        s = md_system(ncell, rho, T, seed=seed)
        r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 15, eps=eps, sigma=sig, thermo=False)
        out.append((r["x"], r["v"], s.L, eps, sig))
    return out


def _batch(states, **sched):
    g = System.batch([p.shape[0] for p, *_ in states], [L for _, _, L, _, _ in states],
                     [dict(epsilon=e, sigma=s, max_neighbors=160) for *_, e, s in states])
    if sched:
        g.set_schedule(**sched)
    g.set_state(torch.from_numpy(np.concatenate([p for p, *_ in states])),
                torch.from_numpy(np.concatenate([v for _, v, *_ in states])))
    return g


def _mic(d, L):
    return d - L * np.round(d / L)


def test_cells_per_axis_of_the_cases():
    assert [oracle.cells_per_axis(L, 2.8) for _, _, L, _, _ in _states()] == [2, 3, 4, 5, 7]


@pytest.mark.parametrize("sched", [{}, {"lds_atoms": 64}, {"threads": 64}, {"threads": 256, "lds_atoms": 2560},
                                   {"block_parts": 2}, {"block_parts": 4, "threads": 64}, {"lanes_per_atom": 2},
                                   {"lanes_per_atom": 2, "lds_atoms": 64}, {"lanes_per_atom": 2, "block_edge": 3},
                                   {"lanes_per_atom": 4}, {"lanes_per_atom": 4, "lds_atoms": 64}])
def test_batch_lists_and_forces_match_oracle(sched):
    states = _states()
    g = _batch(states, **sched)
    g.build_neighbors()
    F, ev = g.compute_forces()
    counts, ids = g.get_neighbors()
    g.sync()
    F, ev, counts, ids = F.cpu().numpy(), ev.cpu().numpy(), counts.cpu().numpy(), ids.cpu().numpy()
    off = 0
    for k, (p, v, L, eps, sig) in enumerate(states):
        n = p.shape[0]
        c_o, n_o, _ = oracle.build_list(p[:, 0], p[:, 1], p[:, 2], L, 2.8, maxnb=160)
        assert np.array_equal(counts[off:off + n], c_o), k
        for i in range(n):
            assert np.array_equal(ids[off + i, : c_o[i]] - off, n_o[i, : c_o[i]]), (k, i)
        Fo, sc, Uo, Wo = oracle.forces(p[:, 0], p[:, 1], p[:, 2], L, c_o, n_o, eps=eps, sigma=sig)
        err = np.linalg.norm(F[off:off + n] - Fo, axis=1)
        assert (err <= 1e-12 * sc).all(), k
        assert ev[k, 0] == pytest.approx(Uo, rel=1e-12)
        assert ev[k, 1] == pytest.approx(Wo, rel=1e-12)
        off += n


def test_batch_trajectory_matches_oracle():
    states = _states()
    g = _batch(states)
    th = g.integrate(60, thermo_every=20)
    P, V, step = g.get_state()
    g.sync()
    P, V, th = P.cpu().numpy(), V.cpu().numpy(), th.cpu().numpy()
    assert step == 60 and th.shape == (3, len(states), 5)
    off = 0
    for k, (p, v, L, eps, sig) in enumerate(states):
        n = p.shape[0]
        r = oracle.run(p[:, 0], p[:, 1], p[:, 2], v[:, 0], v[:, 1], v[:, 2], L, 60, eps=eps, sigma=sig)
        assert np.abs(_mic(P[off:off + n] - r["x"], L)).max() < 1e-9, k
        assert np.abs(V[off:off + n] - r["v"]).max() < 1e-9, k
        np.testing.assert_allclose(th[:, k, :], r["thermo"][[20, 40, 60]], rtol=1e-9, atol=1e-9)
        off += n


def test_batch_equals_single_box_runs_bitwise():
    states = _states()
    g = _batch(states)
    g.integrate(45)
    P, V, _ = g.get_state()
    g.sync()
    off = 0
    for p, v, L, eps, sig in states:
        n = p.shape[0]
        s = System(n, L, epsilon=eps, sigma=sig, max_neighbors=160)
        s.set_state(torch.from_numpy(p), torch.from_numpy(v))
        s.integrate(45)
        p1, v1, _ = s.get_state()
        s.sync()
        assert torch.equal(p1, P[off:off + n]) and torch.equal(v1, V[off:off + n])
        off += n


@pytest.mark.parametrize("threads,lds,edge,parts,lpa,bthreads", [
    (64, 0, 2, 1, 1, 0), (128, 0, 2, 1, 1, 0), (192, 0, 2, 1, 1, 0), (256, 0, 2, 1, 1, 0), (0, 64, 2, 1, 1, 0),
    (0, 0, 3, 1, 1, 0), (384, 0, 3, 1, 1, 0), (1024, 0, 3, 1, 1, 0), (0, 64, 3, 1, 1, 0), (0, 0, 2, 2, 1, 0),
    (64, 0, 2, 4, 1, 0), (0, 0, 3, 2, 1, 0), (128, 0, 3, 4, 1, 0), (0, 64, 3, 4, 1, 0), (0, 0, 2, 1, 2, 0),
    (128, 0, 2, 2, 2, 0), (0, 64, 2, 1, 2, 0), (0, 0, 3, 1, 2, 0), (256, 0, 3, 4, 2, 0), (0, 64, 3, 2, 2, 0),
    (0, 0, 2, 1, 4, 0), (0, 64, 2, 2, 4, 0), (512, 0, 3, 1, 4, 0), (0, 0, 2, 1, 1, 64), (0, 64, 3, 1, 2, 64),
    (0, 0, 3, 2, 1, 1024), (0, 64, 2, 1, 4, 1024), (0, 0, 2, 1, 1, -2), (0, 0, 3, 2, 2, -2), (0, 64, 2, 1, 1, -2),
    (64, 0, 3, 4, 1, -2), (0, 1536, 2, 1, 1, 0), (0, 1536, 2, 1, 1, -2), (0, 3072, 3, 1, 2, 0)])
def test_schedule_does_not_change_trajectory(threads, lds, edge, parts, lpa, bthreads):
    """Any schedule gives the trajectory of the default one bit for bit -
    against the default with the same lanes per atom (two lanes sum each
    atom's force as two interleaved halves, a different rounding).  The list
    build visits candidates in one order on every path: lds_atoms 64 sends
    every neighborhood to global gathers, 1536 (E = 2) and 3072 (E = 3) leave
    room for the force kernel's copy but not for the build's subcell-row copy
    (global gathers writing LDS slots)."""
    s = md_system(9, seed=21)  # 5 cells per axis: edge blocks 1 (E = 2) or 2 (E = 3) cells thick
    ref = System(s.n, s.L)
    ref.set_schedule(lanes_per_atom=lpa)
    ref.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    ref.integrate(30)
    p0, v0, _ = ref.get_state()
    g = System(s.n, s.L)
    # bthreads -2: two lanes per atom in the list build, at its default threads
    g.set_schedule(threads=threads, lds_atoms=lds, block_edge=edge, block_parts=parts, lanes_per_atom=lpa,
                   build_threads=max(bthreads, 0), build_lanes=2 if bthreads == -2 else 0)
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    g.integrate(30)
    p1, v1, _ = g.get_state()
    g.sync()
    ref.sync()
    assert torch.equal(p0, p1) and torch.equal(v0, v1)


@pytest.mark.parametrize("lpa,sched", [(1, dict(block_edge=2)), (1, dict(block_edge=3)), (1, dict(lds_atoms=64)),
                                        (1, dict(block_edge=3, block_parts=2)), (2, dict(lds_atoms=64)),
                                        (2, dict(block_edge=3, threads=512)), (4, dict(block_edge=2, lds_atoms=64)),
                                        (1, dict(build_lanes=2)), (2, dict(block_edge=3, build_lanes=2))])
def test_image_path_schedules_bitwise(lpa, sched):
    """8 cells per axis (>= E + 4 for both block edges): blocks stage their
    neighborhood moved to periodic images near the block and take plain
    differences; a neighborhood too large for LDS (lds_atoms=64) takes the
    partner's nearest image per pair from global memory instead.  Both give
    the same trajectory bit for bit, at either block edge."""
    s = md_system(14, seed=23)
    ref = System(s.n, s.L)
    assert ref.info()["cells_per_axis"] == 8
    ref.set_schedule(lanes_per_atom=lpa)
    ref.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    ref.integrate(30)
    p0, v0, _ = ref.get_state()
    g = System(s.n, s.L)
    g.set_schedule(lanes_per_atom=lpa, **sched)
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    g.integrate(30)
    p1, v1, _ = g.get_state()
    g.sync()
    ref.sync()
    assert torch.equal(p0, p1) and torch.equal(v0, v1)


def test_autotune_keeps_state():
    s = md_system(10, seed=22)
    g = System(s.n, s.L)
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    g.integrate(5)
    p0, v0, _ = g.get_state()
    sc = g.autotune(repeats=2)
    p1, v1, _ = g.get_state()
    g.sync()
    assert sc["block_edge"] in (2, 3) and sc["block_parts"] in (1, 2, 4) and sc["lanes_per_atom"] in (1, 2, 4)
    assert sc["block_threads"] % 64 == 0 and 64 <= sc["block_threads"] <= 1024
    assert sc["build_threads"] % 64 == 0 and 64 <= sc["build_threads"] <= 1024 and sc["build_lanes"] in (1, 2)
    assert torch.equal(p0, p1) and torch.equal(v0, v1)


def test_autotune_cache_applies_the_stored_schedule(tmp_path):
    s = md_system(10, seed=23)
    cache = str(tmp_path / "tune.json")
    picks = []
    for _ in range(2):
        g = System(s.n, s.L)
        g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
        g.integrate(5)
        picks.append((g.autotune(repeats=2, cache=cache), g.info()))
        g.integrate(25)  # runs on the applied schedule (list rebuilt)
        g.sync()
        g.close()
    (first, info1), (second, info2) = picks
    assert first["cached"] is False and second["cached"] is True
    keys = ("block_threads", "lds_atoms", "block_edge", "block_parts", "lanes_per_atom", "build_threads",
            "build_lanes", "half_list", "layout")
    assert {k: first[k] for k in keys} == {k: second[k] for k in keys}
    assert all(info1[k] == info2[k] for k in keys)


def test_replica_workload_generator_batch_small():
    """A slice of the 512-box replica workload (first 12 boxes) through the
    batch path, 40 steps, each box against the oracle."""
    specs = batched_box_specs()[:12]
    systems = [md_system(n, rho, T, seed=seed) for n, rho, T, seed in specs]
    g = System.batch([s.n for s in systems], [s.L for s in systems], max_neighbors_default())
    g.set_state(torch.from_numpy(np.concatenate([s.pos() for s in systems])),
                torch.from_numpy(np.concatenate([s.vel() for s in systems])))
    g.integrate(40)
    P, _, _ = g.get_state()
    g.sync()
    P = P.cpu().numpy()
    off = 0
    for s in systems:
        r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 40, thermo=False)
        assert np.abs(_mic(P[off:off + s.n] - r["x"], s.L)).max() < 1e-9
        off += s.n


def max_neighbors_default():
    return {"max_neighbors": 160}
