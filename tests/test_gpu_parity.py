"""HIP path against the CPU oracle, element by element, through the C ABI.

Bars: neighbor sets bit-exact (sorted per atom, original ids); forces within
1e-12 of each atom's conditioning scale sum_j |f_ij x_ij|; energy and virial
within 1e-12 relative; positions within 1e-9 (minimum-image difference)
after 100 steps.
"""

import numpy as np
import pytest

import oracle
from images_helper import wrong_staged_images
from workloads import SplitMix64, fcc_positions, md_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_2009_07400_amd import System, TmdError  # noqa: E402
from paper_2009_07400_amd import _abi as abi  # noqa: E402

FORCE_TOL = 1e-12
POS_TOL = 1e-9


def _mic(d, L):
    return d - L * np.round(d / L)


def _gpu_system(pos, vel, L, **kw):
    s = System(pos.shape[0], L, **kw)
    s.set_state(torch.from_numpy(pos), torch.from_numpy(vel))
    return s


def _check_lists(sysg, pos, L, r=2.8):
    counts, ids = sysg.get_neighbors()
    sysg.sync()
    counts = counts.cpu().numpy()
    ids = ids.cpu().numpy()
    c_o, n_o, _ = oracle.build_list(pos[:, 0], pos[:, 1], pos[:, 2], L, r, maxnb=ids.shape[1])
    assert np.array_equal(counts, c_o)
    for i in range(pos.shape[0]):
        assert np.array_equal(ids[i, : counts[i]], n_o[i, : c_o[i]]), i
    assert (ids[np.arange(ids.shape[1])[None, :] >= counts[:, None]] == -1).all()
    return c_o, n_o


def _check_forces(sysg, pos, L, c_o, n_o, eps=1.0, sigma=1.0):
    F, ev = sysg.compute_forces()
    sysg.sync()
    F = F.cpu().numpy()
    U, W = ev.cpu().numpy()
    Fo, sc, Uo, Wo = oracle.forces(pos[:, 0], pos[:, 1], pos[:, 2], L, c_o, n_o, eps=eps, sigma=sigma)
    err = np.linalg.norm(F - Fo, axis=1)
    assert (err <= FORCE_TOL * np.maximum(sc, 1e-300)).all(), float((err / np.maximum(sc, 1e-300)).max())
    assert U == pytest.approx(Uo, rel=FORCE_TOL, abs=1e-12)
    assert W == pytest.approx(Wo, rel=FORCE_TOL, abs=1e-12)
    return F


def _liquid(ncell, steps=40, seed=1000, T=1.44, rho=0.8442):
    s = md_system(ncell, rho, T, seed=seed)
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, steps, thermo=False)
    return r["x"], r["v"], s.L


CASES = {
    "fcc8": lambda: (lambda s: (s.pos(), s.vel(), s.L))(md_system(8)),
    "liquid8": lambda: _liquid(8),
    "nc2_liquid4": lambda: _liquid(4, seed=7),
    "nc3_liquid6": lambda: _liquid(6, seed=8),
    "jitter7": lambda: (lambda s: (s.pos(), s.vel(), s.L))(md_system(7, jitter=0.02, seed=1002)),
    "ragged_uniform": lambda: (SplitMix64(5).next_double(3 * 1001).reshape(1001, 3) * 12.5,
                               np.zeros((1001, 3)), 12.5),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("build_lanes", [1, 2])
def test_neighbors_and_forces_match_oracle(case, build_lanes):
    pos, vel, L = CASES[case]()
    g = _gpu_system(pos, vel, L, max_neighbors=256)
    g.set_schedule(build_lanes=build_lanes)
    g.build_neighbors()
    c_o, n_o = _check_lists(g, pos, L)
    _check_forces(g, pos, L, c_o, n_o)


@pytest.mark.parametrize("lpa,lds,bl", [(1, 0, 1), (2, 0, 1), (4, 0, 1), (4, 64, 1), (1, 0, 2), (2, 64, 2)])
def test_short_list_capacity_and_lanes_per_atom(lpa, lds, bl):
    """A dilute gas with max_neighbors = 8 (a list area of three rows): the
    force kernel's row look-ahead and the build's padding stay inside each
    atom's area for every lanes-per-atom setting of either kernel."""
    pos = SplitMix64(11).next_double(3 * 300).reshape(300, 3) * 30.0
    g = _gpu_system(pos, np.zeros_like(pos), 30.0, max_neighbors=8)
    g.set_schedule(lanes_per_atom=lpa, lds_atoms=lds, build_lanes=bl)
    g.build_neighbors()
    c_o, n_o = _check_lists(g, pos, 30.0)
    assert c_o.max() <= 8
    _check_forces(g, pos, 30.0, c_o, n_o)


def test_fcc_lattice_sums_on_gpu():
    pos, L = fcc_positions(8, 0.8442)
    g = _gpu_system(pos, np.zeros_like(pos), L)
    g.build_neighbors()
    F, ev = g.compute_forces()
    g.sync()
    U, W = ev.cpu().numpy()
    n = pos.shape[0]
    assert U / n == pytest.approx(-6.773368053252957, rel=1e-12)
    assert W / n == pytest.approx(-22.158199254035498, rel=1e-12)
    counts, _ = g.get_neighbors()
    assert (counts.cpu().numpy() == 78).all()
    assert (g.neighbor_counts().cpu().numpy() == 78).all()  # counts-only export


def test_parameters_epsilon_sigma():
    pos, vel, L = _liquid(6, seed=9)
    g = _gpu_system(pos, vel, L, epsilon=1.05, sigma=0.98)
    g.build_neighbors()
    c_o, n_o = _check_lists(g, pos, L)
    _check_forces(g, pos, L, c_o, n_o, eps=1.05, sigma=0.98)


def test_single_and_two_atoms():
    L = 8.0
    pos = np.array([[1.0, 1.0, 1.0]])
    g = _gpu_system(pos, np.zeros((1, 3)), L)
    g.build_neighbors()
    F, ev = g.compute_forces()
    g.sync()
    assert (F.cpu().numpy() == 0).all() and (ev.cpu().numpy() == 0).all()
    # two atoms across the periodic face at the potential minimum
    r0 = 2 ** (1 / 6)
    pos = np.array([[0.1, 4.0, 4.0], [0.1 - r0 + L, 4.0, 4.0]])
    g = _gpu_system(pos, np.zeros((2, 3)), L)
    g.build_neighbors()
    F, _ = g.compute_forces()
    g.sync()
    assert np.abs(F.cpu().numpy()).max() < 1e-13


def _run_both(pos, vel, L, steps, thermo_every=0, **kw):
    g = _gpu_system(pos, vel, L, **kw)
    th = g.integrate(steps, thermo_every=thermo_every)
    p, v, step = g.get_state()
    g.sync()
    okw = {k: kw[k] for k in ("epsilon", "sigma", "rebuild_every") if k in kw}
    r = oracle.run(pos[:, 0], pos[:, 1], pos[:, 2], vel[:, 0], vel[:, 1], vel[:, 2], L, steps, **okw)
    return p.cpu().numpy(), v.cpu().numpy(), step, (th.cpu().numpy() if th is not None else None), r


def test_trajectory_100_steps_config0():
    s = md_system(8, seed=1000)
    p, v, step, th, r = _run_both(s.pos(), s.vel(), s.L, 100, thermo_every=1)
    assert step == 100
    assert np.abs(_mic(p - r["x"], s.L)).max() < POS_TOL
    assert np.abs(v - r["v"]).max() < POS_TOL
    assert th.shape == (100, 5)
    np.testing.assert_allclose(th, r["thermo"][1:], rtol=1e-9, atol=1e-9)


def test_split_integrate_is_bitwise_identical():
    s = md_system(6, seed=11)
    g1 = _gpu_system(s.pos(), s.vel(), s.L)
    g1.integrate(100)
    p1, v1, _ = g1.get_state()
    g2 = _gpu_system(s.pos(), s.vel(), s.L)
    g2.integrate(37)
    g2.integrate(1)
    g2.integrate(62)
    p2, v2, step = g2.get_state()
    g1.sync()
    g2.sync()
    assert step == 100
    assert torch.equal(p1, p2) and torch.equal(v1, v2)


def test_runs_are_deterministic():
    s = md_system(7, seed=12)
    out = []
    for _ in range(2):
        g = _gpu_system(s.pos(), s.vel(), s.L)
        th = g.integrate(60, thermo_every=20)
        p, v, _ = g.get_state()
        g.sync()
        out.append((p.cpu(), v.cpu(), th.cpu()))
    assert all(torch.equal(a, b) for a, b in zip(out[0], out[1]))


def test_rebuild_schedule_and_small_box_trajectory():
    p0, v0, L = _liquid(4, steps=5, seed=13)  # two cells per axis
    p, v, step, _, r = _run_both(p0, v0, L, 60, rebuild_every=7)
    assert np.abs(_mic(p - r["x"], L)).max() < POS_TOL
    assert np.abs(v - r["v"]).max() < POS_TOL


@pytest.mark.parametrize("build_lanes", [1, 2])
def test_error_overflow_is_deferred(build_lanes):
    s = md_system(5)
    g = _gpu_system(s.pos(), s.vel(), s.L, max_neighbors=8)
    g.set_schedule(build_lanes=build_lanes)
    g.build_neighbors()
    with pytest.raises(TmdError) as e:
        g.sync()
    assert e.value.status == abi.TMD_ENBR_OVERFLOW
    assert "78" in str(e.value)


def test_overflowing_lists_keep_the_same_entries_on_both_build_paths():
    """With max_neighbors below every list's length both list builds store
    the same first max_neighbors candidates of the canonical walk (the
    16-bit entries past the capacity are dropped on both paths alike)."""
    s = md_system(5)
    out = []
    for lanes in (1, 2):
        g = _gpu_system(s.pos(), s.vel(), s.L, max_neighbors=8)
        g.set_schedule(build_lanes=lanes)
        g.build_neighbors()
        counts, ids = g.get_neighbors()
        with pytest.raises(TmdError) as e:
            g.sync()
        assert e.value.status == abi.TMD_ENBR_OVERFLOW
        out.append((counts.cpu().numpy(), ids.cpu().numpy()))
        g.close()
    (c1, i1), (c2, i2) = out
    assert (c1 == 8).all() and np.array_equal(c1, c2) and np.array_equal(i1, i2)
    assert (i1 >= 0).all() and (i1 < s.n).all()
    assert not (i1 == np.arange(s.n)[:, None]).any()  # no atom lists itself


def test_error_nonfinite_and_call_order():
    s = md_system(5)
    pos = s.pos()
    g = _gpu_system(pos, s.vel(), s.L)
    with pytest.raises(TmdError) as e:
        g.compute_forces()
    assert e.value.status == abi.TMD_ESTATE
    pos = pos.copy()
    pos[3] = pos[4]  # coincident atoms
    g.set_state(torch.from_numpy(pos), torch.from_numpy(s.vel()))
    g.build_neighbors()
    g.compute_forces()
    with pytest.raises(TmdError) as e:
        g.sync()
    assert e.value.status == abi.TMD_ENONFINITE
    pos[3, 0] = np.nan
    g.set_state(torch.from_numpy(pos), torch.from_numpy(s.vel()))
    with pytest.raises(TmdError) as e:
        g.sync()
    assert e.value.status == abi.TMD_ENONFINITE
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    g.integrate(3)
    g.sync()  # cleared by set_state


@pytest.mark.parametrize("ncell,jitter,seed", [(32, 0.0, 1001), (96, 0.02, 1002)])
def test_full_size_sampled_parity(ncell, jitter, seed):
    """Benchmark sizes (131,072 and 3,538,944 atoms): the list and forces of
    sampled atoms against the oracle's all-pairs definitions, plus the
    lattice invariant that every atom has exactly 78 neighbors."""
    s = md_system(ncell, jitter=jitter, seed=seed)
    pos = s.pos()
    g = _gpu_system(pos, s.vel(), s.L)
    g.build_neighbors()
    F, ev = g.compute_forces()
    counts, ids = g.get_neighbors()
    g.sync()
    counts = counts.cpu().numpy()
    assert (counts == 78).all()
    idx = np.unique(SplitMix64(seed).next_u64(48) % np.uint64(s.n)).astype(np.int64)
    idx = np.concatenate([idx, [0, s.n - 1]])
    rows = ids[torch.from_numpy(idx).to(ids.device)].cpu().numpy()
    Fs = F[torch.from_numpy(idx).to(F.device)].cpu().numpy()
    for k, i in enumerate(idx):
        nb = oracle.atom_neighbors(s.x, s.y, s.z, s.L, 2.8, int(i))
        assert np.array_equal(rows[k, :78], nb)
        fo, sc = oracle.atom_force(s.x, s.y, s.z, s.L, int(i))
        assert np.linalg.norm(Fs[k] - fo) <= FORCE_TOL * sc
    U, W = ev.cpu().numpy()
    if jitter == 0.0:
        assert U / s.n == pytest.approx(-6.773368053252957, rel=1e-12)
        assert W / s.n == pytest.approx(-22.158199254035498, rel=1e-12)


@pytest.mark.parametrize("edge,n", [(2, 9), (3, 11)])
def test_checked_images_after_large_drift(edge, n):
    """Boxes of E + 3 cells per axis stage each neighborhood at the images
    nearest to its block and test every difference against L/2.  Here the
    atoms fly up to three sigma (ballistic: a negligible epsilon) on the
    list of the first step, so some partners' staged images are not the
    ones nearest to their atom (about 150 pairs): those pairs take the
    minimum image per pair, and the forces of the kept list match the
    oracle's."""
    s = md_system(n, seed=31 + n)
    rng = np.random.default_rng(n)
    u = rng.standard_normal((s.n, 3))
    vel = u / np.linalg.norm(u, axis=1, keepdims=True) * rng.uniform(0.0, 60.0, (s.n, 1))
    g = System(s.n, s.L, epsilon=1e-30, rebuild_every=1000)
    assert g.info()["cells_per_axis"] == edge + 3
    g.set_schedule(block_edge=edge)
    x0 = s.pos()
    g.set_state(torch.from_numpy(x0), torch.from_numpy(vel))
    g.integrate(10)  # the list of step 0 stays: rebuild every 1000 steps
    g.set_lj_params([1.0], [1.0])
    F, ev = g.compute_forces()
    p, _, _ = g.get_state()
    counts, ids = g.get_neighbors()
    g.sync()
    x = p.cpu().numpy()
    c0, n0, _ = oracle.build_list(x0[:, 0], x0[:, 1], x0[:, 2], s.L, 2.8, maxnb=160)
    assert np.array_equal(counts.cpu().numpy(), c0)  # still the list of step 0
    assert wrong_staged_images(x0, x, s.L, c0, n0, edge) > 0
    Fo, scale, Uo, Wo = oracle.forces(x[:, 0], x[:, 1], x[:, 2], s.L, c0, n0)
    err = np.linalg.norm(F.cpu().numpy() - Fo, axis=1)
    assert (err <= FORCE_TOL * np.maximum(scale, 1e-300)).all(), float((err / np.maximum(scale, 1e-300)).max())
    U, W = ev.cpu().numpy().reshape(-1)[:2]
    assert U == pytest.approx(Uo, rel=FORCE_TOL) and W == pytest.approx(Wo, rel=FORCE_TOL)
    g.close()
