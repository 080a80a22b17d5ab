"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses a closed form,
an invariant, a textbook special case or an independent brute force.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from workloads import SplitMix64, fcc_positions, md_system

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _mic_np(d, L):
    return d - L * np.round(d / L)


# ---------------------------------------------------------------- generator

def test_splitmix64_published_vector():
    g = json.load(open(os.path.join(GOLD, "splitmix64_vector.json")))
    out = SplitMix64(g["seed"]).next_u64(5)
    assert [int(v) for v in out] == [int(s) for s in g["outputs"]]


def test_fcc_workload_shape():
    s = md_system(8, 0.8442, 1.44, seed=1000)
    assert s.n == 2048
    assert s.L == pytest.approx(8 * (4 / 0.8442) ** (1 / 3), rel=1e-15)
    v = s.vel()
    assert np.abs(v.mean(axis=0)).max() < 1e-15
    assert np.sum(v * v) / (3 * s.n - 3) == pytest.approx(1.44, rel=1e-14)
    j = md_system(6, jitter=0.02, seed=1002)
    p, _ = fcc_positions(6, 0.8442)
    d = _mic_np(j.pos() - p, j.L)
    assert np.abs(d).max() <= 0.01 + 1e-12 and np.abs(d).max() > 0.009
    assert j.pos().min() >= 0.0 and j.pos().max() < j.L


def test_paper_setup_constants():
    g = json.load(open(os.path.join(GOLD, "paper_benchmark_setup.json")))
    assert (g["epsilon"], g["sigma"], g["cutoff"], g["verlet_buffer"]) == (1.0, 1.0, 2.5, 0.3)
    assert 4 * g["cpu_unit_cells_per_axis"] ** 3 == 131072
    assert 4 * g["cpu_weak_scaling_unit_cells_per_axis_per_node"] ** 3 == 3538944


# ---------------------------------------------------------------- pair law

def test_force_zero_at_potential_minimum():
    # V'(r) = 0 at r = 2^(1/6) sigma, so the pair force vanishes there
    for sigma in (1.0, 0.98, 1.3):
        r = 2 ** (1 / 6) * sigma
        assert abs(oracle.pair_force(r * r, 1.0, sigma) * r) < 1e-13


def test_force_at_cutoff_and_listing_equivalence():
    # closed value at the cutoff: |F(2.5)| = 24 (2 * 2.5^-12 - 2.5^-6) / 2.5
    r = 2.5
    assert oracle.pair_force(r * r) * r == pytest.approx(-0.0389994774528, abs=1e-12)
    # the oracle follows Eq. 2; the compute_potential example of Sec. 4.2
    # writes the same factor as 48 sr6 (sr6 - 1/2) sr2 eps with sr2 = 1/s and
    # sr6 = sr2^3 sigma^6, an algebraically different evaluation
    for s in np.linspace(0.7, 6.5, 37):
        for eps, sig in ((1.0, 1.0), (1.05, 0.98), (0.5, 1.2)):
            sr2 = 1.0 / s
            sr6 = sr2 * sr2 * sr2 * sig ** 6
            listing = 48.0 * sr6 * (sr6 - 0.5) * sr2 * eps
            assert oracle.pair_force(s, eps, sig) == pytest.approx(listing, rel=1e-13)


def test_force_is_minus_energy_gradient():
    # F(r) = -dV/dr along x_ij: f(s) * r = -V'(r); central difference on V
    for r in (0.95, 1.1, 1.5, 2.0, 2.45):
        for eps, sig in ((1.0, 1.0), (1.05, 0.98)):
            hstep = 1e-6
            dv = (oracle.pair_energy((r + hstep) ** 2, eps, sig) - oracle.pair_energy((r - hstep) ** 2, eps, sig)) / (2 * hstep)
            assert oracle.pair_force(r * r, eps, sig) * r == pytest.approx(-dv, rel=1e-7, abs=1e-9)
    assert oracle.pair_energy(1.0) == 0.0  # V(sigma) = 0
    assert oracle.pair_energy(2 ** (1 / 3)) == pytest.approx(-1.0, rel=1e-15)  # well depth eps


# ---------------------------------------------------------------- lists

def _fcc_shells(a, rmax):
    """FCC shells from lattice vectors (h,k,l)*a/2 with h+k+l even."""
    shells = {}
    R = int(2 * rmax / a) + 2
    for h, k, l in itertools.product(range(-R, R + 1), repeat=3):
        if (h + k + l) % 2 or (h, k, l) == (0, 0, 0):
            continue
        q = h * h + k * k + l * l
        if a / 2 * math.sqrt(q) < rmax:
            shells[q] = shells.get(q, 0) + 1
    return [(a / 2 * math.sqrt(q), m) for q, m in sorted(shells.items())]


@pytest.mark.parametrize("rho", [0.75, 0.8442, 0.90])
def test_fcc_neighbor_counts(rho):
    pos, L = fcc_positions(8, rho)
    a = (4 / rho) ** (1 / 3)
    n28 = sum(m for r, m in _fcc_shells(a, 2.8))
    n25 = sum(m for r, m in _fcc_shells(a, 2.5))
    assert (n25, n28) == (54, 78)
    c, _, _ = oracle.build_list(pos[:, 0], pos[:, 1], pos[:, 2], L, 2.8)
    assert (c == 78).all()
    c, _, _ = oracle.build_list(pos[:, 0], pos[:, 1], pos[:, 2], L, 2.5)
    assert (c == 54).all()


def test_jittered_lattice_counts():
    s = md_system(12, jitter=0.02, seed=1002)
    c, _, _ = oracle.build_list(s.x, s.y, s.z, s.L, 2.8)
    assert (c == 78).all()


def test_fcc_energy_virial_closed_form():
    rho = 0.8442
    a = (4 / rho) ** (1 / 3)
    u = sum(0.5 * m * 4 * (r ** -12 - r ** -6) for r, m in _fcc_shells(a, 2.5))
    w = sum(0.5 * m * 24 * (2 * r ** -12 - r ** -6) for r, m in _fcc_shells(a, 2.5))
    assert u == pytest.approx(-6.773368053252957, rel=1e-13)
    assert w == pytest.approx(-22.158199254035498, rel=1e-13)
    pos, L = fcc_positions(8, rho)
    c, nb, _ = oracle.build_list(pos[:, 0], pos[:, 1], pos[:, 2], L, 2.8)
    F, sc, U, W = oracle.forces(pos[:, 0], pos[:, 1], pos[:, 2], L, c, nb)
    n = pos.shape[0]
    assert U / n == pytest.approx(u, rel=1e-12)
    assert W / n == pytest.approx(w, rel=1e-12)
    assert np.abs(F).max() < 1e-12 * sc.max()


@pytest.mark.slow
def test_fcc_energy_virial_closed_form_at_131k_atoms():
    """The same lattice sums over 32^3 unit cells: 131,072 equal per-atom
    terms, whose plain left-to-right total drifts by 2e-12 from the exact
    sum; the oracle's totals stay within 1e-14 of it."""
    rho = 0.8442
    pos, L = fcc_positions(32, rho)
    c, nb, _ = oracle.build_list(pos[:, 0], pos[:, 1], pos[:, 2], L, 2.8, maxnb=128)
    _, _, U, W = oracle.forces(pos[:, 0], pos[:, 1], pos[:, 2], L, c, nb)
    n = pos.shape[0]
    assert U / n == pytest.approx(-6.773368053252957, rel=1e-14)
    assert W / n == pytest.approx(-22.158199254035498, rel=1e-14)


def _liquid(ncell=6, steps=30, seed=1000, T=1.44, rho=0.8442):
    s = md_system(ncell, rho, T, seed=seed)
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, steps, thermo=False)
    return r["x"], s.L


def _uniform(n, L, seed):
    u = SplitMix64(seed).next_double(3 * n).reshape(n, 3)
    return u * L


@pytest.mark.parametrize("case", ["liquid6", "jitter5", "nc2", "nc3", "uniform", "tiny"])
def test_cell_list_equals_all_pairs(case):
    if case == "liquid6":
        x, L = _liquid(7)
        assert oracle.cells_per_axis(L, 2.8) == 4
    elif case == "jitter5":
        s = md_system(5, jitter=0.3, seed=7)
        x, L = s.pos(), s.L
    elif case == "nc2":  # 4^3 cells: L = 6.72 -> 2 cells per axis, stencil deduplicated to 8 cells
        x, L = _liquid(4)
        assert oracle.cells_per_axis(L, 2.8) == 2
    elif case == "nc3":
        x, L = _liquid(6, seed=3)
        assert oracle.cells_per_axis(L, 2.8) == 3
    elif case == "uniform":
        L = 12.0
        x = _uniform(900, L, 11)
    else:
        L = 6.0
        x = _uniform(7, L, 12)
    c1, n1, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, 2.8, maxnb=400)
    c2, n2, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, 2.8, maxnb=400, brute=True)
    assert oracle.list_as_sets(c1, n1) == oracle.list_as_sets(c2, n2)
    # independent numpy brute force over all image-free pairs
    d = _mic_np(x[:, None, :] - x[None, :, :], L)
    s = (d * d).sum(-1)
    np.fill_diagonal(s, np.inf)
    assert (c1 == (s < 2.8 ** 2).sum(1)).all()


@pytest.mark.parametrize("case", ["liquid6", "jitter5", "nc2", "uniform"])
def test_atom_neighbors_equals_all_pairs(case):
    """orc_atom_neighbors (the per-atom list checker used at full size) against
    the cell-list build and an independent numpy all-pairs distance matrix,
    for every atom of the box."""
    if case == "liquid6":
        x, L = _liquid(7)
    elif case == "jitter5":
        s = md_system(5, jitter=0.3, seed=7)
        x, L = s.pos(), s.L
    elif case == "nc2":
        x, L = _liquid(4)
    else:
        L = 12.0
        x = _uniform(900, L, 11)
    c, nb, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, 2.8, maxnb=400)
    d = _mic_np(x[:, None, :] - x[None, :, :], L)
    s2 = (d * d).sum(-1)
    np.fill_diagonal(s2, np.inf)
    for i in range(x.shape[0]):
        got = oracle.atom_neighbors(x[:, 0], x[:, 1], x[:, 2], L, 2.8, i)
        assert np.array_equal(got, nb[i, : c[i]]), i
        assert np.array_equal(got, np.nonzero(s2[i] < 2.8 ** 2)[0]), i


# ---------------------------------------------------------------- forces

def test_forces_equal_numpy_all_pairs():
    x, L = _liquid(4)
    c, nb, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, 2.8)
    F, sc, U, W = oracle.forces(x[:, 0], x[:, 1], x[:, 2], L, c, nb)
    d = _mic_np(x[:, None, :] - x[None, :, :], L)
    s = (d * d).sum(-1)
    np.fill_diagonal(s, np.inf)
    m = s < 6.25
    q = np.where(m, 1.0 / s ** 3, 0.0)
    f = np.where(m, 24.0 * q * (2.0 * q - 1.0) / s, 0.0)  # Eq. 2 form
    Fn = (f[:, :, None] * d).sum(1)
    assert np.abs(F - Fn).max() <= 1e-12 * sc.max()
    Un = 0.5 * np.where(m, 4.0 * (q * q - q), 0.0).sum()
    Wn = 0.5 * (np.where(m, s, 0.0) * f).sum()
    assert U == pytest.approx(Un, rel=1e-12)
    assert W == pytest.approx(Wn, rel=1e-12)
    for i in (0, 17, 255):
        fi, sci = oracle.atom_force(x[:, 0], x[:, 1], x[:, 2], L, i)
        assert np.abs(fi - F[i]).max() <= 1e-13 * sci


def test_newton_third_law_and_translation():
    x, L = _liquid(6)
    c, nb, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, 2.8)
    F, sc, U, _ = oracle.forces(x[:, 0], x[:, 1], x[:, 2], L, c, nb)
    assert np.abs(F.sum(0)).max() <= 1e-13 * np.abs(F).sum()
    shift = np.array([0.37, -5.1, 2.25])
    y = np.mod(x + shift, L)
    c2, nb2, _ = oracle.build_list(y[:, 0], y[:, 1], y[:, 2], L, 2.8)
    assert oracle.list_as_sets(c, nb) == oracle.list_as_sets(c2, nb2)
    F2, _, U2, _ = oracle.forces(y[:, 0], y[:, 1], y[:, 2], L, c2, nb2)
    assert np.abs(F2 - F).max() <= 1e-12 * sc.max()
    assert U2 == pytest.approx(U, rel=1e-12)


def test_rebuild_schedule_uses_stale_list():
    """Between rebuilds the forces come from the list built at the last rebuild
    (fixed schedule, no displacement check): at step 19 of a 20-step window the
    returned forces equal the step-0 list's forces at the step-19 positions."""
    s = md_system(6, seed=5)
    c, nb, _ = oracle.build_list(s.x, s.y, s.z, s.L, 2.8)
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 19, rebuild_every=20, thermo=False)
    x = r["x"]
    F_stale, sc, _, _ = oracle.forces(x[:, 0], x[:, 1], x[:, 2], s.L, c, nb)
    assert np.array_equal(F_stale, r["f"])
    r20 = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 20, rebuild_every=20, thermo=False)
    y = r20["x"]
    c2, nb2, _ = oracle.build_list(y[:, 0], y[:, 1], y[:, 2], s.L, 2.8)
    F_fresh, _, _, _ = oracle.forces(y[:, 0], y[:, 1], y[:, 2], s.L, c2, nb2)
    assert np.array_equal(F_fresh, r20["f"])
