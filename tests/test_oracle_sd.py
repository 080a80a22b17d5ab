"""Pins of the oracle's Spring-Dashpot contact model (Sec. 3.2, Eq. 3) that do
not come from the oracle itself: closed forms of one pair, the damped
oscillator of a head-on collision (its restitution coefficient),
the elastic limit, all-pairs brute force, Newton's third law and
dissipation."""

import math

import numpy as np
import pytest

import oracle
from workloads import sd_system


def test_pair_static_overlap_is_a_linear_spring():
    k, sigma = 250.0, 1.0
    for r in (0.6, 0.9, 0.999):
        d = np.array([r, 0.0, 0.0]) @ np.array([[0.6, 0.8, 0.0], [-0.8, 0.6, 0.0], [0.0, 0.0, 1.0]])
        F, fm = oracle.sd_pair(d, [0.0, 0.0, 0.0], k, 7.0, sigma)
        assert fm == pytest.approx(k * (sigma - r), rel=1e-14)
        assert F == pytest.approx(k * (sigma - r) * d / r, rel=1e-14)  # along x_ij: pushes i away from j
    for r in (1.0, 1.2):  # touching (Theta(0) = 0) and apart
        F, fm = oracle.sd_pair([r, 0.0, 0.0], [-3.0, 1.0, 0.0], k, 7.0, sigma)
        assert fm == 0.0 and not F.any()


def test_pair_dashpot_acts_along_the_normal_only():
    k, g, sigma = 100.0, 3.0, 1.0
    d = np.array([0.0, 0.8, 0.0])
    # approaching along the normal (u . v_ij = -0.5): extra repulsion gamma * 0.5
    F, fm = oracle.sd_pair(d, [0.0, -0.5, 0.0], k, g, sigma)
    assert fm == pytest.approx(k * 0.2 + g * 0.5, rel=1e-14)
    assert F == pytest.approx([0.0, fm, 0.0], rel=1e-14)
    # sliding (v_ij perpendicular to u): no damping
    F2, fm2 = oracle.sd_pair(d, [0.7, 0.0, -0.3], k, g, sigma)
    assert fm2 == pytest.approx(k * 0.2, rel=1e-14)


def _collide(k, gamma, dt, v_in=1.0, m=1.0):
    """Head-on collision of two spheres (diameter 1) starting 0.01 apart;
    returns (restitution coefficient, closed-form contact time)."""
    L = 10.0
    x = np.array([[4.0, 5.0, 5.0], [5.01, 5.0, 5.0]])
    v = np.array([[0.5 * v_in, 0.0, 0.0], [-0.5 * v_in, 0.0, 0.0]])
    mu = 0.5 * m
    tc = math.pi / math.sqrt(k / mu - (gamma / (2 * mu)) ** 2)
    nsteps = int((0.01 / v_in + 1.5 * tc) / dt) + 10
    r = oracle.sd_run(x, v, L, nsteps, k, gamma, sigma=1.0, mass=m, cutoff=1.0, skin=0.3, dt=dt, rebuild_every=20,
                      maxnb=4)
    vout = r["v"][1, 0] - r["v"][0, 0]  # separating: positive
    return vout / v_in, tc


@pytest.mark.parametrize("gamma", [2.0, 5.0, 12.0])
def test_head_on_collision_restitution_closed_form(gamma):
    """Relative motion of two equal spheres in contact is the damped
    oscillator mu d'' = -K d - gamma d' (mu = m / 2), which leaves contact
    after pi / omega_d with restitution exp(-pi zeta / sqrt(1 - zeta^2)),
    zeta = gamma / (2 sqrt(K mu)).  The discrete run converges to it as dt
    shrinks."""
    k, m = 1000.0, 1.0
    mu = 0.5 * m
    zeta = gamma / (2.0 * math.sqrt(k * mu))
    e_exact = math.exp(-math.pi * zeta / math.sqrt(1.0 - zeta * zeta))
    # the contact starts and ends between steps: the error is O(dt) but
    # not monotone in dt
    for dt, tol in ((4e-4, 6e-3), (1e-4, 2e-3), (5e-5, 1e-3)):
        e, _ = _collide(k, gamma, dt)
        assert abs(e - e_exact) < tol * e_exact, (dt, e, e_exact)


def test_elastic_collision_keeps_energy():
    """gamma = 0: the contact is a conservative spring; the spheres leave
    with their speed, to second order in dt."""
    e1, _ = _collide(1000.0, 0.0, 4e-4)
    e2, _ = _collide(1000.0, 0.0, 1e-4)
    assert abs(e1 - 1.0) < 1e-4 and abs(e2 - 1.0) < 1e-5


def test_list_forces_equal_all_pairs_and_newton():
    s = sd_system(6, seed=5)
    x, v, L = s.pos(), s.vel(), s.L
    c, nb, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, s.cutoff + s.skin, maxnb=64)
    F, scale, U, W = oracle.sd_forces(x, v, L, c, nb, s.k, s.gamma, s.sigma)
    assert (scale > 0).sum() > 0.5 * s.n  # most spheres touch something
    for i in range(s.n):
        Fi = oracle.sd_atom_force(x, v, L, i, s.k, s.gamma, s.sigma)
        assert np.abs(F[i] - Fi).max() <= 1e-13 * max(scale[i], 1e-300), i
    assert np.abs(F.sum(0)).max() <= 1e-13 * scale.sum()
    # elastic energy from an independent numpy all-pairs sum
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, np.inf)
    ov = np.clip(s.sigma - r, 0.0, None)
    assert U == pytest.approx(0.25 * s.k * (ov * ov).sum(), rel=1e-12)


def test_damping_dissipates_and_springs_alone_conserve():
    s = sd_system(5, seed=6)
    r0 = oracle.sd_run(s.pos(), s.vel(), s.L, 400, s.k, 0.0, sigma=s.sigma, cutoff=s.cutoff, skin=s.skin, dt=s.dt)
    E = r0["thermo"][:, 4]
    assert np.abs(E - E[0]).max() < 2e-3 * abs(E[0])
    r1 = oracle.sd_run(s.pos(), s.vel(), s.L, 400, s.k, s.gamma, sigma=s.sigma, cutoff=s.cutoff, skin=s.skin,
                       dt=s.dt)
    E1 = r1["thermo"][:, 4]
    assert E1[-1] < 0.9 * E1[0]
    # E never rises by more than the O(dt^2) error of the conservative part
    assert (np.diff(E1) < 2e-3 * abs(E1[0])).all()
