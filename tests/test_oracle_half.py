"""Pins of the oracle's half neighbor list and its Newton's-third-law forces
(Sec. 3.2, the half-list paragraph; the half_nb variant of Sec. 4.2) that do
not come from the half-list code itself: every unordered pair of the full
list exactly once, forces equal to the all-pairs definition of each atom's
force and to the full-list sum, total momentum conserved, energy and virial
equal to the full list's."""

import numpy as np
import pytest

import oracle
from workloads import md_system


def _liquid(ncell, seed, steps=30):
    s = md_system(ncell, 0.8442, 1.44, seed=seed)
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, steps, thermo=False)
    return r["x"], s.L


@pytest.mark.parametrize("ncell,seed", [(5, 11), (4, 12)])
def test_half_list_holds_every_pair_once(ncell, seed):
    x, L = _liquid(ncell, seed)
    c, nb, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, 2.8, maxnb=160)
    hc, hn = oracle.half_list(c, nb)
    full = {(min(i, j), max(i, j)) for i in range(x.shape[0]) for j in nb[i, : c[i]]}
    half = [(i, j) for i in range(x.shape[0]) for j in hn[i, : hc[i]]]
    assert len(half) == len(set(half)) == len(full) == int(c.sum()) // 2
    assert set(half) == full and all(i < j for i, j in half)


@pytest.mark.parametrize("ncell,seed", [(5, 21), (6, 22)])
def test_half_list_forces_equal_all_pairs_and_full_list(ncell, seed):
    x, L = _liquid(ncell, seed)
    c, nb, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, 2.8, maxnb=160)
    F, sc, U, W = oracle.forces(x[:, 0], x[:, 1], x[:, 2], L, c, nb)
    hc, hn = oracle.half_list(c, nb)
    Fh, Uh, Wh = oracle.forces_half(x[:, 0], x[:, 1], x[:, 2], L, hc, hn)
    assert (np.linalg.norm(Fh - F, axis=1) <= 1e-13 * sc).all()
    for i in range(0, x.shape[0], 7):  # the all-pairs definition, no list
        Fi, sci = oracle.atom_force(x[:, 0], x[:, 1], x[:, 2], L, i)
        assert np.linalg.norm(Fh[i] - Fi) <= 1e-13 * sci, i
    assert np.abs(Fh.sum(0)).max() <= 1e-13 * sc.sum()  # each pair adds f d and -f d
    assert Uh == pytest.approx(U, rel=1e-13) and Wh == pytest.approx(W, rel=1e-13)


def test_half_list_energy_equals_numpy_all_pairs():
    x, L = _liquid(4, 31)
    c, nb, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], L, 2.8, maxnb=160)
    hc, hn = oracle.half_list(c, nb)
    _, Uh, Wh = oracle.forces_half(x[:, 0], x[:, 1], x[:, 2], L, hc, hn)
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.round(d / L)
    s = (d * d).sum(-1)
    iu = np.triu_indices(x.shape[0], 1)
    s = s[iu]
    s = s[s < 2.5 ** 2]
    q = (1.0 / s) ** 3
    assert Uh == pytest.approx((4.0 * (q * q - q)).sum(), rel=1e-12)
    assert Wh == pytest.approx((24.0 * q * (2.0 * q - 1.0)).sum(), rel=1e-12)  # sum of s f(s)
