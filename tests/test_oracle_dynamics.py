"""Pins of the oracle's integrator and of its derivatives.

Integrator: harmonic dimer period (closed form), second-order convergence in
dt, time reversibility, energy conservation.  Derivatives: closed-form single
step, adjoint/tangent-linear dot-product identity, central finite differences
with a detector for pairs crossing the cutoff.
"""

import math

import numpy as np
import pytest

import oracle
from workloads import md_system

R0 = 2 ** (1 / 6)


def _dimer(sep, L=12.0):
    x = np.array([[5.0, 6.0, 6.0], [5.0 + sep, 6.0, 6.0]])
    return x, np.zeros((2, 3)), L


def _steps(x, v, L, n, dt, **kw):
    """n single steps; with one pair that never leaves the list this equals one run."""
    out = []
    for _ in range(n):
        r = oracle.run(x[:, 0], x[:, 1], x[:, 2], v[:, 0], v[:, 1], v[:, 2], L, 1, dt=dt, thermo=False, **kw)
        x, v = r["x"], r["v"]
        out.append(x[1, 0] - x[0, 0])
    return np.array(out), x, v


def test_dimer_small_amplitude_period():
    # V''(r0) = 36 * 2^(2/3) eps / sigma^2, reduced mass m/2
    omega = math.sqrt(36 * 2 ** (2 / 3) / 0.5)
    period = 2 * math.pi / omega
    assert period == pytest.approx(0.58772, abs=1e-5)
    dt = 0.001
    x, v, L = _dimer(R0 + 1e-3)
    sep, _, _ = _steps(x, v, L, 2000, dt)
    u = sep - R0
    idx = np.where(np.sign(u[:-1]) != np.sign(u[1:]))[0]
    t = (idx + 1 + u[idx] / (u[idx] - u[idx + 1])) * dt  # linearly interpolated zero crossings
    measured = 2 * (t[-1] - t[0]) / (len(t) - 1)
    assert measured == pytest.approx(period, rel=2e-4)


def test_velocity_verlet_second_order():
    x, v, L = _dimer(R0 + 0.08)
    T = 0.4
    ref, _, _ = _steps(x, v, L, int(round(T / 0.0000625)), 0.0000625)
    errs = []
    for dt in (0.004, 0.002, 0.001):
        s, _, _ = _steps(x, v, L, int(round(T / dt)), dt)
        errs.append(abs(s[-1] - ref[-1]))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.08)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.08)


def test_time_reversal():
    s = md_system(5, T=0.6, seed=21)
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 100, rebuild_every=1, thermo=False)
    x, v = r["x"], -r["v"]
    b = oracle.run(x[:, 0], x[:, 1], x[:, 2], v[:, 0], v[:, 1], v[:, 2], s.L, 100, rebuild_every=1, thermo=False)
    d = b["x"] - s.pos()
    d -= s.L * np.round(d / s.L)
    assert np.abs(d).max() < 1e-10
    assert np.abs(b["v"] + s.vel()).max() < 1e-9


def test_nve_shifted_energy_and_thermo():
    s = md_system(8, seed=1000)
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 100)
    th = r["thermo"]
    assert th.shape == (101, 5)
    assert th[0, 1] == pytest.approx(1.44, rel=1e-13)  # generator's temperature
    v = r["v"]
    assert th[-1, 0] == pytest.approx(0.5 * np.sum(v * v), rel=1e-13)
    vrc = 4.0 * (2.5 ** -12 - 2.5 ** -6)
    assert vrc == pytest.approx(-0.016316891136, abs=1e-12)

    def npairs(p):
        c, _, _ = oracle.build_list(p[:, 0], p[:, 1], p[:, 2], s.L, 2.5)
        return c.sum() // 2

    e0 = th[0, 4] - npairs(s.pos()) * vrc
    e1 = th[-1, 4] - npairs(r["x"]) * vrc  # step 100 is a rebuild step: list fresh
    assert abs(e1 - e0) / abs(e0) < 2e-4
    # momentum stays zero (Newton's third law through the integrator)
    assert np.abs(v.sum(0)).max() < 1e-10


# ---------------------------------------------------------------- derivatives

def test_single_step_dimer_closed_form():
    """One step, two atoms, loss = |x1_T - t|^2 on atom 1's x coordinate only:
    x1 = x0 + dt (v0 + h F(x0))  =>  dL/deps = 2 (x1-t) dt h F(x0)/eps."""
    dt, h = 0.005, 0.0025
    sep = 1.3
    x, v, L = _dimer(sep)
    eps, sig = 1.1, 0.97
    r = oracle.run(x[:, 0], x[:, 1], x[:, 2], v[:, 0], v[:, 1], v[:, 2], L, 1, eps=eps, sigma=sig, thermo=False)
    q = (sig / sep) ** 6
    f_closed = 24.0 * eps * q * (2 * q - 1.0) / sep ** 2 * (-sep)  # force on atom 0 along x (d_01 = -sep)
    f1 = -f_closed
    x1 = x[1, 0] + dt * h * f1
    assert r["x"][1, 0] == pytest.approx(x1, rel=1e-15)
    t = x1 - 0.01
    lam = np.zeros((2, 3))
    lam[1, 0] = 2 * (x1 - t)
    gx, gv, ge, gs = oracle.adjoint(x, v, L, 1, lam, np.zeros((2, 3)), eps=eps, sigma=sig)
    assert ge == pytest.approx(2 * (x1 - t) * dt * h * f1 / eps, rel=1e-12)
    # d f1 / d sigma with f1 = 24 eps (sig^6/r^6)(2 sig^6/r^6 - 1)/r: derivative of q in sigma is 6q/sig
    dq = 6 * q / sig
    df1 = 24.0 * eps * (dq * (2 * q - 1.0) + q * 2 * dq) / sep
    assert gs == pytest.approx(2 * (x1 - t) * dt * h * df1, rel=1e-12)
    # d x1 / d x1_0 = 1 + dt h dF1/dx1 with dF1/dx1 = -V''(r) (along the bond)
    vpp = eps * (4 * 156 * sig ** 12 / sep ** 14 - 4 * 42 * sig ** 6 / sep ** 8)
    assert gx[1, 0] == pytest.approx(2 * (x1 - t) * (1 - dt * h * vpp), rel=1e-12)
    assert gv[1, 0] == pytest.approx(2 * (x1 - t) * dt, rel=1e-12)


def _small_case(steps=40):
    s = md_system(4, T=1.0, seed=3000)
    return s.pos(), s.vel(), s.L, steps


def test_adjoint_tangent_dot_product():
    x0, v0, L, steps = _small_case(40)
    rng = np.random.default_rng(1)
    dx, dv = rng.standard_normal(x0.shape), rng.standard_normal(x0.shape)
    de, ds = 0.7, -0.4
    lx, lv = rng.standard_normal(x0.shape), rng.standard_normal(x0.shape)
    tx, tv = oracle.tangent(x0, v0, L, steps, dx, dv, de, ds)
    ax, av, ge, gs = oracle.adjoint(x0, v0, L, steps, lx, lv)
    lhs = np.sum(tx * lx) + np.sum(tv * lv)
    rhs = np.sum(dx * ax) + np.sum(dv * av) + de * ge + ds * gs
    assert lhs == pytest.approx(rhs, rel=1e-11)


def _loss_run(x0, v0, L, steps, tgt, **kw):
    r = oracle.run(x0[:, 0], x0[:, 1], x0[:, 2], v0[:, 0], v0[:, 1], v0[:, 2], L, steps, thermo=False,
                   hashes=True, **kw)
    d = r["x"] - tgt
    d -= L * np.round(d / L)
    return float(np.sum(d * d)), r["hashes"]


def test_adjoint_matches_flip_free_finite_differences():
    x0, v0, L, steps = _small_case(40)
    tr = oracle.run(x0[:, 0], x0[:, 1], x0[:, 2], v0[:, 0], v0[:, 1], v0[:, 2], L, steps, eps=1.05, sigma=0.98,
                    thermo=False)
    tgt = tr["x"]
    r = oracle.run(x0[:, 0], x0[:, 1], x0[:, 2], v0[:, 0], v0[:, 1], v0[:, 2], L, steps, thermo=False)
    d = r["x"] - tgt
    d -= L * np.round(d / L)
    gx, gv, ge, gs = oracle.adjoint(x0, v0, L, steps, 2 * d, np.zeros_like(d))
    h = 1e-6
    checked = 0
    for name, kp, km, g in (("eps", dict(eps=1 + h), dict(eps=1 - h), ge),
                            ("sigma", dict(sigma=1 + h), dict(sigma=1 - h), gs)):
        lp, hp = _loss_run(x0, v0, L, steps, tgt, **kp)
        lm, hm = _loss_run(x0, v0, L, steps, tgt, **km)
        if np.any(hp != hm):
            continue  # a pair crossed the cutoff between the two runs: FD is not the a.e. derivative
        assert (lp - lm) / (2 * h) == pytest.approx(g, rel=1e-6), name
        checked += 1
    u = np.random.default_rng(2).standard_normal(x0.shape)
    lp, hp = _loss_run(x0 + h * u, v0, L, steps, tgt)
    lm, hm = _loss_run(x0 - h * u, v0, L, steps, tgt)
    if np.all(hp == hm):
        assert (lp - lm) / (2 * h) == pytest.approx(np.sum(gx * u), rel=1e-6)
        checked += 1
    assert checked >= 2


def test_jvp_matches_force_differences():
    """J w against central differences of the force field at a fixed list."""
    s = md_system(4, T=1.0, seed=4)
    r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, 10, thermo=False)
    x = r["x"]
    c, nb, _ = oracle.build_list(x[:, 0], x[:, 1], x[:, 2], s.L, 2.8)
    w = np.random.default_rng(3).standard_normal(x.shape)
    jw = oracle.jvp(x[:, 0], x[:, 1], x[:, 2], s.L, c, nb, w)
    h = 1e-6
    xp, xm = x + h * w, x - h * w
    Fp, _, _, _ = oracle.forces(xp[:, 0], xp[:, 1], xp[:, 2], s.L, c, nb)
    Fm, _, _, _ = oracle.forces(xm[:, 0], xm[:, 1], xm[:, 2], s.L, c, nb)
    fd = (Fp - Fm) / (2 * h)
    assert np.abs(fd - jw).max() <= 1e-6 * np.abs(jw).max()
    # symmetry of J: <u, J w> = <J u, w>
    u = np.random.default_rng(4).standard_normal(x.shape)
    ju = oracle.jvp(x[:, 0], x[:, 1], x[:, 2], s.L, c, nb, u)
    assert np.sum(u * jw) == pytest.approx(np.sum(ju * w), rel=1e-12)


@pytest.mark.slow
def test_adjoint_workload_rounding_floor():
    """Bar of the GPU test on the 64 x 4,000-atom adjoint workload (200 steps,
    rebuild 20, loss against the trajectory at eps = 1.05, sigma = 0.98 from
    the same start): on replica 0 (seed 3000), moving every start coordinate
    by one ulp moves x_T by ~1e-13 and the gradients by ~1e-13 relative, so
    two correct implementations that round differently stay far inside 1e-9
    over this horizon (no pair crosses the cutoff between the two runs)."""
    s = md_system(10, 0.8442, 1.0, seed=3000)
    x0, v0, L, steps = s.pos(), s.vel(), s.L, 200
    tgt = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, L, steps, eps=1.05, sigma=0.98, thermo=False)["x"]

    def grads(x):
        r = oracle.run(x[:, 0], x[:, 1], x[:, 2], v0[:, 0], v0[:, 1], v0[:, 2], L, steps, thermo=False,
                       hashes=True)
        d = r["x"] - tgt
        d -= L * np.round(d / L)
        return r, oracle.adjoint(x, v0, L, steps, 2 * d, np.zeros_like(d))

    r0, (gx0, _, ge0, gs0) = grads(x0)
    r1, (gx1, _, ge1, gs1) = grads(np.nextafter(x0, np.inf))
    assert np.array_equal(r0["hashes"], r1["hashes"])  # same interacting pairs at every step
    dxT = r1["x"] - r0["x"]
    assert np.abs(dxT - L * np.round(dxT / L)).max() < 1e-11
    assert np.abs(gx1 - gx0).max() <= 1e-11 * np.abs(gx0).max()
    assert ge1 == pytest.approx(ge0, rel=1e-11)
    assert gs1 == pytest.approx(gs0, rel=1e-11)
