"""Reverse-mode gradients of the HIP path against the oracle's adjoint.

The oracle adjoint is itself pinned (closed form, dot-product identity,
flip-free finite differences; tests/test_oracle_dynamics.py).  Bar: 1e-9
relative (to the largest component for vectors) for dL/dx0, dL/dv0,
dL/deps and dL/dsigma.
"""

import numpy as np
import pytest

import oracle
from images_helper import wrong_staged_images
from workloads import md_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_2009_07400_amd import System, TmdError, lj_md  # noqa: E402
from paper_2009_07400_amd import _abi as abi  # noqa: E402

REL = 1e-9


def _close(a, b, rel=REL):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    assert np.abs(a - b).max() <= rel * scale, (np.abs(a - b).max(), scale)


def _boxes():
    # (ncell, rho, T, seed, eps, sigma): 2, 3 and 3 cells per axis
    spec = [(4, 0.8442, 1.0, 31, 1.05, 0.98), (5, 0.80, 1.2, 32, 1.0, 1.0), (6, 0.75, 0.9, 33, 0.95, 1.03)]
    return [(md_system(n, rho, T, seed=seed), eps, sig) for n, rho, T, seed, eps, sig in spec]


def _batch(boxes):
    g = System.batch([s.n for s, _, _ in boxes], [s.L for s, _, _ in boxes],
                     [dict(epsilon=e, sigma=sg, max_neighbors=160) for _, e, sg in boxes])
    g.set_state(torch.from_numpy(np.concatenate([s.pos() for s, _, _ in boxes])),
                torch.from_numpy(np.concatenate([s.vel() for s, _, _ in boxes])))
    return g


@pytest.mark.parametrize("steps", [1, 20, 45])
def test_adjoint_matches_oracle(steps):
    boxes = _boxes()
    g = _batch(boxes)
    n = g.n
    rng = np.random.default_rng(steps)
    lx = rng.standard_normal((n, 3))
    lv = rng.standard_normal((n, 3))
    g.adjoint_forward(steps)
    gx, gv, ge, gs = g.adjoint_backward(torch.from_numpy(lx), torch.from_numpy(lv))
    p, v, step = g.get_state()
    g.sync()
    assert step == steps
    gx, gv, ge, gs = gx.cpu().numpy(), gv.cpu().numpy(), ge.cpu().numpy(), gs.cpu().numpy()
    off = 0
    for k, (s, eps, sig) in enumerate(boxes):
        sl = slice(off, off + s.n)
        r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, steps, eps=eps, sigma=sig, thermo=False)
        d = p.cpu().numpy()[sl] - r["x"]
        assert np.abs(d - s.L * np.round(d / s.L)).max() < 1e-9  # left in the final state
        ox, ov, oe, os_ = oracle.adjoint(s.pos(), s.vel(), s.L, steps, lx[sl], lv[sl], eps=eps, sigma=sig)
        _close(gx[sl], ox)
        _close(gv[sl], ov)
        assert ge[k] == pytest.approx(oe, rel=REL)
        assert gs[k] == pytest.approx(os_, rel=REL)
        off += s.n


def test_adjoint_image_path():
    """A box of 7 cells per axis stages neighborhoods moved to periodic
    images near each block (the step and the reverse kernels alike): the
    gradients match the oracle's adjoint, and equal bit for bit those of a
    run whose neighborhoods do not fit in LDS (partner images taken per pair
    from global memory)."""
    s = md_system(12, 0.8442, 1.0, seed=34)
    rng = np.random.default_rng(7)
    lx = rng.standard_normal((s.n, 3))
    lv = rng.standard_normal((s.n, 3))
    out = []
    for lds in (0, 64):
        g = System(s.n, s.L, epsilon=1.02, sigma=0.99)
        assert g.info()["cells_per_axis"] == 7
        g.set_schedule(lds_atoms=lds)
        g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
        g.adjoint_forward(20)
        r = g.adjoint_backward(torch.from_numpy(lx), torch.from_numpy(lv))
        g.sync()
        out.append([t.cpu() for t in r])
        g.close()
    for a, b in zip(*out):
        assert torch.equal(a, b)
    ox, ov, oe, os_ = oracle.adjoint(s.pos(), s.vel(), s.L, 20, lx, lv, eps=1.02, sigma=0.99)
    gx, gv, ge, gs = (t.numpy() for t in out[0])
    _close(gx, ox)
    _close(gv, ov)
    assert float(ge.reshape(-1)[0]) == pytest.approx(oe, rel=REL)
    assert float(gs.reshape(-1)[0]) == pytest.approx(os_, rel=REL)


def test_adjoint_forward_ends_in_the_integrate_state_bitwise():
    """The recorded forward run takes the steps of integrate() (each later
    interval continues from the state the previous one left, which is the
    state a reload of its checkpoint gives): positions and velocities equal
    integrate()'s bit for bit, over whole and partial rebuild intervals, and
    so do the list it leaves and the steps that follow."""
    for steps in (45, 60):
        s = md_system(10, 0.8442, 1.0, seed=3000)
        a = System(s.n, s.L)
        a.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
        a.integrate(steps)
        pa, va, _ = a.get_state()
        b = System(s.n, s.L)
        b.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
        b.adjoint_forward(steps)
        pb, vb, step = b.get_state()
        a.sync()
        b.sync()
        assert step == steps
        assert torch.equal(pa, pb) and torch.equal(va, vb), steps
        # the list the forward leaves (built into the workspace, then the
        # system's own) is integrate()'s, and later steps run on it alike
        ca, ia = a.get_neighbors()
        cb, ib = b.get_neighbors()
        assert torch.equal(ca, cb) and torch.equal(ia, ib), steps
        a.integrate(12)
        b.integrate(12)
        pa, va, _ = a.get_state()
        pb, vb, _ = b.get_state()
        a.sync()
        b.sync()
        assert torch.equal(pa, pb) and torch.equal(va, vb), steps
        a.close()
        b.close()


def test_adjoint_checked_images_after_large_drift():
    """A box of E + 3 cells per axis (staged images, each difference tested
    against L/2) with atoms flying up to three sigma on the list of the
    first step (a negligible epsilon: ballistic; rebuild every 1000 steps),
    so the last steps see pairs whose staged image is wrong: the gradients,
    dL/deps above all (dF/deps = F/eps does not vanish with eps), match the
    oracle's adjoint, which takes every pair's minimum image."""
    s = md_system(9, seed=40)
    rng = np.random.default_rng(40)
    u = rng.standard_normal((s.n, 3))
    vel = u / np.linalg.norm(u, axis=1, keepdims=True) * rng.uniform(0.0, 60.0, (s.n, 1))
    x0 = s.pos()
    steps, eps = 10, 1e-30
    g = System(s.n, s.L, epsilon=eps, rebuild_every=1000)
    assert g.info()["cells_per_axis"] == 5
    g.set_schedule(block_edge=2)
    g.set_state(torch.from_numpy(x0), torch.from_numpy(vel))
    lx = rng.standard_normal((s.n, 3))
    lv = rng.standard_normal((s.n, 3))
    g.adjoint_forward(steps)
    gx, gv, ge, gs = g.adjoint_backward(torch.from_numpy(lx), torch.from_numpy(lv))
    p, _, _ = g.get_state()
    g.sync()
    c0, n0, _ = oracle.build_list(x0[:, 0], x0[:, 1], x0[:, 2], s.L, 2.8, maxnb=160)
    assert wrong_staged_images(x0, p.cpu().numpy(), s.L, c0, n0, 2) > 0
    ox, ov, oe, os_ = oracle.adjoint(x0, vel, s.L, steps, lx, lv, eps=eps, sigma=1.0, rebuild_every=1000)
    _close(gx.cpu().numpy(), ox)
    _close(gv.cpu().numpy(), ov)
    assert float(ge.reshape(-1)[0]) == pytest.approx(oe, rel=REL)
    assert float(gs.reshape(-1)[0]) == pytest.approx(os_, rel=REL)
    g.close()


def test_adjoint_call_order():
    boxes = _boxes()[:1]
    g = _batch(boxes)
    z = torch.zeros(g.n, 3, dtype=torch.float64)
    with pytest.raises((TmdError, AttributeError)):
        g.adjoint_backward(z)
    g.adjoint_forward(10)
    g.integrate(1)  # changes the state: the recorded run no longer matches
    with pytest.raises(TmdError) as e:
        g.adjoint_backward(z)
    assert e.value.status == abi.TMD_ESTATE
    g.set_state(torch.from_numpy(boxes[0][0].pos()), torch.from_numpy(boxes[0][0].vel()))
    g.adjoint_forward(10)
    g.set_layout("aos")  # the recorded run reads the state as SoA positions
    with pytest.raises(TmdError) as e:
        g.adjoint_backward(z)
    assert e.value.status == abi.TMD_ESTATE
    g.set_layout("soa")
    g.set_state(torch.from_numpy(boxes[0][0].pos()), torch.from_numpy(boxes[0][0].vel()), step=3)
    with pytest.raises(TmdError) as e:  # not at a rebuild step
        g.adjoint_forward(10)
    assert e.value.status == abi.TMD_ESTATE


REPLICAS = 64
STEPS = 200


@pytest.fixture(scope="module")
def replica_grads():
    """The 64 x 4,000-atom adjoint workload on the GPU, as the benchmark runs
    it: FCC 10^3 replicas (rho 0.8442, T 1.0, seeds 3000 + r), 200 steps,
    rebuild every 20, schedule autotuned one rebuild interval into the run;
    loss sum |x_T - x_T^target|^2 with the target run at eps = 1.05,
    sigma = 0.98 from the same start.  Returns the gradients through
    LJMDFunction and the start states."""
    reps = [md_system(10, 0.8442, 1.0, seed=3000 + r) for r in range(REPLICAS)]
    n1, L = reps[0].n, reps[0].L
    x0 = np.concatenate([s.pos() for s in reps])
    v0 = np.concatenate([s.vel() for s in reps])
    g = System.batch([n1] * REPLICAS, [L] * REPLICAS, dict(max_neighbors=128))
    g.set_state(torch.from_numpy(x0), torch.from_numpy(v0))
    g.integrate(20)
    g.autotune(repeats=3, for_adjoint=True)
    ones = torch.ones(REPLICAS, dtype=torch.float64)
    with torch.no_grad():
        tgt = lj_md(1.05 * ones, 0.98 * ones, torch.from_numpy(x0), g, torch.from_numpy(v0), STEPS)
    eps = ones.clone().requires_grad_(True)
    sig = ones.clone().requires_grad_(True)
    xin = torch.from_numpy(x0).clone().requires_grad_(True)
    xT = lj_md(eps, sig, xin, g, torch.from_numpy(v0), STEPS)
    d = xT - tgt
    d = d - L * torch.round(d / L)
    (d * d).sum().backward()
    sched = g.info()
    g.close()
    print(f"adjoint workload: GPU gradients of {REPLICAS} replicas at schedule E{sched['block_edge']} "
          f"L{sched['lanes_per_atom']} T{sched['block_threads']}", flush=True)
    return reps, xin.grad.numpy(), eps.grad.numpy(), sig.grad.numpy()


@pytest.mark.parametrize("group", range(4))
def test_adjoint_workload_all_replicas(replica_grads, group):
    """Every replica of the adjoint workload against the oracle's adjoint at
    1e-9 relative: dL/dx0 (to its largest component), dL/deps, dL/dsigma.
    Rounding differences between the two paths stay near 1e-13 over these
    200 steps (a one-ulp change of every start coordinate moves the oracle's
    gradients by 1.2e-13), so 1e-9 leaves four orders of magnitude."""
    reps, gx, ge, gs = replica_grads
    n1, L = reps[0].n, reps[0].L
    worst = 0.0
    for k in range(16 * group, 16 * group + 16):
        s = reps[k]
        sl = slice(k * n1, (k + 1) * n1)
        tr = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, L, STEPS, eps=1.05, sigma=0.98, thermo=False)
        r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, L, STEPS, thermo=False)
        dd = r["x"] - tr["x"]
        dd -= L * np.round(dd / L)
        ox, _, oe, os_ = oracle.adjoint(s.pos(), s.vel(), L, STEPS, 2 * dd, np.zeros_like(dd))
        _close(gx[sl], ox)
        assert ge[k] == pytest.approx(oe, rel=REL), k
        assert gs[k] == pytest.approx(os_, rel=REL), k
        worst = max(worst, np.abs(gx[sl] - ox).max() / np.abs(ox).max(), abs(ge[k] - oe) / abs(oe),
                    abs(gs[k] - os_) / abs(os_))
    print(f"replicas {16 * group}..{16 * group + 15}: worst relative gradient difference {worst:.2e}", flush=True)


def _gpu_loss(s, steps, tgt, x0=None, eps=1.0, sigma=1.0):
    g = System(s.n, s.L, epsilon=eps, sigma=sigma, max_neighbors=128)
    g.set_state(torch.from_numpy(s.pos() if x0 is None else x0), torch.from_numpy(s.vel()))
    g.integrate(steps)
    p, _, _ = g.get_state()
    g.sync()
    g.close()
    d = p.cpu().numpy() - tgt
    d -= s.L * np.round(d / s.L)
    return float(np.sum(d * d))


def _flips(s, steps, x0=None, **kw):
    x = s.pos() if x0 is None else x0
    return oracle.run(x[:, 0], x[:, 1], x[:, 2], s.vx, s.vy, s.vz, s.L, steps, thermo=False, hashes=True,
                      **kw)["hashes"]


def _gpu_grads(s, steps, tgt):
    g = System(s.n, s.L, max_neighbors=128)
    g.set_state(torch.from_numpy(s.pos()), torch.from_numpy(s.vel()))
    g.adjoint_forward(steps)
    p, _, _ = g.get_state()
    d = p.cpu().numpy() - tgt
    d -= s.L * np.round(d / s.L)
    gx, _, ge, gs = g.adjoint_backward(torch.from_numpy(2 * d))
    g.sync()
    g.close()
    return gx.cpu().numpy(), float(ge[0].item()), float(gs[0].item())


def test_gpu_gradients_against_central_differences():
    """GPU gradients against central finite differences of the GPU's own
    trajectories at h = 1e-6, wherever no pair crosses the cutoff between
    the +h and -h runs (the oracle's per-step hash of interacting pairs; a
    crossing makes the difference quotient measure the force's jump, not
    the derivative).  dL/dx0: four single coordinates of replica 0 of the
    adjoint workload over its full 200 steps; dL/deps: the same replica
    over 40 steps; dL/dsigma: an 864-atom box (FCC 6^3, seed 3000) over 40
    steps, the longest horizons on which these perturbations cross no
    cutoff.  Bars: 5e-5 relative (200 steps) and 1e-7 (40 steps), above
    the difference quotient's own truncation and rounding error."""
    h = 1e-6
    rep = md_system(10, 0.8442, 1.0, seed=3000)
    small = md_system(6, 0.8442, 1.0, seed=3000)
    checked = []
    for s, steps, what in ((rep, 200, "x0"), (rep, 40, "eps"), (small, 40, "sigma")):
        tgt = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.L, steps, eps=1.05, sigma=0.98, thermo=False)["x"]
        gx, ge, gs = _gpu_grads(s, steps, tgt)
        if what == "x0":
            for i, a in ((0, 0), (1234, 1), (2777, 2), (3999, 0)):
                e = np.zeros((s.n, 3))
                e[i, a] = h
                if np.any(_flips(s, steps, x0=s.pos() + e) != _flips(s, steps, x0=s.pos() - e)):
                    continue
                fd = (_gpu_loss(s, steps, tgt, x0=s.pos() + e) - _gpu_loss(s, steps, tgt, x0=s.pos() - e)) / (2 * h)
                assert gx[i, a] == pytest.approx(fd, rel=5e-5), (i, a)
                checked.append((what, i, a, abs(gx[i, a] - fd) / abs(fd)))
        else:
            kp, km = ({"eps": 1 + h}, {"eps": 1 - h}) if what == "eps" else ({"sigma": 1 + h}, {"sigma": 1 - h})
            if np.any(_flips(s, steps, **kp) != _flips(s, steps, **km)):
                continue
            fd = (_gpu_loss(s, steps, tgt, **kp) - _gpu_loss(s, steps, tgt, **km)) / (2 * h)
            g = ge if what == "eps" else gs
            assert g == pytest.approx(fd, rel=1e-7), what
            checked.append((what, abs(g - fd) / abs(fd)))
    print("central differences checked:", checked, flush=True)
    assert sum(1 for c in checked if c[0] == "x0") >= 3
    assert {"eps", "sigma"} <= {c[0] for c in checked}
