"""Reverse-mode gradients of the HIP path against the oracle's adjoint.

The oracle adjoint is itself pinned (closed form, dot-product identity,
flip-free finite differences; tests/test_oracle_dynamics.py).  Bar: 1e-9
relative (to the largest component for vectors) for dL/dx0, dL/dv0,
dL/deps and dL/dsigma.
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
    g.set_state(torch.from_numpy(boxes[0][0].pos()), torch.from_numpy(boxes[0][0].vel()), step=3)
    with pytest.raises(TmdError) as e:  # not at a rebuild step
        g.adjoint_forward(10)
    assert e.value.status == abi.TMD_ESTATE


def test_autograd_function_replica_workload_sample():
    """Two replicas of the adjoint workload (FCC 10^3 = 4,000 atoms, rho
    0.8442, T 1.0, 200 steps, rebuild 20): loss = sum |x_T - x_T^target|^2
    with the target run at eps = 1.05, sigma = 0.98 from the same start.

    Over 200 steps the dynamics amplify the ~1e-16 rounding differences
    between the GPU and oracle trajectories (summation order, fused
    multiply-add) by several orders of magnitude, in the forward run and
    again in the adjoint, so agreement is bounded at 3e-4 relative here; the
    1e-9 bar applies to the short horizons of test_adjoint_matches_oracle."""
    reps = [md_system(10, 0.8442, 1.0, seed=3000 + r) for r in (0, 63)]
    n1 = reps[0].n
    L = reps[0].L
    x0 = np.concatenate([s.pos() for s in reps])
    v0 = np.concatenate([s.vel() for s in reps])
    g = System.batch([n1, n1], [L, L], dict(max_neighbors=160))
    with torch.no_grad():
        tgt = lj_md(torch.tensor([1.05, 1.05]), torch.tensor([0.98, 0.98]), torch.from_numpy(x0), g,
                    torch.from_numpy(v0), 200)
    eps = torch.tensor([1.0, 1.0], dtype=torch.float64, requires_grad=True)
    sig = torch.tensor([1.0, 1.0], dtype=torch.float64, requires_grad=True)
    xin = torch.from_numpy(x0).clone().requires_grad_(True)
    xT = lj_md(eps, sig, xin, g, torch.from_numpy(v0), 200)
    d = xT - tgt
    d = d - L * torch.round(d / L)
    loss = (d * d).sum()
    loss.backward()
    for k, s in enumerate(reps):
        sl = slice(k * n1, (k + 1) * n1)
        tr = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, L, 200, eps=1.05, sigma=0.98, thermo=False)
        r = oracle.run(s.x, s.y, s.z, s.vx, s.vy, s.vz, L, 200, thermo=False)
        dd = r["x"] - tr["x"]
        dd -= L * np.round(dd / L)
        ox, _, oe, os_ = oracle.adjoint(s.pos(), s.vel(), L, 200, 2 * dd, np.zeros_like(dd))
        _close(xin.grad[sl].numpy(), ox, rel=3e-4)
        assert eps.grad[k].item() == pytest.approx(oe, rel=3e-4)
        assert sig.grad[k].item() == pytest.approx(os_, rel=3e-4)
