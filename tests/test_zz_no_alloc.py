"""tmd_compute_forces_static (the entry point that allocates nothing: its
intermediates live in the library's own device array) against the existing
entry points it stands for - create, bind a workspace, set_state, build the
list, compute_forces - on the same positions, through the C ABI.

Bar: forces, energy and virial bitwise equal (same kernels, same default
schedule), on two calls in a row, the second with fewer atoms (the shared
array keeps the first call's contents); both also within the force bar of
the oracle (1e-12 of each atom's scale sum_j |f_ij x_ij|).
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


from paper_2009_07400_amd import System, compute_forces_static  # noqa: E402
from paper_2009_07400_amd import _abi as abi  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _existing_path(pos, L, **kw):
    g = System(pos.shape[0], L, **kw)
    try:
        g.set_state(torch.from_numpy(pos), torch.zeros(pos.shape[0], 3, dtype=torch.float64))
        g.build_neighbors()
        F, ev = g.compute_forces()
        g.sync()
        return F.cpu().numpy(), ev.cpu().numpy()
    finally:
        g.close()


def _check(pos, L, label, **kw):
    _say(f"static forces: {label}, {pos.shape[0]} atoms, L {L:.4f}")
    F, ev, st = compute_forces_static(torch.from_numpy(pos), L, **kw)
    torch.cuda.synchronize()
    F, ev, st = F.cpu().numpy(), ev.cpu().numpy(), st.cpu().numpy()
    assert st[0] == abi.TMD_OK, (label, st)
    Fr, evr = _existing_path(pos, L, **kw)
    assert np.array_equal(F, Fr), (label, float(np.abs(F - Fr).max()))
    assert np.array_equal(ev, evr), (label, ev, evr)
    r = kw.get("cutoff", 2.5) + kw.get("skin", 0.3)
    c, nb, _ = oracle.build_list(pos[:, 0], pos[:, 1], pos[:, 2], L, r, maxnb=kw.get("max_neighbors", 128))
    Fo, sc, Uo, Wo = oracle.forces(pos[:, 0], pos[:, 1], pos[:, 2], L, c, nb)
    assert (np.linalg.norm(F - Fo, axis=1) <= 1e-12 * sc).all(), label
    assert ev[0] == pytest.approx(Uo, rel=1e-12) and ev[1] == pytest.approx(Wo, rel=1e-12), label


def test_static_forces_equal_existing_entry_points_on_two_calls():
    big = md_system(14, seed=41, jitter=0.25)   # 10,976 atoms, 6 cells per axis
    small = md_system(6, seed=42, jitter=0.25)  # 864 atoms, 3 cells per axis
    _check(big.pos(), big.L, "first call")
    _check(small.pos(), small.L, "second call, smaller")


def test_static_forces_reports_overflow_on_the_device():
    s = md_system(8, seed=43, jitter=0.1)
    F, ev, st = compute_forces_static(torch.from_numpy(s.pos()), s.L, max_neighbors=40)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert st[0] == abi.TMD_ENBR_OVERFLOW and st[1] > 40
    # the next call starts from a clear error word
    _check(s.pos(), s.L, "after an overflowing call")
