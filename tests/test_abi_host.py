"""Host-side checks of the C ABI: the library loads, exports every entry
point declared in include/tmd.h, and validates arguments synchronously.
Nothing here launches GPU work."""

import ctypes as C
import math
import os
import re

import pytest

from paper_2009_07400_amd import _abi as abi
from paper_2009_07400_amd.system import make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tmd_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = abi.load_library()
    names = _declared("tmd.h")
    assert "tmd_create" in names and "tmd_integrate" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    for st in range(0, -8, -1):
        s = abi.tmd_status_string(st)
        assert s and s != "unknown status"
    assert abi.tmd_status_string(-99) == "unknown status"


def _create(n=2048, L=13.43677, **kw):
    return abi.tmd_create(make_params(**kw), n, L)


def test_create_and_info():
    h = _create()
    try:
        info = abi.tmd_get_info(h)
        assert info["n_atoms"] == 2048
        assert info["cells_per_axis"] == math.floor(13.43677 / 2.8) == 4
        assert info["n_cells"] == 64
        assert info["n_padded"] % 256 == 0 and info["n_padded"] >= 2048
        assert info["workspace_bytes"] == abi.tmd_workspace_size(h)
        # the list alone needs max_neighbors int32 per padded atom
        assert info["workspace_bytes"] > info["n_padded"] * 128 * 4
        assert info["graph_captures"] == 0 and info["graph_launches"] == 0
    finally:
        abi.tmd_destroy(h)


def test_graph_mode_switch_needs_no_gpu():
    # enabling captures nothing until tmd_integrate; disabling drops nothing
    h = _create()
    try:
        abi.tmd_set_graphs(h, True)
        abi.tmd_set_graphs(h, False)
        abi.tmd_set_graphs(h, True)
        info = abi.tmd_get_info(h)
        assert info["graph_captures"] == 0 and info["graph_launches"] == 0
    finally:
        abi.tmd_destroy(h)


@pytest.mark.parametrize("kw,n,L,status", [
    ({}, 0, 13.4, abi.TMD_EINVAL),
    ({}, -5, 13.4, abi.TMD_EINVAL),
    ({"epsilon": -1.0}, 10, 13.4, abi.TMD_EINVAL),
    ({"sigma": 0.0}, 10, 13.4, abi.TMD_EINVAL),
    ({"dt": float("nan")}, 10, 13.4, abi.TMD_EINVAL),
    ({"mass": float("inf")}, 10, 13.4, abi.TMD_EINVAL),
    ({"skin": -0.1}, 10, 13.4, abi.TMD_EINVAL),
    ({"rebuild_every": 0}, 10, 13.4, abi.TMD_EINVAL),
    ({"max_neighbors": 0}, 10, 13.4, abi.TMD_EINVAL),
    ({"max_neighbors": 5000}, 10, 13.4, abi.TMD_EINVAL),
    ({}, 10, float("nan"), abi.TMD_EINVAL),
    ({}, 10, 5.6, abi.TMD_EBOX),      # cutoff + skin = 2.8 = L/2
    ({}, 10, 5.0, abi.TMD_EBOX),
    ({}, 700_000_001, 2000.0, abi.TMD_EINVAL),  # 3 n_padded doubles addressed with 32-bit offsets
    # Spring-Dashpot (Eq. 3): non-negative finite K and gamma, list radius
    # base cutoff >= the diameter sigma
    (dict(model="spring_dashpot", stiffness=-1.0, cutoff=1.0), 10, 13.4, abi.TMD_EINVAL),
    (dict(model="spring_dashpot", stiffness=100.0, damping=float("nan"), cutoff=1.0), 10, 13.4, abi.TMD_EINVAL),
    (dict(model="spring_dashpot", stiffness=100.0, sigma=1.0, cutoff=0.9), 10, 13.4, abi.TMD_EINVAL),
])
def test_create_rejects(kw, n, L, status):
    with pytest.raises(abi.TmdError) as e:
        _create(n=n, L=L, **kw)
    assert e.value.status == status


def test_smallest_valid_box_and_cell_counts():
    h = _create(n=10, L=5.6000001)
    assert abi.tmd_get_info(h)["cells_per_axis"] == 2
    abi.tmd_destroy(h)
    h = _create(n=3538944, L=161.24123)
    info = abi.tmd_get_info(h)
    assert info["cells_per_axis"] == 57 and info["n_cells"] == 57 ** 3
    abi.tmd_destroy(h)


def test_call_order_and_workspace_checks():
    h = _create()
    try:
        # no workspace bound: every device call is refused before touching the GPU
        for fn in (lambda: abi.tmd_build_neighbors(h, 0),
                   lambda: abi.tmd_integrate(h, 10, 0, None, 0),
                   lambda: abi.tmd_compute_forces(h, None, None, 0),
                   lambda: abi.tmd_sync(h, 0)):
            with pytest.raises(abi.TmdError) as e:
                fn()
            assert e.value.status == abi.TMD_ESTATE
        need = abi.tmd_workspace_size(h)
        with pytest.raises(abi.TmdError) as e:  # misaligned
            abi.tmd_bind_workspace(h, 0x10000 + 8, need)
        assert e.value.status == abi.TMD_EWORKSPACE
        with pytest.raises(abi.TmdError) as e:  # too small
            abi.tmd_bind_workspace(h, 0x10000, need - 1)
        assert e.value.status == abi.TMD_EWORKSPACE
        assert "256-byte" in abi.tmd_last_error(h)
    finally:
        abi.tmd_destroy(h)


def test_batch_create_and_validation():
    ps = [make_params(), make_params(epsilon=1.05, sigma=0.98), make_params()]
    h = abi.tmd_create_batch(ps, [256, 500, 6912], [6.72, 8.4, 20.9])
    try:
        info = abi.tmd_get_info(h)
        assert info["n_boxes"] == 3 and info["n_atoms"] == 256 + 500 + 6912
        # 2 and 3 cells per axis (<= E + 2): one block of the whole box; 7 -> 4^3 blocks
        assert info["n_blocks"] == 1 + 1 + 64
        assert info["n_cells"] == 8 + 27 + 343
        assert info["block_threads"] % 64 == 0 and 64 <= info["block_threads"] <= 1024
        assert info["lds_atoms"] % 64 == 0 and 64 <= info["lds_atoms"] <= 4096
        assert info["block_edge"] == 2  # too few 3x3x3 blocks to fill the GPU
        abi.tmd_set_schedule(h, 128, 512)
        info = abi.tmd_get_info(h)
        assert (info["block_threads"], info["lds_atoms"]) == (128, 512)
        abi.tmd_set_schedule(h, 0, 0, 3)  # 3 cells per edge: 1 + 1 + 3^3 blocks
        info = abi.tmd_get_info(h)
        assert (info["block_edge"], info["n_blocks"], info["block_parts"]) == (3, 1 + 1 + 27, 1)
        abi.tmd_set_schedule(h, 0, 0, 0, 4)
        assert abi.tmd_get_info(h)["block_parts"] == 4
        assert abi.tmd_get_info(h)["lanes_per_atom"] == 1
        b0 = abi.tmd_get_info(h)["build_threads"]
        assert b0 % 64 == 0 and 64 <= b0 <= 1024
        t0 = abi.tmd_get_info(h)["block_threads"]
        abi.tmd_set_schedule(h, 0, 0, 0, 0, 2)
        info = abi.tmd_get_info(h)
        # a second lane per atom widens the force workgroups, not the build's
        assert info["lanes_per_atom"] == 2 and info["build_threads"] == b0 and info["block_threads"] >= t0
        abi.tmd_set_schedule(h, 0, 0, 0, 0, 0, 320)
        assert abi.tmd_get_info(h)["build_threads"] == 320
        assert abi.tmd_get_info(h)["build_lanes"] == 1
        abi.tmd_set_schedule(h, 0, 0, 0, 0, 0, 0, 2)
        info = abi.tmd_get_info(h)
        # two lanes per atom in the build reset its threads to their (wider) default
        assert info["build_lanes"] == 2 and info["build_threads"] >= b0
        for bad in ((100, 0, 0, 0, 0, 0, 0), (1088, 0, 0, 0, 0, 0, 0), (0, 100, 0, 0, 0, 0, 0),
                    (0, 4160, 0, 0, 0, 0, 0), (-64, 0, 0, 0, 0, 0, 0), (0, 0, 4, 0, 0, 0, 0), (0, 0, 1, 0, 0, 0, 0),
                    (0, 0, 0, 3, 0, 0, 0), (0, 0, 0, 8, 0, 0, 0), (0, 0, 0, -1, 0, 0, 0), (0, 0, 0, 0, 3, 0, 0),
                    (0, 0, 0, 0, 8, 0, 0), (0, 0, 0, 0, -1, 0, 0), (0, 0, 0, 0, 0, 100, 0), (0, 0, 0, 0, 0, 1088, 0),
                    (0, 0, 0, 0, 0, -64, 0), (0, 0, 0, 0, 0, 0, 3), (0, 0, 0, 0, 0, 0, 4), (0, 0, 0, 0, 0, 0, -1)):
            with pytest.raises(abi.TmdError):
                abi.tmd_set_schedule(h, *bad)
    finally:
        abi.tmd_destroy(h)
    with pytest.raises(abi.TmdError) as e:  # rebuild interval must be shared
        abi.tmd_create_batch([make_params(), make_params(rebuild_every=10)], [100, 100], [10.0, 10.0])
    assert e.value.status == abi.TMD_EINVAL
    with pytest.raises(abi.TmdError) as e:  # one box too small for the cutoff
        abi.tmd_create_batch([make_params(), make_params()], [100, 100], [10.0, 5.0])
    assert e.value.status == abi.TMD_EBOX
    with pytest.raises(ValueError):
        abi.tmd_create_batch([make_params()], [100, 100], [10.0, 10.0])


def test_null_arguments():
    lib = abi.load_library()
    assert lib.tmd_create(None, 10, 13.4, None) == abi.TMD_EINVAL
    assert lib.tmd_workspace_size(None, None) == abi.TMD_EINVAL
    assert lib.tmd_get_info(None, None) == abi.TMD_EINVAL
    assert lib.tmd_sync(None, None) == abi.TMD_EINVAL
    lib.tmd_destroy(None)
    assert abi.tmd_last_error(None) == "NULL system"
    out = C.c_void_p()
    p = make_params()
    assert lib.tmd_create(C.byref(p), 10, 13.4, C.byref(out)) == abi.TMD_OK
    assert lib.tmd_set_timing(out, 1) == abi.TMD_OK
    assert lib.tmd_set_graphs(None, 1) == abi.TMD_EINVAL
    lib.tmd_destroy(out)


def test_static_forces_validates_before_the_gpu():
    """tmd_compute_forces_static checks its arguments and the size of its
    intermediates against the library's fixed device array before it touches
    a GPU (these calls return without one)."""
    lib = abi.load_library()
    p = make_params()
    fake = (C.c_void_p * 3)(16, 32, 48)  # never dereferenced: every call below fails its checks first
    args = (C.cast(fake, C.c_void_p), None, None, None, None)
    assert lib.tmd_compute_forces_static(None, 2048, 13.43677, *args) == abi.TMD_EINVAL
    assert lib.tmd_compute_forces_static(C.byref(p), 2048, 13.43677, None, None, None, None, None) == abi.TMD_EINVAL
    assert lib.tmd_compute_forces_static(C.byref(p), 0, 13.43677, *args) == abi.TMD_EINVAL
    assert lib.tmd_compute_forces_static(C.byref(p), 2048, 5.0, *args) == abi.TMD_EBOX
    # 32^3 unit cells (131,072 atoms) need more than the 64 MiB array
    h = abi.tmd_create(p, 131072, 53.74708)
    try:
        assert abi.tmd_workspace_size(h) > 64 * 1024 * 1024
    finally:
        abi.tmd_destroy(h)
    assert lib.tmd_compute_forces_static(C.byref(p), 131072, 53.74708, *args) == abi.TMD_EWORKSPACE


def test_unknown_model_and_mixed_batches_are_rejected():
    p = make_params()
    p.model = 7
    with pytest.raises(abi.TmdError) as e:
        abi.tmd_create(p, 10, 13.4)
    assert e.value.status == abi.TMD_EINVAL
    sd = make_params(model="spring_dashpot", stiffness=100.0, damping=1.0, cutoff=1.0)
    with pytest.raises(abi.TmdError) as e:
        abi.tmd_create_batch([make_params(), sd], [100, 100], [13.4, 13.4])
    assert e.value.status == abi.TMD_EINVAL
    h = abi.tmd_create(sd, 100, 13.4)
    abi.tmd_destroy(h)
    with pytest.raises(ValueError):
        make_params(model="dem")


def test_half_list_switch_validates_on_the_host():
    h = _create()
    try:
        assert abi.tmd_get_info(h)["half_list"] == 0
        for bad in (2, -1):
            with pytest.raises(abi.TmdError) as e:
                abi.tmd_set_half_list(h, bad)
            assert e.value.status == abi.TMD_EINVAL
        abi.tmd_set_half_list(h, 1)
        assert abi.tmd_get_info(h)["half_list"] == 1
        # one workgroup per block and one lane per atom while it is on
        for kw in (dict(block_parts=2), dict(lanes_per_atom=4)):
            with pytest.raises(abi.TmdError):
                abi.tmd_set_schedule(h, 0, 0, **kw)
        abi.tmd_set_half_list(h, 0)
        abi.tmd_set_schedule(h, 0, 0, block_parts=2)
        with pytest.raises(abi.TmdError):
            abi.tmd_set_half_list(h, 1)
    finally:
        abi.tmd_destroy(h)
    sd = abi.tmd_create(make_params(model="spring_dashpot", stiffness=100.0, damping=1.0, cutoff=1.0), 100, 13.4)
    try:
        with pytest.raises(abi.TmdError):
            abi.tmd_set_half_list(sd, 1)
    finally:
        abi.tmd_destroy(sd)


def test_layout_switch_validates_on_the_host():
    h = _create()
    try:
        assert abi.tmd_get_info(h)["layout"] == abi.TMD_LAYOUT_SOA
        for bad in (3, -1):
            with pytest.raises(abi.TmdError) as e:
                abi.tmd_set_layout(h, bad, 0)
            assert e.value.status == abi.TMD_EINVAL
        for lay in (abi.TMD_LAYOUT_AOS, abi.TMD_LAYOUT_AOSOA, abi.TMD_LAYOUT_SOA):
            abi.tmd_set_layout(h, lay, 0)  # no state yet: nothing to convert, no GPU call
            assert abi.tmd_get_info(h)["layout"] == lay
    finally:
        abi.tmd_destroy(h)
    sd = abi.tmd_create(make_params(model="spring_dashpot", stiffness=100.0, damping=1.0, cutoff=1.0), 100, 13.4)
    try:
        with pytest.raises(abi.TmdError):
            abi.tmd_set_layout(sd, abi.TMD_LAYOUT_AOS, 0)
        abi.tmd_set_layout(sd, abi.TMD_LAYOUT_SOA, 0)
    finally:
        abi.tmd_destroy(sd)
