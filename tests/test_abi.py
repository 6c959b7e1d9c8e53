"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching a GPU."""
import ctypes

import pytest

import workloads
from paper_2005_09323_amd import native


def test_library_exports_every_declared_function():
    lib = native.lib()
    names = native.declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    for required in ("lbm_init", "lbm_step_batch", "lbm_drag", "gktl_select_clone", "ams_score_kill_branch"):
        assert required in names


def test_state_floats():
    lib = native.lib()
    wl = workloads.mixed_sizes(per_size=2)
    arr = native.desc_array(wl.members)
    assert lib.lbm_state_floats(arr, len(wl.members)) == sum(9 * m.nx * m.ny for m in wl.members)
    assert lib.lbm_state_floats(None, 0) == 0


def test_score_workspace_serves_every_smaller_batch():
    """The score network's gradient rows depend on how many images a backward
    workgroup takes (one below a batch of 4096, then up to 8), so their count
    drops where that number steps up (4095 images: 4095 rows, 4096: 2048);
    the workspace size must still never decrease with the batch, so that a
    workspace for a batch serves every smaller one."""
    lib = native.lib()
    lib.score_net_workspace_bytes.restype = ctypes.c_size_t
    prev = 0
    for b in list(range(1, 9000)) + list(range(9000, 70000, 7)) + [2 ** 20]:
        n = lib.score_net_workspace_bytes(b)
        assert n >= prev, b
        prev = n
    assert lib.score_net_workspace_bytes(0) == 0


def _create(members, pop_floats=10**9, cap=10, a=256, b=512, series=768, accum=1024):
    lib = native.lib()
    ctx = ctypes.c_void_p()
    arr = native.desc_array(members)
    rc = lib.lbm_create(ctypes.byref(ctx), arr, len(members), a, b, pop_floats, series, cap, accum, None)
    return rc, lib.lbm_last_error().decode()


@pytest.mark.parametrize("member,msg", [
    (workloads.Member(64, 16, 0.5, 0.0, None), "tau"),
    (workloads.Member(64, 16, 0.6, float("nan"), None), "force"),
    (workloads.Member(2, 16, 0.6, 0.0, None), "nx"),
    (workloads.Member(64, 16, 0.6, 0.0, (0, 4, 4)), "square"),
    (workloads.Member(64, 16, 0.6, 0.0, (10, 4, 12)), "square"),
    (workloads.Member(64, 16, 0.6, 0.0, (61, 4, 3)), "square"),
])
def test_create_rejects_bad_members(member, msg):
    rc, err = _create([member])
    assert rc == native.LBM_EINVAL and msg in err


def test_create_rejects_bad_buffers():
    m = workloads.Member(64, 16, 0.6, 0.0, (10, 4, 4))
    assert _create([m], pop_floats=9 * 64 * 16 - 1)[0] == native.LBM_EINVAL
    assert _create([m], a=0)[0] == native.LBM_EINVAL
    assert _create([m], a=256, b=256)[0] == native.LBM_EINVAL
    rc, err = _create([m], a=260)
    assert rc == native.LBM_EINVAL and "aligned" in err
    assert _create([m], cap=0)[0] == native.LBM_EINVAL
    assert _create([])[0] == native.LBM_EINVAL


def test_null_context_calls_fail_cleanly():
    lib = native.lib()
    assert lib.lbm_init(None, 1, 0.0) == native.LBM_EINVAL
    assert lib.lbm_step_batch(None, 1) == native.LBM_EINVAL
    assert lib.lbm_drag(None, 0, 1, None) == native.LBM_EINVAL
    assert lib.lbm_destroy(None) == native.LBM_OK
    assert lib.lbm_tile_count() >= 4


def test_size_limits_are_refused_on_the_host():
    """Every size limit is checked before any device work (the pointers below are never
    dereferenced): ensembles above 4096 members, AMS selections outside 1..2048 series,
    estimator sizes and ranges; empty estimator calls succeed without buffers."""
    lib = native.lib()
    m = workloads.Member(64, 4, 0.6, 0.0, None)
    rc, err = _create([m] * 4097)
    assert rc == native.LBM_EINVAL and "4096" in err
    p = 0x1000
    for n in (0, 2049):
        assert lib.ams_score_kill_branch(p, n, 10, 1, 1, 0, p, p, p, p, p, p, None) == native.LBM_EINVAL
    assert lib.ams_score_kill_branch(p, 8, 0, 1, 1, 0, p, p, p, p, p, p, None) == native.LBM_EINVAL
    assert lib.gktl_scgf(p, 0, 1.0, p, None) == native.LBM_EINVAL
    assert lib.gktl_scgf(p, 3, 0.0, p, None) == native.LBM_EINVAL
    assert lib.gktl_scgf(p, 3, float("inf"), p, None) == native.LBM_EINVAL
    assert lib.return_times(p, 4, 100.0, 100.0, p, None) == native.LBM_EINVAL
    assert lib.return_times(p, -1, 100.0, 10.0, p, None) == native.LBM_EINVAL
    assert lib.return_times(None, 0, 100.0, 10.0, None, None) == native.LBM_OK
    assert lib.ams_probability(p, 3, 0, p, p, 1, p, None) == native.LBM_EINVAL
    assert lib.ams_probability(None, 0, 8, None, None, 0, None, None) == native.LBM_OK


def test_member_size_limit_follows_32_bit_plane_offsets():
    """A member's 9 populations are indexed with 32-bit element offsets: 477,218,588 cells is
    the largest lattice accepted (the buffers below are then too small, a different error)."""
    big = workloads.Member(32768, 14564, 0.6, 0.0, None)   # 477,233,152 cells
    rc, err = _create([big])
    assert rc == native.LBM_EINVAL and "too large" in err
    ok = workloads.Member(32768, 14563, 0.6, 0.0, None)    # 477,200,384 cells
    rc, err = _create([ok])
    assert rc == native.LBM_EINVAL and "too large" not in err
