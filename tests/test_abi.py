"""C interface contract, checked without a GPU: the library loads, exports
every function the header declares, validates parameters on the host and
reports errors by status code."""
import ctypes
import os

import pytest

from paper_2206_01683_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    return lbm.lib()


def test_every_declared_function_is_exported(L):
    names = lbm.header_functions()
    assert "lbm_init" in names and "lbm_ib_step" in names and "lbm_body_forces" in names
    for n in names:
        assert hasattr(L, n), n


def test_population_and_workspace_sizes(L):
    p = lbm.make_params(64, 32, 32, 0.6, lbm.BC_VELOCITY, lbm.BC_OUTFLOW, max_markers=500)
    pb = L.lbm_population_bytes(ctypes.byref(p))
    assert pb >= 27 * 64 * 32 * 32 * 4 and pb % 256 == 0
    p16 = lbm.make_params(64, 32, 32, 0.6, storage="f16")
    assert L.lbm_population_bytes(ctypes.byref(p16)) * 2 == L.lbm_population_bytes(
        ctypes.byref(lbm.make_params(64, 32, 32, 0.6)))
    assert L.lbm_workspace_bytes(ctypes.byref(p)) > 0


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=0.3), dict(nx=3), dict(nz=0),
    dict(bc_lo=lbm.BC_PERIODIC, bc_hi=lbm.BC_OUTFLOW), dict(storage=7), dict(max_bones=0),
    dict(mdf_iters=0), dict(mdf_iters=17), dict(block=(96, 1)), dict(block=(512, 2)), dict(ib_alpha=0.0),
    dict(ib_scheme=2), dict(ib_scheme=-1), dict(collision=2), dict(collision=1, trt_lambda=0.0),
    dict(collision=1, trt_lambda=float("nan")), dict(wall_mode=2),
])
def test_invalid_parameters_are_rejected(L, bad):
    kw = dict(nx=16, ny=16, nz=16, tau=0.6, bc_lo=lbm.BC_VELOCITY, bc_hi=lbm.BC_OUTFLOW)
    kw.update(bad)
    p = lbm.make_params(**kw)
    assert L.lbm_population_bytes(ctypes.byref(p)) == 0
    assert L.lbm_workspace_bytes(ctypes.byref(p)) == 0
    ctx = ctypes.c_void_p()
    dummy = ctypes.c_void_p(256)
    rc = L.lbm_init(ctypes.byref(ctx), ctypes.byref(p), dummy, ctypes.c_void_p(512), ctypes.c_void_p(1024),
                    None, None, None)
    assert rc == -1 and not ctx.value


def test_init_rejects_null_or_aliased_buffers(L):
    p = lbm.make_params(16, 16, 16, 0.6)
    ctx = ctypes.c_void_p()
    assert L.lbm_init(ctypes.byref(ctx), ctypes.byref(p), None, ctypes.c_void_p(512), ctypes.c_void_p(1024),
                      None, None, None) == -1
    assert L.lbm_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(512), ctypes.c_void_p(512),
                      ctypes.c_void_p(1024), None, None, None) == -1
    # misaligned workspace
    assert L.lbm_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(512), ctypes.c_void_p(1024),
                      ctypes.c_void_p(1000), None, None, None) == -1
    assert L.lbm_init(None, ctypes.byref(p), ctypes.c_void_p(512), ctypes.c_void_p(1024),
                      ctypes.c_void_p(1024), None, None, None) == -1


def test_calls_on_null_context_fail_cleanly(L):
    assert L.lbm_ib_step(None, None, None, None, 1, None) == -1
    assert L.lbm_check(None) == -1
    assert L.lbm_read_populations(None, None) == -1
    assert L.lbm_macros(None, None, None, None) == -1
    assert L.lbm_body_forces(None, None, None, None) == -1
    assert L.lbm_step_count(None) == -1
    L.lbm_destroy(None)


def test_strerror_covers_every_status(L):
    for code in lbm.STATUS:
        s = lbm.strerror(code)
        assert s and s != "unknown status"
    assert lbm.strerror(42) == "unknown status"


def test_adjoint_ring_size_is_host_computed(L):
    p = lbm.make_params(128, 64, 64, 0.6, lbm.BC_VELOCITY, lbm.BC_OUTFLOW, max_markers=3000, max_bones=10,
                        max_active_tiles=256, with_adjoint=True)
    one = L.lbm_adjoint_ring_bytes(ctypes.byref(p), 1)
    assert one > 0 and one % 256 == 0
    assert L.lbm_adjoint_ring_bytes(ctypes.byref(p), 20) == 20 * one
    assert L.lbm_adjoint_ring_bytes(ctypes.byref(p), 0) == 0
    big = lbm.make_params(128, 64, 64, 0.6, lbm.BC_VELOCITY, lbm.BC_OUTFLOW, max_markers=6000, max_bones=10,
                          max_active_tiles=256, with_adjoint=True)
    assert L.lbm_adjoint_ring_bytes(ctypes.byref(big), 1) > one
    bad = lbm.make_params(128, 64, 64, 0.5, max_markers=3000)
    assert L.lbm_adjoint_ring_bytes(ctypes.byref(bad), 4) == 0
    # the adjoint buffers enlarge the workspace
    plain = lbm.make_params(128, 64, 64, 0.6, lbm.BC_VELOCITY, lbm.BC_OUTFLOW, max_markers=3000, max_bones=10,
                            max_active_tiles=256)
    assert L.lbm_workspace_bytes(ctypes.byref(p)) > L.lbm_workspace_bytes(ctypes.byref(plain))


def test_adjoint_batch_and_state_calls_on_null_handles_fail_cleanly(L):
    w = (ctypes.c_double * 4)(0, 0, 0, 0)
    assert L.lbm_adjoint_step(None, None, None, None, None, w, None, None, None) == -1
    assert L.lbm_adjoint_segment(None, None, None, 1, None, None, None, w, None, None, None, None) == -1
    assert L.lbm_adjoint_sweep(None, None, None, 1, None, None, None, w, None, None, None, None) == -1
    assert L.lbm_adjoint_record(None, None, None, 1, None, None, None, None, None) == -1
    assert L.lbm_bind_populations(None, None, None) == -1
    assert L.lbm_state_save(None, None) == -1
    assert L.lbm_state_restore(None, None, 0) == -1
    assert L.lbm_set_stream(None, None) == -1
    assert L.lbm_batch_bytes(0) == 0 and L.lbm_batch_bytes(100000) == 0 and L.lbm_batch_bytes(64) > 0
    assert L.lbm_batch_create(None, None, 0, None, None) == -1
    assert L.lbm_batch_run(None, 2, 0, 0) == -1
    assert L.lbm_batch_autotune(None, 1, None) == -1
    assert L.lbm_batch_set_shapes(None, None) == -1
    assert L.lbm_batch_check(None) == -1
    assert L.lbm_batch_set_groups(None, 2, None, None) == -1
    L.lbm_batch_destroy(None)


def test_batch_group_bytes_cover_every_group(L):
    """Each of g groups holds at most nenv - g + 1 environments (the split
    gives every group one), so g such slices cover any split; counts outside
    [2, min(nenv, 8)] are refused."""
    for nenv in (2, 5, 64, 512):
        for g in range(2, min(nenv, 8) + 1):
            assert L.lbm_batch_group_bytes(nenv, g) == g * L.lbm_batch_bytes(nenv - g + 1)
    assert L.lbm_batch_group_bytes(64, 1) == 0
    assert L.lbm_batch_group_bytes(64, 9) == 0
    assert L.lbm_batch_group_bytes(3, 4) == 0
    assert L.lbm_batch_group_bytes(0, 2) == 0


def test_implicit_scheme_workspace_holds_its_buffers(L):
    """The implicit velocity correction's buffers (a second fixed-point force
    per active tile, four marker vectors, dot-product partials) are laid out
    only when asked for."""
    kw = dict(max_markers=3000, max_bones=10, max_active_tiles=256)
    d = lbm.make_params(128, 64, 64, 0.6, **kw)
    i = lbm.make_params(128, 64, 64, 0.6, ib_scheme=lbm.IB_IMPLICIT, **kw)
    extra = L.lbm_workspace_bytes(ctypes.byref(i)) - L.lbm_workspace_bytes(ctypes.byref(d))
    assert extra >= 256 * 1536 * 8 + 12 * 3000 * 4
    assert extra < 256 * 1536 * 8 + 12 * 3000 * 4 + 64 * 1024


def test_static_init_validates_on_the_host(L):
    """lbm_init_static (no caller workspace) refuses bad arguments, and a
    problem whose workspace exceeds the static array, before any device call."""
    ctx = ctypes.c_void_p()
    bad = lbm.make_params(16, 16, 16, 0.5)
    assert L.lbm_init_static(ctypes.byref(ctx), ctypes.byref(bad), ctypes.c_void_p(512), ctypes.c_void_p(1024),
                             None, None, None) == -1
    ok = lbm.make_params(16, 16, 16, 0.6)
    assert L.lbm_init_static(ctypes.byref(ctx), ctypes.byref(ok), None, ctypes.c_void_p(1024), None, None,
                             None) == -1
    assert L.lbm_init_static(ctypes.byref(ctx), ctypes.byref(ok), ctypes.c_void_p(512), ctypes.c_void_p(512),
                             None, None, None) == -1
    assert L.lbm_init_static(None, ctypes.byref(ok), ctypes.c_void_p(512), ctypes.c_void_p(1024), None, None,
                             None) == -1
    big = lbm.make_params(384, 192, 192, 0.6, lbm.BC_VELOCITY, lbm.BC_OUTFLOW, max_markers=12000, max_bones=10)
    assert L.lbm_workspace_bytes(ctypes.byref(big)) > lbm.STATIC_WORKSPACE_BYTES
    assert L.lbm_init_static(ctypes.byref(ctx), ctypes.byref(big), ctypes.c_void_p(512), ctypes.c_void_p(1024),
                             None, None, None) == lbm.ERR_CAPACITY
    assert not ctx.value
    # the fish fits once its active tiles are bounded
    fish = lbm.make_params(384, 192, 192, 0.6, lbm.BC_VELOCITY, lbm.BC_OUTFLOW, max_markers=12000, max_bones=10,
                           max_active_tiles=1024)
    assert L.lbm_workspace_bytes(ctypes.byref(fish)) <= lbm.STATIC_WORKSPACE_BYTES


def test_population_layout_strides(L):
    """Rows ([nz][ny][27][nx]) by default when nx is a multiple of 32, planes
    otherwise or on request; the strides address element (i, x, y, z) at
    (z ny + y) rs + i ps + x inside lbm_population_bytes."""
    st = (ctypes.c_int64 * 3)()
    for nx, layout, want_rows in ((384, lbm.LAYOUT_AUTO, True), (48, lbm.LAYOUT_AUTO, False),
                                  (384, lbm.LAYOUT_PLANES, False), (37, lbm.LAYOUT_ROWS, True)):
        for storage in ("f32", "f16"):
            p = lbm.make_params(nx, 20, 12, 0.6, storage=storage, layout=layout)
            assert L.lbm_population_strides(ctypes.byref(p), st) == 0
            ps, rs, rows = st[0], st[1], st[2]
            assert rows == (1 if want_rows else 0)
            if want_rows:
                assert (ps, rs) == (nx, 27 * nx)
            else:
                assert rs == nx and ps >= nx * 20 * 12
            # the last element of the last population fits in the buffer
            last = (12 * 20 - 1) * rs + 26 * ps + nx - 1
            assert (last + 1) * (4 if storage == "f32" else 2) <= L.lbm_population_bytes(ctypes.byref(p))
    bad = lbm.make_params(64, 16, 16, 0.6, layout=3)
    assert L.lbm_population_strides(ctypes.byref(bad), st) == -1
    assert L.lbm_population_bytes(ctypes.byref(bad)) == 0
    assert L.lbm_population_strides(ctypes.byref(lbm.make_params(64, 16, 16, 0.6)), None) == -1
    # block (bx, -1): bx consecutive cells; needs bx
    assert L.lbm_population_bytes(ctypes.byref(lbm.make_params(64, 16, 16, 0.6, block=(256, -1)))) > 0
    assert L.lbm_population_bytes(ctypes.byref(lbm.make_params(64, 16, 16, 0.6, block=(0, -1)))) == 0
    assert L.lbm_population_bytes(ctypes.byref(lbm.make_params(64, 16, 16, 0.6, block=(576, -1)))) == 0


def test_ceiling_library_exports_and_validates():
    """The reference streaming kernels (include/hbm_ceiling.h): every declared
    function is exported, and bad arguments are refused before any launch."""
    import re

    from paper_2206_01683_amd import hbm_ceiling
    C = hbm_ceiling.lib()
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "hbm_ceiling.h")).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(hbm_[a-z_0-9]+)\s*\(", text)))
    assert names == ["hbm_copy", "hbm_pull27", "hbm_read"]
    for n in names:
        assert hasattr(C, n), n
    p, q = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    assert C.hbm_copy(p, q, 100, None) == -1          # not a multiple of 16
    assert C.hbm_copy(ctypes.c_void_p(4100), q, 160, None) == -1  # misaligned
    assert C.hbm_copy(None, q, 160, None) == -1
    assert C.hbm_read(p, 0, q, None) == -1
    assert C.hbm_pull27(p, p, 8, 8, 8, 8, 216, 0, None) == -1      # aliased
    assert C.hbm_pull27(p, q, 8, 8, 8, 8, 64, 0, None) == -1       # rows need rs = 27 nx
    assert C.hbm_pull27(p, q, 8, 8, 8, 100, 8, 0, None) == -1      # planes need ps >= cells
    assert C.hbm_pull27(p, q, 0, 8, 8, 8, 216, 0, None) == -1
    assert C.hbm_pull27(p, q, 8, 8, 8, 8, 216, -1, None) == -1     # blocks per compute unit
    assert C.hbm_pull27(p, q, 8, 8, 8, 8, 216, 33, None) == -1


def test_ib_workgroups_parameter_is_validated(L):
    for v in (-1, 0, 1, 64, 1024):
        assert L.lbm_population_bytes(ctypes.byref(lbm.make_params(64, 16, 16, 0.6, ib_workgroups=v))) > 0
    for v in (-2, 1025):
        assert L.lbm_population_bytes(ctypes.byref(lbm.make_params(64, 16, 16, 0.6, ib_workgroups=v))) == 0
