"""CPU checks of the C ABI: the library loads, exports exactly what the
header declares, and rejects bad arguments on the host before touching the
device."""
import ctypes as C
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT


@pytest.fixture(scope="module")
def L():
    from paper_1110_0995_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1110_0995_amd import build
        build.build()
    return _lib.load()


def _header_functions():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, h)).read() for h in sorted(os.listdir(inc)) if h.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?[a-z0-9_]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M))


def test_header_and_exports_agree(L):
    from paper_1110_0995_amd import _lib
    decl = _header_functions()
    assert decl == set(_lib.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert decl <= exported
    # nothing but the C ABI is exported (kernels and helpers stay hidden)
    assert {s for s in exported if not s.startswith("_")} == decl
    for name in decl:
        getattr(L, name)


def test_plane_stride(L):
    for n, prec in [(1, 0), (16384, 1), (16777216, 2), (2097152, 1), (327680, 1), (100, 0)]:
        s = L.lbm_plane_stride(n, prec)
        assert s >= n and s % 64 == 0
        es = 8 if prec == 0 else 4
        assert (s * es) % 65536 != 0
    assert L.lbm_plane_stride(0, 1) == 0


def _params(**kw):
    from paper_1110_0995_amd import _lib
    p = _lib.LbmParams()
    p.nx, p.ny, p.nz = 8, 8, 8
    p.periodic[:] = [1, 1, 1]
    p.tau = 0.8
    p.prec = 2
    p.solid, p.f_a, p.f_b = 4096, 8192, 16384  # never dereferenced: every case below fails validation
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw,msg", [
    (dict(tau=0.5), "tau"), (dict(tau=float("nan")), "tau"), (dict(nx=0), "size"), (dict(nz=-3), "size"),
    (dict(prec=7), "prec"), (dict(plane_stride=100), "plane_stride"), (dict(plane_stride=448), "plane_stride"),
    (dict(solid=None), "non-NULL"), (dict(f_b=8192), "distinct"), (dict(f_a=8196), "aligned"),
    (dict(gfield=4098, prec=0), "misaligned"), (dict(body_force=(C.c_double * 3)(0, float("inf"), 0)), "body_force"),
])
def test_init_rejects_bad_params(L, kw, msg):
    from paper_1110_0995_amd import _lib
    p = _params(**kw)
    ctx = C.c_void_p(1234)
    rc = L.lbm_init(C.byref(p), C.byref(ctx))
    assert rc == _lib.LBM_EINVAL
    assert ctx.value is None
    assert msg in L.lbm_last_error().decode()
    assert L.lbm_workspace_bytes(C.byref(p)) == -1


def test_null_context_calls(L):
    from paper_1110_0995_amd import _lib
    assert L.lbm_step(None, 1) == _lib.LBM_EINVAL
    assert L.lbm_step_timed(None, None, None) == _lib.LBM_EINVAL
    assert L.ibm_couple(None, None) == _lib.LBM_EINVAL
    assert L.ibm_rest_shape(None, None) == _lib.LBM_EINVAL
    assert L.lbm_read_fields(None, None, None, None) == _lib.LBM_EINVAL
    assert L.lbm_current(None, None, None) == _lib.LBM_EINVAL
    assert L.lbm_store_f64(None, None) == _lib.LBM_EINVAL
    assert L.lbm_init(None, None) == _lib.LBM_EINVAL
    assert L.lbm_init_channels(None, 1, None, None) == _lib.LBM_EINVAL
    assert L.lbm_set_launch(None, 4, 0) == _lib.LBM_EINVAL
    assert L.lbm_set_ibm_overlap(None, 1) == _lib.LBM_EINVAL
    assert L.lbm_run(None, None, 1, 0) == _lib.LBM_EINVAL
    L.lbm_destroy(None)
    assert b"NULL" in L.lbm_last_error()


CHAN_BYTES = 32  # one channel record: nx, ny, nz, tiles per row, first node (8 bytes), first tile, pad


def test_workspace_bytes(L):
    p = _params()
    n = 512
    tiles = 8 * 8  # one 64-wide tile per x-row
    # node class + link mask + spread force, fallback accumulator and velocity
    # field (4 floats each) + node marks + tile marks and tile fallback flags
    # (each padded to 16) and tile list (4 bytes each) + the solid/wall masks
    # (16 bytes) and stencil-node mask (8 bytes) of each tile + list length +
    # claim epoch + reduction partials + sums + the channel record + the
    # collide-stream workgroup table (4 bytes per workgroup of 8 one-tile
    # rows: 8 of them)
    one = n + 4 * n + 12 * n * 4 + n + 2 * tiles + 4 * tiles + 24 * tiles + 4 + 4 + 2 * 32 + 32 + CHAN_BYTES + 4 * 8
    assert L.lbm_workspace_bytes(C.byref(p)) == one
    dims = (C.c_int32 * 3)(8, 8, 8)
    assert L.lbm_workspace_bytes_channels(C.byref(p), 1, dims) == one


def test_workspace_bytes_channels(L):
    p = _params()
    dims = (C.c_int32 * 6)(100, 3, 2, 8, 8, 8)
    n = 600 + 512
    tiles = 2 * 3 * 2 + 8 * 8
    # as for one channel, plus a 2-byte channel id per tile; workgroups: the
    # 6 two-tile rows of channel 0 in groups of 4 rows (2), 8 of channel 1
    expect = (n + 4 * n + 12 * n * 4 + n + 2 * 80 + 4 * tiles + 24 * tiles + 4 + 4 + 5 * 32 + 32 + 2 * CHAN_BYTES
              + 2 * tiles + 4 * (2 + 8))
    assert L.lbm_workspace_bytes_channels(C.byref(p), 2, dims) == expect


@pytest.mark.parametrize("nch,dims,msg", [
    (0, [8, 8, 8], "nch"), (70000, [8, 8, 8], "nch"), (2, [8, 8, 8, 8, 0, 8], "channel 1 size"),
    (1, [-1, 8, 8], "channel 0 size"), (2, [1024, 1024, 1024, 8, 8, 8], "too large"),
])
def test_init_channels_rejects(L, nch, dims, msg):
    from paper_1110_0995_amd import _lib
    p = _params()
    arr = (C.c_int32 * max(len(dims), 3 * max(nch, 1)))(*dims)
    ctx = C.c_void_p(1234)
    rc = L.lbm_init_channels(C.byref(p), nch, arr, C.byref(ctx))
    assert rc == _lib.LBM_EINVAL and ctx.value is None
    assert msg in L.lbm_last_error().decode()
    assert L.lbm_init_channels(C.byref(p), 1, None, C.byref(ctx)) == _lib.LBM_EINVAL
    assert "dims" in L.lbm_last_error().decode()
    assert L.lbm_workspace_bytes_channels(C.byref(p), nch, arr) == -1


def test_init_channels_checks_params(L):
    from paper_1110_0995_amd import _lib
    p = _params(tau=0.4)
    dims = (C.c_int32 * 3)(8, 8, 8)
    ctx = C.c_void_p(1234)
    assert L.lbm_init_channels(C.byref(p), 1, dims, C.byref(ctx)) == _lib.LBM_EINVAL
    assert "tau" in L.lbm_last_error().decode() and ctx.value is None
