"""CPU checks of the magnetic-stage C ABI (include/magnet.h): the ctypes
struct has the C layout, the workspace size follows its stated layout, and
bad arguments are rejected on the host before anything touches the device."""
import ctypes as C
import os
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


def _params(n=1000, **kw):
    from paper_1110_0995_amd import _lib
    p = _lib.MagParams()
    p.n = n
    p.nsheets = 1
    for i, v in enumerate((-4.0, 0.0, 64.0, 0.0, 32.0, 1.0)):
        p.sheets[0][i] = v
    p.bias[2] = 0.5
    p.a, p.chi, p.eta, p.dt = 1.5, 4.0, 1.0, 0.1
    p.rep_a, p.rep_n, p.rep_cut = 0.1, 2.0, 1.0
    p.nx, p.ny, p.nz = 64, 32, 16
    p.periodic[0] = p.periodic[1] = 1
    p.walls_z = 1
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_struct_layout_matches_header(tmp_path):
    from paper_1110_0995_amd import _lib
    src = tmp_path / "lay.c"
    fields = [f for f, _ in _lib.MagParams._fields_]
    body = "".join(f'printf("{f} %zu\\n", offsetof(mag_params, {f}));' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "magnet.h"\n'
                   f'int main(void) {{ {body} printf("size %zu\\n", sizeof(mag_params)); return 0; }}\n')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(ln.split() for ln in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for f in fields:
        assert int(out[f]) == getattr(_lib.MagParams, f).offset, f
    assert int(out["size"]) == C.sizeof(_lib.MagParams)


def test_workspace_bytes(L):
    # moments and one-bead forces, then one [3][n] force array per block of
    # b beads, each 256-byte aligned; b = 256, 128 or 64: the largest giving
    # at least 2048 block pairs (else 64)
    def expect(n):
        b = 64
        for bb in (256, 128):
            nb = -(-n // bb)
            if nb * (nb + 1) // 2 >= 2048:
                b = bb
                break
        plane = -(-(24 * n) // 256) * 256
        return plane * (2 + -(-n // b))

    for n in (1, 255, 256, 1000, 4096, 8191, 8192, 16384, 100000, 1 << 17):
        p = _params(n)
        assert L.mag_workspace_bytes(C.byref(p)) == expect(n), n
    assert expect(1) == 256 * 3 and expect(16384) == 24 * 16384 * (2 + 64)
    assert expect(4096) == 24 * 4096 * (2 + 64)  # blocks of 64: 2080 block pairs
    p = _params((1 << 17) + 1)
    assert L.mag_workspace_bytes(C.byref(p)) == 0


@pytest.mark.parametrize("kw,msg", [
    (dict(n=0), b"n must be"),
    (dict(nsheets=9), b"nsheets"),
    (dict(a=0.0), b"a must be"),
    (dict(chi=-1.0), b"chi"),
    (dict(eta=0.0), b"eta"),
    (dict(dt=float("nan")), b"dt"),
    (dict(rep_n=0.0), b"rep_n"),
    (dict(rep_cut=0.0), b"rep_cut"),
    (dict(nz=0), b"nx, ny, nz"),
    (dict(walls_z=2), b"walls_z"),
])
def test_rejects_bad_params(L, kw, msg):
    from paper_1110_0995_amd import _lib
    p = _params(**kw)
    assert L.mag_workspace_bytes(C.byref(p)) == 0
    assert msg in L.lbm_last_error()
    buf = C.c_void_p(256)  # never dereferenced: the checks fail first
    assert L.mag_run(C.byref(p), buf, 1, buf) == _lib.LBM_EINVAL
    assert L.mag_forces(C.byref(p), buf, buf, buf, buf) == _lib.LBM_EINVAL
    assert L.mag_freeze(C.byref(p), buf, buf) == _lib.LBM_EINVAL


def test_rejects_bad_sheet_and_buffers(L):
    from paper_1110_0995_amd import _lib
    p = _params()
    p.sheets[0][2] = p.sheets[0][1]  # x1 == x0
    assert L.mag_field(C.byref(p), C.c_void_p(256), 4, C.c_void_p(256), None) == _lib.LBM_EINVAL
    assert b"sheet 0" in L.lbm_last_error()
    p = _params()
    assert L.mag_run(C.byref(p), C.c_void_p(256), 1, C.c_void_p(128)) == _lib.LBM_EINVAL
    assert b"256-byte" in L.lbm_last_error()
    assert L.mag_run(C.byref(p), C.c_void_p(256), -1, C.c_void_p(256)) == _lib.LBM_EINVAL
    assert L.mag_run(C.byref(p), None, 1, C.c_void_p(256)) == _lib.LBM_EINVAL
    assert L.mag_field(C.byref(p), None, 4, C.c_void_p(256), None) == _lib.LBM_EINVAL
    assert L.mag_field(C.byref(p), C.c_void_p(256), -1, C.c_void_p(256), None) == _lib.LBM_EINVAL
    # empty work is fine and enqueues nothing
    assert L.mag_field(C.byref(p), None, 0, None, None) == _lib.LBM_OK
    assert L.mag_run(C.byref(p), C.c_void_p(256), 0, C.c_void_p(256)) == _lib.LBM_OK
