"""GPU test of mag_run_static, the variant of mag_run for callers that
cannot allocate: its work lives in the library's static device array
instead of a caller's buffer.  Called through the C-ABI, it must give
bit-for-bit the positions mag_run gives with a workspace of its own, on two
calls in a row (the second with fewer beads, so that the array holds the
first call's larger contents when it starts), and refuse a bead count whose
work does not fit, before enqueueing anything."""
import ctypes as C

import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def magnet():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import magnet as mod
    return mod


def _static_run(b, nsteps):
    import torch
    from paper_1110_0995_amd import _lib
    b.p.stream = torch.cuda.current_stream(b.device).cuda_stream
    _lib.check(b.L.mag_run_static(C.byref(b.p), C.c_void_p(b.x.data_ptr()), int(nsteps)))


def _pair(magnet, st, nsteps):
    """Positions after nsteps of mag_run (own workspace) and of mag_run_static."""
    b = magnet.Beads(st)
    x0 = b.x.clone()
    b.run(nsteps)
    ref = b.positions()
    b.x.copy_(x0)
    _static_run(b, nsteps)
    out = b.positions()
    return ref, out, b


def test_static_work_matches_workspace_twice(magnet):
    big = S.bead_stage(n=16384)                     # 24.75 MiB of work
    small = S.bead_stage(192, 96, 64, n=1500, seed=3)
    for st, nsteps in ((big, 12), (small, 40)):
        ref, out, b = _pair(magnet, st, nsteps)
        assert np.isfinite(ref).all()
        assert np.abs(ref - st.x).max() > 0  # the beads moved
        assert np.array_equal(ref, out), st.n
    # and once more at the small size right after the large one
    b = magnet.Beads(big)
    _static_run(b, 2)
    ref, out, _ = _pair(magnet, small, 40)
    assert np.array_equal(ref, out)


def test_static_work_refuses_too_many_beads(magnet):
    import torch
    from paper_1110_0995_amd import _lib
    st = S.bead_stage(n=20000)  # blocks of 128 beads: about 38 MB of work
    b = magnet.Beads(st)
    assert b.L.mag_workspace_bytes(C.byref(b.p)) > 32 << 20
    x0 = b.x.clone()
    b.p.stream = torch.cuda.current_stream(b.device).cuda_stream
    rc = b.L.mag_run_static(C.byref(b.p), C.c_void_p(b.x.data_ptr()), 5)
    assert rc == _lib.LBM_EINVAL
    assert "mag_run_static" in b.L.lbm_last_error().decode()
    torch.cuda.synchronize()
    assert torch.equal(b.x, x0)
