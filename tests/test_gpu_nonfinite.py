"""Failure detection on the device: a node whose populations are not finite
is flagged by the collide-stream pass itself, and the library reports it
(LBM_ENONFINITE) from a later lbm_run / lbm_step call, or at once from
lbm_check_finite, without host sums.  The bad value is put into the state
from the host (lbm_load_f64); the kernels only compute with it."""
import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import lbm as mod
    return mod


@pytest.mark.parametrize("prec", ["f32dev", "f32", "f64"])
def test_nan_population_is_reported(lbm, prec):
    import torch
    from paper_1110_0995_amd import _lib
    s = S.posts_and_cells(64, 32, 24, posts_x=1, posts_y=1, post_radius=4, gap=6, ncells=1, cell_radius=3.0,
                          level=2, tau=0.8, gx=1e-5, seed=1)
    lat = lbm.Lattice.from_scenario(s, prec=prec)
    mesh = lbm.Mesh(lat, s.cells)
    lat.run(6, mesh, steps_per_graph=2)
    assert lat.check_finite()
    lat.run(2, mesh)  # a clean run leaves nothing to report
    lat.run(2, mesh)
    assert lat.check_finite()
    f = lat.populations_f64().cpu().numpy()
    fluid = np.flatnonzero(s.solid.reshape(-1) == 0)
    f[7, int(fluid[len(fluid) // 2])] = float("nan")
    lat.load_f64(f)
    lat.step(1)  # the pass meets the NaN; nothing has been copied back yet
    assert not lat.check_finite()
    with pytest.raises(_lib.LbmError) as e:
        lat.run(1, mesh)
    assert e.value.code == _lib.LBM_ENONFINITE
    with pytest.raises(_lib.LbmError):
        lat.step(1)
    # a fresh state clears the report
    lat.load_f64(np.nan_to_num(f, nan=1.0 / 18))
    lat.run(4, mesh, steps_per_graph=2)
    assert lat.check_finite()
    lat.close()


def test_report_reaches_a_later_run_without_waiting(lbm):
    """lbm_run queues the copy of the flag; a later call that finds it set
    fails (the copy has landed once the stream is idle)."""
    import torch
    from paper_1110_0995_amd import _lib
    s = S.poiseuille(32, 8, 8)
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    f = lat.populations_f64().cpu().numpy()
    f[3, 5 + 32 * (2 + 8 * 3)] = float("inf")  # x 5, y 2, z 3: a fluid node
    lat.load_f64(f)
    lat.run(2, None)
    torch.cuda.synchronize()
    with pytest.raises(_lib.LbmError) as e:
        lat.run(2, None)
    assert e.value.code == _lib.LBM_ENONFINITE
    lat.close()
