"""Local registration (Euler grid around an initial guess, small translation box):
oracle parity on sampled rotations and recovery of the known displacement."""
import numpy as np
import pytest

import oracle
from paper_2502_00115_amd import synth
from parity import compare_records

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2502_00115_amd import dses  # noqa: E402


@pytest.mark.parametrize("seed", [0, 1])
def test_local_registration_parity_and_recovery(seed):
    p = synth.make_local(seed)
    box = p.meta["t_box"]
    g = dses.register(p.src, p.tgt, p.rotations, p.eps, t_min=-box, t_max=box, records=True)
    rng = np.random.default_rng(seed)
    which = np.unique(np.concatenate([rng.choice(len(p.rotations), 150, replace=False),
                                      [g.rot_index]]))
    orc = oracle.records(p.src, p.tgt, p.rotations, p.eps, t_min=-box, t_max=box, which=which)
    compare_records(g.records[which], orc, len(p.src), label=f"local {seed}")
    # the selected pose is near the displacement applied to the source: 1 mm noise on a
    # 0.1 m object and 2 mm translation bins allow errors of a few tenths of a bin in
    # angle (~1 deg) and of a bin or so in translation
    ang = np.rad2deg(np.arccos(np.clip((np.trace(g.R.astype(np.float64).T @ p.R_true) - 1) / 2,
                                       -1, 1)))
    assert ang < 3.0, ang
    assert np.linalg.norm(g.t - p.t_true) < 3 * p.eps


def test_euler_grid_of_the_library_equals_the_generator():
    step = np.deg2rad(0.5)
    a = dses.euler_grid(10, step)
    b = synth.euler_grid(10, np.float32(step)).reshape(-1, 9)
    np.testing.assert_allclose(a, b, atol=1e-6)
