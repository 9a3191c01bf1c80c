"""Light-cone windows (the basis of the full-size parity checks): an explicit
leapfrog moves information by at most one cell per step, so after n steps a
window of the grid with PEC cut faces holds the same fields as the full grid
on every cell more than n + 1 cells from a cut face.  Checked here on the
oracle itself, on a layered, lossy microstrip with its source and layers
inside the window."""
import numpy as np

import oracle
import workloads as W


def test_window_matches_full_grid_inside_light_cone():
    n = 24
    p = W.small_microstrip(nsteps=n, fp32=False, seed=9, sigma_strip=5.8e7)
    full = oracle.Oracle(p).run(n)
    box = (0, 70, 4, p.ny, 0, p.nz)              # cut faces: x = 70, y = 4
    sub = W.window(p, box)
    assert sub.faces[1] == W.PEC and sub.faces[2] == W.PEC
    assert sub.faces[0] == p.faces[0] and sub.pml_cells[0] == p.pml_cells[0]
    win = oracle.Oracle(sub).run(n)
    m = n + 2
    scale = max(np.max(np.abs(full.field(c))) for c in range(3))
    assert scale > 0
    for c in range(6):
        a = full.field(c)[:, box[2] + m:, :box[1] - m]
        b = win.field(c)[:, m:, :box[1] - box[0] - m]
        assert a.shape == b.shape
        assert np.max(np.abs(a - b)) <= 1e-13 * scale, c
    # near a cut face the window differs (the check above is not vacuous)
    a = full.field(W.EZ)[:, box[2]:, :box[1]]
    b = win.field(W.EZ)[:, :, :box[1] - box[0]]
    assert np.max(np.abs(a - b)) > 1e-6 * scale
