"""The sampled-cell oracle used by the full-size GPU paint check
(cell_oracle.oracle_cells: particles moved down by whole cells onto a 16^3
mesh) against the oracle's paint of the whole mesh, on the CPU: the synthetic
C5 state (256^3 mesh) with tile-face positions, 300 random cells and 300 on
faces and the wrap must agree bit for bit."""
import numpy as np
import torch

import oracle as O
from cell_oracle import oracle_cells
from paper_2007_13394_amd import inputs as I


def test_sampled_cells_equal_the_whole_mesh_paint():
    cfg = I.config("C5")
    n = cfg["n_mesh"]
    x, _ = I.synthetic_state(cfg, seed=5)
    nc, nn, per = I.counts(cfg)
    x[:, :nc // 4] = I.tile_face_positions(n, nc // 4, seed=6)
    x = np.ascontiguousarray(x)
    off, _, q = O.segments(O.make_sim(cfg))
    mesh = np.zeros((n, n, n), dtype=np.int64)
    x64 = x.astype(np.float64)
    for g in range(len(off) - 1):
        O.paint_q(x64, int(off[g]), int(off[g + 1] - off[g]), int(q[g]), n, mesh)
    rng = np.random.default_rng(1)
    special = np.array([0, 15, 16, n // 2, n - 16, n - 1])
    cells = np.concatenate([rng.integers(0, n, size=(300, 3)), rng.choice(special, size=(300, 3))])
    want, nfound = oracle_cells(torch.from_numpy(x), np.asarray(off), np.asarray(q), n, cells, "cpu")
    got = mesh[cells[:, 0], cells[:, 1], cells[:, 2]]
    assert nfound > 100 and np.count_nonzero(got) > 300
    assert np.array_equal(got, want)
