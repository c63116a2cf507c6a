"""Sampled cells of a full-size painted mesh, computed by the FP64 oracle
(test infrastructure: the full-size GPU paint check uses it, and
test_oracle_cells pins it against a whole-mesh oracle paint)."""
import numpy as np
import torch

import oracle as O


def oracle_cells(x, off, q, n, cells, dev):
    """The FP64 oracle's int64 value of each sampled cell of the full mesh.
    The particles whose eight corners include a sampled cell c are found on
    the device (their floor cell lies in c - {0,1}^3); each cell's particles
    are then moved down by whole cells so that c lands on cell L = min(c, 8)
    of a 16^3 mesh (a particle one cell below c = 0 lands on cell 15, the
    wrap).  Moving a float32 position down by an integer keeps it a float32
    value with the same fraction, so each cloud-in-cell weight is unchanged,
    and the oracle's painted cell L is the value of c."""
    P = x.shape[1]
    deltas = np.array([[a, b, e] for a in (0, 1) for b in (0, 1) for e in (0, 1)], dtype=np.int64)
    bases = (cells[:, None, :] - deltas[None]) % n
    blin = np.unique(((bases[..., 0] * n + bases[..., 1]) * n + bases[..., 2]).ravel())
    bset = torch.from_numpy(blin).to(dev)
    found = []
    step = 1 << 24
    for lo in range(0, P, step):
        c = torch.floor(x[:, lo:lo + step]).to(torch.int64) & (n - 1)
        lin = (c[0] * n + c[1]) * n + c[2]
        del c
        found.append((torch.nonzero(torch.isin(lin, bset)).squeeze(1) + lo).cpu())
        del lin
    idx = torch.cat(found)
    pos = x[:, idx.to(dev)].cpu().numpy()
    idx = idx.numpy()
    seg = np.searchsorted(off, idx, side="right") - 1
    base = np.floor(pos).astype(np.int64) % n
    out = np.zeros(len(cells), dtype=np.int64)
    for j, cc in enumerate(cells):
        rel = (cc[:, None] - base) % n
        sel = np.nonzero(np.all(rel <= 1, axis=0))[0]
        L = np.minimum(cc, 8)
        u = np.mod(pos[:, sel].astype(np.float64) - (cc - L)[:, None], float(n))
        u = np.where(u >= n - 1, u - (n - 16), u)
        assert np.all(u < 16) and np.all(u >= np.maximum(L - 1, 0)[:, None])
        assert np.array_equal(u.astype(np.float32).astype(np.float64), u)   # still float32 values
        mesh = np.zeros((16, 16, 16), dtype=np.int64)
        for g in np.unique(seg[sel]):
            k = np.nonzero(seg[sel] == g)[0]
            O.paint_q(np.ascontiguousarray(u[:, k]), 0, len(k), int(q[g]), 16, mesh)
        out[j] = mesh[L[0], L[1], L[2]]
    return out, len(idx)
