"""Oracle of the two-grid fast-LGF far-field approximation (test
infrastructure).  The paper evaluates the lattice convolution with an
FMM-type fast summation on the block octree (Sec. 2.2, Sec. 5; its defining
paper is not at hand), so this is a reading derived from first principles:

* near field: block pairs (t, s) with max_i |t_i - s_i| <= D summed exactly,
      u_near(n) = dx^2 sum_{m: |b(n) - b(m)|_inf <= D} G(n - m) f(m);
* far field: the kernel between the cells of two far blocks is replaced by
  its cubic interpolation in both arguments from nodes twice as coarse as
  the cells, nb/2 per block and axis, node k of a block at fine position
  2k + 1 (so node differences are even lattice vectors and G is sampled at
  G(2 j)).  Every block interpolates from its own nodes only: a cell takes
  the 4 nodes nearest to it along each axis, the window shifted to stay in
  the block, with Lagrange weights (exact for cubics), tensorised.  Then
      A f (node j of block s) = sum_{m in s} w_j(m) f(m)     (A = I^T),
      U (node i of block t) = dx^2 sum_{s: |t - s|_inf > D} sum_{j in s} G(2 (i - j)) (A f)(j),
      u_far(n) = sum_{i in b(n)} w_i(n) U(i)                 (interpolation I),
  and near and far split the block pairs exactly the same way.
* u = u_near + u_far.

The cut between near and far is by block offset, the same in both terms,
so with D >= the extent of the support nothing is far and u is the exact
convolution.
"""
import numpy as np

from . import direct, lgf_table


def node_weights(i, nb):
    """Block-local nodes and weights of the cubic interpolation to local cell
    index i (0 <= i < nb) along one axis: the 4 nodes (of nb/2) nearest to
    the cell centre, the window shifted to stay in the block.  Positions in
    node units: node k at k + 1/2, cell i at (i + 1/2) / 2."""
    h = nb // 2
    x = (i + 0.5) / 2.0
    start = min(max(int(np.floor(x - 0.5)) - 1, 0), h - 4)
    nodes = np.arange(start, start + 4)
    pos = nodes + 0.5
    w = np.ones(4)
    for j in range(4):
        for k in range(4):
            if k != j:
                w[j] *= (x - pos[k]) / (pos[j] - pos[k])
    return nodes, w


def interp_pairs(cells, nb):
    """For fine cells (n, 3): global node coordinates (n, 64, 3) and weights (n, 64)."""
    cells = np.asarray(cells, dtype=np.int64)
    blk = np.floor_divide(cells, nb)
    loc = cells - blk * nb
    table = [node_weights(i, nb) for i in range(nb)]
    tn = np.array([t[0] for t in table])          # (nb, 4)
    tw = np.array([t[1] for t in table])
    offs = [tn[loc[:, a]] + (nb // 2) * blk[:, a:a + 1] for a in range(3)]
    ws = [tw[loc[:, a]] for a in range(3)]
    nodes = np.stack(np.broadcast_arrays(offs[0][:, :, None, None], offs[1][:, None, :, None],
                                         offs[2][:, None, None, :]), axis=-1).reshape(len(cells), 64, 3)
    wt = (ws[0][:, :, None, None] * ws[1][:, None, :, None] * ws[2][:, None, None, :]).reshape(len(cells), 64)
    return nodes, wt


def anterpolate(cells, f, nb):
    """A f = I^T f: (node coordinates (k, 3), values (k,))."""
    nodes, wt = interp_pairs(cells, nb)
    vals = (wt * np.asarray(f, dtype=np.float64)[:, None]).reshape(-1)
    keys, inv = np.unique(nodes.reshape(-1, 3), axis=0, return_inverse=True)
    return keys, np.bincount(inv.ravel(), weights=vals, minlength=len(keys))


def interpolate(node_cells, node_vals, cells, nb):
    """I U at fine cells, U given at node_cells (others 0)."""
    nodes, wt = interp_pairs(cells, nb)
    lut = {tuple(k): v for k, v in zip(np.asarray(node_cells).tolist(), node_vals)}
    vals = np.array([lut.get(tuple(k), 0.0) for k in nodes.reshape(-1, 3).tolist()]).reshape(nodes.shape[:2])
    return (wt * vals).sum(axis=1)


def _block_of(cells, nb):
    return np.floor_divide(np.asarray(cells, dtype=np.int64), nb)


def near_sum(src, f, tgt, dx, nb, D):
    """dx^2 sum over source cells whose block is within D blocks of the target's."""
    src = np.asarray(src, dtype=np.int64)
    tgt = np.asarray(tgt, dtype=np.int64)
    bs, bt = _block_of(src, nb), _block_of(tgt, nb)
    out = np.zeros(len(tgt))
    keys, inv = np.unique(bt, axis=0, return_inverse=True)
    inv = inv.ravel()
    for i, kb in enumerate(keys):
        sel = np.nonzero(inv == i)[0]
        near = np.abs(bs - kb).max(axis=1) <= D
        if near.any():
            out[sel] = direct.direct_sum(src[near], f[near], tgt[sel], dx)
    return out


def far_sum(src, f, tgt, dx, nb, D):
    """The interpolated far field at target cells."""
    nodes, Af = anterpolate(src, f, nb)
    keep = Af != 0.0
    nodes, Af = nodes[keep], Af[keep]
    tnodes = np.unique(interp_pairs(tgt, nb)[0].reshape(-1, 3), axis=0)
    bn, bt = _block_of(nodes, nb // 2), _block_of(tnodes, nb // 2)
    U = np.zeros(len(tnodes))
    keys, inv = np.unique(bt, axis=0, return_inverse=True)
    inv = inv.ravel()
    for i, kb in enumerate(keys):
        sel = np.nonzero(inv == i)[0]
        far = np.abs(bn - kb).max(axis=1) > D
        if far.any():
            # G(2 (i - j)) = the LGF at the even lattice vector between the nodes
            d = (tnodes[sel][:, None, :] - nodes[far][None, :, :]) * 2
            G = lgf_table.G(d.reshape(-1, 3)).reshape(d.shape[:2])
            U[sel] = dx * dx * (G @ Af[far])
    return interpolate(tnodes, U, tgt, nb)


def flgf(src, f, tgt, dx, nb, D):
    """u = u_near + u_far (the two-grid fast-LGF reading)."""
    f = np.asarray(f, dtype=np.float64)
    return near_sum(src, f, tgt, dx, nb, D) + far_sum(src, f, tgt, dx, nb, D)
