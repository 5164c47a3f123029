"""Test-side statement of the activation rules of "Updating active cells"
(update after every step, no shutdown), written from the paper's text and
used to check the CPU TCM oracle step by step.

Given the active cells A of step n, phi^{n+1} computed on them and phi^n:

* keep (item 3, with the hysteresis level): a cell of A stays when any
  |phi^{n+1}| or |phi^n| in it is strictly above ``retire``;
* trigger (item 4, Figure 3a): for a cell of A, every face whose
  |phi^{n+1}| is strictly above ``trigger`` activates the in-domain cell
  across that face;
* source insertion: a cell whose source still has samples for step n+1 is
  active.

Nothing here calls into the oracle's bookkeeping: the rules are evaluated on
plain arrays with NumPy.
"""
from __future__ import annotations

import numpy as np


def cells_shape(shape_zyx, B):
    nz, ny, nx = shape_zyx
    return (-(-nz // B), -(-ny // B), -(-nx // B))


def _blocks(a, B):
    """|a| padded with zeros to whole cells, as (mz, B, my, B, mx, B)."""
    nz, ny, nx = a.shape
    mz, my, mx = cells_shape(a.shape, B)
    p = np.zeros((mz * B, my * B, mx * B), a.dtype)
    p[:nz, :ny, :nx] = np.abs(a)
    return p.reshape(mz, B, my, B, mx, B)


def cell_max(a, B):
    return _blocks(a, B).max(axis=(1, 3, 5))


def face_max(a, B):
    """(6, mz, my, mx): max |a| on face f of each cell (0:-x 1:+x 2:-y 3:+y
    4:-z 5:+z); nodes beyond the domain count as zero."""
    r = _blocks(a, B)
    return np.stack([r[:, :, :, :, :, 0].max(axis=(1, 3)), r[:, :, :, :, :, B - 1].max(axis=(1, 3)),
                     r[:, :, :, 0, :, :].max(axis=(1, 4)), r[:, :, :, B - 1, :, :].max(axis=(1, 4)),
                     r[:, 0].max(axis=(2, 4)), r[:, B - 1].max(axis=(2, 4))])


def node_mask(cells, shape_zyx, B):
    """Cell flags (mz, my, mx) expanded to the nodes of the grid."""
    nz, ny, nx = shape_zyx
    m = np.repeat(np.repeat(np.repeat(cells, B, axis=0), B, axis=1), B, axis=2)
    return m[:nz, :ny, :nx]


def next_active(new, cur, active, trigger, retire, pinned, B):
    """Active cells after the update of step n.

    new: phi^{n+1} on the cells of ``active`` (zero elsewhere); cur: phi^n;
    active: bool (mz, my, mx); pinned: cell indices (cz, cy, cx) whose source
    still inserts at step n+1.  Comparisons are in the fields' precision.
    """
    t = new.dtype.type(trigger)
    r = new.dtype.type(retire)
    nxt = active & ((cell_max(new, B) > r) | (cell_max(cur, B) > r))
    f = (face_max(new, B) > t) & active[None]
    nxt[:, :, :-1] |= f[0][:, :, 1:]
    nxt[:, :, 1:] |= f[1][:, :, :-1]
    nxt[:, :-1, :] |= f[2][:, 1:, :]
    nxt[:, 1:, :] |= f[3][:, :-1, :]
    nxt[:-1] |= f[4][1:]
    nxt[1:] |= f[5][:-1]
    for cz, cy, cx in pinned:
        nxt[cz, cy, cx] = True
    return nxt
