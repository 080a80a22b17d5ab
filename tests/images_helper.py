"""Which listed pairs a neighborhood staged at periodic images near its block
would give a wrong image (a test helper, numpy only)."""

import numpy as np

import oracle


def wrong_staged_images(x0, x, L, counts, nbr, edge, rl=2.8):
    """Listed pairs whose partner, staged at its image nearest to the centre
    of the atom's block (blocks of `edge` cells, binned at x0), is not the
    image nearest to the atom at positions x: a difference beyond L/2 along
    some axis."""
    nc = oracle.cells_per_axis(L, rl)
    a = L / nc
    cell = np.clip(np.floor(np.mod(x0, L) / a).astype(int), 0, nc - 1)
    c0 = cell // edge * edge
    centre = (c0 + 0.5 * np.minimum(edge, nc - c0)) * a

    def near(y, c):  # the image of y nearest to c
        d = y - c
        return y - L * (d > L / 2) + L * (d < -L / 2)

    wrong = 0
    for i in range(x.shape[0]):
        js = nbr[i, : counts[i]]
        d = near(x[i], centre[i]) - near(x[js], centre[i])
        wrong += int((np.abs(d) > L / 2).any(axis=1).sum())
    return wrong
