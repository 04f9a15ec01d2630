"""Oracle of the cell binning that precedes pairing (Sec. 3.1: the particles
of a species are grouped by collision cell before pairs are formed) -- TEST
INFRASTRUCTURE ONLY, like the rest of this package.

Definition: given each particle's cell id, the cell-sorted order is the
stable sort of the particles by cell id (particles of one cell keep their
input order), and the CSR offsets give each cell's first position.  Ids
outside [0, n_cells) belong to no cell: such particles are dropped and
counted.  A library sort (numpy's stable merge sort) serves as the sorting
step; ``bin_particles_loop`` restates the definition with plain loops for
small inputs.
"""
import numpy as np


def bin_order(cell, n_cells):
    """(order, off, n_invalid): order[k] is the input index of the k-th
    particle in cell order (valid particles only), off[c] the first position
    of cell c (off[n_cells] = number of valid particles)."""
    cell = np.asarray(cell, dtype=np.int64)
    valid = (cell >= 0) & (cell < n_cells)
    idx = np.nonzero(valid)[0]
    order = idx[np.argsort(cell[idx], kind="stable")]
    counts = np.bincount(cell[idx], minlength=n_cells) if n_cells > 0 else np.zeros(0, np.int64)
    off = np.zeros(n_cells + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return order, off, int(cell.size - idx.size)


def bin_particles(species, cell, n_cells):
    """Apply bin_order to a species dict {x, y, z, w}: returns (sorted
    species with the valid particles only, off, n_invalid)."""
    order, off, n_invalid = bin_order(cell, n_cells)
    out = {k: np.asarray(species[k])[order] for k in "xyzw"}
    return out, off, n_invalid


def bin_particles_loop(cell, n_cells):
    """The same order by the definition, written out: for each cell in
    increasing order, the particles whose id is that cell, in input order."""
    order = []
    off = [0]
    for c in range(n_cells):
        for i, ci in enumerate(cell):
            if ci == c:
                order.append(i)
        off.append(len(order))
    n_invalid = sum(1 for ci in cell if not (0 <= ci < n_cells))
    return np.array(order, dtype=np.int64), np.array(off, dtype=np.int64), n_invalid
