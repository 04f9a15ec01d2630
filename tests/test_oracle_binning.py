"""Pins of the binning oracle (cell-sorted order and CSR offsets) against
the definition written out with loops, against invariants that hold at any
size, and against hand-worked examples."""
import numpy as np

from oracle import binning


def test_hand_worked_example():
    # cells of six particles; cell 1 is empty; id 5 is outside [0, 4)
    cell = [2, 0, 3, 0, 5, 2]
    order, off, n_inv = binning.bin_order(cell, 4)
    assert order.tolist() == [1, 3, 0, 5, 2]
    assert off.tolist() == [0, 2, 2, 4, 5]
    assert n_inv == 1


def test_matches_loop_definition_on_small_inputs():
    rng = np.random.default_rng(3)
    for n, n_cells in [(0, 1), (1, 1), (7, 3), (50, 1), (64, 9), (200, 17), (300, 300)]:
        cell = rng.integers(-2, n_cells + 2, size=n)
        a = binning.bin_order(cell, n_cells)
        b = binning.bin_particles_loop(cell.tolist(), n_cells)
        assert np.array_equal(a[0], b[0]), (n, n_cells)
        assert np.array_equal(a[1], b[1]), (n, n_cells)
        assert a[2] == b[2]


def test_invariants_at_size():
    rng = np.random.default_rng(5)
    n, n_cells = 200_000, 70_000
    cell = rng.integers(0, n_cells, size=n)
    cell[::97] = -1  # some invalid ids
    order, off, n_inv = binning.bin_order(cell, n_cells)
    valid = cell >= 0
    assert n_inv == int((~valid).sum())
    assert off[0] == 0 and off[-1] == order.size == int(valid.sum())
    assert np.all(np.diff(off) >= 0)
    # every valid particle appears once
    assert np.array_equal(np.sort(order), np.nonzero(valid)[0])
    # sorted by cell, stable inside a cell, and each cell's range holds its particles
    c_sorted = cell[order]
    assert np.all(np.diff(c_sorted) >= 0)
    same = np.diff(c_sorted) == 0
    assert np.all(np.diff(order)[same] > 0)
    for c in rng.integers(0, n_cells, size=50):
        assert np.all(c_sorted[off[c]:off[c + 1]] == c)
        assert off[c + 1] - off[c] == int((cell == c).sum())


def test_species_values_follow_the_order():
    rng = np.random.default_rng(9)
    n, n_cells = 1000, 13
    sp = {k: rng.standard_normal(n).astype(np.float32) for k in "xyzw"}
    cell = rng.integers(0, n_cells, size=n)
    out, off, n_inv = binning.bin_particles(sp, cell, n_cells)
    order = np.argsort(cell, kind="stable")
    for k in "xyzw":
        assert np.array_equal(out[k], sp[k][order])
    assert n_inv == 0 and off[-1] == n
