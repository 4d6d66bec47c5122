"""Pins of the stray-pixel filter (Section 3's clean-up step: a pixel none of
whose 4-neighbours shares its label adopts theirs): hand-worked cases,
border pixels, majority and tie order, and invariants on random maps (the
pixels a pass changes are exactly those without a same-label neighbour,
computed here with array shifts; two passes equal one pass applied twice)."""
import numpy as np

import oracle


def test_isolated_pixel_takes_the_surrounding_label():
    lb = np.full((5, 5), 7, np.int32)
    lb[2, 2] = 3
    assert np.all(oracle.stray_filter(lb, 1) == 7)


def test_majority_and_tie_order():
    # up = 1, left = 2, right = 2, down = 3: the majority is 2
    lb = np.array([[9, 1, 9], [2, 0, 2], [9, 3, 9]], np.int32)
    assert oracle.stray_filter(lb, 1)[1, 1] == 2
    # four different labels: the first in the order up, left, right, down
    lb = np.array([[9, 1, 9], [2, 0, 4], [9, 3, 9]], np.int32)
    assert oracle.stray_filter(lb, 1)[1, 1] == 1
    # up = 5, down = 5, left = 6, right = 6: a tie between two pairs, up first
    lb = np.array([[9, 5, 9], [6, 0, 6], [9, 5, 9]], np.int32)
    assert oracle.stray_filter(lb, 1)[1, 1] == 5


def test_border_pixels_use_their_neighbours_inside_the_image():
    lb = np.array([[4, 1], [1, 1]], np.int32)  # the corner has neighbours right, down
    assert oracle.stray_filter(lb, 1)[0, 0] == 1
    lb = np.array([[4, 5, 6]], np.int32)  # a single row: left and right only
    out = oracle.stray_filter(lb, 1)
    assert out.tolist() == [[5, 4, 5]]
    assert oracle.stray_filter(np.array([[3]], np.int32), 2)[0, 0] == 3


def test_pixel_with_a_same_label_neighbour_is_kept_and_strays_change():
    rng = np.random.default_rng(0)
    for _ in range(20):
        lb = rng.integers(0, 3, (13, 17)).astype(np.int32)
        same = np.zeros(lb.shape, bool)
        same[1:, :] |= lb[1:, :] == lb[:-1, :]
        same[:-1, :] |= lb[:-1, :] == lb[1:, :]
        same[:, 1:] |= lb[:, 1:] == lb[:, :-1]
        same[:, :-1] |= lb[:, :-1] == lb[:, 1:]
        out = oracle.stray_filter(lb, 1)
        assert np.array_equal(out[same], lb[same])
        assert np.all(out[~same] != lb[~same])


def test_two_passes_are_one_pass_twice():
    rng = np.random.default_rng(1)
    lb = rng.integers(0, 4, (20, 20)).astype(np.int32)
    assert np.array_equal(oracle.stray_filter(lb, 2),
                          oracle.stray_filter(oracle.stray_filter(lb, 1), 1))
    assert np.array_equal(oracle.stray_filter(lb, 0), lb)
