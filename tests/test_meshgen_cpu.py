"""Host checks of the seeded input generators that both sides draw from."""
import numpy as np

from meshgen import gen as mg


def test_splitmix64_published_vector():
    # the first outputs of SplitMix64 from state 1234567, as published with
    # the generator's reference implementation
    got = [int(x) for x in mg.splitmix64(1234567, np.arange(2))]
    assert got == [6457827717110365317, 3203168211198807973]


def test_tiled_grid_id_is_a_bijection_with_tiles():
    for g in (1, 2, 31, 32, 33, 70, 129):
        j, i = np.divmod(np.arange(g * g), g)
        ids = mg.tiled_grid_id(i, j, g)
        assert np.array_equal(np.sort(ids), np.arange(g * g))
        # a full 32 x 32 tile holds 1024 consecutive ids
        if g >= 64:
            t = ids[(i < 32) & (j >= 32) & (j < 64)]
            assert t.min() == 32 * g and t.max() == 32 * g + 1023


def test_counter_grid_points_stay_in_their_cells():
    g, jit = 50, 0.45
    p = mg.counter_grid_points(g, jit, 3)
    j, i = np.divmod(np.arange(g * g), g)
    assert np.all(np.abs(p[:, 0] * g - (i + 0.5)) <= jit + 1e-12)
    assert np.all(np.abs(p[:, 1] * g - (j + 0.5)) <= jit + 1e-12)
    # jitter 0 is the exact cell centres
    q = mg.counter_grid_points(g, 0.0, 3)
    assert np.array_equal(q[:, 0], (i + 0.5) / g)
