"""Input generators: balance, sizes and determinism."""
import numpy as np

from synth.configs import config_heat_gaussian, config_tiny, patch_sizes
from synth.hierarchy import is_balanced, random_balanced_hierarchy


def test_heat_config_shape():
    p = config_heat_gaussian()
    assert {l: len(o) for l, o in p.hierarchy.octs.items()} == {4: 512, 5: 512}
    assert is_balanced(p.hierarchy)
    assert p.dt_coarse == 4.0 / 256.0


def test_random_hierarchies_balanced_and_seeded():
    for seed in range(6):
        a = random_balanced_hierarchy(seed, 2, 5, p_refine=0.5)
        b = random_balanced_hierarchy(seed, 2, 5, p_refine=0.5)
        assert is_balanced(a)
        assert a.octs.keys() == b.octs.keys()
        for l in a.octs:
            assert np.array_equal(a.octs[l], b.octs[l])


def test_unbalanced_detected():
    h = random_balanced_hierarchy(0, 2, 3, p_refine=0.5)
    h.octs[4] = np.array([[0, 0, 0]], dtype=np.int32)  # parent cell may not exist at level 3
    bad = dict(h.octs)
    assert (not is_balanced(h)) or len(bad[3]) and np.any(np.all(bad[3] == 0, axis=1))


def test_patch_sizes_range():
    s = patch_sizes(4000, 512)
    assert s.min() >= 8 and s.max() <= 128 and np.all(s % 2 == 0)
    assert 0.9e8 < np.sum(s.astype(np.int64) ** 3) < 2.0e8


def test_tiny_fields_positive():
    p = config_tiny(3)
    for l in p.hierarchy.levels:
        from synth.hierarchy import cell_coords_of_octs
        c = cell_coords_of_octs(p.hierarchy.octs[l])
        assert np.all(p.rho(l, c) > 0) and np.all(p.E(l, c) > 0)
