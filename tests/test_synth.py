"""Input generators: balance, sizes and determinism."""
import numpy as np
import pytest

from synth.configs import config_heat_gaussian, config_tiny, patch_sizes
from synth.hierarchy import cell_coords_of_octs, is_balanced, random_balanced_hierarchy


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


def test_collapse_config_shape():
    # Jeans-refined hierarchy around the softened sphere: balanced, nested towards the
    # centre, every refined cell dense enough, contrast as asked, fields positive
    from synth.configs import config_collapse
    from synth.hierarchy import cell_coords_of_octs, is_balanced
    p = config_collapse(base_level=3, max_level=7, jeans=1.5, contrast=1e4, field_n=64, shared_dt_levels=2)
    h = p.hierarchy
    assert is_balanced(h)
    assert h.levels == [3, 4, 5, 6, 7]
    assert p.nsub == {4: 1, 5: 2, 6: 2, 7: 2}
    for l in h.levels[1:]:
        parents = np.asarray(h.octs[l], dtype=np.int64)
        rho = p.rho(l - 1, parents)
        crit = 8.0 * np.sqrt(rho) / ((1 << (l - 1)) * 1.5 * np.sqrt(0.75))
        assert np.all(crit > 1.0)
        x = (parents + 0.5) / (1 << (l - 1))
        assert np.max(np.linalg.norm(x - 0.5, axis=1)) < 0.9 / (1 << (l - 4)) + 0.1
    c = cell_coords_of_octs(h.octs[7])
    assert np.all(p.rho(7, c) > 0) and np.all(p.E(7, c) > 0)
    assert np.allclose(p.T(7, c) ** 4, p.E(7, c))
    # centre-to-corner contrast without the 5% perturbation
    from synth.configs import _collapse_rho
    rho0, rc = _collapse_rho(1e4, 64, 1, amp=0.0)
    n = 1 << 20
    centre = np.array([[n // 2, n // 2, n // 2]])
    assert rc == pytest.approx(np.sqrt(3) / 2)
    assert rho0(20, centre)[0] / rho0(20, np.array([[0, 0, 0]]))[0] == pytest.approx(1e4, rel=1e-4)


def test_equilibrium_mesh_has_the_papers_cell_count():
    # 8 coarse cells, four more levels, refined where the profile changes by more than
    # 10 % over a cell or a neighbour: 3 + 5 + 5 + 5 + 10 = 28 cells along x, the count
    # the paper gives for its most resolved adaptive runs (Sect. 4.2); plane-parallel, so
    # every level covers whole y-z planes
    from synth.configs import config_equilibrium
    from synth.hierarchy import is_balanced
    p = config_equilibrium()
    h = p.hierarchy
    assert is_balanced(h) and h.levels == [3, 4, 5, 6, 7]
    leaves_along_x = 0
    for l in h.levels:
        c = cell_coords_of_octs(h.octs[l]).astype(np.int64)
        per_x = np.bincount(c[:, 0], minlength=1 << l)
        xs = np.nonzero(per_x)[0]
        assert np.all(per_x[xs] == (1 << l) ** 2)  # whole planes
        refined = set()
        if l + 1 in h.octs:
            refined = set(np.asarray(h.octs[l + 1])[:, 0].tolist())
        leaves_along_x += len([x for x in xs if x not in refined])
    assert leaves_along_x == 28
