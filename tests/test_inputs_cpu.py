"""Host-side checks of the seeded input generators."""
import numpy as np

from paper_2605_01774_amd import inputs as I


def test_porous_material_table_expands_to_the_field():
    """The porous workload's material table indexed by its per-node material gives exactly
    its per-node tensor field (the two tensor input forms describe the same medium)."""
    prob = I.porous_spheres(n=24, steps=1)
    tab, ph = prob.meta["d6_table"], prob.meta["phase"]
    assert ph.dtype == np.uint8 and tab.shape == (2, 6)
    assert np.array_equal(np.moveaxis(tab[ph.astype(np.int64)], -1, 0), prob.d6)
    assert 0.5 < prob.meta["solid_fraction"] < 0.7
