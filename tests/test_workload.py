"""Seeded input generators: properties the synthetic workloads promise."""
import numpy as np

from paper_1810_04289_amd import workload as W


def test_uneven_partition_follows_lognormal_targets():
    # every subdomain gets its share of the lognormal target sizes, up to one vertex of
    # rounding per bisection level, and the result is reproducible from the seed
    m = W.tree_mesh(depth=1, h=W.TREE_H[1])
    nsub, sigma = 9, 0.5
    p = W.uneven_partition(m, nsub, sigma=sigma, seed=4)
    w = np.random.default_rng(4).lognormal(0.0, sigma, nsub)
    sizes = np.bincount(p, minlength=nsub)
    expect = m.nverts * w / w.sum()
    assert sizes.sum() == m.nverts and sizes.min() > 0
    assert np.all(np.abs(sizes - expect) <= np.ceil(np.log2(nsub)) + 1)
    assert np.array_equal(p, W.uneven_partition(m, nsub, sigma=sigma, seed=4))
    # compact pieces: each subdomain's bounding box is a small part of the tree's
    ext = m.X.max(0) - m.X.min(0)
    for s in range(nsub):
        P = m.X[p == s]
        assert np.prod(P.max(0) - P.min(0)) < 0.5 * np.prod(ext)
