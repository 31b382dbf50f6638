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


def _fingerprint(m):
    import hashlib
    h = hashlib.sha256()
    for a in (m.X, m.tets, m.tet_domain, m.bfaces, m.bface_tag):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def test_tree_meshes_are_reproducible_and_valid():
    # The generator evaluates each branch only near its own bounding box; these meshes are
    # the ones it produced when every branch was evaluated on every lattice tet
    for depth, h, V, E, fp in ((1, 0.08, 26451, 134330, "b47a29227ec0b42b"),
                               (2, 0.06, 86285, 445860, "a1f9d1859787ba07")):
        m = W.tree_mesh(depth=depth, h=h)
        assert (m.nverts, m.ntets) == (V, E)
        assert _fingerprint(m) == fp
        a, b, c = (m.X[m.tets[:, k]] - m.X[m.tets[:, 0]] for k in (1, 2, 3))
        assert np.all(np.einsum("ij,ij->i", a, np.cross(b, c)) > 0)
        # one inlet cap and 2^depth outlet caps of fluid faces
        assert np.sum(m.bface_tag == W.TAG_FLUID_INLET) > 0
        assert m.info["noutlets"] == 2 ** depth

