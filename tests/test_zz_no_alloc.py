"""fsi_pc_apply_noalloc, the Schwarz application for callers that cannot allocate, against
fsi_pc_apply through the C ABI.

Both run the same sweep kernels in the same order; only the location of the sweeps' work
values and error flags differs (the library's static per-GPU scratch instead of the
solver's buffers), so the results must be identical.  Two calls in a row, the second on a
smaller input (the scratch keeps the first call's values), then FP32 sweeps, then a solver
whose sweeps need more scratch than there is (rejected with ERR_ARG).
"""
import numpy as np
import pytest

from paper_1810_04289_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PH = W.physics_config1()


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def fsi_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_04289_amd import fsi
    fsi.load_library()
    return fsi


def factored(fsi, mesh, y0, opts, seed):
    s = fsi.Solver(mesh, PH, opts)
    g = W.dirichlet_values(mesh, 30.0)
    s.set_step(1e-3, 1e-3, s.vec(y0), s.vec(g))
    y = s.vec(W.perturbed_state(mesh, y0, seed=seed))
    s.impose_dirichlet(y)
    s.jacobian(y)
    s.pc_setup()
    return s


def compare(s, seed):
    v = s.vec(np.random.default_rng(seed).standard_normal(s.n))
    z0 = s.vec()
    s.pc_apply(v, z0)
    z1 = torch.full_like(z0, float("nan"))
    s.pc_apply_noalloc(v, z1)
    torch.cuda.synchronize()
    return z0, z1


def test_noalloc_pc_apply_equals_pc_apply(fsi_mod):
    tree = W.tree_mesh(depth=1, h=W.TREE_H[1])
    tube = W.tube_mesh()
    cases = [
        ("depth-1 tree, 33 subdomains, ILU(3), FP64", tree, np.zeros(tree.n), dict(nsub=33, overlap=1, ilu_level=3)),
        ("tube, 4 subdomains, ILU(2), FP64 (smaller)", tube,
         W.poiseuille_state(tube, 30.0, PH["mu_f"], 5.0), dict(nsub=4, overlap=1, ilu_level=2)),
        ("tube, 4 subdomains, ILU(2), FP32 sweeps", tube,
         W.poiseuille_state(tube, 30.0, PH["mu_f"], 5.0), dict(nsub=4, overlap=1, ilu_level=2, precision=1)),
    ]
    for k, (name, mesh, y0, opts) in enumerate(cases):
        say(f"[noalloc] {name}: V={mesh.nverts}")
        s = factored(fsi_mod, mesh, y0, opts, seed=3 + k)
        z0, z1 = compare(s, seed=10 + k)
        say(f"  identical {torch.equal(z0, z1)}, |z| {float(torch.linalg.vector_norm(z0)):.3e}")
        assert bool(torch.isfinite(z0).all())
        assert torch.equal(z0, z1)
        # a second call on the same solver (scratch flags cleared again, values rewritten)
        z2 = torch.full_like(z0, float("nan"))
        s.pc_apply_noalloc(s.vec(np.random.default_rng(10 + k).standard_normal(s.n)), z2)
        assert torch.equal(z0, z2)
        s.close()


def test_noalloc_pc_apply_rejects_oversized_solvers(fsi_mod):
    # 300 subdomains whose overlap covers the whole tube: 300 x 2025 = 607,500 local rows,
    # 34 MB of FP64 sweep values, above the 32 MiB scratch
    tube = W.tube_mesh()
    y0 = W.poiseuille_state(tube, 30.0, PH["mu_f"], 5.0)
    s = factored(fsi_mod, tube, y0, dict(nsub=300, overlap=40, ilu_level=0), seed=5)
    v = s.vec(np.random.default_rng(1).standard_normal(s.n))
    z = s.vec()
    rc = s.pc_apply_noalloc(v, z, check=False)
    msg = s.last_error()
    say(f"[noalloc] oversized: rc {rc}, {msg}")
    assert rc == 1 and "scratch" in msg
    s.pc_apply(v, z)       # the solver's own buffers still serve it
    assert bool(torch.isfinite(z).all())
    s.close()
