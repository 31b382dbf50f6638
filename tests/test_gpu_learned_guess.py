"""Learned Newton initial guess: the perceptron's kernels against the FP64 oracle
(oracle/mlp.py), and the guess's effect on the Newton solve at an equal target.

Tolerances follow from FP32 arithmetic (unit roundoff u = 2^-24) against FP64:
  GEMM      elementwise |C - C_ref| <= 4 (K + 2) u (|alpha| |A| |B| + |beta| |C0|), the
            standard inner-product bound gamma_K with a factor for the final scaling;
  network   normwise relative errors of the forward output and each layer's gradient
            stated per check (FP32 sums over up to 5000 rows);
  Adam      one step from the GPU's own gradient: |p - p_ref| <= 2 u |p| + 16 u |d| + 2 e_d,
            d the update (a few FP32 operations on it and the final subtraction) and
            e_d the effect of the FP32 first moment's carried rounding error, which
            a partial cancellation in b1 m + (1 - b1) g can make large relative to m;
  features  one rounding of an FP64 value to FP32: |x - x_ref| <= u |x_ref|.
"""
import numpy as np
import pytest

from oracle import mlp as OM
from paper_1810_04289_amd import workload as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def fsi_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_04289_amd import fsi
    fsi.load_library()
    return fsi


def dev32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def dev64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("M,N,K,ta,tb,alpha,beta,nsplit", [
    (1, 1, 1, False, False, 1.0, 0.0, 1),
    (64, 64, 16, False, False, 1.0, 0.0, 1),
    (70, 130, 33, False, False, 1.0, 0.0, 1),
    (130, 7, 1000, True, False, 1.0, 0.0, 1),      # the weight-gradient shape: A^T B, long K
    (130, 7, 5000, True, False, 1.0, 0.0, 8),      # ... split over K
    (64, 64, 100, False, False, 1.0, 0.5, 3),      # ragged last split, C accumulated
    (20, 30, 40, True, True, 2.0, 0.0, 16),        # more splits asked for than 16-wide K steps
    (300, 18, 128, False, True, 0.5, 0.0, 1),      # the back-propagation shape: A B^T
    (65, 65, 17, True, True, -1.25, 0.75, 1),      # both transposed, C accumulated
    (5, 9, 0, False, False, 1.0, 2.0, 1),          # K = 0: C = beta C
])
def test_gemm_matches_fp64(fsi_mod, M, N, K, ta, tb, alpha, beta, nsplit):
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    C0 = rng.standard_normal((M, N)).astype(np.float32)
    Ad = A.astype(np.float64).T if ta else A.astype(np.float64)
    Bd = B.astype(np.float64).T if tb else B.astype(np.float64)
    ref = alpha * Ad @ Bd + beta * C0.astype(np.float64)
    bound = 4 * (K + 2) * U * (abs(alpha) * np.abs(Ad) @ np.abs(Bd) + abs(beta) * np.abs(C0))
    Cd = dev32(C0)
    fsi_mod.gemm_f32(dev32(A), dev32(B), Cd, alpha=alpha, beta=beta, transA=ta, transB=tb, nsplit=nsplit)
    C = Cd.cpu().numpy().astype(np.float64)
    err = np.abs(C - ref)
    say(f"[gemm {M}x{N}x{K} tA={ta} tB={tb} splits {nsplit}] max err / bound {np.max(err / np.maximum(bound, 1e-300)):.3f}")
    assert np.all(err <= bound + 1e-30)


def random_problem(nin, hidden, nlayers, nout, n, seed):
    rng = np.random.default_rng(seed)
    dims = OM.layer_dims(nin, hidden, nlayers, nout)
    p = np.concatenate([np.concatenate([rng.uniform(-1, 1, a * b) * np.sqrt(3.0 / a), rng.uniform(-0.1, 0.1, b)])
                        for a, b in dims]).astype(np.float32)
    X = rng.standard_normal((n, nin)).astype(np.float32)
    T = rng.standard_normal((n, nout)).astype(np.float32)
    return dims, p, X, T


def layer_blocks(v, dims):
    out, o = [], 0
    for a, b in dims:
        out.append(v[o:o + a * b + b])
        o += a * b + b
    return out


@pytest.mark.parametrize("hidden,nlayers,n", [(48, 3, 5000), (128, 4, 777), (16, 1, 100)])
def test_mlp_forward_and_gradient(fsi_mod, hidden, nlayers, n):
    """Forward output, loss and every layer's gradient against FP64 back-propagation, at
    ragged sizes: hidden widths not a multiple of the 64-wide tile, a ragged last chunk of
    the bias column sums (777 rows in chunks of 4), and the weight gradient split over K
    (5000 rows in 39 splits)."""
    dims, p, X, T = random_problem(18, hidden, nlayers, 7, n, seed=hidden + n)
    net = fsi_mod.MLP(18, hidden, nlayers, 7, nmax=n + 5)
    net.set_params(p)
    Y = net.forward(dev32(X)).cpu().numpy()
    Yr = OM.forward(p, dims, X)[-1]
    ef = np.linalg.norm(Y - Yr) / np.linalg.norm(Yr)
    loss = net.loss_grad(dev32(X), dev32(T))
    lr_, gr = OM.loss_grad(p, dims, X, T)
    _, g = net.get_params()
    el = abs(loss - lr_) / lr_
    eg = [np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(layer_blocks(g, dims), layer_blocks(gr, dims))]
    say(f"[mlp h={hidden} L={nlayers} n={n}] forward {ef:.2e} loss {el:.2e} grad per layer "
        + " ".join(f"{e:.2e}" for e in eg))
    assert ef <= 1e-5
    assert el <= 1e-5
    assert max(eg) <= 1e-4
    net.close()


def test_mlp_adam_steps(fsi_mod):
    """Adam arithmetic per step from the GPU's own gradient, and the 5-step trajectory
    against an FP64 run from the same start."""
    dims, p0, X, T = random_problem(18, 64, 3, 7, 3000, seed=5)
    # the hyperparameters as the library receives them (FP32): 0.999 rounds to 0.99900001,
    # which moves 1 - b2 by 1.3e-5 relative
    f32 = lambda x: float(np.float32(x))
    lr, hp = f32(1e-2), dict(b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8))
    net = fsi_mod.MLP(18, 64, 3, 7, nmax=3000)
    net.set_params(p0)
    Xd, Td = dev32(X), dev32(T)
    po = p0.astype(np.float64)
    m = np.zeros_like(po)
    v = np.zeros_like(po)
    pt, mt, vt = po.copy(), m.copy(), v.copy()
    losses = []
    em = np.zeros_like(po)  # bound on the FP32 first moment's accumulated rounding error
    b1, b2, eps = hp["b1"], hp["b2"], hp["eps"]
    for t in range(1, 6):
        pprev, _ = net.get_params()
        losses.append(net.train_step(Xd, Td, lr=lr, **hp))
        pg, g = net.get_params()
        # per step: the oracle's Adam applied to the GPU's gradient and parameters
        g = g.astype(np.float64)
        em = b1 * em + 2 * U * (b1 * np.abs(m) + (1 - b1) * np.abs(g))
        pref, m, v = OM.adam_step(pprev.astype(np.float64), g, m, v, t, lr=lr, **hp)
        d = np.abs(pprev.astype(np.float64) - pref)
        # m may cancel (b1 m and (1 - b1) g of opposite signs): its error enters through
        # em; v sums positive terms and the update's own operations cost a few u of d
        dm = lr * (em / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        err = np.abs(pg - pref)
        bound = 2 * U * np.abs(pref) + 16 * U * d + 2 * dm + 1e-40
        assert np.all(err <= bound), f"step {t}: max err/bound {np.max(err / bound):.2f}"
        # trajectory: the FP64 network trained from the same start
        _, gt = OM.loss_grad(pt, dims, X, T)
        pt, mt, vt = OM.adam_step(pt, gt, mt, vt, t, lr=lr, **hp)
    pg, _ = net.get_params()
    et = np.linalg.norm(pg - pt) / np.linalg.norm(pt - po)
    say(f"[adam] losses {['%.4f' % x for x in losses]}; 5-step parameter change vs FP64: rel. error {et:.2e}")
    assert losses[-1] < losses[0]
    assert et <= 1e-3
    net.close()


def test_guess_features_target_predict(fsi_mod):
    fsi = fsi_mod
    rng = np.random.default_rng(11)
    V = 1000
    y2, y1, y = (rng.standard_normal(7 * V) * np.tile([30, 30, 30, 1e3, 1e-3, 1e-3, 1e-3], V) for _ in range(3))
    # scales: s, a sigma floor that is active for component 5 only, gains (one switched off)
    sig = np.sqrt(np.mean((y1 - y2).reshape(-1, 7) ** 2, axis=0))
    floor = np.zeros(7)
    floor[5] = 2.0 * sig[5]
    gain = np.array([1.0, 0.5, 1.0, 0.0, 1.0, 1.0, 2.0])
    sc = np.concatenate([rng.uniform(0.5, 2.0, 7), floor, gain]).astype(np.float32)
    tf = np.array([0.3, -0.9, 1.2, 0.1], dtype=np.float32)
    dims, p, _, _ = random_problem(18, 32, 2, 7, 1, seed=2)
    net = fsi.MLP(18, 32, 2, 7, nmax=V)
    net.set_params(p)
    net.set_scales(sc)
    X = net.features(dev64(y1), dev64(y2), tf).cpu().numpy()
    Xr = OM.features(y1, y2, sc, tf)
    # one rounding to FP32, plus sigma's FP64 sum in another order (relative 1e-15)
    assert np.all(np.abs(X - Xr) <= 1.01 * U * np.abs(Xr))
    T = net.target(dev64(y), dev64(y1), dev64(y2)).cpu().numpy()
    Tr = OM.target(y, y1, y2, sc)
    assert np.all(np.abs(T - Tr) <= 1.01 * U * np.abs(Tr) + 1e-12 * np.abs(Tr).max())
    # the extrapolation alone, and corrected by the network output on the same features
    g0 = net.predict(dev64(y1), dev64(y2)).cpu().numpy()
    g0r = OM.guess(y1, y2, None, sc)
    assert np.allclose(g0, g0r, rtol=1e-15, atol=1e-15 * np.abs(g0r).max())
    out = net.forward(dev32(X)).cpu().numpy()
    g1 = net.predict(dev64(y1), dev64(y2), tf).cpu().numpy()
    g1r = OM.guess(y1, y2, out, sc)
    assert np.allclose(g1, g1r, rtol=1e-14, atol=1e-15 * np.abs(g1r).max())
    # the switched-off component is the extrapolation's
    assert np.array_equal(g1.reshape(-1, 7)[:, 3], g0.reshape(-1, 7)[:, 3])
    # the network itself against the oracle on these features
    assert np.linalg.norm(out - OM.forward(p, dims, X)[-1]) <= 1e-5 * np.linalg.norm(OM.forward(p, dims, X)[-1])
    # edge cases: zero rows, too many rows, wrong network shape for the guess
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert net.predict(e, e).numel() == 0
    with pytest.raises(fsi.FsiError):
        net.forward(torch.zeros((V + 1, 18), dtype=torch.float32, device="cuda"))
    other = fsi.MLP(17, 8, 2, 7, nmax=4)
    with pytest.raises(fsi.FsiError):
        other.features(dev64(y1[:28]), dev64(y2[:28]), tf)
    other.close()
    net.close()


def test_learned_guess_on_the_tube(fsi_mod):
    """Straight compliant tube, dt = 2 ms: the network trained on one inflow period of the
    plain solver's steps at amplitude 15 cm/s (the first 100 steps of the start from rest
    left out), then, 100 steps into the next period with the amplitude raised by 20%
    (18 cm/s), every guess solved to the same absolute target.

    What the network gains over the method without it: the velocity error of the guess
    and the initial Newton residual, both against the linear extrapolation (measured:
    velocity error 1.8% vs 6.6% of the step's change, initial residual 0.017 vs 0.071 of
    the previous state's).  The Newton iteration count stays at 2 for every guess: one
    GMRES solve to rtol 1e-3 cannot reach 1e-6 from either start."""
    from paper_1810_04289_amd import guess as G
    r = G.run(case="tube", dt=2e-3, train_steps=400, eval_steps=20, amp_eval=18.0, train_iters=1500, skip=100,
              eval_offset=100, log=say)
    say(f"[learned guess, tube] {r}")
    for name in ("previous", "extrapolation", "learned"):
        assert r[name]["failures"] == 0
        assert r[name]["max_fnorm_over_target"] <= 1.0
    assert r["loss_last"] < 0.1 * r["loss_first"]
    assert r["extrapolation"]["F0_rel"] < 1.0
    # the residual test picks the better start, so the learned guess is never worse
    assert r["learned"]["F0_rel"] <= r["extrapolation"]["F0_rel"]
    # and the trained network is better: velocity error and initial residual
    assert r["rel_err_upd"]["network"][0] < 0.5 * r["rel_err_upd"]["extrapolation"][0]
    assert r["network_picked"] >= 0.9 * r["eval_steps"]
    assert r["learned"]["F0_rel"] < 0.5 * r["extrapolation"]["F0_rel"]
    assert r["learned"]["NI"] <= r["extrapolation"]["NI"]
    # what the step pays for, against the paper's start from the previous state: fewer
    # GMRES iterations at the same Newton target (measured 44.2 against 48.1 per step)
    assert r["learned"]["NI"] <= r["previous"]["NI"]
    assert r["learned"]["LI_per_step"] < r["previous"]["LI_per_step"]
