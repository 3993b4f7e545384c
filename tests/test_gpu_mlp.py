"""HIP kernels of the learned-guess network against the FP64 reference."""
import numpy as np
import pytest

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_04991_amd import perrk
    perrk.lib()
    return perrk


def data(n, seed):
    rng = np.random.default_rng(seed)
    w = (rng.normal(scale=0.3, size=M.NPARAM)).astype(np.float32)
    X = rng.normal(size=(n, 8)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    return w, X, t


def dev(a):
    return torch.tensor(a, device="cuda").contiguous()


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4099])
def test_forward_and_gradient_match_fp64_reference(P, n):
    w, X, t = data(n, n)
    y = P.mlp_forward(dev(w), dev(X)).cpu().numpy()
    yref = M.forward(w.astype(np.float64), X.astype(np.float64))
    assert np.abs(y - yref).max() <= 2e-6 * (1 + np.abs(yref).max())
    loss, g = P.mlp_loss_grad(dev(w), dev(X), dev(t))
    lref, gref = M.loss_grad(w.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert abs(loss.item() - lref) <= 1e-5 * (1 + lref)
    assert np.abs(g.cpu().numpy() - gref).max() <= 2e-5 * (1 + np.abs(gref).max())


def test_gradient_is_bitwise_reproducible(P):
    w, X, t = data(3000, 7)
    g1 = P.mlp_loss_grad(dev(w), dev(X), dev(t))[1]
    g2 = P.mlp_loss_grad(dev(w), dev(X), dev(t))[1]
    assert torch.equal(g1, g2)


def test_adam_step_matches_reference(P):
    rng = np.random.default_rng(3)
    w = rng.normal(size=M.NPARAM).astype(np.float32)
    g = rng.normal(size=M.NPARAM).astype(np.float32)
    m = rng.normal(size=M.NPARAM).astype(np.float32) * 0.1
    v = np.abs(rng.normal(size=M.NPARAM)).astype(np.float32) * 0.1
    wd, md, vd = dev(w), dev(m), dev(v)
    P.mlp_adam(wd, dev(g), md, vd, 5, lr=1e-2)
    b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-2
    m1 = b1 * m.astype(np.float64) + (1 - b1) * g
    v1 = b2 * v.astype(np.float64) + (1 - b2) * g.astype(np.float64) ** 2
    w1 = w - lr * (m1 / (1 - b1 ** 5)) / (np.sqrt(v1 / (1 - b2 ** 5)) + eps)
    assert np.abs(md.cpu().numpy() - m1).max() < 1e-6
    assert np.abs(vd.cpu().numpy() - v1).max() < 1e-6
    assert np.abs(wd.cpu().numpy() - w1).max() < 1e-5


def test_training_fits_a_smooth_target(P):
    from paper_2507_04991_amd import learned_guess as L
    rng = np.random.default_rng(4)
    X = rng.normal(size=(4000, 8))
    Y = 1e-6 * (0.5 * X[:, 0] - 0.3 * X[:, 1] + 0.2 * np.tanh(X[:, 2]))
    model, mean, scale, hist = L.train(X, Y, epochs=400, lr=3e-3)
    pred = L.predict((model, mean, scale), X)
    assert np.sqrt(np.mean((pred - Y) ** 2)) < 0.05 * np.std(Y)


def test_step_uses_learned_increment(P):
    """With every first evaluation accepted (tol_r huge), the accepted gamma is the
    first evaluation point: gamma_prev for the first three steps of a case, then the
    previous root (the case's gamma history, one Newton step from the previous
    accepted point) plus the network's increment for the features of that step."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from helpers import problem_2d
    from paper_2507_04991_amd import learned_guess as L

    f, U0, tab, dt, lev = problem_2d(nx=8, ny=6, order=3, E=(4, 6, 8, 12))
    rng = np.random.default_rng(11)
    w = (rng.normal(scale=0.4, size=M.NPARAM)).astype(np.float32)
    mean = rng.normal(scale=0.1, size=8).astype(np.float32)
    scale = np.abs(rng.normal(size=8)).astype(np.float32) + 0.5
    scale[:3] = 1.0e5  # increments and gamma - 1 are small
    full = np.concatenate([w, np.array([1.0e-4, 2.0e-5], dtype=np.float32)])
    d = P.Descriptors([f], [lev], tab)
    st = P.Stepper(d, P.default_options(guess=P.GUESS_MLP, tol_r=1.0e30))
    st.set_guess_model(full, mean, scale)
    u = dev(U0)
    nb_pre = L.pre_last_count(tab)
    for step in range(6):
        rs = st.relaxation_state()
        hist, gamma_prev = rs.gamma_hist[0].copy(), rs.gamma_prev[0]
        inf = st.step(u, np.array([dt]))[0]
        expect = gamma_prev
        if step >= 3:
            x = L.features(hist, dt, np.asarray(inf["e"]), nb_pre)
            xn = ((x - mean.astype(np.float64)) * scale.astype(np.float64)).astype(np.float32)
            y = M.forward(w.astype(np.float64), xn[None, :].astype(np.float64))[0]
            expect = (1.0 + hist[0]) + (y * float(full[-2]) + float(full[-1]))
            assert abs(expect - gamma_prev) > 1e-6  # the guess moved the point
        assert inf["passes"] == 1
        assert abs(inf["gamma"] - expect) <= 1e-9, (step, inf["gamma"], expect)
        # the history holds the root one Newton step from the accepted point
        after = st.relaxation_state()
        assert abs(after.gamma_prev[0] - inf["gamma"]) == 0.0
        assert abs((1.0 + after.gamma_hist[0, 0]) - inf["gamma"]) <= 1e-6
    st.close()
