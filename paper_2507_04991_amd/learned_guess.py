"""Learned initial guess for the relaxation solve.

A small network (8 -> 32 -> 32 -> 1, tanh) predicts the increment
gamma*_n - gamma*_{n-1} of the root of a case's relaxation equation from: the
last two increments, gamma*_{n-1} - 1, the step size and the entropy-production
terms of this step's stages with b_i != 0 that come before the last stage
(divided by the sum of their magnitudes, zero-padded to four).  gamma*_n is the
root located by one Newton step from the accepted point of step n (whose
evaluation gave r and r'), which the library keeps as the case's gamma history;
the accepted points themselves scatter inside the acceptance band |r| <= tol_r.  It is trained on (features,
increment) pairs logged from the method's own solves, with the library's HIP
forward / gradient / Adam kernels; the step evaluates it before the last stage
(whose epilogue makes the first residual evaluation at the predicted point)
once a case has taken three steps.  Newton and bisection still decide the
accepted gamma, so the guess only changes how many evaluations a step needs.

The feature definition here matches the one evaluated on the device.
"""
from __future__ import annotations

import os

import numpy as np

from . import perrk as P

NFEAT = 8
MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models")
DEFAULT_MODEL = os.path.join(MODEL_DIR, "guess_vortex_ensemble_p3.npz")


def pre_last_count(tab):
    """Stages with b_i != 0 before the last stage (their entropy production is known
    when the guess is made)."""
    b = np.asarray(tab["b"])
    return int(np.count_nonzero(b[:-1]))


def features(ghist, dt, e, nb_pre):
    """ghist: [3] previous gamma - 1 (most recent first); e: entropy production of the
    b_i != 0 stages in stage order, of which the first nb_pre come before the last stage."""
    x = np.zeros(NFEAT)
    x[0] = ghist[0] - ghist[1]
    x[1] = ghist[1] - ghist[2]
    x[2] = ghist[0]
    x[3] = dt
    s = float(np.sum(np.abs(e[:nb_pre])))
    m = min(nb_pre, 4)
    if s > 0.0:
        x[4:4 + m] = np.asarray(e[:m]) / s
    return x


def collect(stepper, u, dt, steps, nb_pre):
    """Advance `steps` synchronous steps, logging one (features, gamma*_n - gamma*_{n-1})
    pair per case and step once the case has three earlier roots (the library's
    gamma history, read after every step).  Steps whose solve fell back or was
    trivial are skipped.  Returns X, Y, the passes of the logged steps and the
    previous root - 1 of each logged pair."""
    n = stepper.n_cases
    dt = np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,))
    hist = stepper.relaxation_state().gamma_hist.copy()
    X, Y, passes, prev = [], [], [], []
    for step in range(steps):
        infos = stepper.step(u, dt)
        new = stepper.relaxation_state().gamma_hist
        for c, inf in enumerate(infos):
            if inf["flags"] == 0 and step >= 3:
                X.append(features(hist[c], dt[c], np.asarray(inf["e"]), nb_pre))
                Y.append(new[c, 0] - hist[c, 0])
                passes.append(inf["passes"])
                prev.append(hist[c, 0])
        hist = new.copy()
    return np.array(X), np.array(Y), np.array(passes), np.array(prev)


def normalisation(X, Y):
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    scale = np.where(std > 0, 1.0 / np.where(std > 0, std, 1.0), 0.0)
    ymean, ystd = float(Y.mean()), float(Y.std() if Y.std() > 0 else 1.0)
    return mean.astype(np.float32), scale.astype(np.float32), ymean, ystd


def init_weights(seed=0):
    rng = np.random.default_rng(seed)
    w = np.zeros(P.MLP_NW, dtype=np.float32)
    w[0:256] = rng.normal(0, np.sqrt(1.0 / 8), 256)
    w[288:1312] = rng.normal(0, np.sqrt(1.0 / 32), 1024)
    w[1344:1376] = rng.normal(0, np.sqrt(1.0 / 32), 32)
    return w


def train(X, Y, epochs=3000, lr=3e-3, seed=0, log_every=0):
    """Full-batch Adam on the normalised data with the HIP kernels.
    Returns (weights[1379] float32 incl. output scale/shift, mean[8], scale[8], loss history)."""
    import torch

    mean, scale, ymean, ystd = normalisation(X, Y)
    Xn = ((X - mean) * scale).astype(np.float32)
    Yn = ((Y - ymean) / ystd).astype(np.float32)
    dev = "cuda"
    x = torch.tensor(Xn, device=dev).contiguous()
    t = torch.tensor(Yn, device=dev).contiguous()
    w = torch.tensor(init_weights(seed), device=dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    work = torch.empty(P.lib().perrk_mlp_workspace_bytes(x.shape[0]), dtype=torch.uint8, device=dev)
    hist = []
    for k in range(1, epochs + 1):
        loss, g = P.mlp_loss_grad(w, x, t, work)
        P.mlp_adam(w, g, m, v, k, lr=lr)
        if log_every and (k % log_every == 0 or k == 1):
            hist.append((k, float(loss.item())))
    loss, _ = P.mlp_loss_grad(w, x, t, work)
    hist.append((epochs, float(loss.item())))
    full = np.concatenate([w.cpu().numpy(), np.array([ystd, ymean], dtype=np.float32)])
    return full, mean, scale, hist


def predict(model, X):
    """Host-side helper: gamma - 1 predicted for feature rows X (runs the HIP forward kernel)."""
    import torch

    w, mean, scale = model
    xn = torch.tensor(((X - mean) * scale).astype(np.float32), device="cuda").contiguous()
    y = P.mlp_forward(torch.tensor(w[:P.MLP_NW], device="cuda"), xn).cpu().numpy().astype(np.float64)
    return y * float(w[P.MLP_NW]) + float(w[P.MLP_NW + 1])


def save(path, model, meta=None):
    w, mean, scale = model
    np.savez(path, weights=w, mean=mean, scale=scale, **({} if meta is None else meta))


def load(path):
    d = np.load(path, allow_pickle=False)
    return d["weights"].astype(np.float32), d["mean"].astype(np.float32), d["scale"].astype(np.float32)


def evaluate(problem, model, steps, precision=P.MIXED):
    """Mean residual passes per step with the previous-gamma guess and with the
    learned guess on the same problem (synchronous steps, fresh contexts)."""
    import torch

    out = {}
    for name, guess in (("prev", P.GUESS_PREV), ("learned", P.GUESS_MLP)):
        d = P.Descriptors(problem["faces"], problem["lev"], problem["tab"], precision=precision)
        st = P.Stepper(d, P.default_options(guess=guess))
        if guess == P.GUESS_MLP:
            st.set_guess_model(*model)
        u = torch.tensor(problem["U0"], device="cuda").contiguous()
        passes, rmax, flags = [], 0.0, 0
        for _ in range(steps):
            infos = st.step(u, problem["dt"])
            passes += [i["passes"] for i in infos]
            rmax = max(rmax, max(abs(i["r"]) for i in infos))
            flags |= int(np.bitwise_or.reduce([i["flags"] for i in infos]))
        out[name] = dict(passes_mean=float(np.mean(passes)), r_max=rmax, flags=flags)
        st.close()
    return out


def main(argv=None):
    """Log training pairs on an ensemble with training seeds, train the network on the
    GPU and write the model; evaluate on a held-out seed."""
    import argparse
    import json

    import torch

    from . import problems

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--train-seed", type=int, default=1000)
    ap.add_argument("--eval-seed", type=int, default=7)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--cases", type=int, default=256)
    ap.add_argument("--eval-steps", type=int, default=60)
    ap.add_argument("--save-data", default=None, help="also write the logged pairs (npz)")
    args = ap.parse_args(argv)
    P.lib()
    prob = problems.ensemble(args.train_seed, args.cases)
    d = P.Descriptors(prob["faces"], prob["lev"], prob["tab"], precision=P.MIXED)
    st = P.Stepper(d, P.default_options())
    u = torch.tensor(prob["U0"], device="cuda").contiguous()
    X, Y, passes, prev = collect(st, u, prob["dt"], args.steps, nb_pre=pre_last_count(prob["tab"]))
    st.close()
    if args.save_data:
        np.savez(args.save_data, X=X, Y=Y, passes=passes, prev=prev)
    print(f"# collected {len(Y)} pairs, increment in [{Y.min():.3e}, {Y.max():.3e}], passes {passes.mean():.3f}",
          flush=True)
    model_w, mean, scale, hist = train(X, Y, epochs=args.epochs, log_every=500)
    print("# loss", hist, flush=True)
    model = (model_w, mean, scale)
    pred = predict(model, X)
    res = dict(pairs=int(len(Y)), train_rmse=float(np.sqrt(np.mean((pred - Y) ** 2))),
               prev_rmse=float(np.sqrt(np.mean(Y ** 2))),
               linear_extrapolation_rmse=float(np.sqrt(np.mean((X[:, 0] - Y) ** 2))), y_std=float(Y.std()),
               loss=hist)
    evalp = problems.ensemble(args.eval_seed, args.cases)
    res["heldout"] = evaluate(evalp, model, args.eval_steps)
    save(args.out, model, dict(train_seed=np.array(args.train_seed), steps=np.array(args.steps),
                               cases=np.array(args.cases), epochs=np.array(args.epochs)))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
