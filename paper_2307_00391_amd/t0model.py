"""Learned choice of the clock time T0.

The QPE stage resolves the eigenphases lambda_j T0 / 2 pi on a 2^n_c-point
grid, so the solution fidelity of HHL depends strongly on T0 (the T Q phase
diagrams of Fig. 3c; the paper's optimiser picks T0 from kappa, Sec. 3.2 and
Fig. 4b).  Here a 5 -> 64 -> 64 -> 1 perceptron predicts

    y = log(T0* lambda_max / 2 pi)

from the cheap spectrum features [log lambda_min, log lambda_max, log kappa,
n_c, n_s] (lambda from GPU Lanczos).  Labels T0* come from the simulator's
own batched 16-point sweeps (sv_batch_*): the grid factor of largest
fidelity, refined by a parabola through its neighbours in log T0.  Training
is full-batch Adam on the library's MLP kernels; the feature and label
standardisation used in training is folded into the first and last layers
afterwards, so prediction takes raw features.

The learned path solves the predicted T0 and four more candidates
(candidate_factors) in one batched graph and keeps the best, against the
16 solves of the plain sweep.

Everything numeric runs in the library (sweeps, Lanczos, forward, backward,
Adam); this module only arranges batches and standardises inputs.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as B
from . import inputs

N_FEATURES = B.SV_MLP_IN
GRID = 16


def grid_factors(count: int = GRID) -> np.ndarray:
    """T0 = factor * 2 pi / lambda_max; factors 2^(-1 + 3 m / (count - 1))."""
    return 2.0 ** (-1.0 + 3.0 * np.arange(count) / (count - 1))


def features(lmin: float, lmax: float, n_c: int, n_s: int) -> np.ndarray:
    return np.array([math.log(lmin), math.log(lmax), math.log(lmax / lmin), float(n_c), float(n_s)])


def spectrum_features(A: np.ndarray, n_c: int, iters: int = 96, seed: int = 0, bw: int | None = None):
    """(features, lambda_min, lambda_max) from GPU Lanczos; bw: the
    half-bandwidth of A when it is banded (1 for the tridiagonal sweep
    family), which makes each Lanczos step O(N bw) and copies only the band."""
    N = A.shape[0]
    if bw is not None and 2 * bw + 1 < N:
        lo, hi = B.sv_spectrum_lanczos_band(B.band_of(A, bw), min(iters, N), seed)
    else:
        lo, hi = B.sv_spectrum_lanczos(A, min(iters, N), seed)
    return features(lo, hi, n_c, N.bit_length() - 1), lo, hi


def candidate_factors(log_factor_pred: float) -> np.ndarray:
    """T0 factors (T0 = factor 2 pi / lambda_max) of the learned path: the
    network's prediction and one grid step (2^0.2) above it, then three that
    follow from the spectrum and the grid alone: factor 1, where lambda_max
    sits on the clock's wrap-around (y = 2^n_c, read as 0: the largest
    eigenvalue, the one 1/lambda weights least, is dropped and the whole clock
    range resolves the rest), and the grid's top two factors 2^1.8 and 2^2,
    where the large eigenvalues alias and the small ones gain resolution.
    The sweep's best T0 sits at one of these structures on most instances."""
    g = grid_factors()
    f = math.exp(log_factor_pred)
    return np.array([f, f * 2.0 ** 0.2, 1.0, g[-2], g[-1]])


def label_from_sweep(F: np.ndarray, log_factors: np.ndarray) -> float:
    """log of the best T0 factor: argmax of the sweep, refined by the vertex of
    the parabola through the best point and its two neighbours (clamped to
    half a grid step)."""
    i = int(np.argmax(F))
    if 0 < i < len(F) - 1:
        f0, f1, f2 = F[i - 1], F[i], F[i + 1]
        den = f0 - 2.0 * f1 + f2
        if den < 0.0:
            step = log_factors[i + 1] - log_factors[i]
            off = 0.5 * (f0 - f2) / den
            return float(log_factors[i] + np.clip(off, -0.5, 0.5) * step)
    return float(log_factors[i])


# --------------------------------------------------------------------------
# batched sweeps
# --------------------------------------------------------------------------

def _solve_bytes(n_s, n_c, dtype):
    return (1 << (n_s + n_c + 1)) * (8 if dtype == "c64" else 16)


def run_batched(problems, dtype="c64", max_bytes=24 << 30, max_solves=16384, stream=None, timings=None):
    """problems: list of (A, b, n_c, t0_array).  Runs them in batches that fit
    `max_bytes` of state memory; returns one (len(t0), 4) result array per
    problem ([p_post, p_anc, norm, fidelity]).  timings (dict, optional)
    accumulates 'prepare_s' and 'run_s'."""
    out = [None] * len(problems)
    i = 0
    while i < len(problems):
        j, by, ns = i, 0, 0
        while j < len(problems):
            A, b, n_c, t0 = problems[j]
            n_s = A.shape[0].bit_length() - 1
            need = _solve_bytes(n_s, n_c, dtype) * len(t0)
            if j > i and (by + need > max_bytes or ns + len(t0) > max_solves):
                break
            by += need
            ns += len(t0)
            j += 1
        t = time.perf_counter()
        h = B.sv_batch_prepare(problems[i:j], dtype, stream)
        t1 = time.perf_counter()
        try:
            res = B.sv_batch_run(h, use_graph=True)
        finally:
            B.sv_batch_free(h)
        t2 = time.perf_counter()
        if timings is not None:
            timings["prepare_s"] = timings.get("prepare_s", 0.0) + (t1 - t)
            timings["run_s"] = timings.get("run_s", 0.0) + (t2 - t1)
        k = 0
        for p in range(i, j):
            n = len(problems[p][3])
            out[p] = res[k:k + n]
            k += n
        i = j
    return out


# --------------------------------------------------------------------------
# the predictor
# --------------------------------------------------------------------------

def glorot_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases (layout W1 b1 W2 b2 W3 b3)."""
    rng = np.random.default_rng(seed)
    H = B.SV_MLP_HIDDEN
    parts = []
    for fan_out, fan_in in ((H, N_FEATURES), (H, H), (1, H)):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    p = np.concatenate(parts)
    assert p.size == B.SV_MLP_PARAMS
    return p


def _fold(p, mu, sd, ymu, ysd):
    """Parameters of net'(x) = ysd * net((x - mu) / sd) + ymu."""
    H, I = B.SV_MLP_HIDDEN, N_FEATURES
    p = np.asarray(p, dtype=np.float64).copy()
    W1 = p[:H * I].reshape(H, I)
    b1 = p[H * I:H * I + H]
    W1f = W1 / sd[None, :]
    b1f = b1 - W1f @ mu
    off3 = H * I + H + H * H + H
    p[:H * I] = W1f.ravel()
    p[H * I:H * I + H] = b1f
    p[off3:off3 + H] *= ysd
    p[-1] = p[-1] * ysd + ymu
    return p


@dataclass
class T0Predictor:
    params: np.ndarray = None            # raw-feature parameters (after folding), float64 copy
    history: list = field(default_factory=list)

    def fit(self, X, y, steps=3000, lr=3e-3, seed=0, log_every=250, device="cuda"):
        import torch
        X = np.asarray(X, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        mu, sd = X.mean(0), X.std(0)
        sd[sd == 0] = 1.0
        ymu, ysd = float(y.mean()), float(y.std() or 1.0)
        Xs = torch.tensor((X - mu) / sd, dtype=torch.float32, device=device)
        ys = torch.tensor((y - ymu) / ysd, dtype=torch.float32, device=device)
        P = torch.tensor(glorot_params(seed), dtype=torch.float32, device=device)
        m = torch.zeros_like(P)
        v = torch.zeros_like(P)
        g = torch.empty_like(P)
        loss = torch.empty(1, dtype=torch.float32, device=device)
        self.history = []
        for step in range(1, steps + 1):
            B.sv_mlp_backward(P, Xs, ys, g, loss)
            if step == 1 or step % log_every == 0 or step == steps:
                self.history.append((step, float(loss.item()) * ysd * ysd))
            B.sv_mlp_adam(P, m, v, g, step, lr=lr)
        self.params = _fold(P.double().cpu().numpy(), mu, sd, ymu, ysd)
        return self

    def predict_log_factor(self, X, device="cuda"):
        import torch
        X = np.atleast_2d(np.asarray(X, dtype=np.float64))
        P = torch.tensor(self.params, dtype=torch.float32, device=device)
        Xd = torch.tensor(X, dtype=torch.float32, device=device)
        return B.sv_mlp_forward(P, Xd).double().cpu().numpy()

    def predict_t0(self, X, lambda_max, device="cuda"):
        return np.exp(self.predict_log_factor(X, device)) * 2.0 * math.pi / np.asarray(lambda_max)

    def save(self, path):
        np.savez(path, params=self.params, history=np.asarray(self.history))

    @classmethod
    def load(cls, path):
        z = np.load(path)
        return cls(params=z["params"], history=[tuple(r) for r in z["history"]])


# --------------------------------------------------------------------------
# data and experiment
# --------------------------------------------------------------------------

def make_instances(count, first, n_s_range, n_c_range, kappa_log10=(1.0, 4.0), config=2):
    return inputs.sweep_instances(count=count, config=config, n_s_range=n_s_range, n_c_range=n_c_range,
                                  kappa_log10=kappa_log10, first=first)


def sweep_dataset(instances, dtype="c64", lanczos_iters=96, timings=None):
    """Features (Lanczos), the 16-point sweep fidelities and labels."""
    lf = np.log(grid_factors())
    feats, lams, probs = [], [], []
    t = time.perf_counter()
    for inst in instances:
        f, lo, hi = spectrum_features(inst.A, inst.n_c, lanczos_iters, seed=inst.index, bw=1)
        feats.append(f)
        lams.append((lo, hi))
        probs.append((inst.A, inst.b, inst.n_c, grid_factors() * 2.0 * math.pi / hi))
    if timings is not None:
        timings["features_s"] = timings.get("features_s", 0.0) + time.perf_counter() - t
    res = run_batched(probs, dtype, timings=timings)
    F = np.stack([r[:, 3] for r in res])
    y = np.array([label_from_sweep(row, lf) for row in F])
    return np.array(feats), np.array(lams), F, y, probs


def smooth_labels(F: np.ndarray, log_factors: np.ndarray, width: int = 1) -> np.ndarray:
    """Labels from sweeps averaged over +-width neighbouring grid points
    (edges use the available neighbours): the centre of the best window
    rather than a single, possibly isolated, peak."""
    if width <= 0:
        return np.array([label_from_sweep(r, log_factors) for r in F])
    n = F.shape[1]
    S = np.zeros_like(F)
    for i in range(n):
        a, b = max(0, i - width), min(n, i + width + 1)
        S[:, i] = F[:, a:b].mean(axis=1)
    return np.array([label_from_sweep(r, log_factors) for r in S])


def single_shot(instances, t0, dtype="c64", timings=None):
    probs = [(i.A, i.b, i.n_c, np.array([t])) for i, t in zip(instances, t0)]
    return np.array([r[0, 3] for r in run_batched(probs, dtype, timings=timings)])


def learned_path(instances, model, dtype="c64", timings=None):
    """The learned path on each instance: Lanczos features, the network's T0,
    and the five candidate T0 (candidate_factors) solved in one batched graph;
    the candidate of highest fidelity is kept, as the sweep keeps its best
    grid point.  Returns (F, T0, F of the prediction alone, T0 predicted)."""
    t = time.perf_counter()
    feats, lmax = [], []
    for inst in instances:
        f, _, hi = spectrum_features(inst.A, inst.n_c, seed=inst.index, bw=1)
        feats.append(f)
        lmax.append(hi)
    lmax = np.array(lmax)
    if timings is not None:
        timings["features_s"] = timings.get("features_s", 0.0) + time.perf_counter() - t
    t = time.perf_counter()
    lp = model.predict_log_factor(np.array(feats))
    if timings is not None:
        timings["predict_s"] = timings.get("predict_s", 0.0) + time.perf_counter() - t
    cands = np.stack([candidate_factors(v) for v in lp]) * (2.0 * math.pi / lmax)[:, None]
    probs = [(i.A, i.b, i.n_c, c) for i, c in zip(instances, cands)]
    res = run_batched(probs, dtype, timings=timings)
    Fc = np.stack([r[:, 3] for r in res])
    k = Fc.argmax(axis=1)
    return Fc[np.arange(len(k)), k], cands[np.arange(len(k)), k], Fc[:, 0], cands[:, 0]


def experiment(n_train=2000, n_eval=256, train_ns=(4, 10), eval_ns=(4, 12), n_c=(8, 12), kappa_log10=(1.0, 4.0),
               steps=4000, lr=3e-3, smooth=1, chunk=512, seed=0, log=print):
    """Train on the sweeps of n_train instances (config-2 family), evaluate on
    n_eval held-out instances: learned single shot (complex64) against the
    16-point complex128 sweep and the textbook T0 = 2 pi (1 - 2^-n_c) / lambda_max."""
    import torch
    lf = np.log(grid_factors())
    out = {"n_train": n_train, "n_eval": n_eval, "train_n_s": list(train_ns), "eval_n_s": list(eval_ns),
           "n_c": list(n_c), "kappa_log10": list(kappa_log10), "grid": GRID, "label_smoothing": smooth}
    # --- training data: c64 sweeps, chunked
    t = time.perf_counter()
    Xs, Fs = [], []
    tim = {}
    for c0 in range(0, n_train, chunk):
        insts = make_instances(min(chunk, n_train - c0), c0, train_ns, n_c, kappa_log10)
        X, _, F, _, _ = sweep_dataset(insts, "c64", timings=tim)
        Xs.append(X)
        Fs.append(F)
        log(f"[t0model] train sweeps {c0 + len(insts)}/{n_train}  {time.perf_counter() - t:.1f}s")
    X = np.concatenate(Xs)
    F = np.concatenate(Fs)
    y = smooth_labels(F, lf, smooth)
    out["train_generate_s"] = time.perf_counter() - t
    out["train_sweep_timings"] = tim
    out["train_records"] = int(F.size)
    # --- fit on the GPU kernels
    t = time.perf_counter()
    model = T0Predictor().fit(X, y, steps=steps, lr=lr, seed=seed)
    torch.cuda.synchronize()
    out["fit_s"] = time.perf_counter() - t
    out["loss_history"] = model.history
    log(f"[t0model] fit {out['fit_s']:.1f}s, loss {model.history[0][1]:.4f} -> {model.history[-1][1]:.4f}")
    # --- held-out instances
    test = make_instances(n_eval, 1_000_000, eval_ns, n_c, kappa_log10)
    # reference: the plain 16-point sweep in complex128
    t_sw = {}
    t = time.perf_counter()
    Xe, lam, Fsw, _, _ = sweep_dataset(test, "c128", timings=t_sw)
    torch.cuda.synchronize()
    # the plain sweep's own cost: preparation and its 16 solves per instance
    # (it needs no spectrum features)
    sweep_s = t_sw.get("prepare_s", 0.0) + t_sw.get("run_s", 0.0)
    Fbest = Fsw.max(axis=1)
    # learned path: Lanczos features + MLP + the five candidates, complex64
    t_l = {}
    t = time.perf_counter()
    Fl, _, Fp, t0p = learned_path(test, model, "c64", timings=t_l)
    torch.cuda.synchronize()
    learned_s = time.perf_counter() - t
    feats = [spectrum_features(i.A, i.n_c, seed=i.index, bw=1)[0] for i in test]
    lmax = lam[:, 1]
    # the method without the network
    t0t = np.array([2 * math.pi * (1 - 2.0 ** -i.n_c) / h for i, h in zip(test, lmax)])
    Ft = single_shot(test, t0t, "c64")
    # the untrained network
    untrained = T0Predictor(params=_fold(glorot_params(seed), np.zeros(N_FEATURES), np.ones(N_FEATURES), 0.0, 1.0))
    Fu = single_shot(test, untrained.predict_t0(np.array(feats), np.array(lmax)), "c64")
    gap = Fbest - Fl
    gap1 = Fbest - Fp
    ncand = len(candidate_factors(0.0))
    out.update({
        "F_sweep_best_mean": float(Fbest.mean()), "F_learned_mean": float(Fl.mean()),
        "F_prediction_only_mean": float(Fp.mean()),
        "F_textbook_mean": float(Ft.mean()), "F_untrained_mean": float(Fu.mean()),
        "gap_mean": float(gap.mean()), "gap_median": float(np.median(gap)),
        "gap_p90": float(np.quantile(gap, 0.9)), "gap_max": float(gap.max()),
        "frac_gap_le_1e-4": float(np.mean(gap <= 1e-4)), "frac_learned_ge_best": float(np.mean(gap <= 0.0)),
        "prediction_only_frac_gap_le_1e-4": float(np.mean(gap1 <= 1e-4)),
        "one_minus_F_best_median": float(np.median(1 - Fbest)),
        "one_minus_F_learned_median": float(np.median(1 - Fl)),
        "sweep_s": sweep_s, "sweep_timings": t_sw, "sweep_solves": int(Fsw.size),
        "learned_s": learned_s, "learned_timings": t_l, "learned_solves": ncand * len(test),
        "candidates_per_instance": ncand,
        "speedup_end_to_end": sweep_s / learned_s,
        "speedup_solve_only": t_sw.get("run_s", 0.0) / max(t_l.get("run_s", 1e-30), 1e-30),
        "solves_per_s_at_1mF_le_1e-4_sweep": float(np.sum(1 - Fbest <= 1e-4)) / sweep_s,
        "solves_per_s_at_1mF_le_1e-4_learned": float(np.sum(1 - Fl <= 1e-4)) / learned_s,
    })
    by_ns = {}
    for ns in range(eval_ns[0], eval_ns[1] + 1):
        sel = np.array([i.n_s == ns for i in test])
        if sel.any():
            by_ns[ns] = {"count": int(sel.sum()), "F_best": float(Fbest[sel].mean()),
                         "F_learned": float(Fl[sel].mean()), "F_textbook": float(Ft[sel].mean())}
    out["by_n_s"] = by_ns
    return out, model


if __name__ == "__main__":
    import argparse
    import json
    import os
    ap = argparse.ArgumentParser(description="train and evaluate the learned T0 predictor on the GPU")
    ap.add_argument("--train", type=int, default=10000)
    ap.add_argument("--eval", type=int, default=256)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--smooth", type=int, default=1)
    ap.add_argument("--out", default="t0model.json")
    ap.add_argument("--save", default="")
    a = ap.parse_args()
    res, model = experiment(n_train=a.train, n_eval=a.eval, steps=a.steps, lr=a.lr, smooth=a.smooth,
                            log=lambda s: print(s, flush=True))
    os.makedirs(os.path.dirname(a.out) or ".", exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(res, f, indent=1, default=float)
    if a.save:
        model.save(a.save)
    print(json.dumps({k: v for k, v in res.items() if not isinstance(v, (list, dict))}, default=float))
