"""Learned plan selection for the Rosko SpMM (auto-tuning the exposed tiling
parameters, which Sec. 6 leaves to future work, in place of the analytic tiling model of
Sec. 4.2).

Per matrix, a Linear(16,64)-ReLU-Linear(64,64)-ReLU-Linear(64,C) network
predicts log(runtime / best runtime) of each candidate plan
(rosko_sched_candidate: panel height mr, register tile, sparse or
dense-MFMA path) from 16 packing statistics (rosko_features); the candidate
with the smallest prediction is used.  The committed network
(sched_data/weights.json) scores the six sparse candidates (C = 6); the
analytic rule (rosko_sched_analytic) is used when no network is loaded.

Everything numerical runs in the library's HIP kernels through the C ABI:
statistics, normalisation, forward, the MSE gradient, backward, Adam and
the arg-min.  This module marshals arguments, holds the device buffers and
drives the timing sweeps and the training:

- `measure`: measured SpMM runtimes of every sparse candidate on the
  matrices of synth.sweep_specs() at every N of synth.SWEEP_N
  (sched_data/measured.jsonl);
- `fit`: full-batch Adam on the training matrices of that sweep, then the
  slowdown t(choice) / t(fastest) of the network, the analytic rule and the
  best fixed candidate on the held-out matrices.  The time is repack plus
  SpMM by default (a step that packs afresh), or the SpMM alone
  (`--objective spmm`, a matrix packed once);
- `sweep` / `train` / `eval`: the same over the seeded random-shape corpus
  (synth.corpus_spec).
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import time

import numpy as np
import torch

from . import _lib as L
from . import ops, synth

F = L.ROSKO_NFEAT
HID = 64
NCAND = L.ROSKO_SCHED_CANDIDATES
DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sched_data")
WEIGHTS = os.path.join(DATA_DIR, "weights.json")
REPORT = os.path.join(DATA_DIR, "fit_report.json")
CORPUS = os.path.join(DATA_DIR, "corpus.jsonl")
MEASURED = os.path.join(DATA_DIR, "measured.jsonl")
N_TRAIN = 1800
OBJECTIVES = ("step", "spmm")


def _p(t):
    return ops._ptr(t)


def _s():
    return ops._stream_ptr()


# ------------------------------------------------------------- statistics
def features(A: torch.Tensor, N: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """The 16 statistics of A (M x K float32 CUDA) times N columns, on the
    device (rosko_features)."""
    ops._check_dense(A, "A")
    M, K = A.shape
    n = C.c_size_t(0)
    L.check(L.lib().rosko_features_workspace_size(M, K, C.byref(n)))
    ws = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=A.device)
    if out is None:
        out = torch.empty(F, dtype=torch.float32, device=A.device)
    L.check(L.lib().rosko_features(_p(A), M, K, max(A.stride(0), 1), N, _p(ws), ws.numel(),
                                   _p(out), _s()))
    return out


def candidate(index: int):
    """(mr, rosko_plan) of candidate `index`."""
    mr = C.c_int32(0)
    plan = L.RoskoPlan()
    L.check(L.lib().rosko_sched_candidate(int(index), C.byref(mr), C.byref(plan)))
    return int(mr.value), plan


def analytic(f_host: np.ndarray) -> int:
    f = np.ascontiguousarray(f_host, np.float32)
    idx = C.c_int32(0)
    L.check(L.lib().rosko_sched_analytic(f.ctypes.data_as(C.c_void_p), C.byref(idx)))
    return int(idx.value)


# -------------------------------------------------------------------- MLP
def param_count(Fi=F, H=HID, Cn=NCAND) -> int:
    n = C.c_int64(0)
    L.check(L.lib().rosko_mlp_param_count(Fi, H, Cn, C.byref(n)))
    return int(n.value)


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], np.float32).ravel()
                           for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unflatten(flat: np.ndarray, Fi=F, H=HID, Cn=NCAND) -> dict:
    shapes = [("W1", (Fi, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, Cn)),
              ("b3", (Cn,))]
    out, o = {}, 0
    for k, sh in shapes:
        n = int(np.prod(sh))
        out[k] = np.asarray(flat[o:o + n], np.float32).reshape(sh)
        o += n
    return out


class MLP:
    """Device parameters, Adam state and the kernel calls of the network."""

    def __init__(self, flat: np.ndarray, mu: np.ndarray, sigma: np.ndarray, device="cuda",
                 Fi=F, H=HID, Cn=NCAND):
        self.F, self.H, self.C = Fi, H, Cn
        self.n = param_count(Fi, H, Cn)
        assert flat.size == self.n
        self.params = torch.from_numpy(np.asarray(flat, np.float32).copy()).to(device)
        self.mu = torch.from_numpy(np.asarray(mu, np.float32)).to(device)
        self.sigma = torch.from_numpy(np.asarray(sigma, np.float32)).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.t = 0

    def normalize(self, X: torch.Tensor) -> torch.Tensor:
        Xn = torch.empty_like(X)
        L.check(L.lib().rosko_mlp_normalize(_p(X), X.shape[0], self.F, _p(self.mu),
                                            _p(self.sigma), _p(Xn), _s()))
        return Xn

    def forward(self, Xn: torch.Tensor):
        B = Xn.shape[0]
        dev = Xn.device
        H1 = torch.empty((B, self.H), dtype=torch.float32, device=dev)
        H2 = torch.empty((B, self.H), dtype=torch.float32, device=dev)
        Y = torch.empty((B, self.C), dtype=torch.float32, device=dev)
        L.check(L.lib().rosko_mlp_forward(_p(self.params), self.F, self.H, self.C, _p(Xn), B,
                                          _p(H1), _p(H2), _p(Y), _s()))
        return H1, H2, Y

    def backward(self, Xn, H1, H2, Y, T, mask) -> torch.Tensor:
        B = Xn.shape[0]
        ws = torch.empty(B * (self.C + 2 * self.H), dtype=torch.float32, device=Xn.device)
        loss = torch.empty(1, dtype=torch.float32, device=Xn.device)
        L.check(L.lib().rosko_mlp_backward(_p(self.params), self.F, self.H, self.C, _p(Xn),
                                           _p(H1), _p(H2), _p(Y), _p(T), _p(mask), B,
                                           _p(self.grads), _p(ws), _p(loss), _s()))
        return loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        L.check(L.lib().rosko_adam_step(_p(self.params), _p(self.grads), _p(self.m), _p(self.v),
                                        self.n, lr, beta1, beta2, eps, self.t, _s()))

    def choose(self, X: torch.Tensor) -> torch.Tensor:
        """Arg-min of the predicted log slowdown per row of raw features X."""
        _, _, Y = self.forward(self.normalize(X))
        out = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
        L.check(L.lib().rosko_argmin_rows(_p(Y), X.shape[0], self.C, _p(out), _s()))
        return out

    def to_json(self) -> dict:
        return {"F": self.F, "H": self.H, "C": self.C,
                "mu": self.mu.cpu().tolist(), "sigma": self.sigma.cpu().tolist(),
                "params": self.params.cpu().tolist()}

    @staticmethod
    def from_json(d: dict, device="cuda") -> "MLP":
        net = MLP(np.array(d["params"], np.float32), np.array(d["mu"], np.float32),
                  np.array(d["sigma"], np.float32), device, d["F"], d["H"], d["C"])
        net.objective = d.get("objective", "step")
        return net


def load(device="cuda", path: str = WEIGHTS) -> MLP | None:
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return MLP.from_json(json.load(f), device)


_NETS: dict = {}


_DT = {"f32": L.ROSKO_F32, "bf16": L.ROSKO_BF16, "fp8": L.ROSKO_FP8_E4M3}


def precision_rule(f_host: np.ndarray, index: int, val_dtype="f32", b_dtype="f32") -> int:
    """The library's value-type rule (rosko_sched_precision) applied to a
    candidate index chosen for FP32 operands."""
    f = np.ascontiguousarray(f_host, np.float32)
    idx = C.c_int32(int(index))
    L.check(L.lib().rosko_sched_precision(f.ctypes.data_as(C.c_void_p), _DT[val_dtype],
                                          _DT[b_dtype], C.byref(idx)))
    return int(idx.value)


def plan_select(f_host: np.ndarray, weights: dict | None = None, val_dtype="f32",
                b_dtype="f32"):
    """(candidate index, panel height, plan) from rosko_plan_select: the host
    forward pass of the network given as its JSON dict (weights.json), or
    the analytic rule when None, then the value-type rule."""
    f = np.ascontiguousarray(f_host, np.float32)
    idx, mr, plan = C.c_int32(-1), C.c_int32(0), L.RoskoPlan()
    if weights is None:
        args = (None, None, None)
    else:
        keep = [np.ascontiguousarray(weights[k], np.float32) for k in ("params", "mu", "sigma")]
        args = tuple(x.ctypes.data_as(C.c_void_p) for x in keep)
    L.check(L.lib().rosko_plan_select(f.ctypes.data_as(C.c_void_p), *args, _DT[val_dtype],
                                      _DT[b_dtype], C.byref(idx), C.byref(mr), C.byref(plan)))
    return int(idx.value), int(mr.value), plan


def network_beats_rule(path: str = REPORT) -> bool:
    """True when the committed fit report shows the network strictly ahead of
    the analytic rule on its held-out problems (geomean slowdown)."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        rep = json.load(f)["held_out"]
    return rep["mlp"]["geomean"] < rep["analytic"]["geomean"]


def default_net(device=None) -> MLP | None:
    """The committed network on `device` (the current CUDA device if None),
    loaded once per device; None when no weights file is present or when the
    network does not beat the analytic rule on its held-out problems (then
    the rule, the method's own tiling choice, is used)."""
    dev = torch.device(device) if device is not None else torch.device(
        "cuda", torch.cuda.current_device())
    key = str(dev)
    if key not in _NETS:
        _NETS[key] = load(dev) if network_beats_rule() else None
    return _NETS[key]


def choose(A: torch.Tensor, N: int, net: MLP | None = None, rule: str = "auto",
           val_dtype: str = "f32", b_dtype: str = "f32") -> int:
    """Candidate index for A (stored as val_dtype) times N columns of a B of
    b_dtype.  rule "auto": the network `net`, else the committed network,
    else the analytic rule; rule "analytic": the analytic rule; then the
    library's value-type rule."""
    if rule not in ("auto", "analytic"):
        raise ValueError(f"unknown rule {rule!r}")
    f = features(A, N)
    if rule == "auto" and net is None:
        net = default_net(A.device)
    fh = f.cpu().numpy().reshape(-1)
    if rule == "analytic" or net is None:
        idx = analytic(fh)
    else:
        idx = int(net.choose(f.view(1, F)).item())
    return precision_rule(fh, idx, val_dtype, b_dtype)


def chooser_name(device=None) -> str:
    """Which rule choose(..., rule="auto") applies on `device`."""
    return "mlp" if default_net(device) is not None else "analytic"


# ---------------------------------------------------------------- corpus
def sparse_candidates() -> list:
    """Indices of the candidates whose plan takes the sparse path."""
    return [c for c in range(NCAND) if candidate(c)[1].path == L.ROSKO_PATH_SPARSE]


def time_packed(P, B: torch.Tensor, plan, reps: int = 5) -> float:
    """Median time (microseconds) of rosko_spmm of packed P times B under
    `plan`, one warm-up call first."""
    N = B.shape[1]
    Cm = torch.empty((P.M, N), dtype=torch.float32, device=B.device)
    need = ops.spmm_workspace_size(P, N, plan)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=B.device)
    ops.spmm(P, B, Cm, plan=plan, ws=ws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ops.spmm(P, B, Cm, plan=plan, ws=ws)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e3)
    del Cm, ws
    return float(np.median(ts))


def time_pack(A: torch.Tensor, P, reps: int = 5) -> float:
    """Median time (microseconds) of repacking A into P's buffers (the
    count, offset and write passes), one warm-up call first."""
    M, K = A.shape
    ws = torch.empty(max(ops.workspace_size(M, K, P.mr), 1), dtype=torch.uint8, device=A.device)
    ops.pack_into(A, P, ws)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ops.pack_into(A, P, ws)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) * 1e3)
    del ws
    return float(np.median(ts))


def time_candidate(A: torch.Tensor, B: torch.Tensor, index: int, reps: int = 5) -> float:
    """Median SpMM time (microseconds) of candidate `index`, packing excluded."""
    mr, plan = candidate(index)
    P = ops.pack(A, mr, "f32")
    t = time_packed(P, B, plan, reps)
    del P
    return t


def sweep(first: int, last: int, path: str, log_every: int = 1, reps: int = 5) -> None:
    """Measure every candidate (sparse and dense-MFMA) on corpus problems
    [first, last) and append one JSON line per problem to `path`: the
    statistics, the SpMM time of each candidate and the time to repack the
    matrix at the candidate's panel height, in microseconds."""
    dev = torch.device("cuda")
    done = set()
    if os.path.exists(path):
        with open(path) as f:
            done = {json.loads(line)["i"] for line in f if line.strip()}
    t0 = time.time()
    with open(path, "a") as out:
        for i in range(first, last):
            if i in done:
                continue
            A, B, sp = synth.corpus_problem_device(i, dev)
            print(f"corpus {i}: {sp['M']}x{sp['K']}x{sp['N']} s={sp['sparsity']:.3f} "
                  f"{sp['kind']}", flush=True)
            f = features(A, B.shape[1]).cpu().numpy().tolist()
            times, packs, packed = [], [], {}
            for c in range(NCAND):
                mr, plan = candidate(c)
                if mr not in packed:
                    P = ops.pack(A, mr, "f32")
                    packed[mr] = (P, time_pack(A, P, reps))
                P, tp = packed[mr]
                times.append(time_packed(P, B, plan, reps))
                packs.append(tp)
            del packed
            out.write(json.dumps({"i": i, "M": sp["M"], "K": sp["K"], "N": sp["N"],
                                  "sparsity": sp["sparsity"], "kind": sp["kind"],
                                  "features": f, "times_us": times, "pack_us": packs}) + "\n")
            out.flush()
            del A, B
            if (i - first) % log_every == 0:
                print(f"  best={int(np.argmin(times))} t={min(times):.1f}us "
                      f"({time.time() - t0:.0f}s)", flush=True)


def read_corpus(path: str = CORPUS, objective: str = "spmm"):
    """Problem indices, statistics X and times Tm (problems x candidates) of
    the corpus; objective "spmm" (a matrix packed once) or "step" (repack
    plus SpMM)."""
    if objective not in OBJECTIVES:
        raise ValueError(f"unknown objective {objective!r}")
    rows = [json.loads(line) for line in open(path) if line.strip()]
    rows.sort(key=lambda r: r["i"])
    X = np.array([r["features"] for r in rows], np.float32)
    Tm = np.array([r["times_us"] for r in rows], np.float64)
    if objective == "step":
        Tm = Tm + np.array([r["pack_us"] for r in rows], np.float64)
    idx = np.array([r["i"] for r in rows])
    return idx, X, Tm


def measured_sweep(path: str = MEASURED, reps: int = 7) -> None:
    """Time every candidate (sparse and dense-MFMA) on every matrix of
    synth.sweep_specs() at every N of synth.SWEEP_N and write one JSON line
    per (matrix, N): the spec, the 16 statistics, the SpMM times and the
    times to repack the matrix at the candidate's panel height (FP32
    values), in microseconds, in candidate order.  Inputs are generated on
    the host, as in the parity tests, and copied to the device."""
    dev = torch.device("cuda")
    cands = list(range(NCAND))
    plans = [candidate(c) for c in cands]
    Bs = {}
    t0 = time.time()
    with open(path, "w") as out:
        for sp in synth.sweep_specs():
            M, K = sp["M"], sp["K"]
            print(f"sweep {sp['j']}: {M}x{K} s={sp['sparsity']} {sp['kind']}", flush=True)
            A = torch.from_numpy(synth.sparse_matrix(M, K, 1.0 - sp["sparsity"], sp["seed"],
                                                     sp["kind"])).to(dev)
            for N in synth.SWEEP_N:
                if (K, N) not in Bs:
                    Bs[(K, N)] = torch.from_numpy(synth.dense_normal(K, N, 30000 + K + N)).to(dev)
            times = {N: [] for N in synth.SWEEP_N}
            packs, packed = [], {}
            for mr, plan in plans:
                if mr not in packed:
                    P = ops.pack(A, mr, "f32")
                    packed[mr] = (P, time_pack(A, P, reps))
                P, tp = packed[mr]
                packs.append(tp)
                for N in synth.SWEEP_N:
                    times[N].append(time_packed(P, Bs[(K, N)], plan, reps))
            del packed
            for N in synth.SWEEP_N:
                f = features(A, N).cpu().numpy().tolist()
                out.write(json.dumps(dict(sp, N=N, candidates=cands, features=f,
                                          times_us=times[N], pack_us=packs)) + "\n")
            out.flush()
            del A
            best = {N: int(np.argmin(times[N])) for N in synth.SWEEP_N}
            print(f"  best {best} ({time.time() - t0:.0f}s)", flush=True)


def read_measured(path: str = MEASURED, objective: str = "step"):
    """Statistics X, times Tm (problems x candidates) and the held-out flag
    of the measured sweep.  objective "step": repack plus SpMM, the cost of
    a step that packs its matrix afresh (training, and the benchmark step);
    "spmm": the SpMM alone, for a matrix packed once and reused."""
    if objective not in OBJECTIVES:
        raise ValueError(f"unknown objective {objective!r}")
    rows = [json.loads(line) for line in open(path) if line.strip()]
    rows.sort(key=lambda r: (r["j"], r["N"]))
    X = np.array([r["features"] for r in rows], np.float32)
    Tm = np.array([r["times_us"] for r in rows], np.float64)
    if objective == "step":
        Tm = Tm + np.array([r["pack_us"] for r in rows], np.float64)
    held = np.array([bool(r["held_out"]) for r in rows])
    return X, Tm, held


def targets(Tm: np.ndarray) -> np.ndarray:
    """log(t / best t) per problem and candidate."""
    return np.log(Tm / Tm.min(axis=1, keepdims=True)).astype(np.float32)


def train(X: np.ndarray, Tm: np.ndarray, steps: int = 4000, lr: float = 3e-3, seed: int = 17,
          device="cuda", log_every: int = 500) -> MLP:
    """Full-batch Adam on the GPU through the library's kernels."""
    mu = X.mean(axis=0)
    sigma = X.std(axis=0)
    sigma[sigma < 1e-6] = 1.0
    Cn = Tm.shape[1]
    net = MLP(flatten(synth.mlp_init_params(F, HID, Cn, seed)), mu, sigma, device, F, HID, Cn)
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(device)
    Td = torch.from_numpy(targets(Tm)).to(device)
    mask = torch.ones_like(Td)
    Xn = net.normalize(Xd)
    for step in range(1, steps + 1):
        H1, H2, Y = net.forward(Xn)
        loss = net.backward(Xn, H1, H2, Y, Td, mask)
        net.adam(lr=lr)
        if step % log_every == 0 or step == 1:
            print(f"train step {step}: loss {loss.item():.5f}", flush=True)
    return net


def evaluate(net: MLP | None, X: np.ndarray, Tm: np.ndarray) -> dict:
    """Slowdown t(choice) / t(best) of the network, the analytic rule and
    the best single fixed candidate on the given problems."""
    best = Tm.min(axis=1)
    out = {}
    if net is not None:
        ch = net.choose(torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()).cpu().numpy()
        r = Tm[np.arange(len(ch)), ch] / best
        out["mlp"] = {"mean": float(r.mean()), "median": float(np.median(r)),
                      "geomean": float(np.exp(np.log(r).mean())),
                      "within_5pct": float((r <= 1.05).mean()), "max": float(r.max())}
    ana = np.array([analytic(x) for x in X])
    r = Tm[np.arange(len(ana)), ana] / best
    if net is not None:
        out["mlp"]["vs_analytic_geomean"] = float(
            np.exp(np.log(Tm[np.arange(len(ch)), ch] / Tm[np.arange(len(ana)), ana]).mean()))
    out["analytic"] = {"mean": float(r.mean()), "median": float(np.median(r)),
                       "geomean": float(np.exp(np.log(r).mean())),
                       "within_5pct": float((r <= 1.05).mean()), "max": float(r.max())}
    fixed = [float(np.exp(np.log(Tm[:, c] / best).mean())) for c in range(Tm.shape[1])]
    c = int(np.argmin(fixed))
    r = Tm[:, c] / best
    out["best_fixed"] = {"candidate": c, "mean": float(r.mean()), "geomean": fixed[c],
                         "within_5pct": float((r <= 1.05).mean())}
    return out


def main(argv=None):
    """python -m paper_2307_03930_amd.sched measure | fit | sweep FIRST LAST | train | eval"""
    import argparse
    ap = argparse.ArgumentParser(prog="python -m paper_2307_03930_amd.sched")
    sub = ap.add_subparsers(dest="cmd", required=True)
    m = sub.add_parser("measure")
    m.add_argument("--out", default=MEASURED)
    m.add_argument("--reps", type=int, default=7)
    fi = sub.add_parser("fit")
    fi.add_argument("--data", default=MEASURED)
    fi.add_argument("--steps", type=int, default=3000)
    fi.add_argument("--lr", type=float, default=3e-3)
    fi.add_argument("--out", default=WEIGHTS)
    fi.add_argument("--objective", choices=OBJECTIVES, default="step")
    s = sub.add_parser("sweep")
    s.add_argument("first", type=int)
    s.add_argument("last", type=int)
    s.add_argument("--out", default=CORPUS)
    t = sub.add_parser("train")
    t.add_argument("--steps", type=int, default=6000)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--corpus", default=CORPUS)
    t.add_argument("--out", default=WEIGHTS)
    t.add_argument("--report", default=REPORT)
    t.add_argument("--objective", choices=OBJECTIVES, default="step")
    e = sub.add_parser("eval")
    e.add_argument("--corpus", default=CORPUS)
    a = ap.parse_args(argv)
    if a.cmd == "measure":
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        measured_sweep(a.out, a.reps)
    elif a.cmd == "fit":
        X, Tm, held = read_measured(a.data, a.objective)
        net = train(X[~held], Tm[~held], steps=a.steps, lr=a.lr)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            json.dump(dict(net.to_json(), objective=a.objective), f)
        print(json.dumps({"objective": a.objective,
                          "n_train": int((~held).sum()), "n_held_out": int(held.sum()),
                          "train": evaluate(net, X[~held], Tm[~held]),
                          "held_out": evaluate(net, X[held], Tm[held])}), flush=True)
    elif a.cmd == "sweep":
        os.makedirs(os.path.dirname(a.out), exist_ok=True)
        sweep(a.first, a.last, a.out)
    elif a.cmd == "train":
        # training set: the corpus's first N_TRAIN problems and the
        # benchmark-shape sweep's training matrices; held out: the corpus's
        # last 200 problems and the sweep's held-out matrices
        idx, X, Tm = read_corpus(a.corpus, a.objective)
        tr = idx < N_TRAIN
        Xs, Ts, held_s = read_measured(MEASURED, a.objective)
        Xtr = np.concatenate([X[tr], Xs[~held_s]])
        Ttr = np.concatenate([Tm[tr], Ts[~held_s]])
        net = train(Xtr, Ttr, steps=a.steps, lr=a.lr)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            json.dump(dict(net.to_json(), objective=a.objective), f)
        rep = {"data": "corpus+sweep", "objective": a.objective, "steps": a.steps, "lr": a.lr,
               "n_train": int(len(Xtr)), "n_held_out": int((~tr).sum()),
               "n_held_out_sweep": int(held_s.sum()),
               "train": evaluate(net, Xtr, Ttr), "held_out": evaluate(net, X[~tr], Tm[~tr]),
               "held_out_sweep": evaluate(net, Xs[held_s], Ts[held_s])}
        with open(a.report, "w") as f:
            json.dump(rep, f)
        print(json.dumps(rep), flush=True)
    else:
        net = load()
        idx, X, Tm = read_corpus(a.corpus, net.objective if net is not None else "step")
        ho = idx >= N_TRAIN
        print(json.dumps({"held_out": evaluate(net, X[ho], Tm[ho])}), flush=True)


if __name__ == "__main__":
    main()
