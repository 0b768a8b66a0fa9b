"""Learned spectral schedule for the sign iteration.

A small MLP (library kernels: nolsm_mlp_forward / _backward / _mse / _adam) maps the
per-submatrix descriptors of A_k = M_k - mu I (nolsm_features) to log10 l_k, a
lower bound on min |eig(A_k)| / b_k with b_k the Gershgorin bound.  The sign
iteration then uses the spectrum-interval scaling of Newton-Schulz driven by l_k
(nolsm_schedule.lower_log10) and still stops on its residual, so a poor prediction
costs iterations, never accuracy; submatrices that miss the tolerance fall back to
plain FP32 Newton-Schulz.

Training data come from runs of the plain method: the number of plain FP32
Newton-Schulz iterations a submatrix needs from the Gershgorin scale fixes, through
the scalar Newton-Schulz map x -> x (3 - x^2) / 2, the smallest starting eigenvalue
that converges in that many steps; that value is the label (a lower bound within a
factor of about 1.5).

Input and target standardisation are folded into the first and last layers when
training ends, so inference runs on raw descriptors through the kernels alone.
"""
from __future__ import annotations

import hashlib
import io
import math

import numpy as np
import torch

from . import _lib as L

NIN, NH = L.NFEAT, L.MLP_HIDDEN


# ----------------------------------------------------------------------------- labels

def ns_steps(x0: float, tol: float, cap: int = 200) -> int:
    """Newton-Schulz steps until |1 - x^2| <= tol for a starting eigenvalue x0 in (0, 1]."""
    x = x0
    for t in range(cap):
        if abs(1.0 - x * x) <= tol:
            return t
        x = 0.5 * x * (3.0 - x * x)
    return cap


def lower_from_steps(n: int, tol: float) -> float:
    """Smallest x0 in (0, 1] whose scalar iteration converges within n steps."""
    lo, hi = 1e-12, 1.0
    if ns_steps(lo, tol) <= n:
        return lo
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if ns_steps(mid, tol) <= n:
            hi = mid
        else:
            lo = mid
        if hi / lo < 1.0 + 1e-9:
            break
    return hi


def labels_from_plain_run(iters, extra: int, tol: float) -> np.ndarray:
    """log10 lower-bound labels from plain-run iteration counts (iters include `extra`)."""
    cache = {}
    out = np.empty(len(iters))
    for i, it in enumerate(np.asarray(iters, dtype=int)):
        n = max(int(it) - extra, 0)
        if n not in cache:
            cache[n] = math.log10(lower_from_steps(n, tol))
        out[i] = cache[n]
    return out


# ----------------------------------------------------------------------------- network

def _glorot(nout: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((NIN, NH), (NH, NH), (NH, nout)):
        lim = math.sqrt(6.0 / (fi + fo))
        parts += [rng.uniform(-lim, lim, (fo, fi)).ravel(), np.zeros(fo)]
    return np.concatenate(parts).astype(np.float32)


class ScheduleMLP:
    """Parameters, Adam state and the training loop, all on the GPU."""

    def __init__(self, nout: int = 1, seed: int = 0, params: np.ndarray | None = None,
                 device: str = "cuda"):
        self.nout = nout
        self.device = device
        self.P = L.nolsm_mlp_param_count(nout)
        p = _glorot(nout, seed) if params is None else np.asarray(params, np.float32)
        assert p.size == self.P
        self.params = torch.from_numpy(p.copy()).to(device)

    # -- inference
    def predict(self, feat: torch.Tensor) -> torch.Tensor:
        y = torch.empty(feat.shape[0], self.nout, device=self.device)
        if feat.shape[0]:
            L.nolsm_mlp_forward(self.params, self.nout, feat, y)
        return y

    # -- training (full batch Adam on standardised data; standardisation folded in at the end)
    def fit(self, x: np.ndarray, t: np.ndarray, steps: int = 2000, lr: float = 3e-3,
            beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, log_every: int = 50):
        x = np.asarray(x, np.float64)
        t = np.asarray(t, np.float64).reshape(len(x), self.nout)
        mx, sx = x.mean(0), x.std(0)
        sx[sx < 1e-8] = 1.0
        mt, st = t.mean(0), t.std(0)
        st[st < 1e-8] = 1.0
        X = torch.from_numpy(((x - mx) / sx).astype(np.float32)).to(self.device)
        T = torch.from_numpy(((t - mt) / st).astype(np.float32)).to(self.device)
        B = X.shape[0]
        y = torch.empty(B, self.nout, device=self.device)
        act = torch.empty(B, 2 * NH, device=self.device)
        dy = torch.empty_like(y)
        loss = torch.empty(1, device=self.device)
        grad = torch.empty(self.P, device=self.device)
        m = torch.zeros(self.P, device=self.device)
        v = torch.zeros(self.P, device=self.device)
        scratch = torch.empty(L.nolsm_mlp_scratch_floats(B, self.nout), device=self.device)
        hist = []
        for step in range(1, steps + 1):
            L.nolsm_mlp_forward(self.params, self.nout, X, y, act)
            L.nolsm_mlp_mse(y, T, dy, loss, scratch)
            L.nolsm_mlp_backward(self.params, self.nout, X, act, dy, grad, scratch)
            L.nolsm_mlp_adam(self.params, grad, m, v, lr, beta1, beta2, eps, step)
            if step == 1 or step % log_every == 0 or step == steps:
                hist.append(float(loss.item()))
        self._fold(mx, sx, mt, st)
        return hist

    def _fold(self, mx, sx, mt, st):
        """Fold x' = (x - mx)/sx and y = st y' + mt into the first and last layers."""
        p = self.params.cpu().numpy().astype(np.float64)
        o = 0
        W1 = p[o:o + NH * NIN].reshape(NH, NIN)
        b1 = p[o + NH * NIN:o + NH * NIN + NH]
        W1n = W1 / sx[None, :]
        b1n = b1 - W1n @ mx
        p[o:o + NH * NIN] = W1n.ravel()
        p[o + NH * NIN:o + NH * NIN + NH] = b1n
        o3 = NH * NIN + NH + NH * NH + NH
        W3 = p[o3:o3 + self.nout * NH].reshape(self.nout, NH)
        b3 = p[o3 + self.nout * NH:]
        p[o3:o3 + self.nout * NH] = (st[:, None] * W3).ravel()
        p[o3 + self.nout * NH:] = st * b3 + mt
        self.params = torch.from_numpy(p.astype(np.float32)).to(self.device)

    # -- persistence (npz + content hash)
    def save(self, path: str, meta: dict | None = None) -> str:
        p = self.params.cpu().numpy()
        digest = hashlib.sha256(p.tobytes()).hexdigest()
        np.savez(path, params=p, nout=np.int32(self.nout), sha256=np.array(digest),
                 meta=np.array(repr(meta or {})))
        return digest

    @classmethod
    def load(cls, path: str, device: str = "cuda") -> "ScheduleMLP":
        with np.load(path, allow_pickle=False) as z:
            p = z["params"]
            digest = str(z["sha256"])
            nout = int(z["nout"])
        if hashlib.sha256(p.tobytes()).hexdigest() != digest:
            raise ValueError(f"{path}: parameter hash mismatch")
        return cls(nout=nout, params=p, device=device)


def pick_molecules(nmol: int, count: int, seed: int, salt: int = 0x5EED) -> np.ndarray:
    """A seeded, sorted sample of `count` molecules (all of them if count >= nmol)."""
    if count >= nmol:
        return np.arange(nmol, dtype=np.int32)
    rng = np.random.default_rng([salt, seed])
    return np.sort(rng.choice(nmol, count, replace=False)).astype(np.int32)


def collect(inst, mols, tol: float = 1e-3, extra: int = 2, mus=None):
    """Descriptors and labels for the submatrices of `mols` (one batch on the GPU).

    The label is log10 of the smallest starting eigenvalue that the plain FP32
    Newton-Schulz iteration (Gershgorin scale, run to ||X^2 - I||_F <= tol plus
    `extra` steps) would bring to tolerance in the number of steps it took.
    mus: chemical potentials to collect at (default: the instance's mu); the set-up
    is shared, and the rows for each mu follow each other.
    Returns (features [K m, NFEAT] float64, labels, plain iterations, ok, mu per row).
    """
    from .runner import Runner, plain_fp32_schedule
    mus = [inst.mu] if mus is None else list(mus)
    r = Runner(inst, mols=mols)
    L.nolsm_build_submatrices(r.plans[0], r.dpat, r.H, r.S)
    out = []
    for mu in mus:
        feat = features(r, 0, mu).cpu().numpy().astype(np.float64)
        r.run(mu=mu, sched=plain_fp32_schedule(tol=tol, extra=extra), energy=False,
              regather=False)
        st = r.stats_host()
        ok = (st["status"] == 0) & (st["fell_back"] == 0)
        lab = labels_from_plain_run(st["iters_lo"], extra, tol)
        out.append((feat, lab, st["iters_lo"].astype(np.int32), ok, np.full(len(lab), mu)))
    del r
    return tuple(np.concatenate([o[i] for o in out]) for i in range(5))


def compare_schedules(inst, mols, model: "ScheduleMLP", lower_factor: float = 0.5, mu=None):
    """Plain FP32, default mixed and learned mixed on one batch of `mols`.

    mu: the chemical potential (default: the instance's).
    Returns a dict per schedule: mean low-precision and fallback iterations, sign
    and GEMM time (HIP events), paper-convention sign-phase TFLOP/s, fallbacks, and
    for the mixed forms the largest density difference, the energy difference per
    atom of the sampled molecules together, and the largest single-molecule energy
    difference per atom, all against the plain FP32 result of the same submatrices.
    """
    from .runner import Runner, default_mixed_schedule, learned_schedule, plain_fp32_schedule
    r = Runner(inst, mols=mols)
    p = r.plans[0]
    atoms = np.asarray(inst.atoms)[mols].astype(np.float64)
    out, ref = {}, None
    for name, sched, pred in (("plain_fp32", plain_fp32_schedule(), None),
                              ("mixed_default", default_mixed_schedule(), None),
                              ("mixed_learned", learned_schedule(), model)):
        r.run(mu=mu, sched=sched, energy=False, predictor=pred,
              lower_factor=lower_factor)                                            # warm-up
        L.nolsm_plan_get_timings(p, reset=True)
        L.nolsm_plan_set_timing(p, True)
        r.run(mu=mu, sched=sched, energy=False, predictor=pred, lower_factor=lower_factor)
        torch.cuda.synchronize()
        tm = L.nolsm_plan_get_timings(p, reset=True).as_dict()
        L.nolsm_plan_set_timing(p, False)
        st = r.stats_host()
        n3 = st["n"].astype(np.float64) ** 3
        flops = float((4.0 * n3 * (st["iters_lo"] + st["iters_fb"])).sum())
        rec = {"iters_lo_mean": float(st["iters_lo"].mean()),
               "iters_fb_mean": float(st["iters_fb"].mean()),
               "fallbacks": int(st["fell_back"].sum()),
               "failed": int((st["status"] != 0).sum()),
               "ms_sign": tm["ms_sign"], "ms_gemm": tm["ms_gemm"],
               "sign_tflops": flops / (tm["ms_sign"] * 1e-3) / 1e12 if tm["ms_sign"] > 0 else None}
        if ref is None:
            ref = (r.D.clone(), st["tr_dh"].copy())
        else:
            rec["max_abs_dD_vs_plain"] = float((r.D - ref[0]).abs().max().item())
            # energy of these molecules' columns per atom (the whole-system measure
            # restricted to the sample), and the largest single-molecule error
            rec["dE_per_atom_vs_plain"] = float(abs(np.sum(st["tr_dh"] - ref[1])) / atoms.sum())
            rec["max_sub_dE_per_atom_vs_plain"] = float(np.max(np.abs(st["tr_dh"] - ref[1]) / atoms))
        out[name] = rec
    del r
    return out


def features(runner, batch_index: int, mu: float) -> torch.Tensor:
    """nolsm_features for one batch of a Runner (runs the FP64 set-up if needed)."""
    K = len(runner.batches[batch_index])
    feat = torch.empty(K, NIN, device=runner.device)
    runner._bind(batch_index)
    L.nolsm_features(runner.plans[batch_index], mu, feat)
    return feat
