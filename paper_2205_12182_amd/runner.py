"""Drive the C ABI over a whole instance (device buffers from PyTorch).

The runner owns device copies of H0, S and D, the device pattern, and one plan
per batch of molecules.  All batches share one workspace (sized for the largest
batch) and are bound in turn; with persist=True each batch also keeps its set-up
(M_k, L^-1) in a buffer of its own, so that several runs at different chemical
potentials gather and set up every batch once.  Nothing here computes on the data.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L


def default_mixed_schedule(fixed_iters=None, panel_steps=1, prec="fp16", fallback_iters=60,
                           tol=0.1, cap=30, scale=None, lower=None, order=2, extra=1):
    """Low-precision bulk, then one FP32 Newton-Schulz step on the own-column panel.

    By default the bulk runs until ||X^2 - I||_F <= tol (every eigenvalue within
    |1 - x^2| <= 0.1) plus one more iteration; with fixed_iters it runs exactly
    that many.  Submatrices that miss the tolerance restart in plain FP32.  order 3
    takes the third-order polynomial step in the bulk.
    """
    phase = (prec, fixed_iters, 0.0, 0, order) if fixed_iters else (prec, cap, tol, extra, order)
    return L.schedule([phase], fallback_tol=tol, fallback_iters=fallback_iters,
                      panel_steps=panel_steps, scale=scale, lower=lower)


# Cap of the low-precision phase under the learned (scaled) schedule.  The scaled
# iteration reaches the tolerance from a lower bound l ~ 1e-6 in about 16 steps,
# the unscaled one in about 30 (the default cap), so both send the same kind of
# submatrix -- a tiny gap at mu, where FP16 rounding is amplified most -- to the
# FP32 restart instead of accepting a low-precision result.
LEARNED_CAP = 16


def learned_schedule(panel_steps=1, prec="fp16", fallback_iters=60, tol=0.1, extra=1):
    """The mixed schedule used with a learned lower bound (Runner.run(predictor=...))."""
    return default_mixed_schedule(panel_steps=panel_steps, prec=prec,
                                  fallback_iters=fallback_iters, tol=tol, cap=LEARNED_CAP,
                                  extra=extra)


def plain_fp32_schedule(tol=1e-3, extra=2, cap=100, order=2):
    """Plain FP32 Newton-Schulz (order 2) or third-order (order 3) iteration to
    convergence (no panel step, no fallback)."""
    return L.schedule([("fp32", cap, tol, extra, order)], fallback_iters=0, panel_steps=0)


def tuned_tile_policy():
    """big_tile_min_npad from the autotuner's table (data/tile_policy.json), or None
    (the library default) when there is no table or it was measured on another GPU
    architecture."""
    import json
    import os
    import warnings
    from .autotune import POLICY_PATH, policy_applies
    if not os.path.exists(POLICY_PATH):
        return None
    with open(POLICY_PATH) as fh:
        policy = json.load(fh)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    ok, note = policy_applies(policy, arch)
    if note and note not in _policy_notes:
        _policy_notes.add(note)
        warnings.warn(f"tile policy: {note}", stacklevel=2)
    return int(policy["big_tile_min_npad"]) if ok else None


_policy_notes = set()


class Runner:
    def __init__(self, inst, batch: int | None = None, mols=None, device="cuda",
                 big_tile_min_npad="tuned", setup_products=None, persist=False, groups=None,
                 overlap=False, factor_tiles=None, form=None):
        """groups: lists of molecules that share one submatrix each (combined
        submatrices, e.g. from nolsm_combine); then `batch` counts submatrices and
        the stats hold one record per group, in the order of `groups`.
        persist: True keeps every batch's gather and set-up in buffers of its own (a new
        chemical potential then reruns only the sign iteration); "auto" does so where
        those buffers fit the free device memory.
        overlap (with persist and several batches): two shared workspaces, and each
        step gathers and sets up batch i + 1 on a second stream while batch i
        iterates on the current one."""
        if not torch.cuda.is_available():
            raise RuntimeError("the NOLSM path runs on the GPU only")
        L.lib()
        self.inst = inst
        self.device = device
        self.H = torch.from_numpy(inst.H_val).to(device)
        self.S = torch.from_numpy(inst.S_val).to(device)
        self.D = torch.zeros_like(self.H)
        self.hpat = L.HostPattern(inst)
        self.dpat = L.DevicePattern(inst, device)
        if groups is not None:
            groups = [list(map(int, g)) for g in groups]
            self.groups = groups
            mols = np.asarray([k for g in groups for k in g], dtype=np.int32)
            units = groups
        else:
            mols = (np.arange(inst.nmol, dtype=np.int32) if mols is None
                    else np.asarray(mols, np.int32))
            self.groups = None
            units = mols
        self.mols = mols
        batch = len(units) if batch is None else batch
        self.batches = [units[i:i + batch] for i in range(0, len(units), batch)]
        if big_tile_min_npad == "tuned":
            big_tile_min_npad = tuned_tile_policy()
        self.big_tile_min_npad = big_tile_min_npad
        self.setup_products = setup_products
        self.factor_tiles = factor_tiles
        self.form = form
        self.persist = bool(persist)
        self.plans = self._create_plans()
        need = max(L.nolsm_plan_workspace_bytes(p) for p in self.plans)
        if persist == "auto":
            # keep every batch's set-up only where the set-up buffers fit beside the
            # workspace in 90% of the free device memory
            free, _ = torch.cuda.mem_get_info(torch.device(device))
            keep = sum(L.nolsm_plan_persist_bytes(p) for p in self.plans)
            if keep + need > 0.9 * free:
                for p in self.plans:
                    L.nolsm_plan_destroy(p)
                self.persist = False
                self.plans = self._create_plans()
                need = max(L.nolsm_plan_workspace_bytes(p) for p in self.plans)
        self.overlap = bool(overlap) and self.persist and len(self.plans) > 1
        self.workspaces = [torch.empty(need, dtype=torch.uint8, device=device)
                           for _ in range(2 if self.overlap else 1)]
        self.workspace = self.workspaces[0]
        self.persist_bufs = ([torch.empty(max(L.nolsm_plan_persist_bytes(p), 256),
                                          dtype=torch.uint8, device=device)
                              for p in self.plans] if self.persist else None)
        self.tables = [torch.empty(L.nolsm_plan_table_bytes(p), dtype=torch.uint8, device=device)
                       for p in self.plans]
        self.stats = [torch.zeros(len(b) * L.STATS_DTYPE.itemsize, dtype=torch.uint8,
                                  device=device) for b in self.batches]
        self.col_traces = torch.zeros(2 * inst.nmol, dtype=torch.float64, device=device)
        self.out2 = torch.zeros(2, dtype=torch.float64, device=device)
        self.bound = None
        self._feat = None
        self._side = None
        if len(self.plans) == 1:
            self._bind(0)
        if self.overlap:
            for i in range(len(self.plans)):     # first binds upload the tables (not async)
                self._bind(i)

    def _create_plans(self):
        if self.groups is not None:
            return [L.nolsm_plan_create_groups(self.hpat, b, self.big_tile_min_npad,
                                               self.setup_products, persist=self.persist,
                                               factor_tiles=self.factor_tiles, form=self.form)
                    for b in self.batches]
        return [L.nolsm_plan_create(self.hpat, b, self.big_tile_min_npad, self.setup_products,
                                    persist=self.persist, factor_tiles=self.factor_tiles,
                                    form=self.form)
                for b in self.batches]

    def __del__(self):
        try:
            for p in getattr(self, "plans", []):
                L.nolsm_plan_destroy(p)
        except Exception:     # interpreter shutdown
            pass

    def _bind(self, i):
        if self.bound != i:
            if self.persist:
                L.nolsm_plan_bind_persist(self.plans[i], self.tables[i],
                                          self.workspaces[i % len(self.workspaces)],
                                          self.persist_bufs[i])
            else:
                L.nolsm_plan_bind(self.plans[i], self.tables[i], self.workspace)
            self.bound = i

    @property
    def keeps_setup(self):
        """Whether every batch's set-up survives the other batches' runs."""
        return self.persist or len(self.plans) == 1

    def run_batch(self, i, mu, sched, predictor=None, lower_factor=0.5, regather=True):
        """Gather, sign iteration and write-back for batch i.

        predictor: a learn.ScheduleMLP; its prediction of log10 l_k from the batch's
        nolsm_features drives the scaled iteration (lower_factor is the safety
        factor applied to l_k).  regather=False reuses the batch's gather and set-up
        from its last run (only where they survive: keeps_setup).
        """
        self._bind(i)
        p = self.plans[i]
        if regather or not self.keeps_setup:
            L.nolsm_build_submatrices(p, self.dpat, self.H, self.S)
        self._sign_and_scatter(i, mu, sched, predictor, lower_factor)

    def _sign_and_scatter(self, i, mu, sched, predictor, lower_factor):
        p = self.plans[i]
        if predictor is not None:
            K = len(self.batches[i])
            if self._feat is None or self._feat.shape[0] < K:
                self._feat = torch.empty(K, L.NFEAT, device=self.device)
            feat = self._feat[:K]
            L.nolsm_features(p, mu, feat)
            y = predictor.predict(feat)
            s2 = L.Schedule.from_buffer_copy(sched)
            s2.lower_log10 = y.data_ptr()
            s2.lower_factor = lower_factor
            s2._keep = (getattr(sched, "_keep", None), y)
            sched = s2
        L.nolsm_sign_batched(p, mu, sched, self.stats[i])
        L.nolsm_scatter_density(p, self.dpat, self.D, self.H, self.S, self.stats[i])

    def run(self, mu=None, sched=None, energy=True, predictor=None, lower_factor=0.5,
            regather=True, serial=False):
        mu = self.inst.mu if mu is None else mu
        if self.overlap and regather and not serial:
            self._run_overlapped(mu, sched, predictor, lower_factor)
        else:
            for i in range(len(self.plans)):
                self.run_batch(i, mu, sched, predictor, lower_factor, regather)
        if energy:
            L.nolsm_energy(self.dpat, self.D, self.H, self.S, self.col_traces, self.out2)

    def _run_overlapped(self, mu, sched, predictor, lower_factor):
        """Batch i + 1's gather and set-up (second stream) run while batch i iterates
        (current stream).  Batches i and i + 2 share a workspace, so batch i + 2's
        gather waits for batch i's write-back.  Every kernel sees the same inputs as
        in the serial order, so the results are the same bit for bit."""
        main = torch.cuda.current_stream()
        if self._side is None:
            self._side = torch.cuda.Stream(device=self.device)
        side = self._side
        side.wait_stream(main)
        n = len(self.plans)
        ready = [torch.cuda.Event() for _ in range(n)]
        done = [torch.cuda.Event() for _ in range(n)]
        for i in range(n):
            self._bind(i)
            p = self.plans[i]
            with torch.cuda.stream(side):
                if i >= 2:
                    side.wait_event(done[i - 2])
                L.nolsm_build_submatrices(p, self.dpat, self.H, self.S)
                L.nolsm_setup_batched(p)
                ready[i].record(side)
            main.wait_event(ready[i])
            self._sign_and_scatter(i, mu, sched, predictor, lower_factor)
            done[i].record(main)
        main.wait_stream(side)

    def mu_search(self, n_target, mu_lo, mu_hi, tol=0.5, max_iter=40, sched=None,
                  predictor=None, lower_factor=0.5, on_trial=None):
        """Chemical potential with Tr(D S) = n_target (nolsm_mu_search_* bisection).

        Every trial runs the whole instance at the trial mu; the gather and set-up
        run at the first trial only when every batch keeps its set-up (persist or a
        single batch).  on_trial(t, mu, N, E) is called after each trial.
        Returns the search record, the trial history [(mu, Tr(DS), Tr(DH))] and
        whether it converged; D, out2 and the stats hold the result at the final mu.
        """
        m = L.nolsm_mu_search_init(n_target, mu_lo, mu_hi, tol, max_iter)
        hist = []
        while m.done == 0:
            mu = m.mu
            self.run(mu, sched, True, predictor, lower_factor, regather=not hist)
            e, ne = self.energy_host()
            hist.append((mu, ne, e))
            if on_trial is not None:
                on_trial(len(hist), mu, ne, e)
            L.nolsm_mu_search_update(m, ne)
        if m.mu != hist[-1][0]:      # cannot happen: the result is the last trial
            raise RuntimeError("mu search ended away from its last trial")
        return m, hist

    def capture(self, mu=None, sched=None, energy=True, predictor=None, lower_factor=0.5):
        """Record one whole step (every batch in turn, then the energy) as a HIP graph.

        Every plan is bound once before the capture (the table uploads are not
        capturable); inside the capture the batches take turns on the shared
        workspace with host-only binds.  graph.replay() repeats the step on the
        current contents of H, S with the captured mu and schedule.
        """
        for i in range(len(self.plans)):
            self._bind(i)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):            # warm-up outside the capture
            self.run(mu, sched, energy, predictor, lower_factor, serial=True)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):            # one stream: the batches in turn
            self.run(mu, sched, energy, predictor, lower_factor, serial=True)
        return graph

    def check(self):
        """Status of every batch (after the last run): the first failing batch's code
        (self.last_check_message names the batch and the failure) or OK."""
        first = L.OK
        msg = None
        for i, p in enumerate(self.plans):
            code = L.nolsm_check(p)
            if code != L.OK and first == L.OK:
                first, msg = code, f"batch {i}: {L.nolsm_last_error()}"
        self.last_check_message = msg
        return first

    def stats_host(self, i=None):
        torch.cuda.synchronize()
        idx = range(len(self.plans)) if i is None else [i]
        recs = [np.frombuffer(self.stats[j].cpu().numpy().tobytes(), dtype=L.STATS_DTYPE)
                for j in idx]
        return np.concatenate(recs)

    def energy_host(self):
        torch.cuda.synchronize()
        e = self.out2.cpu().numpy()
        return float(e[0]), float(e[1])

    # ------------------------------------------------------------- inspection (tests)
    def sub_info(self, batch, i):
        return L.nolsm_plan_query(self.plans[batch], i)

    def ws_view(self, off, count, dtype):
        """View `count` elements of `dtype` at byte offset `off` of the workspace."""
        itemsize = torch.tensor([], dtype=dtype).element_size()
        return self.workspace[off:off + count * itemsize].view(dtype)
