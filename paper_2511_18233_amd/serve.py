"""Continuous-batching request loop for gradient + NAC requests.

Shaped like surface-hopping dynamics: requests (one molecule geometry with its
orbitals and amplitudes, asking for some state gradients and NAC numerators)
arrive over time.  The server keeps a pool of slots; each slot owns one
library context on its own HIP stream (default priority) and keeps its device
regions between requests (grow-only), so the basis tables, integrals, MO blocks
and densities of a request stay resident while it runs and a steady stream of
similar sizes allocates nothing.

Admission: a request waits in FIFO order until a slot is free and the HBM it
needs -- the library's own sizing (ris_request_bytes), minus what the chosen
slot already holds -- fits in the server's budget next to what the other slots
hold.  When it fits only without the regions idle slots keep, those regions are
released (ris_ctx_release) and the request is admitted, so an idle pool never
blocks the head of the queue.  A request larger than the whole budget is
rejected.  The bytes each slot holds are read by the slot's own thread after
each request and kept on the host; the scheduler never calls into a context
that another thread may be using.  Work of different
slots overlaps on the device (one host thread per slot; the ctypes calls drop
the GIL while the library waits on its stream).

Each slot computes a request exactly as a lone call would (same kernels, same
ordered reductions), so results in the mix are bitwise equal to results alone.

The executor is pluggable so the scheduler can be exercised on the CPU.
"""
from __future__ import annotations

import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import md


@dataclass
class Request:
    rid: int
    arrival: float                  # seconds after the trace start
    Z: np.ndarray
    xyz: np.ndarray
    shell_atom: np.ndarray
    shell_l: np.ndarray
    shell_exp: np.ndarray
    C: np.ndarray                   # [nao][nmo]
    eps: np.ndarray
    nocc: int
    X: np.ndarray                   # [nstate][nvir][nocc]
    Y: np.ndarray | None
    sel: list                       # gradients wanted
    pairs: list                     # NAC numerators wanted
    j_p_on_heavy: bool = True
    velocity: np.ndarray | None = None  # [natm][3] nuclear velocities (for T_IJ)


@dataclass
class Result:
    rid: int
    grad: np.ndarray | None = None
    nac: np.ndarray | None = None
    arrival: float = 0.0
    admitted: float = 0.0
    done: float = 0.0
    slot: int = -1
    need_bytes: int = 0
    error: str | None = None
    tdc: np.ndarray | None = None   # T_IJ = g_IJ . v per requested pair (NAC numerators)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class GpuExecutor:
    """Runs one request through the C ABI on a slot's context and stream."""

    def __init__(self, slot: int, device: int, radius_bohr, precision: str, theta: float = 0.2,
                 alpha_J: float = 2.0, c_x: float = 0.25, hbm_budget: int = 0):
        import torch
        from .ris import RisContext
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.stream = torch.cuda.Stream(device=self.dev)
        self.ctx = RisContext(device, stream=self.stream, hbm_budget=hbm_budget)
        self.rad = radius_bohr
        self.precision = precision
        self.theta, self.alpha_J, self.c_x = theta, alpha_J, c_x

    def held_bytes(self) -> int:
        return self.ctx.bytes_held

    def release(self):
        """Free the slot's regions (called only while the slot is idle)."""
        self.ctx.release()

    def need_bytes(self, r: Request) -> int:
        from .ris import request_bytes
        return request_bytes(r.Z, r.shell_atom, r.shell_l, self.rad, r.C.shape[1], r.nocc, r.X.shape[0], 0,
                             len(r.sel) + len(r.pairs), self.theta, r.j_p_on_heavy, xyz=r.xyz,
                             shell_exp=r.shell_exp)

    def run(self, r: Request):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            C = torch.as_tensor(r.C, device=self.dev)
            eps = torch.as_tensor(r.eps, device=self.dev)
            X = torch.as_tensor(r.X, device=self.dev)
            Y = None if r.Y is None else torch.as_tensor(r.Y, device=self.dev)
            self.ctx.aux_build(r.Z, r.xyz, r.shell_atom, r.shell_l, r.shell_exp, self.rad, self.theta,
                               r.j_p_on_heavy)
            self.ctx.int3c(C, eps, r.nocc, self.alpha_J, self.c_x, precision=self.precision)
            g, n = self.ctx.grad_nac_contract(X, Y, r.sel, r.pairs)
            g = g.cpu().numpy() if len(r.sel) else None
            n = n.cpu().numpy() if len(r.pairs) else None
        return g, n

    def close(self):
        self.ctx.close()


class Server:
    """Slot pool + FIFO admission by HBM footprint + one worker thread per slot."""

    def __init__(self, executors, hbm_budget: int):
        self.ex = list(executors)
        self.budget = int(hbm_budget)
        self.lock = threading.Condition()
        self.free = list(range(len(self.ex)))
        self.reserved = [0] * len(self.ex)   # bytes a busy slot may grow to
        # bytes each slot holds, as its own thread last read them
        self.held = [int(e.held_bytes()) for e in self.ex]
        self.pending: list[Request] = []
        self.results: dict[int, Result] = {}
        self.t0 = 0.0
        self.jobs = [queue.Queue() for _ in self.ex]
        self.workers = [threading.Thread(target=self._work, args=(k,), daemon=True) for k in range(len(self.ex))]
        self.closed = False
        for w in self.workers:
            w.start()

    # -- admission ---------------------------------------------------------
    def _held(self, k: int) -> int:
        return self.held[k]

    def _release_idle(self, keep: int):
        """Release the regions of the idle slots other than `keep` (their
        threads wait on their queues, so nothing else touches them)."""
        for j in self.free:
            if j != keep and self.held[j] > 0 and hasattr(self.ex[j], "release"):
                self.ex[j].release()
                self.held[j] = 0

    def _try_admit(self):
        """Admit pending requests in FIFO order while a slot and memory allow."""
        while self.pending and self.free:
            r = self.pending[0]
            need = self.ex[self.free[0]].need_bytes(r)
            if need > self.budget:
                self.pending.pop(0)
                self.results[r.rid] = Result(r.rid, arrival=r.arrival, admitted=self.now(), done=self.now(),
                                             need_bytes=need, error="request larger than the HBM budget")
                self.lock.notify_all()
                continue
            # a slot keeps its regions: it needs max(held, need); the others hold
            # what they hold now or what their running request may grow to
            busy = [j for j in range(len(self.ex)) if j not in self.free]
            best = None
            for k in self.free:
                others = sum(max(self._held(j), self.reserved[j]) for j in range(len(self.ex)) if j != k)
                if others + max(self._held(k), need) <= self.budget:
                    best = k
                    break
            if best is None:
                # does it fit once the idle slots give their regions back?
                k = self.free[0]
                if sum(max(self._held(j), self.reserved[j]) for j in busy) + need <= self.budget:
                    self._release_idle(keep=k)
                    if sum(max(self._held(j), self.reserved[j]) for j in busy) + max(self._held(k), need) \
                            > self.budget and hasattr(self.ex[k], "release"):
                        self.ex[k].release()
                        self.held[k] = 0
                    best = k
                else:
                    return  # head of the queue waits (FIFO) until a busy slot finishes
            self.pending.pop(0)
            self.free.remove(best)
            self.reserved[best] = max(self._held(best), need)
            res = Result(r.rid, arrival=r.arrival, admitted=self.now(), slot=best, need_bytes=need)
            self.results[r.rid] = res
            self.jobs[best].put((r, res))

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, r: Request):
        with self.lock:
            self.pending.append(r)
            self._try_admit()

    def _work(self, k: int):
        while True:
            item = self.jobs[k].get()
            if item is None:
                return
            r, res = item
            try:
                res.grad, res.nac = self.ex[k].run(r)
                if r.velocity is not None and res.nac is not None:
                    res.tdc = np.array([md.time_derivative_coupling(n, r.velocity) for n in res.nac])
            except Exception as e:  # one failing request does not stop the others
                res.error = f"{type(e).__name__}: {e}"
            res.done = self.now()
            held = int(self.ex[k].held_bytes())   # this slot's own thread, after its request
            with self.lock:
                self.held[k] = held
                self.free.append(k)
                self.free.sort()
                self.reserved[k] = 0
                self._try_admit()
                self.lock.notify_all()

    # -- driving a trace ---------------------------------------------------
    def run_trace(self, requests, realtime: bool = True, timeout: float = 3600.0):
        """Submit requests at their arrival times; return {rid: Result}."""
        self.t0 = time.perf_counter()
        for r in sorted(requests, key=lambda q: q.arrival):
            if realtime:
                dt = r.arrival - self.now()
                if dt > 0:
                    time.sleep(dt)
            self.submit(r)
        deadline = time.perf_counter() + timeout
        with self.lock:
            while len(self.results) < len(requests) or any(x.done == 0.0 for x in self.results.values()):
                left = deadline - time.perf_counter()
                if left <= 0:
                    raise TimeoutError("trace did not finish")
                self.lock.wait(timeout=min(left, 1.0))
        return dict(self.results)

    def close(self, executors: bool = True):
        """Stop the worker threads; executors=False keeps the slots' contexts
        (and their warm regions) for another server."""
        if self.closed:
            return
        self.closed = True
        for q in self.jobs:
            q.put(None)
        for w in self.workers:
            w.join(timeout=60)
        if executors:
            for e in self.ex:
                if hasattr(e, "close"):
                    e.close()


def latency_stats(results) -> dict:
    lat = np.array([r.latency for r in results.values() if r.error is None])
    if lat.size == 0:
        return {"p50_ms": None, "p99_ms": None, "n": 0}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "n": int(lat.size)}


# --------------------------------------------------------------- traces --
def make_trace(n_requests: int, n_traj: int, rate_hz: float, seed: int = 1000, natm_range=(20, 120),
               nstate: int = 3, step_ang: float = 0.01, progress=None, random_phase: bool = True):
    """Surface-hopping-shaped trace: n_traj seeded trajectories of chain
    molecules (size uniform in natm_range), each request one step of its
    trajectory (previous geometry + N(0, step_ang) per coordinate, C = S^-1/2 Q
    recomputed, Q, eps and amplitudes fixed per trajectory), asking for the
    gradients of states 0 and 1 and the NAC numerator (0, 1); arrivals Poisson
    with the given rate.  progress(done, total), if given, is called every 32
    requests built.  Each request carries seeded nuclear velocities (the
    server returns T_IJ = g_IJ . v).  With random_phase, every step's
    amplitudes get an arbitrary sign per state, as an eigensolver would
    return them, and are then aligned to the previous step with
    md.phase_signs, as an MD driver does before using the NACs."""
    import molgen
    rng = np.random.default_rng(seed)
    trajs = []
    for t in range(n_traj):
        natm = int(rng.integers(natm_range[0], natm_range[1] + 1))
        p = molgen.make_chain_problem(natm, seed=seed + t, nstate=nstate, tda=False)
        S = molgen.overlap_matrix(p.mol)
        w, V = np.linalg.eigh(S)
        Q = (V * np.sqrt(w)) @ V.T @ p.C          # C = S^-1/2 Q  =>  Q = S^1/2 C
        trajs.append([p, Q, p.mol.xyz.copy(), None, None])  # ..., previous C, previous aligned X
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    bohr = molgen.ANGSTROM_TO_BOHR
    for k in range(n_requests):
        t = k % n_traj
        p, Q, xyz, C_prev, X_prev = trajs[t]
        xyz = xyz + rng.normal(0.0, step_ang * bohr, xyz.shape)
        trajs[t][2] = xyz
        mol = p.mol.with_xyz(xyz)
        S = molgen.overlap_matrix(mol)
        w, V = np.linalg.eigh(S)
        C = (V * (1.0 / np.sqrt(w))) @ V.T @ Q
        X, Y = p.X, p.Y
        if random_phase:
            sg = np.where(rng.random(X.shape[0]) < 0.5, -1.0, 1.0)
            X = sg[:, None, None] * X
            Y = None if Y is None else sg[:, None, None] * Y
            if X_prev is not None:
                fix = md.phase_signs(X_prev, X, C_prev, C, S, p.nocc)
                X = fix[:, None, None] * X
                Y = None if Y is None else fix[:, None, None] * Y
        trajs[t][3], trajs[t][4] = C, X
        vel = rng.normal(0.0, 1e-3, xyz.shape)
        reqs.append(Request(k, float(arrivals[k]), mol.Z, mol.xyz, mol.shell_atom, mol.shell_l, mol.shell_exp,
                            np.ascontiguousarray(C), p.eps, p.nocc, np.ascontiguousarray(X),
                            None if Y is None else np.ascontiguousarray(Y), [0, 1], [(0, 1)], velocity=vel))
        if progress is not None and (k + 1) % 32 == 0:
            progress(k + 1, n_requests)
    return reqs
