"""Benchmark: TDDFT-ris excited-state gradients + NAC numerators per second.

One step = the whole hot path on one seeded molecule, inputs resident in HBM:
ris_aux_build (aux basis, metric, Cholesky, inverse) -> ris_int3c ((mu nu|P)
and MO blocks) -> ris_response_matvec ((A+B) R_I and (A-B) L_I for every
state) -> ris_grad_nac_contract (gradients of every state and NAC numerators of
adjacent pairs, one call).
Default workload: 200-atom C/N/O chain (seed 2), 10 TDDFT states, 10 gradients
+ 9 NAC numerators per step.  `value` is the plain-FP64 rate.  The same line
carries the step in each reduced-precision mode (rate, Gamma roofline against
that mode's peak, max |d grad| and |d NAC| per result against the FP64 step),
a bounded serving replay (saturation throughput and p50/p99 latency under
Poisson arrivals, against the sequential FP64 loop) and the CPU oracle timed on
a bounded sample (all threads and one thread).

    python bench.py [--steps K] [--warmup W] [--workload chain200|chain60|ring12]
                    [--mode-steps S] [--serve N] [--no-cpu-baseline]

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "excited-state grads+NACs/s at 200 atoms; p50/p99 latency; vs plain FP64"
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 (matrix)
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 (matrix)
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the Gamma back-transform GEMM (listed lower tiles) from the
# FETCH_SIZE / WRITE_SIZE counter runs on the 199-atom workload (fetch scaled by
# 2.0, write by 1.0 after a 1 GiB copy calibration), averaged over the 28
# launches of a step; valid only for the GEMM source it was measured on (sha256
# prefix), null otherwise.
GAMMA_TRAFFIC = {"gemm_src_sha256": "38c892350b37dabc", "workload": "chain200", "bytes_per_launch": 17.41e9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name):
    import molgen
    prob = molgen.make_problem(name)
    jp = name != "ring12"
    ns = prob.nstate
    outs = [(i, i) for i in range(ns)] + [(i, i + 1) for i in range(ns - 1)]
    return prob, jp, outs


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample(prob, jp, outs, radii, scale=1.0):
    """Time the CPU oracle on bounded samples of the same workload and scale
    each stage linearly to one full step: (mu nu|P) for 24 s and 8 p auxiliary
    shells, the exchange weights of 24 K functions for one output pair, and
    the derivative contraction over the sampled functions for one output
    (about 10 s of host work at scale 1; `scale` shrinks the sample)."""
    from oracle import ris_oracle as O
    mol = prob.mol
    ao = O.ao_shells(mol)
    aux = O.aux_build(mol, radii, 0.2, jp)
    nJs, nKs = aux.J.n, aux.K.n
    nJ, nK = aux.J.nfunc, aux.K.nfunc
    # (1) three-centre integrals on 24 s + 8 p auxiliary shells
    ks = max(1, min(int(round(24 * scale)), nKs))
    kp = (max(1, min(int(round(8 * scale)), nJs - nKs)) if nJs > nKs else 0)
    pick = list(range(ks)) + list(range(nKs, nKs + kp))
    sub = O.Shells(aux.J.xyz[pick], aux.J.l[pick], aux.J.exp[pick], aux.J.atom[pick])
    t = time.perf_counter()
    t3 = O.int3c(ao, sub)
    t_int = time.perf_counter() - t
    nf = sub.nfunc
    full_int = t_int * (nJ + nK) / nf
    # (2) exchange weights (Gamma^P, V) for the ks sampled K (s) functions of one output pair
    RS, LA = O.ao_densities(prob.C, prob.nocc, prob.X[:2], None if prob.Y is None else prob.Y[:2])
    M2 = O.int2c(sub)
    Ssub = O.Setup(ao, aux, t3[:1], t3[:ks], M2[:1, :1], M2[:ks, :ks])
    t = time.perf_counter()
    O.pair_weights(Ssub, RS[0], RS[1], 0.0, 0.25)
    t_pw = time.perf_counter() - t
    full_pw = t_pw * nK / ks * 2 * len(outs)         # per K function, two pairs per output
    # (3) derivative contraction over the sampled aux shells, one output
    W = np.random.default_rng(0).standard_normal((1, nf, mol.nao, mol.nao))
    t = time.perf_counter()
    O.int3c_grad(ao, sub, mol.natm, W)
    t_dr = time.perf_counter() - t
    full_dr = t_dr * (nJ + nK) / nf * len(outs)     # the oracle contracts one output per pass here
    total = full_int + full_pw + full_dr
    return total, (f"int3c on {nf} of {nJ}+{nK} aux functions ({t_int:.1f} s), exchange weights for {ks} of "
                   f"{nK} K functions x 1 pair ({t_pw:.1f} s), derivative contraction on {nf} aux functions x 1 "
                   f"output ({t_dr:.1f} s)")


def cpu_baseline(prob, jp, outs, radii):
    """The oracle on the host: all threads (OpenMP integrals, BLAS), then one
    thread on an eighth-size sample; both scaled to one full step."""
    import threadpoolctl
    from oracle import ris_oracle as O
    O.lib()  # load the oracle's integrals (and their OpenMP runtime) first
    info = threadpoolctl.threadpool_info()
    blas = ", ".join(sorted({f"{d.get('internal_api')} {d.get('version')}" for d in info
                             if d.get("user_api") == "blas"}))
    nthreads = max([d.get("num_threads", 1) for d in info] + [1])
    total, what = oracle_sample(prob, jp, outs, radii)
    with threadpoolctl.threadpool_limits(limits=1):
        total1, what1 = oracle_sample(prob, jp, outs, radii, scale=0.125)
    return {
        "value": len(outs) / total, "unit": "grads+NACs/s", "cores": nthreads, "kind": "oracle",
        "sample": (f"{prob.mol.natm}-atom workload, {nthreads} threads: {what}; each scaled linearly to "
                   f"{len(outs)} outputs: est. {total:.0f} s per step"),
        "one_thread": {"value": len(outs) / total1, "sample": f"1 thread: {what1}; est. {total1:.0f} s per step"},
        "cpu_model": _cpu_model(), "blas": blas,
    }


def zvector_bench(ctx, prob, jp, radii, C, eps, nrhs, tol, maxit=20):
    """ris Z-vector solve (A+B)^ris Z = rhs for nrhs seeded right-hand sides on
    the workload (FP64), capped at maxit iterations: wall time, matvecs per
    second and the true relative residual reached.  With model orbitals the
    operator is indefinite and nearly singular at this size, so the cap, not
    the tolerance, ends the run; the rate is what is measured."""
    import time as _t
    import torch
    m = prob.mol
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    ctx.int3c(C, eps, prob.nocc, 2.0, 0.25)
    rng = np.random.default_rng(2024)
    rhs = torch.as_tensor(rng.standard_normal((nrhs,) + prob.X.shape[1:]), device=C.device)
    ctx.zvector_solve(rhs, tol=1e-2, maxit=2, allow_noconv=True)  # warm the regions
    torch.cuda.synchronize()
    t = _t.perf_counter()
    Z, it, res = ctx.zvector_solve(rhs, tol=tol, maxit=maxit, allow_noconv=True)
    torch.cuda.synchronize()
    dt = _t.perf_counter() - t
    out = {"nrhs": nrhs, "tol": tol, "iterations": it, "seconds": round(dt, 4),
           "matvecs_per_s": round(nrhs * (it + 1) / dt, 2), "true_rel_residual": res}
    log(f"[bench] zvector: {nrhs} rhs, {it} iterations, {dt:.2f} s, {out['matvecs_per_s']} matvecs/s, "
        f"residual {res:.2e}")
    return out


def zrhs_bench(ctx, prob, jp, radii, C, eps, X, Y, outs):
    """ris terms of the Z-vector right-hand side for the step's outputs (FP64):
    wall time of one ris_zrhs_contract call after ris_int3c."""
    import time as _t
    import torch
    m = prob.mol
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    ctx.int3c(C, eps, prob.nocc, 2.0, 0.25)
    G = ctx.zrhs_contract(X, Y, outs)  # warm the scratch
    torch.cuda.synchronize()
    t = _t.perf_counter()
    G = ctx.zrhs_contract(X, Y, outs, out=G)
    torch.cuda.synchronize()
    dt = _t.perf_counter() - t
    log(f"[bench] zrhs: {len(outs)} outputs in {dt:.3f} s")
    return {"outputs": len(outs), "seconds": round(dt, 4), "outputs_per_s": round(len(outs) / dt, 3)}


def davidson_bench(ctx, prob, jp, radii, C, eps, nroots, tol=1e-6, maxit=15):
    """TDA-ris excitation energies of the workload (FP64) by block Davidson,
    capped at maxit iterations: wall time per iteration and the lowest Ritz
    values reached (model orbitals make A^ris indefinite and slow to converge
    at this size, so the rate is what is measured)."""
    import time as _t
    import torch
    m = prob.mol
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
    ctx.int3c(C, eps, prob.nocc, 2.0, 0.25)
    torch.cuda.synchronize()
    t = _t.perf_counter()
    w, X, it = ctx.tda_davidson(nroots, tol=tol, maxit=maxit, allow_noconv=True)
    torch.cuda.synchronize()
    dt = _t.perf_counter() - t
    out = {"nroots": nroots, "tol": tol, "iterations": it, "seconds": round(dt, 4),
           "seconds_per_iteration": round(dt / max(it, 1), 4),
           "omega_ha": [round(float(x), 8) for x in w], "converged": it < maxit}
    log(f"[bench] davidson: {nroots} roots, {it} iterations, {dt:.2f} s, lowest {w[0]:.6f} Ha")
    return out


def run_steps(ctx, step, steps, warmup, label):
    """W untimed steps, then K timed ones with per-stage event timing on."""
    import torch
    for w in range(warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"[bench] {label} warmup {w}: {time.perf_counter() - t:.3f} s")
    ctx.set_profiling(True)
    times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        log(f"[bench] {label} step {k}: {times[-1]:.3f} s")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    stats = ctx.stage_stats()
    ctx.set_profiling(False)
    return times, total, stats


KERNELS = {
    "fp64": ("k_gemm<0,false,true,*> listed lower tiles, f64 (Gamma^P = (F_I W^P) F_J^T, batched over P)",
             PEAK_FP64_TFLOPS, 1.0),
    "fp32": ("k_gemm<1,false,true,*,float,float,double> listed lower tiles, f32 inputs "
             "(Gamma^P = (F_I W^P) F_J^T, batched over P)", PEAK_FP32_TFLOPS, 1.0),
    "bf16x3": ("k_pgemm<2,...> listed lower tiles, three bf16 products on pre-split bf16 planes (Gamma^P = "
               "(F_I W^P) F_J^T, batched over P; for two states Y^P F_J^T + F_J Y^P^T in one launch)", PEAK_BF16_TFLOPS, 3.0),
    "bf16x6": ("k_pgemm<3,...> listed lower tiles, six bf16 products on pre-split bf16 planes (Gamma^P = "
               "(F_I W^P) F_J^T, batched over P; for two states Y^P F_J^T + F_J Y^P^T in one launch)", PEAK_BF16_TFLOPS, 6.0),
}


def gamma_roofline(stats, precision, workload):
    """Roofline of the Gamma back-transform launches: algorithmic FLOPs per
    launch over their average event-timed duration, against the matrix-core
    peak of the type the launch multiplies in (split-BF16 modes count every
    BF16 product they issue)."""
    gms, gfl, gby, gn = stats["gamma"]
    if gn <= 0 or gms <= 0:
        return None
    kern, peak, nprod = KERNELS[precision]
    ach = gfl / gn / (gms * 1e-3 / gn) / 1e12 * nprod
    import hashlib
    src = os.path.join(ROOT, "paper_2511_18233_amd", "csrc", "ris_gemm.hip")
    same = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] == GAMMA_TRAFFIC["gemm_src_sha256"]
    traffic = GAMMA_TRAFFIC["bytes_per_launch"] if (same and workload == GAMMA_TRAFFIC["workload"]
                                                    and precision == "fp64") else None
    return {"bound": "mfma", "kernel": kern, "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 4), "traffic": traffic, "flops_per_launch": gfl / gn,
            "avg_launch_ms": gms / gn, "algorithmic_bytes_per_launch": gby / gn}


def stage_table(stats, steps):
    out = {}
    for name, (ms, fl, by, n) in stats.items():
        out[name] = {"ms_per_step": ms / steps, "launches": n,
                     "tflops": (fl / (ms * 1e-3) / 1e12) if ms > 0 and fl > 0 else None,
                     "gbs": (by / (ms * 1e-3) / 1e9) if ms > 0 and by > 0 else None}
    return out


def serve_bench(nreq, nslots, radii, mixed=("fp32", "bf16x6", "bf16x3")):
    """Serving replay (chain molecules 20-120 atoms from seeded trajectories,
    2 gradients + 1 NAC numerator each):
      * sequential FP64: one slot, requests back to back (the reference loop
        and the reference results);
      * saturation: every request queued at t = 0, through nslots FP64 slots
        (equal accuracy) and nslots slots in each mixed mode;
      * Poisson arrivals at 1.5x the sequential rate: p50/p99 latency of the
        sequential loop, of nslots FP64 slots and of nslots slots in the
        faster mixed mode.
    Each slot's regions are warmed on the largest requests first (grow-only
    regions: no allocation inside the timed replays).  Results of every run
    are compared with the sequential FP64 ones."""
    from paper_2511_18233_amd.serve import GpuExecutor, Server, latency_stats, make_trace
    log(f"[bench] serving: building a {nreq}-request trace")
    t = time.perf_counter()
    reqs = make_trace(nreq, max(1, nreq // 8), rate_hz=1.0, seed=1000,
                      progress=lambda k, n: log(f"[bench] serving: built {k}/{n} requests"))
    log(f"[bench] serving: trace built in {time.perf_counter() - t:.1f} s")
    big = sorted(reqs, key=lambda r: -r.C.shape[0])[:2]
    budget = 200 << 30
    pools = {}

    def pool(kind, n):
        key = (kind, n)
        if key not in pools:
            ex = [GpuExecutor(k, 0, radii, kind) for k in range(n)]
            for e in ex:            # grow each slot's regions to the largest requests
                for r in big:
                    e.run(r)
            pools[key] = ex
        return pools[key]

    def replay(kind, n, arrivals, realtime):
        for r, a in zip(reqs, arrivals):
            r.arrival = float(a)
        srv = Server(pool(kind, n), budget)
        t0 = time.perf_counter()
        rr = srv.run_trace(reqs, realtime=realtime)
        wall = time.perf_counter() - t0
        srv.close(executors=False)
        return rr, wall

    zero = np.zeros(nreq)
    r0, t_seq = replay("fp64", 1, zero, False)
    rate = nreq / t_seq
    log(f"[bench] serving sequential fp64: {rate:.2f} req/s")

    def dev(rr):
        return max(float(max(np.abs(rr[k].grad - r0[k].grad).max(), np.abs(rr[k].nac - r0[k].nac).max()))
                   for k in rr if rr[k].error is None)

    out = {"requests": nreq, "outputs_per_request": 3,
           "sizes_atoms": [int(min(r.Z.shape[0] for r in reqs)), int(max(r.Z.shape[0] for r in reqs))],
           "sequential_fp64": {"req_s": rate, "grads_nacs_s": 3 * rate}}
    sat = {}
    for kind in ("fp64",) + tuple(mixed):
        rr, wall = replay(kind, nslots, zero, False)
        errs = sum(1 for x in rr.values() if x.error)
        sat[kind] = {"slots": nslots, "req_s": nreq / wall, "grads_nacs_s": 3 * nreq / wall,
                     "vs_sequential_fp64": (nreq / wall) / rate, "max_abs_diff_vs_fp64": dev(rr), "errors": errs}
        log(f"[bench] serving saturation {kind} x{nslots}: {nreq / wall:.2f} req/s ({sat[kind]['vs_sequential_fp64']:.2f}x)")
    out["saturation"] = sat
    best = max(mixed, key=lambda k: sat[k]["req_s"])
    lam = 1.5 * rate
    gaps = np.random.default_rng(7).exponential(1.0 / lam, nreq)
    arr = np.cumsum(gaps) - gaps[0]
    pois = {"arrival_rate_req_s": lam}
    for name, kind, n in (("sequential_fp64", "fp64", 1), (f"fp64_x{nslots}", "fp64", nslots),
                          (f"{best}_x{nslots}", best, nslots)):
        rr, wall = replay(kind, n, arr, True)
        st = latency_stats(rr)
        pois[name] = {"req_s": nreq / wall, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                      "max_abs_diff_vs_fp64": dev(rr), "errors": sum(1 for x in rr.values() if x.error)}
        log(f"[bench] serving poisson {name}: {nreq / wall:.2f} req/s p50 {st['p50_ms']:.1f} ms "
            f"p99 {st['p99_ms']:.1f} ms")
    out["poisson"] = pois
    out["mixed_mode"] = best
    for ex in pools.values():
        for e in ex:
            e.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="chain200")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3", "bf16x6"],
                    help="arithmetic of the headline steps (default plain FP64)")
    ap.add_argument("--mode-steps", type=int, default=5,
                    help="timed steps per reduced-precision mode (0: skip the modes)")
    ap.add_argument("--serve", type=int, default=128,
                    help="requests of the serving replay (20-120 atoms; 0: skip)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-next", action="store_true",
                    help="skip the timing of the rows beyond the step (Z-vector right-hand side, Davidson, MINRES)")
    ap.add_argument("--davidson", type=int, default=10,
                    help="roots of the timed TDA-ris Davidson solve (0: skip)")
    ap.add_argument("--zvector", type=int, default=10,
                    help="right-hand sides of the timed ris Z-vector solve (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is "
              f"design-only for this path", file=sys.stderr)
        sys.exit(2)

    import torch
    import molgen
    from paper_2511_18233_amd import RisContext

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda", 0)
    radii = molgen.radii_bohr_table()
    log(f"[bench] building workload {args.workload}")
    prob, jp, outs = make_workload(args.workload)
    m = prob.mol
    ns = prob.nstate
    grads = [i for (i, j) in outs if i == j]
    pairs = [(i, j) for (i, j) in outs if i != j]
    C = torch.as_tensor(prob.C, device=dev).contiguous()
    eps = torch.as_tensor(prob.eps, device=dev).contiguous()
    X = torch.as_tensor(prob.X, device=dev).contiguous()
    Y = None if prob.Y is None else torch.as_tensor(prob.Y, device=dev).contiguous()
    R = (X + Y) if Y is not None else X.clone()
    L = (X - Y) if Y is not None else X.clone()
    g_out = torch.empty((len(grads), m.natm, 3), dtype=torch.float64, device=dev)
    n_out = torch.empty((len(pairs), m.natm, 3), dtype=torch.float64, device=dev)
    mv_out = torch.empty_like(R)
    torch.cuda.synchronize()
    ctx = RisContext(0)

    # the 500-atom solve runs for minutes: its outputs go out a few per call
    # with a progress line each (same results; the context blocks over the
    # auxiliary index by itself when the unblocked scratch does not fit)
    big = len(outs) > 19

    def make_step(precision):
        def step():
            ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radii, 0.2, jp)
            ctx.int3c(C, eps, prob.nocc, 2.0, 0.25, precision=precision)
            if big:
                torch.cuda.synchronize()
                log("[bench]   int3c + MO transforms done")
            ctx.response_matvec("A+B", R, mv_out)
            ctx.response_matvec("A-B", L, mv_out)
            if not big:
                ctx.grad_nac_contract(X, Y, grads, pairs, None, g_out, n_out)
                return
            torch.cuda.synchronize()
            log("[bench]   matvecs done")
            # gradient J together with the NAC (J-1, J): in one call they share
            # the exchange products of state J
            for k, J in enumerate(grads):
                pk = [q for q, (a, b) in enumerate(pairs) if b == J]
                assert len(pk) <= 1  # adjacent-pair NACs: at most one ends in state J
                ctx.grad_nac_contract(X, Y, [J], [pairs[q] for q in pk], None, g_out[k:k + 1],
                                      n_out[pk[0]:pk[0] + 1] if pk else n_out[:0])
                torch.cuda.synchronize()
                log(f"[bench]   gradient {J}" + (f" + NAC {pairs[pk[0]]}" if pk else "") + " done")
        return step

    log(f"[bench] natm={m.natm} nao={m.nao} nocc={prob.nocc} states={ns} outputs/step={len(outs)}")
    times, total, stats = run_steps(ctx, make_step(args.precision), args.steps, args.warmup, args.precision)
    per_stage = stage_table(stats, args.steps)
    for name, st in per_stage.items():
        log(f"[bench] stage {name:7s} {st['ms_per_step']:10.2f} ms/step  launches={st['launches']}"
            + (f"  {st['tflops']:7.2f} TFLOP/s" if st["tflops"] else ""))
    roof = gamma_roofline(stats, args.precision, args.workload)
    # whole step: the algorithmic FLOPs the stage timers count, over the measured step time
    step_fl = sum(fl for (ms, fl, by, n) in stats.values()) / args.steps
    step_roof = {"achieved_tflops": round(step_fl / (total / args.steps) / 1e12, 3),
                 "peak": PEAK_FP64_TFLOPS,
                 "unit": "TFLOP/s", "algorithmic_flops_per_step": step_fl}
    # a fraction of the FP64 peak only for the FP64 step (the reduced modes mix
    # FP64 stages with stages on other matrix-core types)
    step_roof["frac"] = (round(step_roof["achieved_tflops"] / step_roof["peak"], 4)
                         if args.precision == "fp64" else None)
    g_ref = g_out.cpu().numpy().copy()
    n_ref = n_out.cpu().numpy().copy()

    # translational invariance of the gradients (sum over atoms vanishes)
    inv = float(np.abs(g_ref.sum(1)).max()) if len(grads) else 0.0
    from paper_2511_18233_amd.ris import request_bytes
    plan0 = request_bytes(m.Z, m.shell_atom, m.shell_l, radii, m.nao, prob.nocc, ns, ns, len(outs), xyz=m.xyz,
                          shell_exp=m.shell_exp)
    hbm = {"held_gb": round(ctx.bytes_held / 1e9, 2),
           "unblocked_plan_gb": round(plan0 / 1e9, 2)}
    log(f"[bench] translational invariance max |sum_A grad| {inv:.2e}; HBM held {hbm['held_gb']} GB "
        f"(unblocked plan {hbm['unblocked_plan_gb']} GB)")

    value = len(outs) * args.steps / total
    tsorted = np.sort(np.array(times))
    res = {
        "metric": METRIC, "value": round(value, 4), "unit": "grads+NACs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * total / args.steps, 2),
        "ms_per_step_min": round(1e3 * float(tsorted[0]), 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 (exchange contractions), f64 elsewhere",
                  "bf16x3": "bf16x3 (exchange contractions), f64 elsewhere",
                  "bf16x6": "bf16x6 (exchange contractions), f64 elsewhere"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: seeded C/N/O chain, {m.natm} atoms, nao={m.nao}, "
                               f"nocc={prob.nocc}, nauxJ={ctx.nJ}, nauxK={ctx.nK}, {ns} TDDFT states, "
                               f"{len(grads)} gradients + {len(pairs)} NAC numerators per step",
                   "natm": m.natm, "nao": m.nao, "nocc": prob.nocc, "nauxJ": ctx.nJ, "nauxK": ctx.nK,
                   "nstate": ns, "outputs_per_step": len(outs), "precision": args.precision},
        "step_latency_ms": {"p50": round(1e3 * float(np.percentile(tsorted, 50)), 2),
                            "p99": round(1e3 * float(np.percentile(tsorted, 99)), 2),
                            "min": round(1e3 * float(tsorted[0]), 2)},
        "roofline": roof,
        "step_roofline": step_roof,
        "stages": per_stage,
        "grad_sum_max": inv,
        "hbm": hbm,
    }
    mv = per_stage.get("matvec")
    if mv and mv["ms_per_step"] > 0:
        res["matvecs_per_s"] = round(2 * ns / (mv["ms_per_step"] * 1e-3), 2)

    # the same step in each reduced-precision mode, against the FP64 step's outputs
    if args.mode_steps > 0 and args.precision == "fp64":
        modes = {}
        # the exchange contractions in each reduced precision; "+transforms": the
        # MO transforms of (mu nu|P) in it as well
        for mode in ("fp32", "bf16x6", "bf16x3", "fp32+transforms", "bf16x3+transforms"):
            mt, mtot, mst = run_steps(ctx, make_step(mode), args.mode_steps, 1, mode)
            g = g_out.cpu().numpy()
            n = n_out.cpu().numpy()
            per = [float(np.abs(g[k] - g_ref[k]).max()) for k in range(len(grads))] + \
                  [float(np.abs(n[k] - n_ref[k]).max()) for k in range(len(pairs))]
            rate = len(outs) * args.mode_steps / mtot
            modes[mode] = {
                "grads_nacs_per_s": round(rate, 4), "ms_per_step": round(1e3 * mtot / args.mode_steps, 2),
                "ms_per_step_min": round(1e3 * min(mt), 2), "steps": args.mode_steps,
                "vs_plain_fp64": round(rate / value, 4),
                "roofline": gamma_roofline(mst, mode.split("+")[0], args.workload),
                "max_abs_dgrad_vs_fp64": max(per[:len(grads)]) if grads else None,
                "max_abs_dnac_vs_fp64": max(per[len(grads):]) if pairs else None,
                "max_abs_grad": float(np.abs(g_ref).max()),
                "per_result_max_abs_d": [round(x, 15) for x in per],
                "stages_ms_per_step": {k: round(v["ms_per_step"], 2) for k, v in stage_table(mst, args.mode_steps).items()},
            }
            log(f"[bench] {mode}: {rate:.2f} grads+NACs/s ({rate / value:.2f}x fp64), max|dgrad| "
                f"{modes[mode]['max_abs_dgrad_vs_fp64']:.2e} max|dNAC| {modes[mode]['max_abs_dnac_vs_fp64']:.2e}")
        res["precision_modes"] = modes
    if not args.no_next and not big:
        # the rows beyond the step, timed on the same workload (FP64)
        res["zrhs"] = zrhs_bench(ctx, prob, jp, radii, C, eps, X, Y, outs)
        if args.davidson > 0:
            res["davidson"] = davidson_bench(ctx, prob, jp, radii, C, eps, args.davidson, maxit=10)
        if args.zvector > 0:
            res["zvector"] = zvector_bench(ctx, prob, jp, radii, C, eps, args.zvector, 1e-8)
    ctx.close()
    if args.serve > 0:
        sv = serve_bench(args.serve, args.serve_slots, radii)
        res["serving"] = sv
        best = sv["mixed_mode"]
        pb = sv["poisson"][f"{best}_x{args.serve_slots}"]
        # the metric's latency: requests of the serving replay under Poisson arrivals
        res["latency_ms"] = {"p50": round(pb["p50_ms"], 2), "p99": round(pb["p99_ms"], 2),
                             "of": f"serving replay, {best} x{args.serve_slots} slots, Poisson "
                                   f"{sv['poisson']['arrival_rate_req_s']:.1f} req/s",
                             "sequential_fp64_p50": round(sv["poisson"]["sequential_fp64"]["p50_ms"], 2),
                             "sequential_fp64_p99": round(sv["poisson"]["sequential_fp64"]["p99_ms"], 2)}
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(prob, jp, outs, radii)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
