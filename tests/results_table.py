"""Measure the per-workload results table: GPU throughput of each path, its
force error against the oracle on the same inputs and k-set, and the oracle's
own throughput on the host cores.  Test infrastructure, run by hand on a GPU
machine (python -m tests.results_table); prints a markdown table.

Small workloads are timed per force evaluation (eager calls, launch-latency
bound); errors are over all particles there, and over sampled particles of
the replica batch and of the 1e6-ion slab (the oracle's per-target forces)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2405_06333_amd import inputs  # noqa: E402
from tests.gpu_common import oracle_slab, rel_rms, to_dev  # noqa: E402


def gpu_rate(torch, fn, n_particles, calls):
    """particle-steps/s of fn() (one evaluation of n_particles)."""
    fn()
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(calls):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return n_particles * calls / (t0.elapsed_time(t1) * 1e-3)


def oracle_rate(orc, o, pos, q, n, targets=None):
    """(result, particle-steps/s of the oracle) for one evaluation; with
    targets, the k-space sums still run over all particles and the rate is
    per evaluated target."""
    t = time.perf_counter()
    ref = orc.evaluate(o, pos, q, n, targets=targets)
    dt = time.perf_counter() - t
    n_eval = len(pos) if targets is None else len(targets)
    return ref, n_eval / dt


def main():
    import torch
    from oracle import oracle as orc
    from paper_2405_06333_amd import rbe2d as R
    assert torch.cuda.is_available()
    R.lib()
    orc.lib()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rows = []

    def single(w, precision, calls):
        pos, q = inputs.sample(w)
        s = R.Slab(**w.slab_kwargs(), precision=precision, n_max=w.N)
        n = s.draw_kset(w.seed, 0)
        s.set_kset(n)
        P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
        F = s.forces(P_, Q_)
        s.check()
        rate = gpu_rate(torch, lambda: s.forces(P_, Q_, want_energy=True), w.N, calls)
        return s, pos, q, n, F.cpu().numpy(), rate

    # C1, C2: full evaluations
    for w, precs, calls in ((inputs.SMALL_FP64, ("fp64",), 200), (inputs.DIELECTRIC, ("fp64", "fp32"), 100)):
        ref = cpu = None
        for prec in precs:
            s, pos, q, n, F, rate = single(w, prec, calls)
            if ref is None:
                ref, cpu = oracle_rate(orc, oracle_slab(orc, w, s.Lz_ext), pos, q, n)
            rows.append((w.name, f"{prec} forces + energy", rate, rel_rms(F, ref.F), cpu))
            print(rows[-1], flush=True)

    # C3: the replica batch, sampled particles of every replica
    ws = inputs.replicas()
    pos = np.concatenate([inputs.sample(w)[0] for w in ws]).reshape(-1, 3)
    q = np.concatenate([inputs.sample(w)[1] for w in ws])
    counts = [w.N for w in ws]
    rng = np.random.default_rng(5)
    for prec in ("fp32", "fp64"):
        b = R.BatchedSlab([dict(w.slab_kwargs(), precision=prec, n_max=w.N) for w in ws])
        off = b.offsets(counts)
        b.sample_kset(ws[0].seed, 0)
        kset = b.get_kset()
        P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
        F = b.forces(off, P_, Q_).cpu().numpy()
        b.check()
        rate = gpu_rate(torch, lambda: b.forces(off, P_, Q_, want_energy=True), int(off[-1]), 20)
        errs, cpu_t, cpu_n = [], 0.0, 0
        for r, w in enumerate(ws):
            tg = np.sort(rng.choice(w.N, 8, replace=False))
            t = time.perf_counter()
            ref = orc.evaluate(oracle_slab(orc, w, b.Lz_ext[r]), pos[off[r]:off[r + 1]], q[off[r]:off[r + 1]],
                               kset[r], targets=tg)
            cpu_t += time.perf_counter() - t
            cpu_n += len(tg)
            errs.append((F[off[r] + tg], ref.F))
        err = rel_rms(np.concatenate([e[0] for e in errs]), np.concatenate([e[1] for e in errs]))
        rows.append(("replicas", f"{prec} batch forces + energy (64 slabs, {int(off[-1])} ions)", rate, err,
                     cpu_n / cpu_t))
        print(rows[-1], flush=True)

    # C4: the 1e6-ion slab, sampled particles
    w = inputs.LARGE_MD
    tg = np.sort(np.random.default_rng(11).choice(w.N, 48, replace=False))
    ref = cpu = None
    for prec in ("fp32", "fp64"):
        s, pos, q, n, F, rate = single(w, prec, 10)
        if ref is None:
            ref, cpu = oracle_rate(orc, oracle_slab(orc, w, s.Lz_ext), pos, q, n, targets=tg)
        rows.append((w.name, f"{prec} forces + energy", rate, rel_rms(F[tg], ref.F), cpu))
        print(rows[-1], flush=True)
        del s

    # C5: energy and its adjoint
    w = inputs.GRADIENT
    pos, q = inputs.sample(w)
    s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=w.N)
    n = s.draw_kset(w.seed, 0)
    s.set_kset(n)
    P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
    g = torch.tensor(1.0, dtype=torch.float64, device="cuda")

    def fwd_bwd():
        s.energy(P_, Q_)
        return s.energy_backward(P_, Q_, g)

    dr, dq, _ = fwd_bwd()
    s.check()
    rate = gpu_rate(torch, fwd_bwd, w.N, 20)
    t = time.perf_counter()
    o = oracle_slab(orc, w, s.Lz_ext)
    ref = orc.evaluate(o, pos, q, n)
    cpu = w.N / (time.perf_counter() - t)
    err = max(rel_rms(dr.cpu().numpy(), -ref.F), rel_rms(dq.cpu().numpy(), ref.phi))
    rows.append((w.name, "fp64 energy + backward (dE/dr, dE/dq, dE/dgamma)", rate, err, cpu))
    print(rows[-1], flush=True)

    print()
    print(f"| Workload | Path | GPU particle-steps/s | rel-RMS force error vs oracle | "
          f"oracle particle-steps/s ({threads} threads) |")
    print("|---|---|---|---|---|")
    for name, path, rate, err, cpu in rows:
        print(f"| {name} | {path} | {rate:.3g} | {err:.1e} | {cpu:.3g} |")


if __name__ == "__main__":
    main()
