"""Throughput benchmark of the RBE2D hot path on one MI355X.

One step = one velocity-Verlet MD step of the 1e6-ion slab (800 x 800 x 40,
gamma_top = +0.95, gamma_bot = -0.95, M = 10, alpha = 0.3, r_c = 10, P = 500,
FP32 phases with FP64 accumulation): half kick + drift, a fresh k-set drawn
on the device, real space (cell list + erfc pairs with images), k-space
(structure factors, recalibration, force scatter), IBC, half kick.

Prints one JSON line: particle-steps/s, the live roofline of the dominant
kernel (HIP events around its launches in the timed region) and the CPU
oracle timed on a bounded sample of the same workload.  Side measurements
in the same line: the same MD step replayed from a captured HIP graph, the
64-replica batch (one graph-captured launch sequence per MD step for all
replicas) and the differentiable energy (forward + adjoint), each next to
the plain single-system FP64 path on the same GPU.
"""
import argparse
import subprocess
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RBE2D force+grad particle-steps/s at N=1e6 and 64-replica batch vs plain FP64"

# MI355X published peaks and the VALU issue rate (256 CUs x 64 lanes x 2.4 GHz)
PEAK_HBM_GBS = 8000.0
VALU_LANE_SLOTS = 256 * 64 * 2.4e9          # lane-instruction slots per second
# algorithmic VALU lane-slots per (particle, k) pair; a transcendental
# (v_sin/v_cos/v_exp/v_rsq/v_rcp) occupies 2 slots (half rate on gfx950)
SLOTS_SF = 16      # k.r (3), khat.r (1), sin+cos of both (8), 4 accumulating FMAs
SLOTS_FORCE = 16   # k.r (3), khat.r (1), angle offsets of the polar amplitudes (2), two sines (4),
                   # |cA| sin (1), X +- |cB| sin (2), 3 force FMAs
SLOTS_REAL = 22    # per pair within r_c: d2 (5), cutoff (1), rsqrt (2), exp (2+1), erfc fit
                   # (rcp 2 + 7 FMA), force factor (2); pairs outside r_c not counted
# the FP64 path (FP64 FMA issues at the FP32 rate on gfx950): software sincos
# on revolutions (quarter-turn reduction 4, 6 + 7 polynomial FMAs and products,
# t^2, 4 for the quadrant rotation: 21 per sincos)
SLOTS_SF64 = 51      # k.r and khat.r (5), two sincos (42), 4 accumulating FMAs
SLOTS_FORCE64 = 46   # phases (3), two half-turn-reduced sines (2 x 16) with their angle offsets
                     # and amplitudes (2 x 3), X +- Y (2), 3 force FMAs
SLOTS_REAL64 = 66    # per pair within r_c: d2 and cutoff (6), 1/sqrt refined twice (9), d and
                     # 1/r^2 (2), exp (25), 1/(1 + p x) refined twice (6), erfcx fit (12),
                     # products (6)
SLOTS = {"fp32": {"sf_pass": SLOTS_SF, "force_scatter": SLOTS_FORCE, "real_pairs": SLOTS_REAL},
         "fp64": {"sf_pass": SLOTS_SF64, "force_scatter": SLOTS_FORCE64, "real_pairs": SLOTS_REAL64}}


# HBM traffic of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# (profiles/), valid only while the kernel sources are the ones it was taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "real_pairs_large_md_traffic.txt")
TRAFFIC_SOURCES = ("realspace.hip", "rbe2d_internal.h", "devmath.h", "erfcx_fit.h", "api.hip")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_06333_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """Bytes per launch from the committed counter summary, or None when it is
    missing, for another kernel, or taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("bench_kernel") != kernel or kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


SIDE_STREAM = ("prep", "sf_pass", "assemble", "force_scatter")
BREAKDOWN_STEPS = 5   # profiled steps for the per-kernel breakdown, before the timed ones


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed MD steps (the workload's run is 100 steps)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=20, help="steps of the plain FP64 path (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=20000, help="particles in the oracle's rho sample")
    ap.add_argument("--cpu-targets", type=int, default=256,
                    help="oracle real-space targets (the oracle parallelises over targets in chunks of 16)")
    ap.add_argument("--side-steps", type=int, default=10, help="steps of each side measurement (0 = skip)")
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in launch heuristics")
    ap.add_argument("--parts-only", type=int, default=0,
                    help="only time this many force calls of each half alone (for counter runs)")
    ap.add_argument("--batch-only", type=int, default=0,
                    help="only run this many steps of the 64-replica batch (for kernel traces and counters)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only time the CPU oracle on its sample (prints one JSON object; no GPU)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    return ap.parse_args()


def expected_real_pairs(w, nz=4000):
    """Expected number of (target, source) pairs within r_c for uniform
    density in [margin, H - margin], real sources plus first images; a
    target's own image counts too (at distance 2 z below, 2 (H - z) above)."""
    rho = w.N / (w.Lx * w.Ly * (w.H - 2 * w.margin))
    z = np.linspace(w.margin, w.H - w.margin, nz)
    rc = w.r_c

    def cap_volume(zc, lo, hi):
        # volume of the ball of radius rc at height zc inside the layer lo < z < hi
        a = np.clip(lo - zc, -rc, rc)
        b = np.clip(hi - zc, -rc, rc)
        f = lambda t: math.pi * (rc * rc * t - t ** 3 / 3.0)  # noqa: E731
        return f(b) - f(a)

    lo, hi = w.margin, w.H - w.margin
    direct = cap_volume(z, lo, hi)
    img = cap_volume(-z, lo, hi) + cap_volume(2 * w.H - z, lo, hi)   # first-order images
    # a target's own image is within r_c below for z < r_c / 2, above for H - z < r_c / 2
    own = (min(max(0.5 * rc - lo, 0.0), hi - lo) + min(max(hi - (w.H - 0.5 * rc), 0.0), hi - lo)) / (hi - lo)
    return float(w.N * (rho * np.mean(direct + img) + own))


def run_md(R, torch, w, precision, steps, warmup, profile, use_graph=False, autotune=True):
    from paper_2405_06333_amd import inputs
    pos, q = inputs.sample(w)
    dev = "cuda"
    P_ = torch.as_tensor(pos, device=dev)
    Q_ = torch.as_tensor(q, device=dev)
    V_ = torch.zeros_like(P_)
    F_ = torch.zeros_like(P_)
    slab = R.Slab(**w.slab_kwargs(), precision=precision, n_max=w.N)
    slab.sample_kset(w.seed, 0)
    tuned = slab.autotune(P_, Q_) if autotune else None
    slab.forces(P_, Q_, out=F_)
    err = None
    if profile:
        # stochastic error of the k-space force at this P (Theorem 2.2) on the
        # starting configuration: rms of the per-particle variance estimate
        var = slab.force_variance(P_, Q_)
        err = {"kspace_force_sigma_rms": float(var.mean().sqrt().item()),
               "total_force_rms": float((F_ * F_).sum(dim=1).mean().sqrt().item())}
    zlo, zhi = w.margin, w.H - w.margin
    step = 1
    slab.md_run(P_, V_, Q_, F_, w.dt, zlo, zhi, w.seed, step, warmup, use_graph=use_graph)
    step += warmup
    torch.cuda.synchronize()
    slab.check()
    prof = None
    if profile:
        # per-kernel breakdown: a short run with every kernel class bracketed
        # by events (outside the timed region: the events of all classes add
        # tens of microseconds per step); then the timed run brackets only
        # the dominant caller-stream kernel
        nb = min(steps, BREAKDOWN_STEPS)
        slab.profile_enable(nb + 4)
        slab.profile_read()
        slab.md_run(P_, V_, Q_, F_, w.dt, zlo, zhi, w.seed, step, nb, use_graph=use_graph)
        step += nb
        breakdown = slab.profile_read()
        dom = dominant_kernel(breakdown)
        slab.profile_enable(steps + 4)
        slab.profile_classes([dom])
        slab.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slab.md_run(P_, V_, Q_, F_, w.dt, zlo, zhi, w.seed, step, steps, use_graph=use_graph)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if profile:
        prof = {"breakdown": breakdown, "dominant": dom, "timed": slab.profile_read()[dom]}
        slab.profile_enable(0)
    slab.check()
    finite = bool(torch.isfinite(F_).all().item() and torch.isfinite(P_).all().item())
    if profile:
        tuned = dict(err, launch_params=tuned)
    return (t1 - t0), prof, finite, tuned


def roofline_of(breakdown, precision, NP, pairs, dom=None, t_dom=None):
    """Per-kernel algorithmic fractions of the VALU issue peak from a breakdown
    {class: (ms, launches)}, and the roofline block of the dominant
    caller-stream kernel (its timed duration when given, else the breakdown's)."""
    slots = SLOTS[precision]
    units = {"sf_pass": NP, "force_scatter": NP, "real_pairs": pairs}
    fr = {}
    for k in ("sf_pass", "force_scatter", "real_pairs"):
        t, n = breakdown.get(k, (0.0, 0))
        if n:
            fr[k] = {"ms_per_launch": round(t / n, 4),
                     "valu_frac": round(slots[k] * units[k] / (t / n * 1e-3) / VALU_LANE_SLOTS, 4)}
    dom = dom or dominant_kernel(breakdown)
    if t_dom is None:
        t, n = breakdown[dom]
        t_dom = t / max(n, 1) * 1e-3
    roof = None
    if dom in slots:
        ach = slots[dom] * units[dom] / t_dom / 1e12
        peak = VALU_LANE_SLOTS / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": round(peak, 3),
                "unit": "Tlane-slot/s", "frac": round(ach / peak, 4), "traffic": None,
                "slots_per_unit": slots[dom],
                "concurrent_with": list(SIDE_STREAM) if dom == "real_pairs" else []}
    return roof, fr


def dominant_kernel(prof):
    """The k-space chain (with its force scatter) runs on a second stream,
    overlapped with the cell list and the pair kernel: its event durations
    include the time it shares the chip, so the dominant kernel is taken
    among the caller-stream kernels."""
    return max((k for k in prof if k not in SIDE_STREAM), key=lambda k: prof[k][0])


def run_parts(R, torch, w, precision, calls):
    """Each half of the force call alone on the same configuration: k-space
    (with IBC) and real space (cell list and pairs), every kernel class timed
    by HIP events.  Standalone durations of the structure-factor pass, the
    force scatter and the pair kernel (in the MD step they share the chip)."""
    from paper_2405_06333_amd import inputs
    pos, q = inputs.sample(w)
    P_ = torch.as_tensor(pos, device="cuda")
    Q_ = torch.as_tensor(q, device="cuda")
    slab = R.Slab(**w.slab_kwargs(), precision=precision, n_max=w.N)
    slab.sample_kset(w.seed, 0)
    out = {}
    for name, flags in (("kspace", R.KSPACE | R.IBC), ("real", R.REAL)):
        for _ in range(2):
            slab.forces(P_, Q_, flags=flags)
        torch.cuda.synchronize()
        slab.profile_enable(calls + 4)
        slab.profile_read()
        for _ in range(calls):
            slab.forces(P_, Q_, flags=flags)
        torch.cuda.synchronize()
        out[name] = slab.profile_read()
        slab.profile_enable(0)
    slab.check()
    return out


def timed(torch, fn, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def run_batch(R, torch, steps, autotune=True, plain=True):
    """64 replicas of uneven N and different contrasts: batched MD steps
    (graph replays) in FP32 phases and in FP64, against the plain path --
    one single-system FP64 handle per replica, stepped one after another."""
    from paper_2405_06333_amd import inputs
    ws = inputs.replicas()
    pos = np.concatenate([inputs.sample(w)[0] for w in ws])
    q = np.concatenate([inputs.sample(w)[1] for w in ws])
    counts = [w.N for w in ws]
    ntot = int(sum(counts))
    margin = min(w.margin for w in ws)
    pairs = sum(expected_real_pairs(w) for w in ws)
    out = {"workload": f"replicas: {len(ws)} slabs, N in [{min(counts)}, {max(counts)}], total {ntot}, "
                       f"2:1 ions, P={ws[0].P}, M={ws[0].M}", "particles": ntot,
           "expected_real_pairs": pairs}
    for prec in ("fp32", "fp64"):
        b = R.BatchedSlab([dict(w.slab_kwargs(), precision=prec, n_max=w.N) for w in ws])
        off = b.offsets(counts)
        P_ = torch.as_tensor(pos, device="cuda")
        Q_ = torch.as_tensor(q, device="cuda")
        V_ = torch.zeros_like(P_)
        b.sample_kset(ws[0].seed, 0)
        if autotune:
            out[f"tuned_{prec}"] = b.autotune(off, P_, Q_)
        F_ = b.forces(off, P_, Q_)
        b.md_run(off, P_, V_, Q_, F_, ws[0].dt, margin, ws[0].seed, 1, 2, use_graph=True)
        t = timed(torch, lambda: b.md_run(off, P_, V_, Q_, F_, ws[0].dt, margin, ws[0].seed, 3, steps,
                                          use_graph=True), 1)
        b.check()
        out[f"batch_{prec}_graph"] = ntot * steps / t
        out[f"batch_{prec}_ms_per_step"] = t * 1e3 / steps
        # per-kernel breakdown of the same step from eager steps with every
        # kernel class bracketed by events (a captured graph holds none)
        nb = 3
        b.profile_enable(nb + 4)
        b.profile_read()
        b.md_run(off, P_, V_, Q_, F_, ws[0].dt, margin, ws[0].seed, 3 + steps, nb, use_graph=False)
        bd = b.profile_read()
        b.profile_enable(0)
        b.check()
        roof, fr = roofline_of(bd, prec, ntot * ws[0].P, pairs)
        out[f"roofline_{prec}"] = roof
        out[f"kernels_{prec}"] = {k: {"ms_per_launch": (t_ / n_ if n_ else None), "launches": n_}
                                  for k, (t_, n_) in bd.items() if n_}
        for k, v in fr.items():
            out[f"kernels_{prec}"][k]["valu_frac"] = v["valu_frac"]
        del b
    if not plain:
        return out
    slabs = [R.Slab(**w.slab_kwargs(), precision="fp64", n_max=w.N) for w in ws]
    offs = np.concatenate([[0], np.cumsum(counts)])
    P_ = torch.as_tensor(pos, device="cuda")
    Q_ = torch.as_tensor(q, device="cuda")
    V_ = torch.zeros_like(P_)
    F_ = torch.zeros_like(P_)
    views = [(P_[offs[r]:offs[r + 1]], V_[offs[r]:offs[r + 1]], Q_[offs[r]:offs[r + 1]], F_[offs[r]:offs[r + 1]])
             for r in range(len(ws))]
    for r, s in enumerate(slabs):
        s.sample_kset(ws[r].seed, 0)
        if autotune:
            s.autotune(views[r][0], views[r][2])
        s.forces(views[r][0], views[r][2], out=views[r][3])

    def plain_steps(step0, n):
        for it in range(n):
            for r, s in enumerate(slabs):
                pv, vv, qv, fv = views[r]
                s.md_run(pv, vv, qv, fv, ws[r].dt, margin, ws[r].H - margin, ws[r].seed, step0 + it, 1)
    plain_steps(1, 1)
    n_plain = max(1, steps // 2)
    t = timed(torch, lambda: plain_steps(2, n_plain), 1)
    out["plain_fp64_per_replica"] = ntot * n_plain / t
    out["batch_fp32_vs_plain_fp64"] = out["batch_fp32_graph"] / out["plain_fp64_per_replica"]
    out["batch_fp64_vs_plain_fp64"] = out["batch_fp64_graph"] / out["plain_fp64_per_replica"]
    out["unit"] = "particle-steps/s"
    return out


def run_grad(R, torch, steps, autotune=True):
    """Differentiable energy: forward energy + hand-written adjoint (dE/dr,
    dE/dq, dE/dgamma, rho(k) recomputed) per step, against plain FP64 forces
    on the same system and k-set."""
    from paper_2405_06333_amd import inputs
    w = inputs.GRADIENT
    pos, q = inputs.sample(w)
    P_ = torch.as_tensor(pos, device="cuda")
    Q_ = torch.as_tensor(q, device="cuda")
    out = {"workload": f"gradient: N={w.N}, {w.Lx:g}x{w.Ly:g}x{w.H:g}, P={w.P}, M={w.M}", "unit": "particle-steps/s"}
    s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=w.N)
    s.set_kset(s.draw_kset(w.seed, 0))
    if autotune:
        out["tuned"] = s.autotune(P_, Q_)
    gE = torch.ones((), dtype=torch.float64, device="cuda")
    E = torch.empty(5, dtype=torch.float64, device="cuda")
    F = torch.empty_like(P_)

    def fwd_bwd():
        s.energy(P_, Q_, out=E)
        s.energy_backward(P_, Q_, gE)
    for _ in range(3):
        fwd_bwd()
    out["energy_fwd_bwd_fp64"] = w.N * steps / timed(torch, fwd_bwd, steps)
    fn = R.energy_function()
    gamma = torch.tensor([w.gamma_top, w.gamma_bot], dtype=torch.float64, device="cuda", requires_grad=True)
    Pg = P_.clone().requires_grad_(True)
    Qg = Q_.clone().requires_grad_(True)

    def autograd_step():
        e = fn.apply(Pg, Qg, gamma, s)
        e.backward()
    for _ in range(3):
        autograd_step()
    out["autograd_fp64"] = w.N * steps / timed(torch, autograd_step, steps)
    s.forces(P_, Q_, out=F)
    out["plain_fp64_forces"] = w.N * steps / timed(torch, lambda: s.forces(P_, Q_, out=F), steps)
    out["fwd_bwd_vs_plain_fp64"] = out["energy_fwd_bwd_fp64"] / out["plain_fp64_forces"]
    return out


def run_langevin(R, torch, w, precision, steps, autotune=True):
    """The large slab as charged soft spheres: positions thinned to a 0.9
    minimum distance, WCA ions (sigma = eps = 1) and walls (sigma = 0.5,
    eps = 1), BAOAB at kT = 1, gamma = 1; graph-replayed steps."""
    from paper_2405_06333_amd import inputs
    wt = w.with_(extra={"dmin": 0.9})
    pos, q = inputs.sample(wt)
    md = R.md_params(gamma=1.0, kT=1.0, sigma=1.0, eps=1.0, sigma_wall=0.5, eps_wall=1.0, wall_margin=0.1)
    P_ = torch.as_tensor(pos, device="cuda")
    Q_ = torch.as_tensor(q, device="cuda")
    V_ = torch.zeros_like(P_)
    slab = R.Slab(**w.slab_kwargs(), precision=precision, n_max=w.N)
    slab.sample_kset(w.seed, 0)
    if autotune:
        slab.autotune(P_, Q_)
    F_ = slab.forces(P_, Q_)
    slab.short_forces(P_, Q_, md, F=F_)
    slab.md_run_ex(P_, V_, Q_, F_, w.dt, md, w.seed, 1, 2, use_graph=True)
    t = timed(torch, lambda: slab.md_run_ex(P_, V_, Q_, F_, w.dt, md, w.seed, 3, steps, use_graph=True), 1)
    slab.check()
    kin = float((V_ ** 2).mean().item())
    return {"value": w.N * steps / t, "unit": "particle-steps/s", "steps": steps,
            "thermostat": "BAOAB Langevin kT=1 gamma=1", "short_range": "WCA ions sigma=1 eps=1, walls sigma=0.5",
            "kinetic_T_after": round(kin, 4), "finite": bool(torch.isfinite(P_).all().item())}


def run_surface(R, torch, w, precision, steps, sigma=0.01, autotune=True):
    """The large slab between two like-charged interfaces: density -sigma on
    z = 0 and on z = H, the ions' signs set so that their net charge cancels
    the sheets' (2 sigma Lx Ly more cations than anions); velocity-Verlet
    steps replayed from a hipGraph, as md_graph."""
    from paper_2405_06333_amd import inputs
    pos, _ = inputs.sample(w)
    excess = int(round(2.0 * sigma * w.Lx * w.Ly))
    if (w.N + excess) % 2:
        excess += 1
    q = np.where(np.arange(w.N) < (w.N + excess) // 2, 1.0, -1.0)
    P_ = torch.as_tensor(pos, device="cuda")
    Q_ = torch.as_tensor(q, device="cuda")
    V_ = torch.zeros_like(P_)
    slab = R.Slab(**w.slab_kwargs(), precision=precision, n_max=w.N)
    slab.set_surface_charges(-sigma, -sigma)
    slab.sample_kset(w.seed, 0)
    if autotune:
        slab.autotune(P_, Q_)
    F_ = slab.forces(P_, Q_)
    zlo, zhi = w.margin, w.H - w.margin
    slab.md_run(P_, V_, Q_, F_, w.dt, zlo, zhi, w.seed, 1, 2, use_graph=True)
    t = timed(torch, lambda: slab.md_run(P_, V_, Q_, F_, w.dt, zlo, zhi, w.seed, 3, steps, use_graph=True), 1)
    slab.check()
    return {"value": w.N * steps / t, "unit": "particle-steps/s", "steps": steps,
            "sigma_top": -sigma, "sigma_bot": -sigma, "net_ionic_charge": float(q.sum()),
            "finite": bool(torch.isfinite(P_).all().item() and torch.isfinite(F_).all().item())}


def copy_probe(torch, mib):
    """A plain device copy of `mib` MiB, three times: the reference reading
    for the HBM byte counters."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}), flush=True)


def cpu_baseline(w, n_sample, n_targets):
    """The CPU oracle on a bounded sample of the workload, scaled to one full
    step: its k-space pass (rho over the particles, then the force on each,
    both linear in the particle count) timed on n_sample particles, and its
    real-space sum (every real charge and image within r_c of the target,
    linear in the number of targets) timed for n_targets particles of the
    whole N-particle system."""
    from oracle import oracle as orc
    from paper_2405_06333_amd import inputs
    pos, q = inputs.sample(w)
    o = orc.Slab(Lx=w.Lx, Ly=w.Ly, H=w.H, g_top=w.gamma_top, g_bot=w.gamma_bot, alpha=w.alpha, rc=w.r_c,
                 M=w.M, P=w.P)
    n = orc.draw_kset(o, w.seed, 0)
    c = orc.rbe_weights(o, n)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sub = slice(0, n_sample)
    t0 = time.perf_counter()
    orc.kspace(o, pos[sub], q[sub], n, c)
    t_k = time.perf_counter() - t0
    rng = np.random.default_rng(5)
    tg = np.sort(rng.choice(w.N, n_targets, replace=False))
    t0 = time.perf_counter()
    orc.real_space(o, pos, q, targets=tg)
    t_r = time.perf_counter() - t0
    t_step = t_k * w.N / n_sample + t_r * w.N / n_targets
    return {
        "value": w.N / t_step,
        "unit": "particle-steps/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle k-space (rho and forces) over {n_sample} of the {w.N} particles ({t_k:.2f} s) "
                   f"and real space for {n_targets} sampled particles of the whole system ({t_r:.2f} s), "
                   f"scaled to one step of all {w.N} particles ({t_step:.3g} s/step)"),
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: runs on one GPU only (the kernels work on one GPU's share); --gpus {a.gpus} is not supported", file=sys.stderr)
        return 2
    if a.cpu_only:
        from paper_2405_06333_amd import inputs as _inputs
        print(json.dumps(cpu_baseline(_inputs.LARGE_MD, a.cpu_sample, a.cpu_targets)), flush=True)
        return 0
    # the single-threaded oracle figure, in a child process started before
    # this one touches the GPU: an eighth of the k-space sample and four
    # real-space targets at OMP_NUM_THREADS=1
    single = None
    if not (a.no_cpu_baseline or a.parts_only or a.batch_only or a.copy_mib):
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-only",
                            "--cpu-sample", str(max(1000, a.cpu_sample // 8)),
                            "--cpu-targets", str(max(2, a.cpu_targets // 64))],
                           env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0 and r.stdout.strip():
            single = json.loads(r.stdout.strip().splitlines()[-1])
        else:
            print(f"bench.py: single-threaded oracle run failed: {r.stderr[-400:]}", file=sys.stderr)
    import torch
    if a.copy_mib:
        copy_probe(torch, a.copy_mib)
        return 0
    if a.parts_only:
        from paper_2405_06333_amd import inputs as _inputs, rbe2d as _R
        _R.lib()
        alone = run_parts(_R, torch, _inputs.LARGE_MD, a.precision, a.parts_only)
        print(json.dumps({h: {k: {"ms_total": t, "launches": n} for k, (t, n) in v.items() if n}
                          for h, v in alone.items()}), flush=True)
        return 0
    from paper_2405_06333_amd import inputs, rbe2d as R
    R.lib()
    if a.batch_only:
        print(json.dumps(run_batch(R, torch, a.batch_only, autotune=not a.no_autotune, plain=False)), flush=True)
        return 0
    w = inputs.LARGE_MD
    secs, prof, finite, tuned = run_md(R, torch, w, a.precision, a.steps, a.warmup, profile=True,
                                       autotune=not a.no_autotune)
    ms_step = secs * 1e3 / a.steps
    value = w.N * a.steps / secs

    # per-kernel breakdown (separate profiled steps) and the roofline of the
    # dominant kernel (its events inside the timed region)
    bd = prof["breakdown"]
    kern = {k: {"ms_per_launch": (t / n if n else None), "launches": n} for k, (t, n) in bd.items()}
    for k in SIDE_STREAM:
        if k in kern:
            kern[k]["overlapped"] = True
    dom = prof["dominant"]
    t_dom = prof["timed"][0] / max(prof["timed"][1], 1) * 1e-3
    kern[dom]["ms_per_launch_timed"] = t_dom * 1e3
    kern[dom]["launches_timed"] = prof["timed"][1]
    NP = w.N * w.P
    pairs_real = expected_real_pairs(w)
    if dom == "sf_pass":
        work = SLOTS_SF * NP
    elif dom == "force_scatter":
        work = SLOTS_FORCE * NP
    elif dom == "real_pairs":
        work = SLOTS_REAL * pairs_real
    else:
        work = None
    roof = None
    if work is not None:
        ach = work / t_dom / 1e12
        peak = VALU_LANE_SLOTS / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": round(peak, 3),
                "unit": "Tlane-slot/s", "frac": round(ach / peak, 4), "traffic": measured_traffic(dom),
                "concurrent_with": list(SIDE_STREAM) if dom == "real_pairs" else []}
    for k, slots, units in (("sf_pass", SLOTS_SF, NP), ("force_scatter", SLOTS_FORCE, NP),
                            ("real_pairs", SLOTS_REAL, pairs_real)):
        t, n = bd[k]
        if n:
            kern[k]["valu_frac"] = round(slots * units / (t / n * 1e-3) / VALU_LANE_SLOTS, 4)
    t, n = bd["real_pairs"]
    if n:   # algorithmic HBM bytes of the pair kernel: read (x, y, z, q) + index, write F and phi
        kern["real_pairs"]["hbm_GBs"] = round(w.N * (32 + 4 + 32) / (t / n * 1e-3) / 1e9, 1)

    fp64 = None
    if a.fp64_steps > 0 and a.precision != "fp64":
        s64, p64, _, _ = run_md(R, torch, w, "fp64", a.fp64_steps, 1, profile=True, autotune=not a.no_autotune)
        fp64 = {"value": w.N * a.fp64_steps / s64, "unit": "particle-steps/s", "steps": a.fp64_steps,
                "ms_per_step": s64 * 1e3 / a.fp64_steps}
        t64 = p64["timed"][0] / max(p64["timed"][1], 1) * 1e-3
        fp64["roofline"], fp64["kernels"] = roofline_of(p64["breakdown"], "fp64", NP, pairs_real,
                                                         p64["dominant"], t64)
        if a.side_steps > 0:
            alone64 = run_parts(R, torch, w, "fp64", max(2, a.side_steps // 2))
            _, fp64["kernels_alone"] = roofline_of({**alone64["kspace"], "real_pairs": alone64["real"]["real_pairs"]},
                                                   "fp64", NP, pairs_real, dom="real_pairs")

    graph = batch = grad = langevin = surface = parts = None
    if a.side_steps > 0:
        alone = run_parts(R, torch, w, a.precision, a.side_steps)
        parts = {"calls": a.side_steps, "unit": "ms per launch"}
        for half, k, slots, units in (("kspace", "sf_pass", SLOTS_SF, NP), ("kspace", "force_scatter", SLOTS_FORCE, NP),
                                      ("real", "real_pairs", SLOTS_REAL, pairs_real),
                                      ("real", "cell_build", None, None)):
            t, n = alone[half].get(k, (0.0, 0))
            if not n:
                continue
            ms = t / n
            parts[k] = {"ms": round(ms, 4)}
            if slots:
                parts[k]["valu_frac"] = round(slots * units / (ms * 1e-3) / VALU_LANE_SLOTS, 4)
        # as many steps as the headline run: the capture, the opening pass and
        # the last (eager) step are spread over the same count
        sg, _, _, _ = run_md(R, torch, w, a.precision, a.steps, 1, profile=False, use_graph=True,
                             autotune=not a.no_autotune)
        graph = {"value": w.N * a.steps / sg, "unit": "particle-steps/s", "steps": a.steps}
        langevin = run_langevin(R, torch, w, a.precision, a.side_steps, autotune=not a.no_autotune)
        surface = run_surface(R, torch, w, a.precision, a.side_steps, autotune=not a.no_autotune)
        batch = run_batch(R, torch, a.side_steps, autotune=not a.no_autotune)
        grad = run_grad(R, torch, a.side_steps, autotune=not a.no_autotune)
    cpu = None if a.no_cpu_baseline else cpu_baseline(w, a.cpu_sample, a.cpu_targets)
    if cpu is not None and single is not None:
        cpu["single_thread"] = {"value": single["value"], "unit": single["unit"], "cores": single["cores"],
                                "sample": single["sample"]}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"large_md: N={w.N} 1:1 ions, {w.Lx:g}x{w.Ly:g}x{w.H:g} slab, "
                                f"gamma_top={w.gamma_top}, gamma_bot={w.gamma_bot}, M={w.M}, alpha={w.alpha}, "
                                f"r_c={w.r_c}, P={w.P}, velocity-Verlet dt={w.dt}"),
                   "precision": "FP32 phases and transcendentals, FP64 geometry and accumulation"
                   if a.precision == "fp32" else "FP64"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain_fp64_gpu": fp64,
        "md_graph": graph,
        "md_langevin_wca": langevin,
        "md_surface_charges": surface,
        "batched_replicas": batch,
        "differentiable": grad,
        "launch_params": tuned["launch_params"] if tuned else None,
        "kspace_force_error": ({"sigma_rms": tuned["kspace_force_sigma_rms"], "force_rms": tuned["total_force_rms"],
                                "P": w.P, "estimator": "sample variance of the per-k force terms (Theorem 2.2)"}
                               if tuned else None),
        "kernels": kern,
        "kernels_alone": parts,
        "finite": finite,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
