"""GPU parity of the MD steps whose ions cross the reflecting walls.

Ions start 1e-3 from a wall moving towards it (v_z = -+20), and a few fly
fast enough (|v_z| dt > z_hi - z_lo) to fold twice in one step.  Every
integrator path that folds z is compared element by element with the
oracle's step (``oracle.baoab_step``, whose wall fold is pinned against
repeated mirror reflections and the closed-form triangle wave):
  - rbe2d_md_run, eager and replayed from a captured graph (FP64, FP32);
  - rbe2d_batch_md_run over two systems with different heights;
  - rbe2d_md_run_ex (BAOAB Langevin with WCA ions and walls), eager and graph.
Tolerances: positions 1e-11 absolute, velocities 1e-11 and forces 1e-9
relative RMS (FP64); the FP32-phase path 1e-5 on forces.
"""
import numpy as np
import pytest

from paper_2405_06333_amd import inputs
from tests.gpu_common import oracle_slab, rel_rms, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def R():
    from paper_2405_06333_amd import rbe2d
    rbe2d.lib()
    return rbe2d


def wall_start(pos, zlo, zhi, dt, seed, n_near=40, n_fast=6):
    """Velocities (normal, sd 1) with n_near ions put 1e-3 inside each wall
    and moving at it with |v_z| = 20, and n_fast ions whose |v_z| dt exceeds
    2 (zhi - zlo), so that they fold at least twice in every step."""
    rng = np.random.default_rng(seed)
    pos = pos.copy()
    vel = rng.normal(0.0, 1.0, pos.shape)
    idx = rng.permutation(len(pos))
    lo, hi, fast = idx[:n_near], idx[n_near:2 * n_near], idx[2 * n_near:2 * n_near + n_fast]
    pos[lo, 2] = zlo + 1e-3
    vel[lo, 2] = -20.0
    pos[hi, 2] = zhi - 1e-3
    vel[hi, 2] = 20.0
    W = zhi - zlo
    vel[fast, 2] = rng.choice([-1.0, 1.0], n_fast) * rng.uniform(2.05, 2.9, n_fast) * W / dt
    vel[fast, 0] = rng.normal(0.0, 3.0, n_fast) / dt      # several periods in x as well
    return pos, vel, lo, hi, fast


def crossings(p_before, v_before, dt, zlo, zhi, F):
    """Per ion, how many walls its drift crosses in the coming step (the
    drift uses v after the opening half kick)."""
    z = p_before[:, 2] + dt * (v_before[:, 2] + 0.5 * dt * F[:, 2])
    W = zhi - zlo
    return np.floor((z - zlo) / W).astype(int)


def oracle_vv(orc, o, w, pos, vel, q, F, dt, zlo, zhi, seed, step0, n_steps, stream_of):
    p, v, Fc = pos, vel, F
    folds = []
    for st in range(step0, step0 + n_steps):
        n = orc.draw_kset(o, seed, stream_of(st))
        folds.append(crossings(p, v, dt, zlo, zhi, Fc))
        p, v, Fc = orc.baoab_step(p, v, Fc, dt, 0.0, 0.0, np.zeros_like(p), w.Lx, w.Ly, zlo, zhi,
                                  lambda x: orc.evaluate(o, x, q, n).F)
    return p, v, Fc, np.stack(folds)


def assert_walls_hit(folds, lo, hi, fast):
    """The compared steps did fold: the near ions crossed their wall in the
    first step, the fast ones folded at least twice in every step."""
    assert np.all(folds[0][lo] == -1) and np.all(folds[0][hi] == 1)
    assert np.all(np.abs(folds[:, fast]) >= 2)


@pytest.mark.parametrize("precision,use_graph", [("fp64", False), ("fp64", True), ("fp32", True)])
def test_md_run_wall_crossings_match_oracle(torch, R, orc, precision, use_graph):
    w = inputs.small_random(71, 500, L=12.0, H=6.0, gamma_top=0.6, gamma_bot=-0.4, alpha=0.9, r_c=4.0, P=40,
                            M=4, margin=0.5)
    pos, q = inputs.sample(w)
    seed, dt, step0, zlo, zhi = 19, 2e-3, 2, 0.3, w.H - 0.3
    pos, vel, lo, hi, fast = wall_start(pos, zlo, zhi, dt, 5)
    s = R.Slab(**w.slab_kwargs(), precision=precision, n_max=w.N)
    o = oracle_slab(orc, w, s.Lz_ext)
    F0 = orc.evaluate(o, pos, q, s.draw_kset(seed, 0)).F
    P_, V_, Q_, F_ = to_dev(torch, pos), to_dev(torch, vel), to_dev(torch, q), to_dev(torch, F0)
    print(f"md_run walls {precision} graph={use_graph} N={w.N}", flush=True)
    s.md_run(P_, V_, Q_, F_, dt, zlo, zhi, seed, step0, 4, use_graph=use_graph)
    s.check()
    p, v, F, folds = oracle_vv(orc, o, w, pos, vel, q, F0, dt, zlo, zhi, seed, step0, 4, lambda st: st)
    assert_walls_hit(folds, lo, hi, fast)
    pg, vg, Fg = P_.cpu().numpy(), V_.cpu().numpy(), F_.cpu().numpy()
    assert np.all((pg[:, 2] >= zlo) & (pg[:, 2] <= zhi))
    if precision == "fp64":
        assert np.abs(pg - p).max() <= 1e-11
        assert rel_rms(vg, v) <= 1e-11
        assert rel_rms(Fg, F) <= 1e-9
    else:
        # FP32-phase forces move the positions by about dt^2 times their
        # error; the forces left in F are those of the final positions
        assert np.abs(pg - p).max() <= 1e-6
        ref = orc.evaluate(o, pg, q, s.get_kset()).F
        assert rel_rms(Fg, ref) <= 1e-5
    # the sign of v_z after the last step follows the oracle's folds
    assert np.array_equal(np.sign(vg[fast, 2]), np.sign(v[fast, 2]))


def test_batch_md_run_wall_crossings_match_oracle(torch, R, orc):
    """Two systems of different height: the wall margin applies to each."""
    ws = [inputs.small_random(72, 300, L=11.0, H=6.0, gamma_top=0.5, gamma_bot=0.5, alpha=0.9, r_c=4.0, P=30,
                              M=3, margin=0.5),
          inputs.small_random(73, 257, L=10.0, H=4.5, gamma_top=-0.7, gamma_bot=0.8, alpha=1.0, r_c=3.5, P=30,
                              M=5, margin=0.5)]
    seed, dt, step0, margin = 23, 2e-3, 1, 0.25
    starts = []
    for r, w in enumerate(ws):
        pos, q = inputs.sample(w)
        pos, vel, lo, hi, fast = wall_start(pos, margin, w.H - margin, dt, 10 + r, n_near=25, n_fast=4)
        starts.append((pos, q, vel, lo, hi, fast))
    pos = np.concatenate([s_[0] for s_ in starts])
    q = np.concatenate([s_[1] for s_ in starts])
    vel = np.concatenate([s_[2] for s_ in starts])
    b = R.BatchedSlab([dict(w.slab_kwargs(), precision="fp64", n_max=w.N) for w in ws])
    off = b.offsets([w.N for w in ws])
    k0 = b.draw_kset(seed, 0)
    F0 = np.concatenate([orc.evaluate(oracle_slab(orc, w, b.Lz_ext[r]), starts[r][0], starts[r][1], k0[r]).F
                         for r, w in enumerate(ws)])
    P_, V_, Q_, F_ = to_dev(torch, pos), to_dev(torch, vel), to_dev(torch, q), to_dev(torch, F0)
    print("batch md_run walls", flush=True)
    b.md_run(off, P_, V_, Q_, F_, dt, margin, seed, step0, 3, use_graph=True)
    b.check()
    pg, vg, Fg = P_.cpu().numpy(), V_.cpu().numpy(), F_.cpu().numpy()
    for r, w in enumerate(ws):
        o = oracle_slab(orc, w, b.Lz_ext[r])
        p0, q0, v0, lo, hi, fast = starts[r]
        zlo, zhi = margin, w.H - margin
        p, v, F, folds = oracle_vv(orc, o, w, p0, v0, q0, F0[off[r]:off[r + 1]], dt, zlo, zhi, seed, step0, 3,
                                   lambda st: st * len(ws) + r)
        assert_walls_hit(folds, lo, hi, fast)
        sl = slice(off[r], off[r + 1])
        assert np.abs(pg[sl] - p).max() <= 1e-11, r
        assert rel_rms(vg[sl], v) <= 1e-11, r
        assert rel_rms(Fg[sl], F) <= 1e-9, r


@pytest.mark.parametrize("use_graph", [False, True])
def test_md_run_ex_wall_crossings_match_oracle(torch, R, orc, use_graph):
    """BAOAB with WCA walls: ions 1e-3 from the integrator's walls moving out
    at 20, and fast ones folding at least twice per step, fold exactly as in
    the oracle's step fed with the same noise and k-sets.  The integrator's
    walls (margin 0.6) lie beyond the WCA walls' range (2^(1/6) 0.5), and the
    ion-ion WCA term is off so that a fast ion landing next to another one
    cannot be shot across the box many times over (the WCA ion-ion forces
    are covered by the Langevin test of the MD module)."""
    w = inputs.small_random(74, 300, L=10.0, H=6.0, gamma_top=0.7, gamma_bot=-0.5, alpha=0.9, r_c=4.0, P=40,
                            M=4, margin=0.3).with_(extra={"dmin": 0.85})
    pos, q = inputs.sample(w)
    mdk = dict(gamma=2.0, kT=1.2, sigma=1.0, eps=0.0, sigma_wall=0.5, eps_wall=1.0, wall_margin=0.6)
    md = R.md_params(**mdk)
    seed, dt, step0 = 31, 2e-3, 3
    zlo, zhi = 0.6, w.H - 0.6
    pos, vel, lo, hi, fast = wall_start(pos, zlo, zhi, dt, 8, n_near=20, n_fast=4)
    s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=w.N)
    o = oracle_slab(orc, w, s.Lz_ext)

    def total(x, n):
        Fs, _, _ = orc.short_range(x, w.Lx, w.Ly, w.H, mdk["sigma"], mdk["eps"], mdk["sigma_wall"],
                                   mdk["eps_wall"])
        return orc.evaluate(o, x, q, n).F + Fs

    F0 = total(pos, s.draw_kset(seed, step0 - 1))
    P_, V_, Q_, F_ = to_dev(torch, pos), to_dev(torch, vel), to_dev(torch, q), to_dev(torch, F0)
    print(f"md_run_ex walls graph={use_graph}", flush=True)
    s.md_run_ex(P_, V_, Q_, F_, dt, md, seed, step0, 3, use_graph=use_graph)
    s.check()
    p, v, F = pos, vel, F0
    first_v = None
    W = zhi - zlo
    for st in range(step0, step0 + 3):
        n = orc.draw_kset(o, seed, st)
        xi = orc.thermo_normals(seed, st, w.N)
        # BAOAB drifts by dt times v after the kick (the O step between the
        # two half drifts rescales v; both halves carry the same sign)
        zpre = p[fast, 2] + dt * (v[fast, 2] + 0.5 * dt * F[fast, 2])
        assert np.all(np.abs(np.floor((zpre - zlo) / W)) >= 1)
        p, v, F = orc.baoab_step(p, v, F, dt, mdk["gamma"], mdk["kT"], xi, w.Lx, w.Ly, zlo, zhi,
                                 lambda x: total(x, n))
        if first_v is None:
            first_v = v[:, 2].copy()
    # the near ions were reflected in the first step (v_z changed sign)
    assert np.all(first_v[lo] > 0) and np.all(first_v[hi] < 0)
    pg, vg, Fg = P_.cpu().numpy(), V_.cpu().numpy(), F_.cpu().numpy()
    assert np.abs(pg - p).max() <= 1e-11
    assert rel_rms(vg, v) <= 1e-11
    assert rel_rms(Fg, F) <= 1e-9
