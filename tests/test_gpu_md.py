"""GPU parity of the MD around the path: short-range repulsion (ions and
walls), BAOAB Langevin steps against the oracle's step, graph replays, and
the thermostat's temperature."""
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


def packed(seed, N, L, H, dmin=0.85, margin=0.3, **kw):
    """A workload whose ions touch (WCA overlaps) but do not collapse."""
    return inputs.small_random(seed, N, L=L, H=H, margin=margin, **kw).with_(extra={"dmin": dmin})


SHORT_CASES = [
    # seed, N, L, H, r_c: boxes from 3 columns of cells (all searched once) to many
    (1, 250, 9.0, 6.0, 4.0),
    (2, 1500, 16.0, 8.0, 3.0),
    (3, 40, 4.5, 3.0, 2.0),
]


@pytest.mark.parametrize("case", SHORT_CASES, ids=[f"N{c[1]}L{c[2]}" for c in SHORT_CASES])
def test_short_forces_match_oracle(torch, R, orc, case):
    seed, N, L, H, rc = case
    w = packed(seed, N, L, H, r_c=rc, P=10)
    pos, q = inputs.sample(w)
    md = R.md_params(sigma=1.0, eps=1.3, sigma_wall=0.5, eps_wall=0.8, wall_margin=0.1)
    s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=N)
    F0 = to_dev(torch, np.full((N, 3), 0.25))
    F, E = s.short_forces(to_dev(torch, pos), to_dev(torch, q), md, F=F0, want_energy=True)
    s.check()
    ref, ep, ew = orc.short_range(pos, L, L, H, 1.0, 1.3, 0.5, 0.8)
    assert np.abs(ref).max() > 1.0                       # the case has overlaps
    assert rel_rms(F.cpu().numpy() - 0.25, ref) <= 1e-12  # added to F
    E = E.cpu().numpy()[0]
    assert abs(E[0] - ep) <= 1e-12 * abs(ep) and abs(E[1] - ew) <= 1e-12 * max(abs(ew), 1e-300)


def test_short_forces_batch(torch, R, orc):
    ws = [packed(11, 320, 10.0, 6.0, r_c=4.0, P=10), packed(12, 0, 8.0, 5.0, r_c=3.0, P=10),
          packed(13, 700, 14.0, 7.0, r_c=5.0, P=10)]
    pos = np.concatenate([inputs.sample(w)[0] for w in ws]).reshape(-1, 3)
    q = np.concatenate([inputs.sample(w)[1] for w in ws])
    b = R.BatchedSlab([dict(w.slab_kwargs(), precision="fp64", n_max=w.N) for w in ws])
    off = b.offsets([w.N for w in ws])
    md = R.md_params(sigma=1.0, eps=1.0, sigma_wall=0.5, eps_wall=1.0, wall_margin=0.1)
    F, E = b.short_forces(off, to_dev(torch, pos), to_dev(torch, q), md, want_energy=True)
    F, E = F.cpu().numpy(), E.cpu().numpy()
    for r, w in enumerate(ws):
        if not w.N:
            assert np.array_equal(E[r], [0.0, 0.0])
            continue
        ref, ep, ew = orc.short_range(pos[off[r]:off[r + 1]], w.Lx, w.Ly, w.H, 1.0, 1.0, 0.5, 1.0)
        assert rel_rms(F[off[r]:off[r + 1]], ref) <= 1e-12
        assert abs(E[r][0] - ep) <= 1e-12 * abs(ep)


def _total_force(orc, o, w, pos, q, n, mdk):
    ref = orc.evaluate(o, pos, q, n)
    Fs, _, _ = orc.short_range(pos, w.Lx, w.Ly, w.H, mdk["sigma"], mdk["eps"], mdk["sigma_wall"],
                               mdk["eps_wall"])
    return ref.F + Fs


def test_langevin_steps_match_oracle(torch, R, orc):
    """Three BAOAB steps with RBE2D + WCA forces: same positions, velocities
    and forces as the oracle's step fed with its own noise and k-sets."""
    w = packed(21, 300, 10.0, 6.0, gamma_top=0.7, gamma_bot=-0.5, alpha=0.9, r_c=4.0, P=40, M=4)
    pos, q = inputs.sample(w)
    mdk = dict(gamma=2.0, kT=1.2, sigma=1.0, eps=1.0, sigma_wall=0.5, eps_wall=1.0, wall_margin=0.1)
    md = R.md_params(**mdk)
    seed, dt, step0 = 77, 2e-3, 5
    s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=w.N)
    o = oracle_slab(orc, w, s.Lz_ext)
    vel = np.random.default_rng(4).normal(0.0, 1.0, pos.shape)
    n0 = s.draw_kset(seed, step0 - 1)
    F0 = _total_force(orc, o, w, pos, q, n0, mdk)
    P_, V_, Q_, F_ = to_dev(torch, pos), to_dev(torch, vel), to_dev(torch, q), to_dev(torch, F0)
    s.md_run_ex(P_, V_, Q_, F_, dt, md, seed, step0, 3)
    s.check()
    p, v, F = pos, vel, F0
    for st in range(step0, step0 + 3):
        n = orc.draw_kset(o, seed, st)
        xi = orc.thermo_normals(seed, st, w.N)
        p, v, F = orc.baoab_step(p, v, F, dt, mdk["gamma"], mdk["kT"], xi, w.Lx, w.Ly, 0.1, w.H - 0.1,
                                 lambda x: _total_force(orc, o, w, x, q, n, mdk))
    assert np.abs(P_.cpu().numpy() - p).max() <= 1e-11
    assert rel_rms(V_.cpu().numpy(), v) <= 1e-11
    assert rel_rms(F_.cpu().numpy(), F) <= 1e-9
    assert np.array_equal(s.get_kset(), orc.draw_kset(o, seed, step0 + 2))


def test_langevin_graph_equals_eager_batch(torch, R):
    ws = [packed(31, 450, 12.0, 6.0, gamma_top=0.5, gamma_bot=0.5, r_c=4.0, P=30, M=3),
          packed(32, 250, 10.0, 5.0, r_c=4.0, P=30)]
    pos = np.concatenate([inputs.sample(w)[0] for w in ws]).reshape(-1, 3)
    q = np.concatenate([inputs.sample(w)[1] for w in ws])
    md = R.md_params(gamma=1.0, kT=1.0, sigma=1.0, eps=1.0, sigma_wall=0.5, eps_wall=1.0, wall_margin=0.1)
    runs = []
    for use_graph in (False, True):
        b = R.BatchedSlab([dict(w.slab_kwargs(), precision="fp32", n_max=w.N) for w in ws])
        off = b.offsets([w.N for w in ws])
        P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
        V_ = torch.zeros_like(P_)
        b.set_kset(b.draw_kset(3, 0))
        F_ = b.forces(off, P_, Q_)
        b.short_forces(off, P_, Q_, md, F=F_)
        for step0, n in ((1, 2), (3, 2)):
            b.md_run_ex(off, P_, V_, Q_, F_, 1e-3, md, 9, step0, n, use_graph=use_graph)
            torch.cuda.synchronize()
        b.check()
        runs.append([t.cpu().numpy() for t in (P_, V_, F_)])
    for x, y in zip(runs[0], runs[1]):
        assert np.array_equal(x, y)


def test_thermostat_reaches_target_temperature(torch, R):
    """Uncharged WCA spheres between WCA walls: the kinetic temperature
    settles at kT (equipartition, unit masses)."""
    # start beyond the walls' range (2^(1/6) sigma_wall) so no ion begins deep in it
    w = packed(41, 1500, 20.0, 8.0, margin=0.6, r_c=4.0, P=8)
    pos, _ = inputs.sample(w)
    q = np.zeros(w.N)
    kT = 1.5
    md = R.md_params(gamma=4.0, kT=kT, sigma=1.0, eps=1.0, sigma_wall=0.5, eps_wall=1.0, wall_margin=0.05)
    s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=w.N)
    P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
    V_ = torch.zeros_like(P_)
    s.sample_kset(1, 0)
    F_ = s.forces(P_, Q_)
    s.short_forces(P_, Q_, md, F=F_)
    s.md_run_ex(P_, V_, Q_, F_, 5e-3, md, 1, 0, 300, use_graph=True)
    temps = []
    for k in range(20):
        s.md_run_ex(P_, V_, Q_, F_, 5e-3, md, 1, 300 + 10 * k, 10, use_graph=True)
        temps.append(float((V_ ** 2).mean().item()))
    s.check()
    assert abs(np.mean(temps) - kT) < 0.05 * kT, temps


@pytest.mark.parametrize("use_graph", [False, True])
def test_velocity_verlet_steps_match_oracle(torch, R, orc, use_graph):
    """Four plain velocity-Verlet steps (md_run: chained half kicks, the next
    k-set drawn beside the force pass) against the oracle's step with no
    friction, fed with the same k-sets."""
    w = inputs.small_random(51, 400, L=11.0, H=6.0, gamma_top=0.6, gamma_bot=-0.4, alpha=0.9, r_c=4.0, P=40,
                            M=4, margin=0.5)
    pos, q = inputs.sample(w)
    s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=w.N)
    o = oracle_slab(orc, w, s.Lz_ext)
    seed, dt, step0, zlo, zhi = 13, 2e-3, 3, 0.3, w.H - 0.3
    vel = np.random.default_rng(6).normal(0.0, 2.0, pos.shape)
    n0 = s.draw_kset(seed, 1)
    F0 = orc.evaluate(o, pos, q, n0).F
    P_, V_, Q_, F_ = to_dev(torch, pos), to_dev(torch, vel), to_dev(torch, q), to_dev(torch, F0)
    s.md_run(P_, V_, Q_, F_, dt, zlo, zhi, seed, step0, 4, use_graph=use_graph)
    s.check()
    p, v, F = pos, vel, F0
    for st in range(step0, step0 + 4):
        n = orc.draw_kset(o, seed, st)
        p, v, F = orc.baoab_step(p, v, F, dt, 0.0, 0.0, np.zeros_like(p), w.Lx, w.Ly, zlo, zhi,
                                 lambda x: orc.evaluate(o, x, q, n).F)
    assert np.abs(P_.cpu().numpy() - p).max() <= 1e-11
    assert rel_rms(V_.cpu().numpy(), v) <= 1e-11
    assert rel_rms(F_.cpu().numpy(), F) <= 1e-9
    assert np.array_equal(s.get_kset(), orc.draw_kset(o, seed, step0 + 3))


def _wall_fractions(torch, R, gamma, seed=61, N=600, L=24.0, H=8.0, band=1.0):
    """Langevin + WCA run of a 2:1 electrolyte (Bjerrum length 3.5 sigma) with
    dielectric contrast gamma at both faces: the fraction of cation and of
    anion positions within `band` of either wall, over 100 snapshots after
    3000 steps of equilibration."""
    w = inputs.small_random(seed, N, L=L, H=H, gamma_top=gamma, gamma_bot=gamma, alpha=0.6, r_c=6.0, P=64, M=8,
                            valence=(2, -1), margin=0.6).with_(extra={"dmin": 0.9})
    pos, q = inputs.sample(w)
    md = R.md_params(gamma=1.0, kT=1.0, sigma=1.0, eps=1.0, sigma_wall=0.5, eps_wall=1.0, wall_margin=0.05)
    s = R.Slab(**w.slab_kwargs(), precision="fp32", n_max=N, coulomb_prefactor=3.5)
    P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
    V_ = torch.zeros_like(P_)
    s.sample_kset(7, 0)
    F_ = s.forces(P_, Q_)
    s.short_forces(P_, Q_, md, F=F_)
    s.md_run_ex(P_, V_, Q_, F_, 5e-3, md, 7, 0, 3000, use_graph=True)
    zs, step = [], 3000
    for _ in range(100):
        s.md_run_ex(P_, V_, Q_, F_, 5e-3, md, 7, step, 30, use_graph=True)
        step += 30
        zs.append(P_[:, 2].cpu().numpy().copy())
    s.check()
    z = np.stack(zs)
    near = (z < band) | (z > H - band)
    return float(near[:, q > 0].mean()), float(near[:, q < 0].mean())


def test_ion_depletion_near_insulating_interfaces(torch, R):
    """The MD around the path reproduces the ion-depletion effect near
    insulator-like interfaces (gamma = 0.939 at both faces, Sec. 4): images of
    the same sign push every ion away from the walls (energy ~ gamma q^2
    l_B / 4d at distance d), strongest for the divalent cations, and images of
    the opposite sign (gamma = -0.939) draw them in.  Same ions, seeds and
    steps with gamma = 0 as the reference; measured 0.101 of the cation
    positions within one sigma of a wall at gamma = 0, 0.058 at +0.939, 0.19
    at -0.939 (two seeds agree to 0.005)."""
    c0, a0 = _wall_fractions(torch, R, 0.0)
    cp, ap = _wall_fractions(torch, R, 0.939)
    cm, am = _wall_fractions(torch, R, -0.939)
    assert cp < 0.75 * c0 and cm > 1.4 * c0, (c0, cp, cm)
    assert ap < a0 < am, (a0, ap, am)
