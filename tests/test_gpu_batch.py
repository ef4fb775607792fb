"""GPU parity of the batched path: one handle over many independent slabs.

Each system of a batch must give what the oracle gives for that system alone
(same k-set), and what a single-system handle gives (up to summation order).
MD steps replayed from a captured hipGraph must equal eager steps bitwise.
"""
import numpy as np
import pytest

from paper_2405_06333_amd import inputs
from tests.gpu_common import energy_scale, oracle_slab, rel_rms, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-5}


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


# systems of mixed size, box, contrast and image order; one is empty and
# several are not multiples of a wave or a tile
MIXED = [
    inputs.small_random(501, 300, L=12.0, H=5.0, gamma_top=0.6, gamma_bot=-0.8, alpha=0.9, r_c=5.0, P=40, M=4),
    inputs.small_random(502, 0, L=10.0, H=4.0, P=40),
    inputs.small_random(503, 65, L=10.0, H=2.0, gamma_top=0.7, gamma_bot=-0.6, alpha=1.1, r_c=3.0, P=40, M=3,
                        margin=0.05),
    inputs.small_random(504, 1, L=9.0, H=4.0, gamma_top=-1.0, gamma_bot=-1.0, r_c=3.0, P=40, M=6),
    inputs.small_random(505, 1031, L=20.0, H=6.0, gamma_top=0.95, gamma_bot=0.95, alpha=0.8, r_c=5.0, P=40, M=8),
    inputs.small_random(506, 4097, L=30.0, H=8.0, gamma_top=-0.5, gamma_bot=0.3, alpha=0.7, r_c=6.0, P=40, M=2,
                        valence=(2, -1)),
]


def batch_inputs(ws):
    pos, q = zip(*(inputs.sample(w) for w in ws))
    counts = [w.N for w in ws]
    return np.concatenate(pos).reshape(-1, 3), np.concatenate(q), counts


def make_batch(R, ws, precision, n_max=None):
    kws = [dict(w.slab_kwargs(), precision=precision, n_max=w.N if n_max is None else n_max[i])
           for i, w in enumerate(ws)]
    return R.BatchedSlab(kws)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_oracle_per_system(torch, R, orc, precision):
    ws = MIXED
    pos, q, counts = batch_inputs(ws)
    b = make_batch(R, ws, precision)
    kset = b.draw_kset(7, 100)
    b.set_kset(kset)
    off = b.offsets(counts)
    F, E = b.forces(off, to_dev(torch, pos), to_dev(torch, q), want_energy=True)
    b.check()
    F, E = F.cpu().numpy(), E.cpu().numpy()
    for r, w in enumerate(ws):
        o = oracle_slab(orc, w, b.Lz_ext[r])
        p_r, q_r = pos[off[r]:off[r + 1]], q[off[r]:off[r + 1]]
        ref = orc.evaluate(o, p_r, q_r, kset[r])
        if w.N:
            err = rel_rms(F[off[r]:off[r + 1]], ref.F)
            assert err <= TOL[precision], f"system {r}: force rel-RMS {err:.3e}"
        scale = energy_scale(ref)
        for k, (eg, er) in enumerate(zip(E[r], ref.energies())):
            assert abs(eg - er) <= TOL[precision] * scale, f"system {r} energy[{k}] {eg!r} vs {er!r}"


def test_batch_matches_single_handles(torch, R, orc):
    ws = MIXED
    pos, q, counts = batch_inputs(ws)
    b = make_batch(R, ws, "fp64")
    b.sample_kset(11, 5)
    kset = b.get_kset()
    off = b.offsets(counts)
    F, E = b.forces(off, to_dev(torch, pos), to_dev(torch, q), want_energy=True)
    F, E = F.cpu().numpy(), E.cpu().numpy()
    for r, w in enumerate(ws):
        s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=max(w.N, 1))
        assert s.Lz_ext == b.Lz_ext[r] and s.V == b.V[r] and s.S == b.S[r]
        # device sampler of system r = stream id 5 + r
        assert np.array_equal(kset[r], s.draw_kset(11, 5 + r))
        s.set_kset(kset[r])
        Fs, Es = s.forces(to_dev(torch, pos[off[r]:off[r + 1]]), to_dev(torch, q[off[r]:off[r + 1]]),
                          want_energy=True)
        Fs, Es = Fs.cpu().numpy(), Es.cpu().numpy()
        if w.N:
            assert rel_rms(F[off[r]:off[r + 1]], Fs) <= 1e-12
        assert np.allclose(E[r], Es, rtol=1e-12, atol=1e-12 * np.abs(Es).sum())


def test_batch_layout_changes_between_calls(torch, R, orc):
    """Counts below n_max, changed from call to call, including all-empty."""
    ws = MIXED[:3]
    n_max = [w.N + 50 for w in ws]
    b = make_batch(R, ws, "fp64", n_max=n_max)
    kset = b.draw_kset(3, 0)
    b.set_kset(kset)
    pos, q, counts = batch_inputs(ws)
    off = b.offsets(counts)
    for cut in ([w.N for w in ws], [w.N // 2 for w in ws], [0, 0, 0], [w.N for w in ws]):
        sel = np.concatenate([np.arange(off[r], off[r] + cut[r]) for r in range(len(ws))]).astype(int)
        sub_off = b.offsets(cut)
        F, E = b.forces(sub_off, to_dev(torch, pos[sel]), to_dev(torch, q[sel]), want_energy=True)
        F, E = F.cpu().numpy(), E.cpu().numpy()
        for r, w in enumerate(ws):
            p_r = pos[off[r]:off[r] + cut[r]]
            q_r = q[off[r]:off[r] + cut[r]]
            ref = orc.evaluate(oracle_slab(orc, w, b.Lz_ext[r]), p_r, q_r, kset[r])
            if cut[r]:
                assert rel_rms(F[sub_off[r]:sub_off[r + 1]], ref.F) <= 1e-9
            assert abs(E[r][0] - ref.E_total) <= 1e-9 * energy_scale(ref)


def test_batch_rejects_bad_offsets(torch, R):
    ws = MIXED[:2]
    b = make_batch(R, ws, "fp64")
    b.set_kset(b.draw_kset(0, 0))
    pos = torch.zeros((400, 3), dtype=torch.float64, device="cuda")
    q = torch.zeros(400, dtype=torch.float64, device="cuda")
    for off in ([1, 2, 3], [0, 301, 301], [0, 10, 5]):
        with pytest.raises(R.RBE2DError) as ei:
            n = off[-1] if off[-1] >= 0 else 0
            b.forces(off, pos[:n].contiguous(), q[:n].contiguous())
        assert ei.value.status == R.RBE2D_E_INVAL
    # single-system calls are refused on a batched handle
    st = R.lib().rbe2d_forces(b.handle, 0, None, None, None, None, 7, None)
    assert st == R.RBE2D_E_STATE


def test_batch_mixed_precision_or_P_rejected(R):
    w = MIXED[0]
    with pytest.raises(R.RBE2DError):
        R.BatchedSlab([dict(w.slab_kwargs(), precision="fp64", n_max=10),
                       dict(w.slab_kwargs(), precision="fp32", n_max=10)])
    with pytest.raises(R.RBE2DError):
        R.BatchedSlab([dict(w.slab_kwargs(), n_max=10), dict(w.slab_kwargs(P=41), n_max=10)])


def _md_state(torch, pos, q, vel_seed=0):
    rng = np.random.default_rng(vel_seed)
    vel = rng.normal(0.0, 1.0, pos.shape)
    return to_dev(torch, pos), to_dev(torch, vel), to_dev(torch, q)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_md_graph_replays_equal_eager_single(torch, R, precision):
    w = inputs.small_random(601, 700, L=14.0, H=6.0, gamma_top=0.8, gamma_bot=-0.7, alpha=0.9, r_c=4.5, P=50,
                            M=5)
    pos, q = inputs.sample(w)
    runs = []
    for use_graph in (False, True):
        s = R.Slab(**w.slab_kwargs(), precision=precision, n_max=w.N)
        P_, V_, Q_ = _md_state(torch, pos, q)
        s.set_kset(s.draw_kset(9, 0))
        F_ = s.forces(P_, Q_)
        s.md_run(P_, V_, Q_, F_, 2e-3, 0.3, w.H - 0.3, 9, 1, 3, use_graph=use_graph)
        # eager work of the program between replays
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        s.md_run(P_, V_, Q_, F_, 2e-3, 0.3, w.H - 0.3, 9, 4, 2, use_graph=use_graph)
        s.md_run(P_, V_, Q_, F_, 2e-3, 0.3, w.H - 0.3, 9, 6, 1, use_graph=use_graph)
        s.check()
        del junk
        runs.append([t.cpu().numpy() for t in (P_, V_, F_)] + [s.get_kset()])
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)
    assert np.array_equal(runs[1][3], R.draw_kset(s.params, 9, 6))


def test_md_graph_replays_equal_eager_batch(torch, R):
    ws = [MIXED[0], MIXED[2], MIXED[4]]
    pos, q, counts = batch_inputs(ws)
    runs = []
    for use_graph in (False, True):
        b = make_batch(R, ws, "fp32")
        off = b.offsets(counts)
        P_, V_, Q_ = _md_state(torch, pos, q, 1)
        b.set_kset(b.draw_kset(4, 0))
        F_ = b.forces(off, P_, Q_)
        for step0, n in ((0, 2), (2, 3)):
            b.md_run(off, P_, V_, Q_, F_, 1e-3, 0.04, 4, step0, n, use_graph=use_graph)
            torch.cuda.synchronize()
        b.check()
        runs.append([t.cpu().numpy() for t in (P_, V_, F_)] + [b.get_kset()])
    for a, c in zip(runs[0], runs[1]):
        assert np.array_equal(a, c)
    # last step was step 4: system r drew stream id 4 * n_sys + r
    ks = runs[1][3]
    for r in range(len(ws)):
        assert np.array_equal(ks[r], R.draw_kset(b._params_arr[r], 4, 4 * len(ws) + r))


def test_batch_md_step_forces_match_oracle(torch, R, orc):
    """After batched MD steps the forces left in F are the forces of the
    final positions under the final k-set."""
    ws = [MIXED[0], MIXED[4]]
    pos, q, counts = batch_inputs(ws)
    b = make_batch(R, ws, "fp64")
    off = b.offsets(counts)
    P_, V_, Q_ = _md_state(torch, pos, q, 2)
    b.set_kset(b.draw_kset(1, 0))
    F_ = b.forces(off, P_, Q_)
    b.md_run(off, P_, V_, Q_, F_, 1e-3, 0.2, 1, 0, 3, use_graph=True)
    b.check()
    pf, F, ks = P_.cpu().numpy(), F_.cpu().numpy(), b.get_kset()
    for r, w in enumerate(ws):
        assert np.all(pf[off[r]:off[r + 1], 2] >= 0.2) and np.all(pf[off[r]:off[r + 1], 2] <= w.H - 0.2)
        ref = orc.evaluate(oracle_slab(orc, w, b.Lz_ext[r]), pf[off[r]:off[r + 1]], q[off[r]:off[r + 1]], ks[r])
        assert rel_rms(F[off[r]:off[r + 1]], ref.F) <= 1e-9


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_replica_batch_sampled_parity(torch, R, orc, precision):
    """The 64-replica batch at full size, in the launch configuration the
    benchmark times (FP32 phases, and the FP64 batch it reports beside it):
    sampled particles of four replicas against the oracle's per-target
    forces, and the k-space, self and IBC energies of every replica (the
    oracle sums them over all particles of the replica)."""
    ws = inputs.replicas()
    pos, q, counts = batch_inputs(ws)
    b = make_batch(R, ws, precision)
    off = b.offsets(counts)
    b.sample_kset(ws[0].seed, 0)
    kset = b.get_kset()
    print(f"replicas {precision} total N={off[-1]}", flush=True)
    F, E = b.forces(off, to_dev(torch, pos), to_dev(torch, q), want_energy=True)
    b.check()
    F, E = F.cpu().numpy(), E.cpu().numpy()
    assert np.isfinite(F).all() and np.isfinite(E).all()
    tol = TOL[precision]
    rng = np.random.default_rng(0)
    sampled = (0, 17, 40, 63)
    for r, w in enumerate(ws):
        tg = np.sort(rng.choice(w.N, 24, replace=False)) if r in sampled else np.zeros(1, dtype=np.int64)
        ref = orc.evaluate(oracle_slab(orc, w, b.Lz_ext[r]), pos[off[r]:off[r + 1]], q[off[r]:off[r + 1]],
                           kset[r], targets=tg)
        if r in sampled:
            err = rel_rms(F[off[r] + tg], ref.F)
            assert err <= tol, f"replica {r}: sampled force rel-RMS {err:.3e}"
        scale = abs(E[r][1]) + abs(ref.E_k) + abs(ref.E_self) + abs(ref.E_ibc)
        for k, er in ((2, ref.E_k), (3, ref.E_self), (4, ref.E_ibc)):
            assert abs(E[r][k] - er) <= tol * scale, f"replica {r} energy[{k}] {E[r][k]!r} vs {er!r}"


def test_autotune_single_keeps_results(torch, R, orc):
    w = inputs.DIELECTRIC
    pos, q = inputs.sample(w)
    s = R.Slab(**w.slab_kwargs(), precision="fp64", n_max=w.N)
    kset = s.draw_kset(w.seed, 0)
    s.set_kset(kset)
    P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
    F0, E0 = s.forces(P_, Q_, want_energy=True)
    ch = s.autotune(P_, Q_)
    assert ch["per"] in (1, 2, 4, 8, 16) and ch["ksplit"] in (1, 2, 4, 8, 16, 32, 64) and 1 <= ch["rsplit"] <= 5
    F1, E1 = s.forces(P_, Q_, want_energy=True)
    s.check()
    F0, F1 = F0.cpu().numpy(), F1.cpu().numpy()
    assert rel_rms(F1, F0) <= 1e-12
    assert np.allclose(E1.cpu().numpy(), E0.cpu().numpy(), rtol=1e-12, atol=1e-12 * float(np.abs(E0.cpu().numpy()).sum()))
    ref = orc.evaluate(oracle_slab(orc, w, s.Lz_ext), pos, q, kset)
    assert rel_rms(F1, ref.F) <= 1e-9


def test_autotune_batch_then_graph(torch, R, orc):
    ws = MIXED
    pos, q, counts = batch_inputs(ws)
    b = make_batch(R, ws, "fp32")
    off = b.offsets(counts)
    b.set_kset(b.draw_kset(5, 0))
    P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
    ch = b.autotune(off, P_, Q_)
    assert ch["per"] in (1, 2, 4, 8, 16)
    kset = b.get_kset()
    F = b.forces(off, P_, Q_).cpu().numpy()
    for r, w in enumerate(ws):
        if not w.N:
            continue
        ref = orc.evaluate(oracle_slab(orc, w, b.Lz_ext[r]), pos[off[r]:off[r + 1]], q[off[r]:off[r + 1]], kset[r])
        assert rel_rms(F[off[r]:off[r + 1]], ref.F) <= 1e-5
    # tuned launch parameters inside a captured MD step
    runs = []
    for use_graph in (False, True):
        P2, V2, Q2 = _md_state(torch, pos, q, 3)
        b.set_kset(kset)
        F2 = b.forces(off, P2, Q2)
        b.md_run(off, P2, V2, Q2, F2, 1e-3, 0.04, 6, 0, 3, use_graph=use_graph)
        b.check()
        runs.append([t.cpu().numpy() for t in (P2, V2, F2)])
    for x, y in zip(runs[0], runs[1]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_force_variance_matches_oracle(torch, R, orc, precision, tol):
    """The per-particle variance estimate of the k-space force (Theorem 2.2)
    against the oracle's estimate from the same batch."""
    ws = [MIXED[0], MIXED[4], MIXED[1]]
    pos, q, counts = batch_inputs(ws)
    b = make_batch(R, ws, precision)
    off = b.offsets(counts)
    kset = b.draw_kset(13, 2)
    b.set_kset(kset)
    var = b.force_variance(off, to_dev(torch, pos), to_dev(torch, q)).cpu().numpy()
    b.check()
    for r, w in enumerate(ws):
        if not w.N:
            continue
        ref = orc.force_variance_estimate(oracle_slab(orc, w, b.Lz_ext[r]), pos[off[r]:off[r + 1]],
                                          q[off[r]:off[r + 1]], kset[r])
        assert (ref > 0).all()
        assert rel_rms(var[off[r]:off[r + 1]], ref) <= tol


def test_force_variance_single_batch_of_one_k(torch, R):
    w = MIXED[0]
    pos, q = inputs.sample(w)
    s = R.Slab(**w.slab_kwargs(P=1), precision="fp64", n_max=w.N)
    s.set_kset(s.draw_kset(1, 0))
    var = s.force_variance(to_dev(torch, pos), to_dev(torch, q)).cpu().numpy()
    assert np.array_equal(var, np.zeros(w.N))
