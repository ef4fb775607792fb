"""The entry point without allocation (rbe2d_forces_noalloc) against
rbe2d_forces on a handle with the same parameters and k-set, and against the
oracle: two calls in a row, the second with fewer particles, in both
precisions; the largest sizes it accepts; the first sizes it refuses; the
device error word."""
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


def _workload(seed, N):
    return inputs.small_random(seed, N, L=24.0, H=6.0, gamma_top=0.7, gamma_bot=-0.55, alpha=0.8, r_c=5.0, P=64,
                               M=5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_handle_two_calls(torch, R, orc, precision):
    n_max = 4000
    for call, N in enumerate((3000, 1100)):
        w = _workload(40 + call, N)
        pos, q = inputs.sample(w)
        slab = R.Slab(**w.slab_kwargs(), precision=precision, n_max=n_max)
        kset = slab.draw_kset(5 + call)
        slab.set_kset(kset)
        P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
        K_ = torch.as_tensor(kset, dtype=torch.int32, device="cuda")
        print(f"noalloc {precision} call {call} N={N}", flush=True)
        Fh, Eh = slab.forces(P_, Q_, want_energy=True)
        err = torch.full((), -1, dtype=torch.int32, device="cuda")
        Fs, Es = R.forces_noalloc(slab.params, K_, P_, Q_, want_energy=True, err_out=err)
        torch.cuda.synchronize()
        slab.check()
        assert int(err.item()) == 0
        Fh, Fs, Eh, Es = (t.cpu().numpy() for t in (Fh, Fs, Eh, Es))
        # same kernels and launch parameters as the handle: equal up to rounding order
        assert rel_rms(Fs, Fh) <= 1e-12
        assert np.abs(Es - Eh).max() <= 1e-12 * np.abs(Eh).sum()
        ref = orc.evaluate(oracle_slab(orc, w, slab.Lz_ext), pos, q, kset)
        assert rel_rms(Fs, ref.F) <= TOL[precision]
        for eg, er in zip(Es, ref.energies()):
            assert abs(eg - er) <= TOL[precision] * energy_scale(ref)


def test_noalloc_largest_sizes_and_refusals(torch, R):
    """n_max = 32768 and P = 1024 are accepted (equal to the handle's result);
    one particle or one k-vector more is refused with a message."""
    N = 32768
    w = inputs.small_random(47, N, L=60.0, H=10.0, gamma_top=0.9, gamma_bot=0.9, alpha=0.6, r_c=6.0, P=1024, M=8)
    pos, q = inputs.sample(w)
    slab = R.Slab(**w.slab_kwargs(), precision="fp32", n_max=N)
    kset = slab.draw_kset(9)
    slab.set_kset(kset)
    P_, Q_ = to_dev(torch, pos), to_dev(torch, q)
    K_ = torch.as_tensor(kset, dtype=torch.int32, device="cuda")
    print("noalloc largest", flush=True)
    Fh = slab.forces(P_, Q_)
    Fs = R.forces_noalloc(slab.params, K_, P_, Q_)
    torch.cuda.synchronize()
    assert rel_rms(Fs.cpu().numpy(), Fh.cpu().numpy()) <= 1e-12
    for over in (dict(n_max=N + 1), dict(P=1025)):
        kw = dict(w.slab_kwargs(), precision="fp32", n_max=N)
        kw.update(over)
        p = R.make_params(**kw)
        Kx = torch.zeros((p.P, 3), dtype=torch.int32, device="cuda")
        Kx[:, 0] = 1
        with pytest.raises(R.RBE2DError) as ei:
            R.forces_noalloc(p, Kx, P_[:10], Q_[:10])
        assert ei.value.status == R.RBE2D_E_INVAL and "noalloc" in str(ei.value)


def test_noalloc_error_word(torch, R):
    """A particle outside the slab sets bit 0 of the call's error word; the
    next call with valid positions reports 0."""
    w = _workload(44, 500)
    pos, q = inputs.sample(w)
    p = R.make_params(**w.slab_kwargs(), precision="fp64", n_max=500)
    K_ = torch.as_tensor(R.draw_kset(p, 3), dtype=torch.int32, device="cuda")
    bad = pos.copy()
    bad[7, 2] = w.H + 0.5
    err = torch.zeros((), dtype=torch.int32, device="cuda")
    R.forces_noalloc(p, K_, to_dev(torch, bad), to_dev(torch, q), err_out=err)
    torch.cuda.synchronize()
    assert int(err.item()) & 1
    R.forces_noalloc(p, K_, to_dev(torch, pos), to_dev(torch, q), err_out=err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
