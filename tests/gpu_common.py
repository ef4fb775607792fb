"""Helpers of the GPU parity tests: run the library and the oracle on the
same seeded inputs and k-set, and compare."""
import numpy as np


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt((b * b).sum())
    return float(np.sqrt(((a - b) ** 2).sum()) / den) if den > 0 else float(np.sqrt((a * a).sum()))


def energy_scale(ref):
    """|E_real| + |E_k| + |E_self| + |E_ibc| of an oracle result."""
    return abs(ref.E_real) + abs(ref.E_k) + abs(ref.E_self) + abs(ref.E_ibc) + 1e-300


def oracle_slab(orc, w, Lz):
    return orc.Slab(Lx=w.Lx, Ly=w.Ly, H=w.H, g_top=w.gamma_top, g_bot=w.gamma_bot, alpha=w.alpha,
                    rc=w.r_c, M=w.M, P=w.P, Lz=Lz)


def gpu_slab(R, w, precision=None, n_max=None, **over):
    kw = w.slab_kwargs(**over)
    return R.Slab(**kw, precision=precision or w.precision, n_max=w.N if n_max is None else n_max)


def to_dev(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")
