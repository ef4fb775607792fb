"""RBE2D oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.

Plain FP64 CPU reference for the random batch Ewald method for dielectrically
confined quasi-2D Coulomb systems (Gan, Gao, Liang, Xu, arXiv:2405.06333).
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library.

Contents
  * ctypes wrapper around ``liborc.so`` (``rbe2d_oracle.c``): k-space with
    explicit images or Y-recalibration, IBC, self, brute-force real space;
  * host parameters written out from the paper: the extended height
    (Eq. (3.23)), the normalising constant S (Eq. (2.21)), the k-sampling
    distribution (Sec. 2.3) and its seeded exact sampler;
  * exact definitions used to pin the above: Ewald2D applied to the charges
    plus their images (Eqs. (2.6)-(2.9) with Eq. (3.2) as the source set),
    brute-force lattice summation of Eq. (3.2), the deterministic k-sum of
    Theorem 3.3.

Readings of garbled passages are listed at the top of ``rbe2d_oracle.c``.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle  # noqa: WPS433 (local import on demand)
            build_oracle.build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


class _Box(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("H", ctypes.c_double),
                ("Lz", ctypes.c_double), ("g_top", ctypes.c_double), ("g_bot", ctypes.c_double),
                ("alpha", ctypes.c_double), ("rc", ctypes.c_double), ("M", ctypes.c_int)]


_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _declare(L):
    L.orc_image_coeffs.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _D, _D]
    L.orc_image_z.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.orc_image_z.restype = ctypes.c_double
    L.orc_rho.argtypes = [ctypes.c_int64, _D, _D, ctypes.POINTER(_Box), ctypes.c_int, _I32,
                          ctypes.c_int, _D]
    L.orc_rhoM_explicit.argtypes = [ctypes.c_int64, _D, _D, ctypes.POINTER(_Box), ctypes.c_int,
                                    _I32, _D]
    L.orc_Y.argtypes = [ctypes.POINTER(_Box), ctypes.c_int, _I32, _D, _D]
    L.orc_kspace.argtypes = [ctypes.c_int64, _D, _D, ctypes.POINTER(_Box), ctypes.c_int, _I32,
                             _D, ctypes.c_int, ctypes.c_int64, _I64, _D, _D, _D, _D, _D, _D]
    L.orc_kspace_dgamma.argtypes = [ctypes.c_int64, _D, _D, ctypes.POINTER(_Box), ctypes.c_int,
                                    _I32, _D, ctypes.c_int]
    L.orc_kspace_dgamma.restype = ctypes.c_double
    L.orc_ibc.argtypes = [ctypes.c_int64, _D, _D, ctypes.POINTER(_Box), ctypes.c_int64, _I64,
                          _D, _D, _D, _D]
    L.orc_self.argtypes = [ctypes.c_int64, _D, ctypes.c_double]
    L.orc_self.restype = ctypes.c_double
    L.orc_real.argtypes = [ctypes.c_int64, _D, _D, ctypes.POINTER(_Box), ctypes.c_int64, _I64,
                           _D, _D, _D, _D]
    L.orc_surface.argtypes = [ctypes.c_int64, _D, _D, ctypes.POINTER(_Box), ctypes.c_double, ctypes.c_double,
                              ctypes.c_int64, _I64, _D, _D, _D, _D]
    L.orc_short.argtypes = [ctypes.c_int64, _D, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D, _D]


def _p(a, t=_D):
    return None if a is None else a.ctypes.data_as(t)


@dataclass
class Slab:
    """Parameters of one dielectrically confined slab (Sec. 3.1).

    ``Lz`` is the extended periodic height of Theorem 3.3; ``Lz=None`` takes
    the smallest value allowed by Eq. (3.23) at tolerance ``eps_lz``.
    """
    Lx: float
    Ly: float
    H: float
    g_top: float
    g_bot: float
    alpha: float
    rc: float
    M: int
    P: int
    Lz: float | None = None
    eps_lz: float = 1e-6

    def __post_init__(self):
        if self.Lz is None or self.Lz <= 0:
            self.Lz = lz_ext(self.Lx, self.Ly, self.H, self.M, self.alpha, self.eps_lz)

    @property
    def V(self) -> float:
        return self.Lx * self.Ly * self.Lz

    def box(self, g_top=None, g_bot=None) -> _Box:
        return _Box(self.Lx, self.Ly, self.H, self.Lz,
                    self.g_top if g_top is None else g_top,
                    self.g_bot if g_bot is None else g_bot,
                    self.alpha, self.rc, self.M)


# ---------------------------------------------------------------------------
# Host parameters
# ---------------------------------------------------------------------------

def lz_ext(Lx, Ly, H, M, alpha, eps):
    """Extended height from the criterion of Eq. (3.23), taken with equality."""
    lg = math.log(1.0 / eps)
    return (M + 1) * H + max(max(Lx, Ly) / (2.0 * math.pi) * lg, math.sqrt(lg) / alpha)


def theta(alpha, L):
    """sum over n in Z of exp(-pi^2 n^2 / (alpha^2 L^2)): the one-axis factor of S."""
    s = 1.0
    n = 1
    while True:
        t = math.exp(-(math.pi * math.pi) * float(n * n) / (alpha * alpha * L * L))
        if t < 1e-300:
            break
        s += 2.0 * t
        n += 1
    return s


def norm_S(alpha, Lx, Ly, Lz):
    """S = sum_{k != 0} exp(-k^2 / 4 alpha^2), Eq. (2.21): the sum factorises
    over the three axes of the extended box."""
    return theta(alpha, Lx) * theta(alpha, Ly) * theta(alpha, Lz) - 1.0


def image_coeffs(M, g_top, g_bot):
    gp = np.zeros(max(M, 1))
    gm = np.zeros(max(M, 1))
    lib().orc_image_coeffs(M, g_top, g_bot, _p(gp), _p(gm))
    return gp[:M].copy(), gm[:M].copy()


def image_z(l, sign, z, H):
    return lib().orc_image_z(l, sign, z, H)


# ---------------------------------------------------------------------------
# Seeded exact sampler of the k-set (Sec. 2.3; R: i.i.d. with replacement)
# ---------------------------------------------------------------------------
# SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
# generators", OOPSLA 2014) used in counter mode.

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def _mix64(z):
    z &= _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _stream_key(seed, stream):
    base = _mix64(seed)
    return _mix64((base + (stream + 1) * _GOLDEN) & _M64)


def _uniform(key, counter):
    return (_mix64((key + (counter + 1) * _GOLDEN) & _M64) >> 11) * (1.0 / 9007199254740992.0)


def axis_cdf(alpha, L):
    """Cumulative distribution of n on one axis, P(n) ~ exp(-pi^2 n^2/(alpha^2 L^2)),
    truncated at |n| <= nmax = ceil(10 sigma) + 1, sigma = alpha L / (sqrt(2) pi)."""
    sigma = 10.0 * alpha * L / (math.sqrt(2.0) * math.pi)
    nmax = int(math.ceil(sigma)) + 1
    w = []
    for v in range(-nmax, nmax + 1):
        w.append(math.exp(-(math.pi * math.pi) * float(v * v) / (alpha * alpha * L * L)))
    cdf = []
    acc = 0.0
    for x in w:
        acc += x
        cdf.append(acc)
    tot = acc
    return nmax, [c / tot for c in cdf]


def _draw_axis(nmax, cdf, u):
    lo, hi = 0, len(cdf) - 1
    while lo < hi:                       # smallest m with u < cdf[m]
        mid = (lo + hi) // 2
        if u < cdf[mid]:
            hi = mid
        else:
            lo = mid + 1
    return lo - nmax


def draw_kset(slab: Slab, seed: int, stream: int = 0, P: int | None = None):
    """P i.i.d. integer vectors n != 0 with P(n) ~ exp(-k^2/4 alpha^2),
    k = 2 pi (nx/Lx, ny/Ly, nz/Lz): per-axis inverse CDF, redraw on n = 0
    (at most 64 attempts per vector)."""
    P = slab.P if P is None else P
    tabs = [axis_cdf(slab.alpha, L) for L in (slab.Lx, slab.Ly, slab.Lz)]
    key = _stream_key(seed & _M64, stream & _M64)
    out = np.zeros((P, 3), dtype=np.int32)
    for l in range(P):
        for a in range(64):
            n = [_draw_axis(*tabs[d], _uniform(key, (l * 64 + a) * 3 + d)) for d in range(3)]
            if n != [0, 0, 0]:
                out[l] = n
                break
        else:
            raise RuntimeError("k-sampler: 64 consecutive zero vectors")
    return out


def kvectors(slab: Slab, n):
    n = np.asarray(n, dtype=np.float64)
    return 2.0 * np.pi * n / np.array([slab.Lx, slab.Ly, slab.Lz])


def rbe_weights(slab: Slab, n, S=None):
    """Importance weights of the RBE estimator, Eq. (3.26): 2 pi S / (V P k^2)."""
    S = norm_S(slab.alpha, slab.Lx, slab.Ly, slab.Lz) if S is None else S
    k = kvectors(slab, n)
    k2 = (k * k).sum(axis=1)
    return 2.0 * np.pi * S / (slab.V * len(n) * k2)


def full_kset(slab: Slab, cut=40.0):
    """Every n != 0 with k^2/(4 alpha^2) <= cut, and the deterministic weights
    (2 pi / V) exp(-k^2/4 alpha^2)/k^2 of Eq. (3.16)."""
    lim = [int(math.ceil(math.sqrt(cut) * slab.alpha * L / math.pi)) + 1
           for L in (slab.Lx, slab.Ly, slab.Lz)]
    ax = [np.arange(-m, m + 1) for m in lim]
    g = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1).reshape(-1, 3)
    k = kvectors(slab, g)
    x = (k * k).sum(axis=1) / (4.0 * slab.alpha ** 2)
    keep = (x <= cut) & (np.abs(g).sum(axis=1) > 0)
    g = g[keep].astype(np.int32)
    k2 = (k[keep] ** 2).sum(axis=1)
    c = 2.0 * np.pi / slab.V * np.exp(-k2 / (4.0 * slab.alpha ** 2)) / k2
    return g, c


# ---------------------------------------------------------------------------
# The RBE2D evaluation (Algorithm 2 / Theorem 3.3 / Eq. (3.26))
# ---------------------------------------------------------------------------

@dataclass
class Result:
    E_total: float
    E_real: float
    E_k: float
    E_self: float
    E_ibc: float
    F: np.ndarray          # (n_t, 3) total force
    F_real: np.ndarray
    F_k: np.ndarray
    F_ibc: np.ndarray
    phi: np.ndarray        # (n_t,) dE/dq

    def energies(self):
        return np.array([self.E_total, self.E_real, self.E_k, self.E_self, self.E_ibc])


def _prep(pos, q):
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    return pos, q


def kspace(slab: Slab, pos, q, n, c, explicit_images=False, targets=None, box=None):
    """E_k, F_k (targets), phi_k (targets), rho, rhohat, rhoM."""
    pos, q = _prep(pos, q)
    n = np.ascontiguousarray(n, dtype=np.int32).reshape(-1, 3)
    c = np.ascontiguousarray(c, dtype=np.float64)
    P = n.shape[0]
    tgt = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = len(q) if tgt is None else len(tgt)
    E = np.zeros(1)
    F = np.zeros((nt, 3))
    phi = np.zeros(nt)
    rho = np.zeros(2 * P)
    rhohat = np.zeros(2 * P)
    rhoM = np.zeros(2 * P)
    b = slab.box() if box is None else box
    lib().orc_kspace(len(q), _p(pos), _p(q), ctypes.byref(b), P, _p(n, _I32), _p(c),
                     int(bool(explicit_images)), nt, _p(tgt, _I64), _p(E), _p(F), _p(phi),
                     _p(rho), _p(rhohat), _p(rhoM))
    cz = lambda a: a[0::2] + 1j * a[1::2]  # noqa: E731
    return E[0], F, phi, cz(rho), cz(rhohat), cz(rhoM)


def ibc(slab: Slab, pos, q, targets=None, box=None):
    pos, q = _prep(pos, q)
    tgt = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = len(q) if tgt is None else len(tgt)
    E = np.zeros(1)
    F = np.zeros((nt, 3))
    phi = np.zeros(nt)
    dg = np.zeros(2)
    b = slab.box() if box is None else box
    lib().orc_ibc(len(q), _p(pos), _p(q), ctypes.byref(b), nt, _p(tgt, _I64),
                  _p(E), _p(F), _p(phi), _p(dg))
    return E[0], F, phi, dg


def real_space(slab: Slab, pos, q, targets=None, want_dgamma=False, box=None):
    pos, q = _prep(pos, q)
    tgt = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = len(q) if tgt is None else len(tgt)
    E = np.zeros(1)
    F = np.zeros((nt, 3))
    phi = np.zeros(nt)
    dphig = np.zeros((nt, 2)) if want_dgamma else None
    b = slab.box() if box is None else box
    lib().orc_real(len(q), _p(pos), _p(q), ctypes.byref(b), nt, _p(tgt, _I64),
                   _p(E), _p(F), _p(phi), _p(dphig))
    return E[0], F, phi, dphig


def surface(slab: Slab, pos, q, sig_top, sig_bot, targets=None, box=None):
    """Surface charge densities sig_top on z = H and sig_bot on z = 0 (the
    remark after Eq. (3.26); readings R7, R8 in rbe2d_oracle.c): the sheets'
    field on the ions and the net-charge term of the Lz-periodic k-sum.
    Returns (E, F (n_t, 3), phi (n_t,), dE/dgamma (2,))."""
    pos, q = _prep(pos, q)
    tgt = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = len(q) if tgt is None else len(tgt)
    E = np.zeros(1)
    F = np.zeros((nt, 3))
    phi = np.zeros(nt)
    dg = np.zeros(2)
    b = slab.box() if box is None else box
    lib().orc_surface(len(q), _p(pos), _p(q), ctypes.byref(b), float(sig_top), float(sig_bot), nt,
                      _p(tgt, _I64), _p(E), _p(F), _p(phi), _p(dg))
    return E[0], F, phi, dg


def self_energy(slab: Slab, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().orc_self(len(q), _p(q), slab.alpha)


def evaluate(slab: Slab, pos, q, n, c=None, explicit_images=False, targets=None,
             parts=("real", "kspace", "ibc"), sigma=None) -> Result:
    """Energy components, forces and dE/dq of the RBE2D splitting for a given
    k-set ``n`` with weights ``c`` (default: RBE weights of Eq. (3.26)).
    sigma = (sig_top, sig_bot): surface charge densities on the interfaces;
    their terms (``surface``) go with the IBC part."""
    pos, q = _prep(pos, q)
    nt = len(q) if targets is None else len(targets)
    z3 = np.zeros((nt, 3))
    if c is None:
        c = rbe_weights(slab, n)
    Er = Ek = Ei = 0.0
    Fr = Fk = Fi = z3
    phr = phk = phi_ = np.zeros(nt)
    if "real" in parts:
        Er, Fr, phr, _ = real_space(slab, pos, q, targets)
    if "kspace" in parts:
        Ek, Fk, phk, *_ = kspace(slab, pos, q, n, c, explicit_images, targets)
    if "ibc" in parts:
        Ei, Fi, phi_, _ = ibc(slab, pos, q, targets)
        if sigma is not None and (sigma[0] != 0.0 or sigma[1] != 0.0):
            Eu, Fu, phu, _ = surface(slab, pos, q, sigma[0], sigma[1], targets)
            Ei, Fi, phi_ = Ei + Eu, Fi + Fu, phi_ + phu
    Es = self_energy(slab, q) if "kspace" in parts else 0.0
    tq = q if targets is None else q[np.asarray(targets)]
    ph = phr + phk + phi_ + (-2.0 * slab.alpha / math.sqrt(math.pi) * tq if "kspace" in parts else 0.0)
    return Result(Er + Ek + Es + Ei, Er, Ek, Es, Ei, Fr + Fk + Fi, Fr, Fk, Fi, ph)


def dE_dgamma(slab: Slab, pos, q, n, c=None, sigma=None):
    """dE/dgamma_top, dE/dgamma_bot of the RBE2D energy at fixed k-set:
    real-space image weights (Eq. (3.12)), rho^M (Eq. (3.17)), the IBC
    image dipole (Theorem 3.3) and, with sigma, the surface terms."""
    pos, q = _prep(pos, q)
    if c is None:
        c = rbe_weights(slab, n)
    n = np.ascontiguousarray(n, dtype=np.int32).reshape(-1, 3)
    c = np.ascontiguousarray(c, dtype=np.float64)
    _, _, _, dphig = real_space(slab, pos, q, want_dgamma=True)
    dreal = 0.5 * (q[:, None] * dphig).sum(axis=0)
    b = slab.box()
    dk = np.array([lib().orc_kspace_dgamma(len(q), _p(pos), _p(q), ctypes.byref(b), len(n),
                                           _p(n, _I32), _p(c), w) for w in (0, 1)])
    _, _, _, dibc = ibc(slab, pos, q)
    if sigma is not None and (sigma[0] != 0.0 or sigma[1] != 0.0):
        dibc = dibc + surface(slab, pos, q, sigma[0], sigma[1])[3]
    return dreal + dk + dibc


# ---------------------------------------------------------------------------
# Exact definitions used as pins
# ---------------------------------------------------------------------------

def image_sources(slab: Slab, pos, q, M=None):
    """Real charges plus every image up to order M (Eq. (3.2), (3.3)):
    returns (src_pos, src_charge_times_weight, owner_index, is_real)."""
    pos, q = _prep(pos, q)
    M = slab.M if M is None else M
    gp, gm = image_coeffs(M, slab.g_top, slab.g_bot)
    sp, sq, own, real = [], [], [], []
    for j in range(len(q)):
        sp.append(pos[j]); sq.append(q[j]); own.append(j); real.append(True)
        for l in range(1, M + 1):
            for sgn, g in ((+1, gp[l - 1]), (-1, gm[l - 1])):
                p = pos[j].copy()
                p[2] = image_z(l, sgn, pos[j, 2], slab.H)
                sp.append(p); sq.append(q[j] * g); own.append(j); real.append(False)
    return np.array(sp), np.array(sq), np.array(own), np.array(real)


def ewald2d_images(slab: Slab, pos, q, alpha=None, nreal=4, hcut=40.0, parts=("real", "fourier")):
    """Energy of the truncated image system, U^c_M = 1/2 sum_i q_i phi_M(r_i),
    by the exact Ewald2D formulas (Eqs. (2.6)-(2.9)) applied with the real
    charges as targets and the real charges plus their images as sources.
    ``parts`` selects the erfc (real-space) part and/or the long-range part
    (the reciprocal sum of Eq. (2.7), the zero mode of Eq. (2.9) and the
    self-energy correction), whose sum is the energy; the long-range part
    alone is what the Fourier expression of Theorem 3.3 approximates.
    O(N^2 M) -- for small N only."""
    from scipy.special import erfc, erf, erfcx
    pos, q = _prep(pos, q)
    a = slab.alpha if alpha is None else alpha
    Lx, Ly = slab.Lx, slab.Ly
    sp, sq, own, real = image_sources(slab, pos, q)
    N = len(q)
    U = 0.0
    # reciprocal lattice h != 0 with h^2/(4 a^2) <= hcut
    mx = int(math.ceil(2 * a * math.sqrt(hcut) * Lx / (2 * math.pi))) + 1
    my = int(math.ceil(2 * a * math.sqrt(hcut) * Ly / (2 * math.pi))) + 1
    hx, hy = np.meshgrid(2 * np.pi * np.arange(-mx, mx + 1) / Lx,
                         2 * np.pi * np.arange(-my, my + 1) / Ly, indexing="ij")
    hx, hy = hx.ravel(), hy.ravel()
    h = np.hypot(hx, hy)
    keep = (h > 0) & (h * h / (4 * a * a) <= hcut)
    hx, hy, h = hx[keep], hy[keep], h[keep]
    nx, ny = np.meshgrid(np.arange(-nreal, nreal + 1), np.arange(-nreal, nreal + 1), indexing="ij")
    shifts = np.stack([nx.ravel() * Lx, ny.ravel() * Ly, 0 * nx.ravel()], axis=1)
    for i in range(N):
        phi = 0.0
        d = pos[i][None, :] - sp                       # (S,3)
        if "real" in parts:
            # real space: all lattice shifts, excluding the (i, n=0) self term
            r = d[:, None, :] + shifts[None, :, :]
            rr = np.sqrt((r ** 2).sum(axis=2))
            self_mask = (own == i) & real
            zero_shift = (shifts[:, 0] == 0) & (shifts[:, 1] == 0)
            excl = self_mask[:, None] & zero_shift[None, :]
            rr_safe = np.where(excl, 1.0, rr)
            phi += (sq[:, None] * np.where(excl, 0.0, erfc(a * rr_safe) / rr_safe)).sum()
        if "fourier" not in parts:
            U += 0.5 * q[i] * phi
            continue
        # Fourier part, Eq. (2.7): (pi/(Lx Ly)) sum_h' e^{i h.rho} G_a(h, z)/h
        z = d[:, 2]
        ph = np.cos(np.outer(d[:, 0], hx) + np.outer(d[:, 1], hy))   # (S, nh)
        u1 = h[None, :] / (2 * a) + a * z[:, None]
        u2 = h[None, :] / (2 * a) - a * z[:, None]
        base = np.exp(-h[None, :] ** 2 / (4 * a * a) - a * a * z[:, None] ** 2)

        def term(u, sgn):
            # e^{sgn h z} erfc(u), evaluated through erfcx where u >= 0
            with np.errstate(over="ignore", under="ignore"):
                direct = np.exp(sgn * h[None, :] * z[:, None]) * erfc(np.minimum(u, 0.0))
            return np.where(u >= 0, erfcx(np.maximum(u, 0.0)) * base, direct)

        G = term(u1, +1.0) + term(u2, -1.0)
        phi += math.pi / (Lx * Ly) * (sq[:, None] * ph * G / h[None, :]).sum()
        # zero mode J0, Eq. (2.9)
        phi += (-2 * math.pi / (Lx * Ly) * sq * (z * erf(a * z) + np.exp(-a * a * z * z) / (a * math.sqrt(math.pi)))).sum()
        # self-energy correction
        phi += -2 * a / math.sqrt(math.pi) * q[i]
        U += 0.5 * q[i] * phi
    return U


def brute_force_images(slab: Slab, pos, q, R):
    """1/2 sum_i q_i sum_s' q_s w_s / |r_i - r_s + l| over the lattice vectors
    |n| <= R (a disk), Eq. (3.2) truncated at order M.  The disk sum
    converges like 1/R; use ``richardson`` on (R, 2R)."""
    pos, q = _prep(pos, q)
    sp, sq, own, real = image_sources(slab, pos, q)
    n = np.arange(-R, R + 1)
    nx, ny = np.meshgrid(n, n, indexing="ij")
    disk = (nx ** 2 + ny ** 2) <= R * R
    sh = np.stack([nx[disk] * slab.Lx, ny[disk] * slab.Ly], axis=1)
    zero = (sh[:, 0] == 0) & (sh[:, 1] == 0)
    U = 0.0
    for i in range(len(q)):
        acc = 0.0
        for s in range(len(sq)):
            d = pos[i] - sp[s]
            dx = d[0] + sh[:, 0]
            dy = d[1] + sh[:, 1]
            r = np.sqrt(dx * dx + dy * dy + d[2] * d[2])
            if own[s] == i and real[s]:
                r = r[~zero]
            acc += sq[s] * np.sum(1.0 / r)
        U += 0.5 * q[i] * acc
    return U


def richardson(u_r, u_2r):
    """Eliminates the 1/R term of the disk summation."""
    return 2.0 * u_2r - u_r


def deterministic_energy(slab: Slab, pos, q, cut=40.0):
    """U^c_M from the reformulation of Theorem 3.3 with the full k-sum
    (ELC and remainder terms dropped) -- the quantity RBE estimates."""
    n, c = full_kset(slab, cut)
    return evaluate(slab, pos, q, n, c)


# ---------------------------------------------------------------------------
# MD around the path (Sec. 3.5 and Sec. 4.1): short-range forces and one
# Langevin step.  Test infrastructure like everything in this module.
# ---------------------------------------------------------------------------

def short_range(pos, Lx, Ly, H, sigma, eps, sigma_w, eps_w):
    """Purely repulsive shifted-truncated LJ between ions and against the two
    walls (brute force).  Returns (F (N,3), E_pair, E_wall)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    N = pos.shape[0]
    F = np.zeros((N, 3))
    ep = ctypes.c_double()
    ew = ctypes.c_double()
    lib().orc_short(N, _p(pos), Lx, Ly, H, sigma, eps, sigma_w, eps_w, _p(F), ctypes.byref(ep),
                    ctypes.byref(ew))
    return F, ep.value, ew.value


THERMO_STREAM = 1 << 63   # stream ids of the thermostat noise: this bit set


def thermo_normals(seed, stream, n):
    """n x 3 standard normals of the Langevin noise: SplitMix64 counter-mode
    uniforms (the k-sampler's generator, stream id with the top bit set) and
    the Box-Muller transform (cosine branch): for particle i and component c,
    u1, u2 = uniforms 2(3i+c), 2(3i+c)+1 and xi = sqrt(-2 ln(1-u1)) cos(2 pi u2)."""
    key = _stream_key(seed, (THERMO_STREAM + stream) & _M64)
    out = np.empty((n, 3))
    for i in range(n):
        for c in range(3):
            k = 3 * i + c
            u1 = _uniform(key, 2 * k)
            u2 = _uniform(key, 2 * k + 1)
            out[i, c] = math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)
    return out


def fold_z(z, v, zlo, zhi):
    """Specular reflection at zlo and zhi, applied as often as needed."""
    W = zhi - zlo
    u = z - zlo
    m = math.floor(u / W)
    rem = u - m * W
    if int(abs(m)) % 2 == 1:
        return zhi - rem, -v
    return zlo + rem, v


def baoab_step(pos, vel, F, dt, gamma, kT, normals, Lx, Ly, zlo, zhi, force):
    """One BAOAB step (Leimkuhler and Matthews, 2013) of the Langevin equation
    of Sec. 3.5 with unit masses: v += dt/2 F; r += dt/2 v;
    v = c1 v + c2 xi (c1 = exp(-gamma dt), c2 = sqrt((1 - c1^2) kT));
    r += dt/2 v; x, y wrapped, z reflected at zlo, zhi; F = force(r);
    v += dt/2 F.  With gamma = 0 it is velocity Verlet."""
    c1 = math.exp(-gamma * dt)
    c2 = math.sqrt((1.0 - c1 * c1) * kT)
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    vel = vel + 0.5 * dt * F
    pos = pos + 0.5 * dt * vel
    vel = c1 * vel + c2 * normals
    pos = pos + 0.5 * dt * vel
    pos[:, 0] -= Lx * np.floor(pos[:, 0] / Lx)
    pos[:, 1] -= Ly * np.floor(pos[:, 1] / Ly)
    for i in range(pos.shape[0]):
        pos[i, 2], vel[i, 2] = fold_z(pos[i, 2], vel[i, 2], zlo, zhi)
    Fn = force(pos)
    vel = vel + 0.5 * dt * Fn
    return pos, vel, Fn


# ---------------------------------------------------------------------------
# Parameter selection (Sec. 2.4, Theorem 3.2, Eq. (3.23)) and the stochastic
# error of the k-space force (Theorem 2.2).  Test infrastructure.
# ---------------------------------------------------------------------------

def image_truncation_estimate(M, g_top, g_bot, H, Lmax):
    """Eq. (3.9) with unit constant: |g_top|^floor((M+1)/2) |g_bot|^ceil((M+1)/2)
    exp(-2 pi H (M-1) / max(Lx, Ly))."""
    a = abs(g_top) ** ((M + 1) // 2) if (M + 1) // 2 else 1.0
    b = abs(g_bot) ** ((M + 2) // 2) if (M + 2) // 2 else 1.0
    return a * b * math.exp(-2.0 * math.pi * H * (M - 1) / Lmax)


def image_order_for(tol, g_top, g_bot, H, Lmax, M_max=64):
    """Smallest M >= 0 whose Eq. (3.9) estimate is at most tol (Theorem 3.2)."""
    for M in range(0, M_max + 1):
        if image_truncation_estimate(M, g_top, g_bot, H, Lmax) <= tol:
            return M
    return M_max


def suggest_params(N, Lx, Ly, H, g_top, g_bot, tol):
    """alpha = (N / (Lx Ly H))^(1/3) (Sec. 2.4, independent of Lz); r_c such
    that the real-space tail exp(-alpha^2 r_c^2) is tol, at most min(Lx, Ly)/2
    (then alpha follows r_c); M from Theorem 3.2; Lz from Eq. (3.23) at tol."""
    lg = math.log(1.0 / tol)
    alpha = (N / (Lx * Ly * H)) ** (1.0 / 3.0)
    rc = math.sqrt(lg) / alpha
    if rc > 0.5 * min(Lx, Ly):
        rc = 0.5 * min(Lx, Ly)
        alpha = math.sqrt(lg) / rc
    M = image_order_for(tol, g_top, g_bot, H, max(Lx, Ly))
    Lz = lz_ext(Lx, Ly, H, M, alpha, tol)
    return dict(alpha=alpha, r_c=rc, M=M, Lz=Lz)


def kspace_terms(slab: Slab, pos, q, n, c):
    """Per-k contributions t_l(i) to the k-space force (Eqs. (3.25)-(3.26),
    reading R2): -q_i c_l [k_l Im(e^{-i k_l.r_i} A_l) + khat_l Im(e^{-i khat_l.r_i} B_l)],
    A = rho^M + (1 + conj Y_even) rho, B = conj(Y_odd) rho.  Shape (P, N, 3)."""
    pos, q = _prep(pos, q)
    n = np.ascontiguousarray(n, dtype=np.int32).reshape(-1, 3)
    P = n.shape[0]
    b = slab.box()
    rho = np.zeros(2 * P)
    rhohat = np.zeros(2 * P)
    lib().orc_rho(len(q), _p(pos), _p(q), ctypes.byref(b), P, _p(n, _I32), 0, _p(rho))
    lib().orc_rho(len(q), _p(pos), _p(q), ctypes.byref(b), P, _p(n, _I32), 1, _p(rhohat))
    Yo = np.zeros(2 * P)
    Ye = np.zeros(2 * P)
    lib().orc_Y(ctypes.byref(b), P, _p(n, _I32), _p(Yo), _p(Ye))
    cz = lambda a: a[0::2] + 1j * a[1::2]  # noqa: E731
    rho, rhohat, Yo, Ye = cz(rho), cz(rhohat), cz(Yo), cz(Ye)
    rhoM = (1 + Ye) * rho + Yo * rhohat
    A = rhoM + (1 + np.conj(Ye)) * rho
    B = np.conj(Yo) * rho
    k = kvectors(slab, n)
    kh = k * np.array([1.0, 1.0, -1.0])
    ph = pos @ k.T          # (N, P)
    phh = pos @ kh.T
    X = np.imag(np.exp(-1j * ph) * A[None, :])
    Y = np.imag(np.exp(-1j * phh) * B[None, :])
    t = -(q[:, None, None] * np.asarray(c)[None, :, None]) * (X[:, :, None] * k[None] + Y[:, :, None] * kh[None])
    return np.transpose(t, (1, 0, 2))


def force_variance_estimate(slab: Slab, pos, q, n, c=None):
    """Unbiased estimate, from one batch, of E|Xi_i|^2 of Theorem 2.2 (the
    variance of the RBE k-space force of particle i): the per-k terms are
    i.i.d. given the positions, F = sum_l t_l, so the sample variance gives
    (P sum_l |t_l|^2 - |F|^2) / (P - 1)."""
    n = np.asarray(n).reshape(-1, 3)
    P = n.shape[0]
    c = rbe_weights(slab, n) if c is None else c
    t = kspace_terms(slab, pos, q, n, c)
    F = t.sum(axis=0)
    return (P * (t * t).sum(axis=(0, 2)) - (F * F).sum(axis=1)) / (P - 1)


def force_variance_exact(slab: Slab, pos, q, P, cut=40.0):
    """Theorem 2.2 written out over every k (deterministic sum): with per-k force
    g(k) = P t(k) at batch weight 2 pi S/(V P k^2) and sampling probability
    p(k) = exp(-k^2/4alpha^2)/S, E|Xi_i|^2 = (sum_k p(k) |g_i(k)|^2 - |F_i|^2)/P,
    F_i = sum_k p(k) g_i(k) the deterministic k-space force."""
    n, _ = full_kset(slab, cut)
    S = norm_S(slab.alpha, slab.Lx, slab.Ly, slab.Lz)
    k = kvectors(slab, n)
    k2 = (k * k).sum(axis=1)
    pk = np.exp(-k2 / (4.0 * slab.alpha ** 2)) / S
    g = kspace_terms(slab, pos, q, n, 2.0 * np.pi * S / (slab.V * k2))   # one sample's force, P = 1
    F = (pk[:, None, None] * g).sum(axis=0)
    second = (pk[:, None] * (g * g).sum(axis=2)).sum(axis=0)
    return (second - (F * F).sum(axis=1)) / P
