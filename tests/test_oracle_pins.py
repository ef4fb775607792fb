"""Pins of the CPU oracle against what the paper and the mathematics fix.

No test here compares the oracle with itself: each checks it against an
independent definition (Ewald2D, brute-force lattice sums, the interface
conditions of electrostatics), an exact identity, an invariant, or a
statistical property stated by the paper's theorems.
"""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def small_system(seed, N=6, L=10.0, H=4.0, margin=0.5, q=None):
    rng = np.random.default_rng(seed)
    pos = np.c_[rng.uniform(0, L, N), rng.uniform(0, L, N), rng.uniform(margin, H - margin, N)]
    if q is None:
        q = np.array([1.0, -1.0] * (N // 2))
    return pos, q


# --------------------------------------------------------------------------
# Image series (Sec. 3.1): weights and positions
# --------------------------------------------------------------------------

def test_single_interface_is_one_jackson_image(orc):
    """With gamma_top = 0 the only image is the one of the lower interface,
    at -z with weight gamma_bot (textbook single dielectric interface)."""
    H = 3.0
    gp, gm = orc.image_coeffs(6, 0.0, 0.6)
    assert np.all(gp == 0.0)
    assert gm[0] == pytest.approx(0.6) and np.all(gm[1:] == 0.0)
    assert orc.image_z(1, -1, 0.7, H) == pytest.approx(-0.7)
    gp, gm = orc.image_coeffs(6, -0.3, 0.0)
    assert np.all(gm == 0.0)
    assert gp[0] == pytest.approx(-0.3) and np.all(gp[1:] == 0.0)
    assert orc.image_z(1, +1, 0.7, H) == pytest.approx(2 * H - 0.7)


def _layered_reflection(h, z, zp, H, g_top, g_bot, deriv=False):
    """Reflected part of the xy-Fourier-transformed potential of a unit charge
    at z' in the middle layer of a three-layer dielectric (eps_c = 1),
    obtained by imposing continuity of phi and of eps dphi/dz at z = 0 and
    z = H (4x4 linear solve).  Returns R(z) with phi_hat = 2pi/h e^{-h|z-z'|} + R
    (with deriv, dR/dz instead)."""
    e_top = (1 - g_top) / (1 + g_top)
    e_bot = (1 - g_bot) / (1 + g_bot)
    G0 = 2 * np.pi / h
    # unknowns [A (top: A e^{-hz}), B, C (middle: B e^{hz} + C e^{-hz}), D (bottom: D e^{hz})]
    eH, emH = np.exp(h * H), np.exp(-h * H)
    Amat = np.array([
        [0.0, 1.0, 1.0, -1.0],                     # phi continuous at 0
        [0.0, 1.0, -1.0, -e_bot],                  # eps dphi/dz continuous at 0 (divided by h)
        [-emH, eH, emH, 0.0],                      # phi continuous at H
        [e_top * emH, eH, -emH, 0.0],              # eps dphi/dz continuous at H (divided by h)
    ])
    rhs = np.array([
        -G0 * np.exp(-h * zp),
        -G0 * np.exp(-h * zp),
        -G0 * np.exp(-h * (H - zp)),
        G0 * np.exp(-h * (H - zp)),
    ])
    A, B, C, D = np.linalg.solve(Amat, rhs)
    if deriv:
        return h * (B * np.exp(h * z) - C * np.exp(-h * z))
    return B * np.exp(h * z) + C * np.exp(-h * z)


@pytest.mark.parametrize("g_top,g_bot", [(0.7, -0.4), (-0.9, 0.95), (0.5, 0.5), (0.0, 0.8), (-0.6, 0.0)])
def test_image_series_solves_interface_conditions(orc, g_top, g_bot):
    """The image series with the oracle's weights and positions reproduces
    the exact layered-medium response (this pins reading R1: the printed
    exponent assignment fails this test whenever gamma_top != gamma_bot)."""
    H = 1.3
    M = 120
    gp, gm = orc.image_coeffs(M, g_top, g_bot)
    rng = np.random.default_rng(0)
    for _ in range(20):
        h = rng.uniform(0.2, 3.0)
        z, zp = rng.uniform(0.05, H - 0.05, 2)
        beta = sum(gp[l - 1] * np.exp(-h * abs(z - orc.image_z(l, +1, zp, H)))
                   + gm[l - 1] * np.exp(-h * abs(z - orc.image_z(l, -1, zp, H)))
                   for l in range(1, M + 1))
        ref = _layered_reflection(h, z, zp, H, g_top, g_bot)
        assert 2 * np.pi / h * beta == pytest.approx(ref, rel=1e-10, abs=1e-12)


def test_image_series_matches_closed_form_beta(orc):
    """Eqs. (3.6)-(3.8): the summed image series equals the closed form
    beta_ij(h) = [g_b e^{-h|zi+zj|} + g_t e^{-h|2H-(zi+zj)|}
                  + g_t g_b (e^{-h|2H-zij|} + e^{-h|2H+zij|})] zeta(h)."""
    H, gt, gb = 2.0, 0.8, -0.6
    gp, gm = orc.image_coeffs(200, gt, gb)
    for h, zi, zj in [(0.3, 0.4, 1.7), (1.1, 1.9, 0.2), (2.5, 1.0, 1.0)]:
        s = sum(gp[l - 1] * np.exp(-h * abs(zi - orc.image_z(l, +1, zj, H)))
                + gm[l - 1] * np.exp(-h * abs(zi - orc.image_z(l, -1, zj, H)))
                for l in range(1, 201))
        zij = zi - zj
        closed = (gb * np.exp(-h * abs(zi + zj)) + gt * np.exp(-h * abs(2 * H - zi - zj))
                  + gt * gb * (np.exp(-h * abs(2 * H - zij)) + np.exp(-h * abs(2 * H + zij)))) \
            / (1 - gt * gb * np.exp(-2 * h * H))
        assert s == pytest.approx(closed, rel=1e-12)


# --------------------------------------------------------------------------
# Host parameters
# --------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,Lx,Ly,Lz", [(1.0, 20, 20, 49.0), (0.5, 50, 50, 199.9), (0.3, 800, 800, 2199.0),
                                          (2.0, 3.0, 4.0, 5.0)])
def test_S_by_poisson_summation(orc, alpha, Lx, Ly, Lz):
    """S of Eq. (2.21) against the Poisson-dual form of each theta factor,
    sum_n e^{-pi^2 n^2/(a L)^2} = (a L/sqrt(pi)) sum_m e^{-a^2 L^2 m^2}."""
    S = orc.norm_S(alpha, Lx, Ly, Lz)

    def dual(L):
        return alpha * L / math.sqrt(math.pi) * (1 + 2 * sum(math.exp(-(alpha * L * m) ** 2) for m in range(1, 20)))

    assert S == pytest.approx(dual(Lx) * dual(Ly) * dual(Lz) - 1.0, rel=1e-13)
    # and the bound of Eq. (2.25)
    assert S <= alpha ** 3 * Lx * Ly * Lz / math.pi ** 1.5 * (1 + 1e-9) or alpha * min(Lx, Ly, Lz) < 2


def test_S_by_direct_lattice_sum(orc):
    a, L = 0.9, (3.0, 3.5, 6.0)
    S = orc.norm_S(a, *L)
    rng = range(-40, 41)
    direct = 0.0
    for nx in rng:
        for ny in rng:
            for nz in rng:
                if nx == ny == nz == 0:
                    continue
                k2 = sum((2 * math.pi * n / l) ** 2 for n, l in zip((nx, ny, nz), L))
                direct += math.exp(-k2 / (4 * a * a))
    assert S == pytest.approx(direct, rel=1e-13)


# --------------------------------------------------------------------------
# Exact definitions: Ewald2D with images vs brute-force lattice summation
# --------------------------------------------------------------------------

CASES = [(0.0, 0.0, 0), (0.7, -0.4, 3), (0.5, 0.5, 2), (-0.95, 0.9, 1)]


@pytest.mark.parametrize("g_top,g_bot,M", CASES)
def test_ewald2d_images_alpha_independent(orc, g_top, g_bot, M):
    pos, q = small_system(1)
    s = orc.Slab(Lx=10, Ly=10, H=4, g_top=g_top, g_bot=g_bot, alpha=1.0, rc=4.9, M=M, P=10)
    u1 = orc.ewald2d_images(s, pos, q, alpha=1.0)
    u2 = orc.ewald2d_images(s, pos, q, alpha=0.6, nreal=6)
    assert u1 == pytest.approx(u2, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("g_top,g_bot,M", CASES[:3])
def test_ewald2d_images_equals_bruteforce(orc, g_top, g_bot, M):
    """Eq. (3.2) truncated at M by direct 1/r summation over a disk of lattice
    cells (radius R, 2R cells), Richardson-extrapolated, vs Ewald2D."""
    pos, q = small_system(2, N=4)
    s = orc.Slab(Lx=10, Ly=10, H=4, g_top=g_top, g_bot=g_bot, alpha=1.0, rc=4.9, M=M, P=10)
    u = orc.ewald2d_images(s, pos, q)
    ub = orc.richardson(orc.brute_force_images(s, pos, q, 80), orc.brute_force_images(s, pos, q, 160))
    assert ub == pytest.approx(u, rel=2e-6)


# --------------------------------------------------------------------------
# The reformulation of Theorem 3.3 (oracle k-space + IBC + self + real)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("g_top,g_bot,M", CASES)
def test_reformulation_converges_to_ewald2d(orc, g_top, g_bot, M):
    """Deterministic k-sum + U_IBC^M + self + real space (the oracle's pieces,
    all weights deterministic) tends to Ewald2D with images as the vacuum
    layer grows, at the rate exp(-2 pi (Lz - (M+1)H)/L) of Eq. (3.21)."""
    pos, q = small_system(3)
    H = 4.0
    s = orc.Slab(Lx=10, Ly=10, H=H, g_top=g_top, g_bot=g_bot, alpha=1.0, rc=4.9, M=M, P=10)
    u = orc.ewald2d_images(s, pos, q)
    errs = []
    for extra in (8.0, 14.0, 26.0):
        s2 = orc.Slab(Lx=10, Ly=10, H=H, g_top=g_top, g_bot=g_bot, alpha=1.0, rc=4.9, M=M, P=10,
                      Lz=(M + 1) * H + extra)
        errs.append(abs(orc.deterministic_energy(s2, pos, q).E_total - u))
    assert errs[-1] < 2e-6 * max(1.0, abs(u))
    assert errs[0] > errs[1] > errs[2] or errs[0] < 1e-9


LZ_CASES = [
    # g_top, g_bot, M, alpha, L, eps, branch of Eq. (3.23) that sets the height
    (1.0, 1.0, 2, 1.0, 10.0, 1e-3, "elc"),
    (1.0, 1.0, 2, 1.0, 10.0, 1e-5, "elc"),
    (0.95, -0.95, 3, 1.0, 10.0, 1e-5, "elc"),
    (1.0, 1.0, 2, 0.1, 10.0, 1e-5, "err"),
    (-1.0, 1.0, 1, 0.12, 8.0, 1e-3, "err"),
]


@pytest.mark.parametrize("g_top,g_bot,M,alpha,L,eps,branch", LZ_CASES)
def test_extended_height_meets_its_tolerance(orc, g_top, g_bot, M, alpha, L, eps, branch):
    """Eq. (3.23) pinned by the error it is meant to bound (Theorem 3.3): the
    deterministic k-sum + self + IBC terms at L_z = lz_ext(eps) reproduce the
    long-range (erf) part of Ewald2D with images to within ~eps relative, and
    the error grows when L_z is cut below it.  The two branches of the max are
    exercised separately: the lateral term (ELC error, Eq. (3.21)) for
    alpha L >> 1 and the Gaussian term (remainder, Eq. (3.22)) for small
    alpha.  A dropped (M+1)H, a min for the max or a decimal logarithm each
    fail at least one case."""
    H = 3.0
    pos, q = small_system(3, N=6, L=L, H=H)
    base = dict(Lx=L, Ly=L, H=H, g_top=g_top, g_bot=g_bot, alpha=alpha, rc=L / 2 - 0.01, M=M, P=10)
    u = orc.ewald2d_images(orc.Slab(**base), pos, q, parts=("fourier",))

    def err(Lz):
        s = orc.Slab(**base, Lz=Lz)
        r = orc.evaluate(s, pos, q, *orc.full_kset(s, 40.0), parts=("kspace", "ibc"))
        return abs(r.E_k + r.E_self + r.E_ibc - u) / abs(u)

    lg = math.log(1.0 / eps)
    lateral, gauss = L / (2 * math.pi) * lg, math.sqrt(lg) / alpha
    assert (lateral > gauss) == (branch == "elc")
    lz = orc.lz_ext(L, L, H, M, alpha, eps)
    assert err(lz) <= 2.0 * eps
    if branch == "elc":
        lg10 = math.log10(1.0 / eps)
        wrong = [max(lateral, gauss) + H,                                  # (M+1)H dropped
                 (M + 1) * H + min(lateral, gauss),                        # min for max
                 (M + 1) * H + max(L / (2 * math.pi) * lg10, math.sqrt(lg10) / alpha)]   # log10
        for w in wrong:
            assert err(w) >= 20.0 * eps, w
    else:
        # the lateral term alone is not enough where the Gaussian one is larger
        assert err((M + 1) * H + lateral) >= 1.5 * eps


def _fold_by_reflections(z, v, zlo, zhi):
    """Specular walls by definition: mirror the point in the wall it has
    crossed, flip v, repeat until it lies between the walls."""
    while z < zlo or z > zhi:
        z = 2.0 * zlo - z if z < zlo else 2.0 * zhi - z
        v = -v
    return z, v


def test_fold_z_is_specular_reflection(orc):
    """The integrator's wall fold against (a) repeated mirror reflections and
    (b) the closed form of free flight between two reflecting walls: the
    unfolded coordinate u = z - zlo maps to the triangle wave
    zlo + (W/pi) arccos(cos(pi u / W)), W = zhi - zlo, with v_z multiplied by
    sign(sin(pi u / W)).  Covers no crossing, one crossing of either wall,
    and several folds in one step in both directions."""
    rng = np.random.default_rng(12)
    zlo, zhi = 0.3, 5.7
    W = zhi - zlo
    n_multi = 0
    for k in range(4000):
        z0 = rng.uniform(zlo, zhi)
        v = rng.normal(0.0, 1.0) * (10.0 ** rng.uniform(-2, 1.2)) * W   # up to ~16 W per unit time
        z1 = z0 + v
        zf, vf = orc.fold_z(z1, v, zlo, zhi)
        zb, vb = _fold_by_reflections(z1, v, zlo, zhi)
        assert abs(zf - zb) <= 1e-12 * max(1.0, abs(z1)) and vf == vb, (z0, v)
        u = z1 - zlo
        zc = zlo + W / math.pi * math.acos(math.cos(math.pi * u / W))
        sgn = math.copysign(1.0, math.sin(math.pi * u / W))
        assert abs(zf - zc) <= 1e-9 * max(1.0, abs(u)) and vf == sgn * v
        assert zlo <= zf <= zhi
        n_multi += abs(u) > 2 * W
    assert n_multi > 200
    # exact cases: one crossing of each wall, two folds (below, then above)
    assert orc.fold_z(zlo - 0.25, -3.0, zlo, zhi) == pytest.approx((zlo + 0.25, 3.0))
    assert orc.fold_z(zhi + 0.5, 2.0, zlo, zhi) == pytest.approx((zhi - 0.5, -2.0))
    z, v = orc.fold_z(zlo - (W + 0.5), -7.0, zlo, zhi)
    assert (z, v) == pytest.approx((zhi - 0.5, -7.0))


# --------------------------------------------------------------------------
# Surface charges on the interfaces (remark after Eq. (3.26); readings R7,
# R8 of the oracle)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("g_top,g_bot", [(0.7, -0.4), (-0.9, 0.95), (0.5, 0.5), (0.0, 0.8), (-0.6, 0.0)])
def test_sheet_field_is_the_layered_solution(orc, g_top, g_bot):
    """The field of a uniform sheet on either interface inside the slab is the
    zero lateral mode of the layered-medium Poisson problem (its h -> 0
    limit, Richardson-extrapolated from h = 1e-5 and 1e-6, with the
    interface conditions imposed directly): it does not depend on z, and for
    one interface it is 2 pi sigma (1 + gamma)."""
    H = 1.3
    s = orc.Slab(Lx=10, Ly=10, H=H, g_top=g_top, g_bot=g_bot, alpha=1.0, rc=4.9, M=400, P=10)
    z = np.array([0.2, 0.7, 1.1])
    pos = np.c_[np.ones(3), np.ones(3), z]
    q = np.ones(3)
    _, F0, _, _ = orc.surface(s, pos, q, 0.0, 0.0)           # the net-charge term alone
    for top in (False, True):
        zp = H - 1e-9 if top else 1e-9
        _, F1, _, _ = orc.surface(s, pos, q, 1.0 if top else 0.0, 0.0 if top else 1.0)
        field = (F1 - F0)[:, 2]
        for zz, f in zip(z, field):
            def lay(h):
                dR = _layered_reflection(h, zz, zp, H, g_top, g_bot, deriv=True)
                return 2 * np.pi * np.sign(zz - zp) * np.exp(-h * abs(zz - zp)) - dR
            ref = (10.0 * lay(1e-6) - lay(1e-5)) / 9.0
            assert f == pytest.approx(ref, rel=1e-6, abs=1e-7)
    if g_top == 0.0:
        _, F1, _, _ = orc.surface(s, pos, q, 0.0, 1.0)
        assert (F1 - F0)[0, 2] == pytest.approx(2 * np.pi * (1 + g_bot), rel=1e-12)


def _lattice(L, n, z, sigma):
    g = (np.arange(n) + 0.5) * L / n
    X, Y = np.meshgrid(g, g, indexing="ij")
    return np.c_[X.ravel(), Y.ravel(), np.full(n * n, z)], np.full(n * n, sigma * L * L / (n * n))


@pytest.mark.parametrize("g_top,g_bot,M", [(0.0, 0.0, 0), (0.6, -0.3, 3), (-0.8, 0.7, 4)])
def test_surface_charges_match_point_charge_lattice(orc, g_top, g_bot, M):
    """Non-neutral ions between charged interfaces (the whole system neutral):
    the ions' forces with the surface terms (sheet field R7 and net-charge
    term R8) equal those of the same ions plus a 24 x 24 lattice of point
    charges standing in for each sheet (1e-3 inside the slab), evaluated
    with the neutral reformulation of Theorem 3.3 and the full k-sum.  The
    sheet field alone, or no surface term, is off by 1e-2 to 1e-1.  Energy
    differences between two ion configurations agree as well."""
    L, H = 10.0, 4.0
    rng = np.random.default_rng(5)
    qi = np.array([1.0, -1.0, 2.0, 1.0, -1.0, 1.0])           # Q = 3
    sb, st = -0.01, -0.02                                        # -Q / L^2 on the two sheets
    s = orc.Slab(Lx=L, Ly=L, H=H, g_top=g_top, g_bot=g_bot, alpha=1.0, rc=4.9, M=M, P=10)
    kn, kc = orc.full_kset(s, 40.0)
    pb, qb = _lattice(L, 24, 1e-3, sb)
    pt, qt = _lattice(L, 24, H - 1e-3, st)
    energies = []
    for conf in range(2):
        ions = np.c_[rng.uniform(0, L, 6), rng.uniform(0, L, 6), rng.uniform(1.2, H - 1.2, 6)]
        ref = orc.evaluate(s, np.r_[ions, pb, pt], np.r_[qi, qb, qt], kn, kc, targets=np.arange(6))
        sur = orc.evaluate(s, ions, qi, kn, kc, sigma=(st, sb))
        scale = np.abs(ref.F).max()
        assert np.abs(sur.F - ref.F).max() <= 1e-8 * scale
        lit = orc.evaluate(s, ions, qi, kn, kc)
        sheets_only = lit.F + orc.surface(s, ions, qi, st, sb)[1] - orc.surface(s, ions, qi, 0.0, 0.0)[1]
        assert np.abs(lit.F - ref.F).max() > 1e-2 * scale
        assert np.abs(sheets_only - ref.F).max() > 1e-3 * scale
        full = orc.evaluate(s, np.r_[ions, pb, pt], np.r_[qi, qb, qt], kn, kc)
        energies.append((full.E_total, sur.E_total))
    d_ref = energies[1][0] - energies[0][0]
    d_sur = energies[1][1] - energies[0][1]
    assert d_sur == pytest.approx(d_ref, rel=1e-7, abs=1e-9)


def test_surface_terms_are_derivatives(orc):
    """F = -dE/dz, phi = dE/dq and dE/dgamma of the surface terms against
    central finite differences."""
    H = 3.0
    s = orc.Slab(Lx=8, Ly=8, H=H, g_top=0.55, g_bot=-0.7, alpha=1.0, rc=3.9, M=5, P=10)
    rng = np.random.default_rng(8)
    pos = np.c_[rng.uniform(0, 8, 5), rng.uniform(0, 8, 5), rng.uniform(0.3, H - 0.3, 5)]
    q = np.array([1.0, -2.0, 1.5, 1.0, 0.5])
    sig = (0.02, -0.035)
    E, F, phi, dg = orc.surface(s, pos, q, *sig)
    h = 1e-6
    for i in range(5):
        p1, p2 = pos.copy(), pos.copy()
        p1[i, 2] += h
        p2[i, 2] -= h
        fd = -(orc.surface(s, p1, q, *sig)[0] - orc.surface(s, p2, q, *sig)[0]) / (2 * h)
        assert F[i, 2] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        q1, q2 = q.copy(), q.copy()
        q1[i] += h
        q2[i] -= h
        fdq = (orc.surface(s, pos, q1, *sig)[0] - orc.surface(s, pos, q2, *sig)[0]) / (2 * h)
        assert phi[i] == pytest.approx(fdq, rel=1e-6, abs=1e-9)
    for c, key in ((0, "g_top"), (1, "g_bot")):
        b1 = s.box(**{key: getattr(s, key) + h})
        b2 = s.box(**{key: getattr(s, key) - h})
        fdg = (orc.surface(s, pos, q, *sig, box=b1)[0] - orc.surface(s, pos, q, *sig, box=b2)[0]) / (2 * h)
        assert dg[c] == pytest.approx(fdg, rel=1e-6, abs=1e-9)


# --------------------------------------------------------------------------
# Recalibration identity (Sec. 3.4): Y_odd / Y_even folding == explicit images
# --------------------------------------------------------------------------

@pytest.mark.parametrize("g_top,g_bot,M", [(0.7, -0.4, 3), (0.95, -0.95, 10), (0.9, 0.9, 8), (0.3, 0.0, 1)])
def test_recalibration_equals_explicit_images(orc, g_top, g_bot, M):
    pos, q = small_system(4, N=30, L=12.0, H=3.0)
    s = orc.Slab(Lx=12, Ly=12, H=3, g_top=g_top, g_bot=g_bot, alpha=0.8, rc=5.0, M=M, P=40)
    n = orc.draw_kset(s, seed=7)
    c = orc.rbe_weights(s, n)
    Ea, Fa, pa, _, _, rMa = orc.kspace(s, pos, q, n, c, explicit_images=True)
    Eb, Fb, pb, _, _, rMb = orc.kspace(s, pos, q, n, c, explicit_images=False)
    assert np.allclose(rMa, rMb, rtol=1e-12, atol=1e-12 * np.abs(rMa).max())
    assert Ea == pytest.approx(Eb, rel=1e-12)
    assert np.allclose(Fa, Fb, rtol=1e-11, atol=1e-12 * np.abs(Fa).max())
    assert np.allclose(pa, pb, rtol=1e-11, atol=1e-12 * np.abs(pa).max())


# --------------------------------------------------------------------------
# Forces and gradients are the gradients of the energy (R2, R4, R5)
# --------------------------------------------------------------------------

def fd_system(seed=5):
    """Eight charges; the tests use alpha = 1.5, rc = 4.9 so that
    erfc(alpha rc) ~ 1e-24 and the hard cutoff cannot show up in a
    difference quotient."""
    return small_system(seed, N=8, L=10.0, H=4.0)


@pytest.mark.parametrize("g_top,g_bot,M", [(0.0, 0.0, 0), (0.7, -0.4, 3), (0.9, 0.9, 4)])
def test_total_force_is_minus_gradient(orc, g_top, g_bot, M):
    pos, q = fd_system()
    s = orc.Slab(Lx=10, Ly=10, H=4, g_top=g_top, g_bot=g_bot, alpha=1.5, rc=4.9, M=M, P=30)
    n = orc.draw_kset(s, seed=11)
    r = orc.evaluate(s, pos, q, n)
    h = 1e-5
    for part, getF in (("real", lambda x: x.F_real), ("kspace", lambda x: x.F_k), ("ibc", lambda x: x.F_ibc)):
        ref = getF(orc.evaluate(s, pos, q, n, parts=(part,)))
        for i in range(len(q)):
            for d in range(3):
                pp, pm = pos.copy(), pos.copy()
                pp[i, d] += h
                pm[i, d] -= h
                ep = orc.evaluate(s, pp, q, n, parts=(part,)).E_total
                em = orc.evaluate(s, pm, q, n, parts=(part,)).E_total
                fd = -(ep - em) / (2 * h)
                scale = np.abs(ref).max() + 1e-30
                assert abs(fd - ref[i, d]) < 2e-7 * scale + 1e-9, (part, i, d, fd, ref[i, d])
    assert np.allclose(r.F, r.F_real + r.F_k + r.F_ibc)


@pytest.mark.parametrize("g_top,g_bot,M", [(0.7, -0.4, 3), (0.0, 0.0, 0)])
def test_dE_dq_is_derivative(orc, g_top, g_bot, M):
    pos, q = fd_system()
    s = orc.Slab(Lx=10, Ly=10, H=4, g_top=g_top, g_bot=g_bot, alpha=1.5, rc=4.9, M=M, P=30)
    n = orc.draw_kset(s, seed=12)
    r = orc.evaluate(s, pos, q, n)
    h = 1e-4
    for i in range(len(q)):
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qm[i] -= h
        fd = (orc.evaluate(s, pos, qp, n).E_total - orc.evaluate(s, pos, qm, n).E_total) / (2 * h)
        assert fd == pytest.approx(r.phi[i], rel=1e-8, abs=1e-9)


def test_dE_dgamma_is_derivative(orc):
    pos, q = fd_system()
    n = None
    h = 1e-6
    for gt, gb, M in [(0.7, -0.4, 3), (0.9, 0.9, 6), (0.3, -0.95, 1)]:
        s = orc.Slab(Lx=10, Ly=10, H=4, g_top=gt, g_bot=gb, alpha=1.5, rc=4.9, M=M, P=30)
        n = orc.draw_kset(s, seed=13)
        c = orc.rbe_weights(s, n)
        g = orc.dE_dgamma(s, pos, q, n, c)
        for w in (0, 1):
            sp = orc.Slab(**{**s.__dict__, "g_top": gt + h * (w == 0), "g_bot": gb + h * (w == 1)})
            sm = orc.Slab(**{**s.__dict__, "g_top": gt - h * (w == 0), "g_bot": gb - h * (w == 1)})
            fd = (orc.evaluate(sp, pos, q, n, c).E_total - orc.evaluate(sm, pos, q, n, c).E_total) / (2 * h)
            assert fd == pytest.approx(g[w], rel=1e-6, abs=1e-8), (gt, gb, M, w)


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------

def test_kspace_xy_momentum_conserved_per_k(orc):
    """Each k alone gives sum_i F_xy = 0 for any gamma (lateral translation
    invariance); at gamma = 0 also sum_i F_z = 0."""
    pos, q = small_system(6, N=20)
    for gt, gb, M in [(0.8, -0.7, 5), (0.0, 0.0, 0)]:
        s = orc.Slab(Lx=10, Ly=10, H=4, g_top=gt, g_bot=gb, alpha=1.0, rc=4.9, M=M, P=25)
        n = orc.draw_kset(s, seed=3)
        c = orc.rbe_weights(s, n)
        for l in range(5):
            _, F, *_ = orc.kspace(s, pos, q, n[l:l + 1], c[l:l + 1])
            tot = F.sum(axis=0)
            sc = np.abs(F).sum()
            assert abs(tot[0]) < 1e-12 * sc and abs(tot[1]) < 1e-12 * sc
            if gt == 0 and gb == 0:
                assert abs(tot[2]) < 1e-12 * sc


def test_real_space_xy_momentum_conserved(orc):
    pos, q = small_system(7, N=30)
    s = orc.Slab(Lx=10, Ly=10, H=4, g_top=0.6, g_bot=-0.8, alpha=1.0, rc=4.0, M=4, P=10)
    _, F, _, _ = orc.real_space(s, pos, q)
    tot = F.sum(axis=0)
    assert abs(tot[0]) < 1e-12 * np.abs(F).sum() and abs(tot[1]) < 1e-12 * np.abs(F).sum()


def test_gamma0_reduces_to_homogeneous_rbe_force(orc):
    """At gamma = 0 the k-space force is Eq. (2.20) without its Gaussian
    factor (reading R3): -sum (S/P) 4 pi q_i k / (V k^2) Im(e^{-ik.r_i} rho(k))."""
    pos, q = small_system(8, N=16)
    s = orc.Slab(Lx=10, Ly=10, H=4, g_top=0.0, g_bot=0.0, alpha=1.0, rc=4.9, M=3, P=40)
    n = orc.draw_kset(s, seed=5)
    _, F, *_ = orc.kspace(s, pos, q, n, orc.rbe_weights(s, n))
    S = orc.norm_S(s.alpha, s.Lx, s.Ly, s.Lz)
    k = orc.kvectors(s, n)
    rho = (q[None, :] * np.exp(1j * (k @ pos.T))).sum(axis=1)
    ref = np.zeros_like(F)
    for l in range(len(n)):
        ph = np.exp(-1j * (pos @ k[l]))
        ref -= (S / s.P) * 4 * np.pi * q[:, None] * k[l][None, :] / (s.V * (k[l] @ k[l])) * np.imag(ph * rho[l])[:, None]
    assert np.allclose(F, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def test_mirror_symmetry(orc):
    """z -> H - z with gamma_top <-> gamma_bot and n_z -> -n_z: E unchanged,
    F_z -> -F_z, F_xy unchanged."""
    pos, q = small_system(9, N=12)
    s1 = orc.Slab(Lx=10, Ly=10, H=4, g_top=0.7, g_bot=-0.5, alpha=1.2, rc=4.5, M=5, P=30)
    s2 = orc.Slab(Lx=10, Ly=10, H=4, g_top=-0.5, g_bot=0.7, alpha=1.2, rc=4.5, M=5, P=30)
    n = orc.draw_kset(s1, seed=9)
    n2 = n * np.array([1, 1, -1], dtype=np.int32)
    pos2 = pos.copy()
    pos2[:, 2] = 4.0 - pos[:, 2]
    r1 = orc.evaluate(s1, pos, q, n)
    r2 = orc.evaluate(s2, pos2, q, n2)
    assert r1.E_total == pytest.approx(r2.E_total, rel=1e-11)
    assert np.allclose(r1.F * [1, 1, -1], r2.F, rtol=1e-9, atol=1e-11 * np.abs(r1.F).max())


def test_lateral_translation_and_charge_scaling(orc):
    pos, q = small_system(10, N=12)
    s = orc.Slab(Lx=10, Ly=10, H=4, g_top=0.4, g_bot=0.9, alpha=1.2, rc=4.5, M=4, P=30)
    n = orc.draw_kset(s, seed=10)
    r = orc.evaluate(s, pos, q, n)
    sh = pos + np.array([3.3, -7.1, 0.0])
    r2 = orc.evaluate(s, sh, q, n)
    assert r.E_total == pytest.approx(r2.E_total, rel=1e-10)
    assert np.allclose(r.F, r2.F, rtol=1e-8, atol=1e-10 * np.abs(r.F).max())
    r3 = orc.evaluate(s, pos, 2.5 * q, n)
    assert r3.E_total == pytest.approx(6.25 * r.E_total, rel=1e-12)
    assert np.allclose(r3.F, 6.25 * r.F, rtol=1e-11)


# --------------------------------------------------------------------------
# Statistics of the random batch estimator (Theorem 2.2 and Sec. 3.4)
# --------------------------------------------------------------------------

def test_rbe_estimator_is_unbiased_and_variance_scales_as_1_over_P(orc):
    pos, q = small_system(11, N=20, L=8.0, H=3.0)
    s = orc.Slab(Lx=8, Ly=8, H=3, g_top=0.6, g_bot=-0.7, alpha=0.9, rc=3.9, M=4, P=20)
    nfull, cfull = orc.full_kset(s)
    Eref, Fref, *_ = orc.kspace(s, pos, q, nfull, cfull)
    S = orc.norm_S(s.alpha, s.Lx, s.Ly, s.Lz)
    samples = {}
    for P in (10, 40):
        Es, Fs = [], []
        for r in range(300):
            n = orc.draw_kset(s, seed=1000 + r, stream=P, P=P)
            E, F, *_ = orc.kspace(s, pos, q, n, orc.rbe_weights(s, n, S))
            Es.append(E)
            Fs.append(F[0])
        Es, Fs = np.array(Es), np.array(Fs)
        samples[P] = (Es, Fs)
        z = (Es.mean() - Eref) / (Es.std(ddof=1) / math.sqrt(len(Es)))
        assert abs(z) < 4.5, (P, z)
        zf = (Fs.mean(axis=0) - Fref[0]) / (Fs.std(axis=0, ddof=1) / math.sqrt(len(Fs)))
        assert np.all(np.abs(zf) < 4.5), (P, zf)
    ratio = samples[10][1].var(axis=0).sum() / samples[40][1].var(axis=0).sum()
    assert 2.5 < ratio < 6.5, ratio


# --------------------------------------------------------------------------
# The k-sampler's distribution (Sec. 2.3)
# --------------------------------------------------------------------------

def test_sampler_marginals_chi2(orc):
    from scipy.stats import chi2
    s = orc.Slab(Lx=6, Ly=9, H=2, g_top=0, g_bot=0, alpha=0.8, rc=2.9, M=0, P=6000, Lz=12.0)
    n = orc.draw_kset(s, seed=2024)
    assert not np.any(np.all(n == 0, axis=1))
    Ls = (s.Lx, s.Ly, s.Lz)
    w = [lambda v, L=L: math.exp(-(math.pi * v / (s.alpha * L)) ** 2) for L in Ls]
    Z = [sum(f(v) for v in range(-200, 201)) for f in w]
    p0 = [f(0) / z for f, z in zip(w, Z)]
    for d in range(3):
        others0 = np.prod([p0[e] for e in range(3) if e != d])
        vals, counts = np.unique(n[:, d], return_counts=True)
        cmap = dict(zip(vals.tolist(), counts.tolist()))
        top = int(max(abs(vals.min()), abs(vals.max())))
        exp_, obs = [], []
        for v in range(-top, top + 1):
            p = w[d](v) / Z[d] * (1 - (others0 if v == 0 else 0.0)) / (1 - np.prod(p0))
            exp_.append(p * len(n))
            obs.append(cmap.get(v, 0))
        exp_, obs = np.array(exp_), np.array(obs)
        # pool bins with expected count < 5 into the tails
        big = exp_ >= 5
        e2 = np.append(exp_[big], exp_[~big].sum())
        o2 = np.append(obs[big], obs[~big].sum())
        if e2[-1] < 5:
            e2, o2 = e2[:-1], o2[:-1]
        stat = ((o2 - e2) ** 2 / e2).sum()
        assert stat < chi2.ppf(0.9999, len(e2) - 1), (d, stat)


def test_sampler_is_deterministic_per_seed_and_stream(orc):
    s = orc.Slab(Lx=20, Ly=20, H=5, g_top=0, g_bot=0, alpha=1.0, rc=4, M=0, P=50)
    a = orc.draw_kset(s, seed=0)
    b = orc.draw_kset(s, seed=0)
    c = orc.draw_kset(s, seed=0, stream=1)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


# ---------------------------------------------------------------------------
# MD around the path: short-range forces, thermostat noise, BAOAB step
# ---------------------------------------------------------------------------

def _wca_pair(orc, r, sigma=1.0, eps=1.0):
    pos = np.array([[1.0, 1.0, 2.0], [1.0 + r, 1.0, 2.0]])
    return orc.short_range(pos, 10.0, 10.0, 4.0, sigma, eps, 0.5, 0.0)


def test_wca_special_values_and_cutoff(orc):
    """At r = sigma the shifted-truncated LJ equals eps; at its minimum
    r = 2^(1/6) sigma both energy and force vanish (continuous truncation);
    beyond it nothing acts; the pair forces are equal and opposite."""
    F, e, _ = _wca_pair(orc, 1.0)
    assert abs(e - 1.0) < 1e-14
    rc = 2.0 ** (1.0 / 6.0)
    F, e, _ = _wca_pair(orc, rc * (1 - 1e-9))
    assert abs(e) < 1e-12 and np.abs(F).max() < 1e-6
    F, e, _ = _wca_pair(orc, rc * (1 + 1e-9))
    assert e == 0.0 and np.abs(F).max() == 0.0
    F, e, _ = _wca_pair(orc, 0.95)
    assert np.allclose(F[0], -F[1], rtol=0, atol=1e-12) and F[0, 0] < 0 < F[1, 0]


def test_wca_and_wall_forces_are_minus_gradients(orc):
    # jittered lattice of spacing 1.05 (pairs straddle the 1.12 cutoff), a few
    # closer pairs, and particles near both walls; periodic in x and y
    rng = np.random.default_rng(3)
    L, H = 6.3, 5.0
    g = np.arange(6) * 1.05
    pos = np.array([[x, y, z] for x in g for y in g for z in (0.9, 1.95, 3.0, 4.05)])
    pos += rng.uniform(-0.08, 0.08, pos.shape)
    pos[1] = pos[0] + [0.8, 0.3, 0.2]
    pos[3, 2] = 0.4
    pos[4, 2] = H - 0.35
    sig, eps, sw, ew = 1.0, 1.3, 0.5, 0.7
    F, _, _ = orc.short_range(pos, L, L, H, sig, eps, sw, ew)
    h = 1e-6
    for i in (0, 1, 3, 4, 7):
        for c in range(3):
            pp = pos.copy(); pp[i, c] += h
            pm = pos.copy(); pm[i, c] -= h
            _, e1, w1 = orc.short_range(pp, L, L, H, sig, eps, sw, ew)
            _, e2, w2 = orc.short_range(pm, L, L, H, sig, eps, sw, ew)
            fd = -((e1 + w1) - (e2 + w2)) / (2 * h)
            assert abs(fd - F[i, c]) <= 1e-5 * (1 + abs(F[i, c])), (i, c, fd, F[i, c])
    assert np.abs(F[:, :2].sum(0)).max() < 1e-9     # walls act in z only


def test_wall_force_mirror_symmetry(orc):
    H = 5.0
    for z in (0.2, 0.4, 0.55):
        F1, _, w1 = orc.short_range(np.array([[1.0, 1.0, z]]), 4.0, 4.0, H, 1.0, 0.0, 0.5, 1.0)
        F2, _, w2 = orc.short_range(np.array([[1.0, 1.0, H - z]]), 4.0, 4.0, H, 1.0, 0.0, 0.5, 1.0)
        assert abs(w1 - w2) <= 1e-12 * abs(w1) and abs(F1[0, 2] + F2[0, 2]) <= 1e-12 * abs(F1[0, 2])
        assert (F1[0, 2] > 0) == (z < 0.5 * 2 ** (1 / 6))


def test_thermo_normals_are_standard_normal(orc):
    from scipy import stats
    x = orc.thermo_normals(5, 17, 3000).ravel()
    assert abs(x.mean()) < 4 / np.sqrt(x.size)
    assert abs(x.var() - 1) < 4 * np.sqrt(2 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-3
    y = orc.thermo_normals(5, 18, 10).ravel()
    z = orc.thermo_normals(6, 17, 10).ravel()
    assert not np.allclose(x[:30], y) and not np.allclose(x[:30], z)
    assert np.array_equal(orc.thermo_normals(5, 17, 10).ravel(), x[:30])


def _harmonic(center, k=1.0):
    return lambda p: -k * (p - center)


def test_baoab_without_friction_is_time_reversible(orc):
    """gamma = 0: one step forward, then one step with the velocities
    reversed, returns to the start (velocity Verlet is time-reversible)."""
    rng = np.random.default_rng(1)
    c = np.array([5.0, 5.0, 5.0])
    force = _harmonic(c, 2.0)
    pos = c + rng.normal(0, 0.5, (20, 3))
    vel = rng.normal(0, 1, (20, 3))
    F = force(pos)
    z = np.zeros((20, 3))
    p1, v1, F1 = orc.baoab_step(pos, vel, F, 0.01, 0.0, 1.0, z, 100.0, 100.0, 0.0, 10.0, force)
    p2, v2, _ = orc.baoab_step(p1, -v1, F1, 0.01, 0.0, 1.0, z, 100.0, 100.0, 0.0, 10.0, force)
    assert np.allclose(p2, pos, atol=1e-12) and np.allclose(-v2, vel, atol=1e-12)
    # and energy stays within O(dt^2) over many steps
    e0 = 0.5 * (vel ** 2).sum() + (pos - c).var(axis=None) * 0 + ((pos - c) ** 2).sum()
    p, v, Fc = pos, vel, F
    for _ in range(500):
        p, v, Fc = orc.baoab_step(p, v, Fc, 0.01, 0.0, 1.0, z, 100.0, 100.0, 0.0, 10.0, force)
    e1 = 0.5 * (v ** 2).sum() + ((p - c) ** 2).sum()
    assert abs(e1 - e0) < 1e-3 * e0


def test_baoab_thermostat_reaches_equipartition(orc):
    """No forces: the O step alone drives every velocity component to the
    Maxwell distribution of temperature kT (fluctuation-dissipation)."""
    n, kT = 400, 2.0
    pos = np.tile([5.0, 5.0, 5.0], (n, 1))
    vel = np.zeros((n, 3))
    F = np.zeros((n, 3))
    zero = lambda p: np.zeros_like(p)  # noqa: E731
    v2 = []
    for step in range(60):
        xi = orc.thermo_normals(9, step, n)
        pos, vel, F = orc.baoab_step(pos, vel, F, 0.05, 2.0, kT, xi, 10.0, 10.0, 0.0, 10.0, zero)
        if step >= 30:
            v2.append((vel ** 2).mean())
    assert abs(np.mean(v2) - kT) < 0.06 * kT


# ---------------------------------------------------------------------------
# Parameter selection and the stochastic force error
# ---------------------------------------------------------------------------

def test_image_order_reproduces_the_papers_example(orc):
    """After Theorem 3.2: for H about max(Lx, Ly) and |gamma| = 1, an accuracy
    of 1e-5 needs M = 3 image levels (fixture tests/golden/image_order_example.txt)."""
    rows = []
    with open(os.path.join(GOLDEN, "image_order_example.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert rows
    for tol, gt, gb, H, L, M in rows:
        assert orc.image_order_for(float(tol), float(gt), float(gb), float(H), float(L)) == int(M)
    # no interface: no image is needed; one interface: its single image
    assert orc.image_order_for(1e-5, 0.0, 0.0, 10.0, 100.0) == 0
    assert orc.image_order_for(1e-5, 0.0, 0.9, 10.0, 100.0) == 1


@pytest.mark.parametrize("g,H,L,tol", [(0.9, 10.0, 50.0, 1e-5), (0.95, 40.0, 800.0, 1e-5), (0.5, 5.0, 20.0, 1e-8),
                                       (1.0, 3.0, 9.0, 1e-4)])
def test_image_order_matches_closed_form(orc, g, H, L, tol):
    """For |gamma_top| = |gamma_bot| the smallest admissible M is Eq. (3.10)
    rounded up."""
    a = 4 * np.pi * H / L
    lg = np.log(g * g)
    closed = (2 * np.log(tol) - a - lg) / (lg - a)
    assert orc.image_order_for(tol, g, -g, H, L) == max(0, int(np.ceil(closed - 1e-12)))


def test_suggested_parameters(orc):
    s = orc.suggest_params(10_000, 50.0, 50.0, 10.0, 0.9, 0.9, 1e-5)
    assert abs(s["alpha"] - (10_000 / 25_000.0) ** (1 / 3)) < 1e-15
    assert abs(np.exp(-(s["alpha"] * s["r_c"]) ** 2) - 1e-5) < 1e-12
    assert s["Lz"] >= (s["M"] + 1) * 10.0
    assert orc.image_truncation_estimate(s["M"], 0.9, 0.9, 10.0, 50.0) <= 1e-5 < \
        orc.image_truncation_estimate(s["M"] - 1, 0.9, 0.9, 10.0, 50.0)
    # a dilute small box: r_c is capped at half the box and alpha follows it
    s = orc.suggest_params(10, 10.0, 10.0, 5.0, 0.0, 0.0, 1e-5)
    assert s["r_c"] == 5.0 and abs(s["alpha"] * 5.0 - np.sqrt(np.log(1e5))) < 1e-12 and s["M"] == 0


@pytest.mark.parametrize("gammas,M", [((0.0, 0.0), 0), ((0.8, -0.6), 4)])
def test_force_variance_estimate_is_unbiased(orc, gammas, M):
    """Theorem 2.2: over many independent batches, the mean of the one-batch
    estimates and the observed variance of the force both equal the variance
    written out over every k."""
    sl = orc.Slab(Lx=8, Ly=8, H=4, g_top=gammas[0], g_bot=gammas[1], alpha=0.8, rc=3.5, M=M, P=10)
    rng = np.random.default_rng(0)
    N = 24
    pos = np.column_stack([rng.uniform(0, 8, N), rng.uniform(0, 8, N), rng.uniform(0.3, 3.7, N)])
    q = np.where(np.arange(N) < N // 2, 1.0, -1.0)
    exact = orc.force_variance_exact(sl, pos, q, 10)
    est, Fs = [], []
    for s in range(400):
        n = orc.draw_kset(sl, 3, s)
        c = orc.rbe_weights(sl, n)
        t = orc.kspace_terms(sl, pos, q, n, c)
        Fs.append(t.sum(axis=0))
        est.append(orc.force_variance_estimate(sl, pos, q, n, c))
    Fs = np.array(Fs)
    emp = ((Fs - Fs.mean(axis=0)) ** 2).sum(axis=2).mean(axis=0)
    assert abs(np.mean(est, axis=0).sum() / exact.sum() - 1) < 0.05
    assert abs(emp.sum() / exact.sum() - 1) < 0.08
    # and the per-k terms add up to the oracle's k-space force
    _, F, *_ = orc.kspace(sl, pos, q, n, c)
    assert np.abs(Fs[-1] - F).max() < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("gammas,M", [((0.0, 0.0), 0), ((0.8, -0.6), 4)])
def test_force_variance_is_flat_in_Lz(orc, gammas, M):
    """Theorem 2.2: with alpha fixed, the force variance does not grow with
    the extended height once L_z is past the image layers (S and V both scale
    with L_z, and the k_z sum becomes an integral; the k_z = 0 plane leaves an
    O(1/L_z) remainder: 0.55 % between L_z = 12 H and 48 H here).  A wrong power of V or S
    would change it by factors of 2 and 4."""
    rng = np.random.default_rng(0)
    N = 24
    pos = np.column_stack([rng.uniform(0, 8, N), rng.uniform(0, 8, N), rng.uniform(0.3, 3.7, N)])
    q = np.where(np.arange(N) < N // 2, 1.0, -1.0)
    v = {}
    for Lz in (48.0, 96.0, 192.0):
        sl = orc.Slab(Lx=8, Ly=8, H=4, g_top=gammas[0], g_bot=gammas[1], alpha=0.8, rc=3.5, M=M, P=10, Lz=Lz)
        v[Lz] = orc.force_variance_exact(sl, pos, q, 10)
    for Lz in (48.0, 96.0):
        assert np.abs(v[Lz] / v[192.0] - 1).max() < 1e-2, (Lz, np.abs(v[Lz] / v[192.0] - 1).max())
