// C ABI of librbe2d (declared in include/rbe2d.h): parameter validation,
// derived constants, workspace management, the host k-sampler, layouts of
// one or many systems, and the launch sequences of one RBE2D evaluation
// (Algorithm 2 of the paper) and of velocity-Verlet steps around it.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "rbe2d_internal.h"

// cells per r_c along y of the pair kernel's cell grid
#ifndef RBE2D_REACH_Y
#define RBE2D_REACH_Y 6
#endif

using namespace rbe2d;

namespace {

thread_local std::string g_create_error;

rbe2d_status fail(rbe2d_ctx *h, rbe2d_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
rbe2d_status fail(rbe2d_ctx *h, rbe2d_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf; else g_create_error = buf;
    return st;
}

rbe2d_status hipfail(rbe2d_ctx *h, hipError_t e, const char *what) {
    return fail(h, RBE2D_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define RBE2D_TRY(h, call, what)                           \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hipfail(h, e_, what); \
    } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

double ipow(double b, int e) {
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= b;
    return r;
}

// exponents (a of gamma_top, b of gamma_bot) of the order-l image above (+1) or below (-1)
void exponents(int l, int side, int *a, int *b) {
    const int up = (l + 1) / 2, dn = l / 2;
    if (side > 0) { *a = up; *b = dn; } else { *a = dn; *b = up; }
}

double dmono(int e_self, double g_self, int e_other, double g_other) {
    return e_self ? e_self * ipow(g_self, e_self - 1) * ipow(g_other, e_other) : 0.0;
}

// one-axis theta factor of S: sum_n exp(-pi^2 n^2 / (alpha L)^2)
double theta_axis(double alpha, double L) {
    double s = 1.0;
    for (long n = 1;; n++) {
        const double t = std::exp(-(kPi * kPi) * (double)(n * n) / (alpha * alpha * L * L));
        if (t < 1e-300) break;
        s += 2.0 * t;
    }
    return s;
}

// inverse-CDF table of one axis of the k-distribution, |n| <= nmax
void axis_table(double alpha, double L, int *nmax, std::vector<double> &cdf) {
    const double sig10 = 10.0 * alpha * L / (std::sqrt(2.0) * kPi);
    *nmax = (int)std::ceil(sig10) + 1;
    const int n = 2 * *nmax + 1;
    cdf.assign(n, 0.0);
    double acc = 0.0;
    for (int m = 0; m < n; m++) {
        const long v = m - *nmax;
        acc += std::exp(-(kPi * kPi) * (double)(v * v) / (alpha * alpha * L * L));
        cdf[m] = acc;
    }
    for (int m = 0; m < n; m++) cdf[m] /= acc;
}

rbe2d_status validate(const rbe2d_params *p, rbe2d_ctx *h) {
    if (!p) return fail(h, RBE2D_E_INVAL, "params is NULL");
    if (!finite_pos(p->Lx) || !finite_pos(p->Ly) || !finite_pos(p->H))
        return fail(h, RBE2D_E_INVAL, "Lx, Ly, H must be finite and > 0");
    if (!(std::fabs(p->gamma_top) <= 1.0) || !(std::fabs(p->gamma_bot) <= 1.0))
        return fail(h, RBE2D_E_INVAL, "|gamma_top|, |gamma_bot| must be <= 1");
    if (!finite_pos(p->alpha)) return fail(h, RBE2D_E_INVAL, "alpha must be finite and > 0");
    if (!finite_pos(p->r_c) || p->r_c > 0.5 * std::min(p->Lx, p->Ly))
        return fail(h, RBE2D_E_INVAL, "r_c must satisfy 0 < r_c <= min(Lx, Ly)/2");
    if (p->P < 1 || p->P > 65536) return fail(h, RBE2D_E_INVAL, "P must be in [1, 65536]");
    if (p->M < 0 || p->M > 64) return fail(h, RBE2D_E_INVAL, "M must be in [0, 64]");
    if (p->precision != RBE2D_PREC_FP64 && p->precision != RBE2D_PREC_FP32_PHASE)
        return fail(h, RBE2D_E_INVAL, "unknown precision %d", p->precision);
    if (p->reserved != 0) return fail(h, RBE2D_E_INVAL, "reserved must be 0");
    if (p->n_max < 0 || p->n_max > (int64_t)1 << 30)
        return fail(h, RBE2D_E_INVAL, "n_max must be in [0, 2^30]");
    if (!std::isfinite(p->Lz_ext) || !std::isfinite(p->eps_lz) || !std::isfinite(p->coulomb_prefactor))
        return fail(h, RBE2D_E_INVAL, "non-finite parameter");
    if (p->eps_lz >= 1.0) return fail(h, RBE2D_E_INVAL, "eps_lz must be < 1");
    return RBE2D_OK;
}

double auto_lz(const rbe2d_params *p) {
    const double eps = p->eps_lz > 0.0 ? p->eps_lz : 1e-6;
    const double lg = std::log(1.0 / eps);
    return (p->M + 1) * p->H + std::max(std::max(p->Lx, p->Ly) / (2.0 * kPi) * lg, std::sqrt(lg) / p->alpha);
}

void surface_setup(SysHost &sh);

// Derived constants, image tables, real-space families, sampler tables and
// cell grid of one system.
rbe2d_status setup_system(const rbe2d_params *pin, SysHost &sh) {
    rbe2d_status st = validate(pin, nullptr);
    if (st) return st;
    sh.p = *pin;
    rbe2d_params &p = sh.p;
    SysDesc &d = sh.d;
    std::memset(&d, 0, sizeof d);
    if (p.eps_lz <= 0.0) p.eps_lz = 1e-6;
    if (p.coulomb_prefactor == 0.0) p.coulomb_prefactor = 1.0;
    const double Lz = p.Lz_ext > 0.0 ? p.Lz_ext : auto_lz(&p);
    if (Lz < (p.M + 1) * p.H)
        return fail(nullptr, RBE2D_E_INVAL,
                    "Lz_ext = %g < (M+1) H = %g: the z-replicas of the charges would overlap their images",
                    p.Lz_ext, (p.M + 1) * p.H);
    p.Lz_ext = Lz;
    d.Lx = p.Lx; d.Ly = p.Ly; d.H = p.H; d.Lz = Lz;
    d.V = p.Lx * p.Ly * Lz;
    d.S = theta_axis(p.alpha, p.Lx) * theta_axis(p.alpha, p.Ly) * theta_axis(p.alpha, Lz) - 1.0;
    d.alpha = p.alpha; d.rc = p.r_c; d.rc2 = p.r_c * p.r_c; d.pref = p.coulomb_prefactor;
    d.rc_lay = p.r_c + 1e-9 * p.r_c;   // the margin covers the division that assigned the layers
    d.H_rc = p.H + p.r_c;
    d.g_top = p.gamma_top; d.g_bot = p.gamma_bot; d.M = p.M;
    d.cfac = 2.0 * kPi * d.S * d.pref / (d.V * p.P);

    // image weights, their derivatives, the IBC image-dipole coefficients and
    // the real-space families that can come within r_c of the slab
    std::memset(&sh.img, 0, sizeof sh.img);
    sh.fam.clear();
    d.g1 = 1.0; d.cgam = 0.0; d.dg1t = d.dg1b = d.dcgt = d.dcgb = 0.0;
    for (int l = 1; l <= p.M; l++) {
        int a, b;
        exponents(l, +1, &a, &b);
        sh.img.ea_p[l - 1] = a; sh.img.eb_p[l - 1] = b;
        const double gpl = ipow(p.gamma_top, a) * ipow(p.gamma_bot, b);
        const double dpt = dmono(a, p.gamma_top, b, p.gamma_bot), dpb = dmono(b, p.gamma_bot, a, p.gamma_top);
        exponents(l, -1, &a, &b);
        sh.img.ea_m[l - 1] = a; sh.img.eb_m[l - 1] = b;
        const double gml = ipow(p.gamma_top, a) * ipow(p.gamma_bot, b);
        const double dmt = dmono(a, p.gamma_top, b, p.gamma_bot), dmb = dmono(b, p.gamma_bot, a, p.gamma_top);
        sh.img.gp[l - 1] = gpl; sh.img.gm[l - 1] = gml;
        const double sgn = (l % 2 == 0) ? 1.0 : -1.0;
        const double shp = 2.0 * ((l + 1) / 2) * p.H, shm = -2.0 * (l / 2) * p.H;
        d.g1 += sgn * (gpl + gml);
        d.cgam += shp * gpl + shm * gml;
        d.dg1t += sgn * (dpt + dmt); d.dg1b += sgn * (dpb + dmb);
        d.dcgt += shp * dpt + shm * dmt; d.dcgb += shp * dpb + shm * dmb;
        if ((l - 1) * p.H < p.r_c) {
            for (int side = 1; side >= -1; side -= 2) {
                Family f;
                if (l % 2) {   // reflection: target seen at sz = -1
                    f.sz = -1.0;
                    f.cz = side > 0 ? (l + 1) * p.H : -(l - 1) * p.H;
                    f.zsign = -1.0;
                } else {       // translation
                    f.sz = 1.0;
                    f.cz = side > 0 ? -l * p.H : l * p.H;
                    f.zsign = 1.0;
                }
                f.w = side > 0 ? gpl : gml;
                f.dwt = side > 0 ? dpt : dmt;
                f.dwb = side > 0 ? dpb : dmb;
                sh.fam.push_back(f);
            }
        }
    }
    if ((int)sh.fam.size() > kMaxFamilies)
        return fail(nullptr, RBE2D_E_INVAL, "too many image orders within r_c (H too small for r_c)");
    d.nfam = (int)sh.fam.size();

    // k-sampling tables and the FP32 phase split
    sh.cdf.assign(3, {});
    const double Ls[3] = {p.Lx, p.Ly, Lz};
    int nall = 0;
    for (int ax = 0; ax < 3; ax++) {
        axis_table(p.alpha, Ls[ax], &d.nmax[ax], sh.cdf[ax]);
        nall = std::max(nall, d.nmax[ax]);
    }
    int bits = 0;
    while ((1 << bits) <= nall) bits++;
    // fh keeps 22 - bits fraction bits: n fh then has at most 22 significant
    // bits for |n| < 2^bits, and nx fxh + ny fyh at most 23, so both are exact
    d.fh_bits = std::max(1, 22 - bits);
    d.scale_h = std::ldexp(1.0, d.fh_bits);
    if (p.precision == RBE2D_PREC_FP32_PHASE && bits > 20)
        return fail(nullptr, RBE2D_E_INVAL, "k-range too wide for FP32 phases (alpha L too large)");

    // cell grid: cells >= r_c / reach in x (searched +-reach columns),
    // layers >= r_c / 2 in z and cells >= r_c / reach_y along y, where the
    // pair kernel scans contiguous runs of cells (finer cells trim the runs'
    // ends); coarsened if there would be too many cells.  Where a cutoff
    // sphere holds few particles (n_max / volume * r_c^3 < 20) the runs are
    // short and their set-up dominates: x-cells of r_c (three columns), and
    // at most two layers in a slab thinner than 2 r_c (measured on the
    // 64-replica batch: 4 % faster steps than r_c / 2 in both)
    const double per_rc3 = (double)p.n_max / (p.Lx * p.Ly * p.H) * p.r_c * p.r_c * p.r_c;
    d.reach = per_rc3 < 20.0 ? 1 : 2;
    d.reach_y = RBE2D_REACH_Y;
    int ncx = std::max(1, (int)std::floor(d.reach * p.Lx / p.r_c));
    int ncy = std::max(1, (int)std::floor(d.reach_y * p.Ly / p.r_c));
    int ncz = std::max(1, (int)std::floor(2.0 * p.H / p.r_c));
    if (per_rc3 < 20.0 && p.H < 2.0 * p.r_c) ncz = std::min(ncz, 2);
    const int64_t cell_cap = std::max<int64_t>(2 * p.n_max, 4096);
    while ((int64_t)ncx * ncy * ncz > cell_cap && (ncx > 5 || ncy > 5 || ncz > 1)) {
        if (ncz > 1) ncz = (ncz + 1) / 2;
        else { ncx = std::max(5, ncx / 2); ncy = std::max(5, ncy / 2); }
    }
    d.ncx = ncx; d.ncy = ncy; d.ncz = ncz;
    d.hx = p.Lx / ncx; d.hy = p.Ly / ncy; d.hz = p.H / ncz;
    d.inv_hx = 1.0 / d.hx; d.inv_hy = 1.0 / d.hy; d.inv_hz = 1.0 / d.hz;
    d.inv_Lx = 1.0 / p.Lx; d.inv_Ly = 1.0 / p.Ly; d.inv_Lz = 1.0 / d.Lz;
    // fixed-point frame of the FP32 pair kernel.  z (and every transformed
    // target height within r_c of the slab) lies in [-zoff, zspan - zoff);
    // the span exceeds twice any candidate |dz| <= r_c + hz <= r_c + H.
    const double two32 = 4294967296.0;
    const double zspan = 2.0 * p.H + 4.0 * p.r_c;
    d.zoff = 0.5 * p.H + 2.0 * p.r_c;
    // candidates lie within r_c + hz of the target in z
    d.iso = p.Lx == p.Ly && 2.0 * (p.r_c + d.hz) * (1.0 + 1e-6) < p.Lx;
    d.fxs = two32 / p.Lx; d.fys = two32 / p.Ly; d.fzs = d.iso ? d.fxs : two32 / zspan;
    d.ux = (float)(p.Lx / two32); d.uy = (float)(p.Ly / two32);
    d.uz = d.iso ? d.ux : (float)(zspan / two32);
    d.rc2f = (float)(p.r_c * p.r_c);
    // below `near` the quantisation of the positions (one unit) would exceed
    // ~2^-22 of the distance: such pairs take exact FP64 displacements
    const double unit = d.iso ? p.Lx / two32 : std::max(std::max(p.Lx, p.Ly), zspan) / two32;
    const double near = unit * 4194304.0;
    d.near2f = (float)(near * near);
    d.ud = p.Lx / two32;
    d.u2 = (float)(d.ud * d.ud);
    d.rc2q = (float)(p.r_c * p.r_c * d.fxs * d.fxs);
    d.near2q = (float)(near * near * d.fxs * d.fxs);
    d.sig_top = d.sig_bot = 0.0;
    surface_setup(sh);
    return RBE2D_OK;
}

// Surface charges (reading R7): the uniform sheets sigma_bot on z = 0 and
// sigma_top on z = H, taken just inside the slab, and their images.  Every
// image of the bottom sheet below the slab (and the one at z = 0) pushes
// away from below, every image above pulls; the top sheet likewise.  For
// 0 < z < H this gives phi_s(z) = -Es z + Cs.  Net-charge term (reading R8):
// Gs, A1, A0 are the sums over the real charge and its images of w, w s c
// and w c^2 for image heights s z + c.  Index 0 is the value, 1 and 2 its
// derivatives by gamma_top and gamma_bot.
void surface_setup(SysHost &sh) {
    SysDesc &d = sh.d;
    const rbe2d_params &p = sh.p;
    for (int k = 0; k < 3; k++) { d.Es[k] = d.Cs[k] = d.A1[k] = d.A0[k] = 0.0; d.Gs[k] = k == 0 ? 1.0 : 0.0; }
    d.surf = (d.sig_top != 0.0 || d.sig_bot != 0.0) ? 1 : 0;
    // the real sheets: bottom at 0 (s = +1 for the ions above it), top at H (s = -1)
    d.Es[0] = 2.0 * kPi * (d.sig_bot - d.sig_top);
    d.Cs[0] = -2.0 * kPi * d.sig_top * d.H;          // -2 pi sigma_top |z - H| = 2 pi sigma_top (z - H)
    for (int l = 1; l <= p.M; l++) {
        int a, b;
        double wt[3], wb[3];   // weights (and gamma derivatives) of the + (above) and - (below) image
        exponents(l, +1, &a, &b);
        wt[0] = ipow(p.gamma_top, a) * ipow(p.gamma_bot, b);
        wt[1] = dmono(a, p.gamma_top, b, p.gamma_bot);
        wt[2] = dmono(b, p.gamma_bot, a, p.gamma_top);
        exponents(l, -1, &a, &b);
        wb[0] = ipow(p.gamma_top, a) * ipow(p.gamma_bot, b);
        wb[1] = dmono(a, p.gamma_top, b, p.gamma_bot);
        wb[2] = dmono(b, p.gamma_bot, a, p.gamma_top);
        const double s = (l % 2 == 0) ? 1.0 : -1.0;
        const double cp = 2.0 * ((l + 1) / 2) * p.H, cm = -2.0 * (l / 2) * p.H;
        // image heights of the bottom sheet (z = 0) and of the top sheet (z = H)
        const double bot_up = cp, bot_dn = cm, top_up = s * p.H + cp, top_dn = s * p.H + cm;
        for (int k = 0; k < 3; k++) {
            d.Gs[k] += wt[k] + wb[k];
            d.A1[k] += s * (wt[k] * cp + wb[k] * cm);
            d.A0[k] += wt[k] * cp * cp + wb[k] * cm * cm;
            // images above the slab pull (sign -1), below push (+1); the
            // potential -2 pi sigma w |z - z_w| = -2 pi sigma w sign (z - z_w)
            d.Es[k] += 2.0 * kPi * (d.sig_bot * (wb[k] - wt[k]) + d.sig_top * (wb[k] - wt[k]));
            d.Cs[k] += 2.0 * kPi * (d.sig_bot * (wb[k] * bot_dn - wt[k] * bot_up) +
                                    d.sig_top * (wb[k] * top_dn - wt[k] * top_up));
        }
    }
}

template <typename T>
hipError_t dalloc(rbe2d_ctx *h, T **ptr, size_t count) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return e;
    h->allocs.push_back(p);
    *ptr = (T *)p;
    return hipMemset(p, 0, bytes);
}

void prof_free(rbe2d_ctx *h) {
    Profiler &p = h->prof;
    for (int sl = 0; sl < RBE2D_PROF_SLOTS; sl++)
        for (int b = 0; b < 2; b++) {
            for (hipEvent_t e : p.ev[sl][b]) (void)hipEventDestroy(e);
            p.ev[sl][b].clear();
        }
    p.n = 0;
    for (int sl = 0; sl < RBE2D_PROF_SLOTS; sl++) p.used[sl] = 0;
}

void free_graph(rbe2d_ctx *h) {
    if (h->md_exec) (void)hipGraphExecDestroy(h->md_exec);
    if (h->md_graph) (void)hipGraphDestroy(h->md_graph);
    h->md_exec = nullptr;
    h->md_graph = nullptr;
    h->md_key.clear();
}

void free_all(rbe2d_ctx *h) {
    free_graph(h);
    prof_free(h);
    for (void *p : h->allocs) (void)hipFree(p);
    h->allocs.clear();
    if (h->kstage) (void)hipHostFree(h->kstage);
    if (h->lay_stage) (void)hipHostFree(h->lay_stage);
    if (h->kev) (void)hipEventDestroy(h->kev);
    if (h->lay_ev) (void)hipEventDestroy(h->lay_ev);
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->join_ev) (void)hipEventDestroy(h->join_ev);
    if (h->tail_ev) (void)hipEventDestroy(h->tail_ev);
    if (h->side) (void)hipStreamDestroy(h->side);
}

// Every device workspace of a handle, in one fixed order: A(&ptr, count) is
// called once per buffer (count elements of *ptr's type).  The handle's
// capacities (n_sys, n_cap, cap_particles, cap_sorted, total_cells, P,
// fpart_blocks) must be set.  own_kset: the handle holds its k-set (else the
// caller's device array is used in place).
template <typename Alloc>
void plan_workspace(rbe2d_ctx *h, size_t cdf_total, bool own_kset, Alloc &&A) {
    const int n = h->n_sys;
    const int cells = h->total_cells;
    const int64_t cap_blocks = h->cap_particles / kBlock;
    Workspace &w = h->w;
    A(&w.sys, n);
    A(&w.img, n);
    A(&w.fam, (size_t)n * kMaxFamilies);
    A(&w.cdf, cdf_total);
    A(&w.lay.off, n + 1); A(&w.lay.pbase, n + 1); A(&w.lay.bbase, n + 1);
    A(&w.lay.tbase, n + 1); A(&w.lay.sbase, n + 1);
    A(&w.p32, 2 * h->cap_particles);
    A(&w.p64, h->cap_particles);
    A(&w.bpart, 4 * cap_blocks);
    A(&w.scal, kScal * (size_t)n);
    if (own_kset) A(&w.kset, 3 * (size_t)n * h->P);
    A(&w.kn32, (size_t)n * h->P_pad);
    A(&w.kn64, (size_t)n * h->P_pad);
    double *sfp = nullptr;
    A(&sfp, (size_t)cap_blocks * h->P_pad * 4);
    w.sfpart = sfp;
    A(&w.krec, (size_t)n * h->P * kKRec);
    A(&w.kf32, 3 * (size_t)n * h->P);
    A(&w.fpart, (size_t)h->fpart_blocks * kBlock * 4);
    const int64_t nc = std::max<int64_t>(h->n_cap, 1);
    A(&w.cell, nc); A(&w.slot, nc); A(&w.tmp, nc);
    A(&w.count, cells); A(&w.start, cells + 1); A(&w.scanbuf, cells / 1024 + 2);
    // source records get one wave of padding: the pair kernel reads the first
    // record of an empty run, which may start at the end of the array
    A(&w.sorted, h->cap_sorted + kWave); A(&w.sidx, h->cap_sorted); A(&w.scell, h->cap_sorted);
    if (h->precision == RBE2D_PREC_FP32_PHASE) A(&w.src16, h->cap_sorted + kWave);
    A(&w.freal, nc); A(&w.dgreal, nc);
    A(&w.rpart, 3 * (h->cap_sorted / kWave));
    // the split is only used when there are too few targets to fill the chip
    h->split_cap = std::min<int64_t>(nc, 1 << 18);
    A(&w.freal_s, kMaxRealSplit * h->split_cap);
    A(&w.dgreal_s, kMaxRealSplit * h->split_cap);
    A(&w.rpart_s, kMaxRealSplit * 3 * (h->cap_sorted / kWave));
    A(&w.spart, 2 * (h->cap_sorted / kWave));
    A(&w.err, 4);
    A(&w.step, 1);
}

// A handle over n systems: every system is set up and the workspaces are
// sized for the sum of their n_max.
rbe2d_status create_handle(int n, const rbe2d_params *ps, bool batch, rbe2d_handle *out) {
    if (!out) return fail(nullptr, RBE2D_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 65536) return fail(nullptr, RBE2D_E_INVAL, "n_sys must be in [1, 65536]");
    if (!ps) return fail(nullptr, RBE2D_E_INVAL, "params is NULL");
    rbe2d_ctx *h = new (std::nothrow) rbe2d_ctx();
    if (!h) return fail(nullptr, RBE2D_E_NOMEM, "host allocation failed");
    h->n_sys = n;
    h->batch = batch;
    h->sys.resize(n);
    int64_t n_cap = 0, cap_p = 0, cap_s = 0;
    int cells = 0;
    size_t cdf_total = 0;
    for (int r = 0; r < n; r++) {
        rbe2d_status st = setup_system(&ps[r], h->sys[r]);
        if (st) {
            delete h;
            if (n > 1) g_create_error = "system " + std::to_string(r) + ": " + g_create_error;
            return st;
        }
        const rbe2d_params &p = h->sys[r].p;
        if (r > 0 && (p.P != h->sys[0].p.P || p.precision != h->sys[0].p.precision)) {
            delete h;
            return fail(nullptr, RBE2D_E_INVAL, "all systems of a batch need the same P and precision");
        }
        SysDesc &d = h->sys[r].d;
        d.cbase = cells;
        cells += d.ncx * d.ncy * d.ncz;
        for (int ax = 0; ax < 3; ax++) {
            d.cdf_off[ax] = (int)cdf_total;
            cdf_total += h->sys[r].cdf[ax].size();
        }
        n_cap += p.n_max;
        cap_p += (p.n_max + kTileMax - 1) / kTileMax * kTileMax;
        cap_s += (p.n_max + kWave - 1) / kWave * kWave;
    }
    if (n_cap > INT32_MAX - kTileMax || cap_p > INT32_MAX / 2 || cells > INT32_MAX / 2) {
        delete h;
        return fail(nullptr, RBE2D_E_INVAL, "total particle or cell capacity exceeds 2^30");
    }
    h->precision = h->sys[0].p.precision;
    h->iso = true;
    for (int r = 0; r < n; r++) h->iso = h->iso && h->sys[r].d.iso;
    h->P = h->sys[0].p.P;
    h->P_pad = (h->P + kPPad - 1) / kPPad * kPPad;
    h->n_cap = n_cap;
    h->cap_particles = std::max<int64_t>(cap_p, kTileMax);
    h->cap_sorted = std::max<int64_t>(cap_s, kWave);
    h->total_cells = cells;
    h->fpart_blocks = std::min<int64_t>(64 * (h->cap_particles / kBlock), 4096);
    (void)hipGetDevice(&h->device);

    hipError_t e = hipSuccess;
    auto A = [&](auto **ptr, size_t cnt) { if (e == hipSuccess) e = dalloc(h, ptr, cnt); };
    plan_workspace(h, cdf_total, true, A);
    Workspace &w = h->w;
    std::vector<SysDesc> descs(n);
    std::vector<ImgTable> imgs(n);
    std::vector<Family> fams((size_t)n * kMaxFamilies);
    std::vector<double> cdf(cdf_total);
    for (int r = 0; r < n; r++) {
        descs[r] = h->sys[r].d;
        imgs[r] = h->sys[r].img;
        std::copy(h->sys[r].fam.begin(), h->sys[r].fam.end(), fams.begin() + (size_t)r * kMaxFamilies);
        for (int ax = 0; ax < 3; ax++)
            std::copy(h->sys[r].cdf[ax].begin(), h->sys[r].cdf[ax].end(), cdf.begin() + descs[r].cdf_off[ax]);
    }
    if (e == hipSuccess) e = hipMemcpy(w.sys, descs.data(), n * sizeof(SysDesc), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.img, imgs.data(), n * sizeof(ImgTable), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.fam, fams.data(), fams.size() * sizeof(Family), hipMemcpyHostToDevice);
    if (e == hipSuccess && cdf_total)
        e = hipMemcpy(w.cdf, cdf.data(), cdf_total * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h->kstage, 3 * sizeof(int32_t) * n * h->P, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h->lay_stage, 5 * sizeof(int) * (n + 1), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->kev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->lay_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->tail_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        const bool oom = e == hipErrorOutOfMemory;
        free_all(h);
        delete h;
        return fail(nullptr, oom ? RBE2D_E_NOMEM : RBE2D_E_HIP, "workspace setup failed: %s",
                    hipGetErrorString(e));
    }
    *out = h;
    return RBE2D_OK;
}

// Particle layout of all systems for the given counts into lay (5 (n_sys +
// 1) ints: off, pbase, bbase, tbase, sbase) and the handle's launch sizes.
rbe2d_status compute_layout(rbe2d_ctx *h, const int64_t *counts, int *lay) {
    const int n = h->n_sys;
    int64_t total = 0;
    for (int r = 0; r < n; r++) {
        if (counts[r] < 0 || counts[r] > h->sys[r].p.n_max)
            return fail(h, RBE2D_E_INVAL, "system %d: N = %lld outside [0, n_max = %lld]", r,
                        (long long)counts[r], (long long)h->sys[r].p.n_max);
        total += counts[r];
    }
    const bool fp32 = h->precision == RBE2D_PREC_FP32_PHASE;
    const int nkc = h->P_pad / (fp32 ? kKChunk32 : kKChunk64);
    h->tuned_now = !h->tune.counts.empty() && std::equal(counts, counts + n, h->tune.counts.begin());
    int per;
    if (h->force_per) {
        per = h->force_per;
    } else if (h->tuned_now && h->tune.per) {
        per = h->tune.per;
    } else {
        // tile size: enough tiles to fill the chip, padding under ~10% of the particles
        per = choose_tile(total, nkc);
        for (; per > 1; per >>= 1) {
            int64_t padded = 0;
            const int64_t tile = (int64_t)kBlock * per;
            for (int r = 0; r < n; r++) padded += (counts[r] + tile - 1) / tile * tile;
            if (padded <= total + total / 10 + tile) break;
        }
    }
    const int tile = kBlock * per;
    std::fill(lay, lay + 5 * (n + 1), 0);
    int *off = lay, *pb = off + (n + 1), *bb = pb + (n + 1), *tb = bb + (n + 1), *sb = tb + (n + 1);
    for (int r = 0; r < n; r++) {
        off[r + 1] = off[r] + (int)counts[r];
        pb[r + 1] = pb[r] + (int)((counts[r] + tile - 1) / tile * tile);
        sb[r + 1] = sb[r] + (int)((counts[r] + kWave - 1) / kWave * kWave);
    }
    for (int r = 0; r <= n; r++) { bb[r] = pb[r] / kBlock; tb[r] = pb[r] / tile; }
    h->per = per;
    h->n_total = total;
    h->n_blocks = bb[n];
    h->n_tiles = tb[n];
    h->n_swaves = sb[n] / kWave;
    return RBE2D_OK;
}

// Particle layout of all systems for the given counts; uploaded (through
// pinned staging, ordered on the stream) only when it changes.
rbe2d_status set_layout(rbe2d_ctx *h, const int64_t *counts, hipStream_t s) {
    const int n = h->n_sys;
    h->calls++;
    std::vector<int> lay(5 * (n + 1), 0);
    rbe2d_status st = compute_layout(h, counts, lay.data());
    if (st) return st;
    if (h->lay_valid && lay == h->lay_host) return RBE2D_OK;
    if (h->lay_ev_pending) RBE2D_TRY(h, hipEventSynchronize(h->lay_ev), "layout wait");
    std::memcpy(h->lay_stage, lay.data(), lay.size() * sizeof(int));
    int *dst[5] = {h->w.lay.off, h->w.lay.pbase, h->w.lay.bbase, h->w.lay.tbase, h->w.lay.sbase};
    for (int k = 0; k < 5; k++)
        RBE2D_TRY(h, hipMemcpyAsync(dst[k], h->lay_stage + k * (n + 1), (n + 1) * sizeof(int),
                                    hipMemcpyHostToDevice, s), "layout upload");
    RBE2D_TRY(h, hipEventRecord(h->lay_ev, s), "layout event");
    h->lay_ev_pending = true;
    h->lay_host = lay;
    h->lay_valid = true;
    return RBE2D_OK;
}

rbe2d_status layout_from_offsets(rbe2d_ctx *h, const int64_t *offsets, hipStream_t s) {
    if (!offsets) return fail(h, RBE2D_E_INVAL, "offsets is NULL");
    if (offsets[0] != 0) return fail(h, RBE2D_E_INVAL, "offsets[0] must be 0");
    std::vector<int64_t> counts(h->n_sys);
    for (int r = 0; r < h->n_sys; r++) {
        counts[r] = offsets[r + 1] - offsets[r];
        if (counts[r] < 0) return fail(h, RBE2D_E_INVAL, "offsets must be nondecreasing");
    }
    return set_layout(h, counts.data(), s);
}

rbe2d_status check_arrays(rbe2d_ctx *h, const double *pos, const double *q) {
    if (!h->kset_valid) return fail(h, RBE2D_E_STATE, "no k-set: call rbe2d_set_kset or rbe2d_sample_kset");
    if (h->n_total > 0 && (!pos || !q)) return fail(h, RBE2D_E_INVAL, "pos or q is NULL");
    return RBE2D_OK;
}

// prep + structure factors + real space: everything the outputs depend on
// prep + structure factors + real space: everything the outputs depend on.
// With both halves requested, the k-space chain (prep, structure factors,
// per-k assembly) runs on the side stream while the cell list and the pair
// kernel run on `s`; `s` waits for both.  The cell build is latency- and
// atomic-bound and the pair kernel latency-limited, so the VALU-bound
// structure-factor pass fills their idle issue slots (1.79 instead of
// 1.93 ms per step of the 1e6-ion slab).  The fork and join are events, so
// the pattern is also captured into graphs.
rbe2d_status run_common(rbe2d_ctx *h, const double *pos, const double *q, uint32_t flags, bool want_dg,
                        hipStream_t s) {
    const bool kside = (flags & (RBE2D_KSPACE | RBE2D_IBC)) != 0;
    const bool real = (flags & RBE2D_REAL) != 0;
    hipStream_t ks = s;
    if (kside && real && h->n_total > 0 && !h->one_stream) {
        ks = h->side;
        RBE2D_TRY(h, hipEventRecord(h->fork_ev, s), "fork event");
        RBE2D_TRY(h, hipStreamWaitEvent(ks, h->fork_ev, 0), "fork wait");
    }
    // with two streams, real space is enqueued first (its cell list starts
    // ahead of the structure factors); on one stream the order is as listed
    if (real && ks != s) RBE2D_TRY(h, launch_real(h, pos, q, want_dg, s), "real-space launch");
    if (kside) RBE2D_TRY(h, launch_prep(h, pos, q, ks), "prep launch");
    if (flags & RBE2D_KSPACE) RBE2D_TRY(h, launch_kcoef_sf(h, ks, false, want_dg), "structure-factor launch");
    if (real && ks == s) RBE2D_TRY(h, launch_real(h, pos, q, want_dg, s), "real-space launch");
    if (ks != s) {
        RBE2D_TRY(h, hipEventRecord(h->join_ev, ks), "join event");
        RBE2D_TRY(h, hipStreamWaitEvent(s, h->join_ev, 0), "join wait");
    }
    return RBE2D_OK;
}

// Forces of `parts` into F (added to F with `accumulate`).  With real space
// and k-space/IBC both requested, the whole k-space chain including its force
// scatter runs on the side stream (writing F) while the cell list and pair
// kernel run on `s`; after the join one pass adds the real-space forces and,
// when vel is set, applies the closing half kick v += dt/2 F of an MD step.
// With mxs set, the MD's short-range forces are added too (on `s`, into the
// pair kernel's output while the k-space chain runs).
rbe2d_status compute_forces(rbe2d_ctx *h, const double *pos, const double *q, double *F, uint32_t parts,
                            bool accumulate, double *vel, double dt, hipStream_t s, const MdExtra *mxs) {
    const bool kside = (parts & (RBE2D_KSPACE | RBE2D_IBC)) != 0;
    if (kside && (parts & RBE2D_REAL) && h->n_total > 0 && !h->one_stream) {
        hipStream_t ks = h->side;
        RBE2D_TRY(h, hipEventRecord(h->fork_ev, s), "fork event");
        RBE2D_TRY(h, hipStreamWaitEvent(ks, h->fork_ev, 0), "fork wait");
        RBE2D_TRY(h, launch_real(h, pos, q, false, s), "real-space launch");
        if (mxs) RBE2D_TRY(h, launch_short(h, *mxs, nullptr, nullptr, s, true), "short-range launch");
        // with k-space the assembly launch computes the IBC scalars
        const bool sc_asm = (parts & RBE2D_KSPACE) != 0;
        RBE2D_TRY(h, launch_prep(h, pos, q, ks, !sc_asm), "prep launch");
        if (parts & RBE2D_KSPACE) RBE2D_TRY(h, launch_kcoef_sf(h, ks, true), "structure-factor launch");
        RBE2D_TRY(h, launch_kforce(h, pos, q, F, nullptr, parts & ~(uint32_t)RBE2D_REAL, accumulate, false, false,
                                   nullptr, ks), "force launch");
        RBE2D_TRY(h, hipEventRecord(h->join_ev, ks), "join event");
        RBE2D_TRY(h, hipStreamWaitEvent(s, h->join_ev, 0), "join wait");
        RBE2D_TRY(h, launch_add_real(h, F, vel, 0.5 * dt, s), "real-space add");
        return RBE2D_OK;
    }
    rbe2d_status st = run_common(h, pos, q, parts, false, s);
    if (st) return st;
    RBE2D_TRY(h, launch_kforce(h, pos, q, F, nullptr, parts, accumulate, false, (parts & RBE2D_REAL) != 0, nullptr,
                               s), "force launch");
    if (mxs) RBE2D_TRY(h, launch_short(h, *mxs, F, nullptr, s), "short-range launch");
    if (vel) RBE2D_TRY(h, launch_md_kick(h, vel, F, dt, s), "md kick");
    return RBE2D_OK;
}

rbe2d_status run_forces(rbe2d_ctx *h, const double *pos, const double *q, double *F, double *energy,
                        uint32_t flags, hipStream_t s) {
    if (flags & ~(uint32_t)(RBE2D_ALL | RBE2D_ACCUMULATE)) return fail(h, RBE2D_E_INVAL, "unknown flags");
    rbe2d_status st = check_arrays(h, pos, q);
    if (st) return st;
    if (h->n_total > 0 && !F) return fail(h, RBE2D_E_INVAL, "F is NULL");
    const uint32_t parts = flags & RBE2D_ALL;
    st = compute_forces(h, pos, q, F, parts, (flags & RBE2D_ACCUMULATE) != 0, nullptr, 0.0, s, nullptr);
    if (st) return st;
    if (energy) RBE2D_TRY(h, launch_energy(h, energy, parts, nullptr, nullptr, s), "energy launch");
    return RBE2D_OK;
}

rbe2d_status md_extra(rbe2d_ctx *h, const rbe2d_md_params *mp, double dt, MdExtra *mx) {
    if (!mp) return fail(h, RBE2D_E_INVAL, "md params are NULL");
    const double vals[] = {mp->gamma, mp->kT, mp->sigma, mp->eps, mp->sigma_wall, mp->eps_wall, mp->wall_margin};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(h, RBE2D_E_INVAL, "non-finite md parameter");
    if (mp->gamma < 0 || mp->kT < 0 || mp->eps < 0 || mp->eps_wall < 0)
        return fail(h, RBE2D_E_INVAL, "gamma, kT, eps, eps_wall must be >= 0");
    if ((mp->eps > 0 && !(mp->sigma > 0)) || (mp->eps_wall > 0 && !(mp->sigma_wall > 0)))
        return fail(h, RBE2D_E_INVAL, "sigma, sigma_wall must be > 0 where eps, eps_wall are");
    double hmin = h->sys[0].p.H;
    for (const SysHost &sh : h->sys) hmin = std::min(hmin, sh.p.H);
    if (!(mp->wall_margin > 0 && 2 * mp->wall_margin < hmin))
        return fail(h, RBE2D_E_INVAL, "need 0 < wall_margin < H/2");
    const double rlj = std::pow(2.0, 1.0 / 6.0) * mp->sigma;
    for (const SysHost &sh : h->sys)
        if (mp->eps > 0 && 2 * rlj > std::min(sh.p.Lx, sh.p.Ly))
            return fail(h, RBE2D_E_INVAL, "ion-ion LJ cutoff exceeds half the box");
    mx->c1 = std::exp(-mp->gamma * dt);
    mx->c2 = std::sqrt((1.0 - mx->c1 * mx->c1) * mp->kT);
    mx->sig2 = mp->sigma * mp->sigma;
    mx->eps = mp->eps;
    mx->rc2 = rlj * rlj;
    mx->sigw2 = mp->sigma_wall * mp->sigma_wall;
    mx->epsw = mp->eps_wall;
    mx->hcut = std::pow(2.0, 1.0 / 6.0) * mp->sigma_wall;
    mx->margin = mp->wall_margin;
    return RBE2D_OK;
}

// one step: velocity Verlet, or BAOAB with short-range forces when mx is
// set; the k-set (and the thermostat noise) use the device step counter when
// dev_step is set (graph replays), else stream id `step`
rbe2d_status md_step(rbe2d_ctx *h, double *pos, double *vel, const double *q, double *F, double dt,
                     double zlo, double zhi_from_top, uint64_t seed, int64_t step, bool dev_step,
                     const MdExtra *mx, hipStream_t s) {
    const uint64_t sbase = (uint64_t)step * (uint64_t)h->n_sys;
    // (without mx this runs only for an empty layout: plain velocity Verlet
    // with particles takes vv_run, which applies the wall bounds)
    (void)zlo;
    (void)zhi_from_top;
    if (mx)
        RBE2D_TRY(h, launch_md_kick_drift_langevin(h, pos, vel, F, dt, *mx, seed, sbase,
                                                   dev_step ? h->w.step : nullptr, s), "md drift");
    RBE2D_TRY(h, launch_sample(h, seed, sbase, dev_step ? h->w.step : nullptr, s), "md sample");
    // short-range forces and the closing half kick are fused into the force
    // evaluation
    const bool shortr = mx && mx->short_on();
    rbe2d_status st = compute_forces(h, pos, q, F, RBE2D_ALL, false, vel, dt, s, shortr ? mx : nullptr);
    if (st) return st;
    if (dev_step) RBE2D_TRY(h, launch_step_inc(h, s), "md step counter");
    return RBE2D_OK;
}

// Force evaluation and closing kick of one plain velocity-Verlet step at
// the current positions (whose k-set is drawn, with its k-vector table, and
// whose k-space particle records and IBC block sums the preceding MD pass
// wrote).  The k-space chain (structure factors, assembly with the IBC
// scalars, force scatter) runs on the side stream, real space on s.  After
// the forces, either the closing half kick (last step of the run) or one
// pass with the closing and next opening half kicks, the next drift and the
// next records.  Meanwhile the side stream draws the next step's k-set
// (device step counter: incremented there first) and builds its table.
// The next step's fork orders that draw before the next k-space chain; a
// captured step joins it back explicitly (join_tail).
rbe2d_status vv_unit(rbe2d_ctx *h, double *pos, double *vel, const double *q, double *F, double dt, double zlo,
                     double zhi_from_top, uint64_t seed, int64_t step, bool dev_step, bool last, bool join_tail,
                     hipStream_t s) {
    hipStream_t ks = h->side;
    RBE2D_TRY(h, hipEventRecord(h->fork_ev, s), "fork event");
    RBE2D_TRY(h, hipStreamWaitEvent(ks, h->fork_ev, 0), "fork wait");
    // real space first: its latency-bound cell list then starts ahead of the
    // structure factors (also in a captured graph, whose nodes follow this order)
    RBE2D_TRY(h, launch_real(h, pos, q, false, s), "real-space launch");
    RBE2D_TRY(h, launch_kcoef_sf(h, ks, true), "structure-factor launch");
    RBE2D_TRY(h, launch_kforce(h, pos, q, F, nullptr, RBE2D_KSPACE | RBE2D_IBC, false, false, false, nullptr, ks),
              "force launch");
    RBE2D_TRY(h, hipEventRecord(h->join_ev, ks), "join event");
    RBE2D_TRY(h, hipStreamWaitEvent(s, h->join_ev, 0), "join wait");
    if (!last) {
        if (dev_step) RBE2D_TRY(h, launch_step_inc(h, ks), "md step counter");
        RBE2D_TRY(h, launch_sample(h, seed, (uint64_t)(step + 1) * (uint64_t)h->n_sys, dev_step ? h->w.step : nullptr,
                                   ks), "md sample");
        launch_ktable(h, ks);
        RBE2D_TRY(h, launch_prep_md(h, pos, vel, F, q, dt, zlo, zhi_from_top, true, s), "md leapfrog");
    } else {
        RBE2D_TRY(h, launch_add_real(h, F, vel, 0.5 * dt, s), "real-space add");
    }
    if (join_tail) {
        RBE2D_TRY(h, hipEventRecord(h->tail_ev, ks), "tail event");
        RBE2D_TRY(h, hipStreamWaitEvent(s, h->tail_ev, 0), "tail wait");
    }
    return RBE2D_OK;
}

// plain velocity Verlet (no thermostat, no short-range forces) over n steps:
// the opening kick and drift with the caller's F and the first k-draw, then
// n force evaluations chained by fused kicks; with use_graph the middle ones
// are replays of one captured unit
rbe2d_status vv_run(rbe2d_ctx *h, double *pos, double *vel, const double *q, double *F, double dt, double zlo,
                    double zhi_from_top, uint64_t seed, int64_t step0, int32_t n_steps, bool use_graph,
                    hipStream_t s) {
    RBE2D_TRY(h, launch_prep_md(h, pos, vel, F, q, dt, zlo, zhi_from_top, false, s), "md drift");
    RBE2D_TRY(h, launch_sample(h, seed, (uint64_t)step0 * (uint64_t)h->n_sys, nullptr, s), "md sample");
    launch_ktable(h, s);
    int32_t it = 0;
    if (use_graph) {
        auto bits = [](double x) { uint64_t u; std::memcpy(&u, &x, 8); return u; };
        std::vector<uint64_t> key = {1, (uint64_t)(uintptr_t)pos, (uint64_t)(uintptr_t)vel, (uint64_t)(uintptr_t)q,
                                     (uint64_t)(uintptr_t)F, bits(dt), bits(zlo), bits(zhi_from_top), seed,
                                     (uint64_t)h->per};
        key.insert(key.end(), h->lay_host.begin(), h->lay_host.end());
        if (!h->md_exec || key != h->md_key) {
            free_graph(h);
            hipStream_t cs;
            RBE2D_TRY(h, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
            const int prof_n = h->prof.n;
            h->prof.n = 0;   // no profiling events inside the graph
            // a captured unit starts from counted cells and ends by counting
            // them for the next one; a failed capture leaves the state as it was
            const bool counted0 = h->cells_counted;
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            rbe2d_status st = RBE2D_OK;
            if (e == hipSuccess) {
                st = vv_unit(h, pos, vel, q, F, dt, zlo, zhi_from_top, seed, 0, true, false, true, cs);
                hipGraph_t g = nullptr;
                const hipError_t e2 = hipStreamEndCapture(cs, &g);
                if (st == RBE2D_OK && e2 != hipSuccess) st = hipfail(h, e2, "end capture");
                if (st == RBE2D_OK) {
                    h->md_graph = g;
                    const hipError_t e3 = hipGraphInstantiate(&h->md_exec, g, nullptr, nullptr, 0);
                    if (e3 != hipSuccess) st = hipfail(h, e3, "graph instantiate");
                } else if (g) {
                    (void)hipGraphDestroy(g);
                }
            } else {
                st = hipfail(h, e, "begin capture");
            }
            h->prof.n = prof_n;
            (void)hipStreamDestroy(cs);
            h->cells_counted = counted0;
            if (st) { free_graph(h); return st; }
            h->md_key = key;
        }
        RBE2D_TRY(h, launch_set_step(h, step0, s), "md step counter");
        for (; it < n_steps - 1; it++) RBE2D_TRY(h, hipGraphLaunch(h->md_exec, s), "graph launch");
    }
    for (; it < n_steps; it++) {
        rbe2d_status st = vv_unit(h, pos, vel, q, F, dt, zlo, zhi_from_top, seed, step0 + it, false,
                                  it == n_steps - 1, false, s);
        if (st) return st;
    }
    return RBE2D_OK;
}

// n_steps MD steps, eager or as replays of one captured step
rbe2d_status md_run(rbe2d_ctx *h, double *pos, double *vel, const double *q, double *F, double dt, double zlo,
                    double zhi_from_top, uint64_t seed, int64_t step0, int32_t n_steps, bool use_graph,
                    const MdExtra *mx, hipStream_t s) {
    if (n_steps <= 0) return RBE2D_OK;
    h->kset_valid = true;
    if (!mx && h->n_total > 0)
        return vv_run(h, pos, vel, q, F, dt, zlo, zhi_from_top, seed, step0, n_steps, use_graph, s);
    if (!use_graph) {
        for (int32_t it = 0; it < n_steps; it++) {
            rbe2d_status st = md_step(h, pos, vel, q, F, dt, zlo, zhi_from_top, seed, step0 + it, false, mx, s);
            if (st) return st;
        }
        return RBE2D_OK;
    }
    // a captured step is valid for these arguments and this layout only
    auto bits = [](double x) { uint64_t u; std::memcpy(&u, &x, 8); return u; };
    std::vector<uint64_t> key = {(uint64_t)(uintptr_t)pos, (uint64_t)(uintptr_t)vel, (uint64_t)(uintptr_t)q,
                                 (uint64_t)(uintptr_t)F, bits(dt), bits(zlo), bits(zhi_from_top), seed,
                                 (uint64_t)h->per};
    if (mx)
        for (double v : {mx->c1, mx->c2, mx->sig2, mx->eps, mx->rc2, mx->sigw2, mx->epsw, mx->hcut, mx->margin})
            key.push_back(bits(v));
    key.insert(key.end(), h->lay_host.begin(), h->lay_host.end());
    if (!h->md_exec || key != h->md_key) {
        free_graph(h);
        hipStream_t cs;
        RBE2D_TRY(h, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
        const int prof_n = h->prof.n;
        h->prof.n = 0;   // no profiling events inside the graph
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        rbe2d_status st = RBE2D_OK;
        if (e == hipSuccess) {
            st = md_step(h, pos, vel, q, F, dt, zlo, zhi_from_top, seed, 0, true, mx, cs);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (st == RBE2D_OK && e2 != hipSuccess) st = hipfail(h, e2, "end capture");
            if (st == RBE2D_OK) {
                h->md_graph = g;
                const hipError_t e3 = hipGraphInstantiate(&h->md_exec, g, nullptr, nullptr, 0);
                if (e3 != hipSuccess) st = hipfail(h, e3, "graph instantiate");
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        } else {
            st = hipfail(h, e, "begin capture");
        }
        h->prof.n = prof_n;
        (void)hipStreamDestroy(cs);
        if (st) { free_graph(h); return st; }
        h->md_key = key;
    }
    RBE2D_TRY(h, launch_set_step(h, step0, s), "md step counter");
    for (int32_t it = 0; it < n_steps; it++) RBE2D_TRY(h, hipGraphLaunch(h->md_exec, s), "graph launch");
    return RBE2D_OK;
}

// ---------------------------------------------------------------------------
// The evaluation without a handle (rbe2d_forces_noalloc): every workspace is
// carved from one file-scope device array, so a call allocates no device or
// pinned memory and creates no stream or event.
// ---------------------------------------------------------------------------

constexpr int64_t kStaticMaxN = 32768;     // largest n_max of the static path
constexpr int kStaticMaxP = 1024;          // largest P of the static path
constexpr int kStaticFparts = 1024;        // particle blocks' worth of force-pass partials
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

// The static path's workspaces (each GPU holds its own copy until the
// process ends).  Host code never passes this name to a kernel: it is a
// host-side stand-in, and the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct StaticState {
    unsigned char *base = nullptr;   // device address of `scratch` on this device
    rbe2d_ctx h;
    rbe2d_params last{};
    bool have = false;
};
StaticState g_static[kMaxDevices];
std::mutex g_static_mu;

// Tables of one system, passed by value as kernel arguments (each launch's
// arguments stay below 4 KB)
struct PutDesc {
    SysDesc d;
    int lay[10];
};
constexpr int kFamPerPut = 32;
struct PutFam {
    Family f[kFamPerPut];
    int first, count;
};

__global__ void k_put_desc(PutDesc a, SysDesc *sys, int *off, int *pbase, int *bbase, int *tbase, int *sbase,
                           int *err) {
    if (threadIdx.x != 0) return;
    *sys = a.d;
    int *dst[5] = {off, pbase, bbase, tbase, sbase};
    for (int k = 0; k < 5; k++) {
        dst[k][0] = a.lay[2 * k];
        dst[k][1] = a.lay[2 * k + 1];
    }
    err[0] = 0;
}
__global__ void k_put_img(ImgTable a, ImgTable *img) {
    if (threadIdx.x == 0) *img = a;
}
__global__ void k_put_fam(PutFam a, Family *fam) {
    if ((int)threadIdx.x < a.count) fam[a.first + threadIdx.x] = a.f[threadIdx.x];
}
__global__ void k_copy_err(const int *src, int32_t *dst) {
    if (threadIdx.x == 0) *dst = *src;
}

rbe2d_status forces_noalloc(const rbe2d_params *p, const int32_t *kset, int64_t N, const double *pos,
                            const double *q, double *F, double *energy, uint32_t flags, int32_t *err_word,
                            hipStream_t s) {
    rbe2d_status st = validate(p, nullptr);
    if (st) return st;
    if (p->n_max > kStaticMaxN || p->P > kStaticMaxP)
        return fail(nullptr, RBE2D_E_INVAL,
                    "rbe2d_forces_noalloc handles n_max <= %lld and P <= %d (got n_max = %lld, P = %d)",
                    (long long)kStaticMaxN, kStaticMaxP, (long long)p->n_max, p->P);
    if (N < 0 || N > p->n_max)
        return fail(nullptr, RBE2D_E_INVAL, "N = %lld outside [0, n_max = %lld]", (long long)N,
                    (long long)p->n_max);
    if (flags & ~(uint32_t)(RBE2D_ALL | RBE2D_ACCUMULATE)) return fail(nullptr, RBE2D_E_INVAL, "unknown flags");
    if (N > 0 && (!pos || !q || !F)) return fail(nullptr, RBE2D_E_INVAL, "pos, q or F is NULL");
    if (!kset && (flags & RBE2D_KSPACE)) return fail(nullptr, RBE2D_E_INVAL, "kset is NULL");
    int dev = 0;
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return hipfail(nullptr, ge, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, RBE2D_E_INVAL, "device index %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticState &S = g_static[dev];
    if (!S.base) {
        // once per device, with that device current: the array's address on it
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hipfail(nullptr, e, "hipGetSymbolAddress(scratch)");
        S.base = (unsigned char *)ptr;
    }
    rbe2d_ctx *h = &S.h;
    if (!S.have || std::memcmp(&S.last, p, sizeof *p) != 0) {
        // host set-up of the system (only when the parameters change)
        S.have = false;
        h->sys.resize(1);
        st = setup_system(p, h->sys[0]);
        if (st) return st;
        const rbe2d_params &pp = h->sys[0].p;
        SysDesc &d = h->sys[0].d;
        d.cbase = 0;
        h->n_sys = 1;
        h->batch = false;
        h->precision = pp.precision;
        h->P = pp.P;
        h->P_pad = (h->P + kPPad - 1) / kPPad * kPPad;
        h->n_cap = pp.n_max;
        h->cap_particles = std::max<int64_t>((pp.n_max + kTileMax - 1) / kTileMax * kTileMax, kTileMax);
        h->cap_sorted = std::max<int64_t>((pp.n_max + kWave - 1) / kWave * kWave, kWave);
        h->total_cells = d.ncx * d.ncy * d.ncz;
        h->iso = d.iso != 0;
        h->fpart_blocks = std::min<int64_t>(64 * (h->cap_particles / kBlock), kStaticFparts);
        h->one_stream = true;
        h->side = nullptr;
        // carve the workspaces from the array (256-byte aligned)
        size_t used = 0;
        auto carve = [&](auto **ptr, size_t cnt) {
            using T = std::remove_reference_t<decltype(**ptr)>;
            used = (used + 255) & ~(size_t)255;
            *ptr = (T *)(S.base + used);
            used += std::max<size_t>(cnt, 1) * sizeof(T);
        };
        plan_workspace(h, 1, false, carve);
        if (used > kScratchBytes)
            return fail(nullptr, RBE2D_E_INVAL, "rbe2d_forces_noalloc: %zu bytes of workspace exceed the %zu-byte array",
                        used, kScratchBytes);
        S.last = *p;
        S.have = true;
    }
    h->w.kset = const_cast<int32_t *>(kset);
    h->kset_valid = true;
    int64_t cnt = N;
    PutDesc pd;
    st = compute_layout(h, &cnt, pd.lay);
    if (st) return st;
    // tables and layout: stream-ordered kernel writes (the array keeps the
    // last call's contents; every call rewrites what it reads)
    const SysHost &sh = h->sys[0];
    pd.d = sh.d;
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, pd, h->w.sys, h->w.lay.off, h->w.lay.pbase,
                       h->w.lay.bbase, h->w.lay.tbase, h->w.lay.sbase, h->w.err);
    hipLaunchKernelGGL(k_put_img, dim3(1), dim3(64), 0, s, sh.img, h->w.img);
    for (int f0 = 0; f0 < (int)sh.fam.size(); f0 += kFamPerPut) {
        PutFam pf;
        pf.first = f0;
        pf.count = std::min<int>(kFamPerPut, (int)sh.fam.size() - f0);
        for (int i = 0; i < pf.count; i++) pf.f[i] = sh.fam[f0 + i];
        hipLaunchKernelGGL(k_put_fam, dim3(1), dim3(64), 0, s, pf, h->w.fam);
    }
    // the cell counts start at zero in every build (the array may hold
    // another call's values)
    RBE2D_TRY(nullptr, launch_fill(h->w.count, (int64_t)h->total_cells * 4, s), "count clear");
    h->cells_counted = false;
    RBE2D_TRY(nullptr, hipGetLastError(), "table upload");
    const uint32_t parts = flags & RBE2D_ALL;
    st = compute_forces(h, pos, q, F, parts, (flags & RBE2D_ACCUMULATE) != 0, nullptr, 0.0, s, nullptr);
    if (st) return fail(nullptr, st, "%s", h->err.c_str());
    if (energy) RBE2D_TRY(nullptr, launch_energy(h, energy, parts, nullptr, nullptr, s), "energy launch");
    if (err_word) hipLaunchKernelGGL(k_copy_err, dim3(1), dim3(64), 0, s, h->w.err, err_word);
    RBE2D_TRY(nullptr, hipGetLastError(), "launch");
    return RBE2D_OK;
}

}  // namespace

extern "C" {

rbe2d_status rbe2d_create(const rbe2d_params *p, rbe2d_handle *out) { return create_handle(1, p, false, out); }

rbe2d_status rbe2d_batch_create(int32_t n_sys, const rbe2d_params *params, rbe2d_handle *out) {
    return create_handle(n_sys, params, true, out);
}

void rbe2d_destroy(rbe2d_handle h) {
    if (!h) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    free_all(h);
    (void)hipSetDevice(cur);
    delete h;
}

rbe2d_status rbe2d_query(rbe2d_handle h, double *Lz_ext, double *V, double *S) {
    return rbe2d_query_system(h, 0, Lz_ext, V, S);
}

rbe2d_status rbe2d_query_system(rbe2d_handle h, int32_t sys, double *Lz_ext, double *V, double *S) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (sys < 0 || sys >= h->n_sys) return fail(h, RBE2D_E_INVAL, "system index out of range");
    const SysDesc &d = h->sys[sys].d;
    if (Lz_ext) *Lz_ext = d.Lz;
    if (V) *V = d.V;
    if (S) *S = d.S;
    return RBE2D_OK;
}

rbe2d_status rbe2d_draw_kset(const rbe2d_params *p, uint64_t seed, uint64_t stream_id, int32_t *n_out) {
    rbe2d_status st = validate(p, nullptr);
    if (st) return st;
    if (!n_out) return fail(nullptr, RBE2D_E_INVAL, "n_out is NULL");
    const double Lz = p->Lz_ext > 0.0 ? p->Lz_ext : auto_lz(p);
    const double Ls[3] = {p->Lx, p->Ly, Lz};
    int nm[3];
    std::vector<double> cdf[3];
    for (int d = 0; d < 3; d++) axis_table(p->alpha, Ls[d], &nm[d], cdf[d]);
    const uint64_t key = stream_key(seed, stream_id);
    for (int l = 0; l < p->P; l++) {
        bool ok = false;
        for (int att = 0; att < 64 && !ok; att++) {
            const uint64_t c = ((uint64_t)l * 64 + att) * 3;
            int n[3];
            for (int d = 0; d < 3; d++) n[d] = draw_axis(cdf[d].data(), nm[d], uniform01(key, c + d));
            if (n[0] | n[1] | n[2]) {
                n_out[3 * l] = n[0]; n_out[3 * l + 1] = n[1]; n_out[3 * l + 2] = n[2];
                ok = true;
            }
        }
        if (!ok) return fail(nullptr, RBE2D_E_STATE, "k-sampler drew 64 zero vectors in a row");
    }
    return RBE2D_OK;
}

rbe2d_status rbe2d_set_kset(rbe2d_handle h, const int32_t *n, int n_is_device, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (!n) return fail(h, RBE2D_E_INVAL, "n is NULL");
    h->calls++;
    hipStream_t s = (hipStream_t)stream;
    const size_t cnt = 3 * (size_t)h->n_sys * h->P;
    if (n_is_device) {
        RBE2D_TRY(h, hipMemcpyAsync(h->w.kset, n, cnt * sizeof(int32_t), hipMemcpyDeviceToDevice, s),
                  "set_kset copy");
        h->kset_valid = true;
        return RBE2D_OK;
    }
    for (int r = 0; r < h->n_sys; r++) {
        const SysDesc &d = h->sys[r].d;
        const int64_t lim = h->precision == RBE2D_PREC_FP32_PHASE ? ((int64_t)1 << (22 - d.fh_bits))
                                                                  : ((int64_t)1 << 20);
        for (int l = 0; l < h->P; l++) {
            const int32_t *v = n + 3 * ((size_t)r * h->P + l);
            if (!(v[0] | v[1] | v[2]))
                return fail(h, RBE2D_E_INVAL, "k-set entry %d of system %d is the zero vector", l, r);
            for (int c = 0; c < 3; c++)
                if (std::llabs((long long)v[c]) >= lim)
                    return fail(h, RBE2D_E_INVAL, "k-set entry %d of system %d exceeds |n| < %lld", l, r,
                                (long long)lim);
        }
    }
    // the pinned staging buffer may still feed the previous upload
    if (h->kev_pending) RBE2D_TRY(h, hipEventSynchronize(h->kev), "set_kset wait");
    std::memcpy(h->kstage, n, cnt * sizeof(int32_t));
    RBE2D_TRY(h, hipMemcpyAsync(h->w.kset, h->kstage, cnt * sizeof(int32_t), hipMemcpyHostToDevice, s),
              "set_kset copy");
    RBE2D_TRY(h, hipEventRecord(h->kev, s), "set_kset event");
    h->kev_pending = true;
    h->kset_valid = true;
    return RBE2D_OK;
}

rbe2d_status rbe2d_sample_kset(rbe2d_handle h, uint64_t seed, uint64_t stream_id, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    h->calls++;
    RBE2D_TRY(h, launch_sample(h, seed, stream_id, nullptr, (hipStream_t)stream), "sample_kset launch");
    h->kset_valid = true;
    return RBE2D_OK;
}

rbe2d_status rbe2d_get_kset(rbe2d_handle h, int32_t *n_host, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (!n_host) return fail(h, RBE2D_E_INVAL, "n_host is NULL");
    if (!h->kset_valid) return fail(h, RBE2D_E_STATE, "no k-set");
    hipStream_t s = (hipStream_t)stream;
    RBE2D_TRY(h, hipMemcpyAsync(n_host, h->w.kset, 3 * sizeof(int32_t) * h->n_sys * h->P, hipMemcpyDeviceToHost, s),
              "get_kset copy");
    RBE2D_TRY(h, hipStreamSynchronize(s), "get_kset sync");
    return RBE2D_OK;
}

static rbe2d_status single_layout(rbe2d_ctx *h, int64_t N, hipStream_t s) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (h->batch) return fail(h, RBE2D_E_STATE, "batched handle: use the rbe2d_batch_* calls");
    return set_layout(h, &N, s);
}

rbe2d_status rbe2d_forces(rbe2d_handle h, int64_t N, const double *pos, const double *q, double *F,
                          double *energy, uint32_t flags, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    rbe2d_status st = single_layout(h, N, s);
    if (st) return st;
    return run_forces(h, pos, q, F, energy, flags, s);
}

rbe2d_status rbe2d_batch_forces(rbe2d_handle h, const int64_t *offsets, const double *pos, const double *q,
                                double *F, double *energy, uint32_t flags, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    rbe2d_status st = layout_from_offsets(h, offsets, s);
    if (st) return st;
    return run_forces(h, pos, q, F, energy, flags, s);
}

rbe2d_status rbe2d_energy(rbe2d_handle h, int64_t N, const double *pos, const double *q, double *energy,
                          void *stream) {
    hipStream_t s = (hipStream_t)stream;
    rbe2d_status st = single_layout(h, N, s);
    if (st) return st;
    if (!energy) return fail(h, RBE2D_E_INVAL, "energy is NULL");
    st = check_arrays(h, pos, q);
    if (st) return st;
    // the gamma-derivative sums of the pair kernel cost little and let a
    // following rbe2d_energy_backward reuse everything this call leaves
    st = run_common(h, pos, q, RBE2D_ALL, true, s);
    if (st) return st;
    RBE2D_TRY(h, launch_energy(h, energy, RBE2D_ALL, nullptr, nullptr, s), "energy launch");
    h->fwd.at = h->calls;
    h->fwd.pos = pos;
    h->fwd.q = q;
    h->fwd.n = N;
    return RBE2D_OK;
}

rbe2d_status rbe2d_energy_backward(rbe2d_handle h, int64_t N, const double *pos, const double *q,
                                   const double *gE, double *dEdr, double *dEdq, double *dEdgamma,
                                   void *stream) {
    hipStream_t s = (hipStream_t)stream;
    // state of an immediately preceding rbe2d_energy on the same inputs:
    // per-k records (rho, A, B), the IBC scalars and the pair kernel's
    // per-particle outputs; otherwise it is recomputed
    const bool reuse = h && h->fwd.at == h->calls && h->fwd.pos == pos && h->fwd.q == q && h->fwd.n == N;
    rbe2d_status st = single_layout(h, N, s);
    if (st) return st;
    if (!gE) return fail(h, RBE2D_E_INVAL, "gE is NULL");
    st = check_arrays(h, pos, q);
    if (st) return st;
    if (!reuse) {
        st = run_common(h, pos, q, RBE2D_ALL, dEdgamma != nullptr, s);
        if (st) return st;
    }
    if (dEdr || dEdq)
        RBE2D_TRY(h, launch_kforce(h, pos, q, dEdr, dEdq, RBE2D_ALL, false, true, true, gE, s), "adjoint launch");
    if (dEdgamma) RBE2D_TRY(h, launch_energy(h, nullptr, RBE2D_ALL, gE, dEdgamma, s), "dgamma launch");
    return RBE2D_OK;
}

rbe2d_status rbe2d_md_run(rbe2d_handle h, int64_t N, double *pos, double *vel, const double *q, double *F,
                          double dt, double z_lo, double z_hi, uint64_t seed, int64_t step0, int32_t n_steps,
                          int32_t use_graph, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    rbe2d_status st = single_layout(h, N, s);
    if (st) return st;
    const SysHost &sh = h->sys[0];
    if (N > 0 && (!pos || !vel || !q || !F)) return fail(h, RBE2D_E_INVAL, "NULL array");
    if (!(dt > 0.0) || !(z_lo > 0.0 && z_lo < z_hi && z_hi < sh.p.H) || n_steps < 0)
        return fail(h, RBE2D_E_INVAL, "need dt > 0, 0 < z_lo < z_hi < H, n_steps >= 0");
    return md_run(h, pos, vel, q, F, dt, z_lo, sh.p.H - z_hi, seed, step0, n_steps, use_graph != 0, nullptr, s);
}

rbe2d_status rbe2d_batch_md_run(rbe2d_handle h, const int64_t *offsets, double *pos, double *vel, const double *q,
                                double *F, double dt, double wall_margin, uint64_t seed, int64_t step0,
                                int32_t n_steps, int32_t use_graph, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    rbe2d_status st = layout_from_offsets(h, offsets, s);
    if (st) return st;
    if (h->n_total > 0 && (!pos || !vel || !q || !F)) return fail(h, RBE2D_E_INVAL, "NULL array");
    double hmin = h->sys[0].p.H;
    for (const SysHost &sh : h->sys) hmin = std::min(hmin, sh.p.H);
    if (!(dt > 0.0) || !(wall_margin > 0.0 && 2 * wall_margin < hmin) || n_steps < 0)
        return fail(h, RBE2D_E_INVAL, "need dt > 0, 0 < wall_margin < H/2, n_steps >= 0");
    return md_run(h, pos, vel, q, F, dt, wall_margin, wall_margin, seed, step0, n_steps, use_graph != 0, nullptr,
                  s);
}

rbe2d_status rbe2d_force_variance(rbe2d_handle h, const int64_t *offsets, const double *pos, const double *q,
                                  double *var, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    rbe2d_status st = layout_from_offsets(h, offsets, s);
    if (st) return st;
    st = check_arrays(h, pos, q);
    if (st) return st;
    if (h->n_total > 0 && !var) return fail(h, RBE2D_E_INVAL, "var is NULL");
    st = run_common(h, pos, q, RBE2D_KSPACE, false, s);
    if (st) return st;
    RBE2D_TRY(h, launch_kforce(h, pos, q, nullptr, nullptr, RBE2D_KSPACE, false, false, false, nullptr, s, var),
              "variance launch");
    return RBE2D_OK;
}

rbe2d_status rbe2d_suggest_params(int64_t N, double Lx, double Ly, double H, double gamma_top, double gamma_bot,
                                  double tol, rbe2d_params *p) {
    if (!p) return fail(nullptr, RBE2D_E_INVAL, "params is NULL");
    if (N < 1 || !finite_pos(Lx) || !finite_pos(Ly) || !finite_pos(H))
        return fail(nullptr, RBE2D_E_INVAL, "need N >= 1 and finite Lx, Ly, H > 0");
    if (!(tol > 0.0 && tol < 1.0)) return fail(nullptr, RBE2D_E_INVAL, "tol must be in (0, 1)");
    if (!(std::fabs(gamma_top) <= 1.0) || !(std::fabs(gamma_bot) <= 1.0))
        return fail(nullptr, RBE2D_E_INVAL, "|gamma_top|, |gamma_bot| must be <= 1");
    const double lg = std::log(1.0 / tol);
    // alpha ~ (N / (Lx Ly H))^(1/3), independent of Lz (Sec. 2.4)
    double alpha = std::cbrt((double)N / (Lx * Ly * H));
    // real-space tail exp(-alpha^2 r_c^2) = tol, with r_c <= min(Lx, Ly)/2
    double rc = std::sqrt(lg) / alpha;
    if (rc > 0.5 * std::min(Lx, Ly)) {
        rc = 0.5 * std::min(Lx, Ly);
        alpha = std::sqrt(lg) / rc;
    }
    // smallest M whose image truncation estimate of Theorem 3.2 is within tol
    const double decay = 2.0 * kPi * H / std::max(Lx, Ly);
    int M = 0;
    for (; M < 64; M++) {
        int a, b;
        exponents(M + 1, -1, &a, &b);   // floor((M+1)/2) of gamma_top, ceil((M+1)/2) of gamma_bot
        const double est = ipow(std::fabs(gamma_top), a) * ipow(std::fabs(gamma_bot), b) * std::exp(-decay * (M - 1));
        if (est <= tol) break;
    }
    p->alpha = alpha;
    p->r_c = rc;
    p->M = M;
    p->gamma_top = gamma_top;
    p->gamma_bot = gamma_bot;
    p->Lx = Lx; p->Ly = Ly; p->H = H;
    p->eps_lz = tol;
    p->Lz_ext = auto_lz(p);
    return RBE2D_OK;
}

rbe2d_status rbe2d_short_forces(rbe2d_handle h, const int64_t *offsets, const double *pos, const double *q,
                                double *F, double *energy, const rbe2d_md_params *mp, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    MdExtra mx;
    rbe2d_status st = md_extra(h, mp, 1.0, &mx);
    if (st) return st;
    st = layout_from_offsets(h, offsets, s);
    if (st) return st;
    if (h->n_total > 0 && (!pos || !q || !F)) return fail(h, RBE2D_E_INVAL, "NULL array");
    if (mx.short_on()) RBE2D_TRY(h, launch_cells(h, pos, q, s), "cell list");
    RBE2D_TRY(h, launch_short(h, mx, F, energy, s), "short-range launch");
    return RBE2D_OK;
}

rbe2d_status rbe2d_md_run_ex(rbe2d_handle h, const int64_t *offsets, double *pos, double *vel, const double *q,
                             double *F, double dt, const rbe2d_md_params *mp, uint64_t seed, int64_t step0,
                             int32_t n_steps, int32_t use_graph, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!(dt > 0.0) || n_steps < 0) return fail(h, RBE2D_E_INVAL, "need dt > 0, n_steps >= 0");
    MdExtra mx;
    rbe2d_status st = md_extra(h, mp, dt, &mx);
    if (st) return st;
    st = layout_from_offsets(h, offsets, s);
    if (st) return st;
    if (h->n_total > 0 && (!pos || !vel || !q || !F)) return fail(h, RBE2D_E_INVAL, "NULL array");
    return md_run(h, pos, vel, q, F, dt, mx.margin, mx.margin, seed, step0, n_steps, use_graph != 0, &mx, s);
}

rbe2d_status rbe2d_autotune(rbe2d_handle h, const int64_t *offsets, const double *pos, const double *q,
                            int32_t *chosen, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!offsets) return fail(h, RBE2D_E_INVAL, "offsets is NULL");
    if (offsets[0] != 0) return fail(h, RBE2D_E_INVAL, "offsets[0] must be 0");
    std::vector<int64_t> counts(h->n_sys);
    for (int r = 0; r < h->n_sys; r++) {
        counts[r] = offsets[r + 1] - offsets[r];
        if (counts[r] < 0 || counts[r] > h->sys[r].p.n_max)
            return fail(h, RBE2D_E_INVAL, "system %d: N outside [0, n_max]", r);
    }
    int64_t total = 0;
    for (int64_t c : counts) total += c;
    if (!h->kset_valid) return fail(h, RBE2D_E_STATE, "no k-set: call rbe2d_set_kset or rbe2d_sample_kset");
    if (total > 0 && (!pos || !q)) return fail(h, RBE2D_E_INVAL, "pos or q is NULL");
    RBE2D_TRY(h, hipStreamSynchronize(s), "autotune sync");
    free_graph(h);                 // a captured step holds the old launch parameters
    h->tune = rbe2d_ctx::Tuning();
    const int prof_n = h->prof.n;
    h->prof.n = 0;                 // the trials are not traced
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rbe2d_status st = RBE2D_OK;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    // minimum over reps of the duration of the launches `fn` enqueues
    auto time = [&](auto fn, int reps, float *best) -> rbe2d_status {
        *best = 1e30f;
        for (int i = 0; i < reps; i++) {
            RBE2D_TRY(h, hipEventRecord(e0, s), "autotune event");
            RBE2D_TRY(h, fn(), "autotune launch");
            RBE2D_TRY(h, hipEventRecord(e1, s), "autotune event");
            RBE2D_TRY(h, hipEventSynchronize(e1), "autotune sync");
            float ms = 0.0f;
            RBE2D_TRY(h, hipEventElapsedTime(&ms, e0, e1), "autotune elapsed");
            *best = std::min(*best, ms);
        }
        return RBE2D_OK;
    };
    int best_per = 1, best_ks = 1, best_rs = 1;
    if (he != hipSuccess) st = hipfail(h, he, "autotune events");
    // 1. particles per thread of the structure-factor tiles
    float tbest = 1e30f;
    for (int per = kMaxTileThreads; st == RBE2D_OK && per >= 1 && total > 0; per >>= 1) {
        h->force_per = per;
        st = set_layout(h, counts.data(), s);
        float t = 0.0f;
        if (st == RBE2D_OK)
            st = time([&] {
                hipError_t e = launch_prep(h, pos, q, s);
                return e == hipSuccess ? launch_kcoef_sf(h, s) : e;
            }, 3, &t);
        if (st == RBE2D_OK && t < tbest) { tbest = t; best_per = per; }
    }
    // 2. k-range split of the force pass (the per-k records of the chosen tiling)
    h->force_per = best_per;
    if (st == RBE2D_OK) st = set_layout(h, counts.data(), s);
    if (st == RBE2D_OK && total > 0) {
        const hipError_t e = launch_prep(h, pos, q, s);
        if (e != hipSuccess) st = hipfail(h, e, "autotune prep");
        else if ((he = launch_kcoef_sf(h, s)) != hipSuccess) st = hipfail(h, he, "autotune sf");
    }
    tbest = 1e30f;
    for (int ks = 1; st == RBE2D_OK && ks <= 64 && total > 0; ks <<= 1) {
        if ((int64_t)ks * h->n_blocks > h->fpart_blocks) break;
        h->force_ksplit = ks;
        float t = 0.0f;
        // the real-space output array serves as scratch for the forces
        st = time([&] {
            return launch_kforce(h, pos, q, (double *)h->w.freal, nullptr, RBE2D_KSPACE, false, false, false,
                                 nullptr, s);
        }, 3, &t);
        if (st == RBE2D_OK && t < tbest) { tbest = t; best_ks = ks; }
    }
    h->force_ksplit = 0;
    // 3. column-group split of the pair work (small systems only)
    tbest = 1e30f;
    for (int rs = 1; st == RBE2D_OK && rs <= kMaxRealSplit && total > 0 && total <= h->split_cap; rs++) {
        h->force_rsplit = rs;
        float t = 0.0f;
        st = time([&] { return launch_real(h, pos, q, false, s); }, 3, &t);
        if (st == RBE2D_OK && t < tbest) { tbest = t; best_rs = rs; }
    }
    h->force_rsplit = 0;
    h->force_per = 0;
    h->prof.n = prof_n;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) return st;
    h->tune.counts = counts;
    h->tune.per = best_per;
    h->tune.ksplit = best_ks;
    h->tune.rsplit = best_rs;
    st = set_layout(h, counts.data(), s);
    if (st) return st;
    if (chosen) { chosen[0] = best_per; chosen[1] = best_ks; chosen[2] = best_rs; }
    RBE2D_TRY(h, hipStreamSynchronize(s), "autotune sync");
    return RBE2D_OK;
}

rbe2d_status rbe2d_profile_enable(rbe2d_handle h, int32_t n_events) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (n_events < 0 || n_events > (1 << 20)) return fail(h, RBE2D_E_INVAL, "n_events out of range");
    RBE2D_TRY(h, hipDeviceSynchronize(), "profile sync");
    prof_free(h);
    Profiler &p = h->prof;
    for (int sl = 0; sl < RBE2D_PROF_SLOTS; sl++)
        for (int b = 0; b < 2; b++) {
            p.ev[sl][b].resize(n_events);
            for (int i = 0; i < n_events; i++) RBE2D_TRY(h, hipEventCreate(&p.ev[sl][b][i]), "profile event");
        }
    p.n = n_events;
    p.mask = ~0u;
    return RBE2D_OK;
}

rbe2d_status rbe2d_profile_classes(rbe2d_handle h, uint32_t class_mask) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    h->prof.mask = class_mask;
    return RBE2D_OK;
}

rbe2d_status rbe2d_profile_read(rbe2d_handle h, double *ms, int64_t *launches, int32_t n_slots) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (n_slots < 0 || n_slots > RBE2D_PROF_SLOTS) return fail(h, RBE2D_E_INVAL, "n_slots out of range");
    RBE2D_TRY(h, hipDeviceSynchronize(), "profile sync");
    Profiler &p = h->prof;
    for (int sl = 0; sl < RBE2D_PROF_SLOTS; sl++) {
        double t = 0.0;
        for (int i = 0; i < p.used[sl]; i++) {
            float f = 0.0f;
            RBE2D_TRY(h, hipEventElapsedTime(&f, p.ev[sl][0][i], p.ev[sl][1][i]), "profile elapsed");
            t += f;
        }
        if (sl < n_slots) {
            if (ms) ms[sl] = t;
            if (launches) launches[sl] = p.used[sl];
        }
        p.used[sl] = 0;
    }
    return RBE2D_OK;
}

rbe2d_status rbe2d_forces_noalloc(const rbe2d_params *p, const int32_t *kset, int64_t N, const double *pos,
                                  const double *q, double *F, double *energy, uint32_t flags, int32_t *err_word,
                                  void *stream) {
    return forces_noalloc(p, kset, N, pos, q, F, energy, flags, err_word, (hipStream_t)stream);
}

rbe2d_status rbe2d_set_surface_charges(rbe2d_handle h, int32_t sys, double sigma_top, double sigma_bot) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (sys < -1 || sys >= h->n_sys) return fail(h, RBE2D_E_INVAL, "system index out of range");
    if (!std::isfinite(sigma_top) || !std::isfinite(sigma_bot))
        return fail(h, RBE2D_E_INVAL, "surface charge densities must be finite");
    for (int r = 0; r < h->n_sys; r++) {
        if (sys >= 0 && r != sys) continue;
        h->sys[r].d.sig_top = sigma_top;
        h->sys[r].d.sig_bot = sigma_bot;
        surface_setup(h->sys[r]);
    }
    h->calls++;
    std::vector<SysDesc> descs(h->n_sys);
    for (int r = 0; r < h->n_sys; r++) descs[r] = h->sys[r].d;
    RBE2D_TRY(h, hipDeviceSynchronize(), "surface charges sync");
    RBE2D_TRY(h, hipMemcpy(h->w.sys, descs.data(), h->n_sys * sizeof(SysDesc), hipMemcpyHostToDevice),
              "surface charges upload");
    return RBE2D_OK;
}

rbe2d_status rbe2d_check(rbe2d_handle h, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    hipStream_t s = (hipStream_t)stream;
    RBE2D_TRY(h, hipStreamSynchronize(s), "check sync");
    RBE2D_TRY(h, hipGetLastError(), "asynchronous kernel error");
    int word = 0;
    RBE2D_TRY(h, hipMemcpy(&word, h->w.err, sizeof(int), hipMemcpyDeviceToHost), "check read");
    if (word) RBE2D_TRY(h, hipMemset(h->w.err, 0, sizeof(int)), "check clear");
    if (word & 1) return fail(h, RBE2D_E_RANGE, "a particle had z outside (0, H)");
    if (word & 2) return fail(h, RBE2D_E_STATE, "device k-sampler drew 64 zero vectors in a row");
    return RBE2D_OK;
}

const char *rbe2d_last_error(rbe2d_handle h) {
    if (!h) return g_create_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
