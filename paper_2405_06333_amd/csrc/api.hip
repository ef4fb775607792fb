// C ABI of librbe2d (declared in include/rbe2d.h): parameter validation,
// derived constants, workspace management, the host k-sampler and the
// launch sequences of one RBE2D evaluation (Algorithm 2 of the paper).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdarg>
#include <cstdlib>
#include <cstring>

#include "rbe2d_internal.h"

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

#define RBE2D_TRY(h, call, what)                       \
    do {                                               \
        hipError_t e_ = (call);                        \
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

}  // namespace

extern "C" {

rbe2d_status rbe2d_create(const rbe2d_params *pin, rbe2d_handle *out) {
    if (!out) return fail(nullptr, RBE2D_E_INVAL, "out is NULL");
    *out = nullptr;
    rbe2d_status st = validate(pin, nullptr);
    if (st) return st;
    rbe2d_ctx *h = new (std::nothrow) rbe2d_ctx();
    if (!h) return fail(nullptr, RBE2D_E_NOMEM, "host allocation failed");
    h->p = *pin;
    rbe2d_params &p = h->p;
    if (p.eps_lz <= 0.0) p.eps_lz = 1e-6;
    if (p.coulomb_prefactor == 0.0) p.coulomb_prefactor = 1.0;
    h->pref = p.coulomb_prefactor;
    h->Lz = p.Lz_ext > 0.0 ? p.Lz_ext : auto_lz(&p);
    if (h->Lz < (p.M + 1) * p.H) {
        delete h;
        return fail(nullptr, RBE2D_E_INVAL,
                    "Lz_ext = %g < (M+1) H = %g: the z-replicas of the charges would overlap their images",
                    p.Lz_ext, (p.M + 1) * p.H);
    }
    p.Lz_ext = h->Lz;
    h->V = p.Lx * p.Ly * h->Lz;
    h->S = theta_axis(p.alpha, p.Lx) * theta_axis(p.alpha, p.Ly) * theta_axis(p.alpha, h->Lz) - 1.0;
    h->M = p.M;
    h->P = p.P;
    h->P_pad = (p.P + kPPad - 1) / kPPad * kPPad;

    // image weights, their derivatives and the IBC image-dipole coefficients
    ImgTable img;
    std::memset(&img, 0, sizeof img);
    h->gp.assign(std::max(1, p.M), 0.0);
    h->gm.assign(std::max(1, p.M), 0.0);
    h->g1 = 1.0; h->cgam = 0.0;
    for (int l = 1; l <= p.M; l++) {
        int a, b;
        exponents(l, +1, &a, &b);
        img.ea_p[l - 1] = a; img.eb_p[l - 1] = b;
        const double gpl = ipow(p.gamma_top, a) * ipow(p.gamma_bot, b);
        const double dpt = dmono(a, p.gamma_top, b, p.gamma_bot), dpb = dmono(b, p.gamma_bot, a, p.gamma_top);
        exponents(l, -1, &a, &b);
        img.ea_m[l - 1] = a; img.eb_m[l - 1] = b;
        const double gml = ipow(p.gamma_top, a) * ipow(p.gamma_bot, b);
        const double dmt = dmono(a, p.gamma_top, b, p.gamma_bot), dmb = dmono(b, p.gamma_bot, a, p.gamma_top);
        h->gp[l - 1] = gpl; h->gm[l - 1] = gml;
        img.gp[l - 1] = gpl; img.gm[l - 1] = gml;
        const double sgn = (l % 2 == 0) ? 1.0 : -1.0;
        const double shp = 2.0 * ((l + 1) / 2) * p.H, shm = -2.0 * (l / 2) * p.H;
        h->g1 += sgn * (gpl + gml);
        h->cgam += shp * gpl + shm * gml;
        h->dg1[0] += sgn * (dpt + dmt); h->dg1[1] += sgn * (dpb + dmb);
        h->dcgam[0] += shp * dpt + shm * dmt; h->dcgam[1] += shp * dpb + shm * dmb;
        // real-space families that can come within r_c of the slab
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
                h->fam.push_back(f);
            }
        }
    }
    if ((int)h->fam.size() > kMaxFamilies) {
        delete h;
        return fail(nullptr, RBE2D_E_INVAL, "too many image orders within r_c (H too small for r_c)");
    }

    // k-sampling tables and the FP32 phase split
    h->cdf_host.resize(3);
    const double Ls[3] = {p.Lx, p.Ly, h->Lz};
    int nall = 0;
    for (int d = 0; d < 3; d++) {
        axis_table(p.alpha, Ls[d], &h->nmax[d], h->cdf_host[d]);
        nall = std::max(nall, h->nmax[d]);
    }
    int bits = 0;
    while ((1 << bits) <= nall) bits++;
    h->fh_bits = std::max(1, 23 - bits);
    if (p.precision == RBE2D_PREC_FP32_PHASE && bits > 20) {
        delete h;
        return fail(nullptr, RBE2D_E_INVAL, "k-range too wide for FP32 phases (alpha L too large)");
    }

    // cell grid: cells >= r_c / reach in x and y (searched +-reach columns),
    // >= r_c / reach in z; coarsened if there would be too many cells
    h->reach = 2;
    h->ncx = std::max(1, (int)std::floor(h->reach * p.Lx / p.r_c));
    h->ncy = std::max(1, (int)std::floor(h->reach * p.Ly / p.r_c));
    h->ncz = std::max(1, (int)std::floor(h->reach * p.H / p.r_c));
    const int64_t cell_cap = std::max<int64_t>(2 * p.n_max, 4096);
    while ((int64_t)h->ncx * h->ncy * h->ncz > cell_cap && (h->ncx > 5 || h->ncy > 5 || h->ncz > 1)) {
        if (h->ncz > 1) h->ncz = (h->ncz + 1) / 2;
        else { h->ncx = std::max(5, h->ncx / 2); h->ncy = std::max(5, h->ncy / 2); }
    }
    h->ncells = h->ncx * h->ncy * h->ncz;
    if (const char *env = std::getenv("RBE2D_REAL_ROUND_MIN")) h->round_min = std::max(1, std::min(64, std::atoi(env)));
    h->hx = p.Lx / h->ncx; h->hy = p.Ly / h->ncy; h->hz = p.H / h->ncz;

    (void)hipGetDevice(&h->device);
    const int64_t ncap = (std::max<int64_t>(p.n_max, 1) + kTileMax - 1) / kTileMax * kTileMax;
    h->n_cap = ncap;
    const int64_t nblk = ncap / kBlock;
    Workspace &w = h->w;
    hipError_t e = hipSuccess;
    auto A = [&](auto **ptr, size_t n) { if (e == hipSuccess) e = dalloc(h, ptr, n); };
    A(&w.p32, 2 * ncap);
    A(&w.p64, ncap);
    A(&w.bpart, 4 * nblk);
    A(&w.scal, 16);
    A(&w.kn32, h->P_pad);
    A(&w.kn64, h->P_pad);
    double *sfp = nullptr;
    A(&sfp, (size_t)nblk * h->P_pad * 4);
    w.sfpart = sfp;
    A(&w.krec, (size_t)h->P * kKRec);
    A(&w.kf32, 2 * (size_t)h->P);
    A(&w.fpart, (size_t)std::min<int64_t>(64 * ncap, 4096 * kBlock) * 4);
    A(&w.cell, ncap); A(&w.slot, ncap); A(&w.tmp, ncap); A(&w.sidx, ncap); A(&w.scell, ncap);
    A(&w.count, h->ncells); A(&w.start, h->ncells + 1); A(&w.scanbuf, h->ncells / 1024 + 2);
    A(&w.sorted, ncap); A(&w.freal, ncap); A(&w.dgreal, ncap);
    A(&w.rpart, 3 * nblk);
    A(&w.fam, std::max<size_t>(1, h->fam.size()));
    A(&w.img, 1);
    A(&w.err, 4);
    A(&w.kset, 3 * (size_t)h->P);
    for (int d = 0; d < 3; d++) A(&w.cdf[d], h->cdf_host[d].size());
    if (e == hipSuccess && !h->fam.empty())
        e = hipMemcpy(w.fam, h->fam.data(), h->fam.size() * sizeof(Family), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w.img, &img, sizeof img, hipMemcpyHostToDevice);
    for (int d = 0; d < 3 && e == hipSuccess; d++)
        e = hipMemcpy(w.cdf[d], h->cdf_host[d].data(), h->cdf_host[d].size() * sizeof(double),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h->kstage, 3 * sizeof(int32_t) * h->P, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->kev, hipEventDisableTiming);
    if (e != hipSuccess) {
        const bool oom = e == hipErrorOutOfMemory;
        for (void *ptr : h->allocs) (void)hipFree(ptr);
        if (h->kstage) (void)hipHostFree(h->kstage);
        if (h->kev) (void)hipEventDestroy(h->kev);
        delete h;
        return fail(nullptr, oom ? RBE2D_E_NOMEM : RBE2D_E_HIP, "workspace setup failed: %s",
                    hipGetErrorString(e));
    }
    *out = h;
    return RBE2D_OK;
}

void rbe2d_destroy(rbe2d_handle h) {
    if (!h) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    prof_free(h);
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->kstage) (void)hipHostFree(h->kstage);
    if (h->kev) (void)hipEventDestroy(h->kev);
    (void)hipSetDevice(cur);
    delete h;
}

rbe2d_status rbe2d_query(rbe2d_handle h, double *Lz_ext, double *V, double *S) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (Lz_ext) *Lz_ext = h->Lz;
    if (V) *V = h->V;
    if (S) *S = h->S;
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
    hipStream_t s = (hipStream_t)stream;
    if (n_is_device) {
        RBE2D_TRY(h, hipMemcpyAsync(h->w.kset, n, 3 * sizeof(int32_t) * h->P, hipMemcpyDeviceToDevice, s),
                  "set_kset copy");
        h->kset_valid = true;
        return RBE2D_OK;
    }
    const int64_t lim = h->p.precision == RBE2D_PREC_FP32_PHASE ? ((int64_t)1 << (24 - h->fh_bits)) : ((int64_t)1 << 20);
    for (int l = 0; l < h->P; l++) {
        if (!(n[3 * l] | n[3 * l + 1] | n[3 * l + 2]))
            return fail(h, RBE2D_E_INVAL, "k-set entry %d is the zero vector", l);
        for (int d = 0; d < 3; d++)
            if (std::llabs((long long)n[3 * l + d]) >= lim)
                return fail(h, RBE2D_E_INVAL, "k-set entry %d exceeds |n| < %lld", l, (long long)lim);
    }
    // the pinned staging buffer may still feed the previous upload
    if (h->kev_pending) RBE2D_TRY(h, hipEventSynchronize(h->kev), "set_kset wait");
    std::memcpy(h->kstage, n, 3 * sizeof(int32_t) * h->P);
    RBE2D_TRY(h, hipMemcpyAsync(h->w.kset, h->kstage, 3 * sizeof(int32_t) * h->P, hipMemcpyHostToDevice, s),
              "set_kset copy");
    RBE2D_TRY(h, hipEventRecord(h->kev, s), "set_kset event");
    h->kev_pending = true;
    h->kset_valid = true;
    return RBE2D_OK;
}

rbe2d_status rbe2d_sample_kset(rbe2d_handle h, uint64_t seed, uint64_t stream_id, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    RBE2D_TRY(h, launch_sample(h, seed, stream_id, (hipStream_t)stream), "sample_kset launch");
    h->kset_valid = true;
    return RBE2D_OK;
}

rbe2d_status rbe2d_get_kset(rbe2d_handle h, int32_t *n_host, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (!n_host) return fail(h, RBE2D_E_INVAL, "n_host is NULL");
    if (!h->kset_valid) return fail(h, RBE2D_E_STATE, "no k-set");
    hipStream_t s = (hipStream_t)stream;
    RBE2D_TRY(h, hipMemcpyAsync(n_host, h->w.kset, 3 * sizeof(int32_t) * h->P, hipMemcpyDeviceToHost, s),
              "get_kset copy");
    RBE2D_TRY(h, hipStreamSynchronize(s), "get_kset sync");
    return RBE2D_OK;
}

static rbe2d_status check_call(rbe2d_ctx *h, int64_t N, const double *pos, const double *q) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (N < 0 || N > h->p.n_max) return fail(h, RBE2D_E_INVAL, "N = %lld outside [0, n_max = %lld]",
                                             (long long)N, (long long)h->p.n_max);
    if (N > 0 && (!pos || !q)) return fail(h, RBE2D_E_INVAL, "pos or q is NULL");
    if (!h->kset_valid) return fail(h, RBE2D_E_STATE, "no k-set: call rbe2d_set_kset or rbe2d_sample_kset");
    return RBE2D_OK;
}

// prep + structure factors + real space: everything the outputs depend on
static rbe2d_status run_common(rbe2d_ctx *h, int64_t N, const double *pos, const double *q,
                               uint32_t flags, bool want_dg, hipStream_t s) {
    const bool fp32 = h->p.precision == RBE2D_PREC_FP32_PHASE;
    const int nkc = h->P_pad / (fp32 ? kKChunk32 : kKChunk64);
    const int per = choose_tile(N, nkc);
    const int64_t tile = (int64_t)kBlock * per;
    const int64_t N_pad = (N + tile - 1) / tile * tile;
    if (flags & (RBE2D_KSPACE | RBE2D_IBC))
        RBE2D_TRY(h, launch_prep(h, N, N_pad, pos, q, s), "prep launch");
    if (flags & RBE2D_KSPACE) RBE2D_TRY(h, launch_kcoef_sf(h, N_pad, per, s), "structure-factor launch");
    if (flags & RBE2D_REAL) RBE2D_TRY(h, launch_real(h, N, pos, q, want_dg, s), "real-space launch");
    return RBE2D_OK;
}

rbe2d_status rbe2d_forces(rbe2d_handle h, int64_t N, const double *pos, const double *q, double *F,
                          double *energy, uint32_t flags, void *stream) {
    rbe2d_status st = check_call(h, N, pos, q);
    if (st) return st;
    if (flags & ~(uint32_t)(RBE2D_ALL | RBE2D_ACCUMULATE)) return fail(h, RBE2D_E_INVAL, "unknown flags");
    if (N > 0 && !F) return fail(h, RBE2D_E_INVAL, "F is NULL");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t parts = flags & RBE2D_ALL;
    st = run_common(h, N, pos, q, parts, false, s);
    if (st) return st;
    RBE2D_TRY(h, launch_kforce(h, N, pos, q, F, nullptr, parts, (flags & RBE2D_ACCUMULATE) != 0, false,
                               (parts & RBE2D_REAL) != 0, nullptr, s), "force launch");
    if (energy) RBE2D_TRY(h, launch_energy(h, N, energy, parts, nullptr, nullptr, s), "energy launch");
    return RBE2D_OK;
}

rbe2d_status rbe2d_energy(rbe2d_handle h, int64_t N, const double *pos, const double *q, double *energy,
                          void *stream) {
    rbe2d_status st = check_call(h, N, pos, q);
    if (st) return st;
    if (!energy) return fail(h, RBE2D_E_INVAL, "energy is NULL");
    hipStream_t s = (hipStream_t)stream;
    st = run_common(h, N, pos, q, RBE2D_ALL, false, s);
    if (st) return st;
    RBE2D_TRY(h, launch_energy(h, N, energy, RBE2D_ALL, nullptr, nullptr, s), "energy launch");
    return RBE2D_OK;
}

rbe2d_status rbe2d_energy_backward(rbe2d_handle h, int64_t N, const double *pos, const double *q,
                                   const double *gE, double *dEdr, double *dEdq, double *dEdgamma,
                                   void *stream) {
    rbe2d_status st = check_call(h, N, pos, q);
    if (st) return st;
    if (!gE) return fail(h, RBE2D_E_INVAL, "gE is NULL");
    hipStream_t s = (hipStream_t)stream;
    st = run_common(h, N, pos, q, RBE2D_ALL, dEdgamma != nullptr, s);
    if (st) return st;
    if (dEdr || dEdq)
        RBE2D_TRY(h, launch_kforce(h, N, pos, q, dEdr, dEdq, RBE2D_ALL, false, true, true, gE, s),
                  "adjoint launch");
    if (dEdgamma) RBE2D_TRY(h, launch_energy(h, N, nullptr, RBE2D_ALL, gE, dEdgamma, s), "dgamma launch");
    return RBE2D_OK;
}

rbe2d_status rbe2d_md_run(rbe2d_handle h, int64_t N, double *pos, double *vel, const double *q, double *F,
                          double dt, double z_lo, double z_hi, uint64_t seed, int64_t step0,
                          int32_t n_steps, void *stream) {
    if (!h) return fail(nullptr, RBE2D_E_INVAL, "handle is NULL");
    if (N < 0 || N > h->p.n_max) return fail(h, RBE2D_E_INVAL, "N outside [0, n_max]");
    if (N > 0 && (!pos || !vel || !q || !F)) return fail(h, RBE2D_E_INVAL, "NULL array");
    if (!(dt > 0.0) || !(z_lo > 0.0 && z_lo < z_hi && z_hi < h->p.H) || n_steps < 0)
        return fail(h, RBE2D_E_INVAL, "need dt > 0, 0 < z_lo < z_hi < H, n_steps >= 0");
    hipStream_t s = (hipStream_t)stream;
    for (int32_t it = 0; it < n_steps; it++) {
        RBE2D_TRY(h, launch_md_kick_drift(h, N, pos, vel, F, dt, z_lo, z_hi, s), "md drift");
        RBE2D_TRY(h, launch_sample(h, seed, (uint64_t)(step0 + it), s), "md sample");
        h->kset_valid = true;
        rbe2d_status st = run_common(h, N, pos, q, RBE2D_ALL, false, s);
        if (st) return st;
        RBE2D_TRY(h, launch_kforce(h, N, pos, q, F, nullptr, RBE2D_ALL, false, false, true, nullptr, s), "md force");
        RBE2D_TRY(h, launch_md_kick(h, N, vel, F, dt, s), "md kick");
    }
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
