// Real-space half of RBE2D on gfx950 (Eq. (3.12)): a cell list over the
// slab built by counting sort with a deterministic in-cell order, and the
// erfc pair sum over real charges and truncated image charges within r_c.
//
// Images are never materialised: the order-l image of source j is at the
// same distance from target i as the real source j is from a transformed
// target (x_i, y_i, sz z_i + cz) -- a reflection for odd l, a shift for even
// l -- so every image family is a second cell search around the transformed
// target, done only when that point lies within r_c of the slab.
#include "devmath.h"
#include "erfcx_fit.h"
#include "rbe2d_internal.h"

namespace rbe2d {

__global__ void k_fill(uint32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_fill(void *p, int64_t nbytes, hipStream_t s) {
    const int64_t n = nbytes / 4;
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t *)p, n);
    return hipGetLastError();
}

struct CellArgs {
    const double *pos, *q;
    int64_t N;
    double Lx, Ly, hx, hy, hz;
    int ncx, ncy, ncz, ncells;
    int *cell, *slot, *count, *start, *tmp, *sidx;
    double4 *sorted;
};

__device__ __forceinline__ int cell_of(double x, double y, double z, const CellArgs &a, double *xw,
                                       double *yw) {
    double fx = x / a.Lx; fx -= floor(fx);
    double fy = y / a.Ly; fy -= floor(fy);
    *xw = fx * a.Lx;
    *yw = fy * a.Ly;
    int cx = min(a.ncx - 1, max(0, (int)(*xw / a.hx)));
    int cy = min(a.ncy - 1, max(0, (int)(*yw / a.hy)));
    int cz = min(a.ncz - 1, max(0, (int)(z / a.hz)));   // z outside (0,H) is flagged by prep
    return (cx * a.ncy + cy) * a.ncz + cz;
}

__global__ __launch_bounds__(kBlock) void k_cell_assign(CellArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    double xw, yw;
    const int c = cell_of(a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2], a, &xw, &yw);
    a.cell[i] = c;
    a.slot[i] = atomicAdd(&a.count[c], 1);
}

// exclusive scan of count[0..ncells) into start[0..ncells], one block of 1024 threads
__global__ __launch_bounds__(1024) void k_cell_scan(CellArgs a) {
    __shared__ int sh[1024];
    const int n = a.ncells;
    const int per = (n + 1023) / 1024;
    const int b = threadIdx.x * per;
    const int e = min(n, b + per);
    int sum = 0;
    for (int c = b; c < e; c++) sum += a.count[c];
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // Hillis-Steele inclusive scan
        int v = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int run = threadIdx.x ? sh[threadIdx.x - 1] : 0;
    for (int c = b; c < e; c++) {
        a.start[c] = run;
        run += a.count[c];
    }
    if (threadIdx.x == 1023) a.start[n] = sh[1023];
}

__global__ __launch_bounds__(kBlock) void k_cell_scatter(CellArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    a.tmp[a.start[a.cell[i]] + a.slot[i]] = (int)i;
}

// position within the cell = number of members with a smaller original index
__global__ __launch_bounds__(kBlock) void k_cell_rank(CellArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    const int c = a.cell[i];
    const int b = a.start[c], e = a.start[c + 1];
    int r = 0;
    for (int j = b; j < e; j++) r += a.tmp[j] < (int)i;
    double xw, yw;
    cell_of(a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2], a, &xw, &yw);
    a.sorted[b + r] = make_double4(xw, yw, a.pos[3 * i + 2], a.q[i]);
    a.sidx[b + r] = (int)i;
}

struct RealArgs {
    const double4 *sorted;
    const int *sidx, *start;
    const Family *fam;
    int nfam;
    int64_t N;
    double Lx, Ly, H, hx, hy, hz, rc, rc2, alpha, pref;
    int ncx, ncy, ncz;
    double4 *freal;
    double2 *dgreal;
    double *rpart;
};

// erfc(alpha d)/d and the radial force factor [erfc(ad)/d + 2a/sqrt(pi) e^{-a^2 d^2}]/d^2
template <bool FP32>
__device__ __forceinline__ void pair_terms(double r2, double alpha, double *ec, double *fs) {
    if (FP32) {
        const float r2f = (float)r2;
        const float rinv = __builtin_amdgcn_rsqf(r2f);
        const float af = (float)alpha;
        const float x = af * r2f * rinv;
        const float e = __builtin_amdgcn_exp2f(-(af * af * 1.4426950408889634f) * r2f);
        const float t = __builtin_amdgcn_rcpf(fmaf(RBE2D_ERFCX_P, x, 1.0f));
        float p = rbe2d_erfcx_a[RBE2D_ERFCX_DEG - 1];
#pragma unroll
        for (int k = RBE2D_ERFCX_DEG - 2; k >= 0; k--) p = fmaf(p, t, rbe2d_erfcx_a[k]);
        const float erfc_v = e * p * t;
        const float ecf = erfc_v * rinv;
        *ec = (double)ecf;
        *fs = (double)((ecf + (float)(1.1283791670955126 * alpha) * e) * (rinv * rinv));
    } else {
        const double d = sqrt(r2);
        const double e = exp(-alpha * alpha * r2);
        const double v = erfc(alpha * d) / d;
        *ec = v;
        *fs = (v + 1.1283791670955126 * alpha * e) / r2;
    }
}

template <bool FP32, bool WANT_DG>
__global__ __launch_bounds__(kBlock) void k_real(RealArgs a) {
    __shared__ double sh[kBlock / 64];
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double qphi = 0.0, qdt = 0.0, qdb = 0.0;
    if (t < a.N) {
        const double4 me = a.sorted[t];
        const int cx = min(a.ncx - 1, max(0, (int)(me.x / a.hx)));
        const int cy = min(a.ncy - 1, max(0, (int)(me.y / a.hy)));
        const bool allx = a.ncx < 3, ally = a.ncy < 3;
        double fx = 0, fy = 0, fz = 0, phi = 0, dpt = 0, dpb = 0;
        for (int f = 0; f <= a.nfam; f++) {
            double sz = 1.0, czs = 0.0, w = 1.0, zsign = 1.0, dwt = 0.0, dwb = 0.0;
            if (f > 0) {
                const Family fm = a.fam[f - 1];
                sz = fm.sz; czs = fm.cz; w = fm.w; zsign = fm.zsign; dwt = fm.dwt; dwb = fm.dwb;
            }
            const double tz = sz * me.z + czs;
            if (!(tz > -a.rc && tz < a.H + a.rc)) continue;
            const int czlo = max(0, (int)floor((tz - a.rc) / a.hz));
            const int czhi = min(a.ncz - 1, (int)floor((tz + a.rc) / a.hz));
            if (czlo > czhi) continue;
            double gfx = 0, gfy = 0, gfz = 0, gph = 0;
            const int ylo = ally ? 0 : -1, yhi = ally ? a.ncy - 1 : 1;
            const int xlo = allx ? 0 : -1, xhi = allx ? a.ncx - 1 : 1;
            for (int oy = ylo; oy <= yhi; oy++) {
                int cyy = ally ? oy : cy + oy;
                double sy = 0.0;
                if (cyy < 0) { cyy += a.ncy; sy = -a.Ly; }
                else if (cyy >= a.ncy) { cyy -= a.ncy; sy = a.Ly; }
                for (int ox = xlo; ox <= xhi; ox++) {
                    int cxx = allx ? ox : cx + ox;
                    double sx = 0.0;
                    if (cxx < 0) { cxx += a.ncx; sx = -a.Lx; }
                    else if (cxx >= a.ncx) { cxx -= a.ncx; sx = a.Lx; }
                    const int col = (cxx * a.ncy + cyy) * a.ncz;
                    const int jb = a.start[col + czlo], je = a.start[col + czhi + 1];
                    for (int j = jb; j < je; j++) {
                        const double4 s = a.sorted[j];
                        double dx = me.x - s.x - sx;
                        double dy = me.y - s.y - sy;
                        if (allx) dx -= a.Lx * rint(dx / a.Lx);
                        if (ally) dy -= a.Ly * rint(dy / a.Ly);
                        const double dz = tz - s.z;
                        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                        if (r2 < a.rc2 && (f > 0 || j != (int)t)) {
                            double ec, fs;
                            pair_terms<FP32>(r2, a.alpha, &ec, &fs);
                            const double qf = s.w * fs;
                            gfx = fma(qf, dx, gfx);
                            gfy = fma(qf, dy, gfy);
                            gfz = fma(qf, dz, gfz);
                            gph = fma(s.w, ec, gph);
                        }
                    }
                }
            }
            fx = fma(w, gfx, fx);
            fy = fma(w, gfy, fy);
            fz = fma(w * zsign, gfz, fz);
            phi = fma(w, gph, phi);
            if (WANT_DG) { dpt = fma(dwt, gph, dpt); dpb = fma(dwb, gph, dpb); }
        }
        const int i = a.sidx[t];
        const double qi = me.w * a.pref;
        a.freal[i] = make_double4(qi * fx, qi * fy, qi * fz, a.pref * phi);
        qphi = me.w * a.pref * phi;
        if (WANT_DG) {
            a.dgreal[i] = make_double2(a.pref * dpt, a.pref * dpb);
            qdt = me.w * a.pref * dpt;
            qdb = me.w * a.pref * dpb;
        }
    }
    const double s0 = block_sum_r(qphi, sh);
    double s1 = 0.0, s2 = 0.0;
    if (WANT_DG) { s1 = block_sum_r(qdt, sh); s2 = block_sum_r(qdb, sh); }
    if (threadIdx.x == 0) {
        a.rpart[3 * blockIdx.x] = s0;
        a.rpart[3 * blockIdx.x + 1] = s1;
        a.rpart[3 * blockIdx.x + 2] = s2;
    }
}

hipError_t launch_real(rbe2d_ctx *h, int64_t N, const double *pos, const double *q, bool want_dg,
                       hipStream_t s) {
    if (N == 0) return hipSuccess;
    CellArgs c;
    c.pos = pos; c.q = q; c.N = N;
    c.Lx = h->p.Lx; c.Ly = h->p.Ly; c.hx = h->hx; c.hy = h->hy; c.hz = h->hz;
    c.ncx = h->ncx; c.ncy = h->ncy; c.ncz = h->ncz; c.ncells = h->ncells;
    c.cell = h->w.cell; c.slot = h->w.slot; c.count = h->w.count; c.start = h->w.start;
    c.tmp = h->w.tmp; c.sidx = h->w.sidx; c.sorted = h->w.sorted;
    const int nb = (int)((N + kBlock - 1) / kBlock);
    prof_begin(h, 3, s);
    (void)launch_fill(h->w.count, (int64_t)h->ncells * 4, s);
    hipLaunchKernelGGL(k_cell_assign, dim3(nb), dim3(kBlock), 0, s, c);
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, s, c);
    hipLaunchKernelGGL(k_cell_scatter, dim3(nb), dim3(kBlock), 0, s, c);
    hipLaunchKernelGGL(k_cell_rank, dim3(nb), dim3(kBlock), 0, s, c);
    prof_end(h, 3, s);
    RealArgs r;
    r.sorted = h->w.sorted; r.sidx = h->w.sidx; r.start = h->w.start; r.fam = h->w.fam;
    r.nfam = (int)h->fam.size(); r.N = N;
    r.Lx = h->p.Lx; r.Ly = h->p.Ly; r.H = h->p.H; r.hx = h->hx; r.hy = h->hy; r.hz = h->hz;
    r.rc = h->p.r_c; r.rc2 = h->p.r_c * h->p.r_c; r.alpha = h->p.alpha; r.pref = h->pref;
    r.ncx = h->ncx; r.ncy = h->ncy; r.ncz = h->ncz;
    r.freal = h->w.freal; r.dgreal = h->w.dgreal; r.rpart = h->w.rpart;
    const bool fp32 = h->p.precision == RBE2D_PREC_FP32_PHASE;
    prof_begin(h, 4, s);
    if (fp32) {
        if (want_dg) hipLaunchKernelGGL((k_real<true, true>), dim3(nb), dim3(kBlock), 0, s, r);
        else hipLaunchKernelGGL((k_real<true, false>), dim3(nb), dim3(kBlock), 0, s, r);
    } else {
        if (want_dg) hipLaunchKernelGGL((k_real<false, true>), dim3(nb), dim3(kBlock), 0, s, r);
        else hipLaunchKernelGGL((k_real<false, false>), dim3(nb), dim3(kBlock), 0, s, r);
    }
    prof_end(h, 4, s);
    return hipGetLastError();
}

}  // namespace rbe2d
