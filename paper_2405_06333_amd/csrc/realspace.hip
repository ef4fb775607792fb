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
    int *cell, *slot, *count, *start, *tmp, *sidx, *scell;
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
    return (cz * a.ncx + cx) * a.ncy + cy;             // rows along y are contiguous
}

__global__ __launch_bounds__(kBlock) void k_cell_assign(CellArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.N) return;
    double xw, yw;
    const int c = cell_of(a.pos[3 * i], a.pos[3 * i + 1], a.pos[3 * i + 2], a, &xw, &yw);
    a.cell[i] = c;
    a.slot[i] = atomicAdd(&a.count[c], 1);
}

// exclusive scan of count[0..ncells) into start[0..ncells] in three phases:
// per-block totals, a scan of the block totals, per-block scans plus offset.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ int block_exclusive_scan(int v, int *sh, int *total) {
    // Hillis-Steele inclusive scan in shared memory (blockDim.x = kScanBlock)
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kScanBlock; o <<= 1) {
        const int add = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const int incl = sh[threadIdx.x];
    *total = sh[kScanBlock - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_totals(const int *count, int n, int *btot) {
    __shared__ int sh[kScanBlock / 64];
    const int c = blockIdx.x * kScanBlock + threadIdx.x;
    int v = c < n ? count[c] : 0;
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kScanBlock / 64; w++) t += sh[w];
        btot[blockIdx.x] = t;
    }
}

// one block: exclusive scan of the block totals (nb may exceed the block size)
__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(int *btot, int nb) {
    __shared__ int sh[kScanBlock];
    int carry = 0;
    for (int base = 0; base < nb; base += kScanBlock) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? btot[i] : 0;
        int tot;
        const int ex = block_exclusive_scan(v, sh, &tot);
        if (i < nb) btot[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const int *count, int n, const int *btot,
                                                           int *start) {
    __shared__ int sh[kScanBlock];
    const int c = blockIdx.x * kScanBlock + threadIdx.x;
    const int v = c < n ? count[c] : 0;
    int tot;
    const int ex = block_exclusive_scan(v, sh, &tot);
    if (c < n) start[c] = btot[blockIdx.x] + ex;
    if (c == n - 1) start[n] = btot[blockIdx.x] + ex + v;
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
    // x relative to the cell's lower x edge (a row along y shares it), y wrapped, z as given
    const int cx = (c / a.ncy) % a.ncx;
    const double xr = xw - cx * a.hx;
    a.sorted[b + r] = make_double4(xr, yw, a.pos[3 * i + 2], a.q[i]);
    a.sidx[b + r] = (int)i;
    a.scell[b + r] = c;
}

struct RealArgs {
    const void *src;            // sorted sources: (x - x0(cell), y, z, q) as double4
    const int *sidx, *scell, *start;
    const Family *fam;
    int nfam;
    int64_t N;
    double Lx, Ly, H, hx, hy, hz, inv_hy, inv_hz, rc, rc2, alpha, pref;
    int ncx, ncy, ncz, reach;   // reach: neighbour columns on each side (cells are >= r_c / reach)
    int nblocks;                // logical blocks (the grid is rounded up to a multiple of 8)
    int round_min;              // keep draining the pair queues while this many lanes hold work
    double4 *freal;
    double2 *dgreal;
    double *rpart;
};

template <bool FP32> struct RealTypes;
template <> struct RealTypes<true> { using T = float; using V4 = float4; static constexpr int Q = 8; };
template <> struct RealTypes<false> { using T = double; using V4 = double4; static constexpr int Q = 4; };
// (Q must be a power of two: the queues are rings)

// erfc(alpha d)/d (ec) and the radial force factor fs = [erfc(a d)/d + 2a/sqrt(pi) e^{-a^2 d^2}]/d^2
__device__ __forceinline__ void pair_terms(float r2, float alpha, float c2a, float *ec, float *fs) {
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float x = alpha * r2 * rinv;
    const float e = __builtin_amdgcn_exp2f(-(alpha * alpha * 1.4426950408889634f) * r2);
    const float t = __builtin_amdgcn_rcpf(fmaf(RBE2D_ERFCX_P, x, 1.0f));
    float p = rbe2d_erfcx_a[RBE2D_ERFCX_DEG - 1];
#pragma unroll
    for (int k = RBE2D_ERFCX_DEG - 2; k >= 0; k--) p = fmaf(p, t, rbe2d_erfcx_a[k]);
    const float v = e * p * t * rinv;
    *ec = v;
    *fs = fmaf(c2a, e, v) * (rinv * rinv);
}
__device__ __forceinline__ void pair_terms(double r2, double alpha, double c2a, double *ec, double *fs) {
    const double d = sqrt(r2);
    const double e = exp(-alpha * alpha * r2);
    const double v = erfc(alpha * d) / d;
    *ec = v;
    *fs = fma(c2a, e, v) / r2;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// One thread per target, targets in cell order (z-layer slowest, then x,
// then y), so the lanes of a wave share a z-layer and see neighbour rows of
// similar length.  For each image family, each z-layer within r_c and each
// x-column, the sources lie in one contiguous run of cells along y (two
// runs where the range wraps around the periodic y boundary), culled to the
// y-extent the sphere of radius r_c allows in that layer and column.  Pairs
// within r_c go to a per-lane queue in LDS; the queue is drained (erfc/exp)
// whenever some lane's queue is full, with all lanes taking part, so the
// transcendental work is spent on accepted pairs only.  Pair geometry is
// FP64 in both variants (the closest pairs dominate the force); the FP32
// variant evaluates erfc/exp and the per-drain partial sums in FP32 and
// accumulates the drains in FP64.
template <bool FP32, bool WANT_DG>
__global__ __launch_bounds__(kBlock) void k_real(RealArgs a) {
    using T = typename RealTypes<FP32>::T;
    using V4 = typename RealTypes<FP32>::V4;
    constexpr int Q = RealTypes<FP32>::Q;
    __shared__ V4 queue[Q][kBlock];
    __shared__ double sh[kBlock / 64];
    const double4 *src = (const double4 *)a.src;
    const int tid = threadIdx.x;
    // Blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous
    // range of targets, so neighbouring cells share that XCD's L2.
    const int per_xcd = (int)(gridDim.x >> 3);
    const int lb = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (lb >= a.nblocks) return;
    const int64_t t = (int64_t)lb * kBlock + tid;
    const bool active = t < a.N;
    double4 me = make_double4(0.0, 0.0, 0.0, 0.0);
    int cid = 0;
    if (active) { me = src[t]; cid = a.scell[t]; }
    const int cy = cid % a.ncy;
    const int cx = (cid / a.ncy) % a.ncx;
    const bool allx = a.ncx < 2 * a.reach + 1, ally = a.ncy < 2 * a.reach + 1;
    const double yrel = me.y - cy * a.hy;           // y within the target's cell
    const double rcm2 = a.rc2 * (1.0 + 2e-9);       // culling bounds get a 1e-9 margin:
    const double rmarg = 1e-9 * a.rc;               // cells were assigned by division
    const T alpha = (T)a.alpha;
    const T c2a = (T)(1.1283791670955126 * a.alpha);
    double fx = 0, fy = 0, fz = 0, phi = 0, dpt = 0, dpb = 0;
    for (int f = 0; f <= a.nfam; f++) {
        double sz = 1.0, czs = 0.0, w = 1.0, zsign = 1.0, dwt = 0.0, dwb = 0.0;
        if (f > 0) {
            const Family fm = a.fam[f - 1];
            sz = fm.sz; czs = fm.cz; w = fm.w; zsign = fm.zsign; dwt = fm.dwt; dwb = fm.dwb;
        }
        const double tz = sz * me.z + czs;
        const bool fam_on = active && tz > -a.rc && tz < a.H + a.rc;
        if (__ballot(fam_on) == 0) continue;
        int lzlo = a.ncz, lzhi = -1;
        if (fam_on) {
            lzlo = max(0, (int)floor((tz - a.rc - rmarg) * a.inv_hz));
            lzhi = min(a.ncz - 1, (int)floor((tz + a.rc + rmarg) * a.inv_hz));
        }
        const int wzlo = wave_min(lzlo), wzhi = wave_max(lzhi);
        double gfx = 0, gfy = 0, gfz = 0, gph = 0;
        T sx = 0, sy = 0, szz = 0, sp = 0;   // FP32 partial sums within one drain
        int head = 0, cnt = 0;               // per-lane ring buffer of accepted pairs in LDS
        // one round: every lane with a queued pair evaluates its oldest one
        auto round = [&]() {
            if (cnt > 0) {
                const V4 e = queue[head][tid];
                head = (head + 1) & (Q - 1);
                cnt--;
                const T r2 = e.x * e.x + e.y * e.y + e.z * e.z;
                T ec, fs;
                pair_terms(r2, alpha, c2a, &ec, &fs);
                const T qf = e.w * fs;
                sx += qf * e.x;
                sy += qf * e.y;
                szz += qf * e.z;
                sp += e.w * ec;
            }
        };
        auto fold = [&]() {
            gfx += (double)sx; gfy += (double)sy; gfz += (double)szz; gph += (double)sp;
            sx = sy = szz = sp = 0;
        };
        // when some lane's ring is full: rounds while enough lanes still hold work
        // (a lane evaluates at most Q pairs per drain before the FP64 fold)
        auto drain = [&]() {
            do {
                round();
            } while (__popcll(__ballot(cnt > 0)) >= a.round_min);
            fold();
        };
        // scan one run of sources p[0..len) for pairs within r_c; the trip
        // count is the wave maximum, so drains always run with every lane
        auto scan = [&](const double4 *p, int len, double xt, double yt, int self) {
            const int maxlen = wave_max(len);
            for (int m = 0; m < maxlen; m++) {
                if (m < len) {
                    const double4 s = p[m];
                    double dx = xt - s.x;
                    double dy = yt - s.y;
                    if (allx) dx -= a.Lx * rint(dx / a.Lx);
                    if (ally) dy -= a.Ly * rint(dy / a.Ly);
                    const double dz = tz - s.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    if (r2 < a.rc2 && m != self) {
                        V4 e;
                        e.x = (T)dx; e.y = (T)dy; e.z = (T)dz; e.w = (T)s.w;
                        queue[(head + cnt) & (Q - 1)][tid] = e;
                        cnt++;
                    }
                }
                if (__ballot(cnt == Q) != 0) drain();
            }
        };
        const int xlo = allx ? 0 : -a.reach, xhi = allx ? a.ncx - 1 : a.reach;
        for (int lz = wzlo; lz <= wzhi; lz++) {
            const bool lay_on = lz >= lzlo && lz <= lzhi;
            const double dzmin = fmax(0.0, fmax(lz * a.hz - tz, tz - (lz + 1) * a.hz));
            for (int ox = xlo; ox <= xhi; ox++) {
                const int dxc = allx ? ox - cx : ox;       // column offset in cells
                int cxx = allx ? ox : cx + ox;
                if (!allx) cxx += cxx < 0 ? a.ncx : (cxx >= a.ncx ? -a.ncx : 0);
                double dxmin = 0;
                if (!allx) dxmin = dxc > 0 ? dxc * a.hx - me.x : (dxc < 0 ? me.x - (dxc + 1) * a.hx : 0.0);
                const double xt = me.x - dxc * a.hx;
                const double ye2 = rcm2 - dxmin * dxmin - dzmin * dzmin;
                // up to two runs of cells along y: [ya, yb] unshifted, the wrapped one shifted by sy2
                int jb1 = 0, len1 = 0, jb2 = 0, len2 = 0;
                double sy2 = 0.0;
                if (lay_on && ye2 > 0.0) {
                    const int row = (lz * a.ncx + cxx) * a.ncy;
                    if (ally) {
                        jb1 = a.start[row];
                        len1 = a.start[row + a.ncy] - jb1;
                    } else {
                        const double ye = sqrt(ye2) + rmarg;
                        int cylo = cy + (int)floor((yrel - ye) * a.inv_hy);
                        int cyhi = cy + (int)floor((yrel + ye) * a.inv_hy);
                        cylo = max(cylo, cy - a.reach);
                        cyhi = min(cyhi, cy + a.reach);
                        const int ya = max(cylo, 0), yb = min(cyhi, a.ncy - 1);
                        if (ya <= yb) { jb1 = a.start[row + ya]; len1 = a.start[row + yb + 1] - jb1; }
                        if (cylo < 0) {
                            jb2 = a.start[row + cylo + a.ncy];
                            len2 = a.start[row + a.ncy] - jb2;
                            sy2 = -a.Ly;
                        } else if (cyhi >= a.ncy) {
                            jb2 = a.start[row];
                            len2 = a.start[row + cyhi - a.ncy + 1] - jb2;
                            sy2 = a.Ly;
                        }
                    }
                }
                // the target itself is excluded from the direct family only
                const int self1 = f == 0 ? (int)(t - jb1) : -1;
                const int self2 = f == 0 ? (int)(t - jb2) : -1;
                scan(src + jb1, len1, xt, me.y, self1);
                if (__ballot(len2 > 0) != 0) scan(src + jb2, len2, xt, me.y - sy2, self2);
            }
        }
        while (__ballot(cnt > 0) != 0) round();
        fold();
        fx = fma(w, gfx, fx);
        fy = fma(w, gfy, fy);
        fz = fma(w * zsign, gfz, fz);
        phi = fma(w, gph, phi);
        if (WANT_DG) { dpt = fma(dwt, gph, dpt); dpb = fma(dwb, gph, dpb); }
    }
    double qphi = 0.0, qdt = 0.0, qdb = 0.0;
    if (active) {
        const int i = a.sidx[t];
        const double qi = me.w * a.pref;
        a.freal[i] = make_double4(qi * fx, qi * fy, qi * fz, a.pref * phi);
        qphi = qi * phi;
        if (WANT_DG) {
            a.dgreal[i] = make_double2(a.pref * dpt, a.pref * dpb);
            qdt = qi * dpt;
            qdb = qi * dpb;
        }
    }
    const double s0 = block_sum_r(qphi, sh);
    double s1 = 0.0, s2 = 0.0;
    if (WANT_DG) { s1 = block_sum_r(qdt, sh); s2 = block_sum_r(qdb, sh); }
    if (threadIdx.x == 0) {
        a.rpart[3 * lb] = s0;
        a.rpart[3 * lb + 1] = s1;
        a.rpart[3 * lb + 2] = s2;
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
    const bool fp32 = h->p.precision == RBE2D_PREC_FP32_PHASE;
    c.tmp = h->w.tmp; c.sidx = h->w.sidx; c.scell = h->w.scell; c.sorted = h->w.sorted;
    const int nb = (int)((N + kBlock - 1) / kBlock);
    prof_begin(h, 3, s);
    (void)launch_fill(h->w.count, (int64_t)h->ncells * 4, s);
    hipLaunchKernelGGL(k_cell_assign, dim3(nb), dim3(kBlock), 0, s, c);
    const int nsb = (h->ncells + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_totals, dim3(nsb), dim3(kScanBlock), 0, s, h->w.count, h->ncells, h->w.scanbuf);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, s, h->w.scanbuf, nsb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nsb), dim3(kScanBlock), 0, s, h->w.count, h->ncells, h->w.scanbuf,
                       h->w.start);
    hipLaunchKernelGGL(k_cell_scatter, dim3(nb), dim3(kBlock), 0, s, c);
    hipLaunchKernelGGL(k_cell_rank, dim3(nb), dim3(kBlock), 0, s, c);
    prof_end(h, 3, s);
    RealArgs r;
    r.src = h->w.sorted; r.sidx = h->w.sidx; r.scell = h->w.scell; r.start = h->w.start; r.fam = h->w.fam;
    r.nfam = (int)h->fam.size(); r.N = N;
    r.Lx = h->p.Lx; r.Ly = h->p.Ly; r.H = h->p.H; r.hx = h->hx; r.hy = h->hy; r.hz = h->hz;
    r.rc = h->p.r_c; r.rc2 = h->p.r_c * h->p.r_c; r.alpha = h->p.alpha; r.pref = h->pref;
    r.inv_hy = 1.0 / h->hy; r.inv_hz = 1.0 / h->hz; r.nblocks = nb; r.round_min = h->round_min;
    const int nb8 = (nb + 7) / 8 * 8;
    r.ncx = h->ncx; r.ncy = h->ncy; r.ncz = h->ncz; r.reach = h->reach;
    r.freal = h->w.freal; r.dgreal = h->w.dgreal; r.rpart = h->w.rpart;
    prof_begin(h, 4, s);
    if (fp32) {
        if (want_dg) hipLaunchKernelGGL((k_real<true, true>), dim3(nb8), dim3(kBlock), 0, s, r);
        else hipLaunchKernelGGL((k_real<true, false>), dim3(nb8), dim3(kBlock), 0, s, r);
    } else {
        if (want_dg) hipLaunchKernelGGL((k_real<false, true>), dim3(nb8), dim3(kBlock), 0, s, r);
        else hipLaunchKernelGGL((k_real<false, false>), dim3(nb8), dim3(kBlock), 0, s, r);
    }
    prof_end(h, 4, s);
    return hipGetLastError();
}

}  // namespace rbe2d
