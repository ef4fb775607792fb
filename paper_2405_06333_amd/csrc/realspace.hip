// Real-space half of RBE2D on gfx950 (Eq. (3.12)): a cell list over each
// slab built by counting sort with a deterministic in-cell order, and the
// erfc pair sum over real charges and truncated image charges within r_c.
// All systems of a handle share one sort (their cells are numbered
// consecutively) and one launch of the pair kernel.
//
// Images are never materialised: the order-l image of source j is at the
// same distance from target i as the real source j is from a transformed
// target (x_i, y_i, sz z_i + cz) -- a reflection for odd l, a shift for even
// l -- so every image family is another cell search around the transformed
// target, done only when that point lies within r_c of the slab.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "devmath.h"
#include "erfcx_fit.h"
#include "rbe2d_internal.h"

// Compile-time parameters of the FP32 pair kernel (measured best on the
// 1e6-ion slab: 16-entry rings halve the occupancy, batches of 2 loads leave
// latency exposed, the drain threshold hardly matters).  Register cap: the
// double-buffered scan of paired columns fits 4 waves per SIMD without
// spills (122 VGPRs); at 5 waves it spills and is 5 % slower, uncapped at 3
// waves slower still.  The FP64 variant is capped at 4 waves per SIMD too
// (no spills; 4.5 % faster alone than at its uncapped 3).
#ifndef RBE2D_REAL_U32
#define RBE2D_REAL_U32 4      // source loads per batch (two batches in flight per lane)
#endif
#ifndef RBE2D_RING_Q
#define RBE2D_RING_Q 8        // ring entries per lane (a power of two)
#endif
#ifndef RBE2D_ROUND_MIN
#define RBE2D_ROUND_MIN 40    // keep draining while this many lanes hold pairs
#endif
#ifndef RBE2D_REAL_CHUNKS
#define RBE2D_REAL_CHUNKS 8   // contiguous target chunks per XCD
#endif
#ifndef RBE2D_REAL_WAVES32
#define RBE2D_REAL_WAVES32 4  // FP32 pair kernel: waves per SIMD its register budget must allow
#endif

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
    const SysDesc *sys;
    Layout lay;
    int n_sys, n_total, ncells;
    int *cell, *slot, *count, *start, *sidx, *scell;
    int2 *tmp;      // unordered cell lists: (caller index, global cell)
    int n_waves;    // padded sorted positions / 64 (the rank pass runs one wave per system chunk)
    // set when the MD pass that moved the particles (and counted them) also
    // wrote their k-space records on this stream: the rank pass reads those
    // (one aligned record per particle) instead of positions and charges
    const float4 *p32;
    const double4 *p64;
    double4 *sorted;
    uint4 *src16;   // written when set (FP32 pair kernel)
};

// position -> 32-bit fixed point; the wrap of 2^32 is the period (x, y)
__device__ __forceinline__ uint32_t to_fixed(double v, double scale) {
    return (uint32_t)(unsigned long long)llrint(v * scale);
}

__global__ __launch_bounds__(kBlock) void k_cell_count(CellArgs a) {
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= a.n_total) return;
    const int r = find_sys(a.lay.off, a.n_sys, g);
    const SysDesc &d = a.sys[r];
    double xw, yw;
    const int c = d.cbase + cell_of(a.pos[3 * (int64_t)g], a.pos[3 * (int64_t)g + 1], a.pos[3 * (int64_t)g + 2], d,
                                    &xw, &yw);
    a.cell[g] = c;
    a.slot[g] = atomicAdd(&a.count[c], 1);
}

// exclusive scan of count[0..ncells) into start[0..ncells] in two launches:
// per-block totals of 4096 cells, then each block adds the totals before it
// (at most a few hundred) to the scan of its own cells.  The second launch
// also clears the counts for the next build.  Integer sums: the order does
// not matter.
constexpr int kScanPer = 16;                      // cells per thread
constexpr int kScanCells = kBlock * kScanPer;     // cells per scan block

__device__ __forceinline__ void load_counts(const int *count, int n, int c0, int (&v)[kScanPer]) {
    if (c0 + kScanPer <= n && (c0 & 3) == 0) {
        const int4 *p = reinterpret_cast<const int4 *>(count + c0);
#pragma unroll
        for (int k = 0; k < kScanPer / 4; k++) {
            const int4 w = p[k];
            v[4 * k] = w.x; v[4 * k + 1] = w.y; v[4 * k + 2] = w.z; v[4 * k + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanPer; k++) v[k] = c0 + k < n ? count[c0 + k] : 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_totals(const int *count, int n, int *btot) {
    __shared__ int sh[kBlock / 64];
    int v[kScanPer];
    load_counts(count, n, blockIdx.x * kScanCells + threadIdx.x * kScanPer, v);
    int t = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; k++) t += v[k];
    t = wave_sum(t);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        int b = 0;
        for (int w = 0; w < kBlock / 64; w++) b += sh[w];
        btot[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(int *count, int n, const int *btot, int *start) {
    __shared__ int sh_wave[kBlock / 64];
    __shared__ int sh_base;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (wid == 0) {
        // cells before this block: the totals of the blocks before it
        int b = 0;
        for (int k = lane; k < (int)blockIdx.x; k += 64) b += btot[k];
        b = wave_sum(b);
        if (lane == 0) sh_base = b;
    }
    const int c0 = blockIdx.x * kScanCells + threadIdx.x * kScanPer;
    int v[kScanPer];
    load_counts(count, n, c0, v);
    int t = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; k++) t += v[k];
    // inclusive scan of the thread totals over the wave, then over the waves
    int incl = t;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) sh_wave[wid] = incl;
    __syncthreads();
    int before = sh_base;
    for (int w = 0; w < wid; w++) before += sh_wave[w];
    int run = before + incl - t;
#pragma unroll
    for (int k = 0; k < kScanPer; k++) {
        const int c = c0 + k;
        if (c < n) {
            start[c] = run;
            count[c] = 0;       // the next build counts from zero
        }
        run += v[k];
        if (c == n - 1) start[n] = run;
    }
}

__global__ __launch_bounds__(kBlock) void k_cell_scatter(CellArgs a) {
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= a.n_total) return;
    const int c = a.cell[g];
    a.tmp[a.start[c] + a.slot[g]] = make_int2(g, c);
}

// position within the cell = number of members with a smaller caller index;
// sorted positions are padded per system to whole waves.  One thread per
// padded sorted position, so a wave belongs to one system (its constants
// are scalar loads); the thread takes slot j of the unordered cell lists
// (tmp), gathers the particle it holds and writes its record within the
// same cell, so the stores of a wave stay within a few neighbouring cells.
__global__ __launch_bounds__(kBlock) void k_cell_rank(CellArgs a) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= a.n_waves * kWave) return;
    const int r = __builtin_amdgcn_readfirstlane(find_sys(a.lay.sbase, a.n_sys, t & ~(kWave - 1)));
    const SysDesc d = a.sys[r];   // a copy: wave-uniform values in scalar registers
    const int j = t - a.lay.sbase[r] + a.lay.off[r];   // position in the unpadded cell lists
    if (j >= a.lay.off[r + 1]) return;                   // padding of this system
    const int2 gc = a.tmp[j];
    const int g = gc.x, c = gc.y;
    const int b = a.start[c], e = a.start[c + 1];
    int rank = 0;
    for (int k = b; k < e; k++) rank += a.tmp[k].x < g;
    const int s = b + rank + (a.lay.sbase[r] - a.lay.off[r]);
    double xw, yw, z, qg;
    int cl;
    if (a.p32 || a.p64) {
        // the particle's k-space record: fractional x, y (wrapped) and z / L_z,
        // split hi + lo in FP32 (46 significant bits) or exact in FP64, and q
        // (FP32 in the FP32 records, as the FP32 pair kernel uses it)
        const int64_t ii = (int64_t)a.lay.pbase[r] + (g - a.lay.off[r]);
        double fx, fy, fz;
        if (a.p32) {
            const float4 u = a.p32[2 * ii], v = a.p32[2 * ii + 1];
            fx = (double)u.x + (double)u.y; fy = (double)u.z + (double)u.w; fz = (double)v.x + (double)v.y;
            qg = (double)v.z;
        } else {
            const double4 u = a.p64[ii];
            fx = u.x; fy = u.y; fz = u.z; qg = u.w;
        }
        xw = fx * d.Lx; yw = fy * d.Ly; z = fz * d.Lz;
        cl = c - d.cbase;   // the cell it was counted in
    } else {
        cl = cell_of(a.pos[3 * (int64_t)g], a.pos[3 * (int64_t)g + 1], a.pos[3 * (int64_t)g + 2], d, &xw, &yw);
        z = a.pos[3 * (int64_t)g + 2];
        qg = a.q[g];
    }
    // x relative to the cell's lower x edge (a row along y shares it), y wrapped, z as given
    const int cx = (cl / d.ncy) % d.ncx;
    a.sorted[s] = make_double4(xw - cx * d.hx, yw, z, qg);
    a.sidx[s] = g;
    a.scell[s] = cl;
    if (a.src16) {
        // z clamped into the frame (z outside (0, H) is flagged by prep)
        const double zc = fmin(fmax(z, -d.rc), d.H + d.rc);
        a.src16[s] = make_uint4(to_fixed(xw, d.fxs), to_fixed(yw, d.fys), to_fixed(zc + d.zoff, d.fzs),
                                __float_as_uint((float)qg));
    }
}

struct RealArgs {
    const double4 *src;         // sorted sources: (x - x0(cell), y, z, q)
    const uint4 *src16;         // the same in fixed point (FP32 kernel)
    const int *sidx, *scell, *start;
    const SysDesc *sys;
    const Family *fam;          // kMaxFamilies per system
    Layout lay;
    int n_sys, n_waves;         // n_waves: padded real-space waves of all systems
    int nblocks;                // logical blocks (the grid is rounded up to 8 * RBE2D_REAL_CHUNKS chunks)
    double4 *freal;
    double2 *dgreal;
    double *rpart;              // per wave
    int nsplit;                 // > 1: block row y handles x-columns y, y + nsplit, ... of every target
    int64_t split_stride;       // targets per split in the partial outputs
    int rsplit_stride;          // waves per split in the partial wave sums
    double4 *freal_s;
    double2 *dgreal_s;
    double *rpart_s;
};

template <bool FP32> struct RealTypes;
// U: source loads in flight per lane
template <> struct RealTypes<true> { using T = float; using V4 = float4; static constexpr int U = RBE2D_REAL_U32; };
template <> struct RealTypes<false> { using T = double; using V4 = double4; static constexpr int U = 2; };

// Wave-uniform values computed by vector instructions, moved to scalar
// registers (the compiler keeps them in vector registers otherwise).
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
    const int2 h = make_int2(__builtin_amdgcn_readfirstlane(__double2loint(v)),
                             __builtin_amdgcn_readfirstlane(__double2hiint(v)));
    return __hiloint2double(h.y, h.x);
}

// Constants of the FP32 pair terms in the units of the displacements: with
// displacements in units u (r = u rq), ec and fs below come out as u erfc(a r)/r
// and u^3 [erfc(a r)/r + 2a/sqrt(pi) e^{-a^2 r^2}]/r^2; the sums are rescaled
// by 1/u and 1/u^2 when they are folded into FP64.
struct PairConst32 {
    float ce;    // -a^2 u^2 log2(e): exp(-a^2 r^2) = 2^(ce rq^2)
    float cpx;   // p a u: the fit's argument p a r = cpx rq
    float c2a;   // 2a/sqrt(pi) u
    double fscale, pscale;   // 1/u^2 (forces), 1/u (potential)
    __device__ PairConst32(double alpha, double u)
        : ce(uniform((float)(-alpha * alpha * u * u * 1.4426950408889634))),
          cpx(uniform((float)(RBE2D_ERFCX_P * alpha * u))), c2a(uniform((float)(1.1283791670955126 * alpha * u))),
          fscale(uniform(1.0 / (u * u))), pscale(uniform(1.0 / u)) {}
};

// erfc(a r)/r (ec) and the radial force factor fs = [erfc(a r)/r + 2a/sqrt(pi)
// e^{-a^2 r^2}]/r^2 from rq^2, both in the units of PairConst32; erfc(x) =
// e^{-x^2} t P7(t), t = 1/(1 + p x), the fitted erfcx.
__device__ __forceinline__ void pair_terms(float r2, const PairConst32 &c, float *ec, float *fs) {
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float e = __builtin_amdgcn_exp2f(c.ce * r2);
    const float t = __builtin_amdgcn_rcpf(fmaf(c.cpx, r2 * rinv, 1.0f));
    float p = rbe2d_erfcx_a[RBE2D_ERFCX_DEG - 1];
#pragma unroll
    for (int k = RBE2D_ERFCX_DEG - 2; k >= 0; k--) p = fmaf(p, t, rbe2d_erfcx_a[k]);
    const float v = e * p * t * rinv;
    *ec = v;
    *fs = fmaf(c.c2a, e, v) * (rinv * rinv);
}
// FP64: erfc(x) = exp(-x^2) erfcx(x) with the fitted erfcx (relative error
// below 2e-11), sharing the exponential of the force term; for x beyond the
// fitted range erfc(x) < 1.2e-29 and the term is dropped.  1/sqrt(r^2) and
// 1/(1 + p x) are the hardware estimates refined by two Newton steps each
// (relative error near 1e-16; r^2 > 0 for every accepted pair).
// The coefficients are read from LDS (`coef`, a copy of rbe2d_erfcx64_a): as
// FP64 literals they would hold 24 registers for the whole kernel.
__device__ __forceinline__ void pair_terms(double r2, double alpha, double c2a, double *ec, double *fs,
                                           const double *coef) {
    double y = __builtin_amdgcn_rsq(r2);
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const double en = fma(-r2 * y, y, 1.0);     // 1 - r^2 y^2
        y = fma(0.5 * y, en, y);
    }
    const double d = r2 * y;
    const double rinv2 = y * y;
    const double e = exp(-alpha * alpha * r2);
    const double x = alpha * d;
    const double a1 = fma(RBE2D_ERFCX64_P, x, 1.0);
    double t = __builtin_amdgcn_rcp(a1);
#pragma unroll
    for (int it = 0; it < 2; it++) t = fma(t, fma(-a1, t, 1.0), t);
    double p = coef[RBE2D_ERFCX64_DEG - 1];
#pragma unroll
    for (int k = RBE2D_ERFCX64_DEG - 2; k >= 0; k--) p = fma(p, t, coef[k]);
    const double v = x < RBE2D_ERFCX_XMAX ? e * (p * t) * (d * rinv2) : 0.0;
    *ec = v;
    *fs = fma(c2a, e, v) * rinv2;
}

// ---------------------------------------------------------------------------
// Queues of accepted pairs.  The scan appends pairs (displacement from the
// source to the target, source charge); evaluating erfc/exp for them is
// deferred so that it runs with as many lanes busy as possible.  Both give
// the sums of the queued pairs' force and potential terms in FP64.
// ---------------------------------------------------------------------------

// Per-target FP64 sums over all image families.  Each drain's sums are
// added with the current family's weights: w for x, y and the potential,
// w * zsign for z (the image height moves against the target's for odd
// orders), dw / dgamma for the gamma derivatives of the potential; `scale`
// converts force sums kept in other units.
template <bool DG>
struct TargetSums {
    double fx = 0, fy = 0, fz = 0, phi = 0, dpt = 0, dpb = 0;
    double wxy = 1, wz = 1, wp = 1, wt = 0, wb = 0;
    // fscale, pscale: unit conversions of the force and potential sums
    __device__ void family(double w, double zsign, double dwt, double dwb, double fscale, double pscale) {
        wxy = uniform(w * fscale); wz = uniform(w * zsign * fscale); wp = uniform(w * pscale);
        if (DG) { wt = uniform(dwt * pscale); wb = uniform(dwb * pscale); }
    }
    __device__ void add(double sx, double sy, double sz, double sp) {
        fx = fma(sx, wxy, fx); fy = fma(sy, wxy, fy); fz = fma(sz, wz, fz); phi = fma(sp, wp, phi);
        if (DG) { dpt = fma(sp, wt, dpt); dpb = fma(sp, wb, dpb); }
    }
};

// popcount of a wave mask as two 32-bit halves (scalar instructions only)
__device__ __forceinline__ int busy_lanes(uint64_t m) {
    return __builtin_popcount((uint32_t)m) + __builtin_popcount((uint32_t)(m >> 32));
}

// FP32 kernel: a ring of Q entries per lane.  A round evaluates the oldest
// entry of every lane that holds one; the FP32 sums of a drain (at most Q
// pairs per lane) are folded into FP64.  Cheap routing (every result stays in
// its lane) at the price of idle lanes in the rounds.  The lane's read and
// write positions are byte counters into the slot-major rings (one 16-byte
// entry per thread and slot), masked only to form an address; their
// difference is the fill.  ISO: entries hold displacements in units of the
// isotropic fixed-point frame and the pair terms are evaluated in those units.
template <int Q, int U, bool ISO, bool DG>
struct LaneRings : TargetSums<DG> {
    static constexpr int kRoundMin = RBE2D_ROUND_MIN;   // keep draining while this many lanes hold pairs
    static constexpr uint32_t kSlot = kBlock * (uint32_t)sizeof(float4);
    static constexpr uint32_t kMask = Q * kSlot - 1;    // Q * kSlot is a power of two
    static constexpr uint32_t kRoom = (Q - U) * kSlot;  // fill beyond which U more pushes may not fit
    unsigned char *base;
    uint32_t wpos, rpos;   // unsigned: the counters may wrap, their difference stays exact
    PairConst32 pc;
    float sx = 0, sy = 0, sz = 0, sp = 0;
    __device__ LaneRings(unsigned char *b, int t, const SysDesc &d)
        : base(b), wpos((uint32_t)t * (uint32_t)sizeof(float4)), rpos(wpos), pc(d.alpha, ISO ? d.ud : 1.0) {}
    __device__ void family(double w, double zsign, double dwt, double dwb) {
        TargetSums<DG>::family(w, zsign, dwt, dwb, pc.fscale, pc.pscale);
    }
    __device__ void push(bool acc, float dx, float dy, float dz, float qs) {
        if (acc) {
            const uint32_t at = wpos & kMask;
            wpos += kSlot;
            *reinterpret_cast<float4 *>(base + at) = make_float4(dx, dy, dz, qs);
        }
    }
    __device__ bool full() const { return __ballot(wpos - rpos > kRoom) != 0; }
    // one round: evaluate the oldest entry of every lane with fill f > 0
    __device__ void round(uint32_t f) {
        if (f != 0) {
            const float4 e = *reinterpret_cast<const float4 *>(base + (rpos & kMask));
            rpos += kSlot;
            const float r2 = e.x * e.x + e.y * e.y + e.z * e.z;
            float ec, fs;
            pair_terms(r2, pc, &ec, &fs);
            const float qf = e.w * fs;
            sx += qf * e.x; sy += qf * e.y; sz += qf * e.z; sp += e.w * ec;
        }
    }
    __device__ void fold() {
        this->add((double)sx, (double)sy, (double)sz, (double)sp);
        sx = sy = sz = sp = 0;
    }
    // make room for U more pairs per lane: rounds while a lane could
    // overflow or while enough lanes hold pairs
    __device__ void drain() {
        uint32_t f = wpos - rpos;
        do {
            round(f);
            f = wpos - rpos;
        } while (__ballot(f > kRoom) != 0 || busy_lanes(__ballot(f != 0)) >= kRoundMin);
        fold();
    }
    __device__ void flush() {
        uint32_t f = wpos - rpos;
        while (__ballot(f != 0) != 0) {
            round(f);
            f = wpos - rpos;
        }
        fold();
    }
};

// FP64 kernel: one queue shared by the wave (compacted with a ballot prefix,
// entries tagged with the target's lane), evaluated 64 entries at a time with
// every lane busy; results go to per-target LDS accumulators by LDS atomic
// adds.  Worth its routing cost where a pair evaluation is expensive.
template <int QW, int U, bool DG>
struct WaveQueue : TargetSums<DG> {
    double4 *ent;         // [QW] entries of this wave
    unsigned char *own;   // [QW] owning lane
    double *acc;          // [4][64] per-target sums
    const double *coef;   // erfcx fit coefficients (LDS)
    double alpha, c2a;    // a and 2a/sqrt(pi)
    int lane, qn = 0;     // qn: entries queued (wave-uniform)
    __device__ WaveQueue(double4 *e, unsigned char *o, double *a, const double *c, double al, int l)
        : ent(e), own(o), acc(a), coef(c), alpha(al), c2a(1.1283791670955126 * al), lane(l) {
        for (int c = 0; c < 4; c++) acc[c * kWave + lane] = 0.0;
    }
    __device__ void family(double w, double zsign, double dwt, double dwb) {
        TargetSums<DG>::family(w, zsign, dwt, dwb, 1.0, 1.0);
    }
    __device__ void push(bool ok, double dx, double dy, double dz, double qs) {
        const uint64_t m = __ballot(ok);
        if (ok) {
            const int slot = qn + __popcll(m & ((1ull << lane) - 1ull));
            ent[slot] = make_double4(dx, dy, dz, qs);
            own[slot] = (unsigned char)lane;
        }
        qn += __popcll(m);
    }
    __device__ bool full() const { return qn > QW - U * kWave; }
    // evaluate the top n <= 64 entries, one per lane
    __device__ void round(int n) {
        __builtin_amdgcn_wave_barrier();   // entries were written by other lanes of the wave
        const int base = qn - n;
        if (lane < n) {
            const double4 e = ent[base + lane];
            const int o = own[base + lane];
            const double r2 = e.x * e.x + e.y * e.y + e.z * e.z;
            double ec, fs;
            pair_terms(r2, alpha, c2a, &ec, &fs, coef);
            const double qf = e.w * fs;
            atomicAdd(&acc[o], qf * e.x);
            atomicAdd(&acc[kWave + o], qf * e.y);
            atomicAdd(&acc[2 * kWave + o], qf * e.z);
            atomicAdd(&acc[3 * kWave + o], e.w * ec);
        }
        qn = base;
    }
    __device__ void fold() {
        __builtin_amdgcn_wave_barrier();
        this->add(acc[lane], acc[kWave + lane], acc[2 * kWave + lane], acc[3 * kWave + lane]);
        for (int c = 0; c < 4; c++) acc[c * kWave + lane] = 0.0;
    }
    __device__ void drain() {
        while (qn >= kWave) round(kWave);
        fold();
    }
    __device__ void flush() {
        while (qn > 0) round(min(qn, kWave));
        fold();
    }
};

// Wave-wide max / min of an int with DPP lane moves (no LDS round trips):
// within quads, within rows of 16 (half-mirror, mirror), then row 3 takes
// rows 0-2 by the row broadcasts; the result is read from lane 63 into a
// scalar register.  Every lane of the wave must be active.
template <bool MAX>
__device__ __forceinline__ int wave_reduce(int v) {
    // lanes outside the row mask see the identity of the operation
    constexpr int id = MAX ? INT_MIN : INT_MAX;
    auto op = [](int x, int y) { return MAX ? max(x, y) : min(x, y); };
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0xb1, 0xf, 0xf, false));    // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x4e, 0xf, 0xf, false));    // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x141, 0xf, 0xf, false));   // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x140, 0xf, 0xf, false));   // row_mirror
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));   // row_bcast:15 -> rows 1, 3
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));   // row_bcast:31 -> rows 2, 3
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max(int v) { return wave_reduce<true>(v); }
__device__ __forceinline__ int wave_min(int v) { return wave_reduce<false>(v); }

// One thread per target, targets in cell order (z-layer slowest, then x,
// then y), so the lanes of a wave share a z-layer and see neighbour rows of
// similar length; every wave belongs to one system.  For each image family,
// each z-layer within r_c and each x-column, the sources lie in one
// contiguous run of cells along y (two runs where the range wraps around the
// periodic y boundary), culled to the y-extent the sphere of radius r_c
// allows in that layer and column.  Pairs within r_c are queued and their
// erfc/exp terms evaluated later in rounds (LaneRings for FP32, WaveQueue
// for FP64, above).  The FP64 variant reads 32-byte FP64 source records.
// The FP32 variant reads 16-byte fixed-point records: a displacement is an
// exact integer difference rounded once to FP32, so its error is one
// position quantum (period / 2^32); pairs so close that this would matter
// (the closest pairs dominate the force) are recomputed from the FP64
// records.  It evaluates erfc/exp and the per-drain partial sums in FP32 and
// accumulates the drains in FP64.  The order of every sum is fixed by the
// data, so the results are bitwise reproducible.
template <int QW, int U, bool DG>
__device__ WaveQueue<QW, U, DG> make_wave_queue(unsigned char *lds, int tid, const double *coef, double alpha) {
    const int wid = tid / kWave, lane = tid % kWave;
    double4 *ent = reinterpret_cast<double4 *>(lds) + wid * QW;
    double *acc = reinterpret_cast<double *>(lds + (kBlock / kWave) * QW * sizeof(double4)) + wid * 4 * kWave;
    unsigned char *own = lds + (kBlock / kWave) * (QW * sizeof(double4) + 4 * kWave * sizeof(double)) + wid * QW;
    return WaveQueue<QW, U, DG>(ent, own, acc, coef, alpha, lane);
}

template <bool FP32, bool WANT_DG, bool ISO>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(FP32 ? RBE2D_REAL_WAVES32 : 4, 8)))
void k_real(RealArgs a) {
    static_assert(FP32 || !ISO, "the isotropic frame is a property of the fixed-point records");
    using T = typename RealTypes<FP32>::T;
    constexpr int U = RealTypes<FP32>::U;
    constexpr int NW = kBlock / kWave;
    constexpr int kRingQ = RBE2D_RING_Q;   // FP32: ring entries per lane
    // FP64: queue entries per wave.  A drain leaves at most 63 and a batch
    // adds at most U * 64, so the queue never holds more than 191; 240
    // keeps the block's LDS under 40 KB (four blocks, four waves per SIMD)
    constexpr int kWaveQ = 240;
    static_assert(FP32 || kWaveQ >= (kWave - 1) + U * kWave, "a batch must fit behind a drained queue");
    using Queue = typename std::conditional<FP32, LaneRings<kRingQ, U, ISO, WANT_DG>,
                                            WaveQueue<kWaveQ, U, WANT_DG>>::type;
    constexpr size_t kLds = FP32 ? sizeof(float4) * kRingQ * kBlock
                                 : NW * (kWaveQ * (sizeof(double4) + 1) + 4 * kWave * sizeof(double));
    __shared__ __align__(16) unsigned char lds[kLds];
    __shared__ double coef64[FP32 ? 1 : RBE2D_ERFCX64_DEG];
    if (!FP32) {
        if (threadIdx.x < RBE2D_ERFCX64_DEG) coef64[threadIdx.x] = rbe2d_erfcx64_a[threadIdx.x];
        __syncthreads();
    }
    const double4 *src = a.src;
    const int tid = threadIdx.x;
    // Blocks are dealt round-robin to the 8 XCDs.  Each XCD runs C contiguous
    // chunks of targets (chunk k of XCD x is chunk 8k + x of the range), so
    // neighbouring cells share that XCD's L2, and the targets near the walls
    // (cell order is z-slowest; they search extra image families) are shared
    // by all XCDs instead of loading the first and last ones.
    const int cs = (int)(gridDim.x >> 3) / RBE2D_REAL_CHUNKS;   // blocks per chunk
    const int j = (int)(blockIdx.x >> 3);
    const int lb = ((j / cs) * 8 + (int)(blockIdx.x & 7)) * cs + j % cs;
    if (lb >= a.nblocks) return;
    const int t = lb * kBlock + tid;
    // the system of this wave (system ranges are padded to whole waves)
    const int r = __builtin_amdgcn_readfirstlane(find_sys(a.lay.sbase, a.n_sys, t & ~(kWave - 1)));
    const SysDesc d = a.sys[r];   // a copy: loop-invariant values stay in registers
    const int shift = a.lay.sbase[r] - a.lay.off[r];    // unpadded -> padded sorted position
    const bool active = t - a.lay.sbase[r] < a.lay.off[r + 1] - a.lay.off[r];
    const Family *fams = a.fam + (int64_t)r * kMaxFamilies;
    const int *start = a.start + d.cbase;
    double4 me = make_double4(0.0, 0.0, 0.0, 0.0);
    int cid = 0;
    uint32_t xtf = 0, ytf = 0;   // target in fixed point (FP32 kernel)
    if (active) {
        me = src[t];
        cid = a.scell[t];
        if (FP32) { const uint4 m16 = a.src16[t]; xtf = m16.x; ytf = m16.y; }
    }
    const int cy = cid % d.ncy;
    const int cx = (cid / d.ncy) % d.ncx;
    const bool allx = d.ncx < 2 * d.reach + 1, ally = d.ncy < 2 * d.reach_y + 1;
    // Culling bounds are computed in FP32 with margins that cover its
    // rounding (and the division that assigned the cells): 1e-4 r_c^2 on the
    // squared y-extent, 1e-5 r_c on the extent.  They only decide which cells
    // are scanned; every candidate is then tested against r_c.
    const float yrel = (float)(me.y - cy * d.hy);   // y within the target's cell
    const float xrel = (float)me.x;                 // x within the target's cell
    const float hxf = (float)d.hx, inv_hyf = (float)d.inv_hy;
    const float rcm2 = (float)(d.rc2 * (1.0 + 1e-4));
    const float rmarg = (float)(1e-5 * d.rc);
    Queue qu = [&]() {
        if constexpr (FP32) return Queue(lds, tid, d);
        else return make_wave_queue<kWaveQ, U, WANT_DG>(lds, tid, coef64, d.alpha);
    }();
    for (int f = 0; f <= d.nfam; f++) {
        double sz = 1.0, czs = 0.0, w = 1.0, zsign = 1.0, dwt = 0.0, dwb = 0.0;
        if (f > 0) {
            const Family fm = fams[f - 1];
            sz = fm.sz; czs = fm.cz; w = fm.w; zsign = fm.zsign; dwt = fm.dwt; dwb = fm.dwb;
        }
        const double tz = sz * me.z + czs;
        const bool fam_on = active && tz > -d.rc && tz < d.H_rc;
        if (__ballot(fam_on) == 0) continue;
        const uint32_t tzf = fam_on ? to_fixed(tz + d.zoff, d.fzs) : 0u;
        int lzlo = d.ncz, lzhi = -1;
        if (fam_on) {
            lzlo = max(0, (int)floor((tz - d.rc_lay) * d.inv_hz));
            lzhi = min(d.ncz - 1, (int)floor((tz + d.rc_lay) * d.inv_hz));
        }
        const int wzlo = wave_min(lzlo), wzhi = wave_max(lzhi);
        qu.family(w, zsign, dwt, dwb);
        // FP32: scan run A [jbA, jbA + lenA), then run B, for pairs within
        // r_c.  Each lane walks its two runs as one sequence: A's batches of U
        // (the last one padded), then B's.  The trip count is the wave
        // maximum, so drains always run with every lane; pairing the columns
        // on either side of the target's (one long where the other is short)
        // evens out the lanes' trip counts.  A lone run is B empty.  Loads are
        // issued U at a time, double-buffered: the next U records are in
        // flight while these are tested (and while a drain runs); without
        // the gamma derivatives the two buffers swap roles every batch (the
        // loop body is unrolled by two), so no records are copied between them.
        auto scan32 = [&](int jbA, int lenA, double xtA, double ytA, int jbB, int lenB, double xtB, double ytB) {
            if constexpr (FP32) {
                const int c4a = (lenA + U - 1) / U * U;
                const int tot = c4a + lenB;
                const int maxtot = wave_max(tot);
                // loads from run B are clamped to min(m - c4a, lenB - 1): past a
                // run they stay within the padded arrays (jb + len - 1 + U - 1 <
                // capacity + 64) and are rejected
                const int lmB = max(lenB - 1, 0);
                auto rec = [&](int m0) { return m0 < c4a ? jbA + m0 : jbB + min(m0 - c4a, lmB); };
                // fixed-point displacements: exact integer differences (the
                // int32 wrap is the minimum image in x and y), one rounding
                // each to FP32; exact FP64 geometry for pairs within `near`
                const float rc2s = ISO ? d.rc2q : d.rc2f;
                const float near2s = ISO ? d.near2q : d.near2f;
                auto body = [&](const uint4 (&sv)[U], int m0) {
                    if (qu.full()) qu.drain();
                    const bool inA = m0 < c4a;
                    const int lim = inA ? lenA : tot;          // candidates m < lim
#pragma unroll
                    for (int k = 0; k < U; k++) {
                        const int m = m0 + k;
                        float dx = (float)(int)(xtf - sv[k].x);
                        float dy = (float)(int)(ytf - sv[k].y);
                        float dz = (float)(int)(tzf - sv[k].z);
                        if (!ISO) { dx *= d.ux; dy *= d.uy; dz *= d.uz; }
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        bool acc = m < lim && r2 < rc2s;
                        if (acc && r2 < near2s) {
                            const double4 s64 = src[inA ? jbA + m : jbB + (m - c4a)];
                            double ex = (inA ? xtA : xtB) - s64.x, ey = (inA ? ytA : ytB) - s64.y;
                            // the true displacement is below `near`, far from half a
                            // period, so rounding by the reciprocal finds the same image
                            ex -= d.Lx * rint(ex * d.inv_Lx);
                            ey -= d.Ly * rint(ey * d.inv_Ly);
                            const double ez = tz - s64.z;
                            // zero displacement only for the target itself (direct family)
                            acc = ex != 0.0 || ey != 0.0 || ez != 0.0;
                            if (ISO) { ex *= d.fxs; ey *= d.fxs; }
                            dx = (float)ex; dy = (float)ey; dz = (float)(ISO ? ez * d.fxs : ez);
                        }
                        qu.push(acc, dx, dy, dz, __uint_as_float(sv[k].w));
                    }
                };
                uint4 sa[U], sb[U];
                {
                    const uint4 *pq = a.src16 + rec(0);
#pragma unroll
                    for (int k = 0; k < U; k++) sa[k] = pq[k];
                }
                if constexpr (WANT_DG) {
                    // the gamma-derivative sums hold more registers: one loop
                    // body, the prefetched records copied into place
                    for (int m0 = 0; m0 < maxtot; m0 += U) {
                        if (m0 + U < maxtot) {
                            const uint4 *pq = a.src16 + rec(m0 + U);
#pragma unroll
                            for (int k = 0; k < U; k++) sb[k] = pq[k];
                        }
                        body(sa, m0);
#pragma unroll
                        for (int k = 0; k < U; k++) sa[k] = sb[k];
                    }
                } else {
                    for (int m0 = 0; m0 < maxtot; m0 += 2 * U) {
                        if (m0 + U < maxtot) {
                            const uint4 *pq = a.src16 + rec(m0 + U);
#pragma unroll
                            for (int k = 0; k < U; k++) sb[k] = pq[k];
                        }
                        body(sa, m0);
                        if (m0 + U >= maxtot) break;
                        if (m0 + 2 * U < maxtot) {
                            const uint4 *pq = a.src16 + rec(m0 + 2 * U);
#pragma unroll
                            for (int k = 0; k < U; k++) sa[k] = pq[k];
                        }
                        body(sb, m0 + U);
                    }
                }
            }
        };
        // FP64: scan one run [jb, jb + len); loads U at a time from
        // min(m0, len - 1), past the run inside the padded arrays and rejected
        auto scan64 = [&](int jb, int len, double xt, double yt, int self) {
            if constexpr (!FP32) {
                const int maxlen = wave_max(len);
                const double4 *p = src + jb;
                const int lm = max(len - 1, 0);
                for (int m0 = 0; m0 < maxlen; m0 += U) {
                    if (qu.full()) qu.drain();
                    const double4 *pq = p + min(m0, lm);
                    double4 sv[U];
#pragma unroll
                    for (int k = 0; k < U; k++) sv[k] = pq[k];
#pragma unroll
                    for (int k = 0; k < U; k++) {
                        const int m = m0 + k;
                        double dx = xt - sv[k].x;
                        double dy = yt - sv[k].y;
                        // the images differ only where |dx| is near half a period,
                        // beyond r_c <= period / 2 either way
                        if (allx) dx -= d.Lx * rint(dx * d.inv_Lx);
                        if (ally) dy -= d.Ly * rint(dy * d.inv_Ly);
                        const double dz = tz - sv[k].z;
                        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                        qu.push(m < len && r2 < d.rc2 && m != self, (T)dx, (T)dy, (T)dz, (T)sv[k].w);
                    }
                }
            }
        };
        // the runs of one column (cells along y within the sphere's extent
        // in this layer): [jb1, jb1 + len1) unshifted and, where the range
        // wraps around the periodic y boundary, [jb2, jb2 + len2) shifted by sy2
        struct Runs {
            int jb1, len1, jb2, len2;
            double xt, sy2;
        };
        auto col_runs = [&](bool lay_on, int lz, float dzmin, int ox) {
            Runs R{0, 0, 0, 0, 0.0, 0.0};
            const int dxc = allx ? ox - cx : ox;       // column offset in cells
            int cxx = allx ? ox : cx + ox;
            if (!allx) cxx += cxx < 0 ? d.ncx : (cxx >= d.ncx ? -d.ncx : 0);
            float dxmin = 0.0f;
            if (!allx) dxmin = dxc > 0 ? dxc * hxf - xrel : (dxc < 0 ? xrel - (dxc + 1) * hxf : 0.0f);
            R.xt = me.x - dxc * d.hx;
            const float ye2 = rcm2 - dxmin * dxmin - dzmin * dzmin;
            if (lay_on && ye2 > 0.0f) {
                const int row = (lz * d.ncx + cxx) * d.ncy;
                if (ally) {
                    R.jb1 = start[row];
                    R.len1 = start[row + d.ncy] - R.jb1;
                } else {
                    const float ye = __builtin_amdgcn_sqrtf(ye2) + rmarg;
                    int cylo = cy + (int)floorf((yrel - ye) * inv_hyf);
                    int cyhi = cy + (int)floorf((yrel + ye) * inv_hyf);
                    cylo = max(cylo, cy - d.reach_y);
                    cyhi = min(cyhi, cy + d.reach_y);
                    const int ya = max(cylo, 0), yb = min(cyhi, d.ncy - 1);
                    if (ya <= yb) { R.jb1 = start[row + ya]; R.len1 = start[row + yb + 1] - R.jb1; }
                    if (cylo < 0) {
                        R.jb2 = start[row + cylo + d.ncy];
                        R.len2 = start[row + d.ncy] - R.jb2;
                        R.sy2 = -d.Ly;
                    } else if (cyhi >= d.ncy) {
                        R.jb2 = start[row];
                        R.len2 = start[row + cyhi - d.ncy + 1] - R.jb2;
                        R.sy2 = d.Ly;
                    }
                }
            }
            R.jb1 += shift;
            R.jb2 += shift;
            return R;
        };
        // one column alone (its wrapped run too); the target itself is
        // excluded from the direct family only
        auto scan_col = [&](const Runs &R) {
            if constexpr (FP32) {
                scan32(R.jb1, R.len1, R.xt, me.y, R.jb1, 0, R.xt, me.y);
                if (__ballot(R.len2 > 0) != 0) scan32(R.jb2, R.len2, R.xt, me.y - R.sy2, R.jb2, 0, R.xt, me.y);
            } else {
                scan64(R.jb1, R.len1, R.xt, me.y, f == 0 ? t - R.jb1 : -1);
                if (__ballot(R.len2 > 0) != 0) scan64(R.jb2, R.len2, R.xt, me.y - R.sy2, f == 0 ? t - R.jb2 : -1);
            }
        };
        const int xlo = allx ? 0 : -d.reach, xhi = allx ? d.ncx - 1 : d.reach;
        const int ncol = xhi - xlo + 1;
        for (int lz = wzlo; lz <= wzhi; lz++) {
            const bool lay_on = lz >= lzlo && lz <= lzhi;
            const float dzmin = (float)fmax(0.0, fmax(lz * d.hz - tz, tz - (lz + 1) * d.hz));
            if (FP32 && a.nsplit == 1) {
                // columns in the order 0, -1, +1, -2, +2 (every column in
                // index order when all are searched): the first alone, then
                // pairs scanned as one sequence per lane
                auto col = [&](int i) { return allx ? i : (i == 0 ? 0 : ((i & 1) ? -((i + 1) >> 1) : (i >> 1))); };
                scan_col(col_runs(lay_on, lz, dzmin, col(0)));
                for (int i = 1; i < ncol; i += 2) {
                    const Runs A = col_runs(lay_on, lz, dzmin, col(i));
                    if (i + 1 < ncol) {
                        const Runs B = col_runs(lay_on, lz, dzmin, col(i + 1));
                        scan32(A.jb1, A.len1, A.xt, me.y, B.jb1, B.len1, B.xt, me.y);
                        if (__ballot(A.len2 > 0) != 0)
                            scan32(A.jb2, A.len2, A.xt, me.y - A.sy2, A.jb2, 0, A.xt, me.y);
                        if (__ballot(B.len2 > 0) != 0)
                            scan32(B.jb2, B.len2, B.xt, me.y - B.sy2, B.jb2, 0, B.xt, me.y);
                    } else {
                        scan_col(A);
                    }
                }
            } else {
                for (int ox = xlo + (int)blockIdx.y; ox <= xhi; ox += a.nsplit)
                    scan_col(col_runs(lay_on, lz, dzmin, ox));
            }
        }
        qu.flush();
    }
    const double fx = qu.fx, fy = qu.fy, fz = qu.fz, phi = qu.phi, dpt = qu.dpt, dpb = qu.dpb;
    double qphi = 0.0, qdt = 0.0, qdb = 0.0;
    if (active) {
        const int i = a.sidx[t];
        const double qi = me.w * d.pref;
        const double4 fo = make_double4(qi * fx, qi * fy, qi * fz, d.pref * phi);
        const double2 go = make_double2(d.pref * dpt, d.pref * dpb);
        if (a.nsplit > 1) {
            const int64_t o = (int64_t)blockIdx.y * a.split_stride + i;
            a.freal_s[o] = fo;
            if (WANT_DG) a.dgreal_s[o] = go;
        } else {
            a.freal[i] = fo;
            if (WANT_DG) a.dgreal[i] = go;
        }
        qphi = qi * phi;
        if (WANT_DG) {
            qdt = qi * dpt;
            qdb = qi * dpb;
        }
    }
    // per-wave partial sums (a wave never straddles two systems)
    qphi = wave_sum(qphi);
    if (WANT_DG) { qdt = wave_sum(qdt); qdb = wave_sum(qdb); }
    if ((tid & (kWave - 1)) == 0 && t / kWave < a.n_waves) {
        const int wv = t / kWave;
        double *o = a.nsplit > 1 ? a.rpart_s + 3 * ((int64_t)blockIdx.y * a.rsplit_stride + wv) : a.rpart + 3 * wv;
        o[0] = qphi;
        o[1] = qdt;
        o[2] = qdb;
    }
}

// sum of the split partial outputs, in split order
__global__ __launch_bounds__(kBlock) void k_real_combine(RealArgs a, int n_total, int want_dg) {
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g < n_total) {
        double4 f = a.freal_s[g];
        double2 dg = want_dg ? a.dgreal_s[g] : make_double2(0.0, 0.0);
        for (int s = 1; s < a.nsplit; s++) {
            const double4 v = a.freal_s[(int64_t)s * a.split_stride + g];
            f.x += v.x; f.y += v.y; f.z += v.z; f.w += v.w;
            if (want_dg) {
                const double2 u = a.dgreal_s[(int64_t)s * a.split_stride + g];
                dg.x += u.x; dg.y += u.y;
            }
        }
        a.freal[g] = f;
        if (want_dg) a.dgreal[g] = dg;
    }
    if (g < a.n_waves) {
        for (int c = 0; c < 3; c++) {
            double v = 0.0;
            for (int s = 0; s < a.nsplit; s++) v += a.rpart_s[3 * ((int64_t)s * a.rsplit_stride + g) + c];
            a.rpart[3 * g + c] = v;
        }
    }
}

hipError_t launch_real(rbe2d_ctx *h, const double *pos, const double *q, bool want_dg, hipStream_t s) {
    hipError_t e = launch_cells(h, pos, q, s);
    return e == hipSuccess ? launch_pairs(h, want_dg, s) : e;
}

hipError_t launch_cells(rbe2d_ctx *h, const double *pos, const double *q, hipStream_t s) {
    if (h->n_total == 0) return hipSuccess;
    CellArgs c;
    c.pos = pos; c.q = q; c.sys = h->w.sys; c.lay = h->w.lay; c.n_sys = h->n_sys;
    c.n_total = (int)h->n_total; c.ncells = h->total_cells;
    c.cell = h->w.cell; c.slot = h->w.slot; c.count = h->w.count; c.start = h->w.start;
    c.tmp = h->w.tmp; c.n_waves = h->n_swaves; c.sidx = h->w.sidx; c.scell = h->w.scell; c.sorted = h->w.sorted; c.src16 = h->w.src16;
    // counted by the MD pass: its k-space records of these positions precede this build on s
    const bool fp32 = h->precision == RBE2D_PREC_FP32_PHASE;
    c.p32 = h->cells_counted && fp32 ? h->w.p32 : nullptr;
    c.p64 = h->cells_counted && !fp32 ? h->w.p64 : nullptr;
    const int nb = (int)((h->n_total + kBlock - 1) / kBlock);
    prof_begin(h, 3, s);
    // the counts start at zero (the previous build's scan cleared them); the
    // MD pass that moved the particles may have counted them already
    if (!h->cells_counted) hipLaunchKernelGGL(k_cell_count, dim3(nb), dim3(kBlock), 0, s, c);
    h->cells_counted = false;
    const int nsb = (h->total_cells + kScanCells - 1) / kScanCells;
    hipLaunchKernelGGL(k_scan_totals, dim3(nsb), dim3(kBlock), 0, s, h->w.count, h->total_cells, h->w.scanbuf);
    hipLaunchKernelGGL(k_scan_apply, dim3(nsb), dim3(kBlock), 0, s, h->w.count, h->total_cells, h->w.scanbuf,
                       h->w.start);
    hipLaunchKernelGGL(k_cell_scatter, dim3(nb), dim3(kBlock), 0, s, c);
    hipLaunchKernelGGL(k_cell_rank, dim3((h->n_swaves * kWave + kBlock - 1) / kBlock), dim3(kBlock), 0, s, c);
    prof_end(h, 3, s);
    return hipGetLastError();
}

hipError_t launch_pairs(rbe2d_ctx *h, bool want_dg, hipStream_t s) {
    if (h->n_total == 0) return hipSuccess;
    RealArgs r;
    r.src = h->w.sorted; r.src16 = h->w.src16; r.sidx = h->w.sidx; r.scell = h->w.scell; r.start = h->w.start;
    r.sys = h->w.sys; r.fam = h->w.fam; r.lay = h->w.lay; r.n_sys = h->n_sys; r.n_waves = h->n_swaves;
    r.freal = h->w.freal; r.dgreal = h->w.dgreal; r.rpart = h->w.rpart;
    r.freal_s = h->w.freal_s; r.dgreal_s = h->w.dgreal_s; r.rpart_s = h->w.rpart_s;
    r.split_stride = h->split_cap;
    r.rsplit_stride = (int)(h->cap_sorted / kWave);
    // too few targets to fill the chip: split each target's x-columns over
    // several blocks (about 4096 waves in flight is enough)
    r.nsplit = 1;
    if (h->n_total <= h->split_cap) {
        if (h->force_rsplit) r.nsplit = h->force_rsplit;
        else if (h->tuned_now && h->tune.rsplit) r.nsplit = h->tune.rsplit;
        else r.nsplit = (int)std::min<int64_t>(kMaxRealSplit, std::max<int64_t>(1, 4096 / std::max(1, h->n_swaves)));
        r.nsplit = std::max(1, std::min(kMaxRealSplit, r.nsplit));
    }
    const int nbs = (h->n_swaves * kWave + kBlock - 1) / kBlock;
    r.nblocks = nbs;
    const int nch = 8 * RBE2D_REAL_CHUNKS;
    const int nbc = (nbs + nch - 1) / nch * nch;
    const bool fp32 = h->precision == RBE2D_PREC_FP32_PHASE;
    const dim3 grid(nbc, r.nsplit);
    prof_begin(h, 4, s);
    if (fp32 && h->iso) {
        if (want_dg) hipLaunchKernelGGL((k_real<true, true, true>), grid, dim3(kBlock), 0, s, r);
        else hipLaunchKernelGGL((k_real<true, false, true>), grid, dim3(kBlock), 0, s, r);
    } else if (fp32) {
        if (want_dg) hipLaunchKernelGGL((k_real<true, true, false>), grid, dim3(kBlock), 0, s, r);
        else hipLaunchKernelGGL((k_real<true, false, false>), grid, dim3(kBlock), 0, s, r);
    } else {
        if (want_dg) hipLaunchKernelGGL((k_real<false, true, false>), grid, dim3(kBlock), 0, s, r);
        else hipLaunchKernelGGL((k_real<false, false, false>), grid, dim3(kBlock), 0, s, r);
    }
    if (r.nsplit > 1) {
        const int64_t n = std::max<int64_t>(h->n_total, h->n_swaves);
        hipLaunchKernelGGL(k_real_combine, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, r,
                           (int)h->n_total, (int)want_dg);
    }
    prof_end(h, 4, s);
    return hipGetLastError();
}

// F += F_real (the pair kernel's per-particle output), and in MD steps the
// closing half kick v += dt/2 F with the completed force
__global__ __launch_bounds__(kBlock) void k_add_real(int64_t n, const double4 *freal, double *F, double *vel,
                                                     double half_dt) {
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n) return;
    const double4 fr = freal[g];
    const double add[3] = {fr.x, fr.y, fr.z};
    for (int c = 0; c < 3; c++) {
        const double f = F[3 * g + c] + add[c];
        F[3 * g + c] = f;
        if (vel) vel[3 * g + c] = fma(half_dt, f, vel[3 * g + c]);
    }
}

hipError_t launch_add_real(rbe2d_ctx *h, double *F, double *vel, double half_dt, hipStream_t s) {
    if (h->n_total == 0) return hipSuccess;
    prof_begin(h, 10, s);
    hipLaunchKernelGGL(k_add_real, dim3((unsigned)((h->n_total + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       h->n_total, h->w.freal, F, vel, half_dt);
    prof_end(h, 10, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Short-range forces of the MD (purely repulsive shifted-truncated LJ between
// ions and against the walls), on the cell list of the pair kernel.  One
// thread per target in cell order; within the layers and x-columns that come
// within the LJ cutoff of the target, the cells along y within its y-extent
// (all columns or rows of a small box once).  Forces are added to
// F[stride * i + 0..2] (the caller's N x 3 forces, or the pair kernel's
// per-particle output); per-wave energy sums go to spart.
// ---------------------------------------------------------------------------

struct ShortArgs {
    const double4 *src;
    const int *sidx, *scell, *start;
    const SysDesc *sys;
    Layout lay;
    int n_sys, n_waves;
    MdExtra mx;
    double *F;
    int stride;
    double *spart;
};

__device__ __forceinline__ double lj_rep(double s2_over_r2, double eps, double *r_times_f) {
    const double s6 = s2_over_r2 * s2_over_r2 * s2_over_r2;
    *r_times_f = 24.0 * eps * (2.0 * s6 * s6 - s6);
    return 4.0 * eps * (s6 * s6 - s6 + 0.25);
}

__global__ __launch_bounds__(kBlock) void k_short(ShortArgs a) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int r = __builtin_amdgcn_readfirstlane(find_sys(a.lay.sbase, a.n_sys, t & ~(kWave - 1)));
    const SysDesc d = a.sys[r];
    const int shift = a.lay.sbase[r] - a.lay.off[r];
    const bool active = t - a.lay.sbase[r] < a.lay.off[r + 1] - a.lay.off[r];
    double fx = 0, fy = 0, fz = 0, ep = 0, ew = 0;
    if (active) {
        const double4 me = a.src[t];
        const int cid = a.scell[t];
        const int cy = cid % d.ncy, cx = (cid / d.ncy) % d.ncx;
        const double xt = me.x + cx * d.hx;   // wrapped x of the target
        if (a.mx.eps != 0.0) {
            // cell ranges within the cutoff, with a 1e-9 margin (cells were
            // assigned by division); a small box searches each column or row once
            const double rc = sqrt(a.mx.rc2) * (1.0 + 1e-9);
            const int rx = (int)ceil(rc / d.hx), ry = (int)ceil(rc / d.hy);
            const bool allx = d.ncx <= 2 * rx, ally = d.ncy <= 2 * ry;
            const int x0 = allx ? 0 : cx + (int)floor((me.x - rc) * d.inv_hx);
            const int x1 = allx ? d.ncx - 1 : cx + (int)floor((me.x + rc) * d.inv_hx);
            const double yrel = me.y - cy * d.hy;
            const int y0 = ally ? 0 : cy + (int)floor((yrel - rc) * d.inv_hy);
            const int y1 = ally ? d.ncy - 1 : cy + (int)floor((yrel + rc) * d.inv_hy);
            const int z0 = max(0, (int)floor((me.z - rc) * d.inv_hz));
            const int z1 = min(d.ncz - 1, (int)floor((me.z + rc) * d.inv_hz));
            const int *start = a.start + d.cbase;
            for (int lz = z0; lz <= z1; lz++)
                for (int ix = x0; ix <= x1; ix++) {
                    const int cxx = (ix % d.ncx + d.ncx) % d.ncx;
                    const int row = (lz * d.ncx + cxx) * d.ncy;
                    // along y: one run of cells, or two where it wraps
                    for (int part = 0; part < 2; part++) {
                        int ya = y0, yb = y1;
                        if (!ally) {
                            if (part == 0) { ya = max(y0, 0); yb = min(y1, d.ncy - 1); }
                            else if (y0 < 0) { ya = y0 + d.ncy; yb = d.ncy - 1; }
                            else if (y1 >= d.ncy) { ya = 0; yb = y1 - d.ncy; }
                            else break;
                        } else if (part == 1) {
                            break;
                        }
                        if (ya > yb) continue;
                        const int b = start[row + ya] + shift, e = start[row + yb + 1] + shift;
                        for (int j = b; j < e; j++) {
                            if (j == t) continue;
                            const double4 sj = a.src[j];
                            double dx = xt - (sj.x + cxx * d.hx);
                            double dy = me.y - sj.y;
                            dx -= d.Lx * rint(dx * d.inv_Lx);
                            dy -= d.Ly * rint(dy * d.inv_Ly);
                            const double dz = me.z - sj.z;
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 < a.mx.rc2) {
                                double rf;
                                ep += 0.5 * lj_rep(a.mx.sig2 / r2, a.mx.eps, &rf);
                                fx += rf / r2 * dx; fy += rf / r2 * dy; fz += rf / r2 * dz;
                            }
                        }
                    }
                }
        }
        if (a.mx.epsw != 0.0) {
            const double hb = me.z, ht = d.H - me.z;
            double rf;
            if (hb > 0.0 && hb < a.mx.hcut) { ew += lj_rep(a.mx.sigw2 / (hb * hb), a.mx.epsw, &rf); fz += rf / hb; }
            if (ht > 0.0 && ht < a.mx.hcut) { ew += lj_rep(a.mx.sigw2 / (ht * ht), a.mx.epsw, &rf); fz -= rf / ht; }
        }
        const int i = a.sidx[t];
        double *o = a.F + (int64_t)a.stride * i;
        o[0] += fx;
        o[1] += fy;
        o[2] += fz;
    }
    ep = wave_sum(ep);
    ew = wave_sum(ew);
    if ((threadIdx.x & (kWave - 1)) == 0 && t / kWave < a.n_waves) {
        a.spart[2 * (t / kWave)] = ep;
        a.spart[2 * (t / kWave) + 1] = ew;
    }
}

// per-system sums of the wave energies, fixed order
__global__ __launch_bounds__(kBlock) void k_short_energy(const double *spart, Layout lay, double *energy) {
    __shared__ double sh[kBlock / 64];
    const int r = blockIdx.x;
    double ep = 0, ew = 0;
    for (int wv = lay.sbase[r] / kWave + threadIdx.x; wv < lay.sbase[r + 1] / kWave; wv += kBlock) {
        ep += spart[2 * wv];
        ew += spart[2 * wv + 1];
    }
    ep = block_sum(ep, sh);
    ew = block_sum(ew, sh);
    if (threadIdx.x == 0) {
        energy[2 * r] = ep;
        energy[2 * r + 1] = ew;
    }
}

hipError_t launch_short(rbe2d_ctx *h, const MdExtra &mx, double *F, double *energy, hipStream_t s, bool into_real) {
    prof_begin(h, 9, s);
    if (h->n_total > 0 && mx.short_on()) {
        ShortArgs a;
        a.src = h->w.sorted; a.sidx = h->w.sidx; a.scell = h->w.scell; a.start = h->w.start;
        a.sys = h->w.sys; a.lay = h->w.lay; a.n_sys = h->n_sys; a.n_waves = h->n_swaves;
        a.mx = mx; a.spart = h->w.spart;
        // into_real: add to the pair kernel's per-particle output (x, y, z, phi)
        a.F = into_real ? (double *)h->w.freal : F;
        a.stride = into_real ? 4 : 3;
        hipLaunchKernelGGL(k_short, dim3((h->n_swaves * kWave + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
    }
    if (energy) {
        if (h->n_total > 0 && mx.short_on()) {
            hipLaunchKernelGGL(k_short_energy, dim3(h->n_sys), dim3(kBlock), 0, s, h->w.spart, h->w.lay, energy);
        } else {
            (void)launch_fill(energy, (int64_t)h->n_sys * 2 * sizeof(double), s);
        }
    }
    prof_end(h, 9, s);
    return hipGetLastError();
}

}  // namespace rbe2d
