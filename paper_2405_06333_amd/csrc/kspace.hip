// k-space half of RBE2D on gfx950: particle preparation, the N x P
// structure-factor pass, the FP64 reduction/recalibration per k, the force
// scatter.  Every launch covers all systems of a handle; a block finds its
// system in the layout tables (particles are padded per system to whole
// tiles, so blocks never straddle systems and k-data stay wave-uniform).
//
// Phases are carried in revolutions: k.r / 2pi = nx fx + ny fy + nz fz with
// fx = x/Lx wrapped into [0,1), fy = y/Ly, fz = z/Lz_ext.
//  * FP32 path: f is split into fh (fh_bits = 22 - b fraction bits, where
//    every |n| < 2^b) and fl = f - fh.  Then n fh has at most 22 significant
//    bits and nx fxh + ny fyh at most 23, so both are exact in FP32; the
//    phase fract(nx fxh + ny fyh) + nx fxl + ny fyl (and likewise in z)
//    keeps ~1e-8 revolution accuracy, and the hardware v_sin_f32/v_cos_f32
//    take revolutions directly.
//  * FP64 path: plain FP64 phase and a quarter-turn-reduced Taylor sincos.
#include <algorithm>

#include "devmath.h"
#include "rbe2d_internal.h"

namespace rbe2d {

// ---------------------------------------------------------------------------
// 1. particle preparation
// ---------------------------------------------------------------------------

struct PrepArgs {
    const double *pos, *q;
    const SysDesc *sys;
    Layout lay;
    int n_sys;
    float4 *p32;
    double4 *p64;
    double *bpart;
    int *err;
    // MD update first (MD > 0): positions and velocities are updated in place
    double *pos_md, *vel;
    const double *F;
    const double4 *freal;       // MD == 2: the pair kernel's part of the force
    double dt, zlo, zhi_from_top;
    // MD > 0 with count set: the cell and in-cell slot of each moved
    // particle for the next cell-list build (the counts start at zero)
    int *cell, *slot, *count;
};

// MD: 0 none; 1 opening half kick with F and drift; 2 closing half kick and
// the next opening half kick, both with F + freal (the same force, the same
// roundings as two separate kicks), and drift.  Then the k-space particle
// records of the (new) positions and the block sums of the IBC.
template <bool FP32, int MD>
__global__ __launch_bounds__(kBlock) void k_prep(PrepArgs a) {
    __shared__ double sh[4][kBlock / 64];
    const int b = blockIdx.x;
    const int r = find_sys(a.lay.bbase, a.n_sys, b);
    const SysDesc &d = a.sys[r];
    const int iloc = (b - a.lay.bbase[r]) * kBlock + threadIdx.x;
    const int Nr = a.lay.off[r + 1] - a.lay.off[r];
    const int64_t ii = (int64_t)a.lay.pbase[r] + iloc;      // internal (padded) index
    double sqz = 0.0, sq = 0.0, sq2 = 0.0, sqzz = 0.0;
    double fx = 0, fy = 0, fz = 0, qi = 0;
    if (iloc < Nr) {
        const int64_t g = (int64_t)a.lay.off[r] + iloc;      // caller index
        double x, y, z;
        if (MD > 0) {
            double v[3], rr[3], add[3] = {0.0, 0.0, 0.0};
            if (MD == 2) {
                const double4 fr = a.freal[g];
                add[0] = fr.x; add[1] = fr.y; add[2] = fr.z;
            }
            for (int c = 0; c < 3; c++) {
                const double f = MD == 2 ? a.F[3 * g + c] + add[c] : a.F[3 * g + c];
                v[c] = fma(0.5 * a.dt, f, a.vel[3 * g + c]);
                if (MD == 2) v[c] = fma(0.5 * a.dt, f, v[c]);
                rr[c] = a.pos_md[3 * g + c];
            }
            drift_fold(d, a.dt, a.zlo, a.zhi_from_top, v, rr);
            for (int c = 0; c < 3; c++) {
                a.vel[3 * g + c] = v[c];
                a.pos_md[3 * g + c] = rr[c];
            }
            x = rr[0]; y = rr[1]; z = rr[2];
            if (a.count) {
                double xw, yw;
                const int c = d.cbase + cell_of(x, y, z, d, &xw, &yw);
                a.cell[g] = c;
                a.slot[g] = atomicAdd(&a.count[c], 1);
            }
        } else {
            x = a.pos[3 * g]; y = a.pos[3 * g + 1]; z = a.pos[3 * g + 2];
        }
        qi = a.q[g];
        if (!(z > 0.0 && z < d.H)) atomicOr(a.err, 1);
        fx = x * d.inv_Lx; fx -= floor(fx);
        fy = y * d.inv_Ly; fy -= floor(fy);
        fz = z * d.inv_Lz;
        sqz = qi * z; sq = qi; sq2 = qi * qi; sqzz = qi * z * z;
    }
    if (FP32) {
        // scale_h = 2^fh_bits: the split is exact
        const double hx = ldexp(rint(fx * d.scale_h), -d.fh_bits);
        const double hy = ldexp(rint(fy * d.scale_h), -d.fh_bits);
        const double hz = ldexp(rint(fz * d.scale_h), -d.fh_bits);
        a.p32[2 * ii] = make_float4((float)hx, (float)(fx - hx), (float)hy, (float)(fy - hy));
        a.p32[2 * ii + 1] = make_float4((float)hz, (float)(fz - hz), (float)qi, 0.0f);
    } else {
        a.p64[ii] = make_double4(fx, fy, fz, qi);
    }
    // block sums of q z, q, q^2, q z^2 (one barrier for the four)
    sqz = wave_sum(sqz);
    sq = wave_sum(sq);
    sq2 = wave_sum(sq2);
    sqzz = wave_sum(sqzz);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sh[0][wid] = sqz; sh[1][wid] = sq; sh[2][wid] = sq2; sh[3][wid] = sqzz; }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; k++) t += sh[threadIdx.x][k];
        a.bpart[4 * b + threadIdx.x] = t;
    }
}

// scal layout (kScal per system): 0 mu = sum q z, 1 Q = sum q, 2 sum q^2,
// 3 muM (image dipole of Theorem 3.3), 4 F_ibc,z / q_i, 5 offset of the
// IBC potential, 6 dmuM/dgamma_top, 7 dmuM/dgamma_bot, 8 S2 = sum q z^2;
// with surface charges (zero otherwise): F_z / q_i gains 10 + 9 z, the
// potential dE/dq_i gains 11 + 12 z + 13 z^2, the energy 14, and
// dE/dgamma_{top,bot} 15, 16
struct ScalArgs {
    const double *bpart;
    const SysDesc *sys;
    Layout lay;
    double *scal;
};

// IBC scalars of system r from the prep pass's block sums, by one wave
// (fixed summation order: the same in both launches that use it)
__device__ void ibc_scalars(const ScalArgs &a, int r, int lane) {
    const SysDesc &d = a.sys[r];
    double v[4] = {0, 0, 0, 0};
    for (int b = a.lay.bbase[r] + lane; b < a.lay.bbase[r + 1]; b += 64)
        for (int c = 0; c < 4; c++) v[c] += a.bpart[4 * b + c];
    for (int c = 0; c < 4; c++) v[c] = wave_sum(v[c]);
    if (lane == 0) {
        const double mu = v[0], Q = v[1], S2 = v[3];
        const double muM = d.g1 * mu + d.cgam * Q;
        const double tv = 2.0 * kPi / d.V * d.pref;
        double *o = a.scal + kScal * r;
        o[0] = mu;
        o[1] = Q;
        o[2] = v[2];
        o[3] = muM;
        o[4] = -tv * (muM + d.g1 * mu);
        o[5] = tv * mu * d.cgam;
        o[6] = d.dg1t * mu + d.dcgt * Q;
        o[7] = d.dg1b * mu + d.dcgb * Q;
        o[8] = S2;
        for (int c = 9; c < kScal; c++) o[c] = 0.0;
        if (d.surf) {
            // sheets: phi_s = -Es z + Cs; net charge: U_Q = -(tv / 2) Q (2 Gs S2 + 2 A1 mu + A0 Q)
            const double pe = d.pref;
            o[9] = 2.0 * tv * Q * d.Gs[0];
            o[10] = pe * d.Es[0] + tv * Q * d.A1[0];
            o[11] = pe * d.Cs[0] - tv * (d.Gs[0] * S2 + d.A1[0] * mu + d.A0[0] * Q);
            o[12] = -pe * d.Es[0] - tv * Q * d.A1[0];
            o[13] = -tv * Q * d.Gs[0];
            for (int k = 0; k < 3; k++) {
                const double e = -0.5 * tv * Q * (2.0 * d.Gs[k] * S2 + 2.0 * d.A1[k] * mu + d.A0[k] * Q) +
                                 pe * (-d.Es[k] * mu + d.Cs[k] * Q);
                o[k == 0 ? 14 : 14 + k] = e;
            }
        }
    }
}

__global__ __launch_bounds__(64) void k_scalars(ScalArgs a) { ibc_scalars(a, blockIdx.x, threadIdx.x); }

__global__ void k_ktable(const int32_t *kset, int n_sys, int P, int P_pad, float4 *kn32, double4 *kn64);

static PrepArgs prep_args(rbe2d_ctx *h, const double *pos, const double *q) {
    PrepArgs a{};
    a.pos = pos; a.q = q; a.sys = h->w.sys; a.lay = h->w.lay; a.n_sys = h->n_sys;
    a.p32 = h->w.p32; a.p64 = h->w.p64; a.bpart = h->w.bpart; a.err = h->w.err;
    return a;
}

void launch_ktable(rbe2d_ctx *h, hipStream_t s) {
    const int nk = h->n_sys * h->P_pad;
    hipLaunchKernelGGL(k_ktable, dim3((nk + 63) / 64), dim3(64), 0, s, h->w.kset, h->n_sys, h->P, h->P_pad,
                       h->w.kn32, h->w.kn64);
}

static ScalArgs scal_args(rbe2d_ctx *h) {
    ScalArgs b;
    b.bpart = h->w.bpart; b.sys = h->w.sys; b.lay = h->w.lay; b.scal = h->w.scal;
    return b;
}

static void launch_scalars(rbe2d_ctx *h, hipStream_t s) {
    hipLaunchKernelGGL(k_scalars, dim3(h->n_sys), dim3(64), 0, s, scal_args(h));
}

template <int MD>
static void launch_prep_kernel(rbe2d_ctx *h, const PrepArgs &a, hipStream_t s) {
    if (h->n_blocks <= 0) return;
    if (h->precision == RBE2D_PREC_FP32_PHASE)
        hipLaunchKernelGGL((k_prep<true, MD>), dim3(h->n_blocks), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_prep<false, MD>), dim3(h->n_blocks), dim3(kBlock), 0, s, a);
}

hipError_t launch_prep(rbe2d_ctx *h, const double *pos, const double *q, hipStream_t s, bool scalars) {
    // the k-vector table needs only the k-set: first, off the particles' path
    launch_ktable(h, s);
    prof_begin(h, 0, s);
    launch_prep_kernel<0>(h, prep_args(h, pos, q), s);
    if (scalars) launch_scalars(h, s);
    prof_end(h, 0, s);
    return hipGetLastError();
}

hipError_t launch_prep_md(rbe2d_ctx *h, double *pos, double *vel, const double *F, const double *q, double dt,
                          double zlo, double zhi_from_top, bool with_real, hipStream_t s) {
    PrepArgs a = prep_args(h, pos, q);
    a.pos_md = pos; a.vel = vel; a.F = F; a.freal = h->w.freal;
    a.dt = dt; a.zlo = zlo; a.zhi_from_top = zhi_from_top;
    // a force evaluation with real space follows: count the particles per
    // cell here, where their new positions are at hand
    a.cell = h->w.cell; a.slot = h->w.slot; a.count = h->w.count;
    prof_begin(h, 7, s);
    if (with_real) launch_prep_kernel<2>(h, a, s);
    else launch_prep_kernel<1>(h, a, s);
    prof_end(h, 7, s);
    h->cells_counted = h->n_total > 0;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 2. k-vector table (nx, ny, nz as floats / doubles, padded with zeros)
// ---------------------------------------------------------------------------

__global__ void k_ktable(const int32_t *kset, int n_sys, int P, int P_pad, float4 *kn32, double4 *kn64) {
    const int kg = blockIdx.x * blockDim.x + threadIdx.x;
    if (kg >= n_sys * P_pad) return;
    const int r = kg / P_pad, l = kg - r * P_pad;
    int nx = 0, ny = 0, nz = 0;
    if (l < P) {
        const int32_t *n = kset + 3 * ((int64_t)r * P + l);
        nx = n[0]; ny = n[1]; nz = n[2];
    }
    kn32[kg] = make_float4((float)nx, (float)ny, (float)nz, 0.0f);
    kn64[kg] = make_double4((double)nx, (double)ny, (double)nz, 0.0);
}

// ---------------------------------------------------------------------------
// 3. structure-factor pass: per (particle tile, k-chunk) partial sums of
//    rho(k) = sum q e^{2 pi i phi} and rhohat(k) = sum q e^{2 pi i phihat}
//    with phi = phi_xy + phi_z, phihat = phi_xy - phi_z.
//    Lanes own particles, the k-chunk is wave-uniform (scalar loads).
// ---------------------------------------------------------------------------

// Blocks are dealt round-robin to the 8 XCDs.  Map block b to (tile, k-chunk)
// so that XCD b mod 8 runs all k-chunks of its tiles back to back: a tile is
// then fetched into one XCD's L2 once instead of once per k-chunk.  The grid
// has ceil(n_tiles / 8) * 8 * nkc blocks; blocks past the last tile exit.
struct TileChunk {
    int tile, kc;
};
__device__ __forceinline__ TileChunk tile_chunk(int b, int nkc) {
    const int j = b >> 3;
    return TileChunk{(j / nkc) * 8 + (b & 7), j % nkc};
}

// FP32 phases and transcendentals; each thread sums its (at most 16)
// particles in FP32, and every sum after that -- across the 64 lanes, the
// waves of the block and (in the assembly) the tiles -- is in FP64.
template <int KC>
__global__ __launch_bounds__(kBlock) void k_sf32(const float4 *__restrict__ p32,
                                                 const float4 *__restrict__ kn, const int *tbase,
                                                 int n_sys, int per_thread, int P_pad, int n_tiles,
                                                 double *__restrict__ part) {
    static_assert(4 * KC == 64, "one wave-transposed value per lane");
    __shared__ double sh[kBlock / 64][64];
    const TileChunk tc = tile_chunk((int)blockIdx.x, P_pad / KC);
    if (tc.tile >= n_tiles) return;
    const int r = find_sys(tbase, n_sys, tc.tile);
    const float4 *knr = kn + (int64_t)r * P_pad + tc.kc * KC;
    float acc[4 * KC];
#pragma unroll
    for (int v = 0; v < 4 * KC; v++) acc[v] = 0.0f;
    const int64_t base = (int64_t)tc.tile * kBlock * per_thread + threadIdx.x;
    for (int m = 0; m < per_thread; m++) {
        const int64_t i = base + (int64_t)m * kBlock;
        const float4 a = p32[2 * i];
        const float4 b = p32[2 * i + 1];
#pragma unroll
        for (int kk = 0; kk < KC; kk++) {
            const float4 n = knr[kk];
            // nx fxh + ny fyh is exact (see the header comment)
            float pxy = fractf(fmaf(n.y, a.z, n.x * a.x));
            pxy = fmaf(n.x, a.y, pxy);
            pxy = fmaf(n.y, a.w, pxy);
            const float pz = fmaf(n.z, b.y, fractf(n.z * b.x));
            const float ph = pxy + pz, phh = pxy - pz;
            acc[4 * kk + 0] = fmaf(b.z, cos_rev(ph), acc[4 * kk + 0]);
            acc[4 * kk + 1] = fmaf(b.z, sin_rev(ph), acc[4 * kk + 1]);
            acc[4 * kk + 2] = fmaf(b.z, cos_rev(phh), acc[4 * kk + 2]);
            acc[4 * kk + 3] = fmaf(b.z, sin_rev(phh), acc[4 * kk + 3]);
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // first butterfly stage of the wave transpose-reduce: the FP32 values are
    // exchanged, then widened and added in FP64; the other stages run in FP64
    double v[2 * KC];
    {
        const bool upper = (lane & 32) != 0;
#pragma unroll
        for (int i = 0; i < 2 * KC; i++) {
            const float send = upper ? acc[i] : acc[i + 2 * KC];
            const float keep = upper ? acc[i + 2 * KC] : acc[i];
            v[i] = (double)keep + (double)__shfl_xor(send, 32, 64);
        }
    }
    TransposeStage<KC, 2 * KC, double>::run(v, lane);
    sh[wid][lane] = v[0];
    __syncthreads();
    if (threadIdx.x < 4 * KC) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; w++) t += sh[w][threadIdx.x];
        part[((int64_t)tc.tile * P_pad + tc.kc * KC) * 4 + threadIdx.x] = t;
    }
}

template <int KC>
__global__ __launch_bounds__(kBlock) void k_sf64(const double4 *__restrict__ p64,
                                                 const double4 *__restrict__ kn, const int *tbase,
                                                 int n_sys, int per_thread, int P_pad, int n_tiles,
                                                 double *__restrict__ part) {
    __shared__ double sh[kBlock / 64][4 * KC];
    const TileChunk tc = tile_chunk((int)blockIdx.x, P_pad / KC);
    if (tc.tile >= n_tiles) return;
    const int r = find_sys(tbase, n_sys, tc.tile);
    const double4 *knr = kn + (int64_t)r * P_pad + tc.kc * KC;
    double acc[4 * KC];
#pragma unroll
    for (int v = 0; v < 4 * KC; v++) acc[v] = 0.0;
    const int64_t base = (int64_t)tc.tile * kBlock * per_thread + threadIdx.x;
    for (int m = 0; m < per_thread; m++) {
        const int64_t i = base + (int64_t)m * kBlock;
        const double4 a = p64[i];
#pragma unroll
        for (int kk = 0; kk < KC; kk++) {
            const double4 n = knr[kk];
            const double pxy = fma(n.y, a.y, n.x * a.x);
            const double pz = n.z * a.z;
            double c1, s1, c2, s2;
            sincos_rev64(pxy + pz, &s1, &c1);
            sincos_rev64(pxy - pz, &s2, &c2);
            acc[4 * kk + 0] = fma(a.w, c1, acc[4 * kk + 0]);
            acc[4 * kk + 1] = fma(a.w, s1, acc[4 * kk + 1]);
            acc[4 * kk + 2] = fma(a.w, c2, acc[4 * kk + 2]);
            acc[4 * kk + 3] = fma(a.w, s2, acc[4 * kk + 3]);
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    wave_transpose_reduce<4 * KC>(acc, lane);
    if (lane < 4 * KC) sh[wid][lane] = acc[0];
    __syncthreads();
    if (threadIdx.x < 4 * KC) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; w++) t += sh[w][threadIdx.x];
        part[((int64_t)tc.tile * P_pad + tc.kc * KC) * 4 + threadIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// 4. reduce over tiles (FP64, fixed order) and recalibrate (Sec. 3.4):
//    rho^M = (1 + Y_even) rho + Y_odd rhohat,
//    A = rho^M + (1 + conj Y_even) rho,  B = conj(Y_odd) rho,
//    c = 2 pi S pref / (V P |k|^2),  e = c Re(rho conj(rho^M)).
//    One wave per (system, k); lanes split the tiles and the image orders.
// ---------------------------------------------------------------------------

struct AssembleArgs {
    const double *part;         // structure-factor partials [tile][P_pad][4], FP64 in both precisions
    int P, P_pad;
    const int *tbase;
    const int32_t *kset;
    const SysDesc *sys;
    const ImgTable *img;
    double *krec;
    float4 *kf32;
    int n_sys, with_scalars;   // with_scalars: n_sys more blocks compute the IBC scalars
    ScalArgs sc;
};

__device__ __forceinline__ double dmono(int e_self, double g_self, int e_other, double g_other) {
    // d/dg_self of g_self^e_self g_other^e_other
    if (e_self == 0) return 0.0;
    double r = (double)e_self;
    for (int i = 0; i < e_self - 1; i++) r *= g_self;
    for (int i = 0; i < e_other; i++) r *= g_other;
    return r;
}

// a double held by lane `src`, read by every lane
__device__ __forceinline__ double lane_value(double v, int src) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), src),
                            __builtin_amdgcn_readlane(__double2loint(v), src));
}

// One wave per (system, k).  DG: also the gamma derivatives of Y_odd and
// Y_even (for dE/dgamma; zero otherwise).
template <bool DG>
__global__ __launch_bounds__(64) void k_assemble(AssembleArgs a) {
    if ((int)blockIdx.x >= a.n_sys * a.P) {
        ibc_scalars(a.sc, blockIdx.x - a.n_sys * a.P, threadIdx.x);
        return;
    }
    const int r = blockIdx.x / a.P, l = blockIdx.x - r * a.P;
    const SysDesc &d = a.sys[r];
    const ImgTable &it = a.img[r];
    const int lane = threadIdx.x;
    // v[0..3]: this lane's share of rho and rhohat (lanes split the tiles);
    // v[4..7]: Yo, Ye; v[8..15]: dYo/dg_top, dYe/dg_top, dYo/dg_bot,
    // dYe/dg_bot (lanes split the image orders o = lane+1, lane+65, ...)
    constexpr int NV = DG ? 16 : 8;
    double v[NV];
#pragma unroll
    for (int c = 0; c < NV; c++) v[c] = 0.0;
    for (int t = a.tbase[r] + lane; t < a.tbase[r + 1]; t += 64) {
        const int64_t o = ((int64_t)t * a.P_pad + l) * 4;
        for (int c = 0; c < 4; c++) v[c] += a.part[o + c];
    }
    const int64_t kg = (int64_t)r * a.P + l;
    const int nx = a.kset[3 * kg], ny = a.kset[3 * kg + 1], nz = a.kset[3 * kg + 2];
    const double rev_per_H = (double)nz * d.H / d.Lz;   // kz H / (2 pi)
    for (int o = lane + 1; o <= d.M; o += 64) {
        const double gpl = it.gp[o - 1], gml = it.gm[o - 1];
        double mp, mm;   // multiples of kz H in the exponents of the + and - terms
        int slot;
        if (o & 1) { mp = (double)(o + 1); mm = -(double)(o - 1); slot = 4; }
        else       { mp = (double)o;       mm = -(double)o;       slot = 6; }
        double sp, cp, sm, cm;
        sincos_rev64(mp * rev_per_H, &sp, &cp);
        sincos_rev64(mm * rev_per_H, &sm, &cm);
        v[slot] += gpl * cp + gml * cm;
        v[slot + 1] += gpl * sp + gml * sm;
        if constexpr (DG) {
            const double dpt = dmono(it.ea_p[o - 1], d.g_top, it.eb_p[o - 1], d.g_bot);
            const double dmt = dmono(it.ea_m[o - 1], d.g_top, it.eb_m[o - 1], d.g_bot);
            const double dpb = dmono(it.eb_p[o - 1], d.g_bot, it.ea_p[o - 1], d.g_top);
            const double dmb = dmono(it.eb_m[o - 1], d.g_bot, it.ea_m[o - 1], d.g_top);
            v[4 + slot] += dpt * cp + dmt * cm;
            v[5 + slot] += dpt * sp + dmt * sm;
            v[8 + slot] += dpb * cp + dmb * cm;
            v[9 + slot] += dpb * sp + dmb * sm;
        }
    }
    // the NV wave sums at once (fixed-order butterfly): lane c then holds
    // the sum of value c, which every lane reads
    wave_transpose_reduce<NV>(v, lane);
    double S[NV];
#pragma unroll
    for (int c = 0; c < NV; c++) S[c] = lane_value(v[0], c);
    const double rr = S[0], ri = S[1], hr = S[2], hi = S[3];
    const double *y = S + 4;   // Yo, Ye (re, im), then the derivatives
    const double kx = 2.0 * kPi * nx / d.Lx, ky = 2.0 * kPi * ny / d.Ly, kz = 2.0 * kPi * nz / d.Lz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    const double c = d.cfac / k2;
    // rho^M = (1 + Ye) rho + Yo rhohat
    const double er = 1.0 + y[2], ei = y[3];
    const double mr = er * rr - ei * ri + y[0] * hr - y[1] * hi;
    const double mi = er * ri + ei * rr + y[0] * hi + y[1] * hr;
    // A = rho^M + (1 + conj Ye) rho ; B = conj(Yo) rho
    const double Ar = mr + er * rr + ei * ri;
    const double Ai = mi + er * ri - ei * rr;
    const double Br = y[0] * rr + y[1] * ri;
    const double Bi = y[0] * ri - y[1] * rr;
    // polar form for the force passes, Im(e^{-i ph} cA) = |cA| sin(arg cA - ph):
    // lane 1 for A, lane 2 for B, in parallel
    constexpr double inv2pi = 0.15915494309189535;
    double mag = 0.0, arg = 0.0;
    if (lane == 1 || lane == 2) {
        const double xr = lane == 1 ? Ar : Br, xi = lane == 1 ? Ai : Bi;
        mag = c * hypot(xr, xi);
        arg = atan2(xi, xr) * inv2pi;
    }
    const double magA = lane_value(mag, 1), argA = lane_value(arg, 1);
    const double magB = lane_value(mag, 2), argB = lane_value(arg, 2);
    if (lane != 0) return;
    const double e = c * (rr * mr + ri * mi);
    // d e / d gamma = c Re(rho conj(dYe rho + dYo rhohat))
    double de[2] = {0.0, 0.0};
    if constexpr (DG) {
        for (int w = 0; w < 2; w++) {
            const double *dy = y + 4 + 4 * w;
            const double tr = dy[2] * rr - dy[3] * ri + dy[0] * hr - dy[1] * hi;
            const double ti = dy[2] * ri + dy[3] * rr + dy[0] * hi + dy[1] * hr;
            de[w] = c * (rr * tr + ri * ti);
        }
    }
    double *rec = a.krec + kg * kKRec;
    rec[0] = kx; rec[1] = ky; rec[2] = kz;
    rec[3] = c * Ar; rec[4] = c * Ai; rec[5] = c * Br; rec[6] = c * Bi;
    rec[7] = e; rec[8] = de[0]; rec[9] = de[1];
    rec[10] = nx; rec[11] = ny; rec[12] = nz;
    rec[13] = rr; rec[14] = ri; rec[15] = kx * kx + ky * ky;
    rec[16] = magA; rec[17] = argA; rec[18] = magB; rec[19] = argB;
    a.kf32[3 * kg] = make_float4((float)kx, (float)ky, (float)kz, (float)(kx * kx + ky * ky));
    a.kf32[3 * kg + 1] = make_float4((float)(c * Ar), (float)(c * Ai), (float)(c * Br), (float)(c * Bi));
    a.kf32[3 * kg + 2] = make_float4((float)magA, (float)argA, (float)magB, (float)argB);
}

int choose_tile(int64_t N, int n_kchunks) {
    // particles per thread: fill the chip with >= ~4096 blocks if N allows,
    // but keep tiles long enough to amortise the block reduction.
    int per = kMaxTileThreads;
    while (per > 1) {
        const int64_t tiles = (N + (int64_t)kBlock * per - 1) / ((int64_t)kBlock * per);
        if (tiles * n_kchunks >= 4096) break;
        per >>= 1;
    }
    return per;
}

hipError_t launch_kcoef_sf(rbe2d_ctx *h, hipStream_t s, bool with_scalars, bool want_dg) {
    const bool fp32 = h->precision == RBE2D_PREC_FP32_PHASE;
    prof_begin(h, 1, s);
    if (h->n_tiles > 0) {
        const int tiles8 = (h->n_tiles + 7) / 8 * 8;
        if (fp32) {
            const dim3 g((unsigned)tiles8 * (h->P_pad / kKChunk32));
            hipLaunchKernelGGL(k_sf32<kKChunk32>, g, dim3(kBlock), 0, s, h->w.p32, h->w.kn32, h->w.lay.tbase,
                               h->n_sys, h->per, h->P_pad, h->n_tiles, (double *)h->w.sfpart);
        } else {
            const dim3 g((unsigned)tiles8 * (h->P_pad / kKChunk64));
            hipLaunchKernelGGL(k_sf64<kKChunk64>, g, dim3(kBlock), 0, s, h->w.p64, h->w.kn64, h->w.lay.tbase,
                               h->n_sys, h->per, h->P_pad, h->n_tiles, (double *)h->w.sfpart);
        }
    }
    prof_end(h, 1, s);
    AssembleArgs a;
    a.part = (const double *)h->w.sfpart; a.P = h->P; a.P_pad = h->P_pad;
    a.tbase = h->w.lay.tbase; a.kset = h->w.kset; a.sys = h->w.sys; a.img = h->w.img;
    a.krec = h->w.krec; a.kf32 = h->w.kf32;
    a.n_sys = h->n_sys; a.with_scalars = with_scalars; a.sc = scal_args(h);
    prof_begin(h, 2, s);
    const dim3 ga(h->n_sys * h->P + (with_scalars ? h->n_sys : 0));
    if (want_dg) hipLaunchKernelGGL(k_assemble<true>, ga, dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_assemble<false>, ga, dim3(64), 0, s, a);
    prof_end(h, 2, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 5. force scatter: one thread per particle, all k (or a k-range) uniform:
//    F_i = -q_i sum_l [k_l Im(e^{-i phi} cA_l) + khat_l Im(e^{-i phihat} cB_l)]
//    pot_i = sum_l [Re(e^{-i phi} cA_l) + Re(e^{-i phihat} cB_l)]   (dE_k/dq_i)
// ---------------------------------------------------------------------------

struct ForceArgs {
    const float4 *p32;
    const double4 *p64;
    const float4 *kn32;
    const double4 *kn64;
    const float4 *kf32;
    const double *krec;
    Layout lay;
    const SysDesc *sys;
    int n_sys, P, P_pad, k_per_split, n_threads;   // n_threads = particle blocks * kBlock
    const double *pos;       // for the IBC potential (z_i)
    const double *q;
    const double *scal;
    const double4 *freal;    // added when add_real
    double *fpart;           // [split][n_threads][4] when splitting
    double *F;               // final output (caller order, N x 3)
    double *dEdq;            // final dE/dq when want_pot
    double *var;             // force-variance estimate per particle (variance mode)
    const double *gE;        // scale of the backward outputs (device scalar) or null
    int accumulate, add_real, want_pot, want_var, do_kspace, do_ibc, split;
};

__device__ __forceinline__ void finish_particle(const ForceArgs &a, int r, int64_t g, double fx,
                                                double fy, double fz, double pot) {
    const SysDesc &d = a.sys[r];
    const double *sc = a.scal + kScal * r;
    const double qi = a.q[g];
    if (a.want_var) {
        // pot carries sum_l |t_l|^2 / q_i^2: (P sum |t|^2 - |F|^2) / (P - 1)
        const double P = (double)a.P;
        a.var[g] = a.P > 1 ? qi * qi * (P * pot - (fx * fx + fy * fy + fz * fz)) / (P - 1.0) : 0.0;
        return;
    }
    double Fx = 0, Fy = 0, Fz = 0, ph = 0;
    if (a.do_kspace) {
        Fx = -qi * fx; Fy = -qi * fy; Fz = -qi * fz;
        ph = pot - 2.0 * d.alpha * d.pref / sqrt(kPi) * qi;   // + dE_self/dq_i
    }
    if (a.do_ibc) {
        if (d.surf) {
            // IBC with the surface terms: linear (and quadratic) in z
            const double z = a.pos[3 * g + 2];
            Fz += qi * (sc[4] + sc[10] + sc[9] * z);
            ph += -sc[4] * z + sc[5] + sc[11] + z * (sc[12] + sc[13] * z);
        } else {
            Fz += qi * sc[4];
            ph += -sc[4] * a.pos[3 * g + 2] + sc[5];
        }
    }
    if (a.add_real) {
        const double4 rr = a.freal[g];
        Fx += rr.x; Fy += rr.y; Fz += rr.z; ph += rr.w;
    }
    if (a.want_pot) {
        // backward: dL/dr = -gE F, dL/dq = gE phi
        const double gs = a.gE ? *a.gE : 1.0;
        if (a.F) {
            a.F[3 * g] = -gs * Fx; a.F[3 * g + 1] = -gs * Fy; a.F[3 * g + 2] = -gs * Fz;
        }
        if (a.dEdq) a.dEdq[g] = gs * ph;
        return;
    }
    if (a.accumulate) {
        a.F[3 * g] += Fx; a.F[3 * g + 1] += Fy; a.F[3 * g + 2] += Fz;
    } else {
        a.F[3 * g] = Fx; a.F[3 * g + 1] = Fy; a.F[3 * g + 2] = Fz;
    }
}

// MODE 0: forces; 1: forces and potentials (adjoint); 2: forces and the sum
// of the squared per-k force terms (variance estimate)
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_force32(ForceArgs a) {
    const int b = blockIdx.x;
    const int r = find_sys(a.lay.bbase, a.n_sys, b);
    const int iloc = (b - a.lay.bbase[r]) * kBlock + threadIdx.x;
    if (iloc >= a.lay.off[r + 1] - a.lay.off[r]) return;
    const int64_t ii = (int64_t)a.lay.pbase[r] + iloc;
    const int64_t g = (int64_t)a.lay.off[r] + iloc;
    const float4 pa = a.p32[2 * ii];
    const float4 pb = a.p32[2 * ii + 1];
    const float4 *kn = a.kn32 + (int64_t)r * a.P_pad;
    const float4 *kf = a.kf32 + 3 * (int64_t)r * a.P;
    const int l0 = blockIdx.y * a.k_per_split;
    const int l1 = min(a.P, l0 + a.k_per_split);
    double Fx = 0, Fy = 0, Fz = 0, Pt = 0;
    if (a.do_kspace) {
        // per k: n (kn), k and |k_xy|^2 (kv), and the amplitudes (ab for the
        // potentials, else their polar form)
        constexpr int kExtra = MODE == 1 ? 1 : 2;
        float fx = 0, fy = 0, fz = 0, pt = 0;
        auto one = [&](const float4 &n, const float4 &kv, const float4 &ex) {
            float pxy = fractf(fmaf(n.y, pa.z, n.x * pa.x));
            pxy = fmaf(n.x, pa.y, pxy);
            pxy = fmaf(n.y, pa.w, pxy);
            const float pz = fmaf(n.z, pb.y, fractf(n.z * pb.x));
            float X, Y;   // Im(e^{-i ph} cA), Im(e^{-i phh} cB)
            if (MODE == 1) {
                // the potential needs the real parts too (ex = cA, cB)
                const float ph = pxy + pz, phh = pxy - pz;
                const float c1f = cos_rev(ph), s1f = sin_rev(ph);
                const float c2f = cos_rev(phh), s2f = sin_rev(phh);
                X = fmaf(ex.y, c1f, -ex.x * s1f);
                Y = fmaf(ex.w, c2f, -ex.z * s2f);
                pt = fmaf(ex.x, c1f, pt); pt = fmaf(ex.y, s1f, pt);
                pt = fmaf(ex.z, c2f, pt); pt = fmaf(ex.w, s2f, pt);
            } else {
                // polar form: one transcendental per product
                X = ex.x * sin_rev((ex.y - pxy) - pz);
                Y = ex.z * sin_rev((ex.w - pxy) + pz);
            }
            const float sp = X + Y, sm = X - Y;
            fx = fmaf(kv.x, sp, fx);
            fy = fmaf(kv.y, sp, fy);
            fz = fmaf(kv.z, sm, fz);
            if (MODE == 2) pt = fmaf(kv.w * sp, sp, fmaf(kv.z * sm, kv.z * sm, pt));
        };
        for (int c0 = l0; c0 < l1; c0 += 64) {
            const int c1 = min(l1, c0 + 64);
            fx = fy = fz = pt = 0;
            int l = c0;
            // four k at a time: their records are fetched together (scalar
            // loads), one wait per four instead of one per k
            for (; l + 4 <= c1; l += 4) {
                float4 n[4], kv[4], ex[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    n[j] = kn[l + j];
                    kv[j] = kf[3 * (l + j)];
                    ex[j] = kf[3 * (l + j) + kExtra];
                }
#pragma unroll
                for (int j = 0; j < 4; j++) one(n[j], kv[j], ex[j]);
            }
            for (; l < c1; l++) one(kn[l], kf[3 * l], kf[3 * l + kExtra]);
            Fx += fx; Fy += fy; Fz += fz; Pt += pt;
        }
    }
    if (a.split) {
        double *o = a.fpart + ((int64_t)blockIdx.y * a.n_threads + (int64_t)b * kBlock + threadIdx.x) * 4;
        o[0] = Fx; o[1] = Fy; o[2] = Fz; o[3] = Pt;
    } else {
        finish_particle(a, r, g, Fx, Fy, Fz, Pt);
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_force64(ForceArgs a) {
    const int b = blockIdx.x;
    const int r = find_sys(a.lay.bbase, a.n_sys, b);
    const int iloc = (b - a.lay.bbase[r]) * kBlock + threadIdx.x;
    if (iloc >= a.lay.off[r + 1] - a.lay.off[r]) return;
    const int64_t ii = (int64_t)a.lay.pbase[r] + iloc;
    const int64_t g = (int64_t)a.lay.off[r] + iloc;
    const double4 p = a.p64[ii];
    const double4 *kn = a.kn64 + (int64_t)r * a.P_pad;
    const double *kr = a.krec + (int64_t)r * a.P * kKRec;
    const int l0 = blockIdx.y * a.k_per_split;
    const int l1 = min(a.P, l0 + a.k_per_split);
    double fx = 0, fy = 0, fz = 0, pt = 0;
    if (a.do_kspace) {
        for (int l = l0; l < l1; l++) {
            const double4 n = kn[l];
            const double *rec = kr + (int64_t)l * kKRec;
            const double pxy = fma(n.y, p.y, n.x * p.x);
            const double pz = n.z * p.z;
            double X, Y;   // Im(e^{-i ph} cA), Im(e^{-i phh} cB)
            if (MODE == 1) {
                // the potential needs the real parts too
                double c1, s1, c2, s2;
                sincos_rev64(pxy + pz, &s1, &c1);
                sincos_rev64(pxy - pz, &s2, &c2);
                X = fma(rec[4], c1, -rec[3] * s1);
                Y = fma(rec[6], c2, -rec[5] * s2);
                pt = fma(rec[3], c1, pt); pt = fma(rec[4], s1, pt);
                pt = fma(rec[5], c2, pt); pt = fma(rec[6], s2, pt);
            } else {
                // polar form: one sine per product
                X = rec[16] * sin_rev64((rec[17] - pxy) - pz);
                Y = rec[18] * sin_rev64((rec[19] - pxy) + pz);
            }
            const double sp = X + Y, sm = X - Y;
            fx = fma(rec[0], sp, fx);
            fy = fma(rec[1], sp, fy);
            fz = fma(rec[2], sm, fz);
            if (MODE == 2) pt = fma(rec[15] * sp, sp, fma(rec[2] * sm, rec[2] * sm, pt));
        }
    }
    if (a.split) {
        double *o = a.fpart + ((int64_t)blockIdx.y * a.n_threads + (int64_t)b * kBlock + threadIdx.x) * 4;
        o[0] = fx; o[1] = fy; o[2] = fz; o[3] = pt;
    } else {
        finish_particle(a, r, g, fx, fy, fz, pt);
    }
}

__global__ __launch_bounds__(kBlock) void k_force_combine(ForceArgs a, int nsplit) {
    const int b = blockIdx.x;
    const int r = find_sys(a.lay.bbase, a.n_sys, b);
    const int iloc = (b - a.lay.bbase[r]) * kBlock + threadIdx.x;
    if (iloc >= a.lay.off[r + 1] - a.lay.off[r]) return;
    const int64_t g = (int64_t)a.lay.off[r] + iloc;
    double fx = 0, fy = 0, fz = 0, pt = 0;
    for (int sidx = 0; sidx < nsplit; sidx++) {
        const double *o = a.fpart + ((int64_t)sidx * a.n_threads + (int64_t)b * kBlock + threadIdx.x) * 4;
        fx += o[0]; fy += o[1]; fz += o[2]; pt += o[3];
    }
    finish_particle(a, r, g, fx, fy, fz, pt);
}

int choose_ksplit(int64_t nb, int P) {
    // split the k-loop across blocks when there are too few particles to fill the chip
    int split = 1;
    while (nb * split < 2048 && split * 2 <= 64 && (P + split * 2 - 1) / (split * 2) >= 8) split *= 2;
    return split;
}

hipError_t launch_kforce(rbe2d_ctx *h, const double *pos, const double *q, double *F, double *dEdq,
                         uint32_t flags, bool accumulate, bool want_pot, bool add_real, const double *gE,
                         hipStream_t s, double *var) {
    if (h->n_total == 0) return hipSuccess;
    ForceArgs a;
    a.p32 = h->w.p32; a.p64 = h->w.p64; a.kn32 = h->w.kn32; a.kn64 = h->w.kn64;
    a.kf32 = h->w.kf32; a.krec = h->w.krec; a.lay = h->w.lay; a.sys = h->w.sys;
    a.n_sys = h->n_sys; a.P = h->P; a.P_pad = h->P_pad; a.n_threads = h->n_blocks * kBlock;
    a.pos = pos; a.q = q; a.scal = h->w.scal; a.freal = h->w.freal;
    a.fpart = h->w.fpart; a.F = F; a.dEdq = dEdq; a.gE = gE; a.var = var;
    a.accumulate = accumulate; a.add_real = add_real; a.want_pot = want_pot; a.want_var = var != nullptr;
    a.do_kspace = (flags & RBE2D_KSPACE) != 0; a.do_ibc = (flags & RBE2D_IBC) != 0;
    int split = 1;
    if (a.do_kspace) {
        split = h->force_ksplit ? h->force_ksplit
                                : (h->tuned_now && h->tune.ksplit ? h->tune.ksplit : choose_ksplit(h->n_blocks, h->P));
        // the partial buffer holds fpart_blocks blocks' worth
        while (split > 1 && (int64_t)split * h->n_blocks > h->fpart_blocks) split >>= 1;
    }
    a.k_per_split = (h->P + split - 1) / split;
    a.split = split > 1;
    const bool fp32 = h->precision == RBE2D_PREC_FP32_PHASE;
    dim3 g(h->n_blocks, split);
    prof_begin(h, 5, s);
    if (fp32) {
        if (var) hipLaunchKernelGGL(k_force32<2>, g, dim3(kBlock), 0, s, a);
        else if (want_pot) hipLaunchKernelGGL(k_force32<1>, g, dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL(k_force32<0>, g, dim3(kBlock), 0, s, a);
    } else {
        if (var) hipLaunchKernelGGL(k_force64<2>, g, dim3(kBlock), 0, s, a);
        else if (want_pot) hipLaunchKernelGGL(k_force64<1>, g, dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL(k_force64<0>, g, dim3(kBlock), 0, s, a);
    }
    if (a.split) hipLaunchKernelGGL(k_force_combine, dim3(h->n_blocks), dim3(kBlock), 0, s, a, split);
    prof_end(h, 5, s);
    return hipGetLastError();
}

}  // namespace rbe2d
