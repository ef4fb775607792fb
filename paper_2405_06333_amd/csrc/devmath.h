// Device helpers shared by the kernels of librbe2d: FP64 sincos on
// revolutions, wave and block reductions with a fixed summation order.
#pragma once

#include "rbe2d_internal.h"
#include "sincos_fit.h"

namespace rbe2d {

// sin and cos of 2 pi r: r is reduced to the nearest quarter turn
// (r - q/4 is exact by Sterbenz' lemma), then the polynomials of
// sincos_fit.h (Chebyshev interpolants in t^2, gen_sincos_fit.py) on
// |t| <= pi/4, within 1.2e-16 of sin and cos.
__device__ __forceinline__ void sincos_rev64(double r, double *s_out, double *c_out) {
    const double qd = rint(4.0 * r);
    const double f = fma(-0.25, qd, r);
    // quarter turns mod 4 (|4 r| < 2^31 for every phase of the method; the
    // two's-complement low bits are the residue for negative counts too)
    const int qi = (int)qd;
    const double t = f * (2.0 * kPi);
    const double t2 = t * t;
    double ps = kSinQuarter[kSinQuarterTerms - 1];
#pragma unroll
    for (int k = kSinQuarterTerms - 2; k >= 0; k--) ps = fma(ps, t2, kSinQuarter[k]);
    const double sn = fma(t * t2, ps, t);
    double pc = kCosQuarter[kCosQuarterTerms - 1];
#pragma unroll
    for (int k = kCosQuarterTerms - 2; k >= 0; k--) pc = fma(pc, t2, kCosQuarter[k]);
    pc = fma(pc, t2, -0.5);
    const double cs = fma(t2, pc, 1.0);
    // rotate by qi quarter turns: swap for odd qi, then flip the sign bits
    // (sin for qi = 2, 3; cos for qi = 1, 2 mod 4)
    const bool swap = qi & 1;
    const double s0 = swap ? cs : sn;
    const double c0 = swap ? sn : cs;
    const int ssign = (qi & 2) << 30, csign = ((qi + 1) & 2) << 30;
    *s_out = __hiloint2double(__double2hiint(s0) ^ ssign, __double2loint(s0));
    *c_out = __hiloint2double(__double2hiint(c0) ^ csign, __double2loint(c0));
}

// sin of 2 pi r alone: r is reduced to the nearest half turn (exact, as
// above), then the half-turn polynomial of sincos_fit.h on |t| <= pi/2,
// within 2.3e-16 of sin; an odd half turn flips the sign.
__device__ __forceinline__ double sin_rev64(double r) {
    const double kd = rint(2.0 * r);
    const double f = fma(-0.5, kd, r);
    const double t = f * (2.0 * kPi);
    const double t2 = t * t;
    double p = kSinHalf[kSinHalfTerms - 1];
#pragma unroll
    for (int k = kSinHalfTerms - 2; k >= 0; k--) p = fma(p, t2, kSinHalf[k]);
    const double s = fma(t * t2, p, t);
    // an odd half turn flips the sign bit (|2 r| < 2^31, as above)
    const int sign = ((int)kd & 1) << 31;
    return __hiloint2double(__double2hiint(s) ^ sign, __double2loint(s));
}

// x += dt v, then x, y wrapped into the box and z folded into [zlo, zhi]:
// every crossing of a wall is a specular reflection (v_z flips)
__device__ __forceinline__ void drift_fold(const SysDesc &d, double dt, double zlo, double zhi_from_top, double v[3],
                                           double r[3]) {
    for (int c = 0; c < 3; c++) r[c] = fma(dt, v[c], r[c]);
    r[0] -= d.Lx * floor(r[0] / d.Lx);
    r[1] -= d.Ly * floor(r[1] / d.Ly);
    const double zhi = d.H - zhi_from_top;
    const double W = zhi - zlo;
    const double u = r[2] - zlo;
    const double m = floor(u / W);
    const double rem = u - m * W;
    const bool odd = fmod(fabs(m), 2.0) == 1.0;
    r[2] = odd ? zhi - rem : zlo + rem;
    if (odd) v[2] = -v[2];
    r[2] = fmin(fmax(r[2], zlo), zhi);
}

__device__ __forceinline__ float fractf(float x) { return __builtin_amdgcn_fractf(x); }
__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }
__device__ __forceinline__ float cos_rev(float x) { return __builtin_amdgcn_cosf(x); }

// Butterfly reduction of NV values held by every lane of a wave64: after it,
// lane L holds (in v[0]) the wave-wide sum of value index L mod NV.  At each
// stage a lane keeps one half of its values and swaps the other half with
// the partner lane (lane ^ half).  Fixed order, so deterministic.
template <int HALF, int NV, typename T>
struct TransposeStage {
    __device__ __forceinline__ static void run(T (&v)[NV], int lane) {
        const bool upper = (lane & HALF) != 0;
#pragma unroll
        for (int i = 0; i < HALF; i++) {
            const T send = upper ? v[i] : v[i + HALF];
            const T keep = upper ? v[i + HALF] : v[i];
            v[i] = keep + __shfl_xor(send, HALF, 64);
        }
        TransposeStage<HALF / 2, NV, T>::run(v, lane);
    }
};
template <int NV, typename T>
struct TransposeStage<0, NV, T> {
    __device__ __forceinline__ static void run(T (&)[NV], int) {}
};

template <int NV, typename T>
__device__ __forceinline__ void wave_transpose_reduce(T (&v)[NV], int lane) {
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two <= 64");
    TransposeStage<NV / 2, NV, T>::run(v, lane);
    // lanes L and L ^ NV, L ^ 2NV, ... hold partial sums of the same index
#pragma unroll
    for (int o = NV; o < 64; o <<= 1) v[0] += __shfl_xor(v[0], o, 64);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// deterministic block sum (blockDim.x = kBlock) of one double; result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) r += sh[k];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum_r(double v, double *sh) { return block_sum(v, sh); }

}  // namespace rbe2d
